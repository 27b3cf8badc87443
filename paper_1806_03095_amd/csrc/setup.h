// Host-side setup of the DG operator: 1D rules and bases, the mesh, metric terms
// and penalty parameters, as plain host arrays (no HIP runtime calls here).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "dg_common.h"
#include "dgns.h"

namespace dgns {

// Fills the 1D tables of degree k, n_q flux points, basis DGNS_BASIS_*.
void build_tables(int k, int q, int basis, Tables1D& t);

struct HostSetup {
    Tables1D tab;
    bool gen = false;              // per-quadrature-point metric (curved or stretched meshes)
    int64_t ncell = 0, n3 = 0;
    double h_min = 0;
    std::vector<double> geo;       // [E][3][N3] geometry nodes (LGL)
    std::vector<double> node_x;    // [3][E][N3] coordinates of the basis nodes
    std::vector<double> metric;    // see OpArgs::cell_metric
    std::vector<double> mass_jxw;  // general meshes only
    std::vector<double> face[3];   // general meshes only
    std::vector<double> tau[3];    // penalty per face
};

// Builds everything for a context; returns 0, or a DGNS_E* code with err set.
int build_setup(const dgns_params& prm, const dgns_box_mesh& msh, HostSetup& out, std::string& err);

}  // namespace dgns
