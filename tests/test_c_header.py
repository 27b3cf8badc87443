"""The C ABI from C: include/dgns.h compiles as C99 with warnings as errors, a C program
links against libdgns.so and gets the documented error codes back (no GPU needed: only
argument checks are exercised)."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1806_03095_amd")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "dgns.h"

int main(void) {
    dgns_params p;
    dgns_box_mesh m;
    dgns_ctx* ctx = (dgns_ctx*)0;
    double out[8];
    memset(&p, 0, sizeof p);
    memset(&m, 0, sizeof m);
    if (dgns_create((const dgns_params*)0, &m, (void*)0, &ctx) != DGNS_EINVAL) return 1;
    p.degree = 0;   /* out of range */
    p.n_q = 4;
    p.gamma = 1.4;
    p.R = 287.0;
    p.rho_ref = 1.0;
    m.n[0] = m.n[1] = m.n[2] = 2;
    m.hi[0] = m.hi[1] = m.hi[2] = 1.0;
    m.periodic[0] = m.periodic[1] = m.periodic[2] = 1;
    if (dgns_create(&p, &m, (void*)0, &ctx) != DGNS_EINVAL || ctx != (dgns_ctx*)0) return 2;
    if (strlen(dgns_last_error()) == 0) return 3;
    if (dgns_diagnostics((dgns_ctx*)0, (const double*)0, (const double*)0, out) != DGNS_EINVAL) return 4;
    if (dgns_rk_step((dgns_ctx*)0, (double*)0, (double*)0, 0.0, 1e-3) != DGNS_EINVAL) return 5;
    if (dgns_channel_statistics((dgns_ctx*)0, (const double*)0, out) != DGNS_EINVAL) return 6;
    printf("ok: %s\n", dgns_last_error());
    return 0;
}
"""


def test_header_is_c99_and_links():
    lib = os.path.join(LIBDIR, "libdgns.so")
    if not os.path.exists(lib):
        pytest.skip("libdgns.so is not built")
    with tempfile.TemporaryDirectory() as td:
        src, exe = os.path.join(td, "abi.c"), os.path.join(td, "abi")
        open(src, "w").write(PROGRAM)
        r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                            src, "-L", LIBDIR, "-ldgns", "-Wl,-rpath," + LIBDIR, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
        assert r.stdout.startswith("ok")
