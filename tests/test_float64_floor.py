"""The float64 rounding floor of the oracle, measured against extended precision (CPU).

tests/extended.py evaluates the same operator in x87 extended precision.  Pinned here
against the oracle where both are accurate (Mach 0.3, small meshes: agreement to
rounding), and against exact rules.  Then the oracle's own float64 error is measured
on the workloads whose GPU parity bounds are derived from it (tests/floor.py): it grows
at low Mach number (momentum rows cancel the background pressure p0 = 71 against an
O(1) result) and as the mesh is refined (each quadrature term of a momentum row is of
order p0 h^2 against a result of order h^3).  The asserted ceilings are the measured
values rounded up by about 1.5, so that a change of the oracle's rounding is noticed.
"""
import math

import numpy as np
import pytest
import torch

from oracle import initial, mesh as omesh, operator as ooperator, timeint
from tests import floor
from tests.extended import LD, gauss, lobatto
from tests.gpu_cases import channel_input, patched_state, sample_cells, tgv_fluid, tgv_input

PI3 = ((-math.pi,) * 3, (math.pi,) * 3)


def test_extended_rules_are_exact():
    for n in (2, 4, 7, 11):
        x, w = gauss(n)
        for p in range(2 * n):
            assert abs((w * x ** p).sum() - LD(1) / (p + 1)) < 1e-18, (n, p)
        xl = lobatto(n)
        # the Gauss-Lobatto rule with its weights integrates degree 2n - 3 exactly
        V = np.array([[xi ** p for xi in xl] for p in range(n)], dtype=LD)
        b = np.array([LD(1) / (p + 1) for p in range(n)], dtype=LD)
        wl = np.linalg.solve(V.astype(np.float64), b.astype(np.float64))     # weights (float64 suffice)
        assert abs(float((wl * xl.astype(np.float64) ** (2 * n - 3)).sum()) - 1.0 / (2 * n - 2)) < 1e-12


@pytest.mark.parametrize("n,k,nq,kind,amp,basis", [
    ((2, 2, 2), 2, 3, omesh.AFFINE, 0.0, "LGL"),
    ((2, 2, 3), 2, 4, omesh.CURVED, 0.1, "LGL"),
    ((2, 3, 2), 3, 5, omesh.AFFINE, 0.0, "GL"),
])
def test_extended_matches_oracle_at_mach_03(n, k, nq, kind, amp, basis):
    oop = ooperator.DGOperator(omesh.BoxMesh(n, *PI3, k, kind=kind, deform_amp=amp), tgv_fluid(), nq, basis=basis)
    U = tgv_input(oop, mach=0.3)
    cells = list(range(oop.mesh.n_cells))
    e = floor.oracle_floor(oop, U, cells, "R")
    assert max(e) < 1e-12, e


def test_extended_matches_oracle_channel_walls_force():
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (1.4 * 287.0)
    om = omesh.BoxMesh((2, 4, 1), (0, -1, 0), (2 * math.pi, 1, math.pi), 4, periodic=(True, False, True),
                       kind=omesh.CHANNEL)
    oop = ooperator.DGOperator(om, fl, 7, body_force=(1.0, 0.0, 0.0), wall_T=T0)
    U = channel_input(oop)
    e = floor.oracle_floor(oop, U, list(range(oop.mesh.n_cells)), "R")
    assert max(e) < 2e-12, e


def _tgv_floor(n, k, nq, count, seed):
    oop = ooperator.DGOperator(omesh.BoxMesh((n,) * 3, *PI3, k), tgv_fluid(), nq)
    if n == 4:
        U = tgv_input(oop)
        cells = list(range(64))
    else:
        cells = sample_cells((n,) * 3, count, seed)[:count]
        p0 = 1.0 / (oop.fl.gamma * 0.01)
        U = patched_state(oop, cells, lambda x: initial.taylor_green(x, oop.fl, mach=0.1),
                          [1.0, 0.0, 0.0, 0.0, p0 / (oop.fl.gamma - 1.0)], seed=seed + 1, noise=1e-3)
    return floor.oracle_floor(oop, U, cells, "L")


# measured per-field floors of L (rho, rho u, rho v, rho w, rho E), Mach 0.1 Taylor-Green
# plus 1e-3 noise; ceilings about 1.5 times the measurement
@pytest.mark.parametrize("n,k,nq,count,ceiling", [
    (4, 3, 6, 64, (4e-13, 8e-12, 8e-12, 8e-12, 4e-13)),
    (32, 3, 6, 6, (1e-12, 6e-11, 6e-11, 6e-11, 1.5e-12)),
    (24, 5, 8, 3, (2e-12, 1.5e-10, 1.5e-10, 1.5e-10, 2e-12)),
])
def test_oracle_float64_floor(n, k, nq, count, ceiling):
    e = _tgv_floor(n, k, nq, count, seed=11)
    print("oracle float64 floor of L, %d^3 k=%d n_q=%d:" % (n, k, nq), ["%.1e" % v for v in e])
    assert all(v < c for v, c in zip(e, ceiling)), (e, ceiling)
    # low Mach number: the momentum rows are the worst by an order of magnitude
    assert min(e[1:4]) > 5 * max(e[0], e[4])


def test_rk_increment_floor():
    """Two RK steps at 4^3 k=3 n_q=6: the oracle's increment against extended-precision
    steps is within 1.2 times (L floor + 10 u |U| / |dU|), the bound the GPU RK test uses."""
    oop = ooperator.DGOperator(omesh.BoxMesh((4, 4, 4), *PI3, 3), tgv_fluid(), 6)
    U0 = tgv_input(oop, seed=9)
    ext = floor.extended_for(oop)
    cells = list(range(64))
    dt = timeint.time_step(0.3, 0.02, 1.5, 3.0, 3, oop.mesh.h_min(), 1.0, 0.1, oop.fl.nu)
    A = [LD(f.numerator) / LD(f.denominator) for f in timeint.CK54_A]
    B = [LD(f.numerator) / LD(f.denominator) for f in timeint.CK54_B]
    Ux = U0.numpy().astype(LD)
    for s in range(2):
        for i in range(5):
            R = np.stack([ext.residual_cell(Ux, e) for e in cells], axis=1)
            L = np.stack([ext.inverse_mass(e, R[:, e]) for e in cells], axis=1)
            dU = LD(dt) * L if i == 0 else A[i] * dU + LD(dt) * L
            Ux = Ux + B[i] * dU
    U = U0.clone()
    for s in range(2):
        U = timeint.lsrk_step(lambda V, t: oop.apply(V), U, s * dt, dt)
    inc_ext = Ux - U0.numpy().astype(LD)
    e_inc = floor.errs(U - U0, inc_ext)
    e_L = floor.oracle_floor(oop, U0)
    st = [10 * 2.0 ** -53 * float(np.linalg.norm(U0.numpy()[c]) / np.linalg.norm(inc_ext[c].astype(np.float64)))
          for c in range(5)]
    print("increment floor", e_inc, "L floor", e_L, "state rounding", st)
    for c in range(5):
        assert e_inc[c] <= 1.2 * (e_L[c] + st[c]), (c, e_inc, e_L, st)
