"""GPU parity of the high-degree kernels (k = 8..15: hd_impl.h, the cell streamed through
LDS plane by plane, faces once per face, stand-alone inverse mass) against the oracle.

Every compiled (k, n_q) -- n_q = k+1 for k = 8..15 and the 3/2 rule for k = 8..10 -- on a
two-cell periodic mesh, affine and curved in turn, LGL and Gauss nodes in turn:
  - float64 R and L at Mach 0.3 (Taylor-Green plus noise) against the oracle with the
    floor rule of tests/floor.py, the extended-precision reference on one cell, for
    k = 8, 9 at n_q = k+1 (its dense evaluation takes 14 s per cell at k = 9, 40 s at 10);
  - otherwise per field |gpu - oracle| <= 1e-12 ((k+1)/4)^4 for R and the same times
    10 for L: the measured floors grow like the square of the 1D derivative matrices'
    norms, ((k+1)/4)^2 -- at k = 8: 3e-13 (R) and 1.2e-11 (L) -- and the bound leaves
    another factor ((k+1)/4)^2 (5 at k = 8, 16 at k = 15);
  - the stand-alone inverse mass (backward error through the oracle's mass matrix);
  - float32 R and L per field within 50 times what rounding the input alone to float32
    costs, and the stand-alone inverse mass by its backward error (the float64 bound times
    2^29, the ratio of the unit roundoffs).
Also: two Runge-Kutta steps at k = 8 (stages 1-4 through the high-degree stage path,
which writes L into the next-state buffer and updates from there) against the oracle's
steps, the initial-state projection at k = 8, both again at k = 12 and 15 on a curved
mesh under the per-field float64 bound, the wall branches on a channel with isothermal
no-slip walls at k = 8, 13 and 15, the diagnostics at k = 8, 12 and 15 against the oracle's,
and the entry points without high-degree kernels (adjoint) and body forces rejected with
DGNS_EUNSUPPORTED.
"""
import math

import numpy as np
import pytest
import torch

from oracle import diagnostics as odiag, initial, timeint
from tests import floor
from tests.gpu_cases import announce, channel_input, make_pair, rel_err_fields, tgv_fluid, tgv_input

pytestmark = pytest.mark.gpu

HD = [(8, 9), (8, 13), (9, 10), (9, 14), (10, 11), (10, 16), (11, 12), (12, 13), (13, 14), (14, 15), (15, 16)]


def _cuda(t):
    return t.to("cuda").contiguous()


def _projection_errors(Ug, Uo):
    """Per-field relative error of a projected state; a field that is identically zero in the
    oracle (rho w of the Taylor-Green state) must be exactly zero on the GPU too."""
    errs = []
    for c in range(5):
        if float(torch.linalg.norm(Uo[c])) == 0.0:
            assert float(torch.linalg.norm(Ug[c])) == 0.0, c
            errs.append(0.0)
        else:
            errs.append(float(torch.linalg.norm(Ug[c] - Uo[c]) / torch.linalg.norm(Uo[c])))
    return errs


def _case(i):
    n = [(2, 1, 1), (1, 2, 1)][i % 2]
    kind, amp = ("curved", 0.1) if i % 2 else ("affine", 0.0)
    basis = "GL" if i % 3 == 2 else "LGL"
    return n, kind, amp, basis


@pytest.mark.parametrize("kq", HD)
def test_high_degree_float64(kq):
    k, nq = kq
    i = HD.index(kq)
    n, kind, amp, basis = _case(i)
    announce("high degree fp64 n=%s k=%d nq=%d %s %s" % (n, k, nq, kind, basis))
    oop, gop = make_pair(n, k, nq, kind=kind, amp=amp, basis=basis)
    U = tgv_input(oop, seed=40 + i, mach=0.3)
    R_gpu = gop.residual(_cuda(U)).cpu()
    L_gpu = gop.apply(_cuda(U)).cpu()
    torch.cuda.synchronize()
    R_ora, L_ora = oop.residual(U), oop.apply(U)
    if nq == k + 1 and k <= 9:
        R_ext, L_ext = floor.reference_RL(oop, U, [0])
        floor.check(R_gpu, R_ora, R_ext, "R k=%d" % k, sub=[0])
        floor.check(L_gpu, L_ora, L_ext, "L k=%d" % k, sub=[0])
    else:
        tol = 1e-12 * ((k + 1) / 4.0) ** 4
        eR = rel_err_fields(R_gpu, R_ora)
        eL = rel_err_fields(L_gpu, L_ora)
        print("k=%d: R vs oracle %s, L vs oracle %s (bounds %.1e, %.1e)"
              % (k, ["%.1e" % e for e in eR], ["%.1e" % e for e in eL], tol, 10 * tol), flush=True)
        assert max(eR) <= tol, eR
        assert max(eL) <= 10 * tol, eL
    # stand-alone inverse mass: backward error through the oracle's mass matrix
    X = gop.inverse_mass(_cuda(U)).cpu()
    torch.cuda.synchronize()
    M = oop.mass_matrices()
    MX = torch.einsum("eij,cej->cei", M, X)
    err = float(torch.linalg.norm(MX - U) / torch.linalg.norm(U))
    assert err < 1e-13 * ((k + 1) / 4.0) ** 2, err


@pytest.mark.parametrize("kq", HD)
def test_high_degree_float32(kq):
    k, nq = kq
    i = HD.index(kq)
    n, kind, amp, basis = _case(i + 1)
    announce("high degree fp32 n=%s k=%d nq=%d %s %s" % (n, k, nq, kind, basis))
    oop, gop = make_pair(n, k, nq, kind=kind, amp=amp, basis=basis, precision="fp32")
    U = tgv_input(oop, seed=60 + i, mach=0.3)
    U32 = U.float().double()
    R32 = gop.residual(_cuda(U)).cpu()
    L32 = gop.apply(_cuda(U)).cpu()
    X32 = gop.inverse_mass(_cuda(U)).cpu()
    torch.cuda.synchronize()
    # R and L per field within 50 times what rounding the input alone to float32 costs in the
    # oracle
    for name, got, f in (("R", R32, oop.residual), ("L", L32, oop.apply)):
        ref = f(U)
        cast = rel_err_fields(f(U32), ref)
        errs = rel_err_fields(got, ref)
        print("fp32 k=%d %s per field %s; input-rounding floor %s" % (k, name, ["%.1e" % e for e in errs],
                                                                     ["%.1e" % e for e in cast]), flush=True)
        for c in range(5):
            assert errs[c] <= max(50 * cast[c], 1e-6), (name, c, errs, cast)
    # the stand-alone inverse mass of the streamed path (the register form at N <= 11, one
    # output at a time from LDS above): backward error through the oracle's mass matrix within
    # the float64 bound times the ratio of the unit roundoffs, 2^29
    M = oop.mass_matrices()
    MX = torch.einsum("eij,cej->cei", M, X32)
    err = float(torch.linalg.norm(MX - U) / torch.linalg.norm(U))
    print("fp32 k=%d M^-1 backward error %.1e" % (k, err), flush=True)
    assert err < 1e-13 * 2.0 ** 29 * ((k + 1) / 4.0) ** 2, err


def test_high_degree_rk_steps_and_projection():
    announce("high degree k=8 nq=9: projection and two RK steps")
    oop, gop = make_pair((2, 1, 1), 8, 9)
    Ug = gop.project_ic("taylor_green", [1.0, 1.0, 0.3, 1.0])
    torch.cuda.synchronize()
    Uo = initial.l2_project(oop, lambda x: initial.taylor_green(x, oop.fl, mach=0.3))
    errs = _projection_errors(Ug.cpu(), Uo)
    print("projection vs oracle", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < 1e-12, errs
    U0 = tgv_input(oop, seed=77, mach=0.3)
    dt = gop.compute_dt(0.2, 0.02, 1.5, 3.0, 1.0, 0.3)
    Ug = _cuda(U0.clone())
    work = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    for s in range(2):
        gop.rk_step(Ug, work, s * dt, dt)
    torch.cuda.synchronize()
    U = U0.clone()
    for s in range(2):
        U = timeint.lsrk_step(lambda V, t: oop.apply(V), U, s * dt, dt)
    e_L = floor.oracle_floor(oop, U0, cells=[0])
    inc = rel_err_fields(Ug.cpu() - U0, U - U0)
    print("two RK steps: increment vs oracle %s, oracle L floor %s" % (["%.1e" % e for e in inc],
                                                                       ["%.1e" % e for e in e_L]), flush=True)
    st = [20 * 2.0 ** -53 * float(torch.linalg.norm(U0[c]) / torch.linalg.norm((U - U0)[c])) for c in range(5)]
    for c in range(5):
        assert inc[c] <= max(1e-12, 4.0 * (e_L[c] + st[c])), (c, inc, e_L, st)


@pytest.mark.parametrize("kq", [(12, 13), (15, 16)])
def test_high_degree_rk_steps_and_projection_large_k(kq):
    # the stage path of the streamed kernels (L into the next-state buffer, the residual
    # through the cell's scratch, M^{-1} in place, the update from there) at degrees whose
    # extended-precision floor is too slow to evaluate: the increment of two RK steps per
    # field within 10 times the float64 bound of L above, 1e-11 ((k+1)/4)^4 relative; the
    # projection within 1e-12 ((k+1)/4)^2
    k, nq = kq
    announce("high degree k=%d nq=%d: projection and two RK steps" % (k, nq))
    oop, gop = make_pair((2, 1, 1), k, nq, kind="curved", amp=0.1)
    Ug = gop.project_ic("taylor_green", [1.0, 1.0, 0.3, 1.0])
    torch.cuda.synchronize()
    Uo = initial.l2_project(oop, lambda x: initial.taylor_green(x, oop.fl, mach=0.3))
    errs = _projection_errors(Ug.cpu(), Uo)
    print("projection vs oracle", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < 1e-12 * ((k + 1) / 4.0) ** 2, errs
    U0 = tgv_input(oop, seed=78, mach=0.3)
    dt = gop.compute_dt(0.2, 0.02, 1.5, 3.0, 1.0, 0.3)
    Ug = _cuda(U0.clone())
    work = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    for s in range(2):
        gop.rk_step(Ug, work, s * dt, dt)
    torch.cuda.synchronize()
    U = U0.clone()
    for s in range(2):
        U = timeint.lsrk_step(lambda V, t: oop.apply(V), U, s * dt, dt)
    inc = rel_err_fields(Ug.cpu() - U0, U - U0)
    tol = 10 * 1e-12 * ((k + 1) / 4.0) ** 4
    print("two RK steps: increment vs oracle %s (bound %.1e)" % (["%.1e" % e for e in inc], tol), flush=True)
    assert max(inc) <= tol, inc


@pytest.mark.parametrize("kq", [(8, 9), (13, 14), (15, 16)])
def test_high_degree_channel_walls(kq):
    # the streamed kernels' wall branches (the face kernel's own-side-only lower wall faces and
    # upper faces without an exterior side, in its 128- and 256-thread forms) on a 1x2x1
    # stretched channel with isothermal no-slip walls at both ends of x2, no body force: float64
    # R and L at k = 8 under the floor rule against the extended evaluation, above per field
    # within 1e-12 ((k+1)/4)^4 (L: 10 times) of the oracle; float32 R and L within 50 times the
    # input-rounding floor
    k, nq = kq
    announce("high degree channel 1x2x1 k=%d nq=%d walls" % (k, nq))
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (1.4 * 287.0)
    geo = dict(lo=(0, -1, 0), hi=(2 * math.pi, 1, math.pi), periodic=(1, 0, 1), kind="channel", fluid=fl,
               wall_T=T0)
    oop, gop = make_pair((1, 2, 1), k, nq, **geo)
    U = channel_input(oop)
    R_gpu = gop.residual(_cuda(U)).cpu()
    L_gpu = gop.apply(_cuda(U)).cpu()
    torch.cuda.synchronize()
    R_ora, L_ora = oop.residual(U), oop.apply(U)
    if k == 8:
        R_ext, L_ext = floor.reference_RL(oop, U, [0, 1])
        floor.check(R_gpu, R_ora, R_ext, "R channel k=8")
        floor.check(L_gpu, L_ora, L_ext, "L channel k=8")
    else:
        tol = 1e-12 * ((k + 1) / 4.0) ** 4
        eR, eL = rel_err_fields(R_gpu, R_ora), rel_err_fields(L_gpu, L_ora)
        print("channel k=%d: R vs oracle %s, L vs oracle %s (bounds %.1e, %.1e)"
              % (k, ["%.1e" % e for e in eR], ["%.1e" % e for e in eL], tol, 10 * tol), flush=True)
        assert max(eR) <= tol, eR
        assert max(eL) <= 10 * tol, eL
    _, g32 = make_pair((1, 2, 1), k, nq, precision="fp32", **geo)
    U32 = U.float().double()
    for name, got, f in (("R", g32.residual(_cuda(U)).cpu(), oop.residual), ("L", g32.apply(_cuda(U)).cpu(), oop.apply)):
        ref = f(U)
        cast = rel_err_fields(f(U32), ref)
        errs = rel_err_fields(got, ref)
        print("channel fp32 k=%d %s per field %s; input-rounding floor %s"
              % (k, name, ["%.1e" % e for e in errs], ["%.1e" % e for e in cast]), flush=True)
        for c in range(5):
            assert errs[c] <= max(50 * cast[c], 1e-6), (name, c, errs, cast)


@pytest.mark.parametrize("kq", [(8, 9), (12, 13), (15, 16)])
def test_high_degree_diagnostics(kq):
    # the streamed diagnostics (one quadrature plane at a time, the conserved totals one plane
    # of mass points at a time) against the oracle's on the same U and L: e_k, eps, mass and
    # energy to 1e-13 relative, -de_k/dt to 1e-12, the momentum totals (sums that cancel) to
    # 1e-13 of the mass; affine at k = 8, 15, curved at k = 12
    k, nq = kq
    curved = k == 12
    announce("high degree diagnostics k=%d nq=%d %s" % (k, nq, "curved" if curved else "affine"))
    oop, gop = make_pair((2, 1, 1), k, nq, kind="curved" if curved else "affine", amp=0.1 if curved else 0.0)
    U = tgv_input(oop, seed=90 + k, mach=0.1)
    L = oop.apply(U)
    dg = gop.diagnostics(_cuda(U), _cuda(L))
    torch.cuda.synchronize()
    do = odiag.diagnostics(oop, U, L)
    print("k=%d diagnostics:" % k, {key: "%.2e" % (abs(dg[key] - do[key]) / abs(do[key]))
                                    for key in ("e_k", "eps", "rate", "mass", "energy")}, flush=True)
    for key in ("e_k", "eps", "mass", "energy"):
        assert abs(dg[key] - do[key]) <= 1e-13 * abs(do[key]), (key, dg[key], do[key])
    assert abs(dg["rate"] - do["rate"]) <= 1e-12 * abs(do["rate"]), (dg["rate"], do["rate"])
    assert np.allclose(dg["mom"], do["mom"], rtol=0.0, atol=1e-13 * abs(do["mass"])), (dg["mom"], do["mom"])


def test_high_degree_unsupported_entry_points():
    from paper_1806_03095_amd import binding
    oop, gop = make_pair((2, 1, 1), 8, 9)
    U = _cuda(tgv_input(oop, seed=5, mach=0.3))
    with pytest.raises(RuntimeError, match="degree|unsupported|kernel"):
        gop.residual_vjp(U, torch.ones_like(U))
    with pytest.raises(RuntimeError, match="body force"):
        make_pair((2, 1, 1), 8, 9, force=(1.0, 0.0, 0.0))
    assert binding is not None
