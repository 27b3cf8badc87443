"""GPU parity of the HIP operator against the oracle (float64).

Inputs are the oracle's L2-projected states plus seeded noise; both sides get the
same array.  Every float64 comparison follows the rule of tests/floor.py: the oracle's
own rounding error is measured against an extended-precision evaluation of the same
operator on the same input, the HIP result must be at least half as accurate as the
oracle (|gpu - ext| <= 2 |oracle - ext|), and it must match the oracle to 1e-12 per
field or, where the oracle's own measured error does not allow that (low Mach number,
fine meshes), to three times that error.  Covered: the Taylor-Green configuration of
4^3 cells, k=3, n_q=6 (LGL and GL bases), a range of (k, n_q) on ragged meshes, curved
meshes (per quadrature-point metric), the stretched channel with walls and body force,
each term separately, the inverse mass matrix, Runge-Kutta steps, diagnostics, the
initial-state projection, and run-to-run bitwise determinism.
"""
import math

import numpy as np
import pytest
import torch

from oracle import diagnostics as odiag, initial, timeint
from tests import floor
from tests.gpu_cases import announce, make_pair, tgv_input, channel_input, rel_err_fields, tgv_fluid

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _cuda(t):
    return t.to("cuda").contiguous()


def _check_fields(got, want, tol, what):
    errs = rel_err_fields(got, want)
    assert max(errs) < tol, (what, errs)
    return errs


def _floor_L_and_R(oop, U, L_gpu, R_gpu, what, sub_max=None):
    """L and R of the whole mesh against the oracle with the floor rule; the extended
    reference is evaluated on the first sub_max cells (all if None)."""
    E = oop.mesh.n_cells
    sub = list(range(E if sub_max is None else min(E, sub_max)))
    R_ext, L_ext = floor.reference_RL(oop, U, sub)
    floor.check(R_gpu, oop.residual(U), R_ext, "R " + what, sub=sub)
    floor.check(L_gpu, oop.apply(U), L_ext, "L " + what, sub=sub)


@pytest.mark.parametrize("basis", ["LGL", "GL"])
def test_tgv_4cubed_k3_nq6_operator(basis):
    announce("tgv 4^3 k=3 nq=6 %s apply_operator" % basis)
    oop, gop = make_pair((4, 4, 4), 3, 6, basis=basis)
    U = tgv_input(oop)
    L_gpu = gop.apply(_cuda(U))
    R_gpu = gop.residual(_cuda(U))
    torch.cuda.synchronize()
    _floor_L_and_R(oop, U, L_gpu, R_gpu, "tgv 4^3 k=3 nq=6 %s" % basis)


@pytest.mark.parametrize("terms,mask", [("c", 1), ("v", 2), ("cv", 3)])
def test_tgv_residual_terms(terms, mask):
    announce("tgv 4^3 k=3 nq=6 residual terms=%s" % terms)
    oop, gop = make_pair((4, 4, 4), 3, 6)
    U = tgv_input(oop, seed=5)
    R_gpu = gop.residual(_cuda(U), terms=mask)
    torch.cuda.synchronize()
    cells = list(range(oop.mesh.n_cells))
    ref = floor.reference(oop, U, cells, "R", terms)
    floor.check(R_gpu, oop.residual(U, terms=terms), ref, "R_" + terms)


CASES = [
    # n, k, nq, kind, amp, basis
    ((3, 2, 2), 1, 2, "affine", 0.0, "LGL"),
    ((3, 2, 2), 1, 3, "affine", 0.0, "GL"),
    ((2, 3, 2), 2, 3, "affine", 0.0, "LGL"),
    ((2, 2, 3), 2, 4, "curved", 0.1, "LGL"),
    ((3, 3, 2), 3, 4, "affine", 0.0, "LGL"),
    ((2, 3, 3), 3, 5, "curved", 0.15, "GL"),
    ((2, 2, 2), 4, 7, "affine", 0.0, "LGL"),
    ((2, 2, 2), 4, 6, "curved", 0.1, "LGL"),
    ((2, 3, 1), 4, 5, "affine", 0.0, "GL"),
    ((2, 2, 2), 5, 8, "affine", 0.0, "LGL"),
    ((2, 1, 2), 7, 11, "affine", 0.0, "LGL"),
    ((1, 2, 2), 7, 11, "curved", 0.1, "LGL"),
    # n_q = 2k+1
    ((2, 2, 2), 2, 5, "curved", 0.1, "LGL"),
    ((2, 2, 1), 3, 7, "affine", 0.0, "GL"),
    ((2, 1, 1), 4, 9, "curved", 0.1, "LGL"),
    # the remaining compiled (k, n_q) pairs
    ((2, 2, 2), 5, 6, "curved", 0.1, "LGL"),
    ((2, 1, 2), 6, 7, "affine", 0.0, "GL"),
    ((1, 2, 2), 7, 8, "curved", 0.1, "LGL"),
    # degenerate meshes: one cell per direction is its own periodic neighbour
    ((1, 1, 1), 2, 4, "affine", 0.0, "LGL"),
    ((1, 1, 1), 3, 6, "curved", 0.1, "GL"),
    ((1, 1, 3), 1, 2, "affine", 0.0, "LGL"),
    ((3, 1, 1), 6, 10, "affine", 0.0, "LGL"),
]


@pytest.mark.parametrize("case", CASES)
def test_operator_parity_range(case):
    n, k, nq, kind, amp, basis = case
    announce("parity n=%s k=%d nq=%d kind=%s amp=%g basis=%s" % (n, k, nq, kind, amp, basis))
    oop, gop = make_pair(n, k, nq, kind=kind, amp=amp, basis=basis)
    U = tgv_input(oop, seed=11 + k, mach=0.3)
    L_gpu = gop.apply(_cuda(U))
    R_gpu = gop.residual(_cuda(U))
    torch.cuda.synchronize()
    _floor_L_and_R(oop, U, L_gpu, R_gpu, "n=%s k=%d nq=%d %s" % (n, k, nq, kind), sub_max=4 if k >= 6 else None)


@pytest.mark.parametrize("k,nq", [(4, 7), (3, 5), (4, 5), (2, 3)])
def test_channel_walls_force(k, nq):
    # the workload's k=4, n_q=7, and kernels with fused face traces (k <= 3) and
    # one-wave workgroups (n_q <= 4): walls at both ends of x2 and the body force
    announce("channel 2x4x2 k=%d nq=%d walls+force" % (k, nq))
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (1.4 * 287.0)
    oop, gop = make_pair((2, 4, 2), k, nq, lo=(0, -1, 0), hi=(2 * math.pi, 1, math.pi), periodic=(1, 0, 1),
                         kind="channel", fluid=fl, force=(1.0, 0.0, 0.0), wall_T=T0)
    U = channel_input(oop)
    cells = list(range(oop.mesh.n_cells))
    ext = floor.extended_for(oop)
    for mask, terms in ((1, "c"), (2, "v"), (4, "f"), (7, "cvf")):
        R_gpu = gop.residual(_cuda(U), terms=mask)
        torch.cuda.synchronize()
        R_ora = oop.residual(U, terms=terms)
        ref = ext.residual(U.numpy(), cells, terms)
        if terms == "f":   # the body force has no mass row
            assert float(R_gpu[0].abs().max()) == 0.0
            floor.check(R_gpu, R_ora, ref, "R_f", fields=(1, 4))   # f = (1, 0, 0)
        else:
            floor.check(R_gpu, R_ora, ref, "R_" + terms)
    L_gpu = gop.apply(_cuda(U))
    torch.cuda.synchronize()
    L_ext = np.stack([ext.inverse_mass(e, ref[:, e]) for e in cells], axis=1)
    floor.check(L_gpu, oop.apply(U), L_ext, "L channel")


def test_inverse_mass_in_place_and_curved():
    announce("inverse mass 2x2x3 k=3 curved, in place")
    oop, gop = make_pair((2, 2, 3), 3, 5, kind="curved", amp=0.2)
    R = torch.as_tensor(np.random.default_rng(3).standard_normal((5, oop.mesh.n_cells, oop.N)))
    Rg = _cuda(R)
    out = gop.inverse_mass(Rg)
    gop.inverse_mass(Rg, out=Rg)          # in place
    torch.cuda.synchronize()
    cells = list(range(oop.mesh.n_cells))
    ref = floor.reference_minv(oop, R, cells)
    ora = oop.apply_inverse_mass(R)
    floor.check(out, ora, ref, "M^-1 R")
    floor.check(Rg, ora, ref, "M^-1 R in place")


def test_rk_steps_tgv_4cubed():
    announce("tgv 4^3 k=3 nq=6: 10 RK steps")
    oop, gop = make_pair((4, 4, 4), 3, 6)
    U0 = tgv_input(oop, seed=9)
    dt = gop.compute_dt(0.3, 0.02, 1.5, 3.0, 1.0, 0.1)
    assert abs(dt - timeint.time_step(0.3, 0.02, 1.5, 3.0, 3, oop.mesh.h_min(), 1.0, 0.1, oop.fl.nu)) < 1e-15
    Ug = _cuda(U0.clone())
    work = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    for s in range(10):
        gop.rk_step(Ug, work, s * dt, dt)
    torch.cuda.synchronize()
    U = U0.clone()
    for s in range(10):
        U = timeint.lsrk_step(lambda V, t: oop.apply(V), U, s * dt, dt)
    inc_gpu = Ug.cpu() - U0
    inc_ora = U - U0
    # Floor of the increment: the oracle's single-evaluation floor of L (measured here on
    # the initial state against the extended evaluation) plus the rounding of the fifty
    # state updates U <- U + B dU, at most 50 u |U| against |U10 - U0| (u = 2^-53).  On
    # the CPU (tests/test_float64_floor.py) the oracle's increment after two steps is
    # within 1.2 times this sum of the extended-precision steps.
    e_L = floor.oracle_floor(oop, U0)
    st = [50 * 2.0 ** -53 * float(torch.linalg.norm(U0[c]) / torch.linalg.norm(inc_ora[c])) for c in range(5)]
    errs = rel_err_fields(inc_gpu, inc_ora)
    print("U10 - U0: gpu vs oracle %s, oracle L floor %s, state rounding %s" % (errs, e_L, st), flush=True)
    for c in range(5):
        assert errs[c] <= max(TOL, 4.0 * (e_L[c] + st[c])), (c, errs, e_L, st)


@pytest.mark.parametrize("case", ["channel_k4_fp64", "curved_k3_fp32", "tgv_k2_fp64"])
def test_rk_step_fused_stages_match_stage_by_stage(case):
    """rk_step fuses the update of stages 1-4 into the operator kernel; the same two
    steps taken stage by stage (L from the operator, the update in torch with the
    scheme's coefficients) must agree to rounding."""
    announce("rk_step fused stages vs stage by stage: " + case)
    if case == "channel_k4_fp64":
        fl = tgv_fluid(mu=1.0 / 180.0)
        T0 = (18.3 / 0.1) ** 2 / (fl.gamma * fl.R)
        oop, gop = make_pair((2, 4, 2), 4, 7, lo=(0.0, -1.0, 0.0), hi=(2 * math.pi, 1.0, math.pi),
                             periodic=(1, 0, 1), kind="channel", fluid=fl, force=(1.0, 0.0, 0.0), wall_T=T0)
        U0 = channel_input(oop)
        umax = 18.3
    elif case == "curved_k3_fp32":
        oop, gop = make_pair((3, 3, 3), 3, 6, kind="curved", amp=0.1, precision="fp32")
        U0 = tgv_input(oop, seed=5)
        umax = 1.0
    else:
        oop, gop = make_pair((3, 2, 2), 2, 4)
        U0 = tgv_input(oop, seed=6)
        umax = 1.0
    dt = gop.compute_dt(0.3, 0.02, 1.5, 3.0, umax, 0.1)
    Ug = _cuda(U0.clone())
    work = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    for s in range(2):
        gop.rk_step(Ug, work, s * dt, dt)
    U = _cuda(U0.clone())
    dU = torch.zeros_like(U)
    A = [float(v) for v in timeint.CK54_A]
    B = [float(v) for v in timeint.CK54_B]
    for s in range(2):
        for i in range(5):
            L = gop.apply(U)
            dU = dt * L if i == 0 else A[i] * dU + dt * L
            U = U + B[i] * dU
    torch.cuda.synchronize()
    inc = (U - _cuda(U0)).abs().amax(dim=(1, 2))
    diff = (Ug - U).abs().amax(dim=(1, 2))
    rel = [float(d / max(i, 1e-300)) for d, i in zip(diff, inc)]
    print("fused vs stage-by-stage, max difference relative to the increment per field:", rel, flush=True)
    assert max(rel) < 1e-12, rel


def test_rk_step_hip_graph_replays():
    """One rk_step captured in a HIP graph and replayed three times, with eager work
    on the same state between the replays, against three eager steps (bitwise)."""
    announce("rk_step captured in a HIP graph: three replays vs eager steps")
    oop, gop = make_pair((4, 4, 4), 3, 6)
    U0 = tgv_input(oop, seed=21)
    dt = gop.compute_dt(0.3, 0.02, 1.5, 3.0, 1.0, 0.1)
    Ue = _cuda(U0.clone())
    we = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    ref = []
    for s in range(3):
        gop.rk_step(Ue, we, s * dt, dt)
        ref.append(Ue.clone())
    Ug = _cuda(U0.clone())
    wg = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    graph = gop.rk_graph(Ug, wg, dt, steps=1)
    for s in range(3):
        graph.replay()
        torch.cuda.synchronize()
        L = gop.apply(Ug)            # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(L).all()
        assert torch.equal(Ug, ref[s]), s


def test_rk_stage_update_alone():
    announce("rk_stage_update: stages 0 and 3 against the scheme's coefficients; argument checks")
    from paper_1806_03095_amd.binding import DgnsError
    oop, gop = make_pair((3, 2, 1), 2, 3)
    g = torch.Generator().manual_seed(3)
    U0, dU0, L = (torch.randn(gop.shape, generator=g, dtype=torch.float64) for _ in range(3))
    A = [float(v) for v in timeint.CK54_A]
    B = [float(v) for v in timeint.CK54_B]
    dt = 0.37
    for stage in (0, 3):
        U, dU = _cuda(U0.clone()), _cuda(dU0.clone())
        if stage == 0:
            dU.fill_(float("nan"))   # the first stage must not read dU
        gop.rk_stage_update(U, dU, _cuda(L), stage, dt)
        torch.cuda.synchronize()
        d = dt * L if stage == 0 else A[stage] * dU0 + dt * L
        assert torch.allclose(dU.cpu(), d, rtol=1e-15, atol=1e-15)
        assert torch.allclose(U.cpu(), U0 + B[stage] * d, rtol=1e-15, atol=1e-15)
    U, dU = _cuda(U0.clone()), _cuda(dU0.clone())
    with pytest.raises(DgnsError):
        gop.rk_stage_update(U, dU, _cuda(L), 5, dt)
    with pytest.raises(DgnsError):
        gop.rk_stage_update(U, U, _cuda(L), 1, dt)


@pytest.mark.parametrize("case", ["channel_k4", "tgv_k3"])
def test_channel_statistics(case):
    announce("channel statistics (plane averages) vs oracle: " + case)
    if case == "channel_k4":
        fl = tgv_fluid(mu=1.0 / 180.0)
        T0 = (18.3 / 0.1) ** 2 / (fl.gamma * fl.R)
        oop, gop = make_pair((2, 4, 2), 4, 7, lo=(0.0, -1.0, 0.0), hi=(2 * math.pi, 1.0, math.pi),
                             periodic=(1, 0, 1), kind="channel", fluid=fl, force=(1.0, 0.0, 0.0), wall_T=T0)
        U = channel_input(oop)
    else:
        oop, gop = make_pair((3, 2, 2), 3, 6)
        U = tgv_input(oop, seed=8)
    got = gop.channel_statistics(_cuda(U))
    want = odiag.channel_statistics(oop, U)
    assert got.shape == want.shape
    # Averages of sign-changing quantities (the Taylor-Green <u>, <uv> over a period)
    # cancel to far below their summands, so each column's error is measured against
    # the size of its summands: |y|, rho, |u| <= sqrt(max <uu>), |uv| <= max <uu>.
    q2 = np.abs(want[:, 5:8]).max()
    scale = [np.abs(want[:, 0]).max(), np.abs(want[:, 1]).max()] + [np.sqrt(q2)] * 3 + [q2] * 4
    for m in range(9):
        err = np.abs(got[:, m] - want[:, m]).max() / scale[m]
        assert err < 1e-12, (m, err)


def test_channel_statistics_rejects_curved_mesh():
    from paper_1806_03095_amd.binding import DgnsError
    oop, gop = make_pair((2, 2, 2), 2, 3, kind="curved", amp=0.1)
    with pytest.raises(DgnsError):
        gop.channel_statistics(_cuda(tgv_input(oop)))


def test_diagnostics_and_projection():
    announce("tgv 4^3 k=3 nq=6: diagnostics and IC projection")
    oop, gop = make_pair((4, 4, 4), 3, 6)
    Ug = gop.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
    torch.cuda.synchronize()
    Uo = initial.l2_project(oop, lambda x: initial.taylor_green(x, oop.fl))
    _check_fields(Ug, Uo, TOL, "IC")
    U = tgv_input(oop, seed=4)
    Lg = gop.apply(_cuda(U))
    dg = gop.diagnostics(_cuda(U), Lg)
    do = odiag.diagnostics(oop, U, oop.apply(U))
    for key in ("e_k", "eps", "mass", "energy"):
        assert abs(dg[key] - do[key]) <= 1e-12 * abs(do[key]), (key, dg[key], do[key])
    # -de_k/dt is a functional of L: its floor is the oracle's rate from its own L against
    # the rate from the extended-precision L
    _, L_ext = floor.reference_RL(oop, U, list(range(oop.mesh.n_cells)))
    r_ext = odiag.diagnostics(oop, U, torch.as_tensor(L_ext.astype(np.float64)))["rate"]
    e_rate = abs(do["rate"] - r_ext) / abs(r_ext)
    print("rate: gpu vs oracle %.2e, oracle floor %.2e" % (abs(dg["rate"] - do["rate"]) / abs(do["rate"]), e_rate))
    assert abs(dg["rate"] - do["rate"]) <= max(TOL, 3.0 * e_rate) * abs(do["rate"]), (dg["rate"], do["rate"])
    assert np.allclose(dg["mom"], do["mom"], rtol=1e-10, atol=1e-12 * abs(do["mass"]))


def test_determinism_bitwise():
    announce("tgv 4^3 k=3 nq=6: bitwise determinism")
    oop, gop = make_pair((4, 4, 4), 3, 6)
    U = _cuda(tgv_input(oop, seed=1))
    a = gop.apply(U)
    b = gop.apply(U)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# every compiled (k, n_q): (n, kind) alternate between ragged affine and curved meshes
FP32_CASES = [(1, 2), (1, 3), (2, 3), (2, 4), (2, 5), (3, 4), (3, 5), (3, 6), (3, 7), (4, 5), (4, 6), (4, 7),
              (4, 9), (5, 6), (5, 8), (6, 7), (6, 10), (7, 8), (7, 11)]


def _cast_floor(oop, U, cells=None):
    """Per-field relative change of the float64 oracle's L when only its input is rounded to
    float32: the error that representing the state in float32 costs before any arithmetic
    (the operator's conditioning at low Mach number amplifies it; see test below)."""
    L = oop.apply(U, cells=cells)
    Lc = oop.apply(U.float().double(), cells=cells)
    return rel_err_fields(Lc, L), L


@pytest.mark.parametrize("kq", FP32_CASES)
def test_fp32_every_kernel(kq):
    # Bug detection for every float32 instantiation: a seeded Mach 0.3 state on a small
    # mesh, per-field error against the float64 oracle.  A wrong table, index or branch
    # gives O(1); float32 rounding gives 1e-6..1e-4 here (measured in the CPU emulation:
    # at most 4.5e-4), at most 50 times what rounding the input alone costs.
    k, nq = kq
    i = FP32_CASES.index(kq)
    n = [(3, 2, 2), (2, 2, 3), (2, 3, 1)][i % 3] if k <= 4 else [(2, 1, 2), (1, 2, 2)][i % 2]
    kind, amp = ("curved", 0.1) if i % 2 else ("affine", 0.0)
    announce("fp32 n=%s k=%d nq=%d %s" % (n, k, nq, kind))
    oop, gop = make_pair(n, k, nq, kind=kind, amp=amp, precision="fp32")
    U = tgv_input(oop, seed=2 + i, mach=0.3)
    L32 = gop.apply(_cuda(U))
    torch.cuda.synchronize()
    cast, L64 = _cast_floor(oop, U)
    errs = rel_err_fields(L32, L64)
    print("fp32 per field %s; input-rounding floor %s" % (["%.1e" % e for e in errs], ["%.1e" % e for e in cast]),
          flush=True)
    assert max(errs) < 1e-3, errs
    for c in range(5):
        assert errs[c] <= max(50 * cast[c], 1e-6), (c, errs, cast)


def test_fp32_smooth_taylor_green_error_is_rounding():
    # The smooth Taylor-Green state at Mach 0.1 (no noise), 4^3 cells k=3 n_q=6: per-field
    # error of the float32 operator against the float64 oracle.  Measured in the CPU
    # emulation of this kernel: 1.1e-4 (rho), 1.2e-3 (momentum), 1.4e-4 (rho E), 15 to 25
    # times the change of the float64 L when only its input is rounded to float32.  The
    # cause is the conditioning of L at low Mach number: a perturbation of relative size
    # 6e-8 of the state (|rho E| = 179, p0 = 71) reaches L amplified by about
    # (|u| + c) (k+1)^2 / h * |U| / |L|, against rates of order 1 (rho: div m ~ 0).
    announce("fp32 smooth tgv 4^3 k=3 nq=6 Mach 0.1")
    oop, gop = make_pair((4, 4, 4), 3, 6, precision="fp32")
    U = initial.l2_project(oop, lambda x: initial.taylor_green(x, oop.fl))
    L32 = gop.apply(_cuda(U))
    torch.cuda.synchronize()
    cast, L64 = _cast_floor(oop, U)
    errs = rel_err_fields(L32, L64)
    print("fp32 smooth tgv per field %s; input-rounding floor %s" % (["%.2e" % e for e in errs],
                                                                     ["%.2e" % e for e in cast]), flush=True)
    for c in range(5):
        assert errs[c] <= 50 * cast[c], (c, errs, cast)
    assert max(errs) < 1e-2, errs


def test_rk_step_adjacent_buffers_and_alias_rejection():
    announce("rk_step with U and work adjacent in one allocation; aliasing rejected")
    from paper_1806_03095_amd.binding import DgnsError
    oop, gop = make_pair((2, 2, 2), 2, 3)
    n = gop.n_dof
    buf = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    U = buf[:n].view(gop.shape)
    U.copy_(_cuda(tgv_input(oop, mach=0.3)))
    work = buf[n:]
    gop.rk_step(U, work, 0.0, 1e-4)          # adjacent, not overlapping: accepted
    torch.cuda.synchronize()
    assert torch.isfinite(U).all()
    with pytest.raises(DgnsError):
        gop.rk_step(U, buf[n // 2: n // 2 + 2 * n], 0.0, 1e-4)   # overlapping: rejected
    with pytest.raises(DgnsError):
        gop.apply(U, out=U)


def test_misaligned_vectors_rejected_before_launch():
    # every entry point that takes device vectors checks their 8-byte alignment before
    # it launches anything: a pointer 4 bytes into an allocation returns DGNS_EINVAL
    announce("misaligned vector arguments rejected by every entry point")
    import ctypes
    from paper_1806_03095_amd import binding
    oop, gop = make_pair((2, 2, 2), 2, 3)
    lib, h, n = gop.lib, gop.h, gop.n_dof
    buf = torch.zeros(12 * n + 1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    good = [ctypes.c_void_p(buf.data_ptr() + 8 * n * i) for i in range(3)]
    bad = ctypes.c_void_p(buf.data_ptr() + 4)
    work = ctypes.c_void_p(buf.data_ptr() + 8 * 3 * n)
    out8 = (ctypes.c_double * 8)()
    icp = (ctypes.c_double * 5)(1.0, 1.0, 0.1, 1.0, 0.0)
    stats = (ctypes.c_double * (gop.n[1] * gop.n_q * 9))()
    calls = {
        "apply_operator": lambda x: lib.dgns_apply_operator(h, x, good[1], 0.0),
        "apply_operator out": lambda x: lib.dgns_apply_operator(h, good[0], x, 0.0),
        "apply_residual": lambda x: lib.dgns_apply_residual(h, x, good[1], binding.TERM_ALL),
        "apply_inverse_mass": lambda x: lib.dgns_apply_inverse_mass(h, good[0], x),
        "rk_step": lambda x: lib.dgns_rk_step(h, x, work, 0.0, 1e-4),
        "rk_step work": lambda x: lib.dgns_rk_step(h, good[0], x, 0.0, 1e-4),
        "rk_stage_update": lambda x: lib.dgns_rk_stage_update(h, good[0], x, good[2], 0, 1e-4),
        "diagnostics": lambda x: lib.dgns_diagnostics(h, x, None, out8),
        "diagnostics L": lambda x: lib.dgns_diagnostics(h, good[0], x, out8),
        "kinetic_energy": lambda x: lib.dgns_kinetic_energy(h, x, out8),
        "kinetic_energy_vjp": lambda x: lib.dgns_kinetic_energy_vjp(h, good[0], x),
        "channel_statistics": lambda x: lib.dgns_channel_statistics(h, x, stats),
        "project_ic": lambda x: lib.dgns_project_ic(h, 0, icp, None, x),
        "apply_residual_vjp": lambda x: lib.dgns_apply_residual_vjp(h, good[0], good[1], x, binding.TERM_ALL),
        "apply_operator_vjp": lambda x: lib.dgns_apply_operator_vjp(h, good[0], x, good[2]),
        "rk_step_vjp": lambda x: lib.dgns_rk_step_vjp(h, good[0], 0.0, 1e-4, good[1], good[2], x),
    }
    for name, call in calls.items():
        assert call(bad) == binding.EINVAL, name
    torch.cuda.synchronize()
    assert float(buf.abs().max()) == 0.0   # nothing was written


@pytest.mark.parametrize("scheme", ["williamson3", "four_stage"])
def test_rk_step_with_another_scheme(scheme):
    # dgns_set_rk_scheme: a three-stage third-order scheme (two fused stages) and a four-stage
    # coefficient table (three fused stages: the state ends in the work buffer and is copied
    # back) against the oracle's 2N recurrence with the same coefficients; then the default
    # is restored and matches the five-stage scheme's stage times
    announce("rk_step with the %s scheme" % scheme)
    if scheme == "williamson3":
        A = [float(v) for v in timeint.WS33_A]
        B = [float(v) for v in timeint.WS33_B]
    else:
        A, B = [0.0, -0.41, -0.93, -1.17], [0.31, 0.52, 0.71, 0.23]
    oop, gop = make_pair((3, 2, 2), 3, 5)
    U0 = tgv_input(oop, seed=12, mach=0.3)
    gop.set_rk_scheme(A, B)
    got_A, got_B, got_c = gop.rk_scheme()
    assert got_A == A and got_B == B
    dt = gop.compute_dt(0.3, 0.02, 1.5, 3.0, 1.0, 0.3)
    Ug = _cuda(U0.clone())
    work = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    for s in range(2):
        gop.rk_step(Ug, work, s * dt, dt)
    torch.cuda.synchronize()
    U = U0.clone()
    for s in range(2):
        U = timeint.lsrk_step(lambda V, t: oop.apply(V), U, s * dt, dt, A=A, B=B, C=got_c)
    errs = rel_err_fields(Ug.cpu() - U0, U - U0)
    print("%s: two steps, increment per field vs oracle %s" % (scheme, ["%.1e" % e for e in errs]), flush=True)
    assert max(errs) < 1e-11, errs
    # the stage update takes stage indices of this scheme only
    from paper_1806_03095_amd.binding import DgnsError
    with pytest.raises(DgnsError):
        gop.rk_stage_update(_cuda(U0.clone()), torch.zeros_like(Ug), Ug, len(A), dt)
    gop.set_rk_scheme()
    A5, B5, c5 = gop.rk_scheme()
    assert len(A5) == 5 and max(abs(x - float(y)) for x, y in zip(c5, timeint.CK54_C)) < 1e-15
    with pytest.raises(DgnsError):
        gop.set_rk_scheme([0.5, 0.1], [0.5, 0.5])     # A[0] must be 0


def test_rk_step_vjp_with_another_scheme():
    announce("rk_step_vjp with the three-stage scheme vs oracle autograd")
    A = [float(v) for v in timeint.WS33_A]
    B = [float(v) for v in timeint.WS33_B]
    oop, gop = make_pair((2, 2, 2), 2, 4)
    gop.set_rk_scheme(A, B)
    U = tgv_input(oop, seed=13, mach=0.3)
    dt = gop.compute_dt(0.3, 0.02, 1.5, 3.0, 1.0, 0.3)
    Ub1 = torch.as_tensor(np.random.default_rng(5).standard_normal(tuple(U.shape)))
    got = gop.rk_step_vjp(_cuda(U), 0.0, dt, _cuda(Ub1))
    torch.cuda.synchronize()
    V = U.clone().requires_grad_(True)
    out = timeint.lsrk_step(lambda W, t: oop.apply(W), V, 0.0, dt, A=A, B=B, C=gop.rk_scheme()[2])
    (want,) = torch.autograd.grad(out, V, grad_outputs=Ub1)
    errs = rel_err_fields(got, want)
    print("rk_step_vjp three-stage per field", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < 1e-11, errs
