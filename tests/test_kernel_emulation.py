"""The operator kernel source, compiled for the CPU (tests/emul: one host thread per
thread of a workgroup, real barriers) and run against the oracle -- with
AddressSanitizer and UBSan on.

This checks the kernels' indexing, face handling, geometry and arithmetic without
a GPU (it does not replace the GPU parity tests: it catches a race only when the host
threads happen to interleave badly, and it does not see the device compiler).
Float64 results follow the rule of tests/floor.py: against an extended-precision
evaluation of the same operator the kernel must be at least half as accurate as the
oracle, and it must match the oracle within 1e-12 per field or three times the oracle's
measured error.  test_lds_plan_layout checks the LDS plan of every compiled kernel on the host.
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import torch
import pytest

from oracle import diagnostics as odiag, mesh as omesh, operator as ooperator
from tests import emul_driver as ed, floor
from tests.gpu_cases import channel_input, rel_err_fields, tgv_fluid, tgv_input

PI3 = ((-math.pi,) * 3, (math.pi,) * 3)


def _tgv_case(n, k, nq, kind=0, amp=0.0, basis="LGL"):
    fl = tgv_fluid()
    om = omesh.BoxMesh(n, PI3[0], PI3[1], k, kind=kind, deform_amp=amp)
    oop = ooperator.DGOperator(om, fl, nq, basis=basis)
    return fl, oop, tgv_input(oop, mach=0.3, seed=31)


@pytest.mark.parametrize("n,k,nq,kind,amp,basis", [
    ((3, 2, 2), 1, 2, 0, 0.0, "LGL"),
    ((2, 2, 2), 2, 3, 2, 0.15, "GL"),
    ((2, 1, 2), 3, 6, 0, 0.0, "LGL"),
    ((1, 2, 2), 3, 6, 2, 0.1, "GL"),
    # k = 4, n_q = 5 in float64: traces fused into the t0 sweep so that 128 threads fit
    ((2, 1, 2), 4, 5, 2, 0.1, "LGL"),
    # k = 7, n_q = 11 in float64: one face per face phase (the three-face layout leaves
    # no room in LDS for the 1D tables), 256-thread workgroups
    ((2, 1, 1), 7, 11, 0, 0.0, "LGL"),
])
def test_emulated_residual_per_term(n, k, nq, kind, amp, basis):
    fl, oop, U = _tgv_case(n, k, nq, kind, amp, basis)
    b = 0 if basis == "LGL" else 1
    cells = list(range(oop.mesh.n_cells))
    ext = floor.extended_for(oop)
    for mask, t in ((1, "c"), (2, "v"), (3, "cv")):
        R = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, mu=fl.mu, lam=fl.lam, terms=mask)
        floor.check(R, oop.residual(U, terms=t), ext.residual(U.numpy(), cells, t), "emulated R_" + t)
    L = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, mu=fl.mu, lam=fl.lam, terms=7, fuse=1)
    R_ext = ext.residual(U.numpy(), cells)
    L_ext = np.stack([ext.inverse_mass(e, R_ext[:, e]) for e in cells], axis=1)
    floor.check(L, oop.apply(U), L_ext, "emulated L")


# walls and body force for kernels with unfused (k=4, n_q=7) and fused (k=3, n_q=6) face
# traces, and k=4, n_q=5 (both face terms once per face in the face kernel)
@pytest.mark.parametrize("k,nq", [(4, 7), (3, 6), (4, 5)])
def test_emulated_channel_walls_and_force(k, nq):
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (1.4 * 287.0)
    lo, hi = (0, -1, 0), (2 * math.pi, 1, math.pi)
    om = omesh.BoxMesh((2, 4, 1), lo, hi, k, periodic=(True, False, True), kind=omesh.CHANNEL)
    oop = ooperator.DGOperator(om, fl, nq, body_force=(1.0, 0.0, 0.0), wall_T=T0)
    U = channel_input(oop)
    ext = floor.extended_for(oop)
    cells = list(range(oop.mesh.n_cells))
    for mask, t in ((1, "c"), (2, "v"), (4, "f"), (7, "cvf")):
        R = ed.run(U.numpy(), k, nq, (2, 4, 1), lo, hi, periodic=(1, 0, 1), kind=1, mu=fl.mu, lam=fl.lam,
                   force=(1.0, 0, 0), wall_T=T0, terms=mask)
        Ro = oop.residual(U, terms=t)
        floor.check(R, Ro, ext.residual(U.numpy(), cells, t), "emulated channel R_" + t,
                    fields=(1, 4) if t == "f" else range(5))


@pytest.mark.parametrize("n,k,nq,kind,amp,basis,prec", [
    ((3, 2, 2), 1, 2, 0, 0.0, "LGL", 0),
    ((2, 2, 2), 2, 3, 2, 0.15, "GL", 0),
    ((3, 1, 2), 3, 6, 0, 0.0, "LGL", 0),
    # 240 blocks: seven full workgroups of 32 blocks and a ragged eighth
    ((4, 4, 3), 3, 6, 0, 0.0, "LGL", 0),
    ((1, 2, 2), 3, 6, 2, 0.1, "GL", 1),
    ((2, 1, 1), 4, 7, 2, 0.1, "LGL", 0),
    ((2, 1, 1), 7, 11, 0, 0.0, "LGL", 0),
])
def test_emulated_standalone_inverse_mass(n, k, nq, kind, amp, basis, prec):
    # M^{-1} of a seeded vector, checked by its backward error M L - R (cond(M) grows with k)
    fl, oop, U = _tgv_case(n, k, nq, kind, amp, basis)
    b = 0 if basis == "LGL" else 1
    L = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, precision=prec, mu=fl.mu, lam=fl.lam,
               fuse=3)
    M = oop.mass_matrices()
    ML = torch.einsum("eij,cej->cei", M, torch.as_tensor(L))
    errs = rel_err_fields(ML, U)
    tol = (1e-5 if prec else 1e-13) * max(1.0, ((k + 1) / 4.0) ** 2)
    assert max(errs) < tol, errs


@pytest.mark.parametrize("n,k,nq", [
    ((2, 2, 2), 3, 6),
    # k = 7, n_q = 11 in float32: one face per face phase, so that two waves per SIMD fit
    ((2, 1, 1), 7, 11),
])
def test_emulated_fp32_error_scale(n, k, nq):
    fl, oop, U = _tgv_case(n, k, nq)
    L = ed.run(U.numpy(), k, nq, n, *PI3, precision=1, mu=fl.mu, lam=fl.lam, terms=7, fuse=1)
    errs = rel_err_fields(L, oop.apply(U))
    # float32 rounding, not float64; M^{-1} amplifies it like the derivative matrices, ((k+1)/4)^2
    assert 1e-8 < max(errs) < 1e-4 * max(1.0, ((k + 1) / 4.0) ** 2), errs


def _oracle_vjp(oop, U, Rb, terms):
    import torch
    V = U.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(oop.residual(V, terms=terms), V, grad_outputs=Rb)
    return g


@pytest.mark.parametrize("n,k,nq,kind,amp,basis", [
    ((3, 2, 2), 1, 2, 0, 0.0, "LGL"),
    ((2, 2, 2), 2, 3, 2, 0.15, "GL"),
    ((2, 1, 2), 3, 6, 0, 0.0, "LGL"),
])
def test_emulated_adjoint_per_term(n, k, nq, kind, amp, basis):
    import torch
    fl, oop, U = _tgv_case(n, k, nq, kind, amp, basis)
    b = 0 if basis == "LGL" else 1
    Rb = torch.as_tensor(np.random.default_rng(41).standard_normal(tuple(U.shape)))
    for mask, t in ((1, "c"), (2, "v"), (3, "cv")):
        Ub = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, mu=fl.mu, lam=fl.lam, terms=mask,
                    fuse=2, Rbar=Rb.numpy())
        errs = rel_err_fields(Ub, _oracle_vjp(oop, U, Rb, t))
        assert max(errs) < 1e-12, (t, errs)


def test_emulated_adjoint_channel_walls_and_force():
    import torch
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (1.4 * 287.0)
    lo, hi = (0, -1, 0), (2 * math.pi, 1, math.pi)
    om = omesh.BoxMesh((2, 4, 1), lo, hi, 4, periodic=(True, False, True), kind=omesh.CHANNEL)
    oop = ooperator.DGOperator(om, fl, 7, body_force=(1.0, 0.0, 0.0), wall_T=T0)
    U = channel_input(oop)
    Rb = torch.as_tensor(np.random.default_rng(43).standard_normal(tuple(U.shape)))
    for mask, t in ((1, "c"), (2, "v"), (4, "f"), (7, "cvf")):
        Ub = ed.run(U.numpy(), 4, 7, (2, 4, 1), lo, hi, periodic=(1, 0, 1), kind=1, mu=fl.mu, lam=fl.lam,
                    force=(1.0, 0, 0), wall_T=T0, terms=mask, fuse=2, Rbar=Rb.numpy())
        want = _oracle_vjp(oop, U, Rb, t)
        errs = rel_err_fields(Ub[:2], want[:2]) if t == "f" else rel_err_fields(Ub, want)
        assert max(errs) < 1e-12, (t, errs)


@pytest.mark.parametrize("n,k,nq,kind", [((2, 3, 2), 3, 6, 0), ((2, 4, 1), 4, 7, 1)])
def test_emulated_channel_statistics(n, k, nq, kind):
    # per-cell partial sums of the statistics kernel, reduced here over each plane of
    # cells, against the oracle's plane averages (the y column comes from the host)
    lo, hi = (0.0, -1.0, 0.0), (2 * math.pi, 1.0, math.pi)
    fl = tgv_fluid(mu=1.0 / 180.0)
    om = omesh.BoxMesh(n, lo, hi, k, periodic=(True, kind == 0, True), kind=kind)
    oop = ooperator.DGOperator(om, fl, nq, wall_T=None if kind == 0 else 100.0)
    U = channel_input(oop)
    part = ed.run(U.numpy(), k, nq, n, lo, hi, periodic=(1, int(kind == 0), 1), kind=kind, mu=fl.mu, lam=fl.lam,
                  wall_T=0.0 if kind == 0 else 100.0, fuse=4)
    nx, ny, nz = n
    want = odiag.channel_statistics(oop, U)
    for j in range(ny):
        cells = [i + nx * (j + ny * kk) for kk in range(nz) for i in range(nx)]
        tot = part[cells].sum(axis=0)              # [n_q, 9]
        got = tot[:, 1:] / tot[:, :1]
        ref = want[j * nq:(j + 1) * nq, 1:]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), j


@pytest.mark.parametrize("k,nq,kind", [(3, 6, 0), (4, 7, 1)])
def test_emulated_wall_shear(k, nq, kind):
    # per-wall-cell sums of the wall-shear kernel, totalled here, against the oracle's
    # mean wall shear, wall density and area
    lo, hi = (0.0, -1.0, 0.0), (2 * math.pi, 1.0, math.pi)
    fl = tgv_fluid(mu=1.0 / 180.0)
    n = (2, 3, 2)
    om = omesh.BoxMesh(n, lo, hi, k, periodic=(True, False, True), kind=kind)
    oop = ooperator.DGOperator(om, fl, nq, wall_T=100.0)
    U = channel_input(oop)
    part = ed.run(U.numpy(), k, nq, n, lo, hi, periodic=(1, 0, 1), kind=kind, mu=fl.mu, lam=fl.lam, wall_T=100.0,
                  fuse=5)
    tot = part.sum(axis=0)
    tau, rho_w, area = odiag.channel_wall_shear(oop, U)
    assert abs(tot[0] / tot[2] - tau) <= 1e-12 * abs(tau)
    assert abs(tot[1] / tot[2] - rho_w) <= 1e-13 * rho_w
    assert abs(tot[2] - area) <= 1e-13 * area


def test_lds_plan_layout():
    # every compiled (degree, n_q) in both precisions: the work area holds every phase,
    # regions used at once are disjoint, the fused trace items fill whole waves, and the
    # footprint fits a compute unit (tests/emul/plan_check.cpp)
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "plan_check")
        cmd = ["g++", "-std=c++17", "-O0", "-Wno-unknown-pragmas", "-I", ed.EMU, "-I",
               os.path.join(ed.ROOT, "include"), "-I", ed.CSRC, os.path.join(ed.EMU, "plan_check.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        r = subprocess.run([exe], capture_output=True, text=True)
        assert r.returncode == 0 and r.stdout.strip().endswith("all ok"), r.stdout[-4000:]


@pytest.mark.parametrize("k,nq,kind,amp", [(8, 9, 0, 0.0), (15, 16, 2, 0.1)])
def test_emulated_high_degree_diagnostics(k, nq, kind, amp):
    # the streamed diagnostics (one quadrature plane at a time, the totals one plane of mass
    # points at a time): the nine per-cell partial sums summed over the cells against the
    # oracle's unnormalised integrals of the same U and L -- |u|^2/2, grad u : grad u,
    # -u.du/dt, the conserved totals at the mass points and the volume -- to 1e-13 relative
    # (the rate 1e-12; the momentum totals, sums that cancel to 1e-5 of their terms, to 1e-13
    # of the mass), affine at k = 8, curved at k = 15 (measured: 3e-15, 7e-14, 5e-17)
    fl = tgv_fluid()
    n = (2, 1, 1)
    om = omesh.BoxMesh(n, PI3[0], PI3[1], k, kind=kind, deform_amp=amp)
    oop = ooperator.DGOperator(om, fl, nq)
    U = tgv_input(oop, mach=0.1, seed=33)
    L = oop.apply(U)
    part = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, mu=fl.mu, lam=fl.lam, fuse=6, Rbar=L.numpy())
    got = part.sum(axis=0)
    d = odiag.diagnostics(oop, U, L)
    V = d["volume"]
    want = [d["e_k"] * V, d["eps"] * V / fl.nu, d["rate"] * V, d["mass"], *d["mom"], d["energy"], V]
    for m in range(9):
        bound = 1e-13 * abs(want[3]) if m in (4, 5, 6) else (1e-12 if m == 2 else 1e-13) * abs(want[m])
        assert abs(got[m] - want[m]) <= bound, (m, got[m], want[m])


@pytest.mark.parametrize("k,nq", [(8, 9), (15, 16)])
def test_emulated_high_degree_channel_walls(k, nq):
    # the streamed kernels' wall branches on a 1x2x1 stretched channel with isothermal no-slip
    # walls at both ends of x2 (each cell has one wall face: the lower one lifted on the own
    # side only, the upper one with no exterior side), no body force: at k = 8 R and L under the
    # floor rule against the extended evaluation, at k = 15 per field within 1e-12 ((k+1)/4)^4
    # (L: 10 times) of the oracle as on the GPU; float32 R within 50 times the input-rounding
    # floor
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (1.4 * 287.0)
    lo, hi, n = (0, -1, 0), (2 * math.pi, 1, math.pi), (1, 2, 1)
    om = omesh.BoxMesh(n, lo, hi, k, periodic=(True, False, True), kind=omesh.CHANNEL)
    oop = ooperator.DGOperator(om, fl, nq, wall_T=T0)
    U = channel_input(oop)
    args = dict(periodic=(1, 0, 1), kind=1, mu=fl.mu, lam=fl.lam, wall_T=T0)
    R = ed.run(U.numpy(), k, nq, n, lo, hi, fuse=0, **args)
    L = ed.run(U.numpy(), k, nq, n, lo, hi, fuse=1, **args)
    Ro, Lo = oop.residual(U), oop.apply(U)
    if k == 8:
        R_ext, L_ext = floor.reference_RL(oop, U, [0, 1])
        floor.check(R, Ro, R_ext, "emulated channel k=8 R")
        floor.check(L, Lo, L_ext, "emulated channel k=8 L")
    else:
        tol = 1e-12 * ((k + 1) / 4.0) ** 4
        eR = rel_err_fields(torch.as_tensor(R), Ro)
        eL = rel_err_fields(torch.as_tensor(L), Lo)
        assert max(eR) <= tol, eR
        assert max(eL) <= 10 * tol, eL
    R32 = ed.run(U.numpy(), k, nq, n, lo, hi, fuse=0, precision=1, **args)
    cast = rel_err_fields(oop.residual(U.float().double()), Ro)
    errs = rel_err_fields(torch.as_tensor(R32), Ro)
    for c in range(5):
        assert errs[c] <= max(50 * cast[c], 1e-6), (c, errs, cast)


@pytest.mark.parametrize("n,kind,amp,basis", [((2, 1, 1), 0, 0.0, "LGL"), ((1, 2, 1), 2, 0.1, "GL")])
def test_emulated_high_degree(n, kind, amp, basis):
    # degree 8 (hd_impl.h: the cell streamed plane by plane, faces once per face, the
    # stand-alone inverse mass) at Mach 0.1: R and L under the floor rule against the
    # extended evaluation, M^{-1} by its backward error, float32 R within 50 times the
    # input-rounding floor
    k, nq = 8, 9
    fl = tgv_fluid()
    om = omesh.BoxMesh(n, PI3[0], PI3[1], k, kind=kind, deform_amp=amp)
    oop = ooperator.DGOperator(om, fl, nq, basis=basis)
    U = tgv_input(oop, mach=0.1, seed=31)
    b = 0 if basis == "LGL" else 1
    cells = list(range(om.n_cells))
    R_ext, L_ext = floor.reference_RL(oop, U, cells)
    R = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, mu=fl.mu, lam=fl.lam, fuse=0)
    floor.check(R, oop.residual(U), R_ext, "emulated k=8 R")
    L = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, mu=fl.mu, lam=fl.lam, fuse=1)
    floor.check(L, oop.apply(U), L_ext, "emulated k=8 L")
    X = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, mu=fl.mu, lam=fl.lam, fuse=3)
    MX = torch.einsum("eij,cej->cei", oop.mass_matrices(), torch.as_tensor(X))
    assert float(torch.linalg.norm(MX - U) / torch.linalg.norm(U)) < 1e-13
    R32 = ed.run(U.numpy(), k, nq, n, *PI3, kind=kind, amp=amp, basis=b, precision=1, mu=fl.mu, lam=fl.lam, fuse=0)
    R64 = oop.residual(U)
    cast = rel_err_fields(oop.residual(U.float().double()), R64)
    errs = rel_err_fields(torch.as_tensor(R32), R64)
    for c in range(5):
        assert errs[c] <= 50 * cast[c], (c, errs, cast)


def test_emulated_degree_15_padded_rows():
    # degree 15, n_q = 16: the streamed cell kernel's flux and y-swept rows and the
    # stand-alone inverse mass's x-lines are padded in float64 (128-byte rows); R and L per
    # field within 1e-12 ((k+1)/4)^4 (L: 10 times) of the oracle as on the GPU, M^{-1} by its
    # backward error, float32 R within 50 times the input-rounding floor
    k, nq, n = 15, 16, (2, 1, 1)
    fl, oop, U = _tgv_case(n, k, nq)
    tol = 1e-12 * ((k + 1) / 4.0) ** 4
    R = ed.run(U.numpy(), k, nq, n, *PI3, mu=fl.mu, lam=fl.lam, fuse=0)
    eR = rel_err_fields(torch.as_tensor(R), oop.residual(U))
    assert max(eR) <= tol, eR
    L = ed.run(U.numpy(), k, nq, n, *PI3, mu=fl.mu, lam=fl.lam, fuse=1)
    eL = rel_err_fields(torch.as_tensor(L), oop.apply(U))
    assert max(eL) <= 10 * tol, eL
    X = ed.run(U.numpy(), k, nq, n, *PI3, mu=fl.mu, lam=fl.lam, fuse=3)
    MX = torch.einsum("eij,cej->cei", oop.mass_matrices(), torch.as_tensor(X))
    assert float(torch.linalg.norm(MX - U) / torch.linalg.norm(U)) < 1e-13 * ((k + 1) / 4.0) ** 2
    R32 = ed.run(U.numpy(), k, nq, n, *PI3, precision=1, mu=fl.mu, lam=fl.lam, fuse=0)
    R64 = oop.residual(U)
    cast = rel_err_fields(oop.residual(U.float().double()), R64)
    errs = rel_err_fields(torch.as_tensor(R32), R64)
    for c in range(5):
        assert errs[c] <= max(50 * cast[c], 1e-6), (c, errs, cast)
