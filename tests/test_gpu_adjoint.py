"""GPU parity of the hand-written adjoint against the oracle's reverse-mode derivative.

The oracle's gradient is torch autograd applied to its direct evaluation of the
weak form (a library primitive on the plain definition).  Checked: the residual
VJP per term and the operator VJP on the Taylor-Green 4^3, k=3, n_q=6 setup, on
curved meshes and on the stretched channel with walls and body force; one Runge-
Kutta step's VJP; a dot-product test against finite differences of the GPU
operator; and the gradient of the kinetic energy after 50 steps with checkpoints
every 10 steps (16^3 cells, k=3) against central finite differences on 20 seeded
directions.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import timeint
from tests.gpu_cases import announce, make_pair, tgv_input, channel_input, rel_err_fields, tgv_fluid

pytestmark = pytest.mark.gpu


def _cuda(t):
    return t.to("cuda").contiguous()


def _oracle_vjp(fn, U, cot):
    V = U.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(fn(V), V, grad_outputs=cot)
    return g


def _check(got, want, tol, what):
    errs = rel_err_fields(got, want)
    assert max(errs) < tol, (what, errs)


@pytest.mark.parametrize("terms,mask", [("c", 1), ("v", 2), ("cv", 3)])
def test_residual_vjp_tgv(terms, mask):
    announce("adjoint: residual VJP tgv 4^3 k=3 nq=6 terms=%s" % terms)
    oop, gop = make_pair((4, 4, 4), 3, 6)
    U = tgv_input(oop, seed=21)
    Rb = torch.as_tensor(synth.normal(tuple(U.shape), 22))
    Ub = gop.residual_vjp(_cuda(U), _cuda(Rb), terms=mask)
    torch.cuda.synchronize()
    _check(Ub, _oracle_vjp(lambda V: oop.residual(V, terms=terms), U, Rb), 1e-12, "Ubar_" + terms)


@pytest.mark.parametrize("case", [((2, 2, 3), 2, 4, "curved", 0.1, "LGL"), ((2, 3, 2), 3, 5, "curved", 0.15, "GL"),
                                  ((3, 2, 2), 1, 2, "affine", 0.0, "LGL"), ((2, 2, 2), 4, 7, "affine", 0.0, "LGL"),
                                  ((2, 2, 2), 5, 8, "curved", 0.05, "LGL"),
                                  # n_q = 2k+1
                                  ((2, 2, 1), 3, 7, "affine", 0.0, "LGL"), ((2, 1, 1), 4, 9, "curved", 0.1, "GL")])
def test_operator_vjp_range(case):
    n, k, nq, kind, amp, basis = case
    announce("adjoint: operator VJP n=%s k=%d nq=%d %s %s" % (n, k, nq, kind, basis))
    oop, gop = make_pair(n, k, nq, kind=kind, amp=amp, basis=basis)
    U = tgv_input(oop, seed=23, mach=0.3)
    Lb = torch.as_tensor(synth.normal(tuple(U.shape), 24))
    Ub = gop.operator_vjp(_cuda(U), _cuda(Lb))
    torch.cuda.synchronize()
    _check(Ub, _oracle_vjp(lambda V: oop.apply(V), U, Lb), 1e-11, "Ubar")


def test_operator_vjp_channel_walls_force():
    announce("adjoint: channel 2x4x2 k=4 nq=7 walls+force")
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (1.4 * 287.0)
    oop, gop = make_pair((2, 4, 2), 4, 7, lo=(0, -1, 0), hi=(2 * math.pi, 1, math.pi), periodic=(1, 0, 1),
                         kind="channel", fluid=fl, force=(1.0, 0.0, 0.0), wall_T=T0)
    U = channel_input(oop)
    Lb = torch.as_tensor(synth.normal(tuple(U.shape), 25))
    Ub = gop.operator_vjp(_cuda(U), _cuda(Lb))
    torch.cuda.synchronize()
    _check(Ub, _oracle_vjp(lambda V: oop.apply(V), U, Lb), 1e-11, "Ubar")


def test_rk_step_vjp_against_oracle():
    announce("adjoint: one RK step VJP, tgv 2^3 k=3 nq=6")
    oop, gop = make_pair((2, 2, 2), 3, 6)
    U = tgv_input(oop, seed=26, mach=0.3)
    dt = 2e-3
    Ub1 = torch.as_tensor(synth.normal(tuple(U.shape), 27))
    got = gop.rk_step_vjp(_cuda(U), 0.0, dt, _cuda(Ub1))
    torch.cuda.synchronize()
    want = _oracle_vjp(lambda V: timeint.lsrk_step(lambda W, t: oop.apply(W), V, 0.0, dt), U, Ub1)
    _check(got, want, 1e-12, "rk step")
    # in place
    Ubg = _cuda(Ub1)
    gop.rk_step_vjp(_cuda(U), 0.0, dt, Ubg, out=Ubg)
    torch.cuda.synchronize()
    _check(Ubg, want, 1e-12, "rk step in place")


def test_operator_dot_product_test():
    announce("adjoint: dot-product test of the operator, tgv 4^3 k=3 nq=6")
    oop, gop = make_pair((4, 4, 4), 3, 6)
    U = _cuda(tgv_input(oop, seed=28, mach=0.3))
    d = _cuda(torch.as_tensor(synth.normal(tuple(U.shape), 29))) * U.abs() * 1e-3
    lb = _cuda(torch.as_tensor(synth.normal(tuple(U.shape), 30)))
    h = 1e-3
    Jd = (gop.apply(U + h * d) - gop.apply(U - h * d)) / (2 * h)
    lhs = float((lb * Jd).sum())
    rhs = float((gop.operator_vjp(U, lb) * d).sum())
    # central differences with this step agree to ~1e-6 (the same check on the oracle alone)
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs), (lhs, rhs)


def _oracle_ke(oop, V):
    _, _, detJ = oop._geometry(np.arange(oop.mesh.n_cells), oop.cell_pts)
    Uq = torch.einsum("pi,cei->epc", oop.Phi, V)
    u = Uq[..., 1:4] / Uq[..., 0:1]
    return (0.5 * (u * u).sum(-1) * detJ * torch.as_tensor(oop.cell_w)).sum()


def test_kinetic_energy_and_vjp_against_oracle():
    announce("adjoint: kinetic energy and its VJP, tgv 2^3 k=3 nq=6")
    oop, gop = make_pair((2, 2, 2), 3, 6)
    U = tgv_input(oop, seed=32, mach=0.3)
    K = gop.kinetic_energy(_cuda(U))
    Kb = gop.kinetic_energy_vjp(_cuda(U))
    torch.cuda.synchronize()
    V = U.clone().requires_grad_(True)
    Ko = _oracle_ke(oop, V)
    (g,) = torch.autograd.grad(Ko, V)
    assert abs(K - float(Ko)) <= 1e-13 * abs(float(Ko))
    _check(Kb[:4], g[:4], 1e-13, "dK/dU")
    assert float(Kb[4].abs().max()) == 0.0


def test_rollout_gradient_against_oracle():
    from paper_1806_03095_amd.autograd import kinetic_energy, rk_rollout
    announce("adjoint: dK(U_5)/dU_0 with checkpoints every 2 steps, tgv 2^3 k=3 nq=6, vs oracle")
    oop, gop = make_pair((2, 2, 2), 3, 6)
    U0 = tgv_input(oop, seed=33, mach=0.3)
    dt = 2e-3
    x = _cuda(U0).clone().requires_grad_(True)
    (g,) = torch.autograd.grad(kinetic_energy(rk_rollout(x, gop, 5, dt, ckpt_every=2), gop), x)
    V = U0.clone().requires_grad_(True)
    W = V
    for s in range(5):
        W = timeint.lsrk_step(lambda Z, t: oop.apply(Z), W, s * dt, dt)
    (go,) = torch.autograd.grad(_oracle_ke(oop, W), V)
    _check(g, go, 1e-11, "dK/dU0")


def test_kinetic_energy_gradient_50_steps_against_fd():
    """16^3 cells, k=3, 50 RK steps, checkpoints every 10: gradient of int |u|^2/2 vs central FD."""
    from paper_1806_03095_amd import taylor_green
    from paper_1806_03095_amd.autograd import kinetic_energy, rk_rollout
    announce("adjoint: dK(U_50)/dU_0, tgv 16^3 k=3 nq=6, 20 FD directions")
    op = taylor_green(3, 16, n_q=6)
    U0 = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
    U0 = U0 * (1.0 + 1e-3 * _cuda(torch.as_tensor(synth.normal(tuple(U0.shape), 31))))
    dt = op.compute_dt(0.3, 0.02, 1.5, 3.0, 1.0, 0.1)   # about 2/3 of the stability limit
    x = U0.clone().requires_grad_(True)
    K = kinetic_energy(rk_rollout(x, op, 50, dt, ckpt_every=10), op)
    (g,) = torch.autograd.grad(K, x)

    def K_of(V):
        W = V.clone()
        work = torch.empty(2 * op.n_dof, dtype=torch.float64, device="cuda")
        for s in range(50):
            op.rk_step(W, work, s * dt, dt)
        return op.kinetic_energy(W)

    errs = []
    for j in range(20):
        d = _cuda(torch.as_tensor(synth.normal(tuple(U0.shape), 100 + j)))
        h = 1e-6 * float(torch.linalg.norm(U0)) / float(torch.linalg.norm(d))
        fd = (K_of(U0 + h * d) - K_of(U0 - h * d)) / (2 * h)
        ad = float((g * d).sum())
        errs.append(abs(fd - ad) / abs(ad))
    print("FD vs adjoint, relative differences:", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < 1e-5, errs
