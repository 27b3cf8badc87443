"""Pins of the oracle's dissipation rate, Taylor-Green pressure and perturbed channel state.

CPU only.  Each pin compares the oracle with something the mathematics fixes
independently of the oracle's own formula, and each has a planted-mistake twin that
must make it fail:
  * -de_k/dt (Sec. 5.2.3): the chain rule makes the exact rate equal to the derivative
    of e_k along dU/dt = L, which a centred difference of e_k(U +- delta L) gives to
    O(delta^2);
  * the Taylor-Green pressure (Sec. 5.2.1): for the divergence-free initial velocity the
    incompressible pressure satisfies the Poisson identity lap p = -rho0 d_i u_j d_j u_i,
    which fixes the amplitude rho0 V0^2/16 and the shape of the perturbation; the mean
    state fixes p0 through the Mach number (c0 = V0 / M) and the uniform temperature;
  * the perturbed channel state (Sec. 5.3.1): density and temperature of every node
    are kept, the perturbation vanishes at the walls and is bounded by amp * u1(x2).
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import diagnostics, initial, mesh, operator, physics
from tests.oracle_cases import make, random_state


# ----------------------------------------------------------------- -de_k/dt


def _rate_pin(op, U):
    """(oracle rate, centred difference -(e_k(U + d L) - e_k(U - d L)) / (2 d)) for two d."""
    L = op.apply(U)
    rate = diagnostics.diagnostics(op, U, L)["rate"]
    fds = []
    for delta in (2e-4, 1e-4):
        ep = diagnostics.diagnostics(op, U + delta * L)["e_k"]
        em = diagnostics.diagnostics(op, U - delta * L)["e_k"]
        fds.append(-(ep - em) / (2 * delta))
    return rate, fds


def _rate_case():
    # a compressible state (mean flow plus 5 % noise), so that L_rho is O(1) and the
    # u L_rho term of du/dt = (L_m - u L_rho)/rho matters
    op = make(n=(2, 2, 1), k=2, nq=4, mu=0.02, lam=0.03)
    U = random_state(op.mesh.n_cells, op.N, seed=17, amp=0.05)
    return op, U


def test_dissipation_rate_is_the_derivative_of_ek_along_L():
    op, U = _rate_case()
    rate, fds = _rate_pin(op, U)
    err = [abs(rate - fd) / abs(rate) for fd in fds]
    # O(delta^2): halving delta divides the difference by about four
    assert err[1] < 1e-7, (rate, fds, err)
    assert err[1] < 0.35 * err[0] or err[1] < 1e-11, err


@pytest.mark.parametrize("plant", ["flipped_sign", "dropped_density_rate"])
def test_dissipation_rate_pin_detects_planted_mistakes(plant, monkeypatch):
    orig = physics.velocity_rate
    if plant == "flipped_sign":
        monkeypatch.setattr(physics, "velocity_rate", lambda U, dUdt: -orig(U, dUdt))
    else:
        monkeypatch.setattr(physics, "velocity_rate",
                            lambda U, dUdt: dUdt[..., 1:4] / U[..., 0:1])
    op, U = _rate_case()
    rate, fds = _rate_pin(op, U)
    assert abs(rate - fds[1]) / abs(fds[1]) > 1e-3, (plant, rate, fds)


# ----------------------------------------------------------------- Taylor-Green pressure


def _tgv_fields(x, fl):
    """Primitive p, u, T recovered from the oracle's conserved Taylor-Green state at x."""
    U = initial.taylor_green(x, fl).numpy()
    rho = U[..., 0]
    u = U[..., 1:4] / rho[..., None]
    p = (fl.gamma - 1.0) * (U[..., 4] - 0.5 * rho * (u * u).sum(-1))
    return p, u, p / (rho * fl.R), rho


def _poisson_pin(fl, n_pts=40, seed=3):
    """max |lap p + rho0 d_i u_j d_j u_i| / max |lap p| over random points, derivatives by
    sixth-order central differences of the oracle's function."""
    x0 = synth.rng(seed).uniform(-math.pi, math.pi, (n_pts, 3))
    h = 2e-2
    # sixth-order stencils for the first and second derivative
    c1 = {1: 3 / 4, 2: -3 / 20, 3: 1 / 60}
    c2 = {0: -49 / 18, 1: 3 / 2, 2: -3 / 20, 3: 1 / 90}
    lap = np.zeros(n_pts)
    du = np.zeros((n_pts, 3, 3))                       # du[:, a, j] = d u_a / d x_j
    p0, _, _, _ = _tgv_fields(x0, fl)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        lap += c2[0] * p0 / h ** 2
        for m in (1, 2, 3):
            pp, up, _, _ = _tgv_fields(x0 + m * e, fl)
            pm, um, _, _ = _tgv_fields(x0 - m * e, fl)
            lap += c2[m] * (pp + pm) / h ** 2
            du[:, :, j] += c1[m] * (up - um) / h
    rhs = -np.einsum("nij,nji->n", du, du)             # rho0 = 1
    return float(np.max(np.abs(lap - rhs)) / np.max(np.abs(lap)))


def test_taylor_green_pressure_solves_the_poisson_identity():
    fl = physics.Fluid.from_reynolds(1600.0, 0.71)
    assert _poisson_pin(fl) < 1e-6


def test_taylor_green_mean_state_and_uniform_temperature():
    fl = physics.Fluid.from_reynolds(1600.0, 0.71)
    mach = 0.1
    x = synth.rng(5).uniform(-math.pi, math.pi, (200, 3))
    p, u, T, rho = _tgv_fields(x, fl)
    # isothermal start: T = T0 everywhere with gamma R T0 = c0^2 = (V0 / M)^2
    assert np.allclose(T, T[0], rtol=1e-14, atol=0.0)
    assert abs(math.sqrt(fl.gamma * fl.R * T[0]) - 1.0 / mach) < 1e-12
    # the pressure perturbation averages to zero over a period, so the mean pressure is
    # p0 = rho0 R T0 with rho0 = 1 (checked on a tensor grid, where the trapezoidal rule is exact)
    g = np.linspace(-math.pi, math.pi, 16, endpoint=False)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pg, _, Tg, rhog = _tgv_fields(X, fl)
    assert abs(pg.mean() - fl.R * Tg[0]) < 1e-12 * pg.mean()
    assert abs(rhog.mean() - 1.0) < 1e-13


def test_taylor_green_pressure_pin_detects_doubled_amplitude(monkeypatch):
    # plant rho0 V0^2 / 8 instead of / 16: the perturbation p - p0 doubles
    orig = initial.taylor_green

    def planted(x, fl, U0=1.0, L=1.0, mach=0.1, rho0=1.0):
        U = orig(x, fl, U0, L, mach, rho0)
        p0 = rho0 * (U0 / mach) ** 2 / fl.gamma
        rho = U[..., 0]
        ke = 0.5 * (U[..., 1:4] ** 2).sum(-1) / rho
        p = (fl.gamma - 1.0) * (U[..., 4] - ke)
        p2 = p0 + 2.0 * (p - p0)
        T0 = p0 / (rho0 * fl.R)
        rho2 = p2 / (fl.R * T0)
        u = U[..., 1:4] / rho[..., None]
        return physics.conserved_from_primitive(rho2, u, p2, fl)

    monkeypatch.setattr(initial, "taylor_green", planted)
    fl = physics.Fluid.from_reynolds(1600.0, 0.71)
    assert _poisson_pin(fl) > 0.3


# ----------------------------------------------------------------- perturbed channel


def _channel_op(k=3, basis="LGL"):
    m = mesh.BoxMesh((2, 3, 2), (0.0, -1.0, 0.0), (2 * math.pi, 1.0, math.pi), k,
                     periodic=(True, False, True), kind=mesh.CHANNEL)
    fl = physics.Fluid(gamma=1.4, R=287.0, mu=1.0 / 180.0, lam=0.0, rho_ref=1.0)
    return operator.DGOperator(m, fl, k + 2, basis=basis, wall_T=1.0)


def _node_T(U, fl):
    """Temperature at the nodes, by its own formula: T = (gamma-1)(rho E - |m|^2/(2 rho)) / (rho R)."""
    U = np.asarray(U)
    return (fl.gamma - 1.0) * (U[4] - 0.5 * (U[1:4] ** 2).sum(0) / U[0]) / (U[0] * fl.R)


def _perturbation_pin(basis="LGL"):
    op = _channel_op(basis=basis)
    umax, amp = 18.3, 0.1
    U = initial.l2_project(op, lambda x: initial.channel_laminar(x, op.fl, umax=umax, mach=0.1))
    r = synth.uniform_pm1((3, op.mesh.n_cells, op.N), 7)
    Up = initial.channel_perturbed(op, U, r, umax=umax, power=2, amp=amp)
    T0, T1 = _node_T(U, op.fl), _node_T(Up, op.fl)
    return op, U, Up, r, umax, amp, float(np.abs(T1 - T0).max() / np.abs(T0).max())


@pytest.mark.parametrize("basis", ["LGL", "GL"])
def test_channel_perturbation_keeps_density_and_temperature(basis):
    op, U, Up, r, umax, amp, dT = _perturbation_pin(basis)
    assert torch.equal(Up[0], U[0])
    assert dT < 1e-13
    du = (Up[1:4] / Up[0] - U[1:4] / U[0]).numpy()             # (3, E, N)
    k = op.k
    pts = np.array([[op.nodes[a0], op.nodes[a1], op.nodes[a2]]
                    for a2 in range(k + 1) for a1 in range(k + 1) for a0 in range(k + 1)])
    x, _ = op.mesh.map_at(pts)
    bound = amp * umax * (1.0 - x[..., 1] ** 2)                # (E, N)
    assert np.all(np.abs(du) <= bound[None] * (1 + 1e-12) + 1e-12)
    # the perturbation is the noise scaled by amp u1(x2): recovered exactly where u1 > 0
    inner = bound > 1e-8
    assert np.allclose(du[:, inner] / bound[inner][None], r[:, inner], rtol=1e-9, atol=1e-12)
    if basis == "LGL":
        # LGL nodes include the walls, where the perturbation vanishes
        wall = np.abs(np.abs(x[..., 1]) - 1.0) < 1e-14
        assert wall.any() and np.all(du[:, wall] == 0.0)


def test_channel_perturbation_pin_detects_wrong_temperature(monkeypatch):
    # plant a 0.1 % error in the oracle's temperature: rho E is then rebuilt from the
    # wrong T and the temperature-invariance pin must fail
    orig = physics.temperature
    monkeypatch.setattr(physics, "temperature", lambda U, fl: 1.001 * orig(U, fl))
    *_, dT = _perturbation_pin()
    assert dT > 1e-4
