"""Pins of the oracle's DG operator (paper Sec. 2.2-2.4) against things other than itself.

* brute force: an independent pure-Python scalar implementation (face-centric,
  cofactor geometry, pressure-gradient physics) on meshes of 1-8 cells;
* free-stream preservation on affine and curved meshes;
* discrete conservation under periodic boundaries, and of mass with walls;
* the SIPG viscous operator is symmetric and negative semi-definite where the
  diffusion operator is (momentum block at rest), and the LLF operator
  linearised about a uniform flow is dissipative (no eigenvalue with Re > 0);
* the tensor-product inverse mass matrix equals the dense inverse;
* the Taylor-Green initial kinetic energy and dissipation converge to their
  closed forms at the expected rate; nodal bases LGL and GL give the same L;
* the wall state: a fluid at rest at the wall temperature is steady, heat flows from
  the warmer of wall and fluid and friction opposes a flow along the wall (planted
  adiabatic and slip walls fail), and the residual of the exact steady compressible
  Poiseuille flow converges at the order of the scheme.
"""
import math

import numpy as np
import pytest
import torch

from oracle import mesh, operator, physics, rules, initial, diagnostics
from tests.brute_force import BruteForce
from tests.oracle_cases import make, random_state


def rel(a, b):
    return float(torch.linalg.norm(torch.as_tensor(a) - torch.as_tensor(b)) / torch.linalg.norm(torch.as_tensor(b)))


BRUTE_CASES = [
    # (mesh n, k, nq, basis, kind, periodic, amp, wall_T, force)
    ((1, 1, 1), 2, 3, "LGL", mesh.AFFINE, (True, True, True), 0.0, None, None),
    ((2, 2, 2), 1, 3, "GL", mesh.AFFINE, (True, True, True), 0.0, None, None),
    ((2, 1, 2), 2, 3, "LGL", mesh.CURVED, (True, True, True), 0.04, None, None),
    ((1, 4, 1), 2, 3, "LGL", mesh.CHANNEL, (True, False, True), 0.0, 7e-3, (0.7, 0.0, 0.2)),
    ((1, 1, 1), 3, 4, "GL", mesh.AFFINE, (True, True, True), 0.0, None, None),
]


@pytest.mark.parametrize("case", BRUTE_CASES)
def test_oracle_matches_brute_force(case):
    n, k, nq, basis, kind, periodic, amp, wall_T, force = case
    lo, hi = (0.0, -1.0, 0.0), (1.0, 1.0, 0.8)
    op = make(n=n, k=k, nq=nq, basis=basis, kind=kind, periodic=periodic, lo=lo, hi=hi, amp=amp,
              wall_T=wall_T, force=force)
    bf = BruteForce(n, lo, hi, k, nq, basis=basis, periodic=periodic, kind=kind, amp=amp,
                    mu=op.fl.mu, lam=op.fl.lam, wall_T=wall_T, body_force=force)
    U = random_state(op.mesh.n_cells, op.N, seed=3)
    R_or = op.residual(U, terms="cvf")
    R_bf = bf.residual(U.numpy(), terms="cvf")
    assert rel(R_or, R_bf) < 1e-13
    for t in ("c", "v"):
        assert rel(op.residual(U, terms=t), bf.residual(U.numpy(), terms=t)) < 1e-13


def test_free_stream_affine():
    op = make(n=(3, 2, 2), k=3, nq=5, mu=0.01, lam=0.02)
    fl = op.fl
    x = op.physical_cell_points().numpy()
    U = initial.l2_project(op, lambda x: initial.uniform(x, fl))
    R = op.residual(U)
    vol = op.residual(U, terms="c").abs().max()            # scale: the largest single term
    scale = float(op.residual(torch.ones_like(U) * U[:, :1, :1], cells=[0], terms="c").abs().max()) + 1.0
    assert float(R.abs().max()) < 1e-13 * max(scale, 1.0) * 10


@pytest.mark.parametrize("k,nq", [(2, 3), (3, 5), (4, 6)])
def test_free_stream_curved(k, nq):
    # nq >= ceil(3k/2) integrates the metric terms exactly, so a constant state stays constant
    op = make(n=(2, 2, 2), k=k, nq=nq, kind=mesh.CURVED, amp=0.08, lo=(0, 0, 0), hi=(1, 1, 1))
    _, Jinv, _ = op._geometry(np.arange(8), op.cell_pts)
    assert float(Jinv.std(dim=1).max()) > 1e-2            # the metric really varies inside cells
    fl = op.fl
    Uc = physics.conserved_from_primitive(torch.tensor(1.0, dtype=torch.float64),
                                          torch.tensor([0.3, -0.2, 0.1], dtype=torch.float64),
                                          torch.tensor(1.0 / 1.4, dtype=torch.float64), fl)
    U = Uc[:, None, None].expand(5, op.mesh.n_cells, op.N).clone()  # nodal constants = constant function
    R = op.residual(U, terms="cv")
    assert float(R.abs().max()) < 1e-13


def test_conservation_periodic():
    op = make(n=(2, 3, 2), k=2, nq=4, kind=mesh.CURVED, amp=0.05, lo=(0, 0, 0), hi=(1, 1, 1))
    U = random_state(op.mesh.n_cells, op.N, seed=11, amp=0.1)
    R = op.residual(U, terms="cv")
    # sum_i phi_i = 1: the totals of R are the integrals of -div F, i.e. zero
    tot = R.sum((1, 2))
    scale = float(op.residual(U, terms="c").abs().sum())
    assert float(tot.abs().max()) < 1e-14 * scale


def test_mass_conservation_with_walls():
    op = make(n=(2, 4, 1), k=2, nq=4, kind=mesh.CHANNEL, periodic=(True, False, True), lo=(0, -1, 0),
              hi=(2, 1, 1), wall_T=7e-3, force=(1.0, 0, 0))
    U = random_state(op.mesh.n_cells, op.N, seed=5, amp=0.1)
    R = op.residual(U)
    scale = float(op.residual(U, terms="c").abs().sum())
    assert abs(float(R[0].sum())) < 1e-14 * scale


def _jacobian(op, U, terms, comps=slice(0, 5)):
    """d R[comps] / d U[comps] as a dense matrix (forward-mode, one column per input)."""
    E, N = U.shape[1], U.shape[2]
    idx = range(5)[comps]
    cols = []
    for c in idx:
        for e in range(E):
            for i in range(N):
                T = torch.zeros_like(U)
                T[c, e, i] = 1.0
                _, jv = torch.func.jvp(lambda V: op.residual(V, terms=terms), (U,), (T,))
                cols.append(jv[comps].reshape(-1))
    return torch.stack(cols, dim=1)


def _rest_state(op):
    U = torch.zeros(5, op.mesh.n_cells, op.N, dtype=torch.float64)
    U[0] = 1.0
    U[4] = 2.5
    return U


def _viscous_blocks(op):
    U = _rest_state(op)
    Jm = _jacobian(op, U, "v", slice(1, 4))
    return Jm


def test_sipg_symmetric_and_semidefinite():
    # at a state at rest with uniform rho, p the momentum-momentum block of the viscous
    # residual's Jacobian is -B(phi_j, phi_i) with B the SIPG bilinear form of the
    # Navier-Lame operator: symmetric, and negative semi-definite (rigid motions in its kernel)
    op = make(n=(2, 1, 1), k=1, nq=3, mu=0.05, lam=0.0, lo=(0, 0, 0), hi=(1, 1, 1))
    Jm = _viscous_blocks(op)
    asym = float((Jm - Jm.T).abs().max() / Jm.abs().max())
    assert asym < 1e-12
    ev = torch.linalg.eigvalsh(0.5 * (Jm + Jm.T))
    assert float(ev.max()) < 1e-12 * float(ev.abs().max())
    # energy block with lambda > 0 and mu = 0: a penalised diffusion of rho E, also symmetric
    op2 = make(n=(2, 1, 1), k=1, nq=3, mu=0.0, lam=0.3, lo=(0, 0, 0), hi=(1, 1, 1))
    J2 = _jacobian(op2, _rest_state(op2), "v", slice(4, 5))
    assert float((J2 - J2.T).abs().max() / J2.abs().max()) < 1e-12


@pytest.mark.parametrize("planted", [-0.5, 1.0, 0.0])
def test_sipg_symmetry_pin_detects_planted_mistakes(planted, monkeypatch):
    # plant a wrong factor on the symmetry term in the oracle: the symmetry pin must fail
    monkeypatch.setattr(operator, "SYMMETRY_FACTOR", planted)
    op = make(n=(2, 1, 1), k=1, nq=3, mu=0.05, lam=0.0, lo=(0, 0, 0), hi=(1, 1, 1))
    Jm = _viscous_blocks(op)
    assert float((Jm - Jm.T).abs().max() / Jm.abs().max()) > 1e-3


def test_sipg_definiteness_pin_detects_missing_penalty(monkeypatch):
    # plant a zero interior penalty: the SIPG form loses coercivity and the negative
    # semi-definiteness pin must fail
    monkeypatch.setattr(operator.DGOperator, "tau_of", lambda self, cells: np.zeros(len(np.atleast_1d(cells))))
    op = make(n=(2, 1, 1), k=1, nq=3, mu=0.05, lam=0.0, lo=(0, 0, 0), hi=(1, 1, 1))
    Jm = _viscous_blocks(op)
    ev = torch.linalg.eigvalsh(0.5 * (Jm + Jm.T))
    assert float(ev.max()) > 1e-6 * float(ev.abs().max())


def test_llf_dissipation_pin_detects_wrong_wave_speed(monkeypatch):
    # plant a wave speed |u| - 3c < 0 (the LLF term then anti-dissipates): the pin below must fail
    orig = physics.speed_of_sound
    monkeypatch.setattr(physics, "speed_of_sound", lambda U, fl: -3.0 * orig(U, fl))
    op = make(n=(2, 1, 1), k=1, nq=2, mu=0.0, lam=0.0, lo=(0, 0, 0), hi=(1, 1, 1))
    E, N = op.mesh.n_cells, op.N
    Uc = physics.conserved_from_primitive(torch.tensor(1.0, dtype=torch.float64),
                                          torch.tensor([0.4, 0.25, -0.3], dtype=torch.float64),
                                          torch.tensor(1.0, dtype=torch.float64), op.fl)
    U = Uc[:, None, None].expand(5, E, N).clone()
    J = _jacobian(op, U, "c")
    M = op.mass_matrices()
    Minv = torch.block_diag(*[torch.linalg.inv(M[e]) for e in range(E)])
    ev = torch.linalg.eigvals(torch.kron(torch.eye(5, dtype=torch.float64), Minv) @ J)
    assert float(ev.real.max()) > 1e-6 * float(ev.abs().max())


def test_llf_linearisation_is_dissipative():
    op = make(n=(2, 1, 1), k=1, nq=2, mu=0.0, lam=0.0, lo=(0, 0, 0), hi=(1, 1, 1))
    E, N = op.mesh.n_cells, op.N
    fl = op.fl
    Uc = physics.conserved_from_primitive(torch.tensor(1.0, dtype=torch.float64),
                                          torch.tensor([0.4, 0.25, -0.3], dtype=torch.float64),
                                          torch.tensor(1.0, dtype=torch.float64), fl)
    U = Uc[:, None, None].expand(5, E, N).clone()
    J = _jacobian(op, U, "c")
    M = op.mass_matrices()
    assert J.shape == (5 * E * N, 5 * E * N)
    Minv = torch.block_diag(*[torch.linalg.inv(M[e]) for e in range(E)])
    # dL/dU in (c, e, i) ordering: apply M^{-1} per component
    P = torch.kron(torch.eye(5, dtype=torch.float64), Minv)
    ev = torch.linalg.eigvals(P @ J)
    assert float(ev.real.max()) < 1e-10 * float(ev.abs().max())
    # and the dissipation is really there: some modes are damped
    assert float(ev.real.min()) < -1e-3 * float(ev.abs().max())


@pytest.mark.parametrize("kind,amp", [(mesh.AFFINE, 0.0), (mesh.CURVED, 0.05)])
def test_tensor_product_inverse_mass(kind, amp):
    # M_e = Phi^T W Phi with Phi = S (x) S (x) S square: M^{-1} = (S^{-1})^{x3} W^{-1} (S^{-T})^{x3}
    op = make(n=(2, 1, 1), k=3, nq=4, kind=kind, amp=amp, lo=(0, 0, 0), hi=(1, 1, 1))
    M = op.mass_matrices()
    for e in range(op.mesh.n_cells):
        assert torch.allclose(M[e], M[e].T, atol=0)
        assert float(torch.linalg.eigvalsh(M[e]).min()) > 0
    xm, wm = rules.gauss_legendre(op.k + 1)
    S = rules.lagrange_values(op.nodes, xm)
    Si = np.linalg.inv(S)
    Si3 = np.kron(np.kron(Si, Si), Si)                     # node index a0 fastest <-> last kron factor
    _, _, detJ = op._geometry(np.arange(op.mesh.n_cells), op.mass_pts)
    W = detJ.numpy() * op.mass_w[None, :]
    R = np.random.default_rng(0).standard_normal((op.mesh.n_cells, op.N))
    for e in range(op.mesh.n_cells):
        direct = np.linalg.solve(M[e].numpy(), R[e])
        tens = Si3 @ ((Si3.T @ R[e]) / W[e])
        assert np.allclose(tens, direct, rtol=1e-12, atol=1e-13 * np.abs(direct).max())


def test_taylor_green_initial_energy_and_dissipation_converge():
    fl = physics.Fluid.from_reynolds(1600, 0.71)
    ek, eps, mass_err = [], [], []
    k = 2
    for ne in (2, 4, 8):
        m = mesh.BoxMesh((ne,) * 3, (-math.pi,) * 3, (math.pi,) * 3, k)
        op = operator.DGOperator(m, fl, rules.nq_three_halves(k) + 1)
        U = initial.l2_project(op, lambda x: initial.taylor_green(x, fl))
        d = diagnostics.diagnostics(op, U)
        ek.append(abs(d["e_k"] - 0.125))
        eps.append(abs(d["eps"] - 3 * fl.nu / 4))
        # mass -> (2 pi)^3 rho0 (the projection integrates cos(2x) with the n_q rule);
        # zero momentum by the odd symmetry of the velocity field, to rounding
        mass_err.append(abs(d["mass"] / (2 * math.pi) ** 3 - 1.0))
        assert np.abs(d["mom"]).max() < 1e-11
    # e_k: projection error O(h^{k+1}) enters squared; eps: the broken gradient's
    # face terms leave O(h^k)
    rate_e = math.log2(ek[1] / ek[2])
    rate_eps = math.log2(eps[1] / eps[2])
    assert rate_e > 2 * k + 0.5 and rate_eps > k - 0.5, (ek, eps)
    assert ek[2] < 1e-5 and eps[2] / (3 * fl.nu / 4) < 0.05
    assert mass_err[2] < 1e-12 and mass_err[0] < 1e-6


def test_basis_independence():
    fl = physics.Fluid(gamma=1.4, R=287.0, mu=0.02, lam=0.05)
    res = {}
    for basis in ("LGL", "GL"):
        m = mesh.BoxMesh((2, 2, 2), (-math.pi,) * 3, (math.pi,) * 3, 3, kind=mesh.CURVED, deform_amp=0.2)
        op = operator.DGOperator(m, fl, 6, basis=basis)
        U = initial.l2_project(op, lambda x: initial.taylor_green(x, fl, mach=0.3))
        L = op.apply(U)
        pts = np.random.default_rng(1).uniform(0, 1, (20, 3))
        from oracle.mesh import tensor_basis
        Phi, _ = tensor_basis(op.nodes, pts)
        res[basis] = (np.einsum("pi,cei->cep", Phi, L.numpy()), diagnostics.diagnostics(op, U, L))
    a, b = res["LGL"], res["GL"]
    assert np.abs(a[0] - b[0]).max() < 1e-11 * np.abs(a[0]).max()
    for key in ("e_k", "eps", "rate"):
        assert abs(a[1][key] - b[1][key]) < 1e-12 * abs(a[1][key])


def _rest(op, rho, T):
    E, N = op.mesh.n_cells, op.N
    p = rho * op.fl.R * T
    Uc = physics.conserved_from_primitive(torch.tensor(rho, dtype=torch.float64),
                                          torch.zeros(3, dtype=torch.float64),
                                          torch.tensor(p, dtype=torch.float64), op.fl)
    return Uc[:, None, None].expand(5, E, N).clone()


def test_wall_rest_state_at_wall_temperature_is_steady():
    # a fluid at rest at the wall temperature is a steady state of the channel with
    # isothermal no-slip walls (no body force): the mirror state equals the interior one
    Tw = 300.0
    op = make(n=(2, 3, 1), k=2, nq=4, kind=mesh.CHANNEL, periodic=(True, False, True), lo=(0, -1, 0),
              hi=(2.0, 1.0, 1.0), wall_T=Tw)
    U = _rest(op, 1.2, Tw)
    R = op.residual(U)
    scale = float(op.residual(U, terms="c").abs().max()) + 1.2 * op.fl.R * Tw
    assert float(R.abs().max()) < 1e-12 * scale


@pytest.mark.parametrize("T_fluid,sign", [(250.0, 1.0), (350.0, -1.0)])
def test_wall_heat_flux_direction(T_fluid, sign):
    # a fluid at rest colder than the walls gains energy next to them, a warmer one loses
    # it (heat flows from hot to cold); mass and momentum stay at rest
    Tw = 300.0
    op = make(n=(1, 4, 1), k=2, nq=4, periodic=(True, False, True), lo=(0, -1, 0), hi=(1.0, 1.0, 1.0), wall_T=Tw)
    U = _rest(op, 1.0, T_fluid)
    R = op.residual(U)
    wall_cells = [0, 3]
    E_wall = float(R[4, wall_cells, :].sum())
    assert sign * E_wall > 0
    interior = float(R[4, [1, 2], :].abs().max())
    assert interior < 1e-10 * abs(E_wall)
    assert float(R[0].abs().max()) < 1e-10 * abs(E_wall)


def _poiseuille(op, f, p0, Tw):
    """Steady compressible channel flow driven by the body force f (per volume) between
    isothermal no-slip walls at y = -1, 1, constant mu and lambda: the x-momentum balance
    mu u'' + f = 0 gives u = U (1 - y^2), U = f / (2 mu); the pressure is uniform; the
    energy balance (mu u u')' + lambda T'' + f u = 0 gives T = Tw + mu U^2 (1 - y^4) / (3
    lambda); rho = p0 / (R T)."""
    fl = op.fl
    U = f / (2.0 * fl.mu)

    def field(x):
        y = torch.as_tensor(x[..., 1])
        T = Tw + fl.mu * U ** 2 * (1.0 - y ** 4) / (3.0 * fl.lam)
        rho = p0 / (fl.R * T)
        u = torch.zeros(y.shape + (3,), dtype=torch.float64)
        u[..., 0] = U * (1.0 - y ** 2)
        return physics.conserved_from_primitive(rho, u, p0 * torch.ones_like(y), fl)

    return initial.l2_project(op, field)


def _poiseuille_residuals(k, ny_list):
    f, Tw = 0.04, 1.0
    out = []
    for ny in ny_list:
        op = make(n=(1, ny, 1), k=k, nq=k + 2, periodic=(True, False, True), lo=(0.0, -1.0, 0.0),
                  hi=(0.5, 1.0, 0.5), wall_T=Tw, force=(f, 0.0, 0.0))
        U = _poiseuille(op, f, op.fl.R * Tw, Tw)
        out.append(float(op.residual(U).abs().max()))
    return out


def test_wall_state_poiseuille_steady_state_converges():
    # The wall state (no-slip and isothermal through the mirror exterior state, a reading
    # of Sec. 2.2 / 5.3) against a closed form: the residual of the projected steady
    # Poiseuille state (shear and heat flux at the walls) vanishes under refinement; its
    # largest entries sit in the wall cells' energy rows and fall at about the order k of
    # the scheme (measured at k = 3: rates 2.5 and 2.9 over ny = 2, 4, 8)
    k = 3
    e = _poiseuille_residuals(k, (2, 4, 8))
    rates = [math.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
    print("Poiseuille residual:", ["%.2e" % v for v in e], "rates", ["%.2f" % r for r in rates])
    assert min(rates) > k - 0.75, rates


def _uniform_flow(op, rho, u0, T):
    E, N = op.mesh.n_cells, (op.mesh.k + 1) ** 3
    u = torch.tensor([u0, 0.0, 0.0], dtype=torch.float64)
    Uc = physics.conserved_from_primitive(torch.tensor(rho, dtype=torch.float64), u,
                                          torch.tensor(rho * op.fl.R * T, dtype=torch.float64), op.fl)
    return Uc[:, None, None].expand(5, E, N).clone()


def _wall_friction(op):
    U = _uniform_flow(op, 1.0, 0.5, op.wall_T)
    R = op.residual(U)
    return float(R[1, [0, 3], :].sum()), float(R[1, [1, 2], :].abs().max()), float(R[0].abs().max())


def test_wall_friction_opposes_the_flow():
    # fluid moving uniformly along the walls at the wall temperature: the no-slip wall
    # decelerates it (x-momentum rows of the wall cells negative), the interior cells and
    # the mass rows see nothing
    op = make(n=(1, 4, 1), k=2, nq=4, periodic=(True, False, True), lo=(0, -1, 0), hi=(1.0, 1.0, 1.0), wall_T=1.0)
    wall, interior, mass = _wall_friction(op)
    assert wall < 0
    assert interior < 1e-10 * abs(wall)
    assert mass < 1e-10 * abs(wall)


def test_wall_friction_pin_detects_planted_slip():
    # the same with a slip wall planted in the oracle's mirror state (u+ = u-): no friction
    def slip(self, Um, Gm):
        Up, Gp = operator.DGOperator._mirror(self, Um, Gm)
        Up = Up.clone()
        Up[..., 1:4] = Um[..., 1:4]
        return Up, Gp

    good = make(n=(1, 4, 1), k=2, nq=4, periodic=(True, False, True), lo=(0, -1, 0), hi=(1.0, 1.0, 1.0), wall_T=1.0)
    bad = make(n=(1, 4, 1), k=2, nq=4, periodic=(True, False, True), lo=(0, -1, 0), hi=(1.0, 1.0, 1.0), wall_T=1.0)
    bad._mirror = slip.__get__(bad)
    w_good, _, _ = _wall_friction(good)
    w_bad, _, _ = _wall_friction(bad)
    print("wall friction: no-slip %.3e, planted slip %.3e" % (w_good, w_bad))
    assert abs(w_bad) < 1e-6 * abs(w_good)


def test_wall_heat_flux_pin_detects_planted_adiabatic_wall():
    # the heat-flux direction pin with an adiabatic wall planted in the oracle's mirror
    # state (T+ = T-, no-slip kept): a fluid colder than the walls no longer gains energy
    def adiabatic(self, Um, Gm):
        Up = Um.clone()
        Up[..., 1:4] = -Um[..., 1:4]
        return Up, Gm

    Tw = 300.0
    good = make(n=(1, 4, 1), k=2, nq=4, periodic=(True, False, True), lo=(0, -1, 0), hi=(1.0, 1.0, 1.0), wall_T=Tw)
    bad = make(n=(1, 4, 1), k=2, nq=4, periodic=(True, False, True), lo=(0, -1, 0), hi=(1.0, 1.0, 1.0), wall_T=Tw)
    bad._mirror = adiabatic.__get__(bad)
    e_good = float(good.residual(_rest(good, 1.0, 250.0))[4, [0, 3], :].sum())
    e_bad = float(bad.residual(_rest(bad, 1.0, 250.0))[4, [0, 3], :].sum())
    print("wall heat gain: isothermal %.3e, planted adiabatic %.3e" % (e_good, e_bad))
    assert e_good > 0 and abs(e_bad) < 1e-6 * e_good
