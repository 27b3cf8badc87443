"""Pointwise pins of the oracle's constitutive laws and fluxes (paper Sec. 2.1).

Each check is a closed form of continuum mechanics that the flux must satisfy,
not a retyped formula: rigid motions carry no viscous stress, an isotropic
expansion none either (zero bulk viscosity), simple shear gives mu * rate, a
uniform temperature gives no heat flux, a fluid at rest has F_c = p I, and
F_c is rotation-equivariant and homogeneous of degree one.
"""
import numpy as np
import torch

from oracle import physics as ph

FL = ph.Fluid(gamma=1.4, R=287.0, mu=0.013, lam=0.7, rho_ref=1.0)
rng = np.random.default_rng(7)




def _conserved_gradient(rho, grho, u, A, p, gp):
    """Exact gradient of U for given primitive values/gradients at one point (chain rule by hand)."""
    # m = rho u -> dm_a/dx_j = u_a d rho/dx_j + rho A_aj
    gm = np.outer(u, grho) + rho * A
    # rho E = p/(g-1) + rho |u|^2 / 2 -> d/dx_j = dp_j/(g-1) + |u|^2/2 drho_j + rho u.A[:, j]
    gE = gp / (FL.gamma - 1) + 0.5 * (u @ u) * grho + rho * (u @ A)
    G = np.zeros((5, 3))
    G[0] = grho
    G[1:4] = gm
    G[4] = gE
    U = ph.conserved_from_primitive(torch.tensor(rho, dtype=torch.float64), torch.tensor(u, dtype=torch.float64), torch.tensor(p, dtype=torch.float64), FL)
    return U, torch.tensor(G)


def test_rigid_rotation_has_no_stress():
    W = rng.standard_normal((3, 3))
    A = W - W.T                                   # antisymmetric velocity gradient
    U, G = _conserved_gradient(1.3, rng.standard_normal(3), rng.standard_normal(3), A, 2.0, np.zeros(3))
    tau = ph.viscous_stress(ph.velocity_gradient(U, G), FL)
    assert torch.allclose(tau, torch.zeros(3, 3, dtype=torch.float64), atol=1e-14)


def test_isotropic_expansion_has_no_stress():
    A = 0.37 * np.eye(3)                         # zero bulk viscosity: pure dilatation is stress free
    U, G = _conserved_gradient(0.8, rng.standard_normal(3), rng.standard_normal(3), A, 1.0, np.zeros(3))
    tau = ph.viscous_stress(ph.velocity_gradient(U, G), FL)
    assert torch.allclose(tau, torch.zeros(3, 3, dtype=torch.float64), atol=1e-14)


def test_simple_shear_stress():
    A = np.zeros((3, 3))
    A[0, 1] = 2.5                                # u1 = 2.5 x2
    U, G = _conserved_gradient(1.1, np.zeros(3), np.array([0.2, 0.0, 0.0]), A, 1.0, np.zeros(3))
    tau = ph.viscous_stress(ph.velocity_gradient(U, G), FL).numpy()
    expect = np.zeros((3, 3))
    expect[0, 1] = expect[1, 0] = FL.mu * 2.5
    assert np.allclose(tau, expect, atol=1e-14)


def test_uniform_temperature_has_no_heat_flux():
    # p = rho R T0 with rho varying: grad p = R T0 grad rho, grad T = 0; with a velocity gradient too
    T0 = 3.7
    rho, grho = 1.2, rng.standard_normal(3)
    u, A = rng.standard_normal(3), rng.standard_normal((3, 3))
    U, G = _conserved_gradient(rho, grho, u, A, rho * FL.R * T0, FL.R * T0 * grho)
    gT = ph.temperature_gradient(U, G, FL)
    assert torch.allclose(gT, torch.zeros(3, dtype=torch.float64), atol=1e-12)
    assert abs(float(ph.temperature(U, FL)) - T0) < 1e-12


def test_linear_temperature_heat_flux():
    # rho const, p linear -> T = p/(rho R) linear with slope grad p / (rho R); energy flux = tau.u + lam grad T
    rho = 0.9
    gp = np.array([0.3, -1.2, 0.5])
    U, G = _conserved_gradient(rho, np.zeros(3), np.zeros(3), np.zeros((3, 3)), 2.0, gp)
    F = ph.viscous_flux(U, G, FL).numpy()
    assert np.allclose(F[4], FL.lam * gp / (rho * FL.R), atol=1e-14)
    assert np.allclose(F[:4], 0.0, atol=1e-15)


def test_convective_flux_at_rest_and_mass_row():
    U = ph.conserved_from_primitive(torch.tensor(1.3, dtype=torch.float64), torch.zeros(3, dtype=torch.float64), torch.tensor(2.5, dtype=torch.float64), FL)
    F = ph.convective_flux(U, FL).numpy()
    assert np.allclose(F[0], 0) and np.allclose(F[4], 0)
    assert np.allclose(F[1:4], 2.5 * np.eye(3))


def test_convective_flux_rotation_equivariance_and_homogeneity():
    rho, u, p = 1.1, rng.standard_normal(3), 3.0
    U = ph.conserved_from_primitive(torch.tensor(rho, dtype=torch.float64), torch.tensor(u, dtype=torch.float64), torch.tensor(p, dtype=torch.float64), FL)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    UR = ph.conserved_from_primitive(torch.tensor(rho, dtype=torch.float64), torch.tensor(Q @ u, dtype=torch.float64), torch.tensor(p, dtype=torch.float64), FL)
    F, FR = ph.convective_flux(U, FL).numpy(), ph.convective_flux(UR, FL).numpy()
    n = rng.standard_normal(3)
    Fn, FRn = F @ n, FR @ (Q @ n)
    assert np.isclose(Fn[0], FRn[0]) and np.isclose(Fn[4], FRn[4])
    assert np.allclose(Q @ Fn[1:4], FRn[1:4])
    # homogeneous of degree one in U, so F(U) = dF/dU U (Euler's theorem)
    assert np.allclose(ph.convective_flux(2.5 * U, FL).numpy(), 2.5 * F)
    J = torch.autograd.functional.jacobian(lambda V: ph.convective_flux(V, FL), U)
    assert np.allclose(torch.einsum("cjd,d->cj", J, U).numpy(), F)


def test_viscous_flux_is_linear_in_gradient():
    U = ph.conserved_from_primitive(torch.tensor(1.2, dtype=torch.float64), torch.tensor(rng.standard_normal(3)), torch.tensor(2.0, dtype=torch.float64), FL)
    G1 = torch.tensor(rng.standard_normal((5, 3)))
    G2 = torch.tensor(rng.standard_normal((5, 3)))
    lhs = ph.viscous_flux(U, 2.0 * G1 - 3.0 * G2, FL)
    rhs = 2.0 * ph.viscous_flux(U, G1, FL) - 3.0 * ph.viscous_flux(U, G2, FL)
    assert torch.allclose(lhs, rhs, atol=1e-13)


def test_speed_of_sound_ideal_gas():
    # c^2 = gamma R T for an ideal gas
    U = ph.conserved_from_primitive(torch.tensor(1.3, dtype=torch.float64), torch.tensor([1.0, 2.0, 0.5], dtype=torch.float64), torch.tensor(1e5, dtype=torch.float64), FL)
    T = ph.temperature(U, FL)
    assert abs(float(ph.speed_of_sound(U, FL)) ** 2 - FL.gamma * FL.R * float(T)) < 1e-8
