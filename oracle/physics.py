"""Pointwise physics of the compressible Navier--Stokes equations.

Oracle (test infrastructure only).

Paper Sec. 2.1: conserved variables U = (rho, rho u, rho E); Newtonian stress
with zero bulk viscosity tau = mu (grad u + grad u^T - 2/3 div(u) I); Fourier heat
flux q = -lambda grad T; ideal gas p = rho R T; E = c_v T + |u|^2/2 with
c_v = R/(gamma-1); fluxes eq. (CompressibleNavierStokesFluxes)
    F_c = ((rho u)^T ; rho u (x) u + p I ; (rho E + p) u^T)
    F_v = (0 ; tau ; (tau . u)^T - q^T)
    F_rhs = (0 ; f ; f . u).

Array conventions: U[..., c] with c = 0..4; gradients G[..., c, j] = dU_c/dx_j;
fluxes F[..., c, j] (row c of the flux tensor, spatial column j).
All functions take and return torch float64 tensors.
"""

from dataclasses import dataclass

import torch


@dataclass(frozen=True)
class Fluid:
    gamma: float = 1.4
    R: float = 287.0
    mu: float = 1.0 / 1600.0
    lam: float = 0.0          # thermal conductivity lambda
    rho_ref: float = 1.0      # reference density rho_0 in nu = mu / rho_0 (Sec. 2.2.2)

    @property
    def c_v(self):
        return self.R / (self.gamma - 1.0)

    @property
    def c_p(self):
        return self.gamma * self.R / (self.gamma - 1.0)

    @property
    def nu(self):
        return self.mu / self.rho_ref

    @staticmethod
    def from_reynolds(Re, Pr, gamma=1.4, R=287.0, rho0=1.0, U0=1.0, L=1.0):
        """mu from Re = rho0 U0 L / mu and lambda from Pr = mu c_p / lambda (Sec. 5.2.1)."""
        mu = rho0 * U0 * L / Re
        c_p = gamma * R / (gamma - 1.0)
        return Fluid(gamma=gamma, R=R, mu=mu, lam=mu * c_p / Pr, rho_ref=rho0)


def velocity(U):
    return U[..., 1:4] / U[..., 0:1]


def pressure(U, fl):
    """p = (gamma - 1) (rho E - rho |u|^2 / 2), from E = c_v T + |u|^2/2 and p = rho R T."""
    m = U[..., 1:4]
    return (fl.gamma - 1.0) * (U[..., 4] - 0.5 * (m * m).sum(-1) / U[..., 0])


def temperature(U, fl):
    return pressure(U, fl) / (U[..., 0] * fl.R)


def speed_of_sound(U, fl):
    """c = sqrt(|gamma p / rho|) as in the Lax-Friedrichs flux definition (Sec. 2.2.2)."""
    return torch.sqrt(torch.abs(fl.gamma * pressure(U, fl) / U[..., 0]))


def convective_flux(U, fl):
    """F_c(U)[..., c, j] (Sec. 2.1, eq. CompressibleNavierStokesFluxes)."""
    u = velocity(U)
    p = pressure(U, fl)
    F = torch.zeros(U.shape + (3,), dtype=U.dtype)
    F[..., 0, :] = U[..., 1:4]
    eye = torch.eye(3, dtype=torch.float64)
    F[..., 1:4, :] = U[..., 1:4, None] * u[..., None, :] + p[..., None, None] * eye
    F[..., 4, :] = (U[..., 4] + p)[..., None] * u
    return F


def velocity_rate(U, dUdt):
    """du/dt from dU/dt along a trajectory: d(m/rho)/dt = (dm/dt - u drho/dt)/rho (quotient rule)."""
    return (dUdt[..., 1:4] - velocity(U) * dUdt[..., 0:1]) / U[..., 0:1]


def velocity_gradient(U, G):
    """gu[..., a, j] = d u_a / d x_j from the conserved gradients (quotient rule)."""
    rho = U[..., 0]
    u = velocity(U)
    return (G[..., 1:4, :] - u[..., :, None] * G[..., 0:1, :]) / rho[..., None, None]


def temperature_gradient(U, G, fl):
    """d T / d x_j with T = (E - |u|^2/2)/c_v and E = rho E / rho (quotient and chain rule)."""
    rho = U[..., 0]
    u = velocity(U)
    gu = velocity_gradient(U, G)
    gE = (G[..., 4, :] - (U[..., 4] / rho)[..., None] * G[..., 0, :]) / rho[..., None]
    return (gE - torch.einsum("...a,...aj->...j", u, gu)) / fl.c_v


def viscous_stress(gu, fl):
    """tau = mu (grad u + grad u^T - 2/3 div(u) I), zero bulk viscosity (Sec. 2.1)."""
    div = gu[..., 0, 0] + gu[..., 1, 1] + gu[..., 2, 2]
    eye = torch.eye(3, dtype=torch.float64)
    return fl.mu * (gu + gu.transpose(-1, -2) - (2.0 / 3.0) * div[..., None, None] * eye)


def viscous_flux(U, G, fl):
    """F_v(U, G)[..., c, j]; linear in the gradient slot G (Sec. 2.1, F_v = G(U):grad U)."""
    u = velocity(U)
    gu = velocity_gradient(U, G)
    tau = viscous_stress(gu, fl)
    gT = temperature_gradient(U, G, fl)
    F = torch.zeros(U.shape + (3,), dtype=torch.promote_types(U.dtype, G.dtype))
    F[..., 1:4, :] = tau
    F[..., 4, :] = torch.einsum("...ja,...a->...j", tau, u) + fl.lam * gT
    return F


def body_force_source(U, f):
    """F_rhs = (0, f, f . u) for a constant body force f (Sec. 2.1)."""
    u = velocity(U)
    f = torch.as_tensor(f, dtype=torch.float64)
    S = torch.zeros_like(U)
    S[..., 1:4] = f
    S[..., 4] = (u * f).sum(-1)
    return S


def _f64(a):
    if isinstance(a, torch.Tensor) and a.dtype != torch.float64:
        raise TypeError("oracle inputs must be float64, got %s" % a.dtype)
    return torch.as_tensor(a, dtype=torch.float64)


def conserved_from_primitive(rho, u, p, fl):
    """U from density, velocity (..., 3) and pressure: rho E = p/(gamma-1) + rho |u|^2 / 2."""
    rho, u, p = _f64(rho), _f64(u), _f64(p)
    U = torch.zeros(rho.shape + (5,), dtype=torch.float64)
    U[..., 0] = rho
    U[..., 1:4] = rho[..., None] * u
    U[..., 4] = p / (fl.gamma - 1.0) + 0.5 * rho * (u * u).sum(-1)
    return U
