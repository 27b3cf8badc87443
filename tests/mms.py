"""Manufactured solution for the compressible Navier-Stokes equations (tests only).

Primitive fields rho, u, p are smooth, periodic on [0,1]^3 and vary in all three
directions and in time.  The source S = dU/dt + div(F_c - F_v) is derived with
sympy from the equations of the paper's Sec. 2.1 written in primitive variables
(T = p/(rho R), tau from grad u, q = -lambda grad T, E = p/((gamma-1) rho) + |u|^2/2),
independently of the oracle's conserved-variable gradient formulas.
"""
import functools

import numpy as np
import sympy as sp

GAMMA, RGAS, MU, PR = 1.4, 1.0, 0.01, 0.71
CP = GAMMA * RGAS / (GAMMA - 1)
LAM = MU * CP / PR

x, y, z, t = sp.symbols("x y z t", real=True)
tp = 2 * sp.pi
RHO = 1 + sp.Rational(1, 10) * sp.sin(tp * (x + 2 * y) + t) * sp.cos(tp * z)
UVEL = [sp.Rational(3, 10) + sp.Rational(1, 10) * sp.sin(tp * y) * sp.cos(tp * (z - x) + t),
        -sp.Rational(1, 5) + sp.Rational(1, 10) * sp.cos(tp * x) * sp.sin(tp * z + 2 * t),
        sp.Rational(1, 10) + sp.Rational(1, 10) * sp.sin(tp * (x + y)) * sp.cos(tp * z - t)]
PRES = sp.Rational(4, 5) + sp.Rational(1, 20) * sp.cos(tp * x) * sp.sin(tp * (y - z) + t)


@functools.lru_cache(maxsize=1)
def _compiled():
    X = [x, y, z]
    rho, u, p = RHO, UVEL, PRES
    T = p / (rho * RGAS)
    E = p / ((GAMMA - 1) * rho) + sum(ui ** 2 for ui in u) / 2
    gu = [[sp.diff(u[a], X[j]) for j in range(3)] for a in range(3)]
    div = sum(gu[a][a] for a in range(3))
    tau = [[MU * (gu[a][j] + gu[j][a] - sp.Rational(2, 3) * div * (1 if a == j else 0)) for j in range(3)]
           for a in range(3)]
    q = [-LAM * sp.diff(T, X[j]) for j in range(3)]
    S = [sp.diff(rho, t) + sum(sp.diff(rho * u[j], X[j]) for j in range(3))]
    for a in range(3):
        S.append(sp.diff(rho * u[a], t) + sum(sp.diff(rho * u[a] * u[j] + (p if a == j else 0) - tau[a][j], X[j])
                                              for j in range(3)))
    S.append(sp.diff(rho * E, t) + sum(sp.diff((rho * E + p) * u[j] - sum(tau[j][a] * u[a] for a in range(3)) + q[j], X[j])
                                       for j in range(3)))
    U = [rho] + [rho * ui for ui in u] + [rho * E]
    fS = sp.lambdify((x, y, z, t), S, "numpy")
    fU = sp.lambdify((x, y, z, t), U, "numpy")
    return fS, fU


def _stack(vals, like):
    return np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), like.shape) for v in vals], axis=-1)


def source(X, t):
    fS, _ = _compiled()
    return _stack(fS(X[..., 0], X[..., 1], X[..., 2], t), X[..., 0])


def exact(X, t):
    _, fU = _compiled()
    return _stack(fU(X[..., 0], X[..., 1], X[..., 2], t), X[..., 0])
