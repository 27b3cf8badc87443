"""Explicit low-storage Runge-Kutta time stepping and the time-step formula.

Oracle (test infrastructure only).

Paper Sec. 2.4: the semi-discrete system dU/dt = L(U, t) (eq.
SpatiallyDiscretizedProblem) is advanced by an explicit s-stage Runge-Kutta
method, one evaluation of L per stage; the step is the minimum of a convective
and a viscous restriction (eq. TimeStepRestrictions_Compressible)
    dt_c = Cr / k^e * h_min / (|u|_max + c),  c = |u|_max / M,
    dt_v = D  / k^f * h_min^2 / nu.

The paper's own 7-stage scheme is not printed in it; the scheme used here is the
five-stage, fourth-order 2N-storage scheme of Carpenter and Kennedy (1994),
written in Williamson's two-register form
    dU <- A_i dU + dt L(U, t + c_i dt);   U <- U + B_i dU,   i = 1..5.
Its coefficients are stated as exact rationals so that tests can convert them to
Butcher form and check the order conditions in exact arithmetic.
"""

import math
from fractions import Fraction as Fr

CK54_A = [Fr(0), Fr(-567301805773, 1357537059087), Fr(-2404267990393, 2016746695238),
          Fr(-3550918686646, 2091501179385), Fr(-1275806237668, 842570457699)]
CK54_B = [Fr(1432997174477, 9575080441755), Fr(5161836677717, 13612068292357),
          Fr(1720146321549, 2090206949498), Fr(3134564353537, 4481467310338),
          Fr(2277821191437, 14882151754819)]
CK54_C = [Fr(0), Fr(1432997174477, 9575080441755), Fr(2526269341429, 6820363962896),
          Fr(2006345519317, 3224310063776), Fr(2802321613138, 2924317926251)]


# Williamson (1980), three stages, third order, 2N storage: a second published scheme,
# used to exercise a scheme other than the default (the library takes its table at run time).
WS33_A = [Fr(0), Fr(-5, 9), Fr(-153, 128)]
WS33_B = [Fr(1, 3), Fr(15, 16), Fr(8, 15)]


def butcher_from_2n(A, B):
    """Butcher (a, b, c) of a 2N scheme with the exact arithmetic of its inputs.

    Unrolling the two registers: after stage l, dU_l = sum_j (prod_{m=j+1..l} A_m) dt k_j
    and U_l = U_0 + sum_{l' <= l} B_l' dU_l'; stage i+1 evaluates L at U_i.
    """
    s = len(A)

    def coef(j, upto):
        tot = 0
        for l in range(j, upto + 1):
            prod = 1
            for m in range(j + 1, l + 1):
                prod = prod * A[m]
            tot = tot + B[l] * prod
        return tot

    a = [[0] * s for _ in range(s)]
    for i in range(1, s):
        for j in range(i):
            a[i][j] = coef(j, i - 1)
    b = [coef(j, s - 1) for j in range(s)]
    c = [sum(a[i]) for i in range(s)]
    return a, b, c


def lsrk_step(L, U, t, dt, A=CK54_A, B=CK54_B, C=CK54_C):
    """One 2N-storage step; L(U, t) -> dU/dt.  Returns the new U."""
    dU = None
    for i in range(len(A)):
        k = L(U, t + float(C[i]) * dt)
        dU = dt * k if dU is None else float(A[i]) * dU + dt * k
        U = U + float(B[i]) * dU
    return U


def time_step(Cr, D, e, f, k, h_min, umax, mach, nu):
    """dt = min(dt_c, dt_v) of eq. (TimeStepRestrictions_Compressible); c = umax / M."""
    c = umax / mach
    dt_c = Cr / k ** e * h_min / (umax + c)
    dt_v = D / k ** f * h_min ** 2 / nu if nu > 0 else math.inf
    return min(dt_c, dt_v)


def n_steps(t_final, dt):
    """Number of steps to reach t_final with the fixed step dt (the last one may overshoot)."""
    return math.ceil(t_final / dt)
