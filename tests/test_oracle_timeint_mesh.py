"""Pins of the time integrator, the time-step formula and the mesh generator.

* Table 3 of the paper (Sec. 5.2.4): all 25 printed step counts follow from
  eq. TimeStepRestrictions_Compressible with Cr=0.5, e=1.5, M=0.1, |u|_max=1,
  t_f=20 and h_min = the cell edge 2 pi / 2^l.
* Sec. 5.3.1: the channel mesh's printed maximum aspect ratios.
* The 2N Runge-Kutta scheme: the order conditions up to order 4 in exact
  rational arithmetic, and the observed order on a non-autonomous ODE.
"""
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import mesh, timeint

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append([float(v) for v in line.split()])
    return out


def test_table3_step_counts():
    rows = _rows("table3_steps.txt")
    assert len(rows) == 25
    for k, l, N in rows:
        k, l = int(k), int(l)
        if l <= 4:   # the min-vertex-distance reading of h_min, on the actual mesh
            m = mesh.BoxMesh((2 ** l,) * 3, (-math.pi,) * 3, (math.pi,) * 3, 1)
            h = m.h_min()
            assert abs(h - 2 * math.pi / 2 ** l) < 1e-14
        else:
            h = 2 * math.pi / 2 ** l
        dt = timeint.time_step(0.5, 1e9, 1.5, 3.0, k, h, 1.0, 0.1, 1.0 / 1600)
        assert timeint.n_steps(20.0, dt) == int(N), (k, l)


def test_table3_convective_restriction_binds():
    # with the paper's D ~ 0.035 (Table 2 scale) the viscous step is larger for every Table 3 row
    for k, l, _ in _rows("table3_steps.txt"):
        h = 2 * math.pi / 2 ** int(l)
        dtc = 0.5 / k ** 1.5 * h / 11.0
        dtv = 0.035 / k ** 3 * h * h * 1600
        assert dtc < dtv


def test_channel_aspect_ratios():
    for l, ratio in _rows("channel_aspect.txt"):
        n = 2 ** int(l)
        m = mesh.BoxMesh((n, n, n), (0, -1, 0), (2 * math.pi, 1, math.pi), 1, periodic=(True, False, True),
                         kind=mesh.CHANNEL, stretch_C=1.8)
        hx = 2 * math.pi / n
        # thinnest cell layer: at the wall, x2 in [-1, f(1/n)]
        assert abs(hx / m.h_min() - ratio) < 0.05 + 1e-9, (l, hx / m.h_min())


def test_channel_mesh_walls_and_periodicity():
    m = mesh.BoxMesh((4, 4, 4), (0, -1, 0), (2 * math.pi, 1, math.pi), 3, periodic=(True, False, True),
                     kind=mesh.CHANNEL)
    assert (m.nb[:, 1, 0] < 0).sum() == 16 and (m.nb[:, 1, 1] < 0).sum() == 16
    assert (m.nb[:, 0, :] >= 0).all() and (m.nb[:, 2, :] >= 0).all()
    # neighbor relation is symmetric
    for e in range(m.n_cells):
        for d in range(3):
            for s in range(2):
                f = m.nb[e, d, s]
                if f >= 0:
                    assert m.nb[f, d, 1 - s] == e
    assert abs(m.volume() - 4 * math.pi ** 2) < 1e-12
    ys = m.X[:, 1, :]
    assert ys.min() == -1.0 and ys.max() == 1.0


def test_curved_mesh_is_periodic_and_volume_preserving():
    m = mesh.BoxMesh((3, 3, 3), (0, 0, 0), (1, 1, 1), 3, kind=mesh.CURVED, deform_amp=0.03)
    # the warp vanishes on the box faces; it is odd, so the enclosed volume is unchanged
    assert abs(m.volume() - 1.0) < 1e-13
    assert np.allclose(m.global_map(np.array([0.0, 0.3, 0.7])), [0.0, 0.3, 0.7])


def butcher():
    return timeint.butcher_from_2n(timeint.CK54_A, timeint.CK54_B)


def test_rk_order_conditions_exact():
    a, b, c = butcher()
    s = len(b)
    assert all(isinstance(x, Fr) for x in b)
    # abscissae: the stated c_i are the row sums (the published rationals carry ~1e-17 rounding)
    assert all(abs(float(c[i] - timeint.CK54_C[i])) < 1e-15 for i in range(s))
    A = a
    sb = lambda f: sum(b[i] * f(i) for i in range(s))
    conds = [
        (sb(lambda i: 1), Fr(1)),
        (sb(lambda i: c[i]), Fr(1, 2)),
        (sb(lambda i: c[i] ** 2), Fr(1, 3)),
        (sb(lambda i: sum(A[i][j] * c[j] for j in range(s))), Fr(1, 6)),
        (sb(lambda i: c[i] ** 3), Fr(1, 4)),
        (sb(lambda i: c[i] * sum(A[i][j] * c[j] for j in range(s))), Fr(1, 8)),
        (sb(lambda i: sum(A[i][j] * c[j] ** 2 for j in range(s))), Fr(1, 12)),
        (sb(lambda i: sum(A[i][j] * sum(A[j][m] * c[m] for m in range(s)) for j in range(s))), Fr(1, 24)),
    ]
    for got, want in conds:
        assert abs(float(got - want)) < 1e-15
    # and it is not fifth order (one of the order-5 conditions fails clearly)
    assert abs(float(sb(lambda i: c[i] ** 4) - Fr(1, 5))) > 1e-6


def test_williamson_scheme_is_third_order():
    # the second 2N scheme the library is tested with: order conditions up to three hold
    # exactly, the first fourth-order one does not
    a, b, c = timeint.butcher_from_2n(timeint.WS33_A, timeint.WS33_B)
    s = len(b)
    sb = lambda f: sum(b[i] * f(i) for i in range(s))
    assert sb(lambda i: 1) == 1
    assert sb(lambda i: c[i]) == Fr(1, 2)
    assert sb(lambda i: c[i] ** 2) == Fr(1, 3)
    assert sb(lambda i: sum(a[i][j] * c[j] for j in range(s))) == Fr(1, 6)
    assert sb(lambda i: c[i] ** 3) != Fr(1, 4)


def test_rk_observed_order_nonautonomous():
    # y' = -y + sin(t) + t cos(t) ... exact solution y = t sin(t) + exp(-t) (y(0) = 1)
    f = lambda y, t: -y + np.sin(t) + t * np.cos(t) + t * np.sin(t)
    exact = lambda t: t * np.sin(t) + np.exp(-t)
    errs = []
    for n in (20, 40, 80):
        dt, y, t = 1.0 / n, 1.0, 0.0
        for _ in range(n):
            y = timeint.lsrk_step(f, y, t, dt)
            t += dt
        errs.append(abs(y - exact(1.0)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.8, rates


def test_blowup_at_large_courant_number_is_non_finite():
    """Far past the stability limit of the explicit scheme (Cr = 3 against a critical value
    near 0.4, Sec. 5.2.2), the oracle's solution blows up within a few steps and its
    diagnostics turn non-finite -- the signal the GPU diagnostics report as
    DGNS_ENONFINITE; at Cr = 0.3 the same steps stay finite."""
    import math
    import torch
    from oracle import diagnostics, initial, mesh, operator, physics, timeint
    m = mesh.BoxMesh((3, 3, 3), (-math.pi,) * 3, (math.pi,) * 3, 2)
    fl = physics.Fluid.from_reynolds(1600.0, 0.71)
    op = operator.DGOperator(m, fl, 3)
    U0 = initial.l2_project(op, lambda x: initial.taylor_green(x, fl))
    finite = {}
    for Cr in (0.3, 3.0):
        dt = timeint.time_step(Cr, 10.0, 1.5, 3.0, 2, m.h_min(), 1.0, 0.1, fl.nu)
        U = U0.clone()
        for s in range(6):
            U = timeint.lsrk_step(lambda V, t: op.apply(V), U, s * dt, dt)
        d = diagnostics.diagnostics(op, U)
        finite[Cr] = all(math.isfinite(v) for v in (d["e_k"], d["eps"], d["mass"], d["energy"]))
        finite[Cr] = finite[Cr] and bool(torch.isfinite(U).all())
    assert finite[0.3] and not finite[3.0], finite
