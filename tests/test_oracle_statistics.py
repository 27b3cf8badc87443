"""Pins of the oracle's channel statistics (plane averages over the homogeneous
directions x and z, Sec. 5.3) by closed forms on states the k = 4 space holds exactly."""
import math

import numpy as np
import torch

from oracle import diagnostics as odiag, initial, mesh as omesh, operator as ooperator, physics as ph, rules
from tests.gpu_cases import tgv_fluid

LO, HI = (0.0, -1.0, 0.0), (2 * math.pi, 1.0, math.pi)


def _box(n, k=4, nq=7):
    fl = tgv_fluid(mu=1.0 / 180.0)
    om = omesh.BoxMesh(n, LO, HI, k, periodic=(True, False, True))
    return fl, ooperator.DGOperator(om, fl, nq, wall_T=100.0)


def _y_points(ny, q):
    xg, _ = rules.gauss_legendre(q)
    h = (HI[1] - LO[1]) / ny
    return np.array([LO[1] + (j + xg[p]) * h for j in range(ny) for p in range(q)])


def test_laminar_profile_closed_form():
    # u = u_max (1 - y^2), rho = 1, T uniform: degree <= 4 in each coordinate on a box,
    # so the L2 projection is exact and every plane average has a closed form
    fl, oop = _box((2, 3, 2))
    umax = 18.3
    U = initial.l2_project(oop, lambda x: initial.channel_laminar(x, fl, umax=umax, mach=0.1))
    s = odiag.channel_statistics(oop, U)
    y = _y_points(3, 7)
    assert np.abs(s[:, 0] - y).max() < 1e-14
    ue = umax * (1.0 - y ** 2)
    assert np.abs(s[:, 1] - 1.0).max() < 1e-12
    assert np.abs(s[:, 2] - ue).max() < 1e-11 * umax
    assert np.abs(s[:, [3, 4, 6, 7, 8]]).max() < 1e-11 * umax ** 2
    assert np.abs(s[:, 5] - ue ** 2).max() < 1e-10 * umax ** 2


def test_linear_variation_across_the_planes():
    # rho = 2 + y, u = 1 + c (x - x_m)/L_x, v = b (z - z_m)/L_z: the plane averages are
    # <rho> = 2 + y, <u> = 1, <uu> = 1 + c^2/12, <v> = 0, <vv> = b^2/12, <uv> = 0,
    # <w> = <ww> = 0 (u is m / rho, not m)
    fl, oop = _box((3, 2, 2))
    c, b = 0.6, 0.5
    Lx, Lz = HI[0] - LO[0], HI[2] - LO[2]

    def state(x):
        rho = 2.0 + x[..., 1]
        u = np.zeros(x.shape)
        u[..., 0] = 1.0 + c * (x[..., 0] - 0.5 * (LO[0] + HI[0])) / Lx
        u[..., 1] = b * (x[..., 2] - 0.5 * (LO[2] + HI[2])) / Lz
        return ph.conserved_from_primitive(torch.as_tensor(rho), torch.as_tensor(u),
                                           torch.as_tensor(np.full(x.shape[:-1], 10.0)), fl)

    s = odiag.channel_statistics(oop, initial.l2_project(oop, state))
    assert np.abs(s[:, 1] - (2.0 + _y_points(2, 7))).max() < 1e-12
    want = [None, None, 1.0, 0.0, 0.0, 1.0 + c * c / 12.0, b * b / 12.0, 0.0, 0.0]
    for m in range(2, 9):
        assert np.abs(s[:, m] - want[m]).max() < 1e-12, (m, s[:, m], want[m])


def test_channel_mesh_points_are_symmetric():
    # the tanh stretching is odd about y = 0 and the Gauss points are symmetric in the
    # cell, so the wall-normal points mirror: y(j, p) = -y(n - 1 - j, q - 1 - p)
    fl = tgv_fluid(mu=1.0 / 180.0)
    om = omesh.BoxMesh((2, 4, 1), LO, HI, 4, periodic=(True, False, True), kind=omesh.CHANNEL, stretch_C=1.8)
    oop = ooperator.DGOperator(om, fl, 7, wall_T=100.0)
    U = initial.l2_project(oop, lambda x: initial.channel_laminar(x, fl))
    y = odiag.channel_statistics(oop, U)[:, 0]
    assert np.abs(y + y[::-1]).max() < 1e-14
    assert np.all(np.diff(y) > 0) and -1.0 < y[0] and y[-1] < 1.0


def _wall_box(k=2, nq=3):
    m = omesh.BoxMesh((3, 2, 2), (0.0, -1.0, 0.0), (2 * math.pi, 1.0, math.pi), k, periodic=(True, False, True))
    fl = ph.Fluid(gamma=1.4, R=287.0, mu=0.01, lam=0.0, rho_ref=1.0)
    return ooperator.DGOperator(m, fl, nq, wall_T=300.0)


def _state(op, ufun, p=1.0e5):
    def f(x):
        u = np.zeros(x.shape)
        u[..., 0] = ufun(x[..., 1])
        return ph.conserved_from_primitive(torch.ones(x.shape[:-1], dtype=torch.float64), torch.as_tensor(u),
                                           torch.full(x.shape[:-1], p, dtype=torch.float64), op.fl)
    return initial.l2_project(op, f)


def _poiseuille_pin():
    op = _wall_box()
    tau, rho_w, area = odiag.channel_wall_shear(op, _state(op, lambda y: 3.0 * (1.0 - y ** 2)))
    return op, tau, rho_w, area


def test_wall_shear_of_poiseuille_and_couette_profiles():
    # the k = 2 space holds u = a (1 - y^2) and u = b (y + 1) exactly on an affine box:
    # Poiseuille has tau_w = 2 mu a at both walls, a linear (Couette) profile +mu b at the
    # lower and -mu b at the upper wall (the normal into the fluid flips), mean 0
    op, tau, rho_w, area = _poiseuille_pin()
    assert abs(tau - 2 * op.fl.mu * 3.0) < 1e-12 and abs(rho_w - 1.0) < 1e-13
    assert abs(area - 2 * (2 * math.pi) * math.pi) < 1e-12
    tau, _, _ = odiag.channel_wall_shear(op, _state(op, lambda y: 2.0 * (y + 1.0)))
    assert abs(tau) < 1e-13


def test_wall_shear_pin_detects_a_transposed_velocity_gradient(monkeypatch):
    # plant: du_j/dx_a in place of du_a/dx_j -- the shear then reads du_2/dx_1 = 0
    orig = ph.velocity_gradient
    monkeypatch.setattr(ph, "velocity_gradient", lambda U, G: orig(U, G).transpose(-1, -2))
    op, tau, _, _ = _poiseuille_pin()
    assert abs(tau - 2 * op.fl.mu * 3.0) > 0.5 * 2 * op.fl.mu * 3.0


def test_plus_statistics_of_one_laminar_sample():
    # one sample of the Poiseuille state: u_tau = sqrt(2 mu a), u+ = u / u_tau, no fluctuations
    op = _wall_box(k=2, nq=4)
    a = 3.0
    U = _state(op, lambda y: a * (1.0 - y ** 2))
    prof = odiag.channel_statistics(op, U)
    rows, u_tau = odiag.channel_plus_statistics([prof], [odiag.channel_wall_shear(op, U)], op.fl.nu, -1.0)
    assert abs(u_tau - math.sqrt(2 * op.fl.mu * a)) < 1e-12
    y = rows[:, 0]
    assert np.allclose(rows[:, 1], (y + 1.0) * u_tau / op.fl.nu, rtol=1e-13)
    assert np.allclose(rows[:, 2], a * (1.0 - y ** 2) / u_tau, rtol=1e-12)
    assert np.all(rows[:, 3:6] < 1e-5) and np.all(np.abs(rows[:, 6]) < 1e-10)
