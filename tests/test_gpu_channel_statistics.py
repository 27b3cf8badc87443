"""GPU tests of the channel statistics pipeline (Sec. 5.3): the wall shear stress against
the oracle, and the time-averaged profiles in wall units (sampled while the solver advances
the channel with rk_step) against the same pipeline run with the oracle."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import diagnostics as odiag, initial, timeint
from tests.gpu_cases import announce, make_pair, tgv_fluid

pytestmark = pytest.mark.gpu
LO, HI = (0.0, -1.0, 0.0), (2 * math.pi, 1.0, math.pi)


def _cuda(t):
    return t.to("cuda").contiguous()


def _channel(k, nq, n=(2, 4, 2), kind="channel"):
    fl = tgv_fluid(mu=1.0 / 180.0)
    T0 = (18.3 / 0.1) ** 2 / (fl.gamma * fl.R)
    return make_pair(n, k, nq, lo=LO, hi=HI, periodic=(1, 0, 1), kind=kind, fluid=fl, force=(1.0, 0.0, 0.0),
                     wall_T=T0)


def _perturbed(oop, seed, amp=0.1):
    U = initial.l2_project(oop, lambda x: initial.channel_laminar(x, oop.fl))
    r = synth.uniform_pm1((3, oop.mesh.n_cells, oop.N), seed)
    return initial.channel_perturbed(oop, U, r, amp=amp)


@pytest.mark.parametrize("k,nq", [(4, 7), (3, 5)])
def test_wall_shear_matches_oracle(k, nq):
    announce("channel wall shear k=%d nq=%d" % (k, nq))
    oop, gop = _channel(k, nq)
    U = _perturbed(oop, seed=3)
    got = gop.channel_wall_shear(_cuda(U))
    want = odiag.channel_wall_shear(oop, U)
    print("wall shear gpu %s oracle %s" % (got, want), flush=True)
    for g, w in zip(got, want):
        assert abs(g - w) <= 1e-12 * abs(w), (got, want)


def test_wall_shear_of_poiseuille_flow_on_an_affine_box():
    # the k = 2 space holds u = a (1 - y^2) exactly: tau_w = 2 mu a at both walls
    announce("wall shear of a Poiseuille profile")
    oop, gop = _channel(2, 4, n=(3, 2, 2), kind="affine")
    a = 18.3
    U = initial.l2_project(oop, lambda x: initial.channel_laminar(x, oop.fl, umax=a))
    tau, rho_w, area = gop.channel_wall_shear(_cuda(U))
    assert abs(tau - 2 * oop.fl.mu * a) <= 1e-12 * 2 * oop.fl.mu * a, tau
    assert abs(rho_w - 1.0) <= 1e-13 and abs(area - 4 * math.pi ** 2) <= 1e-12 * area


def test_time_averaged_statistics_in_wall_units_match_the_oracle_pipeline():
    # the perturbed channel advanced 10 steps, sampled every 2nd step, on both sides
    announce("channel statistics pipeline: 10 steps, sampled every 2nd")
    oop, gop = _channel(2, 3)
    U0 = _perturbed(oop, seed=5)
    dt = gop.compute_dt(0.2, 0.1, 1.5, 3.0, 18.3, 0.1)
    Ug = _cuda(U0.clone())
    work = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    prof, sc = gop.run_channel_statistics(Ug, work, dt, 10, every=2)
    U = U0.clone()
    profiles, walls = [], []
    for s in range(1, 11):
        U = timeint.lsrk_step(lambda V, t: oop.apply(V), U, (s - 1) * dt, dt)
        if s % 2 == 0:
            profiles.append(odiag.channel_statistics(oop, U))
            walls.append(odiag.channel_wall_shear(oop, U))
    want, u_tau = odiag.channel_plus_statistics(profiles, walls, oop.fl.nu, LO[1])
    assert sc["samples"] == 5
    print("u_tau gpu %.15f oracle %.15f" % (sc["u_tau"], u_tau), flush=True)
    assert abs(sc["u_tau"] - u_tau) <= 1e-12 * u_tau
    assert prof.shape == want.shape
    for m in range(8):
        scale = np.abs(want[:, m]).max()
        err = np.abs(prof[:, m] - want[:, m]).max() / scale
        print("column %d: max error %.2e of scale %.3e" % (m, err, scale), flush=True)
        assert err <= 1e-10, (m, err)
    # rms and Reynolds stress are non-trivial: the perturbation is 10% of the laminar profile
    assert want[:, 3].max() > 0.1 and np.abs(want[:, 6]).max() > 1e-3


def test_statistics_pipeline_argument_errors():
    from paper_1806_03095_amd.binding import DgnsError
    oop, gop = _channel(2, 3)
    gop.channel_stats_reset()
    with pytest.raises(DgnsError):
        gop.channel_stats_result()             # no samples
    pop, pg = make_pair((2, 2, 2), 2, 3)
    with pytest.raises(DgnsError):
        pg.channel_wall_shear(_cuda(initial.l2_project(pop, lambda x: initial.taylor_green(x, pop.fl))))
