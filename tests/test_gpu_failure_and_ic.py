"""GPU tests of the failure path of the diagnostics and of the perturbed channel state.

* A state holding a NaN (or one that has blown up past the stability limit of the
  explicit scheme, Sec. 5.2.2) makes dgns_diagnostics and dgns_kinetic_energy return
  DGNS_ENONFINITE and leave their host outputs untouched.  This is NaN arithmetic in
  ordinary kernels, not a fault.
* dgns_project_ic for the channel with a velocity perturbation (Sec. 5.3.1) against the
  oracle's projection followed by its perturbation, on the same seeded noise.
"""
import ctypes
import math

import pytest
import torch

import synth
from oracle import initial
from tests.gpu_cases import announce, make_pair, rel_err_fields, tgv_fluid, tgv_input

pytestmark = pytest.mark.gpu


def _cuda(t):
    return t.to("cuda").contiguous()


def test_nan_state_returns_enonfinite_and_leaves_outputs_untouched():
    announce("diagnostics and kinetic energy of a state with one NaN")
    from paper_1806_03095_amd import binding
    oop, gop = make_pair((3, 2, 2), 2, 4)
    U = _cuda(tgv_input(oop))
    U[1, 5, 3] = float("nan")
    torch.cuda.synchronize()
    lib, h = gop.lib, gop.h
    out8 = (ctypes.c_double * 8)(*([12345.0] * 8))
    rc = lib.dgns_diagnostics(h, ctypes.c_void_p(U.data_ptr()), None, out8)
    assert rc == binding.ENONFINITE, rc
    assert list(out8) == [12345.0] * 8
    ke = ctypes.c_double(777.0)
    rc = lib.dgns_kinetic_energy(h, ctypes.c_void_p(U.data_ptr()), ctypes.byref(ke))
    assert rc == binding.ENONFINITE, rc
    assert ke.value == 777.0
    d = gop.diagnostics(U)
    assert d["nonfinite"] and math.isnan(d["e_k"]) and "not finite" in d["error"]
    # the same state without the NaN is fine
    U[1, 5, 3] = 1.0
    assert not gop.diagnostics(U).get("nonfinite")


def test_blowup_past_the_stability_limit_is_flagged():
    announce("tgv 4^3 k=3 nq=6: Cr = 3 blows up and the diagnostics flag it; Cr = 0.3 stays finite")
    oop, gop = make_pair((4, 4, 4), 3, 6)
    U0 = gop.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
    work = torch.empty(2 * gop.n_dof, dtype=torch.float64, device="cuda")
    flagged = {}
    for Cr in (0.3, 3.0):
        dt = gop.compute_dt(Cr, 10.0, 1.5, 3.0, 1.0, 0.1)
        U = U0.clone()
        for s in range(20):
            gop.rk_step(U, work, s * dt, dt)
        torch.cuda.synchronize()
        flagged[Cr] = bool(gop.diagnostics(U).get("nonfinite"))
    assert flagged == {0.3: False, 3.0: True}, flagged


@pytest.mark.parametrize("basis", ["LGL", "GL"])
def test_channel_perturbed_projection_matches_oracle(basis):
    announce("channel 2x4x2 k=4 nq=7 %s: projected laminar state plus perturbation" % basis)
    fl = tgv_fluid(mu=1.0 / 180.0)
    umax, mach, amp = 18.3, 0.1, 0.1
    T0 = (umax / mach) ** 2 / (fl.gamma * fl.R)
    oop, gop = make_pair((2, 4, 2), 4, 7, lo=(0.0, -1.0, 0.0), hi=(2 * math.pi, 1.0, math.pi),
                         periodic=(1, 0, 1), kind="channel", fluid=fl, force=(1.0, 0.0, 0.0), wall_T=T0,
                         basis=basis)
    r = synth.uniform_pm1((3, gop.n_cells, gop.nodes_per_cell), 41)
    Ug = gop.project_ic("channel", [umax, mach, 2.0, amp], noise=_cuda(torch.as_tensor(r)))
    torch.cuda.synchronize()
    U = initial.l2_project(oop, lambda x: initial.channel_laminar(x, oop.fl, umax=umax, mach=mach))
    Uo = initial.channel_perturbed(oop, U, r, umax=umax, power=2, amp=amp)
    errs = rel_err_fields(Ug, Uo)
    print("perturbed channel state, per-field relative error:", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) < 1e-12, errs
