"""Matched oracle / GPU setups for the parity tests.

The oracle builds its own mesh, geometry and operator from the same problem
statement; the only shared data are the input arrays: an oracle-projected
initial state plus seeded noise from the `synth` module.
"""
import math
import sys

import numpy as np
import torch

import synth
from oracle import initial, mesh as omesh, operator as ooperator, physics

TGV_MU = 1.0 / 1600.0
GAMMA, RGAS = 1.4, 287.0


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def tgv_fluid(mu=TGV_MU, Pr=0.71):
    return physics.Fluid(gamma=GAMMA, R=RGAS, mu=mu, lam=mu * GAMMA * RGAS / (GAMMA - 1) / Pr, rho_ref=1.0)


KIND = {"affine": omesh.AFFINE, "channel": omesh.CHANNEL, "curved": omesh.CURVED}


def make_pair(n, k, nq, lo=(-math.pi,) * 3, hi=(math.pi,) * 3, periodic=(1, 1, 1), kind="affine", amp=0.0,
              basis="LGL", precision="fp64", fluid=None, force=(0.0, 0.0, 0.0), wall_T=0.0):
    from paper_1806_03095_amd import Operator
    fl = fluid or tgv_fluid()
    om = omesh.BoxMesh(n, lo, hi, k, periodic=tuple(bool(p) for p in periodic), kind=KIND[kind],
                       deform_amp=amp, stretch_C=1.8)
    has_force = any(f != 0.0 for f in force)
    oop = ooperator.DGOperator(om, fl, nq, basis=basis, body_force=force if has_force else None,
                               wall_T=wall_T if not all(periodic) else None)
    gop = Operator(k, nq, n, lo, hi, periodic=periodic, kind=kind, basis=basis, precision=precision,
                   gamma=fl.gamma, R=fl.R, mu=fl.mu, lam=fl.lam, rho_ref=fl.rho_ref, body_force=force,
                   wall_T=wall_T, deform_amp=amp, stretch_C=1.8)
    return oop, gop


def tgv_input(oop, seed=2024, noise=1e-3, mach=0.1):
    """Oracle L2 projection of the Taylor-Green state (scaled to the box) plus seeded noise."""
    lo, hi = oop.mesh.lo, oop.mesh.hi

    def f(x):
        xs = (x - lo) / (hi - lo) * 2 * math.pi - math.pi
        return initial.taylor_green(xs, oop.fl, mach=mach)

    U = initial.l2_project(oop, f).numpy()
    return torch.as_tensor(synth.relative_noise(U, seed, noise))


def channel_input(oop, seed=7, noise=1e-2, umax=18.3, mach=0.1):
    U = initial.l2_project(oop, lambda x: initial.channel_laminar(x, oop.fl, umax=umax, mach=mach)).numpy()
    return torch.as_tensor(synth.relative_noise(U, seed, noise))


def rel_err_fields(a, b):
    """Per-field ||a - b||_2 / ||b||_2.  A field that is identically zero in b (rho w of the
    Taylor-Green state) is measured against the norm of the whole of b instead, so that it
    gives 0 when a's field is zero too and a finite error otherwise, never NaN."""
    a = torch.as_tensor(a, dtype=torch.float64).cpu()
    b = torch.as_tensor(b, dtype=torch.float64).cpu()
    whole = float(torch.linalg.norm(b))
    out = []
    for c in range(a.shape[0]):
        d, nb = float(torch.linalg.norm(a[c] - b[c])), float(torch.linalg.norm(b[c]))
        out.append(d / nb if nb > 0 else (d / whole if whole > 0 else d))
    return out


def sample_cells(n, count, seed):
    """Corner and edge cells of the box (periodic wrap-around) plus seeded random ones."""
    nx, ny, nz = n
    corners = [0, nx - 1, nx * (ny - 1), nx * ny - 1, nx * ny * (nz - 1), nx * ny * nz - 1]
    rng = synth.rng(seed)
    rest = rng.choice(nx * ny * nz, size=count, replace=False)
    return np.unique(np.concatenate([np.asarray(corners, dtype=np.int64), rest.astype(np.int64)]))


def patched_state(oop, cells, func, background, seed, noise):
    """Uniform `background` everywhere; oracle projection of func plus noise on
    `cells` and their face neighbours."""
    m = oop.mesh
    nbs = m.nb[cells].reshape(-1)
    need = np.unique(np.concatenate([cells, nbs[nbs >= 0]]))
    U = torch.empty(5, m.n_cells, oop.N, dtype=torch.float64)
    U[:] = torch.as_tensor(background, dtype=torch.float64)[:, None, None]
    P = initial.l2_project(oop, func, cells=need).numpy()
    U[:, need, :] = torch.as_tensor(synth.relative_noise(P, seed, noise))
    return U
