"""Float64 rounding floors measured against the extended-precision evaluation.

A float64 evaluation of the operator cannot be more accurate than its rounding allows,
and at low Mach number that floor is far above the unit roundoff: the momentum rows
cancel the background pressure p0 = 1/(gamma M^2) (71 at M = 0.1) against an O(1)
result, and the energy row cancels (rho E + p) u against its O(1) divergence.  These
helpers measure, per conserved field, the error of the oracle and of the HIP path
against tests/extended.py on the same float64 inputs, so that the parity bound of a
workload is a stated multiple of the oracle's own measured error rather than a guess.

Rule used by the parity tests (per field c, relative 2-norms over the compared cells):
    accuracy:  |gpu - ext| <= max(ACC_FACTOR * |oracle - ext|, ACC_MIN)
    parity:    |gpu - oracle| <= max(1e-12, (ACC_FACTOR + 1) * |oracle - ext|)
so the HIP path must be at least half as accurate as the oracle (measured in the CPU
emulation of the kernels: 2-10 times MORE accurate, since sum factorisation performs
fewer operations per result), and 1e-12 against the oracle is kept wherever the
oracle's own floor allows it.
"""
import numpy as np
import torch

from tests.extended import Extended, LD

ACC_FACTOR = 2.0
ACC_MIN = 2e-14
PARITY = 1e-12


def extended_for(oop):
    """The extended-precision evaluator of the same discretisation as the oracle operator oop."""
    m, fl = oop.mesh, oop.fl
    return Extended(m.n, tuple(float(v) for v in m.lo), tuple(float(v) for v in m.hi), m.k, oop.n_q,
                    basis=oop.basis, periodic=tuple(int(p) for p in m.periodic), kind=m.kind,
                    stretch_C=m.stretch_C, amp=m.deform_amp, gamma=fl.gamma, R=fl.R, mu=fl.mu, lam=fl.lam,
                    rho_ref=fl.rho_ref, wall_T=oop.wall_T,
                    body_force=None if oop.body_force is None else tuple(float(v) for v in oop.body_force))


def errs(a, ref, fields=range(5)):
    """Per-field |a - ref|_2 / |ref|_2 with ref in extended precision (a: (5, E, N))."""
    a = np.asarray(torch.as_tensor(a).cpu().numpy() if isinstance(a, torch.Tensor) else a, dtype=LD)
    return [float(np.linalg.norm((a[c] - ref[c]).ravel()) / np.linalg.norm(ref[c].ravel())) for c in fields]


def reference(oop, U, cells, what="L", terms="cvf"):
    """Extended-precision L (what='L') or R restricted to terms (what='R') on the given cells."""
    ext = extended_for(oop)
    U = U.numpy() if isinstance(U, torch.Tensor) else np.asarray(U)
    return ext.operator(U, cells) if what == "L" else ext.residual(U, cells, terms)


def reference_RL(oop, U, cells, terms="cvf"):
    """(R, L = M^{-1} R) in extended precision on the given cells, from one residual evaluation."""
    ext = extended_for(oop)
    U = U.numpy() if isinstance(U, torch.Tensor) else np.asarray(U)
    R = ext.residual(U, cells, terms)
    L = np.stack([ext.inverse_mass(int(e), R[:, i]) for i, e in enumerate(cells)], axis=1)
    return R, L


def reference_minv(oop, R, cells):
    """M^{-1} R in extended precision for the given cells; R: (5, len(cells), N) float64."""
    ext = extended_for(oop)
    R = R.numpy() if isinstance(R, torch.Tensor) else np.asarray(R)
    return np.stack([ext.inverse_mass(int(e), R[:, i]) for i, e in enumerate(cells)], axis=1)


def _fmt(v):
    return " ".join("%.1e" % x for x in v)


def check(got, ora, ref, what, sub=None, fields=range(5), acc_factor=ACC_FACTOR, acc_min=ACC_MIN,
          parity=PARITY):
    """Asserts the accuracy and parity rule above; returns (oracle floor, gpu error, parity) per field.

    got, ora: (5, E, N) on the compared cells; ref: the extended-precision values on the
    cells sub (indices into the E compared cells; all of them if None), where the floor
    and the accuracy are measured.  Parity is checked on all E cells."""
    fields = list(fields)
    g = torch.as_tensor(got).cpu().double()
    o = torch.as_tensor(ora).cpu().double()
    gs, os_ = (g, o) if sub is None else (g[:, sub], o[:, sub])
    e_ora = errs(os_, ref, fields)
    e_gpu = errs(gs, ref, fields)
    par = [float(torch.linalg.norm(g[c] - o[c]) / torch.linalg.norm(o[c])) for c in fields]
    print("%s (fields %s): oracle floor %s | gpu vs extended %s | gpu vs oracle %s"
          % (what, fields, _fmt(e_ora), _fmt(e_gpu), _fmt(par)), flush=True)
    for i, c in enumerate(fields):
        assert e_gpu[i] <= max(acc_factor * e_ora[i], acc_min), (what, "accuracy", c, e_gpu, e_ora)
        assert par[i] <= max(parity, (acc_factor + 1) * e_ora[i]), (what, "parity", c, par, e_ora)
    return e_ora, e_gpu, par


def oracle_floor(oop, U, cells=None, what="L", terms="cvf"):
    """The oracle's measured per-field error against the extended evaluation on `cells`."""
    cells = list(range(oop.mesh.n_cells)) if cells is None else list(cells)
    ref = reference(oop, U, cells, what, terms)
    ora = oop.apply(U, cells=cells) if what == "L" else oop.residual(U, cells=cells, terms=terms)
    return errs(ora, ref)
