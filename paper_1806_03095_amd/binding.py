"""ctypes binding of libdgns.so (include/dgns.h): argument marshalling only.

Every computation runs in the HIP library; tensors are torch float64 CUDA tensors
used as device memory, and the library runs on torch's current stream unless a
stream is given.  There is no CPU fallback: if the library is missing or no GPU
is present, the calls raise.
"""

import ctypes
import math
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdgns.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ENONFINITE = 0, -1, -2, -3, -4, -5
BASIS = {"LGL": 0, "GL": 1}
PRECISION = {"fp64": 0, "fp32": 1}
MESH = {"affine": 0, "channel": 1, "curved": 2}
TERM_CONVECTIVE, TERM_VISCOUS, TERM_FORCE, TERM_ALL = 1, 2, 4, 7
IC = {"taylor_green": 0, "channel": 1, "uniform": 2}


class DgnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dgns error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("n_q", ctypes.c_int), ("basis", ctypes.c_int),
                ("precision", ctypes.c_int), ("gamma", ctypes.c_double), ("R", ctypes.c_double),
                ("mu", ctypes.c_double), ("lambda_", ctypes.c_double), ("rho_ref", ctypes.c_double),
                ("body_force", ctypes.c_double * 3), ("wall_T", ctypes.c_double)]


class BoxMesh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int * 3), ("kind", ctypes.c_int), ("stretch_C", ctypes.c_double),
                ("deform_amp", ctypes.c_double)]


EXPORTS = ["dgns_last_error", "dgns_create", "dgns_destroy", "dgns_sizes", "dgns_set_stream",
           "dgns_apply_residual", "dgns_apply_inverse_mass", "dgns_apply_operator", "dgns_rk_step",
           "dgns_rk_stage_update", "dgns_compute_dt", "dgns_channel_statistics", "dgns_diagnostics",
           "dgns_diagnostics_noalloc", "dgns_project_ic", "dgns_apply_residual_vjp",
           "dgns_apply_operator_vjp", "dgns_rk_step_vjp", "dgns_kinetic_energy", "dgns_kinetic_energy_vjp",
           "dgns_set_rk_scheme", "dgns_get_rk_scheme", "dgns_channel_wall_shear", "dgns_channel_stats_reset",
           "dgns_channel_stats_sample", "dgns_channel_stats_result"]

_lib = None


def load_library(path=LIB_PATH):
    """Loads libdgns.so and declares the prototypes; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libdgns.so is not built (%s); run python -m paper_1806_03095_amd.build" % path)
    lib = ctypes.CDLL(path)
    vp, dp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
    lib.dgns_last_error.restype = ctypes.c_char_p
    lib.dgns_last_error.argtypes = []
    lib.dgns_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(BoxMesh), vp, ctypes.POINTER(vp)]
    lib.dgns_destroy.argtypes = [vp]
    lib.dgns_sizes.argtypes = [vp, i64p, i64p, i64p]
    lib.dgns_set_stream.argtypes = [vp, vp]
    lib.dgns_apply_residual.argtypes = [vp, vp, vp, ctypes.c_uint]
    lib.dgns_apply_inverse_mass.argtypes = [vp, vp, vp]
    lib.dgns_apply_operator.argtypes = [vp, vp, vp, ctypes.c_double]
    lib.dgns_rk_step.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double]
    lib.dgns_rk_stage_update.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_double]
    lib.dgns_channel_statistics.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.dgns_compute_dt.argtypes = [vp] + [ctypes.c_double] * 6 + [dp]
    lib.dgns_diagnostics.argtypes = [vp, vp, vp, dp]
    lib.dgns_diagnostics_noalloc.argtypes = [vp, vp, vp, vp]
    lib.dgns_project_ic.argtypes = [vp, ctypes.c_int, dp, vp, vp]
    lib.dgns_apply_residual_vjp.argtypes = [vp, vp, vp, vp, ctypes.c_uint]
    lib.dgns_apply_operator_vjp.argtypes = [vp, vp, vp, vp]
    lib.dgns_rk_step_vjp.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp]
    lib.dgns_kinetic_energy.argtypes = [vp, vp, dp]
    lib.dgns_kinetic_energy_vjp.argtypes = [vp, vp, vp]
    lib.dgns_set_rk_scheme.argtypes = [vp, ctypes.c_int, dp, dp, dp]
    lib.dgns_channel_wall_shear.argtypes = [vp, vp, dp]
    lib.dgns_channel_stats_reset.argtypes = [vp]
    lib.dgns_channel_stats_sample.argtypes = [vp, vp]
    lib.dgns_channel_stats_result.argtypes = [vp, dp, dp]
    lib.dgns_get_rk_scheme.argtypes = [vp, ctypes.POINTER(ctypes.c_int), dp, dp, dp]
    for name in EXPORTS:
        if name != "dgns_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise DgnsError(rc, _lib.dgns_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Operator:
    """One discretisation (degree, n_q, basis, precision, fluid) on one box mesh.

    Vectors are float64 CUDA tensors of shape (5, n_cells, (k+1)^3).
    """

    def __init__(self, degree, n_q, n, lo, hi, periodic=(1, 1, 1), kind="affine", basis="LGL",
                 precision="fp64", gamma=1.4, R=287.0, mu=0.0, lam=0.0, rho_ref=1.0,
                 body_force=(0.0, 0.0, 0.0), wall_T=0.0, stretch_C=1.8, deform_amp=0.0, stream=None):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the DG operator runs on the GPU only; no GPU is visible")
        self.lib = lib
        self.degree, self.n_q = int(degree), int(n_q)
        self.n = tuple(int(v) for v in n)
        p = Params(self.degree, self.n_q, BASIS[basis], PRECISION[precision], gamma, R, mu, lam, rho_ref,
                   (ctypes.c_double * 3)(*body_force), wall_T)
        m = BoxMesh((ctypes.c_int * 3)(*n), (ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi),
                    (ctypes.c_int * 3)(*[int(bool(v)) for v in periodic]), MESH[kind], stretch_C, deform_amp)
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib.dgns_create(ctypes.byref(p), ctypes.byref(m), self._stream_handle(), ctypes.byref(h)))
        self.h = h
        ne, nn, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.dgns_sizes(self.h, ctypes.byref(ne), ctypes.byref(nn), ctypes.byref(nd)))
        self.n_cells, self.nodes_per_cell, self.n_dof = ne.value, nn.value, nd.value
        self.shape = (5, self.n_cells, self.nodes_per_cell)
        self.mu = mu

    def _stream_handle(self):
        s = self._stream if self._stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def _bind(self):
        _check(self.lib.dgns_set_stream(self.h, self._stream_handle()))

    def _vec(self, t, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("%s must be a contiguous float64 CUDA tensor" % name)
        if t.numel() != self.n_dof:
            raise ValueError("%s has %d entries, expected %d" % (name, t.numel(), self.n_dof))
        return t

    def empty(self):
        return torch.empty(self.shape, dtype=torch.float64, device="cuda")

    def close(self):
        if getattr(self, "h", None):
            self.lib.dgns_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operators ---------------------------------------------------------
    def apply(self, U, out=None, t=0.0):
        """L = M^{-1}(-F_c - F_v + F_rhs)(U)."""
        self._vec(U, "U")
        out = self.empty() if out is None else self._vec(out, "out")
        self._bind()
        _check(self.lib.dgns_apply_operator(self.h, _ptr(U), _ptr(out), t))
        return out

    def residual(self, U, out=None, terms=TERM_ALL):
        """R = -F_c - F_v + F_rhs before the inverse mass matrix, restricted to `terms`."""
        self._vec(U, "U")
        out = self.empty() if out is None else self._vec(out, "out")
        self._bind()
        _check(self.lib.dgns_apply_residual(self.h, _ptr(U), _ptr(out), terms))
        return out

    def inverse_mass(self, R, out=None):
        self._vec(R, "R")
        out = self.empty() if out is None else self._vec(out, "out")
        self._bind()
        _check(self.lib.dgns_apply_inverse_mass(self.h, _ptr(R), _ptr(out)))
        return out

    def rk_step(self, U, work, t, dt):
        """One 5-stage 2N Runge-Kutta step in place; work holds >= 2 n_dof doubles."""
        self._vec(U, "U")
        if not (work.is_cuda and work.dtype == torch.float64 and work.is_contiguous() and work.numel() >= 2 * self.n_dof):
            raise ValueError("work must be a contiguous float64 CUDA tensor of >= 2 n_dof entries")
        self._bind()
        _check(self.lib.dgns_rk_step(self.h, _ptr(U), _ptr(work), t, dt))
        return U

    def set_rk_scheme(self, A=None, B=None, c=None):
        """Sets the 2N Runge-Kutta scheme (Williamson form; A[0] = 0) used by rk_step and its
        adjoint; no arguments restore the default five-stage fourth-order scheme."""
        if A is None and B is None:
            _check(self.lib.dgns_set_rk_scheme(self.h, 0, None, None, None))
            return
        s = len(A)
        arr = lambda v: (ctypes.c_double * s)(*[float(x) for x in v])
        _check(self.lib.dgns_set_rk_scheme(self.h, s, arr(A), arr(B), None if c is None else arr(c)))

    def rk_scheme(self):
        """(A, B, c) of the scheme in use."""
        s = ctypes.c_int()
        A, B, c = ((ctypes.c_double * 16)() for _ in range(3))
        _check(self.lib.dgns_get_rk_scheme(self.h, ctypes.byref(s), A, B, c))
        n = s.value
        return list(A)[:n], list(B)[:n], list(c)[:n]

    def channel_statistics(self, U):
        """Plane averages at the wall-normal Gauss points: a (n[1] * n_q, 9) numpy array with
        columns y, rho, u, v, w, uu, vv, ww, uv (rows by cell row, then point)."""
        import numpy as np
        self._vec(U, "U")
        self._bind()
        out = np.empty((self.n[1] * self.n_q, 9), dtype=np.float64)
        _check(self.lib.dgns_channel_statistics(self.h, _ptr(U), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def channel_wall_shear(self, U):
        """(tau_w, rho_w, wall area): the mean wall shear stress over both walls in x2."""
        self._vec(U, "U")
        self._bind()
        out = (ctypes.c_double * 3)()
        _check(self.lib.dgns_channel_wall_shear(self.h, _ptr(U), out))
        return tuple(out)

    def channel_stats_reset(self):
        _check(self.lib.dgns_channel_stats_reset(self.h))

    def channel_stats_sample(self, U):
        self._vec(U, "U")
        self._bind()
        _check(self.lib.dgns_channel_stats_sample(self.h, _ptr(U)))

    def channel_stats_result(self):
        """Time-averaged profiles: a (n[1] * n_q, 8) numpy array with columns y, y+, u+, rms u+,
        rms v+, rms w+, <u'v'>+, <rho>, and dict(u_tau, tau_w, rho_w, samples)."""
        import numpy as np
        prof = np.empty((self.n[1] * self.n_q, 8), dtype=np.float64)
        sc = (ctypes.c_double * 4)()
        _check(self.lib.dgns_channel_stats_result(self.h, prof.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sc))
        return prof, dict(u_tau=sc[0], tau_w=sc[1], rho_w=sc[2], samples=int(sc[3]))

    def run_channel_statistics(self, U, work, dt, steps, every=10, t0=0.0):
        """Advances U by `steps` RK steps and samples the channel statistics every `every`-th
        step (Sec. 5.3 samples every 10th); returns channel_stats_result()."""
        self.channel_stats_reset()
        t = t0
        for s in range(1, steps + 1):
            self.rk_step(U, work, t, dt)
            t += dt
            if s % every == 0:
                self.channel_stats_sample(U)
        return self.channel_stats_result()

    def rk_graph(self, U, work, dt, steps=1):
        """Captures `steps` rk_step calls on U (in place, work as in rk_step) into a HIP
        graph (torch.cuda.CUDAGraph): each replay() advances U by `steps` steps with one
        launch from the host.  U and work must stay allocated while the graph is used."""
        self._vec(U, "U")
        if not (work.is_cuda and work.dtype == torch.float64 and work.is_contiguous() and work.numel() >= 2 * self.n_dof):
            raise ValueError("work must be a contiguous float64 CUDA tensor of >= 2 n_dof entries")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for s in range(int(steps)):
                self.rk_step(U, work, s * dt, dt)
        return g

    def rk_stage_update(self, U, dU, L, stage, dt):
        """The stage-`stage` vector update alone: dU <- A dU + dt L, U <- U + B dU (in place)."""
        for t, name in ((U, "U"), (dU, "dU"), (L, "L")):
            self._vec(t, name)
        self._bind()
        _check(self.lib.dgns_rk_stage_update(self.h, _ptr(U), _ptr(dU), _ptr(L), int(stage), dt))
        return U

    def compute_dt(self, Cr, D, e, f, umax, mach):
        out = ctypes.c_double()
        _check(self.lib.dgns_compute_dt(self.h, Cr, D, e, f, umax, mach, ctypes.byref(out)))
        return out.value

    def diagnostics(self, U, L=None):
        """e_k, eps, -de_k/dt (nan without L), mass, momentum (3), energy.

        A state with a NaN or Inf anywhere in these integrals (a blown-up run) does not
        raise: the library reports DGNS_ENONFINITE and writes nothing, and the result is
        then all NaN with nonfinite=True and the library's message under "error"."""
        self._vec(U, "U")
        if L is not None:
            self._vec(L, "L")
        out = (ctypes.c_double * 8)(*([math.nan] * 8))
        self._bind()
        rc = self.lib.dgns_diagnostics(self.h, _ptr(U), _ptr(L), out)
        vals = list(out)
        res = dict(e_k=vals[0], eps=vals[1], rate=vals[2], mass=vals[3], mom=vals[4:7], energy=vals[7])
        if rc == ENONFINITE:
            res["nonfinite"] = True
            res["error"] = self.lib.dgns_last_error().decode()
            return res
        _check(rc)
        return res

    def diagnostics_noalloc(self, U, out, L=None):
        """The diagnostics into out, a float64 CUDA tensor of 8 entries, asynchronously and
        without any allocation (the library's static workspace; meshes up to 64^3 cells)."""
        self._vec(U, "U")
        if L is not None:
            self._vec(L, "L")
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == 8):
            raise ValueError("out must be a contiguous float64 CUDA tensor of 8 entries")
        self._bind()
        _check(self.lib.dgns_diagnostics_noalloc(self.h, _ptr(U), _ptr(L), _ptr(out)))
        return out

    # -- adjoint -------------------------------------------------------------
    def residual_vjp(self, U, Rbar, out=None, terms=TERM_ALL):
        """Ubar = (dR/dU)^T Rbar for the residual restricted to `terms`."""
        self._vec(U, "U")
        self._vec(Rbar, "Rbar")
        out = self.empty() if out is None else self._vec(out, "out")
        self._bind()
        _check(self.lib.dgns_apply_residual_vjp(self.h, _ptr(U), _ptr(Rbar), _ptr(out), terms))
        return out

    def operator_vjp(self, U, Lbar, out=None):
        """Ubar = (dL/dU)^T Lbar."""
        self._vec(U, "U")
        self._vec(Lbar, "Lbar")
        out = self.empty() if out is None else self._vec(out, "out")
        self._bind()
        _check(self.lib.dgns_apply_operator_vjp(self.h, _ptr(U), _ptr(Lbar), _ptr(out)))
        return out

    def rk_step_vjp(self, U_n, t, dt, Ubar_np1, out=None, work=None):
        """Ubar_n = (dU_{n+1}/dU_n)^T Ubar_{n+1} for one rk_step from U_n (out may be Ubar_np1)."""
        self._vec(U_n, "U_n")
        self._vec(Ubar_np1, "Ubar_np1")
        out = self.empty() if out is None else self._vec(out, "out")
        nw = (len(self.rk_scheme()[0]) + 4) * self.n_dof
        if work is None:
            work = torch.empty(nw, dtype=torch.float64, device="cuda")
        elif not (work.is_cuda and work.dtype == torch.float64 and work.is_contiguous() and work.numel() >= nw):
            raise ValueError("work must be a contiguous float64 CUDA tensor of >= (stages + 4) n_dof entries")
        self._bind()
        _check(self.lib.dgns_rk_step_vjp(self.h, _ptr(U_n), t, dt, _ptr(Ubar_np1), _ptr(out), _ptr(work)))
        return out

    def kinetic_energy(self, U):
        """int |u|^2/2 over the domain (host float)."""
        self._vec(U, "U")
        out = ctypes.c_double()
        self._bind()
        _check(self.lib.dgns_kinetic_energy(self.h, _ptr(U), ctypes.byref(out)))
        return out.value

    def kinetic_energy_vjp(self, U, out=None):
        self._vec(U, "U")
        out = self.empty() if out is None else self._vec(out, "out")
        self._bind()
        _check(self.lib.dgns_kinetic_energy_vjp(self.h, _ptr(U), _ptr(out)))
        return out

    def project_ic(self, kind, params, noise=None, out=None):
        out = self.empty() if out is None else self._vec(out, "out")
        if noise is not None:
            if not (noise.is_cuda and noise.dtype == torch.float64 and noise.is_contiguous()
                    and noise.numel() == 3 * self.n_cells * self.nodes_per_cell):
                raise ValueError("noise must be float64 CUDA of shape (3, n_cells, nodes)")
        arr = (ctypes.c_double * 8)(*([float(v) for v in params] + [0.0] * (8 - len(params))))
        self._bind()
        _check(self.lib.dgns_project_ic(self.h, IC[kind], arr, _ptr(noise), _ptr(out)))
        return out


def taylor_green(degree, n_cells_1d, n_q=None, precision="fp64", basis="LGL", Re=1600.0, Pr=0.71,
                 mach=0.1, gamma=1.4, R=287.0, **kw):
    """The Taylor-Green vortex setup of the paper's Sec. 5.2.1 on [-pi, pi]^3."""
    mu = 1.0 / Re
    lam = mu * gamma * R / (gamma - 1.0) / Pr
    n_q = n_q if n_q is not None else (3 * degree + 2) // 2
    n = (n_cells_1d,) * 3 if isinstance(n_cells_1d, int) else tuple(n_cells_1d)
    op = Operator(degree, n_q, n, (-math.pi,) * 3, (math.pi,) * 3, basis=basis, precision=precision,
                  gamma=gamma, R=R, mu=mu, lam=lam, **kw)
    op.mach = mach
    return op
