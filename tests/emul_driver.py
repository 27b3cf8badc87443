"""Runs the CPU emulation of the operator kernels (tests/emul) on given inputs."""
import ctypes
import hashlib
import os
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emul")
CSRC = os.path.join(ROOT, "paper_1806_03095_amd", "csrc")
BUILD = os.path.join(EMU, "_build")
CASES = [(1, 2), (2, 3), (3, 6), (4, 5), (4, 7), (7, 11)]
# degrees >= 8 (hd_impl.h): residual, operator and stand-alone inverse mass; k = 15 for the
# padded LDS rows of n_q = 16 and N = 16 in float64 (and the unpadded float32 ones)
HD_CASES = [(8, 9), (15, 16)]


def build():
    srcs = [os.path.join(EMU, "harness.cpp"), os.path.join(EMU, "hip", "hip_runtime.h"),
            os.path.join(CSRC, "setup.cpp"), os.path.join(CSRC, "setup.h"), os.path.join(CSRC, "op_impl.h"),
            os.path.join(CSRC, "adj_impl.h"), os.path.join(CSRC, "dg_adjoint.h"), os.path.join(CSRC, "diag_impl.h"),
            os.path.join(CSRC, "minv_impl.h"), os.path.join(CSRC, "hd_impl.h"),
            os.path.join(CSRC, "dg_common.h"), os.path.join(ROOT, "include", "dgns.h")]
    h = hashlib.sha1()
    for s in srcs:
        h.update(open(s, "rb").read())
    h.update(repr(CASES).encode())
    h.update(repr(HD_CASES).encode())
    exe = os.path.join(BUILD, "harness_" + h.hexdigest()[:12])
    if os.path.exists(exe):
        return exe
    os.makedirs(BUILD, exist_ok=True)
    cases = " ".join("EMU_CASE(%d,%d)" % kq for kq in CASES)
    hd_cases = " ".join("EMU_HD_CASE(%d,%d)" % kq for kq in HD_CASES)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", EMU, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-DEMU_CASES=" + cases, "-DEMU_HD_CASES=" + hd_cases, os.path.join(EMU, "harness.cpp"), os.path.join(CSRC, "setup.cpp"),
           "-o", exe + ".tmp%d" % os.getpid(), "-lpthread"]
    # a per-process temporary name: parallel test workers may build the same harness at once
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-4000:])
    os.replace(exe + ".tmp%d" % os.getpid(), exe)
    return exe


class _Params(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("n_q", ctypes.c_int), ("basis", ctypes.c_int),
                ("precision", ctypes.c_int), ("gamma", ctypes.c_double), ("R", ctypes.c_double),
                ("mu", ctypes.c_double), ("lambda_", ctypes.c_double), ("rho_ref", ctypes.c_double),
                ("body_force", ctypes.c_double * 3), ("wall_T", ctypes.c_double)]


class _Mesh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int * 3), ("kind", ctypes.c_int), ("stretch_C", ctypes.c_double),
                ("deform_amp", ctypes.c_double)]


def run(U, k, nq, n, lo, hi, periodic=(1, 1, 1), kind=0, basis=0, precision=0, gamma=1.4, R=287.0, mu=0.0,
        lam=0.0, rho_ref=1.0, force=(0, 0, 0), wall_T=0.0, amp=0.0, C=1.8, terms=7, fuse=0, Rbar=None):
    """fuse: 0 residual, 1 operator (with M^{-1}), 2 residual adjoint of Rbar, 3 standalone M^{-1} U,
    4 channel-statistics partial sums (returned as [n_cells, n_q, 9]), 5 wall-shear partial sums
    (returned as [2 n0 n2, 3]), 6 diagnostics partial sums of the streamed kernels (k >= 8) with
    Rbar as L (returned as [n_cells, 9])."""
    exe = build()
    p = _Params(k, nq, basis, precision, gamma, R, mu, lam, rho_ref, (ctypes.c_double * 3)(*force), wall_T)
    m = _Mesh((ctypes.c_int * 3)(*n), (ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi),
              (ctypes.c_int * 3)(*periodic), kind, C, amp)
    U = np.ascontiguousarray(U, dtype=np.float64)
    with tempfile.TemporaryDirectory() as td:
        fi, fo = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        with open(fi, "wb") as f:
            f.write(bytes(p))
            f.write(bytes(m))
            f.write(np.uint32(terms).tobytes())
            f.write(np.int32(fuse).tobytes())
            f.write(U.tobytes())
            if fuse in (2, 6):
                f.write(np.ascontiguousarray(Rbar, dtype=np.float64).tobytes())
        r = subprocess.run([exe, fi, fo], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("emulated kernel failed (%d):\n%s" % (r.returncode, r.stderr[-4000:]))
        out = np.fromfile(fo, dtype=np.float64)
        if fuse == 5:
            return out.reshape(-1, 3)
        if fuse == 6:
            return out.reshape(-1, 9)
        return out.reshape(-1, nq, 9) if fuse == 4 else out.reshape(U.shape)
