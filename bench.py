"""Throughput of the DG compressible Navier-Stokes operator on one MI355X.

Workload (default): Taylor-Green vortex on [-pi, pi]^3, 32^3 affine cells,
degree k = 3 (LGL nodes), n_q = 6 Gauss points per direction (over-integration),
10,485,760 float64 DoFs, Ma = 0.1, Re = 1600, Pr = 0.71.  One step = one time step
of the five-stage 2N Runge-Kutta scheme: five evaluations of L = M^{-1}(-F_c - F_v)
(each a face kernel that evaluates every face once and lifts both sides, then the cell
kernel: cell terms, the gathered face terms, inverse mass matrix, and in stages 1-4 the
stage update) and the fifth stage's update.
The reported value is DoFs processed per second per operator evaluation,
N_dof * stages * steps / time, with the inputs resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.  Extra keys: the float32-operator variant's throughput and
dissipation-rate error, the operator kernel alone, its HBM fraction and the
roofline of the dominant kernel, and the oracle timed on host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoFs/s per DG operator eval (TGV k=3, 32^3 cells) FP64 vs FP32; % HBM roofline"
PEAK_FP64_VALU = 78.6e12        # MI355X FP64 vector, FLOP/s
PEAK_HBM = 8.0e12               # MI355X HBM3E, B/s
# Algorithmic work of one evaluation of L per DoF (k=3, n_q=6): sum factorisation
# without even-odd splitting, faces counted once, ~280 flop per cell point and
# ~700 per face point; and the compulsory traffic, read U + write L.
FLOP_PER_DOF = {(3, 6): 1197.0, (3, 5): 769.0, (3, 4): 474.0, (4, 7): 1049.0, (5, 8): 976.0, (7, 11): 1178.0}
BYTES_PER_DOF = 16.0
# HBM bytes of one evaluation of L (its face-kernel and cell-kernel launches) from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE), scaled by what the counters read for a
# plain copy of known size; valid only for the kernel source they were taken on.
# Critical Courant and diffusion numbers of the five-stage scheme (eq.
# TimeStepRestrictions_Compressible with e = 1.5, f = 3), measured on MI355X with
# `bench.py --critical-cfl` the way Sec. 5.2.2 determines them (largest stable value, Taylor-
# Green at effective resolution 60^3 / 64^3, Re = 1600 to t_f = 20 for Cr, Re = 1 to t_f = 1
# for D; resolution 0.02 and 0.002): k -> (Cr stable, D stable).
CRITICAL = {2: (0.36, 0.018), 3: (0.40, 0.020), 5: (0.42, 0.020), 7: (0.40, 0.018)}
# The runs use the paper's ratio of the Courant number to the critical one (Cr = 0.5
# against 0.74 at k = 3 for its scheme, 0.68): 0.68 x 0.40 = 0.27 at k = 3; the precision
# study at k = 5 and 7 uses 0.25 (0.6 of the critical 0.42 / 0.40).
CR = 0.27
CR_STUDY = 0.25
# diffusion number: the paper's ratio to the critical one (D = 0.02 against 0.036), 0.56 x 0.020;
# at Re = 1600 the viscous restriction does not bind either way
D_RUN = 0.011
MEASURED_TRAFFIC = {"fingerprint": "3e8cab51b4fc250f", "workload": (32, 3, 6), "bytes": 862688972.8}


def kernel_fingerprint():
    """sha1 (first 16 hex digits) of the operator kernel's sources with comments and
    blank lines removed, so that a comment edit does not invalidate the measurement."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in ("op_impl.h", "dg_common.h"):
        text = open(os.path.join(ROOT, "paper_1806_03095_amd", "csrc", f)).read()
        for line in text.split("\n"):
            code = re.sub(r"//.*$", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_rk(op, U, work, dt, steps, warmup):
    import torch
    t = 0.0
    for _ in range(warmup):
        op.rk_step(U, work, t, dt)
        t += dt
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        op.rk_step(U, work, t, dt)
        t += dt
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return e0.elapsed_time(e1) / 1e3, wall


def time_operator(op, U, L, calls):
    import torch
    for _ in range(5):
        op.apply(U, L)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(calls):
        op.apply(U, L)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / calls


def time_call(fn, calls, warm_s=0.0):
    """Average seconds per call of fn() (HIP events on the current stream), after three
    untimed calls and, with warm_s > 0, further untimed calls for at least warm_s seconds
    (a GPU coming out of idle runs its first tens of milliseconds of streaming kernels up
    to 12% slower)."""
    import torch
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(calls):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / calls


def copy_bandwidth(mib=1024, calls=20):
    """Measured device-to-device copy rate in B/s (read + write bytes per second)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    t = time_call(lambda: b.copy_(a), calls, warm_s=0.1)
    return 2 * 8 * n / t


def operations(op, U, t_op, t_step, calls):
    """The paper's six operations timed separately (per launch): F_c, F_v, F (all
    terms, before M^{-1}), M^{-1}, the Runge-Kutta vector update, and L."""
    import torch
    ndof = op.n_dof
    R = torch.empty_like(U)
    out = {}
    for name, mask in (("F_c", 1), ("F_v", 2), ("F", 7)):
        t = time_call(lambda: op.residual(U, R, terms=mask), calls)
        out[name] = {"us": 1e6 * t, "dofs_per_s": ndof / t}
    t = time_call(lambda: op.inverse_mass(U, R), calls)
    out["M_inv"] = {"us": 1e6 * t, "dofs_per_s": ndof / t, "hbm_frac": 16 * ndof / t / PEAK_HBM}
    # the stand-alone stage update (read L, dU, U; write dU, U) on scratch copies
    Uc, dU = U.clone(), torch.zeros_like(U)
    t_upd = time_call(lambda: op.rk_stage_update(Uc, dU, R, 1, 1e-12), calls)
    out["rk_update"] = {"us": 1e6 * t_upd, "hbm_frac": 40 * ndof / t_upd / PEAK_HBM,
                        "in_step_us_per_stage": 1e6 * (t_step / 5.0 - t_op),
                        "note": "stand-alone stage update; inside rk_step stages 1-4 fuse it into the operator "
                                "kernel, and in_step_us_per_stage is the step time / 5 minus one operator launch"}
    del Uc, dU
    out["L"] = {"us": 1e6 * t_op, "dofs_per_s": ndof / t_op}
    return out


def channel_throughput(calls):
    """Operator throughput on the stretched channel of 16^3 cells, k=4, n_q=7 (per-point metric)."""
    import torch
    from paper_1806_03095_amd import Operator
    mu, gamma, R, Pr = 1.0 / 180.0, 1.4, 287.0, 0.71
    umax, mach = 18.3, 0.1
    T0 = (umax / mach) ** 2 / (gamma * R)
    res = {}
    for prec in ("fp64", "fp32"):
        op = Operator(4, 7, (16, 16, 16), (0.0, -1.0, 0.0), (2 * math.pi, 1.0, math.pi), periodic=(1, 0, 1),
                      kind="channel", precision=prec, gamma=gamma, R=R, mu=mu,
                      lam=mu * gamma * R / (gamma - 1) / Pr, body_force=(1.0, 0.0, 0.0), wall_T=T0)
        U = op.project_ic("channel", [umax, mach, 2.0, 0.0])
        L = torch.empty_like(U)
        t = time_call(lambda: op.apply(U, L), calls)
        res[prec] = {"us": 1e6 * t, "dofs_per_s": op.n_dof / t}
        if prec == "fp64":
            # wall-normal statistics profile (synchronous call: host wall time)
            op.channel_statistics(U)
            w0 = time.perf_counter()
            for _ in range(10):
                st = op.channel_statistics(U)
            res["statistics_us_per_call"] = 1e6 * (time.perf_counter() - w0) / 10
            res["statistics_points"] = int(st.shape[0])
        op.close()
    res["workload"] = "channel_16cubed_k4_nq7_tanh1.8"
    return res


def graph_timing(steps=50):
    """RK steps on the small Taylor-Green meshes (4^3 and 8^3 cells, k=3, n_q=6), launched
    eagerly from Python one rk_step at a time and as one HIP graph of `steps` steps: on
    meshes this small the host-side launch cost, not the kernels, sets the step rate."""
    import torch
    from paper_1806_03095_amd import taylor_green
    res = {}
    for ne in (4, 8):
        op = taylor_green(3, ne, 6)
        U = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
        work = torch.empty(2 * op.n_dof, dtype=torch.float64, device="cuda")
        dt = op.compute_dt(CR, D_RUN, 1.5, 3.0, 1.0, 0.1)
        t_eager, _ = time_rk(op, U, work, dt, steps, 5)
        g = op.rk_graph(U, work, dt, steps)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        t_graph = e0.elapsed_time(e1) / 1e3
        res["taylor_green_%dcubed_k3_nq6" % ne] = {"n_dof": op.n_dof, "eager_us_per_step": 1e6 * t_eager / steps,
                                                   "graph_us_per_step": 1e6 * t_graph / steps}
        del g
        op.close()
    return res


def adjoint_timing():
    """The differentiation workload: gradient of the kinetic energy after 50 RK steps
    with respect to the initial state (Taylor-Green 16^3 cells, k=3, n_q=6, float64),
    checkpoints every 10 steps; forward and backward wall time, and the operator VJP
    against the operator on the same mesh."""
    import torch
    from paper_1806_03095_amd import taylor_green
    from paper_1806_03095_amd.autograd import kinetic_energy, rk_rollout
    op = taylor_green(3, 16, n_q=6)
    U0 = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
    dt = op.compute_dt(CR, D_RUN, 1.5, 3.0, 1.0, 0.1)
    L = torch.empty_like(U0)
    t_op = time_call(lambda: op.apply(U0, L), 20)
    Ub = torch.empty_like(U0)
    t_vjp = time_call(lambda: op.operator_vjp(U0, L, out=Ub), 20)
    x = U0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    K = kinetic_energy(rk_rollout(x, op, 50, dt, ckpt_every=10), op)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    (g,) = torch.autograd.grad(K, x)
    torch.cuda.synchronize()
    w2 = time.perf_counter()
    return {"workload": "taylor_green_16cubed_k3_nq6_50steps_ckpt10", "n_dof": op.n_dof,
            "forward_s": w1 - w0, "backward_s": w2 - w1, "backward_over_forward": (w2 - w1) / (w1 - w0),
            "operator_us": 1e6 * t_op, "operator_vjp_us": 1e6 * t_vjp, "vjp_over_operator": t_vjp / t_op,
            "grad_finite": bool(torch.isfinite(g).all())}


def degree_sweep(target_dofs=10_000_000, calls=20):
    """Operator throughput over every compiled (k, n_q), float64 and float32, on
    Taylor-Green meshes of about target_dofs DoFs (the mesh size n^3 with n the
    nearest integer to (target_dofs / (5 (k+1)^3))^(1/3)); also F_c, F_v and M^{-1}
    separately (the paper's operation breakdown); and L on the same mesh deformed
    by the sinusoidal warp (amplitude 0.1 h), where the metric is read per
    quadrature point (the paper's Cartesian versus deformed comparison, Sec. 5.1.1)."""
    import torch
    from paper_1806_03095_amd import taylor_green
    qs = {1: (2, 3), 2: (3, 4, 5), 3: (4, 5, 6, 7), 4: (5, 6, 7, 9), 5: (6, 8), 6: (7, 10), 7: (8, 11),
          8: (9, 13), 9: (10, 14), 10: (11, 16), 11: (12,), 12: (13,), 13: (14,), 14: (15,), 15: (16,)}
    rows = []
    for k, nqs in qs.items():
        ne = max(2, int(round((target_dofs / (5.0 * (k + 1) ** 3)) ** (1.0 / 3.0))))
        for nq in nqs:
            row = {"k": k, "n_q": nq, "cells": ne ** 3}
            for prec, mesh in (("fp64", "affine"), ("fp32", "affine"), ("fp64", "curved"), ("fp32", "curved")):
                kw = {} if mesh == "affine" else {"kind": "curved", "deform_amp": 0.1 * 2 * math.pi / ne}
                op = taylor_green(k, ne, n_q=nq, precision=prec, **kw)
                U = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
                L = torch.empty_like(U)
                t = time_call(lambda: op.apply(U, L), calls)
                row["n_dof"] = op.n_dof
                tag = prec if mesh == "affine" else prec + "_deformed"
                row[tag + "_L_dofs_per_s"] = op.n_dof / t
                if prec == "fp64" and mesh == "affine":
                    for name, mask in (("F_c", 1), ("F_v", 2), ("F", 7)):
                        tt = time_call(lambda: op.residual(U, L, terms=mask), calls)
                        row["fp64_%s_dofs_per_s" % name] = op.n_dof / tt
                    tt = time_call(lambda: op.inverse_mass(U, L), calls)
                    row["fp64_M_inv_dofs_per_s"] = op.n_dof / tt
                    Uc, dU = U.clone(), torch.zeros_like(U)
                    tt = time_call(lambda: op.rk_stage_update(Uc, dU, L, 1, 1e-12), calls)
                    row["fp64_rk_update_dofs_per_s"] = op.n_dof / tt
                    del Uc, dU
                op.close()
            log("k=%d n_q=%d %d^3: L fp64 %.3e fp32 %.3e, deformed fp64 %.3e fp32 %.3e DoF/s"
                % (k, nq, ne, row["fp64_L_dofs_per_s"], row["fp32_L_dofs_per_s"],
                   row["fp64_deformed_L_dofs_per_s"], row["fp32_deformed_L_dofs_per_s"]))
            rows.append(row)
    return rows


def memops_streamed(calls=20):
    """The memory-bound operations with vectors far beyond the 256 MB last-level cache:
    M^{-1} (16 B/DoF) and the stand-alone Runge-Kutta stage update (40 B/DoF) on Taylor-Green
    meshes of about 80M DoFs (k = 3: 64^3 cells, 671 MB per vector; k = 4: 50^3; k = 5:
    42^3), as fractions of the 8 TB/s HBM peak and of a measured device copy."""
    import torch
    from paper_1806_03095_amd import taylor_green
    bw = copy_bandwidth(2048, 10)
    rows = []
    for k, ne in ((3, 64), (4, 50), (5, 42)):
        op = taylor_green(k, ne)
        U = torch.rand(op.shape, dtype=torch.float64, device="cuda") + 1.0
        L = torch.empty_like(U)
        t_m = time_call(lambda: op.inverse_mass(U, L), calls, warm_s=0.1)
        dU = torch.zeros_like(U)
        t_u = time_call(lambda: op.rk_stage_update(U, dU, L, 1, 1e-12), calls, warm_s=0.1)
        row = {"k": k, "cells": ne ** 3, "n_dof": op.n_dof, "vector_MB": 8e-6 * op.n_dof,
               "M_inv_us": 1e6 * t_m, "M_inv_hbm_frac": 16 * op.n_dof / t_m / PEAK_HBM,
               "M_inv_frac_of_copy": 16 * op.n_dof / t_m / bw,
               "rk_update_us": 1e6 * t_u, "rk_update_hbm_frac": 40 * op.n_dof / t_u / PEAK_HBM,
               "rk_update_frac_of_copy": 40 * op.n_dof / t_u / bw}
        log("streamed k=%d %d^3 (%.0f MB/vector): M^-1 %.1f us (%.0f%% of HBM peak), update %.1f us (%.0f%%)"
            % (k, ne, row["vector_MB"], row["M_inv_us"], 100 * row["M_inv_hbm_frac"], row["rk_update_us"],
               100 * row["rk_update_hbm_frac"]))
        rows.append(row)
        op.close()
        del U, L, dU
        torch.cuda.empty_cache()
    return {"copy_bytes_per_s": bw, "rows": rows}


def precision_study(steps):
    """Float32 vs float64 operator over `steps` RK steps from the same state, for
    the Taylor-Green 16^3 k=7 n_q=11 and 24^3 k=5 n_q=8 workloads: relative
    difference of the kinetic energy and of its dissipation rate -de_k/dt after the
    run, and of L at the initial state."""
    import torch
    from paper_1806_03095_amd import taylor_green
    out = []
    for ne, k, nq in ((16, 7, 11), (24, 5, 8)):
        ops = {p: taylor_green(k, ne, n_q=nq, precision=p) for p in ("fp64", "fp32")}
        U0 = ops["fp64"].project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
        dt = ops["fp64"].compute_dt(CR_STUDY, D_RUN, 1.5, 3.0, 1.0, 0.1)
        e0 = fp32_error(ops["fp64"], ops["fp32"], U0)
        row = {"workload": "taylor_green_%dcubed_k%d_nq%d" % (ne, k, nq), "n_dof": ops["fp64"].n_dof,
               "steps": steps, "dt": dt, "L0_rel_err": e0["whole_vector"], "L0_rel_err_per_field": e0["per_field"],
               "L0_rate_rel_err": e0["dissipation_rate"]}
        res = {}
        for p, op in ops.items():
            U = U0.clone()
            work = torch.empty(2 * op.n_dof, dtype=torch.float64, device="cuda")
            t, _ = time_rk(op, U, work, dt, steps, 0)
            d = ops["fp64"].diagnostics(U, ops["fp64"].apply(U))
            res[p] = {"U": U, "e_k": d["e_k"], "rate": d["rate"], "ms_per_step": 1e3 * t / steps}
            log("%s %s: %d steps, %.3f ms/step, e_k=%.8f, -de_k/dt=%.6e"
                % (row["workload"], p, steps, 1e3 * t / steps, d["e_k"], d["rate"]))
        a, b = res["fp32"], res["fp64"]
        row.update(e_k_fp64=b["e_k"], e_k_fp32=a["e_k"], e_k_rel_err=abs(a["e_k"] - b["e_k"]) / abs(b["e_k"]),
                   rate_fp64=b["rate"], rate_fp32=a["rate"], rate_rel_err=abs(a["rate"] - b["rate"]) / abs(b["rate"]),
                   U_rel_err=float(torch.linalg.norm(a["U"] - b["U"]) / torch.linalg.norm(b["U"])),
                   ms_per_step_fp64=b["ms_per_step"], ms_per_step_fp32=a["ms_per_step"],
                   speedup=b["ms_per_step"] / a["ms_per_step"])
        out.append(row)
        del ops, res
    return out


def _stays_stable(op, U0, dt, t_final, check_every=50):
    """True if the run from U0 with the fixed step dt reaches t_final with finite diagnostics
    and a kinetic energy that never exceeds 1.5 times the initial one (blow-up criterion)."""
    import torch
    U = U0.clone()
    work = torch.empty(2 * op.n_dof, dtype=torch.float64, device="cuda")
    ek0 = op.diagnostics(U)["e_k"]
    n = int(math.ceil(t_final / dt))
    for s in range(n):
        op.rk_step(U, work, s * dt, dt)
        if (s + 1) % check_every == 0 or s + 1 == n:
            d = op.diagnostics(U)
            if d.get("nonfinite") or not d["e_k"] <= 1.5 * ek0:
                return False
    return True


def critical_numbers(res_cr=0.02, res_d=0.002):
    """Critical Courant and diffusion numbers of the time-step formula (eq.
    TimeStepRestrictions_Compressible with e = 1.5, f = 3) for the Runge-Kutta scheme in use,
    determined the way Sec. 5.2.2 (Table 2) does: Taylor-Green vortex at an effective
    resolution of 60^3 / 64^3 (k = 2, 3, 5, 7 on 20^3, 16^3, 10^3, 8^3 cells, n_q by the 3/2
    rule); Cr from the convection-dominated Re = 1600 case run to t_f = 20 with D not
    binding, D from the viscous Re = 1 case run to t_f = 1 with Cr not binding.  Each
    value is bracketed by bisection to res_cr / res_d (stable, unstable)."""
    from paper_1806_03095_amd import taylor_green
    rows = []
    for k, ne in ((2, 20), (3, 16), (5, 10), (7, 8)):
        nq = (3 * k + 2) // 2
        row = {"k": k, "cells": ne ** 3, "n_q": nq}
        for which, Re, t_f, lo, hi, res in (("Cr", 1600.0, 20.0, 0.1, 1.3, res_cr), ("D", 1.0, 1.0, 0.005, 0.1, res_d)):
            op = taylor_green(k, ne, n_q=nq, Re=Re)
            U0 = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
            stages = len(op.rk_scheme()[0])

            def dt_of(x):
                if which == "Cr":
                    return op.compute_dt(x, 1e3, 1.5, 3.0, 1.0, 0.1)
                return op.compute_dt(1e3, x, 1.5, 3.0, 1.0, 0.1)

            t0 = time.perf_counter()
            runs = 0
            while hi - lo > res * 1.0001:
                mid = round((lo + hi) / 2 / res) * res
                if mid <= lo or mid >= hi:
                    mid = lo + res
                runs += 1
                if _stays_stable(op, U0, dt_of(mid), t_f):
                    lo = mid
                else:
                    hi = mid
            row[which + "_stable"] = round(lo, 6)
            row[which + "_unstable"] = round(hi, 6)
            row[which + "_stable_per_stage"] = round(lo / stages, 6)
            row["dt_" + which + "_stable"] = dt_of(lo)
            log("k=%d %d^3 n_q=%d: %s stable %.3f, unstable %.3f (%d runs, %.0f s)" % (k, ne, nq, which, lo, hi, runs,
                                                                                   time.perf_counter() - t0))
            op.close()
        row["stages"] = stages
        rows.append(row)
    return rows


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_eval(ne, k, nq, n_sample, threads):
    """Seconds for one oracle evaluation of L on n_sample cells (all cells if n_sample is None)
    of the Taylor-Green workload, with `threads` torch CPU threads; DoFs evaluated."""
    import numpy as np
    import torch
    from oracle import initial, mesh, operator, physics
    fl = physics.Fluid.from_reynolds(1600.0, 0.71)
    m = mesh.BoxMesh((ne,) * 3, (-math.pi,) * 3, (math.pi,) * 3, k)
    op = operator.DGOperator(m, fl, nq)
    if n_sample is None or n_sample >= m.n_cells:
        cells = np.arange(m.n_cells, dtype=np.int64)
    else:
        cells = np.linspace(0, m.n_cells - 1, n_sample).astype(np.int64)
    need = np.unique(np.concatenate([cells, m.nb[cells].reshape(-1)]))
    U = torch.zeros(5, m.n_cells, (k + 1) ** 3, dtype=torch.float64)
    U[:, need, :] = initial.l2_project(op, lambda x: initial.taylor_green(x, fl), cells=need)
    op.tau_of(need)
    old = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        op.apply(U, cells=cells[: min(len(cells), 8)])      # warm the geometry code paths
        t0 = time.perf_counter()
        op.apply(U, cells=cells)
        el = time.perf_counter() - t0
    finally:
        torch.set_num_threads(old)
    return el, len(cells) * 5 * (k + 1) ** 3, len(cells), m.n_cells


def cpu_baseline(ne, k, nq, n_sample, n_sample_1core):
    """The oracle, as it stands, timed on the host: one evaluation of L on the full 4^3
    Taylor-Green mesh (k=3, n_q=6) and on a sample of cells of the headline workload,
    each with all the threads torch uses here and with one thread.  value is the
    headline-workload sample with all threads."""
    import torch
    threads = torch.get_num_threads()
    runs = []
    for name, (e, kk, q), sample in (("taylor_green_4cubed_k3_nq6", (4, 3, 6), None),
                                      ("taylor_green_%dcubed_k%d_nq%d" % (ne, k, nq), (ne, k, nq), n_sample)):
        for th in (threads, 1):
            smp = sample if th == threads or sample is None else n_sample_1core
            el, dofs, nc, ntot = _oracle_eval(e, kk, q, smp, th)
            runs.append({"workload": name, "threads": th, "cells": nc, "of_cells": ntot, "seconds": el,
                         "dofs_per_s": dofs / el})
            log("cpu baseline %s, %d thread(s), %d of %d cells: %.2f s, %.3e DoF/s" % (name, th, nc, ntot, el,
                                                                                          dofs / el))
    head = runs[2]
    return {"value": head["dofs_per_s"], "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": "one evaluation of L on %d of %d cells of the same workload (%d threads, %.2f s); "
                      "host %s with %d logical CPUs" % (head["cells"], head["of_cells"], threads, head["seconds"],
                                                       _cpu_model(), os.cpu_count() or 0),
            "runs": runs}


def fp32_error(op64, op32, U):
    """Float32 operator against float64 on the same state: relative error per conserved
    field and over the whole vector, and of the exact -de_k/dt computed from each L."""
    import torch
    L64, L32 = op64.apply(U), op32.apply(U)
    per = [float(torch.linalg.norm(L32[c] - L64[c]) / torch.linalg.norm(L64[c])) for c in range(5)]
    r64 = op64.diagnostics(U, L64)["rate"]
    r32 = op64.diagnostics(U, L32)["rate"]
    return {"per_field": dict(zip(("rho", "rho_u", "rho_v", "rho_w", "rho_E"), per)),
            "whole_vector": float(torch.linalg.norm(L32 - L64) / torch.linalg.norm(L64)),
            "dissipation_rate": abs(r32 - r64) / abs(r64)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cells", type=int, default=32)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--nq", type=int, default=6)
    ap.add_argument("--op-calls", type=int, default=200)
    ap.add_argument("--cpu-sample-cells", type=int, default=12288)
    ap.add_argument("--cpu-sample-cells-1core", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--op-only", type=int, default=0, metavar="CALLS",
                    help="profiling mode: only CALLS launches of the float64 operator kernel, no JSON")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"), help="precision of --op-only")
    ap.add_argument("--memops-only", type=int, default=0, metavar="CALLS",
                    help="profiling mode: CALLS stand-alone M^{-1} launches, then CALLS RK stage updates, nothing timed")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="profiling mode: one device-to-device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the operation breakdown, copy bandwidth and channel figures")
    ap.add_argument("--sweep", action="store_true",
                    help="study mode: operator throughput over every compiled (k, n_q); one JSON line")
    ap.add_argument("--memops-streamed", action="store_true",
                    help="study mode: M^-1 and the RK update past the last-level cache (k = 3..5); one JSON line")
    ap.add_argument("--critical-cfl", action="store_true",
                    help="study mode: critical Courant and diffusion numbers per degree (Sec. 5.2.2 method); one JSON line")
    ap.add_argument("--precision-study", type=int, default=0, metavar="STEPS",
                    help="study mode: float32 vs float64 over STEPS RK steps (16^3 k=7, 24^3 k=5); one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the operator has no multi-GPU path (no halo exchange "
              "between GPUs is implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_03095_amd import taylor_green

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copied %d MiB (read %d B, write %d B)" % (args.copy_calibration, 8 * n, 8 * n))
        return

    if args.sweep:
        print(json.dumps({"degree_sweep": degree_sweep()}), flush=True)
        return
    if args.memops_streamed:
        print(json.dumps({"memops_streamed": memops_streamed()}), flush=True)
        return
    if args.critical_cfl:
        print(json.dumps({"critical_numbers": critical_numbers()}), flush=True)
        return
    if args.precision_study:
        print(json.dumps({"precision_study": precision_study(args.precision_study)}), flush=True)
        return

    k, nq, ne = args.degree, args.nq, args.cells
    if args.op_only:
        op = taylor_green(k, ne, n_q=nq, precision=args.precision)
        U0 = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
        L = torch.empty_like(U0)
        for _ in range(args.op_only):
            op.apply(U0, L)
        torch.cuda.synchronize()
        log("%d operator launches (%s), %d DoFs each" % (args.op_only, args.precision, op.n_dof))
        return
    if args.memops_only:
        op = taylor_green(k, ne, n_q=nq)
        U0 = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
        L = torch.empty_like(U0)
        for _ in range(args.memops_only):
            op.inverse_mass(U0, L)
        dU = torch.zeros_like(U0)
        for _ in range(args.memops_only):
            op.rk_stage_update(U0, dU, L, 1, 1e-12)
        torch.cuda.synchronize()
        log("%d inverse-mass launches and %d stage updates, %d DoFs each" % (args.memops_only, args.memops_only,
                                                                             op.n_dof))
        return
    log("workload: TGV %d^3 cells, k=%d, n_q=%d" % (ne, k, nq))
    op = taylor_green(k, ne, n_q=nq, precision="fp64")
    ndof = op.n_dof
    U0 = op.project_ic("taylor_green", [1.0, 1.0, 0.1, 1.0])
    dt = op.compute_dt(CR, D_RUN, 1.5, 3.0, 1.0, 0.1)
    work = torch.empty(2 * ndof, dtype=torch.float64, device="cuda")
    U = U0.clone()
    log("fp64: %d warmup + %d timed RK steps, dt=%.4e" % (args.warmup, args.steps, dt))
    t64, wall64 = time_rk(op, U, work, dt, args.steps, args.warmup)
    d = op.diagnostics(U)
    if d.get("nonfinite"):
        raise RuntimeError("the solution became non-finite")
    value = ndof * 5 * args.steps / t64
    log("fp64: %.3e DoF/s per operator evaluation (%.3f ms/step), e_k=%.6f" % (value, 1e3 * t64 / args.steps, d["e_k"]))

    L = torch.empty_like(U0)
    t_op = time_operator(op, U0, L, args.op_calls)
    log("fp64 operator kernel: %.1f us per launch, %.3e DoF/s" % (1e6 * t_op, ndof / t_op))

    # The roofline object covers one evaluation of L: its two launches (face kernel, then
    # cell kernel) back to back on the library's stream, timed together by HIP events on
    # that stream; the per-kernel split is in the rocprofv3 kernel trace under profiles/.
    flop = FLOP_PER_DOF.get((k, nq))
    roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s", "frac": None,
            "traffic": None, "kernels": "dg_face_kernel + dg_operator_kernel (one evaluation of L)"}
    if flop is not None:
        ach = flop * ndof / t_op
        roof.update(achieved=round(ach / 1e12, 3), frac=round(ach / PEAK_FP64_VALU, 4))
    hbm_frac = BYTES_PER_DOF * ndof / t_op / PEAK_HBM
    if MEASURED_TRAFFIC["workload"] == (ne, k, nq) and MEASURED_TRAFFIC["fingerprint"] == kernel_fingerprint():
        roof["traffic"] = MEASURED_TRAFFIC["bytes"]

    out = {"metric": METRIC, "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t64 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "taylor_green_%dcubed_k%d_nq%d" % (ne, k, nq), "cells": ne ** 3, "degree": k,
                      "n_q": nq, "basis": "LGL", "n_dof": ndof, "mach": 0.1, "reynolds": 1600,
                      "time_integrator": "2N low-storage RK, 5 stages, order 4", "dt": dt},
           "roofline": roof,
           "operator_only": {"dofs_per_s": ndof / t_op, "us_per_launch": 1e6 * t_op,
                             "hbm_frac_16B_per_dof": round(hbm_frac, 5)}}

    if not args.no_extras:
        out["operations"] = operations(op, U0, t_op, t64 / args.steps, max(args.op_calls // 4, 10))
        bw = copy_bandwidth()
        out["copy_bandwidth"] = {"bytes_per_s": bw, "frac_of_peak": bw / PEAK_HBM,
                                 "operator_hbm_frac_of_copy": BYTES_PER_DOF * ndof / t_op / bw}
        out["channel"] = channel_throughput(max(args.op_calls // 4, 10))
        out["adjoint"] = adjoint_timing()
        out["hip_graph"] = graph_timing()
        log("operations: " + ", ".join("%s %.1f us" % (n, v["us"]) for n, v in out["operations"].items()))
        log("copy %.2f TB/s; channel fp64 %.3e DoF/s" % (bw / 1e12, out["channel"]["fp64"]["dofs_per_s"]))

    if not args.no_fp32:
        op32 = taylor_green(k, ne, n_q=nq, precision="fp32")
        U32 = U0.clone()
        t32, _ = time_rk(op32, U32, work, dt, args.steps, args.warmup)
        t_op32 = time_operator(op32, U0, L, args.op_calls)
        e0 = fp32_error(op, op32, U0)
        out["fp32"] = {"value": ndof * 5 * args.steps / t32, "speedup_vs_fp64": t64 / t32,
                       "operator_dofs_per_s": ndof / t_op32, "operator_speedup_vs_fp64": t_op / t_op32,
                       "residual_rel_err": e0["whole_vector"], "residual_rel_err_per_field": e0["per_field"],
                       "dissipation_rate_rel_err": e0["dissipation_rate"],
                       "error_state": "projected Taylor-Green initial state (smooth, Mach 0.1)"}
        log("fp32: %.3e DoF/s (x%.2f), operator x%.2f, |L32-L64|/|L64| = %.2e, per field %s, rate %.2e"
            % (out["fp32"]["value"], t64 / t32, t_op / t_op32, e0["whole_vector"],
               " ".join("%.1e" % v for v in e0["per_field"].values()), e0["dissipation_rate"]))
        del op32

    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the 4^3 mesh and on %d / %d sample cells" % (args.cpu_sample_cells,
                                                                               args.cpu_sample_cells_1core))
        out["cpu_baseline"] = cpu_baseline(ne, k, nq, args.cpu_sample_cells, args.cpu_sample_cells_1core)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
