#!/usr/bin/env python3
"""Benchmark of the FP64 SBDF2 Rayleigh-Benard step on one MI355X.

Workload: 2-D Rayleigh-Benard, Fourier x (Nx=1024, Lx=4) x Chebyshev z
(Nz=256), Ra=1e8, Pr=1, dt=1e-5, seeded noise on b (workload seed 1001): 513
pencils of 7*256 unknowns.  A step is one pass of the whole hot path: the
backward z transform, the x pass with the grid products, the forward z
transform with the SBDF2 right-hand side, and the banded pencil solve.  The
two start-up factorisations (SBDF1, then SBDF2) happen in the warm-up steps,
as in any run of the scheme.

Prints one JSON line: metric, value (DOF-updates/s = 7*Nx*Nz per step per
second), roofline of the dominant kernel (HIP-event timing on the launch
stream) and the CPU-oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
WORKLOAD = dict(Nx=1024, Nz=256, Lx=4.0, Ra=1e8, Pr=1.0, dt=1e-5, seed_workload=1)


def b_grid(Nx, Nz, xi, amp=1e-3):
    """b = 1 - z + amp z (1 - z) xi on the scale-1 grid (Gauss-Chebyshev z)."""
    import numpy as np

    j = np.arange(Nz)
    z = 0.5 * (1.0 - np.cos(np.pi * (j + 0.5) / Nz))
    return (1.0 - z)[None, :] + amp * (z * (1.0 - z))[None, :] * xi


def algorithmic_bytes(info):
    """Minimum HBM bytes per launch of each kernel (FP64): every input read
    once, every output written once.  z backward: 6 state fields of N modes
    read (b, u, w, bz, uz, wz), 8 grid fields of M points written; x pass: 8
    fields read on the active pencils, 3 written; z forward + RHS: 3 grid
    fields read, the previous state's evolved rows and the old history read,
    the new history (2 arrays) and the right-hand side written; solve: the
    whole-band factors (kl + kl + ku + 1 doubles and a pivot byte per column)
    and the right-hand side read, the state written."""
    P, Pa, N, M, S, ne = info["P"], info["P_active"], info["Nz"], info["Ngz"], info["S"], info["ne"]
    n, kl, ku = info["n"], info["kl"], info["ku"]
    c16 = 16
    zb = 6 * P * N * c16 + 8 * M * P * c16
    xp = 8 * M * Pa * c16 + 3 * M * P * c16
    zf = 3 * M * P * c16 + 3 * P * N * c16 + 2 * (2 * ne * P * N * c16) + ne * P * N * c16
    solve = Pa * n * ((2 * kl + ku + 1) * 8 + 1) + Pa * ne * N * c16 + P * S * N * c16
    return {"z_backward": zb, "x_pass": xp, "z_forward_rhs": zf, "pencil_solve": solve}


ADJ_WORKLOAD = dict(Nx=512, Nz=128, Lx=4.0, Ra=1e6, Pr=1.0, dt=1e-4, steps=200, checkpoint=20,
                    seed_workload=3)
# mixed-precision adjoint workload: 4096x64, checkpoint every 50
ADJ_WORKLOAD_MIXED = dict(Nx=4096, Nz=64, Lx=16.0, Ra=1e7, Pr=7.0, dt=2e-5, steps=200, checkpoint=50,
                          seed_workload=4)


def adjoint_ratio(reps=3, a=None, precision="fp64", keep_grad=False):
    """Adjoint workload (default 512x128, Ra=1e6, 200 SBDF2 steps, checkpoint
    every 20): time of the forward run vs the full gradient (forward with
    checkpoints + recomputation + reverse steps + initial-condition adjoint)."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1905_10388_amd import RBSolver
    from paper_1905_10388_amd.adjoint import kinetic_energy_and_gradient

    a = a or ADJ_WORKLOAD
    g = RBSolver(a["Nx"], a["Nz"], a["Lx"], a["Ra"], a["Pr"], precision=precision)
    b = torch.from_numpy(b_grid(a["Nx"], a["Nz"], si.workload_noise((a["Nx"], a["Nz"]), a["seed_workload"]))).cuda()

    def fwd():
        g.initial_state(b)
        for _ in range(a["steps"]):
            g.step(a["dt"])
        return g.kinetic_energy()

    fwd()
    kinetic_energy_and_gradient(g, b, a["dt"], a["steps"], a["checkpoint"])  # warm (factor cache)
    tf, tg = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fwd()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kinetic_energy_and_gradient(g, b, a["dt"], a["steps"], a["checkpoint"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tg.append(t2 - t1)
    f, gr = float(np.median(tf)), float(np.median(tg))
    dof = 7 * a["Nx"] * a["Nz"] * a["steps"]
    name = (f"rb2d_{a['Nx']}x{a['Nz']}_Ra{a['Ra']:.0e}_dt{a['dt']:.0e}_{a['steps']}steps"
            f"_ckpt{a['checkpoint']}").replace("e+0", "e").replace("e-0", "e-")
    out = {"workload": name, "forward_ms": f * 1e3,
           "gradient_ms": gr * 1e3, "adjoint_over_forward": gr / f,
           "forward_dof_updates_per_s": dof / f, "adjoint_dof_updates_per_s": dof / (gr - f) if gr > f else None,
           "dtype": "f64" if precision == "fp64" else "f32+f64"}
    if keep_grad:
        J, gg = kinetic_energy_and_gradient(g, b, a["dt"], a["steps"], a["checkpoint"])
        out["_J"], out["_grad"] = J, gg.detach().cpu().numpy()
    g.close()
    return out


def adjoint_mixed():
    """The 4096x64 adjoint workload in FP64 and in mixed precision, with the
    mixed gradient's relative L2 error against the FP64 gradient."""
    import numpy as np

    r64 = adjoint_ratio(a=ADJ_WORKLOAD_MIXED, keep_grad=True)
    rmx = adjoint_ratio(a=ADJ_WORKLOAD_MIXED, precision="mixed", keep_grad=True)
    g64, gmx = r64.pop("_grad"), rmx.pop("_grad")
    J64, Jmx = r64.pop("_J"), rmx.pop("_J")
    rmx["grad_err_vs_fp64"] = float(np.linalg.norm(gmx - g64) / np.linalg.norm(g64))
    rmx["J_err_vs_fp64"] = abs(Jmx - J64) / abs(J64)
    rmx["speedup_vs_fp64"] = r64["gradient_ms"] / rmx["gradient_ms"]
    return {"fp64": r64, "mixed": rmx}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE runs, scaled by the copy-kernel calibration),
    or None if the kernel's sources changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)[kernel]
        m = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                m.update(fh.read())
        return rec["bytes"] if m.hexdigest() == rec["sha256"] else None
    except (OSError, KeyError, ValueError):
        return None


def mixed_run(w, steps, warmup, X_fp64):
    """The mixed-precision step on the same workload and step count; per-field
    relative L2 error of its final state against the FP64 path's final state
    (the FP64 path agrees with the FP64 oracle to 1e-10)."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1905_10388_amd import RBSolver

    Nx, Nz, dt = w["Nx"], w["Nz"], w["dt"]
    g = RBSolver(Nx, Nz, w["Lx"], w["Ra"], w["Pr"], precision="mixed")
    g.initial_state(torch.from_numpy(b_grid(Nx, Nz, si.workload_noise((Nx, Nz), w["seed_workload"]))))
    for _ in range(warmup):
        g.step(dt)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        g.step(dt)
    ev1.record()
    torch.cuda.synchronize()
    ms = max((time.perf_counter() - t0) * 1e3 / steps, ev0.elapsed_time(ev1) / steps)
    g.check()
    Xm = g.X.cpu().numpy()
    Xd = X_fp64.cpu().numpy()
    names = ("p", "b", "u", "w", "bz", "uz", "wz")
    err = {}
    for i, v in enumerate(names):
        den = np.linalg.norm(Xd[:, i])
        err[v] = float(np.linalg.norm(Xm[:, i] - Xd[:, i]) / den) if den > 0 else None
    g.set_kernel_timing(True)
    for _ in range(20):
        g.step(dt)
    kt = {k: round(ms_ * 1e3 / c, 3) for k, (ms_, c) in g.read_kernel_timing().items() if c}
    g.close()
    return {"value": 7 * Nx * Nz / (ms * 1e-3), "unit": "DOF-updates/s", "ms_per_step": ms,
            "dtype": "f32+f64", "err_vs_fp64_per_field": err, "kernels_avg_us": kt,
            "steps_compared": steps + warmup}


def rk_run(w, X_start, steps=100, warmup=3):
    """IMEX Runge-Kutta steps (RK222, RK443; FP64) on the headline workload
    from the state the SBDF2 run reached: ms per step and per stage (one
    explicit term and one pencil solve each), per-kernel averages."""
    import torch

    from paper_1905_10388_amd import RBSolver

    Nx, Nz, dt = w["Nx"], w["Nz"], w["dt"]
    out = {}
    for scheme, stages in (("RK222", 2), ("RK443", 4)):
        g = RBSolver(Nx, Nz, w["Lx"], w["Ra"], w["Pr"])
        g.set_state(X_start)
        for _ in range(warmup):
            g.step_rk(dt, scheme)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(steps):
            g.step_rk(dt, scheme)
        ev1.record()
        torch.cuda.synchronize()
        ms = max((time.perf_counter() - t0) * 1e3 / steps, ev0.elapsed_time(ev1) / steps)
        g.check()
        g.set_kernel_timing(True)
        for _ in range(10):
            g.step_rk(dt, scheme)
        kt = {k: round(v * 1e3 / c, 3) for k, (v, c) in g.read_kernel_timing().items() if c}
        g.close()
        out[scheme] = {"value": 7 * Nx * Nz / (ms * 1e-3), "unit": "DOF-updates/s", "ms_per_step": ms,
                       "stages": stages, "ms_per_stage": ms / stages, "steps": steps,
                       "kernels_avg_us": kt, "dtype": "f64"}
    return out


def lbvp_evp_run(w, reps=50, evp_iters=200):
    """The linear boundary value solve (factors cached) and the shift-invert
    linear-stability iteration on the headline workload's pencils."""
    import torch

    import seeded_inputs as si
    from paper_1905_10388_amd import RBSolver

    Nx, Nz = w["Nx"], w["Nz"]
    g = RBSolver(Nx, Nz, w["Lx"], w["Ra"], w["Pr"])
    F = torch.from_numpy(si.complex_noise(g.ev_shape, 24)).cuda()
    X = g.lbvp(F)  # factors L~
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        g.lbvp(F, out=X)
    ev1.record()
    torch.cuda.synchronize()
    lbvp_ms = ev0.elapsed_time(ev1) / reps
    g.evp(1.0, iters=1)  # factors 1 M~ + L~ + L~'
    torch.cuda.synchronize()
    ev0.record()
    sig, res, _ = g.evp(1.0, iters=evp_iters)
    ev1.record()
    torch.cuda.synchronize()
    evp_ms = ev0.elapsed_time(ev1)
    g.close()
    return {"lbvp_ms": lbvp_ms, "lbvp_pencils": Nx // 2,
            "evp_iterations": evp_iters, "evp_ms": evp_ms, "evp_us_per_iteration": evp_ms * 1e3 / evp_iters,
            "evp_tau": 1.0, "evp_top_sigma": float(sig.max())}


def ncc_run(w, X_start, steps=100, warmup=5):
    """SBDF2 steps of the headline workload with a non-constant coefficient
    Gamma(z) w in the b equation: one Chebyshev term (same band, two-block
    solve) and three terms (band kl = 21, ku = 35: whole-band solve)."""
    import torch

    from paper_1905_10388_amd import RBSolver

    Nx, Nz, dt = w["Nx"], w["Nz"], w["dt"]
    out = {}
    for name, gamma in (("gamma_1term", (0.5,)), ("gamma_3term", (0.2, 0.15, -0.1))):
        g = RBSolver(Nx, Nz, w["Lx"], w["Ra"], w["Pr"], gamma=gamma)
        g.set_state(X_start)
        for _ in range(warmup):
            g.step(dt)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            g.step(dt)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        g.check()
        g.set_kernel_timing(True)
        for _ in range(10):
            g.step(dt)
        kt = {k: round(v * 1e3 / c, 3) for k, (v, c) in g.read_kernel_timing().items() if c}
        out[name] = {"gamma": list(gamma), "kl": g.info["kl"], "ku": g.info["ku"], "ms_per_step": ms,
                     "value": 7 * Nx * Nz / (ms * 1e-3), "kernels_avg_us": kt}
        g.close()
    return out


EXTRA_WORKLOADS = {
    # 3-D Fourier x, y x Chebyshev z: 33,024 pencil slots per launch
    "rb3d_256x256x128_Ra1e7_dt5e-5": dict(dim=3, Nx=256, Ny=256, Nz=128, Lx=4.0, Ly=4.0, Ra=1e7,
                                          Pr=1.0, dt=5e-5, seed_workload=2, steps=50),
    # small-Nz regime: 2049 pencil slots of n = 448
    "rb2d_4096x64_Lx16_Ra1e7_Pr7_dt2e-5": dict(dim=2, Nx=4096, Ny=1, Nz=64, Lx=16.0, Ly=1.0,
                                               Ra=1e7, Pr=7.0, dt=2e-5, seed_workload=4, steps=200),
}


def run_workload(w, precision, steps, warmup=10):
    """Timed steps of one workload at one precision: (ms per step, final state
    on the host, per-kernel average us over 10 extra steps)."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1905_10388_amd import RBSolver

    dim, Nx, Ny, Nz, dt = w["dim"], w["Nx"], w["Ny"], w["Nz"], w["dt"]
    g = RBSolver(Nx, Nz, w["Lx"], w["Ra"], w["Pr"], dim=dim, Ny=Ny, Ly=w["Ly"], precision=precision)
    shape = (Nx, Nz) if dim == 2 else (Nx, Ny, Nz)
    xi = si.workload_noise(shape, w["seed_workload"])
    j = np.arange(Nz)
    z = 0.5 * (1.0 - np.cos(np.pi * (j + 0.5) / Nz))
    prof = z * (1.0 - z)
    bg = (1.0 - z) + 1e-3 * prof * xi
    g.initial_state(torch.from_numpy(bg))
    for _ in range(warmup):
        g.step(dt)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        g.step(dt)
    ev1.record()
    torch.cuda.synchronize()
    ms = max((time.perf_counter() - t0) * 1e3 / steps, ev0.elapsed_time(ev1) / steps)
    g.check()
    X = g.X.cpu().numpy()
    g.set_kernel_timing(True)
    for _ in range(10):
        g.step(dt)
    kt = {k: round(v * 1e3 / c, 3) for k, (v, c) in g.read_kernel_timing().items() if c}
    info = dict(g.info)
    g.close()
    del g
    torch.cuda.empty_cache()
    return ms, X, kt, info


def extra_workloads():
    """The 3-D and small-Nz workloads, FP64 and mixed, with the mixed path's
    per-field error against the FP64 path after the same steps."""
    import numpy as np

    out = {}
    for name, w in EXTRA_WORKLOADS.items():
        steps = w["steps"]
        ms64, X64, kt64, info = run_workload(w, "fp64", steps)
        msmx, Xmx, ktmx, _ = run_workload(w, "mixed", steps)
        S = info["S"]
        names = ("p", "b", "u", "w", "bz", "uz", "wz") if S == 7 else \
            ("p", "b", "u", "v", "w", "bz", "uz", "vz", "wz")
        err = {}
        for i, v in enumerate(names):
            a, b = Xmx[..., i, :], X64[..., i, :]
            den = np.linalg.norm(b)
            err[v] = float(np.linalg.norm(a - b) / den) if den > 0 else None
        dof = S * w["Nx"] * w["Ny"] * w["Nz"]
        out[name] = {"steps": steps, "pencils": info["P_active"], "unknowns_per_pencil": info["n"],
                     "fp64": {"value": dof / (ms64 * 1e-3), "ms_per_step": ms64, "kernels_avg_us": kt64},
                     "mixed": {"value": dof / (msmx * 1e-3), "ms_per_step": msmx, "kernels_avg_us": ktmx,
                               "err_vs_fp64_per_field": err, "steps_compared": steps + 10},
                     "unit": "DOF-updates/s"}
    return out


def cpu_baseline(w, sample_pencils=128, reps=3):
    """The oracle's SBDF2 step on a bounded sample: the explicit term on the
    full grid, then right-hand side + LU solve of `sample_pencils` pencils
    (factorisations done beforehand, untimed), scaled to all pencils."""
    import numpy as np

    import seeded_inputs as si
    from oracle import RBOracle, RBParams, sbdf_coefficients

    try:
        from threadpoolctl import threadpool_info

        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    Nx, Nz = w["Nx"], w["Nz"]
    o = RBOracle(Nx, Nz, w["Lx"], RBParams(w["Ra"], w["Pr"]))
    X = o.initial_state(si.workload_noise((Nx, Nz), w["seed_workload"]))
    dt = w["dt"]
    a0, a1, a2, b0, c1, c2 = sbdf_coefficients(1, dt, dt)
    act = [p for p in o.pencils() if p[4]]
    stride = max(1, len(act) // sample_pencils)
    sample = act[::stride][:sample_pencils]
    solvers = {}
    for key, kx, ky, mean, _ in sample:
        solvers[key] = (o._ML_cached(key, kx, ky, mean), o.solver_for(key, kx, ky, mean, a0, b0))
    t_nl, t_pen = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        F = o.nonlinear(X)
        t1 = time.perf_counter()
        for key, kx, ky, mean, _ in sample:
            (M, L), solve = solvers[key]
            Ft = o.precondition_rhs(F[key], mean)
            MX = M @ X[key].reshape(-1)
            B = c1 * Ft - a1 * MX + c2 * Ft - a2 * MX
            for r, val in o.bc_values(mean).items():
                B[r] = val
            solve(B)
        t2 = time.perf_counter()
        t_nl.append(t1 - t0)
        t_pen.append(t2 - t1)
    t_step = float(np.median(t_nl)) + float(np.median(t_pen)) * len(act) / len(sample)
    dof = 7 * Nx * Nz
    return {
        "value": dof / t_step, "unit": "DOF-updates/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"explicit term on the full 1536x384 grid + RHS and LU solves of "
                   f"{len(sample)}/{len(act)} pencils (factorisations untimed), median of "
                   f"{reps}, solve time scaled by {len(act)}/{len(sample)}; "
                   f"{os.cpu_count()} host cores, {threads} BLAS threads"),
        "seconds_per_step": t_step,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=100,
                    help="steps of the per-kernel HIP-event pass after the timed region")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-rk", action="store_true", help="skip the Runge-Kutta steps")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 3-D and small-Nz workloads")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device-to-device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on exactly one GPU (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1905_10388_amd import RBSolver

    w = WORKLOAD
    Nx, Nz, dt = w["Nx"], w["Nz"], w["dt"]
    g = RBSolver(Nx, Nz, w["Lx"], w["Ra"], w["Pr"])
    xi = si.workload_noise((Nx, Nz), w["seed_workload"])
    g.initial_state(torch.from_numpy(b_grid(Nx, Nz, xi)))
    for _ in range(max(2, args.warmup)):
        g.step(dt)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        g.step(dt)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_wall = (t1 - t0) * 1e3 / args.steps
    ms_ev = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = max(ms_wall, ms_ev)
    g.check()
    dof = 7 * Nx * Nz
    value = dof / (ms_per_step * 1e-3)
    X_end = g.X.clone()
    n_steps_end = g.iteration

    # per-kernel HIP-event timing on the launch stream (separate pass)
    g.set_kernel_timing(True)
    for _ in range(args.timing_steps):
        g.step(dt)
    kt = g.read_kernel_timing()
    g.set_kernel_timing(False)
    nbytes = algorithmic_bytes(g.info)
    kernels = {}
    for k, (ms, cnt) in kt.items():
        if cnt:
            avg_us = ms * 1e3 / cnt
            entry = {"avg_us": round(avg_us, 3), "launches": int(cnt)}
            if k in nbytes:
                entry["bytes"] = nbytes[k]
                entry["GBps"] = round(nbytes[k] / (avg_us * 1e-6) / 1e9, 1)
            kernels[k] = entry
    roofline = None
    timed_kernels = [k for k in kernels if k in nbytes]
    if timed_kernels:
        dom = max(timed_kernels, key=lambda k: kernels[k]["avg_us"])
        ach = kernels[dom]["GBps"]
        roofline = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(dom)}
    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    out = {
        "metric": "DOF-updates/s per SBDF2 step, FP64 vs mixed at stated err; adjoint/forward time",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(2, args.warmup),
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rb2d_1024x256_Ra1e8_dt1e-5", "Nx": Nx, "Nz": Nz, "Lx": w["Lx"],
                   "Ra": w["Ra"], "Pr": w["Pr"], "dt": dt, "pencils": g.info["P_active"],
                   "unknowns_per_pencil": g.info["n"], "kl": g.info["kl"], "ku": g.info["ku"]},
        "kernels": kernels,
        "roofline": roofline,
        "mode_updates_per_s": Nx * Nz / (ms_per_step * 1e-3),
    }
    if not args.no_mixed:
        out["mixed"] = mixed_run(w, args.steps, n_steps_end - args.steps, X_end)
        out["mixed"]["speedup_vs_fp64"] = out["mixed"]["value"] / value
    if not args.no_rk:
        out["runge_kutta"] = rk_run(w, X_end)
        out["lbvp_evp"] = lbvp_evp_run(w)
        out["ncc"] = ncc_run(w, X_end)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio()
        out["adjoint_mixed"] = adjoint_mixed()
    if not args.no_extra:
        out["workloads"] = extra_workloads()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
