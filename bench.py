#!/usr/bin/env python3
"""Benchmark of the FP64 SBDF2 Rayleigh-Benard step on one MI355X.

Headline workload: 3-D Rayleigh-Benard, Fourier x, y (Nx = Ny = 256,
Lx = Ly = 4) x Chebyshev z (Nz = 128), Ra = 1e7, Pr = 1, dt = 5e-5, seeded
noise on b (workload seed 1002): 33,024 pencil slots (32,640 solved) of
9 * 128 unknowns, batched into one solve launch.  A step is one pass of the
whole hot path: the backward z transform, the backward y transform, the x
pass with the grid products, the forward y transform, the forward z transform
with the SBDF2 right-hand side, and the banded pencil solve.  The two
start-up factorisations (SBDF1, then SBDF2) run in the warm-up steps, as in
any run of the scheme, and are timed and reported on their own.

Prints one JSON line: metric, value (DOF-updates/s = 9 Nx Ny Nz per step per
second), the roofline of the dominant kernel (HIP events on the launch
stream), the mixed-precision forms with their errors, the other workloads as
extra keys, and the CPU-oracle baseline on a bounded sample.

    python3 bench.py [--steps K] [--warmup W]
    python3 bench.py --probe fp64|mixed WORKLOAD [--probe-steps K] [--probe-dct auto|fft|matmul]   (counters)
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "DOF-updates/s per SBDF2 step, FP64 vs mixed at stated err; adjoint/forward time"

# The five workloads (seed 1000 + workload number for the b noise).
WORKLOADS = {
    "rb2d_64x32_Ra1e4_dt1e-3": dict(dim=2, Nx=64, Ny=1, Nz=32, Lx=4.0, Ly=1.0, Ra=1e4, Pr=1.0,
                                    dt=1e-3, seed_workload=0, steps=100),
    "rb2d_1024x256_Ra1e8_dt1e-5": dict(dim=2, Nx=1024, Ny=1, Nz=256, Lx=4.0, Ly=1.0, Ra=1e8, Pr=1.0,
                                       dt=1e-5, seed_workload=1, steps=500),
    "rb3d_256x256x128_Ra1e7_dt5e-5": dict(dim=3, Nx=256, Ny=256, Nz=128, Lx=4.0, Ly=4.0, Ra=1e7,
                                          Pr=1.0, dt=5e-5, seed_workload=2, steps=100),
    "rb2d_512x128_Ra1e6_dt1e-4": dict(dim=2, Nx=512, Ny=1, Nz=128, Lx=4.0, Ly=1.0, Ra=1e6, Pr=1.0,
                                      dt=1e-4, seed_workload=3, steps=200, checkpoint=20),
    "rb2d_4096x64_Lx16_Ra1e7_Pr7_dt2e-5": dict(dim=2, Nx=4096, Ny=1, Nz=64, Lx=16.0, Ly=1.0, Ra=1e7,
                                               Pr=7.0, dt=2e-5, seed_workload=4, steps=1000,
                                               checkpoint=50),
}
HEADLINE = "rb3d_256x256x128_Ra1e7_dt5e-5"
C2 = "rb2d_1024x256_Ra1e8_dt1e-5"
C4 = "rb2d_512x128_Ra1e6_dt1e-4"
C5 = "rb2d_4096x64_Lx16_Ra1e7_Pr7_dt2e-5"


def var_names(dim):
    return ("p", "b", "u", "w", "bz", "uz", "wz") if dim == 2 else \
        ("p", "b", "u", "v", "w", "bz", "uz", "vz", "wz")


def b_grid(w, amp=1e-3):
    """b = 1 - z + amp z (1 - z) xi on the scale-1 grid (Gauss-Chebyshev z),
    xi the workload's seeded noise ([ix][jz] in 2-D, [ix][ly][jz] in 3-D)."""
    import numpy as np

    import seeded_inputs as si

    Nz = w["Nz"]
    shape = (w["Nx"], w["Nz"]) if w["dim"] == 2 else (w["Nx"], w["Ny"], w["Nz"])
    xi = si.workload_noise(shape, w["seed_workload"])
    j = np.arange(Nz)
    z = 0.5 * (1.0 - np.cos(np.pi * (j + 0.5) / Nz))
    return (1.0 - z) + amp * (z * (1.0 - z)) * xi


def dof(w):
    S = 7 if w["dim"] == 2 else 9
    return S * w["Nx"] * w["Ny"] * w["Nz"]


def solver(w, precision="fp64", dct="auto", solve="auto", **kw):
    from paper_1905_10388_amd import RBSolver

    return RBSolver(w["Nx"], w["Nz"], w["Lx"], w["Ra"], w["Pr"], dim=w["dim"], Ny=w["Ny"],
                    Ly=w["Ly"], precision=precision, dct=dct, mixed_solve=solve, **kw)


def algorithmic_bytes(info, dim):
    """Minimum HBM bytes per launch of each kernel (FP64 complex = 16 B): every
    input read once, every output written once.
      z backward: the state fields the explicit term needs (2-D b, u, w, bz,
        uz, wz; 3-D also v, vz) read, their transforms (6; 3-D 8) of M points
        written per pencil slot (the x derivatives are formed in the x pass,
        the y derivatives in the backward y pass);
      y passes (3-D): backward, the 8 z-transformed fields of Ny rows read
        and 12 written on Ngy rows (with the y derivatives of b, u, v, w) per
        (z level, kx); forward, 4 fields of Ngy read and Ny written;
      x pass: the transformed fields read on the active kx, 3 (3-D: 4) written;
      z forward + RHS: the explicit term read, the previous state's evolved
        rows and the old history read, the new history (two arrays) and the
        right-hand side written;
      solve: the whole-band factors (kl + kl + ku + 1 doubles and a pivot
        byte per column) and the right-hand side read, the state written.
        This is the banded method's bound; where the solve reads the
        factors' nonzeros from sparse records it moves fewer bytes than this
        (roofline.traffic and traffic_frac give what HBM moved)."""
    P, Pa, N, M, S, ne = info["P"], info["P_active"], info["Nz"], info["Ngz"], info["S"], info["ne"]
    n, kl, ku = info["n"], info["kl"], info["ku"]
    Px, Ny, Ngy = info["Px"], info["Ny"], info["Ngy"]
    c16 = 16
    # state fields read, z-transformed fields, fields of the x pass
    nin, nz, nf = (6, 6, 6) if dim == 2 else (8, 8, 12)
    zb = nin * P * N * c16 + nz * M * P * c16
    if dim == 2:
        xp = nf * M * (Px - 1) * c16 + ne * M * Px * c16
        yp = 0
    else:
        xp = nf * M * Ngy * (Px - 1) * c16 + ne * M * Ngy * Px * c16
        yp = (nz * M * Ny * Px + nf * M * Ngy * Px) * c16 + (ne * M * Ngy * Px + ne * M * Ny * Px) * c16
    zf = ne * M * P * c16 + ne * P * N * c16 + 2 * (2 * ne * P * N * c16) + ne * P * N * c16
    solve = Pa * n * ((2 * kl + ku + 1) * 8 + 1) + Pa * ne * N * c16 + P * S * N * c16
    out = {"z_backward": zb, "x_pass": xp, "z_forward_rhs": zf, "pencil_solve": solve}
    if yp:
        out["y_pass"] = yp  # backward + forward, summed per step (two launches)
    return out


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE runs, scaled by the copy-kernel
    calibration), or None if the kernel's sources changed since the counters
    were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)[workload][kernel]
        m = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                m.update(fh.read())
        return rec["bytes"] if m.hexdigest() == rec["sha256"] else None
    except (OSError, KeyError, ValueError, TypeError):
        return None


def timed_steps(g, dt, steps):
    """ms per step over `steps` steps: HIP events on the current stream and the
    host clock, each bracketed by a device synchronisation; the larger."""
    import torch

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        g.step(dt)
    ev1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return max(wall, ev0.elapsed_time(ev1) / steps)


def kernel_pass(g, dt, steps):
    """Per-kernel average us over `steps` extra steps (HIP events recorded by
    the library on the launch stream)."""
    g.set_kernel_timing(True)
    for _ in range(steps):
        g.step(dt)
    kt = g.read_kernel_timing()
    g.set_kernel_timing(False)
    return {k: (ms * 1e3 / c, c) for k, (ms, c) in kt.items() if c}


def field_err(Xa, Xb, dim):
    """Relative L2 error per variable of Xa against Xb over all coefficients."""
    import numpy as np

    out = {}
    for i, v in enumerate(var_names(dim)):
        a, b = Xa[..., i, :], Xb[..., i, :]
        den = np.linalg.norm(b)
        out[v] = float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))
    return out


def run(w, precision="fp64", dct="auto", steps=None, warmup=10, timing_steps=10, solve="auto"):
    """Warm-up (with the two factorisations timed), timed steps, a per-kernel
    pass; returns the figures and the state after warm-up + timed steps."""
    import torch

    g = solver(w, precision, dct, solve)
    g.initial_state(torch.from_numpy(b_grid(w)))
    steps = w["steps"] if steps is None else steps
    g.set_kernel_timing(True)
    for _ in range(max(2, warmup)):
        g.step(w["dt"])
    fk = g.read_kernel_timing()["pencil_factor"]
    g.set_kernel_timing(False)
    ms = timed_steps(g, w["dt"], steps)
    g.check()
    X = g.X.cpu().numpy()
    kt = kernel_pass(g, w["dt"], timing_steps) if timing_steps else {}
    info = dict(g.info)
    g.close()
    del g
    torch.cuda.empty_cache()
    return {"ms_per_step": ms, "value": dof(w) / (ms * 1e-3), "steps": steps,
            "warmup": max(2, warmup), "factor_ms": fk[0] / max(1, fk[1]), "factorisations": fk[1],
            "kernels": kt, "info": info, "X": X}


# --------------------------------------------------------------------------
# oracle windows (test infrastructure: the oracle is only timed and compared)
# --------------------------------------------------------------------------
def oracle_window(w, steps=3):
    """The FP64 oracle's first `steps` steps (SBDF1, then SBDF2) from the
    workload's seeded state, next to the HIP path's FP64 and mixed steps from
    the same initial state: per-field relative L2 error against the oracle."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from oracle import RBOracle, RBParams

    o = RBOracle(w["Nx"], w["Nz"], w["Lx"], RBParams(w["Ra"], w["Pr"]))
    shape = (w["Nx"], w["Nz"])
    X0 = o.initial_state(si.workload_noise(shape, w["seed_workload"]))
    t0 = time.perf_counter()
    Xo = X0
    for _ in range(steps):
        Xo = o.step(Xo, w["dt"])
    t_oracle = time.perf_counter() - t0
    out = {"steps": steps, "oracle_seconds": t_oracle}
    for prec, dct in (("fp64", "auto"), ("mixed", "auto"), ("mixed", "matmul")):
        if prec == "fp64" and dct != "auto":
            continue
        try:
            g = solver(w, prec, dct)
        except Exception as e:  # unsupported z-transform form for this Nz
            out[f"{prec}_{dct}"] = {"error": str(e)}
            continue
        g.set_state(torch.from_numpy(X0).cuda())
        for _ in range(steps):
            g.step(w["dt"])
        Xg = g.X.cpu().numpy()
        g.close()
        err = field_err(Xg, Xo, 2)
        out[f"{prec}_{dct}"] = {"err_vs_oracle_per_field": err, "max": max(err.values())}
    return out


def cpu_baseline_3d(w, sample_pencils=16):
    """The oracle's 3-D SBDF2 step on a bounded sample, scaled to one full
    step: one backward transform (coefficients to the 3/2 grid) and one
    forward transform of a field, times the 15 backward and 4 forward
    transforms of the explicit term; the grid products; and the right-hand
    side and LU solve of `sample_pencils` pencils (dense getrs on factors made
    beforehand, untimed), times the 32,640 active pencils."""
    import numpy as np

    import seeded_inputs as si
    from oracle import RBOracle, RBParams, sbdf_coefficients

    try:
        from threadpoolctl import threadpool_info

        blas = threadpool_info()
        threads = max([d.get("num_threads", 1) for d in blas] + [1])
        blas_desc = "; ".join(f"{d.get('internal_api')} {d.get('version')} "
                              f"({d.get('threading_layer')}, {d.get('num_threads')} threads, "
                              f"{d.get('architecture')})" for d in blas)
    except Exception:  # pragma: no cover
        threads, blas_desc = os.cpu_count() or 1, "unknown"
    o = RBOracle(w["Nx"], w["Nz"], w["Lx"], RBParams(w["Ra"], w["Pr"]), dim=3, Ny=w["Ny"], Ly=w["Ly"])
    X = o.initial_state(si.workload_noise((w["Nx"], w["Ny"], w["Nz"]), w["seed_workload"]), amp=1e-1)
    X[..., o.vi["u"], :] += 1e-2 * si.complex_noise(X[..., 0, :].shape, 77)
    t0 = time.perf_counter()
    gu = o.to_grid(X[..., o.vi["u"], :])
    t1 = time.perf_counter()
    gb = o.to_grid(X[..., o.vi["b"], :])
    t2 = time.perf_counter()
    prod = -(gu * gb + gu * gb + gu * gb)
    t3 = time.perf_counter()
    o.from_grid(prod)
    t4 = time.perf_counter()
    t_back = 0.5 * (t2 - t0)
    t_fwd = t4 - t3
    t_prod = (t3 - t2) * 4  # four products of three terms
    dt = w["dt"]
    a0, a1, a2, b0, c1, c2 = sbdf_coefficients(1, dt, dt)
    act = [p for p in o.pencils() if p[4]]
    stride = max(1, len(act) // sample_pencils)
    sample = act[::stride][:sample_pencils]
    solvers = {}
    tf0 = time.perf_counter()
    for key, kx, ky, mean, _ in sample:
        solvers[key] = (o._ML_cached(key, kx, ky, mean), o.solver_for(key, kx, ky, mean, a0, b0))
    t_factor = (time.perf_counter() - tf0) / len(sample)
    F = np.zeros((o.ne, o.Nz), complex)
    tp0 = time.perf_counter()
    for key, kx, ky, mean, _ in sample:
        (M, L), solve = solvers[key]
        Ft = o.precondition_rhs(F, mean)
        MX = M @ X[key].reshape(-1)
        B = c1 * Ft - a1 * MX + c2 * Ft - a2 * MX
        for r, val in o.bc_values(mean).items():
            B[r] = val
        solve(B)
    t_pen = (time.perf_counter() - tp0) / len(sample)
    t_step = 15 * t_back + 4 * t_fwd + t_prod + t_pen * len(act)
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        model = platform.processor()
    return {
        "value": dof(w) / t_step, "unit": "DOF-updates/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"oracle (dense transform matrices, dense LU per pencil) on the 256x256x128 "
                   f"workload: one backward transform (median of 2) and one forward transform "
                   f"timed and scaled by 15 and 4, the grid products, and the right-hand side "
                   f"and LU solve of {len(sample)} of {len(act)} pencils (factorisations made "
                   f"before, untimed: {t_factor * 1e3:.1f} ms per pencil) scaled by "
                   f"{len(act)}/{len(sample)}; host '{model}', {os.cpu_count()} logical cores, "
                   f"BLAS: {blas_desc}"),
        "seconds_per_step": t_step,
        "seconds_backward_transform": t_back, "seconds_forward_transform": t_fwd,
        "seconds_per_pencil_solve": t_pen, "seconds_per_pencil_factor": t_factor,
    }


# --------------------------------------------------------------------------
# further legs on the 2-D workloads (extra keys)
# --------------------------------------------------------------------------
def rk_run(w, X_start, steps=100, warmup=3):
    """IMEX Runge-Kutta steps (RK222, RK443; FP64) from the state the SBDF2
    run reached: ms per step and per stage, per-kernel averages."""
    import torch

    out = {}
    for scheme, stages in (("RK222", 2), ("RK443", 4)):
        g = solver(w)
        g.set_state(torch.from_numpy(X_start).cuda())
        for _ in range(warmup):
            g.step_rk(w["dt"], scheme)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            g.step_rk(w["dt"], scheme)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        g.check()
        g.close()
        out[scheme] = {"value": dof(w) / (ms * 1e-3), "unit": "DOF-updates/s", "ms_per_step": ms,
                       "stages": stages, "ms_per_stage": ms / stages, "steps": steps, "dtype": "f64"}
    return out


def lbvp_evp_run(w, reps=50, nev=4, max_ops=3000):
    """The linear boundary value solve (factors cached) and the shift-invert
    Krylov-Schur linear-stability solve (nev modes nearest tau = 1 on every
    pencil, at most max_ops operator applications per pencil)."""
    import torch

    import seeded_inputs as si

    g = solver(w)
    F = torch.from_numpy(si.complex_noise(g.ev_shape, 24)).cuda()
    X = g.lbvp(F)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        g.lbvp(F, out=X)
    ev1.record()
    torch.cuda.synchronize()
    lbvp_ms = ev0.elapsed_time(ev1) / reps
    g.evp(1.0, nev=1, max_ops=20)  # factors of tau M + L + L' and the bases
    torch.cuda.synchronize()
    ev0.record()
    sig, res, nconv, nops, _ = g.evp(1.0, nev=nev, max_ops=max_ops)
    ev1.record()
    torch.cuda.synchronize()
    evp_ms = ev0.elapsed_time(ev1)
    act = w["Nx"] // 2
    nconv, nops = nconv[:act].cpu(), nops[:act].cpu()
    top = sig[:act, 0].real.max().item()
    g.close()
    return {"lbvp_ms": lbvp_ms, "lbvp_pencils": act, "evp_tau": 1.0, "evp_nev": nev, "evp_max_ops": max_ops,
            "evp_ms": evp_ms, "evp_pencils_all_converged": int((nconv == nev).sum()),
            "evp_ops_mean": float(nops.float().mean()), "evp_ops_max": int(nops.max()),
            "evp_top_sigma": top}


def ncc_run(w, X_start, steps=100, warmup=5):
    """SBDF2 steps with a non-constant coefficient Gamma(z) w in the b
    equation: one Chebyshev term (same band) and three terms (wider band)."""
    import torch

    out = {}
    for name, gamma in (("gamma_1term", (0.5,)), ("gamma_3term", (0.2, 0.15, -0.1))):
        g = solver(w, gamma=gamma)
        g.set_state(torch.from_numpy(X_start).cuda())
        for _ in range(warmup):
            g.step(w["dt"])
        ms = timed_steps(g, w["dt"], steps)
        g.check()
        out[name] = {"gamma": list(gamma), "kl": g.info["kl"], "ku": g.info["ku"], "ms_per_step": ms,
                     "value": dof(w) / (ms * 1e-3)}
        g.close()
    return out


def adjoint_ratio(w, precision="fp64", reps=3, keep_grad=False):
    """Forward run of the adjoint workload against the full gradient (forward
    with checkpoints + recomputation + reverse steps + initial-condition
    adjoint) of the final kinetic energy."""
    import numpy as np
    import torch

    from paper_1905_10388_amd.adjoint import kinetic_energy_and_gradient

    g = solver(w, precision)
    b = torch.from_numpy(b_grid(w)).cuda()
    steps, ck, dt = w.get("adj_steps", 200), w["checkpoint"], w["dt"]

    def fwd():
        g.initial_state(b)
        for _ in range(steps):
            g.step(dt)
        return g.kinetic_energy()

    fwd()
    kinetic_energy_and_gradient(g, b, dt, steps, ck)
    tf, tg = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fwd()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kinetic_energy_and_gradient(g, b, dt, steps, ck)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tg.append(t2 - t1)
    f, gr = float(np.median(tf)), float(np.median(tg))
    n = dof(w) * steps
    out = {"steps": steps, "checkpoint": ck, "forward_ms": f * 1e3, "gradient_ms": gr * 1e3,
           "adjoint_over_forward": gr / f, "forward_dof_updates_per_s": n / f,
           "adjoint_dof_updates_per_s": n / (gr - f) if gr > f else None,
           "dtype": "f64" if precision == "fp64" else "f32+f64"}
    if keep_grad:
        J, gg = kinetic_energy_and_gradient(g, b, dt, steps, ck)
        out["_J"], out["_grad"] = J, gg.detach().cpu().numpy()
    g.close()
    return out


def adjoint_mixed(w):
    """The adjoint workload in FP64 and in mixed precision, with the mixed
    gradient's relative L2 difference to the FP64 gradient."""
    import numpy as np

    r64 = adjoint_ratio(w, keep_grad=True)
    rmx = adjoint_ratio(w, precision="mixed", keep_grad=True)
    g64, gmx = r64.pop("_grad"), rmx.pop("_grad")
    J64, Jmx = r64.pop("_J"), rmx.pop("_J")
    rmx["grad_diff_vs_fp64"] = float(np.linalg.norm(gmx - g64) / np.linalg.norm(g64))
    rmx["J_diff_vs_fp64"] = abs(Jmx - J64) / abs(J64)
    rmx["speedup_vs_fp64"] = r64["gradient_ms"] / rmx["gradient_ms"]
    return {"fp64": r64, "mixed": rmx}


def workload_pair(name, w, timing_steps=10, forms=(("auto", "auto"),)):
    """FP64 and mixed steps of one workload over its configured step count,
    with the mixed state's per-field relative difference to the FP64 state
    after the same steps; forms are (z transform, mixed solve) pairs."""
    r64 = run(w, "fp64", timing_steps=timing_steps)
    X64 = r64.pop("X")
    out = {"workload": name, "pencils": r64["info"]["P_active"],
           "unknowns_per_pencil": r64["info"]["n"], "unit": "DOF-updates/s",
           "fp64": _public(r64)}
    for dct, solve in forms:
        key = f"mixed_{dct}" + ("" if solve == "auto" else f"_{solve}")
        try:
            rmx = run(w, "mixed", dct, timing_steps=timing_steps, solve=solve)
        except Exception as e:
            out[key] = {"error": str(e)}
            continue
        Xmx = rmx.pop("X")
        m = _public(rmx)
        m["diff_vs_fp64_per_field"] = field_err(Xmx, X64, w["dim"])
        m["speedup_vs_fp64"] = rmx["value"] / r64["value"]
        out[key] = m
    return out, X64


def _public(r):
    k = {n: round(us, 3) for n, (us, c) in r["kernels"].items()}
    return {"value": r["value"], "ms_per_step": r["ms_per_step"], "steps": r["steps"],
            "factor_ms": r["factor_ms"], "kernels_avg_us": k}


def probe(precision, name, steps, copy_bytes, dct="auto"):
    """A few steps of one workload (for counter collection under a profiler)."""
    import torch

    w = WORKLOADS[name]
    g = solver(w, precision, dct=dct)
    g.initial_state(torch.from_numpy(b_grid(w)))
    for _ in range(steps):
        g.step(w["dt"])
    torch.cuda.synchronize()
    g.check()
    if copy_bytes > 0:
        src = torch.ones(copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print("probe done", precision, dct, name, steps, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--timing-steps", type=int, default=20,
                    help="steps of the per-kernel HIP-event pass after the timed region")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-window", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 2-D workloads (step, Runge-Kutta, LBVP/EVP, NCC, adjoint)")
    ap.add_argument("--probe", nargs=2, metavar=("PRECISION", "WORKLOAD"),
                    help="run --probe-steps steps of one workload and exit (for profilers)")
    ap.add_argument("--probe-steps", type=int, default=12)
    ap.add_argument("--probe-dct", default="auto", choices=("auto", "fft", "matmul"))
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="with --probe: one device-to-device copy of this many bytes after the "
                         "steps (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the stau library runs on exactly one GPU (it has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        prec, name = args.probe
        if name not in WORKLOADS:
            sys.exit(f"unknown workload {name}; one of {', '.join(WORKLOADS)}")
        probe(prec, name, args.probe_steps, args.copy_bytes, args.probe_dct)
        return

    w = WORKLOADS[HEADLINE]
    r = run(w, "fp64", steps=args.steps, warmup=args.warmup, timing_steps=args.timing_steps)
    X64 = r.pop("X")
    info = r["info"]
    nbytes = algorithmic_bytes(info, w["dim"])
    kernels = {}
    for k, (us, cnt) in r["kernels"].items():
        launches_per_step = cnt / args.timing_steps if args.timing_steps else 1
        entry = {"avg_us": round(us, 3), "launches": int(cnt)}
        if k in nbytes:
            per_launch = nbytes[k] / launches_per_step
            entry["bytes_per_launch"] = per_launch
            entry["GBps"] = round(per_launch / (us * 1e-6) / 1e9, 1)
        kernels[k] = entry
    roofline = None
    if "pencil_solve" in kernels:
        dom = max((k for k in kernels if "GBps" in kernels[k]), key=lambda k: kernels[k]["avg_us"] *
                  kernels[k]["launches"])
        ach = kernels[dom]["GBps"]
        traffic = measured_traffic(HEADLINE, dom)
        roofline = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic}
        if traffic:
            # the bytes HBM moved per launch (counters) over the same time
            roofline["traffic_frac"] = round(traffic / (kernels[dom]["avg_us"] * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": r["warmup"],
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": HEADLINE, "dim": 3, "Nx": w["Nx"], "Ny": w["Ny"], "Nz": w["Nz"],
                   "Lx": w["Lx"], "Ly": w["Ly"], "Ra": w["Ra"], "Pr": w["Pr"], "dt": w["dt"],
                   "pencils": info["P_active"], "pencil_slots": info["P"],
                   "unknowns_per_pencil": info["n"], "kl": info["kl"], "ku": info["ku"]},
        "kernels": kernels,
        "roofline": roofline,
        "factorisation": {"ms_per_factorisation": r["factor_ms"], "count_in_warmup": r["factorisations"],
                          "note": "SBDF1 and SBDF2 operators, synchronous, in the warm-up steps"},
        "mode_updates_per_s": w["Nx"] * w["Ny"] * w["Nz"] / (r["ms_per_step"] * 1e-3),
    }
    if not args.no_mixed:
        # the 3-D workload names split-BF16 matrix-core z transforms for the
        # mixed form; the FP32 FFT form beside it
        for dct, solve in (("matmul", "auto"), ("fft", "auto"), ("matmul", "refined")):
            rmx = run(w, "mixed", dct, steps=args.steps, warmup=args.warmup, timing_steps=args.timing_steps,
                      solve=solve)
            Xmx = rmx.pop("X")
            m = _public(rmx)
            m["dtype"] = "f32+f64"
            m["z_transform"] = "split-BF16 matrix-core products" if dct == "matmul" else "FP32 FFT"
            m["pencil_solve"] = ("FP32 sweeps + one FP64 refinement" if solve == "refined"
                                 else "FP64 sweeps")
            m["diff_vs_fp64_per_field"] = field_err(Xmx, X64, 3)
            m["steps_compared"] = r["warmup"] + args.steps
            m["speedup_vs_fp64"] = rmx["value"] / r["value"]
            out[f"mixed_{dct}" + ("" if solve == "auto" else f"_{solve}")] = m
    if not args.no_extra:
        extra = {}
        res, X2 = workload_pair(C2, WORKLOADS[C2], forms=(("auto", "auto"), ("matmul", "auto"),
                                                          ("auto", "refined")))
        extra[C2] = res
        extra[C2]["runge_kutta"] = rk_run(WORKLOADS[C2], X2)
        extra[C2]["lbvp_evp"] = lbvp_evp_run(WORKLOADS[C2])
        extra[C2]["ncc"] = ncc_run(WORKLOADS[C2], X2)
        extra[C5], _ = workload_pair(C5, WORKLOADS[C5], forms=(("auto", "auto"), ("auto", "refined")))
        extra[C4] = {"adjoint": adjoint_ratio(WORKLOADS[C4])}
        extra[C5]["adjoint"] = adjoint_mixed(dict(WORKLOADS[C5], adj_steps=200))
        out["workloads"] = extra
    if not args.no_oracle_window:
        out["oracle_window"] = {C2: oracle_window(WORKLOADS[C2])}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_3d(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
