"""Benchmark of the fused binary-mixture LBM step on one MI355X.

Workload (default): the single Ne-Ar channel, H = 64, L = 1280 (81,920 nodes),
C_l = 0.3, theta = 3, Kn_out = 0.05, populations initialised at local
equilibrium with a linear pressure drop. A step is one time level of the
fused sweep: both species pulled, DBB walls, inlet/outlet correction, moments,
relaxation times, MRT collision and the FP64 reduction to C_l(x), CL and C~_l.
On channels of at most 64 rows one launch advances two levels (temporal
blocking; the states are bitwise those of one level per launch).

Prints one JSON line: the FP32 path's throughput in node-MLUPS (one update =
one node with both species' 9 populations), next to the plain FP64 path, the
CL error of FP32 against FP64, the FP64 path against the CPU oracle on a short
run, the roofline of the sweep kernel and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BYTES_PER_POP = {"f64": 8, "f32": 4, "f16": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1603_08221_amd", "csrc", n)
                  for n in ("lbsep.hip", "lbsep_device.h", "e1_table.h")]


def source_hash() -> str:
    """Hash of the sweep kernel's source code with comments and blank lines
    removed (a comment edit does not change the kernel the counters measured)."""
    import re

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
        h.update("\n".join(lines).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, dtype: str, levels: int = 1, tiles: str = None):
    """HBM bytes per launch (of `levels` time levels) from the committed
    rocprofv3 PMC summary, if it was taken on the current kernel source (and,
    for a batch, with the same tile assignment `tiles`); else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    want = source_hash()
    for line in open(TRAFFIC_FILE):
        if line.startswith("#") or not line.strip():
            continue
        kv = dict(tok.split("=", 1) for tok in line.split())
        if (kv.get("workload") == workload and kv.get("dtype") == dtype and kv.get("source") == want
                and int(kv.get("levels", "1")) == levels and kv.get("tiles") == tiles):
            return float(kv["bytes_per_launch"])
    return None


def levels_per_launch(w, requested: int) -> int:
    """Time levels per sweep launch: as requested, else two on channels of at
    most 64 rows (where the two-level kernel applies), one otherwise."""
    if requested:
        return requested
    return 2 if w.ny <= 64 else 1


def make_channel(lbsep, w, dtype, hist_cap=1024, levels=1):
    r = lbsep.dbb_r_from_cm(w.c_m, w.m_a, w.m_b, w.cl_in)
    p = lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r, accom=w.accom,
                          dtype=dtype, hist_cap=hist_cap, fused_steps=levels)
    return lbsep.Channel(p, device="cuda:0"), r


def time_steps(torch, ch, steps):
    """Run exactly `steps` sweeps between two stream synchronisations; return
    (wall seconds, event milliseconds on the channel's stream)."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(ch.stream)
    ch.step(steps)
    end.record(ch.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, start.elapsed_time(end)


def batch_leg(torch, lbsep, dtype: str, steps: int):
    """The seeded 64-channel parametric sweep (uneven H in {16..128}, L = 20 H)
    as one launch per step: tile shapes from the autotuner, the step loop as a
    captured HIP graph of 100 steps, `steps` steps timed with HIP events."""
    from paper_1603_08221_amd import autotune
    from paper_1603_08221_amd.workloads import batch_instances

    ws = batch_instances()
    ps = [lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out,
                            lbsep.dbb_r_from_cm(w.c_m, w.m_a, w.m_b, w.cl_in), dtype=dtype, hist_cap=64)
          for w in ws]
    tuned = autotune.tune(ps)
    stream = torch.cuda.Stream()
    chans = []
    for p, m, rows in zip(ps, tuned["modes"], tuned["rows"]):
        p.tile_mode = m
        p.tile_rows = rows
        chans.append(lbsep.Channel(p, device="cuda:0", stream=stream))
    b = lbsep.Batch(chans)
    b.capture(100)
    b.step(100)
    stream.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    b.step(steps)
    end.record(stream)
    end.synchronize()
    wall = time.perf_counter() - t0
    nodes = sum(w.nx * w.ny for w in ws)
    per = start.elapsed_time(end) / 1e3 / steps
    alg = nodes * 36 * BYTES_PER_POP[dtype]
    diverged = 0
    for c in chans:
        try:
            c.read_cl()
        except lbsep.LbsepError:
            diverged += 1
    return {"workload": "sweep_table_64 (seed 160308221, H in {16..128}, L = 20 H)", "instances": len(ws),
            "nodes": nodes, "steps": steps, "mlups": round(nodes * steps / wall / 1e6, 1),
            "us_per_step": round(per * 1e6, 2), "gbps_algorithmic": round(alg / per / 1e9, 1),
            "frac_of_hbm_peak": round(alg / per / 1e9 / HBM_PEAK_GBS, 4), "tiles": tuned["name"],
            "tuning_ms_per_step": {k: round(v, 4) for k, v in tuned["timings"].items()},
            "graph_steps": 100, "diverged_members": diverged,
            "traffic": (lambda v: None if v is None else round(v))(measured_traffic("sweep_table_64", dtype, tiles=tuned["name"])),
            "t_final": chans[0].t}


def species_velocity_residual(m_now, m_then, gap: int) -> float:
    """max over species of ||u_s(t) - u_s(t - gap)||_2 / (gap ||u_s(t)||_2), both
    components, from two moment fields [6][ny][nx] (the steady-state test)."""
    import numpy as np

    out = 0.0
    for k in (2, 4):
        du = np.sqrt(np.sum((m_now[k] - m_then[k]) ** 2 + (m_now[k + 1] - m_then[k + 1]) ** 2))
        un = np.sqrt(np.sum(m_now[k] ** 2 + m_now[k + 1] ** 2))
        out = max(out, float(du / (gap * un)))
    return out


def steady_leg(torch, lbsep, w, max_steps: int = 50000, check_every: int = 1000, gap: int = 100,
               tol: float = 1e-8):
    """The headline channel run to steady state (species-velocity residual
    below tol between levels `gap` apart, checked every `check_every` steps, or
    max_steps) in FP32 deviation storage and in FP64: steps taken, residual,
    CL, C~_l and the C_l(x) profile every 64 columns, FP32 against FP64."""
    out = {}
    for dtype in ("f32", "f64"):
        ch, _ = make_channel(lbsep, w, dtype, hist_cap=64)
        t0 = time.perf_counter()
        res = float("inf")
        while ch.t < max_steps:
            ch.step(check_every - gap)
            m_then = ch.read_moments()
            ch.step(gap)
            res = species_velocity_residual(ch.read_moments(), m_then, gap)
            if res < tol:
                break
        cl = ch.read_cl(profile=True)
        out[dtype] = {"steps": ch.t, "residual": res, "seconds": round(time.perf_counter() - t0, 2),
                      "cl": cl["cl"], "cl_tilde": cl["cl_tilde"], "x_min": cl["x_min"],
                      "cl_profile_every_64": [round(v, 9) for v in cl["profile"][::64].tolist()]}
        del ch
    out["cl_err_f32_vs_f64"] = abs(out["f32"]["cl"] - out["f64"]["cl"])
    out["workload"] = w.name
    out["criterion"] = f"residual < {tol} (levels {gap} apart) or {max_steps} steps"
    return out


def precision_leg(torch, lbsep, steps: int):
    """He-Ar 256 x 5120 (C_l 0.5, theta 2, Kn_out 0.2) for `steps` steps in FP64,
    FP32-deviation and FP16-deviation storage: time per step and the CL and
    C~_l error of each reduced-precision run against the FP64 run."""
    from paper_1603_08221_amd.workloads import CONFIGS

    wl = CONFIGS["he_ar_256x5120"]
    res = {"workload": wl.name, "steps": steps}
    ref = None
    for dtype in ("f64", "f32", "f16"):
        ch, _ = make_channel(lbsep, wl, dtype, hist_cap=64)
        ch.step(10)
        wall, ev = time_steps(torch, ch, steps - 10)
        cl = ch.read_cl()
        entry = {"us_per_step": round(ev * 1e3 / (steps - 10), 2),
                 "mlups": round(wl.nodes * (steps - 10) / wall / 1e6, 1),
                 "cl": cl["cl"], "cl_tilde": cl["cl_tilde"]}
        if ref is None:
            ref = cl
        else:
            entry["cl_err_vs_f64"] = abs(cl["cl"] - ref["cl"])
            entry["cl_tilde_err_vs_f64"] = abs(cl["cl_tilde"] - ref["cl_tilde"])
        res[dtype] = entry
        del ch
    return res


def adjoint_leg(torch, lbsep, steps: int):
    """dCL/d(theta, C_in, r) of the He-Ar 64 x 1280 channel (C_l 0.5, theta 2.5,
    Kn_out 0.1, FP64) over `steps` steps with checkpoints every 500: wall time of
    the whole gradient (forward, recomputation, reverse sweep)."""
    from paper_1603_08221_amd.adjoint import cl_gradient
    from paper_1603_08221_amd.workloads import CONFIGS

    w = CONFIGS["he_ar_64x1280"]
    r = lbsep.dbb_r_from_cm(w.c_m, w.m_a, w.m_b, w.cl_in)
    p = lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r, dtype="f64",
                          hist_cap=64)
    cl_gradient(p, 200, checkpoint_every=100)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cl, g = cl_gradient(p, steps, checkpoint_every=500)
    wall = time.perf_counter() - t0
    g = g.cpu().tolist()
    return {"workload": w.name, "steps": steps, "checkpoint_every": 500, "seconds": round(wall, 3),
            "cl": cl, "dcl_dtheta": g[0], "dcl_dcl_in": g[1], "dcl_dr": g[2],
            "us_per_step_forward_recompute_reverse": round(wall / steps * 1e6, 2)}


def cpu_baseline(w, r, seconds: float):
    """The CPU oracle as it stands, on the same workload, for a bounded number
    of steps (about `seconds` of CPU work), single BLAS thread."""
    from threadpoolctl import threadpool_limits

    from oracle import binary_lbm as O

    p = O.Params(nx=w.nx, ny=w.ny, m_a=w.m_a, m_b=w.m_b, cl_in=w.cl_in, cl_out=w.cl_out, theta=w.theta,
                 kn_out=w.kn_out, dbb_r=r, accom=w.accom)
    with threadpool_limits(limits=1):
        f = O.initial_state(p)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < seconds:
            f = O.step(f, p)
            n += 1
        dt = time.perf_counter() - t0
    return {"value": w.nodes * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of {w.name} ({w.ny}x{w.nx}) from the initial state, NumPy FP64, "
                      f"{dt:.1f} s, 1 BLAS thread"}


def oracle_parity(lbsep, w, r, steps: int):
    """CL and moments of the GPU FP64 path against the oracle after `steps` steps."""
    import numpy as np

    from oracle import binary_lbm as O

    p = O.Params(nx=w.nx, ny=w.ny, m_a=w.m_a, m_b=w.m_b, cl_in=w.cl_in, cl_out=w.cl_out, theta=w.theta,
                 kn_out=w.kn_out, dbb_r=r, accom=w.accom)
    f, _ = O.run(p, steps)
    d = O.diagnostics(f, p)
    ref = O.moment_fields(f, p)
    ch, _ = make_channel(lbsep, w, "f64")
    ch.step(steps)
    mom = ch.read_moments()
    cl = ch.read_cl()["cl"]
    rho_err = max(float(np.max(np.abs(mom[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in (0, 1))
    return {"steps": steps, "cl_abs_err": abs(cl - d.cl), "rho_rel_err": rho_err}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="ne_ar_64x1280")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "f64"])
    ap.add_argument("--levels", type=int, default=0, choices=[0, 1, 2],
                    help="time levels per sweep launch (0: two on channels of at most 64 rows, else one)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference leg (profiling runs)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the leg on the 512 x 10240 channel (above the last-level cache)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-channel batched sweep leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-gradient leg")
    ap.add_argument("--no-steady", action="store_true", help="skip the run of the channel to steady state")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP64 / FP32 / FP16 storage comparison on the 256 x 5120 channel")
    ap.add_argument("--precision-steps", type=int, default=100000)
    ap.add_argument("--adjoint-steps", type=int, default=10000)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this size (PMC calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs one channel on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1603_08221_amd import lbsep
    from paper_1603_08221_amd.workloads import CONFIGS

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}))
        return

    w = CONFIGS[args.workload]
    levels = levels_per_launch(w, args.levels)
    if args.steps % levels or args.warmup % levels:
        sys.exit(f"--steps and --warmup must be multiples of the {levels} levels per launch")
    ch, r = make_channel(lbsep, w, args.dtype, levels=levels)
    ch.step(args.warmup)
    torch.cuda.synchronize()
    wall, ev_ms = time_steps(torch, ch, args.steps)
    t_total = ch.t
    cl32 = ch.read_cl()
    mlups = w.nodes * args.steps / wall / 1e6
    per_launch_s = ev_ms / 1e3 / (args.steps // levels)
    alg_bytes = levels * w.nodes * 36 * BYTES_PER_POP[args.dtype]
    achieved = alg_bytes / per_launch_s / 1e9

    out = {
        "metric": "MLUPS (both species) + achieved HBM GB/s vs FP64 plain, at CL error <=1e-5",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "mixture": "Ne-Ar" if w.m_a == 20 else "He-Ar",
                   "cl_in": w.cl_in, "theta": w.theta, "kn_out": w.kn_out, "dbb_r": r,
                   "storage": {"f32": "f32 deviation", "f16": "f16 deviation", "f64": "f64"}[args.dtype],
                   "levels_per_launch": levels,
                   "parallelism": "single GPU"},
        "gbps_algorithmic": round(achieved, 1),
        "cl": cl32["cl"],
        "t_final": t_total,
    }

    traffic = measured_traffic(w.name, args.dtype, levels)
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": None if traffic is None else round(traffic)}
    kname = "k_sweep2" if levels == 2 else "k_sweep"
    out["roofline_note"] = (f"{kname}, algorithmic bytes {alg_bytes} per launch ({levels} level(s) x 36 populations x "
                            f"{BYTES_PER_POP[args.dtype]} B x {w.nodes} nodes) / {per_launch_s * 1e6:.2f} us mean "
                            "launch time (HIP events on the channel stream)")

    if not args.no_fp64:
        ch64, _ = make_channel(lbsep, w, "f64", levels=levels)
        ch64.step(args.warmup)
        wall64, ev64 = time_steps(torch, ch64, args.steps)
        cl64 = ch64.read_cl()
        out["fp64"] = {"mlups": round(w.nodes * args.steps / wall64 / 1e6, 1),
                       "ms_per_step": wall64 * 1e3 / args.steps,
                       "gbps_algorithmic": round(w.nodes * 288 / (ev64 / 1e3 / args.steps) / 1e9, 1),
                       "cl": cl64["cl"]}
        out["cl_err_vs_fp64"] = abs(cl32["cl"] - cl64["cl"])
        out["cl_ok"] = out["cl_err_vs_fp64"] <= 1e-5
        del ch64
    if not args.no_large and w.name != "he_ar_512x10240":
        wl = CONFIGS["he_ar_512x10240"]
        chl, _ = make_channel(lbsep, wl, args.dtype, hist_cap=64)
        chl.step(20)
        nl = 200
        wall_l, ev_l = time_steps(torch, chl, nl)
        bl = wl.nodes * 36 * BYTES_PER_POP[args.dtype]
        gbs = bl / (ev_l / 1e3 / nl) / 1e9
        tr = measured_traffic(wl.name, args.dtype)
        out["large_channel"] = {"workload": wl.name, "steps": nl, "mlups": round(wl.nodes * nl / wall_l / 1e6, 1),
                                "us_per_step": round(ev_l * 1e3 / nl, 2), "gbps_algorithmic": round(gbs, 1),
                                "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                                "traffic": None if tr is None else round(tr), "cl": chl.read_cl()["cl"]}
        del chl
    if not args.no_batch:
        out["batch"] = batch_leg(torch, lbsep, args.dtype, args.batch_steps)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(torch, lbsep, args.adjoint_steps)
    if not args.no_steady:
        out["steady_state"] = steady_leg(torch, lbsep, w)
    if not args.no_precision:
        out["precision"] = precision_leg(torch, lbsep, args.precision_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, r, args.cpu_seconds)
        out["fp64_vs_oracle"] = oracle_parity(lbsep, w, r, 100)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
