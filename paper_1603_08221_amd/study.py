"""The paper's parametric study as batched runs (Table 1, Sec. 4).

Runs the cases of Table 1 (workloads.table1_instances: the theta and Kn_out
sweeps of Cases 2 and 7, the mole-fraction Cases 1, 3, 6, 8 and the
unequal-end Cases 4, 5, 9, 10) on the paper's 20 x 700 lattice, or another
size, as one batch of channels advanced by one sweep launch per step, until
every member is steady, and reports what Sec. 4 reads off its figures:

  - CL(t) and C~_l(t) (Eqs. (CL), (Clline); Figs. 5, 6, 8), sampled;
  - the terminal CL, C~_l and the column of the smallest C_l;
  - the steps to reach half the terminal CL (the separation rate V_s of
    Sec. 4.1 is the initial slope of CL(t); its order across runs is the order
    of these half-times, reversed);
  - the volume flow Q_v (Sec. 4.2, Fig. 7; lbsep_read_volume_flow);
  - C_l(x) every few columns (Fig. 9).

A member is steady when the species-velocity residual of R22 (levels 100
apart) is below 1e-8 and its CL changed by less than `cl_tol` (relative)
over the last chunk of steps. Argument marshalling and orchestration only:
every step runs in the HIP library.

Usage: python -m paper_1603_08221_amd.study [--ny 20] [--nx 700]
           [--max-steps 2000000] [--chunk 20000] [--out study.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import lbsep
from .workloads import table1_instances


def velocity_residual(m_now, m_then, gap: int) -> float:
    """R22: max over species of ||u_s(t) - u_s(t - gap)||_2 / (gap ||u_s(t)||_2)."""
    out = 0.0
    for k in (2, 4):
        du = np.sqrt(np.sum((m_now[k] - m_then[k]) ** 2 + (m_now[k + 1] - m_then[k + 1]) ** 2))
        un = np.sqrt(np.sum(m_now[k] ** 2 + m_now[k + 1] ** 2))
        out = max(out, float(du / (gap * un)))
    return out


def run_study(members, dtype="f64", max_steps=2_000_000, chunk=20_000, sample=1000, cl_tol=1e-4,
              res_tol=1e-8, gap=100, profile_every=10, device="cuda:0", log=None):
    """Advance `members` (Workload list) as one batch until all are steady (or
    max_steps); returns a dict per member name."""
    stream = torch.cuda.Stream(device)
    chans = []
    for w in members:
        r = lbsep.dbb_r_from_cm(w.c_m, w.m_a, w.m_b, w.cl_in)
        p = lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r, accom=w.accom,
                              dtype=dtype, hist_cap=chunk)
        chans.append(lbsep.Channel(p, device=device, stream=stream))
    batch = lbsep.Batch(chans)
    batch.capture(min(1000, chunk - gap))
    hist = {w.name: [] for w in members}
    steady_at = {w.name: None for w in members}
    last_cl = {w.name: None for w in members}
    residual = {w.name: None for w in members}
    diverged = set()
    t0 = time.perf_counter()
    while chans[0].t < max_steps:
        start = chans[0].t
        batch.step(chunk - gap)
        then = {}
        for w, c in zip(members, chans):
            if w.name not in diverged:
                then[w.name] = c.read_moments()
        batch.step(gap)
        for w, c in zip(members, chans):
            if w.name in diverged:
                continue
            try:
                h = c.read_history(start + 1, chunk)
            except lbsep.LbsepError:
                diverged.add(w.name)
                continue
            sel = h[(h[:, 0] % sample) == 0]
            hist[w.name] += [[int(a), float(b), float(cc)] for a, b, cc, _ in sel]
            try:
                cl = c.read_cl()["cl"]
            except lbsep.LbsepError:
                diverged.add(w.name)
                continue
            res = velocity_residual(c.read_moments(), then[w.name], gap)
            residual[w.name] = res
            prev = last_cl[w.name]
            last_cl[w.name] = cl
            ok = prev is not None and res < res_tol and abs(cl - prev) <= cl_tol * max(abs(cl), 1e-12)
            if ok and steady_at[w.name] is None:
                steady_at[w.name] = c.t
            elif not ok:
                steady_at[w.name] = None
        pending = [n for n in steady_at if steady_at[n] is None and n not in diverged]
        if log:
            log(f"step {chans[0].t}: {len(members) - len(pending) - len(diverged)} steady, "
                f"{len(diverged)} diverged, {time.perf_counter() - t0:.1f} s")
        if not pending:
            break
    torch.cuda.synchronize(device)
    out = {}
    for w, c in zip(members, chans):
        rec = {"nx": w.nx, "ny": w.ny, "pair": "He-Ar" if w.m_a == 4.0 else "Ne-Ar", "cl_in": w.cl_in,
               "cl_out": w.cl_out, "theta": w.theta, "kn_out": w.kn_out, "steps": c.t,
               "steady_at": steady_at[w.name], "residual": residual[w.name], "diverged": w.name in diverged}
        if w.name not in diverged:
            d = c.read_cl(profile=True)
            q = c.read_volume_flow()
            rec.update(cl=d["cl"], cl_tilde=d["cl_tilde"], x_min=d["x_min"],
                       profile=[round(v, 10) for v in d["profile"][::profile_every].tolist()],
                       q_v_mean=float(np.mean(q)), q_v_in=float(q[1]), q_v_out=float(q[-2]))
            hs = np.array(hist[w.name])
            rec["history"] = hist[w.name]
            if len(hs) and d["cl"] > 0:
                half = hs[hs[:, 1] >= 0.5 * d["cl"]]
                rec["t_half"] = int(half[0, 0]) if len(half) else None
        out[w.name] = rec
    batch.close()
    for c in chans:
        c.close()
    return out


def trend_signs(res: dict) -> dict:
    """The qualitative results of Sec. 4 from terminal values: per mixture,
    CL against theta at Kn_out = 0.3 (Sec. 4.1: falls), against Kn_out at
    theta = 2 (Sec. 4.2: rises), against C_in at theta = 2 (Sec. 4.3: falls as
    C_in rises), He-Ar above Ne-Ar at equal parameters, and the volume flow
    against Kn_out (Fig. 7: falls)."""
    def val(name, key="cl"):
        r = res.get(name)
        return None if r is None or r.get("diverged") else r.get(key)

    out = {}
    for mix, c2, clo, chi in (("He-Ar", 2, 1, 3), ("Ne-Ar", 7, 6, 8)):
        th = [val(f"c{c2}_th{t:g}_kn0.3") for t in (2, 3, 4, 5)]
        kn = [val(f"c{c2}_th2_kn{k:g}") for k in (0.3, 0.5, 1, 3, 5)]
        qv = [val(f"c{c2}_th2_kn{k:g}", "q_v_mean") for k in (0.3, 0.5, 1, 3, 5)]
        cin = [val(f"c{clo}_th2_kn0.3"), val(f"c{c2}_th2_kn0.3"), val(f"c{chi}_th2_kn0.3")]
        mono = lambda v, sgn: None if None in v else all(sgn * (b - a) > 0 for a, b in zip(v, v[1:]))
        out[mix] = {"cl_vs_theta": th, "falls_with_theta": mono(th, -1),
                    "cl_vs_kn": kn, "rises_with_kn": mono(kn, +1),
                    "q_v_vs_kn": qv, "q_v_falls_with_kn": mono(qv, -1),
                    "cl_vs_cin_0.3_0.5_0.7": cin, "falls_with_cin": mono(cin, -1)}
    he, ne = res, res
    pairs = [(f"c2_th{t:g}_kn0.3", f"c7_th{t:g}_kn0.3") for t in (2, 3, 4, 5)]
    pairs += [(f"c2_th2_kn{k:g}", f"c7_th2_kn{k:g}") for k in (0.5, 1, 3, 5)]
    cmp = [(val(a), val(b)) for a, b in pairs]
    out["he_ar_above_ne_ar"] = None if any(None in p for p in cmp) else all(a > b for a, b in cmp)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--ny", type=int, default=20)
    ap.add_argument("--nx", type=int, default=700)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--max-steps", type=int, default=2_000_000)
    ap.add_argument("--chunk", type=int, default=20_000)
    ap.add_argument("--only", default="", help="comma-separated member names (default: all of Table 1)")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    members = table1_instances(args.ny, args.nx)
    if args.only:
        keep = set(args.only.split(","))
        members = [w for w in members if w.name in keep]
    log = lambda m: (sys.stderr.write(f"[study] {m}\n"), sys.stderr.flush())
    res = run_study(members, dtype=args.dtype, max_steps=args.max_steps, chunk=args.chunk, log=log)
    out = {"lattice": [args.ny, args.nx], "dtype": args.dtype, "members": res, "trends": trend_signs(res)}
    text = json.dumps(out)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    print(json.dumps(out["trends"]))


if __name__ == "__main__":
    main()
