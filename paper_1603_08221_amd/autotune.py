"""Autotuner for the tile shape of batched and single-channel sweeps.

The sweep kernel maps nodes to lanes either as a lane pair per node (species
split; shortest chain per lane, pays when a channel leaves the GPU mostly idle)
or as one lane per node (fewest instructions per node, pays when the work
fills the GPU several times), and each wavefront of a tile walks 1, 2 or 4 rows
(more rows: fewer row-tile partial sums, less parallelism). Which shape is
faster depends on the whole launch: a small channel alone wants the lane pair
and one row, the same channel inside a batch that fills the GPU wants one lane
per node and four rows. The tuner times candidate assignments on scratch
channels (fresh workspaces, same shapes and parameters, so the caller's states
are never touched) and returns the fastest. The states are bitwise independent
of the choice (CL sums may differ in the last bits with the rows), so the
choice is a speed decision.

Choices can be cached in a JSON file keyed by the device name, the dtype and
the member shapes.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import lbsep

SPLIT, NODE = lbsep.TILE_SPLIT, lbsep.TILE_NODE


def _key(params_list, device) -> str:
    h = hashlib.sha256()
    h.update(b"tile modes and rows: by size, 2, 4 (not 4 in FP32)")
    h.update(torch.cuda.get_device_name(device).encode())
    for p in params_list:
        h.update(f"{p.nx},{p.ny},{p.dtype},{p.flags}".encode())
    return h.hexdigest()[:20]


TIE = 0.01  # relative timing difference below which two candidates tie


def candidates(params_list):
    """Assignments to try, {name: {"modes": [...], "rows": [...]}} per member:
    tile modes all lane pairs, all one-lane-per-node, and size thresholds in
    between (lane pairs for members up to T nodes), each with the rows chosen
    by size (0) and with two and four rows per wavefront. FP32 sweeps take no
    four-row candidates: their blocks of 8 wavefronts already cover 16 rows
    with two, and four made every block longer in every case measured (the
    64-member table: 203 against 185 us per step), as the library's own
    default assumes; short trial timings, under a profiler in particular, can
    still rank them first."""
    sizes = [p.nx * p.ny for p in params_list]
    modes = {"split": [SPLIT] * len(sizes), "node": [NODE] * len(sizes)}
    for t in (1 << 14, 1 << 16, 1 << 18):
        a = [SPLIT if n <= t else NODE for n in sizes]
        if a not in modes.values():
            modes[f"split<={t}"] = a
    four = not all(p.dtype == lbsep.F32 for p in params_list)
    out = {}
    for name, m in modes.items():
        out[name] = {"modes": m, "rows": [0] * len(sizes)}
        out[name + ",rows2"] = {"modes": m, "rows": [2] * len(sizes)}
        if four:
            out[name + ",rows4"] = {"modes": m, "rows": [4] * len(sizes)}
    return out


def _with_shape(p, mode, rows):
    q = lbsep.Params.from_buffer_copy(p)
    q.tile_mode = mode
    q.tile_rows = rows
    q.hist_cap = 16
    return q


def _time_batch(params_list, modes, rows, device, trial_steps, warmup):
    stream = torch.cuda.Stream(device)
    chans = [lbsep.Channel(_with_shape(p, m, r), device=device, stream=stream)
             for p, m, r in zip(params_list, modes, rows)]
    b = lbsep.Batch(chans) if len(chans) > 1 else None
    step = b.step if b is not None else chans[0].step
    step(warmup)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    stream.synchronize()
    start.record(stream)
    step(trial_steps)
    end.record(stream)
    end.synchronize()
    ms = start.elapsed_time(end) / trial_steps
    if b is not None:
        b.close()
    for c in chans:
        c.close()
    return ms


def tune(params_list, device="cuda:0", trial_steps=40, warmup=10, cache_file=None, rounds=2):
    """Fastest tile assignment for sweeping `params_list` together (one
    channel: alone). Returns {"name", "modes", "rows", "ms_per_step",
    "timings"}: set each member's tile_mode and tile_rows from modes and rows.
    Every candidate is timed once per round, round after round, and keeps its
    best time: the first round runs while the GPU's clocks are still rising
    (the FP64 table's first candidates came out 5-8% slow in a single round
    and the choice 4% slower than the best)."""
    params_list = list(params_list)
    key = _key(params_list, device)
    cache = {}
    if cache_file and os.path.exists(cache_file):
        with open(cache_file) as fh:
            cache = json.load(fh)
        if key in cache:
            return cache[key]
    timings = {}
    cands = candidates(params_list)
    for _ in range(rounds):
        for name, c in cands.items():
            ms = _time_batch(params_list, c["modes"], c["rows"], device, trial_steps, warmup)
            timings[name] = min(ms, timings.get(name, ms))
    # candidates within 1% of the fastest are a tie (trial timings move by
    # about that much between runs): the first of them in candidate order wins,
    # so the same shapes get the same assignment from run to run
    fastest = min(timings.values())
    best = next(n for n in cands if timings[n] <= fastest * (1.0 + TIE))
    out = {"name": best, "modes": cands[best]["modes"], "rows": cands[best]["rows"], "ms_per_step": timings[best],
           "timings": timings}
    if cache_file:
        cache[key] = out
        tmp = cache_file + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_file)
    return out
