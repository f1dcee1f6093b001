"""Batched sweeps (one launch per step over an instance table, optional HIP
graph of the step loop): each member channel must evolve bitwise as it does
when stepped alone (same kernels, same per-channel reductions), and so match
the FP64 oracle wherever the single-channel path does."""
import numpy as np
import pytest
import torch

from oracle import binary_lbm as O
from paper_1603_08221_amd import lbsep
from paper_1603_08221_amd.workloads import HE_AR, NE_AR, Workload, batch_instances

from gpu_helpers import assert_argmin, assert_cl, assert_moments, oracle_params, r_of

pytestmark = pytest.mark.gpu

# uneven members: lane-pair tiles (small) and one-lane-per-node tiles (the
# 132 x 4000 channel has more than 2^16 nodes), ragged edges in x and y
MEMBERS = [
    Workload("b0", 80, 8, *HE_AR, 0.5, 0.5, 2.0, 0.1, 0),
    Workload("b1", 333, 24, *NE_AR, 0.3, 0.3, 3.0, 0.05, 0),
    Workload("b2", 150, 13, *HE_AR, 0.7, 0.4, 2.5, 0.5, 0),
    Workload("b3", 4000, 132, *HE_AR, 0.5, 0.5, 2.0, 0.2, 0),
    Workload("b4", 640, 32, *NE_AR, 0.6, 0.6, 1.5, 0.01, 0),
]


def _make(ws, dtype, stream=None):
    out = []
    for w in ws:
        p = lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r_of(w),
                              dtype=dtype, hist_cap=512)
        out.append(lbsep.Channel(p, device="cuda:0", stream=stream))
    return out


def _same(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        assert torch.equal(x.get_state(), y.get_state()), f"{what}: member {k} state differs"
        ca, cb = x.read_cl(profile=True), y.read_cl(profile=True)
        assert ca["cl"] == cb["cl"] and np.array_equal(ca["profile"], cb["profile"]), f"{what}: member {k} CL"
        assert x.t == y.t


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
def test_batch_matches_members_stepped_alone(dtype):
    batched = _make(MEMBERS, dtype)
    alone = _make(MEMBERS, dtype)
    b = lbsep.Batch(batched)
    assert len(b) == len(MEMBERS)
    b.step(1)
    b.step(149)
    for c in alone:
        c.step(150)
    _same(batched, alone, "after 150 steps")
    # readouts between batch steps do not disturb the batch
    b.step(7)
    for c in alone:
        c.step(7)
    _same(batched, alone, "after 157 steps")


def test_batch_fp64_members_match_the_oracle():
    ws = MEMBERS[:3]
    chans = _make(ws, "f64")
    b = lbsep.Batch(chans)
    b.step(300)
    for w, c in zip(ws, chans):
        p = oracle_params(w, r_of(w))
        f, _ = O.run(p, 300)
        assert_moments(c.read_moments(), O.moment_fields(f, p), 1e-12, w.name)
        assert_cl(c.read_cl()["cl"], O.diagnostics(f, p).cl, 0.0, 1e-12)


def test_batch_graph_replays_match_eager_steps():
    """The captured step loop, replayed several times with eager work and
    synchronisations between the replays, gives the eager result every time;
    step counts that are not a multiple of the graph length finish eagerly."""
    stream = torch.cuda.Stream()
    batched = _make(MEMBERS, "f32", stream=stream)
    alone = _make(MEMBERS, "f32")
    b = lbsep.Batch(batched)
    b.capture(25)
    total = 0
    for rep, n in enumerate((25, 25, 50, 30, 7)):
        b.step(n)
        total += n
        for c in alone:
            c.step(n)
        torch.cuda.synchronize()
        _same(batched, alone, f"replay round {rep} ({total} steps)")
    b.capture(0)  # dropped: plain launches again
    b.step(5)
    for c in alone:
        c.step(5)
    _same(batched, alone, "after dropping the graph")


def test_batch_rejects_members_stepped_alone_and_mixed_inputs():
    chans = _make(MEMBERS[:2], "f32")
    b = lbsep.Batch(chans)
    b.step(3)
    chans[0].step(1)
    with pytest.raises(lbsep.LbsepError) as e:
        b.step(1)
    assert e.value.code == lbsep.EINVAL and "outside its batch" in str(e.value)
    # a member reset to the level it already has: same t, other state
    chans = _make(MEMBERS[:2], "f32")
    b = lbsep.Batch(chans)
    b.step(4)
    chans[1].set_state(chans[1].get_state(), chans[1].t)
    with pytest.raises(lbsep.LbsepError) as e:
        b.step(1)
    assert e.value.code == lbsep.EINVAL and "outside its batch" in str(e.value)
    # set_state one level back, then one step alone: t is the batch's again
    chans = _make(MEMBERS[:2], "f32")
    b = lbsep.Batch(chans)
    b.step(4)
    chans[0].set_state(chans[0].get_state(), chans[0].t - 1)
    chans[0].step(1)
    with pytest.raises(lbsep.LbsepError) as e:
        b.step(1)
    assert e.value.code == lbsep.EINVAL and "outside its batch" in str(e.value)
    # readouts do not count as changes
    chans = _make(MEMBERS[:2], "f32")
    b = lbsep.Batch(chans)
    b.step(2)
    chans[0].read_cl()
    chans[0].get_state()
    chans[1].read_moments()
    b.step(2)
    mixed = _make(MEMBERS[:1], "f32") + _make(MEMBERS[1:2], "f64")
    with pytest.raises(lbsep.LbsepError):
        lbsep.Batch(mixed)
    with pytest.raises(lbsep.LbsepError):
        lbsep.Batch([chans[1], chans[1]])
    with pytest.raises(lbsep.LbsepError):
        b.capture(10)  # default stream: no capture


def _bits(t):
    return t.view({torch.float64: torch.int64, torch.float32: torch.int32, torch.float16: torch.int16}[t.dtype])


def _cl_or_error(c):
    try:
        return c.read_cl()["cl"]
    except lbsep.LbsepError as e:
        assert e.code == lbsep.ENONFINITE
        return "non-finite"


def test_batch_of_the_sweep_table_matches_members_stepped_alone():
    """The 64-instance parametric table (seeded uneven H, C_l, theta, Kn_out),
    FP32, 300 steps in one launch per step, against the same channels stepped
    alone: bitwise equal states (NaN patterns included) and the same CL or the
    same non-finite report. Some members with a mean free path below about one
    lattice spacing diverge under the scheme itself (the oracle diverges on one
    of them too, see the oracle pins): the batch must reproduce that, not hide it."""
    ws = batch_instances()
    batched = _make(ws, "f32")
    b = lbsep.Batch(batched)
    b.step(300)
    for k, w in enumerate(ws):
        alone = _make([w], "f32")[0]
        alone.step(300)
        assert torch.equal(_bits(batched[k].get_state()), _bits(alone.get_state())), w.name
        assert _cl_or_error(batched[k]) == _cl_or_error(alone), w.name
        del alone


def test_autotuner_picks_a_candidate_and_caches_it(tmp_path):
    from paper_1603_08221_amd import autotune

    ps = [lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r_of(w), dtype="f32")
          for w in MEMBERS]
    cache = str(tmp_path / "tune.json")
    got = autotune.tune(ps, trial_steps=5, warmup=2, cache_file=cache)
    cands = autotune.candidates(ps)
    assert got["name"] in cands and cands[got["name"]] == {"modes": got["modes"], "rows": got["rows"]}
    # an all-FP32 table: two-row candidates, none with four rows per wavefront
    assert any(c["rows"] == [2] * len(ps) for c in cands.values())
    assert not any(4 in c["rows"] for c in cands.values())
    # the tie rule: the first candidate (in candidate order) within TIE of the fastest wins
    fastest = min(got["timings"].values())
    assert fastest > 0
    first = next(n for n in cands if got["timings"][n] <= fastest * (1.0 + autotune.TIE))
    assert got["name"] == first and got["ms_per_step"] == got["timings"][first]
    again = autotune.tune(ps, trial_steps=5, warmup=2, cache_file=cache)
    assert again == got  # served from the cache
    # the tuned assignment runs the same arithmetic: a tuned batch equals the default one
    tuned = []
    for w, m, rows in zip(MEMBERS, got["modes"], got["rows"]):
        p = lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r_of(w),
                              dtype="f32", hist_cap=512, tile_mode=m, tile_rows=rows)
        tuned.append(lbsep.Channel(p, device="cuda:0"))
    plain = _make(MEMBERS, "f32")
    lbsep.Batch(tuned).step(40)
    lbsep.Batch(plain).step(40)
    for a, b in zip(tuned, plain):
        assert torch.equal(a.get_state(), b.get_state())


# two levels per launch: members of at most 128 rows (64 in FP64)
MEMBERS2 = [
    Workload("d0", 80, 8, *HE_AR, 0.5, 0.5, 2.0, 0.1, 0),
    Workload("d1", 333, 24, *NE_AR, 0.3, 0.3, 3.0, 0.05, 0),
    Workload("d2", 150, 13, *HE_AR, 0.7, 0.4, 2.5, 0.5, 0),
    Workload("d3", 1000, 100, *HE_AR, 0.5, 0.5, 2.0, 0.2, 0),
    Workload("d4", 640, 64, *NE_AR, 0.6, 0.6, 1.5, 0.03, 0),
    Workload("d5", 40, 128, *HE_AR, 0.45, 0.45, 1.5, 0.3, 0),
]


def _make2(ws, dtype, fused, stream=None):
    out = []
    for w in ws:
        p = lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r_of(w),
                              dtype=dtype, hist_cap=512, fused_steps=fused)
        out.append(lbsep.Channel(p, device="cuda:0", stream=stream))
    return out


def _same_states(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        assert x.t == y.t, what
        assert torch.equal(_bits(x.get_state()), _bits(y.get_state())), f"{what}: member {k} state"
        assert torch.equal(_bits(x.get_post_collision()), _bits(y.get_post_collision())), f"{what}: member {k} post"
        ca, cb = x.read_cl(profile=True), y.read_cl(profile=True)
        # column sums are grouped per tile, so CL agrees to rounding
        assert abs(ca["cl"] - cb["cl"]) <= 1e-12 * abs(ca["cl"]) + 1e-14, f"{what}: member {k} CL"
        np.testing.assert_allclose(cb["profile"], ca["profile"], rtol=1e-13, atol=0, err_msg=what)


@pytest.mark.parametrize("dtype", ["f32", "f16", "f64"])
def test_two_level_batch_matches_members_stepped_alone(dtype):
    """A batch of two-level channels (one launch per two levels, the last of
    one level when the count is odd) against the same channels stepped alone
    with one level per launch: bitwise equal states, CL to rounding, with
    readouts and a reset between batch steps refused."""
    ws = [w for w in MEMBERS2 if dtype != "f64" or w.ny <= 64]
    stream = torch.cuda.Stream()
    batched = _make2(ws, dtype, 2, stream=stream)
    alone = _make2(ws, dtype, 1)
    b = lbsep.Batch(batched)
    total = 0
    for n in (2, 5, 1, 40):
        b.step(n)
        total += n
        for c in alone:
            c.step(n)
        torch.cuda.synchronize()
        _same_states(batched, alone, f"{dtype}, {total} levels")
    b.capture(10)
    for n in (10, 20, 13):  # replays, then an odd rest
        b.step(n)
        total += n
        for c in alone:
            c.step(n)
        torch.cuda.synchronize()
        _same_states(batched, alone, f"{dtype}, graph, {total} levels")
    t0 = total - 20
    for x, y in zip(batched, alone):
        ha, hb = x.read_history(t0, 21), y.read_history(t0, 21)
        np.testing.assert_array_equal(ha[:, 0], hb[:, 0])
        np.testing.assert_allclose(ha[:, 1:3], hb[:, 1:3], rtol=1e-11, atol=1e-14)
    batched[0].step(1)
    with pytest.raises(lbsep.LbsepError, match="outside its batch"):
        b.step(2)


def test_two_level_batch_of_the_sweep_table_matches_the_one_level_batch():
    """The 64-member parametric table (every member has at most 128 rows) in
    FP32: two levels per launch against one, bitwise equal states after 60
    levels (the members that diverge do so identically)."""
    ws = batch_instances()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    one = _make2(ws, "f32", 1, stream=s1)
    two = _make2(ws, "f32", 2, stream=s2)
    b1, b2 = lbsep.Batch(one), lbsep.Batch(two)
    b2.capture(20)
    b1.step(60)
    b2.step(60)
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(one, two)):
        assert torch.equal(_bits(x.get_state()), _bits(y.get_state())), ws[k].name
        assert _cl_or_error(x) == pytest.approx(_cl_or_error(y), rel=1e-12, abs=1e-14) \
            if _cl_or_error(x) != "non-finite" else _cl_or_error(y) == "non-finite"


def test_table1_runs_as_one_batch_match_the_oracle():
    """Runs of Table 1 (workloads.table1_instances on an 8 x 280 lattice, the
    paper's L/H = 35) of every kind: the theta and Kn_out sweeps of cases 2
    (He-Ar) and 7 (Ne-Ar), the mole fractions of cases 1 and 8, the unequal
    ends of cases 4 and 10. They advance as one FP64 batch through a
    captured graph for 400 steps, and each is checked against the oracle:
    moments to 1e-12, CL, C~_l and x_min, and the CL record every 50 steps."""
    from paper_1603_08221_amd.workloads import table1_instances

    names = ["c2_th4_kn0.3", "c2_th2_kn3", "c7_th3_kn0.3", "c7_th2_kn5", "c1_th2_kn0.3", "c8_th4_kn0.3",
             "c4_th2_kn1", "c10_th2_kn0.3"]
    runs = {w.name: w for w in table1_instances(8, 280)}
    ws = [runs[n] for n in names]
    stream = torch.cuda.Stream()
    chans = _make(ws, "f64", stream)
    b = lbsep.Batch(chans)
    b.capture(100)
    print(f"[case] Table 1 runs {names} as one batch, 400 steps", flush=True)
    b.step(400)
    for w, c in zip(ws, chans):
        p = oracle_params(w, r_of(w))
        f, hist = O.run(p, 400, record_every=50)
        d = O.diagnostics(f, p)
        assert_moments(c.read_moments(), O.moment_fields(f, p), 1e-12, w.name)
        got = c.read_cl(profile=True)
        assert_cl(got["cl"], d.cl, 0.0, 1e-12)
        assert_cl(got["cl_tilde"], d.cl_tilde, 0.0, 1e-12)
        assert_argmin(got["x_min"], d.cl_profile)
        rec = c.read_history(0, 401)
        for t, cl, clt in hist:
            assert abs(rec[t, 1] - cl) <= 1e-12 and abs(rec[t, 2] - clt) <= 1e-12, (w.name, t)
    b.close()
