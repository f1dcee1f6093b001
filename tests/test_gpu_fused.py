"""Two time levels per launch (fused_steps = 2) against single-level launches.

Each node of a two-level launch goes through the same arithmetic as in two
single-level sweeps (the first level kept in LDS in the storage type, kappa
of Eq. (rho2) summed in the same order), so the states must agree bitwise;
CL, the C_l profile and the history come from column sums grouped by other
tiles and agree to rounding. Readouts and checkpoints right after a
two-level launch recompute the level before; they must agree bitwise too.
The FP64 two-level path is also checked against the oracle directly."""
import numpy as np
import pytest
import torch

from oracle import binary_lbm as O
from paper_1603_08221_amd import lbsep
from paper_1603_08221_amd.workloads import CONFIGS, HE_AR, NE_AR, Workload

from gpu_helpers import assert_argmin, assert_cl, assert_moments, oracle_params, r_of

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

# (nx, ny): one tile; ragged tiles in x and y; several tiles; the most rows
# two-level launches take (64); the smallest channel (no tiles: the end blocks
# own every column); one tile column; nine columns (the two ends' LDS strips
# overlap); two rows (both walls)
SHAPES = [(80, 8), (150, 13), (517, 24), (200, 64), (6, 7), (7, 5), (9, 11), (70, 2)]


def _params(w, fused, dtype, hist_cap=512):
    return lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r_of(w),
                             dtype=dtype, hist_cap=hist_cap, fused_steps=fused)


def _pair(w, dtype):
    return lbsep.Channel(_params(w, 1, dtype)), lbsep.Channel(_params(w, 2, dtype))


def _agree(a, b, what, dtype="f64"):
    assert a.t == b.t, what
    assert torch.equal(a.get_post_collision(), b.get_post_collision()), f"{what}: post-collision state"
    assert torch.equal(a.get_populations(), b.get_populations()), f"{what}: pre-collision populations"
    ca, cb = a.read_cl(profile=True), b.read_cl(profile=True)
    # CL = (C_in - min C_l) / C_in: rounding of C_l is absolute, ~1e-16
    assert abs(ca["cl"] - cb["cl"]) <= 1e-12 * abs(ca["cl"]) + 1e-14, what
    np.testing.assert_allclose(cb["profile"], ca["profile"], rtol=1e-13, atol=0, err_msg=what)
    assert_argmin(cb["x_min"], ca["profile"], 1e-12)


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[0]}x{s[1]}" for s in SHAPES])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
def test_two_levels_per_launch_match_single_levels(dtype, shape):
    w = Workload("fused", shape[0], shape[1], *NE_AR, 0.3, 0.6, 2.5, 0.08, 0)
    a, b = _pair(w, dtype)
    _agree(a, b, "initial state", dtype)
    for n in (2, 1, 3, 6, 40):  # odd counts end with a single-level launch
        a.step(n)
        b.step(n)
        _agree(a, b, f"t = {a.t}", dtype)
    if dtype == "f16":
        return
    t0 = max(1, a.t - 50)
    ha, hb = a.read_history(t0, a.t - t0 + 1), b.read_history(t0, b.t - t0 + 1)
    np.testing.assert_array_equal(ha[:, 0], hb[:, 0])
    np.testing.assert_allclose(hb[:, 1:3], ha[:, 1:3], rtol=1e-11, atol=1e-14)


def test_fp64_two_levels_match_single_levels_with_the_piecewise_wall_function():
    """An FP64 channel of more than 2^17 nodes evaluates the wall function from
    the piecewise polynomials: in the single-level sweep compiled for it and,
    switched at run time, in the two-level kernel; the states stay bitwise
    equal."""
    w = Workload("fused-table", 2100, 64, *HE_AR, 0.5, 0.5, 2.0, 0.1, 0)
    assert w.nx * w.ny > 1 << 17
    a, b = _pair(w, "f64")
    for n in (2, 1, 5):
        a.step(n)
        b.step(n)
        _agree(a, b, f"t = {a.t}")


# channels of 65 to 128 rows: two end blocks per end in single-level launches,
# one two-level end block of 512 nodes (deviation storage only)
TALL = [(200, 100), (90, 128), (150, 65), (9, 127)]


@pytest.mark.parametrize("shape", TALL, ids=[f"{s[0]}x{s[1]}" for s in TALL])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_two_levels_per_launch_on_channels_up_to_128_rows(dtype, shape):
    w = Workload("fused_tall", shape[0], shape[1], *HE_AR, 0.4, 0.55, 2.5, 0.1, 0)
    a, b = _pair(w, dtype)
    _agree(a, b, "initial state", dtype)
    for n in (2, 3, 36):
        a.step(n)
        b.step(n)
        _agree(a, b, f"t = {a.t}", dtype)
    t0 = max(1, a.t - 30)
    ha, hb = a.read_history(t0, a.t - t0 + 1), b.read_history(t0, b.t - t0 + 1)
    np.testing.assert_allclose(hb[:, 1:3], ha[:, 1:3], rtol=1e-11, atol=1e-14)


def test_two_levels_per_launch_limits():
    """FP64 end blocks hold at most 64 rows, the deviation modes 128."""
    w = Workload("fused_lim", 90, 65, *HE_AR, 0.4, 0.4, 2.0, 0.1, 0)
    with pytest.raises(lbsep.LbsepError, match="64 in FP64"):
        lbsep.Channel(_params(w, 2, "f64"))
    with pytest.raises(lbsep.LbsepError, match="128"):
        lbsep.Channel(_params(w.with_(ny=129), 2, "f32"))
    lbsep.Channel(_params(w.with_(ny=128), 2, "f32")).step(2)


VARIANTS = {
    # the wall function off (constant relaxation times from the mean free path)
    "mfp_off": dict(flags=lbsep.MFP_OFF),
    # single-relaxation-time test mode
    "bgk": dict(flags=lbsep.BGK_TEST, tau_bgk=0.9),
    # unequal inlet and outlet concentrations, partial accommodation
    "cl_in_ne_cl_out": dict(cl_out=0.45, accom=0.7),
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_levels_per_launch_with_model_variants(dtype, variant):
    kw = dict(VARIANTS[variant])
    w = Workload("fused", 90, 12, *HE_AR, 0.3, kw.pop("cl_out", 0.6), 2.0, 0.1, 0)
    mk = lambda fused: lbsep.Channel(lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta,
                                                       w.kn_out, r_of(w), dtype=dtype, hist_cap=512,
                                                       fused_steps=fused, **kw))
    a, b = mk(1), mk(2)
    for n in (4, 7):
        a.step(n)
        b.step(n)
        _agree(a, b, f"{variant}, t = {a.t}", dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_checkpoint_after_a_two_level_launch_resumes_bitwise(dtype):
    w = CONFIGS["he_ar_8x80"].with_(nx=130, ny=20)
    a = lbsep.Channel(_params(w, 2, dtype))
    a.step(10)  # ends on a two-level launch
    snap, t = a.get_state(), a.t
    a.step(8)
    b = lbsep.Channel(_params(w, 2, dtype))
    b.set_state(snap, t)
    b.step(8)
    assert torch.equal(a.get_post_collision(), b.get_post_collision())
    assert a.read_cl()["cl"] == b.read_cl()["cl"]
    # the same checkpoint resumed by single-level launches: same states
    c = lbsep.Channel(_params(w, 1, dtype))
    c.set_state(snap, t)
    c.step(8)
    assert torch.equal(a.get_post_collision(), c.get_post_collision())


@pytest.mark.parametrize("hist_cap", [1, 3, 4])
def test_history_ring_wraps_inside_two_level_launches(hist_cap):
    """A history ring shorter than a launch's two records: the last hist_cap
    records agree with single-level launches, older levels are out of range."""
    w = CONFIGS["he_ar_8x80"].with_(nx=120, ny=10)
    a = lbsep.Channel(_params(w, 1, "f64", hist_cap=hist_cap))
    b = lbsep.Channel(_params(w, 2, "f64", hist_cap=hist_cap))
    for n in (5, 6, 3):
        a.step(n)
        b.step(n)
        t0 = a.t - hist_cap + 1
        ha, hb = a.read_history(t0, hist_cap), b.read_history(t0, hist_cap)
        np.testing.assert_array_equal(hb[:, 0], ha[:, 0])
        np.testing.assert_array_equal(hb[:, 3], ha[:, 3])
        np.testing.assert_allclose(hb[:, 1:3], ha[:, 1:3], rtol=1e-11, atol=1e-14)
        with pytest.raises(lbsep.LbsepError):
            b.read_history(t0 - 1, 1)


def test_set_populations_restarts_the_two_level_pipeline():
    """Physical populations loaded into a two-level channel mid-run continue
    bitwise like a single-level channel loaded with the same populations."""
    w = CONFIGS["he_ar_8x80"].with_(nx=110, ny=14)
    src = lbsep.Channel(_params(w, 1, "f64"))
    src.step(13)
    f, t = src.get_populations(), src.t
    a = lbsep.Channel(_params(w, 1, "f64"))
    b = lbsep.Channel(_params(w, 2, "f64"))
    b.step(6)  # mid-run: levels pending in the two-level pipeline
    a.set_populations(f, t)
    b.set_populations(f, t)
    for n in (2, 5):
        a.step(n)
        b.step(n)
        _agree(a, b, f"after set_populations, t = {a.t}")


def test_moments_after_a_two_level_launch():
    w = CONFIGS["he_ar_8x80"].with_(nx=100, ny=12)
    a, b = _pair(w, "f64")
    a.step(12)
    b.step(12)
    np.testing.assert_array_equal(a.read_moments(), b.read_moments())
    np.testing.assert_array_equal(a.read_volume_flow(), b.read_volume_flow())


def test_fp64_two_level_path_against_the_oracle():
    w = CONFIGS["he_ar_8x80"]
    r = r_of(w)
    ch = lbsep.Channel(_params(w, 2, "f64", hist_cap=4096))
    ch.step(2000)
    p = oracle_params(w, r)
    f, _ = O.run(p, 2000)
    assert_moments(ch.read_moments(), O.moment_fields(f, p), TOL64, "fused, 2000 steps")
    assert_cl(ch.read_cl()["cl"], O.diagnostics(f, p).cl, 0.0, 1e-12)


def test_one_and_two_level_channels_do_not_share_a_batch():
    w = CONFIGS["he_ar_8x80"]
    a = lbsep.Channel(_params(w, 1, "f32"))
    b = lbsep.Channel(_params(w, 2, "f32"))
    with pytest.raises(lbsep.LbsepError, match="fused_steps"):
        lbsep.Batch([a, b])
