"""The hand-written discrete adjoint (HIP, through the C ABI) against the CPU
FP64 reverse sweep (oracle/adjoint.py: reverse-mode differentiation of the
oracle's step) and against central finite differences of the GPU forward."""
import numpy as np
import pytest
import torch

from oracle import adjoint as A
from oracle import binary_lbm as O
from paper_1603_08221_amd import lbsep
from paper_1603_08221_amd.adjoint import Adjoint, SeparationDegree, cl_gradient
from paper_1603_08221_amd.workloads import CONFIGS, HE_AR, NE_AR, Workload

from gpu_helpers import channel, oracle_params, r_of

pytestmark = pytest.mark.gpu

SMALL = Workload("adj", 40, 6, *HE_AR, 0.5, 0.5, 2.0, 0.1, 0)
MODES = [{}, {"periodic_x": True}, {"periodic_y": True, "mfp_off": True}, {"mfp_off": True}]


def _state(p, seed=3):
    rng = np.random.default_rng(seed)
    f = O.initial_state(p) if not p.periodic_x else O.initial_state(
        O.Params(**{**p.__dict__, "periodic_x": False}))
    return f * (1.0 + 0.02 * rng.uniform(-1, 1, size=f.shape))


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("modes", MODES, ids=["walls+ends", "periodic_x", "periodic_y+mfp_off", "mfp_off"])
def test_adjoint_step_matches_the_cpu_reverse_sweep(modes):
    w = SMALL.with_(ny=9) if "periodic_y" in modes else SMALL
    r = r_of(w)
    ch = channel(w, r, **modes)
    p = oracle_params(w, r, **modes)
    f = _state(p)
    lam = np.random.default_rng(11).standard_normal(f.shape)
    ref_lam, ref_dp = A.step_vjp(f, lam, p)
    adj = Adjoint(ch)
    got = adj.step(torch.from_numpy(f).cuda(), torch.from_numpy(lam).cuda()).cpu().numpy()
    assert _rel(got, ref_lam) <= 1e-12
    dp = adj.dparams.cpu().numpy()
    for k in range(3):
        assert abs(dp[k] - ref_dp[k]) <= 1e-11 * max(abs(ref_dp[k]), 1e-3), (k, dp[k], ref_dp[k])


def test_adjoint_step_with_the_piecewise_wall_function_matches_the_cpu_reverse_sweep():
    """A channel of more than 2^17 nodes takes psi and h from the piecewise
    polynomials, in the adjoint's forward relaxation times as in its sweeps:
    one reverse step against the CPU reverse sweep."""
    w = SMALL.with_(nx=1100, ny=120)
    assert w.nx * w.ny > 1 << 17
    r = r_of(w)
    print(f"[case] adjoint step {w.nx}x{w.ny}", flush=True)
    ch = channel(w, r)
    p = oracle_params(w, r)
    f = _state(p)
    lam = np.random.default_rng(12).standard_normal(f.shape)
    ref_lam, ref_dp = A.step_vjp(f, lam, p)
    adj = Adjoint(ch)
    got = adj.step(torch.from_numpy(f).cuda(), torch.from_numpy(lam).cuda()).cpu().numpy()
    assert _rel(got, ref_lam) <= 1e-12
    dp = adj.dparams.cpu().numpy()
    for k in range(3):
        assert abs(dp[k] - ref_dp[k]) <= 1e-11 * max(abs(ref_dp[k]), 1e-3), (k, dp[k], ref_dp[k])


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_post_collision_state_is_the_collision_of_the_populations(dtype, tol):
    """The forward's own post-collision state f'(t) against the oracle's
    collision of the forward's pre-collision state f(t), after 30 steps."""
    w = SMALL
    r = r_of(w)
    ch = channel(w, r, dtype=dtype)
    ch.step(30)
    f = ch.get_populations().cpu().numpy()
    got = ch.get_post_collision().cpu().numpy()
    ref = O.collide(f, oracle_params(w, r))
    assert _rel(got, ref) <= tol


@pytest.mark.parametrize("shape,tile_mode,modes", [((90, 12), lbsep.TILE_NODE, {}),
                                                   ((90, 12), lbsep.TILE_SPLIT, {}),
                                                   ((70, 130), lbsep.TILE_AUTO, {}),
                                                   ((48, 10), lbsep.TILE_AUTO, {"periodic_x": True}),
                                                   ((1100, 120), lbsep.TILE_AUTO, {})],
                         ids=["node", "pair", "three-end-blocks", "periodic-x", "piecewise-wall-function"])
def test_recording_step_writes_what_the_readouts_return(shape, tile_mode, modes):
    """A recording step's pre- and post-collision outputs are bitwise the
    readouts after a plain step from the same state, and the two channels
    stay bitwise equal."""
    w = SMALL.with_(nx=shape[0], ny=shape[1])
    r = r_of(w)
    a, b = channel(w, r, tile_mode=tile_mode, **modes), channel(w, r, tile_mode=tile_mode, **modes)
    a.step(9)
    b.step(9)
    for _ in range(3):
        pre, post = a.step_record()
        b.step(1)
        assert torch.equal(pre, b.get_populations())
        assert torch.equal(post, b.get_post_collision())
        assert torch.equal(a.get_state(), b.get_state())
    assert a.read_cl()["cl"] == b.read_cl()["cl"]


def test_recording_step_needs_fp64_single_level():
    w = SMALL
    r = r_of(w)
    with pytest.raises(lbsep.LbsepError, match="FP64"):
        channel(w, r, dtype="f32").step_record()
    with pytest.raises(lbsep.LbsepError, match="one level per launch"):
        channel(w, r, fused_steps=2).step_record()


def test_adjoint_step_with_the_forward_post_collision_state():
    """lam(t) and the parameter partials with f_post from the forward agree with
    the step that recomputes C(f_t) itself (same map, two FP64 evaluations)."""
    w = SMALL
    r = r_of(w)
    ch = channel(w, r)
    ch.step(25)
    f, fp = ch.get_populations(), ch.get_post_collision()
    lam = torch.from_numpy(np.random.default_rng(7).standard_normal(tuple(f.shape))).cuda()
    a1, a2 = Adjoint(ch), Adjoint(ch)
    got = a1.step(f, lam, f_post=fp).cpu().numpy()
    ref = a2.step(f, lam).cpu().numpy()
    assert _rel(got, ref) <= 1e-12
    d1, d2 = a1.dparams.cpu().numpy(), a2.dparams.cpu().numpy()
    for k in range(3):
        assert abs(d1[k] - d2[k]) <= 1e-11 * max(abs(d2[k]), 1e-3), (k, d1[k], d2[k])


def test_adjoint_step_bgk_limit():
    w = SMALL
    r = r_of(w)
    ch = channel(w, r, tau_bgk=0.8)
    p = oracle_params(w, r, tau_bgk=0.8)
    f = _state(p)
    lam = np.random.default_rng(5).standard_normal(f.shape)
    ref_lam, _ = A.step_vjp(f, lam, p)
    got = Adjoint(ch).step(torch.from_numpy(f).cuda(), torch.from_numpy(lam).cuda()).cpu().numpy()
    assert _rel(got, ref_lam) <= 1e-12


def test_seed_and_initial_terms_match_the_cpu_reverse_sweep():
    w = SMALL
    r = r_of(w)
    p = oracle_params(w, r)
    f = O.run(p, 60)[0]
    ft = torch.tensor(f, dtype=torch.float64, requires_grad=True)
    cl_in = torch.tensor(p.cl_in, dtype=torch.float64, requires_grad=True)
    g_f, g_c = torch.autograd.grad(A.separation_degree(ft, p, cl_in), (ft, cl_in))
    ch = channel(w, r)
    adj = Adjoint(ch)
    seed = adj.seed_cl(torch.from_numpy(f).cuda()).cpu().numpy()
    assert _rel(seed, g_f.numpy()) <= 1e-13
    assert abs(adj.dparams[1].item() - g_c.item()) <= 1e-13 * abs(g_c.item())
    # initial state: lam0 . d f0 / d(theta, C_in)
    lam0 = np.random.default_rng(9).standard_normal(f.shape)
    th = torch.tensor(p.theta, dtype=torch.float64, requires_grad=True)
    cl = torch.tensor(p.cl_in, dtype=torch.float64, requires_grad=True)
    f0 = A.initial_state(p, th, cl)
    ref = torch.autograd.grad(f0, (th, cl), grad_outputs=torch.from_numpy(lam0))
    adj2 = Adjoint(ch)
    adj2.initial(torch.from_numpy(lam0).cuda())
    got = adj2.dparams.cpu().numpy()
    for k in range(2):
        assert abs(got[k] - ref[k].item()) <= 1e-12 * abs(ref[k].item()), (k, got[k], ref[k].item())
    assert got[2] == 0.0


def _params(w, r, dtype="f64"):
    return lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r, dtype=dtype,
                             hist_cap=64)


def test_checkpointed_gradient_matches_the_cpu_reverse_sweep():
    """150 steps, checkpoints every 40 (four segments, the last one short)."""
    w = SMALL
    r = r_of(w)
    cl, grad = cl_gradient(_params(w, r), 150, checkpoint_every=40)
    cl_ref, g_ref = A.gradients(oracle_params(w, r), 150)
    assert abs(cl - cl_ref) <= 1e-12
    grad = grad.cpu().numpy()
    for k in range(3):
        assert abs(grad[k] - g_ref[k]) <= 1e-9 * abs(g_ref[k]), (k, grad[k], g_ref[k])


def _cl_run(w, r, steps, **over):
    p = _params(w, r)
    for k, v in over.items():
        setattr(p, k, v)
    ch = lbsep.Channel(p, device="cuda:0")
    ch.step(steps)
    out = ch.read_cl()
    return out["cl"], out["x_min"]


_FD_CACHE = {}


def _central_differences(w, r, steps):
    """dCL/d(theta, C_in, r) by central differences of the FP64 GPU forward,
    h = 1e-6 relative (cached: both forward precisions are checked against it)."""
    key = (w.name, steps)
    if key not in _FD_CACHE:
        base = {"theta": w.theta, "cl_in": w.cl_in, "dbb_r": r}
        out = []
        for name in ("theta", "cl_in", "dbb_r"):
            h = 1e-6 * base[name]
            c_up, x_up = _cl_run(w, r, steps, **{name: base[name] + h})
            c_dn, x_dn = _cl_run(w, r, steps, **{name: base[name] - h})
            assert x_up == x_dn  # the column of the smallest C_l is held (R16, R21)
            out.append((c_up - c_dn) / (2 * h))
        _FD_CACHE[key] = out
    return _FD_CACHE[key]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gradient_of_the_adjoint_configuration_matches_central_differences(dtype):
    """He-Ar, H = 64, L = 1280, C_l = 0.5, theta = 2.5, Kn_out = 0.1, 10,000
    steps, checkpoints every 500: the three gradients against central
    differences of the FP64 GPU forward with h = 1e-6 (relative), to 1e-4.
    The forward runs in the given storage precision; the reverse sweep is
    FP64 on its states (FP32: the deviations converted to double, the segments
    recomputed by FP32 steps from FP32 checkpoints)."""
    w = CONFIGS["he_ar_64x1280"]
    steps = 10000
    r = r_of(w)
    cl, grad = cl_gradient(_params(w, r, dtype), steps, checkpoint_every=500)
    grad = grad.cpu().numpy()
    fds = _central_differences(w, r, steps)
    for k, name in enumerate(("theta", "cl_in", "dbb_r")):
        print(f"    {dtype} d CL / d {name}: adjoint {grad[k]:.10e}, differences {fds[k]:.10e}", flush=True)
        assert abs(grad[k] - fds[k]) <= 1e-4 * abs(fds[k]), (name, grad[k], fds[k])


def test_autograd_function_returns_the_adjoint_gradients():
    w = SMALL
    r = r_of(w)
    base = _params(w, r)
    th = torch.tensor(w.theta, dtype=torch.float64, requires_grad=True)
    cl = torch.tensor(w.cl_in, dtype=torch.float64, requires_grad=True)
    rr = torch.tensor(r, dtype=torch.float64, requires_grad=True)
    out = SeparationDegree.apply(th, cl, rr, base, 100, 30)
    (3.0 * out).backward()
    _, g_ref = A.gradients(oracle_params(w, r), 100)
    for t, g in zip((th, cl, rr), g_ref):
        assert abs(t.grad.item() - 3.0 * g) <= 1e-9 * abs(3.0 * g)
