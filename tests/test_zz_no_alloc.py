"""The allocation-free reverse step (lbsep_adjoint_step_noalloc, scratch in a
fixed array of the library) against the reverse step with a caller workspace
(lbsep_adjoint_step), through the C ABI: the same kernels on the same inputs,
so lam(t) and the accumulated parameter partials must agree bitwise. Calls
follow one another on the same GPU with different channel sizes (the second
smaller than the first), with and without the forward's post-collision state,
so stale contents of the shared scratch would show."""
from ctypes import c_void_p

import numpy as np
import pytest
import torch

from paper_1603_08221_amd import lbsep
from paper_1603_08221_amd.adjoint import Adjoint
from paper_1603_08221_amd.workloads import HE_AR, NE_AR, Workload

from gpu_helpers import channel, r_of

pytestmark = pytest.mark.gpu

BIG = Workload("noalloc_big", 70, 130, *HE_AR, 0.5, 0.5, 2.0, 0.1, 0)     # three end blocks per end
SMALL = Workload("noalloc_small", 40, 6, *NE_AR, 0.3, 0.6, 3.0, 0.05, 0)  # unequal C_in, C_out
TALL = Workload("noalloc_tall", 12, 300, *HE_AR, 0.7, 0.7, 1.5, 0.3, 0)   # more rows than threads per block


def _noalloc(ch, f, fp, lam, out, dparams):
    lib = lbsep.load()
    ch._take_over()
    rc = lib.lbsep_adjoint_step_noalloc(ch._h, c_void_p(f.data_ptr()),
                                        c_void_p(fp.data_ptr() if fp is not None else None),
                                        c_void_p(lam.data_ptr()), c_void_p(out.data_ptr()),
                                        c_void_p(dparams.data_ptr()))
    return rc


def _case(w, steps, with_post, seed):
    r = r_of(w)
    ch = channel(w, r)
    ch.step(steps)
    f = ch.get_populations()
    fp = ch.get_post_collision() if with_post else None
    lam = torch.from_numpy(np.random.default_rng(seed).standard_normal(tuple(f.shape))).cuda()
    ref_adj = Adjoint(ch)
    ref = ref_adj.step(f, lam, f_post=fp)
    out = torch.full_like(lam, float("nan"))
    dparams = torch.zeros(3, dtype=torch.float64, device=f.device)
    rc = _noalloc(ch, f, fp, lam, out, dparams)
    assert rc == lbsep.OK, lbsep.last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref), f"{w.name}: lam(t) differs"
    assert torch.equal(dparams, ref_adj.dparams), (w.name, dparams.tolist(), ref_adj.dparams.tolist())
    return ch


def test_noalloc_step_matches_the_workspace_step_on_successive_calls():
    _case(BIG, 20, True, 1)      # first call on this GPU: sets up the scratch address
    _case(SMALL, 15, False, 2)   # smaller, and C(f_t) recomputed inside the scratch
    _case(TALL, 10, True, 3)     # the two-pass end closure (ny > 256)
    _case(SMALL, 15, True, 4)


def test_noalloc_step_rejects_what_does_not_fit_before_enqueuing():
    w = Workload("noalloc_long", 1280, 64, *HE_AR, 0.5, 0.5, 2.5, 0.1, 0)
    r = r_of(w)
    ch = channel(w, r)
    f = ch.get_populations()
    lam = torch.zeros_like(f)
    out = torch.full_like(f, 7.0)
    dparams = torch.zeros(3, dtype=torch.float64, device=f.device)
    # recomputing C(f_t) for 81,920 nodes needs 11.8 MB of scratch: refused
    rc = _noalloc(ch, f, None, lam, out, dparams)
    assert rc == lbsep.ESIZE and "fixed scratch" in lbsep.last_error()
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)  # nothing ran
    # with the forward's post-collision state the same channel fits
    fp = ch.get_post_collision()
    lam = torch.from_numpy(np.random.default_rng(9).standard_normal(tuple(f.shape))).cuda()
    ref_adj = Adjoint(ch)
    ref = ref_adj.step(f, lam, f_post=fp)
    assert _noalloc(ch, f, fp, lam, out, dparams) == lbsep.OK, lbsep.last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(dparams, ref_adj.dparams)
    # the aliasing rule of lbsep_adjoint_step holds here too
    assert _noalloc(ch, f, fp, lam, lam, dparams) == lbsep.EINVAL
