"""Gradients of the separation degree CL through the whole run (discrete
adjoint, reverse mode), with checkpointed recomputation of the forward steps.

Argument marshalling and orchestration only: the forward steps, the adjoint
steps, the CL seed and the initial-state term all run in the HIP library
(``lbsep_step``, ``lbsep_adjoint_step``, ``lbsep_adjoint_seed_cl``,
``lbsep_adjoint_initial``). torch holds the device buffers.

Memory: two FP64 states per step of a checkpoint segment (pre- and
post-collision) are kept during the reverse sweep (2 * checkpoint_every * 18 *
ny * nx doubles) plus one raw state per checkpoint.
"""
from __future__ import annotations

from ctypes import c_size_t, c_void_p

import torch

from . import lbsep


class Adjoint:
    """The adjoint primitives of one channel (FP64 arithmetic on dense
    populations [2][9][ny][nx], whatever the channel's storage type)."""

    def __init__(self, channel: lbsep.Channel):
        self.ch = channel
        L = lbsep.load()
        n = L.lbsep_adjoint_workspace_bytes(channel.params)
        if n == 0:
            raise lbsep.LbsepError(lbsep.EINVAL, lbsep.last_error())
        raw = torch.empty(n + 256, dtype=torch.uint8, device=channel.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + n]
        self.nbytes = n
        self.dparams = torch.zeros(3, dtype=torch.float64, device=channel.device)
        self.shape = (2, 9, channel.ny, channel.nx)

    def _args(self):
        return c_void_p(self.ws.data_ptr()), c_size_t(self.nbytes)

    def _check_state(self, t):
        if t.shape != self.shape or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"expected a contiguous float64 tensor of shape {self.shape}")

    def step(self, f_t: torch.Tensor, lam_next: torch.Tensor, out: torch.Tensor | None = None,
             f_post: torch.Tensor | None = None) -> torch.Tensor:
        """lam(t) from lam(t+1) at the pre-collision state f_t; f_post = C(f_t)
        from Channel.get_post_collision at the same level, or None (recomputed)."""
        self._check_state(f_t)
        self._check_state(lam_next)
        if f_post is not None:
            self._check_state(f_post)
        out = torch.empty_like(lam_next) if out is None else out
        self.ch._take_over()
        lbsep._check(lbsep.load().lbsep_adjoint_step(self.ch._h, c_void_p(f_t.data_ptr()),
                                                     c_void_p(f_post.data_ptr() if f_post is not None else None),
                                                     c_void_p(lam_next.data_ptr()), c_void_p(out.data_ptr()),
                                                     c_void_p(self.dparams.data_ptr()), *self._args()))
        self.ch._hand_over(out)
        return out

    def seed_cl(self, f_T: torch.Tensor) -> torch.Tensor:
        self._check_state(f_T)
        out = torch.empty_like(f_T)
        self.ch._take_over()
        lbsep._check(lbsep.load().lbsep_adjoint_seed_cl(self.ch._h, c_void_p(f_T.data_ptr()), c_void_p(out.data_ptr()),
                                                        c_void_p(self.dparams.data_ptr()), *self._args()))
        self.ch._hand_over(out)
        return out

    def initial(self, lam0: torch.Tensor):
        self._check_state(lam0)
        self.ch._take_over()
        lbsep._check(lbsep.load().lbsep_adjoint_initial(self.ch._h, c_void_p(lam0.data_ptr()),
                                                        c_void_p(self.dparams.data_ptr()), *self._args()))


def cl_gradient(params: lbsep.Params, nsteps: int, checkpoint_every: int = 500, device="cuda:0"):
    """CL after nsteps from the initial state of R18 and dCL/d(theta, C_in, r).

    Forward: nsteps sweeps, a raw checkpoint every `checkpoint_every` levels.
    Reverse: per segment (last first) restore the checkpoint, recompute and keep
    the segment's pre- and post-collision states, then run the adjoint steps
    back through it; finally add the initial state's term. Returns (cl,
    tensor[3])."""
    ch = lbsep.Channel(params, device=device)
    adj = Adjoint(ch)
    record = params.dtype == lbsep.F64 and params.fused_steps != 2
    ckpt = {0: ch.get_state()}
    t = 0
    while t < nsteps:
        n = min(checkpoint_every, nsteps - t)
        ch.step(n)
        t += n
        if t < nsteps:
            ckpt[t] = ch.get_state()
    cl = ch.read_cl()["cl"]
    lam = adj.seed_cl(ch.get_populations())
    spare = torch.empty_like(lam)
    starts = sorted(ckpt)
    for t0 in reversed(starts):
        t1 = min(t0 + checkpoint_every, nsteps)
        ch.set_state(ckpt[t0], t0)
        # the segment's (f(t), C(f(t))) for t = t0 .. t1 - 1: the restored level
        # read out, the following levels written by the steps themselves
        # (recording steps, FP64 one level per launch) or read out after them
        seg = [(ch.get_populations(), ch.get_post_collision())]
        for _ in range(t0 + 1, t1):
            if record:
                seg.append(ch.step_record())
            else:
                ch.step(1)
                seg.append((ch.get_populations(), ch.get_post_collision()))
        for k in range(len(seg) - 1, -1, -1):
            adj.step(seg[k][0], lam, out=spare, f_post=seg[k][1])
            lam, spare = spare, lam
        del seg
    adj.initial(lam)
    torch.cuda.synchronize(device)
    return cl, adj.dparams.clone()


class SeparationDegree(torch.autograd.Function):
    """CL(theta, C_in, r) of a channel run, differentiable by the discrete
    adjoint. forward(theta, cl_in, r, base_params, nsteps, checkpoint_every)
    with 0-dim float64 tensors for the three parameters; base_params supplies
    everything else (sizes, masses, C_out, Kn_out, storage type)."""

    @staticmethod
    def forward(ctx, theta, cl_in, r, base_params, nsteps, checkpoint_every=500):
        p = lbsep.Params.from_buffer_copy(base_params)
        p.theta, p.cl_in, p.dbb_r = float(theta), float(cl_in), float(r)
        cl, grad = cl_gradient(p, int(nsteps), int(checkpoint_every), device=theta.device
                               if theta.device.type == "cuda" else "cuda:0")
        ctx.save_for_backward(grad.to(theta.device))
        return torch.tensor(cl, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad[0], g * grad[1], g * grad[2], None, None, None
