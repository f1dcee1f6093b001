"""FP64 CPU reverse sweep of the oracle's time step (reverse-mode derivatives).

TEST INFRASTRUCTURE, like ``binary_lbm``: only ``tests/`` may use it. It is the
oracle's step (Sec. 3.1 collision, Eq. (MRT) streaming, Eqs. (bot)/(bot2) DBB
walls, Eqs. (rho1)/(rho2) inlet/outlet, Eq. (CL)) written a second time in
plain PyTorch CPU float64 operations, in the same order and with the same
readings, so that PyTorch's reverse-mode automatic differentiation yields the
exact discrete adjoint: dCL/d(theta, C_in, r) through every step, the
relaxation times (the wall function psi included) and the initial state of
R18. The only hand-written derivatives are those of the wall function, whose
values come from the library routine scipy.special.exp1 as in the oracle:
psi'(a) = 2 e^-a - 2 a E1(a) and psi''(a) = -2 E1(a).

Pins (tests/test_oracle_adjoint.py): the step here equals the oracle's NumPy
step to rounding; its gradients equal central finite differences of the
NumPy oracle.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.special import exp1

from . import binary_lbm as O

DT = torch.float64
CX = torch.tensor(O.CX, dtype=DT)
CY = torch.tensor(O.CY, dtype=DT)
W = torch.tensor(O.W, dtype=DT)
M = torch.tensor(O.M, dtype=DT)
M_INV = torch.tensor(O.M_INV, dtype=DT)


class _Psi(torch.autograd.Function):
    """psi(a) of Sec. 3.1 with psi' = 2 e^-a - 2 a E1(a) (E1 from scipy)."""

    @staticmethod
    def forward(ctx, a):
        ctx.save_for_backward(a)
        return torch.from_numpy(O.psi(a.detach().numpy()))

    @staticmethod
    def backward(ctx, g):
        (a,) = ctx.saved_tensors
        return g * _DPsi.apply(a)


class _DPsi(torch.autograd.Function):
    """psi'(a) with psi'' = -2 E1(a) (a > 0)."""

    @staticmethod
    def forward(ctx, a):
        ctx.save_for_backward(a)
        return torch.from_numpy(O.dpsi(a.detach().numpy()))

    @staticmethod
    def backward(ctx, g):
        (a,) = ctx.saved_tensors
        an = a.detach().numpy()
        d2 = np.where(an > 0, -2.0 * exp1(np.where(an > 0, an, 1.0)), -np.inf)
        return g * torch.from_numpy(d2)


def psi(a):
    return _Psi.apply(a)


def dpsi(a):
    return _DPsi.apply(a)


def species_density(p, pressure, c_light):
    s = p.s
    return c_light * pressure / (s[0] * O.CS2), (1.0 - c_light) * pressure / (s[1] * O.CS2)


def f_equilibrium(rho, ux, uy, s):
    ext = (9,) + (1,) * rho.dim()
    cu = CX.reshape(ext) * ux + CY.reshape(ext) * uy
    usq = ux * ux + uy * uy
    alpha = torch.tensor(O.alpha_weights(s), dtype=DT).reshape(ext)
    return W.reshape(ext) * rho * (alpha + cu / O.CS2 + cu * cu / (2 * O.CS2 * O.CS2) - usq / (2 * O.CS2))


def wall_function(y, ell, height):
    return 0.5 * (psi(y / ell) + psi((height - y) / ell))


def relaxation_times(rho_a, rho_b, p):
    """The oracle's relaxation_times (R5-R9), differentiable in the densities."""
    m_a, m_b, m_min, s = p.m_a, p.m_b, p.m_min, p.s
    height = float(p.ny)
    y = (torch.arange(p.ny, dtype=DT) + 0.5)[:, None]
    n_a = rho_a / m_a
    n_b = rho_b / m_b
    n = n_a + n_b
    x_a = n_a / n
    x_b = n_b / n
    m_x = (rho_a + rho_b) / n
    pressure = O.CS2 * (s[0] * rho_a + s[1] * rho_b)
    lam = p.kn_out * height * O.P_OUT / pressure
    lam_a = lam / x_a
    lam_b = lam / x_b
    k = torch.sqrt(6.0 * m_min / (math.pi * m_x))
    if p.tau_bgk is not None:
        t = torch.full(rho_a.shape, float(p.tau_bgk), dtype=DT)
        return t, t, t
    if p.mfp_off:
        psi_m = psi_a = psi_b = 1.0
    else:
        psi_m = wall_function(y, lam, height)
        psi_a = wall_function(y, lam_a, height)
        psi_b = wall_function(y, lam_b, height)
    tau_s = 0.5 + lam * psi_m * k
    lam_ae = lam_a * psi_a
    lam_be = lam_b * psi_b
    pref = 1.5 * torch.sqrt(3.0 * (m_a + m_b) * m_a * m_b / (m_min * m_x * m_x))
    bracket = 1.0 / torch.sqrt(x_a * lam_ae) + 1.0 / torch.sqrt(x_b * lam_be)
    tau_d = 0.5 + pref / (bracket * bracket)
    if p.mfp_off:
        tt0 = k * lam
        dtt0 = torch.zeros_like(tt0)
    else:
        a = height / lam
        tt0 = k * lam * 0.5 * psi(a)                 # psi(0) = 0
        dtt0 = 0.5 * k * (2.0 - dpsi(a))             # psi'(0) = 2
    a1, a2 = O.slip_constants(p.accom)
    vs = math.sqrt(math.pi / 6.0)
    tau_q = (0.5 + (3.0 + 24.0 * vs * vs * tt0 * tt0 * a2) / (16.0 * tt0)
             + dtt0 * (12.0 + 30.0 * tt0 * vs * a1) / (16.0 * tt0 * tt0))
    return tau_s, tau_d, tau_q


def collide(f, p):
    rho_s = f.sum(dim=1)
    jx_s = torch.einsum("i,sijx->sjx", CX, f)
    jy_s = torch.einsum("i,sijx->sjx", CY, f)
    rho = rho_s.sum(dim=0)
    ux = jx_s.sum(dim=0) / rho
    uy = jy_s.sum(dim=0) / rho
    tau_s, tau_d, tau_q = relaxation_times(rho_s[0], rho_s[1], p)
    ones = torch.ones_like(tau_s)
    if p.tau_bgk is not None:
        srate = torch.stack([1.0 / tau_s] * 9)
    else:
        srate = torch.stack([ones / O.TAU_RHO, ones / O.TAU_E, ones / O.TAU_EPS, 1.0 / tau_d, 1.0 / tau_q,
                             1.0 / tau_d, 1.0 / tau_q, 1.0 / tau_s, 1.0 / tau_s])
    out = []
    for sig in range(2):
        feq = f_equilibrium(rho_s[sig], ux, uy, p.s[sig])
        m = torch.einsum("ki,ijx->kjx", M, f[sig])
        meq = torch.einsum("ki,ijx->kjx", M, feq)
        mpost = m - srate * (m - meq)
        out.append(torch.einsum("ki,ijx->kjx", M_INV, mpost))
    return torch.stack(out)


def stream(fpost, p, r, rho_in):
    """Streaming, DBB walls (parameter r) and the inlet/outlet closure (inlet
    densities rho_in, a pair of tensors), as in the oracle."""
    fnew = torch.stack([torch.roll(fpost[:, i], shifts=(int(O.CY[i]), int(O.CX[i])), dims=(-2, -1))
                        for i in range(9)], dim=1)
    if not p.periodic_y:
        fnew = fnew.clone()
        for sig in range(2):
            s = p.s[sig]
            for row, unknown, leaving in ((0, (2, 5, 6), (4, 7, 8)), (p.ny - 1, (4, 7, 8), (2, 5, 6))):
                out_mass = sum(fpost[sig, i, row, :] for i in leaving)
                w_in = sum(O.W[i] * s for i in unknown)
                rho_w = out_mass / w_in
                for iu, il in zip(unknown, leaving):
                    feq_w = O.W[iu] * s * rho_w                      # rest equilibrium of Eq. (feq)
                    fnew[sig, iu, row, :] = r * feq_w + (1.0 - r) * fpost[sig, il, row, :]
    if not p.periodic_x:
        _, rout = O.boundary_densities(p)
        species = []
        for sig in range(2):
            ends = []
            for col, l1, l2, rho_bc, unknown in ((0, 1, 2, rho_in[sig], O.INLET_UNKNOWN),
                                                 (p.nx - 1, p.nx - 2, p.nx - 3, float(rout[sig]),
                                                  O.OUTLET_UNKNOWN)):
                g = torch.stack([2.0 * fnew[sig, i, :, l1] - fnew[sig, i, :, l2] if i in unknown
                                 else fnew[sig, i, :, col] for i in range(9)])
                rho_prime = 2.0 * fnew[sig, :, :, l1].sum(dim=0) - fnew[sig, :, :, l2].sum(dim=0)
                kappa = p.ny * rho_bc / rho_prime.sum()
                rho_node = g.sum(dim=0)
                ends.append(g * (kappa * rho_prime / rho_node))
            species.append(torch.cat([ends[0][..., None], fnew[sig, :, :, 1:p.nx - 1], ends[1][..., None]], dim=-1))
        fnew = torch.stack(species)
    return fnew


def inlet_densities(p, theta, cl_in):
    """rho_sigma at the inlet from P_in = theta P_out and C_in (R13)."""
    return species_density(p, theta * O.P_OUT, cl_in)


def step(f, p, theta, cl_in, r):
    return stream(collide(f, p), p, r, inlet_densities(p, theta, cl_in))


def initial_state(p, theta, cl_in):
    """R18 as in the oracle, differentiable in theta and C_in (C_out held)."""
    x = torch.arange(p.nx, dtype=DT)
    frac = x / (p.nx - 1)
    p_in = theta * O.P_OUT
    pres = p_in + (O.P_OUT - p_in) * frac
    cl = cl_in + (p.cl_out - cl_in) * frac
    rho_a, rho_b = species_density(p, pres, cl)
    zeros = torch.zeros((p.ny, p.nx), dtype=DT)
    fa = f_equilibrium(rho_a.expand(p.ny, p.nx), zeros, zeros, p.s[0])
    fb = f_equilibrium(rho_b.expand(p.ny, p.nx), zeros, zeros, p.s[1])
    return torch.stack([fa, fb])


def separation_degree(f, p, cl_in):
    """CL of Eq. (CL) from the pre-collision state (R16)."""
    rho_s = f.sum(dim=1)
    n_a = (rho_s[0] / p.m_a).sum(dim=0)
    n_b = (rho_s[1] / p.m_b).sum(dim=0)
    cl_x = n_a / (n_a + n_b)
    return (cl_in - cl_x.min()) / cl_in


def gradients(p, nsteps):
    """CL after nsteps from the initial state and dCL/d(theta, C_in, r) by the
    reverse sweep. Returns (CL, [dtheta, dcl_in, dr])."""
    theta = torch.tensor(p.theta, dtype=DT, requires_grad=True)
    cl_in = torch.tensor(p.cl_in, dtype=DT, requires_grad=True)
    r = torch.tensor(p.dbb_r, dtype=DT, requires_grad=True)
    f = initial_state(p, theta, cl_in)
    for _ in range(nsteps):
        f = step(f, p, theta, cl_in, r)
    cl = separation_degree(f, p, cl_in)
    g = torch.autograd.grad(cl, (theta, cl_in, r))
    return float(cl.detach()), [float(v) for v in g]


def step_vjp(f, lam, p):
    """One step's adjoint: lam_t = (d f(t+1) / d f(t))^T lam and the explicit
    partial derivatives lam . d f(t+1) / d(theta, C_in, r) at the state f
    (numpy arrays (2, 9, ny, nx))."""
    ft = torch.tensor(f, dtype=DT, requires_grad=True)
    theta = torch.tensor(p.theta, dtype=DT, requires_grad=True)
    cl_in = torch.tensor(p.cl_in, dtype=DT, requires_grad=True)
    r = torch.tensor(p.dbb_r, dtype=DT, requires_grad=True)
    out = step(ft, p, theta, cl_in, r)
    g = torch.autograd.grad(out, (ft, theta, cl_in, r), grad_outputs=torch.tensor(lam, dtype=DT),
                            allow_unused=True)
    dp = [0.0 if v is None else float(v) for v in g[1:]]
    return g[0].numpy(), dp
