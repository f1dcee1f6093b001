"""Plain FP64 CPU oracle for the binary-mixture MRT lattice Boltzmann channel.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The product path
(the HIP library behind ``include/lbsep.h``) never calls it, and the two share
no code: no kernels, helpers, tables or constant generators.

What it computes: Wang, Xu & Guo, "Lattice Boltzmann simulation of separation
phenomenon in a binary gaseous flow through a microchannel" (arXiv:1603.08221).

* Sec. 3.1, Eq. (MRT): f_si(x + c_i, t + 1) = f_si(x, t) + Omega_si.
* Eq. (MR), (m), (S): MRT collision in the moment space of M.
* Eq. (feq): species equilibrium with alpha_s0 = (9 - 5 s)/4 and alpha_si = s,
  built on the mixture velocity.
* Eq. (rhou): mixture and species moments.
* Eqs. (EQFrb), (taos), (EQFrsp): effective relaxation times with the
  mean-free-path wall function psi / E1.
* Eq. (taoq), (A12): tau_q.
* Sec. 3.2, Eqs. (bot), (bot2): diffuse-bounce-back (DBB) walls.
* Eqs. (rho1), (rho2): extrapolation-correction pressure inlet/outlet.
* Sec. 2, Eqs. (C), (P), (CL), (Clline): mole fraction, separation degree CL,
  mean separation.

The method is a time iteration with no shorter closed form, so this module
takes the paper's steps in the paper's order, whole-grid array by whole-grid
array, with no fusion or reordering. Readings where the paper is silent or
garbled are named ``R<n>`` below; each is listed with its reason in the
design notes of the repository.

Array layout: populations ``f[sigma, i, j, x]`` with sigma in (a, b) (a is the
light species), i the D2Q9 direction, j the row across the channel
(0 .. ny-1, node centre y_j = j + 1/2, walls half-way at y = 0 and y = ny),
x the column along the flow (0 .. nx-1; columns 0 and nx-1 are the inlet and
outlet nodes).

Parity pins: see tests/test_oracle_*.py. tau_d has no closed-form check beyond
its limits and symmetries (documented there); the absolute CL values of the
paper's own runs are unpinned (every figure of the paper is stripped).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
from scipy.special import exp1

# ---------------------------------------------------------------------------
# Lattice (Sec. 3.1).  R2: the text's velocity list is garbled; the rows of M
# (rows 3 and 5 are c_x and c_y) and the DBB pairs 2<->4, 5<->7, 6<->8 fix the
# standard order below.
# ---------------------------------------------------------------------------
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)          # weights after Eq. (feq)
CS2 = 1.0 / 3.0                                                # c_s^2 = 1/3 (R3)

# Eq. (m), as printed.
M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)
M_INV = np.linalg.inv(M)

# Fixed relaxation times of the non-hydrodynamic moments (Sec. 3.3).
TAU_RHO, TAU_E, TAU_EPS = 1.0, 1.1, 1.2

# S0 normalisation: outlet pressure P_out = c_s^2 = 1/3 (then n_out * m_min = 1).
P_OUT = CS2


@dataclass(frozen=True)
class Params:
    """Problem statement of Sec. 2 plus the DBB inputs of Sec. 3.2.

    nx, ny      : lattice columns along the flow (N_x, channel length L) and
                  rows across it (N, channel height H = ny lattice units).
    m_a, m_b    : molecular masses, m_a <= m_b (a is the light species).
    cl_in/out   : light-species mole fraction C_l at inlet / outlet, Eq. (C).
    theta       : P_in / P_out (Sec. 2).
    kn_out      : lambda_out / H (Sec. 2).
    dbb_r       : r_sigma of Eqs. (bot), (bot2), one value for both species (R10).
    accom       : accommodation coefficient alpha of Eq. (A12) (R19: default 1).
    periodic_x  : no inlet/outlet; columns wrap (test mode).
    periodic_y  : no walls; rows wrap (test mode; requires mfp_off).
    mfp_off     : Psi == 1 (unbounded mean free path; test mode).
    tau_bgk     : if set, every relaxation time equals it (BGK limit, test mode).
    """
    nx: int
    ny: int
    m_a: float
    m_b: float
    cl_in: float
    cl_out: float
    theta: float
    kn_out: float
    dbb_r: float
    accom: float = 1.0
    periodic_x: bool = False
    periodic_y: bool = False
    mfp_off: bool = False
    tau_bgk: float | None = None

    @property
    def masses(self) -> np.ndarray:
        return np.array([self.m_a, self.m_b], dtype=np.float64)

    @property
    def m_min(self) -> float:
        return min(self.m_a, self.m_b)

    @property
    def s(self) -> np.ndarray:
        """s_sigma = m_min / m_sigma (after Eq. (feq))."""
        return self.m_min / self.masses


def p_in(p: Params) -> float:
    """Inlet pressure, theta = P_in / P_out (Sec. 2)."""
    return p.theta * P_OUT


def species_density(p: Params, pressure, c_light):
    """rho_sigma from the mixture pressure and light mole fraction.

    Model equation of state: the trace of the equilibrium pressure tensor of
    Eq. (feq) is rho_s s_s c_s^2 = n_s k_B T with k_B T = m_min c_s^2, which is
    Eq. (P) split by species. So rho_s = x_s P / (s_s c_s^2)  (R13).
    """
    s = p.s
    x_a = np.asarray(c_light, dtype=np.float64)
    pressure = np.asarray(pressure, dtype=np.float64)
    return x_a * pressure / (s[0] * CS2), (1.0 - x_a) * pressure / (s[1] * CS2)


def boundary_densities(p: Params):
    """(rho_a_in, rho_b_in), (rho_a_out, rho_b_out) for Eq. (rho2) (R13)."""
    rin = species_density(p, p_in(p), p.cl_in)
    rout = species_density(p, P_OUT, p.cl_out)
    return np.array([float(rin[0]), float(rin[1])]), np.array([float(rout[0]), float(rout[1])])


# ---------------------------------------------------------------------------
# Equilibrium, Eq. (feq).
# ---------------------------------------------------------------------------
def alpha_weights(s: float) -> np.ndarray:
    """alpha_s0 = (9 - 5 s)/4, alpha_si = s for i != 0 (after Eq. (feq))."""
    a = np.full(9, float(s))
    a[0] = (9.0 - 5.0 * s) / 4.0
    return a


def f_equilibrium(rho, ux, uy, s: float) -> np.ndarray:
    """f^eq_si = w_i rho_s [alpha_si + c.u/cs2 + (c.u)^2/(2 cs2^2) - u^2/(2 cs2)].

    rho, ux, uy broadcast together; the result has a leading axis of 9.
    u is the velocity of the mixture (Eq. (feq) text).
    """
    rho = np.asarray(rho, dtype=np.float64)
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    shape = np.broadcast(rho, ux, uy).shape
    ext = (9,) + (1,) * len(shape)
    cu = CX.reshape(ext) * ux + CY.reshape(ext) * uy
    usq = ux * ux + uy * uy
    alpha = alpha_weights(s).reshape(ext)
    return W.reshape(ext) * rho * (alpha + cu / CS2 + cu * cu / (2 * CS2 * CS2) - usq / (2 * CS2))


# ---------------------------------------------------------------------------
# Mean-free-path wall function (Sec. 3.1): psi, E1 and Psi.
# ---------------------------------------------------------------------------
def e1(a):
    """E1(a) = int_1^inf t^-1 exp(-a t) dt (the paper's "E_i", R4); library routine."""
    return exp1(np.asarray(a, dtype=np.float64))


def psi(a):
    """psi(alpha) = 1 + (alpha - 1) e^-alpha - alpha^2 E1(alpha), with psi(0) = 0.

    Evaluated as (1 - e^-alpha) + alpha e^-alpha - alpha^2 E1(alpha) with
    1 - e^-alpha = -expm1(-alpha): the same function, without the cancellation
    of 1 - e^-alpha at small alpha (psi ~ 2 alpha there)."""
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = a > 0
    an = a[nz]
    out[nz] = -np.expm1(-an) + an * np.exp(-an) - an * an * e1(an)
    return out


def dpsi(a):
    """psi'(alpha) = 2 e^-alpha - 2 alpha E1(alpha)  (d/d alpha of psi, using E1' = -e^-a/a)."""
    a = np.asarray(a, dtype=np.float64)
    out = np.full_like(a, 2.0)
    nz = a > 0
    an = a[nz]
    out[nz] = 2.0 * np.exp(-an) - 2.0 * an * e1(an)
    return out


def wall_function(y, ell, height):
    """Psi(y) = [psi(y / ell) + psi((H - y) / ell)] / 2  (effective MFP lambda_e = ell Psi)."""
    return 0.5 * (psi(y / ell) + psi((height - y) / ell))


# ---------------------------------------------------------------------------
# Relaxation times, Eqs. (EQFrb), (taos), (EQFrsp), (taoq), (A12).
# ---------------------------------------------------------------------------
@dataclass
class Relaxation:
    tau_s: np.ndarray
    tau_d: np.ndarray
    tau_q: np.ndarray
    lam: np.ndarray = field(repr=False)
    x_a: np.ndarray = field(repr=False)
    m_x: np.ndarray = field(repr=False)
    pressure: np.ndarray = field(repr=False)


def slip_constants(accom: float):
    """A1 = (2 - alpha)/alpha (1 - 0.1817 alpha), A2 = 1/pi + A1^2 / 2 (Eq. (A12))."""
    a1 = (2.0 - accom) / accom * (1.0 - 0.1817 * accom)
    a2 = 1.0 / math.pi + 0.5 * a1 * a1
    return a1, a2


def tau_q_formula(tt0, dtt0, accom: float):
    """Eq. (taoq) with the wall values tau~_s(0) and tau~'_s(0) (R7: the third term
    carries the wall derivative; delta_x = 1 in lattice units)."""
    a1, a2 = slip_constants(accom)
    vs = math.sqrt(math.pi / 6.0)                      # varsigma (R9: literal)
    return (0.5 + (3.0 + 24.0 * vs * vs * tt0 * tt0 * a2) / (16.0 * tt0)
            + dtt0 * (12.0 + 30.0 * tt0 * vs * a1) / (16.0 * tt0 * tt0))


def relaxation_times(rho_a, rho_b, p: Params, y=None) -> Relaxation:
    """Local relaxation times from the species densities (R17: recomputed every
    step from the node's own pre-collision state).

    rho_a, rho_b have shape (ny, nx) (or broadcast with y); y defaults to the
    node centres j + 1/2 of each row.
    """
    rho_a = np.asarray(rho_a, dtype=np.float64)
    rho_b = np.asarray(rho_b, dtype=np.float64)
    m_a, m_b = p.m_a, p.m_b
    m_min = p.m_min
    s = p.s
    height = float(p.ny)                                   # H = N (delta_x = 1)
    if y is None:
        y = (np.arange(p.ny, dtype=np.float64) + 0.5)[:, None]
    n_a = rho_a / m_a
    n_b = rho_b / m_b
    n = n_a + n_b
    x_a = n_a / n
    x_b = n_b / n
    m_x = (rho_a + rho_b) / n                              # m_x = rho / n = x_a m_a + x_b m_b
    pressure = CS2 * (s[0] * rho_a + s[1] * rho_b)         # P = n k_B T, Eq. (P)
    # R5: mu independent of pressure -> lambda proportional to 1/P, equal to
    # Kn_out * H at the outlet pressure.
    lam = p.kn_out * height * P_OUT / pressure
    # R6: equal molecular diameters -> x_s lambda_s = lambda.
    lam_a = lam / x_a
    lam_b = lam / x_b
    k = np.sqrt(6.0 * m_min / (math.pi * m_x))
    if p.tau_bgk is not None:
        t = np.full(np.broadcast(rho_a, y).shape, float(p.tau_bgk))
        return Relaxation(t, t.copy(), t.copy(), lam, x_a, m_x, pressure)
    if p.mfp_off:
        psi_m = psi_a = psi_b = 1.0
    else:
        psi_m = wall_function(y, lam, height)
        psi_a = wall_function(y, lam_a, height)
        psi_b = wall_function(y, lam_b, height)
    # Eq. (taos)
    tau_s = 0.5 + lam * psi_m * k
    # Eq. (EQFrsp), second form, with lambda_se = lambda_s Psi(y; lambda_s)
    lam_ae = lam_a * psi_a
    lam_be = lam_b * psi_b
    pref = 1.5 * np.sqrt(3.0 * (m_a + m_b) * m_a * m_b / (m_min * m_x * m_x))
    bracket = 1.0 / np.sqrt(x_a * lam_ae) + 1.0 / np.sqrt(x_b * lam_be)
    tau_d = 0.5 + pref / (bracket * bracket)
    # Eq. (taoq) (R7, R8): wall values of tau~_s = tau_s - 1/2 from the node's
    # own lambda and m_x, evaluated at y = 0.
    if p.mfp_off:
        tt0 = k * lam
        dtt0 = np.zeros_like(tt0)
    else:
        a = height / lam
        # tau~_s(0) = k lam Psi(0) = k lam [psi(0) + psi(H/lam)] / 2
        tt0 = k * lam * 0.5 * (psi(np.zeros_like(a)) + psi(a))
        # d/dy [k lam Psi(y)] at y = 0 = (k/2) [psi'(0) - psi'(H/lam)]
        dtt0 = 0.5 * k * (dpsi(np.zeros_like(a)) - dpsi(a))
    tau_q = tau_q_formula(tt0, dtt0, p.accom)
    shape = np.broadcast(rho_a, y).shape
    return Relaxation(np.broadcast_to(tau_s, shape).copy(), np.broadcast_to(tau_d, shape).copy(),
                      np.broadcast_to(tau_q, shape).copy(), lam, x_a, m_x, pressure)


# ---------------------------------------------------------------------------
# Moments, Eq. (rhou).
# ---------------------------------------------------------------------------
def moments(f: np.ndarray):
    """rho_sigma, j_sigma (= sum_i c_i f_si) and the mixture rho, u."""
    rho_s = f.sum(axis=1)                                   # (2, ny, nx)
    jx_s = np.tensordot(CX.astype(np.float64), f, axes=([0], [1]))
    jy_s = np.tensordot(CY.astype(np.float64), f, axes=([0], [1]))
    rho = rho_s.sum(axis=0)
    ux = jx_s.sum(axis=0) / rho
    uy = jy_s.sum(axis=0) / rho
    return rho_s, jx_s, jy_s, rho, ux, uy


def species_velocity(f: np.ndarray, p: Params):
    """rho_s u_s = (2 tau_d - 1)/(2 tau_d) sum_i c_i f_si + rho_s u / (2 tau_d), Eq. (rhou).

    Returns (rho_s, u_sx, u_sy) with shapes (2, ny, nx).
    """
    rho_s, jx_s, jy_s, rho, ux, uy = moments(f)
    tau_d = relaxation_times(rho_s[0], rho_s[1], p).tau_d
    g = (2.0 * tau_d - 1.0) / (2.0 * tau_d)
    px = g * jx_s + rho_s * ux / (2.0 * tau_d)
    py = g * jy_s + rho_s * uy / (2.0 * tau_d)
    return rho_s, px / rho_s, py / rho_s


# ---------------------------------------------------------------------------
# One time step: collide (Eq. (MR)) -> stream (Eq. (MRT)) with DBB walls
# (Eqs. (bot), (bot2)) -> inlet/outlet (Eqs. (rho1), (rho2)).  R17.
# ---------------------------------------------------------------------------
def collide(f: np.ndarray, p: Params) -> np.ndarray:
    """Post-collision populations f' = f - M^-1 S (M f - m^eq) (R1: relaxing sign)."""
    rho_s, jx_s, jy_s, rho, ux, uy = moments(f)
    rt = relaxation_times(rho_s[0], rho_s[1], p)
    inv = lambda t: 1.0 / t                                 # noqa: E731
    ones = np.ones_like(rt.tau_s)
    if p.tau_bgk is not None:
        srate = [inv(rt.tau_s)] * 9
    else:
        srate = [ones / TAU_RHO, ones / TAU_E, ones / TAU_EPS, inv(rt.tau_d), inv(rt.tau_q),
                 inv(rt.tau_d), inv(rt.tau_q), inv(rt.tau_s), inv(rt.tau_s)]   # Eq. (S)
    srate = np.stack(srate)                                  # (9, ny, nx)
    out = np.empty_like(f)
    for sig in range(2):
        feq = f_equilibrium(rho_s[sig], ux, uy, p.s[sig])
        m = np.tensordot(M, f[sig], axes=([1], [0]))
        meq = np.tensordot(M, feq, axes=([1], [0]))
        mpost = m - srate * (m - meq)
        out[sig] = np.tensordot(M_INV, mpost, axes=([1], [0]))
    return out


def dbb_walls(fnew: np.ndarray, fpost: np.ndarray, p: Params) -> None:
    """Diffuse-bounce-back, Eqs. (bot) and (bot2), in place on the streamed array.

    R12: the wall equilibrium is the species equilibrium at the stationary wall
    velocity u_w = 0, and its density rho_w is the one for which the wall
    passes no mass: the populations returned carry the same mass as the
    post-collision populations leaving through the wall at that node.
    """
    r = p.dbb_r
    for sig in range(2):
        s = p.s[sig]
        for row, unknown, leaving in ((0, (2, 5, 6), (4, 7, 8)),
                                      (p.ny - 1, (4, 7, 8), (2, 5, 6))):
            out_mass = sum(fpost[sig, i, row, :] for i in leaving)
            w_in = sum(W[i] * s for i in unknown)            # sum of w_i alpha_si over returned set
            rho_w = out_mass / w_in
            feq_w = f_equilibrium(rho_w, 0.0, 0.0, s)       # (9, nx)
            for iu, il in zip(unknown, leaving):
                fnew[sig, iu, row, :] = r * feq_w[iu] + (1.0 - r) * fpost[sig, il, row, :]


# Populations that enter the channel through the inlet (c_x = +1) and the
# outlet (c_x = -1): after streaming they have no source node.
INLET_UNKNOWN = (1, 5, 8)
OUTLET_UNKNOWN = (3, 6, 7)


def inlet_outlet(fnew: np.ndarray, p: Params) -> None:
    """Extrapolation-correction pressure boundary, Eqs. (rho1), (rho2), in place.

    R14: the unknown populations of the boundary node (those entering from the
    reservoir) are extrapolated linearly from the first and second inner layers,
    f_i(0, j) = 2 f_i(1, j) - f_i(2, j); the extrapolated density
    rho'(0, j) = 2 rho(1, j) - rho(2, j) is corrected to
    rho(0, j) = rho'(0, j) N rho_bc / sum_j rho'(0, j)  (R15: N = ny), and the
    node's populations are rescaled to carry that density.
    """
    rin, rout = boundary_densities(p)
    for sig in range(2):
        for col, l1, l2, rho_bc, unknown in ((0, 1, 2, rin[sig], INLET_UNKNOWN),
                                             (p.nx - 1, p.nx - 2, p.nx - 3, rout[sig], OUTLET_UNKNOWN)):
            for i in unknown:
                fnew[sig, i, :, col] = 2.0 * fnew[sig, i, :, l1] - fnew[sig, i, :, l2]
            rho_prime = 2.0 * fnew[sig, :, :, l1].sum(axis=0) - fnew[sig, :, :, l2].sum(axis=0)   # (ny,)
            kappa = p.ny * rho_bc / rho_prime.sum()
            rho_node = fnew[sig, :, :, col].sum(axis=0)
            fnew[sig, :, :, col] *= kappa * rho_prime / rho_node


def stream(fpost: np.ndarray, p: Params) -> np.ndarray:
    """f(x + c_i, t + 1) = f'(x, t) for every in-range source, then walls and ends."""
    fnew = np.empty_like(fpost)
    for i in range(9):
        fnew[:, i] = np.roll(np.roll(fpost[:, i], int(CY[i]), axis=-2), int(CX[i]), axis=-1)
    if not p.periodic_y:
        dbb_walls(fnew, fpost, p)
    if not p.periodic_x:
        inlet_outlet(fnew, p)
    return fnew


def step(f: np.ndarray, p: Params) -> np.ndarray:
    return stream(collide(f, p), p)


# ---------------------------------------------------------------------------
# Initial state (R18) and diagnostics (Eqs. (C), (CL), (Clline); R16).
# ---------------------------------------------------------------------------
def initial_state(p: Params, x0: int = 0, x1: int | None = None) -> np.ndarray:
    """Local equilibrium at rest with pressure and light mole fraction linear in
    x between (P_in, C_l,in) at column 0 and (P_out, C_l,out) at column nx-1
    (R18). Optionally only the columns [x0, x1) of that state."""
    x1 = p.nx if x1 is None else x1
    x = np.arange(x0, x1, dtype=np.float64)
    frac = x / (p.nx - 1) if p.nx > 1 else np.zeros_like(x)
    pres = p_in(p) + (P_OUT - p_in(p)) * frac
    cl = p.cl_in + (p.cl_out - p.cl_in) * frac
    rho_a, rho_b = species_density(p, pres, cl)
    nx = x1 - x0
    f = np.empty((2, 9, p.ny, nx))
    zeros = np.zeros((p.ny, nx))
    f[0] = f_equilibrium(np.broadcast_to(rho_a, (p.ny, nx)), zeros, zeros, p.s[0])
    f[1] = f_equilibrium(np.broadcast_to(rho_b, (p.ny, nx)), zeros, zeros, p.s[1])
    return f


@dataclass
class Diagnostics:
    n_a: np.ndarray          # sum_j n_a(x, j)  per column
    n_b: np.ndarray          # sum_j n_b(x, j)
    j_a: np.ndarray          # sum_j rho_a u_ax (Eq. (rhou) species velocity)
    j_b: np.ndarray
    cl_profile: np.ndarray   # C_l(x) = N_a / (N_a + N_b), Eq. (C) over the cross-section
    cl: float                # CL, Eq. (CL)
    cl_tilde: float          # C~_l, Eq. (Clline)
    x_min: int               # column of the smallest C_l (first one on ties)


def diagnostics(f: np.ndarray, p: Params) -> Diagnostics:
    rho_s, ux_s, uy_s = species_velocity(f, p)
    n_a = (rho_s[0] / p.m_a).sum(axis=0)
    n_b = (rho_s[1] / p.m_b).sum(axis=0)
    cl_x = n_a / (n_a + n_b)
    x_min = int(np.argmin(cl_x))
    cl = (p.cl_in - cl_x[x_min]) / p.cl_in
    cl_tilde = float(np.sum(cl_x - p.cl_in) / (p.nx * p.cl_in))
    j_a = (rho_s[0] * ux_s[0]).sum(axis=0)
    j_b = (rho_s[1] * ux_s[1]).sum(axis=0)
    return Diagnostics(n_a, n_b, j_a, j_b, cl_x, float(cl), cl_tilde, x_min)


def volume_flow(f: np.ndarray, p: Params) -> np.ndarray:
    """Q_v(x) = sum_j u_x(x, j): volume flow of the mixture through each
    cross-section (Sec. 4, Fig. of Q_v against Kn_out; the formula is not
    printed, R25), u the mixture velocity of Eq. (rhou), delta_y = 1."""
    _, _, _, _, ux, _ = moments(f)
    return ux.sum(axis=0)


def moment_fields(f: np.ndarray, p: Params) -> np.ndarray:
    """(6, ny, nx): rho_a, rho_b, u_ax, u_ay, u_bx, u_by (species velocity of Eq. (rhou))."""
    rho_s, ux_s, uy_s = species_velocity(f, p)
    return np.stack([rho_s[0], rho_s[1], ux_s[0], uy_s[0], ux_s[1], uy_s[1]])


def run(p: Params, nsteps: int, f0: np.ndarray | None = None, record_every: int = 0, strict: bool = True):
    """Advance nsteps from f0 (default: the initial state). Returns (f, history)
    where history lists (t, CL, C~_l) every record_every steps (if > 0).
    strict: raise on overflow / invalid / division by zero (off only for runs
    whose edges are known to be invalid, e.g. a window cut out of a channel)."""
    f = initial_state(p) if f0 is None else np.array(f0, dtype=np.float64, copy=True)
    hist = []
    mode = "raise" if strict else "ignore"
    with np.errstate(over=mode, invalid=mode, divide=mode, under="ignore"):
        for t in range(1, nsteps + 1):
            f = step(f, p)
            if record_every and t % record_every == 0:
                d = diagnostics(f, p)
                hist.append((t, d.cl, d.cl_tilde))
    return f, hist


def dbb_r_from_cm(c_m: float, m_a: float, m_b: float, cl: float) -> float:
    """r = 2 - 2 [1 + (c_m / 3) sqrt(pi m_x / (2 k_B T))]^-1, Eq. (R) first form,
    with k_B T = m_min c_s^2 and m_x of the mixture at light fraction cl (R10)."""
    m_min = min(m_a, m_b)
    m_x = cl * m_a + (1.0 - cl) * m_b
    kbt = m_min * CS2
    return 2.0 - 2.0 / (1.0 + (c_m / 3.0) * math.sqrt(math.pi * m_x / (2.0 * kbt)))
