"""Closed forms and exact identities that fix the constants and weights of the
oracle's relaxation times, species velocity and separation diagnostics, and
the discrete continuity of its streaming (P11). Each test states the passage
it pins; a plausible mistake (a wrong prefactor in Eq. (EQFrsp), the two
weights of Eq. (rhou) swapped, CL divided by C_min instead of C_in, a leaking
wall or a wrong interface flux) fails one of them."""
import json
import math
import os

import numpy as np
import pytest

from oracle import binary_lbm as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _node(m_a, m_b, x_a, kn, ny, pfac, y, mfp_off=False):
    """Relaxation times of one node of mole fraction x_a at pressure pfac P_out."""
    p = O.Params(nx=8, ny=ny, m_a=m_a, m_b=m_b, cl_in=0.5, cl_out=0.5, theta=2.0, kn_out=kn, dbb_r=1.0,
                 mfp_off=mfp_off)
    ra, rb = O.species_density(p, pfac * O.P_OUT, x_a)
    return O.relaxation_times(np.array([[ra]]), np.array([[rb]]), p, y=np.array([[y]]))


def test_tau_d_equal_masses_closed_form():
    """Eq. (EQFrsp) with m_a = m_b = m and Psi == 1: m_0 = 2m, m_x = m_min = m,
    so the prefactor is (3/2) sqrt(6), and with x_s lambda_s = lambda (R6) the
    bracket is (2 / sqrt(lambda))^-2 = lambda / 4: tau_d - 1/2 = 3 sqrt(6) lambda / 8,
    whatever the composition."""
    for x_a in (0.2, 0.5, 0.9):
        for kn, pfac in ((0.1, 1.0), (0.3, 2.5), (1.0, 0.7)):
            rt = _node(7.0, 7.0, x_a, kn, 16, pfac, 3.5, mfp_off=True)
            lam = kn * 16 / pfac  # lambda = Kn_out H P_out / P (R5)
            assert abs(rt.lam[0, 0] - lam) < 1e-14 * lam
            assert abs((rt.tau_d[0, 0] - 0.5) - 3.0 * math.sqrt(6.0) * lam / 8.0) < 1e-13 * lam


def test_tau_d_unequal_masses_closed_form():
    """He-Ar (4 : 40) at x_a = 1/2, Psi == 1: m_0 = 44, m_x = 22, so
    3 m_0 m_a m_b / (m_min m_x^2) = 3 * 44 * 160 / (4 * 484) = 120/11, and the
    bracket is lambda / 4 as above: tau_d - 1/2 = (3/8) sqrt(120/11) lambda."""
    rt = _node(4.0, 40.0, 0.5, 0.1, 8, 1.0, 0.5, mfp_off=True)
    lam = 0.8
    assert abs((rt.tau_d[0, 0] - 0.5) - 0.375 * math.sqrt(120.0 / 11.0) * lam) < 1e-14


def test_relaxation_times_worked_values():
    """tau_s, tau_d, tau_q at four nodes against values worked out by hand from
    Eqs. (taos), (EQFrsp), (taoq) (tests/golden/p6_relaxation_times.json)."""
    g = json.load(open(os.path.join(HERE, "golden", "p6_relaxation_times.json")))
    for m_a, m_b, x_a, kn, ny, pfac, y, lam, ts, td, tq in g["rows"]:
        rt = _node(m_a, m_b, x_a, kn, ny, pfac, y)
        assert abs(rt.lam[0, 0] - lam) < 1e-13
        assert abs(rt.tau_s[0, 0] - ts) < 2e-12, (y, rt.tau_s[0, 0], ts)
        assert abs(rt.tau_d[0, 0] - td) < 2e-12, (y, rt.tau_d[0, 0], td)
        assert abs(rt.tau_q[0, 0] - tq) < 2e-11, (y, rt.tau_q[0, 0], tq)


def test_species_momentum_is_the_mean_of_pre_and_post_collision_momenta():
    """Eq. (rhou): rho_s u_s = (1 - 1/(2 tau_d)) j_s + rho_s u / (2 tau_d). The
    collision relaxes the species momentum at the rate 1/tau_d towards rho_s u
    (Eq. (S), the momentum rows of M), j_s* = j_s - (j_s - rho_s u)/tau_d, so
    Eq. (rhou) is exactly the average (j_s + j_s*)/2 of the momenta before and
    after the collision. Swapping its two weights breaks this."""
    rng = np.random.default_rng(5)
    p = O.Params(nx=12, ny=6, m_a=4.0, m_b=40.0, cl_in=0.4, cl_out=0.4, theta=2.0, kn_out=0.2, dbb_r=1.1)
    f = O.initial_state(p) * (1.0 + 0.05 * rng.uniform(-1, 1, size=(2, 9, 6, 12)))
    post = O.collide(f, p)
    rho_s, ux_s, uy_s = O.species_velocity(f, p)
    for s in (0, 1):
        for c, u in ((O.CX, ux_s), (O.CY, uy_s)):
            j = np.tensordot(c.astype(float), f[s], axes=([0], [0]))
            js = np.tensordot(c.astype(float), post[s], axes=([0], [0]))
            # rounding of momenta summed from populations of order rho_s
            assert np.allclose(rho_s[s] * u[s], 0.5 * (j + js), rtol=0, atol=1e-15 * rho_s[s].max())
    # the mixture momentum is conserved, so the species momenta of Eq. (rhou)
    # add up to rho u
    assert np.allclose(rho_s[0] * ux_s[0] + rho_s[1] * ux_s[1],
                       np.tensordot(O.CX.astype(float), f.sum(axis=0), axes=([0], [0])), atol=1e-14)


def _state_with_composition(p, c_of_x, n_of_j):
    """Local equilibrium at rest (Eq. (feq), u = 0) with number densities
    n_a = c(x) n(j), n_b = (1 - c(x)) n(j)."""
    f = np.empty((2, 9, p.ny, p.nx))
    n = n_of_j[:, None] * np.ones((1, p.nx))
    c = np.ones((p.ny, 1)) * c_of_x[None, :]
    for s, (m, share) in enumerate(((p.m_a, c), (p.m_b, 1.0 - c))):
        rho = m * share * n
        f[s] = O.f_equilibrium(rho, 0.0, 0.0, p.s[s])
    return f


def test_separation_degree_on_a_built_profile():
    """Eqs. (C), (CL), (Clline) on a state whose C_l(x) is known: C_l(x) =
    1/2 - sin(pi x / 10) / 10 on 11 columns (every row at the same composition,
    rows at different densities). The smallest C_l is 0.4 at x = 5, so
    CL = (0.5 - 0.4) / 0.5 = 0.2 (dividing by C_min would give 0.25), and
    C~_l = -sum_x sin(pi x / 10) / (10 * 11 * 0.5) = -cot(pi / 20) / 55."""
    p = O.Params(nx=11, ny=5, m_a=4.0, m_b=40.0, cl_in=0.5, cl_out=0.5, theta=2.0, kn_out=0.2, dbb_r=1.1)
    x = np.arange(11)
    f = _state_with_composition(p, 0.5 - np.sin(np.pi * x / 10) / 10, np.array([1.0, 1.3, 0.8, 2.0, 1.1]))
    d = O.diagnostics(f, p)
    assert np.allclose(d.cl_profile, 0.5 - np.sin(np.pi * x / 10) / 10, rtol=0, atol=1e-15)
    assert abs(d.cl - 0.2) < 1e-15
    assert d.x_min == 5
    assert abs(d.cl_tilde - (-1.0 / math.tan(math.pi / 20) / 55.0)) < 1e-15


def test_cross_section_mole_fraction_is_a_ratio_of_sums():
    """Eq. (C) over a cross-section: C_l,x = sum_j n_a / (sum_j n_a + sum_j n_b),
    not the mean over rows of the local ratios. Two rows: (n_a, n_b) = (1, 3)
    and (3, 1) give 1/2; the mean of the local ratios would also be 1/2, so the
    second pair (1, 1) and (1, 3) separates them: 2/6 = 1/3 against
    (1/2 + 1/4)/2 = 3/8. CL = (C_in - 1/3)/C_in with C_in = 0.45."""
    p = O.Params(nx=6, ny=2, m_a=4.0, m_b=40.0, cl_in=0.45, cl_out=0.45, theta=2.0, kn_out=0.2, dbb_r=1.1)
    na = np.array([[1.0, 1.0, 1.0, 1.0, 1.0, 1.0], [3.0, 1.0, 3.0, 3.0, 3.0, 3.0]])
    nb = np.array([[3.0, 1.0, 3.0, 3.0, 3.0, 3.0], [1.0, 3.0, 1.0, 1.0, 1.0, 1.0]])
    f = np.stack([O.f_equilibrium(4.0 * na, 0.0, 0.0, p.s[0]), O.f_equilibrium(40.0 * nb, 0.0, 0.0, p.s[1])])
    d = O.diagnostics(f, p)
    assert abs(d.cl_profile[1] - 1.0 / 3.0) < 1e-15 and abs(d.cl_profile[0] - 0.5) < 1e-15
    assert d.x_min == 1 and abs(d.cl - (0.45 - 1.0 / 3.0) / 0.45) < 1e-15


def _interface_flux(post, p):
    """Mass of species s crossing from column x to x + 1 in one streaming step,
    per interface x + 1/2 (x = 0 .. nx-2): post-collision populations leaving
    column x with c_x = +1 minus those leaving column x + 1 with c_x = -1.
    On a wall row the diagonal populations that head into the wall cross no
    interface: DBB returns them in the same column (Eqs. (bot), (bot2))."""
    crosses = np.ones((9, p.ny), dtype=bool)
    crosses[O.CY == -1, 0] = False        # leaving through the bottom wall
    crosses[O.CY == 1, p.ny - 1] = False  # leaving through the top wall
    right = (O.CX == 1)[:, None] & crosses
    left = (O.CX == -1)[:, None] & crosses
    out_r = (post * right[None, :, :, None]).sum(axis=(1, 2))   # (2, nx)
    out_l = (post * left[None, :, :, None]).sum(axis=(1, 2))
    return out_r[:, :-1] - out_l[:, 1:]


def test_discrete_continuity_of_each_column():
    """P11 (per step): the collision conserves each species' mass at every
    node (Eq. (MR): tau_rho relaxes rho onto itself) and the DBB walls return
    exactly what leaves through them (R12), so the mass of an interior column
    after a step is its mass before plus the inflow through its left interface
    minus the outflow through its right one, for any state."""
    rng = np.random.default_rng(11)
    p = O.Params(nx=14, ny=5, m_a=20.0, m_b=40.0, cl_in=0.3, cl_out=0.6, theta=2.5, kn_out=0.1, dbb_r=0.9)
    f = O.initial_state(p) * (1.0 + 0.1 * rng.uniform(-1, 1, size=(2, 9, 5, 14)))
    post = O.collide(f, p)
    nxt = O.stream(post, p)
    flux = _interface_flux(post, p)
    mass0 = f.sum(axis=(1, 2))
    mass1 = nxt.sum(axis=(1, 2))
    for x in range(1, p.nx - 1):  # columns 0 and nx-1 are rebuilt by Eqs. (rho1), (rho2)
        expect = mass0[:, x] + flux[:, x - 1] - flux[:, x]
        assert np.allclose(mass1[:, x], expect, rtol=0, atol=1e-13 * mass0.max())


@pytest.mark.slow
def test_steady_state_species_flux_is_the_same_through_every_interface():
    """P11: at steady state every interior column keeps its mass, so by the
    per-step continuity above each species' flux is the same through every
    interior interface. He-Ar, 8 x 80 channel, theta = 2, Kn_out = 0.1: after
    6000 steps the flux profile is flat to 1e-8 of its mean (it reaches 2e-9;
    below that a mode of the inlet/outlet closure that grows by about 3e-5 per
    step, from round-off, sets the floor)."""
    p = O.Params(nx=80, ny=8, m_a=4.0, m_b=40.0, cl_in=0.5, cl_out=0.5, theta=2.0, kn_out=0.1,
                 dbb_r=O.dbb_r_from_cm(0.8183, 4.0, 40.0, 0.5))
    f = O.initial_state(p)
    for _ in range(6000):
        f = O.step(f, p)
    flux = _interface_flux(O.collide(f, p), p)[:, 1:-1]  # interfaces between interior columns
    mean = flux.mean(axis=1, keepdims=True)
    spread = float(np.max(np.abs(flux - mean) / np.abs(mean)))
    assert spread < 1e-8, spread
    # the flux is a real through-flow, in the flow direction for both species
    assert np.all(mean > 0)
