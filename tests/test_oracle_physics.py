"""Physics pins of the CPU oracle: limits in which the binary-mixture method of
Sec. 3 must reduce to something else that is known.

* Equal molecular masses: the mixture is one gas; f_a + f_b must follow a
  single-species D2Q9 MRT solver (Lallemand-Luo basis, textbook equilibrium)
  with the same wall and end conditions. The solver below is written
  independently: its own equilibrium, explicit moment formulas, slicing
  streaming, and the wall function through E_3 instead of E_1.
* Near-continuum single-species flow between the walls: a parabolic profile
  whose curvature is -(dP/dx)/mu with mu = rho c_s^2 (tau_s - 1/2).
"""
import math

import numpy as np
import pytest
from scipy.special import expn

from oracle import binary_lbm as O

# ---------------------------------------------------------------------------
# Independent single-species solver (test-local).
# ---------------------------------------------------------------------------
_C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
_W = [4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36]


def _feq1(rho, ux, uy):
    out = []
    for (cx, cy), w in zip(_C, _W):
        cu = cx * ux + cy * uy
        out.append(w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy)))
    return np.array(out)


def _basis():
    rows = []
    for cx, cy in _C:
        c2 = cx * cx + cy * cy
        rows.append([1, 3 * c2 - 4, 4.5 * c2 * c2 - 10.5 * c2 + 4, cx, (3 * c2 - 5) * cx, cy,
                     (3 * c2 - 5) * cy, cx * cx - cy * cy, cx * cy])
    return np.array(rows, dtype=float).T          # (9 moments, 9 directions)


_B = _basis()
_NORM2 = (_B * _B).sum(axis=1)


def _psi_e3(a):
    a = np.asarray(a, float)
    return 1.0 - 2.0 * expn(3, a)


def _single_species_step(f, ny, nx, kn, r, rho_in, rho_out, accom=1.0):
    rho = f.sum(0)
    ux = sum(c[0] * f[i] for i, c in enumerate(_C)) / rho
    uy = sum(c[1] * f[i] for i, c in enumerate(_C)) / rho
    p = rho / 3.0
    lam = kn * ny * (1 / 3) / p
    y = (np.arange(ny) + 0.5)[:, None]
    k = math.sqrt(6 / math.pi)
    ts = lam * 0.5 * (_psi_e3(y / lam) + _psi_e3((ny - y) / lam)) * k
    a = ny / lam
    tt0 = k * lam * 0.5 * _psi_e3(a)
    # derivative of 1 - 2 E_3(alpha) is 2 E_2(alpha); at 0 it is 2
    dtt0 = 0.5 * k * (2.0 - 2.0 * expn(2, a))
    a1 = (2 - accom) / accom * (1 - 0.1817 * accom)
    a2 = 1 / math.pi + a1 * a1 / 2
    tq = 0.5 + (3 + 4 * math.pi * tt0 ** 2 * a2) / (16 * tt0) \
        + dtt0 * (12 + 30 * tt0 * math.sqrt(math.pi / 6) * a1) / (16 * tt0 ** 2)
    rates = [1.0, 1 / 1.1, 1 / 1.2, 0.0, 1 / tq, 0.0, 1 / tq, 1 / (ts + 0.5), 1 / (ts + 0.5)]
    m = np.tensordot(_B, f, axes=([1], [0]))
    meq = np.tensordot(_B, _feq1(rho, ux, uy), axes=([1], [0]))
    mp = np.stack([m[k_] - rates[k_] * (m[k_] - meq[k_]) for k_ in range(9)])
    fp = np.tensordot(_B.T, mp / _NORM2[:, None, None], axes=([1], [0]))
    fn = np.empty_like(fp)
    for i, (cx, cy) in enumerate(_C):
        src = fp[i]
        # shift by (cx, cy) with periodic wrap, written with slicing
        tmp = np.concatenate([src[:, nx - cx:], src[:, :nx - cx]], axis=1) if cx > 0 else (
            np.concatenate([src[:, -cx:], src[:, :-cx]], axis=1) if cx < 0 else src)
        tmp = np.concatenate([tmp[ny - cy:], tmp[:ny - cy]], axis=0) if cy > 0 else (
            np.concatenate([tmp[-cy:], tmp[:-cy]], axis=0) if cy < 0 else tmp)
        fn[i] = tmp
    # walls: stationary, zero mass flux; equilibrium at rest has weights 4/6, 1/6, 1/6 of the set
    for row, unk, lev in ((0, (2, 5, 6), (4, 7, 8)), (ny - 1, (4, 7, 8), (2, 5, 6))):
        out = fp[lev[0], row] + fp[lev[1], row] + fp[lev[2], row]
        for iu, il, share in zip(unk, lev, (4 / 6, 1 / 6, 1 / 6)):
            fn[iu, row] = r * share * out + (1 - r) * fp[il, row]
    # ends: directions entering from the reservoir are extrapolated, then the
    # node is rescaled to the corrected extrapolated density
    for col, c1, c2, rb, enter in ((0, 1, 2, rho_in, (1, 5, 8)), (nx - 1, nx - 2, nx - 3, rho_out, (3, 6, 7))):
        fn[list(enter), :, col] = 2 * fn[list(enter), :, c1] - fn[list(enter), :, c2]
        target = 2 * fn[:, :, c1].sum(0) - fn[:, :, c2].sum(0)
        target = target * (ny * rb / target.sum())
        fn[:, :, col] = fn[:, :, col] * (target / fn[:, :, col].sum(0))
    return fn


def test_equal_masses_reduce_to_single_species_mrt():
    """P9: with m_a = m_b the mixture sum f_a + f_b follows the single-species
    solver to round-off (tau_d drops out because total momentum is conserved)."""
    ny, nx, kn, r, theta = 6, 24, 0.2, 0.74, 2.0
    p = O.Params(nx=nx, ny=ny, m_a=10, m_b=10, cl_in=0.35, cl_out=0.35, theta=theta, kn_out=kn, dbb_r=r)
    f = O.initial_state(p)
    g = f[0] + f[1]
    for _ in range(200):
        f = O.step(f, p)
        g = _single_species_step(g, ny, nx, kn, r, theta, 1.0)
    assert np.max(np.abs(f[0] + f[1] - g)) / np.max(np.abs(g)) < 1e-12


def test_single_species_solver_self_check():
    """The test-local solver conserves mass with periodic ends removed from the
    picture: a uniform rest state is a fixed point."""
    ny, nx = 5, 12
    g = _feq1(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    g2 = _single_species_step(g, ny, nx, 0.1, 0.74, 1.0, 1.0)
    assert np.allclose(g2, g, atol=1e-15)


@pytest.mark.slow
def test_near_continuum_poiseuille_is_parabolic():
    """P10: single-species limit (m_a = m_b), small pressure ratio, small Kn, MFP
    correction off: the steady cross-channel profile of u_x at mid-channel is a
    parabola whose curvature is -(dP/dx)/mu, mu = rho c_s^2 (tau_s - 1/2)."""
    ny, nx = 16, 96
    p = O.Params(nx=nx, ny=ny, m_a=1, m_b=1, cl_in=0.5, cl_out=0.5, theta=1.01, kn_out=0.01,
                 dbb_r=0.74, mfp_off=True)
    f, _ = O.run(p, 6000)
    mf = O.moment_fields(f, p)
    rho = mf[0] + mf[1]
    ux = (mf[0] * mf[2] + mf[1] * mf[4]) / rho
    xm = nx // 2
    y = np.arange(ny) + 0.5
    u = ux[:, xm]
    coef = np.polyfit(y, u, 2)
    resid = u - np.polyval(coef, y)
    assert np.sqrt(np.mean(resid ** 2)) / np.max(np.abs(u)) < 1e-3
    pres = O.CS2 * rho.mean(axis=0)
    dpdx = (pres[xm + 1] - pres[xm - 1]) / 2
    rt = O.relaxation_times(mf[0], mf[1], p)
    mu = rho[:, xm].mean() * O.CS2 * (rt.tau_s[:, xm].mean() - 0.5)
    curv = 2 * coef[0]
    assert abs(curv - dpdx / mu) / abs(dpdx / mu) < 0.02


def test_volume_flow_equal_masses_matches_the_single_species_solver():
    """R25 (Q_v of Sec. 4): with m_a = m_b the mixture volume flow sum_j u_x
    equals that of the independent single-species solver (its own moments),
    and it is also the density-weighted sum of the species velocities of
    Eq. (rhou) (species momenta add up to the mixture momentum)."""
    ny, nx, kn, r, theta = 6, 24, 0.2, 0.74, 2.0
    p = O.Params(nx=nx, ny=ny, m_a=10, m_b=10, cl_in=0.35, cl_out=0.35, theta=theta, kn_out=kn, dbb_r=r)
    f = O.initial_state(p)
    g = f[0] + f[1]
    for _ in range(150):
        f = O.step(f, p)
        g = _single_species_step(g, ny, nx, kn, r, theta, 1.0)
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
    q_single = (np.tensordot(cx, g, axes=([0], [0])) / g.sum(axis=0)).sum(axis=0)
    q = O.volume_flow(f, p)
    assert np.max(np.abs(q - q_single)) <= 1e-12 * np.max(np.abs(q_single))
    mf = O.moment_fields(f, p)
    q_species = ((mf[0] * mf[2] + mf[1] * mf[4]) / (mf[0] + mf[1])).sum(axis=0)
    assert np.max(np.abs(q - q_species)) <= 1e-12 * np.max(np.abs(q))
    assert np.all(q > 0)  # the pressure drives the flow from inlet to outlet
