"""Shared helpers of the GPU parity tests: build oracle parameters and runs from
the same workload description the HIP path gets, and compare results."""
import numpy as np

from oracle import binary_lbm as O
from paper_1603_08221_amd import lbsep

FLAG_NAMES = {"periodic_x": lbsep.PERIODIC_X, "periodic_y": lbsep.PERIODIC_Y, "mfp_off": lbsep.MFP_OFF}


def oracle_params(w, r, **modes):
    return O.Params(nx=w.nx, ny=w.ny, m_a=w.m_a, m_b=w.m_b, cl_in=w.cl_in, cl_out=w.cl_out, theta=w.theta,
                    kn_out=w.kn_out, dbb_r=r, accom=w.accom, **modes)


def channel(w, r, dtype="f64", tau_bgk=None, hist_cap=4096, tile_mode=0, tile_rows=0, fused_steps=0, **modes):
    flags = 0
    for k, v in modes.items():
        if v:
            flags |= FLAG_NAMES[k]
    if tau_bgk is not None:
        flags |= lbsep.BGK_TEST
    p = lbsep.make_params(w.nx, w.ny, w.m_a, w.m_b, w.cl_in, w.cl_out, w.theta, w.kn_out, r, accom=w.accom,
                          tau_bgk=tau_bgk or 0.0, flags=flags, dtype=dtype, hist_cap=hist_cap,
                          tile_mode=tile_mode, tile_rows=tile_rows, fused_steps=fused_steps)
    return lbsep.Channel(p, device="cuda:0")


def r_of(w):
    """DBB coefficient of the workload, from the oracle's Eq. (R) (the same
    number is handed to both sides)."""
    return O.dbb_r_from_cm(w.c_m, w.m_a, w.m_b, w.cl_in)


def field_errors(got, ref):
    """Normwise relative errors of the species moment vectors (rho_s, rho_s u_s):
    max|d rho_s| / max|rho_s| and max|d (rho_s u_s)| / max|rho_s| (both velocity
    components). The momentum is a sum of O(rho) populations, so its rounding
    error scales with the density, not with the (possibly tiny) velocity; it is
    measured on that scale."""
    errs = []
    for k in (0, 1):
        errs.append(float(np.max(np.abs(got[k] - ref[k])) / max(np.max(np.abs(ref[k])), 1e-300)))
    for k, r in ((2, 0), (4, 1)):
        scale = max(np.max(np.abs(ref[r])), 1e-300)
        dj = max(np.max(np.abs(got[r] * got[k] - ref[r] * ref[k])),
                 np.max(np.abs(got[r] * got[k + 1] - ref[r] * ref[k + 1])))
        errs.append(float(dj / scale))
    return errs


def velocity_errors(got, ref):
    """max|d u_s| / max|u_s| per species (both components): reported, not the
    pass criterion, since it is ill-conditioned where the flow is slow."""
    out = []
    for k in (2, 4):
        scale = max(np.max(np.abs(ref[k])), np.max(np.abs(ref[k + 1])), 1e-300)
        out.append(float(max(np.max(np.abs(got[k] - ref[k])), np.max(np.abs(got[k + 1] - ref[k + 1]))) / scale))
    return out


def assert_moments(got, ref, tol, what=""):
    errs = field_errors(got, ref)
    names = ["rho_a", "rho_b", "j_a", "j_b"]
    bad = {names[k]: e for k, e in enumerate(errs) if not e <= tol}
    assert not bad, f"{what}: moment fields beyond {tol:g}: {bad}"
    return max(errs)


def assert_cl(got, ref, rel, abs_):
    assert abs(got - ref) <= rel * abs(ref) + abs_, (got, ref)


def assert_argmin(got_x, profile_ref, margin=1e-11):
    """The column of the smallest C_l must match where the minimum is unique by
    more than round-off; within the margin any of the tied columns is valid."""
    m = profile_ref.min()
    tied = np.flatnonzero(profile_ref <= m + margin)
    assert got_x in tied, (got_x, tied[:10])
