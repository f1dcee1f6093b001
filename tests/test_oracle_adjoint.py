"""Pins of the CPU reverse sweep (oracle/adjoint.py): its step is the NumPy
oracle's step, and its derivatives are the finite-difference derivatives of
the NumPy oracle (central differences, h = 1e-6 relative)."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import binary_lbm as O

torch = pytest.importorskip("torch")


def _params(**kw):
    base = dict(nx=40, ny=6, m_a=4.0, m_b=40.0, cl_in=0.5, cl_out=0.5, theta=2.0, kn_out=0.1,
                dbb_r=O.dbb_r_from_cm(0.8183, 4.0, 40.0, 0.5))
    base.update(kw)
    return O.Params(**base)


def _perturbed_state(p, seed=3):
    rng = np.random.default_rng(seed)
    f = O.initial_state(p)
    return f * (1.0 + 0.02 * rng.uniform(-1, 1, size=f.shape))


@pytest.mark.parametrize("mode", [{}, {"periodic_x": True}, {"mfp_off": True, "periodic_y": True}])
def test_torch_step_equals_the_numpy_step(mode):
    p = _params(**mode)
    f = _perturbed_state(p)
    g = f.copy()
    ft = torch.tensor(f)
    th, cl, r = (torch.tensor(v, dtype=torch.float64) for v in (p.theta, p.cl_in, p.dbb_r))
    for _ in range(5):
        g = O.step(g, p)
        ft = A.step(ft, p, th, cl, r)
    assert np.max(np.abs(ft.numpy() - g)) <= 1e-13 * np.max(np.abs(g))
    assert np.allclose(A.initial_state(p, th, cl).numpy(), O.initial_state(p), rtol=1e-15, atol=0)


def _oracle_cl(p, nsteps):
    f, _ = O.run(p, nsteps)
    d = O.diagnostics(f, p)
    return d.cl, d.x_min


def test_reverse_sweep_gradients_equal_central_differences():
    p = _params()
    nsteps = 150
    cl, grads = A.gradients(p, nsteps)
    cl_ref, xmin = _oracle_cl(p, nsteps)
    assert abs(cl - cl_ref) <= 1e-14
    for k, name in enumerate(("theta", "cl_in", "dbb_r")):
        v = getattr(p, name)
        h = 1e-6 * v
        up = O.Params(**{**p.__dict__, name: v + h})
        dn = O.Params(**{**p.__dict__, name: v - h})
        (c_up, x_up), (c_dn, x_dn) = _oracle_cl(up, nsteps), _oracle_cl(dn, nsteps)
        assert x_up == x_dn == xmin  # CL is smooth here: the minimum stays in one column
        fd = (c_up - c_dn) / (2 * h)
        assert abs(grads[k] - fd) <= 1e-6 * abs(fd) + 1e-9, (name, grads[k], fd)


def test_single_step_adjoint_satisfies_the_dot_product_identity():
    """lam . (J df) = (J^T lam) . df with J df from central differences of the
    NumPy step, for random lam and df, at a perturbed state (walls and ends)."""
    p = _params()
    f = _perturbed_state(p)
    rng = np.random.default_rng(7)
    lam = rng.standard_normal(f.shape)
    df = rng.standard_normal(f.shape) * f
    h = 1e-6
    jdf = (O.step(f + h * df, p) - O.step(f - h * df, p)) / (2 * h)
    lam_t, dparams = A.step_vjp(f, lam, p)
    lhs = float(np.sum(lam * jdf))
    rhs = float(np.sum(lam_t * df))
    assert abs(lhs - rhs) <= 1e-7 * abs(lhs)
    # explicit parameter derivatives of one step against differences in the parameter
    for k, name in enumerate(("theta", "cl_in", "dbb_r")):
        v = getattr(p, name)
        hp = 1e-6 * v
        up = O.Params(**{**p.__dict__, name: v + hp})
        dn = O.Params(**{**p.__dict__, name: v - hp})
        fd = float(np.sum(lam * (O.step(f, up) - O.step(f, dn)))) / (2 * hp)
        assert abs(dparams[k] - fd) <= 1e-6 * abs(fd) + 1e-9, (name, dparams[k], fd)
