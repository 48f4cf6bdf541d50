"""Pins for the FP64 references of the learned indicator (oracle/mlp.py)."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import mlp


def test_vortex_closed_forms():
    a = 5.0
    rho = mlp.vortex_field(np.array([0.0]), np.array([0.0]), [(0.0, 0.0)], [a])
    dT = -a * a * 0.4 / (16 * 0.5 * 1.4 * math.pi ** 2) * math.exp(1.0)
    T = 1 + dT
    r = T ** 2.5
    assert abs(rho[0, 0] - r) < 1e-14                 # density on the axis
    assert abs(rho[1, 0] - r) < 1e-14                 # rho*u = rho (u = 1 on the axis)
    assert abs(rho[2, 0]) < 1e-15                     # no v on the axis
    far = mlp.vortex_field(np.array([40.0]), np.array([-30.0]), [(0.0, 0.0)], [a])[:, 0]
    np.testing.assert_allclose(far, [1.0, 1.0, 0.0, 0.0, 1.0 / 0.4 + 0.5], atol=1e-14)


def test_vortex_is_isentropic_and_rotational():
    g = np.random.default_rng(0)
    x, y = g.uniform(-4, 4, size=(2, 500))
    q = mlp.vortex_field(x, y, [(0.3, -0.2), (1.0, 2.0)], [4.0, 6.0])
    rho = q[0]
    u, v = q[1] / rho, q[2] / rho
    p = (q[4] - 0.5 * rho * (u * u + v * v)) * 0.4
    np.testing.assert_allclose(p / rho ** 1.4, 1.0, rtol=1e-12)
    # one vortex: the velocity perturbation is tangential with |dv| ~ r e^{phi(1-r^2)}
    q = mlp.vortex_field(x, y, [(0.0, 0.0)], [5.0])
    du, dv = q[1] / q[0] - 1.0, q[2] / q[0]
    np.testing.assert_allclose(du * x + dv * y, 0.0, atol=1e-13)
    r2 = x * x + y * y
    # (rho u)/rho - 1 cancels to ~1e-16 absolute where the perturbation is small
    np.testing.assert_allclose(np.hypot(du, dv), 5 / (2 * math.pi) * np.sqrt(r2) * np.exp(0.5 * (1 - r2)),
                               rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 3), (3, 2)])
def test_modal_exact_and_parseval(dim, p):
    x, w = np.polynomial.legendre.leggauss(p + 1)
    n1 = p + 1
    pts = np.array(np.meshgrid(*([x] * dim), indexing="ij")).reshape(dim, -1)[::-1]  # x fastest
    W = np.ones(1)
    for _ in range(dim):
        W = np.kron(w, W)
    for k in range(n1 ** dim):
        kk = [(k // n1 ** a) % n1 for a in range(dim)]
        val = np.ones(pts.shape[1])
        for a in range(dim):
            c = np.zeros(kk[a] + 1)
            c[kk[a]] = 1.0
            val *= npleg.legval(pts[a], c) * math.sqrt((2 * kk[a] + 1) / 2.0)
        cf = mlp.modal(val[None, :], dim, p)[0]
        e = np.zeros(n1 ** dim)
        e[k] = 1.0
        np.testing.assert_allclose(cf, e, atol=1e-13)
    u = np.random.default_rng(1).standard_normal(n1 ** dim)
    c = mlp.modal(u[None, :], dim, p)[0]
    assert abs((c * c).sum() - (W * u * u).sum()) < 1e-12


def test_mlp_gradients_match_finite_differences():
    g = np.random.default_rng(2)
    B = 7
    X = g.standard_normal((B, 320))
    y = g.integers(0, 3, size=B)
    params = [g.standard_normal((320, 128)) * 0.05, g.standard_normal(128) * 0.1,
              g.standard_normal((128, 64)) * 0.1, g.standard_normal(64) * 0.1,
              g.standard_normal((64, 3)) * 0.1, g.standard_normal(3) * 0.1]
    loss, grads = mlp.loss_and_grads(X, y, *params)
    h = 1e-6
    for pi, (P, G) in enumerate(zip(params, grads)):
        flat = P.reshape(-1)
        for idx in g.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(X, y, *params)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(X, y, *params)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (pi, idx)


def test_stored_activation_gradients():
    """With a storage map on the activations: identity gives the plain
    gradients; with rounding, the last layer's gradients (which do not pass
    through the map) still match finite differences exactly."""
    g = np.random.default_rng(3)
    B = 9
    X = g.standard_normal((B, 320))
    y = g.integers(0, 3, size=B)
    params = [g.standard_normal((320, 128)) * 0.05, g.standard_normal(128) * 0.1,
              g.standard_normal((128, 64)) * 0.1, g.standard_normal(64) * 0.1,
              g.standard_normal((64, 3)) * 0.1, g.standard_normal(3) * 0.1]
    l0, g0 = mlp.loss_and_grads(X, y, *params)
    l1, g1 = mlp.loss_and_grads(X, y, *params, store=lambda a: a)
    assert l0 == l1 and all(np.array_equal(a, b) for a, b in zip(g0, g1))
    rnd = lambda a: np.round(a * 64.0) / 64.0          # a coarse storage grid
    loss, grads = mlp.loss_and_grads(X, y, *params, store=rnd)
    assert abs(loss - l0) > 1e-6                        # the map does act
    h = 1e-6
    for pi in (4, 5):
        flat = params[pi].reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(X, y, *params, store=rnd)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(X, y, *params, store=rnd)
            flat[idx] = old
            assert abs((lp - lm) / (2 * h) - grads[pi].reshape(-1)[idx]) <= 1e-7


def _mode_field(dim, p, degs, scale=1.0):
    """Nodal values at the Gauss-Legendre points of the tensor orthonormal
    Legendre mode with per-axis degrees `degs` (x fastest)."""
    x, _ = np.polynomial.legendre.leggauss(p + 1)
    n1 = p + 1
    val = np.ones(n1 ** dim)
    for i in range(n1 ** dim):
        for a in range(dim):
            c = np.zeros(degs[a] + 1)
            c[degs[a]] = 1.0
            val[i] *= npleg.legval(x[(i // n1 ** a) % n1], c) * math.sqrt((2 * degs[a] + 1) / 2.0)
    return scale * val


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 3), (3, 1), (2, 3)])
def test_modal_energy_single_modes(dim, p):
    """One tensor mode: all its energy is 'top' iff its highest degree is p."""
    import itertools
    for degs in itertools.product(range(p + 1), repeat=dim):
        rho = _mode_field(dim, p, degs, 2.5)[None, :]
        top, tot = mlp.modal_energy(rho, dim, p)
        assert abs(tot[0] - 6.25) < 1e-12
        exp = 6.25 if max(degs) == p else 0.0
        assert abs(top[0] - exp) < 1e-12, degs


def test_modal_energy_two_modes_and_flags():
    """rho = a L0 + b Ltop: s = b^2 / (a^2 + b^2); thresholds and clamps."""
    dim, p = 3, 3
    a0 = _mode_field(dim, p, (0, 0, 0))
    at = _mode_field(dim, p, (1, 3, 0))
    rows, s_exp = [], []
    for a, b in ((1.0, 1e-1), (1.0, 1e-3), (1.0, 1e-6), (2.0, 0.0), (0.0, 0.0)):
        rows.append(a * a0 + b * at)
        s_exp.append(b * b / (a * a + b * b) if a or b else None)
    rho = np.array(rows)
    top, tot = mlp.modal_energy(rho, dim, p)
    for k, s in enumerate(s_exp):
        if s is None:
            assert tot[k] == 0.0
        else:
            # a rounding-level leak (~1e-16) of the mean into the top coefficient
            assert abs(top[k] / tot[k] - s) <= 1e-12 * s + 1e-20
    depth = np.array([5, 5, 5, 5, 5])
    f, ls = mlp.modal_flags(rho, depth, 3, 7, dim, p, tau_r=-4.0, tau_c=-8.0)
    # log10 s = -2, -6, -12, -inf, (zero field)
    assert list(f) == [1, 0, -1, -1, 0]
    f, _ = mlp.modal_flags(rho, np.array([7, 7, 3, 3, 5]), 3, 7, dim, p, tau_r=-4.0, tau_c=-8.0)
    assert list(f) == [0, 0, 0, 0, 0]                   # clamped at d_max / d_min
