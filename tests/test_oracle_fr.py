"""Oracle pins for the flux-reconstruction residual (Section 2.1), the
common fluxes with mortars at hanging faces (Section 4.3) and the
three-stage Runge-Kutta step (eq. rk3).

Pins that do not restate the oracle's formulas:
- the Radau correction recovers DG: g_R'(z_i) = l_i(1)/w_i and
  g_L'(z_i) = -l_i(-1)/w_i, the boundary terms of the strong-form DG method
  with its diagonal Gauss-Legendre mass matrix;
- mortar operators reproduce degree-p polynomials and conserve integrals;
- free-stream preservation on adaptive trees with hanging faces;
- discrete conservation: the residual integrates to zero over the periodic
  domain for any data (conservative common fluxes, L2 projection of the
  mortar fluxes);
- a density wave with constant velocity and pressure whose density is a
  global polynomial of degree <= p per axis: on every element away from the
  periodic seam the residual is exactly -(v . grad rho) (1, v, |v|^2 / 2);
- RK3 on du/dt = lambda u gives the cubic Taylor polynomial of exp(lambda dt)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import fr
from paper_2306_06744_amd import synth

LO, L = -5.0, 10.0


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_radau_correction_recovers_dg(p):
    ops = fr.Operators1D(p)
    assert np.allclose(ops.dgR, ops.l_right / ops.w, rtol=0, atol=1e-12)
    assert np.allclose(ops.dgL, -ops.l_left / ops.w, rtol=0, atol=1e-12)
    # g_L(-1) = 1, g_L(1) = 0 and the mirror for g_R
    from numpy.polynomial import legendre as lg
    assert np.allclose(lg.legval([-1.0, 1.0], ops.g_left), [1.0, 0.0], atol=1e-15)
    assert np.allclose(lg.legval([-1.0, 1.0], ops.g_right), [0.0, 1.0], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mortar_operators_exact_and_conservative(p):
    ops = fr.Operators1D(p)
    g = np.random.default_rng(p)
    c = g.standard_normal(p + 1)
    poly = lambda x: np.polyval(c, x)
    z, w = ops.z, ops.w
    for b in range(2):
        assert np.allclose(ops.to_mortar[b] @ poly(z), poly((z + 2 * b - 1) / 2), atol=1e-13)
    back = sum(ops.from_mortar[b] @ poly((z + 2 * b - 1) / 2) for b in range(2))
    assert np.allclose(back, poly(z), atol=1e-13)
    Fm = g.standard_normal((2, p + 1))  # arbitrary mortar fluxes
    coarse = sum(ops.from_mortar[b] @ Fm[b] for b in range(2))
    assert abs(w @ coarse - sum(w @ Fm[b] / 2 for b in range(2))) < 1e-14


def _adaptive_tree(dim, d_max, seed, cycles=3):
    o = oracle.Tree(dim, 1, d_max, start_depth=2)
    for c in range(cycles):
        o.adapt(synth.random_flags(seed + c, o.size(), 0.35, 0.25))
        o.balance()
    nbr, hang = o.connect()
    assert len(hang) > 0
    return o.keys(), nbr, hang


def _vortex_like(pts, dim):
    """A smooth positive state (for tests that need a physical field)."""
    x = pts[..., 0] / L * 2 * np.pi
    y = pts[..., 1] / L * 2 * np.pi
    rho = 1.0 + 0.2 * np.sin(x) * np.cos(y)
    vel = [0.3 + 0.1 * np.cos(x), -0.2 + 0.1 * np.sin(y)] + ([0.05 * np.sin(x + y)] if dim == 3 else [])
    pr = 1.0 + 0.1 * np.cos(x + 2 * y)
    U = [rho] + [rho * v for v in vel] + [pr / 0.4 + 0.5 * rho * sum(v * v for v in vel)]
    return np.transpose(np.stack(U), (0, 2, 1))  # (nvar, n_p, n)


@pytest.mark.parametrize("dim,d_max,p", [(2, 6, 1), (2, 6, 3), (3, 4, 2), (3, 4, 3)])
def test_free_stream_preserved(dim, d_max, p):
    keys, nbr, hang = _adaptive_tree(dim, d_max, 10 * dim + p)
    n = len(keys)
    state = [1.3] + [0.4, -0.7, 0.2][:dim] + [3.1]
    u = np.array(state)[:, None, None] * np.ones((dim + 2, (p + 1) ** dim, n))
    R, _ = fr.residual(keys, nbr, hang, u, dim, d_max, L, p)
    assert np.abs(R).max() <= 1e-12


@pytest.mark.parametrize("dim,d_max,p", [(2, 6, 2), (3, 4, 3)])
def test_residual_integrates_to_zero(dim, d_max, p):
    keys, nbr, hang = _adaptive_tree(dim, d_max, 5 + dim)
    pts = fr.solution_points(keys, dim, d_max, p, (LO,) * dim, L)
    u = _vortex_like(pts, dim)
    u = u * (1.0 + 0.05 * np.random.default_rng(1).standard_normal(u.shape))  # rough data
    R, _ = fr.residual(keys, nbr, hang, u, dim, d_max, L, p)
    w = oracle.gauss_legendre(p + 1)[1]
    W = np.ones(1)
    for _ in range(dim):
        W = np.kron(w, W)
    h = L / 2.0 ** fr._depths(keys, d_max)
    vol = (h / 2) ** dim
    total = np.einsum("i,vie,e->v", W, R, vol)
    scale = np.einsum("i,vie,e->v", W, np.abs(R), vol)
    assert np.all(np.abs(total) <= 1e-13 * scale), total / scale


@pytest.mark.parametrize("dim,d_max,p", [(2, 6, 1), (2, 6, 2), (2, 6, 3), (3, 4, 2), (3, 4, 3)])
def test_density_wave_exact_away_from_seam(dim, d_max, p):
    keys, nbr, hang = _adaptive_tree(dim, d_max, 40 + dim + p)
    n = len(keys)
    pts = fr.solution_points(keys, dim, d_max, p, (LO,) * dim, L)
    g = np.random.default_rng(p)
    coef = 0.05 * g.standard_normal((p + 1,) * dim)
    coef[(0,) * dim] = 2.0
    x = pts / (L / 2)

    def rho_and_grad(x):
        r = np.zeros(x.shape[:-1])
        gr = np.zeros(x.shape)
        for e in itertools.product(range(p + 1), repeat=dim):
            mono = np.ones(x.shape[:-1])
            for a in range(dim):
                mono = mono * x[..., a] ** e[a]
            r += coef[e] * mono
            for a in range(dim):
                if e[a]:
                    d = np.ones(x.shape[:-1]) * coef[e] * e[a] * x[..., a] ** (e[a] - 1)
                    for b in range(dim):
                        if b != a:
                            d = d * x[..., b] ** e[b]
                    gr[..., a] += d / (L / 2)
        return r, gr
    rho, grad = rho_and_grad(x)
    vel = np.array([0.6, -0.35, 0.25][:dim])
    pr = 1.7
    ke = 0.5 * float(vel @ vel)
    U = np.stack([rho] + [rho * v for v in vel] + [pr / 0.4 + ke * rho])
    u = np.transpose(U, (0, 2, 1))
    R, _ = fr.residual(keys, nbr, hang, u, dim, d_max, L, p)
    adv = -(grad @ vel)                                  # (n, n_p)
    exp = np.stack([adv] + [adv * v for v in vel] + [adv * ke])
    exp = np.transpose(exp, (0, 2, 1))
    # elements whose closed box does not touch the domain boundary
    mb = d_max.bit_length()
    inner = []
    for e, k in enumerate(keys):
        d, a = oracle.decode(dim, d_max, int(k))
        s = 2 ** (d_max - d)
        inner.append(all(0 < a[ax] and a[ax] + s < 2 ** d_max for ax in range(dim)))
    inner = np.array(inner)
    assert inner.sum() > n // 3
    # the elements next to hanging faces are among them
    assert np.isin(hang[:, 0], np.flatnonzero(inner)).any()
    # rounding of a derivative of O(|U|) data: ~ulps of |U| times 2/h; a wrong
    # face or mortar term would be of the size of exp itself (>= 1e-3 here)
    h = L / 2.0 ** fr._depths(keys, d_max)
    bar = 1e-13 * np.abs(u).max() * (2.0 / h).max()
    err = np.abs(R[:, :, inner] - exp[:, :, inner]).max()
    print("density wave", dim, p, err, bar, np.abs(exp[:, :, inner]).max())
    assert err <= bar and np.abs(exp[:, :, inner]).max() > 1e4 * bar


def test_rk3_is_the_cubic_taylor_step():
    for z in (-0.3, 0.7, -1.9):
        lam, dt = z / 0.25, 0.25
        u = np.array([1.0, -2.0])
        got = fr.rk3(u, dt, lambda v: lam * v)
        assert np.allclose(got, u * (1 + z + z * z / 2 + z ** 3 / 6), rtol=1e-15, atol=0)


@pytest.mark.parametrize("dim,d_max,p", [(2, 6, 2), (3, 4, 1)])
def test_density_step_is_l2_stable(dim, d_max, p):
    """A density step carried by constant velocity and pressure: the Euler
    equations reduce to linear advection of rho, for which the Rusanov flux
    (dissipation |v| + c >= |v|) makes the DG-equivalent scheme L2-stable.
    int rho^2 must not grow over RK3 steps (it would with the dissipation's
    sign flipped, or with a face term of the wrong element)."""
    keys, nbr, hang = _adaptive_tree(dim, d_max, 60 + dim)
    pts = fr.solution_points(keys, dim, d_max, p, (LO,) * dim, L)
    rho = np.where(np.abs(pts[..., 0] - 0.7) < 2.0, 1.5, 1.0)
    vel = np.array([0.8, 0.3, -0.2][:dim])
    ke = 0.5 * float(vel @ vel)
    u = np.transpose(np.stack([rho] + [rho * v for v in vel] + [1.0 / 0.4 + ke * rho]), (0, 2, 1))
    w = oracle.gauss_legendre(p + 1)[1]
    W = np.ones(1)
    for _ in range(dim):
        W = np.kron(w, W)
    vol = (L / 2.0 ** fr._depths(keys, d_max) / 2) ** dim
    energy = lambda v: float(np.einsum("i,ie,e->", W, v[0] ** 2, vol))
    h_min = L / 2.0 ** fr._depths(keys, d_max).max()
    dt = 0.1 * h_min / (p + 1) ** 2
    e0 = energy(u)
    for _ in range(4):
        u = fr.rk3_step(keys, nbr, hang, u, dt, dim, d_max, L, p)
        e1 = energy(u)
        assert e1 <= e0 * (1 + 1e-14), (e0, e1)
        e0 = e1
