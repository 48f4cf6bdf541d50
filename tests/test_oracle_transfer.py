"""Oracle pins for the solution transfer (Section 4.2): interpolation of the
parent polynomial (eq. parent_soln) on refinement, L2 projection
M u^P = sum_c S_c u^c on coarsening.  Pinned by closed-form Gauss-Legendre
rules, exactness on tensor polynomials of degree <= p, conservation of cell
means, and projection after interpolation being the identity."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

GL_CLOSED = {
    1: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
    2: ([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    3: ([-math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5)), -math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)),
         math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)), math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))],
        [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36,
         (18 + math.sqrt(30)) / 36, (18 - math.sqrt(30)) / 36]),
}


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gauss_legendre_closed_forms(p):
    x, w = oracle.gauss_legendre(p + 1)
    np.testing.assert_allclose(x, GL_CLOSED[p][0], rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, GL_CLOSED[p][1], rtol=0, atol=4e-16)
    # the shared solution-point table is the same rule mapped to [0, 1]
    np.testing.assert_allclose(synth.gl_nodes01(p), (x + 1) / 2, rtol=0, atol=2e-16)


def _points(dim, p, child=None):
    """Tensor solution points (x fastest) of the parent, or of child c in
    parent coordinates."""
    z = np.array(GL_CLOSED[p][0])
    pts = []
    for idx in itertools.product(range(p + 1), repeat=dim):
        i = idx[::-1]  # idx is (.., y, x) -> reverse so x is fastest
        xi = [z[i[a]] for a in range(dim)]
        if child is not None:
            xi = [(xi[a] + 2 * ((child >> a) & 1) - 1) / 2 for a in range(dim)]
        pts.append(xi)
    return np.array(pts)


def _poly(dim, p, seed):
    g = np.random.default_rng(seed)
    coef = g.standard_normal((p + 1,) * dim)

    def f(pts):
        out = np.zeros(len(pts))
        for e in itertools.product(range(p + 1), repeat=dim):
            term = coef[e] * np.ones(len(pts))
            for a in range(dim):
                term = term * pts[:, a] ** e[a]
            out += term
        return out
    return f


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_operators_exact_on_polynomials(dim, p):
    I, P = oracle.operators(dim, p)
    f = _poly(dim, p, 10 * dim + p)
    up = f(_points(dim, p))
    for c in range(1 << dim):
        np.testing.assert_allclose(I[c] @ up, f(_points(dim, p, c)), rtol=0, atol=1e-13)
    # coarsening children that hold one global polynomial returns it
    acc = sum(P[c] @ f(_points(dim, p, c)) for c in range(1 << dim))
    np.testing.assert_allclose(acc, up, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 3), (3, 2), (3, 3)])
def test_projection_after_interpolation_is_identity(dim, p):
    I, P = oracle.operators(dim, p)
    n = (p + 1) ** dim
    S = sum(P[c] @ I[c] for c in range(1 << dim))
    assert np.abs(S - np.eye(n)).max() < 1e-14


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 3)])
def test_cell_means_conserved(dim, p):
    """Coarsening preserves the integral of arbitrary (non-polynomial) child
    data; refinement preserves the parent's mean."""
    I, P = oracle.operators(dim, p)
    w1 = np.array(GL_CLOSED[p][1])
    W = np.ones(1)
    for _ in range(dim):
        W = np.kron(w1, W)
    g = np.random.default_rng(3)
    kids = g.standard_normal((1 << dim, (p + 1) ** dim))
    parent = sum(P[c] @ kids[c] for c in range(1 << dim))
    child_mean = np.mean([W @ kids[c] for c in range(1 << dim)])
    assert abs(W @ parent - child_mean) < 1e-13
    up = g.standard_normal((p + 1) ** dim)
    assert abs(np.mean([W @ (I[c] @ up) for c in range(1 << dim)]) - W @ up) < 1e-13


@pytest.mark.parametrize("dim,p,nvar", [(2, 2, 4), (3, 1, 5), (3, 3, 2)])
def test_tree_transfer_against_operators(dim, p, nvar):
    """lto_transfer applies copy / I_c / sum_c P_c per the mapping."""
    t = oracle.Tree(dim, 2, 5 if dim == 2 else 4)
    for c in range(3):
        t.adapt(synth.random_flags(40 + c, t.size(), 0.3, 0.4))
        t.balance()
    n_old = t.size()
    t.adapt(synth.random_flags(99, n_old, 0.25, 0.5))
    t.balance()
    np_ = (p + 1) ** dim
    u_old = synth.random_solution(5, nvar, np_, n_old)
    u_new = t.transfer(p, u_old)
    src, kind = t.map()
    I, P = oracle.operators(dim, p)
    assert set(kind.tolist()) >= {0, -1} and (kind > 0).any()
    for j in range(t.size()):
        for v in range(nvar):
            if kind[j] == 0:
                exp = u_old[v, :, src[j]]
            elif kind[j] > 0:
                exp = I[kind[j] - 1] @ u_old[v, :, src[j]]
            else:
                exp = sum(P[c] @ u_old[v, :, src[j] + c] for c in range(1 << dim))
            np.testing.assert_allclose(u_new[v, :, j], exp, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------
# Transfer through a whole tree, pinned by one global polynomial.
#
# Every old leaf holds the same Q_p polynomial (degree <= p per axis) sampled
# at its own physical Gauss-Legendre points.  Interpolation of the parent
# polynomial (eq. parent_soln) and L2 projection of children that hold one
# polynomial (Section 4.2) both reproduce it exactly, so after adapt, balance
# and transfer every new leaf must hold the polynomial at its own points.  The
# expectation is computed from the keys by the definition of the Morton ID
# (Section 2.2), not from the oracle's mapping: a wrong child slot, a swapped
# axis or a wrong projection term fails it.

def _decode(dim, d_max, key):
    """(depth, anchor) of a Morton ID: depth in the low m_b bits, then
    dim*(d_max - depth) zero bits, then the anchor's bits at its own depth
    interleaved with x least significant."""
    key = int(key)
    mb = d_max.bit_length()
    depth = key & ((1 << mb) - 1)
    raw = key >> (mb + dim * (d_max - depth))
    a = [0] * dim
    for k in range(depth):
        for ax in range(dim):
            a[ax] |= ((raw >> (dim * k + ax)) & 1) << k
    return depth, [x << (d_max - depth) for x in a]


def _leaf_points(dim, d_max, p, keys, lo, length):
    """Physical solution points (N, n_p, dim) of every leaf, x fastest."""
    t = (np.array(GL_CLOSED[p][0]) + 1.0) / 2.0
    dx = length / 2 ** d_max
    out = np.zeros((len(keys), (p + 1) ** dim, dim))
    for e, k in enumerate(keys):
        d, a = _decode(dim, d_max, k)
        s = 2 ** (d_max - d)
        for i, idx in enumerate(itertools.product(range(p + 1), repeat=dim)):
            ii = idx[::-1]
            for ax in range(dim):
                out[e, i, ax] = lo + dx * (a[ax] + s * t[ii[ax]])
    return out


def _global_poly(dim, p, nvar, seed, half):
    g = np.random.default_rng(seed)
    coef = g.standard_normal((nvar,) + (p + 1,) * dim)

    def f(pts):  # pts (..., dim) -> (nvar, ...)
        x = pts / half
        out = np.zeros((nvar,) + pts.shape[:-1])
        for e in itertools.product(range(p + 1), repeat=dim):
            mono = np.ones(pts.shape[:-1])
            for ax in range(dim):
                mono = mono * x[..., ax] ** e[ax]
            out += coef[(slice(None),) + e][:, None, None] * mono
        return out
    return f


@pytest.mark.parametrize("dim,p,periodic", [(2, 1, 3), (2, 2, 0), (2, 3, 3), (3, 1, 7), (3, 2, 5),
                                            (3, 3, 7), (3, 3, 0)])
def test_tree_transfer_reproduces_global_polynomial(dim, p, periodic):
    d_max = 6 if dim == 2 else 4
    lo, length = -5.0, 10.0
    t = oracle.Tree(dim, 1, d_max, periodic_mask=periodic, start_depth=2)
    for c in range(3):
        t.adapt(synth.random_flags(70 + c + 10 * dim, t.size(), 0.35, 0.3))
        t.balance()
    t.adapt(synth.random_flags(97 + p, t.size(), 0.1, 0.85))
    t.balance()
    old_keys, new_keys = t.old_keys(), t.keys()
    f = _global_poly(dim, p, 2, 1000 * dim + p, length / 2)
    # f gives (nvar, N, n_p); the solution layout is (nvar, n_p, N)
    u_old = np.ascontiguousarray(f(_leaf_points(dim, d_max, p, old_keys, lo, length))
                                 .transpose(0, 2, 1))
    u_new = t.transfer(p, u_old)
    exp = f(_leaf_points(dim, d_max, p, new_keys, lo, length)).transpose(0, 2, 1)
    src, kind = t.map()
    n_ref, n_fused = int((kind > 0).sum()), int((kind < 0).sum())
    assert n_ref > 0 and n_fused > 0 and (kind == 0).any()
    scale = np.abs(exp).max()
    for cls, sel in (("copy", kind == 0), ("refined", kind > 0), ("fused", kind < 0)):
        err = np.abs(u_new[:, :, sel] - exp[:, :, sel]).max() / scale
        assert err <= 1e-13, (cls, err)


@pytest.mark.parametrize("dim,periodic", [(2, 3), (2, 0), (3, 7), (3, 2)])
def test_map_slots_match_geometry(dim, periodic):
    """The mapping's child slot and fused range agree with the decoded
    anchors: a refined child's slot is its offset bits from the parent
    (x lowest), and a fused parent's old[src + c] is its child c."""
    d_max = 6 if dim == 2 else 4
    t = oracle.Tree(dim, 1, d_max, periodic_mask=periodic, start_depth=2)
    for c in range(3):
        t.adapt(synth.random_flags(50 + c, t.size(), 0.35, 0.35))
        t.balance()
    t.adapt(synth.random_flags(59, t.size(), 0.15, 0.8))
    t.balance()
    old_keys, new_keys = t.old_keys(), t.keys()
    src, kind = t.map()
    assert (kind > 0).any() and (kind < 0).any()
    for j, k in enumerate(new_keys):
        d, a = _decode(dim, d_max, k)
        if kind[j] == 0:
            assert old_keys[src[j]] == k
        elif kind[j] > 0:
            dp, ap = _decode(dim, d_max, old_keys[src[j]])
            half = 2 ** (d_max - d)
            assert dp == d - 1
            slot = sum(((a[ax] - ap[ax]) // half) << ax for ax in range(dim))
            assert all(0 <= a[ax] - ap[ax] <= half for ax in range(dim))
            assert kind[j] - 1 == slot
        else:
            half = 2 ** (d_max - d - 1)
            for c in range(1 << dim):
                dc, ac = _decode(dim, d_max, old_keys[src[j] + c])
                assert dc == d + 1
                assert ac == [a[ax] + ((c >> ax) & 1) * half for ax in range(dim)]
