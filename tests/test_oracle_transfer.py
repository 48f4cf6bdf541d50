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
