"""Oracle pins for bottom-up tree construction (Section 3.1: tree
construction from scattered points and linearization; Section 5.1: a d_min
background with the points encoded at d_max).

The constructed tree is pinned to its definition -- split exactly the
octants shallower than d_min and the octants that strictly contain a point's
finest cell -- evaluated here by a brute force over every octant of tiny
domains, to a closed form for one point, and to the uniform trees it must
reduce to.  Keys in these tests come from the Morton ID definition written
out here (Section 2.2), not from the oracle."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth


def key_of(dim, d_max, depth, anchor):
    """Morton ID: the anchor's finest-unit bits interleaved with x least
    significant, shifted over the m_b depth bits, plus the depth."""
    raw = 0
    for k in range(d_max):
        for a in range(dim):
            raw |= ((anchor[a] >> k) & 1) << (dim * k + a)
    return (raw << d_max.bit_length()) | depth


def brute_leaves(dim, d_min, d_max, cells):
    """Every octant is visited from the root; it is split iff it is shallower
    than d_min or strictly contains a seed cell.  Leaves in depth-first order
    (children in index order c = sum_a b_a 2^a)."""
    seeds = {tuple(c) for c in cells}
    out = []

    def contains_seed(depth, anchor):
        s = 1 << (d_max - depth)
        return any(all(anchor[a] <= q[a] < anchor[a] + s for a in range(dim)) for q in seeds)

    def visit(depth, anchor):
        if depth < d_max and (depth < d_min or contains_seed(depth, anchor)):
            half = 1 << (d_max - depth - 1)
            for c in range(1 << dim):
                visit(depth + 1, [anchor[a] + ((c >> a) & 1) * half for a in range(dim)])
        else:
            out.append(key_of(dim, d_max, depth, anchor))
    visit(0, [0] * dim)
    return np.array(out, dtype=np.uint64)


def _points(dim, n, seed, lo=-5.0, length=10.0):
    g = np.random.default_rng(seed)
    return lo + length * g.random((n, dim))


@pytest.mark.parametrize("dim,d_min,d_max,n", [(2, 0, 4, 5), (2, 2, 5, 12), (2, 1, 5, 40),
                                               (3, 0, 3, 4), (3, 1, 3, 20), (3, 2, 4, 9)])
def test_points_tree_matches_brute_force(dim, d_min, d_max, n):
    pts = _points(dim, n, 100 * dim + n)
    cells = oracle.point_cells(dim, d_max, pts, (-5.0,) * dim, 10.0)
    t = oracle.Tree(dim, d_min, d_max, points=pts, lo=(-5.0,) * dim, length=10.0)
    assert np.array_equal(t.keys(), brute_leaves(dim, d_min, d_max, cells))


@pytest.mark.parametrize("dim,d_min,d_max", [(2, 0, 6), (2, 3, 9), (3, 2, 7), (3, 4, 10)])
def test_one_point_closed_form(dim, d_min, d_max):
    """Uniform 2^(dim d_min) leaves, plus 2^dim - 1 more per split on the path
    from depth d_min down to the point's finest cell."""
    t = oracle.Tree(dim, d_min, d_max, points=_points(dim, 1, 7), lo=(-5.0,) * dim, length=10.0)
    assert t.size() == 2 ** (dim * d_min) + (2 ** dim - 1) * (d_max - d_min)


def test_no_points_duplicates_and_full_cover():
    lo, L = (-5.0, -5.0), 10.0
    t = oracle.Tree(2, 3, 6, points=np.zeros((0, 2)), lo=lo, length=L)
    u = oracle.Tree(2, 3, 6)
    assert np.array_equal(t.keys(), u.keys())
    pts = _points(2, 30, 3)
    a = oracle.Tree(2, 1, 6, points=pts, lo=lo, length=L)
    b = oracle.Tree(2, 1, 6, points=np.concatenate([pts, pts[::-1], pts[:7]]), lo=lo, length=L)
    assert np.array_equal(a.keys(), b.keys())
    # one point at the centre of every finest cell: the uniform finest tree
    W = 1 << 4
    c = (np.array(list(itertools.product(range(W), repeat=2)), dtype=float) + 0.5) * L / W
    full = oracle.Tree(2, 1, 4, points=c[:, ::-1] + np.array(lo), lo=lo, length=L)
    assert np.array_equal(full.keys(), oracle.Tree(2, 4, 4).keys())


def test_point_cells_edges():
    """Cells by floor((x - lo) / dx): the low faces belong to their cell, a
    point just inside the top face to the last cell, points outside fail."""
    lo, L, d = (-5.0, -5.0, -5.0), 10.0, 5
    dx = L / 2 ** d
    pts = np.array([[-5.0, -5.0, -5.0], [5.0 - 1e-12, -5.0 + dx, -5.0 + 3 * dx],
                    [0.0, 0.0, 0.0]])
    got = oracle.point_cells(3, d, pts, lo, L)
    assert got.tolist() == [[0, 0, 0], [31, 1, 3], [16, 16, 16]]
    for bad in ([5.0, 0.0, 0.0], [0.0, -5.000001, 0.0], [np.nan, 0.0, 0.0]):
        with pytest.raises(oracle.OracleError):
            oracle.point_cells(3, d, np.array([bad]), lo, L)
        with pytest.raises(oracle.OracleError):
            oracle.Tree(3, 1, d, points=np.array([bad]), lo=lo, length=L)


@pytest.mark.parametrize("dim", [2, 3])
def test_surface_cloud_tiles_and_keeps_seeds(dim):
    """A sampled sphere surface: the leaves tile the domain, every point's
    finest cell is a leaf, every leaf family that could merge holds a seed
    (minimality), and balance afterwards only refines."""
    d_min, d_max = (2, 9) if dim == 2 else (2, 6)
    pts = synth.surface_points(dim, 20000 if dim == 2 else 8000, 5 + dim)
    t = oracle.Tree(dim, d_min, d_max, points=pts, lo=(-5.0,) * dim, length=10.0)
    keys = t.keys()
    mb = d_max.bit_length()
    depth = (keys & np.uint64((1 << mb) - 1)).astype(np.int64)
    assert int((np.int64(1) << (dim * (d_max - depth))).sum()) == 2 ** (dim * d_max)
    assert depth.min() >= d_min
    cells = oracle.point_cells(dim, d_max, pts, (-5.0,) * dim, 10.0)
    seed_keys = {key_of(dim, d_max, d_max, c) for c in cells.tolist()}
    kset = set(keys.tolist())
    assert seed_keys <= kset
    # minimality: a family of 2^dim sibling leaves above d_min holds a seed
    for i in np.flatnonzero((depth > d_min)):
        k = int(keys[i])
        d = int(depth[i])
        raw = k >> mb
        fam = raw >> (dim * (d_max - d + 1)) << (dim * (d_max - d + 1))
        if raw != fam:
            continue  # not the first child
        sibs = [((fam | (c << (dim * (d_max - d)))) << mb) | d for c in range(1 << dim)]
        if all(s in kset for s in sibs):
            # the parent was split for a seed, which must be one of these leaves
            assert d == d_max and any(s in seed_keys for s in sibs), k
    # balance afterwards only refines: every new leaf lies in an old leaf no deeper
    t.balance()
    new = t.keys()
    j = np.searchsorted(keys, new, side="right") - 1
    assert np.all(depth[j] <= (new & np.uint64((1 << mb) - 1)).astype(np.int64))
