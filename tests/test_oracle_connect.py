"""Oracle pins for face connectivity (Section 3.3, Algorithm "Build face
connectivity").  Faces are numbered f = 2*axis + side (0: -x, 1: +x, 2: -y,
3: +y, 4: -z, 5: +z); a conforming face f meets face f^1 of its neighbour.
Checked against the finest-cell brute force and by symmetry."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

import brute


def _balanced_tree(dim, dmin, dmax, seed, cycles=5, periodic=None):
    t = oracle.Tree(dim, dmin, dmax, periodic_mask=periodic)
    for c in range(cycles):
        t.adapt(synth.random_flags(seed * 13 + c, t.size(), 0.35, 0.3))
        t.balance()
    return t


@pytest.mark.parametrize("dim,dmax", [(2, 5), (3, 3), (3, 4)])
def test_connect_matches_bruteforce(dim, dmax):
    for seed in range(2):
        t = _balanced_tree(dim, 1, dmax, seed)
        nbr, hang = t.connect()
        nbr_b, hang_b = t.connect(brute=True)
        assert np.array_equal(nbr, nbr_b) and np.array_equal(hang, hang_b)
        leaves = brute.leaves_of(dim, dmax, t.keys())
        grid = brute.owner_grid(dim, dmax, leaves)
        rows = {(int(r[0]), int(r[1])): [int(x) for x in r[2:]] for r in hang}
        for e, (d, a) in enumerate(leaves):
            for f in range(2 * dim):
                owners = brute.face_neighbours(dim, dmax, leaves, e, f, grid)
                if nbr[e, f] >= 0:
                    assert owners == {int(nbr[e, f])}
                    assert leaves[nbr[e, f]][0] <= d
                else:
                    assert nbr[e, f] == -1
                    fine = rows[(e, f)]
                    assert set(fine) == owners and len(fine) == 1 << (dim - 1)
                    ax = f // 2
                    for slot, k in enumerate(fine):
                        dk, ak = leaves[k]
                        assert dk == d + 1
                        # slot = tangential child bits, lower axis first
                        h = 1 << (dmax - d - 1)
                        bits, j = 0, 0
                        for b in range(dim):
                            if b == ax:
                                continue
                            if (ak[b] - a[b]) % (1 << dmax) >= h:
                                bits |= 1 << j
                            j += 1
                        assert bits == slot


@pytest.mark.parametrize("dim,dmax", [(2, 6), (3, 4)])
def test_connect_symmetry(dim, dmax):
    t = _balanced_tree(dim, 2, dmax, 5)
    nbr, hang = t.connect()
    leaves = brute.leaves_of(dim, dmax, t.keys())
    depth = np.array([d for d, _ in leaves])
    rows = {(int(r[0]), int(r[1])): [int(x) for x in r[2:]] for r in hang}
    assert len(rows) == len(hang)
    # rows are sorted by (element, face)
    assert [tuple(r[:2]) for r in hang] == sorted(tuple(r[:2]) for r in hang)
    for e in range(len(leaves)):
        for f in range(2 * dim):
            j = nbr[e, f]
            assert j != -2  # fully periodic
            if j >= 0 and depth[j] == depth[e]:
                assert nbr[j, f ^ 1] == e
            elif j >= 0:
                assert depth[j] == depth[e] - 1
                assert nbr[j, f ^ 1] == -1 and e in rows[(int(j), f ^ 1)]
            else:
                for k in rows[(e, f)]:
                    assert nbr[k, f ^ 1] == e


def test_connect_non_periodic_boundary():
    dim, dmax = 2, 5
    t = _balanced_tree(dim, 2, dmax, 9, periodic=0)
    nbr, _ = t.connect()
    nbr_b, _ = t.connect(brute=True)
    assert np.array_equal(nbr, nbr_b)
    leaves = brute.leaves_of(dim, dmax, t.keys())
    W = 1 << dmax
    for e, (d, a) in enumerate(leaves):
        s = 1 << (dmax - d)
        for f in range(4):
            ax, side = divmod(f, 2)
            on_boundary = (a[ax] == 0) if side == 0 else (a[ax] + s == W)
            assert (nbr[e, f] == -2) == on_boundary


def test_uniform_tree_connectivity():
    """On a uniform periodic grid every face is conforming."""
    t = oracle.Tree(3, 3, 5)
    nbr, hang = t.connect()
    assert len(hang) == 0 and (nbr >= 0).all()
