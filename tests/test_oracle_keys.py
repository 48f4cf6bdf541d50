"""Oracle pins for Morton IDs (Section 2.2, Algorithm "Morton Encoding") and
the lower-bound scenarios of Section 3.2 (equation lower_bound)."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth


def test_worked_keys_2d():
    # Hand derivation, 2D, D_max = 6 so m_b = 3 bits of depth:
    #  root: no coordinate bits, depth 0                          -> 0
    #  depth-1 octant, anchor (32, 32): integer coords (1, 1) at depth 1,
    #    bit group y^0 x^0 = 11b = 3, 2*(6-1) = 10 padding zeros -> 3072,
    #    shifted by m_b and depth 1 appended                        -> 24577
    #  its first child (depth 2, same anchor): (2, 2) at depth 2 -> groups
    #    11 00 = 12, 8 padding zeros -> 3072, << 3 | 2             -> 24578
    assert oracle.encode(2, 6, 0, (0, 0)) == 0
    assert oracle.encode(2, 6, 1, (32, 32)) == 24577
    assert oracle.encode(2, 6, 2, (32, 32)) == 24578


def test_worked_key_3d():
    # 3D, D_max = 7 (m_b = 3), depth 2, anchor (96, 32, 64) -> integer
    # coords (3, 1, 2) at depth 2.  Groups z^k y^k x^k: k=1: 1 0 1, k=0: 0 1 1
    # -> 101011b = 43; 3*(7-2) = 15 padding zeros -> 43 * 2^15 = 1409024;
    # << 3 | 2 -> 11272194.
    assert oracle.encode(3, 7, 2, (96, 32, 64)) == 11272194


@pytest.mark.parametrize("dim,dmax", [(2, 6), (2, 10), (3, 7), (3, 10), (2, 29), (3, 19)])
def test_encode_decode_roundtrip(dim, dmax):
    g = synth.rng(7 + dim * 100 + dmax)
    for _ in range(300):
        d = int(g.integers(0, dmax + 1))
        s = 1 << (dmax - d)
        a = [int(g.integers(0, 1 << d)) * s for _ in range(dim)]
        k = oracle.encode(dim, dmax, d, a)
        d2, a2 = oracle.decode(dim, dmax, k)
        assert d2 == d and list(a2) == a


def test_bad_keys_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.decode(2, 6, 7)          # depth 7 > D_max
    with pytest.raises(oracle.OracleError):
        oracle.decode(2, 6, (1 << 3) | 1)  # depth 1 with a set padding bit


def _random_tree(dim, dmin, dmax, seed, cycles=4):
    t = oracle.Tree(dim, dmin, dmax)
    for c in range(cycles):
        t.adapt(synth.random_flags(seed * 31 + c, t.size(), 0.35, 0.3))
        t.balance()
    return t


@pytest.mark.parametrize("dim,dmax", [(2, 5), (3, 4)])
def test_sorted_order_is_depth_first(dim, dmax):
    """Ascending Morton IDs list the leaves in depth-first order, ancestors
    before descendants; a first child's ID is its parent's plus one."""
    for seed in range(4):
        t = _random_tree(dim, 1, dmax, seed)
        k = t.keys()                         # pointer-tree depth-first order
        assert (np.diff(k.astype(np.int64)) > 0).all()
        for key in k[:50]:
            d, a = oracle.decode(dim, dmax, int(key))
            if d < dmax:
                assert oracle.encode(dim, dmax, d + 1, a) == int(key) + 1


def test_tiling():
    """Leaves tile the domain: volumes sum to the whole and consecutive leaves
    cover consecutive Morton ranges."""
    for dim, dmax in [(2, 6), (3, 4)]:
        t = _random_tree(dim, 2, dmax, 3)
        vol = 0
        prev_end = 0
        for key in t.keys():
            d, a = oracle.decode(dim, dmax, int(key))
            raw = int(key) >> dmax.bit_length()   # finest-resolution Morton index of the anchor
            assert raw == prev_end
            prev_end = raw + (1 << (dim * (dmax - d)))
            vol += 1 << (dim * (dmax - d))
        assert vol == 1 << (dim * dmax) and prev_end == vol


def test_lower_bound_scenarios():
    """The three lower-bound cases: the key itself, its parent on the left,
    or its first child at the lower bound (T[B] - O = 1)."""
    dim, dmax = 2, 4
    t = oracle.Tree(dim, 1, dmax)
    f = np.zeros(t.size(), dtype=np.int8)
    f[0] = 1
    t.adapt(f)                      # first depth-1 octant refined to depth 2
    T = t.keys().astype(np.uint64)
    # case 1: an existing leaf
    o = oracle.encode(dim, dmax, 1, (8, 0))
    B = np.searchsorted(T, np.uint64(o))
    assert T[B] == o
    # case 2: a depth-3 octant inside the depth-1 leaf at (8, 8)
    o = oracle.encode(dim, dmax, 3, (10, 10))
    B = np.searchsorted(T, np.uint64(o))
    d, a = oracle.decode(dim, dmax, int(T[B - 1]))
    assert d == 1 and tuple(a) == (8, 8)
    # case 3: the (now internal) depth-1 octant at the origin
    o = oracle.encode(dim, dmax, 1, (0, 0))
    B = np.searchsorted(T, np.uint64(o))
    assert int(T[B]) - o == 1
