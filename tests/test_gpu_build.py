"""GPU: bottom-up construction from scattered points (lt_build_points,
Section 3.1 construction and linearization, Section 5.1 background at d_min
with the points encoded at d_max), then 2:1 balance, bit-exact against the
oracle's construction on the same points: random clouds over several sort
tiles with ragged tails, sampled sphere and torus surfaces up to millions of
points, and the degenerate cases (no point, one point, duplicates, every
point in one cell, points on the low faces and just inside the high ones,
d_min = d_max, d_min = 0, points outside the domain)."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

from gpu_util import np_keys

pytestmark = pytest.mark.gpu
LO, L = -5.0, 10.0


def both_from_points(pts, dim, d_min, d_max, balance=2, periodic=None):
    import torch
    import paper_2306_06744_amd as lt
    pm = (1 << dim) - 1 if periodic is None else periodic
    g = lt.Tree.from_points(torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).reshape(-1, dim),
                            dim, d_min, d_max, (LO,) * dim, L, periodic_mask=pm, balance=balance)
    o = oracle.Tree(dim, d_min, d_max, periodic_mask=pm, balance=balance,
                    points=np.asarray(pts, dtype=np.float64).reshape(-1, dim), lo=(LO,) * dim,
                    length=L)
    return g, o


def check(pts, dim, d_min, d_max, what, balance=2, periodic=None):
    print(what, len(pts), dim, d_min, d_max, flush=True)
    g, o = both_from_points(pts, dim, d_min, d_max, balance, periodic)
    kg, ko = np_keys(g), o.keys()
    assert kg.shape == ko.shape and np.array_equal(kg, ko), f"{what}: construction differs"
    g.balance()
    o.balance()
    assert np.array_equal(np_keys(g), o.keys()), f"{what}: balance differs"
    return g, o


@pytest.mark.parametrize("dim,d_min,d_max,n", [(2, 2, 8, 1), (2, 0, 7, 2049), (2, 3, 12, 20000),
                                               (3, 1, 5, 777), (3, 2, 7, 2048 * 9 + 5),
                                               (3, 4, 9, 100003)])
def test_random_clouds(dim, d_min, d_max, n):
    g = np.random.default_rng(1000 * dim + n)
    check(LO + L * g.random((n, dim)), dim, d_min, d_max, "random")


@pytest.mark.parametrize("dim,kind,n,d_min,d_max", [(2, "sphere", 50000, 3, 13),
                                                    (3, "sphere", 200000, 4, 9),
                                                    (3, "torus", 400000, 3, 9)])
def test_surface_clouds(dim, kind, n, d_min, d_max):
    check(synth.surface_points(dim, n, 77, kind), dim, d_min, d_max, kind)


def test_degenerate_inputs():
    import paper_2306_06744_amd as lt
    g = np.random.default_rng(9)
    check(np.zeros((0, 3)), 3, 2, 6, "no points")
    t, _ = check(np.zeros((0, 2)), 2, 0, 4, "no points, d_min 0")
    assert t.size() == 1
    one = LO + L * g.random((1, 3))
    check(np.repeat(one, 5000, axis=0), 3, 1, 8, "one cell many times")
    pts = LO + L * g.random((300, 2))
    check(np.concatenate([pts, pts, pts[::-1]]), 2, 2, 9, "duplicates")
    dx = L / 2 ** 7
    edge = np.array([[LO, LO, LO], [LO + L - 1e-12, LO, LO + 5 * dx], [LO + dx, LO + L - dx / 2, LO]])
    check(edge, 3, 1, 7, "faces")
    check(LO + L * g.random((4000, 3)), 3, 5, 5, "d_min = d_max")
    check(LO + L * g.random((3000, 2)), 2, 4, 10, "face balance", balance=0, periodic=0)
    for bad in ([[LO + L, 0.0]], [[0.0, LO - 1e-9]], [[np.nan, 0.0]]):
        import torch
        with pytest.raises(lt.LtError) as ei:
            lt.Tree.from_points(torch.tensor(bad, dtype=torch.float64), 2, 1, 6, (LO, LO), L)
        assert ei.value.status == 1


def test_large_torus_cycle_after_construction():
    """A million torus points at levels 4..9 (the paper's bunny runs use
    d_min 4 and d_max 9, 10), then one adaptation cycle on the balanced tree:
    construction, balance and connectivity against the oracle."""
    import torch
    pts = synth.surface_points(3, 1 << 20, 5, "torus")
    t, o = check(pts, 3, 4, 9, "large torus")
    print("leaves", t.size(), flush=True)
    f = synth.random_flags(3, o.size(), 0.05, 0.3)
    t.adapt(torch.from_numpy(f).cuda())
    o.adapt(f)
    t.balance()
    o.balance()
    assert np.array_equal(np_keys(t), o.keys())
    t.connect()
    nbr, hang = o.connect()
    assert np.array_equal(t.nbr().cpu().numpy(), nbr)
    assert np.array_equal(t.hang().cpu().numpy(), hang)
