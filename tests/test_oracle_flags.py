"""Oracle pins for the refinement criterion of Section 5.2: an element is
flagged +1 when more of its solution points lie within r < R_in of the vortex
axis than beyond r > R_out, -1 when fewer, else 0; clamped at D_max / D_min."""
import numpy as np

import oracle
from paper_2306_06744_amd import synth


def test_far_vortex_coarsens_everything():
    t = oracle.Tree(2, 2, 6, start_depth=4)
    f = t.flag([(1e6, 1e6)], 5.0, 6.0, synth.gl_nodes01(2), (-5, -5), 10.0)
    assert (f == -1).all()
    t = oracle.Tree(2, 4, 6)   # at the floor nothing coarsens
    f = t.flag([(1e6, 1e6)], 5.0, 6.0, synth.gl_nodes01(2), (-5, -5), 10.0)
    assert (f == 0).all()


def test_vortex_covering_domain_refines_to_dmax():
    t = oracle.Tree(3, 2, 4)
    f = t.flag([(0, 0, 0)], 100.0, 200.0, synth.gl_nodes01(1), (-5, -5, -5), 10.0)
    assert (f == 1).all()
    t = oracle.Tree(3, 4, 4)   # at D_max nothing refines
    f = t.flag([(0, 0, 0)], 100.0, 200.0, synth.gl_nodes01(1), (-5, -5, -5), 10.0)
    assert (f == 0).all()


def test_annulus_elements_keep():
    """Elements whose points all lie in 5 <= r <= 6 have no inside and no
    outside points: flag 0."""
    # 2D, D_max = 8 on [0, 256): a depth-8 element (size 1) centred near r = 5.5
    t = oracle.Tree(2, 8, 8)
    f = t.flag([(0.0, 0.0)], 5.0, 6.0, synth.gl_nodes01(1), (0.0, 0.0), 256.0)
    keys = t.keys()
    # the element with anchor (5, 0) covers x in [5, 6): all points in the annulus
    k = oracle.encode(2, 8, 8, (5, 0))
    assert f[np.searchsorted(keys, np.uint64(k))] == 0
    k = oracle.encode(2, 8, 8, (2, 0))
    assert f[np.searchsorted(keys, np.uint64(k))] == 0  # +1 clamped at D_max
    k = oracle.encode(2, 8, 8, (9, 0))
    assert f[np.searchsorted(keys, np.uint64(k))] == 0  # -1 clamped at D_min = 8


def test_majority_rule_on_straddling_element():
    """An element straddling r = 5 with 3 of 4 points inside refines; one with
    1 of 4 inside and 3 beyond r = 6 coarsens."""
    # D_max 4 on [0, 16): element (depth 2, size 4) anchored at (4, 0), p = 1
    # points x in {4+4t}, t = (1 -+ 1/sqrt 3)/2 -> x ~ 4.845, 7.155
    t = oracle.Tree(2, 1, 4, start_depth=2)
    keys = t.keys()
    e = np.searchsorted(keys, np.uint64(oracle.encode(2, 4, 2, (4, 0))))
    nodes = synth.gl_nodes01(1)
    # centre (0, 0), R_in = 6, R_out = 7.5: points (4.845, .845): r=4.92 in,
    # (7.155, .845): r=7.20 neither, (4.845, 3.155): r=5.78 in, (7.155, 3.155): 7.82 out
    f = t.flag([(0.0, 0.0)], 6.0, 7.5, nodes, (0.0, 0.0), 16.0)
    assert f[e] == 1
    # R_in = 5, R_out = 5.5: in = 1, out = 3 -> coarsen
    f = t.flag([(0.0, 0.0)], 5.0, 5.5, nodes, (0.0, 0.0), 16.0)
    assert f[e] == -1


def test_extruded_criterion_ignores_z():
    t = oracle.Tree(3, 2, 5, start_depth=3)
    f = t.flag([(0.7, -1.1, 123.0)], 2.0, 3.0, synth.gl_nodes01(2), (-5, -5, -5), 10.0,
               dist_axes=2)
    keys = t.keys()
    by_xy = {}
    for k, fl in zip(keys, f):
        d, a = oracle.decode(3, 5, int(k))
        by_xy.setdefault((a[0], a[1]), set()).add(int(fl))
    assert all(len(v) == 1 for v in by_xy.values())


def test_second_far_vortex_changes_nothing():
    t = oracle.Tree(2, 3, 6, start_depth=4)
    args = (5.0, 6.0, synth.gl_nodes01(3), (-5, -5), 10.0)
    f1 = t.flag([(0.3, 0.1)], *args)
    f2 = t.flag([(0.3, 0.1), (1e5, -1e5)], *args)
    assert np.array_equal(f1, f2)


def test_flag_keys_matches_tree_flag():
    """The key-list form of the criterion gives every leaf of an adapted,
    unbalanced tree the same flag as the tree form, with several vortices,
    3D distances and the periodic minimum image."""
    nodes = synth.gl_nodes01(2)
    t = oracle.Tree(3, 2, 6)
    cen = [(0.4, -0.6, 1.3), (-2.0, 1.0, -1.0), (4.6, 4.4, -4.8)]
    for cyc in range(3):
        c = [(x + 0.3 * cyc, y, z) for x, y, z in cen]
        for per in (False, True):
            f = t.flag(c, 1.5, 2.0, nodes, (-5.0,) * 3, 10.0, dist_axes=3, periodic_dist=per)
            fk = oracle.flag_keys(3, 2, 6, t.keys(), c, 1.5, 2.0, nodes, (-5.0,) * 3, 10.0,
                                  dist_axes=3, periodic_dist=per)
            assert np.array_equal(f, fk)
        t.adapt(f)
    assert (f == 1).any() and (f == -1).any() and (f == 0).any()
    # shuffled keys: one flag per key, independent of order
    k = t.keys()
    perm = np.random.default_rng(0).permutation(len(k))
    fk = oracle.flag_keys(3, 2, 6, k[perm], cen, 1.5, 2.0, nodes, (-5.0,) * 3, 10.0, dist_axes=3)
    assert np.array_equal(fk, t.flag(cen, 1.5, 2.0, nodes, (-5.0,) * 3, 10.0, dist_axes=3)[perm])
