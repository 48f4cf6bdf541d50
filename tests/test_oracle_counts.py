"""Element counts of the two small synthetic workloads, cross-checked against
values an independent scratch replay produced from the same definitions
(criterion of Section 5.2 with strict radii 5 / 6 on Gauss-Legendre points,
the adaptation procedure of Section 4.1 with the d_min floor and d_max
ceiling, corner 2:1 balance of Section 3.2, periodic domain).  These are not
paper values; they pin the oracle's whole cycle to a second implementation.
"""
import pytest

import oracle
from paper_2306_06744_amd import synth


@pytest.mark.parametrize("centre,n_refine,n_leaves", [((0.0, 0.0), 60, 244), ((2.0, 2.0), 41, 187)])
def test_2d_small_one_cycle(centre, n_refine, n_leaves):
    w = synth.workload_2d_small(1000)
    o = oracle.Tree(w.dim, w.d_min, w.d_max)
    f = o.flag([(centre[0], centre[1], 0.0)], w.r_in, w.r_out, synth.gl_nodes01(w.p), w.lo,
               w.length)
    assert int((f == 1).sum()) == n_refine
    assert int((f == -1).sum()) == 0  # every coarsening flag is clamped at d_min = 3
    o.adapt(f)
    o.balance()
    assert o.size() == n_leaves


@pytest.mark.slow
def test_3d_extruded_ten_cycles():
    """3D [-5,5]^3, levels 4..7, p = 3, vortex axis at (0, 0) moving +0.1 in x
    per cycle, xy distance."""
    expect = [29184, 220928, 1703360, 1722624, 1734272, 1747712, 1754880, 1765632, 1774816,
              1783552]
    w = synth.workload_3d_extruded(2000)
    w.centres = [(0.0, 0.0, 0.0)]
    o = oracle.Tree(w.dim, w.d_min, w.d_max)
    nodes = synth.gl_nodes01(w.p)
    got = []
    for cyc in range(len(expect)):
        f = o.flag(w.centres_at(cyc), w.r_in, w.r_out, nodes, w.lo, w.length,
                   dist_axes=w.dist_axes)
        o.adapt(f)
        o.balance()
        got.append(o.size())
        assert got == expect[: cyc + 1]
