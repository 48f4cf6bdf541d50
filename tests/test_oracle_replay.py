"""Paper pin: the oracle replays the mesh histories of the paper's adaptive
runs (Section 5.2) and must reproduce every printed element count exactly.

This pins, jointly, the Gauss-Legendre solution points, the r<5 / r>6
criterion, adapt (one level, complete families only, D_min floor), corner
2:1 balance with periodic wrap, and the adapt-before-step timing."""
import multiprocessing as mp

import numpy as np
import pytest

import oracle
import replay

CPU_RUNS = [
    ("2d_w25_d6_p1", False), ("2d_w25_d6_p2", False), ("2d_w25_d6_p3", False),
    ("2d_w25_d7_p1", False), ("2d_w25_d7_p2", False), ("2d_w25_d7_p3", False),
    ("2d_w25_d8_p1", False), ("2d_w25_d8_p2", False), ("2d_w25_d8_p3", False),
    ("2d_w100_d8_p1", False), ("2d_w100_d8_p2", False), ("2d_w100_d8_p3", False),
    ("3d_slab_d6_p1", True), ("3d_slab_d6_p2", True), ("3d_slab_d6_p3", True),
    ("3d_slab_d7_p1", True), ("3d_slab_d7_p2", True), ("3d_slab_d7_p3", True),
    ("3d_slab_d8_p1", True), ("3d_slab_d8_p2", True),
]


@pytest.fixture(scope="module")
def replayed():
    oracle.build()
    # longest first so the pool stays busy
    order = sorted(CPU_RUNS, key=lambda r: ("d8" not in r[0], "w25" not in r[0]))
    ctx = mp.get_context("fork")
    with ctx.Pool(min(8, mp.cpu_count())) as pool:
        res = pool.starmap(replay.replay_oracle, order)
    return dict(res)


@pytest.mark.slow
@pytest.mark.parametrize("name,as_2d", CPU_RUNS)
def test_paper_element_count(replayed, name, as_2d):
    assert replayed[name] == replay.paper_counts()[name]


@pytest.mark.slow
def test_slab_is_extruded_plane():
    """The direct 3D slab (a cube of 16 identical level-4 layers) has, cycle by
    cycle, exactly the leaves of the 2D run extruded: 16 * sum 2^(l-4)."""
    run = replay.runs()["3d_slab_d6_p2"]
    from paper_2306_06744_amd import synth
    nodes = synth.gl_nodes01(run.p)
    t3 = oracle.Tree(3, 4, run.d_max, start_depth=4)
    t2 = oracle.Tree(2, 4, run.d_max, start_depth=4)
    mb = run.d_max.bit_length()
    for k in [0] * 4 + list(range(0, 400, 10)):
        for t, lo in ((t3, run.lo), (t2, run.lo[:2])):
            f = t.flag([run.centre(k)], 5.0, 6.0, nodes, lo, run.length, dist_axes=2,
                       periodic_dist=True)
            t.adapt(f)
            t.balance()
        depth = (t2.keys() & np.uint64((1 << mb) - 1)).astype(np.int64)
        assert t3.size() == 16 * int((2 ** (depth - 4)).sum())
