"""GPU: the transfer's launch shapes (lt_set_tuning, lt_autotune_transfer)
never change its result: every candidate shape gives the default shape's
output bit for bit, FP64 and split precision."""
import itertools

import numpy as np
import pytest

from paper_2306_06744_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mapped_tree():
    import torch
    import paper_2306_06744_amd as lt
    w = synth.workload_3d_extruded(2008)
    nodes = synth.gl_nodes01(3)
    t = lt.Tree.uniform(3, w.d_min, w.d_max)
    for c in range(3):
        t.adapt(t.flag(w.centres_at(c), w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=2))
        t.balance()
    n_old = t.size()
    g = torch.Generator(device="cuda")
    g.manual_seed(9)
    u_old = torch.randn((5, 64, n_old), dtype=torch.float64, device="cuda", generator=g)
    t.adapt(t.flag(w.centres_at(6), w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=2))
    t.balance()
    t.map()
    src, kind = t.mapping()
    assert (kind.cpu().numpy() != 0).any()
    return t, u_old


@pytest.mark.parametrize("precision", [0, 1])
def test_every_shape_gives_the_same_transfer(mapped_tree, precision):
    t, u_old = mapped_tree
    t.set_tuning(2, 2048)
    ref = t.transfer(3, u_old, precision=precision)
    for epl, grid in itertools.product((1, 2, 4), (1024, 2048, 4096, 7)):
        t.set_tuning(epl, grid)
        out = t.transfer(3, u_old, precision=precision)
        assert bool((out == ref).all()), (epl, grid)
    t.set_tuning(2, 2048)


def test_autotune_keeps_the_result(mapped_tree):
    import torch
    t, u_old = mapped_tree
    t.set_tuning(2, 2048)
    ref = t.transfer(3, u_old)
    scratch = torch.empty_like(ref)
    r = t.autotune_transfer(3, u_old, scratch)
    print("autotune", r, flush=True)
    assert r["copy_elems_per_lane"] in (1, 2, 4) and r["interp_grid"] in (1024, 2048, 4096, 16384, 65535)
    assert 0 < r["ms"] <= r["ms_default"] * 1.0001
    assert t.tuning() == {"copy_elems_per_lane": r["copy_elems_per_lane"], "interp_grid": r["interp_grid"]}
    assert bool((scratch == ref).all())
    assert bool((t.transfer(3, u_old) == ref).all())


def test_tuning_rejects_bad_values(mapped_tree):
    import paper_2306_06744_amd as lt
    t, _ = mapped_tree
    for bad in ((3, 2048), (2, 0), (0, 10)):
        with pytest.raises(lt.LtError):
            t.set_tuning(*bad)
