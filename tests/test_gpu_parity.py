"""GPU parity: every step of the HIP path, called through the C ABI, against
the CPU oracle on identical seeded inputs.

Bar: keys, flags, nbr, hang and the mapping bit-exact; the FP64 transfer
with copies bit-exact and refined and fused elements each within 1e-13, both
in relative L2 over the class and in the largest error relative to the
class's largest value (the two sides differ only in summation order:
sum-factorised tensor products against dense products, about 10^2 roundings
per output, each ~1.1e-16 relative)."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

from gpu_util import (adapt_both, assert_same_connectivity, assert_same_map, assert_same_tree,
                      assert_transfer, both, np_keys, rel_l2)

pytestmark = pytest.mark.gpu
TOL = 1e-13


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    import paper_2306_06744_amd as lt
    assert torch.cuda.is_available()
    lt.lib()
    oracle.build()
    yield
    torch.cuda.synchronize()


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dim,dmax,depth", [(2, 6, 0), (2, 6, 3), (2, 10, 5), (3, 7, 0), (3, 7, 4),
                                            (3, 19, 2), (2, 29, 3)])
def test_uniform_build(dim, dmax, depth):
    say("uniform", dim, dmax, depth)
    g, o = both(dim, 0, dmax, depth=depth)
    assert_same_tree(g, o)


def test_build_from_keys_and_validation():
    import torch
    import paper_2306_06744_amd as lt
    o = oracle.Tree(2, 2, 6)
    for c in range(3):
        o.adapt(synth.random_flags(c, o.size(), 0.3, 0.3))
        o.balance()
    k = o.keys()
    say("from_keys", len(k))
    t = lt.Tree.from_keys(torch.from_numpy(k.view(np.int64)), 2, 2, 6)
    assert np.array_equal(np_keys(t), k)
    bad = k.copy()
    bad[[3, 4]] = bad[[4, 3]]           # not ascending
    with pytest.raises(lt.LtError, match="INVALID_TREE"):
        lt.Tree.from_keys(torch.from_numpy(bad.view(np.int64)), 2, 2, 6)
    with pytest.raises(lt.LtError, match="INVALID_TREE"):
        lt.Tree.from_keys(torch.from_numpy(np.delete(k, 7).view(np.int64)), 2, 2, 6)  # gap


FLAG_CASES = [
    # dim, dmin, dmax, p, centres, r_in, r_out, dist_axes, periodic_dist
    (2, 3, 6, 2, [(0.3, -0.7)], 2.0, 2.5, 2, False),
    (2, 3, 8, 3, [(4.9, 4.9)], 1.0, 1.2, 2, True),
    (2, 2, 7, 1, [(0.1, 0.2), (-3.0, 2.0), (2.5, -2.5)], 0.7, 1.1, 2, True),
    (3, 2, 5, 3, [(0.4, -0.6, 0.0)], 2.0, 2.4, 2, False),
    (3, 2, 5, 2, [(0.4, -0.6, 1.3), (-2.0, 1.0, -1.0)], 1.5, 2.0, 3, True),
    # four vortices, 3D distances, no minimum image (the large configuration's form)
    (3, 2, 5, 3, [(1.1, -0.4, 0.9), (-2.2, 1.7, -0.6), (0.3, 2.5, -2.1), (-1.0, -2.4, 1.8)],
     1.2, 1.5, 3, False),
    # degree 7 (8 points per axis) with several vortices, 2D and 3D
    (2, 2, 6, 7, [(0.3, 0.2), (-2.0, 1.5)], 1.5, 2.0, 2, False),
    (3, 2, 4, 7, [(0.5, 0.5, 0.5), (-1.5, 0.7, -0.4)], 1.8, 2.2, 3, True),
]


@pytest.mark.parametrize("case", range(len(FLAG_CASES)))
def test_flag_adapt_balance_cycles(case):
    """Several full geometric cycles: flags, adapt, balance bit-exact."""
    import torch
    dim, dmin, dmax, p, centres, rin, rout, da, per = FLAG_CASES[case]
    say("flag case", case)
    g, o = both(dim, dmin, dmax)
    lo, L = (-5.0,) * dim, 10.0
    nodes = synth.gl_nodes01(p)
    for cyc in range(dmax - dmin + 2):
        cen = [tuple(c[a] + 0.37 * cyc * (a == 0) for a in range(len(c))) for c in centres]
        f = g.flag(cen, rin, rout, nodes, lo, L, dist_axes=da, periodic_dist=per)
        fo = o.flag(cen, rin, rout, nodes, lo, L, dist_axes=da, periodic_dist=per)
        assert np.array_equal(f.cpu().numpy(), fo), f"flags differ at cycle {cyc}"
        g.adapt(f)
        o.adapt(fo)
        assert_same_tree(g, o, f"adapt {cyc}")
        g.balance()
        o.balance()
        assert_same_tree(g, o, f"balance {cyc}")
    torch.cuda.synchronize()


@pytest.mark.parametrize("dim,dmax,kind,periodic", [(2, 6, 2, 3), (2, 6, 0, 3), (2, 6, 1, 0),
                                                    (3, 4, 2, 7), (3, 4, 0, 7), (3, 4, 1, 5),
                                                    (3, 5, 2, 0)])
def test_random_unbalanced_then_balance(dim, dmax, kind, periodic):
    """Adapt with random flags and no balance (violations pile up), then balance."""
    say("unbalanced", dim, dmax, kind, periodic)
    g, o = both(dim, 1, dmax, periodic_mask=periodic, balance=kind)
    for c in range(dmax):
        adapt_both(g, o, synth.random_flags(1000 * dim + 10 * c + kind, o.size(), 0.35, 0.25))
        assert_same_tree(g, o, f"adapt {c}")
    g.balance()
    o.balance()
    assert_same_tree(g, o, "balance")
    assert o.is_balanced() or o.size() > 3000
    g.balance()  # idempotent
    assert_same_tree(g, o, "balance twice")


@pytest.mark.parametrize("dim,dmax,periodic", [(2, 7, 3), (2, 7, 0), (2, 7, 2), (3, 5, 7), (3, 5, 0),
                                               (3, 5, 6)])
def test_cycle_connect_map_transfer(dim, dmax, periodic):
    """Random balanced cycles: connectivity, mapping bit-exact, transfer <= 1e-13."""
    import torch
    say("cycle", dim, dmax, periodic)
    g, o = both(dim, 2, dmax, periodic_mask=periodic)
    for c in range(4):
        adapt_both(g, o, synth.random_flags(77 + c + 10 * dim, o.size(), 0.3, 0.45))
        g.balance()
        o.balance()
        assert_same_tree(g, o, f"cycle {c}")
        assert_same_connectivity(g, o, f"cycle {c}")
        assert_same_map(g, o, f"cycle {c}")
        for p in (1, 2, 3):
            nvar = 4 if dim == 2 else 5
            n_old = o.old_size()
            u_old = synth.random_solution(5 + c + p, nvar, (p + 1) ** dim, n_old)
            ug = g.transfer(p, torch.from_numpy(u_old).cuda()).cpu().numpy()
            uo = o.transfer(p, u_old)
            assert_transfer(ug, uo, o.map()[1], TOL, f"cycle {c} p{p}")


@pytest.mark.parametrize("dim,dmax", [(2, 8), (3, 6)])
def test_connect_on_side_stream_beside_transfer(dim, dmax):
    """lt_connect on a second stream while lt_transfer runs on the first (the
    two use separate scratch): connectivity, mapping bit-exact and the
    transfer within the bar, cycle after cycle, each cycle with another cap
    on the face search's grid (the search strides over its lanes)."""
    import torch
    import paper_2306_06744_amd as lt
    say("side stream", dim, dmax)
    g, o = both(dim, 2, dmax)
    with pytest.raises(lt.LtError) as ei:
        g.set_connect_grid(-1)
    assert ei.value.status == 1
    side = torch.cuda.Stream()
    p = 3 if dim == 3 else 2
    nvar = 5 if dim == 3 else 4
    for c in range(4):
        adapt_both(g, o, synth.random_flags(300 + c + 10 * dim, o.size(), 0.35, 0.4))
        g.balance()
        o.balance()
        assert_same_tree(g, o, f"cycle {c}")
        g.map()
        u_old = synth.random_solution(400 + c, nvar, (p + 1) ** dim, o.old_size())
        ug = g.transfer(p, torch.from_numpy(u_old).cuda())
        g.set_connect_grid((0, 256, 7, 1)[c])
        with torch.cuda.stream(side):  # no wait on the first stream: the two overlap
            g.connect()
        torch.cuda.synchronize()
        nbr_o, hang_o = o.connect()
        assert np.array_equal(g.nbr().cpu().numpy(), nbr_o), f"cycle {c}: nbr differs"
        assert np.array_equal(g.hang().cpu().numpy(), hang_o), f"cycle {c}: hang differs"
        src, kind = g.mapping()
        src_o, kind_o = o.map()
        assert np.array_equal(src.cpu().numpy(), src_o) and np.array_equal(kind.cpu().numpy(), kind_o)
        assert_transfer(ug.cpu().numpy(), o.transfer(p, u_old), kind_o, TOL, f"cycle {c}")


@pytest.mark.parametrize("p_refine,p_coarsen", [(0.9, 0.0), (0.0, 0.95), (0.3, 0.4)])
def test_transfer_joins_caller_stream(p_refine, p_coarsen):
    """The 3D transfer forks its interpolation passes onto a second stream of
    the tree and joins it back: work enqueued after it on the caller's stream
    (a copy of the result on a non-default stream, with only that stream
    synchronised) sees every interpolated and projected element.  Mostly
    refined or mostly fused mappings make the interpolation passes outlast
    the copy pass, so a missing join would leave elements unwritten."""
    import torch
    say("joined stream", p_refine, p_coarsen)
    g, o = both(3, 2, 7, depth=4)
    adapt_both(g, o, synth.random_flags(511, o.size(), p_refine, p_coarsen))
    g.balance()
    o.balance()
    assert_same_tree(g, o)
    g.map()
    u_old = synth.random_solution(512, 5, 64, o.old_size())
    ud = torch.from_numpy(u_old).cuda()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ug = g.transfer(3, ud)
        host = ug.clone().to("cpu")
    s.synchronize()
    kind = o.map()[1]
    say("refined", int((kind > 0).sum()), "fused", int((kind < 0).sum()), "of", kind.size)
    assert_transfer(host.numpy(), o.transfer(3, u_old), kind, TOL, "joined")


def test_refinement_fallback_for_wide_rows_matches_buffer_form():
    """The 3D refinement pass addresses a wave's rows through a buffer
    resource with 32-bit row offsets; leading dimensions from 2^32 / (8 N^2)
    elements (33.5M at p = 3) take the kernel's earlier form instead.  Both
    must write the same bits: the same mapping transferred once with a tight
    leading dimension and once with 2^25 + 64 (two 17 GB arrays, one
    variable)."""
    import torch
    say("wide rows")
    g, o = both(3, 2, 7, depth=4)
    n_old = g.size()
    adapt_both(g, o, synth.random_flags(611, o.size(), 0.4, 0.3))
    g.balance()
    g.map()
    n = g.size()
    ud = torch.from_numpy(synth.random_solution(612, 1, 64, n_old)).cuda()
    ua = g.transfer(3, ud)
    ld = (1 << 25) + 64
    big = torch.zeros((1, 64, ld), dtype=torch.float64, device="cuda")
    big[:, :, :n_old] = ud
    ub = torch.zeros((1, 64, ld), dtype=torch.float64, device="cuda")
    g.transfer(3, big, u_new=ub)
    torch.cuda.synchronize()
    kind = g.mapping()[1].cpu().numpy()
    say("refined", int((kind > 0).sum()), "fused", int((kind < 0).sum()), "of", n)
    same = bool(torch.equal(ua, ub[:, :, :n]))
    del big, ub
    torch.cuda.empty_cache()
    assert (kind > 0).any() and same


def test_transfer_with_padding_and_high_degree_2d():
    import torch
    say("padding")
    g, o = both(2, 2, 6)
    adapt_both(g, o, synth.random_flags(3, o.size(), 0.3, 0.0))
    g.balance(); o.balance()
    adapt_both(g, o, synth.random_flags(4, o.size(), 0.2, 0.6))
    g.balance(); o.balance()
    for p in (4, 7):
        n_old = o.old_size()
        u = synth.random_solution(9, 3, (p + 1) ** 2, n_old)
        upad = np.zeros((3, (p + 1) ** 2, n_old + 37))
        upad[:, :, :n_old] = u
        out = torch.full((3, (p + 1) ** 2, g.size() + 11), 7.0, dtype=torch.float64, device="cuda")
        g.transfer(p, torch.from_numpy(upad).cuda(), u_new=out)
        res = out.cpu().numpy()
        assert (res[:, :, g.size():] == 7.0).all()
        assert_transfer(res[:, :, :g.size()], o.transfer(p, u), o.map()[1], TOL, f"padded p{p}")


def test_single_leaf_tree():
    """Degenerate tree: the root alone (its own periodic neighbour)."""
    import torch
    say("single leaf")
    for periodic in (3, 0):
        g, o = both(2, 0, 4, depth=0, periodic_mask=periodic)
        assert g.size() == 1
        assert_same_connectivity(g, o, "root")
        adapt_both(g, o, np.array([1], dtype=np.int8))
        g.balance(); o.balance()
        assert_same_tree(g, o, "refined root")
        assert_same_connectivity(g, o, "refined root")
        u = synth.random_solution(1, 2, 9, 1)
        assert_transfer(g.transfer(2, torch.from_numpy(u).cuda()).cpu().numpy(), o.transfer(2, u),
                        o.map()[1], TOL, "refined root")
        adapt_both(g, o, np.full(4, -1, dtype=np.int8))
        assert_same_tree(g, o, "coarsened to root")
        assert g.size() == 1
        assert_same_map(g, o, "fused root")


def test_deep_ripple_at_key_limits():
    """Refine one corner to the finest depth at the 64-bit key limit; the
    balance ripple crosses every level."""
    for dim, dmax in [(3, 19), (2, 29)]:
        say("deep", dim, dmax)
        g, o = both(dim, 0, dmax, depth=1)
        for c in range(dmax - 1):
            f = np.zeros(o.size(), dtype=np.int8)
            f[o.size() - 1] = 1          # always the last (highest-key) leaf
            adapt_both(g, o, f)
            assert_same_tree(g, o, f"deep adapt {c}")
        g.balance()
        o.balance()
        assert_same_tree(g, o, "deep balance")
        assert_same_connectivity(g, o, "deep")


def test_bad_flags_rejected_and_tree_kept():
    import torch
    import paper_2306_06744_amd as lt
    say("bad flags")
    g, o = both(2, 1, 5, depth=3)
    before = np_keys(g).copy()
    f = np.zeros(g.size(), dtype=np.int8)
    f[5] = 3
    with pytest.raises(lt.LtError, match="ARG"):
        g.adapt(torch.from_numpy(f).cuda())
    assert np.array_equal(np_keys(g), before)
    with pytest.raises(lt.LtError, match="STATE"):
        g.map()


def test_deterministic_rerun():
    import torch
    say("determinism")
    res = []
    for _ in range(2):
        g, _o = both(3, 2, 6)
        for c in range(4):
            f = torch.from_numpy(synth.random_flags(50 + c, g.size(), 0.4, 0.3)).cuda()
            g.adapt(f)
            g.balance()
        g.connect()
        res.append((np_keys(g).copy(), g.nbr().cpu().numpy(), g.hang().cpu().numpy()))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
