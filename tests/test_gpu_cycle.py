"""GPU: the cycle captured in a hipGraph (lt_cycle_*) against the eager calls.

Each test replays the graph over several cycles, with the eager reference
cycle (its own launches and synchronisations) run between the replays, and
compares every replay: keys, nbr, hang and mapping bit-exact, the FP64
transfer bit-exact (same kernels, same inputs)."""
import numpy as np
import pytest

from paper_2306_06744_amd import synth

pytestmark = pytest.mark.gpu


def flag_args(w, c, nodes):
    return dict(centres=w.centres_at(c), r_in=w.r_in, r_out=w.r_out, nodes01=nodes, lo=w.lo,
                length=w.length, dist_axes=w.dist_axes, periodic_dist=w.periodic_dist)


def eager_cycle(t, fa, p, u_old):
    t.adapt(t.flag(**fa))
    t.balance()
    t.connect()
    t.map()
    return t.transfer(p, u_old)


def compare(G, E, uG, uE, n):
    assert np.array_equal(G.keys().cpu().numpy(), E.keys().cpu().numpy())
    assert np.array_equal(G.nbr().cpu().numpy(), E.nbr().cpu().numpy())
    assert np.array_equal(G.hang().cpu().numpy(), E.hang().cpu().numpy())
    for a, b in zip(G.mapping(), E.mapping()):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert bool((uG[:, :, :n] == uE).all())


@pytest.mark.parametrize("case,passes", [("3d", 4), ("3d", 2), ("2d", 4)])
def test_captured_cycle_matches_eager(case, passes):
    import torch
    import paper_2306_06744_amd as lt
    if case == "3d":
        w = synth.workload_3d_extruded(2005)
        warm, cycles = 2, 6
    else:
        w = synth.workload_2d_small(1005)
        w.advect = (0.3, 0.2, 0.0)
        warm, cycles = 1, 6
    nodes = synth.gl_nodes01(w.p)
    npts = (w.p + 1) ** w.dim
    E = lt.Tree.uniform(w.dim, w.d_min, w.d_max)
    G = lt.Tree.uniform(w.dim, w.d_min, w.d_max)
    if passes == 2:
        G.set_connect_grid(256)  # the captured face search with a capped grid
    for c in range(warm):
        for t in (E, G):
            t.adapt(t.flag(**flag_args(w, c, nodes)))
            t.balance()
    cap = 4_000_000 if case == "3d" else 20000     # the 3D cycles reach ~1.7M leaves
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    u = [torch.zeros((w.nvar, npts, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    u[0][:, :, :G.size()] = torch.randn((w.nvar, npts, G.size()), dtype=torch.float64, device="cuda",
                                        generator=g)
    uE = u[0][:, :, :E.size()].clone()
    cyc = lt.Cycle(G, w.p, w.nvar, cap, u, flag_args(w, warm, nodes), balance_passes=passes)
    for c in range(warm, warm + cycles):
        fa = flag_args(w, c, nodes)
        ui = cyc.run(fa)
        uE = eager_cycle(E, fa, w.p, uE)
        torch.cuda.synchronize()
        print(case, passes, "cycle", c, G.size(), cyc.stats(), flush=True)
        compare(G, E, u[ui], uE, E.size())
    runs, eager, recap = cyc.stats()
    assert runs == cycles
    if passes == 4 and case == "3d":
        assert eager == 0
    del cyc


def test_captured_cycle_capacity_error_leaves_tree_unchanged():
    import torch
    import paper_2306_06744_amd as lt
    w = synth.workload_3d_extruded(2006)
    nodes = synth.gl_nodes01(w.p)
    G = lt.Tree.uniform(3, w.d_min, w.d_max)
    n0 = G.size()
    keys0 = G.keys().cpu().numpy().copy()
    cap = n0 + 100          # the first cycle refines far beyond this
    u = [torch.zeros((w.nvar, 64, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    cyc = lt.Cycle(G, w.p, w.nvar, cap, u, flag_args(w, 0, nodes))
    with pytest.raises(lt.LtError) as ei:
        cyc.run(flag_args(w, 0, nodes))
    assert ei.value.status == 9
    assert G.size() == n0
    assert np.array_equal(G.keys().cpu().numpy(), keys0)
    del cyc


def test_captured_cycle_balance_overflow_leaves_tree_unchanged():
    # capacity above adapt's output but below the balanced tree: the overflow
    # comes from a balance refinement pass, whose list appends and partial
    # output must stay within the reserved buffers; the tree stays usable
    import torch
    import paper_2306_06744_amd as lt
    w = synth.workload_3d_extruded(2007)
    nodes = synth.gl_nodes01(w.p)
    E = lt.Tree.uniform(3, w.d_min, w.d_max)
    G = lt.Tree.uniform(3, w.d_min, w.d_max)
    for t in (E, G):
        t.adapt(t.flag(**flag_args(w, 0, nodes)))
        t.balance()
    n0 = G.size()
    keys0 = G.keys().cpu().numpy().copy()
    fa = flag_args(w, 1, nodes)
    E.adapt(E.flag(**fa))
    n_adapt = E.size()
    E.balance()
    n_bal = E.size()
    assert n_bal > n_adapt > n0, (n0, n_adapt, n_bal)
    cap = (n_adapt + n_bal) // 2
    print("balance overflow case: n0", n0, "adapt", n_adapt, "balanced", n_bal, "cap", cap, flush=True)
    u = [torch.zeros((w.nvar, 64, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    cyc = lt.Cycle(G, w.p, w.nvar, cap, u, fa)
    with pytest.raises(lt.LtError) as ei:
        cyc.run(fa)
    assert ei.value.status == 9
    del cyc
    assert G.size() == n0
    assert np.array_equal(G.keys().cpu().numpy(), keys0)
    G.adapt(G.flag(**fa))
    G.balance()
    assert np.array_equal(G.keys().cpu().numpy(), E.keys().cpu().numpy())


def test_captured_ensemble_cycle_matches_eager():
    import torch
    import paper_2306_06744_amd as lt
    g = synth.rng(4100)
    M = 5
    d_max = [int(x) for x in g.integers(5, 8, size=M)]
    d_min = [2] * M
    depth = [3] * M
    fargs = []
    for m in range(M):
        cen = [tuple(g.uniform(-3, 3, size=3)) for _ in range(int(g.integers(1, 3)))]
        r = float(g.uniform(1.0, 2.0))
        fargs.append(dict(centres=cen, r_in=r, r_out=1.2 * r, nodes01=synth.gl_nodes01(2),
                          lo=(-5.0,) * 3, length=10.0, dist_axes=3, periodic_dist=False))
    E = lt.Tree.batch(3, 7, d_min, d_max, depth)
    G = lt.Tree.batch(3, 7, d_min, d_max, depth)
    cap = 2_000_000
    u = [torch.zeros((3, 27, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(8)
    u[0][:, :, :G.size()] = torch.randn((3, 27, G.size()), dtype=torch.float64, device="cuda",
                                        generator=gen)
    uE = u[0][:, :, :E.size()].clone()
    cyc = lt.Cycle(G, 2, 3, cap, u, fargs)
    for c in range(5):
        fa = [dict(a, centres=[(x + 0.2 * c, y, z) for x, y, z in a["centres"]]) for a in fargs]
        ui = cyc.run(fa)
        E.adapt(E.flag_batch(fa))
        E.balance()
        E.connect()
        E.map()
        uE = E.transfer(2, uE)
        torch.cuda.synchronize()
        print("ensemble cycle", c, G.size(), cyc.stats(), flush=True)
        compare(G, E, u[ui], uE, E.size())
    del cyc


def test_captured_cycle_finishes_long_ripples_eagerly():
    """Four vortices refined to level 8 over a level-4 background leave a
    five-level staircase around each; moving the vortices ripples the 2:1
    splits down the staircase over several passes.  With two captured passes
    the run finishes such cycles eagerly, with the same result."""
    import torch
    import paper_2306_06744_amd as lt
    w = synth.workload_3d_large(3001)
    w.d_max = 8
    w.p = 2
    nodes = synth.gl_nodes01(w.p)
    E = lt.Tree.uniform(3, w.d_min, w.d_max)
    G = lt.Tree.uniform(3, w.d_min, w.d_max)

    def fa(c):
        return dict(centres=[(x + 0.06 * c, y - 0.04 * c, z) for x, y, z in w.centres], r_in=w.r_in,
                    r_out=w.r_out, nodes01=nodes, lo=w.lo, length=w.length, dist_axes=3)

    for c in range(5):
        for t in (E, G):
            t.adapt(t.flag(**fa(0)))
            t.balance()
    cap = 8 * G.size()
    u = [torch.zeros((2, 27, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    u[0][:, :, :G.size()] = torch.randn((2, 27, G.size()), dtype=torch.float64, device="cuda")
    uE = u[0][:, :, :E.size()].clone()
    cyc = lt.Cycle(G, 2, 2, cap, u, fa(1), balance_passes=2)
    for c in range(1, 7):
        ui = cyc.run(fa(c))
        uE = eager_cycle(E, fa(c), 2, uE)
        torch.cuda.synchronize()
        print("ripple cycle", c, G.size(), cyc.stats(), flush=True)
        compare(G, E, u[ui], uE, E.size())
    runs, eager, recap = cyc.stats()
    assert eager >= 1
    del cyc


def test_captured_chosen_cycle_matches_eager():
    """Learned flags (network over the geometric fallback) and the split
    transfer, captured, against the same calls made eagerly."""
    import torch
    import paper_2306_06744_amd as lt
    w = synth.workload_3d_extruded(2007)
    nodes = synth.gl_nodes01(3)
    m = lt.MLP(synth.mlp_init(21))
    E = lt.Tree.uniform(3, w.d_min, w.d_max)
    G = lt.Tree.uniform(3, w.d_min, w.d_max)
    for c in range(2):
        for t in (E, G):
            t.adapt(t.flag(**flag_args(w, c, nodes)))
            t.balance()
    cap = 4_000_000
    u = [torch.zeros((5, 64, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    cyc = lt.Cycle(G, 3, 5, cap, u, flag_args(w, 2, nodes), balance_passes=2, precision=1, mlp=m)
    cur = 0
    for c in range(2, 6):
        fa = flag_args(w, c, nodes)
        cen = w.centres_at(c)
        G.vortex_field(cen, w.strengths, nodes, w.lo, w.length, out=u[cur])
        uE = E.vortex_field(cen, w.strengths, nodes, w.lo, w.length)
        assert bool((u[cur][:, :, :E.size()] == uE).all())
        cur = cyc.run(fa)
        f, _ = E.flag_mlp(m, uE, cen, w.r_in, w.r_out, nodes, w.lo, w.length, conf_min=0.9,
                          dist_axes=w.dist_axes)
        E.adapt(f)
        E.balance()
        E.connect()
        E.map()
        uE = E.transfer(3, uE, precision=1)
        torch.cuda.synchronize()
        print("chosen cycle", c, G.size(), cyc.stats(), flush=True)
        compare(G, E, u[cur], uE, E.size())
    del cyc
