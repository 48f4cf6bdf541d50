"""GPU: ensembles whose meshes carry different degrees (3D, p 1..3) in one
tree and one solution array (lt_set_mesh_degree, lt_flag_batch with each
mesh's own solution points, lt_transfer_mixed, and the captured cycle with
p = -1).  The solution layout is u[v][i][e] with i < NPM, NPM the largest
(p+1)^3 of the ensemble; an element of a mesh of degree p owns rows
i < (p+1)^3.  Every mesh is compared with its own CPU oracle tree at its own
degree: flags, keys and mapping bit-exact, the transfer per class (copies
bit-exact, refined and fused elements within 1e-13); the captured cycle is
compared with the eager calls bit for bit on every owned row."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

from gpu_util import assert_transfer
from test_gpu_batch import to_mesh_keys

pytestmark = pytest.mark.gpu


def mesh_args(g, p):
    cen = [tuple(g.uniform(-3, 3, size=3)) for _ in range(int(g.integers(1, 3)))]
    r_in = float(g.uniform(1.2, 2.5))
    return dict(centres=cen, r_in=r_in, r_out=1.2 * r_in, nodes01=synth.gl_nodes01(p),
                lo=(-5.0,) * 3, length=10.0, dist_axes=3, periodic_dist=bool(g.integers(2)))


def moved(args, dx):
    return [dict(a, centres=[(x + dx, y, z) for x, y, z in a["centres"]]) for a in args]


def test_mixed_degree_ensemble_matches_per_mesh_oracle():
    import torch
    import paper_2306_06744_amd as lt
    g = synth.rng(4300)
    degs = [1, 2, 3, 3, 1, 2, 3]
    M = len(degs)
    d_fine = 6
    d_max = [int(x) for x in g.integers(4, d_fine + 1, size=M)]
    d_min = [1] * M
    depth = [int(g.integers(2, dm)) for dm in d_max]
    print("mixed ensemble", degs, d_max, depth, flush=True)
    t = lt.Tree.batch(3, d_fine, d_min, d_max, depth)
    t.set_mesh_degree(degs)
    O = [oracle.Tree(3, d_min[m], d_max[m], start_depth=depth[m]) for m in range(M)]
    fargs = [mesh_args(g, degs[m]) for m in range(M)]
    nvar, npm = 3, 64
    saw = {"refined": 0, "fused": 0}
    for cyc in range(4):
        fa = moved(fargs, 0.4 * cyc)
        offs_old = t.mesh_offsets()
        f = t.flag_batch(fa).cpu().numpy()
        for m in range(M):
            fo = O[m].flag(**fa[m])
            assert np.array_equal(f[offs_old[m]:offs_old[m + 1]], fo), f"flags mesh {m} cycle {cyc}"
            O[m].adapt(fo)
            O[m].balance()
        t.adapt(torch.from_numpy(f).cuda())
        t.balance()
        offs = t.mesh_offsets()
        keys = t.keys().cpu().numpy().view(np.uint64)
        u_old = synth.random_solution(90 + cyc, nvar, npm, offs_old[-1])
        u_new = t.transfer_mixed(torch.from_numpy(u_old).cuda()).cpu().numpy()
        src, kind = (a.cpu().numpy() for a in t.mapping())
        for m in range(M):
            a, b = offs[m], offs[m + 1]
            assert np.array_equal(to_mesh_keys(keys[a:b], 3, d_fine, d_max[m]), O[m].keys()), \
                f"keys mesh {m} cycle {cyc}"
            so, ko = O[m].map()
            assert np.array_equal(src[a:b] - offs_old[m], so) and np.array_equal(kind[a:b], ko), \
                f"map mesh {m} cycle {cyc}"
            n_p = (degs[m] + 1) ** 3
            mine = np.ascontiguousarray(u_old[:, :n_p, offs_old[m]:offs_old[m + 1]])
            ref = O[m].transfer(degs[m], mine)
            errs = assert_transfer(u_new[:, :n_p, a:b], ref, ko, 1e-13,
                                   f"mixed transfer mesh {m} p{degs[m]} cycle {cyc}")
            for k in saw:
                saw[k] += errs.get(k, (0, 0, 0))[2]
    assert saw["refined"] > 0 and saw["fused"] > 0, saw


def owned(u, offs, degs):
    """The rows each element owns, gathered per mesh: list of (nvar, n_p, n_m)."""
    return [u[:, :(p + 1) ** 3, offs[m]:offs[m + 1]] for m, p in enumerate(degs)]


def test_captured_mixed_cycle_matches_eager():
    import torch
    import paper_2306_06744_amd as lt
    g = synth.rng(4310)
    degs = [3, 1, 2, 3, 2]
    M = len(degs)
    d_max = [int(x) for x in g.integers(5, 8, size=M)]
    d_min, depth = [2] * M, [3] * M
    fargs = [mesh_args(g, p) for p in degs]
    E = lt.Tree.batch(3, 7, d_min, d_max, depth)
    G = lt.Tree.batch(3, 7, d_min, d_max, depth)
    for t in (E, G):
        t.set_mesh_degree(degs)
    nvar, npm, cap = 2, 64, 1_500_000
    u = [torch.zeros((nvar, npm, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    u[0][:, :, :G.size()] = torch.randn((nvar, npm, G.size()), dtype=torch.float64, device="cuda",
                                        generator=gen)
    uE = u[0][:, :, :E.size()].clone()
    cyc = lt.Cycle(G, -1, nvar, cap, u, fargs)
    for c in range(5):
        fa = moved(fargs, 0.25 * c)
        offs_old = E.mesh_offsets()
        ui = cyc.run(fa)
        E.adapt(E.flag_batch(fa))
        E.balance()
        E.connect()
        E.map()
        uE = E.transfer_mixed(uE)
        torch.cuda.synchronize()
        print("mixed captured cycle", c, offs_old[-1], "->", G.size(), cyc.stats(), flush=True)
        assert np.array_equal(G.keys().cpu().numpy(), E.keys().cpu().numpy())
        for a, b in zip(G.mapping(), E.mapping()):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        offs = E.mesh_offsets()
        for m, (x, y) in enumerate(zip(owned(u[ui], offs, degs), owned(uE, offs, degs))):
            assert bool((x == y).all()), f"mesh {m} (p{degs[m]}) cycle {c}"
    runs, eager, recap = cyc.stats()
    assert runs == 5
    del cyc


def test_mixed_degree_arguments_are_checked():
    import paper_2306_06744_amd as lt
    t = lt.Tree.batch(3, 5, [1, 1], [4, 5], [2, 2])
    with pytest.raises(lt.LtError):
        t.set_mesh_degree([1, 4])
    with pytest.raises(lt.LtError):  # no degrees set yet
        import torch
        t.adapt(torch.zeros(t.size(), dtype=torch.int8, device="cuda"))
        t.transfer_mixed(torch.zeros((1, 8, t.sizes()[1]), dtype=torch.float64, device="cuda"))
    t2 = lt.Tree.uniform(2, 1, 5)
    with pytest.raises(lt.LtError):
        t2.set_mesh_degree([2])


def test_captured_mixed_cycle_64_meshes_matches_eager():
    """The 64-mesh ensemble (p 2 and 3 mixed, finest levels 6..9) captured for
    five cycles, the fourth of which quadruples the leaves (575k -> 2.3M): a
    balance pass whose refinements grow the count across many scan tiles,
    with a capacity-sized grid, against the eager calls bit for bit."""
    import torch
    import paper_2306_06744_amd as lt
    meshes = synth.workload_ensemble(4000)
    degs = [m.p for m in meshes]

    def margs(m, cyc):
        return dict(centres=m.centres_at(cyc), r_in=m.r_in, r_out=m.r_out,
                    nodes01=synth.gl_nodes01(m.p), lo=(-5.0,) * 3, length=10.0, dist_axes=3,
                    periodic_dist=False)

    trees = []
    for _ in range(2):
        t = lt.Tree.batch(3, 9, [m.d_min for m in meshes], [m.d_max for m in meshes],
                          [m.d_min for m in meshes])
        t.set_mesh_degree(degs)
        trees.append(t)
    E, G = trees
    nvar, cap = 1, 6_000_000
    u = [torch.zeros((nvar, 64, cap), dtype=torch.float64, device="cuda") for _ in range(2)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(64)
    u[0][:, :, :G.size()] = torch.randn((nvar, 64, G.size()), dtype=torch.float64, device="cuda",
                                        generator=gen)
    uE = u[0][:, :, :E.size()].clone()
    cyc = lt.Cycle(G, -1, nvar, cap, u, [margs(m, 0) for m in meshes])
    for c in range(5):
        fa = [margs(m, c) for m in meshes]
        ui = cyc.run(fa)
        E.adapt(E.flag_batch(fa))
        E.balance()
        E.map()
        uE = E.transfer_mixed(uE)
        torch.cuda.synchronize()
        print("64-mesh captured cycle", c, G.size(), cyc.stats(), flush=True)
        assert np.array_equal(G.keys().cpu().numpy(), E.keys().cpu().numpy())
        for a, b in zip(G.mapping(), E.mapping()):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        offs = E.mesh_offsets()
        for m, (x, y) in enumerate(zip(owned(u[ui], offs, degs), owned(uE, offs, degs))):
            assert bool((x == y).all()), f"mesh {m} cycle {c}"
    assert G.size() > 2_000_000
    del cyc
