"""GPU, full size of the large configuration (3D, levels 4..10, four
vortices, ~8M leaves, p = 3, 5 variables): properties that hold at any size
on the whole tree, oracle checks on sampled leaves (balance, connectivity,
mapping and FP64 transfer element by element with the oracle's dense
operators), and the split-precision transfer against the FP64 one over every
element."""
import numpy as np
import pytest

import oracle
from paper_2306_06744_amd import synth

from gpu_util import rel_l2

pytestmark = pytest.mark.gpu

NS = 3000       # sampled leaves per check


def decode_all(keys, dim, d_max):
    """Vectorised decode of Morton keys: (depth, anchor (n, dim))."""
    mb = int(d_max).bit_length()
    depth = (keys & np.uint64((1 << mb) - 1)).astype(np.int64)
    m = keys >> np.uint64(mb)
    anc = np.zeros((len(keys), dim), dtype=np.int64)
    for k in range(d_max):
        for a in range(dim):
            bit = (m >> np.uint64(dim * k + a)) & np.uint64(1)
            anc[:, a] |= bit.astype(np.int64) << k
    return depth, anc


@pytest.fixture(scope="module")
def large():
    import torch
    import paper_2306_06744_amd as lt
    w = synth.workload_3d_large(3000)
    nodes = synth.gl_nodes01(w.p)
    t = lt.Tree.uniform(3, w.d_min, w.d_max)
    for c in range(w.cycles - 1):
        f = t.flag(w.centres, w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=3)
        t.adapt(f)
        t.balance()
        print("cycle", c, t.size(), flush=True)
    old_keys = t.keys().cpu().numpy().view(np.uint64).copy()
    g = torch.Generator(device="cuda")
    g.manual_seed(3000)
    u_old = torch.randn((w.nvar, 64, len(old_keys)), dtype=torch.float64, device="cuda",
                        generator=g)
    # the last cycle moves the vortices a little so it refines and coarsens
    cen = [(c[0] + 0.05, c[1], c[2]) for c in w.centres]
    f = t.flag(cen, w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=3)
    flags = f.cpu().numpy().copy()
    t.adapt(f)
    t.balance()
    t.connect()
    t.map()
    u64 = t.transfer(3, u_old)
    u_split = t.transfer(3, u_old, precision=1)
    keys = t.keys().cpu().numpy().view(np.uint64).copy()
    print("leaves", len(old_keys), "->", len(keys), flush=True)
    return dict(w=w, t=t, old_keys=old_keys, keys=keys, u_old=u_old, u64=u64, u_split=u_split,
                cen=cen, flags=flags)


def test_flags_every_leaf(large):
    """The four-vortex criterion on every leaf of the large tree, bit-exact
    against the oracle's key-list form of it."""
    w = large["w"]
    fo = oracle.flag_keys(3, w.d_min, w.d_max, large["old_keys"], large["cen"], w.r_in, w.r_out,
                          synth.gl_nodes01(w.p), w.lo, w.length, dist_axes=3)
    f = large["flags"]
    bad = np.flatnonzero(f != fo)
    assert bad.size == 0, f"{bad.size} flags differ, first at leaf {bad[:5]}"
    assert (f == 1).any() and (f == -1).any() and (f == 0).any()


def test_size_order_tiling_and_centres(large):
    w, keys = large["w"], large["keys"]
    assert 4e6 <= len(keys) <= 16e6
    assert np.all(keys[1:] > keys[:-1])
    depth, anc = decode_all(keys, 3, w.d_max)
    assert depth.min() >= w.d_min and depth.max() <= w.d_max
    vol = (np.uint64(1) << (np.uint64(3) * (np.uint64(w.d_max) - depth.astype(np.uint64)))).sum()
    assert int(vol) == 8 ** w.d_max
    # consecutive leaves abut: anchor(i+1) = end of leaf i in Morton order
    mb = int(w.d_max).bit_length()
    m = (keys >> np.uint64(mb)).astype(np.uint64)
    span = np.uint64(1) << (np.uint64(3) * (np.uint64(w.d_max) - depth[:-1].astype(np.uint64)))
    assert np.all(m[:-1] + span == m[1:])
    # every vortex centre lies in a finest-level leaf
    dx = w.length / 2 ** w.d_max
    for c in large["cen"]:
        a = [int((c[k] - w.lo[k]) / dx) for k in range(3)]
        pk = oracle.encode(3, w.d_max, w.d_max, a)
        j = np.searchsorted(keys, np.uint64(pk), side="right") - 1
        assert depth[j] == w.d_max


def _leaf_at(keys, dim, d_max, point):
    k = oracle.encode(dim, d_max, d_max, [int(x) for x in point])
    return int(np.searchsorted(keys, np.uint64(k), side="right") - 1)


def test_sampled_balance_and_connectivity(large):
    w, keys, t = large["w"], large["keys"], large["t"]
    depth, anc = decode_all(keys, 3, w.d_max)
    W = 1 << w.d_max
    nbr = t.nbr().cpu().numpy().reshape(-1, 6)
    hang = t.hang().cpu().numpy().reshape(-1, 6)
    hang_idx = {(int(r[0]), int(r[1])): r[2:] for r in hang}
    g = np.random.default_rng(5)
    for e in g.choice(len(keys), size=NS, replace=False):
        d = depth[e]
        s = 1 << (w.d_max - d)
        # corner balance: every neighbour box of the leaf's own size, all 26 directions
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    q = [(anc[e, 0] + dx * s) % W, (anc[e, 1] + dy * s) % W, (anc[e, 2] + dz * s) % W]
                    j = _leaf_at(keys, 3, w.d_max, q)
                    assert depth[j] >= d - 1, (e, dx, dy, dz)
        # faces against the same-size box across each face
        for f in range(6):
            a, side = f >> 1, f & 1
            q = list(anc[e])
            q[a] = (q[a] + (s if side else -s)) % W
            j = _leaf_at(keys, 3, w.d_max, q)
            if depth[j] <= d:
                assert nbr[e, f] == j
            else:
                assert nbr[e, f] == -1
                row = hang_idx[(int(e), f)]
                for slot in range(4):
                    tang = [x for x in range(3) if x != a]
                    qq = list(q)
                    if side == 0:
                        qq[a] += s // 2
                    qq[tang[0]] += (slot & 1) * (s // 2)
                    qq[tang[1]] += ((slot >> 1) & 1) * (s // 2)
                    jj = _leaf_at(keys, 3, w.d_max, qq)
                    assert row[slot] == jj and depth[jj] == d + 1


def test_sampled_mapping_and_fp64_transfer(large):
    w, keys, old_keys, t = large["w"], large["keys"], large["old_keys"], large["t"]
    src, kind = (a.cpu().numpy() for a in t.mapping())
    I, P = oracle.operators(3, 3)
    g = np.random.default_rng(6)
    changed = np.flatnonzero(kind != 0)
    pick = np.concatenate([g.choice(len(keys), size=NS, replace=False),
                           g.choice(changed, size=min(NS, len(changed)), replace=False)])
    cols_new = np.unique(pick)
    u_new = large["u64"][:, :, cols_new].cpu().numpy()
    for col, e in enumerate(cols_new):
        e = int(e)
        k = int(kind[e])
        s = int(src[e])
        if k == 0:
            assert old_keys[s] == keys[e]
            exp = large["u_old"][:, :, s].cpu().numpy()
        elif k > 0:
            d_e = int(keys[e]) & ((1 << 4) - 1)
            pk = oracle.decode(3, w.d_max, int(old_keys[s]))
            ck = oracle.decode(3, w.d_max, int(keys[e]))
            assert pk[0] == d_e - 1
            up = large["u_old"][:, :, s].cpu().numpy()
            exp = up @ I[k - 1].T
        else:
            uc = large["u_old"][:, :, s:s + 8].cpu().numpy()
            exp = sum(uc[:, :, c] @ P[c].T for c in range(8))
        got = u_new[:, :, col]
        assert np.linalg.norm(got - exp) <= 1e-13 * max(1.0, np.linalg.norm(exp)), (e, k)


def test_split_transfer_error_bound(large):
    """Split precision over all ~8M elements: <= 2e-6 relative L2 against the
    FP64 transfer (itself checked against the oracle above), cell means
    <= 1e-13 relative."""
    import torch
    a, b = large["u_split"], large["u64"]
    err = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    x, wq = oracle.gauss_legendre(4)
    w3 = torch.from_numpy(np.einsum("i,j,k->ijk", wq, wq, wq).reshape(-1) / 8.0).cuda()
    ma = torch.einsum("vpe,p->ve", a, w3)
    mb = torch.einsum("vpe,p->ve", b, w3)
    merr = float((ma - mb).abs().max() / mb.abs().max())
    print("split rel L2", err, "cell-mean rel", merr, flush=True)
    assert err <= 2e-6
    assert merr <= 1e-13
