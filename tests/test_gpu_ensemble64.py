"""GPU: the 64-mesh ensemble at the benchmark's parameters (3D [-5,5]^3,
1-4 vortices per mesh with 3D distance, finest level U{6..9}, p U{2,3},
uniform start at level 3, nine cycles advected +0.1 in x, ~9.7M leaves in
all), run as the benchmark runs it: one ensemble tree per degree, every phase
one launch for all of its meshes.  Every mesh's flags, keys, connectivity and
mapping of the last cycle are compared bit for bit with SHA-256 hashes of its
own oracle tree (tests/golden/workload_ensemble_64.json, written by
make_workload_golden.py from the oracle only, keys at the mesh's own finest
level and indices local to the mesh), and the leaf count of every cycle.
The last cycle's FP64 transfer is checked on every refined and fused element
and a seeded 1% of the copies against the oracle's dense operators, per class
(the fused class at full size lives here: ~30k fused parents)."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2306_06744_amd import synth

from gpu_util import assert_transfer, changed_and_sampled, dense_expected

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
D_FINE = 9


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def mesh_keys(keys, dim, d_fine, d_max_m):
    """Ensemble keys (shared finest level; mesh bits above the Morton bits)
    re-encoded at the mesh's own finest level: the interleaved anchor bits
    shift down by dim * (d_fine - d_max_m), the depth stays."""
    mb_f, mb_m = d_fine.bit_length(), d_max_m.bit_length()
    k = keys & np.uint64((1 << (mb_f + dim * d_fine)) - 1)
    depth = k & np.uint64((1 << mb_f) - 1)
    raw = (k >> np.uint64(mb_f)) >> np.uint64(dim * (d_fine - d_max_m))
    return (raw << np.uint64(mb_m)) | depth


def test_ensemble_64_bit_exact_per_mesh():
    import torch
    import paper_2306_06744_amd as lt
    with open(os.path.join(HERE, "golden", "workload_ensemble_64.json")) as fh:
        gold = json.load(fh)
    meshes = synth.workload_ensemble(4000)
    cycles = gold["cycles"]

    def margs(m, cyc):
        return dict(centres=m.centres_at(cyc), r_in=m.r_in, r_out=m.r_out,
                    nodes01=synth.gl_nodes01(m.p), lo=(-5.0,) * 3, length=10.0, dist_axes=3,
                    periodic_dist=False)

    checked = 0
    for p in (2, 3):
        ids = [i for i, m in enumerate(meshes) if m.p == p]
        grp = [meshes[i] for i in ids]
        print(f"p{p}: {len(ids)} meshes", flush=True)
        t = lt.Tree.batch(3, D_FINE, [m.d_min for m in grp], [m.d_max for m in grp],
                          [m.d_min for m in grp])
        counts = []
        for cyc in range(cycles):
            offs_old = t.mesh_offsets()
            f = t.flag_batch([margs(m, cyc) for m in grp])
            t.adapt(f)
            t.balance()
            counts.append(t.mesh_offsets())
        flags = f.cpu().numpy()
        t.connect()
        t.map()
        src_all, kind_all = (a.cpu().numpy() for a in t.mapping())
        gen = torch.Generator(device="cuda")
        gen.manual_seed(4000 + p)
        n_old = offs_old[-1]
        u_old = torch.randn((5, (p + 1) ** 3, n_old), dtype=torch.float64, device="cuda", generator=gen)
        u_new = t.transfer(p, u_old)
        js = changed_and_sampled(kind_all, np.random.default_rng(p))
        k_js, s_js = kind_all[js].astype(np.int64), src_all[js].astype(np.int64)
        cols = np.unique(np.concatenate([s_js[k_js >= 0]] + [s_js[k_js < 0] + c for c in range(8)]))
        sub = u_old.index_select(2, torch.from_numpy(cols).cuda()).cpu().numpy()
        src_sub = np.zeros(len(src_all), dtype=np.int64)
        src_sub[js] = np.searchsorted(cols, s_js)
        exp = dense_expected(3, p, sub, src_sub, kind_all, js)
        got = u_new.index_select(2, torch.from_numpy(js).cuda()).cpu().numpy()
        errs = assert_transfer(got, exp, kind_all[js], 1e-13, f"ensemble p{p} FP64")
        assert "fused" in errs or p == 2
        del u_old, u_new
        offs = t.mesh_offsets()
        keys = t.keys().cpu().numpy().view(np.uint64)
        nbr = t.nbr().cpu().numpy()
        hang = t.hang().cpu().numpy()
        src, kind = (a.cpu().numpy() for a in t.mapping())
        print(f"p{p}: {offs[-1]} leaves, {len(hang)} hanging rows", flush=True)
        row_mesh = np.searchsorted(np.array(offs), hang[:, 0], side="right") - 1
        for j, i in enumerate(ids):
            g = gold["meshes"][i]
            m = meshes[i]
            assert g["mesh"] == i and g["p"] == p and g["d_max"] == m.d_max
            assert [c[j + 1] - c[j] for c in counts] == g["counts"], f"mesh {i}: leaf counts"
            a, b = offs[j], offs[j + 1]
            assert sha(flags[offs_old[j]:offs_old[j + 1]]) == g["flags"], f"mesh {i}: flags"
            assert sha(mesh_keys(keys[a:b], 3, D_FINE, m.d_max)) == g["keys"], f"mesh {i}: keys"
            loc = nbr[a:b].copy()
            loc[loc >= 0] -= a
            assert sha(loc) == g["nbr"], f"mesh {i}: nbr"
            h = hang[row_mesh == j].copy()
            h[:, 0] -= a
            h[:, 2:] -= a
            assert len(h) == g["n_hang"] and sha(h) == g["hang"], f"mesh {i}: hang"
            assert sha(src[a:b] - np.int32(offs_old[j])) == g["map_src"], f"mesh {i}: map_src"
            assert sha(kind[a:b]) == g["map_kind"], f"mesh {i}: map_kind"
            checked += 1
        del t
        torch.cuda.empty_cache()
    assert checked == len(meshes)


def test_ensemble_64_one_tree_mixed_degrees():
    """All 64 meshes in one tree with per-mesh degrees (lt_set_mesh_degree,
    one solution array of 64 rows per variable), as the benchmark's one-tree
    runs: the same per-mesh hashes, and the last cycle's lt_transfer_mixed on
    every refined and fused element and a seeded 1% of the copies against the
    oracle's dense operators at each mesh's own degree."""
    import torch
    import paper_2306_06744_amd as lt
    with open(os.path.join(HERE, "golden", "workload_ensemble_64.json")) as fh:
        gold = json.load(fh)
    meshes = synth.workload_ensemble(4000)
    degs = [m.p for m in meshes]

    def margs(m, cyc):
        return dict(centres=m.centres_at(cyc), r_in=m.r_in, r_out=m.r_out,
                    nodes01=synth.gl_nodes01(m.p), lo=(-5.0,) * 3, length=10.0, dist_axes=3,
                    periodic_dist=False)

    t = lt.Tree.batch(3, D_FINE, [m.d_min for m in meshes], [m.d_max for m in meshes],
                      [m.d_min for m in meshes])
    t.set_mesh_degree(degs)
    for cyc in range(gold["cycles"]):
        offs_old = t.mesh_offsets()
        f = t.flag_batch([margs(m, cyc) for m in meshes])
        t.adapt(f)
        t.balance()
    flags = f.cpu().numpy()
    t.map()
    src_all, kind_all = (a.cpu().numpy() for a in t.mapping())
    offs = t.mesh_offsets()
    print(f"one tree: {offs[-1]} leaves", flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4064)
    u_old = torch.randn((5, 64, offs_old[-1]), dtype=torch.float64, device="cuda", generator=gen)
    u_new = t.transfer_mixed(u_old)
    js_all = changed_and_sampled(kind_all, np.random.default_rng(64))
    mesh_of = np.searchsorted(np.array(offs), js_all, side="right") - 1
    deg_of = np.array(degs)[mesh_of]
    for p in (2, 3):
        n_p = (p + 1) ** 3
        js = js_all[deg_of == p]
        k_js, s_js = kind_all[js].astype(np.int64), src_all[js].astype(np.int64)
        cols = np.unique(np.concatenate([s_js[k_js >= 0]] + [s_js[k_js < 0] + c for c in range(8)]))
        sub = u_old[:, :n_p].index_select(2, torch.from_numpy(cols).cuda()).cpu().numpy()
        src_sub = np.zeros(len(src_all), dtype=np.int64)
        src_sub[js] = np.searchsorted(cols, s_js)
        exp = dense_expected(3, p, sub, src_sub, kind_all, js)
        got = u_new[:, :n_p].index_select(2, torch.from_numpy(js).cuda()).cpu().numpy()
        errs = assert_transfer(got, exp, kind_all[js], 1e-13, f"one tree, p{p} meshes")
        assert "refined" in errs and ("fused" in errs or p == 2)
    del u_old, u_new
    keys = t.keys().cpu().numpy().view(np.uint64)
    src, kind = src_all, kind_all
    for i, m in enumerate(meshes):
        g = gold["meshes"][i]
        a, b = offs[i], offs[i + 1]
        assert g["counts"][-1] == b - a, f"mesh {i}: leaf count"
        assert sha(flags[offs_old[i]:offs_old[i + 1]]) == g["flags"], f"mesh {i}: flags"
        assert sha(mesh_keys(keys[a:b], 3, D_FINE, m.d_max)) == g["keys"], f"mesh {i}: keys"
        assert sha(src[a:b] - np.int32(offs_old[i])) == g["map_src"], f"mesh {i}: map_src"
        assert sha(kind[a:b]) == g["map_kind"], f"mesh {i}: map_kind"
