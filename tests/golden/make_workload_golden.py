"""Write tests/golden/workload_<name>.json from the CPU oracle only.

For each cycle of the synthetic workloads (2D [-5,5]^2 levels 3-6 p2, one
cycle; 3D [-5,5]^3 levels 4-7 p3, ten cycles advected +0.1 in x; the large 3D
workload, levels 4-10 and four vortices, six cycles at fixed centres, one with
the centres moved +0.05 in x and one moved +0.1; the 64-mesh ensemble, nine cycles advected
+0.1 in x, every mesh its own tree), the oracle's flags, keys, connectivity
and mapping are hashed (SHA-256 of the little-endian arrays) so the GPU tests
can check full-size outputs bit for bit without storing them.
Run:  python tests/golden/make_workload_golden.py [2d_small 3d_extruded 3d_large ensemble_64]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2306_06744_amd import synth  # noqa: E402


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def run(w: synth.Workload, path: str):
    o = oracle.Tree(w.dim, w.d_min, w.d_max)
    nodes = synth.gl_nodes01(w.p)
    out = {"workload": w.name, "seed_note": "synth.%s" % w.name, "cycles": []}
    for cyc in range(w.cycles):
        t0 = time.time()
        f = o.flag(w.centres_at(cyc), w.r_in, w.r_out, nodes, w.lo, w.length,
                   dist_axes=w.dist_axes, periodic_dist=w.periodic_dist)
        n_old = o.size()
        o.adapt(f)
        n_adapt = o.size()
        o.balance()
        nbr, hang = o.connect()
        src, kind = o.map()
        rec = {"cycle": cyc, "n_old": n_old, "n_adapt": n_adapt, "n_new": o.size(),
               "n_hang": int(len(hang)), "flags": sha(f), "keys": sha(o.keys()),
               "nbr": sha(nbr), "hang": sha(hang), "map_src": sha(src), "map_kind": sha(kind),
               "n_copy": int((kind == 0).sum()), "n_refined": int((kind > 0).sum()),
               "n_fused": int((kind < 0).sum())}
        out["cycles"].append(rec)
        print(cyc, rec["n_old"], "->", rec["n_new"], f"{time.time() - t0:.1f}s", flush=True)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


def cycle_record(o, cyc, f, n_old, n_adapt, t0):
    nbr, hang = o.connect()
    src, kind = o.map()
    rec = {"cycle": cyc, "n_old": n_old, "n_adapt": n_adapt, "n_new": o.size(),
           "n_hang": int(len(hang)), "flags": sha(f), "keys": sha(o.keys()),
           "nbr": sha(nbr), "hang": sha(hang), "map_src": sha(src), "map_kind": sha(kind),
           "n_copy": int((kind == 0).sum()), "n_refined": int((kind > 0).sum()),
           "n_fused": int((kind < 0).sum())}
    print(cyc, rec["n_old"], "->", rec["n_new"], f"{time.time() - t0:.1f}s", flush=True)
    return rec


def large_centres(w: synth.Workload, cyc: int):
    """Centres of cycle cyc of the large workload as the benchmark runs it:
    w.cycles - 1 cycles at the fixed centres, then one with them moved +0.05
    in x and the timed one moved +0.1 (it refines and coarsens)."""
    k = max(0, cyc - (w.cycles - 2))
    return [(c[0] + 0.05 * k, c[1], c[2]) for c in w.centres]


def run_large(w: synth.Workload, path: str):
    """The large workload's cycles as the benchmark runs them (large_centres);
    every cycle is hashed."""
    o = oracle.Tree(w.dim, w.d_min, w.d_max)
    nodes = synth.gl_nodes01(w.p)
    out = {"workload": w.name, "seed_note": "synth.%s" % w.name, "cycles": []}
    for cyc in range(w.cycles + 1):
        t0 = time.time()
        cen = large_centres(w, cyc)
        f = o.flag(cen, w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=w.dist_axes,
                   periodic_dist=w.periodic_dist)
        n_old = o.size()
        o.adapt(f)
        n_adapt = o.size()
        o.balance()
        out["cycles"].append(cycle_record(o, cyc, f, n_old, n_adapt, t0))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


def run_ensemble(seed: int, cycles: int, path: str):
    """Every mesh of the ensemble as its own oracle tree (keys at the mesh's
    own finest level, indices local to the mesh), `cycles` cycles with the
    centres advected +0.1 in x per cycle; the last cycle is hashed per mesh,
    the leaf counts of every cycle are kept."""
    meshes = synth.workload_ensemble(seed)
    out = {"workload": "ensemble_64", "seed_note": "synth.workload_ensemble(%d)" % seed,
           "cycles": cycles, "meshes": []}
    for mi, m in enumerate(meshes):
        t0 = time.time()
        o = oracle.Tree(3, m.d_min, m.d_max)
        nodes = synth.gl_nodes01(m.p)
        counts = []
        for cyc in range(cycles):
            f = o.flag(m.centres_at(cyc), m.r_in, m.r_out, nodes, (-5.0,) * 3, 10.0, dist_axes=3)
            n_old = o.size()
            o.adapt(f)
            n_adapt = o.size()
            o.balance()
            counts.append(o.size())
        rec = cycle_record(o, cycles - 1, f, n_old, n_adapt, t0)
        rec.update({"mesh": mi, "p": m.p, "d_max": m.d_max, "counts": counts})
        out["meshes"].append(rec)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    oracle.build()
    which = sys.argv[1:] or ["2d_small", "3d_extruded", "3d_large", "ensemble_64"]
    if "2d_small" in which:
        run(synth.workload_2d_small(1000), os.path.join(HERE, "workload_2d_small.json"))
    if "3d_extruded" in which:
        run(synth.workload_3d_extruded(2000), os.path.join(HERE, "workload_3d_extruded.json"))
    if "3d_large" in which:
        run_large(synth.workload_3d_large(3000), os.path.join(HERE, "workload_3d_large.json"))
    if "ensemble_64" in which:
        run_ensemble(4000, 9, os.path.join(HERE, "workload_ensemble_64.json"))
