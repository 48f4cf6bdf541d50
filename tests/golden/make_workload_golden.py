"""Write tests/golden/workload_<name>.json from the CPU oracle only.

For each cycle of the two synthetic workloads (2D [-5,5]^2 levels 3-6 p2,
one cycle; 3D [-5,5]^3 levels 4-7 p3, ten cycles advected +0.1 in x), the
oracle's flags, keys, connectivity and mapping are hashed (SHA-256 of the
little-endian arrays) so the GPU tests can check full-size outputs bit for
bit without storing them.  Run:  python tests/golden/make_workload_golden.py
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


if __name__ == "__main__":
    oracle.build()
    which = sys.argv[1:] or ["2d_small", "3d_extruded"]
    if "2d_small" in which:
        run(synth.workload_2d_small(1000), os.path.join(HERE, "workload_2d_small.json"))
    if "3d_extruded" in which:
        run(synth.workload_3d_extruded(2000), os.path.join(HERE, "workload_3d_extruded.json"))
