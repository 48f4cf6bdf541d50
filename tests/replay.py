"""Solver-free replay of the paper's adaptive runs (Section 5.2).

The refinement criterion only looks at the vortex axis, which moves with the
free stream, so the mesh history of each run can be replayed without the FR
solver: at every cycle flag (geometric criterion, min-image distance),
adapt, then 2:1 balance.  Final leaf counts are compared with the paper's
tables (tests/golden/paper_element_counts.csv).

The 3D slab (one level-D_min layer, periodic in z, field independent of z)
is replayed either directly as a cube of identical layers, or as the 2D run
with D_min = 4, counting each 2D leaf of depth l as 2^(l-4) slab octants.
"""
from __future__ import annotations

import csv
import os

import numpy as np

from paper_2306_06744_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "paper_element_counts.csv")


def paper_counts() -> dict:
    out = {}
    with open(GOLDEN) as fh:
        rows = [ln for ln in fh if not ln.startswith("#")]
    for r in csv.DictReader(rows):
        out[r["run"]] = int(r["count"])
    return out


def runs() -> dict:
    return {r.name: r for r in synth.paper_runs()}


def replay_oracle(name: str, as_2d: bool = False, cycles: int | None = None):
    """Run one replay on the CPU oracle; returns (name, count)."""
    import oracle
    run = runs()[name]
    ncyc = run.cycles if cycles is None else cycles
    nodes = synth.gl_nodes01(run.p)
    dim = 2 if as_2d else run.dim
    t = oracle.Tree(dim, run.d_min, run.d_max, start_depth=run.start_depth)
    lo = run.lo[:dim]
    for k in [0] * run.warmup + list(range(ncyc)):
        f = t.flag([run.centre(k)], 5.0, 6.0, nodes, lo, run.length, dist_axes=2,
                   periodic_dist=True)
        t.adapt(f)
        t.balance()
    if run.dim == 3 and as_2d:
        mb = run.d_max.bit_length()
        depth = (t.keys() & np.uint64((1 << mb) - 1)).astype(np.int64)
        return name, int((2 ** (depth - run.d_min)).sum())
    return name, t.size() // run.z_layers
