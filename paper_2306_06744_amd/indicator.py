"""Training data and device training of the learned refinement indicator.

Each seeded field is a config-2 style workload: an isentropic vortex extruded
in z (strength U[3,7], centre U[-2,2]^2) on [-5,5]^3, levels 4..7, p = 3, five
FP64 conserved variables.  Its mesh is adapted with the geometric criterion of
Section 5.2 as in the plain cycle, and at the mesh states the cycle visits
(after the second and third adaptation) the label of a leaf is the geometric
flag before the depth clamps (+1: class 2, 0: class 1, -1: class 0).  Up to
``rows_per_class`` leaves per class and state are drawn, and their features
(lt_mlp_features) become training rows.  Training is mini-batch Adam through
lt_mlp_train_step.  Every step runs in the library's kernels; host code only
picks rows and batches.
"""
from __future__ import annotations

import numpy as np

from . import synth

TRAIN_SEEDS = range(100000, 102000)
HELDOUT_SEEDS = range(200000, 200100)


def _lt():
    import paper_2306_06744_amd as lt
    return lt


def mesh_states(w, states=(1, 2)):
    """Yields (tree, cycle) at each requested state of the plain cycle: the
    tree after cycles 0..k of flag/adapt/balance (centre advected per cycle)."""
    lt = _lt()
    nodes = synth.gl_nodes01(w.p)
    t = lt.Tree.uniform(w.dim, w.d_min, w.d_max)
    for c in range(max(states) + 1):
        f = t.flag(w.centres_at(c), w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=w.dist_axes,
                   periodic_dist=w.periodic_dist)
        t.adapt(f)
        t.balance()
        if c in states:
            yield t, c + 1


def field_rows(mlp, seed, rows_per_class=256, states=(1, 2)):
    """Training rows of one seeded field: (X bf16 (k, 320), y int8 (k,)) on the device."""
    import torch
    w = synth.workload_3d_extruded(seed)
    nodes = synth.gl_nodes01(w.p)
    g = synth.rng(seed)
    Xs, ys = [], []
    for t, c in mesh_states(w, states):
        cen = w.centres_at(c)
        u = t.vortex_field(cen, w.strengths, nodes, w.lo, w.length)
        raw = t.flag(cen, w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=w.dist_axes,
                     periodic_dist=w.periodic_dist, raw=True).cpu().numpy()
        pick = []
        for cls in (-1, 0, 1):
            idx = np.flatnonzero(raw == cls)
            if len(idx) > rows_per_class:
                idx = np.sort(g.choice(idx, size=rows_per_class, replace=False))
            pick.append(idx)
        rows = np.concatenate(pick).astype(np.int32)
        if len(rows) == 0:
            continue
        rows_d = torch.from_numpy(rows).cuda()
        Xs.append(mlp.features(u, rows=rows_d))
        ys.append(torch.from_numpy((raw[rows] + 1).astype(np.int8)).cuda())
    return Xs, ys


def training_set(mlp, seeds=TRAIN_SEEDS, rows_per_class=256):
    import torch
    Xs, ys = [], []
    for sd in seeds:
        a, b = field_rows(mlp, sd, rows_per_class)
        Xs += a
        ys += b
    return torch.cat(Xs), torch.cat(ys)


def train(mlp, X, y, steps=3000, batch=4096, lr=2e-3, seed=7):
    """Mini-batch Adam; returns the mean loss of the first and last 100 steps
    (evaluated by the forward pass on each batch before its update)."""
    import torch
    g = synth.rng(seed)
    n = X.shape[0]
    losses = []
    for s in range(steps):
        idx = torch.from_numpy(g.integers(0, n, size=min(batch, n))).cuda()
        xb = X.index_select(0, idx).contiguous()
        yb = y.index_select(0, idx).contiguous()
        if s < 100 or s >= steps - 100:
            z = mlp.logits(xb).double()
            losses.append(float(torch.nn.functional.cross_entropy(z, yb.long())))
        mlp.train_step(xb, yb, lr)
    k = min(100, len(losses) // 2)
    return float(np.mean(losses[:k])), float(np.mean(losses[-k:]))


def disagreement(mlp, seeds=HELDOUT_SEEDS, conf_min=0.9, taus=None):
    """Over the held-out fields' leaves at the cycle's mesh states: fraction of
    learned flags (geometric fallback below conf_min) that differ from the
    geometric flags, fraction that fell back, the network alone (argmax), and
    the modal-energy indicator (taus = (tau_refine, tau_coarsen)) for
    comparison."""
    tot = 0
    d_learned = d_alone = d_modal = fb = 0
    for sd in seeds:
        w = synth.workload_3d_extruded(sd)
        nodes = synth.gl_nodes01(w.p)
        for t, c in mesh_states(w):
            cen = w.centres_at(c)
            u = t.vortex_field(cen, w.strengths, nodes, w.lo, w.length)
            plain = t.flag(cen, w.r_in, w.r_out, nodes, w.lo, w.length, dist_axes=w.dist_axes)
            f, conf = t.flag_mlp(mlp, u, cen, w.r_in, w.r_out, nodes, w.lo, w.length,
                                 conf_min=conf_min, dist_axes=w.dist_axes)
            f0, _ = t.flag_mlp(mlp, u, cen, w.r_in, w.r_out, nodes, w.lo, w.length, conf_min=0.0,
                               dist_axes=w.dist_axes)
            n = plain.numel()
            tot += n
            d_learned += int((f != plain).sum())
            d_alone += int((f0 != plain).sum())
            fb += int((conf < conf_min).sum())
            if taus is not None:
                fm = t.flag_modal(w.p, u, taus[0], taus[1])
                d_modal += int((fm != plain).sum())
    out = {"leaves": tot, "learned": d_learned / tot, "fallback_rate": fb / tot,
           "network_alone": d_alone / tot}
    if taus is not None:
        out["modal"] = d_modal / tot
    return out
