"""Helpers shared by the GPU parity tests: run one cycle on both the HIP
library (through the C ABI) and the CPU oracle with identical inputs."""
from __future__ import annotations

import numpy as np


def np_keys(t) -> np.ndarray:
    return t.keys().cpu().numpy().view(np.uint64)


def both(dim, d_min, d_max, depth=None, periodic_mask=None, balance=2):
    import oracle
    import paper_2306_06744_amd as lt
    g = lt.Tree.uniform(dim, d_min, d_max, depth=depth, periodic_mask=periodic_mask,
                        balance=balance)
    o = oracle.Tree(dim, d_min, d_max, periodic_mask=periodic_mask, balance=balance,
                    start_depth=depth)
    return g, o


def adapt_both(g, o, flags: np.ndarray):
    import torch
    g.adapt(torch.from_numpy(flags).cuda())
    o.adapt(flags)


def assert_same_tree(g, o, what=""):
    kg, ko = np_keys(g), o.keys()
    assert kg.shape == ko.shape, f"{what}: {kg.shape} vs {ko.shape} leaves"
    assert np.array_equal(kg, ko), f"{what}: keys differ at {np.flatnonzero(kg != ko)[:5]}"


def assert_same_connectivity(g, o, what=""):
    g.connect()
    nbr_o, hang_o = o.connect()
    nbr_g = g.nbr().cpu().numpy()
    hang_g = g.hang().cpu().numpy()
    assert np.array_equal(nbr_g, nbr_o), f"{what}: nbr differs"
    assert hang_g.shape == hang_o.shape and np.array_equal(hang_g, hang_o), f"{what}: hang differs"


def assert_same_map(g, o, what=""):
    g.map()
    src, kind = g.mapping()
    src_o, kind_o = o.map()
    assert np.array_equal(src.cpu().numpy(), src_o), f"{what}: map_src differs"
    assert np.array_equal(kind.cpu().numpy(), kind_o), f"{what}: map_kind differs"


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def class_errors(got: np.ndarray, ref: np.ndarray, kind: np.ndarray) -> dict:
    """Transfer error per class of the mapping, so that exact copies do not
    dilute errors of interpolated or projected elements: for copy (kind 0),
    refined (kind > 0) and fused (kind < 0) elements, (relative L2 over the
    class, largest absolute error over the class's largest |value|, count).
    got, ref: (nvar, n_p, n) over the same n new leaves as kind."""
    out = {}
    for name, sel in (("copy", kind == 0), ("refined", kind > 0), ("fused", kind < 0)):
        if not sel.any():
            continue
        a, b = got[..., sel], ref[..., sel]
        l2 = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        mx = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
        out[name] = (l2, mx, int(sel.sum()))
    return out


def assert_transfer(got, ref, kind, tol, what="", copies_exact=True):
    """Per-class transfer bar: copies bit-exact (unless copies_exact is
    False), refined and fused elements within tol both in relative L2 and in
    the largest error relative to the class's largest value."""
    errs = class_errors(got, ref, kind)
    print(what, " ".join(f"{k}[{n}] l2 {a:.2e} max {b:.2e}" for k, (a, b, n) in errs.items()),
          flush=True)
    for name, (l2, mx, n) in errs.items():
        if name == "copy" and copies_exact:
            assert mx == 0.0, f"{what}: copies differ ({mx:.3e})"
        else:
            assert l2 <= tol and mx <= tol, f"{what}: {name} l2 {l2:.3e} max {mx:.3e} > {tol}"
    return errs


def dense_expected(dim, p, u_old, src, kind, js):
    """What the transfer of Section 4.2 gives the new leaves js, from the
    oracle's dense operators: copy, I_c u_parent (refined child c = kind-1),
    sum_c P_c u_child_c (fused; the children are old[src .. src + 2^dim - 1]).
    u_old: (nvar, n_p, n_old) host array.  Returns (nvar, n_p, len(js))."""
    import oracle
    I, P = oracle.operators(dim, p)
    js = np.asarray(js)
    k, s = kind[js].astype(np.int64), src[js].astype(np.int64)
    exp = np.empty(u_old.shape[:2] + (len(js),))
    sel = k == 0
    exp[:, :, sel] = u_old[:, :, s[sel]]
    for c in range(1 << dim):
        sel = k == c + 1
        if sel.any():
            exp[:, :, sel] = np.matmul(I[c], u_old[:, :, s[sel]])
    sel = k < 0
    if sel.any():
        acc = np.zeros(u_old.shape[:2] + (int(sel.sum()),))
        for c in range(1 << dim):
            acc += np.matmul(P[c], u_old[:, :, s[sel] + c])
        exp[:, :, sel] = acc
    return exp


def changed_and_sampled(kind, rng, copy_frac=0.01, min_copies=200):
    """Every refined and fused new leaf plus a seeded sample of the copies
    (copy_frac of them, at least min_copies)."""
    changed = np.flatnonzero(kind != 0)
    copies = np.flatnonzero(kind == 0)
    m = min(len(copies), max(min_copies, int(copy_frac * len(copies))))
    pick = rng.choice(copies, size=m, replace=False) if m else copies[:0]
    return np.sort(np.concatenate([changed, pick]))
