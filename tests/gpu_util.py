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
