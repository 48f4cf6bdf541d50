"""Brute-force references on tiny trees, formulated on the grid of finest cells.

A leaf is the set of finest-resolution cells it covers; two leaves touch iff
one of their cells is a (periodic) neighbour of one of the other's.  This
formulation shares nothing with the oracle's pointer tree or with the GPU
library, so agreement pins both.
"""
from __future__ import annotations

import itertools

import numpy as np

import oracle


def leaves_of(dim, d_max, keys):
    out = []
    for k in keys:
        d, a = oracle.decode(dim, d_max, int(k))
        out.append((d, tuple(int(x) for x in a)))
    return out


def keys_of(dim, d_max, leaves):
    return np.array(sorted(oracle.encode(dim, d_max, d, a) for d, a in leaves), dtype=np.uint64)


def owner_grid(dim, d_max, leaves):
    W = 1 << d_max
    g = -np.ones((W,) * dim, dtype=np.int64)
    for i, (d, a) in enumerate(leaves):
        s = 1 << (d_max - d)
        sl = tuple(slice(a[ax], a[ax] + s) for ax in range(dim))
        assert (g[sl] == -1).all(), "overlapping leaves"
        g[sl] = i
    assert (g >= 0).all(), "leaves do not tile the domain"
    return g


def directions(dim, kind):
    limit = {0: 1, 1: min(2, dim), 2: dim}[kind]
    for d in itertools.product((-1, 0, 1), repeat=dim):
        nz = sum(1 for x in d if x != 0)
        if 1 <= nz <= limit:
            yield d


def violators(dim, d_max, leaves, kind=2):
    """Set of leaves that touch a leaf two or more levels finer."""
    g = owner_grid(dim, d_max, leaves)
    depth = np.array([d for d, _ in leaves])
    D = depth[g]
    bad = set()
    for d in directions(dim, kind):
        nb = np.roll(g, shift=tuple(-x for x in d), axis=tuple(range(dim)))
        mask = depth[nb] < D - 1
        bad.update(int(v) for v in np.unique(nb[mask]))
    return bad


def split(dim, d_max, leaf):
    d, a = leaf
    h = 1 << (d_max - d - 1)
    kids = []
    for c in range(1 << dim):
        kids.append((d + 1, tuple(a[ax] + (h if (c >> ax) & 1 else 0) for ax in range(dim))))
    return kids


def balance(dim, d_max, leaves, kind=2, seed=0):
    """Split one violating leaf at a time, picked at random, until none is left."""
    rng = np.random.default_rng(seed)
    leaves = list(leaves)
    while True:
        bad = sorted(violators(dim, d_max, leaves, kind))
        if not bad:
            return leaves
        i = bad[rng.integers(len(bad))]
        leaves = leaves[:i] + split(dim, d_max, leaves[i]) + leaves[i + 1:]


def face_neighbours(dim, d_max, leaves, e, f, g=None):
    """Leaves owning the finest cells just across face f = 2*axis + side of leaf e
    (g: the owner grid of ``leaves``, computed here if not given)."""
    if g is None:
        g = owner_grid(dim, d_max, leaves)
    W = 1 << d_max
    d, a = leaves[e]
    s = 1 << (d_max - d)
    ax, side = divmod(f, 2)
    idx = []
    for b in range(dim):
        if b == ax:
            idx.append([(a[b] + s) % W] if side else [(a[b] - 1) % W])
        else:
            idx.append(list(range(a[b], a[b] + s)))
    owners = set()
    for cell in itertools.product(*idx):
        owners.add(int(g[cell]))
    return owners
