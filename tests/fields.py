"""CPU helpers for tests: physical coordinates of the solution points of an
oracle tree's leaves and the FP64 vortex field there (oracle/mlp.py)."""
import numpy as np

import oracle
from oracle import mlp as ref


def leaf_geometry(dim, d_max, keys):
    """(depth (n,), anchor (n, dim)) of each key."""
    depth = np.zeros(len(keys), dtype=np.int64)
    anc = np.zeros((len(keys), dim), dtype=np.int64)
    for e, k in enumerate(keys):
        d, a = oracle.decode(dim, d_max, int(k))
        depth[e] = d
        anc[e] = a[:dim]
    return depth, anc


def point_xy(dim, d_max, depth, anc, nodes, lo, length):
    """x, y of every solution point: (n, (p+1)^dim) each, x fastest."""
    n1 = len(nodes)
    npts = n1 ** dim
    i = np.arange(npts)
    ix, iy = i % n1, (i // n1) % n1
    dx = length / 2 ** d_max
    s = (2.0 ** (d_max - depth))[:, None]
    X = lo[0] + dx * (anc[:, 0:1] + s * np.asarray(nodes)[ix][None, :])
    Y = lo[1] + dx * (anc[:, 1:2] + s * np.asarray(nodes)[iy][None, :])
    return X, Y


def vortex_u(dim, d_max, keys, nodes, lo, length, centres, strengths):
    """FP64 conserved variables (nvar, n_p, n): 5 in 3D, 4 in 2D (no rho w)."""
    depth, anc = leaf_geometry(dim, d_max, keys)
    X, Y = point_xy(dim, d_max, depth, anc, nodes, lo, length)
    q = ref.vortex_field(X, Y, [c[:2] for c in centres], strengths)   # (5, n, n_p)
    if dim == 2:
        q = q[[0, 1, 2, 4]]
    return np.ascontiguousarray(np.transpose(q, (0, 2, 1))), depth
