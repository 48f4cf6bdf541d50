"""FP64 references for the learned refinement indicator and for the
modal-energy indicator it is measured against.

TEST INFRASTRUCTURE ONLY (imported by tests/ and the benchmark's checks).

  * vortex_field: the isentropic vortex of Section 5.2 (phi = 1/2, gamma = 1.4)
    superposed for several z-extruded vortices, on a free stream
    (rho, u, v, w, p) = (1, 1, 0, 0, 1), in conserved variables
    (rho, rho u, rho v, rho w, E); the perturbations are
        du = -a/(2 pi) (y - yc) e^{phi (1 - r2)},  dv = a/(2 pi) (x - xc) e^{phi (1 - r2)},
        dT = -a^2 (gamma - 1) / (16 phi gamma pi^2) e^{2 phi (1 - r2)},
    with r2 the squared xy distance to the axis, T = 1 + dT, rho = T^{1/(gamma-1)},
    p = rho^gamma.
  * modal: coefficients of an element's Gauss-Legendre nodal values in the
    orthonormal tensor Legendre basis (Gauss-Legendre quadrature is exact for
    the degree-2p products, so this is the exact projection).
  * features: log10(|c| + 1e-14) per mode and variable, scaled (f + 7) / 7.
  * modal_energy / modal_flags: the fraction of the density's modal energy in
    the modes whose highest per-axis degree is p, and the thresholded flag
    (+1 above log10 tau_r, -1 below log10 tau_c, else 0; all-zero density 0),
    with the refinement ceiling / coarsening floor clamps.  The thresholds
    are calibrated by this project, not taken from the paper (parity of the
    thresholds themselves is unpinned; the indicator's arithmetic is pinned
    by closed forms).
  * MLP 320 -> 128 -> 64 -> 3 with ReLU, softmax cross-entropy, and its
    gradients written out by hand (checked against finite differences); an
    optional storage map on the hidden activations models a network that
    keeps them in a narrower format.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg

GAMMA = 1.4
PHI = 0.5


def vortex_field(x, y, centres, strengths):
    """Conserved variables (5, ...) at points (x, y), z-extruded vortices."""
    du = np.zeros_like(x)
    dv = np.zeros_like(x)
    dT = np.zeros_like(x)
    for (xc, yc), a in zip(centres, strengths):
        dx = x - xc
        dy = y - yc
        r2 = dx * dx + dy * dy
        e = np.exp(PHI * (1.0 - r2))
        du += -a / (2 * math.pi) * dy * e
        dv += a / (2 * math.pi) * dx * e
        dT += -a * a * (GAMMA - 1) / (16 * PHI * GAMMA * math.pi ** 2) * e * e
    T = 1.0 + dT
    rho = T ** (1.0 / (GAMMA - 1.0))
    p = rho ** GAMMA
    u = 1.0 + du
    v = dv
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, np.zeros_like(x), E])


def gl(npts):
    x, w = npleg.leggauss(npts)
    return x, w


def modal_matrix_1d(p):
    """T[n, i] = w_i * Ln(x_i), Ln orthonormal Legendre on [-1, 1]."""
    x, w = gl(p + 1)
    T = np.zeros((p + 1, p + 1))
    for n in range(p + 1):
        c = np.zeros(n + 1)
        c[n] = 1.0
        T[n] = w * npleg.legval(x, c) * math.sqrt((2 * n + 1) / 2.0)
    return T


def modal(u, dim, p):
    """u: (..., (p+1)^dim) nodal values, x fastest -> modal coefficients
    (same shape, mode index k = kx + (p+1)(ky + (p+1) kz))."""
    T = modal_matrix_1d(p)
    n1 = p + 1
    shape = u.shape[:-1] + (n1,) * dim
    a = u.reshape(shape)              # (..., z, y, x)
    # apply T on every axis
    for ax in range(dim):
        a = np.moveaxis(np.tensordot(a, T, axes=([a.ndim - 1 - ax], [1])), -1, a.ndim - 1 - ax)
    return a.reshape(u.shape)


def features(coeffs):
    """coeffs: (nvar, npts) per element (or (..., nvar, npts)) -> flat features."""
    f = (np.log10(np.abs(coeffs) + 1e-14) + 7.0) / 7.0
    return f.reshape(f.shape[:-2] + (-1,))


def relu(x):
    return np.maximum(x, 0.0)


def forward(X, W1, b1, W2, b2, W3, b3, store=None):
    """X: (B, 320).  Returns logits and the cache for backward.

    ``store`` (optional) maps each hidden activation to the value the network
    keeps and passes on (e.g. rounding to a storage format); the backward
    pass then differentiates through it as the identity."""
    st = store if store is not None else (lambda a: a)
    z1 = X @ W1 + b1
    h1 = st(relu(z1))
    z2 = h1 @ W2 + b2
    h2 = st(relu(z2))
    z3 = h2 @ W3 + b3
    return z3, (X, z1, h1, z2, h2)


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grads(X, y, W1, b1, W2, b2, W3, b3, store=None):
    """Mean softmax cross-entropy over the batch and its gradients (``store``
    as in forward)."""
    z3, (X, z1, h1, z2, h2) = forward(X, W1, b1, W2, b2, W3, b3, store)
    P = softmax(z3)
    B = X.shape[0]
    loss = -np.mean(np.log(P[np.arange(B), y]))
    d3 = P.copy()
    d3[np.arange(B), y] -= 1.0
    d3 /= B
    gW3 = h2.T @ d3
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3.T) * (z2 > 0)
    gW2 = h1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (z1 > 0)
    gW1 = X.T @ d1
    gb1 = d1.sum(axis=0)
    return loss, (gW1, gb1, gW2, gb2, gW3, gb3)


def modal_energy(rho, dim, p):
    """rho: (n, (p+1)^dim) nodal density -> (top-mode energy, total energy)."""
    c = modal(rho, dim, p)
    n1 = p + 1
    k = np.arange(n1 ** dim)
    top = np.zeros(n1 ** dim, dtype=bool)
    for a in range(dim):
        top |= (k // n1 ** a) % n1 == p
    e = c * c
    return e[:, top].sum(axis=1), e.sum(axis=1)


def modal_flags(rho, depth, d_min, d_max, dim, p, tau_r, tau_c):
    """Modal-energy flags with the depth clamps (depth: (n,) ints)."""
    top, tot = modal_energy(rho, dim, p)
    f = np.zeros(len(tot), dtype=np.int8)
    nz = tot > 0
    with np.errstate(divide="ignore"):
        ls = np.where(nz, np.log10(np.where(nz, top, 1.0) / np.where(nz, tot, 1.0)), 0.0)
    f[nz & (ls > tau_r)] = 1
    f[nz & (ls < tau_c)] = -1
    f[(f == 1) & (depth >= d_max)] = 0
    f[(f == -1) & (depth <= d_min)] = 0
    return f, ls
