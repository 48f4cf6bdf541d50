"""FP64 oracle of the flux-reconstruction residual and the three-stage
Runge-Kutta step on a linear tree (2D: 4 Euler variables, 3D: 5).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it and it shares no code with the GPU library.

What it computes, step by step in the paper's order:

* Section 2.1: on each element the conservation law is differentiated axis
  by axis.  Along every line of Gauss-Legendre solution points in axis a the
  flux polynomial f(xi) = sum_i l_i(xi) f_i is corrected at both ends by
  Huynh's correction functions g_L, g_R (the right and left Radau
  polynomials of degree p+1, which recover the discontinuous Galerkin
  method), d f^/d xi = sum_i l_i' f_i + g_L' (f^(-1) - f(-1)) + g_R' (f^(1) - f(1)),
  with f(+-1) the flux polynomial's end values and f^(+-1) the common fluxes;
  d/dx = (2/h) d/d xi, and R = -sum_a d f_a / d x_a.
* Section 4.3, Algorithm "Procedure of common flux calculations": the solution
  is interpolated to the flux points of every face; a conforming face takes
  the Rusanov flux of its two traces; at a hanging face the coarse trace is
  L2-projected onto each of the 2^(dim-1) mortars (eq. interpolation_operator:
  M_Xi u^ = S_Xi u), the fine traces are copied onto them, the Rusanov flux is
  computed on each mortar, each fine face takes its mortar's flux and the
  coarse face takes the L2 projection of the mortar fluxes (eq.
  projection_operator: M F = sum_i S^i F^i).  The face operators are assembled
  by separate Gauss-Legendre quadrature with p+2 points.
* Eq. rk3: u1 = u + dt R(u), u2 = 3/4 u + 1/4 u1 + 1/4 dt R(u1),
  u_next = 1/3 u + 2/3 u2 + 2/3 dt R(u2).

Readings: the Euler equations with gamma given by the caller (1.4 in the
workloads); a periodic domain (the paper considers only periodic
boundaries); face f = 2 axis + side; face points ordered by the tangential
axes in increasing order, the lower fastest; mortar slot s = the fine face's
tangential child bits, lower axis first (the hanging-face table's order).
"""
from __future__ import annotations

import itertools

import numpy as np
from numpy.polynomial import legendre as npleg

import oracle


def lagrange(nodes, k, x):
    """l_k(x) for the Lagrange basis on `nodes`."""
    v = np.ones_like(np.asarray(x, dtype=np.float64))
    for m, zm in enumerate(nodes):
        if m != k:
            v = v * (x - zm) / (nodes[k] - zm)
    return v


def lagrange_deriv(nodes, k, x):
    """l_k'(x) by the product rule."""
    n = len(nodes)
    out = np.zeros_like(np.asarray(x, dtype=np.float64))
    for r in range(n):
        if r == k:
            continue
        term = np.ones_like(out) / (nodes[k] - nodes[r])
        for m in range(n):
            if m != k and m != r:
                term = term * (x - nodes[m]) / (nodes[k] - nodes[m])
        out = out + term
    return out


class Operators1D:
    """One-axis operators of degree p on the Gauss-Legendre points z."""

    def __init__(self, p: int):
        self.p = p
        n = p + 1
        self.z, self.w = oracle.gauss_legendre(n)
        z = self.z
        # basis values at the element ends and the differentiation matrix
        self.l_left = np.array([lagrange(z, j, -1.0) for j in range(n)])
        self.l_right = np.array([lagrange(z, j, 1.0) for j in range(n)])
        self.D = np.array([[lagrange_deriv(z, j, z[i]) for j in range(n)] for i in range(n)])
        # Radau correction functions of degree p+1 (Section 2.1):
        #   g_L = (-1)^(p+1)/2 (P_{p+1} - P_p),  g_R = (P_{p+1} + P_p)/2
        cL = np.zeros(p + 2)
        cL[p + 1], cL[p] = 0.5 * (-1) ** (p + 1), -0.5 * (-1) ** (p + 1)
        cR = np.zeros(p + 2)
        cR[p + 1], cR[p] = 0.5, 0.5
        self.g_left = cL
        self.g_right = cR
        self.dgL = npleg.legval(z, npleg.legder(cL))
        self.dgR = npleg.legval(z, npleg.legder(cR))
        # mortar operators of one half (b = 0 lower, 1 upper), by quadrature
        q, wq = oracle.gauss_legendre(p + 2)
        M = np.array([[np.sum(wq * lagrange(z, j, q) * lagrange(z, i, q)) for i in range(n)]
                      for j in range(n)])
        self.to_mortar = []     # coarse face polynomial -> mortar b (eq. interpolation_operator)
        self.from_mortar = []   # mortar b flux -> coarse face (eq. projection_operator)
        for b in range(2):
            xi = (q + 2 * b - 1) / 2.0       # quadrature points of half b, coarse coordinates
            # mortar b: M_Xi u^ = S_Xi u,  S_Xi[j, i] = int_Xi l^_j l_i
            S_m = np.array([[np.sum(wq * lagrange(z, j, q) * lagrange(z, i, xi)) for i in range(n)]
                            for j in range(n)])
            self.to_mortar.append(np.linalg.solve(M, S_m))
            # coarse face: M F = S^b F^b,  S^b[j, i] = int_{half b} l_j l^_i (d xi = d z / 2)
            S_c = np.array([[np.sum(wq / 2.0 * lagrange(z, j, xi) * lagrange(z, i, q))
                             for i in range(n)] for j in range(n)])
            self.from_mortar.append(np.linalg.solve(M, S_c))


def face_operators(ops: Operators1D, dim: int):
    """Mortar operators on a face of a dim-dimensional element, per slot s
    (tangential child bits, lower axis first), acting on face points ordered
    lower tangential axis fastest."""
    to_m, from_m = [], []
    for s in range(1 << (dim - 1)):
        if dim == 2:
            to_m.append(ops.to_mortar[s])
            from_m.append(ops.from_mortar[s])
        else:
            b0, b1 = s & 1, (s >> 1) & 1
            to_m.append(np.kron(ops.to_mortar[b1], ops.to_mortar[b0]))
            from_m.append(np.kron(ops.from_mortar[b1], ops.from_mortar[b0]))
    return to_m, from_m


# ------------------------------------------------------------------ Euler
def pressure(U, gamma):
    """U: (nvar, ...) conserved (rho, rho u_a..., E)."""
    dim = U.shape[0] - 2
    kin = sum(U[1 + a] ** 2 for a in range(dim)) / U[0]
    return (gamma - 1.0) * (U[-1] - 0.5 * kin)


def flux(U, a, gamma):
    """Euler flux along axis a: (rho u_a, rho u u_a + p delta, (E + p) u_a)."""
    dim = U.shape[0] - 2
    p = pressure(U, gamma)
    ua = U[1 + a] / U[0]
    F = np.empty_like(U)
    F[0] = U[1 + a]
    for b in range(dim):
        F[1 + b] = U[1 + b] * ua + (p if b == a else 0.0)
    F[-1] = (U[-1] + p) * ua
    return F


def rusanov(UL, UR, a, gamma):
    """Common flux across a face normal to axis a, UL on the low side."""
    def speed(U):
        return np.abs(U[1 + a] / U[0]) + np.sqrt(gamma * pressure(U, gamma) / U[0])
    lam = np.maximum(speed(UL), speed(UR))
    return 0.5 * (flux(UL, a, gamma) + flux(UR, a, gamma)) - 0.5 * lam * (UR - UL)


# ------------------------------------------------------------------ residual
def _depths(keys, d_max):
    mb = int(d_max).bit_length()
    return (np.asarray(keys, dtype=np.uint64) & np.uint64((1 << mb) - 1)).astype(np.int64)


def _line_view(U, a, dim):
    """U: (nvar, n_e, (p+1)^dim) -> array with axis a last: (nvar, n_e, *other axes, n1),
    other axes ordered so that flattening them gives the face point index
    (lower tangential axis fastest)."""
    nvar, ne, npts = U.shape
    n1 = round(npts ** (1.0 / dim))
    V = U.reshape((nvar, ne) + (n1,) * dim)          # (..., z, y, x): axis b at position 2 + dim-1-b
    pos = 2 + dim - 1 - a
    V = np.moveaxis(V, pos, -1)                       # remaining tangential axes stay high-to-low
    return V


def _from_line_view(V, a, dim):
    pos = 2 + dim - 1 - a
    W = np.moveaxis(V, -1, pos)
    return W.reshape(W.shape[:2] + (-1,))


def residual(keys, nbr, hang, u, dim, d_max, length, p, gamma=1.4):
    """R(u) of Section 2.1 with the common fluxes of Section 4.3.

    keys: leaf Morton IDs; nbr (n, 2 dim) and hang rows from the oracle's
    connectivity; u: (nvar, n_p, n) nodal conserved variables.  Returns
    (R, faces) with R like u and faces = {"common": (n, 2 dim, nvar, nfp),
    "local": (n, 2 dim, nvar, nfp)} the common and local normal fluxes at
    every element face."""
    ops = Operators1D(p)
    n1 = p + 1
    nvar, npts, ne = u.shape
    assert nvar == dim + 2 and npts == n1 ** dim
    nfp = n1 ** (dim - 1)
    U = np.transpose(u, (0, 2, 1)).astype(np.float64)       # (nvar, ne, npts)
    h = length / 2.0 ** _depths(keys, d_max)
    nbr = np.asarray(nbr).reshape(ne, 2 * dim)
    depth = _depths(keys, d_max)

    trace = np.zeros((ne, 2 * dim, nvar, nfp))     # solution at the face points
    floc = np.zeros((ne, 2 * dim, nvar, nfp))      # flux polynomial's end values
    Fa = []
    for a in range(dim):
        F = flux(U, a, gamma)                               # (nvar, ne, npts)
        Fa.append(F)
        UL, FL = _line_view(U, a, dim), _line_view(F, a, dim)
        for side, lv in ((0, ops.l_left), (1, ops.l_right)):
            tr = np.tensordot(UL, lv, axes=([-1], [0]))     # (nvar, ne, *tangential)
            fl = np.tensordot(FL, lv, axes=([-1], [0]))
            trace[:, 2 * a + side] = np.transpose(tr.reshape(nvar, ne, nfp), (1, 0, 2))
            floc[:, 2 * a + side] = np.transpose(fl.reshape(nvar, ne, nfp), (1, 0, 2))

    common = np.full((ne, 2 * dim, nvar, nfp), np.nan)
    # conforming faces: each pair once, from its low side
    for a in range(dim):
        f = 2 * a + 1
        j_all = nbr[:, f]
        E = np.flatnonzero((j_all >= 0) & (depth[np.maximum(j_all, 0)] == depth))
        J = j_all[E]
        UL = np.transpose(trace[E, f], (1, 0, 2))           # (nvar, pairs, nfp)
        UR = np.transpose(trace[J, f - 1], (1, 0, 2))
        F = np.transpose(rusanov(UL, UR, a, gamma), (1, 0, 2))
        common[E, f] = F
        common[J, f - 1] = F
    # hanging faces through mortars
    to_m, from_m = face_operators(ops, dim)
    for row in np.asarray(hang).reshape(-1, 2 + (1 << (dim - 1))):
        c, f = int(row[0]), int(row[1])
        a, side = f // 2, f % 2
        acc = np.zeros((nvar, nfp))
        for s, k in enumerate(row[2:]):
            k = int(k)
            uc = trace[c, f] @ to_m[s].T                     # (nvar, nfp) on mortar s
            uk = trace[k, f ^ 1]
            UL, UR = (uc, uk) if side == 1 else (uk, uc)
            F = rusanov(UL, UR, a, gamma)
            common[k, f ^ 1] = F
            acc += F @ from_m[s].T
        common[c, f] = acc
    assert not np.isnan(common).any(), "a face has no common flux (tree not periodic or not balanced)"

    R = np.zeros_like(U)
    for a in range(dim):
        FL = _line_view(Fa[a], a, dim)                       # (nvar, ne, *tang, n1)
        dF = np.tensordot(FL, ops.D, axes=([-1], [1]))        # d/dxi along the line
        jl = common[:, 2 * a] - floc[:, 2 * a]                # (ne, nvar, nfp)
        jr = common[:, 2 * a + 1] - floc[:, 2 * a + 1]
        shape = (nvar, ne) + (n1,) * (dim - 1)
        jl = np.transpose(jl, (1, 0, 2)).reshape(shape)
        jr = np.transpose(jr, (1, 0, 2)).reshape(shape)
        dF = dF + jl[..., None] * ops.dgL + jr[..., None] * ops.dgR
        dF = dF * (2.0 / h).reshape((1, ne) + (1,) * dim)
        R -= _from_line_view(dF, a, dim)
    return np.transpose(R, (0, 2, 1)), {"common": common, "local": floc}


def rk3(u, dt, R):
    """One step of eq. rk3 for du/dt = R(u)."""
    u1 = u + dt * R(u)
    u2 = 0.75 * u + 0.25 * u1 + 0.25 * dt * R(u1)
    return u / 3.0 + 2.0 / 3.0 * u2 + 2.0 / 3.0 * dt * R(u2)


def rk3_step(keys, nbr, hang, u, dt, dim, d_max, length, p, gamma=1.4):
    """One step of eq. rk3 with the residual above on a fixed tree."""
    return rk3(u, dt, lambda v: residual(keys, nbr, hang, v, dim, d_max, length, p, gamma)[0])


def solution_points(keys, dim, d_max, p, lo, length):
    """Physical solution points (n, n_p, dim), x fastest (for test fields)."""
    z = (oracle.gauss_legendre(p + 1)[0] + 1.0) / 2.0
    mb = int(d_max).bit_length()
    dx = length / 2 ** d_max
    out = np.zeros((len(keys), (p + 1) ** dim, dim))
    for e, k in enumerate(np.asarray(keys, dtype=np.uint64)):
        d, anc = oracle.decode(dim, d_max, int(k))
        s = 2 ** (d_max - d)
        for i, idx in enumerate(itertools.product(range(p + 1), repeat=dim)):
            ii = idx[::-1]
            for ax in range(dim):
                out[e, i, ax] = lo[ax] + dx * (anc[ax] + s * z[ii[ax]])
    return out
