"""Seeded synthetic inputs for the adaptation cycle.

This module only draws numbers and states workload shapes; it holds none of
the method's arithmetic (no keys, no criterion, no transfer).  Both the GPU
library's callers and the CPU oracle's tests take their inputs from here.

Inputs, each with the passage it stands in for:
  * solution-point positions on one axis (Gauss-Legendre points mapped to
    [0, 1]; the FR solution points of Section 2.1, family read as
    Gauss-Legendre), given as data so both sides use identical bits;
  * isentropic-vortex centres and strengths (Section 5.2) per workload;
  * the vortex path of the paper's adaptive runs: free stream (u, v) = (1, 1),
    time step 0.001 and adaptation every 10 steps (Section 5.2), so the
    centre moves by 0.01 per axis per cycle;
  * random solution arrays (the transfer is linear in u, so any values test
    it) and random refine/keep/coarsen flags.
RNG: numpy PCG64, seed 1000*k + i for parity case i of workload k and
1000*k for timing.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def gl_nodes01(p: int) -> np.ndarray:
    """Gauss-Legendre points of degree-p FR on [0, 1] (closed forms for p <= 3,
    numpy's Golub-Welsch values above)."""
    if p == 0:
        x = [0.0]
    elif p == 1:
        r = 1.0 / math.sqrt(3.0)
        x = [-r, r]
    elif p == 2:
        r = math.sqrt(3.0 / 5.0)
        x = [-r, 0.0, r]
    elif p == 3:
        a = math.sqrt(3.0 / 7.0 - 2.0 / 7.0 * math.sqrt(6.0 / 5.0))
        b = math.sqrt(3.0 / 7.0 + 2.0 / 7.0 * math.sqrt(6.0 / 5.0))
        x = [-b, -a, a, b]
    elif p <= 7:
        x = list(np.polynomial.legendre.leggauss(p + 1)[0])
    else:
        raise ValueError("p must be in 0..7")
    return np.array([(1.0 + v) / 2.0 for v in x], dtype=np.float64)


def gl_weights(p: int) -> np.ndarray:
    """Gauss-Legendre weights of the p+1 points on [-1, 1] (summing to 2)."""
    return np.polynomial.legendre.leggauss(p + 1)[1]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Workload:
    """One synthetic adaptation workload (cubic domain [lo, lo+length)^dim)."""
    name: str
    dim: int
    d_min: int
    d_max: int
    p: int
    nvar: int
    lo: tuple
    length: float
    r_in: float
    r_out: float
    dist_axes: int
    periodic_dist: bool
    centres: list = field(default_factory=list)    # per vortex, 3 coords
    strengths: list = field(default_factory=list)
    cycles: int = 1
    advect: tuple = (0.0, 0.0, 0.0)               # centre shift per cycle
    start_depth: int | None = None                 # uniform start (default d_min)

    def centres_at(self, cycle: int) -> list:
        return [tuple(c[a] + cycle * self.advect[a] for a in range(3)) for c in self.centres]


def workload_2d_small(seed: int = 1000) -> Workload:
    """2D, [-5,5]^2, uniform level 3, max level 6, p=2, 4 variables, one
    vortex of strength 5 centred uniformly in [-2,2]^2; radii 5 / 6."""
    g = rng(seed)
    c = g.uniform(-2.0, 2.0, size=2)
    return Workload("2d_small_p2_l3-6", 2, 3, 6, 2, 4, (-5.0, -5.0), 10.0, 5.0, 6.0, 2, False,
                    centres=[(float(c[0]), float(c[1]), 0.0)], strengths=[5.0], cycles=1)


def workload_3d_extruded(seed: int = 2000) -> Workload:
    """3D, [-5,5]^3, uniform level 4, max level 7, p=3, 5 variables, one
    z-extruded vortex (strength U[3,7], centre U[-2,2]^2, xy distance),
    10 cycles advected by +0.1 in x per cycle."""
    g = rng(seed)
    c = g.uniform(-2.0, 2.0, size=2)
    s = g.uniform(3.0, 7.0)
    return Workload("3d_extruded_p3_l4-7", 3, 4, 7, 3, 5, (-5.0, -5.0, -5.0), 10.0, 5.0, 6.0, 2,
                    False, centres=[(float(c[0]), float(c[1]), 0.0)], strengths=[float(s)],
                    cycles=10, advect=(0.1, 0.0, 0.0))


def workload_3d_large(seed: int = 3000) -> Workload:
    """3D, [-5,5]^3, uniform level 4, max level 10, p=3, 5 variables, four
    vortices (strength U[3,7], centre U[-3,3]^3, 3D distance).  The radius
    aims at ~8M leaves: four balls of radius r_in filled at the finest cell
    size (10/1024)^3 hold 8e6 cells for r_in ~ 0.76; r_out = 1.2 r_in.  Seven
    adaptations at fixed centres take the uniform level-4 mesh to level 10."""
    g = rng(seed)
    cen = [tuple(float(x) for x in g.uniform(-3.0, 3.0, size=3)) for _ in range(4)]
    st = [float(x) for x in g.uniform(3.0, 7.0, size=4)]
    cell = (10.0 / 2 ** 10) ** 3
    r = (8e6 * cell / (4 * 4.0 / 3.0 * math.pi)) ** (1.0 / 3.0)
    return Workload("3d_large_p3_l4-10", 3, 4, 10, 3, 5, (-5.0, -5.0, -5.0), 10.0, r, 1.2 * r, 3,
                    False, centres=cen, strengths=st, cycles=7)


@dataclass
class EnsembleMesh:
    """One mesh of an ensemble: 3D [-5,5]^3, uniform start at level d_min,
    3D-distance vortex criterion (radii r_in, 1.2 r_in)."""
    d_min: int
    d_max: int
    p: int
    centres: list
    strengths: list
    r_in: float

    @property
    def r_out(self):
        return 1.2 * self.r_in

    def centres_at(self, cycle: int) -> list:
        return [(c[0] + 0.1 * cycle, c[1], c[2]) for c in self.centres]


def workload_ensemble(seed: int = 4000, nmesh: int = 64) -> list:
    """Ensemble of independent 3D meshes: 1-4 vortices each (strength U[3,7],
    centre U[-3,3]^3), finest level U{6..9}, p U{2,3}, uniform start at level 3.
    The radius r_in aims each mesh at a log-uniform leaf count in [1e4, 1e6]
    (refined volume ~ n_vort * 4/3 pi r_in^3 at the finest cell size), clipped
    to [0.5, 2.0]; the counts reached are measured, not assumed."""
    g = rng(seed)
    out = []
    for _ in range(nmesh):
        nv = int(g.integers(1, 5))
        d_max = int(g.integers(6, 10))
        p = int(g.integers(2, 4))
        target = 10.0 ** g.uniform(4.0, 6.0)
        cell = (10.0 / 2 ** d_max) ** 3
        r = (target * cell / (nv * 4.0 / 3.0 * math.pi)) ** (1.0 / 3.0)
        r = float(min(max(r, 0.5), 2.0))
        cen = [tuple(float(x) for x in g.uniform(-3.0, 3.0, size=3)) for _ in range(nv)]
        st = [float(x) for x in g.uniform(3.0, 7.0, size=nv)]
        out.append(EnsembleMesh(3, d_max, p, cen, st, r))
    return out


def surface_points(dim: int, n: int, seed: int, kind: str = "sphere") -> np.ndarray:
    """(n, dim) points sampled uniformly on a closed surface inside [-5,5]^dim,
    a stand-in for the surface geometry the paper builds initial trees from
    (Section 5.1): a circle (2D) or sphere (3D) of radius 3, or (3D, kind
    "torus") a torus of radii 3 and 1 about the z axis, centred off the
    origin so that the cloud does not align with the tree."""
    g = rng(seed)
    c = np.array([0.137, -0.211, 0.073][:dim])
    if dim == 2:
        th = g.uniform(0.0, 2.0 * math.pi, n)
        return c + 3.0 * np.stack([np.cos(th), np.sin(th)], axis=1)
    if kind == "torus":
        # area-uniform: accept the tube angle with probability (R + r cos v) / (R + r)
        out = np.zeros((0, 3))
        while len(out) < n:
            u = g.uniform(0.0, 2.0 * math.pi, 2 * n)
            v = g.uniform(0.0, 2.0 * math.pi, 2 * n)
            keep = g.random(2 * n) < (3.0 + np.cos(v)) / 4.0
            u, v = u[keep], v[keep]
            p = np.stack([(3.0 + np.cos(v)) * np.cos(u), (3.0 + np.cos(v)) * np.sin(u), np.sin(v)],
                         axis=1)
            out = np.concatenate([out, p])
        return c + out[:n]
    x = g.standard_normal((n, 3))
    return c + 3.0 * x / np.linalg.norm(x, axis=1, keepdims=True)


def mlp_init(seed: int) -> np.ndarray:
    """He-normal initial parameters of the 320 -> 128 -> 64 -> 3 indicator
    network, flat FP32: W1[128][320], b1[128], W2[64][128], b2[64], W3[3][64], b3[3]."""
    g = rng(seed)
    parts = []
    for n_in, n_out in ((320, 128), (128, 64), (64, 3)):
        parts.append(g.standard_normal((n_out, n_in)) * math.sqrt(2.0 / n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def mlp_split(params: np.ndarray):
    """Flat parameters -> (W1, b1, W2, b2, W3, b3) views ([out][in] weights)."""
    shapes = [(128, 320), (128,), (64, 128), (64,), (3, 64), (3,)]
    out, o = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        out.append(params[o:o + k].reshape(sh))
        o += k
    return out


def random_flags(seed: int, n: int, p_refine: float = 0.3, p_coarsen: float = 0.4) -> np.ndarray:
    g = rng(seed)
    r = g.random(n)
    f = np.zeros(n, dtype=np.int8)
    f[r < p_refine] = 1
    f[(r >= p_refine) & (r < p_refine + p_coarsen)] = -1
    return f


def random_solution(seed: int, nvar: int, npts: int, n: int) -> np.ndarray:
    """(nvar, npts, n) float64 standard-normal values."""
    return rng(seed).standard_normal((nvar, npts, n))


# --------------------------------------------------------------- paper runs
@dataclass
class PaperRun:
    """One adaptive run of Section 5.2 replayed without the solver.

    The criterion depends only on the vortex axis, which moves with the free
    stream (1, 1): the centre at cycle k (time 0.01 k) is (0.01 k, 0.01 k).
    ``cycles`` adaptations run at k = 0 .. cycles-1, after ``warmup`` extra
    adaptations at the k = 0 centre from a uniform mesh at ``start_depth``.
    Distances use the minimum image (the vortex crosses the periodic boundary).
    ``z_layers`` > 1 marks the 3D slab, run as a cube of that many identical
    level-d_min layers (count = leaves / z_layers)."""
    name: str
    dim: int
    d_min: int
    d_max: int
    p: int
    half_width: float
    cycles: int
    start_depth: int
    warmup: int = 12
    z_layers: int = 1

    @property
    def lo(self):
        return tuple([-self.half_width] * self.dim)

    @property
    def length(self):
        return 2.0 * self.half_width

    def centre(self, k: int):
        t = k * 0.01
        return (t, t, 0.0)


def paper_runs() -> list:
    runs = []
    for dmax in (6, 7, 8):
        for p in (1, 2, 3):
            runs.append(PaperRun(f"2d_w25_d{dmax}_p{p}", 2, 3, dmax, p, 12.5, 2500, 3))
    for dmax in (8, 9, 10):
        for p in (1, 2, 3):
            runs.append(PaperRun(f"2d_w100_d{dmax}_p{p}", 2, 3, dmax, p, 50.0, 10000, dmax))
    for dmax in (6, 7, 8):
        for p in (1, 2, 3):
            runs.append(PaperRun(f"3d_slab_d{dmax}_p{p}", 3, 4, dmax, p, 12.5, 2500, 4, z_layers=16))
    return runs
