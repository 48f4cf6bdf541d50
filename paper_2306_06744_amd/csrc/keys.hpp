// keys.hpp -- Morton ID arithmetic on the device (Section 2.2, Algorithm
// "Morton Encoding").
//
// An octant is held as one uint64: key = (m << mb) | depth, where m is the
// bit-interleaved anchor in finest units (bit k of axis a at dim*k + a, x
// least significant) and mb = bitlength(d_max).  Because the anchor's bits
// below the octant's own resolution are zero, m equals the paper's raw ID
// followed by dim*(d_max - depth) padding zeros.  Interleaving uses the
// "magic number" spreading the paper recommends (shift-or-mask ladders).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lt {

// Geometry of one tree, or of an ensemble of independent trees held in one
// key array.  For an ensemble the mesh index sits above the Morton bits
// (bit mesh_shift = mb + dim*dmax and up), so the concatenated keys stay
// globally sorted mesh by mesh, and every search and scan of a single tree
// works on the whole ensemble unchanged; dmax is then the shared finest
// level and each mesh has its own refinement ceiling and coarsening floor.
struct KeyGeom {
  int dim;            // 2 or 3
  int dmax;           // finest depth (key resolution)
  int mb;             // bits that hold the depth
  int dmin;           // coarsening floor (single tree)
  unsigned periodic;  // bit a: axis a wraps
  int balance;        // 0 face, 1 edge, 2 corner
  int mesh_shift;     // first bit of the mesh index
  int nmesh;          // 1 for a single tree
  const int8_t* lim;  // ensemble: per mesh {floor, ceiling} (device), else null

  __host__ __device__ uint64_t width() const { return uint64_t(1) << dmax; }
  __host__ __device__ uint64_t depth_mask() const { return (uint64_t(1) << mb) - 1; }
  __host__ __device__ int nchild() const { return 1 << dim; }
};

__host__ __device__ inline uint64_t spread2(uint64_t x) {
  x &= 0xffffffffull;
  x = (x | (x << 16)) & 0x0000ffff0000ffffull;
  x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
  x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

__host__ __device__ inline uint64_t compact2(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0f0f0f0f0f0f0f0full;
  x = (x | (x >> 4)) & 0x00ff00ff00ff00ffull;
  x = (x | (x >> 8)) & 0x0000ffff0000ffffull;
  x = (x | (x >> 16)) & 0x00000000ffffffffull;
  return x;
}

__host__ __device__ inline uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__host__ __device__ inline uint64_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x | (x >> 4)) & 0x100f00f00f00f00full;
  x = (x | (x >> 8)) & 0x001f0000ff0000ffull;
  x = (x | (x >> 16)) & 0x001f00000000ffffull;
  x = (x | (x >> 32)) & 0x1fffffull;
  return x;
}

// Interleave an anchor (finest units) into the Morton index m.
__host__ __device__ inline uint64_t morton(const KeyGeom& g, const uint64_t* x) {
  if (g.dim == 2) return spread2(x[0]) | (spread2(x[1]) << 1);
  return spread3(x[0]) | (spread3(x[1]) << 1) | (spread3(x[2]) << 2);
}

__host__ __device__ inline void demorton(const KeyGeom& g, uint64_t m, uint64_t* x) {
  if (g.dim == 2) {
    x[0] = compact2(m);
    x[1] = compact2(m >> 1);
    x[2] = 0;
  } else {
    x[0] = compact3(m);
    x[1] = compact3(m >> 1);
    x[2] = compact3(m >> 2);
  }
}

__host__ __device__ inline int key_depth(const KeyGeom& g, uint64_t key) {
  return int(key & g.depth_mask());
}
// The mesh bits of a key, in place (0 for a single tree).
__host__ __device__ inline uint64_t key_mesh_bits(const KeyGeom& g, uint64_t key) {
  return g.nmesh > 1 ? (key >> g.mesh_shift) << g.mesh_shift : 0;
}
__host__ __device__ inline int key_mesh(const KeyGeom& g, uint64_t key) {
  return g.nmesh > 1 ? int(key >> g.mesh_shift) : 0;
}
// Morton index of the anchor without the mesh bits.
__host__ __device__ inline uint64_t key_morton(const KeyGeom& g, uint64_t key) {
  const uint64_t m = key >> g.mb;
  return g.nmesh > 1 ? (m & ((uint64_t(1) << (g.dim * g.dmax)) - 1)) : m;
}
// Coarsening floor and refinement ceiling of the tree a key belongs to.
__device__ inline void depth_limits(const KeyGeom& g, uint64_t key, int* lo, int* hi) {
  if (g.lim) {
    const int m = key_mesh(g, key);
    *lo = g.lim[2 * m];
    *hi = g.lim[2 * m + 1];
  } else {
    *lo = g.dmin;
    *hi = g.dmax;
  }
}
__host__ __device__ inline uint64_t key_m(const KeyGeom& g, uint64_t key) { return key >> g.mb; }
__host__ __device__ inline uint64_t make_key(const KeyGeom& g, uint64_t m, int depth) {
  return (m << g.mb) | uint64_t(depth);
}

// Morton-index span of one octant of depth d (its number of finest cells).
__host__ __device__ inline uint64_t span(const KeyGeom& g, int d) {
  return uint64_t(1) << (g.dim * (g.dmax - d));
}

// Key of child c (c = sum_a b_a 2^a) of the octant (m, d).
__host__ __device__ inline uint64_t child_key(const KeyGeom& g, uint64_t m, int d, int c) {
  return make_key(g, m | (uint64_t(c) << (g.dim * (g.dmax - d - 1))), d + 1);
}

// Child index of an octant of depth d >= 1 within its parent.
__host__ __device__ inline int child_index(const KeyGeom& g, uint64_t m, int d) {
  return int((m >> (g.dim * (g.dmax - d))) & uint64_t(g.nchild() - 1));
}

// Key that sorts right after every octant containing the finest cell with
// Morton index m: the leaf holding that cell is the last key <= it.
__host__ __device__ inline uint64_t point_key(const KeyGeom& g, uint64_t m) {
  return make_key(g, m, g.dmax);
}

// Shift coordinate x by delta along axis a; false outside a non-periodic domain.
__host__ __device__ inline bool shift_coord(const KeyGeom& g, int a, uint64_t x, int64_t delta,
                                            uint64_t* out) {
  const int64_t W = int64_t(g.width());
  int64_t y = int64_t(x) + delta;
  if ((g.periodic >> a) & 1u) {
    y = ((y % W) + W) % W;
  } else if (y < 0 || y >= W) {
    return false;
  }
  *out = uint64_t(y);
  return true;
}

// Index of the last key <= probe in keys[0, n) (or -1): with probe a point
// key, the leaf that holds the point.
__device__ inline int64_t last_le(const uint64_t* __restrict__ keys, int64_t n, uint64_t probe) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] <= probe)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo - 1;
}

// Index of the last key <= probe (or -1), searching outward from a hint index
// h in [0, n): gallop away from h in doubling steps until the probe is
// bracketed, then bisect.  Neighbour keys usually lie close to the querying
// leaf in Morton order, so the probes stay in a few cache lines.
__device__ inline int64_t last_le_near(const uint64_t* __restrict__ keys, int64_t n, uint64_t probe,
                                       int64_t h) {
  int64_t lo, hi;  // invariant: keys[lo] <= probe (lo == -1: none), keys[hi] > probe (hi == n: none)
  if (keys[h] <= probe) {
    lo = h;
    int64_t step = 1;
    for (;;) {
      hi = lo + step;
      if (hi >= n) {
        hi = n;
        break;
      }
      if (keys[hi] > probe) break;
      lo = hi;
      step <<= 1;
    }
  } else {
    hi = h;
    int64_t step = 1;
    for (;;) {
      lo = hi - step;
      if (lo < 0) {
        lo = -1;
        break;
      }
      if (keys[lo] <= probe) break;
      hi = lo;
      step <<= 1;
    }
  }
  while (hi - lo > 1) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] <= probe)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Radix directory over a sorted key array: bucket c covers the keys
// [c << shift, (c + 1) << shift), and d[c] is the index of the last key
// <= c << shift (-1 if none), for c = 0 .. nb; d[nb] = n - 1.  The leaf
// holding a probe then lies in [d[c], d[c + 1]] for c = probe >> shift, so a
// search reads two adjacent words and bisects a range of a few leaves
// instead of walking the whole array.
struct KeyDir {
  const int32_t* d;
  int shift;
  int64_t nb;
};

// Last index with keys[i] <= probe (-1 if none), through the directory.
__device__ inline int64_t dir_last_le(const uint64_t* __restrict__ keys, int64_t n, const KeyDir& D,
                                      uint64_t probe) {
  const uint64_t c = probe >> D.shift;
  int64_t lo, hi;
  if (c >= uint64_t(D.nb)) {
    lo = D.d[D.nb];
    hi = n;
  } else {
    lo = D.d[c];
    hi = int64_t(D.d[c + 1]) + 1;
  }
  // keep every probe inside [0, n) whatever the directory holds
  lo = lo < -1 ? -1 : (lo > n - 1 ? n - 1 : lo);
  hi = hi > n ? n : (hi < lo + 1 ? lo + 1 : hi);
  while (hi - lo > 1) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] <= probe)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// First index with keys[i] >= probe (n if none).
__device__ inline int64_t lower_bound(const uint64_t* __restrict__ keys, int64_t n, uint64_t probe) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < probe)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace lt
