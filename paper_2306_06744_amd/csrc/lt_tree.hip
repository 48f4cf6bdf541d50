// lt_tree.hip -- tree kernels and the C ABI of the adaptation cycle.
//
// Keys stay sorted throughout: every kernel that changes the leaf set counts
// its outputs per input leaf, takes an exclusive scan of the counts with
// decoupled look-back, and writes its outputs in input order, which is
// Morton order.  No sort, no linearisation pass and no atomics decide any
// output position, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tree.hpp"

using lt::KeyGeom;

namespace lt {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }

lt_status fail(lt_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

namespace {
std::mutex g_alloc_mu;
Alloc g_alloc;  // registered by lt_set_allocator; empty: hipMalloc / hipFree
}  // namespace

Alloc registered_alloc() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

void register_alloc(const Alloc& A) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = A;
}

hipError_t dev_malloc(const Alloc& A, void** p, size_t bytes) {
  *p = nullptr;
  if (!A.alloc) return hipMalloc(p, bytes);
  *p = A.alloc(bytes, nullptr, A.ctx);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t dev_free(const Alloc& A, void* p) {
  if (!p) return hipSuccess;
  if (!A.free_) return hipFree(p);
  const hipError_t e = hipDeviceSynchronize();
  A.free_(p, nullptr, A.ctx);
  return e;
}

}  // namespace lt

#define LT_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return lt::fail(LT_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LT_TRY(expr)                \
  do {                              \
    lt_status s_ = (expr);          \
    if (s_ != LT_OK) return s_;     \
  } while (0)

namespace lt {
namespace {


int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------ kernels
// Zero the look-back words and counters before a scan.  converge (captured
// cycles, after a balance marking pass): no fresh marks means the fixpoint.
// Captured cycles also fold their count bookkeeping in here (one launch fewer
// each): *cnt_dst = *cnt_src when both are set, and reset_conv clears the
// fixpoint flag at the start of a cycle.
__global__ void k_clear_scan(uint64_t* status, int64_t ntiles, DevCtr* ctr, int clear_err,
                             int converge, int clear_list, int reset_conv, int64_t* cnt_dst,
                             const int64_t* cnt_src) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < ntiles) status[i] = 0;
  if (i == 0) {
    if (clear_list) {  // the lists adapt and balance refinement build for the next pass
      ctr->nexam = 0;
      ctr->nfused = 0;
    }
    if (converge && ctr->nmarked == 0) ctr->conv = 1;
    if (reset_conv) ctr->conv = 0;
    if (cnt_dst && cnt_src) *cnt_dst = *cnt_src;
    ctr->ticket = 0;
    ctr->total = 0;
    ctr->nmarked = 0;
    ctr->nfgroups = 0;
    if (clear_err) ctr->err = 0;
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Uniform tree: leaf i of depth D has Morton index i * span(D).
__global__ void k_uniform(KeyGeom g, int depth, int64_t n, uint64_t* keys) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = make_key(g, uint64_t(i) << (g.dim * (g.dmax - depth)), depth);
}

// Ensemble of uniform trees: mesh m holds 2^(dim*depth_m) leaves starting at offs[m].
__global__ void k_uniform_batch(KeyGeom g, const int64_t* __restrict__ offs,
                                const int8_t* __restrict__ depth, int nmesh, int64_t n,
                                uint64_t* __restrict__ keys) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = nmesh - 1;
  while (lo < hi) {  // last mesh whose first leaf is <= i
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int d = depth[lo];
  keys[i] = (uint64_t(lo) << g.mesh_shift) |
            make_key(g, uint64_t(i - offs[lo]) << (g.dim * (g.dmax - d)), d);
}

// First leaf of every mesh (offs[nmesh] = n).
__global__ void k_mesh_offsets(KeyGeom g, const uint64_t* __restrict__ keys, int64_t n, int nmesh,
                               int64_t* __restrict__ offs) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m > nmesh) return;
  offs[m] = m == nmesh ? n : lower_bound(keys, n, uint64_t(m) << g.mesh_shift);
}

// Complete linear tree check: each key valid, and the Morton range of leaf i
// ends exactly where leaf i+1 starts (so keys ascend, tile, and do not overlap).
__global__ void k_validate(KeyGeom g, const uint64_t* __restrict__ keys, int64_t n, unsigned* err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  const int d = key_depth(g, k);
  const uint64_t m = key_m(g, k);
  bool ok = d <= g.dmax;
  if (ok) {
    if ((m & (span(g, d) - 1)) != 0) ok = false;                      // padding bits
    if (g.dim * g.dmax < 64 && (m >> (g.dim * g.dmax)) != 0) ok = false;  // outside the domain
  }
  if (ok) {
    const uint64_t end = m + span(g, d);
    if (i + 1 < n) {
      const uint64_t kn = keys[i + 1];
      if (key_depth(g, kn) > g.dmax || key_m(g, kn) != end) ok = false;
    } else {
      const uint64_t full = g.dim * g.dmax >= 64 ? 0 : (uint64_t(1) << (g.dim * g.dmax));
      if (end != full) ok = false;
    }
    if (i == 0 && m != 0) ok = false;
  }
  if (!ok) atomicOr(err, ERR_INVALID_TREE);
}

// Adaptation (Section 4.1).  Per leaf: +1 -> 2^dim children, first leaf of a
// complete all -1 family -> parent, other members of such a family -> nothing,
// everything else -> itself.
// Balance marks written by adapt (see the marking pass): the children of a
// refined leaf are to be examined, a fused parent is to be checked against
// finer neighbours; every other leaf is balanced with its neighbours already.
constexpr uint32_t kMarkExamine = 4u;
// Workgroups of a marking pass over the examine list (it strides over the
// list, whose length is on the device).
constexpr int64_t kMarkGrid = 2048;
constexpr uint32_t kMarkFused = 16u;

// An append to a device-side list.  A captured cycle whose output outgrows
// its capacity keeps running (the host discards the result), so appends past
// the list's capacity are dropped rather than written.
__device__ inline void list_put(int32_t* __restrict__ l, int64_t i, int64_t cap, int32_t v) {
  if (i < cap) l[i] = v;
}

__global__ __launch_bounds__(kScanBig) void k_adapt(KeyGeom g, const uint64_t* __restrict__ in,
                                                  const int8_t* __restrict__ flags,
                                                  uint64_t* __restrict__ out, int64_t cap,
                                                  ScanState st, uint32_t* __restrict__ marks,
                                                  int32_t* __restrict__ elist, int64_t* nexam,
                                                  int64_t ecap, int32_t* __restrict__ flist,
                                                  int64_t* nflist, int64_t fcap) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = st.items.get();
  const int64_t base = tile * kTileMax + int64_t(threadIdx.x) * kItems;
  const int nc = g.nchild();
  uint64_t key[kItems];
  int act[kItems];  // 0 keep, 1 refine, 2 emit parent, 3 drop
  int64_t local = 0;
  unsigned err = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k;
    act[k] = 3;
    key[k] = 0;
    if (i >= n) continue;
    const uint64_t kk = in[i];
    key[k] = kk;
    int f = flags[i];
    if (f < -1 || f > 1) {
      err |= ERR_BAD_FLAG;
      f = 0;
    }
    const int d = key_depth(g, kk);
    int lo, hi;
    depth_limits(g, kk, &lo, &hi);
    if (f == 1 && d >= hi) f = 0;
    if (f == -1 && d <= lo) f = 0;
    int a = 0;
    if (f == 1) {
      a = 1;
    } else if (f == -1) {
      // The family is complete iff the 2^dim keys around i are exactly the
      // siblings (consecutive, same depth, raw IDs incrementing by one).
      const uint64_t m = key_m(g, kk);
      const int c = child_index(g, m, d);
      const int64_t h = i - c;
      const uint64_t step = uint64_t(1) << (g.dim * (g.dmax - d) + g.mb);
      const uint64_t k0 = kk - uint64_t(c) * step;
      bool all = h >= 0 && h + nc <= n;
      if (all) {
        // every sibling's key and flag loaded before any is compared: one
        // round trip instead of a chain of 2^dim dependent ones
        uint64_t sk[8];
        int sf[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < nc) {
            sk[j] = in[h + j];
            sf[j] = flags[h + j];
          }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < nc) all = all && sk[j] == k0 + uint64_t(j) * step && sf[j] == -1;
      }
      if (all) a = c == 0 ? 2 : 3;
    }
    act[k] = a;
    local += a == 1 ? nc : (a == 3 ? 0 : 1);
  }
  // the new children go on the list of leaves the first balance pass examines
  int64_t ex = 0, fx = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    ex += act[k] == 1 ? nc : 0;
    fx += act[k] == 2 ? 1 : 0;
  }
  int64_t eo = elist ? wave_append(ex, nexam) : 0;
  // the fused parents go on the list the first balance pass probes around
  int64_t fo = flist ? wave_append(fx, nflist) : 0;
  int64_t blk;
  const int64_t thr = block_exclusive<kScanBig>(local, &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int a = act[k];
    if (a == 3) continue;
    const int cnt = a == 1 ? nc : 1;
    if (o + cnt > cap) {
      err |= ERR_CAPACITY;
      // the slots below the capacity still get a valid key: the kernels after
      // this one in a captured cycle read them before the result is discarded
      for (int64_t q = o; q < cap && q < o + cnt; ++q) {
        out[q] = key[k];
        if (marks) marks[q] = 0u;
      }
      if (elist && a == 1)
        for (int c = 0; c < nc; ++c) list_put(elist, eo++, ecap, -1);
      if (flist && a == 2) list_put(flist, fo++, fcap, -1);
      o += cnt;
      continue;
    }
    const uint64_t kk = key[k];
    const int d = key_depth(g, kk);
    if (a == 0) {
      out[o] = kk;
      if (marks) marks[o] = 0u;
    } else if (a == 2) {
      out[o] = make_key(g, key_m(g, kk), d - 1);
      if (marks) marks[o] = kMarkFused;
      if (flist) list_put(flist, fo++, fcap, int32_t(o));
    } else {
      const uint64_t m = key_m(g, kk);
      for (int c = 0; c < nc; ++c) {
        out[o + c] = child_key(g, m, d, c);
        if (marks) marks[o + c] = kMarkExamine;
        if (elist) list_put(elist, eo++, ecap, int32_t(o + c));
      }
    }
    o += cnt;
  }
  if (err) atomicOr(st.err, err);
}

// 2:1 balance, marking pass.  For a leaf L of depth D with parent P, the
// leaves that touch L and are two or more levels coarser are exactly the
// leaves strictly containing one of the 2^dim - 1 depth-(D-1) neighbours of P
// around the vertex L shares with P (the searching keys of Section 3.2),
// restricted to face / face+edge neighbours for the weaker balance kinds.
// Such a leaf gets bit 0 (split); L gets bit 1 (check again next pass).
// Only leaves with bit 2 (new or re-checked) are examined unless check_all.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_balance_mark(KeyGeom g, const uint64_t* __restrict__ keys,
                                                         Count cn, KeyDir D, uint32_t* mark,
                                                         int check_all, DevCtr* ctr,
                                                         const unsigned* conv,
                                                         const int32_t* __restrict__ elist,
                                                         int64_t ecap) {
  // 2^DIM lanes per leaf, lane `sub` (1 .. 2^DIM - 1) probes one searching key;
  // waves stride over the (leaf, sub) pairs: every leaf (check_all), or the
  // listed leaves (elist: ctr->nexam entries, the leaves holding bit 2).
  // `conv` (captured cycles): the fixpoint was already reached, nothing to
  // examine.
  if (conv && *conv) return;
  constexpr int SL = 1 << DIM;
  const int64_t n = cn.get();
  const int64_t items = elist ? min(ctr->nexam, ecap) : n;
  const int64_t lanes = items * SL;
  const int lane = threadIdx.x & 63;
  const int limit = g.balance == 0 ? 1 : (g.balance == 1 ? 2 : 3);
  unsigned long long nfresh = 0;
  for (int64_t wb = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63); wb < lanes;
       wb += int64_t(gridDim.x) * blockDim.x) {
    const int64_t tid = wb + lane;
    const int64_t it = tid / SL;
    const int64_t i = elist ? (it < items ? int64_t(elist[it]) : -1) : it;
    const int sub = int(tid % SL);
    bool viol = false, fresh = false;
    if (i >= 0 && i < n && sub != 0 && __popc(unsigned(sub)) <= limit &&
        (check_all || (mark[i] & 4u))) {
      const uint64_t key = keys[i];
      const int d = key_depth(g, key);
      if (d >= 2) {
        uint64_t x[3];
        demorton(g, key_morton(g, key), x);
        const uint64_t mhi = key_mesh_bits(g, key) >> g.mb;
        const uint64_t S = uint64_t(1) << (g.dmax - d + 1);  // parent size
        uint64_t q[3] = {0, 0, 0};
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const uint64_t pa = x[a] & ~(S - 1);
          q[a] = pa;
          if ((sub >> a) & 1) {
            const bool up = (x[a] >> (g.dmax - d)) & 1;
            ok = ok && shift_coord(g, a, pa, up ? int64_t(S) : -int64_t(S), &q[a]);
          }
        }
        if (ok) {
          const int64_t j = dir_last_le(keys, n, D, point_key(g, morton(g, q) | mhi));
          if (j >= 0 && key_depth(g, keys[j]) < d - 1) {
            const uint32_t was = atomicOr(&mark[j], 1u);
            fresh = !(was & 1u);
            viol = true;
          }
        }
      }
    }
    const uint64_t vb = __ballot(viol);
    const uint64_t fb = __ballot(fresh);
    if (sub == 0 && i >= 0 && i < n && ((vb >> lane) & ((uint64_t(1) << SL) - 1)))
      atomicOr(&mark[i], 2u);
    nfresh += __popcll(fb);
  }
  if (lane == 0 && nfresh) atomicAdd(&ctr->nmarked, nfresh);
}

// 2:1 balance after adaptation, fused parents.  A parent P (depth D) that
// replaced 2^dim balanced leaves can touch leaves of depth D+2 (never deeper,
// never coarser than D-1 -- the leaves it replaced were balanced); those sit
// in the shell of depth-(D+2) cells around P.  Adapt lists the fused parents
// (any order, count ctr->nfused); one lane per (parent, shell cell) -- per the
// balance kind, cells across faces only, or also edges, or also corners --
// probes its cell and marks P for splitting on a depth-(D+2) leaf.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_fused_probe(KeyGeom g, const uint64_t* __restrict__ keys,
                                                        Count cn, KeyDir D,
                                                        const int32_t* __restrict__ list, uint32_t* mark,
                                                        DevCtr* ctr) {
  constexpr int W = 6;  // cells per axis around P: -1 .. 4 in units of a depth-(D+2) cell
  constexpr int NCELL = DIM == 3 ? W * W * W : W * W;
  const int64_t n = cn.get();
  const int64_t work = int64_t(ctr->nfused) * NCELL;
  const int limit = g.balance == 0 ? 1 : (g.balance == 1 ? 2 : 3);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < work;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = list[t / NCELL];
    const int cidx = int(t % NCELL);
    const int off[3] = {cidx % W - 1, (cidx / W) % W - 1, DIM == 3 ? cidx / (W * W) - 1 : 0};
    int outside = 0;
    for (int a = 0; a < DIM; ++a) outside += (off[a] < 0 || off[a] > 3) ? 1 : 0;
    if (outside == 0 || outside > limit || i < 0 || i >= n) continue;
    const uint64_t key = keys[i];
    const int d = key_depth(g, key);
    if (d + 2 > g.dmax) continue;
    uint64_t x[3];
    demorton(g, key_morton(g, key), x);
    const uint64_t mhi = key_mesh_bits(g, key) >> g.mb;
    const int64_t q4 = int64_t(1) << (g.dmax - d - 2);
    uint64_t q[3] = {x[0], x[1], x[2]};
    bool ok = true;
    for (int a = 0; a < DIM && ok; ++a) ok = shift_coord(g, a, x[a], int64_t(off[a]) * q4, &q[a]);
    if (!ok) continue;
    const int64_t j = dir_last_le(keys, n, D, point_key(g, morton(g, q) | mhi));
    if (j >= 0 && key_depth(g, keys[j]) >= d + 2) {
      const uint32_t was = atomicOr(&mark[i], 1u);
      if (!(was & 1u)) atomicAdd(&ctr->nmarked, 1ull);
    }
  }
}

// The fused-parent check of the first balance pass after adaptation.
hipError_t launch_fused_check(const KeyGeom& g, const uint64_t* keys, Count cn, const KeyDir& D,
                              uint32_t* mark, const int32_t* list, DevCtr* ctr, hipStream_t s) {
  constexpr int64_t kGrid = 2048;
  if (g.dim == 3)
    k_fused_probe<3><<<unsigned(kGrid), kBlock, 0, s>>>(g, keys, cn, D, list, mark, ctr);
  else
    k_fused_probe<2><<<unsigned(kGrid), kBlock, 0, s>>>(g, keys, cn, D, list, mark, ctr);
  return hipGetLastError();
}

// Radix directory of a sorted key array (see KeyDir): leaf i owns the
// buckets c with keys[i] <= c << shift < keys[i + 1].  Short spans are
// written by their own lane, long ones (coarse leaves) by the whole wave.
__global__ __launch_bounds__(256) void k_build_dir(const uint64_t* __restrict__ keys, Count cn,
                                                   int shift, int64_t nb, int32_t* __restrict__ d,
                                                   const unsigned* conv) {
  if (conv && *conv) return;  // captured cycles: keys unchanged since the last build
  const int64_t n = cn.get();
  const int lane = threadIdx.x & 63;
  auto ceil_sh = [shift](uint64_t k) -> int64_t {
    const uint64_t mask = (uint64_t(1) << shift) - 1;
    return int64_t(k >> shift) + ((k & mask) ? 1 : 0);
  };
  for (int64_t wb = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63); wb < n;
       wb += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = wb + lane;
    int64_t c0 = 0, c1 = 0;
    if (i < n) {
      c0 = ceil_sh(keys[i]);
      c1 = i + 1 < n ? ceil_sh(keys[i + 1]) : nb + 1;
      c1 = c1 < nb + 1 ? c1 : nb + 1;
      c0 = c0 < c1 ? c0 : c1;
      if (i == 0)
        for (int64_t c = 0, e = c0; c < e; ++c) d[c] = -1;
    }
    const bool big = c1 - c0 > 8;
    if (!big)
      for (int64_t c = c0; c < c1; ++c) d[c] = int32_t(i);
    uint64_t bm = __ballot(big);
    while (bm) {
      const int l = __ffsll((unsigned long long)bm) - 1;
      bm &= bm - 1;
      const int64_t a = __shfl(c0, l), b = __shfl(c1, l), v = __shfl(i, l);
      for (int64_t c = a + lane; c < b; c += 64) d[c] = int32_t(v);
    }
  }
}

// 2:1 balance, refinement pass: split bit-0 leaves one level, in order.  The
// new mark array holds bit 2 for leaves to examine next pass: the children of
// split leaves and the leaves that found a violation.
__global__ __launch_bounds__(kScanBig) void k_balance_refine(KeyGeom g, const uint64_t* __restrict__ in,
                                                           const uint32_t* __restrict__ mark,
                                                           uint64_t* __restrict__ out,
                                                           uint32_t* __restrict__ mark_out, int64_t cap,
                                                           ScanState st, const unsigned* conv,
                                                           int32_t* __restrict__ elist, int64_t* nexam,
                                                           int64_t ecap) {
  if (conv && *conv) {
    // captured cycles past the fixpoint: the pass is the identity, a plain copy
    const int64_t n = st.items.get();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = int64_t(blockIdx.x) * kTileMax + int64_t(k) * kScanBig + threadIdx.x;
      if (i < n) {
        out[i] = in[i];
        mark_out[i] = 0u;
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_total(st, n);
    return;
  }
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = st.items.get();
  const int64_t base = tile * kTileMax + int64_t(threadIdx.x) * kItems;
  const int nc = g.nchild();
  uint32_t w[kItems];
  uint64_t key[kItems];  // read with the marks, ahead of the look-back
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k;
    w[k] = 0;
    key[k] = 0;
    if (i >= n) continue;
    w[k] = mark[i] | 8u;  // bit 3: valid item
    key[k] = in[i];
    local += (w[k] & 1u) ? nc : 1;
  }
  // leaves the next pass examines (bit 2): the children of split leaves and
  // the leaves that found a violation, also put on the examine list
  int64_t ex = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (w[k] & 8u) ex += (w[k] & 1u) ? nc : ((w[k] & 2u) ? 1 : 0);
  int64_t eo = wave_append(ex, nexam);
  int64_t blk;
  const int64_t thr = block_exclusive<kScanBig>(local, &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
  unsigned err = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (!(w[k] & 8u)) continue;
    const uint64_t kk = key[k];
    const int cnt = (w[k] & 1u) ? nc : 1;
    const int nex = (w[k] & 1u) ? nc : ((w[k] & 2u) ? 1 : 0);
    if (o + cnt > cap) {
      err |= ERR_CAPACITY;
      for (int64_t q = o; q < cap && q < o + cnt; ++q) {  // valid keys below the capacity
        out[q] = kk;
        mark_out[q] = 0u;
      }
      for (int c = 0; c < nex; ++c) list_put(elist, eo++, ecap, -1);
      o += cnt;
      continue;
    }
    if (w[k] & 1u) {
      const uint64_t m = key_m(g, kk);
      const int d = key_depth(g, kk);
      for (int c = 0; c < nc; ++c) {
        out[o + c] = child_key(g, m, d, c);
        mark_out[o + c] = 4u;
        list_put(elist, eo++, ecap, int32_t(o + c));
      }
    } else {
      out[o] = kk;
      mark_out[o] = (w[k] & 2u) ? 4u : 0u;
      if (w[k] & 2u) list_put(elist, eo++, ecap, int32_t(o));
    }
    o += cnt;
  }
  if (err) atomicOr(st.err, err);
}

// Face connectivity (Section 3.3).  For face f = 2a + side the same-size box
// across the face is located by the leaf that holds its anchor: depth <= D
// means that leaf holds the whole box; deeper means the box is subdivided and
// e is the coarse side of a hanging face, whose 2^(dim-1) fine leaves are the
// box's children on the side facing e.
//
// Pass 1: one lane per (leaf, face), 2^DIM lanes per leaf (2D: 4, 3D: 8, two
// idle); nbr rows are written coalesced and each leaf's hanging faces become
// a bit mask.
template <int DIM>
__global__ __launch_bounds__(256) void k_connect_faces(KeyGeom g, const uint64_t* __restrict__ keys,
                                                       Count cn, KeyDir D, int32_t* __restrict__ nbr,
                                                       uint8_t* __restrict__ hmask) {
  constexpr int SL = 1 << DIM, NF = 2 * DIM;
  const int64_t n = cn.get();
  const int64_t lanes = n * SL;
  const int lane = threadIdx.x & 63;
  for (int64_t wb = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63); wb < lanes;
       wb += int64_t(gridDim.x) * blockDim.x) {
    const int64_t tid = wb + lane;
    const int64_t e = tid / SL;
    const int f = int(tid % SL);
    bool hanging = false;
    if (e < n && f < NF) {
      const uint64_t key = keys[e];
      const int d = key_depth(g, key);
      uint64_t x[3];
      demorton(g, key_morton(g, key), x);
      const uint64_t mhi = key_mesh_bits(g, key) >> g.mb;
      const int64_t sz = int64_t(1) << (g.dmax - d);
      const int a = f >> 1;
      uint64_t q[3] = {x[0], x[1], x[2]};
      int32_t v;
      if (!shift_coord(g, a, x[a], (f & 1) ? sz : -sz, &q[a])) {
        v = -2;
      } else {
        const int64_t j = dir_last_le(keys, n, D, point_key(g, morton(g, q) | mhi));
        if (j < 0) {
          v = -2;  // unreachable for a complete tree (keys[0] has anchor 0)
        } else if (key_depth(g, keys[j]) <= d) {
          v = int32_t(j);
        } else {
          v = -1;
          hanging = true;
        }
      }
      nbr[e * NF + f] = v;
    }
    const uint64_t hb = __ballot(hanging);
    if (f == 0 && e < n) hmask[e] = uint8_t((hb >> lane) & ((1u << SL) - 1));
  }
}

// Pass 2: hanging-face rows in (leaf, face) order: count from the masks,
// decoupled look-back scan, then each row's leaf and face.
__global__ __launch_bounds__(kScanSmall) void k_connect_rows(const uint8_t* __restrict__ hmask, int dim,
                                                         int32_t* __restrict__ hang, int64_t cap_rows,
                                                         ScanState st) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = st.items.get();
  const int64_t base = tile * kTileMin + int64_t(threadIdx.x) * kItems;
  const int nf = 2 * dim;
  const int width = 2 + (1 << (dim - 1));
  uint64_t hm8 = 0;  // kItems masks, one byte each
  if (base + kItems <= n) {
    hm8 = *reinterpret_cast<const uint64_t*>(hmask + base);
  } else {
    for (int k = 0; k < kItems; ++k)
      if (base + k < n) hm8 |= uint64_t(hmask[base + k]) << (8 * k);
  }
  int64_t blk;
  const int64_t thr = block_exclusive<kScanSmall>(__popcll(hm8), &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
  for (int k = 0; k < kItems && hm8; ++k) {
    const unsigned hm = unsigned(hm8 >> (8 * k)) & 0xffu;
    for (int f = 0; f < nf; ++f) {
      if (!((hm >> f) & 1u)) continue;
      if (o < cap_rows) {  // else the host grows the table and runs this pass again
        hang[o * width] = int32_t(base + k);
        hang[o * width + 1] = f;
      }
      o++;
    }
  }
}

// Pass 3: one lane per (row, slot): the fine leaf of the hanging face.  Slot
// bits are the tangential child bits in axis order, lower axis first; the
// fine leaves are the children of the same-size box on the side facing e.
__global__ __launch_bounds__(256) void k_connect_fine(KeyGeom g, const uint64_t* __restrict__ keys,
                                                      Count cn, KeyDir D, int32_t* __restrict__ hang,
                                                      const int64_t* total, int64_t cap_rows,
                                                      unsigned* err) {
  const int64_t n = cn.get();
  const int nh = 1 << (g.dim - 1);
  const int width = 2 + nh;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = tid / nh;
  const int slot = int(tid % nh);
  const int64_t rows = *total < cap_rows ? *total : cap_rows;  // rows the table holds
  if (r >= rows) return;
  int32_t* row = hang + r * width;
  const int64_t e = row[0];
  const int f = row[1];
  if (e < 0 || e >= n || f < 0 || f >= 2 * g.dim) {
    atomicOr(err, ERR_UNBALANCED);
    row[2 + slot] = -1;
    return;
  }
  const uint64_t key = keys[e];
  const int d = key_depth(g, key);
  uint64_t x[3];
  demorton(g, key_morton(g, key), x);
  const uint64_t mhi = key_mesh_bits(g, key) >> g.mb;
  const int64_t sz = int64_t(1) << (g.dmax - d);
  const int a = f >> 1, side = f & 1;
  uint64_t q[3] = {x[0], x[1], x[2]};
  shift_coord(g, a, x[a], side ? sz : -sz, &q[a]);
  int c = (1 - side) << a, j = 0;
  for (int t = 0; t < g.dim; ++t) {
    if (t == a) continue;
    c |= ((slot >> j) & 1) << t;
    ++j;
  }
  const uint64_t ck = child_key(g, morton(g, q) | mhi, d, c);
  const int64_t idx = dir_last_le(keys, n, D, ck);
  if (idx < 0 || keys[idx] != ck) {
    atomicOr(err, ERR_UNBALANCED);
    row[2 + slot] = -1;
  } else {
    row[2 + slot] = int32_t(idx);
  }
}

// Old -> new mapping (Section 4.2): lower bound B of each new key in the old
// tree, then the case it falls in.  old(i) reads old key i.
template <class Old>
__device__ inline void map_case(KeyGeom g, const Old& old, int64_t n_old, uint64_t key, int64_t B,
                                int64_t j, int32_t* __restrict__ src, int8_t* __restrict__ kind,
                                unsigned* err) {
  const int d = key_depth(g, key);
  if (B < n_old && old(B) == key) {
    src[j] = int32_t(B);
    kind[j] = 0;
    return;
  }
  if (B > 0 && d > 0) {
    const uint64_t pk = old(B - 1);
    const uint64_t m = key_m(g, key);
    const uint64_t pm = key_m(g, pk);
    if (key_depth(g, pk) == d - 1 && (m & ~(span(g, d - 1) - 1)) == pm) {
      src[j] = int32_t(B - 1);
      kind[j] = int8_t(1 + child_index(g, m, d));
      return;
    }
  }
  const int nc = g.nchild();
  if (B + nc <= n_old && old(B) == key + 1 && d < g.dmax) {
    const uint64_t last = child_key(g, key_m(g, key), d, nc - 1);
    if (old(B + nc - 1) == last) {
      src[j] = int32_t(B);
      kind[j] = -1;
      return;
    }
  }
  // fits none of the three cases (the old tree was not balanced): report it;
  // the entry stays a valid index so that a captured transfer reads in bounds
  src[j] = 0;
  kind[j] = 0;
  atomicOr(err, ERR_MAP);
}

// First indices of keys[0, n) >= pa and >= pb, found by the whole wave
// together (every lane passes the same two probes): each half of the wave
// probes 32 evenly spaced keys of its remaining range per round and keeps the
// one gap its probe falls in -- one memory round trip per round for both
// searches (five at 1.6M keys) instead of one per halving.
__device__ inline void wave_lower_bound2(const uint64_t* __restrict__ keys, int64_t n, uint64_t pa,
                                         uint64_t pb, int64_t* ra, int64_t* rb) {
  const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  const uint64_t probe = half ? pb : pa;
  int64_t lo = 0, hi = n;  // this half's bound lies in [lo, hi]
  for (;;) {
    const bool wide = hi - lo > 32;
    if (__ballot(wide) == 0) break;  // both halves narrow: the loop is left by the whole wave
    const int64_t step = wide ? (hi - lo + 31) / 32 : 1;
    const int64_t p = lo + int64_t(hl) * step;
    // the probes below the bound are a prefix of the half's lanes (the keys ascend)
    const uint64_t m = __ballot(p < hi && keys[p] < probe);
    const int c = __popc(unsigned(half ? (m >> 32) : m));
    if (wide) {
      if (c == 0) {
        hi = lo;
      } else {
        const int64_t nlo = lo + int64_t(c - 1) * step + 1;
        hi = std::min(hi, lo + int64_t(c) * step);
        lo = nlo;
      }
    }
  }
  const int64_t p = lo + hl;
  const uint64_t m = __ballot(p < hi && keys[p] < probe);
  const int64_t r = lo + __popc(unsigned(half ? (m >> 32) : m));
  *ra = __shfl(r, 0);
  *rb = __shfl(r, 32);
}

__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave maps 64 consecutive new keys.  Their lower bounds lie between those
// of the wave's first and last key, found by one cooperative search; the
// old keys around that range (the case checks read B - 1 and B + 2^d - 1) go
// to the wave's LDS window in one coalesced load, and each lane bisects its
// own bound there.  A range wider than the window is bisected in memory.
constexpr int kMapWin = 640;
__global__ __launch_bounds__(kBlock) void k_map(KeyGeom g, const uint64_t* __restrict__ old_keys,
                                                Count cn_old, const uint64_t* __restrict__ keys,
                                                Count cn, int32_t* __restrict__ src,
                                                int8_t* __restrict__ kind, unsigned* err) {
  __shared__ uint64_t win[kBlock / 64][kMapWin];
  const int64_t n_old = cn_old.get(), n = cn.get();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nc = g.nchild();
  uint64_t* W = win[wv];
  for (int64_t wb = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63); wb < n;
       wb += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = wb + lane;
    const bool live = j < n;
    const uint64_t key = keys[live ? j : n - 1];  // lanes past the end repeat the last key
    int64_t bf, bl;
    wave_lower_bound2(old_keys, n_old, __shfl(key, 0), __shfl(key, 63), &bf, &bl);
    const int64_t w0 = bf > 0 ? bf - 1 : 0;
    const int64_t w1 = std::min(bl + nc, n_old);
    if (w1 - w0 <= kMapWin) {
      for (int64_t q = w0 + lane; q < w1; q += 64) W[q - w0] = old_keys[q];
      wave_lds_fence();
      int64_t lo = bf, hi = bl;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (W[mid - w0] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (live) map_case(g, [&](int64_t i) { return W[i - w0]; }, n_old, key, lo, j, src, kind, err);
      wave_lds_fence();  // every lane done with the window before the next one overwrites it
    } else {
      int64_t lo = bf, hi = bl;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (old_keys[mid] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (live) map_case(g, [&](int64_t i) { return old_keys[i]; }, n_old, key, lo, j, src, kind, err);
    }
  }
}


// ------------------------------------------------------------------ host helpers
}  // namespace

void dir_params(const KeyGeom& g, int64_t n, int* shift, int64_t* nb) {
  int kb = g.mesh_shift;
  if (g.nmesh > 1) {
    int mbits = 0;
    while ((int64_t(1) << mbits) < g.nmesh) ++mbits;
    kb += mbits;
  }
  kb = std::min(kb, 64);
  int L = 0;
  while (L < 62 && (int64_t(1) << L) < n) ++L;
  L = std::max(10, std::min(24, L - 1));
  L = std::min(L, kb);
  *shift = kb - L;
  // The buckets end with the last mesh's key range (nmesh << mesh_shift),
  // not at the next power of two of the mesh count: otherwise the last leaf
  // would own every bucket of the empty mesh slots.
  const int ms = g.mesh_shift;
  const int64_t nm = std::max(1, g.nmesh);
  if (*shift <= ms)
    *nb = nm << (ms - *shift);
  else
    *nb = (nm + (int64_t(1) << (*shift - ms)) - 1) >> (*shift - ms);
}

lt_status prep_scan_fixed(uint64_t* status, int64_t status_cap, DevCtr* ctr, int64_t n_items,
                          int64_t tile, hipStream_t stream, int flags, ScanState* st, int64_t* cnt_dst,
                          const int64_t* cnt_src) {
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(n_items, tile));
  if (ntiles > status_cap) return fail(LT_ERR_ARG, "scan needs more look-back words than provided");
  k_clear_scan<<<unsigned(ceil_div(ntiles, 256)), 256, 0, stream>>>(
      status, ntiles, ctr, flags & 1, (flags >> 1) & 1, (flags >> 2) & 1, (flags >> 3) & 1, cnt_dst,
      cnt_src);
  LT_HIP(hipGetLastError());
  st->status = status;
  st->ticket = &ctr->ticket;
  st->err = &ctr->err;
  st->total = &ctr->total;
  st->items = Count{n_items, nullptr};
  st->tile = tile;
  st->commit = nullptr;
  st->commit_cap = 0;
  return LT_OK;
}

namespace {
lt_status prep_scan_on(const Alloc& A, uint64_t** status, int64_t* status_cap, DevCtr* ctr,
                       int64_t n_items, int64_t tile, hipStream_t stream, int flags, ScanState* st,
                       int64_t* cnt_dst = nullptr, const int64_t* cnt_src = nullptr) {
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(n_items, tile));
  LT_TRY(grow(A, status, status_cap, ntiles));
  return prep_scan_fixed(*status, *status_cap, ctr, n_items, tile, stream, flags, st, cnt_dst, cnt_src);
}
}  // namespace

lt_status prep_scan(lt_tree t, int64_t n_items, int64_t tile, hipStream_t stream, int flags,
                    ScanState* st, int64_t* cnt_dst, const int64_t* cnt_src) {
  return prep_scan_on(t->A, &t->status, &t->status_cap, t->dctr, n_items, tile, stream, flags, st,
                      cnt_dst, cnt_src);
}

lt_status prep_scan_conn(lt_tree t, int64_t n_items, hipStream_t stream, int flags, ScanState* st) {
  return prep_scan_on(t->A, &t->cstatus, &t->cstatus_cap, t->cctr, n_items, kTileMin, stream, flags,
                      st);
}

lt_status read_ctr(lt_tree t, hipStream_t stream) {
  LT_HIP(hipMemcpyAsync(t->hctr, t->dctr, sizeof(DevCtr), hipMemcpyDeviceToHost, stream));
  LT_HIP(hipStreamSynchronize(stream));
  return LT_OK;
}

lt_status clear_err(lt_tree t, hipStream_t stream) {
  k_clear_scan<<<1, 64, 0, stream>>>(t->status, 0, t->dctr, 1, 0, 0, 0, nullptr, nullptr);
  LT_HIP(hipGetLastError());
  return LT_OK;
}

namespace {

lt_status check_geom(const lt_geom* g) {
  if (!g) return fail(LT_ERR_ARG, "geom is NULL");
  if (g->dim != 2 && g->dim != 3) return fail(LT_ERR_ARG, "dim must be 2 or 3");
  if (g->d_max < 1 || g->d_min < 0 || g->d_min > g->d_max)
    return fail(LT_ERR_DEPTH, "need 0 <= d_min <= d_max and d_max >= 1");
  int mb = 0;
  while ((g->d_max >> mb) != 0) ++mb;
  if (g->dim * g->d_max + mb > 64) return fail(LT_ERR_DEPTH, "dim*d_max + bitlength(d_max) > 64");
  if (g->dim == 3 && g->d_max > 21) return fail(LT_ERR_DEPTH, "3D d_max above 21");
  if (g->balance < 0 || g->balance > 2) return fail(LT_ERR_ARG, "balance must be 0, 1 or 2");
  return LT_OK;
}

lt_status new_tree(const lt_geom* geom, lt_tree* out) {
  LT_TRY(check_geom(geom));
  if (!out) return fail(LT_ERR_ARG, "out is NULL");
  lt_tree t = new lt_tree_s;
  int mb = 0;
  while ((geom->d_max >> mb) != 0) ++mb;
  t->g.dim = geom->dim;
  t->g.dmax = geom->d_max;
  t->g.dmin = geom->d_min;
  t->g.mb = mb;
  t->g.periodic = geom->periodic_mask & ((1u << geom->dim) - 1);
  t->g.balance = geom->balance;
  t->g.mesh_shift = mb + geom->dim * geom->d_max;
  t->g.nmesh = 1;
  t->g.lim = nullptr;
  t->A = registered_alloc();
  hipError_t e = hipGetDevice(&t->device);
  if (e == hipSuccess) e = dev_malloc(t->A, reinterpret_cast<void**>(&t->dctr), sizeof(DevCtr));
  if (e == hipSuccess) e = hipHostMalloc(&t->hctr, sizeof(DevCtr), hipHostMallocDefault);
  if (e == hipSuccess) e = dev_malloc(t->A, reinterpret_cast<void**>(&t->cctr), sizeof(DevCtr));
  if (e == hipSuccess) e = hipHostMalloc(&t->hcctr, sizeof(DevCtr), hipHostMallocDefault);
  if (e != hipSuccess) {
    lt_destroy(t);
    return fail(e == hipErrorOutOfMemory ? LT_ERR_OOM : LT_ERR_HIP,
                std::string("tree setup: ") + hipGetErrorString(e));
  }
  std::memset(t->hctr, 0, sizeof(DevCtr));
  std::memset(t->hcctr, 0, sizeof(DevCtr));
  e = hipMemset(t->dctr, 0, sizeof(DevCtr));
  if (e == hipSuccess) e = hipMemset(t->cctr, 0, sizeof(DevCtr));
  if (e != hipSuccess) {
    lt_destroy(t);
    return fail(LT_ERR_HIP, std::string("tree setup: ") + hipGetErrorString(e));
  }
  *out = t;
  return LT_OK;
}

void invalidate(lt_tree t) {
  t->dir_valid = false;
  t->conn_valid = false;
  t->n_hang = -1;
  t->map_valid = false;
}

// Radix directory of the current keys (see KeyDir): about one bucket per
// two leaves (2^10 .. 2^24 buckets) over the range the keys can take.
lt_status ensure_dir(lt_tree t, hipStream_t s, KeyDir* D) {
  const int64_t n = t->n_cur;
  if (!t->dir_valid) {
    dir_params(t->g, n, &t->dir_shift, &t->dir_nb);
    LT_TRY(grow(t->A, &t->dir, &t->dir_cap, t->dir_nb + 1));
    if (n > 0) {
      k_build_dir<<<unsigned(ceil_div(n, 256)), 256, 0, s>>>(t->kbuf[t->cur], Count{n, nullptr},
                                                             t->dir_shift, t->dir_nb, t->dir, nullptr);
      LT_HIP(hipGetLastError());
    }
    t->dir_valid = true;
  }
  D->d = t->dir;
  D->shift = t->dir_shift;
  D->nb = t->dir_nb;
  return LT_OK;
}

lt_status do_map(lt_tree t, hipStream_t stream) {
  if (!t->has_old) return fail(LT_ERR_STATE, "lt_map needs a prior lt_adapt");
  LT_TRY(grow(t->A, &t->map_src, &t->map_cap, t->n_cur));
  LT_TRY(grow(t->A, &t->map_kind, &t->kind_cap, t->n_cur));
  LT_TRY(clear_err(t, stream));
  if (t->n_cur > 0)
    k_map<<<unsigned(ceil_div(t->n_cur, kBlock)), kBlock, 0, stream>>>(
        t->g, t->kbuf[t->old], Count{t->n_old, nullptr}, t->kbuf[t->cur], Count{t->n_cur, nullptr},
        t->map_src, t->map_kind, &t->dctr->err);
  LT_HIP(hipGetLastError());
  LT_TRY(read_ctr(t, stream));
  if (t->hctr->err & ERR_MAP)
    return fail(LT_ERR_UNBALANCED,
                "a new leaf is neither an old leaf, a child of one, nor a parent of 2^dim old leaves");
  if (t->hctr->err) return fail(LT_ERR_INTERNAL, "device check failed in lt_map");
  t->map_valid = true;
  return LT_OK;
}

// ---------------------------------------------------------- captured cycles
// Single-thread bookkeeping kernels of a cycle whose counts stay on the device.

// After the balance passes: marks left mean the fixed passes did not reach
// the fixpoint; and the transfer's groups of 64 leaves, ceil(S[0] / 64), the
// count being final here.
__global__ void k_check_marks(DevCtr* ctr, int64_t* groups, const int64_t* n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (ctr->nmarked != 0) atomicOr(&ctr->err, ERR_BALANCE_PASSES);
    *groups = (*n + 63) / 64;
  }
}

// Also folds connectivity's error word (its branch ran on a side stream)
// into the cycle's.
__global__ void k_copy_keys(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, Count cn,
                            unsigned* err, const unsigned* cerr) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const unsigned ce = *cerr;
  if (i == 0 && ce != 0) atomicOr(err, ce);
  if ((*err | ce) != 0) return;  // keep the pre-cycle keys for the host's recovery
  if (i < cn.get()) dst[i] = src[i];
}

}  // namespace

lt_status record_cycle(lt_tree_s* t, const CycleRec& r, hipStream_t s) {
  const KeyGeom& g = t->g;
  const int64_t C = r.cap;
  int64_t* S = r.dsz;
  uint64_t* K0 = t->kbuf[0];
  uint64_t* K[2] = {t->kbuf[1], t->kbuf[2]};
  const unsigned nb256 = unsigned(ceil_div(C, 256));
  // the search kernels stride over their work: a bounded grid, whatever the capacity
  constexpr int64_t kStrideGrid = 4096;
  const unsigned nlanes = unsigned(std::min<int64_t>(ceil_div(C * g.nchild(), 256), kStrideGrid));
  const unsigned nleaf = unsigned(std::min<int64_t>(ceil_div(C, 256), kStrideGrid));
  const unsigned* conv = &t->dctr->conv;
  unsigned* err = &t->dctr->err;
  int8_t* F = t->map_kind;  // the flags live in the kind array until the mapping overwrites it
  // flags (parameters from the device table)
  LT_TRY(launch_flag_table(g, r.tmpl, r.nmesh, t->flag_tab, K0, Count{C, &S[0]}, F, s));
  if (r.mlp)  // learned flags, the geometric ones as the fallback below conf_min
    LT_TRY(launch_mlp_flag(t, r.mlp, Count{C, &S[0]}, r.uo, r.ld, r.conf_min, F, nullptr, s));
  // adapt K0 -> K[0]; its scan's clear also starts the cycle: leaves before
  // the cycle S[1] <- S[0], the fixpoint flag cleared
  ScanState st;
  LT_TRY(prep_scan(t, C, kTileMax, s, 1 | 4 | 8, &st, &S[1], &S[0]));
  st.items.p = &S[1];
  st.commit = &S[0];
  st.commit_cap = C;
  k_adapt<<<grid_tiles(st), kScanBig, 0, s>>>(g, K0, F, K[0], C, st, t->mbuf[0], t->elist,
                                              &t->dctr->nexam, t->elist_cap, t->fused,
                                              &t->dctr->nfused, t->fused_cap);
  LT_HIP(hipGetLastError());
  // balance: fixed passes, then a check
  // (the tree entering the cycle is balanced, so adapt's marks restrict the
  // first pass to new children and fused parents)
  const KeyDir D{t->dir, r.dir_shift, r.dir_nb};
  int ki = 0, mi = 0;
  for (int pass = 0; pass <= r.passes; ++pass) {
    k_build_dir<<<nleaf, 256, 0, s>>>(K[ki], Count{C, &S[0]}, r.dir_shift, r.dir_nb, t->dir, conv);
    if (pass == 0)
      LT_HIP(launch_fused_check(g, K[ki], Count{C, &S[0]}, D, t->mbuf[mi], t->fused, t->dctr, s));
    const unsigned mgrid = unsigned(std::min<int64_t>(nlanes, kMarkGrid));
    if (g.dim == 3)
      k_balance_mark<3><<<mgrid, kBlock, 0, s>>>(g, K[ki], Count{C, &S[0]}, D, t->mbuf[mi], 0,
                                                 t->dctr, conv, t->elist, t->elist_cap);
    else
      k_balance_mark<2><<<mgrid, kBlock, 0, s>>>(g, K[ki], Count{C, &S[0]}, D, t->mbuf[mi], 0,
                                                 t->dctr, conv, t->elist, t->elist_cap);
    if (pass == r.passes) break;
    // the clear also records convergence, and copies the pass's input count
    // to S[4], where the pass reads it: the last tile commits the new count
    // to S[0] while workgroups of the capacity-sized grid may still be taking
    // tickets, and each must see the count the scan started from
    LT_TRY(prep_scan(t, C, kTileMax, s, 2 | 4, &st, &S[4], &S[0]));
    st.items.p = &S[4];
    st.commit = &S[0];
    st.commit_cap = C;
    k_balance_refine<<<grid_tiles(st), kScanBig, 0, s>>>(g, K[ki], t->mbuf[mi], K[1 - ki],
                                                        t->mbuf[1 - mi], C, st, conv, t->elist,
                                                        &t->dctr->nexam, t->elist_cap);
    ki = 1 - ki;
    mi = 1 - mi;
  }
  k_check_marks<<<1, 64, 0, s>>>(t->dctr, &S[3], &S[0]);
  LT_HIP(hipGetLastError());
  if (ki != 0) return fail(LT_ERR_ARG, "balance passes of a captured cycle must be even");
  // map
  k_map<<<nleaf, kBlock, 0, s>>>(g, K0, Count{C, &S[1]}, K[0], Count{C, &S[0]}, t->map_src,
                                  t->map_kind, err);
  LT_HIP(hipGetLastError());
  // connect on the side stream (the directory of K[0] was built by the check
  // pass); it reads the new keys only, and its scan words and counters are its
  // own, so it runs beside the transfer (forked after the mapping, which runs
  // alone: beside connectivity's searches it took three times as long)
  hipStream_t cs = r.side;
  LT_HIP(hipEventRecord(r.fork, s));
  LT_HIP(hipStreamWaitEvent(cs, r.fork, 0));
  const unsigned cgrid = t->conn_grid > 0 ? std::min<unsigned>(nlanes, unsigned(t->conn_grid)) : nlanes;
  if (g.dim == 3)
    k_connect_faces<3><<<cgrid, 256, 0, cs>>>(g, K[0], Count{C, &S[0]}, D, t->nbr, t->hmask);
  else
    k_connect_faces<2><<<cgrid, 256, 0, cs>>>(g, K[0], Count{C, &S[0]}, D, t->nbr, t->hmask);
  ScanState cst;
  LT_TRY(prep_scan_conn(t, C, cs, 1, &cst));
  cst.items.p = &S[0];
  cst.commit = &S[2];  // rows past the table's capacity raise ERR_CAPACITY
  cst.commit_cap = r.hang_rows;
  k_connect_rows<<<grid_tiles(cst), kScanSmall, 0, cs>>>(t->hmask, g.dim, t->hang, r.hang_rows, cst);
  const int nh = 1 << (g.dim - 1);
  k_connect_fine<<<unsigned(ceil_div(r.hang_rows * nh, 256)), 256, 0, cs>>>(
      g, K[0], Count{C, &S[0]}, D, t->hang, &t->cctr->total, r.hang_rows, &t->cctr->err);
  LT_HIP(hipGetLastError());
  LT_HIP(hipEventRecord(r.join, cs));
  // transfer
  if (r.precision == 1) {
    LT_TRY(launch_split_transfer(t, Count{C, &S[0]}, r.p, r.nvar, r.uo, r.ld, r.un, r.ld, s));
  } else if (r.p < 0) {  // per-mesh degrees
    LT_TRY(launch_transfer_mixed(t, K[0], Count{C, &S[0]}, &S[3], r.nvar, r.uo, r.ld, r.un, r.ld, s));
  } else {
    LT_TRY(launch_transfer(t, Count{C, &S[0], t->n_cur}, &S[3], r.p, r.ops, r.nvar, r.uo, r.ld, r.un, r.ld, s));
  }
  // the new keys become the next cycle's input, once connectivity is done
  LT_HIP(hipStreamWaitEvent(s, r.join, 0));
  k_copy_keys<<<nb256, 256, 0, s>>>(K[0], K0, Count{C, &S[0]}, err, &t->cctr->err);
  LT_HIP(hipGetLastError());
  return LT_OK;
}

namespace {

}  // namespace
// A new tree with no leaves yet (geometry checked, allocator and counters set
// up), for the translation units that build trees of their own.
lt_status create_tree(const lt_geom* geom, lt_tree* out) { return new_tree(geom, out); }

}  // namespace lt

using namespace lt;

// =================================================================== C ABI
extern "C" {

const char* lt_last_error(void) { return lt::g_err.c_str(); }

lt_status lt_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                           void (*free_)(void* ptr, void* stream, void* ctx), void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr))
    return fail(LT_ERR_ARG, "alloc and free must both be set or both be NULL");
  Alloc A;
  A.alloc = alloc;
  A.free_ = free_;
  A.ctx = alloc ? ctx : nullptr;
  register_alloc(A);
  return LT_OK;
}

lt_status lt_build_uniform(const lt_geom* geom, int depth, void* stream, lt_tree* out) {
  lt_tree t = nullptr;
  LT_TRY(new_tree(geom, &t));
  if (depth < 0 || depth > geom->d_max) {
    lt_destroy(t);
    return fail(LT_ERR_DEPTH, "uniform depth outside [0, d_max]");
  }
  if (geom->dim * depth > 40) {
    lt_destroy(t);
    return fail(LT_ERR_ARG, "uniform tree too large");
  }
  const int64_t n = int64_t(1) << (geom->dim * depth);
  hipStream_t s = static_cast<hipStream_t>(stream);
  lt_status st = grow(t->A, &t->kbuf[t->cur], &t->kcap[t->cur], n);
  if (st != LT_OK) {
    lt_destroy(t);
    return st;
  }
  k_uniform<<<unsigned(ceil_div(n, kBlock)), kBlock, 0, s>>>(t->g, depth, n, t->kbuf[t->cur]);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    lt_destroy(t);
    return fail(LT_ERR_HIP, std::string("uniform build: ") + hipGetErrorString(e));
  }
  t->n_cur = n;
  t->balanced = true;  // uniform per mesh
  *out = t;
  return LT_OK;
}

lt_status lt_build(const lt_geom* geom, const uint64_t* keys, int64_t n, void* stream, lt_tree* out) {
  if (!keys || n < 1) return fail(LT_ERR_ARG, "keys must be a non-empty device array");
  lt_tree t = nullptr;
  LT_TRY(new_tree(geom, &t));
  hipStream_t s = static_cast<hipStream_t>(stream);
  lt_status st = grow(t->A, &t->kbuf[t->cur], &t->kcap[t->cur], n);
  if (st != LT_OK) {
    lt_destroy(t);
    return st;
  }
  hipError_t e = hipMemcpyAsync(t->kbuf[t->cur], keys, size_t(n) * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) {
    k_validate<<<unsigned(ceil_div(n, kBlock)), kBlock, 0, s>>>(t->g, t->kbuf[t->cur], n,
                                                                 &t->dctr->err);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(t->hctr, t->dctr, sizeof(DevCtr), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    lt_destroy(t);
    return fail(LT_ERR_HIP, std::string("build: ") + hipGetErrorString(e));
  }
  if (t->hctr->err) {
    lt_destroy(t);
    return fail(LT_ERR_INVALID_TREE, "keys are not the ascending IDs of a complete linear tree");
  }
  t->n_cur = n;
  *out = t;
  return LT_OK;
}

lt_status lt_build_batch(const lt_geom* geom, int nmesh, const int* d_min, const int* d_max,
                         const int* depth, void* stream, lt_tree* out) {
  if (!geom || !d_min || !d_max || !depth || !out || nmesh < 1)
    return fail(LT_ERR_ARG, "NULL argument or no mesh");
  lt_geom g0 = *geom;
  g0.d_min = 0;
  LT_TRY(check_geom(&g0));
  int mb = 0;
  while ((geom->d_max >> mb) != 0) ++mb;
  int mesh_bits = 0;
  while (((nmesh - 1) >> mesh_bits) != 0) ++mesh_bits;
  if (mb + geom->dim * geom->d_max + mesh_bits > 64)
    return fail(LT_ERR_DEPTH, "mesh index does not fit above the Morton bits");
  std::vector<int8_t> lim(2 * size_t(nmesh)), dep(nmesh);
  std::vector<int64_t> offs(size_t(nmesh) + 1, 0);
  for (int m = 0; m < nmesh; ++m) {
    if (d_min[m] < 0 || d_min[m] > d_max[m] || d_max[m] > geom->d_max || depth[m] < 0 ||
        depth[m] > geom->d_max)
      return fail(LT_ERR_DEPTH, "mesh " + std::to_string(m) + ": need 0 <= d_min <= d_max <= finest");
    if (geom->dim * depth[m] > 36) return fail(LT_ERR_ARG, "uniform mesh too large");
    lim[2 * m] = int8_t(d_min[m]);
    lim[2 * m + 1] = int8_t(d_max[m]);
    dep[m] = int8_t(depth[m]);
    offs[m + 1] = offs[m] + (int64_t(1) << (geom->dim * depth[m]));
  }
  const int64_t n = offs[nmesh];
  lt_tree t = nullptr;
  LT_TRY(new_tree(&g0, &t));
  hipStream_t s = static_cast<hipStream_t>(stream);
  int8_t* dep_dev = nullptr;
  lt_status st = grow(t->A, &t->kbuf[t->cur], &t->kcap[t->cur], n);
  hipError_t e = hipSuccess;
  if (st == LT_OK) {
    e = dev_malloc(t->A, reinterpret_cast<void**>(&t->lim), lim.size());
    if (e == hipSuccess)
      e = dev_malloc(t->A, reinterpret_cast<void**>(&t->mesh_offs), sizeof(int64_t) * (nmesh + 1));
    if (e == hipSuccess) e = dev_malloc(t->A, reinterpret_cast<void**>(&dep_dev), dep.size());
    if (e == hipSuccess) e = dev_malloc(t->A, &t->flag_tab, flag_args_size() * nmesh);
    if (e == hipSuccess)
      e = hipMemcpy(t->lim, lim.data(), lim.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dep_dev, dep.data(), dep.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(t->mesh_offs, offs.data(), sizeof(int64_t) * (nmesh + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      t->g.nmesh = nmesh;
      t->g.lim = t->lim;
      k_uniform_batch<<<unsigned(ceil_div(n, kBlock)), kBlock, 0, s>>>(t->g, t->mesh_offs, dep_dev,
                                                                        nmesh, n, t->kbuf[t->cur]);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
      st = fail(e == hipErrorOutOfMemory ? LT_ERR_OOM : LT_ERR_HIP,
                std::string("batch build: ") + hipGetErrorString(e));
  }
  (void)dev_free(t->A, dep_dev);
  if (st != LT_OK) {
    lt_destroy(t);
    return st;
  }
  t->n_cur = n;
  t->balanced = true;  // uniform per mesh
  *out = t;
  return LT_OK;
}

lt_status lt_flag_batch(lt_tree t, const lt_flag_params* per_mesh, int nmesh, int8_t* flags,
                        void* stream) {
  if (!t || !per_mesh || !flags) return fail(LT_ERR_ARG, "NULL argument");
  if (nmesh != t->g.nmesh || !t->flag_tab)
    return fail(LT_ERR_ARG, "nmesh must equal the ensemble's mesh count");
  return launch_flag_batch(t->g, per_mesh, nmesh, t->flag_tab, t->kbuf[t->cur], t->n_cur, flags,
                           static_cast<hipStream_t>(stream));
}

lt_status lt_mesh_offsets(lt_tree t, int64_t* offsets, void* stream) {
  if (!t || !offsets) return fail(LT_ERR_ARG, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nm = t->g.nmesh;
  if (!t->mesh_offs)
    if (dev_malloc(t->A, reinterpret_cast<void**>(&t->mesh_offs), sizeof(int64_t) * (nm + 1)) != hipSuccess)
      return fail(LT_ERR_OOM, "mesh offsets");
  k_mesh_offsets<<<unsigned(ceil_div(nm + 1, 64)), 64, 0, s>>>(t->g, t->kbuf[t->cur], t->n_cur, nm,
                                                                 t->mesh_offs);
  LT_HIP(hipGetLastError());
  LT_HIP(hipMemcpyAsync(offsets, t->mesh_offs, sizeof(int64_t) * (nm + 1), hipMemcpyDeviceToHost, s));
  LT_HIP(hipStreamSynchronize(s));
  return LT_OK;
}

lt_status lt_flag(lt_tree t, const lt_flag_params* fp, int8_t* flags, void* stream) {
  if (!t || !fp || !flags) return fail(LT_ERR_ARG, "NULL argument");
  if (t->g.nmesh > 1) return fail(LT_ERR_ARG, "an ensemble takes lt_flag_batch");
  return launch_flag(t->g, fp, t->kbuf[t->cur], t->n_cur, flags, static_cast<hipStream_t>(stream));
}

lt_status lt_adapt(lt_tree t, const int8_t* flags, void* stream) {
  if (!t || !flags) return fail(LT_ERR_ARG, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = t->n_cur;
  // Output bound: every leaf refined.  The output goes to whichever of the
  // two free key buffers already holds the bound: the buffers rotate roles
  // from cycle to cycle, and growing a small one costs a device-wide free and
  // allocation.  The old snapshot is left alone until the call has succeeded.
  const int64_t need = n * t->g.nchild();
  int out = t->tmp, spare = t->aux;
  if (t->kcap[out] < need && t->kcap[spare] >= need) std::swap(out, spare);
  if (t->kcap[out] < need) {
    // growing: grow the other free buffer with it, so that from now on one of
    // the free buffers holds the bound and steady cycles allocate nothing
    LT_TRY(grow(t->A, &t->kbuf[out], &t->kcap[out], need));
    LT_TRY(grow(t->A, &t->kbuf[spare], &t->kcap[spare], need));
  }
  // From a balanced tree, adapt also writes the first balance pass's marks.
  const bool marks = t->balanced;
  int64_t cap = t->kcap[out];
  if (marks) {
    LT_TRY(grow(t->A, &t->mbuf[0], &t->mcap[0], need));
    LT_TRY(grow(t->A, &t->elist, &t->elist_cap, need));
    LT_TRY(grow(t->A, &t->fused, &t->fused_cap, need));
    cap = std::min(cap, std::min(t->mcap[0], std::min(t->elist_cap, t->fused_cap)));
  }
  ScanState st;
  LT_TRY(prep_scan(t, n, kTileMax, s, 1 | 4, &st));
  k_adapt<<<grid_tiles(st), kScanBig, 0, s>>>(t->g, t->kbuf[t->cur], flags, t->kbuf[out], cap, st,
                                              marks ? t->mbuf[0] : nullptr,
                                              marks ? t->elist : nullptr, &t->dctr->nexam,
                                              t->elist_cap, marks ? t->fused : nullptr,
                                              &t->dctr->nfused, t->fused_cap);
  LT_HIP(hipGetLastError());
  LT_TRY(read_ctr(t, s));
  if (t->hctr->err & ERR_BAD_FLAG) return fail(LT_ERR_ARG, "flags must be -1, 0 or 1");
  if (t->hctr->err) return fail(LT_ERR_INTERNAL, "device check failed in lt_adapt");
  // old <- cur, cur <- the output, the other free buffer and the superseded
  // snapshot become the free ones
  const int prev_old = t->old;
  t->old = t->cur;
  t->cur = out;
  t->tmp = spare;
  t->aux = prev_old;
  t->n_old = n;
  t->n_cur = t->hctr->total;
  t->has_old = true;
  invalidate(t);
  t->balanced = false;
  t->adapt_marks = marks;
  return LT_OK;
}

}  // extern "C"

namespace {
// The balance fixpoint from the leaves in kbuf[t->cur].  Each refinement pass
// reads the current buffer and writes into one of the two free ones (tmp and
// aux in turn), then makes its output current; the buffer that held the
// leaves on entry is never written, so the caller can restore it.
lt_status balance_passes(lt_tree t, hipStream_t s) {
  // One host readback per pass (the number of leaves to split).  The refine
  // pass's own consistency checks land in the error word and are read with
  // the next pass's count.
  // The first pass examines every leaf, or -- right after adapt of a
  // balanced tree -- only the new children and the fused parents.
  int mi = 0;
  const bool restricted = t->adapt_marks && t->mcap[0] >= t->n_cur;
  t->adapt_marks = false;
  if (!restricted) {
    LT_TRY(grow(t->A, &t->mbuf[mi], &t->mcap[mi], t->n_cur));
    k_fill_u32<<<unsigned(ceil_div(t->n_cur, 256)), 256, 0, s>>>(t->mbuf[mi], t->n_cur, 0u);
    LT_HIP(hipGetLastError());
  }
  // Right after a successful adapt the error word, the mark count and the
  // fused-parent count are already zero (adapt's scan preparation cleared
  // them and adapt read the error word back), and the examine list must
  // survive: only other entries need the counters cleared.
  if (!restricted) LT_TRY(clear_err(t, s));
  const int max_pass = 4 * t->g.dmax + 16;
  int64_t expect_total = -1;
  for (int pass = 0;; ++pass) {
    if (pass > max_pass) return fail(LT_ERR_INTERNAL, "balance did not converge");
    KeyDir D;
    LT_TRY(ensure_dir(t, s, &D));
    if (t->n_cur > 0) {
      const int all = pass == 0 && !restricted ? 1 : 0;
      // every leaf: one lane per (leaf, searching key); listed leaves: a
      // bounded grid striding over the device-side list
      const int64_t full = ceil_div(t->n_cur * t->g.nchild(), kBlock);
      const unsigned blocks = unsigned(all ? full : std::min<int64_t>(full, kMarkGrid));
      const int32_t* el = all ? nullptr : t->elist;
      const Count cn{t->n_cur, nullptr};
      if (pass == 0 && restricted)  // adapt listed the fused parents (the list is sized for its output)
        LT_HIP(launch_fused_check(t->g, t->kbuf[t->cur], cn, D, t->mbuf[mi], t->fused, t->dctr, s));
      if (t->g.dim == 3)
        k_balance_mark<3><<<blocks, kBlock, 0, s>>>(t->g, t->kbuf[t->cur], cn, D, t->mbuf[mi], all,
                                                    t->dctr, nullptr, el, t->elist_cap);
      else
        k_balance_mark<2><<<blocks, kBlock, 0, s>>>(t->g, t->kbuf[t->cur], cn, D, t->mbuf[mi], all,
                                                    t->dctr, nullptr, el, t->elist_cap);
      LT_HIP(hipGetLastError());
    }
    LT_TRY(read_ctr(t, s));
    if (t->hctr->err) return fail(LT_ERR_INTERNAL, "device check failed in lt_balance");
    if (expect_total >= 0 && t->hctr->total != expect_total)
      return fail(LT_ERR_INTERNAL, "balance refinement size mismatch");
    const int64_t marked = int64_t(t->hctr->nmarked);
    if (marked == 0) break;
    const int64_t n_new = t->n_cur + marked * (t->g.nchild() - 1);
    const int out = t->cur == t->tmp ? t->aux : t->tmp;
    LT_TRY(grow(t->A, &t->kbuf[out], &t->kcap[out], n_new));
    LT_TRY(grow(t->A, &t->mbuf[1 - mi], &t->mcap[1 - mi], n_new));
    LT_TRY(grow(t->A, &t->elist, &t->elist_cap, n_new));
    ScanState st;
    // also zeroes the mark count and the examine list for the next pass
    LT_TRY(prep_scan(t, t->n_cur, kTileMax, s, 4, &st));
    const int64_t cap = std::min(std::min(t->kcap[out], t->mcap[1 - mi]), t->elist_cap);
    k_balance_refine<<<grid_tiles(st), kScanBig, 0, s>>>(t->g, t->kbuf[t->cur], t->mbuf[mi],
                                                        t->kbuf[out], t->mbuf[1 - mi], cap, st,
                                                        nullptr, t->elist, &t->dctr->nexam,
                                                        t->elist_cap);
    LT_HIP(hipGetLastError());
    expect_total = n_new;
    t->cur = out;
    t->n_cur = n_new;
    mi = 1 - mi;
    invalidate(t);
  }
  return LT_OK;
}
}  // namespace

extern "C" {

lt_status lt_balance(lt_tree t, void* stream) {
  if (!t) return fail(LT_ERR_ARG, "NULL tree");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int cur0 = t->cur;
  const int64_t n0 = t->n_cur;
  const bool conn0 = t->conn_valid, map0 = t->map_valid;
  const int64_t hang0 = t->n_hang;
  const lt_status st = balance_passes(t, s);
  if (st != LT_OK) {
    // strong guarantee: the leaves before the call are still in kbuf[cur0];
    // connectivity and mapping arrays were not touched by the passes
    t->cur = cur0;
    t->n_cur = n0;
    t->conn_valid = conn0;
    t->map_valid = map0;
    t->n_hang = hang0;
    t->dir_valid = false;     // the directory may describe intermediate leaves
    t->adapt_marks = false;   // the first pass's marks were consumed
    return st;
  }
  if (t->cur != cur0) {  // cur0 and the free buffer the passes did not end in are free
    if (t->cur == t->tmp)
      t->tmp = cur0;
    else
      t->aux = cur0;
  }
  t->balanced = true;
  return LT_OK;
}


lt_status lt_connect(lt_tree t, void* stream) {
  if (!t) return fail(LT_ERR_ARG, "NULL tree");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = t->n_cur;
  const int nf = 2 * t->g.dim;
  const int width = 2 + (1 << (t->g.dim - 1));
  LT_TRY(grow(t->A, &t->nbr, &t->nbr_cap, n * nf));
  LT_TRY(grow(t->A, &t->hmask, &t->hmask_cap, n + kItems));
  // initial table: one row per 16 leaves, as a captured cycle reserves (the
  // hanging faces sit on the refinement fronts: one per 90 leaves in the
  // 1.7M-leaf workload, more than one per 64 at 9M leaves)
  LT_TRY(grow(t->A, &t->hang, &t->hang_cap, std::max<int64_t>(1024, n / 16) * width));
  KeyDir D;
  LT_TRY(ensure_dir(t, s, &D));
  if (n > 0) {
    const int64_t lanes = ceil_div(n * t->g.nchild(), 256);
    const unsigned blocks = unsigned(t->conn_grid > 0 ? std::min<int64_t>(lanes, t->conn_grid) : lanes);
    if (t->g.dim == 3)
      k_connect_faces<3><<<blocks, 256, 0, s>>>(t->g, t->kbuf[t->cur], Count{n, nullptr}, D, t->nbr,
                                                t->hmask);
    else
      k_connect_faces<2><<<blocks, 256, 0, s>>>(t->g, t->kbuf[t->cur], Count{n, nullptr}, D, t->nbr,
                                                t->hmask);
    LT_HIP(hipGetLastError());
  }
  const int nh = 1 << (t->g.dim - 1);
  int64_t rows = -1;
  for (int attempt = 0; attempt < 2 && rows < 0; ++attempt) {
    const int64_t cap_rows = t->hang_cap / width;
    ScanState st;
    LT_TRY(prep_scan_conn(t, n, s, 1, &st));
    k_connect_rows<<<grid_tiles(st), kScanSmall, 0, s>>>(t->hmask, t->g.dim, t->hang, cap_rows, st);
    LT_HIP(hipGetLastError());
    // fine leaves of the rows the table holds (the row count stays on the device)
    k_connect_fine<<<unsigned(ceil_div(cap_rows * nh, 256)), 256, 0, s>>>(
        t->g, t->kbuf[t->cur], Count{n, nullptr}, D, t->hang, &t->cctr->total, cap_rows,
        &t->cctr->err);
    LT_HIP(hipGetLastError());
    LT_HIP(hipMemcpyAsync(t->hcctr, t->cctr, sizeof(DevCtr), hipMemcpyDeviceToHost, s));
    LT_HIP(hipStreamSynchronize(s));
    if (t->hcctr->err & ERR_UNBALANCED)
      return fail(LT_ERR_UNBALANCED, "tree is not 2:1 balanced across a face");
    if (t->hcctr->err) return fail(LT_ERR_INTERNAL, "device check failed in lt_connect");
    if (t->hcctr->total <= cap_rows)
      rows = t->hcctr->total;
    else  // the hanging-face table overflowed: grow it (with room for the next
          // cycles: a regrowth frees memory, which waits for the whole device)
          // and emit the rows again
      LT_TRY(grow(t->A, &t->hang, &t->hang_cap, 2 * t->hcctr->total * width));
  }
  if (rows < 0) return fail(LT_ERR_INTERNAL, "hanging-face table overflowed twice");
  t->n_hang = rows;
  t->conn_valid = true;
  return LT_OK;
}

lt_status lt_set_connect_grid(lt_tree t, int blocks) {
  if (!t) return fail(LT_ERR_ARG, "NULL tree");
  if (blocks < 0) return fail(LT_ERR_ARG, "the connectivity grid cap must be >= 0");
  t->conn_grid = blocks;
  return LT_OK;
}

lt_status lt_map(lt_tree t, void* stream) {
  if (!t) return fail(LT_ERR_ARG, "NULL tree");
  return do_map(t, static_cast<hipStream_t>(stream));
}

lt_status lt_transfer(lt_tree t, int p, int nvar, const double* u_old, int64_t ld_old, double* u_new,
                      int64_t ld_new, int precision, void* stream) {
  if (!t || !u_old || !u_new) return fail(LT_ERR_ARG, "NULL argument");
  if (precision != 0 && precision != 1) return fail(LT_ERR_ARG, "precision must be 0 or 1");
  if (nvar < 1) return fail(LT_ERR_ARG, "nvar must be positive");
  if (p < 1 || p > (t->g.dim == 3 ? 3 : LT_MAX_DEGREE))
    return fail(LT_ERR_ARG, "unsupported polynomial degree for this dimension");
  if (!t->has_old) return fail(LT_ERR_STATE, "lt_transfer needs a prior lt_adapt");
  if (ld_old < t->n_old || ld_new < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!t->map_valid) LT_TRY(lt_map(t, stream));
  if (precision == 1) return launch_split_transfer(t, p, nvar, u_old, ld_old, u_new, ld_new, s);
  LT_TRY(build_transfer_ops(t->A, p, &t->ops[p], s));
  return launch_transfer(t, p, t->ops[p], nvar, u_old, ld_old, u_new, ld_new, s);
}

lt_status lt_size(lt_tree t, int64_t* n_cur, int64_t* n_old, int64_t* n_hang) {
  if (!t) return fail(LT_ERR_ARG, "NULL tree");
  if (n_cur) *n_cur = t->n_cur;
  if (n_old) *n_old = t->has_old ? t->n_old : -1;
  if (n_hang) *n_hang = t->conn_valid ? t->n_hang : -1;
  return LT_OK;
}

static lt_status field_info(lt_tree t, lt_field what, const void** ptr, int64_t* count, size_t* elem) {
  const int nf = 2 * t->g.dim, width = 2 + (1 << (t->g.dim - 1));
  switch (what) {
    case LT_KEYS: *ptr = t->kbuf[t->cur]; *count = t->n_cur; *elem = 8; break;
    case LT_OLD_KEYS:
      *ptr = t->has_old ? t->kbuf[t->old] : nullptr; *count = t->has_old ? t->n_old : 0; *elem = 8; break;
    case LT_NBR:
      *ptr = t->conn_valid ? t->nbr : nullptr; *count = t->conn_valid ? t->n_cur * nf : 0; *elem = 4; break;
    case LT_HANG:
      *ptr = t->conn_valid ? t->hang : nullptr; *count = t->conn_valid ? t->n_hang * width : 0; *elem = 4; break;
    case LT_MAP_SRC:
      *ptr = t->map_valid ? t->map_src : nullptr; *count = t->map_valid ? t->n_cur : 0; *elem = 4; break;
    case LT_MAP_KIND:
      *ptr = t->map_valid ? t->map_kind : nullptr; *count = t->map_valid ? t->n_cur : 0; *elem = 1; break;
    default: return fail(LT_ERR_ARG, "unknown field");
  }
  return LT_OK;
}

lt_status lt_view(lt_tree t, lt_field what, const void** ptr, int64_t* count) {
  if (!t || !ptr || !count) return fail(LT_ERR_ARG, "NULL argument");
  size_t elem;
  return field_info(t, what, ptr, count, &elem);
}

lt_status lt_export(lt_tree t, lt_field what, void* dst, int64_t capacity, void* stream) {
  if (!t) return fail(LT_ERR_ARG, "NULL tree");
  const void* p;
  int64_t count;
  size_t elem;
  LT_TRY(field_info(t, what, &p, &count, &elem));
  if (!p && count > 0) return fail(LT_ERR_STATE, "field not computed");
  if (capacity < count) return fail(LT_ERR_ARG, "destination too small");
  if (count > 0 && !dst) return fail(LT_ERR_ARG, "NULL destination");
  if (count > 0)
    LT_HIP(hipMemcpyAsync(dst, p, size_t(count) * elem, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(stream)));
  return LT_OK;
}

void lt_destroy(lt_tree t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  const Alloc A = t->A;
  auto fr = [&](void* p) { (void)dev_free(A, p); };
  for (auto& b : t->kbuf) fr(b);
  for (auto& b : t->mbuf) fr(b);
  for (void* b : {(void*)t->nbr, (void*)t->hmask, (void*)t->fused, (void*)t->dir, (void*)t->hang,
                  (void*)t->map_src, (void*)t->map_kind, (void*)t->status, (void*)t->lim,
                  (void*)t->flag_tab, (void*)t->mesh_offs, (void*)t->dctr, (void*)t->cstatus,
                  (void*)t->elist, (void*)t->cctr, t->split_frags, (void*)t->split_vec,
                  (void*)t->split_R, (void*)t->split_F, (void*)t->copy_delta, (void*)t->grp_list})
    fr(b);
  for (auto& o : t->ops) fr(o);
  for (auto& o : t->fr_tab) fr(o);
  fr(t->mesh_np);
  fr(t->chunk_np);
  fr(t->fr_fb);
  if (t->hctr) (void)hipHostFree(t->hctr);
  if (t->hcctr) (void)hipHostFree(t->hcctr);
  if (t->xs) (void)hipStreamDestroy(t->xs);
  for (hipEvent_t e : t->xev)
    if (e) (void)hipEventDestroy(e);
  delete t;
}

}  // extern "C"
