// lt_build.hip -- bottom-up construction of a complete linear tree from
// scattered points (Section 3.1, tree construction and linearization;
// Section 5.1: a coarse background at d_min with the points encoded at d_max).
//
// The tree built is the coarsest complete linear tree whose leaves all have
// depth >= d_min and in which every point's finest cell (its d_max octant) is
// a leaf.  Its leaves are the point cells themselves plus, in every gap of the
// Morton curve between two consecutive distinct cells, the coarsest aligned
// octants that tile the gap -- at most d_min deep's size -- taken greedily
// from the gap's start.  So the construction is
//
//   1. encode: one lane per point, finest cell -> Morton index;
//   2. sort the indices: LSD radix sort, 8-bit digits, three launches per
//      digit (per-tile histograms, one look-back scan over them, a stable
//      scatter ranked in LDS with wave ballots);
//   3. unique: count -> look-back scan -> emit of the distinct indices;
//   4. completion: per gap, the number of octants of its greedy tiling,
//      scanned into output offsets; then one lane per gap writes them
//      (nearly every gap holds a few leaves).
//
// Where the paper appends the octants between consecutive points through
// shared-memory and atomic counters, sorts and linearizes, the count -> scan
// -> emit form writes every leaf once, already in Morton order and linear.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "tree.hpp"

namespace lt {
namespace {

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kSortItems = 8;
constexpr int64_t kSortTile = int64_t(kSortBlock) * kSortItems;  // keys per workgroup
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
static_assert(kRadix == kSortBlock, "one digit per thread in the per-tile passes");

// shares the error word with the scans' ERR_* bits
enum : unsigned { ERR_POINT = 1u << 12 };

// Finest cell of each point: i_a = floor((x_a - lo_a) / dx), in FP64 in that
// order (this unit is compiled without contraction), interleaved into the
// Morton index at d_max.  Points outside the domain set ERR_POINT.
template <int DIM>
__global__ __launch_bounds__(256) void k_point_codes(const double* __restrict__ pts, int64_t n,
                                                     double lo0, double lo1, double lo2, double dx,
                                                     double W, uint64_t* __restrict__ codes,
                                                     unsigned* err) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double lo[3] = {lo0, lo1, lo2};
  uint64_t c[3] = {0, 0, 0};
  bool ok = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double f = floor((pts[DIM * j + a] - lo[a]) / dx);
    ok = ok && f >= 0.0 && f < W;  // false for NaN too
    c[a] = ok ? uint64_t(f) : 0;
  }
  if (!ok) atomicOr(err, ERR_POINT);
  codes[j] = DIM == 2 ? (spread2(c[0]) | (spread2(c[1]) << 1))
                      : (spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2));
}

// Digit counts of one tile, digit-major: hist[d * ntiles + tile].
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                           int64_t n, int shift, int64_t ntiles,
                                                           uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + int64_t(r) * kSortBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of 32-bit counts into 32-bit offsets (decoupled look-back).
__global__ __launch_bounds__(kScanSmall) void k_exscan_u32(const uint32_t* __restrict__ in,
                                                           uint32_t* __restrict__ out,
                                                           ScanState st) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = st.items.get();
  const int64_t base = tile * kTileMin + int64_t(threadIdx.x) * kItems;
  uint32_t v[kItems];
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    v[k] = base + k < n ? in[base + k] : 0u;
    local += v[k];
  }
  int64_t blk;
  const int64_t thr = block_exclusive<kScanSmall>(local, &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) out[base + k] = uint32_t(o);
    o += v[k];
  }
}

// Stable scatter of one tile by one digit.  Wave w takes the tile's keys
// [w*512, (w+1)*512) in eight rounds of 64 consecutive keys; a key's rank
// among the earlier keys of its wave with the same digit is the running
// count of that digit (LDS, one row per wave) plus the number of lower lanes
// of its round holding the same digit (eight ballots give the lanes whose
// digit matches bit for bit).  The wave rows are then turned into offsets
// over the waves, so keys keep their input order within a digit.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const uint64_t* __restrict__ in,
                                                              int64_t n, int shift, int64_t ntiles,
                                                              const uint32_t* __restrict__ offs,
                                                              uint64_t* __restrict__ out) {
  __shared__ uint32_t cnt[kSortWaves][kRadix];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortBlock) (&cnt[0][0])[i] = 0u;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kSortTile + int64_t(w) * (kSortItems * 64);
  const unsigned long long below = (1ull << lane) - 1ull;
  uint64_t key[kSortItems];
  uint32_t rank[kSortItems];
  int dig[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + int64_t(r) * 64 + lane;
    const bool valid = i < n;
    key[r] = valid ? in[i] : 0;
    const int d = int((key[r] >> shift) & (kRadix - 1));
    dig[r] = valid ? d : -1;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t before = uint32_t(__popcll(peers & below));
    const uint32_t b0 = cnt[w][d];
    rank[r] = b0 + before;
    // the lowest lane of each digit group advances its running count; the
    // wave's LDS accesses complete in order, so the next round reads it
    if (valid && before == 0) cnt[w][d] = b0 + uint32_t(__popcll(peers));
  }
  __syncthreads();
  {
    const int d = threadIdx.x;  // one digit per thread
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < kSortWaves; ++q) {
      const uint32_t c = cnt[q][d];
      cnt[q][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int d = dig[r];
    if (d < 0) continue;
    const uint32_t pos = offs[int64_t(d) * ntiles + blockIdx.x] + cnt[w][d] + rank[r];
    out[pos] = key[r];
  }
}

// Distinct values of a sorted array, in order (count -> scan -> emit).
__global__ __launch_bounds__(kScanSmall) void k_unique(const uint64_t* __restrict__ in,
                                                       uint64_t* __restrict__ out, ScanState st) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = st.items.get();
  const int64_t base = tile * kTileMin + int64_t(threadIdx.x) * kItems;
  bool first[kItems];
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k;
    first[k] = i < n && (i == 0 || in[i] != in[i - 1]);
    local += first[k];
  }
  int64_t blk;
  const int64_t thr = block_exclusive<kScanSmall>(local, &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (first[k]) out[o++] = in[base + k];
}

// Greedy tiling of the Morton interval [lo, hi) of finest cells by aligned
// octants of at most 2^(dim*K) cells (depth >= d_max - K): at every position
// the largest aligned octant that fits.  Let P be the point of [lo, hi]
// aligned to the largest octant size 2^(dim j), j <= K.  No octant of the
// tiling crosses P (an aligned octant across it would put a point aligned to
// a larger size inside [lo, hi]), so the tiling is an ascending run over
// [lo, P) -- d_k octants of size 2^(dim k) for each digit d_k of P - lo in
// base 2^dim, smallest first -- then (hi - P) >> (dim K) octants of the full
// size, then a descending run over the rest, digit by digit from the top.
// Counting and emitting both follow these digits instead of probing the
// largest fitting octant at every position.
struct Gap {
  uint64_t lo, hi;
};

// P for a non-empty gap.
__device__ inline uint64_t gap_pivot(uint64_t lo, uint64_t hi, int dim, int K) {
  for (int j = K; j > 0; --j) {
    const uint64_t b = uint64_t(1) << (dim * j);
    const uint64_t p = (lo + b - 1) & ~(b - 1);
    if (p <= hi) return p;
  }
  return lo;
}

// Leaves of the tiling of [lo, hi).
__device__ inline int64_t gap_leaves(uint64_t lo, uint64_t hi, int dim, int K) {
  if (lo >= hi) return 0;
  const uint64_t P = gap_pivot(lo, hi, dim, K);
  const uint64_t digit = (uint64_t(1) << dim) - 1, rest = hi - P;
  int64_t n = int64_t(rest >> (dim * K));
  for (int k = 0; k < K; ++k)
    n += int64_t(((P - lo) >> (dim * k)) & digit) + int64_t((rest >> (dim * k)) & digit);
  return n;
}

// Gap g of m distinct cells S: [S[g-1] + 1, S[g]) (from 0 for g = 0, up to
// the domain's end for g = m).
__device__ inline Gap gap_of(const uint64_t* __restrict__ S, int64_t m, int64_t g, uint64_t end) {
  Gap q;
  q.lo = g == 0 ? 0 : S[g - 1] + 1;
  q.hi = g == m ? end : S[g];
  return q;
}

// Leaves per gap (its tiling plus the cell closing it), scanned into offsets.
__global__ __launch_bounds__(kScanSmall) void k_gap_count(const uint64_t* __restrict__ S, int64_t m,
                                                          uint64_t end, int dim, int K,
                                                          int64_t* __restrict__ goff, ScanState st) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = st.items.get();  // m + 1 gaps
  const int64_t base = tile * kTileMin + int64_t(threadIdx.x) * kItems;
  int64_t c[kItems];
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t g = base + k;
    c[k] = 0;
    if (g >= n) continue;
    const Gap q = gap_of(S, m, g, end);
    c[k] = gap_leaves(q.lo, q.hi, dim, K) + (g < m ? 1 : 0);
    local += c[k];
  }
  int64_t blk;
  const int64_t thr = block_exclusive<kScanSmall>(local, &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) goff[base + k] = o;
    o += c[k];
  }
}

// One lane per gap writes its leaves at goff[g]: the ascending run, the
// full-size run, the descending run (the digits above) and the closing point
// cell.  Nearly every gap holds a few leaves; the long full-size runs (at
// most the background's 2^(d d_min) octants, in the gaps far from every
// point) are rare, and a lane walks them alone.
__global__ __launch_bounds__(256) void k_gap_emit(const uint64_t* __restrict__ S, int64_t m,
                                                  uint64_t end, KeyGeom g, int K,
                                                  const int64_t* __restrict__ goff,
                                                  uint64_t* __restrict__ keys) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi > m) return;
  const int dim = g.dim;
  const Gap q = gap_of(S, m, gi, end);
  int64_t o = goff[gi];
  if (q.lo < q.hi) {
    const uint64_t P = gap_pivot(q.lo, q.hi, dim, K);
    const uint64_t digit = (uint64_t(1) << dim) - 1, rest = q.hi - P;
    uint64_t x = q.lo;
    for (int k = 0; k < K; ++k)
      for (uint64_t t = ((P - q.lo) >> (dim * k)) & digit; t > 0; --t) {
        keys[o++] = make_key(g, x, g.dmax - k);
        x += uint64_t(1) << (dim * k);
      }
    for (uint64_t t = rest >> (dim * K); t > 0; --t) {
      keys[o++] = make_key(g, x, g.dmax - K);
      x += uint64_t(1) << (dim * K);
    }
    for (int k = K - 1; k >= 0; --k)
      for (uint64_t t = (rest >> (dim * k)) & digit; t > 0; --t) {
        keys[o++] = make_key(g, x, g.dmax - k);
        x += uint64_t(1) << (dim * k);
      }
  }
  if (gi < m) keys[o] = make_key(g, S[gi], g.dmax);
}

// Device temporaries of one construction, freed on every exit path.
struct Temps {
  const Alloc* A;
  void* p[6] = {};
  ~Temps() {
    for (void* q : p) (void)dev_free(*A, q);
  }
};

lt_status sort_codes(lt_tree t, uint64_t** a, uint64_t** b, int64_t n, int bits, uint32_t* hist,
                     uint32_t* offs, hipStream_t s) {
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  for (int shift = 0; shift < bits; shift += kRadixBits) {
    k_radix_hist<<<unsigned(ntiles), kSortBlock, 0, s>>>(*a, n, shift, ntiles, hist);
    ScanState st;
    LT_TRY_STATUS(prep_scan(t, kRadix * ntiles, kTileMin, s, 0, &st));
    k_exscan_u32<<<grid_tiles(st), kScanSmall, 0, s>>>(hist, offs, st);
    k_radix_scatter<<<unsigned(ntiles), kSortBlock, 0, s>>>(*a, n, shift, ntiles, offs, *b);
    if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "radix sort launch");
    std::swap(*a, *b);
  }
  return LT_OK;
}

lt_status build_points(lt_tree t, const double* pts, int64_t n, const double* lo, double len,
                       hipStream_t s) {
  const KeyGeom& g = t->g;
  const int dim = g.dim;
  Temps tmp{&t->A};
  auto al = [&](int i, size_t bytes) -> lt_status {
    if (dev_malloc(t->A, &tmp.p[i], std::max<size_t>(bytes, 256)) != hipSuccess)
      return fail(LT_ERR_OOM, "construction temporaries (" + std::to_string(bytes) + " bytes)");
    return LT_OK;
  };
  const int64_t ntiles = std::max<int64_t>(1, (n + kSortTile - 1) / kSortTile);
  LT_TRY_STATUS(al(0, size_t(n) * 8));                      // codes
  LT_TRY_STATUS(al(1, size_t(n) * 8));                      // sort ping-pong, then the distinct cells
  LT_TRY_STATUS(al(2, size_t(kRadix) * ntiles * 4));        // digit counts
  LT_TRY_STATUS(al(3, size_t(kRadix) * ntiles * 4));        // digit offsets
  LT_TRY_STATUS(al(4, size_t(n + 1) * 8));                  // gap offsets
  uint64_t* a = static_cast<uint64_t*>(tmp.p[0]);
  uint64_t* b = static_cast<uint64_t*>(tmp.p[1]);
  LT_TRY_STATUS(clear_err(t, s));
  int64_t m = 0;
  if (n > 0) {
    const double W = double(int64_t(1) << g.dmax);
    const double dx = len / W;
    if (dim == 2)
      k_point_codes<2><<<unsigned((n + 255) / 256), 256, 0, s>>>(pts, n, lo[0], lo[1], 0.0, dx, W, a,
                                                                 &t->dctr->err);
    else
      k_point_codes<3><<<unsigned((n + 255) / 256), 256, 0, s>>>(pts, n, lo[0], lo[1], lo[2], dx, W,
                                                                 a, &t->dctr->err);
    if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "point encoding launch");
    LT_TRY_STATUS(sort_codes(t, &a, &b, n, dim * g.dmax, static_cast<uint32_t*>(tmp.p[2]),
                             static_cast<uint32_t*>(tmp.p[3]), s));
    // a holds the sorted cells; the distinct ones go to b
    ScanState st;
    LT_TRY_STATUS(prep_scan(t, n, kTileMin, s, 0, &st));
    k_unique<<<grid_tiles(st), kScanSmall, 0, s>>>(a, b, st);
    if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "unique launch");
    LT_TRY_STATUS(read_ctr(t, s));
    if (t->hctr->err & ERR_POINT) return fail(LT_ERR_ARG, "a point lies outside the domain");
    if (t->hctr->err) return fail(LT_ERR_INTERNAL, "device check failed while sorting the points");
    m = t->hctr->total;
  }
  const uint64_t* S = b;
  const uint64_t end = uint64_t(1) << (dim * g.dmax);
  const int K = g.dmax - g.dmin;
  int64_t* goff = static_cast<int64_t*>(tmp.p[4]);
  ScanState st;
  LT_TRY_STATUS(prep_scan(t, m + 1, kTileMin, s, 1, &st));
  k_gap_count<<<grid_tiles(st), kScanSmall, 0, s>>>(S, m, end, dim, K, goff, st);
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "gap count launch");
  LT_TRY_STATUS(read_ctr(t, s));
  if (t->hctr->err) return fail(LT_ERR_INTERNAL, "device check failed while counting the tiling");
  const int64_t total = t->hctr->total;
  if (total > (int64_t(1) << 31) - 1) return fail(LT_ERR_ARG, "the tree would hold 2^31 leaves or more");
  LT_TRY_STATUS(grow(t->A, &t->kbuf[t->cur], &t->kcap[t->cur], total));
  const int64_t threads = m + 1;  // one lane per gap
  k_gap_emit<<<unsigned((threads + 255) / 256), 256, 0, s>>>(S, m, end, g, K, goff,
                                                             t->kbuf[t->cur]);
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "gap emit launch");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LT_ERR_HIP, "construction");
  t->n_cur = total;
  t->balanced = false;
  return LT_OK;
}

}  // namespace
}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_build_points(const lt_geom* geom, const double* pts, int64_t n, const double* lo,
                          double len, void* stream, lt_tree* out) {
  if (!geom || !lo || !out || n < 0 || (n > 0 && !pts)) return fail(LT_ERR_ARG, "NULL argument or n < 0");
  if (n > (int64_t(1) << 31) - 1) return fail(LT_ERR_ARG, "at most 2^31 - 1 points");
  if (!(len > 0.0)) return fail(LT_ERR_ARG, "the domain length must be positive");
  lt_tree t = nullptr;
  LT_TRY_STATUS(create_tree(geom, &t));
  if (geom->dim == 3 && geom->d_max > 21) {
    lt_destroy(t);
    return fail(LT_ERR_DEPTH, "3D d_max above 21");
  }
  const lt_status st = build_points(t, pts, n, lo, len, static_cast<hipStream_t>(stream));
  if (st != LT_OK) {
    lt_destroy(t);
    return st;
  }
  *out = t;
  return LT_OK;
}

}  // extern "C"
