// lt_transfer.hip -- FP64 solution transfer between the old and new tree
// (Section 4.2).
//
// With Gauss-Legendre solution points the operators factor per axis.  On one
// axis with nodes z_i and weights w_i:
//   refinement (interpolation of the parent polynomial, eq. parent_soln):
//       A_b[i][k] = l_k((z_i + 2b - 1) / 2),            child half b in {0, 1}
//   coarsening (L2 projection M u^P = sum_b S_b u^b): the Gauss-Legendre rule
//   integrates the degree-2p products exactly, so M = diag(w) and
//       P_b[i][k] = (1/2) (w_k / w_i) A_b[k][i].
// In d dimensions the child-c operators are tensor products over the axes of
// the factor for that axis's child bit, so each is applied as d passes of a
// (p+1) x (p+1) product along one axis (sum factorisation) instead of one
// dense (p+1)^d x (p+1)^d product: the same result up to rounding order, with
// (p+1)^(d-1) times fewer flops, which keeps the transfer bound by HBM bytes
// rather than by FP64 throughput.
#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <string>
#include <vector>

#include "tree.hpp"

namespace lt {
namespace {

// Gauss-Legendre nodes (Newton on P_n from Chebyshev starting points),
// weights, then the factors A_0, A_1, P_0, P_1 (row-major, n x n each),
// followed by the n weights.
__global__ void k_build_ops(int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double z[LT_MAX_DEGREE + 1], w[LT_MAX_DEGREE + 1];
  for (int i = 0; i < n; ++i) {
    double x = -cos(M_PI * (2.0 * i + 1.0) / (2.0 * n));
    double dp = 1.0;
    for (int it = 0; it < 60; ++it) {
      // P_n(x) and P_n'(x) by the Bonnet recurrence
      double pm = 1.0, pc = x;
      if (n == 1) {
        pc = x;
        pm = 1.0;
      }
      for (int k = 2; k <= n; ++k) {
        const double pn = ((2 * k - 1) * x * pc - (k - 1) * pm) / k;
        pm = pc;
        pc = pn;
      }
      dp = n * (pm - x * pc) / (1.0 - x * x);
      const double dx = pc / dp;
      x -= dx;
      if (fabs(dx) <= 1e-16 * fmax(1.0, fabs(x))) break;
    }
    double pm = 1.0, pc = x;
    for (int k = 2; k <= n; ++k) {
      const double pn = ((2 * k - 1) * x * pc - (k - 1) * pm) / k;
      pm = pc;
      pc = pn;
    }
    dp = n * (pm - x * pc) / (1.0 - x * x);
    z[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  double* A0 = out;
  double* A1 = out + n * n;
  double* P0 = out + 2 * n * n;
  double* P1 = out + 3 * n * n;
  for (int b = 0; b < 2; ++b) {
    double* A = b ? A1 : A0;
    for (int i = 0; i < n; ++i) {
      const double xi = (z[i] + 2.0 * b - 1.0) * 0.5;
      for (int k = 0; k < n; ++k) {
        double l = 1.0;
        for (int m = 0; m < n; ++m)
          if (m != k) l *= (xi - z[m]) / (z[k] - z[m]);
        A[i * n + k] = l;
      }
    }
  }
  for (int b = 0; b < 2; ++b) {
    const double* A = b ? A1 : A0;
    double* P = b ? P1 : P0;
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) P[i * n + k] = 0.5 * (w[k] / w[i]) * A[k * n + i];
  }
  for (int i = 0; i < n; ++i) out[4 * n * n + i] = w[i];
}

// out = (Mz (x) My (x) Mx) in, for a tensor array with x fastest.
template <int DIM, int N>
__device__ inline void tensor_apply(const double* __restrict__ Mx, const double* __restrict__ My,
                                    const double* __restrict__ Mz, const double* in, double* out) {
  constexpr int NZ = DIM == 3 ? N : 1;
  constexpr int NP = N * N * NZ;
  double t[NP];
#pragma unroll
  for (int r = 0; r < N * NZ; ++r)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += Mx[i * N + k] * in[r * N + k];
      t[r * N + i] = acc;
    }
  if constexpr (DIM == 2) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int x = 0; x < N; ++x) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) acc += My[i * N + k] * t[k * N + x];
        out[i * N + x] = acc;
      }
  } else {
    double t2[NP];
#pragma unroll
    for (int z = 0; z < N; ++z)
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int x = 0; x < N; ++x) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < N; ++k) acc += My[i * N + k] * t[(z * N + k) * N + x];
          t2[(z * N + i) * N + x] = acc;
        }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int y = 0; y < N; ++y)
#pragma unroll
        for (int x = 0; x < N; ++x) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < N; ++k) acc += Mz[i * N + k] * t2[(k * N + y) * N + x];
          out[(i * N + y) * N + x] = acc;
        }
  }
}

// One thread per (new element, variable) -- used for 2D.  Consecutive
// threads handle consecutive new elements, so every load and store of one
// point index is a contiguous run across the wave in the element-fastest layout.
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_transfer(const double* __restrict__ ops,
                                                  const int32_t* __restrict__ src,
                                                  const int8_t* __restrict__ kind, Count cn,
                                                  const double* __restrict__ uo, int64_t ldo,
                                                  double* __restrict__ un, int64_t ldn) {
  const int64_t n = cn.get();
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  constexpr int NC = 1 << DIM;
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int v = blockIdx.y;
  const double* U = uo + int64_t(v) * NP * ldo;
  double* O = un + int64_t(v) * NP * ldn;
  const int kd = kind[j];
  const int64_t s = src[j];
  if (kd == 0) {
#pragma unroll
    for (int i = 0; i < NP; ++i) O[i * ldn + j] = U[i * ldo + s];
    return;
  }
  const double* A = ops;
  const double* P = ops + 2 * N * N;
  double in[NP], out[NP];
  if (kd > 0) {
    const int c = kd - 1;
#pragma unroll
    for (int i = 0; i < NP; ++i) in[i] = U[i * ldo + s];
    tensor_apply<DIM, N>(A + (c & 1) * N * N, A + ((c >> 1) & 1) * N * N, A + ((c >> 2) & 1) * N * N,
                         in, out);
#pragma unroll
    for (int i = 0; i < NP; ++i) O[i * ldn + j] = out[i];
    return;
  }
  double acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = 0.0;
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int i = 0; i < NP; ++i) in[i] = U[i * ldo + s + c];
    tensor_apply<DIM, N>(P + (c & 1) * N * N, P + ((c >> 1) & 1) * N * N, P + ((c >> 2) & 1) * N * N,
                         in, out);
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] += out[i];
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) O[i * ldn + j] = acc[i];
}

// Blocks are dealt to the XCDs round-robin (block b to XCD b % 8); this
// permutation gives each XCD one contiguous run of chunks, so the cache lines
// two neighbouring chunks share are fetched into one L2 only.
__device__ inline int64_t xcd_chunk(int64_t b, int64_t nblocks) {
  const int64_t q = nblocks >> 3, r = nblocks & 7;
  const int64_t x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// Copy runs.  Between the refinement fronts the new elements are copies of
// consecutive old elements, so src[j] - j is constant over long runs.  A
// chunk of 256*EPL new elements (one block row of the copy pass, EPL
// elements per lane) that lies inside one such run is "pure": its source
// offset is one word, and the copy of that chunk needs no per-element map
// reads.  cdelta[c] = src[j] - j for a pure chunk, else kImpure.  EPL is a
// tuning parameter (1, 2 or 4; lt_autotune_transfer picks it).
constexpr int64_t kImpure = INT64_MIN;

template <int EPL>
__global__ __launch_bounds__(256) void k_copy_chunks(const int32_t* __restrict__ src,
                                                     const int8_t* __restrict__ kind, Count cn,
                                                     int64_t* __restrict__ cdelta) {
  constexpr int64_t CH = 256 * EPL;
  const int64_t n = cn.get();
  const int64_t c = blockIdx.x;
  const int64_t j0 = c * CH;
  if (j0 >= n) {  // launches sized for a capacity: chunks past the end
    if (threadIdx.x == 0) cdelta[c] = kImpure;
    return;
  }
  const bool head = kind[j0] == 0;
  const int64_t ref = head ? int64_t(src[j0]) - j0 : 0;
  bool ok = head;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int64_t j = j0 + int64_t(e) * 256 + threadIdx.x;
    if (j < n) ok = ok && kind[j] == 0 && int64_t(src[j]) - j == ref;
  }
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) cdelta[c] = ok ? ref : kImpure;
}

// Copy pass (COPY elements).  One block moves one point row (variable v,
// point i) of one chunk: 256 lanes x EPL elements.  Pure chunks read one
// offset and move the row like a plain copy (16-byte pairs for EPL >= 2);
// impure chunks read the map per element and move only the copy elements.
// SKIP: a wave leaves out its 64 elements (one interpolation group) when any
// of them is refined or fused -- the interpolation passes then write the
// group's copies too, so that every row segment of a group is written whole
// by one kernel (pieces written by two kernels reach HBM as partial lines).
// Source loads and output stores are streaming (non-temporal): every copied
// value is touched once, and keeping it out of the caches was measured ~2.5%
// faster for the whole transfer.
template <int EPL, bool SKIP>
__global__ __launch_bounds__(256) void k_copy3(const int32_t* __restrict__ src,
                                               const int8_t* __restrict__ kind, Count cn,
                                               const int64_t* __restrict__ cdelta,
                                               const double* __restrict__ uo, int64_t ldo,
                                               double* __restrict__ un, int64_t ldn) {
  constexpr int64_t CH = 256 * EPL;
  const int64_t n = cn.get();
  const double* U = uo + int64_t(blockIdx.y) * ldo;
  double* O = un + int64_t(blockIdx.y) * ldn;
  // one chunk per block, unless the grid was sized below the count (a
  // captured cycle's launch sized for the count at capture): then stride
  for (int64_t c = xcd_chunk(blockIdx.x, gridDim.x); c * CH < n; c += gridDim.x) {
    const int64_t dl = cdelta[c];
    if (dl != kImpure) {
      if constexpr (EPL == 1) {
        const int64_t j = c * CH + threadIdx.x;
        if (j < n) __builtin_nontemporal_store(__builtin_nontemporal_load(U + j + dl), O + j);
      } else {
#pragma unroll
        for (int h = 0; h < EPL / 2; ++h) {
          const int64_t j = c * CH + int64_t(h) * 512 + int64_t(threadIdx.x) * 2;
          if (j + 1 < n) {
            const d2u t = __builtin_nontemporal_load(reinterpret_cast<const d2u*>(U + j + dl));
            __builtin_nontemporal_store(t, reinterpret_cast<d2u*>(O + j));
          } else if (j < n) {
            __builtin_nontemporal_store(__builtin_nontemporal_load(U + j + dl), O + j);
          }
        }
      }
      continue;
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int64_t jj = c * CH + int64_t(e) * 256 + threadIdx.x;
      const int kd = jj < n ? int(kind[jj]) : 0;
      if (SKIP && __ballot(kd != 0) != 0) continue;  // an interpolation group
      if (jj < n && kd == 0) __builtin_nontemporal_store(__builtin_nontemporal_load(U + src[jj]), O + jj);
    }
  }
}

// x then y pass inside one z-slab (N x N values, x fastest).
template <int N>
__device__ inline void xy_pass(const double* Mx, const double* My, const double* in, double* out) {
  double t[N * N];
#pragma unroll
  for (int y = 0; y < N; ++y)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) a += Mx[i * N + k] * in[y * N + k];
      t[y * N + i] = a;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int x = 0; x < N; ++x) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) a += My[i * N + k] * t[k * N + x];
      out[i * N + x] = a;
    }
}

// Groups of 64 consecutive new elements that hold any refined or fused
// element.  Groups with refined children only are listed in order by a
// look-back scan (count 1 per such group); groups that hold a fused element
// are appended to a second list (flist, count *nflist) in any order, since
// every group is computed on its own.
__global__ __launch_bounds__(kScanSmall) void k_group_list(const int8_t* __restrict__ kind, Count cn,
                                                       int32_t* __restrict__ list, ScanState st,
                                                       int32_t* __restrict__ flist,
                                                       int64_t* __restrict__ nflist) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = cn.get();
  const int64_t ngroups = st.items.get();
  const int64_t base = tile * kTileMin + int64_t(threadIdx.x) * kItems;
  bool ref[kItems];
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t gidx = base + k;
    ref[k] = false;
    if (gidx >= ngroups) continue;
    const int64_t j0 = gidx * 64;
    bool any = false, fus = false;
    if (j0 + 64 <= n) {
      const uint64_t* w8 = reinterpret_cast<const uint64_t*>(kind + j0);
      uint64_t acc = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) acc |= w8[q];
      any = acc != 0;
      fus = (acc & 0x8080808080808080ull) != 0;  // a negative kind byte
    } else {
      for (int64_t j = j0; j < n; ++j) {
        any = any || kind[j] != 0;
        fus = fus || kind[j] < 0;
      }
    }
    if (fus) {
      const int64_t o = int64_t(atomicAdd(reinterpret_cast<unsigned long long*>(nflist), 1ull));
      flist[o] = int32_t(gidx);
    }
    ref[k] = any && !fus;
    local += ref[k] ? 1 : 0;
  }
  int64_t blk;
  const int64_t thr = block_exclusive<kScanSmall>(local, &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (ref[k]) list[o++] = int32_t(base + k);
}

// Ensembles with a degree per mesh (lt_set_mesh_degree): the interpolation
// kernels below also run over (group, degree) entries, entry = group * 4 +
// N - 1, one launch per degree present.  A lane then works only if its
// element's mesh has degree N (the key's mesh bits index the point-count
// table); copies are left to the copy pass, and a variable's rows are npm
// apart (the largest point count of the ensemble).
struct MixedArgs {
  KeyGeom g;
  const uint64_t* keys = nullptr;
  const uint8_t* np_of_mesh = nullptr;
  int npm = 0;
};

// 3D refinement pass over the groups that hold refined children only.  A
// block of N waves takes listed groups of 64 consecutive new elements of one
// variable (grid-stride over the device-side list); lane = element and wave w
// owns z-slab w (N*N points).  The x and y passes of the parent's slab w run
// in registers, the z pass mixes the N slabs through LDS, and each output row
// is stored as soon as it is formed.  Keeping no accumulator across rounds
// holds the register count near half of the general kernel's, so twice as
// many waves hide the load and store latency.  The group's copies are moved
// here as well (the copy pass leaves listed groups out), so that each row
// segment of a group is written whole by this kernel.  MIXED: see MixedArgs.
template <int N, bool MIXED>
__global__ __launch_bounds__(64 * N) void k_interp3_ref(const double* __restrict__ ops,
                                                        const int32_t* __restrict__ src,
                                                        const int8_t* __restrict__ kind, Count cn,
                                                        const int32_t* __restrict__ groups,
                                                        const int64_t* __restrict__ ngroups,
                                                        const double* __restrict__ uo, int64_t ldo,
                                                        double* __restrict__ un, int64_t ldn,
                                                        MixedArgs mx) {
  constexpr int NN = N * N;
  constexpr int NP = NN * N;
  __shared__ double T[N][NN][64];
  __shared__ double M[2][NN];  // A_0, A_1
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = cn.get();
  const int64_t ng = *ngroups;
  if (int64_t(blockIdx.x) >= ng) return;
  for (int i = threadIdx.x; i < 2 * NN; i += blockDim.x) M[i / NN][i % NN] = ops[i];
  const int v = blockIdx.y;
  const int64_t vstride = MIXED ? mx.npm : NP;
  const double* U = uo + int64_t(v) * vstride * ldo + int64_t(w) * NN * ldo;
  double* O0 = un + int64_t(v) * vstride * ldn + int64_t(w) * NN * ldn;
  __syncthreads();
  // Software pipeline over the block's groups: the map and the input rows of
  // the next group are loaded before this group's stores are issued.  Loads
  // and stores share one counter, so a load issued after a group's stores
  // would wait for them; loaded a group ahead, the rows are in registers by
  // the time the stores before them matter.
  auto next = [&](int64_t from) -> int64_t {  // the block's next entry of this degree, or ng
    for (int64_t q = from; q < ng; q += gridDim.x) {
      if constexpr (!MIXED) return q;
      if ((groups[q] & 3) == N - 1) return q;
    }
    return ng;
  };
  struct Item {
    int64_t j;
    int kd;
    bool live;
  };
  auto map_of = [&](int64_t q) -> Item {
    Item it{0, 0, false};
    if (q >= ng) return it;
    int64_t grp = groups[q];
    if constexpr (MIXED) grp >>= 2;
    it.j = grp * 64 + lane;
    it.live = it.j < n;
    if constexpr (MIXED)
      it.live = it.live && int(mx.np_of_mesh[key_mesh(mx.g, mx.keys[it.j])]) == NP;
    it.kd = it.live ? int(kind[it.j]) : 0;
    return it;
  };
  // a copy loads its own source, a refined child its parent: the same rows
  auto load_rows = [&](const Item& it, double* in) {
    if (it.live && (!MIXED || it.kd > 0)) {
      const int64_t s = int64_t(src[it.j]);
#pragma unroll
      for (int r = 0; r < NN; ++r) in[r] = __builtin_nontemporal_load(U + int64_t(r) * ldo + s);
    }
  };
  int64_t gi = next(blockIdx.x);
  Item cur = map_of(gi);
  double in[NN];
  load_rows(cur, in);
  while (gi < ng) {
    const int64_t gn = next(gi + gridDim.x);
    const Item nxt = map_of(gn);
    const int kd = cur.kd;
    const int c = kd > 0 ? kd - 1 : 0;
    if (kd > 0) {
      double sl[NN];
      xy_pass<N>(M[c & 1], M[(c >> 1) & 1], in, sl);
#pragma unroll
      for (int r = 0; r < NN; ++r) T[w][r][lane] = sl[r];
    }
    double cp[NN];  // a copy's rows, kept while the next group's rows arrive
    const bool copy = !MIXED && cur.live && kd == 0;
#pragma unroll
    for (int r = 0; r < NN; ++r) cp[r] = in[r];
    load_rows(nxt, in);
    __syncthreads();
    double* O = O0 + cur.j;
    if (copy) {  // a copy of the group (the copy pass left the group out)
#pragma unroll
      for (int r = 0; r < NN; ++r) __builtin_nontemporal_store(cp[r], O + int64_t(r) * ldn);
    }
    if (kd > 0) {
      const double* Mz = M[(c >> 2) & 1] + w * N;
#pragma unroll
      for (int r = 0; r < NN; ++r) {
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) a += Mz[k] * T[k][r][lane];
        __builtin_nontemporal_store(a, O + int64_t(r) * ldn);
      }
    }
    __syncthreads();
    gi = gn;
    cur = nxt;
  }
}

// Buffer resource over a wave's rows: base address, no stride, no range limit
// (every offset formed below lies inside the caller's arrays).  The fourth
// word is the GFX9-family data format for raw dword access.
__device__ inline __amdgpu_buffer_rsrc_t rows_rsrc(const double* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0, 0xFFFFFFFF, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));
constexpr int kNonTemporal = 2;  // cache-policy bit of the buffer access: streaming

// The refinement pass of k_interp3_ref (one variable and group of 64 new
// elements per block of N waves, wave w = z-slab w, the z pass through LDS),
// in a form without branches around memory accesses:
//  - every lane of a listed group loads and stores each row: a refined child
//    stores its interpolated value, a copy its source value (selected, not
//    branched), and lanes past the end repeat the last element, so that the
//    stores of an iteration are a fixed number;
//  - rows are addressed through a per-wave buffer resource (row r by a scalar
//    offset, the element by a 32-bit vector offset), which keeps no address
//    registers per row;
//  - a group's map (kind, source) is loaded two groups ahead and its rows one
//    group ahead, both issued before the stores of the group in hand.
// With a fixed store count the compiler waits only for loads issued before
// the previous group's stores, never for the stores themselves, and the
// kernel fits 3 waves per SIMD instead of 2.  Row offsets must fit 32 bits:
// the launch checks N*N rows of either array against that.
template <int N>
__global__ __launch_bounds__(64 * N) void k_refine3(const double* __restrict__ ops,
                                                    const int32_t* __restrict__ src,
                                                    const int8_t* __restrict__ kind, Count cn,
                                                    const int32_t* __restrict__ groups,
                                                    const int64_t* __restrict__ ngroups,
                                                    const double* __restrict__ uo, int64_t ldo,
                                                    double* __restrict__ un, int64_t ldn) {
  constexpr int NN = N * N;
  constexpr int NP = NN * N;
  __shared__ double T[N][NN][64];
  __shared__ double M[2][NN];  // A_0, A_1
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int64_t n = cn.get();
  const int64_t ng = *ngroups;
  if (int64_t(blockIdx.x) >= ng) return;
  for (int i = threadIdx.x; i < 2 * NN; i += blockDim.x) M[i / NN][i % NN] = ops[i];
  const int v = blockIdx.y;
  const __amdgpu_buffer_rsrc_t RU = rows_rsrc(uo + (int64_t(v) * NP + int64_t(w) * NN) * ldo);
  const __amdgpu_buffer_rsrc_t RO = rows_rsrc(un + (int64_t(v) * NP + int64_t(w) * NN) * ldn);
  const uint32_t so = uint32_t(ldo * 8), sn = uint32_t(ldn * 8);
  const int64_t G = gridDim.x;
  struct Map {
    uint32_t j, s;
    int kd;
  };
  auto map_of = [&](int64_t q) -> Map {
    const int64_t qc = q < ng ? q : ng - 1;
    int64_t j = int64_t(groups[qc]) * 64 + lane;
    j = j < n ? j : n - 1;  // past the end: the last element again (same values, same address)
    Map m;
    m.j = uint32_t(j);
    m.kd = int(kind[j]);
    m.s = uint32_t(src[j]);
    return m;
  };
  // a copy loads its own source, a refined child its parent: the same rows
  auto load_rows = [&](const Map& m, double* in) {
    const uint32_t off = m.s * 8u;
#pragma unroll
    for (int r = 0; r < NN; ++r)
      in[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(RU, off, uint32_t(r) * so,
                                                                              kNonTemporal));
  };
  __syncthreads();
  int64_t q = blockIdx.x;
  Map m0 = map_of(q), m1 = map_of(q + G);
  double in[NN];
  load_rows(m0, in);
  // Nothing may be in flight where the loop begins: the counter state at its
  // head is then the one its own iterations leave (only stores), and the
  // first wait inside covers loads alone.
#pragma unroll
  for (int r = 0; r < NN; ++r) asm volatile("" ::"v"(in[r]));
  asm volatile("" ::"v"(m0.j), "v"(m0.kd), "v"(m1.j), "v"(m1.s), "v"(m1.kd));
  __builtin_amdgcn_s_waitcnt(0);
  while (q < ng) {
    const Map m2 = map_of(q + 2 * G);
    double nx[NN];
    load_rows(m1, nx);
    const int c = m0.kd > 0 ? m0.kd - 1 : 0;
    {
      double sl[NN];
      xy_pass<N>(M[c & 1], M[(c >> 1) & 1], in, sl);
#pragma unroll
      for (int r = 0; r < NN; ++r) T[w][r][lane] = sl[r];
    }
    __syncthreads();
    const double* Mz = M[(c >> 2) & 1] + w * N;
    const bool refined = m0.kd > 0;
    const uint32_t oj = m0.j * 8u;
#pragma unroll
    for (int r = 0; r < NN; ++r) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) a += Mz[k] * T[k][r][lane];
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, refined ? a : in[r]), RO, oj,
                                            uint32_t(r) * sn, kNonTemporal);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NN; ++r) in[r] = nx[r];
    m0 = m1;
    m1 = m2;
    q += G;
  }
}

// The refinement pass of an ensemble with a degree per mesh (MixedArgs), in
// the form of k_refine3: the block takes the (group, degree N) entries of its
// degree, and a lane whose element has another degree, is a copy (the copy
// pass writes those here) or lies past the end repeats the loads and stores
// of the entry's first refined lane of degree N -- the same values to the
// same address -- so that every lane stores each row.  Every listed entry has
// such a lane (k_group_list_mixed lists (group, N) only for a group with a
// refined element of degree N and no fused one); the entries fetched ahead
// past the end, which are never stored, fall back to the lane's own element.
// The mesh-degree table is read from LDS, so that a group's map needs no
// dependent load.
constexpr int kMeshTab = 4096;  // meshes whose degrees fit the LDS table
template <int N>
__global__ __launch_bounds__(64 * N) void k_refine3_mixed(const double* __restrict__ ops,
                                                          const int32_t* __restrict__ src,
                                                          const int8_t* __restrict__ kind, Count cn,
                                                          const int32_t* __restrict__ groups,
                                                          const int64_t* __restrict__ ngroups,
                                                          const double* __restrict__ uo, int64_t ldo,
                                                          double* __restrict__ un, int64_t ldn,
                                                          MixedArgs mx, int nmesh) {
  constexpr int NN = N * N;
  constexpr int NP = NN * N;
  __shared__ double T[N][NN][64];
  __shared__ double M[2][NN];  // A_0, A_1
  __shared__ uint8_t npt[kMeshTab];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int64_t n = cn.get();
  const int64_t ng = *ngroups;
  if (int64_t(blockIdx.x) >= ng) return;
  for (int i = threadIdx.x; i < 2 * NN; i += blockDim.x) M[i / NN][i % NN] = ops[i];
  for (int i = threadIdx.x; i < nmesh; i += blockDim.x) npt[i] = mx.np_of_mesh[i];
  const int v = blockIdx.y;
  const __amdgpu_buffer_rsrc_t RU = rows_rsrc(uo + (int64_t(v) * mx.npm + int64_t(w) * NN) * ldo);
  const __amdgpu_buffer_rsrc_t RO = rows_rsrc(un + (int64_t(v) * mx.npm + int64_t(w) * NN) * ldn);
  const uint32_t so = uint32_t(ldo * 8), sn = uint32_t(ldn * 8);
  // The block's next entry of degree N, or ng.  The entry index is the same
  // on every lane; said explicitly, and kept in 32 bits (entries < 2^31), so
  // that the list is read by scalar loads and the index stays in scalar
  // registers (a vector load or register here would wait for every store
  // before it).
  const int ngi = int(ng);
  const int G32 = int(gridDim.x);
  auto next = [&](int from) -> int {
    for (int q = __builtin_amdgcn_readfirstlane(from); q < ngi; q = __builtin_amdgcn_readfirstlane(q + G32))
      if ((__builtin_amdgcn_readfirstlane(groups[q]) & 3) == N - 1) return q;
    return ngi;
  };
  struct Map {
    uint32_t j, s;
    int kd;
    uint64_t key;
  };
  auto map_of = [&](int q) -> Map {
    const int qc = __builtin_amdgcn_readfirstlane(q < ngi ? q : ngi - 1);
    int64_t j = int64_t(__builtin_amdgcn_readfirstlane(groups[qc]) >> 2) * 64 + lane;
    j = j < n ? j : n - 1;
    Map m;
    m.j = uint32_t(j);
    m.kd = int(kind[j]);
    m.s = uint32_t(src[j]);
    m.key = mx.keys[j];
    return m;
  };
  // the lane's own element if it is a refined child of degree N, else the donor's
  auto settle = [&](Map& m) {
    const int np = int(npt[key_mesh(mx.g, m.key)]);  // every key names a mesh: no branch
    const bool own = (m.kd > 0) & (np == NP);
    const uint64_t mask = __ballot(own);
    const int d = mask ? __builtin_ffsll(static_cast<long long>(mask)) - 1 : lane;
    const uint32_t dj = __shfl(m.j, d), ds = __shfl(m.s, d);
    const int dk = __shfl(m.kd, d);
    if (!own) {
      m.j = dj;
      m.s = ds;
      m.kd = dk > 0 ? dk : 1;  // the donor's child (an unlisted fallback: any child, never stored)
    }
  };
  auto load_rows = [&](const Map& m, double* in) {
    const uint32_t off = m.s * 8u;
#pragma unroll
    for (int r = 0; r < NN; ++r)
      in[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(RU, off, uint32_t(r) * so,
                                                                              kNonTemporal));
  };
  __syncthreads();
  int q = next(int(blockIdx.x));
  if (q >= ngi) return;
  int q1 = next(q + G32);
  Map m0 = map_of(q), m1 = map_of(q1);
  settle(m0);
  double in[NN];
  load_rows(m0, in);
#pragma unroll
  for (int r = 0; r < NN; ++r) asm volatile("" ::"v"(in[r]));
  asm volatile("" ::"v"(m0.j), "v"(m0.kd), "v"(m1.j), "v"(m1.s), "v"(m1.kd), "v"(m1.key));
  __builtin_amdgcn_s_waitcnt(0);
  while (q < ngi) {
    const int q2 = next(q1 + G32);
    Map m2 = map_of(q2);
    settle(m1);
    double nx[NN];
    load_rows(m1, nx);
    const int c = m0.kd - 1;
    {
      double sl[NN];
      xy_pass<N>(M[c & 1], M[(c >> 1) & 1], in, sl);
#pragma unroll
      for (int r = 0; r < NN; ++r) T[w][r][lane] = sl[r];
    }
    __syncthreads();
    const double* Mz = M[(c >> 2) & 1] + w * N;
    const uint32_t oj = m0.j * 8u;
#pragma unroll
    for (int r = 0; r < NN; ++r) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) a += Mz[k] * T[k][r][lane];
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, a), RO, oj, uint32_t(r) * sn,
                                            kNonTemporal);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NN; ++r) in[r] = nx[r];
    m0 = m1;
    m1 = m2;
    q = q1;
    q1 = q2;
  }
}

// 3D, general interpolation / projection pass, for the groups that hold a
// fused element (refined children in the same group are handled here too).
// A block of N waves takes listed groups of 64 consecutive new elements of
// one variable (grid-stride over the device-side list); lane = element and
// wave w owns z-slab w (N*N points) of the input and of the output.  The x
// and y passes act within a slab and stay in registers; the z pass mixes
// slabs through LDS.  A fused element needs two z rounds (children with z
// bit 0, then 1), a refined one a single round.  The group's copies are moved
// here as well (the copy pass leaves listed groups out).  MIXED: see
// MixedArgs.
template <int N, bool MIXED>
__global__ __launch_bounds__(64 * N) void k_interp3(const double* __restrict__ ops,
                                                    const int32_t* __restrict__ src,
                                                    const int8_t* __restrict__ kind, Count cn,
                                                    const int32_t* __restrict__ groups,
                                                    const int64_t* __restrict__ ngroups,
                                                    const double* __restrict__ uo, int64_t ldo,
                                                    double* __restrict__ un, int64_t ldn,
                                                    MixedArgs mx) {
  constexpr int NN = N * N;
  constexpr int NP = NN * N;
  __shared__ double T[2][N][NN][64];  // the x/y-passed slabs of each z round
  __shared__ double M[4][NN];         // A_0, A_1, P_0, P_1
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = cn.get();
  const int64_t ng = *ngroups;
  if (int64_t(blockIdx.x) >= ng) return;
  for (int i = threadIdx.x; i < 4 * NN; i += blockDim.x) M[i / NN][i % NN] = ops[i];
  const int v = blockIdx.y;
  const int64_t vstride = MIXED ? mx.npm : NP;
  const double* U = uo + int64_t(v) * vstride * ldo + int64_t(w) * NN * ldo;
  __syncthreads();
  for (int64_t gi = blockIdx.x; gi < ng; gi += gridDim.x) {
    int64_t grp = groups[gi];
    if constexpr (MIXED) {
      if ((grp & 3) != N - 1) continue;  // another degree's entry (uniform over the block)
      grp >>= 2;
    }
    const int64_t j = grp * 64 + lane;
    bool live = j < n;
    if constexpr (MIXED) live = live && int(mx.np_of_mesh[key_mesh(mx.g, mx.keys[j])]) == NP;
    const int kd = live ? int(kind[j]) : 0;
    const int64_t s = live ? int64_t(src[j]) : 0;
    const int c = kd > 0 ? kd - 1 : 0;
    const bool copy = !MIXED && live && kd == 0;  // a copy of the group (the copy pass left the group out)
    // x and y passes: a refined child from its parent's slab w (round 0), a
    // fused parent from the slabs w of its four children of each z half
    // (rounds 0 and 1), each child's rows loaded while the one before is
    // projected
    if (kd > 0) {
      double in[NN], sl[NN];
#pragma unroll
      for (int r = 0; r < NN; ++r) in[r] = U[int64_t(r) * ldo + s];
      xy_pass<N>(M[c & 1], M[(c >> 1) & 1], in, sl);
#pragma unroll
      for (int r = 0; r < NN; ++r) T[0][w][r][lane] = sl[r];
    } else if (kd < 0) {
#pragma unroll 1
      for (int rz = 0; rz < 2; ++rz) {
        double sl[NN], in[2][NN];
#pragma unroll
        for (int r = 0; r < NN; ++r) {
          sl[r] = 0.0;
          in[0][r] = U[int64_t(r) * ldo + s + 4 * rz];
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          if (cc < 3) {
#pragma unroll
            for (int r = 0; r < NN; ++r) in[(cc + 1) & 1][r] = U[int64_t(r) * ldo + s + 4 * rz + cc + 1];
          }
          double t[NN];
          xy_pass<N>(M[2 + (cc & 1)], M[2 + (cc >> 1)], in[cc & 1], t);
#pragma unroll
          for (int r = 0; r < NN; ++r) sl[r] += t[r];
        }
#pragma unroll
        for (int r = 0; r < NN; ++r) T[rz][w][r][lane] = sl[r];
      }
    }
    __syncthreads();
    // z pass over the slabs of the block's waves, and the stores
    double* O = un + int64_t(v) * vstride * ldn + int64_t(w) * NN * ldn + j;
    if (kd > 0) {
      const double* Mz = M[(c >> 2) & 1] + w * N;
#pragma unroll
      for (int r = 0; r < NN; ++r) {
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) a += Mz[k] * T[0][k][r][lane];
        __builtin_nontemporal_store(a, O + int64_t(r) * ldn);
      }
    } else if (kd < 0) {
      const double* P0 = M[2] + w * N;
      const double* P1 = M[3] + w * N;
#pragma unroll
      for (int r = 0; r < NN; ++r) {
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) a += P0[k] * T[0][k][r][lane];
#pragma unroll
        for (int k = 0; k < N; ++k) a += P1[k] * T[1][k][r][lane];
        __builtin_nontemporal_store(a, O + int64_t(r) * ldn);
      }
    } else if (copy) {
#pragma unroll
      for (int r = 0; r < NN; ++r)
        __builtin_nontemporal_store(__builtin_nontemporal_load(U + int64_t(r) * ldo + s), O + int64_t(r) * ldn);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------- mixed degrees
// An ensemble whose meshes carry their own degree (3D, p 1..3) in one
// solution layout u[(v * NPM + i) * ld + e], NPM = the largest point count;
// an element of a mesh with N = p+1 points per axis uses rows i < N^3 of each
// variable block.  np_of_mesh[m] = N^3 of mesh m.  The copy pass and the
// group lists below handle all degrees in one launch; the interpolation runs
// the uniform kernels once per degree present over the (group, degree)
// entries (their MIXED form).

__device__ inline int elem_np(const KeyGeom& g, const uint8_t* __restrict__ np_of_mesh, uint64_t key) {
  return np_of_mesh[key_mesh(g, key)];
}

// Pure copy runs as k_copy_chunks, plus the largest point count of the
// chunk's elements (rows beyond it are skipped by the copy pass).
template <int EPL>
__global__ __launch_bounds__(256) void k_copy_chunks_mixed(KeyGeom g, const uint64_t* __restrict__ keys,
                                                           const uint8_t* __restrict__ np_of_mesh,
                                                           const int32_t* __restrict__ src,
                                                           const int8_t* __restrict__ kind, Count cn,
                                                           int64_t* __restrict__ cdelta,
                                                           int32_t* __restrict__ cnp) {
  constexpr int64_t CH = 256 * EPL;
  __shared__ int s_np;
  const int64_t n = cn.get();
  const int64_t c = blockIdx.x;
  const int64_t j0 = c * CH;
  if (j0 >= n) {
    if (threadIdx.x == 0) {
      cdelta[c] = kImpure;
      cnp[c] = 0;
    }
    return;
  }
  if (threadIdx.x == 0) s_np = 0;
  __syncthreads();
  const bool head = kind[j0] == 0;
  const int64_t ref = head ? int64_t(src[j0]) - j0 : 0;
  bool ok = head;
  int mx = 0;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int64_t j = j0 + int64_t(e) * 256 + threadIdx.x;
    if (j < n) {
      ok = ok && kind[j] == 0 && int64_t(src[j]) - j == ref;
      mx = max(mx, elem_np(g, np_of_mesh, keys[j]));
    }
  }
  atomicMax(&s_np, mx);
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) {
    cdelta[c] = ok ? ref : kImpure;
    cnp[c] = s_np;
  }
}

// The copy pass over the rows the chunk's elements own: a workgroup per
// (chunk, variable) walks rows i < the chunk's largest point count (so that
// no workgroup is launched for rows no element of the chunk owns).
template <int EPL>
__global__ __launch_bounds__(256) void k_copy3_mixed(const int32_t* __restrict__ src,
                                                     const int8_t* __restrict__ kind, Count cn,
                                                     const int64_t* __restrict__ cdelta,
                                                     const int32_t* __restrict__ cnp, int npm,
                                                     const double* __restrict__ uo, int64_t ldo,
                                                     double* __restrict__ un, int64_t ldn) {
  constexpr int64_t CH = 256 * EPL;
  const int64_t n = cn.get();
  const int64_t c = xcd_chunk(blockIdx.x, gridDim.x);
  if (c * CH >= n) return;
  const int rows = cnp[c];
  const int64_t r0 = int64_t(blockIdx.y) * npm;
  const int64_t dl = cdelta[c];
  if (dl != kImpure) {
#pragma unroll 4
    for (int i = 0; i < rows; ++i) {
      const double* U = uo + (r0 + i) * ldo;
      double* O = un + (r0 + i) * ldn;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int64_t j = c * CH + int64_t(e) * 256 + threadIdx.x;
        if (j < n) __builtin_nontemporal_store(__builtin_nontemporal_load(U + j + dl), O + j);
      }
    }
    return;
  }
  int64_t sj[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int64_t jj = c * CH + int64_t(e) * 256 + threadIdx.x;
    sj[e] = jj < n && kind[jj] == 0 ? int64_t(src[jj]) : -1;
  }
#pragma unroll 4
  for (int i = 0; i < rows; ++i) {
    const double* U = uo + (r0 + i) * ldo;
    double* O = un + (r0 + i) * ldn;
#pragma unroll
    for (int e = 0; e < EPL; ++e)
      if (sj[e] >= 0)
        __builtin_nontemporal_store(__builtin_nontemporal_load(U + sj[e]),
                                    O + c * CH + int64_t(e) * 256 + threadIdx.x);
  }
}

// Work entries of the interpolation passes: (group << 2) | (N - 1) for every
// degree N present among a group's refined / fused elements.  Groups whose
// elements of degree N are refined only go to the ordered list (look-back
// scan, one entry per such (group, degree)); the others to flist (any order).
__global__ __launch_bounds__(kScanSmall) void k_group_list_mixed(KeyGeom g, const uint64_t* __restrict__ keys,
                                                                 const uint8_t* __restrict__ np_of_mesh,
                                                                 const int8_t* __restrict__ kind, Count cn,
                                                                 int32_t* __restrict__ list, ScanState st,
                                                                 int32_t* __restrict__ flist,
                                                                 int64_t* __restrict__ nflist) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = cn.get();
  const int64_t ngroups = st.items.get();
  const int64_t base = tile * kTileMin + int64_t(threadIdx.x) * kItems;
  unsigned refmask[kItems];  // bit N-1: a degree-N refined-only entry
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t gidx = base + k;
    refmask[k] = 0;
    if (gidx >= ngroups) continue;
    unsigned any = 0, fus = 0;  // bit N-1 per degree
    const int64_t j0 = gidx * 64;
    if (j0 + 64 <= n) {  // a group of copies only (nearly all): eight words, no element loop
      const uint64_t* w8 = reinterpret_cast<const uint64_t*>(kind + j0);
      uint64_t acc = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) acc |= w8[q];
      if (acc == 0) continue;
    }
    for (int64_t j = j0; j < j0 + 64 && j < n; ++j) {
      const int kd = kind[j];
      if (kd == 0) continue;
      const int np = elem_np(g, np_of_mesh, keys[j]);
      const int N = np == 8 ? 2 : (np == 27 ? 3 : 4);
      any |= 1u << (N - 1);
      if (kd < 0) fus |= 1u << (N - 1);
    }
    for (int N = 2; N <= 4; ++N)
      if (fus & (1u << (N - 1))) {
        const int64_t o = int64_t(atomicAdd(reinterpret_cast<unsigned long long*>(nflist), 1ull));
        flist[o] = int32_t(gidx * 4 + (N - 1));
      }
    refmask[k] = any & ~fus;
    local += __popc(refmask[k]);
  }
  int64_t blk;
  const int64_t thr = block_exclusive<kScanSmall>(local, &blk);
  int64_t o = tile_prefix(st, tile, blk) + thr;
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    for (int N = 2; N <= 4; ++N)
      if (refmask[k] & (1u << (N - 1))) list[o++] = int32_t((base + k) * 4 + (N - 1));
}

// Scratch of one FP64 transfer, sized for n new leaves: per copy chunk the
// source offset of a pure copy run (ceil(n / 256) entries at the finest
// tuning), the interpolation-group lists (the ordered list of groups with a
// refined element, then the groups holding a fused one: 2 ceil(n / 64)),
// look-back words and counters.  From the tree's buffers (lt_transfer) or
// from the library's static array (lt_transfer_noalloc).
struct XferScratch {
  int64_t* copy_delta;
  int32_t* grp_list;
  uint64_t* status;
  int64_t status_cap;
  DevCtr* ctr;
  // a second stream for the interpolation passes, forked from and joined to
  // the caller's (null: everything on the caller's stream)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

lt_status copy_pass(const TransferTune& tune, const int32_t* src, const int8_t* kind, Count n,
                    int64_t rows, const double* uo, int64_t ldo, double* un, int64_t ldn,
                    int64_t* copy_delta, bool skip_groups, hipStream_t s);

template <int DIM, int N>
hipError_t launch(const TransferTune& tune, const double* ops, const int32_t* src, const int8_t* kind,
                  Count n, const int64_t* ngroups_dev, int nvar, const double* uo, int64_t ldo,
                  double* un, int64_t ldn, const XferScratch& X, hipStream_t s, lt_status* st_out) {
  *st_out = LT_OK;
  if constexpr (DIM == 3) {
    hipError_t e = hipSuccess;
    const int64_t ngroups = (n.n + 63) / 64;
    // The copy pass leaves out every group the interpolation passes write
    // (their copies included), so the two write disjoint elements and run at
    // once when a second stream is given: the interpolation passes, bound by
    // their dependent loads, then overlap the copy's streaming traffic.  The
    // copy is enqueued first, so that its start waits on no host call of
    // the fork.
    hipStream_t si = s;
    if (X.side) {
      e = hipEventRecord(X.fork, s);
      if (e != hipSuccess) return e;
      si = X.side;
    }
    *st_out = copy_pass(tune, src, kind, n, nvar * N * N * N, uo, ldo, un, ldn, X.copy_delta, true, s);
    if (X.side) e = hipStreamWaitEvent(X.side, X.fork, 0);
    // grp_list holds the ordered list in [0, ngroups) and the list of
    // groups with a fused element in [ngroups, 2 ngroups)
    ScanState st;
    if (*st_out == LT_OK && e == hipSuccess)
      *st_out = prep_scan_fixed(X.status, X.status_cap, X.ctr, ngroups, kTileMin, si, 0, &st);
    if (*st_out == LT_OK && e == hipSuccess) {
      st.items.p = ngroups_dev;
      int32_t* flist = X.grp_list + ngroups;
      k_group_list<<<grid_tiles(st), kScanSmall, 0, si>>>(kind, n, X.grp_list, st, flist,
                                                      &X.ctr->nfgroups);
      const dim3 gi{unsigned(std::max<int64_t>(1, std::min<int64_t>(ngroups, tune.interp_grid))),
                    unsigned(nvar), 1u};
      // the buffer form takes N*N rows of either array by a 32-bit offset
      constexpr int64_t kRowsMax = (int64_t(1) << 32) / (8 * N * N);
      if (ldo < kRowsMax && ldn < kRowsMax)
        k_refine3<N><<<gi, 64 * N, 0, si>>>(ops, src, kind, n, X.grp_list, st.total, uo, ldo, un, ldn);
      else
        k_interp3_ref<N, false><<<gi, 64 * N, 0, si>>>(ops, src, kind, n, X.grp_list, st.total, uo,
                                                       ldo, un, ldn, MixedArgs{});
      k_interp3<N, false><<<gi, 64 * N, 0, si>>>(ops, src, kind, n, flist, &X.ctr->nfgroups, uo, ldo, un,
                                                 ldn, MixedArgs{});
      e = hipGetLastError();
    }
    // the join is recorded on every path that forked, so that a capture
    // in progress stays whole
    if (X.side) {
      const hipError_t ej = hipEventRecord(X.join, X.side);
      const hipError_t ew = ej == hipSuccess ? hipStreamWaitEvent(s, X.join, 0) : ej;
      if (e == hipSuccess) e = ew;
    }
    return e;
  } else {
    dim3 grid(unsigned((n.n + 255) / 256), unsigned(nvar));
    k_transfer<DIM, N><<<grid, 256, 0, s>>>(ops, src, kind, n, uo, ldo, un, ldn);
    return hipGetLastError();
  }
}

}  // namespace

namespace {
lt_status copy_pass(const TransferTune& tune, const int32_t* src, const int8_t* kind, Count n,
                    int64_t rows, const double* uo, int64_t ldo, double* un, int64_t ldn,
                    int64_t* copy_delta, bool skip_groups, hipStream_t s) {
  if (n.n == 0) return LT_OK;
  if (rows < 1 || rows > 65535) return fail(LT_ERR_ARG, "copy pass: rows out of range");
  const int epl = tune.copy_epl;
  const int64_t CH = 256 * int64_t(epl);
  const int64_t nchunks = (n.n + CH - 1) / CH;
  // A capacity-sized launch with a hint: workgroups for the hinted count and
  // a 32nd more, striding over whatever lies beyond.  The slack keeps
  // striding rare (a workgroup's second chunk waits behind its first: a grid
  // of 15/16 of the count made the captured cycle ~12% slower), and it stays
  // small because every workgroup past the count is still dispatched, one per
  // chunk and row, only to exit (an eighth more cost ~58 us per captured
  // cycle at 1.66M leaves).
  const int64_t nlaunch =
      n.hint > 0 ? std::max<int64_t>(1, std::min(nchunks, (n.hint + n.hint / 32 + CH - 1) / CH)) : nchunks;
  const dim3 grid{unsigned(nlaunch), unsigned(rows), 1u};
#define LT_COPY(E)                                                                              \
  do {                                                                                          \
    k_copy_chunks<E><<<unsigned(nchunks), 256, 0, s>>>(src, kind, n, copy_delta);               \
    if (skip_groups)                                                                            \
      k_copy3<E, true><<<grid, 256, 0, s>>>(src, kind, n, copy_delta, uo, ldo, un, ldn);        \
    else                                                                                        \
      k_copy3<E, false><<<grid, 256, 0, s>>>(src, kind, n, copy_delta, uo, ldo, un, ldn);       \
  } while (0)
  if (epl == 1)
    LT_COPY(1);
  else if (epl == 4)
    LT_COPY(4);
  else
    LT_COPY(2);
#undef LT_COPY
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("copy pass launch: ") + hipGetErrorString(e));
  return LT_OK;
}
}  // namespace

lt_status launch_copy(lt_tree_s* t, Count n, int64_t rows, const double* uo, int64_t ldo,
                      double* un, int64_t ldn, hipStream_t s) {
  if (n.n == 0) return LT_OK;
  const int64_t CH = 256 * int64_t(t->tune.copy_epl);
  LT_TRY_STATUS(grow(t->A, &t->copy_delta, &t->copy_delta_cap, (n.n + CH - 1) / CH));
  return copy_pass(t->tune, t->map_src, t->map_kind, n, rows, uo, ldo, un, ldn, t->copy_delta, false, s);
}

lt_status build_transfer_ops(const Alloc& A, int p, double** ops, hipStream_t stream) {
  if (*ops) return LT_OK;
  const int n = p + 1;
  void* q = nullptr;
  hipError_t e = dev_malloc(A, &q, sizeof(double) * (4 * n * n + n));
  if (e != hipSuccess) return fail(LT_ERR_OOM, "transfer operator allocation failed");
  k_build_ops<<<1, 64, 0, stream>>>(n, static_cast<double*>(q));
  e = hipGetLastError();
  if (e != hipSuccess) {
    (void)dev_free(A, q);
    return fail(LT_ERR_HIP, std::string("operator build: ") + hipGetErrorString(e));
  }
  *ops = static_cast<double*>(q);
  return LT_OK;
}

lt_status launch_copy(lt_tree_s* t, int64_t rows, const double* uo, int64_t ldo, double* un,
                      int64_t ldn, hipStream_t s) {
  return launch_copy(t, Count{t->n_cur, nullptr}, rows, uo, ldo, un, ldn, s);
}

lt_status launch_transfer(lt_tree_s* t, int p, const double* ops, int nvar, const double* u_old,
                          int64_t ld_old, double* u_new, int64_t ld_new, hipStream_t s) {
  return launch_transfer(t, Count{t->n_cur, nullptr}, nullptr, p, ops, nvar, u_old, ld_old, u_new,
                         ld_new, s);
}

namespace {
// The FP64 transfer over n new leaves of a mapping (src, kind) with the given
// scratch; no allocation.
lt_status transfer_with(int dim, const TransferTune& tune, const int32_t* src, const int8_t* kind,
                        Count n, const int64_t* ngroups_dev, int p, const double* ops, int nvar,
                        const double* u_old, int64_t ld_old, double* u_new, int64_t ld_new,
                        const XferScratch& X, hipStream_t s) {
  if (n.n == 0) return LT_OK;
  int64_t npts = 1;
  for (int a = 0; a < dim; ++a) npts *= p + 1;
  if (nvar < 1 || int64_t(nvar) * npts > 65535)
    return fail(LT_ERR_ARG, "nvar * (p+1)^dim must be in [1, 65535]");
  hipError_t e = hipErrorInvalidValue;
  lt_status st = LT_OK;
#define LT_L(D, NN) e = launch<D, NN>(tune, ops, src, kind, n, ngroups_dev, nvar, u_old, ld_old, u_new, ld_new, X, s, &st)
  if (dim == 3) {
    switch (p) {
      case 1: LT_L(3, 2); break;
      case 2: LT_L(3, 3); break;
      case 3: LT_L(3, 4); break;
      default: return fail(LT_ERR_ARG, "3D transfer supports p = 1..3");
    }
  } else {
    switch (p) {
      case 1: LT_L(2, 2); break;
      case 2: LT_L(2, 3); break;
      case 3: LT_L(2, 4); break;
      case 4: LT_L(2, 5); break;
      case 5: LT_L(2, 6); break;
      case 6: LT_L(2, 7); break;
      case 7: LT_L(2, 8); break;
      default: return fail(LT_ERR_ARG, "2D transfer supports p = 1..7");
    }
  }
#undef LT_L
  if (st != LT_OK) return st;
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("transfer launch: ") + hipGetErrorString(e));
  return LT_OK;
}
}  // namespace

lt_status transfer_side(lt_tree_s* t, hipStream_t* side, hipEvent_t* fork, hipEvent_t* join) {
  if (!t->xs) {
    hipStream_t q = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (q) (void)hipStreamDestroy(q);
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      return fail(LT_ERR_HIP, std::string("transfer stream: ") + hipGetErrorString(e));
    }
    t->xs = q;
    t->xev[0] = a;
    t->xev[1] = b;
  }
  *side = t->xs;
  *fork = t->xev[0];
  *join = t->xev[1];
  return LT_OK;
}

lt_status launch_transfer_mixed(lt_tree_s* t, const uint64_t* keys, Count n, const int64_t* ngroups_dev,
                                int nvar, const double* uo, int64_t ldo, double* un, int64_t ldn,
                                hipStream_t s) {
  if (n.n == 0) return LT_OK;
  if (!t->mesh_np || t->g.dim != 3) return fail(LT_ERR_STATE, "per-mesh degrees are not set");
  const int npm = t->mesh_npm;
  if (nvar < 1 || int64_t(nvar) * npm > 65535) return fail(LT_ERR_ARG, "nvar * points out of range");
  const double* ops[3] = {nullptr, nullptr, nullptr};
  for (int p = 1; p <= 3; ++p)
    if (t->mesh_degs & (1u << p)) {
      LT_TRY_STATUS(build_transfer_ops(t->A, p, &t->ops[p], s));
      ops[p - 1] = t->ops[p];
    }
  const int epl = t->tune.copy_epl;
  const int64_t CH = 256 * int64_t(epl);
  const int64_t nchunks = (n.n + CH - 1) / CH;
  const int64_t ngroups = (n.n + 63) / 64;
  LT_TRY_STATUS(grow(t->A, &t->copy_delta, &t->copy_delta_cap, nchunks));
  LT_TRY_STATUS(grow(t->A, &t->chunk_np, &t->chunk_np_cap, nchunks));
  LT_TRY_STATUS(grow(t->A, &t->grp_list, &t->grp_cap, 6 * ngroups));
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  LT_TRY_STATUS(transfer_side(t, &side, &fork, &join));
  // The group list first, alone on the caller's stream: beside the copy pass
  // its look-back tiles wait for wave slots behind the copy's workgroups
  // (~0.3 ms alone, ~2 ms beside it at 10M leaves), and the interpolation
  // passes on the second stream need it.  Then the copy pass on the caller's
  // stream and, as in the single-degree form, the interpolation passes
  // (which here write no copies) on the second stream.
  ScanState st;
  LT_TRY_STATUS(prep_scan(t, ngroups, kTileMin, s, 0, &st));
  st.items.p = ngroups_dev;
  int32_t* flist = t->grp_list + 3 * ngroups;
  k_group_list_mixed<<<grid_tiles(st), kScanSmall, 0, s>>>(t->g, keys, t->mesh_np, t->map_kind, n,
                                                           t->grp_list, st, flist, &t->dctr->nfgroups);
  hipError_t ef = hipEventRecord(fork, s);
  if (ef != hipSuccess) return fail(LT_ERR_HIP, std::string("transfer fork: ") + hipGetErrorString(ef));
  const dim3 grid{unsigned(nchunks), unsigned(nvar), 1u};
#define LT_CM(E)                                                                                    \
  do {                                                                                              \
    k_copy_chunks_mixed<E><<<unsigned(nchunks), 256, 0, s>>>(t->g, keys, t->mesh_np, t->map_src,     \
                                                            t->map_kind, n, t->copy_delta,          \
                                                            t->chunk_np);                           \
    k_copy3_mixed<E><<<grid, 256, 0, s>>>(t->map_src, t->map_kind, n, t->copy_delta, t->chunk_np,   \
                                          npm, uo, ldo, un, ldn);                                   \
  } while (0)
  if (epl == 1)
    LT_CM(1);
  else if (epl == 4)
    LT_CM(4);
  else
    LT_CM(2);
#undef LT_CM
  ef = hipStreamWaitEvent(side, fork, 0);
  if (ef == hipSuccess) {
    // one launch of each interpolation kernel per degree present; the blocks
    // of a launch skip the other degrees' entries
    const dim3 gi{unsigned(std::max<int64_t>(1, std::min<int64_t>(3 * ngroups, t->tune.interp_grid))),
                  unsigned(nvar), 1u};
    const MixedArgs mx{t->g, keys, t->mesh_np, npm};
    // the buffer form takes N*N rows of either array by a 32-bit offset and
    // the mesh-degree table in LDS
    auto buffer_ok = [&](int nn) {
      const int64_t rows_max = (int64_t(1) << 32) / (8 * nn * nn);
      return ldo < rows_max && ldn < rows_max && t->g.nmesh <= kMeshTab;
    };
#define LT_MX(NN, OPS)                                                                                 \
  do {                                                                                                 \
    if (buffer_ok(NN))                                                                                 \
      k_refine3_mixed<NN><<<gi, 64 * NN, 0, side>>>(OPS, t->map_src, t->map_kind, n, t->grp_list,      \
                                                    st.total, uo, ldo, un, ldn, mx, t->g.nmesh);       \
    else                                                                                               \
      k_interp3_ref<NN, true><<<gi, 64 * NN, 0, side>>>(OPS, t->map_src, t->map_kind, n, t->grp_list,  \
                                                        st.total, uo, ldo, un, ldn, mx);               \
    k_interp3<NN, true><<<gi, 64 * NN, 0, side>>>(OPS, t->map_src, t->map_kind, n, flist,              \
                                                  &t->dctr->nfgroups, uo, ldo, un, ldn, mx);           \
  } while (0)
    if (ops[0]) LT_MX(2, ops[0]);
    if (ops[1]) LT_MX(3, ops[1]);
    if (ops[2]) LT_MX(4, ops[2]);
#undef LT_MX
  }
  const hipError_t e = hipGetLastError();
  // the join on every path that forked, so that a capture in progress stays whole
  const hipError_t ej = hipEventRecord(join, side);
  const hipError_t ew = ej == hipSuccess ? hipStreamWaitEvent(s, join, 0) : ej;
  if (ef != hipSuccess) return fail(LT_ERR_HIP, std::string("transfer fork: ") + hipGetErrorString(ef));
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("mixed transfer launch: ") + hipGetErrorString(e));
  if (ew != hipSuccess) return fail(LT_ERR_HIP, std::string("transfer join: ") + hipGetErrorString(ew));
  return LT_OK;
}

lt_status launch_transfer(lt_tree_s* t, Count n, const int64_t* ngroups_dev, int p,
                          const double* ops, int nvar, const double* u_old, int64_t ld_old,
                          double* u_new, int64_t ld_new, hipStream_t s) {
  if (n.n == 0) return LT_OK;
  XferScratch X{};
  if (t->g.dim == 3) {
    const int64_t ngroups = (n.n + 63) / 64;
    const int64_t CH = 256 * int64_t(t->tune.copy_epl);
    LT_TRY_STATUS(grow(t->A, &t->copy_delta, &t->copy_delta_cap, (n.n + CH - 1) / CH));
    LT_TRY_STATUS(grow(t->A, &t->grp_list, &t->grp_cap, 2 * ngroups));
    LT_TRY_STATUS(grow(t->A, &t->status, &t->status_cap,
                       std::max<int64_t>(1, (ngroups + kTileMin - 1) / kTileMin)));
    X = XferScratch{t->copy_delta, t->grp_list, t->status, t->status_cap, t->dctr};
    LT_TRY_STATUS(transfer_side(t, &X.side, &X.fork, &X.join));
  }
  return transfer_with(t->g.dim, t->tune, t->map_src, t->map_kind, n, ngroups_dev, p, ops, nvar,
                       u_old, ld_old, u_new, ld_new, X, s);
}

}  // namespace lt

// ------------------------------------------------------- allocation-free form
namespace lt {
namespace {

// Static scratch of lt_transfer_noalloc, one copy per GPU (the device keeps
// it until the process ends), laid out for up to kNoallocLeaves new leaves:
//   [0, 4 KiB)       FP64 1D operators (4 (p+1)^2 + (p+1) doubles, p <= 7)
//   [4 KiB, 8 KiB)   counters (DevCtr)
//   [8 KiB, 16 KiB)  look-back words of the group scan
//   then             copy-chunk source offsets, interpolation-group lists.
constexpr int64_t kNoallocLeaves = int64_t(1) << 25;
constexpr size_t kOffOps = 0, kOffCtr = 4096, kOffStatus = 8192, kOffDelta = 16384;
constexpr int64_t kStatusWords = (kOffDelta - kOffStatus) / 8;
constexpr int64_t kDeltaWords = kNoallocLeaves / 256 + 2;
constexpr size_t kOffGroups = kOffDelta + size_t(kDeltaWords) * 8;
constexpr int64_t kGroupWords = 2 * (kNoallocLeaves / 64 + 2);
constexpr size_t kScratchBytes = (kOffGroups + size_t(kGroupWords) * 4 + 255) / 256 * 256;
static_assert(sizeof(double) * (4 * 8 * 8 + 8) <= kOffCtr - kOffOps, "operators fit");
static_assert(sizeof(DevCtr) <= kOffStatus - kOffCtr, "counters fit");
static_assert((kNoallocLeaves / 64 + kTileMin - 1) / kTileMin <= kStatusWords, "look-back words fit");

// In host code this name is only a stand-in for the symbol: the device
// address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};

// The device address of `scratch` on the current device, looked up on the
// first call there.
lt_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= 64) return fail(LT_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LT_ERR_HIP, std::string("static scratch address: ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_dev[dev]);
  return LT_OK;
}

}  // namespace
}  // namespace lt

// ------------------------------------------------------------------ tuning
using namespace lt;

extern "C" {

lt_status lt_transfer_noalloc(lt_tree t, int p, int nvar, const double* u_old, int64_t ld_old,
                              double* u_new, int64_t ld_new, void* stream) {
  if (!t || !u_old || !u_new) return fail(LT_ERR_ARG, "NULL argument");
  if (nvar < 1) return fail(LT_ERR_ARG, "nvar must be positive");
  if (p < 1 || p > (t->g.dim == 3 ? 3 : LT_MAX_DEGREE))
    return fail(LT_ERR_ARG, "unsupported polynomial degree for this dimension");
  if (t->n_cur > kNoallocLeaves)
    return fail(LT_ERR_ARG, "lt_transfer_noalloc takes at most 2^25 leaves (" +
                                std::to_string(t->n_cur) + " given)");
  if (!t->has_old || !t->map_valid)
    return fail(LT_ERR_STATE, "lt_transfer_noalloc needs the mapping of an adaptation (lt_map)");
  if (ld_old < t->n_old || ld_new < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LT_ERR_HIP, "hipGetDevice");
  if (dev != t->device) return fail(LT_ERR_ARG, "the tree lives on another device than the current one");
  unsigned char* base = nullptr;
  LT_TRY_STATUS(scratch_address(dev, &base));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* ops = reinterpret_cast<double*>(base + kOffOps);
  k_build_ops<<<1, 64, 0, s>>>(p + 1, ops);
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "operator build launch");
  const XferScratch X{reinterpret_cast<int64_t*>(base + kOffDelta),
                      reinterpret_cast<int32_t*>(base + kOffGroups),
                      reinterpret_cast<uint64_t*>(base + kOffStatus), kStatusWords,
                      reinterpret_cast<DevCtr*>(base + kOffCtr)};
  return transfer_with(t->g.dim, t->tune, t->map_src, t->map_kind, Count{t->n_cur, nullptr}, nullptr,
                       p, ops, nvar, u_old, ld_old, u_new, ld_new, X, s);
}

lt_status lt_set_mesh_degree(lt_tree t, const int* p, void* stream) {
  if (!t || !p) return fail(LT_ERR_ARG, "NULL argument");
  if (t->g.dim != 3) return fail(LT_ERR_ARG, "per-mesh degrees are for 3D ensembles");
  const int nm = t->g.nmesh;
  std::vector<uint8_t> np(static_cast<size_t>(nm));
  unsigned degs = 0;
  int npm = 0;
  for (int m = 0; m < nm; ++m) {
    if (p[m] < 1 || p[m] > 3) return fail(LT_ERR_ARG, "mesh degrees must be 1..3");
    np[m] = uint8_t((p[m] + 1) * (p[m] + 1) * (p[m] + 1));
    degs |= 1u << p[m];
    npm = std::max(npm, int(np[m]));
  }
  if (!t->mesh_np &&
      dev_malloc(t->A, reinterpret_cast<void**>(&t->mesh_np), std::max<size_t>(nm, 256)) != hipSuccess)
    return fail(LT_ERR_OOM, "mesh degree table");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(t->mesh_np, np.data(), np.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LT_ERR_HIP, "mesh degree upload");
  t->mesh_degs = degs;
  t->mesh_npm = npm;
  return LT_OK;
}

lt_status lt_transfer_mixed(lt_tree t, int nvar, const double* u_old, int64_t ld_old, double* u_new,
                            int64_t ld_new, void* stream) {
  if (!t || !u_old || !u_new) return fail(LT_ERR_ARG, "NULL argument");
  if (!t->mesh_np) return fail(LT_ERR_STATE, "lt_transfer_mixed needs lt_set_mesh_degree");
  if (!t->has_old) return fail(LT_ERR_STATE, "lt_transfer_mixed needs a prior lt_adapt");
  if (ld_old < t->n_old || ld_new < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  if (!t->map_valid) LT_TRY_STATUS(lt_map(t, stream));
  return launch_transfer_mixed(t, t->kbuf[t->cur], Count{t->n_cur, nullptr}, nullptr, nvar, u_old, ld_old,
                               u_new, ld_new, static_cast<hipStream_t>(stream));
}

lt_status lt_set_tuning(lt_tree t, const lt_tune* tune) {
  if (!t || !tune) return fail(LT_ERR_ARG, "NULL argument");
  const int e = tune->copy_elems_per_lane;
  if (e != 1 && e != 2 && e != 4) return fail(LT_ERR_ARG, "copy_elems_per_lane must be 1, 2 or 4");
  if (tune->interp_grid < 1 || tune->interp_grid > 65535) return fail(LT_ERR_ARG, "interp_grid out of range");
  t->tune.copy_epl = e;
  t->tune.interp_grid = tune->interp_grid;
  return LT_OK;
}

lt_status lt_get_tuning(lt_tree t, lt_tune* tune) {
  if (!t || !tune) return fail(LT_ERR_ARG, "NULL argument");
  tune->copy_elems_per_lane = t->tune.copy_epl;
  tune->interp_grid = t->tune.interp_grid;
  tune->ms = -1.f;
  tune->ms_default = -1.f;
  return LT_OK;
}

lt_status lt_autotune_transfer(lt_tree t, int p, int nvar, const double* u_old, int64_t ld_old,
                               double* u_new, int64_t ld_new, int precision, void* stream, lt_tune* out) {
  if (!t) return fail(LT_ERR_ARG, "NULL tree");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(LT_ERR_HIP, "event create");
  const TransferTune keep = t->tune;
  const int epls[3] = {1, 2, 4};
  const int grids[5] = {1024, 2048, 4096, 16384, 65535};
  TransferTune best = keep;
  float best_ms = 1e30f, default_ms = -1.f;
  lt_status st = LT_OK;
  for (int a = 0; a < 3 && st == LT_OK; ++a)
    for (int b = 0; b < 5 && st == LT_OK; ++b) {
      t->tune.copy_epl = epls[a];
      t->tune.interp_grid = grids[b];
      // one untimed launch, then three timed ones (every candidate writes the same result)
      st = lt_transfer(t, p, nvar, u_old, ld_old, u_new, ld_new, precision, stream);
      if (st != LT_OK) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 3 && st == LT_OK; ++r)
        st = lt_transfer(t, p, nvar, u_old, ld_old, u_new, ld_new, precision, stream);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) st = fail(LT_ERR_HIP, "event sync");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= 3.f;
      if (epls[a] == TransferTune{}.copy_epl && grids[b] == TransferTune{}.interp_grid) default_ms = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = t->tune;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  t->tune = st == LT_OK ? best : keep;
  if (st != LT_OK) return st;
  if (out) {
    out->copy_elems_per_lane = best.copy_epl;
    out->interp_grid = best.interp_grid;
    out->ms = best_ms;
    out->ms_default = default_ms;
  }
  return LT_OK;
}

}  // extern "C"
