// lt_split.hip -- split-precision solution transfer on BF16 MFMA.
//
// The same operators as the FP64 transfer of Section 4.2 (interpolation of
// the parent polynomial on refinement, L2 projection on coarsening), applied
// as dense (p+1)^d x (p+1)^d products on the matrix cores:
//   * every operator entry and every FP64 solution value is split into three
//     BF16 terms, x ~ x0 + x1 + x2 (each the BF16 rounding of the remainder);
//   * the six products a0b0, a0b1, a1b0, a0b2, a1b1, a2b0 are accumulated in
//     FP32 by v_mfma_f32_16x16x32_bf16 (smallest first);
//   * the result is shifted per element so that its cell mean (the
//     Gauss-Legendre quadrature mean) equals the FP64 cell mean: for a refined
//     child the mean of the parent polynomial over the child, for a fused
//     parent the average of its children's means (the projection conserves
//     the integral).
// Supported: 64 points per element (3D p = 3, 2D p = 7).  Copies are copies.
// Work lists (first child of each refined family, each fused parent) are
// built on the device by a look-back scan, so the call never synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "tree.hpp"

namespace lt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNP = 64;        // points per element
constexpr int kMT = kNP / 16;  // 16-row tiles of an operator
constexpr int kKS = kNP / 32;  // 32-deep K steps
constexpr int kTC = 16;        // columns (families / fused parents) per tile
constexpr int64_t kLow31 = (int64_t(1) << 31) - 1;

__device__ inline void split3(double x, __bf16& b0, __bf16& b1, __bf16& b2) {
  b0 = __bf16(float(x));
  const double r1 = x - double(float(b0));
  b1 = __bf16(float(r1));
  const double r2 = r1 - double(float(b1));
  b2 = __bf16(float(r2));
}

// Dense operator entry: op 0 interpolation I_c, op 1 projection P_c, from the
// 1D factors (A_0, A_1, P_0, P_1 row-major n1 x n1) by tensor product.
__device__ inline double dense_entry(const double* ops1d, int n1, int dim, int op, int c, int row,
                                     int k) {
  double v = 1.0;
  for (int a = 0; a < dim; ++a) {
    const int b = (c >> a) & 1;
    const double* M = ops1d + (2 * op + b) * n1 * n1;
    v *= M[(row % n1) * n1 + (k % n1)];
    row /= n1;
    k /= n1;
  }
  return v;
}

// A-operand fragments for v_mfma_f32_16x16x32_bf16: lane l of tile (mt, ks)
// holds rows mt*16 + (l % 16), columns ks*32 + 8*(l / 16) + t, t = 0..7.
// Layout: frags[((((op*nc + c)*3 + s)*kMT + mt)*kKS + ks)*64 + lane].
__global__ void k_build_split(const double* __restrict__ ops1d, int n1, int dim, int nc,
                              bf16x8* __restrict__ frags) {
  const int total = 2 * nc * kMT * kKS * 64;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int lane = id % 64, ks = (id / 64) % kKS, mt = (id / (64 * kKS)) % kMT;
  const int c = (id / (64 * kKS * kMT)) % nc, op = id / (64 * kKS * kMT * nc);
  bf16x8 f0, f1, f2;
  for (int t = 0; t < 8; ++t) {
    const int row = mt * 16 + (lane % 16), k = ks * 32 + 8 * (lane / 16) + t;
    __bf16 x0, x1, x2;
    split3(dense_entry(ops1d, n1, dim, op, c, row, k), x0, x1, x2);
    f0[t] = x0;
    f1[t] = x1;
    f2[t] = x2;
  }
  const int base = (op * nc + c) * 3;
  frags[(((base + 0) * kMT + mt) * kKS + ks) * 64 + lane] = f0;
  frags[(((base + 1) * kMT + mt) * kKS + ks) * 64 + lane] = f1;
  frags[(((base + 2) * kMT + mt) * kKS + ks) * 64 + lane] = f2;
}

// FP64 mean weights: Wn[i] = quadrature weight / element volume (sums to 1),
// and g_c[k] = sum_i Wn[i] I_c[i][k] (mean over child c of parent basis k).
__global__ void k_build_split_vec(const double* __restrict__ ops1d, int n1, int dim, int nc,
                                  double* __restrict__ vec) {
  const double* w = ops1d + 4 * n1 * n1;
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) {
    double W = 1.0;
    int r = i;
    for (int a = 0; a < dim; ++a) {
      W *= 0.5 * w[r % n1];
      r /= n1;
    }
    vec[i] = W;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nc * kNP; q += blockDim.x) {
    const int c = q / kNP, k = q % kNP;
    double s = 0.0;
    for (int i = 0; i < kNP; ++i) s += vec[i] * dense_entry(ops1d, n1, dim, 0, c, i, k);
    vec[kNP + q] = s;
  }
}

// Work lists from the mapping: R = first child of each refined family (kind
// 1), F = each fused parent (kind -1), in new-leaf order.  One scan carries
// both counts packed as nR + (nF << 31).
__global__ __launch_bounds__(kScanSmall) void k_split_lists(const int8_t* __restrict__ kind,
                                                        int32_t* __restrict__ R,
                                                        int32_t* __restrict__ F, ScanState st) {
  const int64_t tile = take_ticket(st);
  if (tile >= scan_tiles(st)) return;
  const int64_t n = st.items.get();
  const int64_t base = tile * kTileMin + int64_t(threadIdx.x) * kItems;
  int8_t kd[kItems];
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t j = base + k;
    kd[k] = j < n ? kind[j] : 0;
    local += (kd[k] == 1 ? 1 : 0) + (kd[k] == -1 ? (int64_t(1) << 31) : 0);
  }
  int64_t blk;
  const int64_t thr = block_exclusive<kScanSmall>(local, &blk);
  const int64_t o = tile_prefix(st, tile, blk) + thr;
  int64_t orr = o & kLow31, of = o >> 31;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (kd[k] == 1) R[orr++] = int32_t(base + k);
    if (kd[k] == -1) F[of++] = int32_t(base + k);
  }
}

__device__ inline f32x4 mma6(const bf16x8& a0, const bf16x8& a1, const bf16x8& a2, const bf16x8& b0,
                             const bf16x8& b1, const bf16x8& b2, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc, 0, 0, 0);
  return acc;
}

// Refinement.  A block of NC waves takes tiles of 16 refined families; wave c
// computes child c of all 16 (I_c in registers, the shared parent tile split
// once into LDS).  The D fragment of lane l holds rows 4*(l/16) + r of a
// 16-row tile, column l % 16.
template <int NC>
__global__ __launch_bounds__(64 * NC) void k_split_refine(
    const bf16x8* __restrict__ fragI, const double* __restrict__ vec, const int32_t* __restrict__ R,
    const int64_t* __restrict__ packed, const int32_t* __restrict__ src,
    const double* __restrict__ uo, int64_t ldo, double* __restrict__ un, int64_t ldn) {
  __shared__ double Bd[kNP][kTC];
  __shared__ bf16x8 Bf[3][kKS][64];
  __shared__ double Out[kNP][kTC * NC];
  __shared__ int32_t s_j0[kTC], s_src[kTC];
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int v = blockIdx.y;
  const int64_t nR = (*packed) & kLow31;
  const int64_t ntile = (nR + kTC - 1) / kTC;
  if (int64_t(blockIdx.x) >= ntile) return;
  bf16x8 a[3][kMT][kKS];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int ks = 0; ks < kKS; ++ks) a[s][mt][ks] = fragI[(((c * 3 + s) * kMT + mt) * kKS + ks) * 64 + lane];
  const double* Wn = vec;
  const double* g = vec + kNP + c * kNP;
  const double* U = uo + int64_t(v) * kNP * ldo;
  double* O = un + int64_t(v) * kNP * ldn;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    if (threadIdx.x < kTC) {
      const int64_t r = tile * kTC + threadIdx.x;
      int32_t j0 = -1, sp = -1;
      if (r < nR) {
        j0 = R[r];
        sp = src[j0];
      }
      s_j0[threadIdx.x] = j0;
      s_src[threadIdx.x] = sp;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kNP * kTC; idx += blockDim.x) {
      const int k = idx / kTC, cc = idx % kTC;
      const int32_t sp = s_src[cc];
      Bd[k][cc] = sp >= 0 ? U[int64_t(k) * ldo + sp] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < kKS * 64) {
      const int ks = threadIdx.x >> 6, l = threadIdx.x & 63;
      bf16x8 b0, b1, b2;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        __bf16 x0, x1, x2;
        split3(Bd[ks * 32 + 8 * (l >> 4) + t][l & 15], x0, x1, x2);
        b0[t] = x0;
        b1[t] = x1;
        b2[t] = x2;
      }
      Bf[0][ks][l] = b0;
      Bf[1][ks][l] = b1;
      Bf[2][ks][l] = b2;
    }
    __syncthreads();
    f32x4 acc[kMT];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kKS; ++ks) {
      const bf16x8 b0 = Bf[0][ks][lane], b1 = Bf[1][ks][lane], b2 = Bf[2][ks][lane];
#pragma unroll
      for (int mt = 0; mt < kMT; ++mt)
        acc[mt] = mma6(a[0][mt][ks], a[1][mt][ks], a[2][mt][ks], b0, b1, b2, acc[mt]);
    }
    // cell-mean correction in FP64
    double ms = 0.0, mf = 0.0;
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) ms += Wn[mt * 16 + 4 * grp + r] * double(acc[mt][r]);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) mf += g[16 * grp + kk] * Bd[16 * grp + kk][col];
    ms += __shfl_xor(ms, 16, 64);
    ms += __shfl_xor(ms, 32, 64);
    mf += __shfl_xor(mf, 16, 64);
    mf += __shfl_xor(mf, 32, 64);
    const double delta = mf - ms;
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) Out[mt * 16 + 4 * grp + r][col * NC + c] = double(acc[mt][r]) + delta;
    __syncthreads();
    for (int idx = threadIdx.x; idx < kNP * kTC * NC; idx += blockDim.x) {
      const int row = idx / (kTC * NC), q = idx % (kTC * NC);
      const int32_t j0 = s_j0[q / NC];
      if (j0 >= 0) O[int64_t(row) * ldn + j0 + (q % NC)] = Out[row][q];
    }
    __syncthreads();
  }
}

// Coarsening.  A block of NC waves takes tiles of 16 fused parents; wave c
// multiplies P_c by the values of child c (split in registers); the partial
// results are summed over the children through LDS.
template <int NC>
__global__ __launch_bounds__(64 * NC) void k_split_fuse(
    const bf16x8* __restrict__ fragP, const double* __restrict__ vec, const int32_t* __restrict__ F,
    const int64_t* __restrict__ packed, const int32_t* __restrict__ src,
    const double* __restrict__ uo, int64_t ldo, double* __restrict__ un, int64_t ldn) {
  __shared__ float Part[NC][kNP][kTC];
  __shared__ double Mc[NC][kTC];
  __shared__ double Osum[kNP][kTC];
  __shared__ double Shift[kTC];
  __shared__ int32_t s_j[kTC], s_src[kTC];
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int v = blockIdx.y;
  const int64_t nF = (*packed) >> 31;
  const int64_t ntile = (nF + kTC - 1) / kTC;
  if (int64_t(blockIdx.x) >= ntile) return;
  bf16x8 a[3][kMT][kKS];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int ks = 0; ks < kKS; ++ks) a[s][mt][ks] = fragP[(((c * 3 + s) * kMT + mt) * kKS + ks) * 64 + lane];
  const double* Wn = vec;
  const double* U = uo + int64_t(v) * kNP * ldo;
  double* O = un + int64_t(v) * kNP * ldn;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    if (threadIdx.x < kTC) {
      const int64_t r = tile * kTC + threadIdx.x;
      int32_t j = -1, sp = -1;
      if (r < nF) {
        j = F[r];
        sp = src[j];
      }
      s_j[threadIdx.x] = j;
      s_src[threadIdx.x] = sp;
    }
    __syncthreads();
    const int32_t sp = s_src[col];
    const bool live = sp >= 0;
    // Rows 8*grp + 32*ks + t of child c.  A padding column (sp < 0) reads
    // column c instead and discards it: a tile exists only when some parent
    // fuses, so the old mesh holds at least 2^d elements.  The per-row offsets
    // are wave-uniform, and one lane address per tile keeps the split
    // operator (96 registers) and the values in registers without scratch.
    const double* Ucol = U + int64_t(8 * grp) * ldo + (live ? sp : 0) + c;
    double mpart = 0.0;
    f32x4 acc[kMT];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kKS; ++ks) {
      bf16x8 b0, b1, b2;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = ks * 32 + 8 * grp + t;
        const double xr = Ucol[int64_t(ks * 32 + t) * ldo];
        const double x = live ? xr : 0.0;
        mpart += Wn[k] * x;
        __bf16 x0, x1, x2;
        split3(x, x0, x1, x2);
        b0[t] = x0;
        b1[t] = x1;
        b2[t] = x2;
      }
#pragma unroll
      for (int mt = 0; mt < kMT; ++mt)
        acc[mt] = mma6(a[0][mt][ks], a[1][mt][ks], a[2][mt][ks], b0, b1, b2, acc[mt]);
      __builtin_amdgcn_sched_barrier(0);
    }
    mpart += __shfl_xor(mpart, 16, 64);
    mpart += __shfl_xor(mpart, 32, 64);
    if (grp == 0) Mc[c][col] = mpart;
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) Part[c][mt * 16 + 4 * grp + r][col] = acc[mt][r];
    __syncthreads();
    for (int idx = threadIdx.x; idx < kNP * kTC; idx += blockDim.x) {
      const int row = idx / kTC, cc = idx % kTC;
      double sum = 0.0;
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) sum += double(Part[ch][row][cc]);
      Osum[row][cc] = sum;
    }
    __syncthreads();
    if (threadIdx.x < kTC) {
      double ms = 0.0, mf = 0.0;
      for (int row = 0; row < kNP; ++row) ms += Wn[row] * Osum[row][threadIdx.x];
      for (int ch = 0; ch < NC; ++ch) mf += Mc[ch][threadIdx.x];
      Shift[threadIdx.x] = mf / NC - ms;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kNP * kTC; idx += blockDim.x) {
      const int row = idx / kTC, cc = idx % kTC;
      const int32_t j = s_j[cc];
      if (j >= 0) O[int64_t(row) * ldn + j] = Osum[row][cc] + Shift[cc];
    }
    __syncthreads();
  }
}

}  // namespace

lt_status prepare_split(lt_tree_s* t, int p, hipStream_t s) {
  const int dim = t->g.dim;
  if (!((dim == 3 && p == 3) || (dim == 2 && p == 7)))
    return fail(LT_ERR_ARG, "split precision needs 64 points per element (3D p=3 or 2D p=7)");
  const int nc = 1 << dim, n1 = p + 1;
  LT_TRY_STATUS(build_transfer_ops(t->A, p, &t->ops[p], s));
  if (!t->split_frags) {
    const size_t nfr = size_t(2) * nc * 3 * kMT * kKS * 64;
    void* q = nullptr;
    if (dev_malloc(t->A, &q, nfr * sizeof(bf16x8)) != hipSuccess) return fail(LT_ERR_OOM, "split operators");
    void* qv = nullptr;
    if (dev_malloc(t->A, &qv, sizeof(double) * (kNP + nc * kNP)) != hipSuccess) {
      (void)dev_free(t->A, q);
      return fail(LT_ERR_OOM, "split operators");
    }
    k_build_split<<<unsigned((nfr / 3 + 255) / 256), 256, 0, s>>>(t->ops[p], n1, dim, nc,
                                                                  static_cast<bf16x8*>(q));
    k_build_split_vec<<<1, 256, 0, s>>>(t->ops[p], n1, dim, nc, static_cast<double*>(qv));
    if (hipGetLastError() != hipSuccess) {
      (void)dev_free(t->A, q);
      (void)dev_free(t->A, qv);
      return fail(LT_ERR_HIP, "split operator build failed to launch");
    }
    t->split_frags = q;
    t->split_vec = static_cast<double*>(qv);
  }
  return LT_OK;
}

lt_status launch_split_transfer(lt_tree_s* t, int p, int nvar, const double* u_old, int64_t ld_old,
                                double* u_new, int64_t ld_new, hipStream_t s) {
  return launch_split_transfer(t, Count{t->n_cur, nullptr}, p, nvar, u_old, ld_old, u_new, ld_new, s);
}

lt_status launch_split_transfer(lt_tree_s* t, Count cn, int p, int nvar, const double* u_old,
                                int64_t ld_old, double* u_new, int64_t ld_new, hipStream_t s) {
  const int dim = t->g.dim;
  if (nvar < 1 || int64_t(nvar) * kNP > 65535) return fail(LT_ERR_ARG, "nvar * 64 must be in [1, 65535]");
  LT_TRY_STATUS(prepare_split(t, p, s));
  const int nc = 1 << dim;
  const int64_t n = cn.n;  // leaves, or the capacity of a launch whose count lives on the device
  if (n == 0) return LT_OK;
  LT_TRY_STATUS(grow(t->A, &t->split_R, &t->split_R_cap, n));
  LT_TRY_STATUS(grow(t->A, &t->split_F, &t->split_F_cap, n));
  const bf16x8* fr = static_cast<const bf16x8*>(t->split_frags);
  const bf16x8* fI = fr;
  const bf16x8* fP = fr + size_t(nc) * 3 * kMT * kKS * 64;
  // The copy pass writes only copies and the refinement and fusion passes
  // only refined and fused elements: the latter run on the tree's second
  // stream beside the copy pass, forked after it is enqueued and joined back.
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  LT_TRY_STATUS(transfer_side(t, &side, &fork, &join));
  hipError_t ef = hipEventRecord(fork, s);
  if (ef != hipSuccess) return fail(LT_ERR_HIP, std::string("split transfer fork: ") + hipGetErrorString(ef));
  lt_status r = launch_copy(t, cn, int64_t(nvar) * kNP, u_old, ld_old, u_new, ld_new, s);
  ef = hipStreamWaitEvent(side, fork, 0);
  ScanState st;
  if (r == LT_OK && ef == hipSuccess) r = prep_scan(t, n, kTileMin, side, 0, &st);
  if (r == LT_OK && ef == hipSuccess) {
    st.items.p = cn.p;
    k_split_lists<<<grid_tiles(st), kScanSmall, 0, side>>>(t->map_kind, t->split_R, t->split_F, st);
    const int64_t max_ref_tiles = (n / nc + kTC - 1) / kTC + 1;
    const int64_t max_fuse_tiles = (n + kTC - 1) / kTC + 1;
    const dim3 gr(unsigned(std::min<int64_t>(max_ref_tiles, 2048)), unsigned(nvar));
    const dim3 gf(unsigned(std::min<int64_t>(max_fuse_tiles, 512)), unsigned(nvar));
    if (nc == 8) {
      k_split_refine<8><<<gr, 512, 0, side>>>(fI, t->split_vec, t->split_R, st.total, t->map_src, u_old,
                                              ld_old, u_new, ld_new);
      k_split_fuse<8><<<gf, 512, 0, side>>>(fP, t->split_vec, t->split_F, st.total, t->map_src, u_old,
                                            ld_old, u_new, ld_new);
    } else {
      k_split_refine<4><<<gr, 256, 0, side>>>(fI, t->split_vec, t->split_R, st.total, t->map_src, u_old,
                                              ld_old, u_new, ld_new);
      k_split_fuse<4><<<gf, 256, 0, side>>>(fP, t->split_vec, t->split_F, st.total, t->map_src, u_old,
                                            ld_old, u_new, ld_new);
    }
  }
  // the join on every path that forked, so that a capture in progress stays whole
  const hipError_t ej = hipEventRecord(join, side);
  const hipError_t ew = ej == hipSuccess ? hipStreamWaitEvent(s, join, 0) : ej;
  if (r != LT_OK) return r;
  if (ef != hipSuccess) return fail(LT_ERR_HIP, std::string("split transfer fork: ") + hipGetErrorString(ef));
  if (ew != hipSuccess) return fail(LT_ERR_HIP, std::string("split transfer join: ") + hipGetErrorString(ew));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("split transfer launch: ") + hipGetErrorString(e));
  return LT_OK;
}

}  // namespace lt
