// lt_mlp.hip -- learned refinement indicator (form 4 of the cycle).
//
// Per element, the FP64 nodal solution (64 Gauss-Legendre points x 5
// variables for p = 3 in 3D) is projected on the orthonormal tensor Legendre
// basis (sum-factorised; Gauss-Legendre quadrature is exact for the degree-2p
// products), each coefficient c becomes f = (log10(|c| + 1e-14) + 7) / 7, and
// an MLP 320 -> 128 -> 64 -> 3 (ReLU, BF16 weights and activations, FP32
// accumulation on the matrix cores) gives refine / keep / coarsen scores.
// Below a softmax confidence threshold the element keeps the geometric flag
// of Section 5.2.  Training runs on the device through the same GEMM kernel
// (forward, backward, Adam on FP32 master weights).
//
// Also here: the isentropic vortex of Section 5.2 evaluated at the solution
// points of a tree's leaves (z-extruded vortices superposed on the free
// stream rho = 1, u = 1, v = w = 0, p = 1; gamma = 1.4, phi = 1/2), used to
// make synthetic solution fields.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "tree.hpp"

namespace lt {
namespace {

constexpr double kGamma = 1.4;
constexpr double kPhi = 0.5;

struct FieldArgs {
  KeyGeom g;
  int nvort;
  double c[LT_MAX_VORTICES][2];
  double a[LT_MAX_VORTICES];
  double lo[3], dx;
  double nodes[LT_MAX_DEGREE + 1];
};

// One thread per (element, point): conserved variables of the vortex field.
template <int N1>
__global__ __launch_bounds__(256) void k_vortex_field(FieldArgs A, const uint64_t* __restrict__ keys,
                                                      int64_t n, double* __restrict__ u, int64_t ld) {
  constexpr int NP = N1 * N1 * N1;
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int npts = A.g.dim == 3 ? NP : N1 * N1;
  const int64_t e = id / npts;
  const int i = int(id % npts);
  if (e >= n) return;
  const uint64_t key = keys[e];
  const int d = key_depth(A.g, key);
  uint64_t x[3];
  demorton(A.g, key_morton(A.g, key), x);
  const double s = double(uint64_t(1) << (A.g.dmax - d));
  const int ix = i % N1, iy = (i / N1) % N1;
  const double X = A.lo[0] + A.dx * (double(x[0]) + s * A.nodes[ix]);
  const double Y = A.lo[1] + A.dx * (double(x[1]) + s * A.nodes[iy]);
  double du = 0.0, dv = 0.0, dT = 0.0;
  for (int v = 0; v < A.nvort; ++v) {
    const double ddx = X - A.c[v][0], ddy = Y - A.c[v][1];
    const double r2 = ddx * ddx + ddy * ddy;
    const double ex = exp(kPhi * (1.0 - r2));
    const double al = A.a[v];
    du += -al / (2.0 * M_PI) * ddy * ex;
    dv += al / (2.0 * M_PI) * ddx * ex;
    dT += -al * al * (kGamma - 1.0) / (16.0 * kPhi * kGamma * M_PI * M_PI) * ex * ex;
  }
  const double T = 1.0 + dT;
  const double rho = pow(T, 1.0 / (kGamma - 1.0));
  const double p = pow(rho, kGamma);
  const double uu = 1.0 + du, vv = dv;
  const double E = p / (kGamma - 1.0) + 0.5 * rho * (uu * uu + vv * vv);
  const double q[5] = {rho, rho * uu, rho * vv, 0.0, E};
  const int nvar = A.g.dim == 3 ? 5 : 4;
  for (int var = 0; var < nvar; ++var) {
    const int slot = A.g.dim == 3 ? var : (var < 3 ? var : 4);  // 2D: rho, rho u, rho v, E
    u[(int64_t(var) * npts + i) * ld + e] = q[slot];
  }
}

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Network input of one modal coefficient magnitude cc = |c| + 1e-14 (>= 1e-14,
// a normal FP32 number): (log10 cc + 7) / 7, formed as the hardware base-2
// logarithm times log10(2), then times 1/7.  Within a few FP32 ulps of the
// exactly rounded expression, far below the BF16 rounding that follows.
__device__ inline float feature_of(float cc) {
  return (__builtin_amdgcn_logf(cc) * 0.30102999566398120f + 7.0f) * (1.0f / 7.0f);
}
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Modal features of 64-point elements: T[n][i] = w_i L~_n(x_i) per axis
// (orthonormal Legendre at the Gauss-Legendre points), applied on the three
// axes; f = (log10(|c| + 1e-14) + 7) / 7 written as BF16 row [v*64 + mode]
// of X (one row of 64*nvar per element; `rows` picks elements, or null for
// all).  A block covers 64 elements of one variable with four lanes per
// element, one z-slab each: x and y passes in registers, the z pass through
// LDS.  Coefficients are FP64; the logarithm is taken in FP32, its result
// being stored in BF16.
__global__ __launch_bounds__(256) void k_mlp_features(const double* __restrict__ T4,
                                                      const double* __restrict__ u, int64_t ld,
                                                      int nvar, const int32_t* __restrict__ rows,
                                                      Count cn, bf16* __restrict__ X) {
  constexpr int kS = 65;  // LDS stride (doubles) of one element's 64 values
  const int64_t n = cn.get();
  __shared__ double sA[64 * kS];
  const int el = threadIdx.x & 63, z = threadIdx.x >> 6;
  const int v = blockIdx.y;
  const int64_t r = int64_t(blockIdx.x) * 64 + el;
  const bool live = r < n;
  const int64_t e = live ? (rows ? int64_t(rows[r]) : r) : 0;
  double T[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) T[i] = T4[i];
  double a[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = live ? u[(int64_t(v) * 64 + z * 16 + i) * ld + e] : 0.0;
  // x pass (stride 1) then y pass (stride 4) on the 4 x 4 slab
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int st = pass == 0 ? 1 : 4;
#pragma unroll
    for (int line = 0; line < 4; ++line) {
      const int base = pass == 0 ? line * 4 : line;
      const double x0 = a[base], x1 = a[base + st], x2 = a[base + 2 * st], x3 = a[base + 3 * st];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        a[base + m * st] = T[m * 4] * x0 + T[m * 4 + 1] * x1 + T[m * 4 + 2] * x2 + T[m * 4 + 3] * x3;
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) sA[el * kS + z * 16 + i] = a[i];
  __syncthreads();
  // z pass: this lane now produces output slab m = z of its element
  const int m = z;
  double c[16];
#pragma unroll
  for (int yx = 0; yx < 16; ++yx) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc += T[m * 4 + i] * sA[el * kS + i * 16 + yx];
    c[yx] = acc;
  }
  if (!live) return;
  typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
  bf16x8v* out = reinterpret_cast<bf16x8v*>(X + r * int64_t(64 * nvar) + v * 64 + m * 16);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    bf16x8v o;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float cc = float(fabs(c[h * 8 + t]) + 1e-14);
      o[t] = bf16(feature_of(cc));
    }
    out[h] = o;
  }
}

// C[m][n] = sum_k A[m][k] Bt[n][k] (+ bias[n]) on BF16 matrix cores with FP32
// accumulation; both operands are K-contiguous.  Optional: ReLU, an FP32
// output, a BF16 output.  One wave per 16 x 16 tile; rows/columns/depth past
// M, N, K read as zero.
__global__ __launch_bounds__(256) void k_gemm_nt(const bf16* __restrict__ A, int64_t lda,
                                                 const bf16* __restrict__ Bt, int64_t ldb, int M, int N,
                                                 int K, const float* __restrict__ bias, int relu,
                                                 float* __restrict__ C, int64_t ldc,
                                                 bf16* __restrict__ Cb, int64_t ldcb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tiles_n = (N + 15) / 16;
  const int64_t tile = int64_t(blockIdx.x) * 4 + w;
  const int64_t tiles = int64_t((M + 15) / 16) * tiles_n;
  if (tile >= tiles) return;
  const int m0 = int(tile / tiles_n) * 16, n0 = int(tile % tiles_n) * 16;
  const int r = lane & 15, kq = 8 * (lane >> 4);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const int am = m0 + r, bn = n0 + r;
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + kq + t;
      a[t] = (am < M && k < K) ? A[int64_t(am) * lda + k] : bf16(0.f);
      b[t] = (bn < N && k < K) ? Bt[int64_t(bn) * ldb + k] : bf16(0.f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  const int cn = n0 + (lane & 15);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cm = m0 + 4 * (lane >> 4) + q;
    if (cm >= M || cn >= N) continue;
    float val = acc[q] + (bias ? bias[cn] : 0.f);
    if (relu) val = val > 0.f ? val : 0.f;
    if (C) C[int64_t(cm) * ldc + cn] = val;
    if (Cb) Cb[int64_t(cm) * ldcb + cn] = bf16(val);
  }
}

// Out[c][r] = In[r][c] (BF16 from FP32 or BF16 sources), R x Cols.
template <class TIn>
__global__ void k_transpose(const TIn* __restrict__ in, int64_t ldi, int R, int Cols,
                            bf16* __restrict__ out, int64_t ldo) {
  __shared__ float tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int j = ty; j < 32; j += 8) {
    const int rr = r0 + j, cc = c0 + tx;
    tile[j][tx] = (rr < R && cc < Cols) ? float(in[int64_t(rr) * ldi + cc]) : 0.f;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int cc = c0 + j, rr = r0 + tx;
    if (cc < Cols && rr < R) out[int64_t(cc) * ldo + rr] = bf16(tile[tx][j]);
  }
}

// Softmax cross-entropy over 3 classes: dZ = (softmax(Z) - onehot(y)) / B and
// the per-row loss.
__global__ void k_xent(const float* __restrict__ Z, const int8_t* __restrict__ y, int B,
                       float* __restrict__ dZ, float* __restrict__ loss) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float z0 = Z[3 * b], z1 = Z[3 * b + 1], z2 = Z[3 * b + 2];
  const float m = fmaxf(z0, fmaxf(z1, z2));
  const float e0 = expf(z0 - m), e1 = expf(z1 - m), e2 = expf(z2 - m);
  const float s = e0 + e1 + e2;
  const int c = min(max(int(y[b]), 0), 2);  // labels outside {0,1,2} clamp
  const float p[3] = {e0 / s, e1 / s, e2 / s};
  for (int k = 0; k < 3; ++k) dZ[3 * b + k] = (p[k] - (k == c ? 1.f : 0.f)) / float(B);
  loss[b] = -logf(p[c]);
}

// G[r][c] *= (H[r][c] > 0)  (ReLU derivative through the stored activation).
__global__ void k_relu_mask(float* __restrict__ G, const bf16* __restrict__ H, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && !(float(H[i]) > 0.f)) G[i] = 0.f;
}

// Column sums of an R x Cols FP32 array (bias gradients).
__global__ void k_colsum(const float* __restrict__ G, int R, int Cols, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Cols) return;
  float s = 0.f;
  for (int r = 0; r < R; ++r) s += G[int64_t(r) * Cols + c];
  out[c] = s;
}

// Adam on FP32 master parameters; refreshes the BF16 copy.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, bf16* __restrict__ wb, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  const float wi = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = bf16(wi);
}

// Modal-energy indicator: the density's nodal values become coefficients in
// the orthonormal tensor Legendre basis (matrix T per axis, sum-factorised);
// s = energy of the modes whose highest per-axis degree is p over the total
// energy; +1 if log10 s > tau_r, -1 if log10 s < tau_c, else 0 (all-zero
// density: 0); then the depth clamps.
struct ModalT {
  double T[16];  // T[n * N1 + i]
};

template <int N1, int DIM>
__global__ __launch_bounds__(256) void k_flag_modal(KeyGeom g, const uint64_t* __restrict__ keys,
                                                    int64_t n, ModalT M, const double* __restrict__ u,
                                                    int64_t ld, double tau_r, double tau_c,
                                                    int8_t* __restrict__ flags) {
  constexpr int NP = DIM == 3 ? N1 * N1 * N1 : N1 * N1;
  constexpr int NZ = DIM == 3 ? N1 : 1;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double a[NP], b[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) a[i] = u[int64_t(i) * ld + e];
  // x: b[zy][m] = sum_i T[m][i] a[zy][i]
#pragma unroll
  for (int zy = 0; zy < NP / N1; ++zy)
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < N1; ++i) acc += M.T[m * N1 + i] * a[zy * N1 + i];
      b[zy * N1 + m] = acc;
    }
  // y: a[z][m][x] = sum_i T[m][i] b[z][i][x]
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int m = 0; m < N1; ++m)
#pragma unroll
      for (int x = 0; x < N1; ++x) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) acc += M.T[m * N1 + i] * b[(z * N1 + i) * N1 + x];
        a[(z * N1 + m) * N1 + x] = acc;
      }
  if (DIM == 3) {
    // z: b[m][yx] = sum_i T[m][i] a[i][yx]
#pragma unroll
    for (int m = 0; m < N1; ++m)
#pragma unroll
      for (int yx = 0; yx < N1 * N1; ++yx) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) acc += M.T[m * N1 + i] * a[i * N1 * N1 + yx];
        b[m * N1 * N1 + yx] = acc;
      }
  } else {
#pragma unroll
    for (int k = 0; k < NP; ++k) b[k] = a[k];
  }
  double tot = 0.0, top = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int kx = k % N1, ky = (k / N1) % N1, kz = DIM == 3 ? k / (N1 * N1) : 0;
    const double c2 = b[k] * b[k];
    tot += c2;
    if (kx == N1 - 1 || ky == N1 - 1 || kz == N1 - 1) top += c2;
  }
  int f = 0;
  if (tot > 0.0) {
    const double ls = log10(top / tot);  // -inf when the top modes vanish
    f = ls > tau_r ? 1 : (ls < tau_c ? -1 : 0);
  }
  const uint64_t key = keys[e];
  const int d = key_depth(g, key);
  int lo, hi;
  depth_limits(g, key, &lo, &hi);
  if (f == 1 && d >= hi) f = 0;
  if (f == -1 && d <= lo) f = 0;
  flags[e] = int8_t(f);
}

// Learned flags over a mesh: workgroups of 8 waves hold W1 and W2 in LDS;
// each wave runs its own 16-element tiles, with its activations in a
// per-wave LDS patch (BF16), W3 in registers, and the logits going straight
// to the decision: argmax class (0 coarsen, 1 keep, 2 refine) when its
// softmax probability reaches conf_min, else the geometric flag already in
// `flags`; then the depth clamps.
constexpr int kW1S = 328;  // LDS row stride (BF16) of W1 (320 + pad)
constexpr int kW2S = 136;  // W2 (128 + pad)
constexpr int kH1S = 136;  // layer-1 activations of a wave's 16 rows (128 + pad)
constexpr int kH2S = 72;   // layer-2 activations (64 + pad)
constexpr int kFlagWaves = 8;

// Features and network in one pass (learned flags over a whole mesh).  The
// same workgroup shape as k_mlp_flag, but each wave builds its 16 rows of
// features itself: lane group g (lanes 16g .. 16g+15, one element each)
// loads z-slab g of the element's 64 values of one variable, transforms it
// along x and y in registers, and the z pass combines the four slabs over
// three rotation rounds of cross-lane exchange (round r: lane group g sends
// its row my = (g + r) mod 4 and receives slab (g - r) mod 4 of row my = g),
// so lane group g ends with the coefficients of row my = g.  The 64 BF16
// features of a variable are staged in the wave's LDS patch and read back as
// matrix-core A fragments.  No feature array is written to memory.
// Orders one wave's LDS writes before its later LDS reads by other lanes of
// the same wave (the patches below are private to a wave; the wave's LDS
// operations execute in program order, the fences keep the compiler's order).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row `row` (per lane) of a 4 x 4 register block, as a masked sum: exact for
// finite values, and branch-free (nested selects on a per-lane index were
// compiled to exec-masked branches).
__device__ inline double pick4(const double* a, int row, int x) {
  return double(row == 0) * a[x] + double(row == 1) * a[4 + x] + double(row == 2) * a[8 + x] +
         double(row == 3) * a[12 + x];
}

__global__ __launch_bounds__(64 * kFlagWaves) void k_mlp_flag_fused(
    KeyGeom g, const uint64_t* __restrict__ keys, const double* __restrict__ u, int64_t ld, Count cn,
    const double* __restrict__ T4, const bf16* __restrict__ W1, const bf16* __restrict__ W2,
    const bf16* __restrict__ W3, const float* __restrict__ P, int64_t off_b1, int64_t off_b2,
    int64_t off_b3, float conf_min, int8_t* __restrict__ flags, float* __restrict__ conf) {
  constexpr int kFS = 72;  // staging row stride (BF16) of one element's 64 features
  __shared__ __attribute__((aligned(16))) bf16 sW1[128 * kW1S];
  __shared__ __attribute__((aligned(16))) bf16 sW2[64 * kW2S];
  __shared__ __attribute__((aligned(16))) bf16 sH1[kFlagWaves][16 * kH1S];
  __shared__ __attribute__((aligned(16))) bf16 sH2[kFlagWaves][16 * kH2S];
  __shared__ float sZ[kFlagWaves][16][4];
  __shared__ float sB[128 + 64 + 4];
  const int64_t n = cn.get();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4, lk = 8 * lg;
  for (int c = tid; c < 128 * 40; c += 64 * kFlagWaves) {
    const int row = c / 40, c16 = c % 40;
    *reinterpret_cast<bf16x8*>(sW1 + row * kW1S + c16 * 8) =
        *reinterpret_cast<const bf16x8*>(W1 + row * 320 + c16 * 8);
  }
  for (int c = tid; c < 64 * 16; c += 64 * kFlagWaves) {
    const int row = c / 16, c16 = c % 16;
    *reinterpret_cast<bf16x8*>(sW2 + row * kW2S + c16 * 8) =
        *reinterpret_cast<const bf16x8*>(W2 + row * 128 + c16 * 8);
  }
  for (int c = tid; c < 128 + 64 + 3; c += 64 * kFlagWaves)
    sB[c] = c < 128 ? P[off_b1 + c] : (c < 192 ? P[off_b2 + c - 128] : P[off_b3 + c - 192]);
  bf16x8 b3f[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    if (lr < 3) {
      b3f[ks] = *reinterpret_cast<const bf16x8*>(W3 + lr * 64 + 32 * ks + lk);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) b3f[ks][t] = bf16(0.f);
    }
  }
  double T[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) T[i] = T4[i];
  __syncthreads();
  bf16* H1 = sH1[w];
  bf16* H2 = sH2[w];
  bf16* FS = sH1[w];  // feature staging shares the layer-1 patch (used one after the other)
  const int64_t ntiles = (n + 15) / 16;
  const int64_t stride = int64_t(gridDim.x) * kFlagWaves;
  // z-slab lg of this lane's element of tile tl, variable v: unconditional
  // loads at a clamped index, so that no branch or select stands between a
  // load and its use.  A lane past the end reads element 0: its row of the
  // network is finite and never written out.
  auto load_slab = [&](int64_t tl, int v, double* dst) {
    const int64_t el = tl * 16 + lr;
    const int64_t ec = (tl < ntiles && el < n) ? el : 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[i] = u[(int64_t(v) * 64 + lg * 16 + i) * ld + ec];
  };
  // The slab of the next variable (or of the next tile's first variable) is
  // loaded while the current one is computed, into the other of two register
  // buffers (the variable loop is unrolled, so the buffers swap roles without
  // copies): with two waves per SIMD (the weights fill the LDS) the loads of
  // one variable would otherwise wait alone.
  int64_t tile = int64_t(blockIdx.x) * kFlagWaves + w;
  double bufA[16], bufB[16];
  if (tile < ntiles) load_slab(tile, 0, bufA);
  // Waves run their tiles independently (every LDS patch in the loop is a
  // wave's own); a wave whose tile lies past the end computes on zeros and
  // writes nothing.
  for (; tile < ntiles; tile += stride) {
    // this tile's keys and fallback flags, read ahead of the prefetches
    const int64_t eo = tile * 16 + lane;
    const bool own = lane < 16 && eo < n;
    const int64_t eoc = own ? eo : 0;
    const uint64_t okey = keys[eoc];
    const int ofl = int(flags[eoc]);
    // layer 1 accumulates variable by variable: acc[ct] += X[:, 64v .. 64v+63] W1^T
    f32x4 acc1[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) acc1[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      // keep each variable's work in its own region, so that the waits for
      // the prefetched slab fall in the next variable, not this one
      __builtin_amdgcn_sched_barrier(0);
      double* a = (v & 1) ? bufB : bufA;
      load_slab(v < 4 ? tile : tile + stride, v < 4 ? v + 1 : 0, (v & 1) ? bufA : bufB);
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        const int st = pass == 0 ? 1 : 4;
#pragma unroll
        for (int line = 0; line < 4; ++line) {
          const int b0 = pass == 0 ? line * 4 : line;
          const double x0 = a[b0], x1 = a[b0 + st], x2 = a[b0 + 2 * st], x3 = a[b0 + 3 * st];
#pragma unroll
          for (int m = 0; m < 4; ++m)
            a[b0 + m * st] = T[m * 4] * x0 + T[m * 4 + 1] * x1 + T[m * 4 + 2] * x2 + T[m * 4 + 3] * x3;
        }
      }
      // a[my*4 + mx] = slab lg's partial coefficients; z pass over the 4 slabs
      double c[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) c[i] = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int z = (lg - r) & 3;         // slab received this round
        const int row = (lg + r) & 3;       // row sent this round
        const int srcl = z * 16 + lr;
        double val[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const double sendv = pick4(a, row, x);
          val[x] = r == 0 ? sendv : __shfl(sendv, srcl);
        }
#pragma unroll
        for (int mz = 0; mz < 4; ++mz) {
          const double tz = double(z == 0) * T[mz * 4] + double(z == 1) * T[mz * 4 + 1] +
                            double(z == 2) * T[mz * 4 + 2] + double(z == 3) * T[mz * 4 + 3];
#pragma unroll
          for (int x = 0; x < 4; ++x) c[mz * 4 + x] += tz * val[x];
        }
      }
      wave_lds_sync();  // the previous variable's fragments have been read
#pragma unroll
      for (int mz = 0; mz < 4; ++mz)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const float cc = float(fabs(c[mz * 4 + x]) + 1e-14);
          FS[lr * kFS + mz * 16 + lg * 4 + x] = bf16(feature_of(cc));
        }
      wave_lds_sync();
      bf16x8 af[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) af[h] = *reinterpret_cast<const bf16x8*>(FS + lr * kFS + 32 * h + lk);
#pragma unroll
      for (int ct = 0; ct < 8; ++ct)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bf16x8 bf =
              *reinterpret_cast<const bf16x8*>(sW1 + (16 * ct + lr) * kW1S + 64 * v + 32 * h + lk);
          acc1[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[h], bf, acc1[ct], 0, 0, 0);
        }
    }
    wave_lds_sync();  // staging reads done before layer 1 writes the patch
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
      const float bias = sB[16 * ct + lr];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float hv = acc1[ct][q] + bias;
        H1[(4 * lg + q) * kH1S + 16 * ct + lr] = bf16(hv > 0.f ? hv : 0.f);
      }
    }
    wave_lds_sync();
    bf16x8 h1f[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) h1f[ks] = *reinterpret_cast<const bf16x8*>(H1 + lr * kH1S + 32 * ks + lk);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bf16x8 bf = *reinterpret_cast<const bf16x8*>(sW2 + (16 * ct + lr) * kW2S + 32 * ks + lk);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1f[ks], bf, acc, 0, 0, 0);
      }
      const float bias = sB[128 + 16 * ct + lr];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float hv = acc[q] + bias;
        H2[(4 * lg + q) * kH2S + 16 * ct + lr] = bf16(hv > 0.f ? hv : 0.f);
      }
    }
    wave_lds_sync();
    f32x4 acc3 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(H2 + lr * kH2S + 32 * ks + lk);
      acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b3f[ks], acc3, 0, 0, 0);
    }
    if (lr < 3)
#pragma unroll
      for (int q = 0; q < 4; ++q) sZ[w][4 * lg + q][lr] = acc3[q] + sB[192 + lr];
    wave_lds_sync();
    if (own) {
      const float z0 = sZ[w][lane][0], z1 = sZ[w][lane][1], z2 = sZ[w][lane][2];
      const float mx = fmaxf(z0, fmaxf(z1, z2));
      const float e0 = expf(z0 - mx), e1 = expf(z1 - mx), e2 = expf(z2 - mx);
      const float sum = e0 + e1 + e2;
      int cls = 0;
      float pc = e0;
      if (e1 > pc) { cls = 1; pc = e1; }
      if (e2 > pc) { cls = 2; pc = e2; }
      pc /= sum;
      if (conf) conf[eo] = pc;
      int f = pc >= conf_min ? cls - 1 : ofl;
      const int d = key_depth(g, okey);
      int lo, hi;
      depth_limits(g, okey, &lo, &hi);
      if (f == 1 && d >= hi) f = 0;
      if (f == -1 && d <= lo) f = 0;
      flags[eo] = int8_t(f);
    }
    wave_lds_sync();  // sZ and the patches are rewritten by the next tile
#pragma unroll
    for (int i = 0; i < 16; ++i) bufA[i] = bufB[i];  // the next tile's first slab
  }
}

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// T[n][i] = w_i sqrt((2n+1)/2) P_n(x_i) at the p+1 Gauss-Legendre points
// (closed forms, p <= 3): the orthonormal-Legendre projection per axis.
bool modal_matrix(int p, double* T) {
  double x[4], w[4];
  if (p == 1) {
    const double r = 1.0 / std::sqrt(3.0);
    x[0] = -r; x[1] = r; w[0] = w[1] = 1.0;
  } else if (p == 2) {
    const double r = std::sqrt(3.0 / 5.0);
    x[0] = -r; x[1] = 0.0; x[2] = r;
    w[0] = w[2] = 5.0 / 9.0; w[1] = 8.0 / 9.0;
  } else if (p == 3) {
    const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
    w[0] = w[3] = (18.0 - std::sqrt(30.0)) / 36.0;
    w[1] = w[2] = (18.0 + std::sqrt(30.0)) / 36.0;
  } else {
    return false;
  }
  const int n1 = p + 1;
  for (int i = 0; i < n1; ++i) {
    double P[4];
    P[0] = 1.0;
    P[1] = x[i];
    for (int k = 2; k < n1; ++k) P[k] = ((2.0 * k - 1.0) * x[i] * P[k - 1] - (k - 1.0) * P[k - 2]) / k;
    for (int m = 0; m < n1; ++m) T[m * n1 + i] = w[i] * std::sqrt((2.0 * m + 1.0) / 2.0) * P[m];
  }
  return true;
}

}  // namespace
}  // namespace lt

// ------------------------------------------------------------------- MLP state
struct lt_mlp_s {
  static constexpr int kIn = 320, kH1 = 128, kH2 = 64, kOut = 3;
  int device = 0;
  lt::Alloc A;  // device allocator of every buffer below
  // FP32 master parameters, BF16 copies (row-major [out][in]) and transposes
  float* P = nullptr;   // W1 b1 W2 b2 W3 b3 (FP32, contiguous)
  float* G = nullptr;   // gradients, same layout
  float* M1 = nullptr;  // Adam moments
  float* M2 = nullptr;
  __bf16* W1 = nullptr; __bf16* W2 = nullptr; __bf16* W3 = nullptr;      // [out][in]
  __bf16* W1T = nullptr; __bf16* W2T = nullptr; __bf16* W3T = nullptr;   // [in][out]
  double* T4 = nullptr;  // 4x4 modal matrix (p = 3)
  int64_t step = 0;
  // scratch sized for `cap` rows
  int64_t cap = 0;
  __bf16 *H1 = nullptr, *H2 = nullptr, *XT = nullptr, *H1T = nullptr, *H2T = nullptr;
  __bf16 *D1T = nullptr, *D2T = nullptr, *D3T = nullptr, *D2b = nullptr, *D3b = nullptr;
  float *Z3 = nullptr, *D1 = nullptr, *D2 = nullptr, *D3 = nullptr, *loss = nullptr;
  __bf16* X = nullptr;  // features for lt_flag_mlp
  int64_t xcap = 0;

  static constexpr int64_t off_W1 = 0, off_b1 = off_W1 + int64_t(kH1) * kIn;
  static constexpr int64_t off_W2 = off_b1 + kH1, off_b2 = off_W2 + int64_t(kH2) * kH1;
  static constexpr int64_t off_W3 = off_b2 + kH2, off_b3 = off_W3 + int64_t(kOut) * kH2;
  static constexpr int64_t nparam = off_b3 + kOut;
};

namespace lt {
namespace {

lt_status mlp_scratch(lt_mlp_s* m, int64_t B) {
  if (B <= m->cap) return LT_OK;
  auto fr = [m](void* p) { (void)dev_free(m->A, p); };
  fr(m->H1); fr(m->H2); fr(m->XT); fr(m->H1T); fr(m->H2T); fr(m->D1T); fr(m->D2T); fr(m->D3T);
  fr(m->D2b); fr(m->D3b); fr(m->Z3); fr(m->D1); fr(m->D2); fr(m->D3); fr(m->loss);
  const int64_t c = B + B / 4 + 64;
  hipError_t e = hipSuccess;
  auto al = [&](void** p, size_t bytes) { if (e == hipSuccess) e = dev_malloc(m->A, p, bytes); };
  al((void**)&m->H1, c * 128 * 2); al((void**)&m->H2, c * 64 * 2); al((void**)&m->XT, c * 320 * 2);
  al((void**)&m->H1T, c * 128 * 2); al((void**)&m->H2T, c * 64 * 2); al((void**)&m->D1T, c * 128 * 2);
  al((void**)&m->D2T, c * 64 * 2); al((void**)&m->D3T, c * 3 * 2); al((void**)&m->D2b, c * 64 * 2);
  al((void**)&m->D3b, c * 3 * 2); al((void**)&m->Z3, c * 3 * 4); al((void**)&m->D1, c * 128 * 4);
  al((void**)&m->D2, c * 64 * 4); al((void**)&m->D3, c * 3 * 4); al((void**)&m->loss, c * 4);
  if (e != hipSuccess) {
    m->cap = 0;
    return fail(LT_ERR_OOM, "MLP scratch allocation failed");
  }
  m->cap = c;
  return LT_OK;
}

hipError_t gemm(const __bf16* A, int64_t lda, const __bf16* Bt, int64_t ldb, int M, int N, int K,
                const float* bias, int relu, float* C, int64_t ldc, __bf16* Cb, int64_t ldcb,
                hipStream_t s) {
  const int64_t tiles = int64_t((M + 15) / 16) * ((N + 15) / 16);
  k_gemm_nt<<<nblk(tiles, 4), 256, 0, s>>>(A, lda, Bt, ldb, M, N, K, bias, relu, C, ldc, Cb, ldcb);
  return hipGetLastError();
}

template <class TIn>
hipError_t transpose(const TIn* in, int64_t ldi, int R, int Cols, __bf16* out, int64_t ldo,
                     hipStream_t s) {
  dim3 grid(nblk(Cols, 32), nblk(R, 32));
  k_transpose<TIn><<<grid, 256, 0, s>>>(in, ldi, R, Cols, out, ldo);
  return hipGetLastError();
}

// BF16 copies and transposes of the weights from the FP32 masters.
lt_status mlp_refresh(lt_mlp_s* m, hipStream_t s) {
  const float* P = m->P;
  hipError_t e = transpose(P + lt_mlp_s::off_W1, 320, 128, 320, m->W1T, 128, s);
  if (e == hipSuccess) e = transpose(P + lt_mlp_s::off_W2, 128, 64, 128, m->W2T, 64, s);
  if (e == hipSuccess) e = transpose(P + lt_mlp_s::off_W3, 64, 3, 64, m->W3T, 3, s);
  if (e == hipSuccess) e = transpose(m->W1T, 128, 320, 128, m->W1, 320, s);
  if (e == hipSuccess) e = transpose(m->W2T, 64, 128, 64, m->W2, 128, s);
  if (e == hipSuccess) e = transpose(m->W3T, 3, 64, 3, m->W3, 64, s);
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("MLP refresh: ") + hipGetErrorString(e));
  return LT_OK;
}

// Forward pass on B rows of X (BF16 [B][320]); logits in Z3 (FP32 [B][3]).
lt_status mlp_forward(lt_mlp_s* m, const __bf16* X, int64_t B, float* Z3, hipStream_t s) {
  const float* P = m->P;
  hipError_t e = gemm(X, 320, m->W1, 320, int(B), 128, 320, P + lt_mlp_s::off_b1, 1, nullptr, 0, m->H1, 128, s);
  if (e == hipSuccess)
    e = gemm(m->H1, 128, m->W2, 128, int(B), 64, 128, P + lt_mlp_s::off_b2, 1, nullptr, 0, m->H2, 64, s);
  if (e == hipSuccess)
    e = gemm(m->H2, 64, m->W3, 64, int(B), 3, 64, P + lt_mlp_s::off_b3, 0, Z3, 3, nullptr, 0, s);
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("MLP forward: ") + hipGetErrorString(e));
  return LT_OK;
}

// Forward + backward on one mini-batch; gradients (FP32) in m->G.
lt_status mlp_backward(lt_mlp_s* m, const __bf16* X, const int8_t* y, int64_t B, hipStream_t s) {
  LT_TRY_STATUS(mlp_scratch(m, B));
  LT_TRY_STATUS(mlp_forward(m, X, B, m->Z3, s));
  float* G = m->G;
  const int b = int(B);
  k_xent<<<nblk(B, 256), 256, 0, s>>>(m->Z3, y, b, m->D3, m->loss);
  hipError_t e = hipGetLastError();
  // layer 3: gW3 = D3^T H2, gb3 = colsum D3, D2 = (D3 W3) * [H2 > 0]
  if (e == hipSuccess) e = transpose(m->D3, 3, b, 3, m->D3T, b, s);
  if (e == hipSuccess) e = transpose(m->H2, 64, b, 64, m->H2T, b, s);
  if (e == hipSuccess) e = gemm(m->D3T, b, m->H2T, b, 3, 64, b, nullptr, 0, G + lt_mlp_s::off_W3, 64, nullptr, 0, s);
  if (e == hipSuccess) { k_colsum<<<1, 64, 0, s>>>(m->D3, b, 3, G + lt_mlp_s::off_b3); e = hipGetLastError(); }
  if (e == hipSuccess) e = transpose(m->D3T, b, 3, b, m->D3b, 3, s);
  if (e == hipSuccess) e = gemm(m->D3b, 3, m->W3T, 3, b, 64, 3, nullptr, 0, m->D2, 64, nullptr, 0, s);
  if (e == hipSuccess) { k_relu_mask<<<nblk(B * 64, 256), 256, 0, s>>>(m->D2, m->H2, B * 64); e = hipGetLastError(); }
  // layer 2: gW2 = D2^T H1, gb2, D1 = (D2 W2) * [H1 > 0]
  if (e == hipSuccess) e = transpose(m->D2, 64, b, 64, m->D2T, b, s);
  if (e == hipSuccess) e = transpose(m->H1, 128, b, 128, m->H1T, b, s);
  if (e == hipSuccess) e = gemm(m->D2T, b, m->H1T, b, 64, 128, b, nullptr, 0, G + lt_mlp_s::off_W2, 128, nullptr, 0, s);
  if (e == hipSuccess) { k_colsum<<<1, 64, 0, s>>>(m->D2, b, 64, G + lt_mlp_s::off_b2); e = hipGetLastError(); }
  if (e == hipSuccess) e = transpose(m->D2T, b, 64, b, m->D2b, 64, s);
  if (e == hipSuccess) e = gemm(m->D2b, 64, m->W2T, 64, b, 128, 64, nullptr, 0, m->D1, 128, nullptr, 0, s);
  if (e == hipSuccess) { k_relu_mask<<<nblk(B * 128, 256), 256, 0, s>>>(m->D1, m->H1, B * 128); e = hipGetLastError(); }
  // layer 1: gW1 = D1^T X, gb1
  if (e == hipSuccess) e = transpose(m->D1, 128, b, 128, m->D1T, b, s);
  if (e == hipSuccess) e = transpose(X, 320, b, 320, m->XT, b, s);
  if (e == hipSuccess) e = gemm(m->D1T, b, m->XT, b, 128, 320, b, nullptr, 0, G + lt_mlp_s::off_W1, 320, nullptr, 0, s);
  if (e == hipSuccess) { k_colsum<<<2, 64, 0, s>>>(m->D1, b, 128, G + lt_mlp_s::off_b1); e = hipGetLastError(); }
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("MLP backward: ") + hipGetErrorString(e));
  return LT_OK;
}

}  // namespace
}  // namespace lt

namespace lt {

lt_status mlp_reserve(lt_mlp m, int64_t n) {
  if (m->xcap >= n) return LT_OK;
  (void)dev_free(m->A, m->X);
  m->X = nullptr;
  m->xcap = 0;
  if (dev_malloc(m->A, reinterpret_cast<void**>(&m->X), size_t(n) * 320 * 2) != hipSuccess)
    return fail(LT_ERR_OOM, "MLP features");
  m->xcap = n;
  return LT_OK;
}

lt_status launch_mlp_flag(lt_tree_s* t, lt_mlp m, Count n, const double* u, int64_t ld, float conf_min,
                          int8_t* flags, float* conf, hipStream_t s) {
  if (t->g.dim != 3) return fail(LT_ERR_ARG, "the learned indicator takes 3D p = 3 elements");
  if (n.n == 0) return LT_OK;
  const int64_t ntiles = (n.n + 16 * kFlagWaves - 1) / (16 * kFlagWaves);
  const unsigned grid = unsigned(std::min<int64_t>(ntiles, 256));
  k_mlp_flag_fused<<<grid, 64 * kFlagWaves, 0, s>>>(t->g, t->kbuf[t->cur], u, ld, n, m->T4, m->W1, m->W2,
                                                    m->W3, m->P, lt_mlp_s::off_b1, lt_mlp_s::off_b2,
                                                    lt_mlp_s::off_b3, conf_min, flags, conf);
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "learned flag launch");
  return LT_OK;
}

}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_mlp_create(const float* params, lt_mlp* out) {
  if (!params || !out) return fail(LT_ERR_ARG, "NULL argument");
  lt_mlp m = new lt_mlp_s;
  m->A = registered_alloc();
  hipError_t e = hipGetDevice(&m->device);
  const size_t np = size_t(lt_mlp_s::nparam);
  auto al = [&](void** p, size_t bytes) { if (e == hipSuccess) e = dev_malloc(m->A, p, bytes); };
  al((void**)&m->P, np * 4); al((void**)&m->G, np * 4); al((void**)&m->M1, np * 4); al((void**)&m->M2, np * 4);
  al((void**)&m->W1, 128 * 320 * 2); al((void**)&m->W2, 64 * 128 * 2); al((void**)&m->W3, 3 * 64 * 2);
  al((void**)&m->W1T, 128 * 320 * 2); al((void**)&m->W2T, 64 * 128 * 2); al((void**)&m->W3T, 3 * 64 * 2);
  al((void**)&m->T4, 16 * 8);
  if (e == hipSuccess) e = hipMemcpy(m->P, params, np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->M1, 0, np * 4);
  if (e == hipSuccess) e = hipMemset(m->M2, 0, np * 4);
  if (e == hipSuccess) {
    double T[16];
    modal_matrix(3, T);
    e = hipMemcpy(m->T4, T, sizeof(T), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    lt_mlp_destroy(m);
    return fail(e == hipErrorOutOfMemory ? LT_ERR_OOM : LT_ERR_HIP,
                std::string("MLP create: ") + hipGetErrorString(e));
  }
  lt_status st = mlp_refresh(m, nullptr);
  if (st == LT_OK && hipDeviceSynchronize() != hipSuccess) st = fail(LT_ERR_HIP, "MLP create sync");
  if (st != LT_OK) {
    lt_mlp_destroy(m);
    return st;
  }
  *out = m;
  return LT_OK;
}

lt_status lt_mlp_params(lt_mlp m, float* params, float* grads, void* stream) {
  if (!m) return fail(LT_ERR_ARG, "NULL model");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = size_t(lt_mlp_s::nparam) * 4;
  if (params) LT_TRY_STATUS(hipMemcpyAsync(params, m->P, bytes, hipMemcpyDeviceToHost, s) == hipSuccess ? LT_OK : fail(LT_ERR_HIP, "copy"));
  if (grads) LT_TRY_STATUS(hipMemcpyAsync(grads, m->G, bytes, hipMemcpyDeviceToHost, s) == hipSuccess ? LT_OK : fail(LT_ERR_HIP, "copy"));
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LT_ERR_HIP, "sync");
  return LT_OK;
}

lt_status lt_mlp_features(lt_mlp m, const double* u, int64_t ld, int nvar, const int32_t* rows,
                          int64_t n, void* X, void* stream) {
  if (!m || !u || !X || nvar != 5) return fail(LT_ERR_ARG, "features need 5 variables of 64 points");
  if (n == 0) return LT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_mlp_features<<<dim3(nblk(n, 64), unsigned(nvar)), 256, 0, s>>>(m->T4, u, ld, nvar, rows,
                                                                    Count{n, nullptr},
                                                                    static_cast<__bf16*>(X));
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "features launch");
  return LT_OK;
}

lt_status lt_mlp_grads(lt_mlp m, const void* X, const int8_t* labels, int64_t B, void* stream) {
  if (!m || !X || !labels || B < 1 || B > (int64_t(1) << 21)) return fail(LT_ERR_ARG, "batch size must be in [1, 2^21]");
  return mlp_backward(m, static_cast<const __bf16*>(X), labels, B, static_cast<hipStream_t>(stream));
}

lt_status lt_mlp_train_step(lt_mlp m, const void* X, const int8_t* labels, int64_t B, float lr,
                            void* stream) {
  LT_TRY_STATUS(lt_mlp_grads(m, X, labels, B, stream));
  hipStream_t s = static_cast<hipStream_t>(stream);
  m->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, float(m->step)), c2 = 1.f - std::pow(b2, float(m->step));
  k_adam<<<nblk(lt_mlp_s::nparam, 256), 256, 0, s>>>(m->P, m->G, m->M1, m->M2, nullptr,
                                                     lt_mlp_s::nparam, lr, b1, b2, 1e-8f, c1, c2);
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "adam launch");
  return mlp_refresh(m, s);
}

lt_status lt_mlp_infer(lt_mlp m, const void* X, int64_t n, float* logits, void* stream) {
  if (!m || !X || !logits) return fail(LT_ERR_ARG, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int64_t b0 = 0; b0 < n; b0 += (int64_t(1) << 20)) {
    const int64_t B = std::min<int64_t>(n - b0, int64_t(1) << 20);
    LT_TRY_STATUS(mlp_scratch(m, B));
    LT_TRY_STATUS(mlp_forward(m, static_cast<const __bf16*>(X) + b0 * 320, B, logits + b0 * 3, s));
  }
  return LT_OK;
}

lt_status lt_flag_mlp(lt_tree t, lt_mlp m, const lt_flag_params* fallback, const double* u, int64_t ld,
                      float conf_min, int8_t* flags, float* conf, void* stream) {
  if (!t || !m || !fallback || !u || !flags) return fail(LT_ERR_ARG, "NULL argument");
  if (t->g.dim != 3) return fail(LT_ERR_ARG, "the learned indicator takes 3D p = 3 elements");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = t->n_cur;
  if (ld < n) return fail(LT_ERR_ARG, "leading dimension too small");
  LT_TRY_STATUS(launch_flag(t->g, fallback, t->kbuf[t->cur], n, flags, s));
  if (n == 0) return LT_OK;
  LT_TRY_STATUS(mlp_reserve(m, n));
  return launch_mlp_flag(t, m, Count{n, nullptr}, u, ld, conf_min, flags, conf, s);
}

lt_status lt_vortex_field(lt_tree t, const lt_flag_params* where, const double* strength, double* u,
                          int64_t ld, void* stream) {
  if (!t || !where || !strength || !u || !where->centre || !where->nodes01)
    return fail(LT_ERR_ARG, "NULL argument");
  if (where->nvort < 1 || where->nvort > LT_MAX_VORTICES) return fail(LT_ERR_ARG, "bad vortex count");
  if (where->p < 0 || where->p > 3) return fail(LT_ERR_ARG, "vortex field supports p <= 3");
  if (ld < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  FieldArgs A{};
  A.g = t->g;
  A.nvort = where->nvort;
  for (int v = 0; v < where->nvort; ++v) {
    A.c[v][0] = where->centre[3 * v];
    A.c[v][1] = where->centre[3 * v + 1];
    A.a[v] = strength[v];
  }
  for (int a = 0; a < 3; ++a) A.lo[a] = where->lo[a];
  A.dx = where->len / double(uint64_t(1) << t->g.dmax);
  for (int k = 0; k <= where->p; ++k) A.nodes[k] = where->nodes01[k];
  const int n1 = where->p + 1;
  const int64_t npts = t->g.dim == 3 ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
  const int64_t total = t->n_cur * npts;
  if (total == 0) return LT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned blocks = nblk(total, 256);
  switch (n1) {
    case 1: k_vortex_field<1><<<blocks, 256, 0, s>>>(A, t->kbuf[t->cur], t->n_cur, u, ld); break;
    case 2: k_vortex_field<2><<<blocks, 256, 0, s>>>(A, t->kbuf[t->cur], t->n_cur, u, ld); break;
    case 3: k_vortex_field<3><<<blocks, 256, 0, s>>>(A, t->kbuf[t->cur], t->n_cur, u, ld); break;
    default: k_vortex_field<4><<<blocks, 256, 0, s>>>(A, t->kbuf[t->cur], t->n_cur, u, ld); break;
  }
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "vortex field launch");
  return LT_OK;
}

lt_status lt_flag_modal(lt_tree t, int p, const double* u, int64_t ld, double tau_refine,
                        double tau_coarsen, int8_t* flags, void* stream) {
  if (!t || !u || !flags) return fail(LT_ERR_ARG, "NULL argument");
  if (p < 1 || p > 3) return fail(LT_ERR_ARG, "modal indicator supports p = 1..3");
  if (ld < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  if (!(tau_coarsen <= tau_refine)) return fail(LT_ERR_ARG, "need tau_coarsen <= tau_refine");
  const int64_t n = t->n_cur;
  if (n == 0) return LT_OK;
  ModalT M{};
  modal_matrix(p, M.T);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned blocks = nblk(n, 256);
  const uint64_t* keys = t->kbuf[t->cur];
#define LT_M(N1, D) k_flag_modal<N1, D><<<blocks, 256, 0, s>>>(t->g, keys, n, M, u, ld, tau_refine, tau_coarsen, flags)
  if (t->g.dim == 3) {
    if (p == 1) LT_M(2, 3); else if (p == 2) LT_M(3, 3); else LT_M(4, 3);
  } else {
    if (p == 1) LT_M(2, 2); else if (p == 2) LT_M(3, 2); else LT_M(4, 2);
  }
#undef LT_M
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "modal indicator launch");
  return LT_OK;
}

void lt_mlp_destroy(lt_mlp m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {m->P, m->G, m->M1, m->M2, m->W1, m->W2, m->W3, m->W1T, m->W2T, m->W3T, m->T4,
                  m->H1, m->H2, m->XT, m->H1T, m->H2T, m->D1T, m->D2T, m->D3T, m->D2b, m->D3b,
                  m->Z3, m->D1, m->D2, m->D3, m->loss, m->X};
  for (void* p : ptrs) (void)dev_free(m->A, p);
  delete m;
}

}  // extern "C"
