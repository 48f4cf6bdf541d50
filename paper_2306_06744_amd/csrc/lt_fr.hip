// lt_fr.hip -- flux reconstruction on the adapted tree: common fluxes with
// mortars at hanging faces (Section 4.3) and the FR residual with the
// three-stage Runge-Kutta step (Section 2.1, eq. rk3), for the Euler
// equations on Gauss-Legendre solution points.
//
// A face buffer FB[f][v][q][ld] (face f = 2 axis + side, variable v, face
// point q with the tangential axes in increasing order, the lower fastest,
// element fastest) first holds the solution's traces, then -- overwritten in
// place -- the common normal fluxes:
//   k_fr_trace   one lane per element: u -> traces of every face;
//   k_fr_conf    one lane per element and axis: a conforming face pair is
//                owned by its low-side element, which reads both traces and
//                writes the Rusanov flux into both slots;
//   k_fr_mortar  one wave per hanging-face row, lane = (mortar s, face point):
//                the coarse trace L2-projected onto the mortar (exact for the
//                same degree: the half-interval interpolation factors A_b),
//                the fine trace, the Rusanov flux on the mortar into the fine
//                slot, and the coarse slot's L2 projection of the mortar
//                fluxes (the half-interval projection factors P_b) summed
//                over the mortars through LDS.
// Every slot is read and written by exactly one owner: no atomics, and the
// result is the same on every run (the paper accumulates the coarse side with
// atomic additions).
//   k_fr_volume  one workgroup per 64 elements (lane = element, so every load
//                of a point row is one contiguous run), one wave per slab of
//                points along the last axis; derivatives along the in-slab
//                axes in registers, along the last axis through LDS, the
//                Radau corrections from the face buffer, and the stage
//                combination out = c0 u0 + c1 u + c2 dt R fused in.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "tree.hpp"

namespace lt {
namespace {

// shares the error word with the scans' ERR_* bits
enum : unsigned { ERR_FR_ROW = 1u << 13 };

// Per-degree FP64 tables (device, n1 = p + 1):
//   D[n1][n1] (D[i][j] = l_j'(z_i)), lL[n1], lR[n1] (l_j(-1), l_j(1)),
//   dgL[n1], dgR[n1] (Radau correction derivatives at z_i),
//   A0, A1 (half-interval interpolation, A_b[i][k] = l_k((z_i + 2b - 1)/2)),
//   P0, P1 (half-interval L2 projection back onto the whole interval).
struct FrTab {
  static constexpr int kD = 0;
  __host__ __device__ static constexpr int lL(int n) { return n * n; }
  __host__ __device__ static constexpr int lR(int n) { return n * n + n; }
  __host__ __device__ static constexpr int dgL(int n) { return n * n + 2 * n; }
  __host__ __device__ static constexpr int dgR(int n) { return n * n + 3 * n; }
  __host__ __device__ static constexpr int A(int n, int b) { return n * n + 4 * n + b * n * n; }
  __host__ __device__ static constexpr int P(int n, int b) { return 3 * n * n + 4 * n + b * n * n; }
  __host__ __device__ static constexpr int size(int n) { return 5 * n * n + 4 * n; }
};

// Host: Gauss-Legendre nodes / weights by Newton on P_n (Bonnet recurrence).
void gl_host(int n, std::vector<double>& z, std::vector<double>& w) {
  z.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p1 = x, p0 = 1.0;
      const double dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (x * p1 - p0) / (x * x - 1.0);
    z[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

double lag(const std::vector<double>& z, int k, double x) {
  double v = 1.0;
  for (size_t m = 0; m < z.size(); ++m)
    if (int(m) != k) v *= (x - z[m]) / (z[k] - z[m]);
  return v;
}

double lag_d(const std::vector<double>& z, int k, double x) {
  double s = 0.0;
  for (size_t r = 0; r < z.size(); ++r) {
    if (int(r) == k) continue;
    double t = 1.0 / (z[k] - z[r]);
    for (size_t m = 0; m < z.size(); ++m)
      if (int(m) != k && m != r) t *= (x - z[m]) / (z[k] - z[m]);
    s += t;
  }
  return s;
}

// Legendre P_n'(x) from the recurrence P_{k+1} = ((2k+1) x P_k - k P_{k-1})/(k+1)
// and P_{k+1}' = P_{k-1}' + (2k+1) P_k.
double leg_d(int n, double x) {
  if (n == 0) return 0.0;
  double pm = 1.0, pc = x, dm = 0.0, dc = 1.0;
  for (int k = 1; k < n; ++k) {
    const double pn = ((2.0 * k + 1.0) * x * pc - k * pm) / (k + 1.0);
    const double dn = dm + (2.0 * k + 1.0) * pc;
    pm = pc;
    pc = pn;
    dm = dc;
    dc = dn;
  }
  return dc;
}

std::vector<double> fr_tables(int p) {
  const int n = p + 1;
  std::vector<double> z, w, zq, wq;
  gl_host(n, z, w);
  gl_host(n + 1, zq, wq);
  std::vector<double> T(FrTab::size(n), 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T[FrTab::kD + i * n + j] = lag_d(z, j, z[i]);
  for (int j = 0; j < n; ++j) {
    T[FrTab::lL(n) + j] = lag(z, j, -1.0);
    T[FrTab::lR(n) + j] = lag(z, j, 1.0);
  }
  // g_L = (-1)^(p+1)/2 (P_{p+1} - P_p), g_R = (P_{p+1} + P_p)/2
  const double sL = (p + 1) % 2 ? -0.5 : 0.5;
  for (int i = 0; i < n; ++i) {
    T[FrTab::dgL(n) + i] = sL * (leg_d(p + 1, z[i]) - leg_d(p, z[i]));
    T[FrTab::dgR(n) + i] = 0.5 * (leg_d(p + 1, z[i]) + leg_d(p, z[i]));
  }
  for (int b = 0; b < 2; ++b) {
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) T[FrTab::A(n, b) + i * n + k] = lag(z, k, (z[i] + 2.0 * b - 1.0) / 2.0);
    // P_b = M^-1 S_b, M = diag(w) (exact for GL), S_b[j][i] = int_{half b} l_j l^_i
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int q = 0; q < n + 1; ++q) s += wq[q] / 2.0 * lag(z, j, (zq[q] + 2.0 * b - 1.0) / 2.0) * lag(z, i, zq[q]);
        T[FrTab::P(n, b) + j * n + i] = s / w[j];
      }
  }
  return T;
}

// ------------------------------------------------------------------ physics
template <int DIM>
__device__ inline double pressure(const double* U, double gm1) {
  double kin = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) kin += U[1 + a] * U[1 + a];
  return gm1 * (U[DIM + 1] - 0.5 * kin / U[0]);
}

// Euler flux along axis a of the state U (nvar = DIM + 2 values).
template <int DIM>
__device__ inline void euler_flux(const double* U, int a, double gm1, double* F) {
  const double p = pressure<DIM>(U, gm1);
  const double ua = U[1 + a] / U[0];
  F[0] = U[1 + a];
#pragma unroll
  for (int b = 0; b < DIM; ++b) F[1 + b] = U[1 + b] * ua + (b == a ? p : 0.0);
  F[DIM + 1] = (U[DIM + 1] + p) * ua;
}

// One component of the flux along axis a (recomputes the pressure).
template <int DIM>
__device__ inline double flux_comp(const double* U, int a, int v, double gm1) {
  const double ua = U[1 + a] / U[0];
  if (v == 0) return U[1 + a];
  const double p = pressure<DIM>(U, gm1);
  if (v == DIM + 1) return (U[DIM + 1] + p) * ua;
  return U[v] * ua + (v - 1 == a ? p : 0.0);
}

// Rusanov flux across a face normal to axis a, UL on the low side.
template <int DIM>
__device__ inline void rusanov(const double* UL, const double* UR, int a, double gamma, double* F) {
  constexpr int NV = DIM + 2;
  const double gm1 = gamma - 1.0;
  double FL[NV], FR[NV];
  euler_flux<DIM>(UL, a, gm1, FL);
  euler_flux<DIM>(UR, a, gm1, FR);
  const double sL = fabs(UL[1 + a] / UL[0]) + sqrt(gamma * pressure<DIM>(UL, gm1) / UL[0]);
  const double sR = fabs(UR[1 + a] / UR[0]) + sqrt(gamma * pressure<DIM>(UR, gm1) / UR[0]);
  const double lam = fmax(sL, sR);
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * (UR[v] - UL[v]);
}

// ------------------------------------------------------------------ indexing
// Point index i = sum_b idx_b N^b; face point q of a face normal to axis a:
// the other axes in increasing order, the lower fastest.
template <int DIM, int N>
__device__ inline int face_point(const int* idx, int a) {
  int q = 0, m = 1;
#pragma unroll
  for (int b = 0; b < DIM; ++b)
    if (b != a) {
      q += idx[b] * m;
      m *= N;
    }
  return q;
}

template <int DIM>
__device__ inline int64_t fb_index(int f, int v, int q, int nfp, int64_t ldf, int64_t e) {
  return (int64_t(f * (DIM + 2) + v) * nfp + q) * ldf + e;
}

// ------------------------------------------------------------------ kernels
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_fr_trace(const double* __restrict__ u, int64_t ld, int64_t n,
                                                  const double* __restrict__ tab,
                                                  double* __restrict__ fb, int64_t ldf) {
  constexpr int NP = DIM == 3 ? N * N * N : N * N;
  constexpr int NFP = NP / N;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double lL[N], lR[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    lL[j] = tab[FrTab::lL(N) + j];
    lR[j] = tab[FrTab::lR(N) + j];
  }
  for (int v = 0; v < DIM + 2; ++v) {
    double x[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) x[i] = u[(int64_t(v) * NP + i) * ld + e];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      int stride = 1;
      for (int b = 0; b < a; ++b) stride *= N;
#pragma unroll
      for (int q = 0; q < NFP; ++q) {
        // first point of the line through face point q
        int idx[3] = {0, 0, 0}, r = q;
#pragma unroll
        for (int b = 0; b < DIM; ++b)
          if (b != a) {
            idx[b] = r % N;
            r /= N;
          }
        int i0 = 0, m = 1;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
          i0 += idx[b] * m;
          m *= N;
        }
        double sl = 0.0, sr = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          sl += lL[j] * x[i0 + j * stride];
          sr += lR[j] * x[i0 + j * stride];
        }
        fb[fb_index<DIM>(2 * a, v, q, NFP, ldf, e)] = sl;
        fb[fb_index<DIM>(2 * a + 1, v, q, NFP, ldf, e)] = sr;
      }
    }
  }
}

template <int DIM, int N>
__global__ __launch_bounds__(256) void k_fr_conf(KeyGeom g, const uint64_t* __restrict__ keys,
                                                 const int32_t* __restrict__ nbr, int64_t n,
                                                 double gamma, double* __restrict__ fb, int64_t ldf,
                                                 unsigned* err) {
  constexpr int NFP = DIM == 3 ? N * N : N;
  constexpr int NV = DIM + 2;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int de = key_depth(g, keys[e]);
#pragma unroll 1
  for (int a = 0; a < DIM; ++a) {
    const int f = 2 * a + 1;
    const int64_t j = nbr[e * 2 * DIM + f];
    if (j == -2 || nbr[e * 2 * DIM + f - 1] == -2) {
      atomicOr(err, ERR_INVALID_TREE);  // a non-periodic face: not supported
      continue;
    }
    if (j < 0 || j >= n || key_depth(g, keys[j]) != de) continue;  // hanging: the mortar kernel
#pragma unroll 1
    for (int q = 0; q < NFP; ++q) {
      double UL[NV], UR[NV], F[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        UL[v] = fb[fb_index<DIM>(f, v, q, NFP, ldf, e)];
        UR[v] = fb[fb_index<DIM>(f - 1, v, q, NFP, ldf, j)];
      }
      rusanov<DIM>(UL, UR, a, gamma, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        fb[fb_index<DIM>(f, v, q, NFP, ldf, e)] = F[v];
        fb[fb_index<DIM>(f - 1, v, q, NFP, ldf, j)] = F[v];
      }
    }
  }
}

// One wave per hanging-face row [c, f, k_0 .. k_{S-1}], lane = s * NFP + q.
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_fr_mortar(const int32_t* __restrict__ hang, int64_t nrows,
                                                   int64_t n, const double* __restrict__ tab,
                                                   double gamma, double* __restrict__ fb, int64_t ldf,
                                                   unsigned* err) {
  constexpr int NFP = DIM == 3 ? N * N : N;
  constexpr int S = 1 << (DIM - 1);
  constexpr int NV = DIM + 2;
  constexpr int W = 2 + S;
  static_assert(S * NFP <= 64, "one wave per row");
  __shared__ double Fm[4][S * NFP][NV];  // mortar fluxes of the wave's row
  __shared__ double Uc[4][NFP][NV];      // coarse trace
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r = int64_t(blockIdx.x) * (blockDim.x >> 6) + wv;
  const bool row_ok = r < nrows;
  const int s = lane / NFP, q = lane % NFP;
  const bool act = row_ok && lane < S * NFP;
  int64_t c = 0, k = 0;
  int f = 0;
  if (row_ok) {
    c = hang[r * W];
    f = hang[r * W + 1];
  }
  if (act) k = hang[r * W + 2 + s];
  const bool ok = !row_ok || (c >= 0 && c < n && f >= 0 && f < 2 * DIM && k >= 0 && k < n);
  if (!ok) atomicOr(err, ERR_FR_ROW);
  const bool go = act && ok;
  if (go && s == 0)
    for (int v = 0; v < NV; ++v) Uc[wv][q][v] = fb[fb_index<DIM>(f, v, q, NFP, ldf, c)];
  __syncthreads();
  const int a = f >> 1, side = f & 1;
  // tangential child bits of mortar s and the face point's tangential indices
  const int b0 = s & 1, b1 = (s >> 1) & 1;
  const int q0 = q % N, q1 = q / N;
  double Um[NV], Uk[NV], F[NV];
  if (go) {
    const double* A0 = tab + FrTab::A(N, b0);
    const double* A1 = tab + FrTab::A(N, b1);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
      if (DIM == 2) {
#pragma unroll
        for (int i = 0; i < N; ++i) acc += A0[q0 * N + i] * Uc[wv][i][v];
      } else {
#pragma unroll
        for (int i1 = 0; i1 < N; ++i1) {
          double t = 0.0;
#pragma unroll
          for (int i0 = 0; i0 < N; ++i0) t += A0[q0 * N + i0] * Uc[wv][i1 * N + i0][v];
          acc += A1[q1 * N + i1] * t;
        }
      }
      Um[v] = acc;
      Uk[v] = fb[fb_index<DIM>(f ^ 1, v, q, NFP, ldf, k)];
    }
    if (side == 1)
      rusanov<DIM>(Um, Uk, a, gamma, F);
    else
      rusanov<DIM>(Uk, Um, a, gamma, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      fb[fb_index<DIM>(f ^ 1, v, q, NFP, ldf, k)] = F[v];
      Fm[wv][lane][v] = F[v];
    }
  }
  __syncthreads();
  // coarse face: sum over the mortars of (P_b1 x P_b0) applied to their fluxes
  if (go && s == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < S; ++m) {
        const double* P0 = tab + FrTab::P(N, m & 1);
        const double* P1 = tab + FrTab::P(N, (m >> 1) & 1);
        if (DIM == 2) {
#pragma unroll
          for (int i = 0; i < N; ++i) acc += P0[q0 * N + i] * Fm[wv][m * NFP + i][v];
        } else {
#pragma unroll
          for (int i1 = 0; i1 < N; ++i1) {
            double t = 0.0;
#pragma unroll
            for (int i0 = 0; i0 < N; ++i0) t += P0[q0 * N + i0] * Fm[wv][m * NFP + i1 * N + i0][v];
            acc += P1[q1 * N + i1] * t;
          }
        }
      }
      fb[fb_index<DIM>(f, v, q, NFP, ldf, c)] = acc;
    }
  }
}

// Volume part and stage combination.  Workgroup: N waves (slab z = wave for
// 3D, y = wave for 2D), 64 elements (lane = element).
template <int DIM, int N>
__global__ __launch_bounds__(64 * N) void k_fr_volume(KeyGeom g, const uint64_t* __restrict__ keys,
                                                      int64_t n, const double* __restrict__ tab,
                                                      double length, double gamma,
                                                      const double* __restrict__ uin, int64_t ld,
                                                      const double* __restrict__ fb, int64_t ldf,
                                                      const double* __restrict__ u0, double c0,
                                                      double c1, double c2,
                                                      double* __restrict__ out, int64_t ldo) {
  constexpr int SP = DIM == 3 ? N * N : N;  // points of a slab
  constexpr int NP = SP * N;
  constexpr int NV = DIM + 2;
  constexpr int NFP = SP;
  constexpr int LA = DIM - 1;  // the slab axis
  __shared__ double H[N][SP][64];
  __shared__ double tb[5 * N * N + 4 * N];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < FrTab::size(N); i += blockDim.x) tb[i] = tab[i];
  const int64_t e = int64_t(blockIdx.x) * 64 + lane;
  const bool live = e < n;
  const double gm1 = gamma - 1.0;
  double U[NV][SP];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int sp = 0; sp < SP; ++sp)
      U[v][sp] = live ? uin[(int64_t(v) * NP + w * SP + sp) * ld + e] : (v == 0 ? 1.0 : 0.0);
  const double h = live ? ldexp(length, -key_depth(g, keys[e])) : 1.0;
  const double scale = -2.0 / h;
  __syncthreads();
  const double* D = tb + FrTab::kD;
  const double* lL = tb + FrTab::lL(N);
  const double* lR = tb + FrTab::lR(N);
  const double* dgL = tb + FrTab::dgL(N);
  const double* dgR = tb + FrTab::dgR(N);
#pragma unroll 1
  for (int v = 0; v < NV; ++v) {
    double R[SP];
#pragma unroll
    for (int sp = 0; sp < SP; ++sp) R[sp] = 0.0;
    // in-slab axes
#pragma unroll
    for (int a = 0; a < DIM - 1; ++a) {
      const int stride = a == 0 ? 1 : N;
#pragma unroll
      for (int l = 0; l < SP / N; ++l) {
        // line l: the other in-slab index (3D) or none (2D)
        const int base = a == 0 ? l * N : l;
        double Fv[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
          double Up[NV];
#pragma unroll
          for (int vv = 0; vv < NV; ++vv) Up[vv] = U[vv][base + j * stride];
          Fv[j] = flux_comp<DIM>(Up, a, v, gm1);
        }
        double FL = 0.0, FR = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          FL += lL[j] * Fv[j];
          FR += lR[j] * Fv[j];
        }
        int idx[3] = {0, 0, 0};
        idx[LA] = w;
        if (DIM == 3) idx[a == 0 ? 1 : 0] = l;  // the in-slab index across the line
        const int q = face_point<DIM, N>(idx, a);
        const double HL = live ? fb[fb_index<DIM>(2 * a, v, q, NFP, ldf, e)] : 0.0;
        const double HR = live ? fb[fb_index<DIM>(2 * a + 1, v, q, NFP, ldf, e)] : 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          double d = 0.0;
#pragma unroll
          for (int j = 0; j < N; ++j) d += D[i * N + j] * Fv[j];
          R[base + i * stride] += d + dgL[i] * (HL - FL) + dgR[i] * (HR - FR);
        }
      }
    }
    // the slab axis through LDS
#pragma unroll
    for (int sp = 0; sp < SP; ++sp) {
      double Up[NV];
#pragma unroll
      for (int vv = 0; vv < NV; ++vv) Up[vv] = U[vv][sp];
      H[w][sp][lane] = flux_comp<DIM>(Up, LA, v, gm1);
    }
    __syncthreads();
#pragma unroll
    for (int sp = 0; sp < SP; ++sp) {
      double d = 0.0, FL = 0.0, FR = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double x = H[k][sp][lane];
        d += D[w * N + k] * x;
        FL += lL[k] * x;
        FR += lR[k] * x;
      }
      const double HL = live ? fb[fb_index<DIM>(2 * LA, v, sp, NFP, ldf, e)] : 0.0;
      const double HR = live ? fb[fb_index<DIM>(2 * LA + 1, v, sp, NFP, ldf, e)] : 0.0;
      R[sp] += d + dgL[w] * (HL - FL) + dgR[w] * (HR - FR);
    }
    __syncthreads();
    if (live) {
#pragma unroll
      for (int sp = 0; sp < SP; ++sp) {
        const int64_t o = (int64_t(v) * NP + w * SP + sp);
        double r = c1 * U[v][sp] + c2 * (scale * R[sp]);
        if (c0 != 0.0) r += c0 * u0[o * ld + e];
        out[o * ldo + e] = r;
      }
    }
  }
}

template <int DIM, int N>
lt_status fr_faces(lt_tree_s* t, const double* u, int64_t ld, const double* tab, double gamma,
                   double* fb, int64_t ldf, hipStream_t s) {
  const int64_t n = t->n_cur;
  k_fr_trace<DIM, N><<<unsigned((n + 255) / 256), 256, 0, s>>>(u, ld, n, tab, fb, ldf);
  k_fr_conf<DIM, N><<<unsigned((n + 255) / 256), 256, 0, s>>>(t->g, t->kbuf[t->cur], t->nbr, n, gamma,
                                                              fb, ldf, &t->dctr->err);
  if (t->n_hang > 0)
    k_fr_mortar<DIM, N><<<unsigned((t->n_hang + 3) / 4), 256, 0, s>>>(t->hang, t->n_hang, n, tab, gamma,
                                                                       fb, ldf, &t->dctr->err);
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "FR face kernels launch");
  return LT_OK;
}

template <int DIM, int N>
lt_status fr_volume(lt_tree_s* t, const double* tab, double length, double gamma, const double* uin,
                    int64_t ld, const double* fb, int64_t ldf, const double* u0, double c0, double c1,
                    double c2, double* out, int64_t ldo, hipStream_t s) {
  const int64_t n = t->n_cur;
  k_fr_volume<DIM, N><<<unsigned((n + 63) / 64), 64 * N, 0, s>>>(t->g, t->kbuf[t->cur], n, tab, length,
                                                                 gamma, uin, ld, fb, ldf, u0, c0, c1,
                                                                 c2, out, ldo);
  if (hipGetLastError() != hipSuccess) return fail(LT_ERR_HIP, "FR volume kernel launch");
  return LT_OK;
}

}  // namespace
}  // namespace lt

// ------------------------------------------------------------------ entry points
namespace lt {
namespace {

lt_status fr_check(lt_tree_s* t, int p, const char* who) {
  if (!t) return fail(LT_ERR_ARG, std::string(who) + ": NULL tree");
  const int dim = t->g.dim;
  if ((dim == 3 && (p < 1 || p > 3)) || (dim == 2 && (p < 1 || p > LT_MAX_DEGREE)))
    return fail(LT_ERR_ARG, std::string(who) + ": p must be 1..3 in 3D, 1..7 in 2D");
  if (t->g.nmesh != 1) return fail(LT_ERR_ARG, std::string(who) + ": one tree, not an ensemble");
  if (t->g.periodic != (1u << dim) - 1u)
    return fail(LT_ERR_ARG, std::string(who) + ": the domain must be periodic on every axis");
  if (!t->conn_valid) return fail(LT_ERR_STATE, std::string(who) + ": needs lt_connect on the current leaves");
  if (t->n_cur < 1) return fail(LT_ERR_ARG, std::string(who) + ": empty tree");
  return LT_OK;
}

lt_status fr_tab(lt_tree_s* t, int p, hipStream_t s, const double** out) {
  if (!t->fr_tab[p]) {
    const std::vector<double> T = fr_tables(p);
    void* q = nullptr;
    if (dev_malloc(t->A, &q, T.size() * sizeof(double)) != hipSuccess) return fail(LT_ERR_OOM, "FR tables");
    if (hipMemcpyAsync(q, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      (void)dev_free(t->A, q);
      return fail(LT_ERR_HIP, "FR table upload");
    }
    t->fr_tab[p] = static_cast<double*>(q);
  }
  *out = t->fr_tab[p];
  return LT_OK;
}

int64_t face_doubles(int dim, int p) {
  int64_t nfp = 1;
  for (int a = 0; a < dim - 1; ++a) nfp *= p + 1;
  return int64_t(2 * dim) * (dim + 2) * nfp;
}

lt_status faces(lt_tree_s* t, int p, const double* u, int64_t ld, const double* tab, double gamma,
                double* fb, int64_t ldf, hipStream_t s) {
#define LT_F(D, NN) return fr_faces<D, NN>(t, u, ld, tab, gamma, fb, ldf, s)
  if (t->g.dim == 3) {
    switch (p) {
      case 1: LT_F(3, 2);
      case 2: LT_F(3, 3);
      default: LT_F(3, 4);
    }
  }
  switch (p) {
    case 1: LT_F(2, 2);
    case 2: LT_F(2, 3);
    case 3: LT_F(2, 4);
    case 4: LT_F(2, 5);
    case 5: LT_F(2, 6);
    case 6: LT_F(2, 7);
    default: LT_F(2, 8);
  }
#undef LT_F
}

lt_status volume(lt_tree_s* t, int p, const double* tab, double length, double gamma, const double* uin,
                 int64_t ld, const double* fb, int64_t ldf, const double* u0, double c0, double c1,
                 double c2, double* out, int64_t ldo, hipStream_t s) {
#define LT_V(D, NN) return fr_volume<D, NN>(t, tab, length, gamma, uin, ld, fb, ldf, u0, c0, c1, c2, out, ldo, s)
  if (t->g.dim == 3) {
    switch (p) {
      case 1: LT_V(3, 2);
      case 2: LT_V(3, 3);
      default: LT_V(3, 4);
    }
  }
  switch (p) {
    case 1: LT_V(2, 2);
    case 2: LT_V(2, 3);
    case 3: LT_V(2, 4);
    case 4: LT_V(2, 5);
    case 5: LT_V(2, 6);
    case 6: LT_V(2, 7);
    default: LT_V(2, 8);
  }
#undef LT_V
}

lt_status internal_faces(lt_tree_s* t, int p, int64_t* ldf) {
  const int64_t n = t->n_cur;
  LT_TRY_STATUS(grow(t->A, &t->fr_fb, &t->fr_fb_cap, face_doubles(t->g.dim, p) * n));
  *ldf = n;
  return LT_OK;
}

}  // namespace
}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_fr_face_flux(lt_tree t, int p, const double* u, int64_t ld, double gamma, double* fhat,
                          int64_t ld_f, void* stream) {
  LT_TRY_STATUS(fr_check(t, p, "lt_fr_face_flux"));
  if (!u || !fhat) return fail(LT_ERR_ARG, "NULL argument");
  if (ld < t->n_cur || ld_f < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  if (!(gamma > 1.0)) return fail(LT_ERR_ARG, "gamma must exceed 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double* tab = nullptr;
  LT_TRY_STATUS(fr_tab(t, p, s, &tab));
  return faces(t, p, u, ld, tab, gamma, fhat, ld_f, s);
}

lt_status lt_fr_residual(lt_tree t, int p, const double* u, int64_t ld, double gamma, double length,
                         double* R, int64_t ld_r, void* stream) {
  LT_TRY_STATUS(fr_check(t, p, "lt_fr_residual"));
  if (!u || !R || u == R) return fail(LT_ERR_ARG, "NULL argument or R aliasing u");
  if (ld < t->n_cur || ld_r < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  if (!(gamma > 1.0) || !(length > 0.0)) return fail(LT_ERR_ARG, "gamma must exceed 1, length be positive");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double* tab = nullptr;
  LT_TRY_STATUS(fr_tab(t, p, s, &tab));
  int64_t ldf = 0;
  LT_TRY_STATUS(internal_faces(t, p, &ldf));
  LT_TRY_STATUS(faces(t, p, u, ld, tab, gamma, t->fr_fb, ldf, s));
  return volume(t, p, tab, length, gamma, u, ld, t->fr_fb, ldf, nullptr, 0.0, 0.0, 1.0, R, ld_r, s);
}

lt_status lt_fr_rk3(lt_tree t, int p, double* u, int64_t ld, double* work, double dt, double gamma,
                    double length, int steps, void* stream) {
  LT_TRY_STATUS(fr_check(t, p, "lt_fr_rk3"));
  if (!u || !work || u == work) return fail(LT_ERR_ARG, "NULL argument or work aliasing u");
  if (ld < t->n_cur) return fail(LT_ERR_ARG, "leading dimension too small");
  if (!(gamma > 1.0) || !(length > 0.0) || !(dt > 0.0) || steps < 0)
    return fail(LT_ERR_ARG, "gamma must exceed 1, length and dt be positive, steps >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double* tab = nullptr;
  LT_TRY_STATUS(fr_tab(t, p, s, &tab));
  int64_t ldf = 0;
  LT_TRY_STATUS(internal_faces(t, p, &ldf));
  double* fb = t->fr_fb;
  for (int k = 0; k < steps; ++k) {
    // u1 = u + dt R(u)
    LT_TRY_STATUS(faces(t, p, u, ld, tab, gamma, fb, ldf, s));
    LT_TRY_STATUS(volume(t, p, tab, length, gamma, u, ld, fb, ldf, nullptr, 0.0, 1.0, dt, work, ld, s));
    // u2 = 3/4 u + 1/4 u1 + 1/4 dt R(u1)   (written over u1)
    LT_TRY_STATUS(faces(t, p, work, ld, tab, gamma, fb, ldf, s));
    LT_TRY_STATUS(volume(t, p, tab, length, gamma, work, ld, fb, ldf, u, 0.75, 0.25, 0.25 * dt, work, ld, s));
    // u_next = 1/3 u + 2/3 u2 + 2/3 dt R(u2)   (written over u)
    LT_TRY_STATUS(faces(t, p, work, ld, tab, gamma, fb, ldf, s));
    LT_TRY_STATUS(volume(t, p, tab, length, gamma, work, ld, fb, ldf, u, 1.0 / 3.0, 2.0 / 3.0,
                         2.0 / 3.0 * dt, u, ld, s));
  }
  return LT_OK;
}

}  // extern "C"
