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
//   k_fr_volume  a lane holds one x-line of points of one element (lanes
//                of a wave part = consecutive elements, so every load of a
//                point row is one contiguous run); the x derivative in
//                registers, the y and z derivatives through LDS, the Radau
//                corrections from the face buffer, and the stage combination
//                out = c0 u0 + c1 u + c2 dt R fused in.
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

// The 1D operators are built by constexpr functions, so that the volume
// kernel takes them as literal constants (no loads, no registers held across
// its loop) and the device tables of the other kernels hold the same values.

// cos by its Taylor series (|x| <= pi; a starting guess only).
constexpr double cx_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr double cx_abs(double x) { return x < 0.0 ? -x : x; }

// P_n(x) and P_{n-1}(x) by the three-term (Bonnet) recurrence.
constexpr void legendre_pair(int n, double x, double* pn, double* pm) {
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = n == 0 ? 1.0 : p1;
  *pm = n == 0 ? 0.0 : p0;
}

template <int Q>
struct GaussLegendre {
  double z[Q] = {};
  double w[Q] = {};
};

// Gauss-Legendre nodes (ascending) and weights: Newton on P_Q from the usual
// cosine guess, w = 2 / ((1 - z^2) P_Q'(z)^2).
template <int Q>
constexpr GaussLegendre<Q> gauss_legendre() {
  GaussLegendre<Q> r;
  for (int i = 0; i < Q; ++i) {
    double x = -cx_cos(M_PI * (i + 0.75) / (Q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn = 0.0, pm = 0.0;
      legendre_pair(Q, x, &pn, &pm);
      const double dp = Q * (x * pn - pm) / (x * x - 1.0);
      const double dx = pn / dp;
      x -= dx;
      if (cx_abs(dx) < 1e-16) break;
    }
    double pn = 0.0, pm = 0.0;
    legendre_pair(Q, x, &pn, &pm);
    const double dp = Q * (x * pn - pm) / (x * x - 1.0);
    r.z[i] = x;
    r.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return r;
}

// Lagrange basis l_k on the nodes z (n of them) and its derivative.
constexpr double lag(const double* z, int n, int k, double x) {
  double v = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != k) v *= (x - z[m]) / (z[k] - z[m]);
  return v;
}

constexpr double lag_d(const double* z, int n, int k, double x) {
  double s = 0.0;
  for (int r = 0; r < n; ++r) {
    if (r == k) continue;
    double t = 1.0 / (z[k] - z[r]);
    for (int m = 0; m < n; ++m)
      if (m != k && m != r) t *= (x - z[m]) / (z[k] - z[m]);
    s += t;
  }
  return s;
}

// P_n'(x) from P_{k+1}' = P_{k-1}' + (2k+1) P_k.
constexpr double leg_d(int n, double x) {
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

// The operators of degree N - 1 on N Gauss-Legendre points, laid out as the
// device table (FrTab).
template <int N>
struct Ops1D {
  double t[5 * N * N + 4 * N] = {};
};

template <int N>
constexpr Ops1D<N> ops_1d() {
  constexpr int p = N - 1;
  const GaussLegendre<N> gl = gauss_legendre<N>();
  const GaussLegendre<N + 1> gq = gauss_legendre<N + 1>();
  Ops1D<N> o;
  double* T = o.t;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) T[FrTab::kD + i * N + j] = lag_d(gl.z, N, j, gl.z[i]);
  for (int j = 0; j < N; ++j) {
    T[FrTab::lL(N) + j] = lag(gl.z, N, j, -1.0);
    T[FrTab::lR(N) + j] = lag(gl.z, N, j, 1.0);
  }
  // g_L = (-1)^(p+1)/2 (P_{p+1} - P_p), g_R = (P_{p+1} + P_p)/2
  const double sL = (p + 1) % 2 ? -0.5 : 0.5;
  for (int i = 0; i < N; ++i) {
    T[FrTab::dgL(N) + i] = sL * (leg_d(p + 1, gl.z[i]) - leg_d(p, gl.z[i]));
    T[FrTab::dgR(N) + i] = 0.5 * (leg_d(p + 1, gl.z[i]) + leg_d(p, gl.z[i]));
  }
  for (int b = 0; b < 2; ++b) {
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < N; ++k) T[FrTab::A(N, b) + i * N + k] = lag(gl.z, N, k, (gl.z[i] + 2.0 * b - 1.0) / 2.0);
    // P_b = M^-1 S_b, M = diag(w) (exact for GL), S_b[j][i] = int_{half b} l_j l^_i
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int q = 0; q < N + 1; ++q)
          s += gq.w[q] / 2.0 * lag(gl.z, N, j, (gq.z[q] + 2.0 * b - 1.0) / 2.0) * lag(gl.z, N, i, gq.z[q]);
        T[FrTab::P(N, b) + j * N + i] = s / gl.w[j];
      }
  }
  return o;
}

template <int N>
std::vector<double> tables_of() {
  constexpr Ops1D<N> o = ops_1d<N>();
  return std::vector<double>(o.t, o.t + FrTab::size(N));
}

std::vector<double> fr_tables(int p) {
  switch (p + 1) {
    case 2: return tables_of<2>();
    case 3: return tables_of<3>();
    case 4: return tables_of<4>();
    case 5: return tables_of<5>();
    case 6: return tables_of<6>();
    case 7: return tables_of<7>();
    default: return tables_of<8>();
  }
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

// Entry r of N compile-time values, r uniform across the wave, as
// sum_k [k == r] row[k] (exact: the other terms are zeros), so that no array
// is indexed at run time (which would place it in scratch memory).
template <int N>
__device__ inline double row_at(const double* row, int r) {
  double x = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) x += (r == k ? 1.0 : 0.0) * row[k];
  return x;
}

// Volume part and stage combination.  A lane holds one x-line of N points
// of one element; a workgroup holds every line of EB = 64 / H elements
// (lane = element within each of the H parts of a wave, so that every load
// of a point row is one contiguous run).  Wave w holds lines w + (NL / H) h,
// h = 0..H-1 (NL = N^2 lines in 3D, N in 2D); NL / H is a multiple of N so
// that the line's y is uniform across the wave.  Each point's inverse density
// and pressure are formed once per pass; the variables are taken one at a
// time (a loop that is not unrolled, to bound the code and the registers),
// with component v of the flux along axis a written as
//   F_a[v] = (U[v] + [v is energy] p) m_a / rho + [v is momentum a] p
// (the mass flux m_a for v = 0).  U[v] is formed as sum_k [k == v] U[k]
// (exact: the other terms are zeros), so that no register array is indexed
// by the loop variable (that would move it to scratch memory).  The x
// derivative stays in registers; the y and z fluxes go through LDS for the
// derivatives across lines.  The 1D operators are literal constants.
template <int DIM, int N, int H>
__global__ __launch_bounds__(64 * (DIM == 3 ? N * N : N) / H) void k_fr_volume(
    KeyGeom g, const uint64_t* __restrict__ keys, int64_t n, double length, double gamma,
    const double* __restrict__ uin, int64_t ld, const double* __restrict__ fb, int64_t ldf,
    const double* __restrict__ u0, double c0, double c1, double c2, double* __restrict__ out,
    int64_t ldo) {
  constexpr int NL = DIM == 3 ? N * N : N;  // x-lines
  constexpr int NP = NL * N;
  constexpr int NV = DIM + 2;
  constexpr int NFP = NL;  // points of a face
  constexpr int EB = 64 / H;  // elements of a workgroup
  static_assert(NL % H == 0 && (NL / H) % N == 0, "the parts of a wave must share y");
  constexpr Ops1D<N> O = ops_1d<N>();
  const double* D = O.t + FrTab::kD;
  const double* lL = O.t + FrTab::lL(N);
  const double* lR = O.t + FrTab::lR(N);
  const double* dgL = O.t + FrTab::dgL(N);
  const double* dgR = O.t + FrTab::dgR(N);
  __shared__ double Hy[NP][EB];
  __shared__ double Hz[DIM == 3 ? NP : 1][EB];
  const int lane = threadIdx.x & 63;
  const int el = lane % EB;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = w + (NL / H) * (lane / EB);  // the lane's line
  const int y = w % N;                       // uniform
  const int z = l / N;                       // uniform when H = 1
  const int64_t e0 = int64_t(blockIdx.x) * EB;
  const bool live = e0 + el < n;
  // lanes past the last element read the last element's values and store nothing
  const int64_t e = live ? e0 + el : n - 1;
  const double gm1 = gamma - 1.0;
  auto row = [&](auto* p, int64_t r, int64_t stride) { return p + (r * stride + e); };
  double U[NV][N];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int i = 0; i < N; ++i) U[v][i] = *row(uin, int64_t(v) * NP + l * N + i, ld);
  const double h = ldexp(length, -key_depth(g, keys[e]));
  const double scale = -2.0 / h;
  // the operators' rows at the line's y and z
  double Dy[N], Dz[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double c[N];
#pragma unroll
    for (int r = 0; r < N; ++r) c[r] = D[r * N + k];
    Dy[k] = row_at<N>(c, y);
    Dz[k] = row_at<N>(c, z);
  }
  const double gLy = row_at<N>(dgL, y), gRy = row_at<N>(dgR, y);
  const double gLz = row_at<N>(dgL, z), gRz = row_at<N>(dgR, z);
#pragma unroll 1
  for (int v = 0; v < NV; ++v) {
    // values derived from the state are not kept across passes
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int i = 0; i < N; ++i) asm volatile("" : "+v"(U[k][i]));
    double ir[N], pr[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      ir[i] = 1.0 / U[0][i];
      double kin = 0.0;
#pragma unroll
      for (int b = 0; b < DIM; ++b) kin += U[1 + b][i] * U[1 + b][i];
      pr[i] = gm1 * (U[NV - 1][i] - 0.5 * kin * ir[i]);
    }
    const double HxL = *row(fb, fb_index<DIM>(0, v, l, NFP, 1, 0), ldf);
    const double HxR = *row(fb, fb_index<DIM>(1, v, l, NFP, 1, 0), ldf);
    // the y and z face values too: consumed (below) before the barrier, so
    // that their loads overlap this variable's flux work instead of being
    // sunk to their use after the barrier, where nothing hides them
    double HyL[N], HyR[N], HzL[N], HzR[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      HyL[i] = *row(fb, fb_index<DIM>(2, v, i + N * z, NFP, 1, 0), ldf);
      HyR[i] = *row(fb, fb_index<DIM>(3, v, i + N * z, NFP, 1, 0), ldf);
      HzL[i] = HzR[i] = 0.0;
      if constexpr (DIM == 3) {
        HzL[i] = *row(fb, fb_index<DIM>(4, v, i + N * y, NFP, 1, 0), ldf);
        HzR[i] = *row(fb, fb_index<DIM>(5, v, i + N * y, NFP, 1, 0), ldf);
      }
    }
    // the stage's u0 term likewise (u0 is read only when c0 is nonzero): one
    // round trip for the line instead of one per point in the store loop
    double U0[N];
#pragma unroll
    for (int i = 0; i < N; ++i) U0[i] = 0.0;
    if (c0 != 0.0)
#pragma unroll
      for (int i = 0; i < N; ++i) U0[i] = *row(u0, int64_t(v) * NP + l * N + i, ld);
    const bool is_e = v == NV - 1;
    double cur[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) x += (v == k ? 1.0 : 0.0) * U[k][i];
      cur[i] = x;
    }
    auto flux = [&](int a, int i) {
      const double x = cur[i] + (is_e ? pr[i] : 0.0);
      return x * (U[1 + a][i] * ir[i]) + (v == 1 + a ? pr[i] : 0.0);
    };
    // fluxes across lines to LDS first, so that the x work below hides the barrier's wait
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Hy[l * N + i][el] = flux(1, i);
      if constexpr (DIM == 3) Hz[l * N + i][el] = flux(2, i);
    }
    double R[N];
    {  // x: the lane's own line
      double F[N];
#pragma unroll
      for (int k = 0; k < N; ++k) F[k] = flux(0, k);
      double FL = 0.0, FR = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        FL += lL[k] * F[k];
        FR += lR[k] * F[k];
      }
      const double jL = HxL - FL, jR = HxR - FR;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double d = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) d += D[i * N + k] * F[k];
        R[i] = d + dgL[i] * jL + dgR[i] * jR;
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
      asm volatile("" ::"v"(HyL[i]), "v"(HyR[i]), "v"(HzL[i]), "v"(HzR[i]), "v"(U0[i]));
    __syncthreads();
    // y: point (i, y, z) on the line of points (i, k, z)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double d = 0.0, FL = 0.0, FR = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double x = Hy[i + N * k + N * N * z][el];
        d += Dy[k] * x;
        FL += lL[k] * x;
        FR += lR[k] * x;
      }
      R[i] += d + gLy * (HyL[i] - FL) + gRy * (HyR[i] - FR);
    }
    if constexpr (DIM == 3) {  // z: the line of points (i, y, k)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double d = 0.0, FL = 0.0, FR = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double x = Hz[i + N * y + N * N * k][el];
          d += Dz[k] * x;
          FL += lL[k] * x;
          FR += lR[k] * x;
        }
        R[i] += d + gLz * (HzL[i] - FL) + gRz * (HzR[i] - FR);
      }
    }
    if (live) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int64_t o = int64_t(v) * NP + l * N + i;
        double r = c1 * cur[i] + c2 * (scale * R[i]);
        if (c0 != 0.0) r += c0 * U0[i];
        *row(out, o, ldo) = r;
      }
    }
    __syncthreads();  // before the next variable overwrites Hy, Hz
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
  // p = 3 in 3D: four parts of 16 elements per wave, 4 waves (16 lines of
  // 16 elements): no spills at 224 VGPRs and two workgroups per CU; else one
  // part of 64 elements, one wave per line
  constexpr int H = (DIM == 3 && N == 4) ? 4 : 1;
  constexpr int waves = (DIM == 3 ? N * N : N) / H;
  constexpr int EB = 64 / H;
  k_fr_volume<DIM, N, H><<<unsigned((n + EB - 1) / EB), 64 * waves, 0, s>>>(
      t->g, t->kbuf[t->cur], n, length, gamma, uin, ld, fb, ldf, u0, c0, c1, c2, out, ldo);
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
