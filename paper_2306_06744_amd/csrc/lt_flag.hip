// lt_flag.hip -- geometric refinement criterion (Section 5.2).
//
// Built with -ffp-contract=off: the physical point coordinates and squared
// distances are evaluated as separately rounded FP64 operations in a fixed
// order, so the integer decision r^2 < R_in^2 / r^2 > R_out^2 is reproducible
// bit for bit on any IEEE FP64 implementation that follows the same order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "tree.hpp"

#pragma clang fp contract(off)

namespace lt {
namespace {

struct FlagArgs {
  KeyGeom g;
  int p, nvort, dist_axes, periodic_dist, raw;
  double lo[3], len, dx, rin2, rout2;
  double nodes[LT_MAX_DEGREE + 1];
  double c[LT_MAX_VORTICES][3];
};

// Squared distance along one axis from a point coordinate to a centre
// coordinate (minimum image when periodic), or an exact 0 for an axis the
// criterion ignores.
__device__ inline double axis_d2(double x, double c, bool on, bool periodic, double len) {
  double dd = x - c;
  if (periodic) {
    const double q = dd / len;
    const double f = floor(q + 0.5);
    const double sh = len * f;
    dd = dd - sh;
  }
  return on ? dd * dd : 0.0;
}

// One thread per element.  The coordinate of point index k on axis a depends
// only on (a, k), so the (p+1) values per axis are computed once, and so are
// the squared distances per axis to a centre: r^2 = (dx^2 + dy^2) + dz^2 is
// then two additions per point, in the same order as point by point (an axis
// outside the criterion adds an exact 0).  With several vortices each point
// keeps the smallest r^2 over the vortices; a z slice of points is handled at
// a time so that this running minimum stays in registers.
// TAB: each element takes the parameters of its mesh from tab (an ensemble);
// otherwise every element uses A0.
template <int N1>
__device__ inline int8_t flag_of(const FlagArgs& A, const KeyGeom& g, uint64_t key) {
  const int d = key_depth(g, key);
  uint64_t x[3];
  demorton(g, key_morton(g, key), x);
  const double s = double(uint64_t(1) << (g.dmax - d));
  const int nvort = A.nvort, da = A.dist_axes;
  const bool per = A.periodic_dist != 0;
  const double len = A.len, rin2 = A.rin2, rout2 = A.rout2;
  double X[2][N1];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const double t = s * A.nodes[k];
      const double u = double(x[a]) + t;
      const double w = A.dx * u;
      X[a][k] = A.lo[a] + w;
    }
  const int nz = g.dim == 3 ? N1 : 1;
  int n_in = 0, n_out = 0;
  // the z coordinate of slice iz, by the same operations as X[a][k]
  auto zcoord = [&](int iz) {
    const double t = s * A.nodes[iz];
    const double u = double(x[2]) + t;
    const double w = A.dx * u;
    return A.lo[2] + w;
  };
  if (nvort == 1) {
    double D2[2][N1];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int k = 0; k < N1; ++k) D2[a][k] = axis_d2(X[a][k], A.c[0][a], a < da, per, len);
    for (int iz = 0; iz < nz; ++iz) {
      const double dz = axis_d2(zcoord(iz), A.c[0][2], 2 < da, per, len);
#pragma unroll
      for (int iy = 0; iy < N1; ++iy)
#pragma unroll
        for (int ix = 0; ix < N1; ++ix) {
          const double xy = D2[0][ix] + D2[1][iy];
          const double r2 = xy + dz;
          n_in += r2 < rin2 ? 1 : 0;
          n_out += r2 > rout2 ? 1 : 0;
        }
    }
  } else {
    for (int iz = 0; iz < nz; ++iz) {
      {
        const double z = zcoord(iz);
        double best[N1 * N1];
#pragma unroll
        for (int i = 0; i < N1 * N1; ++i) best[i] = INFINITY;
        for (int v = 0; v < nvort; ++v) {
          const double cx = A.c[v][0], cy = A.c[v][1], cz = A.c[v][2];
          double Dx[N1], Dy[N1];
#pragma unroll
          for (int k = 0; k < N1; ++k) {
            Dx[k] = axis_d2(X[0][k], cx, 0 < da, per, len);
            Dy[k] = axis_d2(X[1][k], cy, 1 < da, per, len);
          }
          const double dz = axis_d2(z, cz, 2 < da, per, len);
#pragma unroll
          for (int iy = 0; iy < N1; ++iy)
#pragma unroll
            for (int ix = 0; ix < N1; ++ix) {
              const double xy = Dx[ix] + Dy[iy];
              const double r2 = xy + dz;
              double& b = best[iy * N1 + ix];
              b = r2 < b ? r2 : b;
            }
        }
#pragma unroll
        for (int i = 0; i < N1 * N1; ++i) {
          n_in += best[i] < rin2 ? 1 : 0;
          n_out += best[i] > rout2 ? 1 : 0;
        }
      }
    }
  }
  int f = n_in > n_out ? 1 : (n_in < n_out ? -1 : 0);
  if (!A.raw) {
    int lo, hi;
    depth_limits(g, key, &lo, &hi);
    if (f == 1 && d >= hi) f = 0;
    if (f == -1 && d <= lo) f = 0;
  }
  return int8_t(f);
}

template <int N1, bool TAB>
__global__ __launch_bounds__(256) void k_flag(FlagArgs A0, const FlagArgs* __restrict__ tab,
                                              const uint64_t* __restrict__ keys, Count cn,
                                              int8_t* __restrict__ flags) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= cn.get()) return;
  const KeyGeom& g = A0.g;
  const uint64_t key = keys[e];
  const FlagArgs* Ap = &A0;
  if constexpr (TAB) Ap = &tab[key_mesh(g, key)];
  flags[e] = flag_of<N1>(*Ap, g, key);
}

// An ensemble whose meshes have different degrees, in one launch: each
// element takes its mesh's parameters and branches on that mesh's point
// count (the branch is uniform across a wave except at mesh boundaries).
__global__ __launch_bounds__(256) void k_flag_mixed(KeyGeom g, const FlagArgs* __restrict__ tab,
                                                    const uint64_t* __restrict__ keys, Count cn,
                                                    int8_t* __restrict__ flags) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= cn.get()) return;
  const uint64_t key = keys[e];
  const FlagArgs& A = tab[key_mesh(g, key)];
  int8_t f = 0;
  switch (A.p + 1) {
    case 1: f = flag_of<1>(A, g, key); break;
    case 2: f = flag_of<2>(A, g, key); break;
    case 3: f = flag_of<3>(A, g, key); break;
    case 4: f = flag_of<4>(A, g, key); break;
    case 5: f = flag_of<5>(A, g, key); break;
    case 6: f = flag_of<6>(A, g, key); break;
    case 7: f = flag_of<7>(A, g, key); break;
    default: f = flag_of<8>(A, g, key); break;
  }
  flags[e] = f;
}

template <int N1>
hipError_t launch(const FlagArgs& A, const FlagArgs* tab, const uint64_t* keys, Count n, int8_t* flags,
                  hipStream_t s) {
  const unsigned blocks = unsigned((n.n + 255) / 256);
  if (tab)
    k_flag<N1, true><<<blocks, 256, 0, s>>>(A, tab, keys, n, flags);
  else
    k_flag<N1, false><<<blocks, 256, 0, s>>>(A, tab, keys, n, flags);
  return hipGetLastError();
}

lt_status fill_args(const KeyGeom& g, const lt_flag_params* fp, FlagArgs* out) {
  if (fp->nvort < 1 || fp->nvort > LT_MAX_VORTICES || !fp->centre)
    return fail(LT_ERR_ARG, "nvort must be in 1..LT_MAX_VORTICES with centres given");
  if (fp->p < 0 || fp->p > LT_MAX_DEGREE || !fp->nodes01)
    return fail(LT_ERR_ARG, "p must be in 0..LT_MAX_DEGREE with nodes01 given");
  if (fp->dist_axes < 1 || fp->dist_axes > g.dim) return fail(LT_ERR_ARG, "dist_axes out of range");
  if (!(fp->len > 0.0)) return fail(LT_ERR_ARG, "len must be positive");
  FlagArgs A{};
  A.g = g;
  A.p = fp->p;
  A.nvort = fp->nvort;
  A.dist_axes = fp->dist_axes;
  A.periodic_dist = fp->periodic_dist ? 1 : 0;
  A.raw = fp->raw ? 1 : 0;
  for (int a = 0; a < 3; ++a) A.lo[a] = a < g.dim ? fp->lo[a] : 0.0;
  A.len = fp->len;
  A.dx = fp->len / double(uint64_t(1) << g.dmax);
  A.rin2 = fp->r_in * fp->r_in;
  A.rout2 = fp->r_out * fp->r_out;
  for (int k = 0; k <= fp->p; ++k) A.nodes[k] = fp->nodes01[k];
  for (int v = 0; v < fp->nvort; ++v)
    for (int a = 0; a < 3; ++a) A.c[v][a] = fp->centre[3 * v + a];
  *out = A;
  return LT_OK;
}

hipError_t dispatch(int n1, const FlagArgs& A, const FlagArgs* tab, const uint64_t* keys, Count n,
                    int8_t* flags, hipStream_t stream) {
  switch (n1) {
    case 1: return launch<1>(A, tab, keys, n, flags, stream);
    case 2: return launch<2>(A, tab, keys, n, flags, stream);
    case 3: return launch<3>(A, tab, keys, n, flags, stream);
    case 4: return launch<4>(A, tab, keys, n, flags, stream);
    case 5: return launch<5>(A, tab, keys, n, flags, stream);
    case 6: return launch<6>(A, tab, keys, n, flags, stream);
    case 7: return launch<7>(A, tab, keys, n, flags, stream);
    default: return launch<8>(A, tab, keys, n, flags, stream);
  }
}

}  // namespace

lt_status launch_flag(const KeyGeom& g, const lt_flag_params* fp, const uint64_t* keys, int64_t n,
                      int8_t* flags, hipStream_t stream) {
  FlagArgs A;
  LT_TRY_STATUS(fill_args(g, fp, &A));
  if (n == 0) return LT_OK;
  const hipError_t e = dispatch(fp->p + 1, A, nullptr, keys, Count{n, nullptr}, flags, stream);
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("flag launch: ") + hipGetErrorString(e));
  return LT_OK;
}

size_t flag_args_size() { return sizeof(FlagArgs); }

// Copies the per-mesh table from pageable host memory (staged by the runtime
// before the call returns, so the host copy may go out of scope at once).
bool mixed_degrees(const lt_flag_params* fps, int nmesh) {
  for (int m = 1; m < nmesh; ++m)
    if (fps[m].p != fps[0].p) return true;
  return false;
}

hipError_t dispatch_table(const KeyGeom& g, const lt_flag_params* fps, int nmesh, const FlagArgs& A0,
                          const FlagArgs* tab, const uint64_t* keys, Count n, int8_t* flags,
                          hipStream_t stream) {
  if (!mixed_degrees(fps, nmesh)) return dispatch(fps[0].p + 1, A0, tab, keys, n, flags, stream);
  k_flag_mixed<<<unsigned((n.n + 255) / 256), 256, 0, stream>>>(g, tab, keys, n, flags);
  return hipGetLastError();
}

lt_status launch_flag_batch(const KeyGeom& g, const lt_flag_params* fps, int nmesh, void* dev_table,
                            const uint64_t* keys, int64_t n, int8_t* flags, hipStream_t stream) {
  std::vector<FlagArgs> H(static_cast<size_t>(nmesh));
  for (int m = 0; m < nmesh; ++m) LT_TRY_STATUS(fill_args(g, &fps[m], &H[m]));
  hipError_t e = hipMemcpyAsync(dev_table, H.data(), sizeof(FlagArgs) * nmesh, hipMemcpyHostToDevice,
                                stream);
  if (e == hipSuccess && n > 0)
    e = dispatch_table(g, fps, nmesh, H[0], static_cast<const FlagArgs*>(dev_table), keys,
                       Count{n, nullptr}, flags, stream);
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("flag launch: ") + hipGetErrorString(e));
  return LT_OK;
}

// Host table of per-mesh parameters (validated) for a later upload.
lt_status fill_flag_table(const KeyGeom& g, const lt_flag_params* fps, int nmesh, void* host_table) {
  FlagArgs* H = static_cast<FlagArgs*>(host_table);
  for (int m = 0; m < nmesh; ++m) LT_TRY_STATUS(fill_args(g, &fps[m], &H[m]));
  return LT_OK;
}

// Flags from the parameters in dev_table (one entry per mesh), over a count
// that may live on the device; fps (host, nmesh entries) fix each mesh's
// degree (one kernel for one degree, the branching kernel for several) and
// the geometry.
lt_status launch_flag_table(const KeyGeom& g, const lt_flag_params* fps, int nmesh, const void* dev_table,
                            const uint64_t* keys, Count n, int8_t* flags, hipStream_t stream) {
  FlagArgs A;
  LT_TRY_STATUS(fill_args(g, fps, &A));
  if (n.n == 0) return LT_OK;
  const hipError_t e = dispatch_table(g, fps, nmesh, A, static_cast<const FlagArgs*>(dev_table), keys, n,
                                      flags, stream);
  if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("flag launch: ") + hipGetErrorString(e));
  return LT_OK;
}

}  // namespace lt
