/*
 * lt.h -- C ABI of the MI355X (gfx950) adaptation cycle on linear trees.
 *
 * One tree (a 2D linear quadtree or 3D linear octree) lives in device memory
 * as an ascending array of 64-bit Morton IDs.  The cycle of the h-adaptive
 * flux-reconstruction method is
 *
 *     lt_flag -> lt_adapt -> lt_balance -> lt_connect -> lt_map -> lt_transfer
 *
 * Conventions shared by every entry point:
 *   - Pointers documented as "device" are HIP device pointers; "host" ones are
 *     ordinary host memory read during the call only.
 *   - `stream` is a hipStream_t (may be NULL for the null stream).  Kernels are
 *     enqueued on it in call order.  Calls that must learn a size on the host
 *     (lt_build, lt_adapt, lt_balance, lt_connect, lt_map) synchronise the
 *     stream before returning; lt_flag and lt_transfer do not.
 *   - Every call returns an lt_status; no exception crosses the ABI.  The text
 *     of the last error of the calling thread is lt_last_error().  On an
 *     error the tree's leaves, its old tree and its connectivity and mapping
 *     results are as before the call (strong guarantee), except where a
 *     declaration below says otherwise.
 *   - Caller-owned buffers (flags, solution arrays, export targets) stay owned
 *     by the caller.  Everything else (keys, the pre-adapt snapshot, nbr, hang,
 *     map arrays, scratch) is owned by the tree and freed by lt_destroy; its
 *     device memory comes from the allocator registered with lt_set_allocator
 *     when the tree was created (hipMalloc / hipFree if none was).
 *   - A tree is not thread-safe; use one tree per host thread or serialise.
 *     Calls on one tree run one after another in stream order, with a single
 *     exception: lt_connect keeps scratch of its own, so it may run on a
 *     second stream beside lt_map and lt_transfer of the same tree (issue it
 *     after lt_balance has returned; lt_connect returns once its stream is
 *     done).
 *
 * Morton ID layout (Section 2.2, Algorithm "Morton Encoding"): the anchor
 * (lowest corner) of an octant in integer units of the finest resolution
 * 2^-d_max is bit-interleaved with x least significant (bit k of axis a at
 * position dim*k + a), then shifted left by m_b = bitlength(d_max) bits that
 * hold the depth.  Ascending IDs list leaves depth-first, a parent before its
 * children, and a first child's ID is its parent's plus one.
 */
#ifndef LT_H
#define LT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lt_tree_s* lt_tree;

typedef enum {
  LT_OK = 0,
  LT_ERR_ARG = 1,          /* bad argument: null pointer, size or value out of range   */
  LT_ERR_OOM = 2,          /* a device or pinned-host allocation failed                */
  LT_ERR_HIP = 3,          /* a HIP runtime call or kernel launch failed               */
  LT_ERR_DEPTH = 4,        /* dim*d_max + m_b > 64, or a depth outside [0, d_max]      */
  LT_ERR_INVALID_TREE = 5, /* keys not strictly ascending / not a complete linear tree */
  LT_ERR_UNBALANCED = 6,   /* a step that needs a 2:1-balanced tree found it is not    */
  LT_ERR_STATE = 7,        /* call order violated (e.g. lt_map before any lt_adapt)    */
  LT_ERR_INTERNAL = 8,     /* a device-side consistency check failed                   */
  LT_ERR_CAPACITY = 9      /* a captured cycle outgrew the capacity it was created with  */
} lt_status;

/* Export / view selectors. */
typedef enum {
  LT_KEYS = 0,      /* uint64  [n_cur]                                      */
  LT_OLD_KEYS = 1,  /* uint64  [n_old]       keys before the last lt_adapt  */
  LT_NBR = 2,       /* int32   [n_cur * 2*dim]                              */
  LT_HANG = 3,      /* int32   [n_hang * (2 + 2^(dim-1))]                   */
  LT_MAP_SRC = 4,   /* int32   [n_cur]                                      */
  LT_MAP_KIND = 5   /* int8    [n_cur]                                      */
} lt_field;

#define LT_MAX_VORTICES 8
#define LT_MAX_DEGREE 7

/* Tree geometry.  The domain is the cube [0, 2^d_max)^dim in finest units. */
typedef struct {
  int dim;                /* 2 or 3                                                   */
  int d_min;              /* coarsening floor: no leaf coarsens below this depth      */
  int d_max;              /* refinement ceiling; dim*d_max + bitlength(d_max) <= 64   */
  unsigned periodic_mask; /* bit a set: axis a is periodic (neighbour keys wrap)      */
  int balance;            /* 2:1 balance across 0 faces, 1 faces+edges, 2 + corners   */
} lt_geom;

/* Geometric refinement criterion (Section 5.2): an element is flagged +1 when
 * more of its (p+1)^dim solution points lie strictly within r_in of the
 * nearest vortex axis than strictly beyond r_out, -1 when fewer, 0 otherwise;
 * +1 becomes 0 at depth d_max and -1 becomes 0 at depth <= d_min.
 * Point k of an element of depth D with anchor x (finest units) on axis a is
 *   lo[a] + dx * (x_a + s * nodes01[k]),  s = 2^(d_max - D), dx = len / 2^d_max,
 * evaluated in FP64 in exactly that order without fused multiply-adds;
 * r^2 = sum over axes a < dist_axes of (X_a - centre_a)^2 in axis order,
 * with the minimum image d - len*floor(d/len + 0.5) when periodic_dist. */
typedef struct {
  int nvort;              /* 1 .. LT_MAX_VORTICES                                     */
  const double* centre;   /* host, centre[3*v + a]                                    */
  double r_in, r_out;
  int dist_axes;          /* 2: distance in the xy plane (z-extruded field), 3: xyz   */
  int periodic_dist;      /* 1: minimum-image distance with period len               */
  int p;                  /* polynomial degree, 0 .. LT_MAX_DEGREE                   */
  const double* nodes01;  /* host, p+1 solution-point positions in [0,1] on one axis */
  double lo[3];           /* physical position of the domain's lowest corner         */
  double len;             /* physical edge length of the cubic domain                */
  int raw;                /* 1: skip the d_min / d_max clamps (training labels)      */
} lt_flag_params;

/* Device allocator for the trees, captured cycles and models created after
 * this call (each keeps the allocator it was created with until it is
 * destroyed).  alloc(bytes, stream, ctx) returns device memory of the
 * current device or NULL (the call needing it then fails with LT_ERR_OOM and
 * leaves its tree as before); free_(ptr, stream, ctx) releases it.  The
 * library passes stream = NULL and synchronises the device before every
 * free, so a stream-ordered caching allocator may hand the memory out again
 * at once.  Both NULL restores hipMalloc / hipFree; one NULL is LT_ERR_ARG.
 * Process-wide; ctx is passed through untouched. */
lt_status lt_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                           void (*free_)(void* ptr, void* stream, void* ctx), void* ctx);

/* Uniform tree of all 2^(dim*depth) octants at `depth` (d_min <= depth <= d_max
 * is not required: depth may be below d_min or above it up to d_max).
 * Ownership of *out passes to the caller (release with lt_destroy). */
lt_status lt_build_uniform(const lt_geom* geom, int depth, void* stream, lt_tree* out);

/* Tree from `n` device keys (copied).  The keys must be strictly ascending and
 * form a complete linear tree (the leaves tile the domain exactly); otherwise
 * LT_ERR_INVALID_TREE.  Balance is not checked here. */
lt_status lt_build(const lt_geom* geom, const uint64_t* keys, int64_t n, void* stream,
                   lt_tree* out);

/* Tree built bottom-up from n scattered points (Section 3.1, tree
 * construction and linearization; Section 5.1: a coarse background at d_min
 * with the points encoded at d_max).  pts: device FP64 [n][dim], point-major,
 * in the physical cube [lo, lo+len)^dim (lo: host, dim values).  A point's
 * finest cell is i_a = floor((x_a - lo[a]) / dx) with dx = len / 2^d_max,
 * evaluated in FP64 in that order; every cell must lie in [0, 2^d_max)
 * (LT_ERR_ARG otherwise, also for a NaN coordinate).  The result is the
 * coarsest complete linear tree whose leaves all have depth >= d_min and in
 * which every point's finest cell is a leaf (duplicates allowed; n = 0 gives
 * the uniform tree at d_min).  It is not 2:1 balanced: call lt_balance.
 * 0 <= n < 2^31 and fewer than 2^31 leaves.  Synchronises the stream; the
 * temporaries (two sort buffers of n keys, offsets) come from the registered
 * allocator and are freed before returning.  Ownership of *out passes to the
 * caller. */
lt_status lt_build_points(const lt_geom* geom, const double* pts, int64_t n, const double* lo,
                          double len, void* stream, lt_tree* out);

/* Ensemble of `nmesh` independent trees in one key array, each starting
 * uniform at depth[m] (form 2 of the cycle: every later call -- adapt,
 * balance, connect, map, transfer -- then runs each step for all meshes in one
 * launch).  geom->d_max is the shared finest level (the key resolution) and
 * geom->d_min is ignored; mesh m refines no deeper than d_max[m] and coarsens
 * no coarser than d_min[m] (0 <= d_min[m] <= d_max[m] <= geom->d_max).  The
 * mesh index is stored above the Morton bits, so keys sort mesh by mesh and
 * leaves of different meshes never touch; indices in nbr, hang and the
 * mapping are ensemble-global.  LT_ERR_DEPTH if the index does not fit in 64
 * bits.  Host arrays of nmesh entries.  Ownership of *out passes to the caller. */
lt_status lt_build_batch(const lt_geom* geom, int nmesh, const int* d_min, const int* d_max,
                         const int* depth, void* stream, lt_tree* out);

/* Flags of an ensemble: per_mesh[m] (host, nmesh entries, all with the same p)
 * gives the criterion of mesh m.  Point coordinates are computed at the shared
 * finest level, which is exact: the scalings by powers of two commute with
 * the rounding.  flags: device int8 [n_cur]. */
lt_status lt_flag_batch(lt_tree t, const lt_flag_params* per_mesh, int nmesh, int8_t* flags,
                        void* stream);

/* Per-mesh degrees of a 3D ensemble for lt_transfer_mixed and for captured
 * cycles with p = -1 (host array of nmesh values, each 1..3; form 2 of the
 * cycle with meshes of different order).  Synchronises. */
lt_status lt_set_mesh_degree(lt_tree t, const int* p, void* stream);

/* FP64 solution transfer (Section 4.2) of an ensemble whose meshes have
 * their own degree (lt_set_mesh_degree): the copy pass and the group list one
 * launch each for all meshes, each interpolation kernel one launch per degree
 * present.  Layout u[(v * NPM + i) * ld + e] with NPM the largest
 * (p+1)^3 over the meshes; an element of a mesh of degree p uses the rows
 * i < (p+1)^3 of each variable block, and its other rows are neither read nor
 * written.  Otherwise as lt_transfer at precision 0, its second stream
 * included (LT_ERR_STATE without degrees or a prior lt_adapt).  Asynchronous
 * unless the mapping was stale. */
lt_status lt_transfer_mixed(lt_tree t, int nvar, const double* u_old, int64_t ld_old, double* u_new,
                            int64_t ld_new, void* stream);

/* offsets[m] = index of the first leaf of mesh m, offsets[nmesh] = n_cur
 * (host array of nmesh + 1; a single tree has nmesh = 1).  Synchronises. */
lt_status lt_mesh_offsets(lt_tree t, int64_t* offsets, void* stream);

/* Flags of the current leaves (Section 5.2 criterion, see lt_flag_params).
 * flags: device int8 [n_cur], written in key order.  Asynchronous.  An
 * ensemble takes lt_flag_batch instead (LT_ERR_ARG here). */
lt_status lt_flag(lt_tree t, const lt_flag_params* fp, int8_t* flags, void* stream);

/* Adaptation procedure (Section 4.1): every leaf flagged +1 (depth < d_max) is
 * replaced by its 2^dim children; a family of 2^dim sibling leaves all flagged
 * -1 (depth > d_min) is replaced by its parent; every other -1 acts as 0.  No
 * octant changes more than once.  flags: device int8 [n_cur], values -1, 0, 1
 * (others: LT_ERR_ARG detected on the device, tree unchanged).  The keys
 * before the call are kept as the old tree for lt_map / lt_transfer (on an
 * error the previous old tree is kept instead). */
lt_status lt_adapt(lt_tree t, const int8_t* flags, void* stream);

/* Strong 2:1 balance (Section 3.2): replace the tree by its coarsest
 * refinement in which any two leaves touching across a face (or edge /
 * corner, per geom.balance; periodic axes wrap) differ by at most one level.
 * Every pass writes into a spare key buffer, so on any error (LT_ERR_OOM when
 * a buffer cannot grow, LT_ERR_HIP, LT_ERR_INTERNAL) the tree is exactly as
 * before the call. */
lt_status lt_balance(lt_tree t, void* stream);

/* Face connectivity (Section 3.3).  Face f = 2*axis + side (side 0 = low
 * coordinate); a conforming face f meets face f^1 of its neighbour.
 *   nbr[2*dim*e + f] = index of the one leaf of depth <= depth(e) across face f
 *                      (same depth: conforming; one coarser: e is a fine side),
 *                    = -1 when 2^(dim-1) leaves one level finer lie across
 *                      (e is the coarse side; see hang),
 *                    = -2 across a non-periodic domain boundary.
 *   hang row r = [e, f, k_0 .. k_{2^(dim-1)-1}], rows sorted by (e, f); k_s is
 *   the fine leaf whose tangential child bits (lower axis first) equal s.
 * Needs a 2:1-balanced tree (LT_ERR_UNBALANCED otherwise).  It reads only the
 * current keys and uses its own look-back words and counters: it may overlap
 * lt_map / lt_transfer issued on another stream. */
lt_status lt_connect(lt_tree t, void* stream);

/* Caps the workgroups (256 lanes each) of lt_connect's face search, which
 * strides over its lanes: 0, the default, launches one lane per face.  The
 * search is bound by the latency of its key lookups.  Issued on a second
 * stream beside lt_map and lt_transfer, a small grid (256 workgroups on
 * MI355X, one per compute unit) leaves the other wave slots to the
 * bandwidth-bound transfer, which then runs faster while the search still ends
 * first; alone, the search takes longer with a cap.  Applies to later
 * lt_connect calls and to cycles captured later.  LT_ERR_ARG if negative. */
lt_status lt_set_connect_grid(lt_tree t, int blocks);

/* Old->new mapping (Section 4.2, mapping algorithm): for each current leaf j,
 *   map_kind[j] = 0      map_src[j] = old index of the same octant (copy),
 *   map_kind[j] = 1 + c  map_src[j] = old index of its parent (refined, child c),
 *   map_kind[j] = -1     map_src[j] = old index of its first child (fused; the
 *                        2^dim children are old[src .. src + 2^dim - 1]).
 * LT_ERR_STATE without a prior lt_adapt; LT_ERR_UNBALANCED when a leaf fits
 * none of the three cases (the old tree was not balanced). */
lt_status lt_map(lt_tree t, void* stream);

/* Solution transfer (Section 4.2) from the old tree to the current one:
 * copy; interpolation of the parent polynomial at the child's points
 * (eq. parent_soln); L2 projection of the 2^dim children onto the parent.
 * Solution layout: u[(v * n_p + i) * ld + e], n_p = (p+1)^dim, point index
 * i = i_x + (p+1) (i_y + (p+1) i_z) over Gauss-Legendre points, variable v
 * slowest, element e fastest.  u_old: device FP64, ld_old >= n_old; u_new:
 * device FP64, ld_new >= n_cur, written for every current leaf.  Computes the
 * mapping first if lt_map has not run since the last change.
 *   precision 0: FP64 throughout (sum-factorised); p in 1..3 for dim 3,
 *                1..LT_MAX_DEGREE for dim 2.
 *   precision 1: dense operator products on BF16 matrix cores with every
 *                operand split in three BF16 terms and FP32 accumulation,
 *                then an FP64 shift that makes each new element's cell mean
 *                (Gauss-Legendre quadrature mean) equal the FP64 one; copies
 *                are exact.  Needs 64 points per element (dim 3 with p = 3,
 *                or dim 2 with p = 7).  Relative L2 error ~1e-7 against FP64.
 * Other values return LT_ERR_ARG, as does nvar * n_p outside [1, 65535].
 * Asynchronous (unless the mapping was stale).  In 3D at precision 0, and at
 * precision 1, the interpolation passes run on a second stream owned by the
 * tree (made on the first such call), forked from `stream` after the copy
 * pass is enqueued and joined back to it: later work on `stream` sees the
 * whole transfer.  A caller that captures this call into a graph makes one
 * such call eagerly first (or uses lt_transfer_noalloc, which stays on
 * `stream`). */
lt_status lt_transfer(lt_tree t, int p, int nvar, const double* u_old, int64_t ld_old,
                      double* u_new, int64_t ld_new, int precision, void* stream);

/* lt_transfer at precision 0 for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results bit for bit, but the
 * transfer's scratch -- copy-run source offsets, interpolation-group lists,
 * look-back words, counters, the FP64 1D operators -- lives in a static
 * device array of the library (about 5.3 MiB, one copy per GPU, kept until
 * the process ends) instead of buffers the tree grows.  The call allocates
 * nothing: it needs the mapping of the last adaptation already computed
 * (lt_map, or an earlier lt_transfer; LT_ERR_STATE otherwise), at most 2^25
 * current leaves (LT_ERR_ARG otherwise), and the tree's device current.
 * Every call on one GPU shares that array, so calls that overlap on one GPU
 * (on different streams, or from several threads) race; serialise them.
 * Arguments, layout and supported degrees as lt_transfer.  Asynchronous. */
lt_status lt_transfer_noalloc(lt_tree t, int p, int nvar, const double* u_old, int64_t ld_old,
                              double* u_new, int64_t ld_new, void* stream);

/* Tuning of the transfer's launch shapes (results never depend on them):
 * elements per lane of the copy pass (1, 2 or 4; one block row covers 256
 * times that many elements) and persistent workgroups per variable of the
 * 3D interpolation pass.  Defaults 2 and 2048. */
typedef struct {
  int copy_elems_per_lane;
  int interp_grid;
  float ms;          /* lt_autotune_transfer: mean time of the chosen shape     */
  float ms_default;  /*   and of the default shape (ms); -1 from lt_get_tuning  */
} lt_tune;

/* Times lt_transfer (same arguments, same result every time: u_new is
 * written repeatedly) for every tuning candidate -- copy elements per lane
 * {1, 2, 4} x interpolation workgroups {1024, 2048, 4096, 16384, 65535} -- with HIP events,
 * one untimed and three timed launches each, and keeps the fastest in the
 * tree for later transfers (and cycles captured later).  Synchronises. */
lt_status lt_autotune_transfer(lt_tree t, int p, int nvar, const double* u_old, int64_t ld_old,
                               double* u_new, int64_t ld_new, int precision, void* stream,
                               lt_tune* out);
/* Set / read the tree's tuning (LT_ERR_ARG for values outside the ranges). */
lt_status lt_set_tuning(lt_tree t, const lt_tune* tune);
lt_status lt_get_tuning(lt_tree t, lt_tune* tune);

/* ------------------------------------------------------------------------
 * Flux reconstruction on the current (2:1-balanced, connected, periodic)
 * tree for the Euler equations: 2D (rho, rho u, rho v, E), 3D (rho, rho u,
 * rho v, rho w, E); p = (p+1)^dim Gauss-Legendre solution points per element,
 * u[(v * n_p + i) * ld + e] as lt_transfer; gamma > 1; the tree's cube has
 * physical edge `length`.  All three need lt_connect on the current leaves
 * (LT_ERR_STATE otherwise), a tree periodic on every axis and a single mesh
 * (LT_ERR_ARG), p 1..3 in 3D and 1..7 in 2D.  Asynchronous; the tree keeps a
 * face buffer of 2 dim (dim+2) (p+1)^(dim-1) doubles per leaf.
 * ------------------------------------------------------------------------ */

/* Common normal fluxes at every element face (Section 4.3, Algorithm
 * "Procedure of common flux calculations"): the solution's traces at the
 * face points; a conforming face takes the Rusanov flux of its two traces; at
 * a hanging face the coarse trace is L2-projected onto each of the 2^(dim-1)
 * mortars (eq. interpolation_operator), the fine traces are copied onto them,
 * the Rusanov flux is taken on each mortar, each fine face receives its
 * mortar's flux and the coarse face the L2 projection of the mortar fluxes
 * (eq. projection_operator).  Each face slot has one writer: deterministic,
 * no atomics.  fhat: device FP64, fhat[((f * (dim+2) + v) * nfp + q) * ld_f + e]
 * with face f = 2 axis + side, face point q over the tangential axes in
 * increasing order (the lower fastest), nfp = (p+1)^(dim-1); the value is the
 * flux component along the face's axis (not multiplied by an outward sign). */
lt_status lt_fr_face_flux(lt_tree t, int p, const double* u, int64_t ld, double gamma, double* fhat,
                          int64_t ld_f, void* stream);

/* FR residual R = -sum_a d f_a / d x_a (Section 2.1): along every line of
 * solution points the flux polynomial's derivative plus the Radau
 * corrections g_L'(f^(-1) - f(-1)) + g_R'(f^(1) - f(1)) with the common fluxes
 * above, scaled by 2/h.  R: device FP64, layout as u with ld_r >= n_cur, not
 * aliasing u. */
lt_status lt_fr_residual(lt_tree t, int p, const double* u, int64_t ld, double gamma, double length,
                         double* R, int64_t ld_r, void* stream);

/* `steps` steps of the three-stage Runge-Kutta scheme (eq. rk3) in place on
 * u, with time step dt; work: device FP64 of u's shape and ld, not aliasing u
 * (holds the intermediate stages). */
lt_status lt_fr_rk3(lt_tree t, int p, double* u, int64_t ld, double* work, double dt, double gamma,
                    double length, int steps, void* stream);

/* Host-side sizes (no device work): current leaves, leaves before the last
 * lt_adapt (-1 if none), rows of the hanging-face table (-1 before lt_connect).
 * Any pointer may be NULL. */
lt_status lt_size(lt_tree t, int64_t* n_cur, int64_t* n_old, int64_t* n_hang);

/* Borrowed device pointer to one of the tree's arrays (NULL if not computed);
 * valid until the next call that changes the tree. */
lt_status lt_view(lt_tree t, lt_field what, const void** ptr, int64_t* count);

/* Stream-ordered device-to-device copy of one of the tree's arrays into the
 * caller's device buffer `dst` holding `capacity` elements of that field's
 * type; LT_ERR_ARG if it is too small.  dst may be NULL when the field is
 * empty; LT_ERR_STATE if the field has not been computed. */
lt_status lt_export(lt_tree t, lt_field what, void* dst, int64_t capacity, void* stream);

/* ------------------------------------------------------------------------
 * Learned refinement indicator (form 4 of the cycle), for 3D elements of 64
 * Gauss-Legendre points (p = 3) with 5 conserved variables.
 *
 * Features per element: the nodal values of each variable projected on the
 * orthonormal tensor Legendre basis (exact with Gauss-Legendre quadrature),
 * f = (log10(|c| + 1e-14) + 7) / 7, 320 values (variable-major, mode index
 * x fastest), stored BF16.  Network: 320 -> 128 -> 64 -> 3 with ReLU, BF16
 * weights and activations, FP32 accumulation on the matrix cores; classes
 * 0 coarsen, 1 keep, 2 refine.  Parameters (FP32, host layout): W1[128][320],
 * b1[128], W2[64][128], b2[64], W3[3][64], b3[3] (LT_MLP_NPARAM floats).
 * ------------------------------------------------------------------------ */
#define LT_MLP_NPARAM (128 * 320 + 128 + 64 * 128 + 64 + 3 * 64 + 3)
typedef struct lt_mlp_s* lt_mlp;

/* New model from host FP32 parameters (copied); Adam state zeroed. */
lt_status lt_mlp_create(const float* params, lt_mlp* out);
/* Copy the FP32 parameters and/or the last gradients (NULL to skip) to host
 * arrays of LT_MLP_NPARAM floats.  Synchronises. */
lt_status lt_mlp_params(lt_mlp m, float* params, float* grads, void* stream);
/* Features of n elements into X (device BF16 [n][320]): element rows[r] of
 * the solution u[(v*64 + i)*ld + e] (rows == NULL: elements 0..n-1). */
lt_status lt_mlp_features(lt_mlp m, const double* u, int64_t ld, int nvar, const int32_t* rows,
                          int64_t n, void* X, void* stream);
/* Forward + backward of the mean softmax cross-entropy on a batch of B rows
 * (X device BF16 [B][320], labels device int8 in {0,1,2} = coarsen / keep /
 * refine, other values clamped into that range); the gradients are kept in
 * the model (read with lt_mlp_params).  1 <= B <= 2^21, else LT_ERR_ARG. */
lt_status lt_mlp_grads(lt_mlp m, const void* X, const int8_t* labels, int64_t B, void* stream);
/* lt_mlp_grads, then one Adam step (beta 0.9 / 0.999, eps 1e-8) at rate lr. */
lt_status lt_mlp_train_step(lt_mlp m, const void* X, const int8_t* labels, int64_t B, float lr,
                            void* stream);
/* Logits (device FP32 [n][3]) of n feature rows. */
lt_status lt_mlp_infer(lt_mlp m, const void* X, int64_t n, float* logits, void* stream);
/* Flags of the current leaves from the solution u (device FP64, ld >= n_cur):
 * the argmax class of the network where its softmax probability is at least
 * conf_min, else the geometric flag of `fallback`; then the depth clamps.
 * conf (device FP32 [n_cur], may be NULL) receives the top probability. */
lt_status lt_flag_mlp(lt_tree t, lt_mlp m, const lt_flag_params* fallback, const double* u, int64_t ld,
                      float conf_min, int8_t* flags, float* conf, void* stream);
/* Isentropic vortex (Section 5.2; phi = 1/2, gamma = 1.4, free stream rho = 1,
 * u = 1, v = w = 0, p = 1) of z-extruded vortices with the given xy centres
 * (centre[3*v + a]) and strengths, in conserved variables at the solution
 * points of every leaf: u[(v*n_p + i)*ld + e], 5 variables in 3D (rho, rho u,
 * rho v, rho w, E), 4 in 2D (rho, rho u, rho v, E).  Points as in lt_flag.
 * A synthetic-input generator. */
lt_status lt_vortex_field(lt_tree t, const lt_flag_params* where, const double* strength, double* u,
                          int64_t ld, void* stream);
void lt_mlp_destroy(lt_mlp m);

/* Modal-energy indicator (the criterion used when no vortex centre is known,
 * and the baseline the learned indicator is measured against): the density
 * u[(0 * n_p + i) * ld + e] (variable 0, device FP64) of each leaf is projected
 * on the orthonormal tensor Legendre basis at the Gauss-Legendre points;
 * s = (energy of the modes whose highest per-axis degree is p) / (total
 * energy).  flag = +1 if log10 s > tau_refine, -1 if log10 s < tau_coarsen,
 * else 0 (0 for an all-zero density), then the d_max / d_min clamps of
 * lt_flag.  p in 1..3; tau_coarsen <= tau_refine.  flags: device int8
 * [n_cur].  Asynchronous. */
lt_status lt_flag_modal(lt_tree t, int p, const double* u, int64_t ld, double tau_refine,
                        double tau_coarsen, int8_t* flags, void* stream);

/* ------------------------------------------------------------------------
 * Captured cycles (form 2 of the cycle): the whole plain cycle -- flags of
 * Section 5.2, adaptation (Section 4.1), balance (Section 3.2), connectivity
 * (Section 3.3), mapping and FP64 transfer (Section 4.2) -- recorded once in
 * a hipGraph whose kernels keep every count on the device, then replayed with
 * one host synchronisation per cycle instead of one per size readback.
 *
 * The graph is sized for `capacity` leaves: every tree buffer is allocated for
 * it at creation, and u[0], u[1] (caller-owned device FP64 arrays, layout as
 * lt_transfer with a leading dimension ld >= capacity) hold the solution
 * alternately.  Balance runs
 * `balance_passes` one-level passes (even, >= 2) and a check pass.
 * flag_template (host, nmesh entries, nmesh = the tree's mesh count) fixes
 * each mesh's degree p of the flag points (meshes may differ), the geometry
 * and the criterion's form; each run passes the cycle's own parameters (e.g.
 * advected centres) with the same degrees.
 * The transfer may be FP64 (3D p 1..3, 2D p 1..7) or split precision
 * (64 points per element), and the flags geometric or learned (lt_flag_mlp:
 * the network over the geometric fallback below conf_min; the network's
 * weights are read at each replay, so training between runs takes effect). */
typedef struct lt_cycle_s* lt_cycle;
typedef struct {
  int p;                  /* transfer degree, or -1: each mesh's own degree          */
                          /*   (lt_set_mesh_degree; lt_transfer_mixed layout, FP64)  */
  int nvar;               /* variables; nvar * (p+1)^dim <= 65535                   */
  int64_t capacity;       /* leaves the graph's buffers hold (>= current leaves)     */
  int64_t ld;             /* leading dimension of u[0], u[1] (>= capacity)          */
  int balance_passes;     /* fixed balance passes in the graph: even, 2..64          */
  double* u[2];           /* device solution arrays [nvar][(p+1)^dim][ld]           */
  int nmesh;              /* flag parameter sets per run (the tree's mesh count)     */
  const lt_flag_params* flag_template;  /* host, nmesh entries                      */
  int precision;          /* transfer as lt_transfer: 0 FP64, 1 split (64 points)    */
  struct lt_mlp_s* mlp;   /* learned flags over the geometric fallback (lt_flag_mlp  */
  float conf_min;         /*   semantics; 3D p 3, 5 variables), or NULL             */
} lt_cycle_desc;

/* Balances the tree if it is not known to be balanced, allocates its
 * buffers for d->capacity (keeping its leaves; the pre-adapt snapshot is
 * dropped), builds the transfer operators and captures
 * two graphs (u[0] -> u[1] and u[1] -> u[0]).  Synchronises.  The tree must
 * not be used by other calls while the cycle exists, except lt_size, lt_view
 * and lt_export.  LT_ERR_ARG for an invalid descriptor. */
lt_status lt_cycle_create(lt_tree t, const lt_cycle_desc* d, void* stream, lt_cycle* out);

/* One cycle with flag parameters fp (host, nmesh entries, same p as the
 * template).  On return *u_index is the index of the array now holding the
 * solution (the other one held it before).  Synchronises once.
 * If the fixed balance passes did not reach the 2:1 fixpoint, the cycle is
 * finished by the eager calls (same result) and the graphs are recaptured
 * when buffers had to grow.  If a size passed the capacity inside the graph,
 * the tree is restored to its state before the call and LT_ERR_CAPACITY is
 * returned (create a new cycle with a larger capacity).  If finishing
 * eagerly fails (LT_ERR_CAPACITY when the balanced tree outgrew the
 * capacity: the tree then holds the new balanced leaves but u was not
 * transferred; or any error of the eager calls), the cycle drops its graphs
 * and every later lt_cycle_run returns LT_ERR_STATE without launching
 * anything; destroy it.  Other device check failures give LT_ERR_INTERNAL. */
lt_status lt_cycle_run(lt_cycle c, const lt_flag_params* fp, void* stream, int* u_index);

/* Host counters of a cycle: runs, runs whose balance was finished by the
 * eager calls, and recaptures.  Any pointer may be NULL. */
lt_status lt_cycle_stats(lt_cycle c, int64_t* runs, int64_t* eager_finishes, int64_t* recaptures);

/* Frees the graphs and the cycle's own buffers (not the tree). */
void lt_cycle_destroy(lt_cycle c);

/* Text of the calling thread's last error ("" if none). */
const char* lt_last_error(void);

/* Frees the tree and everything it owns (NULL is ignored).  Synchronises the
 * device before freeing. */
void lt_destroy(lt_tree t);

#ifdef __cplusplus
}
#endif
#endif
