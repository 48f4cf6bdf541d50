/*
 * lt_oracle.h -- CPU oracle for the linear-tree adaptation cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the GPU library.
 *
 * The oracle is a plain, slow, single-threaded implementation on a pointer
 * tree (one heap node per octant, children in Morton child order), written
 * from the paper's definitions:
 *   - Morton IDs:                Section 2.2, Algorithm "Morton Encoding"
 *   - refinement criterion:      Section 5.2 (isentropic vortex, r<5 vs r>6)
 *   - adaptation procedure:      Section 4.1, Algorithm "Adaptation procedure"
 *   - 2:1 balance:               Section 3.2 (strong 2:1, balance at depth D)
 *   - face connectivity:         Section 3.3, Algorithm "Build face connectivity"
 *   - old/new mapping:           Section 4.2, Algorithm "Mapping between old and new tree"
 *   - solution transfer:         Section 4.2, eq. parent_soln (interpolation) and
 *                                the L2 projection M u^P = sum_i S_i u^K_i
 * All floating point is FP64.  All functions return 0 on success and a
 * non-zero code on failure (message via lto_last_error()).
 */
#ifndef LT_ORACLE_H
#define LT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lto_tree_s lto_tree;

/* Create a tree over [0, 2^dmax)^dim (integer units).  keys == NULL builds
 * the uniform tree at depth d_min; otherwise keys[0..n) must be the strictly
 * ascending Morton IDs of a complete linear tree.  balance_kind: 0 face,
 * 1 edge, 2 corner.  Returns NULL on error. */
lto_tree* lto_create(int dim, int d_min, int d_max, unsigned periodic_mask,
                     int balance_kind, const uint64_t* keys, int64_t n);
/* Tree built bottom-up from n scattered points (Section 3.1, tree
 * construction and linearization; Section 5.1: a d_min background with the
 * points encoded at d_max).  pts[dim*j + a] is coordinate a of point j in the
 * physical cube [lo, lo+len)^dim; its finest cell is
 *   i_a = floor((pts[dim*j + a] - lo[a]) / dx),  dx = len / 2^d_max
 * (FP64, in that order), which must lie in [0, 2^d_max) (else NULL).  The
 * result is the coarsest complete linear tree whose leaves all have depth
 * >= d_min and in which every point's finest cell is a leaf.  Not balanced. */
lto_tree* lto_create_points(int dim, int d_min, int d_max, unsigned periodic_mask,
                            int balance_kind, const double* pts, int64_t n, const double* lo,
                            double len);
/* The same point -> finest cell conversion: anchors[dim*j + a] = i_a, or
 * non-zero with an error when a point lies outside the domain. */
int lto_point_cells(int dim, int d_max, const double* pts, int64_t n, const double* lo, double len,
                    int64_t* anchors);

/* Uniform tree at start_depth (d_min stays the coarsening floor). */
lto_tree* lto_create_uniform(int dim, int d_min, int d_max, unsigned periodic_mask,
                             int balance_kind, int start_depth);
void lto_destroy(lto_tree* t);

int64_t lto_size(const lto_tree* t);      /* current leaves            */
int64_t lto_old_size(const lto_tree* t);  /* leaves before last adapt  */
int lto_keys(const lto_tree* t, uint64_t* out);      /* DFS order           */
int lto_old_keys(const lto_tree* t, uint64_t* out);  /* snapshot, DFS order */

/* Morton ID of one octant (naive bit loop), and its inverse. */
uint64_t lto_encode(int dim, int d_max, int depth, const int64_t* anchor);
int lto_decode(int dim, int d_max, uint64_t key, int* depth, int64_t* anchor);

/* Geometric refinement flag, one per leaf (DFS order).  Vortex centres are
 * centre[3*v + a]; dist_axes in {2,3}; nodes01[k] are the solution-point
 * positions in [0,1] on one axis (p+1 of them); lo[a], len: the cubic
 * physical domain [lo, lo+len)^dim.  Clamps +1 at d_max and -1 at d_min. */
int lto_flag(const lto_tree* t, int nvort, const double* centre,
             double r_in, double r_out, int dist_axes, int periodic_dist,
             const double* nodes01, int p, const double* lo, double len,
             int8_t* flags);

/* The same criterion for n arbitrary keys (no tree needed): flags[e] is
 * what lto_flag gives the leaf keys[e] in any tree with these depth limits. */
int lto_flag_keys(int dim, int d_min, int d_max, const uint64_t* keys, int64_t n, int nvort,
                  const double* centre, double r_in, double r_out, int dist_axes,
                  int periodic_dist, const double* nodes01, int p, const double* lo, double len,
                  int8_t* flags);

/* Refine/coarsen (one level at most); snapshots the old leaves. */
int lto_adapt(lto_tree* t, const int8_t* flags);

/* Coarsest 2:1-balanced refinement.  brute != 0: all-pairs contact test. */
int lto_balance(lto_tree* t, int brute);

/* 1 if the current tree is 2:1 balanced (all-pairs contact test). */
int lto_is_balanced(const lto_tree* t);

/* Face connectivity.  nbr[2*dim*e + f]; hang rows of 2 + 2^(dim-1) int32:
 * [e, f, fine_0, ...].  *n_hang receives the row count; hang_cap rows of
 * room must be provided (pass hang == NULL to only count). */
int lto_connect(const lto_tree* t, int brute, int32_t* nbr, int32_t* hang,
                int64_t hang_cap, int64_t* n_hang);

/* Old->new mapping: map_src[j] old leaf index, map_kind[j] = 0 copy,
 * 1 + c refined child c, -1 fused (src = old index of child 0). */
int lto_map(const lto_tree* t, int32_t* map_src, int8_t* map_kind);

/* FP64 solution transfer, u[(v*n_p + i)*ld + e], n_p = (p+1)^dim. */
int lto_transfer(const lto_tree* t, int p, int nvar, const double* u_old,
                 int64_t ld_old, double* u_new, int64_t ld_new);

/* Gauss-Legendre nodes/weights on [-1,1] (p+1 points, Newton iteration). */
int lto_gauss_legendre(int npts, double* x, double* w);

/* Dense transfer operators: I[c][i][k] (child c value at point i from parent
 * coefficient k) and P[c][i][k] (parent value i from child-c value k). */
int lto_operators(int dim, int p, double* I, double* P);

const char* lto_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
