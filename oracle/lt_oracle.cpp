// lt_oracle.cpp -- plain CPU oracle of the linear-tree adaptation cycle.
//
// TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
// CPU-baseline leg of the benchmark.  The GPU library never links or calls
// it, and it shares no code with the GPU library.
//
// Representation: a pointer tree.  Every octant is a heap Node holding its
// depth and its anchor (left-front-bottom corner, Section 2.2) in integer
// units of the finest resolution 2^-dmax.  Children are stored in Morton
// child order c = sum_a b_a 2^a (a = 0 x, 1 y, 2 z).  Leaves are listed by a
// depth-first walk that visits a node before its children and children in
// index order.  Morton IDs are produced by a naive bit loop straight from
// Algorithm "Morton Encoding"; they are used only to talk to the caller.
//
// Everything is O(N) or O(N^2) loops with no cleverness: neighbours are found
// either by testing every pair of leaves (brute mode) or by descending from
// the root to the leaf that holds a point.
#include "lt_oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(const std::string& m) {
  g_err = m;
  return 1;
}

struct Node {
  int depth = 0;
  int64_t anchor[3] = {0, 0, 0};
  Node* parent = nullptr;
  Node* child[8] = {nullptr, nullptr, nullptr, nullptr,
                    nullptr, nullptr, nullptr, nullptr};
  int tag = 0;  // scratch used by one operation at a time
  bool leaf() const { return child[0] == nullptr; }
};

struct Cell {
  int depth;
  int64_t a[3];
};

int bit_length(int v) {
  int b = 0;
  while ((v >> b) != 0) b++;
  return b;
}

}  // namespace

struct lto_tree_s {
  int dim = 2, dmin = 0, dmax = 1;
  unsigned periodic = 0;
  int balance_kind = 2;
  Node* root = nullptr;
  std::vector<Node*> leaves;  // depth-first order
  std::vector<Cell> old;      // leaves before the last adapt, same order
  bool has_old = false;

  int64_t width() const { return int64_t(1) << dmax; }
  int nchild() const { return 1 << dim; }
  int64_t size_at(int depth) const { return int64_t(1) << (dmax - depth); }

  void split(Node* n) {
    const int64_t half = size_at(n->depth + 1);
    for (int c = 0; c < nchild(); ++c) {
      Node* k = new Node;
      k->depth = n->depth + 1;
      k->parent = n;
      for (int a = 0; a < dim; ++a)
        k->anchor[a] = n->anchor[a] + (((c >> a) & 1) ? half : 0);
      n->child[c] = k;
    }
  }
  static void free_subtree(Node* n) {
    if (!n) return;
    for (Node* k : n->child) free_subtree(k);
    delete n;
  }
  void merge(Node* n) {
    for (int c = 0; c < 8; ++c) {
      free_subtree(n->child[c]);
      n->child[c] = nullptr;
    }
  }
  void walk(Node* n) {
    if (n->leaf()) {
      leaves.push_back(n);
      return;
    }
    for (int c = 0; c < nchild(); ++c) walk(n->child[c]);
  }
  void relist() {
    leaves.clear();
    walk(root);
  }
  // Leaf that holds the finest-resolution cell with anchor p.
  Node* locate(const int64_t* p) const {
    Node* n = root;
    while (!n->leaf()) {
      const int64_t half = size_at(n->depth + 1);
      int c = 0;
      for (int a = 0; a < dim; ++a)
        if (p[a] >= n->anchor[a] + half) c |= 1 << a;
      n = n->child[c];
    }
    return n;
  }
  // Node at depth <= stop_depth on the path to p (a leaf or the node at stop_depth).
  Node* descend(const int64_t* p, int stop_depth) const {
    Node* n = root;
    while (!n->leaf() && n->depth < stop_depth) {
      const int64_t half = size_at(n->depth + 1);
      int c = 0;
      for (int a = 0; a < dim; ++a)
        if (p[a] >= n->anchor[a] + half) c |= 1 << a;
      n = n->child[c];
    }
    return n;
  }
  // Shift coordinate x by d along axis a; false if it leaves a non-periodic domain.
  bool shifted(int a, int64_t x, int64_t d, int64_t* out) const {
    int64_t y = x + d;
    const int64_t W = width();
    if ((periodic >> a) & 1) {
      y %= W;
      if (y < 0) y += W;
    } else if (y < 0 || y >= W) {
      return false;
    }
    *out = y;
    return true;
  }
  ~lto_tree_s() { free_subtree(root); }
};

namespace {

uint64_t encode_key(int dim, int dmax, int depth, const int64_t* anchor) {
  // Algorithm "Morton Encoding": integer coordinates at the octant's own depth,
  // bit groups x^{D-1} ... x^0 with x^k = (z^k y^k x^k) (x least significant),
  // then dim*(dmax - depth) padding zeros, then the depth in m_b bits.
  const int mb = bit_length(dmax);
  uint64_t raw = 0;
  for (int k = depth - 1; k >= 0; --k) {
    for (int a = dim - 1; a >= 0; --a) {
      const int64_t xi = anchor[a] >> (dmax - depth);
      raw = raw * 2 + uint64_t((xi >> k) & 1);
    }
  }
  uint64_t key = raw;
  for (int i = 0; i < dim * (dmax - depth); ++i) key = key * 2;
  for (int i = 0; i < mb; ++i) key = key * 2;
  return key + uint64_t(depth);
}

bool decode_key(int dim, int dmax, uint64_t key, int* depth, int64_t* anchor) {
  const int mb = bit_length(dmax);
  const int d = int(key & ((uint64_t(1) << mb) - 1));
  if (d > dmax) return false;
  uint64_t rest = key >> mb;
  for (int i = 0; i < dim * (dmax - d); ++i) {
    if (rest & 1) return false;  // padding must be zero
    rest >>= 1;
  }
  if (dim * d < 64 && (rest >> (dim * d)) != 0) return false;
  int64_t xi[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k)
    for (int a = 0; a < dim; ++a)
      if ((rest >> (dim * k + a)) & 1) xi[a] |= int64_t(1) << k;
  for (int a = 0; a < 3; ++a) anchor[a] = a < dim ? (xi[a] << (dmax - d)) : 0;
  *depth = d;
  return true;
}

uint64_t key_of(const lto_tree_s* t, const Node* n) {
  return encode_key(t->dim, t->dmax, n->depth, n->anchor);
}

// ---------------------------------------------------------------- contact
// Contact between two leaves, periodic images included.  Returns the smallest
// number of axes on which the closed boxes only touch (share an end point)
// over all images whose closed boxes intersect; 0 means they overlap, -1
// means no contact at all.
int contact_axes(const lto_tree_s* t, const Node* L, const Node* N) {
  const int64_t W = t->width();
  const int64_t sl = t->size_at(L->depth), sn = t->size_at(N->depth);
  int best = -1;
  int nimg = 1;
  for (int a = 0; a < t->dim; ++a) nimg *= 3;
  for (int img = 0; img < nimg; ++img) {
    int code = img;
    int touching = 0;
    bool ok = true;
    for (int a = 0; a < t->dim; ++a) {
      const int k = code % 3 - 1;
      code /= 3;
      if (k != 0 && !((t->periodic >> a) & 1)) {
        ok = false;
        break;
      }
      const int64_t l0 = L->anchor[a], l1 = l0 + sl;
      const int64_t n0 = N->anchor[a] + k * W, n1 = n0 + sn;
      const int64_t lo = std::max(l0, n0), hi = std::min(l1, n1);
      if (lo > hi) {
        ok = false;
        break;
      }
      if (lo == hi) touching++;
    }
    if (!ok) continue;
    if (best < 0 || touching < best) best = touching;
  }
  return best;
}

int balance_limit(const lto_tree_s* t) {
  if (t->balance_kind == 0) return 1;
  if (t->balance_kind == 1) return std::min(2, t->dim);
  return t->dim;
}

bool is_contact(const lto_tree_s* t, const Node* L, const Node* N) {
  const int k = contact_axes(t, L, N);
  return k >= 1 && k <= balance_limit(t);
}

// ---------------------------------------------------------------- quadrature
// Gauss-Legendre nodes by Newton iteration on P_n (three-term recurrence).
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (n == 0) p1 = 1.0;
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < n; ++k) {
      const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  // ascending order
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (x[j] < x[i]) {
        std::swap(x[i], x[j]);
        std::swap(w[i], w[j]);
      }
}

double lagrange(const std::vector<double>& nodes, int k, double x) {
  double v = 1.0;
  for (size_t m = 0; m < nodes.size(); ++m)
    if (int(m) != k) v *= (x - nodes[m]) / (nodes[k] - nodes[m]);
  return v;
}

// Dense operators of Section 4.2.  Tensor point index i = i0 + (p+1)(i1 + (p+1) i2).
struct Ops {
  int dim, p, np;
  std::vector<double> I;  // [c][i][k]
  std::vector<double> P;  // [c][i][k]
};

int solve_dense(int n, std::vector<double> A, std::vector<double>& B, int ncol) {
  // Gaussian elimination with partial pivoting: A (n x n) X = B (n x ncol).
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
    if (A[piv * n + col] == 0.0) return fail("singular mass matrix");
    if (piv != col) {
      for (int c = 0; c < n; ++c) std::swap(A[col * n + c], A[piv * n + c]);
      for (int c = 0; c < ncol; ++c) std::swap(B[col * ncol + c], B[piv * ncol + c]);
    }
    for (int r = col + 1; r < n; ++r) {
      const double f = A[r * n + col] / A[col * n + col];
      if (f == 0.0) continue;
      for (int c = col; c < n; ++c) A[r * n + c] -= f * A[col * n + c];
      for (int c = 0; c < ncol; ++c) B[r * ncol + c] -= f * B[col * ncol + c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    for (int c = 0; c < ncol; ++c) {
      double s = B[r * ncol + c];
      for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * B[k * ncol + c];
      B[r * ncol + c] = s / A[r * n + r];
    }
  }
  return 0;
}

int build_ops(int dim, int p, Ops* ops) {
  if (dim < 2 || dim > 3 || p < 0 || p > 7) return fail("unsupported dim/p");
  const int n1 = p + 1;
  int np = 1;
  for (int a = 0; a < dim; ++a) np *= n1;
  const int nc = 1 << dim;
  std::vector<double> z(n1), wz(n1);
  gauss_legendre(n1, z.data(), wz.data());
  ops->dim = dim;
  ops->p = p;
  ops->np = np;
  ops->I.assign(size_t(nc) * np * np, 0.0);
  ops->P.assign(size_t(nc) * np * np, 0.0);

  auto idx = [&](int i, int a) { int v = i; for (int b = 0; b < a; ++b) v /= n1; return v % n1; };
  auto basis = [&](int k, const double* xi) {
    double v = 1.0;
    for (int a = 0; a < dim; ++a) v *= lagrange(z, idx(k, a), xi[a]);
    return v;
  };

  // Interpolation: child c's point i, in parent coordinates xi = (z + 2b - 1)/2.
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < np; ++i) {
      double xi[3];
      for (int a = 0; a < dim; ++a) xi[a] = (z[idx(i, a)] + 2.0 * ((c >> a) & 1) - 1.0) / 2.0;
      for (int k = 0; k < np; ++k) ops->I[(size_t(c) * np + i) * np + k] = basis(k, xi);
    }

  // L2 projection: M u^P = sum_c S_c u^c, by separate Gauss-Legendre
  // quadrature with Q = p + 2 points per axis.
  const int Q = p + 2;
  std::vector<double> q(Q), wq(Q);
  gauss_legendre(Q, q.data(), wq.data());
  int nq = 1;
  for (int a = 0; a < dim; ++a) nq *= Q;
  auto qidx = [&](int i, int a) { int v = i; for (int b = 0; b < a; ++b) v /= Q; return v % Q; };

  std::vector<double> M(size_t(np) * np, 0.0);
  for (int qq = 0; qq < nq; ++qq) {
    double xi[3], W = 1.0;
    for (int a = 0; a < dim; ++a) {
      xi[a] = q[qidx(qq, a)];
      W *= wq[qidx(qq, a)];
    }
    std::vector<double> lv(np);
    for (int j = 0; j < np; ++j) lv[j] = basis(j, xi);
    for (int j = 0; j < np; ++j)
      for (int i = 0; i < np; ++i) M[size_t(j) * np + i] += W * lv[j] * lv[i];
  }
  for (int c = 0; c < nc; ++c) {
    std::vector<double> S(size_t(np) * np, 0.0);
    for (int qq = 0; qq < nq; ++qq) {
      double zc[3], xi[3], W = 1.0;
      for (int a = 0; a < dim; ++a) {
        zc[a] = q[qidx(qq, a)];
        xi[a] = (zc[a] + 2.0 * ((c >> a) & 1) - 1.0) / 2.0;
        W *= wq[qidx(qq, a)] / 2.0;  // child volume is 2^-dim of the parent
      }
      for (int j = 0; j < np; ++j) {
        const double lj = basis(j, xi);
        for (int i = 0; i < np; ++i) S[size_t(j) * np + i] += W * lj * basis(i, zc);
      }
    }
    if (solve_dense(np, M, S, np)) return 1;
    std::copy(S.begin(), S.end(), ops->P.begin() + size_t(c) * np * np);
  }
  return 0;
}

}  // namespace

// ====================================================================== API
extern "C" {

const char* lto_last_error(void) { return g_err.c_str(); }

uint64_t lto_encode(int dim, int d_max, int depth, const int64_t* anchor) {
  return encode_key(dim, d_max, depth, anchor);
}

int lto_decode(int dim, int d_max, uint64_t key, int* depth, int64_t* anchor) {
  return decode_key(dim, d_max, key, depth, anchor) ? 0 : fail("invalid key");
}

lto_tree* lto_create_uniform(int dim, int d_min, int d_max, unsigned periodic_mask,
                             int balance_kind, int start_depth);

lto_tree* lto_create(int dim, int d_min, int d_max, unsigned periodic_mask,
                     int balance_kind, const uint64_t* keys, int64_t n) {
  if (!keys) return lto_create_uniform(dim, d_min, d_max, periodic_mask, balance_kind, d_min);
  if (dim < 2 || dim > 3) { fail("dim must be 2 or 3"); return nullptr; }
  if (d_max < 1 || d_min < 0 || d_min > d_max) { fail("bad depth range"); return nullptr; }
  if (dim * d_max + bit_length(d_max) > 64) { fail("d_max too large for 64-bit keys"); return nullptr; }
  if (balance_kind < 0 || balance_kind > 2) { fail("bad balance kind"); return nullptr; }
  lto_tree* t = new lto_tree;
  t->dim = dim;
  t->dmin = d_min;
  t->dmax = d_max;
  t->periodic = periodic_mask & ((1u << dim) - 1);
  t->balance_kind = balance_kind;
  t->root = new Node;
  for (int64_t i = 0; i < n; ++i) {
    if (i > 0 && keys[i] <= keys[i - 1]) { fail("keys not strictly ascending"); delete t; return nullptr; }
    int d;
    int64_t a[3];
    if (!decode_key(dim, d_max, keys[i], &d, a)) { fail("invalid key"); delete t; return nullptr; }
    Node* nd = t->root;
    while (nd->depth < d) {
      if (nd->leaf()) t->split(nd);
      const int64_t half = t->size_at(nd->depth + 1);
      int c = 0;
      for (int ax = 0; ax < dim; ++ax)
        if (a[ax] >= nd->anchor[ax] + half) c |= 1 << ax;
      nd = nd->child[c];
    }
  }
  t->relist();
  if (int64_t(t->leaves.size()) != n) { fail("keys are not a complete linear tree"); delete t; return nullptr; }
  for (int64_t i = 0; i < n; ++i)
    if (key_of(t, t->leaves[i]) != keys[i]) { fail("keys are not a complete linear tree"); delete t; return nullptr; }
  return t;
}

lto_tree* lto_create_uniform(int dim, int d_min, int d_max, unsigned periodic_mask,
                             int balance_kind, int start_depth) {
  if (dim < 2 || dim > 3) { fail("dim must be 2 or 3"); return nullptr; }
  if (d_max < 1 || d_min < 0 || d_min > d_max) { fail("bad depth range"); return nullptr; }
  if (start_depth < 0 || start_depth > d_max) { fail("bad start depth"); return nullptr; }
  if (dim * d_max + bit_length(d_max) > 64) { fail("d_max too large for 64-bit keys"); return nullptr; }
  if (balance_kind < 0 || balance_kind > 2) { fail("bad balance kind"); return nullptr; }
  lto_tree* t = new lto_tree;
  t->dim = dim;
  t->dmin = d_min;
  t->dmax = d_max;
  t->periodic = periodic_mask & ((1u << dim) - 1);
  t->balance_kind = balance_kind;
  t->root = new Node;
  std::vector<Node*> front{t->root};
  for (int d = 0; d < start_depth; ++d) {
    std::vector<Node*> next;
    for (Node* nd : front) {
      t->split(nd);
      for (int c = 0; c < t->nchild(); ++c) next.push_back(nd->child[c]);
    }
    front.swap(next);
  }
  t->relist();
  return t;
}

int lto_point_cells(int dim, int d_max, const double* pts, int64_t n, const double* lo, double len,
                    int64_t* anchors) {
  if (dim < 2 || dim > 3 || d_max < 1 || d_max > 21) return fail("bad dim / d_max");
  if (!(len > 0.0)) return fail("domain length must be positive");
  const int64_t W = int64_t(1) << d_max;
  const double dx = len / double(W);
  for (int64_t j = 0; j < n; ++j)
    for (int a = 0; a < dim; ++a) {
      const double f = std::floor((pts[dim * j + a] - lo[a]) / dx);
      if (!(f >= 0.0 && f < double(W))) return fail("a point lies outside the domain");
      anchors[dim * j + a] = int64_t(f);
    }
  return 0;
}

// Section 3.1: the points' finest cells are the seeds of the tree; every
// octant that strictly contains a seed is split, and so is every octant
// shallower than d_min (the coarse background).  Splitting exactly those
// octants gives the coarsest complete tree with the seeds as leaves: each
// split is forced, and no leaf can merge with its siblings without either
// swallowing a seed or rising above d_min.
lto_tree* lto_create_points(int dim, int d_min, int d_max, unsigned periodic_mask,
                            int balance_kind, const double* pts, int64_t n, const double* lo,
                            double len) {
  if (n < 0 || (n > 0 && !pts)) { fail("bad point array"); return nullptr; }
  std::vector<int64_t> anc(size_t(n) * dim);
  if (n > 0 && lto_point_cells(dim, d_max, pts, n, lo, len, anc.data())) return nullptr;
  lto_tree* t = lto_create_uniform(dim, d_min, d_max, periodic_mask, balance_kind, d_min);
  if (!t) return nullptr;
  for (int64_t j = 0; j < n; ++j) {
    int64_t p[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) p[a] = anc[size_t(j) * dim + a];
    Node* nd = t->locate(p);  // the leaf holding the seed
    while (nd->depth < d_max) {
      t->split(nd);
      const int64_t half = t->size_at(nd->depth + 1);
      int c = 0;
      for (int a = 0; a < dim; ++a)
        if (p[a] >= nd->anchor[a] + half) c |= 1 << a;
      nd = nd->child[c];
    }
  }
  t->relist();
  return t;
}

void lto_destroy(lto_tree* t) { delete t; }

int64_t lto_size(const lto_tree* t) { return int64_t(t->leaves.size()); }
int64_t lto_old_size(const lto_tree* t) { return t->has_old ? int64_t(t->old.size()) : -1; }

int lto_keys(const lto_tree* t, uint64_t* out) {
  for (size_t i = 0; i < t->leaves.size(); ++i) out[i] = key_of(t, t->leaves[i]);
  return 0;
}

int lto_old_keys(const lto_tree* t, uint64_t* out) {
  if (!t->has_old) return fail("no adapt has run");
  for (size_t i = 0; i < t->old.size(); ++i)
    out[i] = encode_key(t->dim, t->dmax, t->old[i].depth, t->old[i].a);
  return 0;
}

// Refinement criterion of Section 5.2: count the element's solution points
// closer than r_in and farther than r_out from the vortex axis.
// The criterion of Section 5.2 for one leaf (depth, anchor): count the
// solution points inside R_in and outside R_out of the nearest vortex axis.
static int8_t leaf_flag(int dim, int dmin, int dmax, int depth, const int64_t* anchor, int nvort,
                        const double* centre, double rin2, double rout2, int dist_axes,
                        int periodic_dist, const double* nodes01, int n1, const double* lo,
                        double len) {
  const double dxmin = len / double(int64_t(1) << dmax);
  const double s = double(int64_t(1) << (dmax - depth));
  int np = 1;
  for (int a = 0; a < dim; ++a) np *= n1;
  int n_in = 0, n_out = 0;
  for (int i = 0; i < np; ++i) {
    int ia[3] = {i % n1, (i / n1) % n1, i / (n1 * n1)};
    double x[3];
    for (int a = 0; a < dim; ++a) x[a] = lo[a] + dxmin * (double(anchor[a]) + s * nodes01[ia[a]]);
    double best = 0.0;
    for (int v = 0; v < nvort; ++v) {
      double r2 = 0.0;
      for (int a = 0; a < dist_axes; ++a) {
        double d = x[a] - centre[3 * v + a];
        if (periodic_dist) d = d - len * std::floor(d / len + 0.5);
        r2 = r2 + d * d;
      }
      if (v == 0 || r2 < best) best = r2;
    }
    if (best < rin2) n_in++;
    if (best > rout2) n_out++;
  }
  int f = n_in > n_out ? 1 : (n_in < n_out ? -1 : 0);
  if (f == 1 && depth >= dmax) f = 0;
  if (f == -1 && depth <= dmin) f = 0;
  return int8_t(f);
}

int lto_flag(const lto_tree* t, int nvort, const double* centre, double r_in,
             double r_out, int dist_axes, int periodic_dist, const double* nodes01,
             int p, const double* lo, double len, int8_t* flags) {
  if (nvort < 1 || dist_axes < 1 || dist_axes > t->dim || p < 0 || p > 7)
    return fail("bad flag parameters");
  const double rin2 = r_in * r_in, rout2 = r_out * r_out;
  for (size_t e = 0; e < t->leaves.size(); ++e) {
    const Node* n = t->leaves[e];
    flags[e] = leaf_flag(t->dim, t->dmin, t->dmax, n->depth, n->anchor, nvort, centre, rin2, rout2,
                         dist_axes, periodic_dist, nodes01, p + 1, lo, len);
  }
  return 0;
}

int lto_flag_keys(int dim, int d_min, int d_max, const uint64_t* keys, int64_t n, int nvort,
                  const double* centre, double r_in, double r_out, int dist_axes,
                  int periodic_dist, const double* nodes01, int p, const double* lo, double len,
                  int8_t* flags) {
  if (dim < 2 || dim > 3 || d_min < 0 || d_min > d_max || nvort < 1 || dist_axes < 1 ||
      dist_axes > dim || p < 0 || p > 7)
    return fail("bad flag parameters");
  const double rin2 = r_in * r_in, rout2 = r_out * r_out;
  for (int64_t e = 0; e < n; ++e) {
    int d;
    int64_t a[3] = {0, 0, 0};
    if (!decode_key(dim, d_max, keys[e], &d, a)) return fail("invalid key");
    flags[e] = leaf_flag(dim, d_min, d_max, d, a, nvort, centre, rin2, rout2, dist_axes,
                         periodic_dist, nodes01, p + 1, lo, len);
  }
  return 0;
}

// Algorithm "Adaptation procedure": refine +1 leaves once; coarsen a family
// only when all of its 2^dim children are leaves flagged -1; every other -1
// is reverted to 0.  No octant changes more than once.
int lto_adapt(lto_tree* t, const int8_t* flags) {
  const size_t N = t->leaves.size();
  for (size_t i = 0; i < N; ++i)
    if (flags[i] < -1 || flags[i] > 1) return fail("flags must be -1, 0 or 1");
  t->old.clear();
  for (Node* n : t->leaves) {
    Cell c;
    c.depth = n->depth;
    for (int a = 0; a < 3; ++a) c.a[a] = n->anchor[a];
    t->old.push_back(c);
  }
  t->has_old = true;
  for (size_t i = 0; i < N; ++i) {
    Node* n = t->leaves[i];
    int f = flags[i];
    if (f == 1 && n->depth >= t->dmax) f = 0;
    if (f == -1 && n->depth <= t->dmin) f = 0;
    n->tag = f;
  }
  std::vector<Node*> parents, refine;
  for (size_t i = 0; i < N; ++i) {
    Node* n = t->leaves[i];
    if (n->tag == 1) refine.push_back(n);
    if (n->tag != -1 || !n->parent) continue;
    Node* P = n->parent;
    if (P->child[0] != n) continue;  // visit each family once
    bool all = true;
    for (int c = 0; c < t->nchild(); ++c)
      if (!P->child[c]->leaf() || P->child[c]->tag != -1) all = false;
    if (all) parents.push_back(P);
  }
  // A family that coarsens holds only -1 leaves, so no refined leaf is freed.
  for (Node* P : parents) t->merge(P);
  for (Node* n : refine) t->split(n);
  t->relist();
  for (Node* n : t->leaves) n->tag = 0;
  return 0;
}

// Coarsest 2:1-balanced refinement (Section 3.2, strong 2:1): split any leaf
// that touches a leaf two or more levels finer, until nothing changes.  Every
// split is forced (the coarse leaf touches a leaf at least two levels finer in
// any refinement), and the loop ends only when no pair violates 2:1, so the
// result is the unique coarsest balanced refinement.
//
// brute != 0: every sweep tests all pairs of leaves for contact.
// brute == 0: for each leaf L the coarser leaves touching it are exactly the
// leaves holding the 3^dim - 1 same-size boxes around L, found by descending
// from the root.  The first sweep checks all leaves; later sweeps check the
// leaves created by the previous sweep and the leaves that found a violation
// in it (one split may leave them still too fine for the new neighbour).  A
// leaf with no violation keeps none: balance never coarsens anything.
int lto_balance(lto_tree* t, int brute) {
  const int limit = balance_limit(t);
  t->relist();
  std::vector<Node*> check = t->leaves;
  for (;;) {
    std::set<Node*> marked, recheck;
    const size_t N = t->leaves.size();
    if (brute) {
      for (size_t i = 0; i < N; ++i)
        for (size_t j = 0; j < N; ++j) {
          Node* L = t->leaves[i];
          Node* M = t->leaves[j];
          if (M->depth < L->depth - 1 && is_contact(t, L, M)) marked.insert(M);
        }
    } else {
      int ndir = 1;
      for (int a = 0; a < t->dim; ++a) ndir *= 3;
      for (Node* L : check) {
        if (!L->leaf()) continue;  // split in the previous sweep; its children are listed
        const int64_t s = t->size_at(L->depth);
        for (int dcode = 0; dcode < ndir; ++dcode) {
          int code = dcode, nz = 0;
          int64_t b[3] = {0, 0, 0};
          bool inside = true;
          for (int a = 0; a < t->dim; ++a) {
            const int dlt = code % 3 - 1;
            code /= 3;
            if (dlt != 0) nz++;
            if (!t->shifted(a, L->anchor[a], dlt * s, &b[a])) inside = false;
          }
          if (nz == 0 || nz > limit || !inside) continue;
          Node* M = t->locate(b);
          if (M->depth < L->depth - 1) {
            marked.insert(M);
            recheck.insert(L);
          }
        }
      }
    }
    if (marked.empty()) break;
    check.assign(recheck.begin(), recheck.end());
    for (Node* M : marked) {
      t->split(M);
      for (int c = 0; c < t->nchild(); ++c) check.push_back(M->child[c]);
    }
    t->relist();
  }
  return 0;
}

int lto_is_balanced(const lto_tree* t) {
  const size_t N = t->leaves.size();
  for (size_t i = 0; i < N; ++i)
    for (size_t j = 0; j < N; ++j) {
      const Node* L = t->leaves[i];
      const Node* M = t->leaves[j];
      if (M->depth < L->depth - 1 && is_contact(t, L, M)) return 0;
    }
  return 1;
}

// Algorithm "Build face connectivity".  Face f = 2*axis + side (side 0 is the
// low-coordinate face).  The same-size box across the face is either inside
// one leaf of depth <= depth(e) (conforming, or e is the fine side of a
// hanging face) or split into 2^(dim-1) finer leaves (e is the coarse side).
int lto_connect(const lto_tree* t, int brute, int32_t* nbr, int32_t* hang,
                int64_t hang_cap, int64_t* n_hang) {
  const int dim = t->dim, nf = 2 * dim, nh = 1 << (dim - 1);
  std::map<const Node*, int32_t> index;
  for (size_t i = 0; i < t->leaves.size(); ++i) index[t->leaves[i]] = int32_t(i);
  int64_t rows = 0;
  const int64_t W = t->width();
  for (size_t e = 0; e < t->leaves.size(); ++e) {
    const Node* E = t->leaves[e];
    const int64_t s = t->size_at(E->depth);
    for (int f = 0; f < nf; ++f) {
      const int ax = f / 2, side = f % 2;
      int64_t b[3] = {E->anchor[0], E->anchor[1], E->anchor[2]};
      if (!t->shifted(ax, E->anchor[ax], side ? s : -s, &b[ax])) {
        nbr[nf * e + f] = -2;
        continue;
      }
      std::vector<std::pair<int, const Node*>> fine;  // (slot, leaf)
      const Node* coarse = nullptr;
      if (!brute) {
        const Node* X = t->descend(b, E->depth);
        if (X->leaf()) {
          coarse = X;
        } else {
          for (int slot = 0; slot < nh; ++slot) {
            int c = (1 - side) << ax, j = 0;
            for (int a = 0; a < dim; ++a) {
              if (a == ax) continue;
              c |= ((slot >> j) & 1) << a;
              j++;
            }
            const Node* K = X->child[c];
            if (!K->leaf()) return fail("tree is not 2:1 balanced across a face");
            fine.push_back({slot, K});
          }
        }
      } else {
        // every leaf whose face lies on the plane across face f and whose
        // tangential extent overlaps the face in a set of positive area
        const int64_t plane = side ? (E->anchor[ax] + s) % W : E->anchor[ax];
        for (const Node* M : t->leaves) {
          const int64_t sm = t->size_at(M->depth);
          const int64_t m_near = side ? M->anchor[ax] : (M->anchor[ax] + sm) % W;
          if (m_near != plane) continue;
          bool overlap = true;
          int slot = 0, j = 0;
          for (int a = 0; a < dim; ++a) {
            if (a == ax) continue;
            bool any = false;
            for (int k = -1; k <= 1; ++k) {
              if (k != 0 && !((t->periodic >> a) & 1)) continue;
              const int64_t m0 = M->anchor[a] + k * W;
              if (std::max(E->anchor[a], m0) < std::min(E->anchor[a] + s, m0 + sm)) {
                any = true;
                if (sm < s && m0 - E->anchor[a] >= sm) slot |= 1 << j;
              }
            }
            if (!any) overlap = false;
            j++;
          }
          if (!overlap) continue;
          if (M->depth <= E->depth) {
            if (coarse && coarse != M) return fail("two coarse neighbours across one face");
            coarse = M;
          } else {
            if (M->depth != E->depth + 1) return fail("tree is not 2:1 balanced across a face");
            fine.push_back({slot, M});
          }
        }
        if (coarse && !fine.empty()) return fail("mixed neighbours across one face");
        if (!coarse && int(fine.size()) != nh) return fail("incomplete fine neighbours");
        std::sort(fine.begin(), fine.end(),
                  [](const std::pair<int, const Node*>& x, const std::pair<int, const Node*>& y) {
                    return x.first < y.first;
                  });
        for (int k = 0; k < int(fine.size()); ++k)
          if (fine[k].first != k) return fail("duplicate fine slot");
      }
      if (coarse) {
        nbr[nf * e + f] = index.at(coarse);
      } else {
        nbr[nf * e + f] = -1;
        if (hang) {
          if (rows >= hang_cap) return fail("hang capacity too small");
          int32_t* row = hang + rows * (2 + nh);
          row[0] = int32_t(e);
          row[1] = f;
          for (int k = 0; k < nh; ++k) row[2 + k] = index.at(fine[k].second);
        }
        rows++;
      }
    }
  }
  *n_hang = rows;
  return 0;
}

// Algorithm "Mapping between old and new tree", done by looking octants up
// by (depth, anchor): each new leaf is an old leaf, a child of one, or the
// parent of 2^dim old leaves.
int lto_map(const lto_tree* t, int32_t* map_src, int8_t* map_kind) {
  if (!t->has_old) return fail("no adapt has run");
  std::map<std::tuple<int, int64_t, int64_t, int64_t>, int32_t> old;
  for (size_t i = 0; i < t->old.size(); ++i) {
    const Cell& c = t->old[i];
    old[std::make_tuple(c.depth, c.a[0], c.a[1], c.a[2])] = int32_t(i);
  }
  for (size_t j = 0; j < t->leaves.size(); ++j) {
    const Node* n = t->leaves[j];
    const int d = n->depth;
    auto it = old.find(std::make_tuple(d, n->anchor[0], n->anchor[1], n->anchor[2]));
    if (it != old.end()) {
      map_src[j] = it->second;
      map_kind[j] = 0;
      continue;
    }
    if (d > 0) {
      const int64_t ps = t->size_at(d - 1);
      int64_t pa[3] = {0, 0, 0};
      int c = 0;
      for (int a = 0; a < t->dim; ++a) {
        pa[a] = n->anchor[a] - n->anchor[a] % ps;
        if (n->anchor[a] != pa[a]) c |= 1 << a;
      }
      it = old.find(std::make_tuple(d - 1, pa[0], pa[1], pa[2]));
      if (it != old.end()) {
        map_src[j] = it->second;
        map_kind[j] = int8_t(1 + c);
        continue;
      }
    }
    if (d < t->dmax) {
      const int64_t hs = t->size_at(d + 1);
      int32_t first = -1;
      bool all = true;
      for (int c = 0; c < t->nchild(); ++c) {
        int64_t ca[3] = {n->anchor[0], n->anchor[1], n->anchor[2]};
        for (int a = 0; a < t->dim; ++a)
          if ((c >> a) & 1) ca[a] += hs;
        auto jt = old.find(std::make_tuple(d + 1, ca[0], ca[1], ca[2]));
        if (jt == old.end()) {
          all = false;
          break;
        }
        if (c == 0) first = jt->second;
      }
      if (all) {
        map_src[j] = first;
        map_kind[j] = -1;
        continue;
      }
    }
    return fail("new leaf is neither copy, refined child nor fused parent");
  }
  return 0;
}

// Solution transfer of Section 4.2: copy, interpolation (eq. parent_soln)
// evaluated densely, and L2 projection with dense M^{-1} S_c.
int lto_transfer(const lto_tree* t, int p, int nvar, const double* u_old,
                 int64_t ld_old, double* u_new, int64_t ld_new) {
  if (!t->has_old) return fail("no adapt has run");
  if (nvar < 1) return fail("nvar must be positive");
  if (ld_old < int64_t(t->old.size()) || ld_new < int64_t(t->leaves.size()))
    return fail("leading dimension too small");
  Ops ops;
  if (build_ops(t->dim, p, &ops)) return 1;
  const int np = ops.np, nc = t->nchild();
  std::vector<int32_t> src(t->leaves.size());
  std::vector<int8_t> kind(t->leaves.size());
  if (lto_map(t, src.data(), kind.data())) return 1;
  std::map<std::tuple<int, int64_t, int64_t, int64_t>, int32_t> old;
  for (size_t i = 0; i < t->old.size(); ++i) {
    const Cell& c = t->old[i];
    old[std::make_tuple(c.depth, c.a[0], c.a[1], c.a[2])] = int32_t(i);
  }
  for (size_t j = 0; j < t->leaves.size(); ++j) {
    const Node* n = t->leaves[j];
    for (int v = 0; v < nvar; ++v) {
      for (int i = 0; i < np; ++i) {
        double acc = 0.0;
        if (kind[j] == 0) {
          acc = u_old[(int64_t(v) * np + i) * ld_old + src[j]];
        } else if (kind[j] > 0) {
          const int c = kind[j] - 1;
          for (int k = 0; k < np; ++k)
            acc += ops.I[(size_t(c) * np + i) * np + k] * u_old[(int64_t(v) * np + k) * ld_old + src[j]];
        } else {
          const int64_t hs = t->size_at(n->depth + 1);
          for (int c = 0; c < nc; ++c) {
            int64_t ca[3] = {n->anchor[0], n->anchor[1], n->anchor[2]};
            for (int a = 0; a < t->dim; ++a)
              if ((c >> a) & 1) ca[a] += hs;
            const int32_t oc = old.at(std::make_tuple(n->depth + 1, ca[0], ca[1], ca[2]));
            for (int k = 0; k < np; ++k)
              acc += ops.P[(size_t(c) * np + i) * np + k] * u_old[(int64_t(v) * np + k) * ld_old + oc];
          }
        }
        u_new[(int64_t(v) * np + i) * ld_new + j] = acc;
      }
    }
  }
  return 0;
}

int lto_gauss_legendre(int npts, double* x, double* w) {
  if (npts < 1 || npts > 16) return fail("bad point count");
  gauss_legendre(npts, x, w);
  return 0;
}

int lto_operators(int dim, int p, double* I, double* P) {
  Ops ops;
  if (build_ops(dim, p, &ops)) return 1;
  std::copy(ops.I.begin(), ops.I.end(), I);
  std::copy(ops.P.begin(), ops.P.end(), P);
  return 0;
}

}  // extern "C"
