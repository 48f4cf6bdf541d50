// tree.hpp -- internal state of one linear tree and the host helpers shared
// by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lt.h"
#include "keys.hpp"
#include "scan.hpp"

namespace lt {

// Small device-side counters, read back in one copy.
struct DevCtr {
  unsigned err;
  unsigned conv;  // captured cycles: the balance fixpoint was reached this cycle
  int64_t total;
  unsigned long long nmarked;
  unsigned long long ticket;
  int64_t nfused;             // fused parents listed for the first balance pass
  int64_t nfgroups;           // transfer groups holding a fused element (second list)
  int64_t nexam;              // balance: leaves listed for the next marking pass
};

void set_error(const std::string& msg);
lt_status fail(lt_status s, const std::string& msg);

#define LT_TRY_STATUS(expr)         \
  do {                              \
    lt_status s_ = (expr);          \
    if (s_ != LT_OK) return s_;     \
  } while (0)

// Flag kernel launcher (its own translation unit: no FP contraction there).
lt_status launch_flag(const KeyGeom& g, const lt_flag_params* fp, const uint64_t* keys, int64_t n,
                      int8_t* flags, hipStream_t stream);

// Ensemble flags: per-mesh parameters copied to dev_table (flag_args_size()
// bytes per mesh), then one launch over all leaves.
size_t flag_args_size();
lt_status launch_flag_batch(const KeyGeom& g, const lt_flag_params* fps, int nmesh, void* dev_table,
                            const uint64_t* keys, int64_t n, int8_t* flags, hipStream_t stream);

// Validated per-mesh flag parameters written to host_table (flag_args_size()
// bytes per mesh), and flags from a device copy of such a table over a count
// that may live on the device (captured cycles).
lt_status fill_flag_table(const KeyGeom& g, const lt_flag_params* fps, int nmesh, void* host_table);
lt_status launch_flag_table(const KeyGeom& g, const lt_flag_params* fps, int nmesh, const void* dev_table,
                            const uint64_t* keys, Count n, int8_t* flags, hipStream_t stream);

// One whole cycle recorded on a stream with every count kept on the device
// (for capture in a graph): flags from the device table, adapt kbuf[0] ->
// kbuf[1], `passes` (even) balance passes between kbuf[1] and kbuf[2] and a
// check pass, connect, map, transfer uo -> un, then the new keys copied back
// to kbuf[0] (skipped when an error bit is set).  dsz[0] = leaves,
// dsz[1] = leaves before the cycle, dsz[2] = hanging rows, dsz[3] = groups of
// 64 leaves, dsz[4] = a balance pass's input count.  Every buffer must already hold `cap` leaves (no allocation).
struct CycleRec {
  int64_t cap;        // leaves
  int64_t hang_rows;  // rows of the hanging-face table
  int passes;
  int p, nvar;
  const double* uo;
  double* un;
  int64_t ld;          // leading dimension of uo and un
  lt_flag_params fp0;  // degree and geometry of the flags (the centres come from the table)
  const lt_flag_params* tmpl;  // every mesh's template (only the degrees are read here)
  int nmesh;
  int64_t* dsz;
  const double* ops;
  int precision;       // transfer: 0 FP64, 1 split
  lt_mlp mlp;          // learned flags (null: geometric only)
  float conf_min;
  int dir_shift;
  int64_t dir_nb;
  // connectivity runs on `side` between the events, beside the mapping and
  // the transfer on the main stream
  hipStream_t side;
  hipEvent_t fork, join;
};
lt_status record_cycle(lt_tree_s* t, const CycleRec& r, hipStream_t s);

// Builds (once per degree) the FP64 1D transfer operators into ops.
struct Alloc;
lt_status build_transfer_ops(const Alloc& A, int p, double** ops, hipStream_t stream);

// Device allocator of a tree (with its cycles) or a model: the one registered
// with lt_set_allocator when the object was created, or hipMalloc / hipFree
// when none was.  Every device buffer an object owns goes through it.
struct Alloc {
  void* (*alloc)(size_t bytes, void* stream, void* ctx) = nullptr;
  void (*free_)(void* ptr, void* stream, void* ctx) = nullptr;
  void* ctx = nullptr;
};
// The allocator registered now (copied into each new object), and its
// replacement (lt_set_allocator).
Alloc registered_alloc();
void register_alloc(const Alloc& A);
// hipMalloc semantics: hipSuccess and *p set, or an error and *p = NULL.
hipError_t dev_malloc(const Alloc& A, void** p, size_t bytes);
// Frees p (NULL is ignored).  The device is synchronised first, as hipFree
// does, so no kernel still in flight can touch the memory a caching
// allocator hands out again.
hipError_t dev_free(const Alloc& A, void* p);

// Grow a device buffer to hold `need` elements (contents are not kept).
template <class T>
inline lt_status grow(const Alloc& A, T** p, int64_t* cap, int64_t need) {
  if (need <= *cap && *p) return LT_OK;
  int64_t ncap = std::max<int64_t>(need + need / 4, 1024);
  if (*p) {
    hipError_t e = dev_free(A, *p);
    *p = nullptr;
    *cap = 0;
    if (e != hipSuccess) return fail(LT_ERR_HIP, std::string("device free: ") + hipGetErrorString(e));
  }
  void* q = nullptr;
  hipError_t e = dev_malloc(A, &q, size_t(ncap) * sizeof(T));
  if (e != hipSuccess || !q)
    return fail(LT_ERR_OOM, "device allocation of " + std::to_string(size_t(ncap) * sizeof(T)) +
                                " bytes failed");
  *p = static_cast<T*>(q);
  *cap = ncap;
  return LT_OK;
}


}  // namespace lt

struct lt_tree_s;

namespace lt {

// Zero the look-back words for n_items of scan work in tiles of `tile`
// items (kTileMax or kTileMin, matching the kernel's workgroup) and the
// counters; fills st for a scan kernel on `stream`.  flags: 1 = also clear
// the error word, 2 = record the balance fixpoint (no marks since the last
// clear; captured cycles), 4 = also clear the lists, 8 = clear the fixpoint
// flag (a captured cycle's start).  cnt_dst / cnt_src (captured cycles): the
// same launch copies one device count to another word.
lt_status prep_scan(lt_tree_s* t, int64_t n_items, int64_t tile, hipStream_t stream, int flags,
                    ScanState* st, int64_t* cnt_dst = nullptr, const int64_t* cnt_src = nullptr);
// The same over caller-provided look-back words (status_cap of them) and
// counters, allocating nothing (LT_ERR_ARG when the words do not suffice).
lt_status prep_scan_fixed(uint64_t* status, int64_t status_cap, DevCtr* ctr, int64_t n_items,
                          int64_t tile, hipStream_t stream, int flags, ScanState* st,
                          int64_t* cnt_dst = nullptr, const int64_t* cnt_src = nullptr);
// The same on connectivity's own look-back words and counters, so that
// lt_connect may run beside lt_map and lt_transfer on another stream.
lt_status prep_scan_conn(lt_tree_s* t, int64_t n_items, hipStream_t stream, int flags,
                         ScanState* st);
// A new tree with no leaves yet (geometry checked, counters allocated).
lt_status create_tree(const lt_geom* geom, lt_tree_s** out);
// Copy the device counters to the pinned mirror and wait for the stream.
lt_status read_ctr(lt_tree_s* t, hipStream_t stream);
// Zero the counters and the error word.
lt_status clear_err(lt_tree_s* t, hipStream_t stream);
// Key-directory size for n leaves: 2^L buckets of 2^shift key values.
void dir_params(const KeyGeom& g, int64_t n, int* shift, int64_t* nb);

// Split-precision (BF16 x 3 on MFMA, FP64 cell means) transfer; asynchronous.
lt_status launch_split_transfer(lt_tree_s* t, int p, int nvar, const double* u_old, int64_t ld_old,
                                double* u_new, int64_t ld_new, hipStream_t s);
lt_status launch_split_transfer(lt_tree_s* t, Count n, int p, int nvar, const double* u_old,
                                int64_t ld_old, double* u_new, int64_t ld_new, hipStream_t s);
// One-time split operator build (before capture).
lt_status prepare_split(lt_tree_s* t, int p, hipStream_t s);

// Learned flags over a count that may live on the device: features of u
// (5 variables x 64 points), the fused network and the decision over the
// geometric flags already in `flags`.  mlp_reserve sizes the feature buffer.
lt_status mlp_reserve(lt_mlp m, int64_t n);
lt_status launch_mlp_flag(lt_tree_s* t, lt_mlp m, Count n, const double* u, int64_t ld, float conf_min,
                          int8_t* flags, float* conf, hipStream_t s);

lt_status launch_transfer(lt_tree_s* t, int p, const double* ops, int nvar, const double* u_old,
                          int64_t ld_old, double* u_new, int64_t ld_new, hipStream_t s);
// FP64 transfer of an ensemble with per-mesh degrees (lt_set_mesh_degree), over
// a count that may live on the device; asynchronous.  keys: the new leaves'
// keys (each element's mesh, hence its degree, comes from its key), which a
// captured cycle holds in another buffer than the tree's current one.
// The tree's second stream for the interpolation passes of a 3D transfer and
// its fork/join events, made on first use (default priority, non-blocking).
lt_status transfer_side(lt_tree_s* t, hipStream_t* side, hipEvent_t* fork, hipEvent_t* join);
lt_status launch_transfer_mixed(lt_tree_s* t, const uint64_t* keys, Count n, const int64_t* ngroups_dev,
                                int nvar, const double* uo, int64_t ldo, double* un, int64_t ldn,
                                hipStream_t s);

// COPY elements of the current mapping, all `rows` point rows (nvar * n_p);
// asynchronous.
lt_status launch_copy(lt_tree_s* t, int64_t rows, const double* uo, int64_t ldo, double* un,
                      int64_t ldn, hipStream_t s);
lt_status launch_copy(lt_tree_s* t, Count n, int64_t rows, const double* uo, int64_t ldo,
                      double* un, int64_t ldn, hipStream_t s);

// Transfer over n new leaves given as a Count (a device count with the
// launch sized for its capacity n.n); ngroups_dev, when set, holds
// ceil(count / 64) on the device.  Asynchronous; no host synchronisation.
lt_status launch_transfer(lt_tree_s* t, Count n, const int64_t* ngroups_dev, int p,
                          const double* ops, int nvar, const double* u_old, int64_t ld_old,
                          double* u_new, int64_t ld_new, hipStream_t s);

}  // namespace lt

// Tuning parameters of the transfer (results never depend on them).
struct TransferTune {
  int copy_epl = 2;        // copy pass: elements per lane (1, 2, 4); chunk = 256 * copy_epl
  int interp_grid = 2048;  // persistent interpolation workgroups per variable
};

struct lt_tree_s {
  lt::KeyGeom g{};
  lt::Alloc A;  // device allocator of every buffer below (and of the tree's cycles)
  TransferTune tune;
  int device = 0;
  // Four key buffers in four roles: the current leaves, the leaves before the
  // last adapt (the old tree of lt_map / lt_transfer), and two free ones that
  // adapt and balance write into.  A call swaps roles only once it has
  // succeeded, so on any error the current and old leaves are as before.
  uint64_t* kbuf[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t kcap[4] = {0, 0, 0, 0};
  int cur = 0, tmp = 1, old = 2, aux = 3;  // roles of the four key buffers
  int64_t n_cur = 0, n_old = -1, n_hang = -1;
  bool has_old = false;
  bool balanced = false;     // the current leaves are known to be 2:1 balanced
  bool adapt_marks = false;  // mbuf[0] holds adapt's marks for the first balance pass
  int conn_grid = 0;         // cap on the face search's workgroups (0: one lane per face)

  uint32_t* mbuf[2] = {nullptr, nullptr};  // balance marks, ping-pong
  int64_t mcap[2] = {0, 0};

  int32_t* dir = nullptr;       // radix directory of the current keys
  int64_t dir_cap = 0;
  int dir_shift = 0;
  int64_t dir_nb = 0;
  bool dir_valid = false;

  int32_t* nbr = nullptr;
  int64_t nbr_cap = 0;
  uint8_t* hmask = nullptr;     // per leaf: faces that are the coarse side of a hanging face
  int64_t hmask_cap = 0;
  int32_t* fused = nullptr;     // fused parents of the last adaptation (first balance pass)
  int64_t fused_cap = 0;
  int32_t* hang = nullptr;
  int64_t hang_cap = 0;  // rows
  bool conn_valid = false;

  int32_t* map_src = nullptr;
  int8_t* map_kind = nullptr;
  int64_t map_cap = 0;
  int64_t kind_cap = 0;
  bool map_valid = false;

  int8_t* lim = nullptr;        // ensemble: per-mesh {floor, ceiling}
  void* flag_tab = nullptr;     // ensemble: per-mesh flag parameters
  int64_t* mesh_offs = nullptr; // ensemble: first leaf of each mesh (nmesh + 1)

  uint64_t* status = nullptr;  // look-back tile words
  int64_t status_cap = 0;
  lt::DevCtr* dctr = nullptr;
  lt::DevCtr* hctr = nullptr;  // pinned mirror
  int32_t* elist = nullptr;     // balance: leaves to examine in the next marking pass
  int64_t elist_cap = 0;
  uint64_t* cstatus = nullptr;  // connectivity's own look-back words and counters
  int64_t cstatus_cap = 0;
  lt::DevCtr* cctr = nullptr;
  lt::DevCtr* hcctr = nullptr;  // pinned mirror

  double* ops[LT_MAX_DEGREE + 1] = {};  // 1D factors A_0, A_1, P_0, P_1 and weights

  void* split_frags = nullptr;  // BF16 x 3 operator fragments (64-point elements)
  double* split_vec = nullptr;  // FP64 mean weights
  int32_t* split_R = nullptr;   // first child of each refined family
  int64_t split_R_cap = 0;
  int32_t* split_F = nullptr;   // fused parents
  int64_t split_F_cap = 0;
  double* fr_tab[LT_MAX_DEGREE + 1] = {};  // flux reconstruction: 1D tables per degree
  double* fr_fb = nullptr;                  // flux reconstruction: face traces / common fluxes
  int64_t fr_fb_cap = 0;
  uint8_t* mesh_np = nullptr;   // ensemble with per-mesh degrees: points per element of each mesh
  int mesh_npm = 0;             //   the largest of them (the solution layout's point stride)
  unsigned mesh_degs = 0;       //   bit p set: some mesh has degree p
  int32_t* chunk_np = nullptr;  // mixed-degree copy pass: largest point count per chunk
  int64_t chunk_np_cap = 0;
  int32_t* grp_list = nullptr;  // 64-element groups holding refined/fused elements
  int64_t grp_cap = 0;
  int64_t* copy_delta = nullptr;  // per copy chunk: source offset of a pure run, or a flag
  int64_t copy_delta_cap = 0;
  hipStream_t xs = nullptr;       // transfer: second stream of the interpolation passes
  hipEvent_t xev[2] = {};         //   its fork and join events
};
