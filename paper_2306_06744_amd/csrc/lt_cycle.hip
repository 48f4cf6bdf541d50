// lt_cycle.hip -- the whole plain cycle captured in a hipGraph (form 2).
//
// record_cycle (lt_tree.hip) enqueues every step with the leaf counts kept on
// the device and every launch sized for a fixed capacity, so the sequence
// needs no host readback and can be captured once.  A run uploads the cycle's
// flag parameters, replays the graph for the current solution parity and
// reads the sizes and the error word back in one synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tree.hpp"

using namespace lt;

struct lt_cycle_s {
  lt_tree t = nullptr;
  lt_cycle_desc d{};
  int nmesh = 1;
  std::vector<lt_flag_params> tmpl;
  std::vector<double> tmpl_nodes;  // the template's point table (fp0 keeps a pointer to it)
  std::vector<double> tmpl_centres;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int parity = 0;                  // u[parity] holds the solution
  int64_t* dsz = nullptr;          // device: leaves, leaves before, hanging rows, groups, a balance pass's input
  int64_t* hsz = nullptr;          // pinned mirror
  void* flag_host = nullptr;       // pinned flag-parameter table
  int64_t hang_rows = 0;
  int64_t runs = 0, eager_finishes = 0, recaptures = 0;
  int dir_shift = 0;
  int64_t dir_nb = 0;
  // Set when finishing a cycle eagerly failed: the graphs were dropped (the
  // eager calls may have moved buffers the graphs point at) and every later
  // run returns LT_ERR_STATE without launching anything.
  bool dead = false;
};

namespace {

// Grow a key buffer to `need` keeping its first `keep` keys.
lt_status grow_keys(lt_tree t, int i, int64_t need, int64_t keep, hipStream_t s) {
  if (t->kcap[i] >= need && t->kbuf[i]) return LT_OK;
  void* q = nullptr;
  const int64_t cap = need + need / 4;
  if (dev_malloc(t->A, &q, size_t(cap) * 8) != hipSuccess) return fail(LT_ERR_OOM, "key buffer for the cycle");
  if (keep > 0 && hipMemcpyAsync(q, t->kbuf[i], size_t(keep) * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
    (void)dev_free(t->A, q);
    return fail(LT_ERR_HIP, "key copy");
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LT_ERR_HIP, "sync");
  (void)dev_free(t->A, t->kbuf[i]);
  t->kbuf[i] = static_cast<uint64_t*>(q);
  t->kcap[i] = cap;
  return LT_OK;
}

// Every buffer the recorded cycle touches, sized for the capacity.
lt_status reserve(lt_cycle c, hipStream_t s) {
  lt_tree t = c->t;
  const int64_t C = c->d.capacity;
  const int dim = t->g.dim;
  // current keys into kbuf[0]
  LT_TRY_STATUS(grow_keys(t, t->cur, C, t->n_cur, s));
  if (t->cur != 0) {
    LT_TRY_STATUS(grow_keys(t, 0, C, 0, s));
    if (hipMemcpyAsync(t->kbuf[0], t->kbuf[t->cur], size_t(t->n_cur) * 8, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return fail(LT_ERR_HIP, "key copy");
  }
  t->cur = 0;
  t->tmp = 1;
  t->old = 2;
  t->aux = 3;
  t->has_old = false;
  t->n_old = -1;
  t->map_valid = false;
  t->conn_valid = false;
  t->dir_valid = false;
  t->n_hang = -1;
  LT_TRY_STATUS(grow_keys(t, 1, C, 0, s));
  LT_TRY_STATUS(grow_keys(t, 2, C, 0, s));
  LT_TRY_STATUS(grow(t->A, &t->mbuf[0], &t->mcap[0], C));
  LT_TRY_STATUS(grow(t->A, &t->mbuf[1], &t->mcap[1], C));
  LT_TRY_STATUS(grow(t->A, &t->nbr, &t->nbr_cap, C * 2 * dim));
  LT_TRY_STATUS(grow(t->A, &t->hmask, &t->hmask_cap, C + kItems));
  LT_TRY_STATUS(grow(t->A, &t->fused, &t->fused_cap, C));
  LT_TRY_STATUS(grow(t->A, &t->elist, &t->elist_cap, C));
  c->hang_rows = std::max<int64_t>(1024, C / 16);
  LT_TRY_STATUS(grow(t->A, &t->hang, &t->hang_cap, c->hang_rows * (2 + (1 << (dim - 1)))));
  c->hang_rows = t->hang_cap / (2 + (1 << (dim - 1)));
  LT_TRY_STATUS(grow(t->A, &t->map_src, &t->map_cap, C));
  LT_TRY_STATUS(grow(t->A, &t->map_kind, &t->kind_cap, C));
  LT_TRY_STATUS(grow(t->A, &t->copy_delta, &t->copy_delta_cap, C / 256 + 2));  // chunks at the finest tuning
  LT_TRY_STATUS(grow(t->A, &t->grp_list, &t->grp_cap, 2 * (C / 64 + 2)));
  LT_TRY_STATUS(grow(t->A, &t->status, &t->status_cap, std::max<int64_t>(1, (C + kTileMin - 1) / kTileMin)));
  LT_TRY_STATUS(grow(t->A, &t->cstatus, &t->cstatus_cap, std::max<int64_t>(1, (C + kTileMin - 1) / kTileMin)));
  dir_params(t->g, C, &c->dir_shift, &c->dir_nb);
  LT_TRY_STATUS(grow(t->A, &t->dir, &t->dir_cap, c->dir_nb + 1));
  if (!t->flag_tab) {
    if (dev_malloc(t->A, &t->flag_tab, flag_args_size() * size_t(c->nmesh)) != hipSuccess)
      return fail(LT_ERR_OOM, "flag table");
  }
  if (c->d.p > 0) {
    LT_TRY_STATUS(build_transfer_ops(t->A, c->d.p, &t->ops[c->d.p], s));
  } else {  // per-mesh degrees: every degree's operators, the chunk table and room for the entries
    for (int p = 1; p <= 3; ++p)
      if (t->mesh_degs & (1u << p)) LT_TRY_STATUS(build_transfer_ops(t->A, p, &t->ops[p], s));
    LT_TRY_STATUS(grow(t->A, &t->chunk_np, &t->chunk_np_cap, C / 256 + 2));
    LT_TRY_STATUS(grow(t->A, &t->grp_list, &t->grp_cap, 6 * (C / 64 + 2)));
  }
  if (c->d.precision == 1) {
    LT_TRY_STATUS(prepare_split(t, c->d.p, s));
    LT_TRY_STATUS(grow(t->A, &t->split_R, &t->split_R_cap, C));
    LT_TRY_STATUS(grow(t->A, &t->split_F, &t->split_F_cap, C));
  }
  if (c->d.mlp) LT_TRY_STATUS(mlp_reserve(c->d.mlp, C));
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LT_ERR_HIP, "sync");
  return LT_OK;
}

void drop_graphs(lt_cycle c) {
  for (int q = 0; q < 2; ++q) {
    if (c->exec[q]) (void)hipGraphExecDestroy(c->exec[q]);
    if (c->graph[q]) (void)hipGraphDestroy(c->graph[q]);
    c->exec[q] = nullptr;
    c->graph[q] = nullptr;
  }
}

lt_status capture(lt_cycle c) {
  drop_graphs(c);
  lt_tree t = c->t;
  hipStream_t cs = nullptr, side = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return fail(LT_ERR_HIP, "capture stream");
  lt_status st = LT_OK;
  if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess)
    st = fail(LT_ERR_HIP, "capture side stream");
  if (st == LT_OK) {  // the transfer's own second stream, made outside the capture
    hipStream_t xs;
    hipEvent_t xf, xj;
    st = transfer_side(t, &xs, &xf, &xj);
  }
  for (int q = 0; q < 2 && st == LT_OK; ++q) {
    CycleRec r{};
    r.cap = c->d.capacity;
    r.hang_rows = c->hang_rows;
    r.passes = c->d.balance_passes;
    r.p = c->d.p;
    r.nvar = c->d.nvar;
    r.uo = c->d.u[q];
    r.un = c->d.u[1 - q];
    r.ld = c->d.ld;
    r.fp0 = c->tmpl[0];
    r.tmpl = c->tmpl.data();
    r.nmesh = c->nmesh;
    r.dsz = c->dsz;
    r.ops = c->d.p > 0 ? t->ops[c->d.p] : nullptr;
    r.precision = c->d.precision;
    r.mlp = c->d.mlp;
    r.conf_min = c->d.conf_min;
    r.dir_shift = c->dir_shift;
    r.dir_nb = c->dir_nb;
    r.side = side;
    r.fork = ev[0];
    r.join = ev[1];
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = fail(LT_ERR_HIP, "begin capture");
      break;
    }
    st = record_cycle(t, r, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (st == LT_OK && (e != hipSuccess || !g)) st = fail(LT_ERR_HIP, "end capture");
    if (st != LT_OK) {
      if (g) (void)hipGraphDestroy(g);
      break;
    }
    c->graph[q] = g;
    if (hipGraphInstantiate(&c->exec[q], g, nullptr, nullptr, 0) != hipSuccess)
      st = fail(LT_ERR_HIP, "graph instantiate");
  }
  (void)hipStreamDestroy(cs);
  if (side) (void)hipStreamDestroy(side);
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st != LT_OK) drop_graphs(c);
  return st;
}

lt_status upload_count(lt_cycle c, hipStream_t s) {
  c->hsz[0] = c->t->n_cur;
  if (hipMemcpyAsync(c->dsz, c->hsz, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LT_ERR_HIP, "count upload");
  return LT_OK;
}

// Finishes a cycle whose fixed balance passes stopped short of the fixpoint
// with the eager calls (same result), then recaptures the graphs when
// buffers moved.  On error the caller drops the graphs.
lt_status finish_eagerly(lt_cycle c, int q, void* stream, int* u_index) {
  lt_tree t = c->t;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto buffers = [t]() {
    return std::vector<const void*>{t->kbuf[0], t->kbuf[1], t->kbuf[2], t->mbuf[0], t->mbuf[1],
                                    t->nbr, t->hmask, t->hang, t->map_src, t->map_kind, t->dir,
                                    t->status, t->cstatus, t->elist, t->copy_delta, t->grp_list,
                                    t->fused, t->split_R, t->split_F, t->chunk_np};
  };
  const std::vector<const void*> before = buffers();
  t->old = 0;
  t->cur = 1;
  t->tmp = 2;
  t->aux = 3;
  t->n_old = c->hsz[1];
  t->n_cur = c->hsz[0];
  t->has_old = true;
  t->dir_valid = t->conn_valid = t->map_valid = false;
  t->n_hang = -1;
  LT_TRY_STATUS(lt_balance(t, stream));
  if (t->n_cur > c->d.capacity)
    return fail(LT_ERR_CAPACITY,
                "the cycle outgrew its capacity while finishing eagerly; u not transferred");
  LT_TRY_STATUS(lt_connect(t, stream));
  LT_TRY_STATUS(lt_map(t, stream));
  if (c->d.p > 0)
    LT_TRY_STATUS(lt_transfer(t, c->d.p, c->d.nvar, c->d.u[q], c->d.ld, c->d.u[1 - q], c->d.ld,
                              c->d.precision, stream));
  else
    LT_TRY_STATUS(lt_transfer_mixed(t, c->d.nvar, c->d.u[q], c->d.ld, c->d.u[1 - q], c->d.ld, stream));
  if (t->cur != 0) {
    if (hipMemcpyAsync(t->kbuf[0], t->kbuf[t->cur], size_t(t->n_cur) * 8, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return fail(LT_ERR_HIP, "key copy");
    t->cur = 0;
    t->tmp = 1;
    t->old = 2;
    t->aux = 3;
  }
  t->has_old = false;
  t->dir_valid = false;
  c->parity = 1 - q;
  if (u_index) *u_index = c->parity;
  LT_TRY_STATUS(upload_count(c, s));
  if (buffers() != before) {
    // buffers moved: size everything for the capacity again and recapture
    c->recaptures++;
    LT_TRY_STATUS(reserve(c, s));
    LT_TRY_STATUS(upload_count(c, s));
    LT_TRY_STATUS(capture(c));
  }
  return LT_OK;
}

}  // namespace

extern "C" {

lt_status lt_cycle_create(lt_tree t, const lt_cycle_desc* d, void* stream, lt_cycle* out) {
  if (!t || !d || !out || !d->flag_template || !d->u[0] || !d->u[1])
    return fail(LT_ERR_ARG, "NULL argument");
  const int dim = t->g.dim;
  if (d->nmesh != t->g.nmesh) return fail(LT_ERR_ARG, "nmesh must equal the tree's mesh count");
  if (d->balance_passes < 2 || d->balance_passes > 64 || (d->balance_passes & 1))
    return fail(LT_ERR_ARG, "balance_passes must be even, 2..64");
  const bool mixed = d->p == -1;
  if (mixed && (!t->mesh_np || d->precision != 0 || d->mlp))
    return fail(LT_ERR_ARG, "p = -1 needs lt_set_mesh_degree, precision 0 and no learned flags");
  if (!mixed && ((dim == 3 && (d->p < 1 || d->p > 3)) || (dim == 2 && (d->p < 1 || d->p > LT_MAX_DEGREE))))
    return fail(LT_ERR_ARG, "transfer degree out of range");
  int64_t npts = 1;
  if (mixed)
    npts = t->mesh_npm;
  else
    for (int a = 0; a < dim; ++a) npts *= d->p + 1;
  if (d->nvar < 1 || int64_t(d->nvar) * npts > 65535) return fail(LT_ERR_ARG, "nvar out of range");
  if (d->capacity < std::max<int64_t>(t->n_cur, 1) || d->capacity > (int64_t(1) << 31) - 1)
    return fail(LT_ERR_ARG, "capacity must hold the current leaves and stay below 2^31");
  if (d->ld < d->capacity) return fail(LT_ERR_ARG, "ld must be at least the capacity");
  if (d->precision != 0 && d->precision != 1) return fail(LT_ERR_ARG, "precision must be 0 or 1");
  if (d->precision == 1 && !((dim == 3 && d->p == 3) || (dim == 2 && d->p == 7)))
    return fail(LT_ERR_ARG, "split precision needs 64 points per element");
  if (d->mlp && (dim != 3 || d->p != 3 || d->nvar != 5))
    return fail(LT_ERR_ARG, "learned flags need 3D p = 3 elements with 5 variables");
  hipStream_t s = static_cast<hipStream_t>(stream);
  lt_cycle c = new lt_cycle_s;
  c->t = t;
  c->d = *d;
  c->nmesh = d->nmesh;
  c->tmpl.assign(d->flag_template, d->flag_template + d->nmesh);
  // keep a private copy of the template's first entry's tables
  const lt_flag_params& f0 = d->flag_template[0];
  c->tmpl_nodes.assign(f0.nodes01, f0.nodes01 + f0.p + 1);
  c->tmpl_centres.assign(f0.centre, f0.centre + 3 * std::max(f0.nvort, 1));
  c->tmpl[0].nodes01 = c->tmpl_nodes.data();
  c->tmpl[0].centre = c->tmpl_centres.data();
  c->d.flag_template = nullptr;
  lt_status st = LT_OK;
  if (dev_malloc(t->A, reinterpret_cast<void**>(&c->dsz), 5 * sizeof(int64_t)) != hipSuccess ||
      hipHostMalloc(&c->hsz, 4 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&c->flag_host, flag_args_size() * size_t(c->nmesh), hipHostMallocDefault) != hipSuccess)
    st = fail(LT_ERR_OOM, "cycle state");
  if (st == LT_OK && !t->balanced) st = lt_balance(t, stream);  // the graph starts from a balanced tree
  if (st == LT_OK) st = reserve(c, s);
  if (st == LT_OK) st = fill_flag_table(t->g, c->tmpl.data(), 1, c->flag_host);  // validate the template
  if (st == LT_OK) st = upload_count(c, s);
  if (st == LT_OK) st = capture(c);
  if (st != LT_OK) {
    lt_cycle_destroy(c);
    return st;
  }
  *out = c;
  return LT_OK;
}

lt_status lt_cycle_run(lt_cycle c, const lt_flag_params* fp, void* stream, int* u_index) {
  if (!c || !fp) return fail(LT_ERR_ARG, "NULL argument");
  if (c->dead)
    return fail(LT_ERR_STATE, "an earlier run of this cycle failed while finishing eagerly; create a new cycle");
  lt_tree t = c->t;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int m = 0; m < c->nmesh; ++m)
    if (fp[m].p != c->tmpl[m].p) return fail(LT_ERR_ARG, "flag parameters need each mesh's template p");
  LT_TRY_STATUS(fill_flag_table(t->g, fp, c->nmesh, c->flag_host));
  const int q = c->parity;
  if (hipMemcpyAsync(t->flag_tab, c->flag_host, flag_args_size() * size_t(c->nmesh), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return fail(LT_ERR_HIP, "flag table upload");
  if (hipGraphLaunch(c->exec[q], s) != hipSuccess) return fail(LT_ERR_HIP, "graph launch");
  if (hipMemcpyAsync(c->hsz, c->dsz, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(LT_ERR_HIP, "size readback");
  LT_TRY_STATUS(read_ctr(t, s));
  unsigned err = t->hctr->err;
  // an unfinished balance also shows as missing fine leaves at hanging faces
  if (err & ERR_BALANCE_PASSES) err &= ~ERR_UNBALANCED;
  c->runs++;
  if (err == 0) {
    t->n_cur = c->hsz[0];
    t->n_old = c->hsz[1];
    t->n_hang = c->hsz[2];
    t->cur = 0;
    t->tmp = 1;
    t->old = 2;
    t->aux = 3;
    t->has_old = false;  // the pre-cycle keys were overwritten by the new ones
    t->balanced = true;
    t->adapt_marks = false;
    t->conn_valid = true;
    t->map_valid = true;
    t->dir_valid = false;
    c->parity = 1 - q;
    if (u_index) *u_index = c->parity;
    return LT_OK;
  }
  // The keys before the cycle are intact in kbuf[0] (the final copy is
  // skipped on any error).
  if (err & ERR_CAPACITY) {  // later checks failing on truncated arrays are its consequences
    t->n_cur = c->hsz[1];
    t->dir_valid = t->conn_valid = t->map_valid = false;
    t->n_hang = -1;
    return fail(LT_ERR_CAPACITY, "a captured cycle outgrew its capacity; the tree is unchanged");
  }
  if (err & ~ERR_BALANCE_PASSES) {
    t->n_cur = c->hsz[1];
    t->dir_valid = t->conn_valid = t->map_valid = false;
    char msg[96];
    snprintf(msg, sizeof msg, "device check failed in a captured cycle (error bits 0x%x)", err);
    return fail(LT_ERR_INTERNAL, msg);
  }
  // The fixed balance passes stopped short of the fixpoint: finish eagerly
  // from the partly balanced keys in kbuf[1].
  c->eager_finishes++;
  const lt_status st = finish_eagerly(c, q, stream, u_index);
  if (st != LT_OK) {
    // The eager calls may have moved or regrown buffers the graphs point at:
    // the graphs are dropped and the cycle refuses later runs.
    drop_graphs(c);
    c->dead = true;
  }
  return st;
}

lt_status lt_cycle_stats(lt_cycle c, int64_t* runs, int64_t* eager_finishes, int64_t* recaptures) {
  if (!c) return fail(LT_ERR_ARG, "NULL cycle");
  if (runs) *runs = c->runs;
  if (eager_finishes) *eager_finishes = c->eager_finishes;
  if (recaptures) *recaptures = c->recaptures;
  return LT_OK;
}

void lt_cycle_destroy(lt_cycle c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  drop_graphs(c);
  (void)dev_free(c->t->A, c->dsz);
  if (c->hsz) (void)hipHostFree(c->hsz);
  if (c->flag_host) (void)hipHostFree(c->flag_host);
  delete c;
}

}  // extern "C"
