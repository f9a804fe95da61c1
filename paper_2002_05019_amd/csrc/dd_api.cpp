// C ABI of the DD solver: argument checking, context, workspace binding and
// the drivers of the numeric phases (see include/dd.h for the contract).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <tuple>
#include <utility>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dd.h"
#include "kernels.h"
#include "plan.h"

namespace {
thread_local std::string g_err;

dd_status fail(dd_status s, const std::string &m) {
  g_err = m;
  return s;
}
}  // namespace

struct dd_ctx_s {
  dd::Plan plan;
  dd_options opt;
  // deep copy of the problem and the setup options, for re-planning (dd_tune)
  dd::SetupOptions so;
  std::vector<int32_t> n;
  std::vector<std::vector<int64_t>> rowptr;
  std::vector<std::vector<int32_t>> colind;
  std::vector<int64_t> imap_ptr, imap_mult;
  std::vector<int32_t> imap_dof;
  std::vector<int8_t> imap_sign;
  std::vector<float> xyz;
  int64_t n_mult = 0;
  uint8_t *ws = nullptr;
  int64_t ws_bytes = 0;
  bool factored = false;
  bool events = false;
  hipEvent_t ev[4];
  bool fact_rec = false, solve_rec = false;
  hipStream_t last = nullptr;
  double t_setup = 0;
  int refine_iters = 0;
  double rel_resid = 0, rel_resid_torn = 0;
  // status words of the last factorisation (see read_status); valid once
  // status_read is set
  bool status_read = false;
  int32_t stat[5] = {0, 0, 0, 0, 0};
  dd::KTimer tm;
  std::vector<hipEvent_t> tev;
  // hipGraph replay: captured on an internal stream, launched on the caller's
  hipStream_t cap = nullptr;
  std::map<const void *, hipGraphExec_t> gfactor;
  std::map<std::pair<int, int>, hipGraphExec_t> gsolve;
  // refined solve of one column block as one graph, per (columns,
  // iterations enqueued, right-hand side pointer, its leading dimension)
  std::map<std::tuple<int, int, const void *, int64_t>, hipGraphExec_t> grefine;
  // correction iterations the last refined solve needed (the next one
  // enqueues as many before it synchronises)
  int refine_guess = 2;
  // side streams of the factorisation and their events
  dd::SideStream side;
  // device whose static workspace array this context is bound to (-1: a
  // caller-owned workspace)
  int static_dev = -1;
  std::string tune_cache;      // dd_options.tune_cache (copied)
  bool tuned_from_cache = false;
};

namespace {
// context bound last to each device's static workspace array (the array
// holds that context's tables and factors; an earlier one is refused)
constexpr int MAX_STATIC_DEV = 64;
dd_ctx_s *g_static_owner[MAX_STATIC_DEV] = {};

bool static_stale(const dd_ctx_s *c) { return c->static_dev >= 0 && g_static_owner[c->static_dev] != c; }

void drop_graphs(dd_ctx_s *c) {
  for (auto &kv : c->gfactor) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : c->gsolve) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : c->grefine) (void)hipGraphExecDestroy(kv.second);
  c->gfactor.clear();
  c->gsolve.clear();
  c->grefine.clear();
}

// Records `enqueue` (launches only) on the capture stream into an executable graph.
template <class F>
hipError_t capture(dd_ctx_s *c, F enqueue, hipGraphExec_t *out) {
  hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e1 = enqueue(c->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap, &g);
  if (e1 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e1;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

// Waits for the last factorisation to finish and reads its status words
// (perturbed pivots, non-finite flag, 2 x 2 pivots, interchanges, lowest
// domain with a perturbed or non-finite pivot) through the internal stream.
hipError_t read_status(dd_ctx_s *c) {
  if (c->status_read) return hipSuccess;
  hipError_t e = hipEventSynchronize(c->ev[1]);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->stat, c->ws + c->plan.b_status, sizeof c->stat, hipMemcpyDeviceToHost, c->cap);
  if (e == hipSuccess) e = hipStreamSynchronize(c->cap);
  if (e == hipSuccess) c->status_read = true;
  return e;
}

std::string where_msg(const dd_ctx_s *c) {
  const int d = c->stat[4];
  if (d >= c->plan.n_dom) return "the auxiliary matrix";
  return "domain " + std::to_string(d);
}

// Status that the solve reports for the factorisation: DD_ERR_NUMERIC for a
// non-finite pivot (nothing is solved), DD_ERR_SINGULAR for perturbed
// pivots (the solve still runs on the perturbed factors), else DD_OK.
dd_status factor_status(const dd_ctx_s *c) {
  if (c->stat[1]) {
    g_err = "non-finite pivot in " + where_msg(c);
    return DD_ERR_NUMERIC;
  }
  if (c->stat[0]) {
    g_err = std::to_string(c->stat[0]) + " pivot block(s) perturbed, the first in " + where_msg(c);
    return DD_ERR_SINGULAR;
  }
  return DD_OK;
}

// Tile-cache key: the device's architecture and CU count, the precision,
// and an FNV-1a hash of every front's (kind, n, s) in plan order.
std::string tune_key(const dd_ctx_s *c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(c->plan.precision);
  for (const dd::FrontDev &d : c->plan.fronts) {
    mix(d.kind);
    mix(d.n);
    mix(d.s);
  }
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char &ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  char buf[256];
  snprintf(buf, sizeof buf, "%s/%dcu/p%d/%016llx", arch.c_str(), cus, c->plan.precision, (unsigned long long)h);
  return buf;
}

// Tiles of `key` from the cache file (false if absent or malformed).
bool cache_lookup(const std::string &path, const std::string &key, int *tiles) {
  FILE *fp = fopen(path.c_str(), "r");
  if (!fp) return false;
  char line[512], k[256];
  bool found = false;
  while (fgets(line, sizeof line, fp)) {
    int t[dd::TILE_BUCKETS];
    if (sscanf(line, "%255s %d %d %d %d %d", k, &t[0], &t[1], &t[2], &t[3], &t[4]) != 6) continue;
    if (key != k) continue;
    bool ok = true;
    for (int b = 0; b < dd::TILE_BUCKETS; ++b) ok = ok && (t[b] == 0 || t[b] == 64 || t[b] == 128);
    if (!ok) continue;
    for (int b = 0; b < dd::TILE_BUCKETS; ++b) tiles[b] = t[b];
    found = true;   // the last matching line wins
  }
  fclose(fp);
  return found;
}

void cache_append(const std::string &path, const std::string &key, const int *tiles) {
  FILE *fp = fopen(path.c_str(), "a");
  if (!fp) return;
  fprintf(fp, "%s %d %d %d %d %d\n", key.c_str(), tiles[0], tiles[1], tiles[2], tiles[3], tiles[4]);
  fclose(fp);
}

hipError_t run_solve_core(dd_ctx_s *c, int nrhs, bool with_c, hipStream_t st, bool subset = false) {
  if (!c->opt.use_graph) return dd::solve_core(c->plan, c->ws, nrhs, with_c, st, nullptr, subset);
  auto key = std::make_pair(nrhs, (with_c ? 1 : 0) + (subset ? 2 : 0));
  auto it = c->gsolve.find(key);
  if (it == c->gsolve.end()) {
    hipGraphExec_t ge;
    hipError_t e = capture(
        c, [&](hipStream_t s) { return dd::solve_core(c->plan, c->ws, nrhs, with_c, s, nullptr, subset); }, &ge);
    if (e != hipSuccess) return e;
    it = c->gsolve.emplace(key, ge).first;
  }
  return hipGraphLaunch(it->second, st);
}
}  // namespace

#define HIPCHECK(x)                                                                                \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess) return fail(DD_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

extern "C" {

void dd_default_options(dd_options *o) {
  if (!o) return;
  o->precision = DD_FP64;
  o->refine_tol = 1e-9;
  o->refine_maxit = 20;
  o->max_rhs = 64;
  o->leaf_size = 48;
  o->use_graph = 0;
  o->verbose = 0;
  for (int b = 0; b < DD_TILE_BUCKETS; ++b) o->schur_tile[b] = 0;
  o->verify_schedule = 0;
  o->tune_cache = nullptr;
}

const char *dd_last_error(void) { return g_err.c_str(); }

dd_status dd_setup(const dd_problem *prob, const dd_options *opt, dd_ctx *out) {
  try {
    g_err.clear();
    if (!out) return fail(DD_ERR_ARG, "out is null");
    *out = nullptr;
    if (!prob) return fail(DD_ERR_ARG, "problem is null");
    dd_options o;
    dd_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != DD_FP64 && o.precision != DD_FP32_REFINE) return fail(DD_ERR_ARG, "unknown precision");
    if (o.max_rhs < 1 || o.max_rhs > 4096) return fail(DD_ERR_ARG, "max_rhs must be in [1, 4096]");
    if (o.leaf_size < 1) return fail(DD_ERR_ARG, "leaf_size must be >= 1");
    if (o.refine_maxit < 0) return fail(DD_ERR_ARG, "refine_maxit must be >= 0");
    if (!(o.refine_tol > 0)) return fail(DD_ERR_ARG, "refine_tol must be > 0");
    if (o.use_graph < 0 || o.use_graph > 2) return fail(DD_ERR_ARG, "use_graph must be 0, 1 or 2");
    for (int b = 0; b < DD_TILE_BUCKETS; ++b)
      if (o.schur_tile[b] != 0 && o.schur_tile[b] != 64 && o.schur_tile[b] != 128)
        return fail(DD_ERR_ARG, "schur_tile entries must be 0, 64 or 128");
    if (prob->n_dom < 1 || !prob->dom) return fail(DD_ERR_ARG, "need at least one domain");
    auto t0 = std::chrono::steady_clock::now();
    dd::ProblemView pv;
    pv.n_dom = prob->n_dom;
    pv.n_mult = prob->n_mult;
    for (int i = 0; i < prob->n_dom; ++i) {
      pv.n.push_back(prob->dom[i].n);
      pv.rowptr.push_back(prob->dom[i].rowptr);
      pv.colind.push_back(prob->dom[i].colind);
      pv.nnz.push_back(prob->dom[i].nnz);
    }
    pv.imap_ptr = prob->imap_ptr;
    pv.imap_dof = prob->imap_dof;
    pv.imap_mult = prob->imap_mult;
    pv.imap_sign = prob->imap_sign;
    pv.xyz = prob->dof_xyz;
    int code = 0;
    std::string m = dd::validate_problem(pv, &code);
    if (!m.empty()) return fail((dd_status)code, m);
    dd::SetupOptions so;
    so.precision = o.precision;
    so.max_rhs = o.max_rhs;
    so.leaf = o.leaf_size;
    so.verbose = o.verbose;
    for (int b = 0; b < DD_TILE_BUCKETS; ++b) so.schur_tile[b] = o.schur_tile[b];
    so.verify = o.verify_schedule;
    dd_ctx_s *c = new dd_ctx_s;
    m = dd::build_plan(pv, so, c->plan);
    if (!m.empty()) {
      delete c;
      return fail(DD_ERR_PATTERN, m);
    }
    if (so.verify) {
      m = dd::check_schedule(c->plan, c->plan.factor_seq);
      if (m.empty()) m = dd::check_layout(c->plan);
      if (!m.empty()) {
        delete c;
        return fail(DD_ERR_STATE, "stream schedule check: " + m);
      }
    }
    c->so = so;
    c->n_mult = prob->n_mult;
    int64_t ntot = 0;
    for (int i = 0; i < prob->n_dom; ++i) {
      const dd_pattern &d = prob->dom[i];
      c->n.push_back(d.n);
      c->rowptr.emplace_back(d.rowptr, d.rowptr + d.n + 1);
      c->colind.emplace_back(d.colind, d.colind + d.nnz);
      ntot += d.n;
    }
    if (prob->imap_ptr) {
      const int64_t ne = prob->imap_ptr[prob->n_dom];
      c->imap_ptr.assign(prob->imap_ptr, prob->imap_ptr + prob->n_dom + 1);
      if (ne > 0) {
        c->imap_dof.assign(prob->imap_dof, prob->imap_dof + ne);
        c->imap_mult.assign(prob->imap_mult, prob->imap_mult + ne);
        c->imap_sign.assign(prob->imap_sign, prob->imap_sign + ne);
      }
    }
    if (prob->dof_xyz) c->xyz.assign(prob->dof_xyz, prob->dof_xyz + 3 * ntot);
    if (o.tune_cache) c->tune_cache = o.tune_cache;
    o.tune_cache = nullptr;   // the context keeps its own copy
    c->opt = o;
    c->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = c;
    return DD_OK;
  } catch (const std::bad_alloc &) {
    return fail(DD_ERR_NOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(DD_ERR_ARG, e.what());
  }
}

dd_status dd_workspace_size(dd_ctx c, int64_t *bytes) {
  if (!c || !bytes) return fail(DD_ERR_ARG, "null argument");
  *bytes = c->plan.b_total;
  return DD_OK;
}

}  // extern "C"

namespace {
// Events and streams of a context (created once, on first need).
dd_status ensure_runtime(dd_ctx_s *c) {
  if (!c->events) {
    for (int i = 0; i < 4; ++i) HIPCHECK(hipEventCreate(&c->ev[i]));
    c->events = true;
  }
  if (!c->cap) HIPCHECK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  for (int x = 0; x < dd::N_SIDE; ++x) {
    if (c->side.stream[x]) continue;
    hipStream_t s2;
    hipEvent_t e0, e1;
    HIPCHECK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&e0, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
    c->side.stream[x] = s2;
    c->side.fork[x] = e0;
    c->side.join[x] = e1;
  }
  return DD_OK;
}

// Uploads the index tables into the workspace and makes it the context's.
dd_status bind_region(dd_ctx_s *c, void *dev, int64_t bytes, int static_dev) {
  HIPCHECK(hipMemcpy((uint8_t *)dev + c->plan.b_meta, c->plan.meta.data(), c->plan.meta.size(),
                     hipMemcpyHostToDevice));
  drop_graphs(c);
  if (c->static_dev >= 0 && g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
  c->static_dev = static_dev;
  if (static_dev >= 0) g_static_owner[static_dev] = c;
  c->ws = (uint8_t *)dev;
  c->ws_bytes = bytes;
  c->factored = false;
  c->fact_rec = c->solve_rec = false;
  c->status_read = false;
  return DD_OK;
}
}  // namespace

namespace dd {
// Binds device `device`'s static workspace array (address dev, capacity
// bytes); called by dd_bind_static_workspace, which owns the array.
dd_status bind_static(dd_ctx c, void *dev, int64_t bytes, int device) {
  if (!c) return fail(DD_ERR_ARG, "null context");
  if (device < 0 || device >= MAX_STATIC_DEV) return fail(DD_ERR_DEVICE, "device id out of range");
  if (c->plan.b_total > bytes)
    return fail(DD_ERR_NOMEM, "workspace of " + std::to_string(c->plan.b_total) +
                                  " bytes exceeds the static workspace array (" + std::to_string(bytes) + " bytes)");
  return bind_region(c, dev, bytes, device);
}
dd_status set_error(dd_status s, const char *msg) { return fail(s, msg); }
}  // namespace dd

extern "C" {

dd_status dd_bind_workspace(dd_ctx c, void *dev, int64_t bytes) {
  if (!c || !dev) return fail(DD_ERR_ARG, "null argument");
  if (bytes < c->plan.b_total) return fail(DD_ERR_NOMEM, "workspace smaller than dd_workspace_size");
  if (((uintptr_t)dev) & 255) return fail(DD_ERR_ARG, "workspace must be 256-byte aligned");
  const dd_status r = ensure_runtime(c);
  if (r != DD_OK) return r;
  return bind_region(c, dev, bytes, -1);
}

dd_status dd_factor(dd_ctx c, const dd_z *vals, void *stream) {
  if (!c) return fail(DD_ERR_ARG, "null context");
  if (!c->ws) return fail(DD_ERR_STATE, "no workspace bound");
  if (static_stale(c)) return fail(DD_ERR_STATE, "the static workspace array was bound to another context");
  {
    const dd_status r = ensure_runtime(c);
    if (r != DD_OK) return r;
  }
  if (!vals && c->plan.nnz_total > 0) return fail(DD_ERR_ARG, "vals is null");
  hipStream_t st = (hipStream_t)stream;
  const void *v = vals;
  // FP64 copy of the operator for the refinement residuals
  if (c->plan.precision != 0) HIPCHECK(dd::operator_copy(c->plan, c->ws, vals, st));
  HIPCHECK(hipEventRecord(c->ev[0], st));
  if (c->opt.use_graph == 1 && c->tm.kind < 0) {
    auto it = c->gfactor.find(v);
    if (it == c->gfactor.end()) {
      hipGraphExec_t ge;
      HIPCHECK(capture(c, [&](hipStream_t s) { return dd::factor(c->plan, c->ws, v, s, nullptr, &c->side); }, &ge));
      it = c->gfactor.emplace(v, ge).first;
    }
    HIPCHECK(hipGraphLaunch(it->second, st));
  } else {
    HIPCHECK(dd::factor(c->plan, c->ws, v, st, c->tm.kind >= 0 ? &c->tm : nullptr, &c->side));
  }
  HIPCHECK(hipEventRecord(c->ev[1], st));
  c->fact_rec = true;
  c->factored = true;
  c->status_read = false;
  c->last = st;
  return DD_OK;
}

dd_status dd_solve(dd_ctx c, int32_t nrhs, const dd_z *f, int64_t ldf, dd_z *u, int64_t ldu, dd_z *lam, int64_t ldl,
                   void *stream) {
  if (!c) return fail(DD_ERR_ARG, "null context");
  if (static_stale(c)) return fail(DD_ERR_STATE, "the static workspace array was bound to another context");
  if (!c->factored) return fail(DD_ERR_STATE, "dd_solve before dd_factor");
  if (nrhs < 0) return fail(DD_ERR_ARG, "nrhs < 0");
  if (nrhs == 0) return DD_OK;
  const dd::Plan &P = c->plan;
  if (!f || !u) return fail(DD_ERR_ARG, "f or u is null");
  if (ldf < P.n_torn || ldu < P.n_torn) return fail(DD_ERR_ARG, "leading dimension below the torn size");
  if (lam && ldl < P.n_mult) return fail(DD_ERR_ARG, "ldl below n_mult");
  if ((const void *)f == (const void *)u) return fail(DD_ERR_ARG, "u may not alias f");
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(read_status(c));
  const dd_status fst = factor_status(c);
  if (fst == DD_ERR_NUMERIC) return fst;
  c->last = st;
  HIPCHECK(hipEventRecord(c->ev[2], st));
  dd_status result = DD_OK;
  c->refine_iters = 0;
  c->rel_resid = 0;
  c->rel_resid_torn = 0;
  for (int32_t j0 = 0; j0 < nrhs; j0 += P.max_rhs) {
    const int nb = std::min<int32_t>(P.max_rhs, nrhs - j0);
    const dd_z *fj = f + (int64_t)j0 * ldf;
    dd_z *uj = u + (int64_t)j0 * ldu;
    dd_z *lj = lam ? lam + (int64_t)j0 * ldl : nullptr;
    if (P.precision == 0) {
      HIPCHECK(dd::rhs_in(P, c->ws, fj, ldf, nb, st));
      HIPCHECK(run_solve_core(c, nb, false, st));
      HIPCHECK(dd::sol_out(P, c->ws, uj, ldu, lj, ldl, nb, st));
      continue;
    }
    // FP64 iterative refinement with the FP32 factors.  Two residuals per
    // column, both relative to the right-hand side: the torn one,
    // [f - K u - B^T lam; -B u], whose FP32 solve gives the correction, and
    // the assembled one, f - A u~ with every DoF taken from its
    // representative copy (the residual of the undecomposed FEM system,
    // A = sum_i R_i^T K_i R_i).  Converged when both are within refine_tol.
    // The test runs on the device: the first solve, the residuals and K
    // correction iterations (as many as the last refined solve needed) are
    // enqueued at once, or replayed as one graph, and the iterations after
    // convergence return at once; the host synchronises once and continues
    // one iteration at a time only if K were not enough.
    const double tol = c->opt.refine_tol;
    const int *gate = dd::refine_ctl(P, c->ws);
    auto iteration = [&](hipStream_t s) -> hipError_t {
      hipError_t e = dd::solve_core(P, c->ws, nb, true, s, nullptr, false, gate);
      if (e == hipSuccess) e = dd::refine_update(P, c->ws, nb, s, gate);
      if (e == hipSuccess) e = dd::refine_resid(P, c->ws, fj, ldf, nb, false, s, gate);
      if (e == hipSuccess) e = dd::refine_test(P, c->ws, nb, tol, true, s);
      return e;
    };
    const int K = std::min(c->opt.refine_maxit, std::max(0, c->refine_guess));
    auto sequence = [&](hipStream_t s) -> hipError_t {
      hipError_t e = dd::rhs_in(P, c->ws, fj, ldf, nb, s);
      if (e == hipSuccess) e = dd::solve_core(P, c->ws, nb, false, s);
      if (e == hipSuccess) e = dd::refine_ctl_reset(P, c->ws, s);
      if (e == hipSuccess) e = dd::refine_init(P, c->ws, nb, s);
      if (e == hipSuccess) e = dd::refine_resid(P, c->ws, fj, ldf, nb, true, s);
      if (e == hipSuccess) e = dd::refine_resid(P, c->ws, fj, ldf, nb, false, s);
      if (e == hipSuccess) e = dd::refine_test(P, c->ws, nb, tol, false, s);
      for (int k = 0; k < K && e == hipSuccess; ++k) e = iteration(s);
      return e;
    };
    if (c->opt.use_graph) {
      const auto key = std::make_tuple(nb, K, (const void *)fj, ldf);
      auto itg = c->grefine.find(key);
      if (itg == c->grefine.end()) {
        hipGraphExec_t ge;
        HIPCHECK(capture(c, sequence, &ge));
        itg = c->grefine.emplace(key, ge).first;
      }
      HIPCHECK(hipGraphLaunch(itg->second, st));
    } else {
      HIPCHECK(sequence(st));
    }
    int ctl[3];
    double relv[2];
    auto fetch = [&]() -> hipError_t {
      hipError_t e = hipMemcpyAsync(ctl, gate, sizeof ctl, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(relv, dd::refine_rel(P, c->ws), sizeof relv, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      return e;
    };
    HIPCHECK(fetch());
    while (!ctl[0] && ctl[1] < c->opt.refine_maxit) {
      HIPCHECK(iteration(st));
      HIPCHECK(fetch());
    }
    const int it = ctl[1];
    const double rel_t = relv[0], rel_g = relv[1];
    c->refine_guess = it;
    if (ctl[2]) {
      result = DD_ERR_NUMERIC;
      g_err = "non-finite residual during refinement";
    } else if (!ctl[0]) {
      // perturbed pivots are the likely cause: report them
      result = fst != DD_OK ? fst : DD_ERR_NOT_CONVERGED;
      if (fst == DD_OK) g_err = "refinement did not reach refine_tol";
    }
    HIPCHECK(dd::refine_out(P, c->ws, uj, ldu, lj, ldl, nb, st));
    c->refine_iters = std::max(c->refine_iters, it);
    c->rel_resid = std::max(c->rel_resid, rel_g);
    c->rel_resid_torn = std::max(c->rel_resid_torn, rel_t);
  }
  HIPCHECK(hipEventRecord(c->ev[3], st));
  c->solve_rec = true;
  // FP64: perturbed pivots make the solution inexact (no refinement repairs
  // it); FP32_REFINE: a refinement that reached refine_tol repaired them
  if (result == DD_OK && P.precision == 0 && fst != DD_OK) {
    factor_status(c);
    result = fst;
  }
  return result;
}

dd_status dd_solve_subset(dd_ctx c, int32_t nrhs, const dd_z *f, int64_t ldf, dd_z *u, int64_t ldu,
                          const uint8_t *domain_mask, void *stream) {
  if (!c) return fail(DD_ERR_ARG, "null context");
  const dd::Plan &P = c->plan;
  if (P.precision != 0)
    return fail(DD_ERR_ARG, "subset recovery needs the FP64 path (refinement uses every domain's solution)");
  if (nrhs < 0) return fail(DD_ERR_ARG, "nrhs < 0");
  if (!domain_mask) return fail(DD_ERR_ARG, "domain_mask is null");
  if (static_stale(c)) return fail(DD_ERR_STATE, "the static workspace array was bound to another context");
  if (!c->factored) return fail(DD_ERR_STATE, "dd_solve_subset before dd_factor");
  if (nrhs == 0) return DD_OK;
  if (!f || !u) return fail(DD_ERR_ARG, "f or u is null");
  if (ldf < P.n_torn || ldu < P.n_torn) return fail(DD_ERR_ARG, "leading dimension below the torn size");
  if ((const void *)f == (const void *)u) return fail(DD_ERR_ARG, "u may not alias f");
  try {
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(read_status(c));
    const dd_status fst = factor_status(c);
    if (fst == DD_ERR_NUMERIC) return fst;
    c->last = st;
    HIPCHECK(hipMemcpyAsync(c->ws + P.b_dmask, domain_mask, (size_t)P.n_dom, hipMemcpyHostToDevice, st));
    HIPCHECK(hipEventRecord(c->ev[2], st));
    c->refine_iters = 0;
    c->rel_resid = 0;
    for (int32_t j0 = 0; j0 < nrhs; j0 += P.max_rhs) {
      const int nb = std::min<int32_t>(P.max_rhs, nrhs - j0);
      HIPCHECK(dd::rhs_in(P, c->ws, f + (int64_t)j0 * ldf, ldf, nb, st));
      HIPCHECK(run_solve_core(c, nb, false, st, true));
      HIPCHECK(dd::sol_out(P, c->ws, u + (int64_t)j0 * ldu, ldu, nullptr, 0, nb, st, true));
    }
    HIPCHECK(hipEventRecord(c->ev[3], st));
    c->solve_rec = true;
    if (fst != DD_OK) {
      factor_status(c);
      return fst;
    }
  } catch (...) {
    return fail(DD_ERR_DEVICE, "unexpected exception");
  }
  return DD_OK;
}

dd_status dd_solve_dofs(dd_ctx c, int32_t nrhs, const dd_z *f, int64_t ldf, int64_t nsel, const int64_t *rows,
                        dd_z *out, int64_t ldo, void *stream) {
  if (!c) return fail(DD_ERR_ARG, "null context");
  const dd::Plan &P = c->plan;
  if (P.precision != 0)
    return fail(DD_ERR_ARG, "subset recovery needs the FP64 path (refinement uses every domain's solution)");
  if (nrhs < 0 || nsel < 0) return fail(DD_ERR_ARG, "negative size");
  if (nsel > 0 && !rows) return fail(DD_ERR_ARG, "rows is null");
  if (static_stale(c)) return fail(DD_ERR_STATE, "the static workspace array was bound to another context");
  if (!c->factored) return fail(DD_ERR_STATE, "dd_solve_dofs before dd_factor");
  if (nrhs == 0 || nsel == 0) return DD_OK;
  if (!f || !out) return fail(DD_ERR_ARG, "f or out is null");
  if (ldf < P.n_torn) return fail(DD_ERR_ARG, "ldf below the torn size");
  if (ldo < nsel) return fail(DD_ERR_ARG, "ldo below the number of selected rows");
  if (nsel > P.n_torn) return fail(DD_ERR_ARG, "more selected rows than torn rows");
  try {
    std::vector<uint8_t> mask(P.n_dom, 0);
    for (int64_t i = 0; i < nsel; ++i) {
      if (rows[i] < 0 || rows[i] >= P.n_torn) return fail(DD_ERR_ARG, "selected row out of range");
      const int d = (int)(std::upper_bound(P.dom_row.begin(), P.dom_row.end(), rows[i]) - P.dom_row.begin()) - 1;
      mask[d] = 1;
    }
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(read_status(c));
    const dd_status fst = factor_status(c);
    if (fst == DD_ERR_NUMERIC) return fst;
    c->last = st;
    HIPCHECK(hipMemcpyAsync(c->ws + P.b_dmask, mask.data(), (size_t)P.n_dom, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(c->ws + P.b_sel, rows, (size_t)nsel * 8, hipMemcpyHostToDevice, st));
    HIPCHECK(hipEventRecord(c->ev[2], st));
    c->refine_iters = 0;
    c->rel_resid = 0;
    for (int32_t j0 = 0; j0 < nrhs; j0 += P.max_rhs) {
      const int nb = std::min<int32_t>(P.max_rhs, nrhs - j0);
      HIPCHECK(dd::rhs_in(P, c->ws, f + (int64_t)j0 * ldf, ldf, nb, st));
      HIPCHECK(run_solve_core(c, nb, false, st, true));
      HIPCHECK(dd::sel_out(P, c->ws, nsel, out + (int64_t)j0 * ldo, ldo, nb, st));
    }
    HIPCHECK(hipEventRecord(c->ev[3], st));
    // the host arrays were staged by the copies above; wait for them before
    // returning (the caller may free them)
    HIPCHECK(hipStreamSynchronize(st));
    c->solve_rec = true;
    if (fst != DD_OK) {
      factor_status(c);
      return fst;
    }
  } catch (const std::bad_alloc &) {
    return fail(DD_ERR_NOMEM, "host allocation failed");
  }
  return DD_OK;
}

dd_status dd_get_info(dd_ctx c, dd_info *info) {
  if (!c || !info) return fail(DD_ERR_ARG, "null argument");
  std::memset(info, 0, sizeof *info);
  const dd::Plan &P = c->plan;
  info->t_setup = c->t_setup;
  info->flops_factor = P.flops_factor;
  info->flops_solve = P.flops_solve_rhs;
  info->bytes_factor = P.bytes_factor;
  info->bytes_solve = P.bytes_solve;
  info->workspace_bytes = P.b_total;
  info->n_fronts_domain = P.n_front_dom;
  info->n_fronts_aux = P.n_front_aux;
  info->max_front_aux = P.max_front_aux;
  info->max_front_domain = P.max_front_dom;
  info->refine_iters = c->refine_iters;
  info->rel_resid = c->rel_resid;
  info->rel_resid_torn = c->rel_resid_torn;
  info->bad_domain = -1;
  info->tuned_from_cache = c->tuned_from_cache ? 1 : 0;
  if (c->events) {
    float ms = 0;
    if (c->fact_rec) {
      HIPCHECK(hipEventSynchronize(c->ev[1]));
      HIPCHECK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
      info->t_factor = ms * 1e-3;
    }
    if (c->solve_rec) {
      HIPCHECK(hipEventSynchronize(c->ev[3]));
      HIPCHECK(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
      info->t_solve = ms * 1e-3;
    }
  }
  if (c->ws && c->factored && !static_stale(c)) {
    HIPCHECK(hipStreamSynchronize(c->last));
    HIPCHECK(read_status(c));
    info->n_perturbed = c->stat[0];
    info->numeric_flags = c->stat[1];
    info->n_pivot_2x2 = c->stat[2];
    info->n_interchanges = c->stat[3];
    if (c->stat[0] || c->stat[1]) info->bad_domain = c->stat[4];
  }
  return DD_OK;
}

dd_status dd_get_interface_dofs(dd_ctx c, int32_t dom, int32_t *count, int32_t *dofs) {
  if (!c || !count) return fail(DD_ERR_ARG, "null argument");
  if (dom < 0 || dom >= c->plan.n_dom) return fail(DD_ERR_ARG, "domain out of range");
  const auto &g = c->plan.gamma[dom];
  *count = (int32_t)g.size();
  if (dofs) std::memcpy(dofs, g.data(), g.size() * sizeof(int32_t));
  return DD_OK;
}

dd_status dd_get_interface_inverse(dd_ctx c, int32_t dom, dd_z *out, void *stream) {
  if (!c || !out) return fail(DD_ERR_ARG, "null argument");
  if (dom < 0 || dom >= c->plan.n_dom) return fail(DD_ERR_ARG, "domain out of range");
  if (static_stale(c)) return fail(DD_ERR_STATE, "the static workspace array was bound to another context");
  if (!c->factored) return fail(DD_ERR_STATE, "no factorisation");
  int f = c->plan.gamma_front[dom];
  if (f < 0) return fail(DD_ERR_ARG, "domain has no interface");
  HIPCHECK(dd::interface_inverse_out(c->plan, c->ws, f, out, (hipStream_t)stream));
  return DD_OK;
}

dd_status dd_get_domain_flops(dd_ctx c, int32_t dom, double *flops) {
  if (!c || !flops) return fail(DD_ERR_ARG, "null argument");
  if (dom < 0 || dom >= c->plan.n_dom) return fail(DD_ERR_ARG, "domain out of range");
  *flops = c->plan.dom_flops.empty() ? 0.0 : c->plan.dom_flops[dom];
  return DD_OK;
}

dd_status dd_kernel_timer_start(dd_ctx c, int32_t kernel) {
  if (!c) return fail(DD_ERR_ARG, "null context");
  static const int kinds[] = {dd::L_SYRK, dd::L_TRSM, dd::L_PANEL, dd::L_INVSYRK, dd::L_UPDPANEL};
  if (kernel < -1 || kernel > 4) return fail(DD_ERR_ARG, "unknown kernel");
  if (c->tev.empty() && kernel >= 0) {
    c->tev.resize(8192);
    for (auto &e : c->tev) HIPCHECK(hipEventCreate(&e));
  }
  c->tm = dd::KTimer();
  c->tm.kind = kernel < 0 ? -1 : kinds[kernel];
  c->tm.ev = c->tev.data();
  c->tm.cap = (int32_t)c->tev.size();
  return DD_OK;
}

dd_status dd_kernel_timer_read(dd_ctx c, double *seconds, int64_t *launches, double *flops) {
  if (!c || !seconds || !launches || !flops) return fail(DD_ERR_ARG, "null argument");
  double t = 0;
  for (int i = 0; i + 1 < c->tm.used; i += 2) {
    float ms = 0;
    HIPCHECK(hipEventSynchronize(c->tev[i + 1]));
    HIPCHECK(hipEventElapsedTime(&ms, c->tev[i], c->tev[i + 1]));
    t += ms * 1e-3;
  }
  *seconds = t;
  *launches = c->tm.launches;
  *flops = c->tm.flops;
  return DD_OK;
}

dd_status dd_tune(dd_ctx c, int32_t *schur_tile, void *stream) {
  if (!c) return fail(DD_ERR_ARG, "null context");
  if (!c->ws) return fail(DD_ERR_STATE, "no workspace bound");
  if (static_stale(c)) return fail(DD_ERR_STATE, "the static workspace array was bound to another context");
  {
    const dd_status r = ensure_runtime(c);
    if (r != DD_OK) return r;
  }
  try {
    hipStream_t st = (hipStream_t)stream;
    int choice[dd::TILE_BUCKETS];
    const std::string key = tune_key(c);
    c->tuned_from_cache = !c->tune_cache.empty() && cache_lookup(c->tune_cache, key, choice);
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    for (int b = 0; b < dd::TILE_BUCKETS && !c->tuned_from_cache; ++b) {
      choice[b] = 0;
      const dd::Launch &l64 = c->plan.tune[b][0], &l128 = c->plan.tune[b][1];
      if (l64.count == 0 || l128.count == 0) continue;
      float best[2] = {1e30f, 1e30f};
      for (int rep = 0; rep < 4; ++rep)
        for (int v = 0; v < 2; ++v) {
          HIPCHECK(hipEventRecord(e0, st));
          HIPCHECK(dd::run_launch(c->plan, c->ws, v ? l128 : l64, st));
          HIPCHECK(hipEventRecord(e1, st));
          HIPCHECK(hipEventSynchronize(e1));
          float ms = 0;
          HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) best[v] = std::min(best[v], ms);   // first round warms up
        }
      choice[b] = best[1] < 0.9f * best[0] ? 128 : 64;   // 128 only when clearly faster
      if (c->opt.verbose)
        fprintf(stderr, "[dd] tile bucket %d: 64 -> %.3f ms, 128 -> %.3f ms: %d\n", b, best[0], best[1], choice[b]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!c->tune_cache.empty() && !c->tuned_from_cache) cache_append(c->tune_cache, key, choice);
    // re-plan with the chosen policy (same workspace layout) and upload
    dd::SetupOptions so = c->so;
    for (int b = 0; b < dd::TILE_BUCKETS; ++b) {
      if (choice[b]) so.schur_tile[b] = choice[b];
      c->opt.schur_tile[b] = so.schur_tile[b];
      if (schur_tile) schur_tile[b] = choice[b];
    }
    dd::ProblemView pv;
    pv.n_dom = (int32_t)c->n.size();
    pv.n_mult = c->n_mult;
    for (size_t i = 0; i < c->n.size(); ++i) {
      pv.n.push_back(c->n[i]);
      pv.rowptr.push_back(c->rowptr[i].data());
      pv.colind.push_back(c->colind[i].data());
      pv.nnz.push_back((int64_t)c->colind[i].size());
    }
    pv.imap_ptr = c->imap_ptr.empty() ? nullptr : c->imap_ptr.data();
    pv.imap_dof = c->imap_dof.empty() ? nullptr : c->imap_dof.data();
    pv.imap_mult = c->imap_mult.empty() ? nullptr : c->imap_mult.data();
    pv.imap_sign = c->imap_sign.empty() ? nullptr : c->imap_sign.data();
    pv.xyz = c->xyz.empty() ? nullptr : c->xyz.data();
    dd::Plan np;
    std::string m = dd::build_plan(pv, so, np);
    if (!m.empty()) return fail(DD_ERR_PATTERN, m);
    if (so.verify) {
      m = dd::check_schedule(np, np.factor_seq);
      if (m.empty()) m = dd::check_layout(np);
      if (!m.empty()) return fail(DD_ERR_STATE, "stream schedule check: " + m);
    }
    if (np.b_total != c->plan.b_total || np.b_meta != c->plan.b_meta || np.meta.size() != c->plan.meta.size())
      return fail(DD_ERR_STATE, "re-planned layout differs");
    HIPCHECK(hipMemcpy(c->ws + np.b_meta, np.meta.data(), np.meta.size(), hipMemcpyHostToDevice));
    c->plan = std::move(np);
    c->so = so;
    drop_graphs(c);
    c->factored = false;
    return DD_OK;
  } catch (const std::bad_alloc &) {
    return fail(DD_ERR_NOMEM, "host allocation failed");
  }
}

void dd_destroy(dd_ctx c) {
  if (!c) return;
  if (c->static_dev >= 0 && g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
  if (c->events)
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(c->ev[i]);
  for (auto &e : c->tev) (void)hipEventDestroy(e);
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (int x = 0; x < dd::N_SIDE; ++x) {
    if (c->side.stream[x]) (void)hipStreamDestroy((hipStream_t)c->side.stream[x]);
    for (void *e : {c->side.fork[x], c->side.join[x]})
      if (e) (void)hipEventDestroy((hipEvent_t)e);
  }
  delete c;
}

}  // extern "C"
