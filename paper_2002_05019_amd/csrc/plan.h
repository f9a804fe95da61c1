// Host-side plan of the DD solver: symbolic structure, workspace layout and
// the launch sequences of the numeric phases.  Built once by dd_setup on the
// CPU (no GPU call), then uploaded into the caller's workspace.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "dd_internal.h"

namespace dd {

enum LaunchKind : int32_t {
  // factorisation
  L_ASM,        // pull extend-add: assign children update blocks (zero elsewhere)
  L_SCAT,       // add original domain-matrix entries
  L_AUXG,       // add interface-inverse blocks into auxiliary fronts
  L_PANEL,      // pivot-tile LDL^T with restricted Bunch-Kaufman
  L_TRSM,       // W = A21 P L11^-T, L21 = W D^-1
  L_SYRK,       // trailing update C -= L21 W^T
  L_ZREC1,      // recursive inverse: T1 = P L21 Z11 (upper triangle)
  L_ZREC2,      // recursive inverse: Z21 = -Z22 T1
  L_INVSYRK,    // X = P^T Z^T Y P with Y = D^-1 Z
  L_SYRK2,      // trailing update on 128 x 128 tiles (512 threads)
  L_FORK,       // the side stream waits for the main stream (no kernel)
  L_JOIN,       // the main stream waits for the side stream (no kernel)
  L_DINVZ,      // Y = D^-1 Z of an interface root, stored transposed above Z
  L_STORE,      // factor columns of a front into its stored-factor place
  L_UPDPANEL,   // column update and pivot tile in one launch (pivot-tile items first)
  // solve
  S_FINIT,      // front vector = gathered right-hand side + children updates (256 rows per item)
  S_FFIN,       // z = D^-1 y over the fully-summed rows (256 rows per item)
  S_BINIT,      // update rows of the front vector from the global solution
  S_BFIN,       // fully-summed rows of the front vector to the global solution
  S_FFRONT,     // whole-front forward substitution, one workgroup per front
  S_BFRONT,     // whole-front backward substitution, one workgroup per front
  // fronts carrying Z = L11^-1: split products (one partial slot per item,
  // item = {front, slot, output tile, K chunk}) and their reductions
  // (item = {front, first slot, output tile, slot count})
  S_ZP0, S_ZR0, // y = Z P v_s;  v_s = y
  S_ZP1, S_ZR1, // v_R -= L21 y
  S_ZP2, S_ZR2, // t = z - L21^T x_R
  S_ZP3, S_ZR3, // x_s = P^T Z^T t
};

// front-size buckets of the Schur-update tile policy: n < 512, < 1024,
// < 2048, < 4096, >= 4096
constexpr int TILE_BUCKETS = 5;
inline int tile_bucket(int n) { return n < 512 ? 0 : n < 1024 ? 1 : n < 2048 ? 2 : n < 4096 ? 3 : 4; }

struct Launch {
  int32_t kind;
  int32_t count;     // number of items / workgroups
  int64_t first;     // first item in the kind's item array
  int32_t p0, p1;    // kind-specific
  double flops;      // algorithmic real flops of the launch (complex FMA = 8)
  int32_t side = 0;  // 1: enqueued on the side stream (look-ahead of the factorisation)
};

// Side streams and their events of the factorisation (owned by the caller;
// null streams = everything on the main stream).  Launch.side = s >= 1 runs
// on stream[s - 1]: 1 the look-ahead of the trailing update, 2 the previous
// level's inverses and stored-factor copies.
constexpr int N_SIDE = 2;
struct SideStream {
  void *stream[N_SIDE] = {nullptr, nullptr};   // hipStream_t
  void *fork[N_SIDE] = {nullptr, nullptr};     // hipEvent_t, recorded on the main stream
  void *join[N_SIDE] = {nullptr, nullptr};     // hipEvent_t, recorded on the side stream
};

// Optional per-kernel event timer (diagnostics): brackets every launch of
// one kind with a pair of events on the launch stream.
struct KTimer {
  int32_t kind = -1;
  void *ev = nullptr;      // hipEvent_t array
  int32_t cap = 0, used = 0;
  int64_t launches = 0;
  double flops = 0;
};

struct Plan {
  // ---- problem
  int32_t n_dom = 0;
  int64_t n_mult = 0, n_torn = 0, nnz_total = 0;
  std::vector<int32_t> dom_n;
  std::vector<int64_t> dom_row;      // first torn row of each domain
  std::vector<int64_t> dom_nnz;      // first value index of each domain
  std::vector<int64_t> csr_ptr;      // torn system CSR (global rows/cols), n_torn + 1
  std::vector<int32_t> csr_col;
  // SELL-64 copy of the torn operator for the FP64 refinement residual:
  // slices of 64 consecutive rows, slice s holds width w_s = (sell_ptr[s+1] -
  // sell_ptr[s]) / 64 entries per row, entry k of row 64 s + l at
  // sell_ptr[s] + 64 k + l; padding entries have column 0 and value 0
  std::vector<int64_t> sell_ptr;
  std::vector<int32_t> sell_col;
  int64_t nnz_sell = 0;
  std::vector<std::vector<int32_t>> gamma;   // sorted interface dofs per domain
  std::vector<int32_t> gamma_front;          // interface-root front id per domain (-1 if none)

  // ---- fronts
  std::vector<FrontDev> fronts;
  std::vector<int32_t> vars;
  std::vector<int32_t> child_front;
  std::vector<int64_t> child_rmap;
  std::vector<int32_t> rmap;
  std::vector<int32_t> urow;   // per front: parent row of each update row (FrontDev::uoff)
  std::vector<SPair> spairs;
  std::vector<AuxItem> aux_items;
  std::vector<int32_t> gpos, gsign;
  std::vector<MultRef> mrefs;
  std::vector<GamRef> grefs;
  std::vector<int32_t> hmult, hsign;
  std::vector<int32_t> row_gam;
  // copies of one global DoF: the torn rows that multipliers tie together
  // (union of the multiplier pairs).  grep[r] = lowest torn row of r's
  // component (its representative); the components in representative order,
  // gcomp_row[gcomp_ptr[c] .. gcomp_ptr[c+1]) their rows (FP64 refinement:
  // residual of the assembled system)
  std::vector<int32_t> grep, gcomp_ptr, gcomp_row;
  int64_t n_gcomp = 0;

  // ---- schedule
  std::vector<Item> items;
  std::vector<Launch> factor_seq;
  std::vector<Launch> solve_dom_fwd;   // interior forward + Gamma assemble
  std::vector<Launch> solve_aux;       // aux forward + backward
  std::vector<Launch> solve_dom_bwd;   // Gamma scatter + interior backward
  std::vector<Item> gemv_items;        // interface GEMV items (one per 64-row tile)
  std::vector<double> dom_flops;       // factor flops per domain (fronts + interface inverse)
  int64_t max_partials = 0;            // partial slots needed by the largest split product

  // ---- options / layout
  int32_t precision = 0;
  int32_t max_rhs = 64;
  int32_t schur_tile[TILE_BUCKETS] = {64, 64, 64, 64, 64};   // resolved policy
  // per bucket: the first outer block's trailing update of all fronts of the
  // bucket with 64 (index 0) and 128 (index 1) tiles, for the tile tuner
  Launch tune[TILE_BUCKETS][2] = {};
  size_t elem = 8;                     // sizeof(T)
  int64_t t_elems = 0;                 // T elements in the numeric region
  // numeric region (T elements): stored factors, W scratch of the widest
  // level, and the arena (peak of the factorisation's live fronts, or the
  // solve's vectors, whichever is larger)
  int64_t e_stored = 0, e_w = 0, e_arena_factor = 0, e_arena_solve = 0;
  // factorisation level of every front and the last level that reads its
  // full matrix (its parent's); the layout check replays them
  std::vector<int32_t> front_lev, front_last;
  int64_t vf_off = 0, vx_off = 0, vd_off = 0, vl_off = 0, vc_off = 0, part_off = 0;
  int64_t side_n = 0;                  // fully-summed positions (side arrays)
  // byte offsets inside the workspace
  int64_t b_meta = 0, b_num = 0, b_side = 0, b_vals = 0, b_r64 = 0, b_status = 0, b_dmask = 0, b_sel = 0,
          b_total = 0;
  // offsets (bytes) of each meta array inside the meta blob
  int64_t m_fronts, m_vars, m_cfront, m_crmap, m_rmap, m_urow, m_spairs, m_aux, m_gpos, m_gsign,
      m_mrefs, m_grefs, m_hmult, m_hsign, m_rowgam, m_items, m_gemv, m_csrp, m_sellp, m_sellc, m_domrow,
      m_grep, m_gcp, m_gcr;
  std::vector<uint8_t> meta;           // serialised meta blob
  // FP64 refinement vectors (doubles, planar) inside the r64 region
  // r_g: per torn row f - K u~ with u~ the representative copies (FP64 planar)
  int64_t r_u = 0, r_l = 0, r_g = 0, r_norm = 0, r_fnorm = 0, r_part = 0, r_ctl = 0;
  int64_t r_nblk = 0;

  // ---- statistics
  double flops_factor = 0, flops_solve_rhs = 0, bytes_factor = 0, bytes_solve = 0;
  int32_t n_front_dom = 0, n_front_aux = 0, max_front_dom = 0, max_front_aux = 0;
};

struct SetupOptions {
  int32_t precision = 0;
  int32_t max_rhs = 64;
  int32_t leaf = 48;
  int32_t aux_leaf = 256;
  int32_t verbose = 0;
  int32_t schur_tile[TILE_BUCKETS] = {0, 0, 0, 0, 0};   // 64 or 128; 0 = default
  int32_t verify = 0;   // check the factorisation's stream ordering
};

struct ProblemView {
  int32_t n_dom;
  int64_t n_mult;
  std::vector<int32_t> n;
  std::vector<const int64_t *> rowptr;
  std::vector<const int32_t *> colind;
  std::vector<int64_t> nnz;
  const int64_t *imap_ptr;
  const int32_t *imap_dof;
  const int64_t *imap_mult;
  const int8_t *imap_sign;
  const float *xyz;
};

// Validates the problem; returns an empty string or the error message and
// sets *code to the dd_status value.
std::string validate_problem(const ProblemView &p, int *code);

// Builds the full plan (symbolic analysis, schedule, workspace layout).
std::string build_plan(const ProblemView &p, const SetupOptions &o, Plan &plan);
// "" if every pair of launches of `seq` on different streams that the
// fork / join points leave unordered touches disjoint data, else a message
std::string check_schedule(const Plan &P, const std::vector<Launch> &seq);
// "" if the numeric layout is consistent: the full matrices of fronts alive
// at the same level (from their own level to their parent's) are disjoint,
// the stored factors and interface inverses are disjoint from each other and
// lie below the W scratch, and the W buffers of one level are disjoint
std::string check_layout(const Plan &P);

}  // namespace dd
