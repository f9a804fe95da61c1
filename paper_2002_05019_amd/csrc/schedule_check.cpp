// Host verification of the factorisation's stream schedule.
//
// The factorisation sequence spreads its launches over the main stream and
// side streams, ordered by fork (a side stream waits for the main stream)
// and join (the main stream waits for a side stream) points.  This check
// replays those ordering rules with vector clocks and, for every pair of
// launches on different streams that are not ordered, compares what their
// work items read and write: rectangles of a front's matrix, of its two W
// buffers and of its pivot arrays.  Kernels other than the column / trailing
// updates, the pivot tile, the panel solve, the inverse recursion and the
// stored-factor copy are treated as touching everything, so they must never
// overlap a side-stream launch.  The work
// items inside one launch of the pivot chain (pivot tile, column update,
// panel solve) run concurrently too: no two of them may conflict.
#include <algorithm>
#include <array>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "dd_internal.h"
#include "plan.h"

namespace dd {
namespace {

enum Space { SP_A = 0, SP_W0 = 1, SP_W1 = 2, SP_PIV = 3, SP_ALL = 4 };

struct Acc {
  int sp;
  int r0, r1, c0, c1;   // half-open row and column ranges
  bool w;
};

using FrontAcc = std::map<int, std::vector<Acc>>;

bool tracked(int kind) {
  return kind == L_SYRK || kind == L_SYRK2 || kind == L_PANEL || kind == L_TRSM || kind == L_UPDPANEL ||
         kind == L_ZREC1 || kind == L_ZREC2 || kind == L_STORE;
}

// Read and write sets of one work item of a tracked launch kind (all in the
// item's front).
void item_accesses(const Plan &P, const Launch &L, const Item &it, std::vector<Acc> &v) {
  const FrontDev &d = P.fronts[it.f];
  const int n = d.n;
  if (L.kind == L_UPDPANEL && it.i < 0) {
    // pivot tile k with its diagonal block's column update by the outer
    // block starting at o; rows past a last, short tile get that update
    const int k = it.k, o = it.j, b = std::min(NB, d.s - k);
    const int wb = (o / KBLK) & 1 ? SP_W1 : SP_W0;
    v.push_back({SP_A, k, std::min(k + NB, n), o, k, false});
    v.push_back({wb, k, k + b, 0, k - o, false});
    v.push_back({SP_A, k, std::min(k + NB, n), k, k + b, true});
    v.push_back({SP_PIV, k, k + b, 0, 1, true});
  } else if (L.kind == L_SYRK || L.kind == L_SYRK2 || L.kind == L_UPDPANEL) {
    // A[r, q] -= sum_kk L[r, kk] W[q, kk - k]: a column update of the pivot
    // tile q0 (q0 inside the outer block) or a trailing tile
    const int ts = L.kind == L_SYRK2 ? 128 : 64;
    const int k = it.k, r0 = it.i, q0 = it.j, bend = std::min(k + KBLK, d.s);
    const bool colupd = q0 < bend;
    const int kend = colupd ? q0 : bend, qend = colupd ? std::min(q0 + NB, d.s) : n;
    const int r1 = std::min(r0 + ts, n), q1 = std::min(q0 + ts, qend);
    const int wb = (k / KBLK) & 1 ? SP_W1 : SP_W0;
    v.push_back({SP_A, r0, r1, k, kend, false});
    v.push_back({wb, q0, q1, 0, kend - k, false});
    v.push_back({SP_A, r0, r1, q0, q1, true});
  } else if (L.kind == L_PANEL) {
    const int k = it.k, b = std::min(NB, d.s - k);
    v.push_back({SP_A, k, k + b, k, k + b, true});
    v.push_back({SP_PIV, k, k + b, 0, 1, true});
  } else if (L.kind == L_ZREC1) {
    // split at m0: T1 = L21 Z11 for output rows [r0, r0 + GT) and columns
    // [c0, c0 + GT), written transposed into the upper triangle
    const int m0 = it.k, r0 = it.i, c0 = it.j, r1 = std::min(r0 + GT, d.s), c1 = std::min(c0 + GT, m0);
    v.push_back({SP_A, r0, r1, c0, m0, false});   // stored rows of L21
    v.push_back({SP_PIV, r0, r1, 0, 1, false});
    v.push_back({SP_A, c0, m0, c0, c1, false});   // Z11
    v.push_back({SP_A, c0, c1, r0, r1, true});    // T1^T
  } else if (L.kind == L_ZREC2) {
    // Z21 = -Z22 T1 for output rows [r0, r0 + GT) and columns [c0, c0 + GT)
    const int m0 = it.k, r0 = it.i, c0 = it.j, r1 = std::min(r0 + GT, d.s), c1 = std::min(c0 + GT, m0);
    v.push_back({SP_A, r0, r1, m0, r1, false});   // Z22
    v.push_back({SP_A, c0, c1, m0, r1, false});   // T1^T
    v.push_back({SP_A, r0, r1, c0, c1, true});    // Z21
  } else if (L.kind == L_STORE) {
    // factor columns [k, k + 16) read into the stored-factor region, which
    // no other kernel of the factorisation touches
    v.push_back({SP_A, 0, n, it.k, std::min(it.k + 16, d.s), false});
  } else {
    // W = A21 P^T L11^-T and L21 for rows [r0, r0 + GT) of pivot tile k
    const int k = it.k, r0 = it.i, j = it.j, b = std::min(NB, d.s - k);
    const int r1 = std::min(r0 + GT, n);
    const int wb = ((k - j) / KBLK) & 1 ? SP_W1 : SP_W0;
    v.push_back({SP_A, k, k + b, k, k + b, false});
    v.push_back({SP_PIV, k, k + b, 0, 1, false});
    v.push_back({SP_A, r0, r1, k, k + b, true});
    v.push_back({wb, r0, r1, j, j + b, true});
  }
}

// Read and write sets of one launch, per front (front -1: everything).
FrontAcc accesses(const Plan &P, const Launch &L) {
  FrontAcc out;
  if (!tracked(L.kind)) {
    out[-1].push_back({SP_ALL, 0, 0, 0, 0, true});
    return out;
  }
  for (int64_t x = 0; x < L.count; ++x) {
    const Item &it = P.items[L.first + x];
    item_accesses(P, L, it, out[it.f]);
  }
  return out;
}

bool clash(const Acc &a, const Acc &b) {
  if (a.sp == SP_ALL || b.sp == SP_ALL) return true;
  if (a.sp != b.sp || !(a.w || b.w)) return false;
  return a.r0 < b.r1 && b.r0 < a.r1 && a.c0 < b.c1 && b.c0 < a.c1;
}

// first conflicting pair of two launches' access sets, or false
bool conflict(const FrontAcc &a, const FrontAcc &b, int *front) {
  for (const auto &ka : a) {
    for (const auto &kb : b) {
      if (ka.first != -1 && kb.first != -1 && ka.first != kb.first) continue;
      for (const Acc &x : ka.second)
        for (const Acc &y : kb.second)
          if (clash(x, y)) {
            *front = ka.first >= 0 ? ka.first : kb.first;
            return true;
          }
    }
  }
  return false;
}

}  // namespace

std::string check_schedule(const Plan &P, const std::vector<Launch> &seq) {
  constexpr int NS = 3;
  using VC = std::array<int64_t, NS>;
  VC clk[NS] = {};
  struct Ev {
    int st;
    size_t pos;   // index in seq
    VC vc;
    FrontAcc acc;
  };
  std::vector<Ev> ev;
  std::vector<size_t> by_stream[NS];   // indices into ev
  for (size_t j = 0; j < seq.size(); ++j) {
    const Launch &L = seq[j];
    if (L.side < 0 || L.side >= NS) return "launch " + std::to_string(j) + ": bad stream";
    if (L.kind == L_FORK || L.kind == L_JOIN) {
      if (L.side == 0) return "sync point " + std::to_string(j) + " on the main stream";
      const int x = L.side;
      VC &to = L.kind == L_FORK ? clk[x] : clk[0];
      const VC &from = L.kind == L_FORK ? clk[0] : clk[x];
      for (int i = 0; i < NS; ++i) to[i] = std::max(to[i], from[i]);
      continue;
    }
    if (L.kind == L_PANEL || L.kind == L_TRSM || L.kind == L_UPDPANEL) {
      // the work items of one pivot-chain launch run concurrently
      std::map<int, std::vector<std::vector<Acc>>> per;
      for (int64_t x = 0; x < L.count; ++x) {
        const Item &it = P.items[L.first + x];
        per[it.f].emplace_back();
        item_accesses(P, L, it, per[it.f].back());
      }
      for (const auto &kv : per)
        for (size_t a = 0; a < kv.second.size(); ++a)
          for (size_t b = a + 1; b < kv.second.size(); ++b)
            for (const Acc &x : kv.second[a])
              for (const Acc &y : kv.second[b])
                if (clash(x, y))
                  return "launch " + std::to_string(j) + " (kind " + std::to_string(L.kind) +
                         "): work items of front " + std::to_string(kv.first) + " conflict";
    }
    const int st = L.side;
    clk[st][st]++;
    Ev e{st, j, clk[st], accesses(P, L)};
    // every earlier launch of another stream that does not happen before this one
    for (int s = 0; s < NS; ++s) {
      if (s == st) continue;
      for (size_t q = by_stream[s].size(); q-- > 0;) {
        const Ev &a = ev[by_stream[s][q]];
        if (a.vc[s] <= e.vc[s]) break;   // a (and all before it on s) happen before e
        int front = -1;
        if (conflict(a.acc, e.acc, &front)) {
          char msg[256];
          snprintf(msg, sizeof msg,
                   "unordered launches %zu (kind %d, stream %d) and %zu (kind %d, stream %d) touch front %d",
                   a.pos, seq[a.pos].kind, a.st, j, L.kind, st, front);
          return msg;
        }
      }
    }
    by_stream[st].push_back(ev.size());
    ev.push_back(std::move(e));
  }
  for (int s = 1; s < NS; ++s)
    for (int i = 0; i < NS; ++i)
      if (clk[s][i] > clk[0][i]) return "side stream " + std::to_string(s) + " not joined at the end";
  return std::string();
}

std::string check_layout(const Plan &P) {
  const int nf = (int)P.fronts.size();
  if ((int)P.front_lev.size() != nf || (int)P.front_last.size() != nf) return "layout: levels missing";
  using R = std::pair<int64_t, int64_t>;   // [begin, end) in T elements
  auto overlap = [](std::vector<std::pair<R, int>> v, const char *what) -> std::string {
    std::sort(v.begin(), v.end());
    for (size_t i = 1; i < v.size(); ++i)
      if (v[i].first.first < v[i - 1].first.second)
        return std::string("layout: ") + what + " of fronts " + std::to_string(v[i - 1].second) + " and " +
               std::to_string(v[i].second) + " overlap";
    return std::string();
  };
  // stored factors and interface inverses: disjoint, below the W scratch
  std::vector<std::pair<R, int>> st;
  for (int f = 0; f < nf; ++f) {
    const FrontDev &d = P.fronts[f];
    if (d.kind == FK_GAMMA) st.push_back({{d.xoff, d.xoff + 2 * (int64_t)d.s * d.s}, f});
    else st.push_back({{d.loff, d.loff + d.lpim + (d.lpim == (int64_t)d.n * d.n ? (int64_t)d.n * d.n : (int64_t)d.n * d.s)}, f});
  }
  std::string m = overlap(st, "stored factors");
  if (!m.empty()) return m;
  for (auto &x : st)
    if (x.first.first < 0 || x.first.second > P.e_stored) return "layout: stored factor outside its region";
  // the backward sweep's parent-row map inverts the parent's extend-add map:
  // update row j of child c sits in row urow[c.uoff + j - c.s] of its parent,
  // whose map sends that row back to j - c.s
  for (int p = 0; p < nf; ++p) {
    const FrontDev &d = P.fronts[p];
    for (int ch = 0; ch < d.nchild; ++ch) {
      const int c = P.child_front[d.child + ch];
      const FrontDev &cd = P.fronts[c];
      if (cd.parent != p) return "layout: child " + std::to_string(c) + " names another parent";
      const int64_t rb = P.child_rmap[d.child + ch];
      if (cd.uoff < 0 || cd.uoff + (cd.n - cd.s) > (int64_t)P.urow.size()) return "layout: parent-row map out of range";
      for (int j = cd.s; j < cd.n; ++j) {
        const int32_t pp = P.urow[cd.uoff + j - cd.s];
        if (pp < 0 || pp >= d.n || P.rmap[rb + pp] != j - cd.s)
          return "layout: parent-row map of front " + std::to_string(c) + " does not invert the extend-add map";
      }
    }
  }
  for (int f = 0; f < nf; ++f)
    if (P.fronts[f].n > P.fronts[f].s && P.fronts[f].parent < 0) return "layout: update rows without a parent";
  int nlev = 0;
  for (int f = 0; f < nf; ++f) nlev = std::max(nlev, P.front_last[f] + 1);
  for (int l = 0; l < nlev; ++l) {
    std::vector<std::pair<R, int>> live, w;
    for (int f = 0; f < nf; ++f) {
      const FrontDev &d = P.fronts[f];
      if (P.front_lev[f] == l) {
        const int64_t wb = (((2 * (int64_t)d.n * d.wcols) + 63) & ~(int64_t)63) + d.wstride;
        w.push_back({{d.woff, d.woff + wb}, f});
        if (d.woff < P.e_stored || d.woff + wb > P.e_stored + P.e_w) return "layout: W outside its region";
      }
      if (P.front_lev[f] > l || P.front_last[f] < l) continue;
      if (d.loff == d.off && d.kind != FK_GAMMA) continue;   // kept whole: a stored factor
      const int64_t arena = P.e_stored + P.e_w;
      const R r{d.off, d.off + 2 * (int64_t)d.n * d.n};
      if (r.first < arena || r.second > arena + P.e_arena_factor) return "layout: front outside the arena";
      live.push_back({r, f});
    }
    m = overlap(live, ("live front matrices at level " + std::to_string(l)).c_str());
    if (!m.empty()) return m;
    m = overlap(w, ("W scratch at level " + std::to_string(l)).c_str());
    if (!m.empty()) return m;
  }
  return std::string();
}

}  // namespace dd
