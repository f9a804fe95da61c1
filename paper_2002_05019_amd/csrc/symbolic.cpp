// Symbolic phase of the DD solver (host only, no GPU call).
//
// * Domain matrices: nested-dissection ordering of the interior DoFs with the
//   interface DoFs (those carrying a multiplier) eliminated last, as the root
//   front; multifrontal tree, update-row sets and extend-add maps.
// * Auxiliary matrix F = sum_i B_i K_i^-1 B_i^T (paper, section II): its
//   nonzero structure is the union of one clique per domain on the domain's
//   multipliers.  Multipliers shared by the same pair of domains are
//   indistinguishable, so they are grouped into blocks; the symbolic
//   factorisation runs on the (much smaller) block graph and every front is a
//   union of whole dense blocks.
// * The launch schedule of the numeric phases and the workspace layout.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <utility>

#include "plan.h"

namespace dd {

// ----------------------------------------------------------------------------
// validation
std::string validate_problem(const ProblemView &p, int *code) {
  char buf[512];
  *code = -1;
  if (p.n_dom < 1) return "n_dom must be >= 1";
  if (p.n_mult < 0) return "n_mult must be >= 0";
  if (p.n_mult > 0x3fffffff) return "n_mult too large";
  for (int i = 0; i < p.n_dom; ++i) {
    const int32_t n = p.n[i];
    if (n < 0) { snprintf(buf, sizeof buf, "domain %d: negative size", i); return buf; }
    if (!p.rowptr[i] || (p.nnz[i] > 0 && !p.colind[i])) {
      snprintf(buf, sizeof buf, "domain %d: null pattern pointer", i);
      return buf;
    }
    *code = -2;
    const int64_t *rp = p.rowptr[i];
    const int32_t *ci = p.colind[i];
    if (rp[0] != 0 || rp[n] != p.nnz[i]) {
      snprintf(buf, sizeof buf, "domain %d: rowptr[0] must be 0 and rowptr[n] = nnz", i);
      return buf;
    }
    std::vector<int64_t> cnt(n, 0);
    for (int32_t r = 0; r < n; ++r) {
      if (rp[r + 1] < rp[r]) { snprintf(buf, sizeof buf, "domain %d: rowptr decreases at row %d", i, r); return buf; }
      bool diag = false;
      for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
        int32_t c = ci[e];
        if (c < 0 || c >= n) { snprintf(buf, sizeof buf, "domain %d: column %d out of range in row %d", i, c, r); return buf; }
        if (e > rp[r] && ci[e - 1] >= c) { snprintf(buf, sizeof buf, "domain %d: columns not strictly increasing in row %d", i, r); return buf; }
        if (c == r) diag = true;
        cnt[c]++;
      }
      if (!diag) { snprintf(buf, sizeof buf, "domain %d: missing diagonal in row %d", i, r); return buf; }
    }
    for (int32_t r = 0; r < n; ++r) {
      if (cnt[r] != rp[r + 1] - rp[r]) { snprintf(buf, sizeof buf, "domain %d: pattern not symmetric (row %d)", i, r); return buf; }
      for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
        int32_t c = ci[e];
        if (!std::binary_search(ci + rp[c], ci + rp[c + 1], r)) {
          snprintf(buf, sizeof buf, "domain %d: pattern not symmetric (%d,%d)", i, r, c);
          return buf;
        }
      }
    }
  }
  *code = -3;
  if (p.n_mult > 0 && (!p.imap_ptr || !p.imap_dof || !p.imap_mult || !p.imap_sign))
    return "interface map pointers must be non-null";
  if (!p.imap_ptr) return p.n_mult == 0 ? (*code = 0, std::string()) : std::string("null imap_ptr");
  if (p.imap_ptr[0] != 0) return "imap_ptr[0] must be 0";
  std::vector<int32_t> mcnt(p.n_mult, 0), mdom(p.n_mult, -1);
  for (int i = 0; i < p.n_dom; ++i) {
    if (p.imap_ptr[i + 1] < p.imap_ptr[i]) return "imap_ptr decreases";
    for (int64_t e = p.imap_ptr[i]; e < p.imap_ptr[i + 1]; ++e) {
      int32_t d = p.imap_dof[e];
      int64_t m = p.imap_mult[e];
      int s = p.imap_sign[e];
      if (d < 0 || d >= p.n[i]) { snprintf(buf, sizeof buf, "interface entry %lld: dof %d out of range for domain %d", (long long)e, d, i); return buf; }
      if (m < 0 || m >= p.n_mult) { snprintf(buf, sizeof buf, "interface entry %lld: multiplier %lld out of range", (long long)e, (long long)m); return buf; }
      if (s != 1 && s != -1) { snprintf(buf, sizeof buf, "interface entry %lld: sign must be +1 or -1", (long long)e); return buf; }
      if (mdom[m] == i) { snprintf(buf, sizeof buf, "multiplier %lld appears twice in domain %d", (long long)m, i); return buf; }
      mdom[m] = i;
      mcnt[m]++;
    }
  }
  for (int64_t m = 0; m < p.n_mult; ++m)
    if (mcnt[m] != 2) {
      snprintf(buf, sizeof buf, "multiplier %lld has %d entries (needs exactly 2)", (long long)m, mcnt[m]);
      return buf;
    }
  *code = 0;
  return std::string();
}

// ----------------------------------------------------------------------------
// nested dissection on a CSR graph (self loops ignored)
namespace {

struct NdGraph {
  int n = 0;
  const int64_t *ptr = nullptr;
  const int32_t *col = nullptr;
  const double *xyz = nullptr;   // 3 per vertex or null
  const double *w = nullptr;     // vertex weights or null (= 1)
};

struct NdTree {
  std::vector<std::vector<int>> vars;
  std::vector<std::vector<int>> kids;
  int add(std::vector<int> v, std::vector<int> k) {
    vars.push_back(std::move(v));
    kids.push_back(std::move(k));
    return (int)vars.size() - 1;
  }
};

class Dissector {
 public:
  Dissector(const NdGraph &g, double leaf_w) : G(g), leaf(leaf_w), stamp(g.n, 0), side(g.n, 0), lev(g.n, -1) {}

  std::vector<int> run(std::vector<int> &V, NdTree &T) {
    double wV = weight(V);
    if (V.size() <= 1 || wV <= leaf) return {T.add(V, {})};
    std::vector<int> L, S, R;
    bool ok = G.xyz && plane_split(V, L, S, R);
    if (!ok) ok = level_split(V, L, S, R);
    if (!ok) return {T.add(V, {})};
    std::vector<int> kids;
    if (!L.empty()) {
      auto a = run(L, T);
      kids.insert(kids.end(), a.begin(), a.end());
    }
    if (!R.empty()) {
      auto b = run(R, T);
      kids.insert(kids.end(), b.begin(), b.end());
    }
    if (S.empty()) return kids;
    std::sort(S.begin(), S.end());
    return {T.add(S, kids)};
  }

 private:
  const NdGraph &G;
  double leaf;
  std::vector<int> stamp;
  std::vector<int8_t> side;
  std::vector<int> lev;
  int cur = 0;

  double wt(int v) const { return G.w ? G.w[v] : 1.0; }
  double weight(const std::vector<int> &V) const {
    double s = 0;
    for (int v : V) s += wt(v);
    return s;
  }
  void mark(const std::vector<int> &V) {
    ++cur;
    for (int v : V) stamp[v] = cur;
  }

  // Plane separator on the coordinates: the vertices lying exactly on an
  // axis-aligned plane, if no edge crosses the plane.
  bool plane_split(const std::vector<int> &V, std::vector<int> &L, std::vector<int> &S, std::vector<int> &R) {
    mark(V);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v : V)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], G.xyz[3 * v + a]);
        hi[a] = std::max(hi[a], G.xyz[3 * v + a]);
      }
    int axes[3] = {0, 1, 2};
    std::sort(axes, axes + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
    const double wV = weight(V);
    for (int ai = 0; ai < 3; ++ai) {
      const int ax = axes[ai];
      if (hi[ax] - lo[ax] <= 0) break;
      std::vector<std::pair<double, double>> xs;  // (coord, weight)
      xs.reserve(V.size());
      for (int v : V) xs.push_back({G.xyz[3 * v + ax], wt(v)});
      std::sort(xs.begin(), xs.end());
      // cumulative weights at distinct values
      std::vector<double> vals, wbelow, won;
      double acc = 0;
      for (size_t i = 0; i < xs.size();) {
        size_t j = i;
        double wo = 0;
        while (j < xs.size() && xs[j].first == xs[i].first) wo += xs[j++].second;
        vals.push_back(xs[i].first);
        wbelow.push_back(acc);
        won.push_back(wo);
        acc += wo;
        i = j;
      }
      // candidates: balanced planes, closest to the weighted median first
      std::vector<std::pair<double, int>> cand;
      for (size_t u = 0; u < vals.size(); ++u) {
        double wl = wbelow[u], wr = wV - wbelow[u] - won[u];
        if (wl >= 0.15 * wV && wr >= 0.15 * wV) cand.push_back({std::fabs(wl - wr) / wV, (int)u});
      }
      std::sort(cand.begin(), cand.end());
      int best = -1;
      double best_score = 1e300;
      int tried = 0;
      for (auto &c : cand) {
        if (tried++ >= 8) break;
        const double u = vals[c.second];
        bool sep = true;
        for (int v : V) {
          if (G.xyz[3 * v + ax] >= u) continue;
          for (int64_t e = G.ptr[v]; e < G.ptr[v + 1] && sep; ++e) {
            int w = G.col[e];
            if (w != v && stamp[w] == cur && G.xyz[3 * w + ax] > u) sep = false;
          }
          if (!sep) break;
        }
        if (!sep) continue;
        double score = won[c.second] * (1.0 + c.first);
        if (score < best_score) {
          best_score = score;
          best = c.second;
        }
      }
      if (best >= 0) {
        const double u = vals[best];
        L.clear(); S.clear(); R.clear();
        for (int v : V) {
          double x = G.xyz[3 * v + ax];
          (x < u ? L : (x > u ? R : S)).push_back(v);
        }
        return true;
      }
    }
    return false;
  }

  int bfs(const std::vector<int> &V, int src, std::vector<int> &order) {
    // BFS inside the marked set; lev[] holds levels; returns depth
    order.clear();
    for (int v : V) lev[v] = -1;
    lev[src] = 0;
    order.push_back(src);
    for (size_t h = 0; h < order.size(); ++h) {
      int v = order[h];
      for (int64_t e = G.ptr[v]; e < G.ptr[v + 1]; ++e) {
        int w = G.col[e];
        if (stamp[w] == cur && lev[w] < 0) {
          lev[w] = lev[v] + 1;
          order.push_back(w);
        }
      }
    }
    return lev[order.back()];
  }

  // Level-set separator of a BFS from a pseudo-peripheral vertex.
  bool level_split(const std::vector<int> &V, std::vector<int> &L, std::vector<int> &S, std::vector<int> &R) {
    mark(V);
    std::vector<int> order;
    bfs(V, V[0], order);
    L.clear(); S.clear(); R.clear();
    if (order.size() < V.size()) {           // disconnected: split off one component
      for (int v : V) (lev[v] >= 0 ? L : R).push_back(v);
      return true;
    }
    int far = order.back();
    for (int it = 0; it < 2; ++it) {
      bfs(V, far, order);
      far = order.back();
    }
    int D = lev[order.back()];
    if (D < 2) return false;
    std::vector<double> wl(D + 1, 0.0);
    for (int v : V) wl[lev[v]] += wt(v);
    const double wV = weight(V);
    double below = 0;
    int best = -1;
    double best_score = 1e300;
    for (int l = 0; l <= D; ++l) {
      double after = wV - below - wl[l];
      if (l >= 1 && l <= D - 1) {
        double imb = std::fabs(below - after) / wV;
        bool balanced = below >= 0.2 * wV && after >= 0.2 * wV;
        double score = wl[l] * (1.0 + imb) + (balanced ? 0.0 : 1e200 * imb);
        if (score < best_score) {
          best_score = score;
          best = l;
        }
      }
      below += wl[l];
    }
    if (best < 0) return false;
    for (int v : V) (lev[v] < best ? L : (lev[v] > best ? R : S)).push_back(v);
    return true;
  }
};

// Multifrontal symbolic factorisation of an elimination forest given by
// NdTree nodes: postorder, ranks, and the update rows of every node.
struct Symb {
  std::vector<int> post;                  // node ids in postorder
  std::vector<int> parent;                // per node
  std::vector<int> rank;                  // per unit
  std::vector<std::vector<int>> rows;     // per node, sorted by rank
  std::vector<int> height;                // per node
};

void symbolic(const NdTree &T, const std::vector<int> &roots, int nunits, const int64_t *ptr,
              const int32_t *col, Symb &S) {
  const int nn = (int)T.vars.size();
  S.parent.assign(nn, -1);
  S.height.assign(nn, 0);
  S.rows.assign(nn, {});
  S.rank.assign(nunits, -1);
  S.post.clear();
  for (int v = 0; v < nn; ++v)
    for (int k : T.kids[v]) S.parent[k] = v;
  // iterative postorder
  std::vector<std::pair<int, size_t>> st;
  for (int r : roots) {
    st.push_back({r, 0});
    while (!st.empty()) {
      auto &top = st.back();
      if (top.second < T.kids[top.first].size()) {
        int k = T.kids[top.first][top.second++];
        st.push_back({k, 0});
      } else {
        S.post.push_back(top.first);
        st.pop_back();
      }
    }
  }
  int rk = 0;
  for (int v : S.post)
    for (int u : T.vars[v]) S.rank[u] = rk++;
  std::vector<int> stamp(nunits, -1);
  for (int v : S.post) {
    int maxr = -1;
    for (int u : T.vars[v]) maxr = std::max(maxr, S.rank[u]);
    std::vector<int> R;
    auto consider = [&](int w) {
      if (S.rank[w] > maxr && stamp[w] != v) {
        stamp[w] = v;
        R.push_back(w);
      }
    };
    for (int u : T.vars[v])
      for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) consider(col[e]);
    int h = 0;
    for (int k : T.kids[v]) {
      for (int w : S.rows[k]) consider(w);
      h = std::max(h, S.height[k] + 1);
    }
    S.height[v] = h;
    std::sort(R.begin(), R.end(), [&](int a, int b) { return S.rank[a] < S.rank[b]; });
    S.rows[v] = std::move(R);
  }
}

inline int ntiles(int x, int t) { return (x + t - 1) / t; }

}  // namespace

// ----------------------------------------------------------------------------
std::string build_plan(const ProblemView &p, const SetupOptions &o, Plan &P) {
  P = Plan();
  P.n_dom = p.n_dom;
  P.n_mult = p.n_mult;
  P.precision = o.precision;
  P.max_rhs = o.max_rhs;
  // default Schur-update tiles: 64 below 1024, 128 from 1024 on
  for (int bkt = 0; bkt < TILE_BUCKETS; ++bkt) {
    const int t = o.schur_tile[bkt];
    P.schur_tile[bkt] = t == 64 || t == 128 ? t : (bkt >= 2 ? 128 : 64);
  }
  P.elem = o.precision == 0 ? sizeof(double) : sizeof(float);
  P.dom_n.assign(p.n.begin(), p.n.end());
  P.dom_row.resize(p.n_dom + 1);
  P.dom_nnz.resize(p.n_dom + 1);
  P.dom_row[0] = 0;
  P.dom_nnz[0] = 0;
  for (int i = 0; i < p.n_dom; ++i) {
    P.dom_row[i + 1] = P.dom_row[i] + p.n[i];
    P.dom_nnz[i + 1] = P.dom_nnz[i] + p.nnz[i];
  }
  P.n_torn = P.dom_row[p.n_dom];
  P.nnz_total = P.dom_nnz[p.n_dom];
  if (P.n_torn > 0x3fffffff) return "too many torn DoFs";

  // torn-system CSR (for the FP64 residual of the refinement)
  P.csr_ptr.resize(P.n_torn + 1);
  P.csr_col.resize(P.nnz_total);
  for (int i = 0; i < p.n_dom; ++i) {
    for (int32_t r = 0; r <= p.n[i]; ++r) P.csr_ptr[P.dom_row[i] + r] = P.dom_nnz[i] + p.rowptr[i][r];
    for (int64_t e = 0; e < p.nnz[i]; ++e) P.csr_col[P.dom_nnz[i] + e] = (int32_t)(P.dom_row[i] + p.colind[i][e]);
  }
  if (o.precision != 0) {
    const int64_t nsl = (P.n_torn + 63) / 64;
    P.sell_ptr.assign(nsl + 1, 0);
    for (int64_t sl = 0; sl < nsl; ++sl) {
      int64_t w = 0;
      for (int64_t r = sl * 64; r < std::min(P.n_torn, sl * 64 + 64); ++r) w = std::max(w, P.csr_ptr[r + 1] - P.csr_ptr[r]);
      P.sell_ptr[sl + 1] = P.sell_ptr[sl] + 64 * w;
    }
    P.nnz_sell = P.sell_ptr[nsl];
    P.sell_col.assign(P.nnz_sell, 0);
    for (int64_t r = 0; r < P.n_torn; ++r) {
      const int64_t base = P.sell_ptr[r / 64] + (r % 64);
      for (int64_t k = 0; k < P.csr_ptr[r + 1] - P.csr_ptr[r]; ++k) P.sell_col[base + 64 * k] = P.csr_col[P.csr_ptr[r] + k];
    }
  }

  // interface dofs per domain (sorted) and the multiplier entries
  P.gamma.assign(p.n_dom, {});
  std::vector<int32_t> m_dom(2 * p.n_mult), m_dof(2 * p.n_mult), m_sg(2 * p.n_mult), m_fill(p.n_mult, 0);
  for (int i = 0; i < p.n_dom; ++i) {
    auto &g = P.gamma[i];
    for (int64_t e = p.imap_ptr ? p.imap_ptr[i] : 0; e < (p.imap_ptr ? p.imap_ptr[i + 1] : 0); ++e) {
      g.push_back(p.imap_dof[e]);
      int64_t m = p.imap_mult[e];
      int slot = m_fill[m]++;
      m_dom[2 * m + slot] = i;
      m_dof[2 * m + slot] = p.imap_dof[e];
      m_sg[2 * m + slot] = p.imap_sign[e];
    }
    std::sort(g.begin(), g.end());
    g.erase(std::unique(g.begin(), g.end()), g.end());
  }
  // order the two entries of each multiplier by domain
  for (int64_t m = 0; m < p.n_mult; ++m)
    if (m_dom[2 * m] > m_dom[2 * m + 1]) {
      std::swap(m_dom[2 * m], m_dom[2 * m + 1]);
      std::swap(m_dof[2 * m], m_dof[2 * m + 1]);
      std::swap(m_sg[2 * m], m_sg[2 * m + 1]);
    }
  auto gpos_of = [&](int d, int dof) {
    auto &g = P.gamma[d];
    return (int32_t)(std::lower_bound(g.begin(), g.end(), dof) - g.begin());
  };

  // ------------------------------------------------------------ domain trees
  struct FH {
    int kind, dom, height, parent = -1;
    std::vector<int> vars, rows, kids;
  };
  std::vector<FH> F;
  std::vector<std::vector<int>> dom_fronts(p.n_dom);
  P.gamma_front.assign(p.n_dom, -1);
  std::vector<double> xyzd;
  for (int i = 0; i < p.n_dom; ++i) {
    const int n = p.n[i];
    NdGraph G;
    G.n = n;
    G.ptr = p.rowptr[i];
    G.col = p.colind[i];
    if (p.xyz) {
      xyzd.resize(3 * (size_t)n);
      for (int64_t k = 0; k < 3 * (int64_t)n; ++k) xyzd[k] = p.xyz[3 * P.dom_row[i] + k];
      G.xyz = xyzd.data();
    }
    std::vector<char> isg(n, 0);
    for (int d : P.gamma[i]) isg[d] = 1;
    std::vector<int> interior;
    for (int v = 0; v < n; ++v)
      if (!isg[v]) interior.push_back(v);
    NdTree T;
    Dissector D(G, (double)o.leaf);
    std::vector<int> roots;
    if (!interior.empty()) roots = D.run(interior, T);
    if (!P.gamma[i].empty()) {
      std::vector<int> g(P.gamma[i].begin(), P.gamma[i].end());
      roots = {T.add(g, roots)};
    }
    Symb S;
    symbolic(T, roots, n, p.rowptr[i], p.colind[i], S);
    // verify the separator property: every child's update rows sit in its parent front
    std::vector<int> id(T.vars.size());
    for (int v : S.post) {
      id[v] = (int)F.size();
      FH f;
      f.kind = (!P.gamma[i].empty() && v == roots[0]) ? FK_GAMMA : FK_INTERIOR;
      f.dom = i;
      f.height = S.height[v];
      f.vars = T.vars[v];
      f.rows = S.rows[v];
      F.push_back(std::move(f));
      dom_fronts[i].push_back(id[v]);
    }
    for (int v : S.post) {
      for (int k : T.kids[v]) {
        F[id[v]].kids.push_back(id[k]);
        F[id[k]].parent = id[v];
      }
    }
    if (!P.gamma[i].empty()) {
      P.gamma_front[i] = id[roots[0]];
      if (!F[id[roots[0]]].rows.empty()) return "internal: interface root has update rows";
    }
  }
  const int n_dom_fronts = (int)F.size();

  // ------------------------------------------------------------ aux block graph
  std::map<std::pair<int, int>, int> bkey;
  std::vector<std::vector<int32_t>> bmult;       // multipliers of each block
  std::vector<std::array<int, 2>> bdom;
  std::vector<int> mblock(p.n_mult);
  for (int64_t m = 0; m < p.n_mult; ++m) {
    auto key = std::make_pair(m_dom[2 * m], m_dom[2 * m + 1]);
    auto it = bkey.find(key);
    int b;
    if (it == bkey.end()) {
      b = (int)bmult.size();
      bkey[key] = b;
      bmult.push_back({});
      bdom.push_back({key.first, key.second});
    } else {
      b = it->second;
    }
    bmult[b].push_back((int32_t)m);
    mblock[m] = b;
  }
  const int nb = (int)bmult.size();
  // block adjacency: share a domain
  std::vector<std::vector<int>> dom_blocks(p.n_dom);
  for (int b = 0; b < nb; ++b) {
    dom_blocks[bdom[b][0]].push_back(b);
    dom_blocks[bdom[b][1]].push_back(b);
  }
  std::vector<int64_t> bptr(nb + 1, 0);
  std::vector<int32_t> bcol;
  {
    std::vector<int> st(nb, -1);
    for (int b = 0; b < nb; ++b) {
      for (int s = 0; s < 2; ++s)
        for (int c : dom_blocks[bdom[b][s]])
          if (st[c] != b) {
            st[c] = b;
            bcol.push_back(c);
          }
      bptr[b + 1] = (int64_t)bcol.size();
    }
  }
  std::vector<double> bw(nb), bxyz;
  for (int b = 0; b < nb; ++b) bw[b] = (double)bmult[b].size();
  if (p.xyz) {
    bxyz.assign(3 * (size_t)nb, 0.0);
    for (int b = 0; b < nb; ++b) {
      for (int32_t m : bmult[b]) {
        int d = m_dom[2 * m], dof = m_dof[2 * m];
        for (int a = 0; a < 3; ++a) bxyz[3 * b + a] += p.xyz[3 * (P.dom_row[d] + dof) + a];
      }
      for (int a = 0; a < 3; ++a) bxyz[3 * b + a] /= (double)bmult[b].size();
    }
  }
  std::vector<int> aux_first(nb, 0);
  if (nb > 0) {
    NdGraph G;
    G.n = nb;
    G.ptr = bptr.data();
    G.col = bcol.data();
    G.xyz = p.xyz ? bxyz.data() : nullptr;
    G.w = bw.data();
    NdTree T;
    Dissector D(G, (double)o.aux_leaf);
    std::vector<int> all(nb);
    std::iota(all.begin(), all.end(), 0);
    std::vector<int> roots = D.run(all, T);
    Symb S;
    symbolic(T, roots, nb, bptr.data(), bcol.data(), S);
    std::vector<int> id(T.vars.size());
    for (int v : S.post) {
      id[v] = (int)F.size();
      FH f;
      f.kind = FK_AUX;
      f.dom = -1;
      f.height = S.height[v];
      f.vars = T.vars[v];      // block ids for now
      f.rows = S.rows[v];
      F.push_back(std::move(f));
    }
    for (int v : S.post)
      for (int k : T.kids[v]) {
        F[id[v]].kids.push_back(id[k]);
        F[id[k]].parent = id[v];
      }
  }

  // ------------------------------------------------------------ front descriptors
  const int nf = (int)F.size();
  P.fronts.resize(nf);
  // block position bookkeeping for aux fronts: unit lists (blocks) kept aside
  std::vector<std::vector<int>> aux_units(nf);
  for (int f = 0; f < nf; ++f) {
    FH &h = F[f];
    FrontDev &d = P.fronts[f];
    std::memset(&d, 0, sizeof d);
    d.kind = h.kind;
    d.dom = h.dom;
    d.xoff = -1;
    d.goff = -1;
    d.idx = (int64_t)P.vars.size();
    if (h.kind == FK_AUX) {
      std::vector<int> units(h.vars);
      units.insert(units.end(), h.rows.begin(), h.rows.end());
      int s = 0;
      for (int b : h.vars) s += (int)bmult[b].size();
      int n = 0;
      for (int b : units) {
        for (int32_t m : bmult[b]) P.vars.push_back(m);
        n += (int)bmult[b].size();
      }
      d.s = s;
      d.n = n;
      d.vbase = 0;
      aux_units[f] = std::move(units);
    } else {
      d.s = (int)h.vars.size();
      d.n = d.s + (int)h.rows.size();
      for (int v : h.vars) P.vars.push_back(v);
      for (int v : h.rows) P.vars.push_back(v);
      d.vbase = P.dom_row[h.dom];
    }
    // W: factorisation scratch (one outer block of columns, at most KBLK);
    // fronts substituted through Z = L11^-1 also keep one intermediate
    // column per right-hand side there
    d.wcols = std::max(NB, std::min(KBLK, (d.s + NB - 1) / NB * NB));
    if (h.kind != FK_GAMMA && d.n > FUSE_N) d.wcols = std::max<int32_t>(d.wcols, P.max_rhs);
  }
  // children + reverse extend-add maps, and each child's parent rows
  {
    std::vector<int32_t> pos;
    for (int f = 0; f < nf; ++f) {
      P.fronts[f].parent = -1;
      P.fronts[f].uoff = 0;
    }
    for (int f = 0; f < nf; ++f) {
      FrontDev &d = P.fronts[f];
      d.child = (int64_t)P.child_front.size();
      d.nchild = (int)F[f].kids.size();
      if (d.nchild == 0) continue;
      // position of every variable in this front
      const int32_t *fv = &P.vars[d.idx];
      std::map<int32_t, int32_t> small;
      int32_t maxv = 0;
      for (int r = 0; r < d.n; ++r) maxv = std::max(maxv, fv[r]);
      pos.assign((size_t)maxv + 1, -1);
      for (int r = 0; r < d.n; ++r) pos[fv[r]] = r;
      for (int c : F[f].kids) {
        FrontDev &cd = P.fronts[c];
        P.child_front.push_back(c);
        P.child_rmap.push_back((int64_t)P.rmap.size());
        size_t base = P.rmap.size();
        P.rmap.resize(base + d.n, -1);
        cd.parent = f;
        cd.uoff = (int64_t)P.urow.size();
        const int32_t *cv = &P.vars[cd.idx];
        int prev = -1;
        for (int j = cd.s; j < cd.n; ++j) {
          int32_t v = cv[j];
          int32_t pp = (v <= maxv) ? pos[v] : -1;
          if (pp < 0) return "internal: update row missing in the parent front";
          if (pp <= prev) return "internal: extend-add map not monotone";
          prev = pp;
          P.rmap[base + pp] = j - cd.s;
          P.urow.push_back(pp);
        }
      }
    }
    for (int f = 0; f < nf; ++f)
      if (P.fronts[f].n > P.fronts[f].s && P.fronts[f].parent < 0)
        return "internal: update rows without a parent front";
  }

  // ------------------------------------------------------------ original entries (domain fronts)
  {
    std::vector<int32_t> pos;
    std::vector<int64_t> rank;
    for (int i = 0; i < p.n_dom; ++i) {
      // rank of every dof = position in the postorder concatenation of vars
      rank.assign(p.n[i], -1);
      int64_t rk = 0;
      for (int f : dom_fronts[i]) {
        const FrontDev &d = P.fronts[f];
        for (int r = 0; r < d.s; ++r) rank[P.vars[d.idx + r]] = rk++;
      }
      if (rk != p.n[i]) return "internal: ordering does not cover the domain";
      pos.assign(p.n[i], -1);
      for (int f : dom_fronts[i]) {
        FrontDev &d = P.fronts[f];
        const int32_t *fv = &P.vars[d.idx];
        for (int r = 0; r < d.n; ++r) pos[fv[r]] = r;
        for (int c = 0; c < d.s; ++c) {
          int32_t vc = fv[c];
          for (int64_t e = p.rowptr[i][vc]; e < p.rowptr[i][vc + 1]; ++e) {
            int32_t vr = p.colind[i][e];
            if (rank[vr] < rank[vc]) continue;
            int32_t pr = pos[vr];
            if (pr < c) return "internal: original entry outside its front";
            SPair sp;
            sp.src = P.dom_nnz[i] + e;
            sp.pos = pr + c * d.n;
            sp.pad = 0;
            P.spairs.push_back(sp);
          }
        }
        for (int r = 0; r < d.n; ++r) pos[fv[r]] = -1;
      }
    }
  }
  // pair ranges per front (the pairs of a front are contiguous)
  std::vector<std::pair<int64_t, int64_t>> prange(nf, {0, 0});
  {
    int64_t at = 0;
    std::vector<int64_t> rank;
    for (int i = 0; i < p.n_dom; ++i) {
      rank.assign(p.n[i], -1);
      int64_t rk = 0;
      for (int f : dom_fronts[i]) {
        const FrontDev &d = P.fronts[f];
        for (int r = 0; r < d.s; ++r) rank[P.vars[d.idx + r]] = rk++;
      }
      for (int f : dom_fronts[i]) {
        const FrontDev &d = P.fronts[f];
        int64_t cnt = 0;
        for (int c = 0; c < d.s; ++c) {
          int32_t vc = P.vars[d.idx + c];
          for (int64_t e = p.rowptr[i][vc]; e < p.rowptr[i][vc + 1]; ++e)
            if (rank[p.colind[i][e]] >= rank[vc]) ++cnt;
        }
        prange[f] = {at, cnt};
        at += cnt;
      }
    }
    if (at != (int64_t)P.spairs.size()) return "internal: pair count mismatch";
  }

  // ------------------------------------------------------------ aux gather items
  P.gpos.clear();
  P.gsign.clear();
  // per block and domain slot: offset of (gpos, gsign) arrays
  std::vector<std::array<int64_t, 2>> boff(nb);
  for (int b = 0; b < nb; ++b)
    for (int s = 0; s < 2; ++s) {
      boff[b][s] = (int64_t)P.gpos.size();
      for (int32_t m : bmult[b]) {
        int slot = (m_dom[2 * m] == bdom[b][s]) ? 0 : 1;
        int d = m_dom[2 * m + slot];
        P.gpos.push_back(gpos_of(d, m_dof[2 * m + slot]));
        P.gsign.push_back(m_sg[2 * m + slot]);
      }
    }
  std::vector<std::pair<int64_t, int64_t>> arange(nf, {0, 0});
  for (int f = n_dom_fronts; f < nf; ++f) {
    const auto &units = aux_units[f];
    int nsep = (int)F[f].vars.size();
    std::vector<int> upos(units.size());
    int at = 0;
    for (size_t u = 0; u < units.size(); ++u) {
      upos[u] = at;
      at += (int)bmult[units[u]].size();
    }
    int64_t first = (int64_t)P.aux_items.size();
    for (int ia = 0; ia < nsep; ++ia) {
      int a = units[ia];
      for (size_t ib = ia; ib < units.size(); ++ib) {
        int b = units[ib];
        AuxItem it;
        std::memset(&it, 0, sizeof it);
        it.f = f;
        it.pa = upos[ia];
        it.pb = upos[ib];
        it.na = (int)bmult[a].size();
        it.nb = (int)bmult[b].size();
        it.same = (a == b);
        int nd = 0;
        for (int sa = 0; sa < 2; ++sa)
          for (int sb = 0; sb < 2; ++sb)
            if (bdom[a][sa] == bdom[b][sb]) {
              it.ga[nd] = boff[a][sa];
              it.gb[nd] = boff[b][sb];
              it.xoff[nd] = bdom[a][sa];   // domain id for now; replaced by the X offset in the layout
              ++nd;
            }
        if (nd == 0) continue;
        it.ndom = nd;
        P.aux_items.push_back(it);
      }
    }
    arange[f] = {first, (int64_t)P.aux_items.size() - first};
  }

  // ------------------------------------------------------------ statistics
  double fl = 0, fs = 0, fb = 0;
  for (int f = 0; f < nf; ++f) {
    const FrontDev &d = P.fronts[f];
    double n = d.n, s = d.s, R = n - s;
    fl += 8.0 * (n * n * n - R * R * R) / 6.0;
    fs += 8.0 * (s * s + 2.0 * s * R);
    fb += (s * n - s * s / 2.0) * 2.0 * (double)P.elem;
    if (d.kind == FK_GAMMA) {
      fl += 8.0 * s * s * s / 3.0;
      fs += 8.0 * 2.0 * s * s;
      fb += s * s * 2.0 * (double)P.elem - (s * n - s * s / 2.0) * 2.0 * (double)P.elem;
    }
    if (d.kind != FK_AUX) {
      if (P.dom_flops.empty()) P.dom_flops.assign(p.n_dom, 0.0);
      P.dom_flops[d.dom] += 8.0 * (n * n * n - R * R * R) / 6.0 + (d.kind == FK_GAMMA ? 8.0 * s * s * s / 3.0 : 0.0);
    }
    if (d.kind == FK_AUX) {
      P.n_front_aux++;
      P.max_front_aux = std::max(P.max_front_aux, d.n);
    } else {
      P.n_front_dom++;
      P.max_front_dom = std::max(P.max_front_dom, d.n);
    }
  }
  P.flops_factor = fl;
  P.flops_solve_rhs = fs;
  P.bytes_factor = fb;
  // one solve of one column block reads every stored factor twice (forward
  // and backward sweeps; the interface inverses in the condensation and in
  // the interface correction)
  P.bytes_solve = 2.0 * fb;

  // ------------------------------------------------------------ numeric layout (T elements)
  // Factor order: domain levels by height, the interface roots, auxiliary
  // levels by height (the schedule below uses the same grouping).
  auto by_height = [&](int kind_lo, int kind_hi, bool include_gamma) {
    std::map<int, std::vector<int>> lv;
    for (int f = 0; f < nf; ++f) {
      int k = P.fronts[f].kind;
      if (k == FK_GAMMA && !include_gamma) continue;
      if (k < kind_lo || k > kind_hi) continue;
      lv[F[f].height].push_back(f);
    }
    std::vector<std::vector<int>> out;
    for (auto &kv : lv) out.push_back(kv.second);
    return out;
  };
  std::vector<std::vector<int>> dom_levels = by_height(FK_INTERIOR, FK_INTERIOR, false);
  std::vector<int> gam;
  for (int i = 0; i < p.n_dom; ++i)
    if (P.gamma_front[i] >= 0) gam.push_back(P.gamma_front[i]);
  // domains without interface: their roots are interior fronts already
  std::vector<std::vector<int>> aux_levels = by_height(FK_AUX, FK_AUX, false);
  std::vector<std::vector<int>> levels(dom_levels);
  if (!gam.empty()) levels.push_back(gam);
  levels.insert(levels.end(), aux_levels.begin(), aux_levels.end());
  const int nlev = (int)levels.size();
  std::vector<int> lev(nf, -1);
  for (int l = 0; l < nlev; ++l)
    for (int f : levels[l]) lev[f] = l;
  for (int f = 0; f < nf; ++f)
    if (lev[f] < 0) return "internal: front without a level";
  // a front's full matrix is read by its own level and by its parent's
  // (extend-add of the update block)
  std::vector<int> last_use(nf);
  for (int f = 0; f < nf; ++f) {
    last_use[f] = F[f].parent >= 0 ? lev[F[f].parent] : lev[f];
    if (last_use[f] < lev[f]) return "internal: parent factored before its child";
  }
  P.front_lev = lev;
  P.front_last = last_use;
  // fronts whose full matrix is kept as the stored factor (no update block);
  // interface roots keep only the interface inverse X
  auto kept = [&](int f) { return P.fronts[f].kind != FK_GAMMA && P.fronts[f].n == P.fronts[f].s; };

  const int64_t mr = P.max_rhs;
  int64_t at = 0;
  auto align = [](int64_t x) { return (x + 63) & ~(int64_t)63; };
  // 1. stored factors (alive from their factorisation to the next one)
  for (int f = 0; f < nf; ++f) {
    FrontDev &d = P.fronts[f];
    if (d.kind == FK_GAMMA) {
      d.xoff = at;
      at = align(at + 2 * (int64_t)d.s * d.s);
      d.loff = -1;
      d.lpim = 0;
    } else if (kept(f)) {
      d.off = d.loff = at;
      d.lpim = (int64_t)d.n * d.n;
      at = align(at + 2 * (int64_t)d.n * d.n);
    } else {
      d.loff = at;
      d.lpim = (int64_t)d.n * d.s;
      at = align(at + 2 * (int64_t)d.n * d.s);
    }
  }
  P.e_stored = at;
  // 2. W scratch: the fronts of one level at a time (factorisation and solve
  // work on one level after the other)
  {
    const int64_t wbase = at;
    int64_t wmax = 0;
    for (int l = 0; l < nlev; ++l) {
      int64_t o = 0;
      for (int f : levels[l]) {
        FrontDev &d = P.fronts[f];
        d.woff = wbase + o;
        const int64_t wbuf = align(2 * (int64_t)d.n * d.wcols);
        d.wstride = d.s > KBLK ? wbuf : 0;   // second buffer for odd outer blocks
        o = align(o + wbuf + d.wstride);
      }
      wmax = std::max(wmax, o);
    }
    at = wbase + wmax;
    P.e_w = wmax;
  }
  // 3. arena.  During a factorisation it holds the full front matrices, each
  // from its level to its parent's (first fit over the level sequence);
  // during a solve, the solve's vectors (the fronts are dead by then).
  const int64_t arena = at;
  {
    std::vector<std::pair<int64_t, int64_t>> freel;   // (start, length), by start
    int64_t top = 0;
    auto take = [&](int64_t len) {
      for (size_t i = 0; i < freel.size(); ++i)
        if (freel[i].second >= len) {
          const int64_t o = freel[i].first;
          freel[i].first += len;
          freel[i].second -= len;
          if (freel[i].second == 0) freel.erase(freel.begin() + (long)i);
          return o;
        }
      const int64_t o = top;
      top += len;
      return o;
    };
    auto give = [&](int64_t o, int64_t len) {
      auto it = std::lower_bound(freel.begin(), freel.end(), std::make_pair(o, (int64_t)0));
      it = freel.insert(it, {o, len});
      size_t i = (size_t)(it - freel.begin());
      if (i + 1 < freel.size() && freel[i].first + freel[i].second == freel[i + 1].first) {
        freel[i].second += freel[i + 1].second;
        freel.erase(freel.begin() + (long)i + 1);
      }
      if (i > 0 && freel[i - 1].first + freel[i - 1].second == freel[i].first) {
        freel[i - 1].second += freel[i].second;
        freel.erase(freel.begin() + (long)i);
      }
      if (!freel.empty() && freel.back().first + freel.back().second == top) {
        top = freel.back().first;
        freel.pop_back();
      }
    };
    int64_t peak = 0;
    std::vector<std::vector<int>> dies(nlev);
    for (int f = 0; f < nf; ++f)
      if (!kept(f)) dies[last_use[f]].push_back(f);
    for (int l = 0; l < nlev; ++l) {
      std::vector<int> fs;
      for (int f : levels[l])
        if (!kept(f)) fs.push_back(f);
      std::stable_sort(fs.begin(), fs.end(), [&](int a, int b) { return P.fronts[a].n > P.fronts[b].n; });
      for (int f : fs) P.fronts[f].off = arena + take(align(2 * (int64_t)P.fronts[f].n * P.fronts[f].n));
      peak = std::max(peak, top);
      for (int f : dies[l]) give(P.fronts[f].off - arena, align(2 * (int64_t)P.fronts[f].n * P.fronts[f].n));
    }
    P.e_arena_factor = peak;
  }
  at = arena;   // the solve's vectors, from the start of the arena
  for (int f = 0; f < nf; ++f) {
    FrontDev &d = P.fronts[f];
    if (d.kind != FK_GAMMA) continue;
    d.goff = at;
    at = align(at + 4 * (int64_t)d.s * mr);
  }
  for (int f = 0; f < nf; ++f) {
    FrontDev &d = P.fronts[f];
    d.voff = at;
    at = align(at + 2 * (int64_t)d.n * mr);
  }
  P.vf_off = at; at = align(at + 2 * P.n_torn * mr);
  P.vx_off = at; at = align(at + 2 * P.n_torn * mr);
  P.vd_off = at; at = align(at + 2 * P.n_mult * mr);
  P.vl_off = at; at = align(at + 2 * P.n_mult * mr);
  P.vc_off = at; at = align(at + 2 * P.n_mult * mr);
  // side arrays
  int64_t sn = 0;
  for (int f = 0; f < nf; ++f) {
    P.fronts[f].soff = sn;
    sn += P.fronts[f].s;
  }
  P.side_n = sn;
  // aux item X offsets
  for (auto &it : P.aux_items)
    for (int t = 0; t < it.ndom; ++t) {
      int d = (int)it.xoff[t];
      const FrontDev &g = P.fronts[P.gamma_front[d]];
      it.xoff[t] = g.xoff;
      it.g[t] = g.s;
    }
  // multiplier references
  P.mrefs.resize(p.n_mult);
  for (int64_t m = 0; m < p.n_mult; ++m) {
    MultRef r;
    for (int s = 0; s < 2; ++s) {
      int d = m_dom[2 * m + s];
      const FrontDev &g = P.fronts[P.gamma_front[d]];
      r.o[s] = g.goff + gpos_of(d, m_dof[2 * m + s]);
      r.g[s] = g.s;
      r.sg[s] = m_sg[2 * m + s];
      r.row[s] = P.dom_row[d] + m_dof[2 * m + s];
    }
    P.mrefs[m] = r;
  }
  // copies of every global DoF (FP64 refinement): union-find over the torn
  // rows that a multiplier ties together; the representative of a component
  // is its lowest torn row (the copy of the lowest-numbered domain)
  if (o.precision != 0) {
    std::vector<int32_t> up(P.n_torn);
    std::iota(up.begin(), up.end(), 0);
    auto find = [&](int32_t x) {
      while (up[x] != x) {
        up[x] = up[up[x]];
        x = up[x];
      }
      return x;
    };
    for (int64_t m = 0; m < p.n_mult; ++m) {
      int32_t a = find((int32_t)P.mrefs[m].row[0]), b = find((int32_t)P.mrefs[m].row[1]);
      if (a != b) up[std::max(a, b)] = std::min(a, b);
    }
    P.grep.resize(P.n_torn);
    std::vector<int32_t> cid(P.n_torn, -1), cnt;
    for (int64_t r = 0; r < P.n_torn; ++r) {
      const int32_t g = find((int32_t)r);
      P.grep[r] = g;
      if (g == r) {
        cid[r] = (int32_t)cnt.size();
        cnt.push_back(0);
      }
      cnt[cid[g]]++;
    }
    P.n_gcomp = (int64_t)cnt.size();
    P.gcomp_ptr.assign(P.n_gcomp + 1, 0);
    for (int64_t c = 0; c < P.n_gcomp; ++c) P.gcomp_ptr[c + 1] = P.gcomp_ptr[c] + cnt[c];
    P.gcomp_row.resize(P.n_torn);
    std::vector<int32_t> fill(P.gcomp_ptr.begin(), P.gcomp_ptr.end() - 1);
    for (int64_t r = 0; r < P.n_torn; ++r) P.gcomp_row[fill[cid[P.grep[r]]]++] = (int32_t)r;
  }
  // interface positions -> multipliers acting on them
  P.row_gam.assign(P.n_torn, -1);
  for (int i = 0; i < p.n_dom; ++i) {
    if (P.gamma[i].empty()) continue;
    const FrontDev &g = P.fronts[P.gamma_front[i]];
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(P.gamma[i].size());
    for (int64_t e = p.imap_ptr[i]; e < p.imap_ptr[i + 1]; ++e)
      lists[gpos_of(i, p.imap_dof[e])].push_back({(int32_t)p.imap_mult[e], p.imap_sign[e]});
    for (size_t q = 0; q < lists.size(); ++q) {
      GamRef r;
      r.o = g.goff + 2 * (int64_t)g.s * mr + (int64_t)q;   // h buffer follows the YG buffer
      r.g = g.s;
      r.beg = (int32_t)P.hmult.size();
      r.cnt = (int32_t)lists[q].size();
      r.pad = 0;
      for (auto &pr : lists[q]) {
        P.hmult.push_back(pr.first);
        P.hsign.push_back(pr.second);
      }
      P.row_gam[P.dom_row[i] + P.gamma[i][q]] = (int32_t)P.grefs.size();
      P.grefs.push_back(r);
    }
  }

  // ------------------------------------------------------------ schedule
  // algorithmic flops of one work item (complex FMA = 8 real flops)
  auto item_flops = [&](int kind, const Item &it) -> double {
    // gathers count no flops (and the assembly items of auxiliary fronts
    // index interface blocks, not fronts)
    if (kind == L_ASM || kind == L_SCAT || kind == L_AUXG) return 0.0;
    const FrontDev &d = P.fronts[it.f];
    const int n = d.n;
    switch (kind) {
      case L_SYRK:
      case L_UPDPANEL: {   // C(r0.., q0..) -= L21 W^T over the lower triangle
        if (kind == L_UPDPANEL && it.i < 0) {
          // pivot tile k and its diagonal block's column update by the
          // outer block's earlier tiles (columns it.j .. k)
          const double b = std::min(NB, d.s - it.k);
          return 8.0 * (b * b * b / 3.0 + b * b * b / 6.0) + 8.0 * (it.k - it.j) * b * (b + 1) / 2;
        }
        // item: k = first column of the outer block; j = q0.  K length:
        // trailing update (i >= block end): block width; column update: q0 - k
        const int kend = std::min(it.k + KBLK, d.s);
        const bool colupd = it.j < kend;
        const double K = colupd ? (it.j - it.k) : (kend - it.k);
        const double rows = std::min(GT, n - it.i);
        const double cols = colupd ? std::min(NB, d.s - it.j) : std::min(GT, n - it.j);
        const double cnt = (it.i == it.j) ? rows * (rows + 1) / 2 : rows * cols;
        return 8.0 * K * cnt;
      }
      case L_SYRK2: {   // trailing update on 128 x 128 tiles
        const double K = std::min(it.k + KBLK, d.s) - it.k;
        const double rows = std::min(128, n - it.i), cols = std::min(128, n - it.j);
        const double cnt = (it.i == it.j) ? rows * (rows + 1) / 2 : rows * cols;
        return 8.0 * K * cnt;
      }
      case L_TRSM: {   // W = A21 P L^-T (triangular), L21 = W D^-1
        const double b = std::min(NB, d.s - it.k);
        const double rows = std::min(GT, n - it.i);
        return 8.0 * rows * (b * (b + 1) / 2 + b);
      }
      case L_PANEL: {
        const double b = std::min(NB, d.s - it.k);
        return 8.0 * (b * b * b / 3.0 + b * b * b / 6.0);
      }
      case L_ZREC1: {   // T1 tile: rows x cols x K (K from the column tile to m0)
        const double rows = std::min(GT, d.s - it.i), cols = std::min(GT, it.k - it.j);
        return 8.0 * rows * cols * (it.k - it.j - cols / 2);
      }
      case L_ZREC2: {
        const double rows = std::min(GT, d.s - it.i), cols = std::min(GT, it.k - it.j);
        return 8.0 * rows * cols * (it.i - it.k + rows / 2);
      }
      case L_INVSYRK: {
        const double rows = std::min(GT, n - it.i), cols = std::min(GT, n - it.j);
        const double cnt = (it.i == it.j) ? rows * (rows + 1) / 2 : rows * cols;
        return 8.0 * cnt * (n - it.i);
      }
      default:
        return 0.0;
    }
  };
  auto push = [&](std::vector<Launch> &seq, int kind, const std::vector<Item> &its, int p0 = 0, int p1 = 0) {
    if (its.empty()) return;
    Launch L;
    L.kind = kind;
    L.count = (int32_t)its.size();
    L.first = (int64_t)P.items.size();
    L.p0 = p0;
    L.p1 = p1;
    L.flops = 0;
    if (kind != L_FORK && kind != L_JOIN && kind < S_FINIT)
      for (const Item &it : its) L.flops += item_flops(kind, it);
    const bool gemm = kind == L_SYRK || kind == L_SYRK2 || kind == L_TRSM || kind == L_ZREC1 ||
                      kind == L_ZREC2 || kind == L_INVSYRK;
    if (gemm && its.size() >= 16) {
      // Workgroup b runs on XCD b % 8: give each XCD a contiguous run of the
      // item list (items sharing an operand panel are adjacent), so that
      // panel is read into one L2.
      const int64_t N = (int64_t)its.size();
      int64_t start[8], at = 0;
      for (int x = 0; x < 8; ++x) {
        start[x] = at;
        at += (N - x + 7) / 8;
      }
      for (int64_t b = 0; b < N; ++b) P.items.push_back(its[start[b % 8] + b / 8]);
    } else {
      P.items.insert(P.items.end(), its.begin(), its.end());
    }
    seq.push_back(L);
  };
  // Blocked right-looking LDL^T with outer blocks of KBLK columns: inside a
  // block every pivot tile first receives the updates of the block's earlier
  // tiles (column update), is factored (pivot tile + panel solve), and after
  // the block one trailing update with K = KBLK is applied.
  int64_t item_pad = 0;
  // lower tiles (edge ts) of the trailing matrix [kend, n) of front f, updated
  // by the outer block starting at column o
  auto trailing = [&](std::vector<Item> &out, int f, int o, int kend, int ts) {
    const int nt = ntiles(P.fronts[f].n - kend, ts);
    for (int ti = 0; ti < nt; ++ti)
      for (int tj = 0; tj <= ti; ++tj) out.push_back({f, o, kend + ti * ts, kend + tj * ts});
  };
  // stream synchronisation points of the look-ahead (no kernel)
  auto sync = [&](std::vector<Launch> &seq, int kind, int side) {
    Launch L{};
    L.kind = kind;
    L.count = 0;
    L.first = 0;
    L.flops = 0;
    L.side = side;
    seq.push_back(L);
  };
  auto push_on = [&](std::vector<Launch> &seq, int kind, const std::vector<Item> &its, int side) {
    const size_t before = seq.size();
    push(seq, kind, its);
    if (seq.size() > before) seq.back().side = side;
  };
  // Z = L11^-1 of the fully-summed block (P basis) by recursive halving of
  // tile ranges: a split (f, a, m, b) of tiles [a, b) at m, whose halves
  // already hold Z, forms the lower-left block (T1 = L21 Z11, then
  // Z21 = -Z22 T1).  All splits of one height (over all fronts) form one pair
  // of launches.  The single tiles already hold L_kk^-1.
  using Split = std::array<int, 4>;   // (f, a, m, b) in tiles
  auto zlaunch = [&](std::vector<Launch> &seq, const std::map<int, std::vector<Split>> &by_h, int side) {
    for (auto &kv : by_h) {
      std::vector<Item> g1, g2;
      for (auto &nd : kv.second) {
        const FrontDev &d = P.fronts[nd[0]];
        const int c0 = nd[1] * NB, m0 = nd[2] * NB, r1 = std::min(nd[3] * NB, d.s);
        // K of a T1 item grows with its column distance, of a Z21 item with
        // its row: each list runs over its K-determining index innermost, so
        // that the contiguous runs handed to the XCDs carry equal work
        for (int r = m0; r < r1; r += GT)
          for (int c = c0; c < m0; c += GT) g1.push_back({nd[0], m0, r, c});
        for (int c = c0; c < m0; c += GT)
          for (int r = m0; r < r1; r += GT) g2.push_back({nd[0], m0, r, c});
      }
      push_on(seq, L_ZREC1, g1, side);
      push_on(seq, L_ZREC2, g2, side);
    }
  };
  // balanced halving of [a, b) into by_h; returns the height
  std::function<int(std::map<int, std::vector<Split>> &, int, int, int)> zrec =
      [&](std::map<int, std::vector<Split>> &by_h, int f, int a, int b) -> int {
    if (b - a <= 1) return 0;
    const int m = (a + b) / 2;
    const int h = 1 + std::max(zrec(by_h, f, a, m), zrec(by_h, f, m, b));
    by_h[h].push_back({f, a, m, b});
    return h;
  };
  auto zsteps = [&](std::vector<Launch> &seq, const std::vector<int> &fs) {
    std::map<int, std::vector<Split>> by_h;
    for (int f : fs) zrec(by_h, f, 0, ntiles(P.fronts[f].s, NB));
    zlaunch(seq, by_h, 0);
  };
  // Z of the tiles [t0, t1) (one outer block) as soon as they are factored
  // (rows of Z depend only on rows of L up to them): their own halving, then
  // merges in binary-counter order, so that the splits stay balanced as in
  // the halving of the whole range: the front's completed ranges (zst, by
  // front) are merged while the last two are equally long, and all of them
  // after the front's last tile.
  using ZStack = std::map<int, std::vector<std::pair<int, int>>>;
  auto zblock = [&](std::vector<Launch> &seq, const std::vector<int> &fs, int t0, int tb, ZStack &zst, int side) {
    std::map<int, std::vector<Split>> by_h;
    int hmax = 0;
    for (int f : fs) {
      const int t1 = std::min(tb, ntiles(P.fronts[f].s, NB));
      if (t0 < t1) hmax = std::max(hmax, zrec(by_h, f, t0, t1));
    }
    for (int f : fs) {
      const int nt = ntiles(P.fronts[f].s, NB), t1 = std::min(tb, nt);
      if (t0 >= t1) continue;
      auto &st = zst[f];
      st.push_back({t0, t1});
      for (int h = hmax + 1; st.size() >= 2; ++h) {
        const auto top = st.back(), below = st[st.size() - 2];
        if (t1 < nt && top.second - top.first != below.second - below.first) break;
        by_h[h].push_back({f, below.first, top.first, top.second});
        st.pop_back();
        st.back() = {below.first, top.second};
      }
    }
    zlaunch(seq, by_h, side);
  };
  // Outer blocks of KBLK columns.  Inside a block each pivot tile gets the
  // block's earlier tiles (column update), its pivot-tile factorisation and
  // its panel solve.  The block's trailing update is split: the strip of the
  // next block's columns runs on the main stream, the rest on the side
  // stream, overlapping the next block's (latency-bound) pivot chain; the
  // main stream waits for it before the next trailing update.  Odd outer
  // blocks use the second W buffer.
  // zinc: fronts whose Z is formed block by block on side stream 2 while the
  // following blocks are factored (the caller joins that stream).
  auto factor_steps = [&](std::vector<Launch> &seq, const std::vector<int> &fs, const std::vector<int> &zinc) {
    int maxt = 0;
    for (int f : fs) maxt = std::max(maxt, ntiles(P.fronts[f].s, NB));
    const int G = KBLK / NB;
    bool pending = false;
    ZStack zst;
    for (int ob = 0; ob < maxt; ob += G) {
      for (int t = ob; t < ob + G && t < maxt; ++t) {
        // the block's first tile: pivot tile alone; later tiles: one launch
        // of the pivot tiles (each with its diagonal block's column update)
        // followed by the column update of the rows below
        std::vector<Item> pan, upd, trs;
        for (int f : fs) {
          const FrontDev &d = P.fronts[f];
          const int k = t * NB, o = ob * NB;
          if (k >= d.s) continue;
          const int b = std::min(NB, d.s - k);
          pan.push_back(t > ob ? Item{f, k, -1, o} : Item{f, k, 0, 0});
          if (t > ob)
            for (int r0 = k + GT; r0 < d.n; r0 += GT) upd.push_back({f, o, r0, k});
          for (int r0 = k + b; r0 < d.n; r0 += GT) trs.push_back({f, k, r0, k - o});
        }
        if (t > ob) {
          pan.insert(pan.end(), upd.begin(), upd.end());
          push(seq, L_UPDPANEL, pan);
        } else {
          push(seq, L_PANEL, pan);
        }
        push(seq, L_TRSM, trs);
      }
      if (!zinc.empty()) {
        sync(seq, L_FORK, 2);
        zblock(seq, zinc, ob, ob + G, zst, 2);
      }
      std::vector<Item> syr[2], syr2[2];   // [0]: next block's strip, [1]: rest
      for (int f : fs) {
        const FrontDev &d = P.fronts[f];
        const int o = ob * NB;
        if (o >= d.s) continue;
        const int kend = std::min(o + KBLK, d.s);
        const int ts = P.schur_tile[tile_bucket(d.n)];
        std::vector<Item> all;
        trailing(all, f, o, kend, ts);
        for (const Item &it : all) (ts == 128 ? syr2 : syr)[it.j < kend + KBLK ? 0 : 1].push_back(it);
        if (ts == 128) {
          // keep the item array as long as with 64-tiles: the workspace
          // layout must not depend on the tile policy
          const int64_t a = ntiles(d.n - kend, 64), c = ntiles(d.n - kend, 128);
          item_pad += a * (a + 1) / 2 - c * (c + 1) / 2;
        }
      }
      if (pending) sync(seq, L_JOIN, 1);
      push(seq, L_SYRK, syr[0]);
      push(seq, L_SYRK2, syr2[0]);
      pending = !syr[1].empty() || !syr2[1].empty();
      if (pending) {
        sync(seq, L_FORK, 1);
        push_on(seq, L_SYRK, syr[1], 1);
        push_on(seq, L_SYRK2, syr2[1], 1);
      }
    }
    if (pending) sync(seq, L_JOIN, 1);
  };
  auto assemble = [&](std::vector<Launch> &seq, const std::vector<int> &fs, bool aux) {
    std::vector<Item> as, sc, ag;
    for (int f : fs) {
      const FrontDev &d = P.fronts[f];
      for (int c0 = 0; c0 < d.n; c0 += 64)
        for (int r0 = c0; r0 < d.n; r0 += 256) as.push_back({f, c0, r0, 0});
      if (!aux) {
        auto pr = prange[f];
        for (int64_t b = 0; b < pr.second; b += 4096)
          sc.push_back({f, (int32_t)(pr.first + b), (int32_t)std::min<int64_t>(4096, pr.second - b), 0});
      } else {
        // 64 x 64 sub-blocks of every block pair (lower part only on the diagonal)
        auto ar = arange[f];
        for (int64_t b = 0; b < ar.second; ++b) {
          const AuxItem &a = P.aux_items[ar.first + b];
          for (int i0 = 0; i0 < a.na; i0 += 64)
            for (int j0 = 0; j0 < a.nb; j0 += 64)
              if (!a.same || j0 + 64 > i0) ag.push_back({(int32_t)(ar.first + b), 0, i0, j0});
        }
      }
    }
    push(seq, L_ASM, as);
    push(seq, L_SCAT, sc);
    push(seq, L_AUXG, ag);
  };
  auto zfront = [&](int f) { return P.fronts[f].kind != FK_GAMMA && P.fronts[f].n > FUSE_N; };
  auto zset = [&](const std::vector<int> &lv) {
    std::vector<int> z;
    for (int f : lv)
      if (zfront(f)) z.push_back(f);
    return z;
  };
  // the factor columns of the level's fronts (except those kept whole) into
  // their stored-factor place: 16 columns x 256 rows per item, from the
  // columns' 64-row diagonal tile down (the solves read nothing above it)
  auto store = [&](std::vector<Launch> &seq, const std::vector<int> &fs) {
    std::vector<Item> st;
    for (int f : fs) {
      const FrontDev &d = P.fronts[f];
      if (d.kind == FK_GAMMA || kept(f)) continue;
      for (int c0 = 0; c0 < d.s; c0 += 16)
        for (int r0 = (c0 / NB) * NB; r0 < d.n; r0 += 256) st.push_back({f, c0, r0, 0});
    }
    push(seq, L_STORE, st);
  };

  // factor.  A level's inverses (Z) and stored-factor copies run on side
  // stream 2 beside the next level's factorisation, which touches only that
  // level's fronts (alive together with the previous level's, so disjoint);
  // the main stream waits for them before the level after (whose fronts may
  // reuse their memory).  The last level keeps them on the main stream; the
  // interface roots form their Z beside their own factorisation (below).
  std::vector<int> prev;
  auto side_inverse = [&]() {
    if (prev.empty()) return false;
    sync(P.factor_seq, L_FORK, 2);
    const size_t a = P.factor_seq.size();
    zsteps(P.factor_seq, zset(prev));
    store(P.factor_seq, prev);
    for (size_t i = a; i < P.factor_seq.size(); ++i) P.factor_seq[i].side = 2;
    return true;
  };
  // The interface roots have nothing after them to overlap their Z with
  // (their X is needed at once): theirs is formed block by block beside their
  // own factorisation instead.  The top auxiliary front keeps the halving
  // after its factorisation: beside its latency-bound chain the merges slow
  // the chain as much as they save, and the final merge is long.
  auto level = [&](const std::vector<int> &lv, bool aux, const std::vector<int> &zinc) {
    assemble(P.factor_seq, lv, aux);
    const bool forked = side_inverse();
    factor_steps(P.factor_seq, lv, zinc);
    if (forked || !zinc.empty()) sync(P.factor_seq, L_JOIN, 2);
    prev = lv;
  };
  const std::vector<int> none;
  for (auto &lv : dom_levels) level(lv, false, none);
  if (!gam.empty()) {
    level(gam, false, gam);
    prev.clear();   // the roots' X follows on the main stream
    std::vector<Item> sy;
    for (int f : gam) {
      const FrontDev &d = P.fronts[f];
      int nt = ntiles(d.s, GT);
      for (int ti = 0; ti < nt; ++ti)
        for (int tj = 0; tj <= ti; ++tj) sy.push_back({f, 0, ti * GT, tj * GT});
    }
    push(P.factor_seq, L_DINVZ, sy);
    push(P.factor_seq, L_INVSYRK, sy);
  }
  for (auto &lv : aux_levels) level(lv, true, none);
  zsteps(P.factor_seq, zset(prev));
  store(P.factor_seq, prev);
  P.items.resize(P.items.size() + item_pad, Item{0, 0, 0, 0});
  // tuner launches: first outer block's trailing update of every front of a
  // bucket, with both tile edges
  for (int bkt = 0; bkt < TILE_BUCKETS; ++bkt) {
    std::vector<Item> t64, t128;
    for (int f = 0; f < (int)P.fronts.size(); ++f) {
      const FrontDev &d = P.fronts[f];
      if (tile_bucket(d.n) != bkt || d.s == 0) continue;
      const int kend = std::min(KBLK, d.s);
      trailing(t64, f, 0, kend, 64);
      trailing(t128, f, 0, kend, 128);
    }
    std::vector<Launch> tmp;
    push(tmp, L_SYRK, t64);
    push(tmp, L_SYRK2, t128);
    if (tmp.size() == 2) {
      P.tune[bkt][0] = tmp[0];
      P.tune[bkt][1] = tmp[1];
    }
  }

  // solve: forward over a set of levels
  int64_t max_part = 0;
  int ns_a = 0, ns_b = 0;   // partial slots of the level's first and second product
  auto rows = [&](std::vector<Item> &v, int f, int lo, int hi) {
    for (int r = lo; r < hi; r += 256) v.push_back({f, 0, r, 0});
  };
  // split product: 64-output tiles [o_lo, o_hi) x K chunks [k_lo(tile), k_hi(tile)).
  // A tile with one chunk is one item that applies the epilogue itself (slot
  // -1); a tile with several has one partial slot per item and one reduction
  // item.
  auto split = [&](std::vector<Item> &prod, std::vector<Item> &red, int &nslot, int f, int o_lo, int o_hi,
                   auto k_lo, auto k_hi) {
    for (int i = o_lo; i < o_hi; i += 64) {
      if (k_hi(i) - k_lo(i) <= ZKC) {
        prod.push_back({f, -1, i, k_lo(i)});
        continue;
      }
      const int sbeg = nslot;
      for (int c = k_lo(i); c < k_hi(i); c += ZKC) prod.push_back({f, nslot++, i, c});
      red.push_back({f, sbeg, i, nslot - sbeg});
    }
  };
  // Small fronts: one workgroup per front.  Fronts carrying Z = L11^-1:
  // row-parallel gathers and split triangular / rectangular products.
  auto fwd = [&](std::vector<Launch> &seq, const std::vector<std::vector<int>> &levels, bool gamma_only_init) {
    for (auto &lv : levels) {
      std::vector<Item> small, in, fin, p0, r0, p1, r1;
      for (int f : lv) {
        const FrontDev &d = P.fronts[f];
        const int s = d.s, n = d.n;
        if (gamma_only_init) {
          rows(in, f, 0, n);
          continue;
        }
        if (!zfront(f)) {
          small.push_back({f, 0, 0, 0});
          continue;
        }
        // without children the update rows hold no extend-add sums: the
        // forward product writes them outright
        rows(in, f, 0, d.nchild ? n : s);
        rows(fin, f, 0, s);
        split(p0, r0, ns_a, f, 0, s, [](int) { return 0; }, [&](int i) { return std::min(i + 64, s); });
        split(p1, r1, ns_b, f, s, n, [](int) { return 0; }, [&](int) { return s; });
      }
      max_part = std::max<int64_t>(max_part, std::max(ns_a, ns_b));
      ns_a = ns_b = 0;
      push(seq, S_FFRONT, small);
      push(seq, S_FINIT, in);
      push(seq, S_ZP0, p0);
      push(seq, S_ZR0, r0);
      push(seq, S_ZP1, p1);
      push(seq, S_ZR1, r1);
      push(seq, S_FFIN, fin);
    }
  };
  auto bwd = [&](std::vector<Launch> &seq, const std::vector<std::vector<int>> &levels) {
    for (auto it = levels.rbegin(); it != levels.rend(); ++it) {
      std::vector<Item> small, in, out, p2, r2, p3, r3;
      for (int f : *it) {
        const FrontDev &d = P.fronts[f];
        const int s = d.s, n = d.n;
        if (!zfront(f)) {
          small.push_back({f, 0, 0, 0});
          continue;
        }
        rows(in, f, s, n);
        rows(out, f, 0, s);
        split(p2, r2, ns_a, f, 0, s, [&](int) { return s; }, [&](int) { return n; });
        split(p3, r3, ns_b, f, 0, s, [](int i) { return i; }, [&](int) { return s; });
      }
      max_part = std::max<int64_t>(max_part, std::max(ns_a, ns_b));
      ns_a = ns_b = 0;
      push(seq, S_BFRONT, small);
      push(seq, S_BINIT, in);
      push(seq, S_ZP2, p2);
      push(seq, S_ZR2, r2);
      push(seq, S_ZP3, p3);
      push(seq, S_ZR3, r3);
      push(seq, S_BFIN, out);
    }
  };
  fwd(P.solve_dom_fwd, dom_levels, false);
  if (!gam.empty()) fwd(P.solve_dom_fwd, {gam}, true);
  fwd(P.solve_aux, aux_levels, false);
  bwd(P.solve_aux, aux_levels);
  if (!gam.empty()) {
    std::vector<Item> out;
    for (int f : gam) rows(out, f, 0, P.fronts[f].s);
    push(P.solve_dom_bwd, S_BFIN, out);
  }
  bwd(P.solve_dom_bwd, dom_levels);
  for (int f : gam)
    for (int r = 0; r < P.fronts[f].s; r += 64) P.gemv_items.push_back({f, 0, r, 0});
  P.max_partials = max_part;
  P.part_off = at;
  at = align(at + std::max<int64_t>(1, max_part) * NB * mr * 2);
  P.e_arena_solve = at - arena;
  P.t_elems = arena + std::max(P.e_arena_factor, P.e_arena_solve);

  // ------------------------------------------------------------ meta blob
  auto put = [&](const void *src, size_t bytes) -> int64_t {
    size_t o = (P.meta.size() + 255) & ~(size_t)255;
    P.meta.resize(o + std::max<size_t>(bytes, 16), 0);
    if (bytes) std::memcpy(P.meta.data() + o, src, bytes);
    return (int64_t)o;
  };
  P.m_fronts = put(P.fronts.data(), P.fronts.size() * sizeof(FrontDev));
  P.m_vars = put(P.vars.data(), P.vars.size() * 4);
  P.m_cfront = put(P.child_front.data(), P.child_front.size() * 4);
  P.m_crmap = put(P.child_rmap.data(), P.child_rmap.size() * 8);
  P.m_rmap = put(P.rmap.data(), P.rmap.size() * 4);
  P.m_urow = put(P.urow.data(), P.urow.size() * 4);
  P.m_spairs = put(P.spairs.data(), P.spairs.size() * sizeof(SPair));
  P.m_aux = put(P.aux_items.data(), P.aux_items.size() * sizeof(AuxItem));
  P.m_gpos = put(P.gpos.data(), P.gpos.size() * 4);
  P.m_gsign = put(P.gsign.data(), P.gsign.size() * 4);
  P.m_mrefs = put(P.mrefs.data(), P.mrefs.size() * sizeof(MultRef));
  P.m_grefs = put(P.grefs.data(), P.grefs.size() * sizeof(GamRef));
  P.m_hmult = put(P.hmult.data(), P.hmult.size() * 4);
  P.m_hsign = put(P.hsign.data(), P.hsign.size() * 4);
  P.m_rowgam = put(P.row_gam.data(), P.row_gam.size() * 4);
  P.m_items = put(P.items.data(), P.items.size() * sizeof(Item));
  P.m_gemv = put(P.gemv_items.data(), P.gemv_items.size() * sizeof(Item));
  P.m_csrp = put(P.csr_ptr.data(), P.csr_ptr.size() * 8);
  P.m_sellp = put(P.sell_ptr.data(), P.sell_ptr.size() * 8);
  P.m_sellc = put(P.sell_col.data(), P.sell_col.size() * 4);
  P.m_domrow = put(P.dom_row.data(), P.dom_row.size() * 8);
  P.m_grep = put(P.grep.data(), P.grep.size() * 4);
  P.m_gcp = put(P.gcomp_ptr.data(), P.gcomp_ptr.size() * 4);
  P.m_gcr = put(P.gcomp_row.data(), P.gcomp_row.size() * 4);

  // ------------------------------------------------------------ workspace (bytes)
  auto A256 = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
  int64_t b = 0;
  P.b_meta = b; b = A256(b + (int64_t)P.meta.size());
  P.b_num = b; b = A256(b + P.t_elems * (int64_t)P.elem);
  P.b_side = b; b = A256(b + P.side_n * (16 + 16 + 4 + 4));
  P.b_vals = b;
  if (P.precision != 0) b = A256(b + P.nnz_sell * 16);   // SELL-64 FP64 operator copy
  P.b_r64 = b;
  if (P.precision != 0) {
    int64_t r = 0;
    P.r_u = r; r += 2 * P.n_torn * mr;
    P.r_l = r; r += 2 * P.n_mult * mr;
    P.r_g = r; r += 2 * P.n_torn * mr;
    P.r_nblk = 1024;
    // [blocks x cols] partial sums: torn residual (or rhs), then the
    // assembled (global) one
    P.r_part = r; r += 2 * P.r_nblk * mr;
    P.r_norm = r; r += 2 * mr;    // squared norms: torn [0, mr), global [mr, 2 mr)
    P.r_fnorm = r; r += 2 * mr;
    P.r_ctl = r; r += 4;          // last torn / assembled residual maxima
    b = A256(b + r * 8);
  }
  P.b_status = b; b = A256(b + 256);
  P.b_dmask = b; b = A256(b + std::max(1, p.n_dom));   // domain mask of the subset solve
  P.b_sel = b; b = A256(b + 8 * std::max<int64_t>(1, P.n_torn));   // selected rows (dd_solve_dofs)
  P.b_total = b;

  if (o.verbose) {
    // workspace breakdown (GB)
    const double e = (double)P.elem / 1e9;
    fprintf(stderr, "[dd] workspace GB: stored factors %.3f, W %.3f, arena %.3f (fronts %.3f, solve vectors %.3f), "
                    "meta %.3f side %.3f r64 %.3f\n",
            P.e_stored * e, P.e_w * e, std::max(P.e_arena_factor, P.e_arena_solve) * e, P.e_arena_factor * e,
            P.e_arena_solve * e, P.meta.size() / 1e9, P.side_n * 40 / 1e9, (P.b_status - P.b_vals) / 1e9);
    fprintf(stderr,
            "[dd] domains %d torn %lld mult %lld | fronts dom %d (max %d) aux %d (max %d) blocks %d\n"
            "[dd] factor %.3e flop, solve %.3e flop/rhs, factors %.3f GB | workspace %.3f GB | launches factor %zu solve %zu\n",
            p.n_dom, (long long)P.n_torn, (long long)P.n_mult, P.n_front_dom, P.max_front_dom, P.n_front_aux,
            P.max_front_aux, nb, P.flops_factor, P.flops_solve_rhs, P.bytes_factor / 1e9, P.b_total / 1e9,
            P.factor_seq.size(), P.solve_dom_fwd.size() + P.solve_aux.size() + P.solve_dom_bwd.size());
  }
  return std::string();
}

}  // namespace dd
