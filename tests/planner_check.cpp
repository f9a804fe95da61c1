// Host-only driver of the symbolic planner, built by the test suite with
// AddressSanitizer and UndefinedBehaviorSanitizer (g++, no GPU code).
//
// Each argument names a problem file written by tests/test_planner_sanitizers.py:
//   int32 n_dom, int64 n_mult, int32 has_xyz, int32 expect_valid
//   per domain: int32 n, int64 nnz, int64 rowptr[n + 1], int32 colind[nnz]
//   int64 imap_ptr[n_dom + 1], int32 imap_dof[m], int64 imap_mult[m], int8 imap_sign[m]
//   float xyz[3 * sum(n)] when has_xyz
// For a valid problem the plan is built in both precisions with the stream
// schedule and the workspace layout checked; an invalid one must be refused
// by validate_problem.  Exit status 0 when every file behaves as expected.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "plan.h"

namespace {

struct Reader {
  FILE *f;
  bool ok = true;
  template <typename X>
  X one() {
    X v{};
    if (std::fread(&v, sizeof(X), 1, f) != 1) ok = false;
    return v;
  }
  template <typename X>
  std::vector<X> many(int64_t count) {
    std::vector<X> v(count < 0 ? 0 : (size_t)count);
    if (count > 0 && std::fread(v.data(), sizeof(X), (size_t)count, f) != (size_t)count) ok = false;
    return v;
  }
};

// The schedule and layout checks must refuse a plan with (1) two work items
// of one panel-solve launch writing the same rows, (2) the main stream's first
// wait for either side stream removed, or (3) a wrong row in the backward
// sweep's parent-row map.  True when all are caught (plans that do not have
// the needed launches count as caught).
bool planted_conflicts_caught(const dd::Plan &P) {
  bool ok = true;
  for (size_t j = 0; j < P.factor_seq.size(); ++j) {
    const dd::Launch &L = P.factor_seq[j];
    if (L.kind != dd::L_TRSM || L.count < 2 || P.items[L.first].f != P.items[L.first + 1].f) continue;
    dd::Plan Q = P;
    Q.items[L.first + 1].i = Q.items[L.first].i;
    if (dd::check_schedule(Q, Q.factor_seq).empty()) {
      std::printf("duplicated panel-solve rows in launch %zu not caught\n", j);
      ok = false;
    }
    break;
  }
  for (int side = 1; side <= 2; ++side)
    for (size_t j = 0; j < P.factor_seq.size(); ++j) {
      if (P.factor_seq[j].kind != dd::L_JOIN || P.factor_seq[j].side != side) continue;
      dd::Plan Q = P;
      Q.factor_seq.erase(Q.factor_seq.begin() + j);
      if (dd::check_schedule(Q, Q.factor_seq).empty()) {
        std::printf("missing join %zu of side stream %d not caught\n", j, side);
        ok = false;
      }
      break;
    }
  // (3) an update row of the backward sweep's parent-row map pointed at the
  // parent's next row
  for (size_t c = 0; c < P.fronts.size(); ++c) {
    const dd::FrontDev &cd = P.fronts[c];
    if (cd.parent < 0 || cd.n <= cd.s) continue;
    dd::Plan Q = P;
    Q.urow[cd.uoff] += 1;
    if (dd::check_layout(Q).empty()) {
      std::printf("shifted parent row of front %zu not caught\n", c);
      ok = false;
    }
    break;
  }
  return ok;
}

int run(const char *path) {
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    std::printf("%s: cannot open\n", path);
    return 1;
  }
  Reader r{f};
  const int32_t n_dom = r.one<int32_t>();
  const int64_t n_mult = r.one<int64_t>();
  const int32_t has_xyz = r.one<int32_t>();
  const int32_t expect_valid = r.one<int32_t>();
  std::vector<std::vector<int64_t>> rowptr(n_dom);
  std::vector<std::vector<int32_t>> colind(n_dom);
  dd::ProblemView pv;
  pv.n_dom = n_dom;
  pv.n_mult = n_mult;
  int64_t n_torn = 0;
  for (int i = 0; i < n_dom && r.ok; ++i) {
    const int32_t n = r.one<int32_t>();
    const int64_t nnz = r.one<int64_t>();
    rowptr[i] = r.many<int64_t>((int64_t)n + 1);
    colind[i] = r.many<int32_t>(nnz);
    pv.n.push_back(n);
    pv.nnz.push_back(nnz);
    n_torn += n;
  }
  const std::vector<int64_t> iptr = r.many<int64_t>((int64_t)n_dom + 1);
  const int64_t m = iptr.empty() ? 0 : iptr.back();
  const std::vector<int32_t> idof = r.many<int32_t>(m);
  const std::vector<int64_t> imult = r.many<int64_t>(m);
  const std::vector<int8_t> isign = r.many<int8_t>(m);
  const std::vector<float> xyz = has_xyz ? r.many<float>(3 * n_torn) : std::vector<float>();
  std::fclose(f);
  if (!r.ok) {
    std::printf("%s: truncated file\n", path);
    return 1;
  }
  for (int i = 0; i < n_dom; ++i) {
    pv.rowptr.push_back(rowptr[i].data());
    pv.colind.push_back(colind[i].data());
  }
  pv.imap_ptr = iptr.data();
  pv.imap_dof = idof.data();
  pv.imap_mult = imult.data();
  pv.imap_sign = isign.data();
  pv.xyz = has_xyz ? xyz.data() : nullptr;

  int code = 0;
  const std::string v = dd::validate_problem(pv, &code);
  if (!expect_valid) {
    std::printf("%s: refused (%d): %s\n", path, code, v.c_str());
    return v.empty() ? 1 : 0;
  }
  if (!v.empty()) {
    std::printf("%s: unexpectedly refused: %s\n", path, v.c_str());
    return 1;
  }
  for (int prec = 0; prec < 2; ++prec) {
    dd::SetupOptions so;
    so.precision = prec;
    so.max_rhs = 8;
    so.verify = 1;
    dd::Plan P;
    std::string e = dd::build_plan(pv, so, P);
    if (e.empty()) e = dd::check_schedule(P, P.factor_seq);
    if (e.empty()) e = dd::check_layout(P);
    if (!e.empty()) {
      std::printf("%s (precision %d): %s\n", path, prec, e.c_str());
      return 1;
    }
    std::printf("%s (precision %d): %zu fronts, %zu factor launches\n", path, prec, P.fronts.size(),
                P.factor_seq.size());
    if (prec == 0 && planted_conflicts_caught(P)) std::printf("%s: planted conflicts caught\n", path);
  }
  return 0;
}

}  // namespace

int main(int argc, char **argv) {
  int bad = 0;
  for (int i = 1; i < argc; ++i) bad += run(argv[i]);
  return bad ? 1 : 0;
}
