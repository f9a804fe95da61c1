"""GPU parity on the method's degenerate cases and at the full bench size.

* One domain: no multipliers and no auxiliary matrix, so the DD solve is a
  single sparse LDL^T of the operator (section II with one domain).
* Two domains: the auxiliary matrix is one dense block (one aux front).
* The 48^3 bench workload, in the configuration ``bench.py`` times (tuned
  tiles, hipGraph replay): interface inverses of sampled domains against the
  oracle's sparse direct inverse (the oracle cannot do the whole case in
  seconds), every column's residual on the host, and the mixed path against
  the FP64 path.
"""
import numpy as np
import pytest

import oracle
from paper_2002_05019_amd.problem import even_cuts
from tests.conftest import cached_case
from tests.test_gpu_parity import DEV, _colerr, _rhs, _solver

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_single_domain_is_one_sparse_solve(precision):
    c = cached_case("cube12", cuts=even_cuts(12, 1))
    assert c.n_dom == 1 and c.n_mult == 0
    print(f"[parity] one domain cube12 {precision}", flush=True)
    s = _solver(c, precision=precision)
    u = s.solve(_rhs(c))
    torch.cuda.synchronize()
    ref = oracle.global_solve(c.A, c.f)
    err = _colerr(c.owner_copy(u.cpu().numpy()), ref)
    assert err < (1e-10 if precision == "fp64" else 1e-9), err
    if precision == "fp32_refine":
        assert s.info()["rel_resid"] <= 1e-9
        assert oracle.global_residual(c, u.cpu().numpy()).max() <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_two_domains_dense_auxiliary_block(precision):
    c = cached_case("cube12", cuts=((0, 12), (0, 12), (0, 6, 12)))
    assert c.n_dom == 2 and c.n_mult > 0
    print(f"[parity] two domains cube12 {precision}", flush=True)
    s = _solver(c, precision=precision)
    u, lam = s.solve(_rhs(c), return_lam=True)
    torch.cuda.synchronize()
    ref = oracle.serial_dd(c)
    tol = 1e-10 if precision == "fp64" else 1e-9
    assert _colerr(u.cpu().numpy(), ref["u"]) < tol
    assert _colerr(lam.cpu().numpy(), ref["lam"]) < tol
    if precision == "fp32_refine":
        assert oracle.global_residual(c, u.cpu().numpy()).max() <= 1e-9


def test_full_size_sampled_parity():
    c = cached_case("cube48")
    print("[parity] cube48 full size: fp64 setup + tune + graph", flush=True)
    f = _rhs(c)
    s = _solver(c, max_rhs=8, use_graph=True)
    s.tune()
    vals = torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV)
    s.factor(vals)
    u64 = s.solve(f)
    torch.cuda.synchronize()
    info = s.info()
    assert info["n_perturbed"] == 0 and info["numeric_flags"] == 0
    # sampled interface inverses: a corner and an interior domain
    for i in (0, 21):
        print(f"[parity] cube48 interface inverse of domain {i}", flush=True)
        g = c.gamma(i)
        assert np.array_equal(s.interface_dofs(i), g)
        X = s.interface_inverse(i).cpu().numpy()
        R, _ = oracle.interface_inverse(c.domains[i].K, g)
        assert np.abs(X - R).max() / np.abs(R).max() < 1e-10
    u64 = u64.cpu().numpy()
    assert oracle.global_residual(c, u64).max() < 1e-11
    print("[parity] cube48 full size: fp32+refine", flush=True)
    m = _solver(c, precision="fp32_refine", max_rhs=8, use_graph=True)
    m.tune()
    m.factor(vals)
    um = m.solve(f)
    torch.cuda.synchronize()
    assert m.last_status == 0 and m.info()["rel_resid"] <= 1e-9
    um = um.cpu().numpy()
    assert oracle.global_residual(c, um).max() <= 1e-9
    assert _colerr(um, u64) <= 1e-9


def test_full_size_reciprocity_and_linearity():
    """Properties of A^-1 that hold at any size, on the 48^3 bench workload in
    the timed configuration (tuned tiles, graph replay, FP64).  Reciprocity:
    A is complex symmetric, so u_j^T f_i = u_i^T f_j (no conjugation); with the
    torn convention f is nonzero only on owner copies, where u is the global
    value, so the torn products are the global ones.  Linearity: the solve
    of F C equals U C for a fixed complex 8 x 8 C.  Each solution is within
    1e-10 of A^-1 f per column (the FP64 gate), so both identities hold to
    2e-10 relative."""
    c = cached_case("cube48")
    print("[parity] cube48 full size: reciprocity and linearity (fp64, tuned, graph)", flush=True)
    f = _rhs(c)
    s = _solver(c, max_rhs=8, use_graph=True)
    s.tune()
    s.factor(torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV))
    U = s.solve(f).cpu().numpy()
    F = f.cpu().numpy()
    M = U.T @ F
    scale = np.linalg.norm(U, axis=0).max() * np.linalg.norm(F, axis=0).max()
    rec = np.abs(M - M.T).max() / scale
    rng = np.random.default_rng(4805)
    C = (rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))) / 4
    UC = s.solve(torch.from_numpy(np.ascontiguousarray(F @ C)).to(DEV)).cpu().numpy()
    lin = _colerr(UC, U @ C)
    print(f"[parity] cube48 reciprocity {rec:.2e} linearity {lin:.2e}", flush=True)
    assert rec < 2e-10, rec
    assert lin < 2e-10, lin


@pytest.mark.parametrize("graph", [False, True])
def test_subset_recovery_matches_full_solve(graph):
    """Section II: after the multipliers, the primal unknowns of only some
    domains are recovered.  The selected domains' rows equal the full solve
    bit for bit (same arithmetic); the other rows are left untouched."""
    c = cached_case("cube18u")
    print(f"[parity] subset recovery cube18u graph={graph}", flush=True)
    s = _solver(c, use_graph=graph)
    f = _rhs(c)
    full = s.solve(f).cpu().numpy()
    offs = np.cumsum([0] + [d.n for d in c.domains])
    pick = [0, 3, c.n_dom - 1]
    sentinel = torch.full_like(f, 7.0 + 7.0j)
    for rep in range(2):
        u = s.solve_subset(f, pick, u=sentinel).cpu().numpy()
        for i in range(c.n_dom):
            rows = slice(offs[i], offs[i + 1])
            if i in pick:
                assert np.array_equal(u[rows], full[rows]), (rep, i)
            else:
                assert np.all(u[rows] == 7.0 + 7.0j), (rep, i)
    # the full solve still works after subset solves
    assert np.array_equal(s.solve(f).cpu().numpy(), full)


def test_subset_recovery_against_oracle():
    """The recovered domains' unknowns against the oracle's serial DD
    solution (1e-10 per column), on an uneven jittered case."""
    c = cached_case("cube18u")
    s = _solver(c, max_rhs=8)
    offs = np.cumsum([0] + [d.n for d in c.domains])
    pick = [1, c.n_dom // 2, c.n_dom - 2]
    print(f"[parity] subset recovery cube18u domains {pick} vs oracle", flush=True)
    u = s.solve_subset(_rhs(c), pick).cpu().numpy()
    ref = oracle.serial_dd(c)["u"]
    for i in pick:
        rows = slice(offs[i], offs[i + 1])
        assert _colerr(u[rows], ref[rows]) < 1e-10, i


def test_dof_recovery_against_oracle():
    """Recovery at the granularity of single DoFs (observation points): the
    selected torn rows equal the full solve's bit for bit and the oracle's
    solution within 1e-10 per column."""
    c = cached_case("cube18u")
    s = _solver(c)
    offs = np.cumsum([0] + [d.n for d in c.domains])
    rng = np.random.default_rng(1802)
    rows = np.concatenate([offs[1] + rng.choice(c.domains[1].n, 40, replace=False),
                           offs[5] + rng.choice(c.domains[5].n, 40, replace=False), [offs[-1] - 1]])
    print(f"[parity] dof recovery cube18u: {len(rows)} rows in 3 domains", flush=True)
    f = _rhs(c)
    out = s.solve_dofs(f, rows).cpu().numpy()
    full = s.solve(f).cpu().numpy()
    assert np.array_equal(out, full[rows])
    ref = oracle.serial_dd(c)["u"][rows]
    assert _colerr(out, ref) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_graph_only_orderings(precision):
    """No DoF coordinates: every domain and the auxiliary block graph are
    ordered by the level-set (graph-only) nested dissection."""
    from paper_2002_05019_amd.binding import Solver
    c = cached_case("cube16")
    print(f"[parity] cube16 without coordinates {precision}", flush=True)
    s = Solver.from_case(c, coordinates=False, precision=precision).bind(DEV)
    s.factor(torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV))
    u = s.solve(_rhs(c))
    torch.cuda.synchronize()
    un = u.cpu().numpy()
    err = _colerr(un, oracle.serial_dd(c)["u"])
    print(f"[parity] cube16 graph-only {precision}: err {err:.2e}", flush=True)
    if precision == "fp64":
        assert err < 1e-10, err
    else:
        assert oracle.global_residual(c, un).max() <= 1e-9 and err <= 1e-9, err


def test_frequency_sweep_reuses_the_symbolic_phase():
    """Many excitations over a frequency sweep: one context (one symbolic
    phase, one workspace) refactored at three wavenumbers; every solution
    against the oracle of its own operator."""
    base = cached_case("cube12")
    s = None
    for scale in (1.0, 0.8, 1.25):
        c = cached_case("cube12", k0=base.spec.k0 * scale)
        print(f"[parity] frequency sweep cube12 k0 x {scale}", flush=True)
        if s is None:
            s = _solver(c)
        else:
            assert all(np.array_equal(a.K.indptr, b.K.indptr) and np.array_equal(a.K.indices, b.K.indices)
                       for a, b in zip(c.domains, base.domains))
            s.factor(torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV))
        u = s.solve(_rhs(c))
        torch.cuda.synchronize()
        assert _colerr(u.cpu().numpy(), oracle.serial_dd(c)["u"]) < 1e-10
