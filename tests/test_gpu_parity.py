"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 path, relative error <= 1e-10 per right-hand-side column on
the solution, the multipliers and the interface inverses; FP32 fronts + FP64
refinement, the residual of the undecomposed system ||f - A u|| / ||f|| <= 1e-9
per column (computed on the host from the owner copies) and the error against
the FP64 oracle <= 1e-9 per column.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import cached_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_REF = {}


def _ref(name):
    if name not in _REF:
        _REF[name] = oracle.serial_dd(cached_case(name))
    return _REF[name]


def _solver(case, precision="fp64", **kw):
    from paper_2002_05019_amd.binding import Solver
    s = Solver.from_case(case, precision=precision, **kw).bind(DEV)
    vals = torch.from_numpy(np.concatenate([d.K.data for d in case.domains])).to(DEV)
    s.factor(vals)
    return s


def _rhs(case):
    return torch.from_numpy(case.torn_rhs()).to(DEV)


def _colerr(u, ref):
    u = np.asarray(u).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return (np.linalg.norm(u - ref, axis=0) / np.linalg.norm(ref, axis=0)).max()


@pytest.mark.parametrize("name", ["cube6", "cube12", "cube16", "cube18u"])
def test_interface_inverse_fp64(name):
    c = cached_case(name)
    print(f"[parity] interface inverse {name}", flush=True)
    s = _solver(c)
    ref = _ref(name)
    worst = 0.0
    for i in range(c.n_dom):
        assert np.array_equal(s.interface_dofs(i), c.gamma(i))
        X = s.interface_inverse(i).cpu().numpy()
        R = ref["S_inv"][i]
        worst = max(worst, np.abs(X - R).max() / np.abs(R).max())
    info = s.info()
    assert info["n_perturbed"] == 0 and info["numeric_flags"] == 0
    assert worst < 1e-10, worst


@pytest.mark.parametrize("name", ["cube6", "cube12", "cube16", "cube18u", "cube24"])
def test_solution_fp64(name):
    c = cached_case(name)
    print(f"[parity] fp64 solve {name}", flush=True)
    s = _solver(c)
    u, lam = s.solve(_rhs(c), return_lam=True)
    torch.cuda.synchronize()
    ref = _ref(name)
    eu = _colerr(u.cpu().numpy(), ref["u"])
    el = _colerr(lam.cpu().numpy(), ref["lam"])
    print(f"[parity] {name} fp64: u err {eu:.2e} lam err {el:.2e}", flush=True)
    assert eu < 1e-10, eu
    assert el < 1e-10, el
    assert oracle.global_residual(c, u.cpu().numpy()).max() < 1e-10


@pytest.mark.parametrize("name", ["cube6", "cube16", "cube18u"])
def test_solution_mixed_refined(name):
    c = cached_case(name)
    print(f"[parity] fp32+refine solve {name}", flush=True)
    s = _solver(c, precision="fp32_refine")
    u = s.solve(_rhs(c))
    torch.cuda.synchronize()
    info = s.info()
    un = u.cpu().numpy()
    gr = oracle.global_residual(c, un).max()
    eu = _colerr(un, _ref(name)["u"])
    print(f"[parity] {name} mixed: iters {info['refine_iters']} resid {info['rel_resid']:.2e} "
          f"(torn {info['rel_resid_torn']:.2e}) host global resid {gr:.2e} err {eu:.2e}", flush=True)
    assert s.last_status == 0
    assert info["rel_resid"] <= 1e-9 and info["rel_resid_torn"] <= 1e-9
    # the device's assembled residual is the host's, up to rounding
    assert abs(info["rel_resid"] - gr) <= 1e-3 * gr + 1e-15
    assert gr <= 1e-9
    assert eu <= 1e-9


def test_many_rhs_blocks_and_vector_rhs():
    """nrhs above max_rhs is solved in column blocks; a 1-D rhs works."""
    c = cached_case("cube12")
    s = _solver(c, max_rhs=2)
    f = _rhs(c)
    f5 = torch.cat([f, 2j * f[:, :2]], dim=1)
    u = s.solve(f5)
    ref = _ref("cube12")["u"]
    assert _colerr(u[:, :3].cpu().numpy(), ref) < 1e-10
    assert _colerr(u[:, 3:].cpu().numpy(), 2j * ref[:, :2]) < 1e-10
    u1 = s.solve(f[:, 1].contiguous())
    assert _colerr(u1.cpu().numpy(), ref[:, 1]) < 1e-10


def test_refactor_same_context():
    """A second factorisation with new values reuses the symbolic phase."""
    c = cached_case("cube6")
    s = _solver(c)
    vals2 = torch.from_numpy(np.concatenate([2.0 * d.K.data for d in c.domains])).to(DEV)
    s.factor(vals2)
    u = s.solve(_rhs(c))
    assert _colerr(u.cpu().numpy(), 0.5 * _ref("cube6")["u"]) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_graph_replay_bitwise_equals_eager(precision):
    """Factor + solve replayed from hipGraphs, three times with eager work and
    synchronisations in between, equal bit for bit to the eager launches."""
    c = cached_case("cube16")
    eager = _solver(c, precision=precision)
    f = _rhs(c)
    ue = eager.solve(f).cpu().numpy()
    s = _solver(c, precision=precision, use_graph=True)
    vals = torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV)
    for rep in range(3):
        s.factor(vals)
        u = s.solve(f).cpu().numpy()
        assert np.array_equal(u, ue), (rep, np.abs(u - ue).max())
        eager.factor(vals)
        ue2 = eager.solve(f).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(ue2, ue)
    assert s.info()["n_perturbed"] == 0


def test_repeat_runs_bitwise_identical():
    c = cached_case("cube18u")
    a = _solver(c).solve(_rhs(c)).cpu().numpy()
    b = _solver(c).solve(_rhs(c)).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("tile", [64, 128])
def test_schur_tile_policy(tile):
    """Every front's trailing update on one tile edge (128 also on fronts far
    smaller than the tile, so ragged tiles everywhere)."""
    c = cached_case("cube18u")
    print(f"[parity] schur tile {tile} cube18u", flush=True)
    s = _solver(c, schur_tile=[tile] * 5)
    u = s.solve(_rhs(c))
    torch.cuda.synchronize()
    assert _colerr(u.cpu().numpy(), _ref("cube18u")["u"]) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_tuned_tiles(precision):
    """The tile tuner re-plans on the bound workspace; the factorisation after
    it must still match the oracle."""
    from paper_2002_05019_amd.binding import Solver
    c = cached_case("cube24")
    print(f"[parity] tuned tiles cube24 {precision}", flush=True)
    s = Solver.from_case(c, precision=precision).bind(DEV)
    tiles = s.tune()
    assert len(tiles) == 5 and all(t in (0, 64, 128) for t in tiles)
    assert any(t != 0 for t in tiles)
    vals = torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV)
    s.factor(vals)
    u = s.solve(_rhs(c))
    torch.cuda.synchronize()
    tol = 1e-10 if precision == "fp64" else 1e-9
    assert _colerr(u.cpu().numpy(), _ref("cube24")["u"]) < tol
    if precision == "fp32_refine":
        assert oracle.global_residual(c, u.cpu().numpy()).max() <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_many_rhs_on_matrix_cores(precision):
    """70 right-hand sides in one block: the substitution products of the wide
    fronts run on the MFMA tile (two 64-column passes)."""
    c = cached_case("cube18u")
    print(f"[parity] 70 rhs cube18u {precision}", flush=True)
    rng = np.random.default_rng(7)
    nr = 70
    nt = sum(d.n for d in c.domains)
    ft = (rng.standard_normal((nt, nr)) + 1j * rng.standard_normal((nt, nr))) / np.sqrt(2)
    offs = np.cumsum([0] + [d.n for d in c.domains])
    ref = oracle.serial_dd(c, F_rhs=[ft[offs[i]:offs[i + 1]] for i in range(c.n_dom)])
    s = _solver(c, precision=precision, max_rhs=80)
    u = s.solve(torch.from_numpy(ft).to(DEV))
    torch.cuda.synchronize()
    tol = 1e-10 if precision == "fp64" else 1e-9
    assert _colerr(u.cpu().numpy(), ref["u"]) < tol
    if precision == "fp32_refine":
        assert s.info()["rel_resid"] <= 1e-9


def test_tune_cache(tmp_path):
    """The tile tuner's cache: the first context measures and appends its
    line, a second context of the same problem takes the tiles from the
    file, and its factorisation matches the oracle."""
    from paper_2002_05019_amd.binding import Solver
    c = cached_case("cube18u")
    path = tmp_path / "tiles.txt"
    print("[parity] tune cache cube18u", flush=True)
    s1 = Solver.from_case(c, tune_cache=path).bind(DEV)
    t1 = s1.tune()
    assert s1.info()["tuned_from_cache"] == 0
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:] == [str(t) for t in t1]
    s2 = Solver.from_case(c, tune_cache=path).bind(DEV)
    t2 = s2.tune()
    assert s2.info()["tuned_from_cache"] == 1 and t2 == t1
    assert len(path.read_text().splitlines()) == 1
    s2.factor(torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV))
    u = s2.solve(_rhs(c))
    assert _colerr(u.cpu().numpy(), _ref("cube18u")["u"]) < 1e-10
    # another shape (FP32 fronts) gets a line of its own
    s3 = Solver.from_case(c, precision="fp32_refine", tune_cache=path).bind(DEV)
    s3.tune()
    assert s3.info()["tuned_from_cache"] == 0 and len(path.read_text().splitlines()) == 2


@pytest.mark.parametrize("graph", [False, True])
def test_refinement_cap_and_device_control(graph):
    """Refinement control on the device: with a cap of one correction the
    solve reports DD_ERR_NOT_CONVERGED (u still written, one iteration
    counted); with the default cap the same context converges, and a repeat
    solve (which enqueues as many corrections as the last one needed)
    returns the same bits."""
    from paper_2002_05019_amd.binding import Solver
    c = cached_case("cube16")
    vals = torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV)
    print(f"[parity] refinement cap cube16 graph={graph}", flush=True)
    s = Solver.from_case(c, precision="fp32_refine", refine_maxit=1, use_graph=graph).bind(DEV)
    s.factor(vals)
    u1 = s.solve(_rhs(c), check=False).cpu().numpy()
    info = s.info()
    assert s.last_status == -8 and info["refine_iters"] == 1
    assert 1e-9 < info["rel_resid"] < 1e-3
    assert np.isfinite(u1).all()
    m = Solver.from_case(c, precision="fp32_refine", use_graph=graph).bind(DEV)
    m.factor(vals)
    ua = m.solve(_rhs(c)).cpu().numpy()
    it = m.info()["refine_iters"]
    ub = m.solve(_rhs(c)).cpu().numpy()
    assert m.last_status == 0 and m.info()["refine_iters"] == it >= 1
    assert np.array_equal(ua, ub)
    assert oracle.global_residual(c, ub).max() <= 1e-9
