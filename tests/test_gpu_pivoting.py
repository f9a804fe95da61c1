"""Restricted Bunch-Kaufman pivoting and the numerical status contract,
through the C ABI.

Section II factors the auxiliary matrix (and, here, every front) by a block
LDL^T with restricted Bunch-Kaufman pivoting, and requires every domain to be
regular.  These tests force the pivot tile's branches on single dense
domains (one front of n >= 200: several 64-wide pivot tiles, a ragged last
tile and, at n = 300, a second 256-column outer block) and compare the
solution entry by entry with the LAPACK brute force:

* zero diagonal: no 1 x 1 pivot passes the test, 2 x 2 pivots throughout;
* alternating zero / large diagonal: 1 x 1 pivots with interchanges;
* tiny diagonal: a mix of both.

A domain that is not regular must be reported: an exactly singular pivot
tile and a zero row give DD_ERR_SINGULAR with the domain that holds it; a
NaN value gives DD_ERR_NUMERIC (FP64 path, nothing solved).
"""
import numpy as np
import pytest

import oracle
from tests.conftest import cached_case
from tests.test_gpu_parity import DEV, _colerr, _rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dense_domain(n, diag, seed):
    """Complex-symmetric dense n x n matrix with the given diagonal rule."""
    rng = np.random.default_rng(seed)
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    A = G + G.T
    k = np.arange(n)
    if diag == "zero":
        d = np.zeros(n, complex)
    elif diag == "alternating":
        d = np.where(k % 2 == 0, 0.0, 3.0 + 1.0j)
    elif diag == "tiny":
        d = 1e-9 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    else:
        raise ValueError(diag)
    A[k, k] = d
    return A


def _dense_solver(A, precision="fp64", **kw):
    from paper_2002_05019_amd.binding import Solver
    n = A.shape[0]
    rowptr = np.arange(n + 1, dtype=np.int64) * n
    colind = np.tile(np.arange(n, dtype=np.int32), n)
    s = Solver([rowptr], [colind], 0, np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64),
               np.zeros(0, np.int8), xyz=None, precision=precision, **kw).bind(DEV)
    s.factor(torch.from_numpy(np.ascontiguousarray(A.ravel())).to(DEV))
    return s


def _rhs_dense(n, nrhs, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))) / np.sqrt(2)


@pytest.mark.parametrize("n,diag", [(200, "zero"), (300, "alternating"), (256, "tiny")])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_bunch_kaufman_branches_against_brute_force(n, diag, precision):
    A = _dense_domain(n, diag, seed=n)
    F = _rhs_dense(n, 3, seed=n + 1)
    print(f"[pivot] dense n={n} diag={diag} {precision}", flush=True)
    s = _dense_solver(A, precision)
    u = s.solve(torch.from_numpy(F).to(DEV)).cpu().numpy()
    info = s.info()
    ref = oracle.dense_solve(A, F)
    err = _colerr(u, ref)
    res = (np.linalg.norm(F - A @ u, axis=0) / np.linalg.norm(F, axis=0)).max()
    print(f"[pivot] n={n} {diag} {precision}: 2x2 {info['n_pivot_2x2']} interchanges "
          f"{info['n_interchanges']} err {err:.2e} resid {res:.2e}", flush=True)
    assert s.last_status == 0
    assert info["n_perturbed"] == 0 and info["numeric_flags"] == 0 and info["bad_domain"] == -1
    if diag == "zero":
        assert info["n_pivot_2x2"] > 0
    if diag == "alternating":
        assert info["n_interchanges"] > 0
    if diag == "tiny":
        assert info["n_pivot_2x2"] > 0 and info["n_interchanges"] > 0
    if precision == "fp64":
        assert err < 1e-10, err
    else:
        assert info["rel_resid"] <= 1e-9 and res <= 1e-9, (info["rel_resid"], res)
        assert err < 1e-9, err


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_singular_pivot_tile_is_reported(precision):
    """A nonsingular matrix whose leading 64 x 64 tile is zero: restricted
    pivoting cannot leave the tile, so its pivots are perturbed."""
    n = 200
    A = _dense_domain(n, "alternating", seed=11)
    A[:64, :64] = 0.0
    print(f"[pivot] singular leading tile {precision}", flush=True)
    s = _dense_solver(A, precision, refine_maxit=2)
    s.solve(torch.from_numpy(_rhs_dense(n, 1, 12)).to(DEV), check=False)
    info = s.info()
    print(f"[pivot] singular tile: status {s.last_status} perturbed {info['n_perturbed']}", flush=True)
    assert info["n_perturbed"] > 0
    assert info["bad_domain"] == 0
    assert s.last_status == -6   # DD_ERR_SINGULAR


def _cube6_with(mutate):
    c = cached_case("cube6")
    vals = [d.K.data.copy() for d in c.domains]
    mutate(c, vals)
    return c, torch.from_numpy(np.concatenate(vals)).to(DEV)


def test_zero_row_reports_its_domain():
    """Domain 3 with one interior row and column zeroed is singular."""
    dom = 3

    def zero_row(c, vals):
        K = c.domains[dom].K
        g = set(c.gamma(dom).tolist())
        r = next(v for v in range(K.shape[0]) if v not in g)
        rows = np.repeat(np.arange(K.shape[0]), np.diff(K.indptr))
        vals[dom][(rows == r) | (K.indices == r)] = 0.0

    from paper_2002_05019_amd.binding import Solver
    c, vals = _cube6_with(zero_row)
    print("[pivot] cube6 zero row in domain 3", flush=True)
    s = Solver.from_case(c).bind(DEV)
    s.factor(vals)
    s.solve(_rhs(c), check=False)
    info = s.info()
    assert s.last_status == -6, s.last_status
    assert info["n_perturbed"] > 0 and info["bad_domain"] == dom


def test_nan_value_is_numeric_error():
    dom = 5

    def put_nan(c, vals):
        # a diagonal entry: it is assembled whatever the elimination order
        K = c.domains[dom].K
        r = K.shape[0] // 2
        vals[dom][K.indptr[r] + np.searchsorted(K.indices[K.indptr[r]:K.indptr[r + 1]], r)] = np.nan

    from paper_2002_05019_amd.binding import DDError, Solver
    c, vals = _cube6_with(put_nan)
    print("[pivot] cube6 NaN in domain 5", flush=True)
    s = Solver.from_case(c).bind(DEV)
    s.factor(vals)
    with pytest.raises(DDError) as e:
        s.solve(_rhs(c))
    assert e.value.status == -7   # DD_ERR_NUMERIC
    info = s.info()
    assert info["numeric_flags"] != 0 and info["bad_domain"] == dom
    # the context recovers with good values
    s.factor(torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV))
    u = s.solve(_rhs(c))
    assert _colerr(u.cpu().numpy(), oracle.serial_dd(c)["u"]) < 1e-10
