"""Host-side checks of the C ABI (no GPU call): the library loads, exports
every entry point declared in include/dd.h, validates its inputs, reports
state errors, and its symbolic phase counts what closed forms predict."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2002_05019_amd import binding as B
from tests.conftest import ROOT, cached_case

HEADER = os.path.join(ROOT, "include", "dd.h")


def _lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libdd.so not built")
    return B.load()


def test_exports_every_declared_symbol():
    lib = _lib()
    text = open(HEADER).read()
    names = sorted(set(re.findall(r"^\s*(?:dd_status|void|const char \*)\s*\*?\s*(dd_\w+)\s*\(", text, re.M)))
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def _problem(rowptrs, colinds, n_mult=0, imap=None, opt=None):
    lib = _lib()
    nd = len(rowptrs)
    keep = []
    pats = (B.dd_pattern * nd)()
    for i in range(nd):
        rp = np.ascontiguousarray(rowptrs[i], np.int64)
        ci = np.ascontiguousarray(colinds[i], np.int32)
        keep += [rp, ci]
        pats[i].n = len(rp) - 1
        pats[i].nnz = int(rp[-1])
        pats[i].rowptr = rp.ctypes.data_as(C.POINTER(C.c_int64))
        pats[i].colind = ci.ctypes.data_as(C.POINTER(C.c_int32))
    prob = B.dd_problem()
    prob.n_dom = nd
    prob.dom = pats
    prob.n_mult = n_mult
    if imap is not None:
        arrs = [np.ascontiguousarray(imap[0], np.int64), np.ascontiguousarray(imap[1], np.int32),
                np.ascontiguousarray(imap[2], np.int64), np.ascontiguousarray(imap[3], np.int8)]
        keep += arrs
        prob.imap_ptr = arrs[0].ctypes.data_as(C.POINTER(C.c_int64))
        prob.imap_dof = arrs[1].ctypes.data_as(C.POINTER(C.c_int32))
        prob.imap_mult = arrs[2].ctypes.data_as(C.POINTER(C.c_int64))
        prob.imap_sign = arrs[3].ctypes.data_as(C.POINTER(C.c_int8))
    ctx = C.c_void_p()
    st = lib.dd_setup(C.byref(prob), opt, C.byref(ctx))
    return st, ctx, lib


def _dense(n):
    return np.arange(0, n * n + 1, n), np.tile(np.arange(n), n)


def test_pattern_errors_are_reported():
    rp, ci = _dense(3)
    bad = ci.copy()
    bad[0], bad[1] = bad[1], bad[0]            # unsorted row
    st, _, lib = _problem([rp], [bad])
    assert st == -2 and b"increasing" in lib.dd_last_error()
    m = sp.csr_matrix(np.array([[1, 1, 0], [1, 0, 1], [0, 1, 1.0]]))
    m.eliminate_zeros()                          # missing diagonal (1,1)
    st, _, lib = _problem([m.indptr], [m.indices])
    assert st == -2 and b"diagonal" in lib.dd_last_error()
    m = sp.csr_matrix(np.array([[1, 1, 0], [0, 1, 0], [0, 0, 1.0]]))  # not symmetric
    st, _, lib = _problem([m.indptr], [m.indices])
    assert st == -2 and b"symmetric" in lib.dd_last_error()
    st, _, _ = _problem([np.array([0, 1, 3]), np.array([0, 1])], [np.array([0, 0, 1]), np.array([0])])
    assert st == -2


def test_map_errors_are_reported():
    rp, ci = _dense(2)
    pats = ([rp, rp], [ci, ci])
    ok = (np.array([0, 1, 2]), np.array([0, 0]), np.array([0, 0]), np.array([1, -1]))
    st, ctx, lib = _problem(*pats, n_mult=1, imap=ok)
    assert st == 0
    lib.dd_destroy(ctx)
    one = (np.array([0, 1, 1]), np.array([0]), np.array([0]), np.array([1]))
    st, _, lib = _problem(*pats, n_mult=1, imap=one)
    assert st == -3 and b"exactly 2" in lib.dd_last_error()
    sign = (np.array([0, 1, 2]), np.array([0, 0]), np.array([0, 0]), np.array([1, 2]))
    assert _problem(*pats, n_mult=1, imap=sign)[0] == -3
    dof = (np.array([0, 1, 2]), np.array([0, 5]), np.array([0, 0]), np.array([1, -1]))
    assert _problem(*pats, n_mult=1, imap=dof)[0] == -3
    same = (np.array([0, 2, 2]), np.array([0, 1]), np.array([0, 0]), np.array([1, -1]))
    assert _problem(*pats, n_mult=1, imap=same)[0] == -3


def test_option_and_state_errors():
    lib = _lib()
    rp, ci = _dense(4)
    opt = B.dd_options()
    lib.dd_default_options(C.byref(opt))
    opt.max_rhs = 0
    assert _problem([rp], [ci], opt=C.byref(opt))[0] == -1
    lib.dd_default_options(C.byref(opt))
    opt.precision = 7
    assert _problem([rp], [ci], opt=C.byref(opt))[0] == -1
    st, ctx, lib = _problem([rp], [ci])
    assert st == 0
    z = C.c_void_p(0)
    assert lib.dd_factor(ctx, z, None) == -4          # no workspace bound
    assert lib.dd_solve(ctx, 1, z, 4, z, 4, None, 0, None) == -4   # before factor
    assert lib.dd_bind_workspace(ctx, C.c_void_p(256), 1) == -5    # too small
    mask = (C.c_uint8 * 1)(1)
    assert lib.dd_solve_subset(ctx, 1, z, 4, z, 4, None, None) == -1   # no mask
    assert lib.dd_solve_subset(ctx, 1, z, 4, z, 4, mask, None) == -4   # before factor
    lib.dd_destroy(ctx)
    lib.dd_default_options(C.byref(opt))
    opt.precision = 1
    st, ctx, lib = _problem([rp], [ci], opt=C.byref(opt))
    assert st == 0
    assert lib.dd_solve_subset(ctx, 1, z, 4, z, 4, mask, None) == -1   # FP64 contexts only
    lib.dd_destroy(ctx)


def test_dense_single_domain_flops_closed_form():
    """A dense pattern cannot be dissected: one front eliminating n pivots,
    (n^3/6) complex FMAs = 8 n^3 / 6 real flops; solve 2 n^2 complex FMAs."""
    n = 40
    rp, ci = _dense(n)
    st, ctx, lib = _problem([rp], [ci])
    assert st == 0
    inf = B.dd_info()
    assert lib.dd_get_info(ctx, C.byref(inf)) == 0
    assert inf.n_fronts_domain == 1 and inf.n_fronts_aux == 0
    assert inf.flops_factor == pytest.approx(8.0 * n ** 3 / 6.0)
    assert inf.flops_solve == pytest.approx(8.0 * n * n)
    lib.dd_destroy(ctx)


def test_symbolic_structure_of_cube_cases():
    for name in ("cube6", "cube16"):
        c = cached_case(name)
        s = B.Solver.from_case(c)
        inf = s.info()
        for i in range(c.n_dom):
            assert np.array_equal(s.interface_dofs(i), c.gamma(i))
        assert sum(s.domain_flops(i) for i in range(c.n_dom)) < inf["flops_factor"]
        assert inf["workspace_bytes"] > 0
        # the auxiliary fronts cover every multiplier exactly once as a pivot
        assert inf["max_front_aux"] <= c.n_mult
        s.close()


def test_interior_domain_flops_match_appendix_model():
    """A 12^3 interior domain: interior elimination plus the interface
    Schur inverse.  A geometric nested-dissection front model (recursive
    longest-side bisection, leaves of at most 2 elements per side, calibrated
    against an exact symbolic factorisation of the 12^3 domain) gives ~8.0e8
    complex FMAs for the interior part, and the interface inverse costs
    g^3/2 (g = 1728).  Our own ordering must land within 25% of that."""
    c = cached_case("cube48")
    s = B.Solver.from_case(c)
    dom = 21                                       # an interior domain of the 4x4x4 grid
    g = len(c.gamma(dom))
    assert g == 1728
    model = 8.0 * (7.97e8 + g ** 3 / 2.0)
    assert s.domain_flops(dom) == pytest.approx(model, rel=0.25)
    s.close()
