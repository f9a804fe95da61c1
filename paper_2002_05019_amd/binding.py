"""Thin ctypes binding of ``libdd.so`` (declared in ``include/dd.h``).

Argument marshalling only: every numeric step runs in the library's HIP
kernels.  PyTorch provides device memory (the workspace, value, right-hand
side and solution tensors) and the stream.  Importing works without a GPU;
``Solver`` raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdd.so")

DD_OK = 0
STATUS = {0: "DD_OK", -1: "DD_ERR_ARG", -2: "DD_ERR_PATTERN", -3: "DD_ERR_MAP", -4: "DD_ERR_STATE",
          -5: "DD_ERR_NOMEM", -6: "DD_ERR_SINGULAR", -7: "DD_ERR_NUMERIC", -8: "DD_ERR_NOT_CONVERGED",
          -9: "DD_ERR_DEVICE"}
PRECISION = {"fp64": 0, "fp32_refine": 1}

_P = C.POINTER


class dd_pattern(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rowptr", _P(C.c_int64)), ("colind", _P(C.c_int32))]


class dd_problem(C.Structure):
    _fields_ = [("n_dom", C.c_int32), ("dom", _P(dd_pattern)), ("n_mult", C.c_int64),
                ("imap_ptr", _P(C.c_int64)), ("imap_dof", _P(C.c_int32)), ("imap_mult", _P(C.c_int64)),
                ("imap_sign", _P(C.c_int8)), ("dof_xyz", _P(C.c_float))]


class dd_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("refine_tol", C.c_double), ("refine_maxit", C.c_int32),
                ("max_rhs", C.c_int32), ("leaf_size", C.c_int32), ("use_graph", C.c_int32),
                ("verbose", C.c_int32), ("schur_tile", C.c_int32 * 5),
                ("verify_schedule", C.c_int32), ("tune_cache", C.c_char_p)]


class dd_info(C.Structure):
    _fields_ = [("t_setup", C.c_double), ("t_factor", C.c_double), ("t_solve", C.c_double),
                ("flops_factor", C.c_double), ("flops_solve", C.c_double), ("bytes_factor", C.c_double),
                ("workspace_bytes", C.c_int64), ("n_fronts_domain", C.c_int32), ("n_fronts_aux", C.c_int32),
                ("max_front_aux", C.c_int32), ("max_front_domain", C.c_int32), ("refine_iters", C.c_int32),
                ("rel_resid", C.c_double), ("n_perturbed", C.c_int32), ("numeric_flags", C.c_int32),
                ("bytes_solve", C.c_double), ("rel_resid_torn", C.c_double), ("bad_domain", C.c_int32),
                ("n_pivot_2x2", C.c_int32), ("n_interchanges", C.c_int32), ("tuned_from_cache", C.c_int32)]


EXPORTS = ["dd_default_options", "dd_setup", "dd_workspace_size", "dd_bind_workspace", "dd_factor",
           "dd_solve", "dd_get_info", "dd_get_interface_dofs", "dd_get_interface_inverse",
           "dd_get_domain_flops", "dd_kernel_timer_start", "dd_kernel_timer_read", "dd_tune", "dd_solve_subset",
           "dd_bind_static_workspace", "dd_solve_dofs", "dd_destroy", "dd_last_error"]
STATIC_WORKSPACE_BYTES = 128 << 20   # DD_STATIC_WORKSPACE_BYTES
TILE_BUCKETS = 5   # front sizes [0,512) [512,1024) [1024,2048) [2048,4096) [4096,...)
KERNELS = {"schur_update": 0, "panel_solve": 1, "pivot_tile": 2, "inverse_update": 3, "column_update": 4}

_lib = None


def load():
    """Load libdd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2002_05019_amd.build`")
    # torch brings its own HIP runtime; loading it first makes the library
    # resolve libamdhip64 to that same runtime, so that torch's device
    # pointers and streams are valid in the library (a second runtime
    # loaded from the system path would not see the device)
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.dd_default_options.argtypes = [_P(dd_options)]
    lib.dd_default_options.restype = None
    lib.dd_setup.argtypes = [_P(dd_problem), _P(dd_options), _P(vp)]
    lib.dd_workspace_size.argtypes = [vp, _P(C.c_int64)]
    lib.dd_bind_workspace.argtypes = [vp, vp, C.c_int64]
    lib.dd_bind_static_workspace.argtypes = [vp]
    lib.dd_factor.argtypes = [vp, vp, vp]
    lib.dd_solve.argtypes = [vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, vp, C.c_int64, vp]
    lib.dd_solve_subset.argtypes = [vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, _P(C.c_uint8), vp]
    lib.dd_get_info.argtypes = [vp, _P(dd_info)]
    lib.dd_solve_dofs.argtypes = [vp, C.c_int32, vp, C.c_int64, C.c_int64, _P(C.c_int64), vp, C.c_int64, vp]
    lib.dd_get_interface_dofs.argtypes = [vp, C.c_int32, _P(C.c_int32), _P(C.c_int32)]
    lib.dd_get_interface_inverse.argtypes = [vp, C.c_int32, vp, vp]
    lib.dd_get_domain_flops.argtypes = [vp, C.c_int32, _P(C.c_double)]
    lib.dd_kernel_timer_start.argtypes = [vp, C.c_int32]
    lib.dd_kernel_timer_read.argtypes = [vp, _P(C.c_double), _P(C.c_int64), _P(C.c_double)]
    lib.dd_tune.argtypes = [vp, _P(C.c_int32), vp]
    lib.dd_destroy.argtypes = [vp]
    lib.dd_destroy.restype = None
    lib.dd_last_error.argtypes = []
    lib.dd_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("dd_default_options", "dd_destroy", "dd_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class DDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st):
    if st != DD_OK:
        raise DDError(st, load().dd_last_error().decode())
    return st


def _ptr(a, ctype):
    return a.ctypes.data_as(_P(ctype))


class Solver:
    """One decomposed problem: symbolic setup at construction (host only),
    then ``bind`` (device workspace), ``factor``, ``solve``.

    Domain ``i`` is given by its CSR pattern (``rowptr[i]``, ``colind[i]``);
    the interface map by ``imap_ptr``, ``imap_dof``, ``imap_mult``,
    ``imap_sign``; ``xyz`` (optional) steers the orderings."""

    def __init__(self, rowptr, colind, n_mult, imap_ptr, imap_dof, imap_mult, imap_sign, xyz=None,
                 precision="fp64", max_rhs=64, leaf_size=48, refine_tol=1e-9, refine_maxit=20,
                 use_graph=False, verbose=False, schur_tile=None, verify_schedule=False, tune_cache=None):
        lib = load()
        self._lib = lib
        nd = len(rowptr)
        self._rowptr = [np.ascontiguousarray(r, dtype=np.int64) for r in rowptr]
        self._colind = [np.ascontiguousarray(c, dtype=np.int32) for c in colind]
        pats = (dd_pattern * nd)()
        for i in range(nd):
            pats[i].n = len(self._rowptr[i]) - 1
            pats[i].nnz = int(self._rowptr[i][-1])
            pats[i].rowptr = _ptr(self._rowptr[i], C.c_int64)
            pats[i].colind = _ptr(self._colind[i], C.c_int32)
        self._imap = [np.ascontiguousarray(imap_ptr, dtype=np.int64), np.ascontiguousarray(imap_dof, dtype=np.int32),
                      np.ascontiguousarray(imap_mult, dtype=np.int64), np.ascontiguousarray(imap_sign, dtype=np.int8)]
        self._xyz = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float32)
        prob = dd_problem()
        prob.n_dom = nd
        prob.dom = pats
        prob.n_mult = int(n_mult)
        prob.imap_ptr = _ptr(self._imap[0], C.c_int64)
        prob.imap_dof = _ptr(self._imap[1], C.c_int32)
        prob.imap_mult = _ptr(self._imap[2], C.c_int64)
        prob.imap_sign = _ptr(self._imap[3], C.c_int8)
        prob.dof_xyz = _ptr(self._xyz, C.c_float) if self._xyz is not None else None
        opt = dd_options()
        lib.dd_default_options(C.byref(opt))
        opt.precision = PRECISION[precision]
        opt.max_rhs = int(max_rhs)
        opt.leaf_size = int(leaf_size)
        opt.refine_tol = float(refine_tol)
        opt.refine_maxit = int(refine_maxit)
        opt.verbose = int(bool(verbose))
        opt.use_graph = 2 if use_graph == "solve" else int(bool(use_graph))
        opt.verify_schedule = int(bool(verify_schedule))
        self._tune_cache = None if tune_cache is None else str(tune_cache).encode()
        opt.tune_cache = self._tune_cache
        if schur_tile is not None:
            assert len(schur_tile) == TILE_BUCKETS
            for b, t in enumerate(schur_tile):
                opt.schur_tile[b] = int(t)
        self.precision = precision
        self.max_rhs = int(max_rhs)
        ctx = C.c_void_p()
        _check(lib.dd_setup(C.byref(prob), C.byref(opt), C.byref(ctx)))
        self._ctx = ctx
        self.n_dom = nd
        self.n_mult = int(n_mult)
        self.dom_n = np.array([len(r) - 1 for r in self._rowptr], dtype=np.int64)
        self.n_torn = int(self.dom_n.sum())
        self.nnz = int(sum(int(r[-1]) for r in self._rowptr))
        ws = C.c_int64()
        _check(lib.dd_workspace_size(ctx, C.byref(ws)))
        self.workspace_bytes = int(ws.value)
        self._ws = None

    @classmethod
    def from_case(cls, case, coordinates=True, **kw):
        """Solver of a generated case; ``coordinates=False`` passes no DoF
        coordinates (graph-only orderings)."""
        doms = case.domains
        xyz = np.concatenate([d.xyz for d in doms]) if coordinates else None
        return cls([d.K.indptr for d in doms], [d.K.indices for d in doms], case.n_mult, case.imap_ptr,
                   case.imap_dof, case.imap_mult, case.imap_sign, xyz=xyz, **kw)

    # ------------------------------------------------------------------ device
    @staticmethod
    def _stream(stream):
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        return C.c_void_p(s.cuda_stream)

    def bind(self, device="cuda:0"):
        import torch
        buf = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self._ws = buf
        self._ws_off = off
        _check(self._lib.dd_bind_workspace(self._ctx, C.c_void_p(buf.data_ptr() + off), self.workspace_bytes))
        self.device = torch.device(device)
        return self

    def bind_static(self, device="cuda:0"):
        """Binds the library's static workspace array of ``device`` (no device
        allocation; problems above STATIC_WORKSPACE_BYTES are refused).  The
        array serves the context bound to it last."""
        import torch
        torch.cuda.set_device(torch.device(device))
        _check(self._lib.dd_bind_static_workspace(self._ctx))
        self._ws = None
        self.device = torch.device(device)
        return self

    def factor(self, vals, stream=None):
        """vals: complex128 device tensor, all domain values concatenated."""
        import torch
        assert vals.dtype == torch.complex128 and vals.is_cuda and vals.is_contiguous()
        assert vals.numel() == self.nnz
        self._vals = vals
        _check(self._lib.dd_factor(self._ctx, C.c_void_p(vals.data_ptr()), self._stream(stream)))

    def solve(self, f, return_lam=False, stream=None, check=True):
        """f: complex128 device tensor (n_torn, nrhs) (or (n_torn,)).  Returns u
        of the same shape (and the multipliers (n_mult, nrhs) if asked).
        A status other than DD_OK raises DDError unless ``check`` is False;
        the status is kept in ``last_status`` either way (u is written on
        DD_ERR_NOT_CONVERGED and DD_ERR_SINGULAR)."""
        import torch
        vec = f.dim() == 1
        F = f.reshape(self.n_torn, -1)
        nrhs = F.shape[1]
        # column-major staging (ld = n_torn), reused across calls: the
        # library's graphs of a refined solve are kept per right-hand-side
        # pointer
        fb = getattr(self, "_fbuf", None)
        if fb is None or fb.shape[0] != nrhs or fb.device != F.device:
            fb = self._fbuf = torch.empty((nrhs, self.n_torn), dtype=torch.complex128, device=F.device)
        fb.copy_(F.t())
        fc = fb
        u = torch.empty_like(fc)
        lam = torch.empty((nrhs, self.n_mult), dtype=torch.complex128, device=fc.device) if return_lam else None
        st = self._lib.dd_solve(self._ctx, nrhs, C.c_void_p(fc.data_ptr()), self.n_torn, C.c_void_p(u.data_ptr()),
                                self.n_torn, C.c_void_p(lam.data_ptr()) if lam is not None else None,
                                max(self.n_mult, 1), self._stream(stream))
        self.last_status = st
        if check:
            _check(st)
        u = u.t()
        if vec:
            u = u.reshape(-1)
        if return_lam:
            return u, lam.t()
        return u

    def solve_subset(self, f, domains, u=None, stream=None, check=True):
        """Recovers the primal unknowns of the listed domains only (FP64
        contexts).  f: complex128 device tensor (n_torn, nrhs); u: optional
        output of the same shape whose other rows are left as they are
        (zeros when u is None).  Returns u."""
        import torch
        F = f.reshape(self.n_torn, -1)
        nrhs = F.shape[1]
        fc = F.t().contiguous()
        uc = torch.zeros_like(fc) if u is None else u.reshape(self.n_torn, -1).t().contiguous()
        mask = np.zeros(self.n_dom, dtype=np.uint8)
        mask[np.asarray(list(domains), dtype=np.int64)] = 1
        st = self._lib.dd_solve_subset(self._ctx, nrhs, C.c_void_p(fc.data_ptr()), self.n_torn,
                                       C.c_void_p(uc.data_ptr()), self.n_torn, _ptr(mask, C.c_uint8),
                                       self._stream(stream))
        self.last_status = st
        if check:
            _check(st)
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        out = uc.t()
        return out.reshape(-1) if f.dim() == 1 else out

    def solve_dofs(self, f, rows, stream=None, check=True):
        """Recovers the primal unknowns at the given torn rows only (FP64
        contexts): returns a (len(rows), nrhs) complex128 device tensor."""
        import torch
        F = f.reshape(self.n_torn, -1)
        nrhs = F.shape[1]
        fc = F.t().contiguous()
        r = np.ascontiguousarray(rows, dtype=np.int64)
        out = torch.empty((nrhs, len(r)), dtype=torch.complex128, device=fc.device)
        st = self._lib.dd_solve_dofs(self._ctx, nrhs, C.c_void_p(fc.data_ptr()), self.n_torn, len(r),
                                     _ptr(r, C.c_int64), C.c_void_p(out.data_ptr()), max(len(r), 1),
                                     self._stream(stream))
        self.last_status = st
        if check:
            _check(st)
        return out.t()

    def info(self):
        inf = dd_info()
        _check(self._lib.dd_get_info(self._ctx, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in dd_info._fields_}

    def interface_dofs(self, dom):
        cnt = C.c_int32()
        _check(self._lib.dd_get_interface_dofs(self._ctx, dom, C.byref(cnt), None))
        out = np.zeros(cnt.value, dtype=np.int32)
        _check(self._lib.dd_get_interface_dofs(self._ctx, dom, C.byref(cnt), _ptr(out, C.c_int32)))
        return out

    def interface_inverse(self, dom, stream=None):
        import torch
        g = len(self.interface_dofs(dom))
        out = torch.empty((g, g), dtype=torch.complex128, device=self.device)
        _check(self._lib.dd_get_interface_inverse(self._ctx, dom, C.c_void_p(out.data_ptr()), self._stream(stream)))
        return out.t()      # column-major result

    def domain_flops(self, dom):
        f = C.c_double()
        _check(self._lib.dd_get_domain_flops(self._ctx, dom, C.byref(f)))
        return f.value

    def tune(self, stream=None):
        """Autotune the Schur-update tile edge per front-size bucket on the
        bound workspace (discards a previous factorisation).  Returns the
        chosen edges (0 for empty buckets)."""
        out = (C.c_int32 * TILE_BUCKETS)()
        _check(self._lib.dd_tune(self._ctx, out, self._stream(stream)))
        return [int(x) for x in out]

    def kernel_timer_start(self, kernel="schur_update"):
        _check(self._lib.dd_kernel_timer_start(self._ctx, -1 if kernel is None else KERNELS[kernel]))

    def kernel_timer_read(self):
        t, n, fl = C.c_double(), C.c_int64(), C.c_double()
        _check(self._lib.dd_kernel_timer_read(self._ctx, C.byref(t), C.byref(n), C.byref(fl)))
        return {"seconds": t.value, "launches": n.value, "flops": fl.value}

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.dd_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
