"""Plain CPU FP64 oracle for the direct domain-decomposition (DD) solve.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the solver.  It shares no code with the
GPU path; its only common input is the seeded problem generator, which holds
none of the method's arithmetic.

What is computed, and where the paper states it (Moshfegh & Vouvakis, "Direct
Solution of FEM Models: Are Sparse Direct Solvers the Best Strategy?"):

* The method is "numerically exact" (Abstract; section II): its result is the
  solution u = A^-1 f of the undecomposed FEM system.  ``global_solve`` is that
  plain definition (SuperLU; ``dense_solve`` is the LAPACK brute force).
* Section II: primal DoFs in the domains plus dual DoFs on the interfaces give
  a sparse arrowhead system [blkdiag(K_i) B^T; B 0] [u; lam] = [f; 0]
  (``arrowhead``).
* Section II: the primal DoFs are eliminated by independent sparse direct
  factorisations of the domain matrices (a FETI-like reduction), leaving the
  symmetric auxiliary matrix F = sum_i B_i K_i^-1 B_i^T with right-hand side
  d = sum_i B_i K_i^-1 f_i.  Only the interface rows/columns of K_i^-1 are
  needed: B_i K_i^-1 B_i^T = B_Gamma (K_i^-1)_GammaGamma B_Gamma^T
  (``interface_inverse``, ``dual_blocks``).
* Section II: the auxiliary system is factored and solved (here with LAPACK /
  SuperLU; the paper's block LDL^T with restricted Bunch-Kaufman pivoting is a
  way of reaching the same lam), then the primal unknowns are recovered by
  independent forward/backward substitutions u_i = K_i^-1 (f_i - B_i^T lam)
  (``serial_dd``).

Every routine is FP64 and uses library primitives (SuperLU, LAPACK) as single
steps, with no blocking or reordering of its own.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def dense_solve(M, F):
    """Brute force: LAPACK zgesv on the densified matrix."""
    M = M.toarray() if sp.issparse(M) else np.asarray(M)
    return np.linalg.solve(M, F)


def global_solve(A, F):
    """Undecomposed sparse direct solve u = A^-1 F (SuperLU, FP64)."""
    lu = spl.splu(sp.csc_matrix(A))
    return lu.solve(np.asarray(F, dtype=np.complex128))


def arrowhead(case, beta_free=False):
    """The assembled saddle-point ("arrowhead") system of section II.

    Returns (M, rhs) with M = [[blkdiag K_i, B^T], [B, 0]] and
    rhs = [f_torn; 0]; unknown ordering = torn domain DoFs then multipliers.
    """
    K = sp.block_diag([d.K for d in case.domains], format="csr")
    B = sp.hstack([case.B(i) for i in range(case.n_dom)], format="csr")
    M = sp.bmat([[K, B.T], [B, None]], format="csr")
    f = case.torn_rhs()
    rhs = np.concatenate([f, np.zeros((case.n_mult, f.shape[1]), complex)])
    return M, rhs


def interface_inverse(K, gamma):
    """(K^-1) restricted to rows/columns ``gamma``: the inverse of the
    interface Schur complement K_GG - K_GI K_II^-1 K_IG.  One sparse direct
    factorisation of K, then solves with the identity columns at gamma."""
    lu = spl.splu(sp.csc_matrix(K))
    E = np.zeros((K.shape[0], len(gamma)), complex)
    E[gamma, np.arange(len(gamma))] = 1.0
    return lu.solve(E)[gamma, :], lu


def dual_blocks(case, i, lu=None):
    """D_i = B_i K_i^-1 B_i^T on the multipliers that touch domain i.

    Returns (mult_ids, D_i dense) with mult_ids the sorted multiplier ids."""
    a, b = case.imap_ptr[i], case.imap_ptr[i + 1]
    mids = case.imap_mult[a:b]
    order = np.argsort(mids, kind="stable")
    mids = mids[order]
    dofs = case.imap_dof[a:b][order]
    sgn = case.imap_sign[a:b][order].astype(float)
    K = case.domains[i].K
    if lu is None:
        lu = spl.splu(sp.csc_matrix(K))
    Bt = np.zeros((K.shape[0], len(mids)), complex)
    Bt[dofs, np.arange(len(mids))] = sgn            # columns of B_i^T
    X = lu.solve(Bt)                                 # K_i^-1 B_i^T
    D = sgn[:, None] * X[dofs, :]                    # B_i X
    return mids, D, lu


def serial_dd(case, F_rhs=None, aux="auto"):
    """Serial DD solve of the arrowhead system (section II), FP64.

    Returns a dict with the per-domain interface inverses, the auxiliary
    matrix F, its right-hand side d, the multipliers lam and the torn
    solution u (stacked by domain)."""
    f_torn = case.f_torn if F_rhs is None else F_rhs
    nm = case.n_mult
    nr = f_torn[0].shape[1]
    rows, cols, vals = [], [], []
    d = np.zeros((nm, nr), complex)
    lus, sinv = [], []
    for i in range(case.n_dom):
        mids, D, lu = dual_blocks(case, i)
        lus.append(lu)
        g = case.gamma(i)
        E = np.zeros((case.domains[i].n, len(g)), complex)
        E[g, np.arange(len(g))] = 1.0
        sinv.append(lu.solve(E)[g, :])
        rr, cc = np.meshgrid(mids, mids, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(D.ravel())
        a, b = case.imap_ptr[i], case.imap_ptr[i + 1]
        y = lu.solve(np.asarray(f_torn[i], complex))
        # d += B_i K_i^-1 f_i
        np.add.at(d, case.imap_mult[a:b], case.imap_sign[a:b][:, None] * y[case.imap_dof[a:b]])
    F = sp.coo_matrix((np.concatenate(vals) if vals else np.zeros(0),
                       (np.concatenate(rows) if rows else np.zeros(0, int),
                        np.concatenate(cols) if cols else np.zeros(0, int))),
                      shape=(nm, nm)).tocsr()
    if nm == 0:
        lam = np.zeros((0, nr), complex)
    elif aux == "dense" or (aux == "auto" and nm <= 4000):
        lam = np.linalg.solve(F.toarray(), d)
    else:
        lam = spl.splu(sp.csc_matrix(F)).solve(d)
    u = []
    for i in range(case.n_dom):
        a, b = case.imap_ptr[i], case.imap_ptr[i + 1]
        rhs = np.array(f_torn[i], complex)
        # f_i - B_i^T lam
        np.add.at(rhs, case.imap_dof[a:b], -case.imap_sign[a:b][:, None] * lam[case.imap_mult[a:b]])
        u.append(lus[i].solve(rhs))
    return dict(S_inv=sinv, F=F, d=d, lam=lam, u=np.concatenate(u, axis=0))


def torn_residual(case, u_torn, lam, f_torn=None):
    """r_i = f_i - K_i u_i - B_i^T lam and r_lam = -sum_i B_i u_i."""
    f_torn = case.f_torn if f_torn is None else f_torn
    off = 0
    r = []
    rl = np.zeros((case.n_mult,) + u_torn.shape[1:], complex)
    for i, dm in enumerate(case.domains):
        ui = u_torn[off:off + dm.n]
        Bi = case.B(i)
        r.append(f_torn[i] - dm.K @ ui - Bi.T @ lam)
        rl -= Bi @ ui
        off += dm.n
    return np.concatenate(r, axis=0), rl


def global_residual(case, u_torn):
    """Per-column ||f - A u|| / ||f|| with u the owner copy of the torn solution."""
    u = case.owner_copy(u_torn)
    r = case.f - case.A @ u
    return np.linalg.norm(r, axis=0) / np.linalg.norm(case.f, axis=0)


def cond1_estimate(A):
    """Estimate of the 1-norm condition number ||A||_1 ||A^-1||_1, the inverse's
    norm by Hager-Higham block estimation (scipy onenormest) on SuperLU
    solves.  It bounds the relative error of a solution by its relative
    residual: err <= cond * resid."""
    lu = spl.splu(sp.csc_matrix(A))
    n = A.shape[0]
    inv = spl.LinearOperator((n, n), matvec=lambda x: lu.solve(np.asarray(x, complex)),
                             rmatvec=lambda x: lu.solve(np.asarray(x, complex), trans="H"),
                             matmat=lambda X: lu.solve(np.asarray(X, complex)), dtype=complex)
    anorm = np.abs(sp.csc_matrix(A)).sum(axis=0).max()
    return float(anorm * spl.onenormest(inv))


def rel_error(u, ref):
    """Per-column ||u - ref||_2 / ||ref||_2."""
    u = np.asarray(u).reshape(ref.shape[0], -1)
    ref = np.asarray(ref).reshape(ref.shape[0], -1)
    return np.linalg.norm(u - ref, axis=0) / np.linalg.norm(ref, axis=0)


def ldl_solve_dense(F, d):
    """Dense symmetric-indefinite (Bunch-Kaufman, LAPACK zsytrf) solve of F lam = d,
    used for the two-domain special case where F is one dense block."""
    lu, dm, perm = sla.ldl(F, lower=True, hermitian=False)
    # F = lu dm lu^T with lu row-permuted: solve in three steps
    L = lu[perm]
    y = sla.solve_triangular(L, d[perm], lower=True, unit_diagonal=True)
    z = np.linalg.solve(dm, y)
    x = sla.solve_triangular(L.T, z, lower=False, unit_diagonal=True)
    out = np.empty_like(x)
    out[perm] = x
    return out
