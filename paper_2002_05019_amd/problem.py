"""Seeded synthetic FEM workloads for the direct domain-decomposition solver.

This module only *builds inputs*: a time-harmonic curl-curl boundary value
problem (curl mu^-1 curl E - k0^2 eps_r E = J) on a hexahedral mesh of the unit
cube, discretised with lowest-order Nedelec (edge) elements, PEC on the outer
boundary, cut into box-shaped domains.  For every domain it produces the
complex-symmetric sparse domain matrix K_i (Robin-regularised, see below), the
signed Boolean interface map B_i (edge Lagrange multipliers), and the torn
right-hand sides.  It contains none of the solver's arithmetic (no
factorisation, no Schur complement, no solve); both the CPU oracle and the GPU
path consume what it returns.

Paper background (section II, Approach): the method re-casts the boundary
value problem on a collection of domains with a mixed/hybrid variational form
in which every domain problem is regular and the whole problem stays
self-adjoint, with primal DoFs in the domain volumes and dual DoFs on the
domain interfaces.  The paper defers the exact formulation to its references,
so the reading used here is:

* +/- Robin regularisation: each interface face mass M_F = int (n x N_a).(n x N_b)
  is added with +j k0 beta to one neighbour and -j k0 beta to the other, so the
  terms cancel on assembly (sum_i R_i^T K_i R_i = A exactly, symmetry kept).
  The sign is +1 on domains of even domain-grid parity.
* Edge multipliers: for an edge owned by domains d1 < d2 < ... < dm, the m-1
  non-redundant "star" constraints u_d1(e) - u_dk(e) = 0 (or the "chain"
  variant u_d(k-1)(e) - u_dk(e) = 0, used to check constraint-choice
  invariance).
* Right-hand side: i.i.d. (N(0,1) + jN(0,1))/sqrt(2) per non-PEC edge and
  column; the full value goes to the lowest-id owner of the edge.

Seeds: ``numpy.random.default_rng([seed, stream])`` with stream 0 = node
jitter, 1 = materials, 2 = domain cuts, 3 = right-hand sides.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------
# 1-D Gauss-Legendre (3 points) on [0, 1]: exact to degree 5.
_G3X = np.array([0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6)])
_G3W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])


def _hat(a, t):
    """1-D hat functions on [0,1]: l_0 = 1 - t, l_1 = t."""
    return t if a else 1.0 - t


def _dhat(a):
    return 1.0 if a else -1.0


# Local edge table of the reference hexahedron [0,1]^3.  Edges 0-3 run along
# xi at (eta0, zeta0); 4-7 along eta at (xi0, zeta0); 8-11 along zeta at
# (xi0, eta0); the corner pairs are (0,0), (1,0), (0,1), (1,1).  All edges are
# oriented along +reference axis, which matches the global +axis orientation of
# the structured mesh, so no orientation signs are needed.
_CORNERS = ((0, 0), (1, 0), (0, 1), (1, 1))


def _reference_basis(xq):
    """Reference edge functions and their curls at points xq (Q,3).

    Returns N (Q,12,3), C (Q,12,3) in reference coordinates.
    """
    Q = xq.shape[0]
    N = np.zeros((Q, 12, 3))
    C = np.zeros((Q, 12, 3))
    xi, eta, zeta = xq[:, 0], xq[:, 1], xq[:, 2]
    for m, (a, b) in enumerate(_CORNERS):
        # xi-edge at (eta=a, zeta=b): N = l_a(eta) l_b(zeta) e_xi
        N[:, m, 0] = _hat(a, eta) * _hat(b, zeta)
        C[:, m, 1] = _hat(a, eta) * _dhat(b)
        C[:, m, 2] = -_dhat(a) * _hat(b, zeta)
        # eta-edge at (xi=a, zeta=b): N = l_a(xi) l_b(zeta) e_eta
        N[:, 4 + m, 1] = _hat(a, xi) * _hat(b, zeta)
        C[:, 4 + m, 0] = -_hat(a, xi) * _dhat(b)
        C[:, 4 + m, 2] = _dhat(a) * _hat(b, zeta)
        # zeta-edge at (xi=a, eta=b): N = l_a(xi) l_b(eta) e_zeta
        N[:, 8 + m, 2] = _hat(a, xi) * _hat(b, eta)
        C[:, 8 + m, 0] = _hat(a, xi) * _dhat(b)
        C[:, 8 + m, 1] = -_dhat(a) * _hat(b, eta)
    return N, C


def _gauss_cube():
    g = np.array([(x, y, z) for z in _G3X for y in _G3X for x in _G3X])
    w = np.array([wx * wy * wz for wz in _G3W for wy in _G3W for wx in _G3W])
    return g, w


_QX, _QW = _gauss_cube()
_NREF, _CREF = _reference_basis(_QX)


def _shape_grads(xq):
    """Trilinear shape functions (Q,8) and reference gradients (Q,8,3)."""
    Q = xq.shape[0]
    phi = np.zeros((Q, 8))
    dphi = np.zeros((Q, 8, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                n = a + 2 * b + 4 * c
                lx, ly, lz = _hat(a, xq[:, 0]), _hat(b, xq[:, 1]), _hat(c, xq[:, 2])
                phi[:, n] = lx * ly * lz
                dphi[:, n, 0] = _dhat(a) * ly * lz
                dphi[:, n, 1] = lx * _dhat(b) * lz
                dphi[:, n, 2] = lx * ly * _dhat(c)
    return phi, dphi


_PHI, _DPHI = _shape_grads(_QX)


def element_jacobians(X):
    """X: (E,8,3) element node coordinates -> J (E,Q,3,3), J[...,a,b] = dx_a/dxi_b."""
    return np.einsum("ena,qnb->eqab", X, _DPHI)


def element_matrices(X):
    """Curl-curl (S) and mass (T) matrices of hexahedral edge elements.

    X: (E,8,3) node coordinates (local node a + 2b + 4c at reference corner
    (a, b, c)).  Covariant map N = J^-T N_ref, curl N = J curl_ref N_ref / det J,
    3x3x3 Gauss quadrature.  Returns S, T of shape (E,12,12), mu_r = eps_r = 1.
    """
    J = element_jacobians(X)
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0):
        raise ValueError("inverted element")
    G = np.einsum("eqab,eqac->eqbc", J, J)          # J^T J
    Ginv = np.linalg.inv(G)
    wS = _QW[None, :] / detJ                          # w / det J
    wT = _QW[None, :] * detJ
    S = np.einsum("eq,qai,eqij,qbj->eab", wS, _CREF, G, _CREF, optimize=True)
    T = np.einsum("eq,qai,eqij,qbj->eab", wT, _NREF, Ginv, _NREF, optimize=True)
    return S, T


# ----------------------------------------------------------------------------
# Face (interface) mass matrices: tangential traces of the 4 edges of a quad
# face.  Face parameters (u, v) in [0,1]^2, face nodes x_{bc} at (u=b, v=c);
# edges 0,1 run along u at v = 0, 1; edges 2,3 run along v at u = 0, 1.
_G2 = np.array([(u, v) for v in _G3X for u in _G3X])
_W2 = np.array([wu * wv for wv in _G3W for wu in _G3W])


def face_mass_matrices(Y):
    """Y: (F,4,3) face node coordinates (index b + 2c) -> M (F,4,4).

    M_ab = int_F (n x N_a).(n x N_b) dS = int N_ref_a^T G^-1 N_ref_b sqrt(det G) du dv
    with G the surface metric (the tangential trace of a covariantly mapped
    edge function has the reference covariant components).
    """
    u, v = _G2[:, 0], _G2[:, 1]
    dphi = np.zeros((len(u), 4, 2))
    for c in range(2):
        for b in range(2):
            n = b + 2 * c
            dphi[:, n, 0] = _dhat(b) * _hat(c, v)
            dphi[:, n, 1] = _hat(b, u) * _dhat(c)
    Nr = np.zeros((len(u), 4, 2))
    Nr[:, 0, 0] = 1 - v
    Nr[:, 1, 0] = v
    Nr[:, 2, 1] = 1 - u
    Nr[:, 3, 1] = u
    Js = np.einsum("fna,qnb->fqab", Y, dphi)          # (F,Q,3,2)
    G = np.einsum("fqab,fqac->fqbc", Js, Js)          # (F,Q,2,2)
    detG = G[..., 0, 0] * G[..., 1, 1] - G[..., 0, 1] * G[..., 1, 0]
    Ginv = np.empty_like(G)
    Ginv[..., 0, 0] = G[..., 1, 1] / detG
    Ginv[..., 1, 1] = G[..., 0, 0] / detG
    Ginv[..., 0, 1] = -G[..., 0, 1] / detG
    Ginv[..., 1, 0] = -G[..., 1, 0] / detG
    w = _W2[None, :] * np.sqrt(detG)
    return np.einsum("fq,qai,fqij,qbj->fab", w, Nr, Ginv, Nr, optimize=True)


# ----------------------------------------------------------------------------
@dataclass
class CaseSpec:
    """Workload description.  ``cuts`` gives, per axis, the element indices of
    the domain boundaries (first 0, last n); ``cuts=None`` with ``random_cuts``
    draws them (stream 2)."""
    n: int
    cuts: tuple | None
    k0: float
    eps_lo: float
    eps_hi: float
    tan_delta: float
    jitter: float = 0.0
    nrhs: int = 1
    seed: int = 0
    beta: float = 1.0
    constraints: str = "star"
    random_cuts: tuple | None = None   # (n_parts, w_min, w_max) per axis
    name: str = ""


def _k0_ppw(n, eps_max, ppw=10.0):
    """k0 giving ``ppw`` elements per wavelength in the densest material."""
    h = 1.0 / n
    return 2.0 * math.pi / (ppw * h * math.sqrt(eps_max))


def even_cuts(n, parts):
    return tuple(tuple(int(round(i * n / parts)) for i in range(parts + 1)) for _ in range(3))


def named_spec(name: str) -> CaseSpec:
    """The workloads the solver is exercised and measured on."""
    if name == "cube6":      # 6^3 elements, 2^3 domains of 3^3, 1 RHS
        return CaseSpec(n=6, cuts=even_cuts(6, 2), k0=2 * math.pi, eps_lo=2.0, eps_hi=2.0,
                        tan_delta=0.02, nrhs=1, seed=1, name=name)
    if name == "cube48":     # 48^3 elements, 4^3 domains of 12^3, 8 RHS
        return CaseSpec(n=48, cuts=even_cuts(48, 4), k0=_k0_ppw(48, 4.0), eps_lo=1.0,
                        eps_hi=4.0, tan_delta=0.02, nrhs=8, seed=2, name=name)
    if name == "cube64j":    # 64^3 jittered, 216 uneven domains (6^3 .. 14^3), 64 RHS
        return CaseSpec(n=64, cuts=None, random_cuts=(6, 6, 14), k0=_k0_ppw(64, 8.0),
                        eps_lo=1.0, eps_hi=8.0, tan_delta=0.02, jitter=0.2, nrhs=64,
                        seed=4, name=name)
    if name == "cube96j":    # 96^3 jittered, 8^3 domains of 12^3, 256 RHS
        return CaseSpec(n=96, cuts=even_cuts(96, 8), k0=_k0_ppw(96, 4.0), eps_lo=1.0,
                        eps_hi=4.0, tan_delta=0.01, jitter=0.2, nrhs=256, seed=5, name=name)
    # small parity cases spanning several tiles
    if name == "cube12":     # 12^3, 2^3 domains of 6^3
        return CaseSpec(n=12, cuts=even_cuts(12, 2), k0=_k0_ppw(12, 3.0), eps_lo=1.0,
                        eps_hi=3.0, tan_delta=0.02, nrhs=3, seed=12, name=name)
    if name == "cube16":     # 16^3, 2^3 domains of 8^3
        return CaseSpec(n=16, cuts=even_cuts(16, 2), k0=_k0_ppw(16, 4.0), eps_lo=1.0,
                        eps_hi=4.0, tan_delta=0.02, nrhs=4, seed=16, name=name)
    if name == "cube18u":    # 18^3 jittered, uneven 3x2x2 cuts
        return CaseSpec(n=18, cuts=((0, 5, 11, 18), (0, 8, 18), (0, 10, 18)),
                        k0=_k0_ppw(18, 4.0), eps_lo=1.0, eps_hi=4.0, tan_delta=0.02,
                        jitter=0.2, nrhs=5, seed=18, name=name)
    if name == "cube24":     # 24^3, 3^3 domains of 8^3
        return CaseSpec(n=24, cuts=even_cuts(24, 3), k0=_k0_ppw(24, 4.0), eps_lo=1.0,
                        eps_hi=4.0, tan_delta=0.02, nrhs=8, seed=24, name=name)
    raise KeyError(name)


# ----------------------------------------------------------------------------
@dataclass
class Domain:
    box: tuple                 # ((x0,x1),(y0,y1),(z0,z1)) in element indices
    n: int                     # local (non-PEC) unknowns
    l2g: np.ndarray            # local -> global non-PEC edge index
    xyz: np.ndarray            # (n,3) float32 logical edge midpoints (units of h)
    sigma: int                 # Robin sign
    A: sp.csr_matrix           # domain stiffness without Robin terms
    K: sp.csr_matrix           # A + j k0 beta sigma sum_F M_F  (sorted, symmetric pattern)


@dataclass
class Case:
    spec: CaseSpec
    n_global: int
    domains: list
    n_mult: int
    imap_ptr: np.ndarray       # (n_dom+1,) int64
    imap_dof: np.ndarray       # int32
    imap_mult: np.ndarray      # int64
    imap_sign: np.ndarray      # int8
    f: np.ndarray              # (n_global, nrhs) complex128
    f_torn: list               # per-domain (n_i, nrhs)
    eps: np.ndarray            # per-element complex eps_r, shape (n,n,n) [i,j,k]
    nodes: np.ndarray          # (n+1,n+1,n+1,3) node coordinates [i,j,k]
    gmap: np.ndarray           # full edge id -> non-PEC index or -1
    _A: sp.csr_matrix | None = field(default=None, repr=False)

    @property
    def n_dom(self):
        return len(self.domains)

    def B(self, i):
        """Signed Boolean interface block B_i (n_mult x n_i)."""
        a, b = self.imap_ptr[i], self.imap_ptr[i + 1]
        d = self.domains[i]
        return sp.csr_matrix((self.imap_sign[a:b].astype(np.float64),
                              (self.imap_mult[a:b], self.imap_dof[a:b])),
                             shape=(self.n_mult, d.n))

    def gamma(self, i):
        """Sorted local dofs of domain i that carry a multiplier."""
        a, b = self.imap_ptr[i], self.imap_ptr[i + 1]
        return np.unique(self.imap_dof[a:b])

    @property
    def A(self):
        if self._A is None:
            self._A = assemble_global(self)
        return self._A

    def torn_rhs(self):
        """(sum n_i, nrhs) torn right-hand side, domains stacked in order."""
        return np.concatenate(self.f_torn, axis=0)

    def owner_copy(self, u_torn):
        """Global solution from the lowest-id owner copy of every edge."""
        u = np.zeros((self.n_global,) + u_torn.shape[1:], dtype=u_torn.dtype)
        off = 0
        seen = np.zeros(self.n_global, bool)
        for d in self.domains:
            blk = u_torn[off:off + d.n]
            new = ~seen[d.l2g]
            u[d.l2g[new]] = blk[new]
            seen[d.l2g] = True
            off += d.n
        return u

    def values_digest(self):
        h = hashlib.sha256()
        for d in self.domains:
            h.update(np.ascontiguousarray(d.K.data).tobytes())
        h.update(np.ascontiguousarray(self.f).tobytes())
        return h.hexdigest()


# ----------------------------------------------------------------------------
# Structured edge numbering on an n^3 element grid.
def _edge_ids(n):
    nx = n * (n + 1) * (n + 1)

    def xe(i, j, k):
        return i + n * (j + (n + 1) * k)

    def ye(i, j, k):
        return nx + i + (n + 1) * (j + n * k)

    def ze(i, j, k):
        return 2 * nx + i + (n + 1) * (j + (n + 1) * k)
    return xe, ye, ze, 3 * nx


def _element_edges(n, I, Jj, K):
    """Global edge ids (E,12) of elements with indices I, Jj, K (arrays)."""
    xe, ye, ze, _ = _edge_ids(n)
    cols = []
    for a, b in _CORNERS:
        cols.append(xe(I, Jj + a, K + b))
    for a, b in _CORNERS:
        cols.append(ye(I + a, Jj, K + b))
    for a, b in _CORNERS:
        cols.append(ze(I + a, Jj + b, K))
    return np.stack(cols, axis=1)


def _edge_midpoints_logical(n):
    """(n_edges,3) logical midpoints of all edges (units of h)."""
    xe, ye, ze, ne = _edge_ids(n)
    out = np.zeros((ne, 3), np.float32)
    r = np.arange(n + 1)
    s = np.arange(n)
    i, j, k = np.meshgrid(s, r, r, indexing="ij")
    out[xe(i, j, k).ravel()] = np.stack([i + 0.5, j, k], -1).reshape(-1, 3)
    i, j, k = np.meshgrid(r, s, r, indexing="ij")
    out[ye(i, j, k).ravel()] = np.stack([i, j + 0.5, k], -1).reshape(-1, 3)
    i, j, k = np.meshgrid(r, r, s, indexing="ij")
    out[ze(i, j, k).ravel()] = np.stack([i, j, k + 0.5], -1).reshape(-1, 3)
    return out


def _pec_mask(n):
    """True for edges lying in the outer boundary (removed by PEC)."""
    xe, ye, ze, ne = _edge_ids(n)
    m = np.zeros(ne, bool)
    r = np.arange(n + 1)
    s = np.arange(n)
    i, j, k = np.meshgrid(s, r, r, indexing="ij")
    m[xe(i, j, k).ravel()] = ((j == 0) | (j == n) | (k == 0) | (k == n)).ravel()
    i, j, k = np.meshgrid(r, s, r, indexing="ij")
    m[ye(i, j, k).ravel()] = ((i == 0) | (i == n) | (k == 0) | (k == n)).ravel()
    i, j, k = np.meshgrid(r, r, s, indexing="ij")
    m[ze(i, j, k).ravel()] = ((i == 0) | (i == n) | (j == 0) | (j == n)).ravel()
    return m


def _random_cuts(rng, n, parts, wmin, wmax):
    """Rejection-sample ``parts`` integer widths in [wmin, wmax] summing to n."""
    for _ in range(100000):
        w = rng.integers(wmin, wmax + 1, size=parts)
        if w.sum() == n:
            return tuple(int(x) for x in np.concatenate([[0], np.cumsum(w)]))
    raise RuntimeError("could not draw cuts")


def make_nodes(spec: CaseSpec):
    n = spec.n
    h = 1.0 / n
    r = np.arange(n + 1) * h
    X = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1)
    if spec.jitter > 0:
        rng = np.random.default_rng([spec.seed, 0])
        J = rng.uniform(-spec.jitter * h, spec.jitter * h, size=X.shape)
        J[0, :, :] = J[n, :, :] = 0.0
        J[:, 0, :] = J[:, n, :] = 0.0
        J[:, :, 0] = J[:, :, n] = 0.0
        X = X + J
    return X


def make_materials(spec: CaseSpec):
    n = spec.n
    if spec.eps_lo == spec.eps_hi:
        ep = np.full((n, n, n), spec.eps_lo)
    else:
        rng = np.random.default_rng([spec.seed, 1])
        ep = rng.uniform(spec.eps_lo, spec.eps_hi, size=(n, n, n))
    return ep * (1.0 - 1j * spec.tan_delta)


def element_nodes(nodes, I, Jj, K):
    cols = []
    for c in range(2):
        for b in range(2):
            for a in range(2):
                cols.append(nodes[I + a, Jj + b, K + c])
    return np.stack(cols, axis=1)


def assemble(n, nodes, eps, k0, elems, gmap, nloc, g2l=None):
    """Assemble S - k0^2 eps T over element index triples ``elems`` (3 arrays)."""
    I, Jj, K = elems
    X = element_nodes(nodes, I, Jj, K)
    rel = X - X[:, :1, :]
    if len(X) > 1 and np.ptp(rel, axis=0).max() <= 1e-13 * max(1.0, np.abs(rel).max()):
        # every element is a translate of the first one: one quadrature suffices
        S1, T1 = element_matrices(X[:1])
        S = np.broadcast_to(S1, (len(X), 12, 12))
        T = np.broadcast_to(T1, (len(X), 12, 12))
    else:
        S, T = element_matrices(X)
    Ae = S - (k0 ** 2) * eps[I, Jj, K][:, None, None] * T
    ge = _element_edges(n, I, Jj, K)
    le = gmap[ge]
    if g2l is not None:
        le = np.where(le >= 0, g2l[np.maximum(le, 0)], -1)
    keep = le >= 0
    rr = np.repeat(le[:, :, None], 12, axis=2)
    cc = np.repeat(le[:, None, :], 12, axis=1)
    m = keep[:, :, None] & keep[:, None, :]
    M = sp.coo_matrix((Ae[m], (rr[m], cc[m])), shape=(nloc, nloc)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return M


def assemble_global(case: Case) -> sp.csr_matrix:
    """Global (undecomposed) FEM matrix A on the non-PEC edges."""
    s = case.spec
    n = s.n
    idx = np.arange(n)
    I, Jj, K = [a.ravel() for a in np.meshgrid(idx, idx, idx, indexing="ij")]
    return assemble(n, case.nodes, case.eps, s.k0, (I, Jj, K), case.gmap, case.n_global)


def make_case(spec: CaseSpec | str) -> Case:
    if isinstance(spec, str):
        spec = named_spec(spec)
    n = spec.n
    xe, ye, ze, ne = _edge_ids(n)
    pec = _pec_mask(n)
    gmap = np.full(ne, -1, np.int64)
    gmap[~pec] = np.arange(int((~pec).sum()))
    n_global = int((~pec).sum())
    mid = _edge_midpoints_logical(n)
    nodes = make_nodes(spec)
    eps = make_materials(spec)

    if spec.cuts is not None:
        cuts = spec.cuts
    else:
        rng = np.random.default_rng([spec.seed, 2])
        p, lo, hi = spec.random_cuts
        cuts = tuple(_random_cuts(rng, n, p, lo, hi) for _ in range(3))
    P = [len(c) - 1 for c in cuts]

    # element -> domain
    dom_of_axis = []
    for ax in range(3):
        a = np.zeros(n, np.int64)
        for p in range(P[ax]):
            a[cuts[ax][p]:cuts[ax][p + 1]] = p
        dom_of_axis.append(a)

    def dom_id(p, q, r):
        return p + P[0] * (q + P[1] * r)

    n_dom = P[0] * P[1] * P[2]
    boxes = [None] * n_dom
    for r in range(P[2]):
        for q in range(P[1]):
            for p in range(P[0]):
                boxes[dom_id(p, q, r)] = ((cuts[0][p], cuts[0][p + 1]), (cuts[1][q], cuts[1][q + 1]),
                                          (cuts[2][r], cuts[2][r + 1]), (p, q, r))

    # ---- per-domain edge sets and local numbering
    dom_edges = []
    for d in range(n_dom):
        (x0, x1), (y0, y1), (z0, z1), _ = boxes[d]
        ids = []
        i, j, k = np.meshgrid(np.arange(x0, x1), np.arange(y0, y1 + 1), np.arange(z0, z1 + 1), indexing="ij")
        ids.append(xe(i, j, k).ravel(order="F"))
        i, j, k = np.meshgrid(np.arange(x0, x1 + 1), np.arange(y0, y1), np.arange(z0, z1 + 1), indexing="ij")
        ids.append(ye(i, j, k).ravel(order="F"))
        i, j, k = np.meshgrid(np.arange(x0, x1 + 1), np.arange(y0, y1 + 1), np.arange(z0, z1), indexing="ij")
        ids.append(ze(i, j, k).ravel(order="F"))
        ids = np.concatenate(ids)
        ids = ids[~pec[ids]]
        dom_edges.append(gmap[ids])          # local -> global non-PEC index

    # owner lists of every global unknown
    cnt = np.zeros(n_global, np.int64)
    for d in range(n_dom):
        cnt[dom_edges[d]] += 1
    shared = np.nonzero(cnt > 1)[0]
    own_ptr = np.zeros(n_global + 1, np.int64)
    own_ptr[1:] = np.cumsum(cnt)
    own = np.empty(own_ptr[-1], np.int64)
    own_loc = np.empty(own_ptr[-1], np.int64)
    fill = own_ptr[:-1].copy()
    for d in range(n_dom):   # ascending d -> owner lists sorted
        g = dom_edges[d]
        own[fill[g]] = d
        own_loc[fill[g]] = np.arange(len(g))
        fill[g] += 1

    # ---- multipliers (star or chain), ordered by global edge then pair
    m_dom, m_dof, m_id, m_sign = [], [], [], []
    mid_count = 0
    for e in shared:
        a, b = own_ptr[e], own_ptr[e + 1]
        ds, ls = own[a:b], own_loc[a:b]
        for kk in range(1, b - a):
            i0 = 0 if spec.constraints == "star" else kk - 1
            m_dom += [ds[i0], ds[kk]]
            m_dof += [ls[i0], ls[kk]]
            m_id += [mid_count, mid_count]
            m_sign += [1, -1]
            mid_count += 1
    m_dom = np.array(m_dom, np.int64)
    order = np.lexsort((np.array(m_id), m_dom))
    imap_ptr = np.zeros(n_dom + 1, np.int64)
    np.add.at(imap_ptr, m_dom + 1, 1)
    imap_ptr = np.cumsum(imap_ptr)
    imap_dof = np.array(m_dof, np.int64)[order].astype(np.int32)
    imap_mult = np.array(m_id, np.int64)[order]
    imap_sign = np.array(m_sign, np.int64)[order].astype(np.int8)

    # ---- domain matrices with +/- Robin face terms
    domains = []
    h = 1.0 / n
    for d in range(n_dom):
        (x0, x1), (y0, y1), (z0, z1), (p, q, r) = boxes[d]
        g = dom_edges[d]
        nloc = len(g)
        g2l = np.full(n_global, -1, np.int64)
        g2l[g] = np.arange(nloc)
        I, Jj, K = [a.ravel() for a in np.meshgrid(np.arange(x0, x1), np.arange(y0, y1),
                                                   np.arange(z0, z1), indexing="ij")]
        A = assemble(n, nodes, eps, spec.k0, (I, Jj, K), gmap, nloc, g2l)
        sigma = 1 if (p + q + r) % 2 == 0 else -1
        R = _robin_faces(n, nodes, gmap, g2l, nloc, boxes[d], cuts)
        K = (A + (1j * spec.k0 * spec.beta * sigma) * R).tocsr()
        K.sum_duplicates()
        K.sort_indices()
        domains.append(Domain(box=boxes[d][:3], n=nloc, l2g=g,
                              xyz=np.ascontiguousarray(mid[np.nonzero(~pec)[0][g]]),
                              sigma=sigma, A=A, K=K))

    # ---- right-hand sides
    rng = np.random.default_rng([spec.seed, 3])
    z = rng.standard_normal((n_global, spec.nrhs, 2))
    f = (z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0)
    first = own[own_ptr[:-1]]
    f_torn = []
    for d in range(n_dom):
        g = dom_edges[d]
        fd = np.where((first[g] == d)[:, None], f[g], 0.0)
        f_torn.append(np.ascontiguousarray(fd))

    return Case(spec=spec, n_global=n_global, domains=domains, n_mult=mid_count,
                imap_ptr=imap_ptr, imap_dof=imap_dof, imap_mult=imap_mult,
                imap_sign=imap_sign, f=f, f_torn=f_torn, eps=eps, nodes=nodes, gmap=gmap)


def _robin_faces(n, nodes, gmap, g2l, nloc, box, cuts):
    """Sum of interface face masses M_F over the domain's faces that lie on an
    internal cut plane (local numbering)."""
    xe, ye, ze, _ = _edge_ids(n)
    (x0, x1), (y0, y1), (z0, z1), _ = box
    rows, cols, vals = [], [], []
    for ax in range(3):
        lo_hi = [(x0, x1), (y0, y1), (z0, z1)][ax]
        for plane in lo_hi:
            if plane == 0 or plane == n:
                continue
            # face grid on this plane over the domain's extent in the other two axes
            o = [a for a in range(3) if a != ax]
            rng_u = np.arange(*[(x0, x1), (y0, y1), (z0, z1)][o[0]])
            rng_v = np.arange(*[(x0, x1), (y0, y1), (z0, z1)][o[1]])
            U, V = [a.ravel() for a in np.meshgrid(rng_u, rng_v, indexing="ij")]
            idx = [None, None, None]
            idx[ax] = np.full_like(U, plane)
            idx[o[0]] = U
            idx[o[1]] = V
            # face nodes (b + 2c) at (u=b, v=c)
            Y = []
            for c in range(2):
                for b in range(2):
                    ii = [idx[0].copy(), idx[1].copy(), idx[2].copy()]
                    ii[o[0]] += b
                    ii[o[1]] += c
                    Y.append(nodes[ii[0], ii[1], ii[2]])
            Y = np.stack(Y, axis=1)
            M = face_mass_matrices(Y)
            # edges: along u at v=0,1 ; along v at u=0,1
            edge_fn = [xe, ye, ze]

            def eid(axis_dir, du, dv):
                ii = [idx[0].copy(), idx[1].copy(), idx[2].copy()]
                ii[o[0]] += du
                ii[o[1]] += dv
                return edge_fn[axis_dir](ii[0], ii[1], ii[2])
            E = np.stack([eid(o[0], 0, 0), eid(o[0], 0, 1), eid(o[1], 0, 0), eid(o[1], 1, 0)], 1)
            le = gmap[E]
            le = np.where(le >= 0, g2l[np.maximum(le, 0)], -1)
            keep = le >= 0
            rr = np.repeat(le[:, :, None], 4, axis=2)
            cc = np.repeat(le[:, None, :], 4, axis=1)
            m = keep[:, :, None] & keep[:, None, :]
            rows.append(rr[m])
            cols.append(cc[m])
            vals.append(M[m])
    if not rows:
        return sp.csr_matrix((nloc, nloc))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nloc, nloc)).tocsr()


# ----------------------------------------------------------------------------
def flat_inputs(case: Case):
    """Concatenated arrays in the layout the C ABI consumes."""
    doms = case.domains
    rowptr = [d.K.indptr.astype(np.int64) for d in doms]
    colind = [d.K.indices.astype(np.int32) for d in doms]
    vals = np.concatenate([d.K.data.astype(np.complex128) for d in doms])
    xyz = np.concatenate([d.xyz for d in doms]).astype(np.float32)
    return dict(rowptr=rowptr, colind=colind, vals=vals, xyz=xyz,
                nnz=[int(d.K.nnz) for d in doms], n=[d.n for d in doms])
