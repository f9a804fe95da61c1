"""Pins of the unstructured tetrahedral generator and its graph partitioner
(no GPU): closed-form Whitney element matrices against quadrature, de Rham
exactness, first-order convergence to an analytic field, Robin cancellation
on irregular interfaces, the partitioner's invariants, and the oracle's DD
solve on these meshes against the undecomposed solve."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
from paper_2002_05019_amd import tetmesh as TM

# 4-point rule on a tetrahedron, exact for quadratics (barycentric a,b,b,b)
_QA, _QB = 0.5854101966249685, 0.1381966011250105
_QL = np.array([[_QA, _QB, _QB, _QB], [_QB, _QA, _QB, _QB], [_QB, _QB, _QA, _QB], [_QB, _QB, _QB, _QA]])
# 3-point rule on a triangle, exact for quadratics
_TL = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])

_CASES = {}


def _case(name):
    if name not in _CASES:
        _CASES[name] = TM.make_tet_case(name)
    return _CASES[name]


def _whitney_at(g, lam):
    """N_e at points with barycentric coordinates lam (Q, 4): (T, Q, 6, 3)."""
    ea, eb = TM.TET_EDGES[:, 0], TM.TET_EDGES[:, 1]
    return (lam[None, :, ea, None] * g[:, None, eb, :] - lam[None, :, eb, None] * g[:, None, ea, :])


def test_element_matrices_against_quadrature():
    rng = np.random.default_rng(5)
    P = rng.standard_normal((20, 4, 3))
    S, T = TM.whitney_matrices(P)
    g, V = TM.barycentric_gradients(P)
    N = _whitney_at(g, _QL)                                      # (T, 4, 6, 3)
    Tq = np.einsum("t,tqei,tqfi->tef", V / 4, N, N)
    assert np.abs(T - Tq).max() <= 1e-12 * np.abs(T).max()
    # curl N_e = 2 grad l_a x grad l_b is constant: S = V curl N . curl N
    c = 2 * np.cross(g[:, TM.TET_EDGES[:, 0]], g[:, TM.TET_EDGES[:, 1]])
    assert np.abs(S - V[:, None, None] * np.einsum("tei,tfi->tef", c, c)).max() <= 1e-12 * np.abs(S).max()
    # symmetric, T positive definite
    assert np.abs(T - T.transpose(0, 2, 1)).max() == 0
    assert np.linalg.eigvalsh(T).min() > 0


def test_face_mass_against_quadrature():
    rng = np.random.default_rng(6)
    Q = rng.standard_normal((15, 3, 3))
    M = TM.face_mass(Q)
    e1, e2 = Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0]
    nrm = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(nrm, axis=1)
    n = nrm / (2 * area[:, None])
    # tangential part of the tetrahedral Whitney function of a face edge: use
    # a tetrahedron on the face with an arbitrary apex, project n x N
    P = np.concatenate([Q, (Q.mean(axis=1) + n)[:, None, :]], axis=1)
    g, _ = TM.barycentric_gradients(P)
    lam = np.concatenate([_TL, np.zeros((3, 1))], axis=1)
    N = _whitney_at(g, lam)                                      # (F, 3, 6, 3)
    face_edges = [0, 1, 3]                                       # (0,1) (0,2) (1,2) among TET_EDGES
    nxN = np.cross(n[:, None, None, :], N[:, :, face_edges, :])
    Mq = np.einsum("f,fqei,fqgi->feg", area / 3, nxN, nxN)
    assert np.abs(M - Mq).max() <= 1e-12 * np.abs(M).max()


@pytest.mark.parametrize("name", ["tet8", "tet12s"])
def test_curl_kills_gradients(name):
    """de Rham exactness on the unstructured mesh: S G = 0 for the discrete
    gradient G (node values -> edge differences, edges oriented low -> high)."""
    c = _case(name)
    nn = c.nodes.shape[0]
    E = len(c.edges)
    G = sp.csr_matrix((np.r_[-np.ones(E), np.ones(E)], (np.r_[np.arange(E), np.arange(E)],
                                                        np.r_[c.edges[:, 0], c.edges[:, 1]])), shape=(E, nn))
    S, _ = TM.whitney_matrices(c.nodes[c.tets])
    sg = c.tet_signs[:, :, None] * c.tet_signs[:, None, :]
    rr = np.repeat(c.tet_edges, 6, axis=1).ravel()
    cc = np.tile(c.tet_edges, (1, 6)).ravel()
    Sg = sp.csr_matrix(((S * sg).ravel(), (rr, cc)), shape=(E, E))
    phi = np.random.default_rng(7).standard_normal(nn)
    assert np.abs(Sg @ (G @ phi)).max() <= 1e-11 * abs(Sg).max() * np.abs(phi).max()


@pytest.mark.parametrize("name", ["tet8", "tet12s", "tet16"])
def test_robin_terms_cancel_and_partition(name):
    """sum_i R_i^T K_i R_i = A on irregular interfaces; the partitioner gives
    every element one domain, balanced parts, and connected growing."""
    c = _case(name)
    acc = sp.csr_matrix((c.n_global, c.n_global), dtype=complex)
    for d in c.domains:
        R = sp.csr_matrix((np.ones(d.n), (np.arange(d.n), d.l2g)), shape=(d.n, c.n_global))
        acc = acc + R.T @ d.K @ R
    assert abs(acc - c.A).max() <= 1e-13 * abs(c.A).max()
    sizes = np.bincount(c.part)
    assert len(sizes) == c.spec.n_dom and sizes.sum() == len(c.tets)
    assert sizes.max() <= 1.2 * len(c.tets) / c.spec.n_dom
    # every multiplier ties two copies of one edge
    own = np.concatenate([c.domains[i].l2g[c.imap_dof[c.imap_ptr[i]:c.imap_ptr[i + 1]]] for i in range(c.n_dom)])
    mult = c.imap_mult
    order = np.argsort(mult, kind="stable")
    pairs = own[order].reshape(-1, 2)
    assert np.all(pairs[:, 0] == pairs[:, 1])


def test_partitioner_refinement_lowers_the_cut():
    c = _case("tet16")
    ptr, adj = TM.dual_graph(c.tets)
    refined = TM.partition(ptr, adj, 8)
    # growing only: with no balance slack no vertex may move
    plain = TM.partition(ptr, adj, 8, imbalance=0.0)
    cr, cp = TM.cut_edges(ptr, adj, refined), TM.cut_edges(ptr, adj, plain)
    print(f"[tet] tet16 into 8: cut {cp} by growing, {cr} refined")
    assert cr < cp
    assert np.bincount(refined).max() <= 1.05 * len(c.tets) / 8


@pytest.mark.parametrize("name", ["tet8", "tet12s"])
def test_dd_on_tetrahedra_is_numerically_exact(name):
    c = _case(name)
    out = oracle.serial_dd(c)
    ref = oracle.global_solve(c.A, c.f)
    assert oracle.rel_error(c.owner_copy(out["u"]), ref).max() < 1e-11
    assert oracle.global_residual(c, out["u"]).max() < 1e-12
    F = out["F"].toarray()
    assert np.abs(F - F.T).max() <= 1e-13 * np.abs(F).max()


def _tet_error(n, k0=1.0):
    """Relative L2 error of the edge-element solution of the analytic field
    on the whole unit cube (uniform Kuhn mesh, PEC walls)."""
    rng = np.random.default_rng(0)
    nodes, tets = TM.kuhn_mesh(n, 0.0, rng)
    edges, te, tsg = TM.mesh_edges(tets)
    faces, _, fcnt = TM.mesh_faces(tets)
    bf = faces[fcnt == 1]
    nn = len(nodes)
    bkey = np.unique(np.concatenate([np.sort(bf[:, p], axis=1) for p in ([0, 1], [0, 2], [1, 2])]) @ [nn, 1])
    pec = np.isin(edges @ [nn, 1], bkey)
    gm = -np.ones(len(edges), np.int64)
    gm[~pec] = np.arange(int((~pec).sum()))
    S, T = TM.whitney_matrices(nodes[tets])
    sg = tsg[:, :, None] * tsg[:, None, :]
    Ae = (S - k0 ** 2 * T) * sg
    li = gm[te]
    rr, cc = np.repeat(li, 6, axis=1).ravel(), np.tile(li, (1, 6)).ravel()
    ok = (rr >= 0) & (cc >= 0)
    A = sp.csr_matrix((Ae.ravel()[ok], (rr[ok], cc[ok])), shape=(int((~pec).sum()),) * 2)
    g, V = TM.barycentric_gradients(nodes[tets])
    N = _whitney_at(g, _QL) * tsg[:, None, :, None]              # global orientation
    xq = np.einsum("ql,tli->tqi", _QL, nodes[tets])
    s = np.sin(math.pi * xq)
    Ef = np.stack([s[..., 1] * s[..., 2], s[..., 2] * s[..., 0], s[..., 0] * s[..., 1]], -1)
    Jsrc = (2 * math.pi ** 2 - k0 ** 2) * Ef
    fe = np.einsum("t,tqi,tqei->te", V / 4, Jsrc, N)
    f = np.zeros(A.shape[0])
    np.add.at(f, li[li >= 0], fe[li >= 0])
    u = spl.splu(sp.csc_matrix(A)).solve(f)
    ue = np.where(li >= 0, u[np.maximum(li, 0)], 0.0)
    Eh = np.einsum("te,tqei->tqi", ue, N)
    err = np.einsum("t,tqi->", V / 4, (Eh - Ef) ** 2)
    nrm = np.einsum("t,tqi->", V / 4, Ef ** 2)
    return math.sqrt(err / nrm)


def test_analytic_field_convergence_on_tetrahedra():
    """The field of the hexahedral pin (tangential-free on the cube, curl
    curl E = 2 pi^2 E): lowest-order Whitney elements converge at first order
    in L2."""
    errs = [_tet_error(n) for n in (4, 8, 16)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(f"[tet] L2 errors {errs}, rates {rates}")
    assert min(rates) >= 0.9, (errs, rates)
