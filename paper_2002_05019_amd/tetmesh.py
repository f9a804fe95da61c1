"""Seeded unstructured tetrahedral workloads for the DD solver.

The paper's models (section III) are unstructured FEM meshes of a dielectric
sphere and of antenna arrays, split into domains by a graph partitioner.
This module builds stand-ins of that kind:

* mesh: a jittered n^3 grid of the unit cube, every cell split into six
  tetrahedra along its main diagonal (Kuhn's subdivision: conforming, all
  cells alike), optionally carved to the ball of radius `ball` around the
  cube's centre (tetrahedra whose centroid lies inside), which leaves a
  jagged, unstructured outer surface; PEC on the outer surface;
* materials: a lossy dielectric sphere of radius `sphere` (eps_in) in a
  lossy background (eps_out), loss tangent `tan_delta`;
* elements: lowest-order Nedelec (Whitney) edge elements, closed-form
  element matrices (`whitney_matrices`), curl-curl operator
  curl curl E - k0^2 eps_r E with mu_r = 1;
* domains: a project-written graph partitioner of the element dual graph
  (`partition`): recursive bisection by graph growing from a
  pseudo-peripheral element, refined by greedy boundary moves under a
  balance bound; domains are irregular, not boxes;
* interfaces: star constraints from the lowest-numbered owner of every
  shared edge; Robin terms on every interface triangle, +j k0 beta M_F on the
  lower-numbered domain's side and -j k0 beta M_F on the other (so that
  they cancel in the assembled operator: sum_i R_i^T K_i R_i = A).

Holds the problem definition only (no DD arithmetic); it serves the oracle
and the GPU path alike.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .problem import Case, Domain

# local edges of a tetrahedron (vertex pairs) and local faces (vertex triples)
TET_EDGES = np.array([[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]])
TET_FACES = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
TRI_EDGES = np.array([[0, 1], [0, 2], [1, 2]])


@dataclass
class TetSpec:
    n: int                     # grid cells per side before the subdivision
    n_dom: int                 # domains produced by the partitioner
    k0: float
    eps_in: float = 4.0        # inside the dielectric sphere
    eps_out: float = 1.0
    tan_delta: float = 0.02
    sphere: float = 0.3        # radius of the dielectric sphere (unit cube centred at 0.5)
    ball: float | None = None  # carve the mesh to this radius (None: the whole cube)
    jitter: float = 0.2        # interior node jitter in units of h
    nrhs: int = 1
    seed: int = 0
    beta: float = 1.0
    imbalance: float = 0.03    # allowed part-size deviation of a bisection
    name: str = ""


def named_tet_spec(name: str) -> TetSpec:
    """Tetrahedral workloads: parity cases and the sphere stand-in."""
    if name == "tet8":       # 8^3 cells (3,072 tets) of the unit cube, 4 domains
        return TetSpec(n=8, n_dom=4, k0=2 * math.pi, nrhs=2, seed=81, name=name)
    if name == "tet12s":     # 12^3 cells carved to a ball, 8 irregular domains
        return TetSpec(n=12, n_dom=8, k0=2 * math.pi * 1.5, ball=0.5, nrhs=3, seed=121, name=name)
    if name == "tet16":      # 16^3 cells, 11 domains (not a power of two)
        return TetSpec(n=16, n_dom=11, k0=2 * math.pi * 2.0, nrhs=4, seed=161, name=name)
    if name == "tet40s":     # 40^3 cells carved to a ball, 64 domains, 8 RHS
        return TetSpec(n=40, n_dom=64, k0=2 * math.pi * 4.0, ball=0.5, sphere=0.25, nrhs=8, seed=401,
                       name=name)
    raise KeyError(name)


# ----------------------------------------------------------------------------
# mesh
def kuhn_mesh(n, jitter, rng):
    """Nodes ((n+1)^3, 3) of the jittered unit-cube grid (boundary nodes stay
    on the boundary) and the six Kuhn tetrahedra of every cell, (6 n^3, 4)."""
    h = 1.0 / n
    g = np.arange(n + 1) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    nodes = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    idx = np.arange((n + 1) ** 3).reshape(n + 1, n + 1, n + 1)
    if jitter:
        d = rng.uniform(-jitter * h, jitter * h, size=nodes.shape)
        inner = np.ones((n + 1,) * 3, bool)
        inner[[0, -1], :, :] = inner[:, [0, -1], :] = inner[:, :, [0, -1]] = False
        nodes[inner.ravel()] += d[inner.ravel()]
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    corner = lambda a, b, c: idx[i + a, j + b, k + c]
    v000, v111 = corner(0, 0, 0), corner(1, 1, 1)
    unit = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    tets = []
    for p in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        a = unit[p[0]]
        b = tuple(x + y for x, y in zip(a, unit[p[1]]))
        tets.append(np.stack([v000, corner(*a), corner(*b), v111], axis=1))
    return nodes, np.concatenate(tets, axis=0)


def carve_ball(nodes, tets, radius):
    """Tetrahedra whose centroid lies within `radius` of the cube's centre,
    with the unused nodes dropped and the rest renumbered."""
    c = nodes[tets].mean(axis=1)
    keep = np.linalg.norm(c - 0.5, axis=1) <= radius
    tets = tets[keep]
    used = np.unique(tets)
    renum = -np.ones(len(nodes), np.int64)
    renum[used] = np.arange(len(used))
    return nodes[used], renum[tets]


def mesh_edges(tets):
    """Unique edges (E, 2) with ascending node ids, the tetrahedra's edge ids
    (T, 6) in TET_EDGES order, and the orientation signs (T, 6): +1 when the
    local pair is ascending in global node ids."""
    a = tets[:, TET_EDGES[:, 0]]
    b = tets[:, TET_EDGES[:, 1]]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo.astype(np.int64) * (tets.max() + 1) + hi
    uk, inv = np.unique(key.ravel(), return_inverse=True)
    edges = np.stack([uk // (tets.max() + 1), uk % (tets.max() + 1)], axis=1)
    return edges, inv.reshape(tets.shape[0], 6), np.where(a < b, 1.0, -1.0)


def mesh_faces(tets):
    """Unique faces (F, 3) with ascending node ids, the tetrahedra's face ids
    (T, 4) in TET_FACES order, and the number of tetrahedra on each face."""
    f = np.sort(tets[:, TET_FACES], axis=2)
    m = tets.max() + 1
    key = (f[..., 0].astype(np.int64) * m + f[..., 1]) * m + f[..., 2]
    uk, inv, cnt = np.unique(key.ravel(), return_inverse=True, return_counts=True)
    faces = np.stack([uk // (m * m), (uk // m) % m, uk % m], axis=1)
    return faces, inv.reshape(tets.shape[0], 4), cnt


# ----------------------------------------------------------------------------
# elements
def barycentric_gradients(P):
    """Gradients of the four barycentric coordinates of tetrahedra P (T, 4, 3)
    -> (T, 4, 3), and their volumes."""
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)   # columns
    Ji = np.linalg.inv(J)                        # rows: gradients of lambda_1..3
    g = np.empty_like(P)
    g[:, 1:] = Ji
    g[:, 0] = -Ji.sum(axis=1)
    return g, np.abs(np.linalg.det(J)) / 6.0


def whitney_matrices(P):
    """Lowest-order Nedelec element matrices of tetrahedra P (T, 4, 3) for
    the local edges TET_EDGES (local orientation a -> b):
    N_e = l_a grad l_b - l_b grad l_a, curl N_e = 2 grad l_a x grad l_b;
    S_ef = int curl N_e . curl N_f, T_ef = int N_e . N_f with
    int l_x l_y = V (1 + delta_xy) / 20.  Returns (S, T), each (T, 6, 6)."""
    g, V = barycentric_gradients(P)
    ea, eb = TET_EDGES[:, 0], TET_EDGES[:, 1]
    c = 2.0 * np.cross(g[:, ea], g[:, eb])                       # (T, 6, 3)
    S = V[:, None, None] * np.einsum("tei,tfi->tef", c, c)
    G = np.einsum("tai,tbi->tab", g, g)                          # grad l_a . grad l_b
    M = (np.ones((4, 4)) + np.eye(4)) / 20.0                     # int l_x l_y / V
    a, b = ea[:, None], eb[:, None]
    cc, d = ea[None, :], eb[None, :]
    Tm = (M[a, cc] * G[:, b, d] - M[a, d] * G[:, b, cc] - M[b, cc] * G[:, a, d] + M[b, d] * G[:, a, cc])
    Tm = V[:, None, None] * Tm
    # exactly symmetric (the two triangles differ in rounding order only)
    return 0.5 * (S + S.transpose(0, 2, 1)), 0.5 * (Tm + Tm.transpose(0, 2, 1))


def face_mass(Q):
    """Tangential-trace mass of triangles Q (F, 3, 3) for the local edges
    TRI_EDGES: int_F (n x N_e).(n x N_f) dS, the traces being the triangle's
    own Whitney functions l_a grad_s l_b - l_b grad_s l_a (surface gradients);
    int l_x l_y = A (1 + delta_xy) / 12.  Returns (F, 3, 3)."""
    e1, e2 = Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0]
    E = np.stack([e1, e2], axis=2)                               # (F, 3, 2)
    Gm = np.linalg.inv(np.einsum("fia,fib->fab", E, E))          # (E^T E)^-1
    G12 = np.einsum("fia,fab->fib", E, Gm)                       # surface gradients of l_1, l_2 (columns)
    g = np.empty_like(Q)
    g[:, 1], g[:, 2] = G12[:, :, 0], G12[:, :, 1]
    g[:, 0] = -g[:, 1] - g[:, 2]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    G = np.einsum("fai,fbi->fab", g, g)
    M = (np.ones((3, 3)) + np.eye(3)) / 12.0
    ea, eb = TRI_EDGES[:, 0], TRI_EDGES[:, 1]
    a, b, cc, d = ea[:, None], eb[:, None], ea[None, :], eb[None, :]
    Fm = area[:, None, None] * (M[a, cc] * G[:, b, d] - M[a, d] * G[:, b, cc] - M[b, cc] * G[:, a, d]
                                + M[b, d] * G[:, a, cc])
    return 0.5 * (Fm + Fm.transpose(0, 2, 1))


# ----------------------------------------------------------------------------
# graph partitioner
def dual_graph(tets):
    """CSR adjacency of tetrahedra sharing a face."""
    _, tf, cnt = mesh_faces(tets)
    T = len(tets)
    owner = np.repeat(np.arange(T), 4)
    order = np.argsort(tf.ravel(), kind="stable")
    fs = tf.ravel()[order]
    ow = owner[order]
    inner = cnt[fs] == 2
    fs, ow = fs[inner], ow[inner]
    a, b = ow[0::2], ow[1::2]                                    # the two sides of each inner face
    r = np.concatenate([a, b])
    c = np.concatenate([b, a])
    G = sp.csr_matrix((np.ones(len(r), np.int8), (r, c)), shape=(T, T))
    return G.indptr, G.indices


def _bfs_order(ptr, adj, start, inset):
    """Breadth-first order of the vertices of `inset` (bool mask) reachable
    from `start`, and their levels."""
    order = [start]
    level = {start: 0}
    head = 0
    while head < len(order):
        v = order[head]
        head += 1
        for w in adj[ptr[v]:ptr[v + 1]]:
            if inset[w] and w not in level:
                level[w] = level[v] + 1
                order.append(w)
    return order, level


def _bisect(ptr, adj, verts, frac, imbalance):
    """Splits `verts` (array) into a part of about `frac` of its vertices and
    the rest: graph growing from a pseudo-peripheral vertex (piece by piece
    when the set is not connected), then sweeps of boundary moves.  A sweep
    moves, from one side, the vertices whose move removes more cut edges
    than it adds (highest gain first, as many as that side's balance slack
    allows); vertices leaving the same side together never do worse than
    the sum of their gains."""
    n_all = len(ptr) - 1
    inset = np.zeros(n_all, bool)
    inset[verts] = True
    order = []
    seen = np.zeros(n_all, bool)
    for s in verts:
        if seen[s]:
            continue
        o1, _ = _bfs_order(ptr, adj, int(s), inset & ~seen)
        o2, _ = _bfs_order(ptr, adj, o1[-1], inset & ~seen)
        seen[o2] = True
        order.extend(o2)
    order = np.asarray(order, dtype=np.int64)
    nA = int(round(frac * len(verts)))
    part = np.zeros(n_all, np.int8)          # 1: part A, 2: part B, 0: elsewhere
    part[order[:nA]] = 1
    part[order[nA:]] = 2
    deg = np.diff(ptr)[verts]
    rows = np.repeat(np.arange(len(verts)), deg)
    cols = adj[np.concatenate([np.arange(ptr[v], ptr[v + 1]) for v in verts])] if len(verts) else np.zeros(0, int)
    target = {1: nA, 2: len(verts) - nA}
    for _ in range(16):
        moved = 0
        for side in (1, 2):
            pv = part[verts]
            pc = part[cols]
            ext = np.bincount(rows, weights=(pc == 3 - pv[rows]), minlength=len(verts))
            own = np.bincount(rows, weights=(pc == pv[rows]), minlength=len(verts))
            gain = ext - own
            cand = np.flatnonzero((pv == side) & (gain > 0))
            slack = int(np.sum(pv == side) - math.ceil((1 - imbalance) * target[side]))
            if slack <= 0 or len(cand) == 0:
                continue
            cand = cand[np.argsort(-gain[cand], kind="stable")[:slack]]
            part[verts[cand]] = 3 - side
            moved += len(cand)
        if not moved:
            break
    return verts[part[verts] == 1], verts[part[verts] == 2]


def partition(ptr, adj, nparts, imbalance=0.03):
    """Recursive bisection of a graph into `nparts` parts (any count: a set
    meant for k parts is split k//2 : k - k//2).  Returns the part of every
    vertex."""
    parts = np.empty(len(ptr) - 1, np.int64)
    stack = [(np.arange(len(ptr) - 1), nparts, 0)]
    while stack:
        verts, k, base = stack.pop()
        if k == 1:
            parts[verts] = base
            continue
        ka = k // 2
        A, B = _bisect(ptr, adj, verts, ka / k, imbalance)
        stack.append((B, k - ka, base + ka))
        stack.append((A, ka, base))
    return parts


def cut_edges(ptr, adj, parts):
    """Number of graph edges between different parts."""
    r = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    return int(np.sum(parts[r] != parts[adj]) // 2)


# ----------------------------------------------------------------------------
# case
def make_tet_case(spec: TetSpec | str) -> Case:
    """The decomposed problem on a tetrahedral mesh, as a `Case` (the same
    interface the hexahedral generator provides)."""
    if isinstance(spec, str):
        spec = named_tet_spec(spec)
    rng_j = np.random.default_rng([spec.seed, 0])
    rng_m = np.random.default_rng([spec.seed, 1])
    rng_f = np.random.default_rng([spec.seed, 3])
    nodes, tets = kuhn_mesh(spec.n, spec.jitter, rng_j)
    if spec.ball is not None:
        nodes, tets = carve_ball(nodes, tets, spec.ball)
    T = len(tets)
    edges, te, tsg = mesh_edges(tets)
    faces, tfc, fcnt = mesh_faces(tets)
    # PEC: edges of the outer surface (faces with one tetrahedron)
    bf = faces[fcnt == 1]
    bedge = np.unique(np.concatenate([np.sort(bf[:, p], axis=1) for p in ([0, 1], [0, 2], [1, 2])]), axis=0)
    key = edges[:, 0] * (len(nodes)) + edges[:, 1]
    pec = np.isin(key, bedge[:, 0] * len(nodes) + bedge[:, 1])
    gmap = -np.ones(len(edges), np.int64)
    gmap[~pec] = np.arange(int((~pec).sum()))
    n_global = int((~pec).sum())
    # materials: dielectric sphere in a lossy background (eps' (1 - j tan d))
    cen = nodes[tets].mean(axis=1)
    inside = np.linalg.norm(cen - 0.5, axis=1) <= spec.sphere
    epsr = np.where(inside, spec.eps_in, spec.eps_out) * (1.0 + rng_m.uniform(-0.05, 0.05, T))
    eps = epsr * (1 - 1j * spec.tan_delta)
    S, Tm = whitney_matrices(nodes[tets])
    sg = tsg[:, :, None] * tsg[:, None, :]
    Ael = (S - spec.k0 ** 2 * eps[:, None, None] * Tm) * sg      # (T, 6, 6), global orientation
    # partition of the element dual graph
    ptr, adj = dual_graph(tets)
    part = partition(ptr, adj, spec.n_dom, spec.imbalance)
    n_dom = int(part.max()) + 1
    # interface faces: inner faces whose two tetrahedra lie in different domains
    owner = np.repeat(np.arange(T), 4)
    order = np.argsort(tfc.ravel(), kind="stable")
    fs, ow = tfc.ravel()[order], owner[order]
    inner = fcnt[fs] == 2
    fs, ow = fs[inner], ow[inner]
    fa, ta, tb = fs[0::2], ow[0::2], ow[1::2]
    iface = part[ta] != part[tb]
    fa, da, db = fa[iface], part[ta[iface]], part[tb[iface]]
    lo_d, hi_d = np.minimum(da, db), np.maximum(da, db)
    tri = faces[fa]                                              # ascending node ids
    Mf = face_mass(nodes[tri])                                   # local edges TRI_EDGES, ascending = global
    te_tri = np.stack([np.searchsorted(key, tri[:, a] * len(nodes) + tri[:, b]) for a, b in TRI_EDGES], axis=1)
    domains = []
    f_glob = (rng_f.standard_normal((n_global, spec.nrhs)) + 1j * rng_f.standard_normal((n_global, spec.nrhs))) \
        / math.sqrt(2.0)
    owners = [[] for _ in range(n_global)]
    for d in range(n_dom):
        tl = np.flatnonzero(part == d)
        ge = np.unique(te[tl])
        ge = ge[~pec[ge]]
        l2g = gmap[ge]
        loc = -np.ones(len(edges), np.int64)
        loc[ge] = np.arange(len(ge))
        li = loc[te[tl]]                                          # (t, 6), -1 for PEC
        rr = np.repeat(li, 6, axis=1).ravel()
        cc = np.tile(li, (1, 6)).ravel()
        vv = Ael[tl].reshape(len(tl), 36).ravel()
        ok = (rr >= 0) & (cc >= 0)
        Ad = sp.csr_matrix((vv[ok], (rr[ok], cc[ok])), shape=(len(ge), len(ge)))
        Ad.sum_duplicates()
        # Robin terms on this domain's interface triangles
        mine = (lo_d == d) | (hi_d == d)
        sgn = np.where(lo_d[mine] == d, 1.0, -1.0)
        lt = loc[te_tri[mine]]
        rr = np.repeat(lt, 3, axis=1).ravel()
        cc = np.tile(lt, (1, 3)).ravel()
        vv = (1j * spec.k0 * spec.beta * sgn[:, None, None] * Mf[mine]).reshape(-1)
        ok = (rr >= 0) & (cc >= 0)
        R = sp.csr_matrix((vv[ok], (rr[ok], cc[ok])), shape=(len(ge), len(ge)))
        # symmetric element and face matrices: a symmetric pattern, and a
        # nonzero diagonal (the loss makes every diagonal entry complex)
        K = (Ad + R).tocsr()
        K.sum_duplicates()
        K.sort_indices()
        xyz = (0.5 * (nodes[edges[ge, 0]] + nodes[edges[ge, 1]])).astype(np.float32)
        domains.append(Domain(box=None, n=len(ge), l2g=l2g, xyz=xyz, sigma=0, A=Ad.tocsr(), K=K))
        for li_, g in enumerate(l2g):
            owners[g].append((d, li_))
    # star constraints from the lowest-numbered owner; the right-hand side to it
    ent = [[] for _ in range(n_dom)]
    m = 0
    for g in range(n_global):
        ow_ = owners[g]
        if len(ow_) < 2:
            continue
        d1, l1 = ow_[0]
        for dk, lk in ow_[1:]:
            ent[d1].append((l1, m, 1))
            ent[dk].append((lk, m, -1))
            m += 1
    imap_ptr = np.zeros(n_dom + 1, np.int64)
    dofs, mults, signs = [], [], []
    for d in range(n_dom):
        e = sorted(ent[d], key=lambda x: x[1])
        imap_ptr[d + 1] = imap_ptr[d] + len(e)
        dofs += [x[0] for x in e]
        mults += [x[1] for x in e]
        signs += [x[2] for x in e]
    f_torn = []
    seen = np.zeros(n_global, bool)
    for dm in domains:
        blk = np.zeros((dm.n, spec.nrhs), complex)
        new = ~seen[dm.l2g]
        blk[new] = f_glob[dm.l2g[new]]
        seen[dm.l2g] = True
        f_torn.append(blk)
    case = Case(spec=spec, n_global=n_global, domains=domains, n_mult=m,
                imap_ptr=imap_ptr, imap_dof=np.asarray(dofs, np.int32), imap_mult=np.asarray(mults, np.int64),
                imap_sign=np.asarray(signs, np.int8), f=f_glob, f_torn=f_torn, eps=eps, nodes=nodes, gmap=gmap)
    # the undecomposed operator from the element matrices directly
    li = gmap[te]
    rr = np.repeat(li, 6, axis=1).ravel()
    cc = np.tile(li, (1, 6)).ravel()
    vv = Ael.reshape(T, 36).ravel()
    ok = (rr >= 0) & (cc >= 0)
    case._A = sp.csr_matrix((vv[ok], (rr[ok], cc[ok])), shape=(n_global, n_global))
    case._A.sum_duplicates()
    case.tets, case.edges, case.tet_edges, case.tet_signs, case.part = tets, edges, te, tsg, part
    return case
