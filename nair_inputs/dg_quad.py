"""Upwind DG-Q_p discretisation of  b . grad(u) + sigma u = q  on [0,1]^2.

The paper's model problem is steady transport with inflow data (numerical
results section, equation "transport"), discretised by fully upwinded
discontinuous Galerkin of orders 1-6.  Its meshes are not available, so this
module builds the same PDE on N x N quadrilaterals (optionally with jittered
interior vertices), giving the block structure the paper relies on: one dense
block per element, coupled only to its upwind neighbours, so the matrix is
block lower triangular in a (hidden) topological order of the cells.

Element matrix (strong upwind form, test index i, trial index j):
    A_KK[i,j]  =  int_K (b . grad phi_j + sigma phi_j) phi_i
                  - int_{dK^-} (b.n_K) phi_j phi_i
    A_KK'[i,j] = + int_{dK^- cap dK'} (b.n_K) phi'_j phi_i
where dK^- is the inflow part of the boundary (b.n_K < 0).  The right-hand
side is M_K q_K for nodal source values q_K (or int q phi_i for a source
function), plus -int_{Gamma_in} (b.n) g phi_i for inflow data g.

Basis: tensor Lagrange polynomials on (p+1)^2 Gauss-Lobatto nodes of the
reference square [0,1]^2, numbered lexicographically with x fastest.
Quadrature: p+2 Gauss-Legendre points per direction on volumes and faces.
Cells are numbered c = ix + N*iy; the block index of cell c is perm[c], where
perm is a seeded permutation, so the solver never sees the flow ordering.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional, Union

import numpy as np

FlowFn = Callable[[np.ndarray, np.ndarray], tuple]


def gauss_lobatto_nodes(p: int) -> np.ndarray:
    """p+1 Gauss-Lobatto nodes on [0,1] (endpoints and roots of P_p')."""
    if p < 1:
        raise ValueError("p >= 1 required")
    if p == 1:
        t = np.array([-1.0, 1.0])
    else:
        c = np.zeros(p + 1)
        c[p] = 1.0
        inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
        t = np.concatenate(([-1.0], np.sort(inner.real), [1.0]))
    return 0.5 * (t + 1.0)


def gauss_legendre(nq: int):
    """nq-point Gauss-Legendre rule on [0,1]."""
    t, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_1d(nodes: np.ndarray, t: np.ndarray):
    """Values and derivatives of the 1-D Lagrange basis on `nodes` at points t.

    Returns (V, D) with V[q, i] = l_i(t_q) and D[q, i] = l_i'(t_q).
    """
    n = len(nodes)
    t = np.asarray(t, dtype=np.float64)
    V = np.ones((len(t), n))
    D = np.zeros((len(t), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            V[:, i] *= (t - nodes[m]) / (nodes[i] - nodes[m])
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(t), 1.0 / (nodes[i] - nodes[m]))
            for s in range(n):
                if s == i or s == m:
                    continue
                term *= (t - nodes[s]) / (nodes[i] - nodes[s])
            D[:, i] += term
    return V, D


def _tensor(Vx, Vy):
    """2-D tensor values: out[qx + nq*qy, ix + n*iy] = Vx[qx,ix] * Vy[qy,iy]."""
    nqx, n = Vx.shape
    nqy = Vy.shape[0]
    out = np.einsum("ai,bj->baji", Vx, Vy).reshape(nqy * nqx, n * n)
    return out


@dataclass
class DGSystem:
    """A block-CSR system A x = b with metadata.  Arrays are host numpy arrays."""
    nb: int
    bs: int
    rowptr: np.ndarray          # int32 [nb+1]
    colidx: np.ndarray          # int32 [nnzb], sorted and unique per row
    vals: np.ndarray            # float64 [nnzb, bs, bs], row-major blocks
    rhs: np.ndarray             # float64 [nb*bs]
    perm: np.ndarray            # int64 [ncell]: block index of cell c
    topo_order: np.ndarray      # int64 [nb]: block indices, upwind first
    N: int = 0
    p: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nb * self.bs

    @property
    def nnzb(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        bs = self.bs
        D = np.zeros((self.n, self.n))
        for I in range(self.nb):
            for t in range(self.rowptr[I], self.rowptr[I + 1]):
                J = self.colidx[t]
                D[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = self.vals[t]
        return D


def _flow_callable(b: Union[tuple, FlowFn]) -> FlowFn:
    if callable(b):
        return b
    bx, by = float(b[0]), float(b[1])
    return lambda x, y: (np.full_like(x, bx), np.full_like(y, by))


def _vertices(N: int, jitter: float, seed: int) -> np.ndarray:
    """(N+1, N+1, 2) vertex array; interior vertices jittered by U[-jitter*h, jitter*h]^2."""
    h = 1.0 / N
    g = np.arange(N + 1) * h
    X = np.empty((N + 1, N + 1, 2))
    X[:, :, 0] = g[None, :]       # X[j, i] -> x = i h
    X[:, :, 1] = g[:, None]       # y = j h
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        d = rng.uniform(-jitter * h, jitter * h, size=(N + 1, N + 1, 2))
        X[1:N, 1:N, :] += d[1:N, 1:N, :]
    return X


def topo_sort_blocks(nb: int, rowptr: np.ndarray, colidx: np.ndarray) -> np.ndarray:
    """Kahn topological order of the block graph (row I depends on column J).

    Returns block indices with every block after all blocks it depends on.
    Raises ValueError if the block graph has a cycle.
    """
    indeg = np.zeros(nb, dtype=np.int64)
    dependents = [[] for _ in range(nb)]
    for I in range(nb):
        for t in range(rowptr[I], rowptr[I + 1]):
            J = int(colidx[t])
            if J != I:
                indeg[I] += 1
                dependents[J].append(I)
    order = []
    stack = [I for I in range(nb) if indeg[I] == 0]
    while stack:
        J = stack.pop()
        order.append(J)
        for I in dependents[J]:
            indeg[I] -= 1
            if indeg[I] == 0:
                stack.append(I)
    if len(order) != nb:
        raise ValueError("block graph has a cycle")
    return np.asarray(order, dtype=np.int64)


def dg_quad(N: int, p: int, b: Union[tuple, FlowFn], sigma: Union[float, np.ndarray] = 1.0,
            jitter: float = 0.0, seed_perm: Optional[int] = 101, seed_q: int = 102,
            seed_jitter: int = 103, q_nodal: Optional[np.ndarray] = None,
            q_fn: Optional[FlowFn] = None, g_fn: Optional[FlowFn] = None,
            check_acyclic: bool = True, chunk: int = 8192, return_mass: bool = False) -> DGSystem:
    """Assemble the upwind DG-Q_p system on an N x N quad mesh of [0,1]^2.

    b         : constant (bx, by) or callable (x, y) -> (bx, by) on arrays.
    sigma     : scalar or per-cell array [N*N] (cell order c = ix + N*iy).
    jitter    : interior vertex jitter as a fraction of h (cells stay convex for <= 0.25).
    seed_perm : seed of the cell -> block permutation; None keeps the natural order.
    q_nodal   : nodal source values [N*N, (p+1)^2] in cell order; default U[-1,1] from seed_q.
    q_fn      : source function; if given, rhs_i = int q phi_i (overrides q_nodal).
    g_fn      : inflow boundary data; default g = 0.
    return_mass: also return the cell mass matrices (block order) in meta["mass"].
    """
    if N < 1:
        raise ValueError("N >= 1 required")
    nloc = p + 1
    bs = nloc * nloc
    ncell = N * N
    flow = _flow_callable(b)
    nodes = gauss_lobatto_nodes(p)
    tq, wq = gauss_legendre(p + 2)
    nq = len(tq)
    V1, D1 = lagrange_1d(nodes, tq)
    Phi = _tensor(V1, V1)                    # [nq*nq, bs]
    Pxi = _tensor(D1, V1)                    # d/dxi
    Peta = _tensor(V1, D1)                   # d/deta
    W2 = np.outer(wq, wq).reshape(-1)        # [qx + nq*qy] -> wq[qy]*wq[qx]; symmetric
    xi2 = np.tile(tq, nq)
    eta2 = np.repeat(tq, nq)

    X = _vertices(N, jitter, seed_jitter)
    iy, ix = np.divmod(np.arange(ncell), N)
    X0 = X[iy, ix]
    X1 = X[iy, ix + 1]
    X2 = X[iy + 1, ix + 1]
    X3 = X[iy + 1, ix]

    if np.ndim(sigma) == 0:
        sig = np.full(ncell, float(sigma))
    else:
        sig = np.asarray(sigma, dtype=np.float64).reshape(ncell)

    if q_fn is None:
        if q_nodal is None:
            rng = np.random.Generator(np.random.PCG64(seed_q))
            q_nodal = rng.uniform(-1.0, 1.0, size=(ncell, bs))
        q_nodal = np.asarray(q_nodal, dtype=np.float64).reshape(ncell, bs)

    diag = np.empty((ncell, bs, bs))
    rhs_cell = np.zeros((ncell, bs))
    mass_cell = np.empty((ncell, bs, bs)) if return_mass else None

    # ---- volume terms, chunked over cells
    for c0 in range(0, ncell, chunk):
        c1 = min(ncell, c0 + chunk)
        a0, a1, a2, a3 = X0[c0:c1], X1[c0:c1], X2[c0:c1], X3[c0:c1]
        xi = xi2[None, :]
        et = eta2[None, :]
        # bilinear map and its Jacobian at the quadrature points: [nc, nq2]
        px = (a0[:, None, 0] * (1 - xi) * (1 - et) + a1[:, None, 0] * xi * (1 - et)
              + a2[:, None, 0] * xi * et + a3[:, None, 0] * (1 - xi) * et)
        py = (a0[:, None, 1] * (1 - xi) * (1 - et) + a1[:, None, 1] * xi * (1 - et)
              + a2[:, None, 1] * xi * et + a3[:, None, 1] * (1 - xi) * et)
        x_xi = (a1[:, None, 0] - a0[:, None, 0]) * (1 - et) + (a2[:, None, 0] - a3[:, None, 0]) * et
        y_xi = (a1[:, None, 1] - a0[:, None, 1]) * (1 - et) + (a2[:, None, 1] - a3[:, None, 1]) * et
        x_et = (a3[:, None, 0] - a0[:, None, 0]) * (1 - xi) + (a2[:, None, 0] - a1[:, None, 0]) * xi
        y_et = (a3[:, None, 1] - a0[:, None, 1]) * (1 - xi) + (a2[:, None, 1] - a1[:, None, 1]) * xi
        det = x_xi * y_et - x_et * y_xi
        if np.any(det <= 0):
            raise ValueError("non-positive Jacobian: mesh is tangled")
        bx, by = flow(px, py)
        bx = np.broadcast_to(bx, px.shape)
        by = np.broadcast_to(by, px.shape)
        c_xi = bx * y_et - by * x_et          # (b . grad phi) * det = c_xi phi_xi + c_eta phi_eta
        c_et = by * x_xi - bx * y_xi
        sd = sig[c0:c1, None] * det
        G = (W2[None, :, None] * (c_xi[:, :, None] * Pxi[None] + c_et[:, :, None] * Peta[None]
                                  + sd[:, :, None] * Phi[None]))
        diag[c0:c1] = np.matmul(Phi.T[None], G)
        if q_fn is None or return_mass:
            M = np.matmul(Phi.T[None], (W2[None, :] * det)[:, :, None] * Phi[None])
            if return_mass:
                mass_cell[c0:c1] = M
        if q_fn is None:
            rhs_cell[c0:c1] = np.einsum("cij,cj->ci", M, q_nodal[c0:c1])
        else:
            qv = np.broadcast_to(q_fn(px, py), px.shape)
            rhs_cell[c0:c1] = np.einsum("qi,cq->ci", Phi, W2[None, :] * det * qv)

    # ---- face terms.  Face f: 0 south (eta=0), 1 east (xi=1), 2 north (eta=1), 3 west (xi=0).
    one = np.ones(nq)
    zero = np.zeros(nq)
    face_ref = [(tq, zero), (one, tq), (tq, one), (zero, tq)]
    face_phi = []
    for (fx, fy) in face_ref:
        Vx, _ = lagrange_1d(nodes, fx)
        Vy, _ = lagrange_1d(nodes, fy)
        face_phi.append(np.einsum("qa,qb->qba", Vx, Vy).reshape(nq, bs))
    opposite = [2, 3, 0, 1]
    # endpoints of each face in CCW orientation and the parameter-start vertex
    verts = [X0, X1, X2, X3]
    ccw = [(0, 1), (1, 2), (2, 3), (3, 0)]
    pstart = [(0, 1), (1, 2), (3, 2), (0, 3)]      # x(t) = Va (1-t) + Vb t
    nbr_dx = [(0, -1), (1, 0), (0, 1), (-1, 0)]

    off_rows, off_cols, off_vals = [], [], []
    for f in range(4):
        va, vb = verts[ccw[f][0]], verts[ccw[f][1]]
        tau = vb - va
        L = np.hypot(tau[:, 0], tau[:, 1])
        nx = tau[:, 1] / L
        ny = -tau[:, 0] / L
        sa, sb = verts[pstart[f][0]], verts[pstart[f][1]]
        qx = sa[:, None, 0] * (1 - tq[None]) + sb[:, None, 0] * tq[None]
        qy = sa[:, None, 1] * (1 - tq[None]) + sb[:, None, 1] * tq[None]
        bxq, byq = flow(qx, qy)
        bxq = np.broadcast_to(bxq, qx.shape)
        byq = np.broadcast_to(byq, qx.shape)
        bn = bxq * nx[:, None] + byq * ny[:, None]          # [ncell, nq]
        inflow = bn < 0
        outflow = bn > 0
        mixed = inflow.any(axis=1) & outflow.any(axis=1)
        if np.any(mixed):
            raise ValueError("b.n changes sign along a face; upwinding is ambiguous")
        is_in = inflow.any(axis=1)
        wbn = wq[None, :] * L[:, None] * bn                  # [ncell, nq]
        Pf = face_phi[f]
        own = np.einsum("qi,cq,qj->cij", Pf, wbn, Pf)
        diag[is_in] -= own[is_in]
        dx, dy = nbr_dx[f]
        jx, jy = ix + dx, iy + dy
        inside = (jx >= 0) & (jx < N) & (jy >= 0) & (jy < N)
        interior_in = is_in & inside
        bnd_in = is_in & ~inside
        if np.any(interior_in):
            cells = np.nonzero(interior_in)[0]
            nbrs = jx[cells] + N * jy[cells]
            Po = face_phi[opposite[f]]
            blk = np.einsum("qi,cq,qj->cij", Pf, wbn[cells], Po)
            off_rows.append(cells)
            off_cols.append(nbrs)
            off_vals.append(blk)
        if g_fn is not None and np.any(bnd_in):
            cells = np.nonzero(bnd_in)[0]
            gv = np.broadcast_to(g_fn(qx[cells], qy[cells]), qx[cells].shape)
            rhs_cell[cells] -= np.einsum("qi,cq->ci", Pf, wbn[cells] * gv)

    # ---- block ordering and BSR assembly
    if seed_perm is None:
        perm = np.arange(ncell, dtype=np.int64)
    else:
        perm = np.random.Generator(np.random.PCG64(seed_perm)).permutation(ncell).astype(np.int64)
    if off_rows:
        orow = perm[np.concatenate(off_rows)]
        ocol = perm[np.concatenate(off_cols)]
        oval = np.concatenate(off_vals)
    else:
        orow = np.zeros(0, dtype=np.int64)
        ocol = np.zeros(0, dtype=np.int64)
        oval = np.zeros((0, bs, bs))
    rows = np.concatenate([perm, orow])
    cols = np.concatenate([perm, ocol])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    nb = ncell
    nnzb = len(rows)
    vals = np.empty((nnzb, bs, bs))
    src_is_diag = order < ncell
    vals[src_is_diag] = diag[order[src_is_diag]]
    vals[~src_is_diag] = oval[order[~src_is_diag] - ncell]
    if np.any((rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])):
        raise ValueError("duplicate block (two faces shared by the same pair of cells)")
    rowptr = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    rhs = np.empty((nb, bs))
    rhs[perm] = rhs_cell
    rowptr32 = rowptr.astype(np.int32)
    colidx32 = cols.astype(np.int32)
    topo = (topo_sort_blocks(nb, rowptr32, colidx32) if check_acyclic
            else np.zeros(0, dtype=np.int64))
    meta = {"jitter": jitter, "sigma_is_array": np.ndim(sigma) != 0}
    if return_mass:
        mass = np.empty_like(mass_cell)
        mass[perm] = mass_cell
        meta["mass"] = mass
    return DGSystem(nb=nb, bs=bs, rowptr=rowptr32, colidx=colidx32,
                    vals=np.ascontiguousarray(vals), rhs=rhs.reshape(-1),
                    perm=perm, topo_order=topo, N=N, p=p, meta=meta)


def sigma_q_model(N: int, p: int, b, jitter: float = 0.0, seed_perm: Optional[int] = 101,
                  seed_sigma: int = 105, seed_q: int = 102, seed_xstar: int = 104):
    """Parts of the differentiable model A(sigma) x = M q of the Q_p transport system.

    The upwind DG matrix is affine in the per-cell reaction coefficient:
    A(sigma) = A(0) + sum_K sigma_K E_KK (x) M_K, and the right-hand side is
    b(q) = M q (M the block-diagonal mass matrix, q nodal).  Returns a dict with
    the sigma = 0 system, the cell mass matrices and the diagonal block positions
    (block order), seeded sigma ~ U[0.5, 2] per cell, q ~ U[-1, 1] per node and a
    target x* ~ U[-1, 1].
    """
    S0 = dg_quad(N, p, b, sigma=0.0, jitter=jitter, seed_perm=seed_perm, return_mass=True,
                 q_nodal=np.zeros((N * N, (p + 1) ** 2)))
    nb, bs = S0.nb, S0.bs
    rows = np.repeat(np.arange(nb), np.diff(S0.rowptr))
    diag_pos = np.nonzero(rows == S0.colidx)[0]
    sig_cell = np.random.Generator(np.random.PCG64(seed_sigma)).uniform(0.5, 2.0, size=N * N)
    q_cell = np.random.Generator(np.random.PCG64(seed_q)).uniform(-1.0, 1.0, size=(N * N, bs))
    sigma = np.empty(nb)
    sigma[S0.perm] = sig_cell
    q = np.empty((nb, bs))
    q[S0.perm] = q_cell
    xstar = np.random.Generator(np.random.PCG64(seed_xstar)).uniform(-1.0, 1.0, size=nb * bs)
    return dict(system=S0, mass=S0.meta["mass"], diag_pos=diag_pos, sigma=sigma, q=q.reshape(-1), xstar=xstar)
