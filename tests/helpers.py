"""Dense linear-algebra helpers for the tests (numpy only; no oracle arithmetic)."""
import numpy as np


def bsr_dense(nb, bs, rowptr, colidx, vals, ncols=None):
    ncols = nb if ncols is None else ncols
    D = np.zeros((nb * bs, ncols * bs))
    for I in range(nb):
        for t in range(rowptr[I], rowptr[I + 1]):
            J = colidx[t]
            D[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = vals[t]
    return D


def dof_index(blocks, bs):
    blocks = np.asarray(blocks, dtype=np.int64)
    return (blocks[:, None] * bs + np.arange(bs)[None, :]).reshape(-1)


def row_blocks(rowptr):
    return np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))


def dense_E(vcycle, A):
    """Error propagator E = I - B A of one cycle application B (a callable on vectors)."""
    n = A.shape[0]
    E = np.eye(n)
    for j in range(n):
        E[:, j] -= vcycle(A[:, j])
    return E


def dense_B(vcycle, n):
    return np.stack([vcycle(np.eye(n)[:, j]) for j in range(n)], axis=1)


def longest_path_edges(nodes, adj):
    """Longest path (in edges) of a DAG given as adj[u] = list of successors, over `nodes`."""
    nodes = list(nodes)
    memo = {}

    def lp(u):
        if u in memo:
            return memo[u]
        best = 0
        for v in adj.get(u, ()):
            best = max(best, 1 + lp(v))
        memo[u] = best
        return best

    return max((lp(u) for u in nodes), default=0)
