"""Seeded random block-sparse matrices for tests.

`layered_block_triangular` gives a matrix that is block lower triangular in a
hidden order: blocks are placed in `layers` layers, each block depends on a few
blocks of earlier layers, so the longest dependency path has at most
layers-1 edges.  Block indices are a seeded permutation of that order.
"""
from __future__ import annotations

import numpy as np


def _to_bsr(nb, bs, entries):
    """entries: dict (I, J) -> block.  Returns sorted BSR arrays."""
    keys = sorted(entries)
    rowptr = np.zeros(nb + 1, dtype=np.int32)
    for (I, _J) in keys:
        rowptr[I + 1] += 1
    rowptr = np.cumsum(rowptr).astype(np.int32)
    colidx = np.array([J for (_I, J) in keys], dtype=np.int32)
    vals = np.array([entries[k] for k in keys], dtype=np.float64).reshape(len(keys), bs, bs)
    return rowptr, colidx, vals


def layered_block_triangular(nb: int, bs: int, layers: int, deps: int = 2, seed: int = 0,
                             offdiag_scale: float = 0.5, back_edges: int = 0,
                             zero_entries: float = 0.0):
    """Random block lower triangular matrix (in a hidden order), as BSR.

    Returns (rowptr, colidx, vals, order, layer) where order lists the block
    indices in a dependency-respecting order and layer[I] is the layer of I.
    back_edges > 0 reverses that many existing dependencies (adding A_JI next
    to A_IJ), which makes the matrix non-triangular in every order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if nb >= layers:
        layer_of_pos = np.sort(np.concatenate([np.arange(layers),
                                               rng.integers(0, layers, size=nb - layers)]))
    else:
        layer_of_pos = np.arange(nb)
    perm = rng.permutation(nb)          # position -> block index
    layer = np.empty(nb, dtype=np.int64)
    layer[perm] = layer_of_pos
    entries = {}
    for pos in range(nb):
        I = int(perm[pos])
        D = rng.uniform(-1.0, 1.0, size=(bs, bs))
        D += np.diag(np.sign(np.diag(D)) * bs + np.where(np.diag(D) == 0, bs, 0))
        entries[(I, I)] = D
        earlier = np.nonzero(layer_of_pos < layer_of_pos[pos])[0]
        if len(earlier):
            pick = rng.choice(earlier, size=min(deps, len(earlier)), replace=False)
            for q in pick:
                B = offdiag_scale * rng.uniform(-1.0, 1.0, size=(bs, bs))
                if zero_entries > 0.0:
                    B[rng.random((bs, bs)) < zero_entries] = 0.0
                entries[(I, int(perm[q]))] = B
    # back edges: reverse existing dependencies, so each one closes a 2-cycle
    deps_list = sorted(k for k in entries if k[0] != k[1])
    if back_edges > 0 and deps_list:
        pick = rng.choice(len(deps_list), size=min(back_edges, len(deps_list)), replace=False)
        for q in pick:
            I, J = deps_list[int(q)]
            entries[(J, I)] = offdiag_scale * rng.uniform(-1.0, 1.0, size=(bs, bs))
    rowptr, colidx, vals = _to_bsr(nb, bs, entries)
    order = perm.astype(np.int64)
    return rowptr, colidx, vals, order, layer


def random_block_sparse(nb: int, bs: int, density: float, seed: int = 0, diag_boost: float = 2.0):
    """Random block-sparse matrix with a dominant diagonal block per row (not triangular)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    entries = {}
    for I in range(nb):
        D = rng.uniform(-1.0, 1.0, size=(bs, bs)) + diag_boost * bs * np.eye(bs)
        entries[(I, I)] = D
        for J in range(nb):
            if J != I and rng.random() < density:
                entries[(I, J)] = rng.uniform(-1.0, 1.0, size=(bs, bs))
    return _to_bsr(nb, bs, entries)
