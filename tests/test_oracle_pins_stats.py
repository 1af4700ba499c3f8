"""Pins of the oracle's cost statistics and of the block red-black special case.

* Cycle complexity (section 6: work units of one level-0 SpMV) on a hand-built
  three-level hierarchy whose every level is fixed by its construction, against
  counts made by hand from the definition, for the V- and the F-cycle and for
  F and FC relaxation.
* The convergence factors rho_avg and rho_last5 on geometric histories, where
  they have closed forms.
* The paper's block red-black example (section 4, the coarsening figure of a
  uniform structured grid): with elements coloured like a chessboard every F
  element depends only on C elements, so A_ff is block diagonal, the Neumann
  restriction of any degree is ideal restriction -A_cf A_ff^{-1}, the coarse
  operator is the Schur complement A_cc - A_cf A_ff^{-1} A_fc, and each coarse
  row couples to at most three coarse elements, all strictly upwind.

No test calls the HIP library.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Hierarchy, Params
from nair_inputs import dg_quad
from helpers import bsr_dense, dof_index, row_blocks


# ------------------------------------------------------ cycle complexity

def _chain4(bs=2):
    """Four blocks, row I depends on block I-1 only (a 1-D upwind chain).

    Diagonal blocks [[2, .5], [0, 3]], off-diagonal blocks [[-1, .25], [.5, -1]].
    With the level-0 splitting forced to C = {0, 2}, F = {1, 3}:
      level 0: nnzb 7; F rows 1, 3 hold 2 + 2 = 4 blocks; C rows 0, 2 hold
               1 + 2 = 3; Z has one block (row of block 2, column 1; the F-F
               part is empty, so Z = -A_21 D_1^{-1} at every degree); one-point
               interpolation maps 1 -> coarse 0 and 3 -> coarse 1.
      level 1: K = R A P is the 2-block chain [[K00], [K10, K11]] with
               K10 = Z_21 A_10 + (Z_21 A_11 + A_21) (nonzero, not dropped):
               nnzb 3.  Its only strong connection is row 1 -> block 0, so
               lambda = (1, 0): block 1 starts F, block 0 becomes C in round 1.
               F rows hold 2 blocks, C rows 1, Z is empty (C row 0 has no F
               column), one F block.
      level 2: one block, the coarsest, dense order bs = 2.
    """
    D = np.array([[2.0, 0.5], [0.0, 3.0]])
    L = np.array([[-1.0, 0.25], [0.5, -1.0]])
    rp = np.array([0, 1, 3, 5, 7], dtype=np.int32)
    ci = np.array([0, 0, 1, 1, 2, 2, 3], dtype=np.int32)
    va = np.stack([D, L, D, L, D, L, D])
    return 4, bs, rp, ci, va


def _hier_chain4(**kw):
    nb, bs, rp, ci, va = _chain4()
    return Hierarchy(nb, bs, rp, ci, va, Params(cf_override=np.array([1, 0, 1, 0], np.int8),
                                                 max_coarse_dofs=2, **kw))


def _check_chain4_structure(H):
    assert H.num_levels == 3
    L0, L1, L2 = H.levels()
    assert list(L0.cf) == [1, 0, 1, 0] and list(L0.pmap) == [0, 0, 1, 1]
    assert list(L0.z_rowptr) == [0, 0, 1] and list(L0.z_colidx) == [1]
    assert L1.nb == 2 and list(L1.rowptr) == [0, 1, 3] and list(L1.colidx) == [0, 0, 1]
    assert list(L1.cf) == [1, 0] and list(L1.z_rowptr) == [0, 0]
    assert L2.coarsest and L2.nb == 1 and L2.dense_lu.shape == (2, 2)


# Hand counts (units of 1/7 WU: level 0 has 7 blocks).  Per non-coarsest level
# the cycle does nu F sweeps over the F rows' blocks, with FC one sweep over the
# C rows' blocks, one restriction over Z's blocks and one interpolation of the
# F blocks; the coarsest level's dense solve costs dense_n^2 entries, i.e.
# dense_n^2 / bs^2 = 1 block; the outer residual is one level-0 SpMV (1 WU).
#   w0 = 4 nu + 3 FC + 1 + 2,  w1 = 2 nu + 1 FC + 0 + 1,  w2 = 1,
#   operators of levels 1 and 2: 3 and 1 blocks.
# V-cycle: 1 + (w0 + w1 + w2) / 7.
# F-cycle: the coarse solve on level l is an F-cycle on l, a residual with A_l
# and a V-cycle on l; at the coarsest both cycles are the dense solve.  So
#   F(2) = w2, F(1) = w1 + [F(2) + 1 + V(2)] = w1 + 2 w2 + 1,
#   F(0) = w0 + [F(1) + 3 + V(1)] = w0 + 2 w1 + 3 w2 + 4,
# and CC = 1 + F(0) / 7.
@pytest.mark.parametrize("degree,relax,cycle,cc_sevenths", [
    (1, 0, 0, 7 + (11 + 5 + 1)),          # nu 2, F:  w0 11, w1 5
    (1, 1, 0, 7 + (14 + 6 + 1)),          # nu 2, FC: w0 14, w1 6
    (2, 0, 0, 7 + (15 + 7 + 1)),          # nu 3, F:  w0 15, w1 7
    (1, 0, 1, 7 + (11 + 10 + 3 + 4)),     # F-cycle, nu 2, F relaxation
    (1, 1, 1, 7 + (14 + 12 + 3 + 4)),     # F-cycle, nu 2, FC relaxation
    (0, 0, 1, 7 + (7 + 6 + 3 + 4)),       # F-cycle, nu 1: w0 7, w1 3
])
def test_cycle_complexity_hand_count(degree, relax, cycle, cc_sevenths):
    H = _hier_chain4(degree=degree, relax=relax, cycle=cycle)
    _check_chain4_structure(H)
    oc, cc = H.complexity()
    assert oc == pytest.approx(11 / 7, rel=1e-15)       # (7 + 3 + 1) / 7
    assert cc == pytest.approx(cc_sevenths / 7, rel=1e-15)


def test_cycle_complexity_two_level_closed_form():
    """A two-level hierarchy of a general matrix: CC = 1 + [nu nnz(F rows) +
    FC nnz(C rows) + nnz(Z) + nb_F] / nnzb_0 + n_c^2 / (bs^2 nnzb_0), counted
    here from the level's arrays with numpy (every term of the definition
    visible).  The F-cycle's coarse solve is two dense solves (the F- and the
    V-cycle on the coarsest level) and one residual with the coarse operator."""
    from nair_inputs import random_blocks
    rp, ci, va = random_blocks.random_block_sparse(30, 2, 0.1, seed=9)
    for relax in (0, 1):
        HV = Hierarchy(30, 2, rp, ci, va, Params(degree=1, relax=relax, max_coarse_dofs=59, max_levels=2))
        HF = Hierarchy(30, 2, rp, ci, va, Params(degree=1, relax=relax, max_coarse_dofs=59, max_levels=2,
                                                 cycle=1))
        assert HV.num_levels == 2
        L0, L1 = HV.levels()
        rl = np.diff(L0.rowptr)
        nnz0 = rl.sum()
        work0 = 2 * rl[L0.cf == 0].sum() + relax * rl[L0.cf == 1].sum() + L0.z_rowptr[-1] + (L0.cf == 0).sum()
        dense = (L1.nb * 2) ** 2 / 4
        assert HV.complexity()[1] == pytest.approx(1 + (work0 + dense) / nnz0, rel=1e-14)
        assert HF.complexity()[1] == pytest.approx(1 + (work0 + 2 * dense + L1.rowptr[-1]) / nnz0, rel=1e-14)


# --------------------------------------------------- convergence factors

@pytest.mark.parametrize("K", [1, 3, 5, 6, 12, 40])
@pytest.mark.parametrize("c,q", [(1.0, 0.25), (3.0, 0.5), (0.125, 0.1)])
def test_rho_stats_on_geometric_histories(K, c, q):
    """h_k = c q^k (k = 1..K): rho_avg = h_K^(1/K) = c^(1/K) q and, once there
    are more than five entries, rho_last5 = (h_K / h_{K-5})^(1/5) = q; with
    five or fewer it falls back to rho_avg."""
    hist = c * q ** np.arange(1, K + 1)
    avg, last5 = oracle.rho_stats(hist)
    assert avg == pytest.approx(c ** (1.0 / K) * q, rel=1e-13)
    if K > 5:
        assert last5 == pytest.approx(q, rel=1e-13)
    else:
        assert last5 == avg


def test_rho_stats_edge_cases():
    assert all(math.isnan(v) for v in oracle.rho_stats([]))
    # a history that stalls after a fast start: the two factors differ
    hist = np.concatenate([1e-3 ** np.arange(1, 4), 1e-9 * 0.9 ** np.arange(1, 8)])
    avg, last5 = oracle.rho_stats(hist)
    assert last5 == pytest.approx(0.9, rel=1e-13)
    assert avg == pytest.approx(hist[-1] ** (1 / 10), rel=1e-13) and avg < 0.2


# ------------------------------------------------ block red-black example

def _red_black(N=8, p=1, angle=math.pi / 8):
    S = dg_quad(N, p, (math.cos(angle), math.sin(angle)), sigma=1.0, seed_perm=17)
    iy, ix = np.divmod(np.arange(N * N), N)
    cf = np.zeros(S.nb, dtype=np.int8)
    cf[S.perm] = ((ix + iy) % 2 == 0).astype(np.int8)
    cell_of = np.empty(S.nb, dtype=np.int64)
    cell_of[S.perm] = np.arange(N * N)
    return S, cf, cell_of


@pytest.mark.parametrize("degree", [0, 1, 2])
def test_red_black_restriction_is_ideal_and_coarse_operator_is_schur(degree):
    """Chessboard splitting of a uniform Q1 grid with a constant flow in the
    first quadrant (every element depends on its west and south neighbours)."""
    N = 8
    S, cf, cell_of = _red_black(N)
    bs = S.bs
    H = Hierarchy(S.nb, bs, S.rowptr, S.colidx, S.vals,
                  Params(degree=degree, cf_override=cf, drop=0.0, max_levels=2, max_coarse_dofs=1))
    L0, L1 = H.levels()
    assert np.array_equal(L0.cf, cf)
    rows = row_blocks(S.rowptr)
    F = np.nonzero(cf == 0)[0]
    C = np.nonzero(cf == 1)[0]
    # A_ff is block diagonal: no F row couples to another F block
    off = rows != S.colidx
    assert not np.any(off & (cf[rows] == 0) & (cf[S.colidx] == 0))
    A = S.to_dense()
    fi, ci_ = dof_index(F, bs), dof_index(C, bs)
    Aff, Afc = A[np.ix_(fi, fi)], A[np.ix_(fi, ci_)]
    Acf, Acc = A[np.ix_(ci_, fi)], A[np.ix_(ci_, ci_)]
    Rid = -Acf @ np.linalg.inv(Aff)                    # ideal restriction's F part
    Z = bsr_dense(L0.nc, bs, L0.z_rowptr, L0.z_colidx, L0.z_vals, ncols=S.nb)[:, fi]
    assert np.abs(Z - Rid).max() <= 1e-13 * np.abs(Rid).max()
    # Z has exactly A_cf's block pattern (the Neumann terms are empty)
    zr = row_blocks(L0.z_rowptr)
    zpairs = {(int(C[i]), int(j)) for i, j in zip(zr, L0.z_colidx)}
    apairs = {(int(I), int(J)) for I, J in zip(rows, S.colidx) if cf[I] == 1 and cf[J] == 0}
    assert zpairs == apairs
    # coarse operator = Schur complement (R A P with R ideal, for any P)
    K = bsr_dense(L1.nb, bs, L1.rowptr, L1.colidx, L1.vals)
    Sch = Acc - Acf @ np.linalg.solve(Aff, Afc)
    assert np.abs(K - Sch).max() <= 1e-13 * np.abs(Sch).max()
    # each coarse row: itself plus at most three coarse elements, all strictly
    # upwind (west/south of it), exactly three in the interior
    iy, ix = np.divmod(cell_of[C], N)
    r1 = row_blocks(L1.rowptr)
    for i in range(L1.nb):
        nbrs = [int(j) for j in L1.colidx[r1 == i] if j != i]
        assert len(nbrs) <= 3
        for j in nbrs:
            assert ix[j] <= ix[i] and iy[j] <= iy[i] and ix[j] + iy[j] < ix[i] + iy[i]
        want = {(ix[i] - 2, iy[i]), (ix[i] - 1, iy[i] - 1), (ix[i], iy[i] - 2)}
        want = {w for w in want if w[0] >= 0 and w[1] >= 0}
        assert {(ix[j], iy[j]) for j in nbrs} == want
        if ix[i] >= 2 and iy[i] >= 2:
            assert len(nbrs) == 3
