"""Tests of the seeded input generators (no GPU, no oracle arithmetic)."""
import math

import numpy as np
import pytest

from nair_inputs import dg_quad, make_config, topo_sort_blocks, gauss_lobatto_nodes
from nair_inputs.random_blocks import layered_block_triangular, random_block_sparse
from helpers import bsr_dense, dof_index


def _nodal_error(S, x, u, N, p, jitter=0.0):
    nodes = gauss_lobatto_nodes(p)
    h = 1.0 / N
    err = 0.0
    for c in range(N * N):
        iy, ix = divmod(c, N)
        blk = S.perm[c]
        for k in range(S.bs):
            ky, kx = divmod(k, p + 1)
            X, Y = (ix + nodes[kx]) * h, (iy + nodes[ky]) * h
            err = max(err, abs(x[blk * S.bs + k] - u(X, Y)))
    return err


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_polynomial_exactness(p):
    """Upwind DG reproduces any u in Q_p exactly on an affine mesh (Galerkin
    orthogonality: u is in the discrete space and continuous, so the upwind jump
    terms vanish)."""
    b = (math.cos(0.3), math.sin(0.3))
    s = 0.7
    u = lambda x, y: (x ** p) * (y ** p) + 2 * x - y + 1
    ux = lambda x, y: p * x ** (p - 1) * y ** p + 2
    uy = lambda x, y: p * x ** p * y ** (p - 1) - 1
    q = lambda x, y: b[0] * ux(x, y) + b[1] * uy(x, y) + s * u(x, y)
    S = dg_quad(4, p, b, sigma=s, q_fn=q, g_fn=u, seed_perm=7)
    x = np.linalg.solve(S.to_dense(), S.rhs)
    assert _nodal_error(S, x, u, 4, p) < 1e-11


def test_polynomial_exactness_curved_flow_linear_u():
    """With b(x,y) = (y+1/4, -(x+1/4)) and u linear, q = b.grad u + sigma u is
    quadratic and still integrated exactly; the solution is u."""
    bfun = lambda x, y: (y + 0.25, -(x + 0.25))
    u = lambda x, y: 3 * x - 2 * y + 0.5
    q = lambda x, y: (y + 0.25) * 3 + (-(x + 0.25)) * (-2) + 0.5 * u(x, y)
    S = dg_quad(5, 2, bfun, sigma=0.5, q_fn=q, g_fn=u, seed_perm=3)
    x = np.linalg.solve(S.to_dense(), S.rhs)
    assert _nodal_error(S, x, u, 5, 2) < 1e-11


@pytest.mark.parametrize("name", ["dg_q1_32", "dg_q2_256_curved", "dg_q4_512_jitter",
                                  "dg_q3_256_curved_sigma"])
def test_block_triangular_after_topo_sort(name):
    S, _ = make_config(name, N=6)
    order = S.topo_order
    pos = np.empty(S.nb, dtype=np.int64)
    pos[order] = np.arange(S.nb)
    rows = np.repeat(np.arange(S.nb), np.diff(S.rowptr))
    assert np.all(pos[S.colidx] <= pos[rows])
    D = S.to_dense()
    idx = dof_index(order, S.bs)
    Dp = D[np.ix_(idx, idx)]
    # strictly block upper part is zero
    for a in range(S.nb):
        assert not np.any(Dp[a * S.bs:(a + 1) * S.bs, (a + 1) * S.bs:])


def test_sizes_match_configs():
    S, k = make_config("dg_q1_32")
    assert (S.nb, S.bs, S.nnzb, S.n, k) == (1024, 4, 3008, 4096, 1)
    # N x N quads: N^2 diagonal blocks plus 2 N (N-1) interior faces, each upwind once
    for N in (8, 17):
        S, _ = make_config("dg_q2_256_curved", N=N)
        assert S.nnzb == N * N + 2 * N * (N - 1)
        assert S.bs == 9


def test_off_diagonal_blocks_touch_one_face():
    """Upwind face coupling only involves the (p+1) nodes on each of the two
    faces: (p+1)^2 nonzeros per off-diagonal block."""
    S, _ = make_config("dg_q2_256_curved", N=6)
    rows = np.repeat(np.arange(S.nb), np.diff(S.rowptr))
    off = rows != S.colidx
    nz = np.count_nonzero(S.vals[off], axis=(1, 2))
    assert np.all(nz == 9)


def test_jittered_mesh_is_valid_and_seeded():
    S1, _ = make_config("dg_q4_512_jitter", N=5)
    S2, _ = make_config("dg_q4_512_jitter", N=5)
    assert np.array_equal(S1.vals, S2.vals) and np.array_equal(S1.rhs, S2.rhs)
    S3, _ = make_config("dg_q4_512_jitter", N=5, seed_jitter=99)
    assert not np.allclose(S1.vals, S3.vals)


def test_cycle_detection():
    rp, ci, va, order, layer = layered_block_triangular(30, 2, 4, seed=2)
    topo_sort_blocks(30, rp, ci)
    rp, ci, va, order, layer = layered_block_triangular(30, 2, 4, seed=2, back_edges=2)
    with pytest.raises(ValueError):
        topo_sort_blocks(30, rp, ci)


def test_random_generators_shapes():
    rp, ci, va = random_block_sparse(12, 3, 0.2, seed=1)
    assert rp[-1] == len(ci) == va.shape[0]
    rows = np.repeat(np.arange(12), np.diff(rp))
    assert np.all(np.isin(np.arange(12), ci[rows == ci]))


def test_sigma_q_model_is_affine_in_sigma():
    """A(sigma) = A(0) + sigma_K M_K on the diagonal blocks and b = M q reproduce
    the direct assembly with that sigma and nodal q."""
    from nair_inputs import sigma_q_model
    import math
    bfun = lambda x, y: (y + 0.25, -(x + 0.25))
    m = sigma_q_model(5, 2, bfun, seed_perm=3)
    S0 = m["system"]
    vals = S0.vals.copy()
    vals[m["diag_pos"]] += m["sigma"][:, None, None] * m["mass"]
    b = np.einsum("kij,kj->ki", m["mass"], m["q"].reshape(S0.nb, S0.bs)).reshape(-1)
    sig_cell = m["sigma"][S0.perm]
    q_cell = m["q"].reshape(S0.nb, S0.bs)[S0.perm]
    S = dg_quad(5, 2, bfun, sigma=sig_cell, seed_perm=3, q_nodal=q_cell)
    assert np.allclose(vals, S.vals, rtol=0, atol=1e-14)
    assert np.allclose(b, S.rhs, rtol=0, atol=1e-14)


def test_batch_concatenation_is_block_diagonal():
    from nair_inputs import make_batch, concat_systems
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(3, 5, 4), nang=5)
    assert k == 2 and [S.N for S in systems] == [3, 5, 4, 3, 5]
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    D = bsr_dense(len(rp) - 1, 9, rp, ci, va)
    o = 0
    for S in systems:
        n = S.n
        assert np.array_equal(D[o:o + n, o:o + n], S.to_dense())
        assert not np.any(D[o:o + n, :o]) and not np.any(D[o:o + n, o + n:])
        assert np.array_equal(rhs[o:o + n], S.rhs)
        o += n
    # directions never axis-aligned, sources differ per angle
    assert not np.array_equal(systems[0].rhs[:9], systems[4].rhs[:9])


def test_batch_generation_in_worker_processes_matches():
    from nair_inputs import make_batch
    a, _ = make_batch("dg_q2_angles64_uneven", sizes=(4, 6), nang=4)
    b, _ = make_batch("dg_q2_angles64_uneven", sizes=(4, 6), nang=4, workers=2)
    for Sa, Sb in zip(a, b):
        assert np.array_equal(Sa.vals, Sb.vals) and np.array_equal(Sa.rhs, Sb.rhs)
