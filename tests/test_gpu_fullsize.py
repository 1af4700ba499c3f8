"""GPU parity at full workload sizes, in the launch configuration bench.py times.

* 256x256 Q2 curved flow (589,824 DOFs): the whole hierarchy, the solve and
  the transposed solve against the oracle.
* The 512x512 jittered Q4 recipe at N = 128 (409,600 DOFs, every default path
  of the full-size workload active): the same complete comparison.
* 512x512 jittered Q4 (6,553,600 DOFs, 25x25 blocks): too large for the oracle
  to set up in a test, so sampled outputs the oracle computes one by one (block
  inverses), brute-force definitions on sampled rows (block sizes, strength,
  one-point), the splitting certificate on the whole level, and the converged
  residuals recomputed independently on the CPU.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nair_inputs import make_config
from test_gpu_parity import build_pair, compare_hierarchies, check_solve, to_dev, np_, _need_gpu, _say
from test_oracle_pins import _splitting_certificate

pytestmark = pytest.mark.gpu


def test_fullsize_bench_workload_parity():
    _say("test: full-size dg_q2_256_curved parity (hierarchy, solve, transposed solve)")
    S, k = make_config("dg_q2_256_curved")
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=k)
    compare_hierarchies(G, O)
    _say("  hierarchy identical; solving")
    check_solve(G, O, S.rhs)
    g = np.random.Generator(np.random.PCG64(300)).uniform(-1, 1, S.n)
    check_solve(G, O, g, trans=True)


def test_q4_jittered_128_full_hierarchy_parity():
    """The Q4 recipe (25x25 blocks, jittered mesh) at N = 128: 409,600 DOFs,
    large enough that every default path of the full-size workload fires on
    the finest levels (face rectangles, F-ordered sweep copies with
    column-major row-compressed blocks, row-compressed Z, the 25x25
    matrix-core products), small enough for the oracle.  Every level, the
    solve and the transposed solve against the oracle."""
    import paper_1704_05001_amd as P
    _say("test: dg_q4_512_jitter recipe at N=128, full hierarchy parity")
    S, k = make_config("dg_q4_512_jitter", N=128)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=k)
    lv0 = G.level(0, fields=())
    assert lv0["face_rmax"] == 5 and lv0["sweep_nnzb"] >= 0
    assert G.level(1, fields=())["sweep_nnzb"] >= 0
    compare_hierarchies(G, O)
    _say("  hierarchy identical; solving")
    check_solve(G, O, S.rhs)
    g = np.random.Generator(np.random.PCG64(300)).uniform(-1, 1, S.n)
    check_solve(G, O, g, trans=True)


def _bsr_matvec(S, x, trans=False):
    import scipy.sparse as sp
    A = sp.bsr_matrix((S.vals, S.colidx, S.rowptr), shape=(S.n, S.n))
    return A.T @ x if trans else A @ x


def test_fullsize_q4_512_sampled():
    import paper_1704_05001_amd as P
    _need_gpu()
    _say("test: full-size dg_q4_512_jitter (6.55M DOFs): generating")
    S, k = make_config("dg_q4_512_jitter")
    _say("  setup + solve on the GPU")
    G = P.Hierarchy(*to_dev(S.rowptr, S.colidx, S.vals), S.bs, P.Params(degree=k))
    b = torch.from_numpy(S.rhs).cuda()
    x, res = G.solve(b, rtol=1e-10)
    assert res.status == "OK", res
    g = np.random.Generator(np.random.PCG64(300)).uniform(-1, 1, S.n)
    y, resT = G.solve_T(torch.from_numpy(g).cuda(), rtol=1e-10)
    assert resT.status == "OK", resT
    _say(f"  {res.iters} / {resT.iters} iterations; checking")
    # independent CPU residuals
    xh = np_(x)
    r = S.rhs - _bsr_matvec(S, xh)
    assert np.linalg.norm(r) / np.linalg.norm(S.rhs) <= 1.0001e-10
    yh = np_(y)
    rT = g - _bsr_matvec(S, yh, trans=True)
    assert np.linalg.norm(rT) / np.linalg.norm(g) <= 1.0001e-10
    L = G.level(0, fields=("rowptr", "colidx", "dinv", "bnorm", "mask", "lam", "cf", "cidx", "pmap", "dround"))
    rp, ci = np_(L["rowptr"]), np_(L["colidx"])
    assert np.array_equal(rp, S.rowptr) and np.array_equal(ci, S.colidx)
    bnorm, mask, cf, pmap = np_(L["bnorm"]), np_(L["mask"]), np_(L["cf"]), np_(L["pmap"])
    theta, phi = P.Params().theta, P.Params().phi   # the defaults the hierarchy was built with
    rng = np.random.default_rng(0)
    rows = rng.choice(S.nb, size=200, replace=False)
    dinv = np_(L["dinv"][torch.from_numpy(rows).cuda().long()])
    cidx = np_(L["cidx"])
    cpts = np.nonzero(cf == 1)[0]
    for n_, I in enumerate(rows):
        lo, hi = rp[I], rp[I + 1]
        d = lo + int(np.nonzero(ci[lo:hi] == I)[0][0])
        # the oracle's block inverse, computed for this block alone: identical bits
        assert np.array_equal(oracle.block_inverse(S.vals[d]), dinv[n_]), I
        size = np.abs(S.vals[lo:hi]).max(axis=(1, 2))
        assert np.array_equal(size, bnorm[lo:hi])
        off = ci[lo:hi] != I
        m = size[off].max() if off.any() else 0.0
        st = off & (m > 0) & (size >= theta * m)
        sp_ = off & (m > 0) & (size >= phi * m)
        assert np.array_equal(mask[lo:hi] & 1, st.astype(np.uint8))
        assert np.array_equal((mask[lo:hi] >> 1) & 1, sp_.astype(np.uint8))
        if cf[I] == 1:
            assert pmap[I] == cidx[I]
        else:
            cand = off & (cf[ci[lo:hi]] == 1) & (size > 0)
            if not cand.any():
                assert pmap[I] == -1
            else:
                best = size[cand].max()
                J = ci[lo:hi][cand][size[cand] == best].min()
                assert cpts[pmap[I]] == J
    # lambda from the GPU's own mask, and the splitting certificate on the whole level
    lam = np_(L["lam"])
    assert np.array_equal(lam, np.bincount(ci[(mask & 1) == 1], minlength=S.nb))

    class Lv:
        pass
    lv = Lv()
    lv.nb, lv.rowptr, lv.colidx, lv.mask, lv.lam, lv.cf, lv.dround = S.nb, rp, ci, mask, lam, cf, np_(L["dround"])
    _say("  splitting certificate")
    _splitting_certificate(lv, 0, 0)
