"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: bit-exact for integer/index/pattern data (strength masks, lambda, C/F
splitting and its rounds, one-point map, Z and coarse-operator patterns,
level count, iteration count); the setup values that feed decisions (block
sizes, D^-1, Z, coarse operators) are computed in the same fixed FP64 order on
both sides and are compared for equality; solve-phase values within 1e-12
(iterates, relative to max |x|) and residual histories within
1e-12 + 1e-6 h_k.  The coarsest level's dense inverse (Gauss-Jordan on the GPU,
LU on the oracle) is compared to 1e-10 relative.
"""
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nair_inputs import dg_quad, make_config
from nair_inputs.random_blocks import layered_block_triangular, random_block_sparse

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(rp, ci, va):
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(np.ascontiguousarray(rp, dtype=np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(ci, dtype=np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(va, dtype=np.float64)).to(dev))


def build_pair(nb, bs, rp, ci, va, gpu_kw=None, **kw):
    """GPU and oracle hierarchies of one matrix; gpu_kw holds GPU-only parameters
    (form="scalar" also selects the oracle's form 1)."""
    import paper_1704_05001_amd as P
    _need_gpu()
    d_rp, d_ci, d_va = to_dev(rp, ci, va)
    gpu_kw = dict(gpu_kw or {})
    G = P.Hierarchy(d_rp, d_ci, d_va, bs, P.Params(**kw, **gpu_kw))
    O = oracle.Hierarchy(nb, bs, rp, ci, va, oracle.Params(**oracle_kw(gpu_kw, kw)))
    return G, O


def oracle_kw(gpu_kw, kw):
    """Oracle parameters for GPU parameters: form "scalar" is the oracle's form 1,
    cycle "F" its cycle 1; precision and tuning have no oracle counterpart."""
    okw = dict(kw)
    if (gpu_kw or {}).get("form") == "scalar":
        okw["form"] = 1
    if (gpu_kw or {}).get("cycle") == "F":
        okw["cycle"] = 1
    return okw


def np_(t):
    return t.detach().cpu().numpy()


def compare_hierarchies(G, O):
    gl = G.info()["levels"]
    assert gl == O.num_levels, (gl, O.num_levels)
    for l in range(gl):
        g = G.level(l)
        o = O.level(l)
        assert (g["nb"], g["bs"], g["nnzb"], g["coarsest"]) == (o.nb, o.bs, len(o.colidx), o.coarsest), l
        assert np.array_equal(np_(g["rowptr"]), o.rowptr), l
        assert np.array_equal(np_(g["colidx"]), o.colidx), l
        assert np.array_equal(np_(g["vals"]), o.vals), f"level {l} operator values differ"
        if o.coarsest:
            n = o.nb * o.bs
            inv = np_(g["dense_inv"])
            lu, piv = o.dense_lu, o.dense_piv
            # oracle inverse from its LU factors
            ref = np.linalg.inv(oracle.bsr_to_dense(o.nb, o.bs, o.rowptr, o.colidx, o.vals))
            assert np.abs(inv - ref).max() <= 1e-10 * np.abs(ref).max(), l
            continue
        assert np.array_equal(np_(g["bnorm"]), o.bnorm), l
        assert np.array_equal(np_(g["dinv"]), o.dinv), f"level {l} D^-1 differs"
        assert np.array_equal(np_(g["mask"]), o.mask), l
        assert np.array_equal(np_(g["lam"]), o.lam), l
        assert np.array_equal(np_(g["cf"]), o.cf), l
        assert np.array_equal(np_(g["dround"]), o.dround), l
        assert g["pmis_rounds"] == o.pmis_rounds, l
        assert tuple(g["margin"]) == tuple(o.margin), (l, g["margin"], o.margin)   # decision-margin audit
        assert np.array_equal(np_(g["cidx"]), o.cidx), l
        assert g["nc"] == o.nc
        assert np.array_equal(np_(g["pmap"]), o.pmap), l
        assert np.array_equal(np_(g["z_rowptr"]), o.z_rowptr), l
        assert np.array_equal(np_(g["z_colidx"]), o.z_colidx), l
        assert np.array_equal(np_(g["z_vals"]), o.z_vals), f"level {l} Z differs"


def check_solve(G, O, b, rtol=1e-10, trans=False, max_iter=200):
    bt = torch.from_numpy(b).cuda()
    if trans:
        xg, rg = G.solve_T(bt, rtol=rtol, max_iter=max_iter)
        xo, ho, so = O.solve_T(b, rtol, max_iter)
    else:
        xg, rg = G.solve(bt, rtol=rtol, max_iter=max_iter)
        xo, ho, so = O.solve(b, rtol, max_iter)
    hg = G.history()
    assert rg.status == so, (rg.status, so)
    assert len(hg) == len(ho) == rg.iters
    assert np.all(np.abs(hg - ho) <= 1e-12 + 1e-6 * ho)
    xg = np_(xg)
    assert np.abs(xg - xo).max() <= 1e-12 * np.abs(xo).max()
    return rg, hg


def small_dg(N=6, p=1, theta=0.4, seed=3):
    return dg_quad(N, p, (math.cos(theta), math.sin(theta)), sigma=1.0, seed_perm=seed)


# ------------------------------------------------------------------ tests

def test_block_inverse_and_strength_bit_exact():
    _say("test: block inverse, strength (dg 6x6 Q2)")
    S = small_dg(6, 2)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=1, max_coarse_dofs=40)
    compare_hierarchies(G, O)


def _tied_blocks(nb, bs, seed):
    """nb nonsingular bs x bs blocks of small integers, so that the pivot search
    meets many ties in |a_ik| (equal values and opposite signs) and zeros."""
    rng = np.random.default_rng(seed)
    out = np.empty((nb, bs, bs))
    n = 0
    while n < nb:
        B = rng.integers(-2, 3, size=(bs, bs)).astype(np.float64)
        if abs(np.linalg.det(B)) < 0.5 or np.linalg.cond(B) > 1e6:
            continue
        out[n] = B
        n += 1
    return out


@pytest.mark.parametrize("bs", [4, 7, 9, 16, 25])
def test_block_inverse_pivot_ties_bit_exact(bs):
    """D^-1 of blocks full of pivot ties against the oracle's LU, block by block:
    the first row of largest magnitude must win on every kernel that forms D^-1
    (one thread per block at bs 4 and 9, a half wave per block at 16 and 25,
    one wave per block otherwise)."""
    import paper_1704_05001_amd as P
    _need_gpu()
    nb = 100
    _say(f"test: block inverse with pivot ties (bs {bs}, {nb} blocks)")
    diag = _tied_blocks(nb, bs, seed=bs)
    # block lower bidiagonal: block I also depends on block I - 1 (weakly)
    rows = [[0]] + [[I - 1, I] for I in range(1, nb)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate([np.array(r) for r in rows]).astype(np.int32)
    va = np.random.default_rng(1).uniform(-1, 1, size=(len(ci), bs, bs)) * 1e-3
    rowid = np.repeat(np.arange(nb), np.diff(rp))
    va[rowid == ci] = diag
    # (two levels: the second is solved directly, whatever the splitting gives)
    G = P.Hierarchy(*to_dev(rp, ci, va), bs, P.Params(degree=1, max_coarse_dofs=bs, max_levels=2))
    dinv = G.level(0, fields=("dinv",))["dinv"].cpu().numpy().reshape(nb, bs, bs)
    for I in range(nb):
        assert np.array_equal(oracle.block_inverse(diag[I]), dinv[I]), I
    G.close()


@pytest.mark.parametrize("name,N", [("dg_q1_32", None), ("dg_q2_256_curved", 24), ("dg_q4_512_jitter", 6),
                                    ("dg_q3_256_curved_sigma", 8)])
def test_setup_parity_configs(name, N):
    _say(f"test: setup parity {name} N={N}")
    S, k = make_config(name, N=N)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=k)
    compare_hierarchies(G, O)
    check_solve(G, O, S.rhs)


@pytest.mark.parametrize("relax,degree", [(0, 0), (1, 1), (0, 3), (1, 2)])
def test_parity_variants(relax, degree):
    _say(f"test: variants relax={relax} degree={degree}")
    S, _ = make_config("dg_q2_256_curved", N=12)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=degree, relax=relax, max_coarse_dofs=60)
    compare_hierarchies(G, O)
    check_solve(G, O, S.rhs)
    g = np.random.default_rng(1).uniform(-1, 1, S.n)
    check_solve(G, O, g, trans=True)


@pytest.mark.parametrize("name,N,degree", [("dg_q2_256_curved", 16, 6), ("dg_q2_256_curved", 12, 16),
                                           ("dg_q4_512_jitter", 8, 4)])
def test_high_neumann_degree(name, N, degree):
    """Neumann degrees past the usual few (up to the limit, 16): the sum of the
    k + 1 terms that Z's product forms without storing it, through the term
    maps composed over k pattern unions, against the oracle's stored sums."""
    _say(f"test: Neumann degree {degree} ({name} N={N})")
    S, _ = make_config(name, N=N)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=degree, max_coarse_dofs=4 * S.bs)
    compare_hierarchies(G, O)
    check_solve(G, O, S.rhs)


def test_parity_random_matrices():
    _say("test: random block matrices")
    rp, ci, va, order, layer = layered_block_triangular(300, 3, 12, deps=3, seed=7, zero_entries=0.3)
    G, O = build_pair(300, 3, rp, ci, va, degree=2, max_coarse_dofs=30)
    compare_hierarchies(G, O)
    b = np.random.default_rng(2).uniform(-1, 1, 900)
    check_solve(G, O, b)
    rp, ci, va = random_block_sparse(200, 2, 0.02, seed=3)
    G, O = build_pair(200, 2, rp, ci, va, degree=1, max_coarse_dofs=20, phi=0.0, drop=0.0)
    compare_hierarchies(G, O)


@pytest.mark.parametrize("bs", [8, 12, 32])
def test_parity_generic_block_sizes(bs):
    """Block sizes off the specialised instances (the gather of kept blocks with
    sixteen 64-word chunks, the generic block kernels, bs 32 at the limit): the
    whole hierarchy bit for bit and the solve against the oracle."""
    _need_gpu()
    _say(f"test: random block matrix at bs {bs}")
    nb = 200
    rp, ci, va, order, layer = layered_block_triangular(nb, bs, 10, deps=3, seed=bs, zero_entries=0.3)
    G, O = build_pair(nb, bs, rp, ci, va, degree=2, max_coarse_dofs=20 * bs)
    assert O.num_levels >= 3   # (two Galerkin products, so two gathers of kept blocks)
    compare_hierarchies(G, O)
    b = np.random.default_rng(5).uniform(-1, 1, nb * bs)
    check_solve(G, O, b)


def test_cf_override_and_seed():
    _say("test: cf override and seed")
    S, k = make_config("dg_q1_32", N=10)
    cf = (np.arange(S.nb) % 3 == 0).astype(np.int8)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=1, cf_override=cf)
    compare_hierarchies(G, O)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=1, seed=987654321)
    compare_hierarchies(G, O)


def test_transposed_cycle_adjoint_on_gpu():
    _say("test: adjointness of the GPU cycle")
    S, k = make_config("dg_q2_256_curved", N=16)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=2)
    rng = np.random.default_rng(5)
    u = torch.from_numpy(rng.uniform(-1, 1, S.n)).cuda()
    v = torch.from_numpy(rng.uniform(-1, 1, S.n)).cuda()
    lhs = float(torch.dot(v, G.vcycle(u)))
    rhs = float(torch.dot(G.vcycle_T(v), u))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # and each application matches the oracle's
    eo = O.vcycle(np_(u))
    assert np.abs(np_(G.vcycle(u)) - eo).max() <= 1e-12 * np.abs(eo).max()
    yo = O.vcycle_T(np_(v))
    assert np.abs(np_(G.vcycle_T(v)) - yo).max() <= 1e-12 * np.abs(yo).max()


def test_edge_cases():
    _say("test: edge cases (single level, one block, empty Neumann terms)")
    # one level: dense solve only
    S = small_dg(3, 1)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, max_coarse_dofs=1000)
    compare_hierarchies(G, O)
    check_solve(G, O, S.rhs)
    # one level larger than the in-LDS dense inverse (576 unknowns: global-memory path)
    S = small_dg(8, 2)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, max_coarse_dofs=600)
    compare_hierarchies(G, O)
    check_solve(G, O, S.rhs)
    # a single block
    va = np.array([[[4.0, 1.0], [0.5, 3.0]]])
    G, O = build_pair(1, 2, np.array([0, 1]), np.array([0]), va, max_coarse_dofs=0)
    compare_hierarchies(G, O)
    check_solve(G, O, np.array([1.0, -2.0]))
    # block-diagonal matrix: no strong connections, the splitting stalls -> dense
    nb, bs = 40, 2
    rp = np.arange(nb + 1)
    ci = np.arange(nb)
    va = np.random.default_rng(0).uniform(-1, 1, (nb, bs, bs)) + 3 * np.eye(bs)
    G, O = build_pair(nb, bs, rp, ci, va, max_coarse_dofs=4)
    compare_hierarchies(G, O)
    check_solve(G, O, np.ones(nb * bs))
    # zero right-hand side
    S, _ = make_config("dg_q1_32", N=8)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals)
    x, r = G.solve(torch.zeros(S.n, dtype=torch.float64, device="cuda"))
    assert r.status == "OK" and r.iters == 0 and float(x.abs().max()) == 0.0


def test_error_codes():
    _say("test: error codes")
    import paper_1704_05001_amd as P
    _need_gpu()
    S = small_dg(4, 1)
    rows = np.repeat(np.arange(S.nb), np.diff(S.rowptr))
    # unsorted columns in one row
    ci = S.colidx.copy()
    r = next(I for I in range(S.nb) if S.rowptr[I + 1] - S.rowptr[I] >= 2)
    ci[S.rowptr[r]:S.rowptr[r + 1]] = ci[S.rowptr[r]:S.rowptr[r + 1]][::-1]
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(*to_dev(S.rowptr, ci, S.vals), S.bs)
    assert e.value.status == "EINVAL"
    # missing diagonal
    keep = ~((rows == 0) & (S.colidx == 0))
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=S.nb))])
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(*to_dev(rp, S.colidx[keep], S.vals[keep]), S.bs)
    assert e.value.status == "EINVAL"
    # singular diagonal block
    va = S.vals.copy()
    va[(rows == 5) & (S.colidx == 5)] = 0.0
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(*to_dev(S.rowptr, S.colidx, va), S.bs, P.Params(max_coarse_dofs=1))
    assert e.value.status == "ESINGULAR"
    # no convergence within max_iter, and a non-finite right-hand side
    G = P.Hierarchy(*to_dev(S.rowptr, S.colidx, S.vals), S.bs, P.Params(max_coarse_dofs=8))
    b = torch.from_numpy(S.rhs).cuda()
    x, r = G.solve(b, rtol=1e-14, max_iter=1)
    assert r.status == "ENOCONV" and r.iters == 1
    b[3] = float("nan")
    x, r = G.solve(b)
    assert r.status == "ENUMERIC"


def test_setup_is_deterministic():
    _say("test: determinism")
    S, k = make_config("dg_q2_256_curved", N=20)
    import paper_1704_05001_amd as P
    _need_gpu()
    dev = to_dev(S.rowptr, S.colidx, S.vals)
    A = P.Hierarchy(*dev, S.bs, P.Params(degree=k))
    B = P.Hierarchy(*dev, S.bs, P.Params(degree=k))
    for l in range(A.info()["levels"]):
        a, b = A.level(l), B.level(l)
        for key in a:
            if isinstance(a[key], torch.Tensor):
                assert torch.equal(a[key], b[key]), (l, key)


def test_margin_audit_matches_oracle():
    """The decision-margin audit (comparisons within 1e-12 relative in the
    strength, one-point and drop decisions) counts the same near-ties as the
    oracle, with ties planted in theta, in the drop tolerance and by a
    diagonal flow on a uniform grid."""
    _say("test: decision-margin audit")
    S = dg_quad(7, 2, (math.cos(0.4), math.sin(0.4)), sigma=1.0, seed_perm=61)
    O = oracle.Hierarchy(S.nb, S.bs, S.rowptr, S.colidx, S.vals, oracle.Params(degree=1, max_coarse_dofs=20))
    L0 = O.level(0)
    rows = np.repeat(np.arange(L0.nb), np.diff(L0.rowptr))
    off = L0.colidx != rows
    m = np.zeros(L0.nb)
    np.maximum.at(m, rows[off], L0.bnorm[off])
    t = next(t for t in np.flatnonzero(off) if 0 < L0.bnorm[t] < m[rows[t]])
    theta = float(L0.bnorm[t] / m[rows[t]])
    K = oracle.Hierarchy(S.nb, S.bs, S.rowptr, S.colidx, S.vals,
                         oracle.Params(degree=1, max_coarse_dofs=20, drop=0.0)).level(1)
    kr = np.repeat(np.arange(K.nb), np.diff(K.rowptr))
    kn = np.abs(K.vals).max(axis=(1, 2))
    dn = np.zeros(K.nb)
    dn[kr[K.colidx == kr]] = kn[K.colidx == kr]
    u = next(u for u in np.flatnonzero(K.colidx != kr) if kn[u] < 0.5 * dn[kr[u]])
    drop = float(kn[u] / dn[kr[u]])
    U = dg_quad(6, 1, (math.sqrt(0.5), math.sqrt(0.5)), sigma=1.0, seed_perm=7)
    totals = []
    for M, kw in ((S, dict(theta=theta)), (S, dict(drop=drop)), (U, dict(max_coarse_dofs=8)),
                  (S, dict(drop=0.0))):
        kw = dict(dict(degree=1, max_coarse_dofs=20), **kw)
        G, O = build_pair(M.nb, M.bs, M.rowptr, M.colidx, M.vals, **kw)
        compare_hierarchies(G, O)
        totals.append(np.sum([O.level(l).margin for l in range(O.num_levels)], axis=0))
    _say(f"  audit totals (theta, phi, one-point, drop): {[tuple(int(v) for v in x) for x in totals]}")
    assert totals[0][0] >= 1 and totals[1][3] >= 1 and totals[2][2] >= 1
