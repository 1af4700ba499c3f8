"""Batched hierarchies on the GPU: many independent systems (discrete-ordinate
angles on uneven meshes) in one setup and one graph-captured solve.

Every system of a batch must get exactly the hierarchy the oracle builds for it
alone (bit-exact patterns, splittings and setup values, per level), and the
batched solve must reproduce each system's own oracle iteration (same
iteration count, histories within 1e-12 + 1e-6 h_k, iterates within 1e-12).
The graph-replayed and the eagerly launched iteration must agree bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nair_inputs import make_batch, concat_systems
from test_gpu_parity import np_, _say, to_dev, oracle_kw

import paper_1704_05001_amd as P

pytestmark = pytest.mark.gpu

BATCH = "dg_q2_angles64_uneven"


def build_batch(systems, gpu_kw=None, oracles=True, **kw):
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    d_rp, d_ci, d_va = to_dev(rp, ci, va)
    G = P.Hierarchy(d_rp, d_ci, d_va, systems[0].bs, P.Params(**kw, **(gpu_kw or {})), sys_nb=sys_nb)
    Os = None
    if oracles:
        okw = oracle_kw(gpu_kw, kw)
        Os = [oracle.Hierarchy(S.nb, S.bs, S.rowptr, S.colidx, S.vals, oracle.Params(**okw)) for S in systems]
    return G, Os, rhs


def compare_batch(G, Os, check=None):
    """Each system's slice of every GPU level against its own oracle hierarchy."""
    L = G.num_levels
    if check is None:
        assert L == max(O.num_levels for O in Os)
    for l in range(L):
        sy = G.systems(l)
        seg, mode, doff = sy["seg"], sy["mode"], sy["dense_off"]
        nxt = G.systems(l + 1)["seg"] if l + 1 < L else None
        g = {k: np_(v) if torch.is_tensor(v) else v for k, v in G.level(l).items()}
        bs = g["bs"]
        for k, O in enumerate(Os):
            if check is not None and k not in check:
                continue
            if l >= O.num_levels:
                assert mode[k] == 0 and seg[k] == seg[k + 1], (l, k)
                continue
            o = O.level(l)
            b0, b1 = int(seg[k]), int(seg[k + 1])
            assert b1 - b0 == o.nb, (l, k)
            t0, t1 = int(g["rowptr"][b0]), int(g["rowptr"][b1])
            assert np.array_equal(g["rowptr"][b0:b1 + 1] - t0, o.rowptr), (l, k)
            assert np.array_equal(g["colidx"][t0:t1] - b0, o.colidx), (l, k)
            assert np.array_equal(g["vals"][t0:t1], o.vals), f"level {l} system {k} operator values"
            if o.coarsest:
                assert mode[k] == 2, (l, k)
                n = o.nb * o.bs
                flat = g["dense_inv"].reshape(-1)
                inv = flat[int(doff[k]):int(doff[k]) + n * n].reshape(n, n)
                ref = np.linalg.inv(oracle.bsr_to_dense(o.nb, o.bs, o.rowptr, o.colidx, o.vals))
                assert np.abs(inv - ref).max() <= 1e-10 * np.abs(ref).max(), (l, k)
                continue
            assert mode[k] == 1, (l, k)
            assert np.array_equal(g["bnorm"][t0:t1], o.bnorm), (l, k)
            assert np.array_equal(g["dinv"][b0:b1], o.dinv), f"level {l} system {k} D^-1"
            assert np.array_equal(g["mask"][t0:t1], o.mask), (l, k)
            assert np.array_equal(g["lam"][b0:b1], o.lam), (l, k)
            assert np.array_equal(g["cf"][b0:b1], o.cf), (l, k)
            assert np.array_equal(g["dround"][b0:b1], o.dround), (l, k)
            c0, c1 = int(nxt[k]), int(nxt[k + 1])
            assert c1 - c0 == o.nc, (l, k)
            cid = g["cidx"][b0:b1].copy()
            cid[cid >= 0] -= c0
            assert np.array_equal(cid, o.cidx), (l, k)
            pm = g["pmap"][b0:b1].copy()
            pm[pm >= 0] -= c0
            assert np.array_equal(pm, o.pmap), (l, k)
            z0, z1 = int(g["z_rowptr"][c0]), int(g["z_rowptr"][c1])
            assert np.array_equal(g["z_rowptr"][c0:c1 + 1] - z0, o.z_rowptr), (l, k)
            assert np.array_equal(g["z_colidx"][z0:z1] - b0, o.z_colidx), (l, k)
            assert np.array_equal(g["z_vals"][z0:z1], o.z_vals), f"level {l} system {k} Z"


def check_batch_solve(G, Os, systems, b, rtol=1e-10, trans=False, graph=True, check=None, fp32=False):
    bt = torch.from_numpy(b).cuda()
    x, res = G.solve_batch(bt, rtol=rtol, trans=trans, graph=graph)
    x = np_(x)
    o = 0
    for k, S in enumerate(systems):
        n = S.n
        r = res[k]
        assert r.status == "OK" and r.relres <= rtol, (k, r)
        if check is None or k in check:
            bk = b[o:o + n]
            xo, ho, so = (Os[k].solve_T if trans else Os[k].solve)(bk, rtol, 200)
            h = G.batch_history(k)
            assert so == "OK"
            err = np.abs(x[o:o + n] - xo).max() / np.abs(xo).max()
            if fp32:
                assert abs(r.iters - len(ho)) <= 2, (k, r.iters, len(ho))
                assert err <= 1e-8, (k, err)
            else:
                assert r.iters == len(ho) == len(h), (k, r.iters, len(ho), len(h))
                assert np.all(np.abs(h - ho) <= 1e-12 + 1e-6 * ho), k
                assert err <= 1e-12, (k, err)
        o += n
    return x, res


@pytest.mark.parametrize("sizes,nang", [((3, 6, 10, 14), 6), ((8, 5), 3)])
def test_batch_setup_and_solve_match_each_system_alone(sizes, nang):
    _say(f"test: batch sizes={sizes} nang={nang}")
    systems, k = make_batch(BATCH, sizes=sizes, nang=nang)
    G, Os, rhs = build_batch(systems, degree=k)
    compare_batch(G, Os)
    check_batch_solve(G, Os, systems, rhs)
    g = np.random.default_rng(2).uniform(-1, 1, rhs.size)
    check_batch_solve(G, Os, systems, g, trans=True)


@pytest.mark.parametrize("relax,degree", [(1, 1), (0, 3)])
def test_batch_variants(relax, degree):
    _say(f"test: batch variants relax={relax} degree={degree}")
    systems, _ = make_batch(BATCH, sizes=(5, 9, 12), nang=4)
    G, Os, rhs = build_batch(systems, degree=degree, relax=relax, max_coarse_dofs=60)
    compare_batch(G, Os)
    check_batch_solve(G, Os, systems, rhs)
    g = np.random.default_rng(3).uniform(-1, 1, rhs.size)
    check_batch_solve(G, Os, systems, g, trans=True)


def test_graph_replay_equals_eager_launches():
    _say("test: graph replay vs eager batch iteration")
    systems, k = make_batch(BATCH, sizes=(6, 11), nang=4)
    G, _, rhs = build_batch(systems, oracles=False, degree=k)
    bt = torch.from_numpy(rhs).cuda()
    for trans in (False, True):
        xg, rg = G.solve_batch(bt, trans=trans, graph=True)
        hg = [G.batch_history(s) for s in range(G.nsys)]
        xe, re = G.solve_batch(bt, trans=trans, graph=False)
        he = [G.batch_history(s) for s in range(G.nsys)]
        assert torch.equal(xg, xe)
        assert [r.iters for r in rg] == [r.iters for r in re]
        for a, b in zip(hg, he):
            assert np.array_equal(a, b)
        # a second replay of the cached graph gives the same answer
        x2, r2 = G.solve_batch(bt, trans=trans, graph=True)
        assert torch.equal(x2, xg)


def test_single_system_batch_solve_equals_plain_solve():
    _say("test: one-system batch solve vs nair_solve")
    systems, k = make_batch(BATCH, sizes=(16,), nang=1)
    S = systems[0]
    d_rp, d_ci, d_va = to_dev(S.rowptr, S.colidx, S.vals)
    G = P.Hierarchy(d_rp, d_ci, d_va, S.bs, P.Params(degree=k))
    bt = torch.from_numpy(S.rhs).cuda()
    x1, r1 = G.solve(bt)
    x2, r2 = G.solve_batch(bt)
    assert r2[0].iters == r1.iters
    assert torch.equal(x1, x2)
    h1, h2 = G.history(), G.batch_history(0)
    assert np.all(np.abs(h1 - h2) <= 1e-13 * h1)
    with pytest.raises(P.NairError):
        B, _, rhs = build_batch(systems + systems, oracles=False, degree=k)
        B.solve(torch.from_numpy(rhs).cuda())


def test_batch_fp32_hierarchy():
    _say("test: batch with the FP32-stored hierarchy")
    systems, k = make_batch(BATCH, sizes=(6, 12, 9), nang=5)
    G, Os, rhs = build_batch(systems, gpu_kw=dict(precision="fp32"), degree=k)
    compare_batch(G, Os)
    check_batch_solve(G, Os, systems, rhs, fp32=True)
    check_batch_solve(G, Os, systems, rhs, trans=True, fp32=True)


def test_batch_rejects_coupled_systems():
    _say("test: batch with a block coupling two systems")
    systems, k = make_batch(BATCH, sizes=(4,), nang=2)
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    # move one off-diagonal block of the second system into the first system's columns
    nb0 = int(sys_nb[0])
    row = nb0 + 5
    t = int(rp[row])
    if ci[t] == row:
        t += 1
    ci = ci.copy()
    ci[t] = 0
    order = np.argsort(ci[rp[row]:rp[row + 1]], kind="stable")
    ci[rp[row]:rp[row + 1]] = ci[rp[row]:rp[row + 1]][order]
    va = va.copy()
    va[rp[row]:rp[row + 1]] = va[rp[row]:rp[row + 1]][order]
    d_rp, d_ci, d_va = to_dev(rp, ci, va)
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(d_rp, d_ci, d_va, 9, P.Params(degree=k), sys_nb=sys_nb)
    assert e.value.status == "EINVAL"


def test_batch_full_size_angles():
    """The 64-angle uneven-mesh workload (17.7M DOFs): FP64 and FP32-stored
    hierarchies, every system converged; systems 0, 1 and 3 (64^2, 128^2 and
    256^2 meshes) against their own oracle hierarchies."""
    systems, k = make_batch(BATCH, workers=8, check_acyclic=False)
    _say(f"test: full batch ({sum(S.n for S in systems)} DOFs, {len(systems)} systems)")
    check = (0, 1, 3)
    assert [systems[j].N for j in check] == [64, 128, 256]
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    d_rp, d_ci, d_va = to_dev(rp, ci, va)
    bt = torch.from_numpy(rhs).cuda()
    Os = {j: oracle.Hierarchy(systems[j].nb, 9, systems[j].rowptr, systems[j].colidx, systems[j].vals,
                              oracle.Params(degree=k)) for j in check}
    Olist = [Os.get(j) for j in range(len(systems))]
    for prec in ("fp64", "fp32"):
        G = P.Hierarchy(d_rp, d_ci, d_va, 9, P.Params(degree=k, precision=prec), sys_nb=sys_nb)
        _say(f"  {prec}: {G.num_levels} levels")
        compare_batch(G, [O if O is not None else _Absent() for O in Olist], check=check)
        x, res = check_batch_solve(G, Olist, systems, rhs, check=check, fp32=(prec == "fp32"))
        its = [r.iters for r in res]
        _say(f"  {prec}: iterations min {min(its)} max {max(its)}")
        G.close()


class _Absent:
    """Stands in for systems without an oracle hierarchy in compare_batch."""
    num_levels = 0
