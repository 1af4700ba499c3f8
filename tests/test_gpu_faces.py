"""Face-compressed finest operator (nair_params.faces): the compact copy holds
exactly the nonzero rows, columns and entries of every off-diagonal block and
the diagonal blocks whole, and every solve reads it without changing a bit
of its result: the same handles with faces off give identical iterates and
histories (forward, transposed, F and FC, F-cycle, FP32-stored, GMRES,
batched), while the oracle comparison of the other GPU tests runs with the
copy on (the default)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config, make_batch, concat_systems
from nair_inputs.random_blocks import layered_block_triangular
from test_gpu_parity import build_pair, small_dg, to_dev, _say, np_, check_solve

pytestmark = pytest.mark.gpu


def _masks(vals):
    nzr = (vals != 0).any(axis=2)           # [nnzb, bs] rows with a nonzero
    nzc = (vals != 0).any(axis=1)           # [nnzb, bs] columns with a nonzero
    return nzr, nzc


def check_face_copy(G, rp, ci, va):
    v = G.level(0)
    assert "face_meta" in v, "no face copy built"
    nb, bs = v["nb"], v["bs"]
    rows = np.repeat(np.arange(nb), np.diff(rp))
    diag = ci == rows
    meta = np_(v["face_meta"]).view(np.uint64)
    rmask = (meta & np.uint64(0xFFFFFFFF)).astype(np.int64)
    cmask = (meta >> np.uint64(32)).astype(np.int64)
    nzr, nzc = _masks(va)
    bit = 1 << np.arange(bs)
    want_r = (nzr * bit).sum(axis=1)
    want_c = (nzc * bit).sum(axis=1)
    assert np.array_equal(rmask[~diag], want_r[~diag])
    assert np.array_equal(cmask[~diag], want_c[~diag])
    assert not meta[diag].any()
    rmax, cmax = v["face_rmax"], v["face_cmax"]
    assert rmax == nzr[~diag].sum(axis=1).max() and cmax == max(1, nzc[~diag].sum(axis=1).max())
    fv = np_(v["face_vals"]).reshape(len(ci), rmax, cmax)
    for t in np.flatnonzero(~diag):
        r = np.flatnonzero(nzr[t])
        c = np.flatnonzero(nzc[t])
        rect = np.zeros((rmax, cmax))
        rect[:len(r), :len(c)] = va[t][np.ix_(r, c)]
        assert np.array_equal(fv[t], rect), t
    # the diagonal blocks by columns
    assert np.array_equal(np_(v["face_dvals"]), va[diag][np.argsort(rows[diag])].transpose(0, 2, 1))
    return rmax, cmax


def pair_on_off(rp, ci, va, bs, **kw):
    import paper_1704_05001_amd as P
    d = to_dev(rp, ci, va)
    on = P.Hierarchy(*d, bs, P.Params(**kw))
    off = P.Hierarchy(*d, bs, P.Params(faces=False, **kw))
    return on, off


def same_solves(on, off, b, trans=False, rtol=1e-10):
    bt = torch.from_numpy(b).cuda()
    f = (lambda H: H.solve_T) if trans else (lambda H: H.solve)
    x1, r1 = f(on)(bt, rtol=rtol)
    h1 = on.history()
    x2, r2 = f(off)(bt, rtol=rtol)
    h2 = off.history()
    assert r1.status == r2.status and r1.iters == r2.iters
    assert np.array_equal(h1, h2), "histories differ"
    assert torch.equal(x1, x2), "iterates differ"
    return r1


@pytest.mark.parametrize("name,N,expect", [("dg_q1_32", None, (2, 2)), ("dg_q2_256_curved", 16, (3, 3)),
                                           ("dg_q4_512_jitter", 5, (5, 5))])
def test_face_copy_holds_the_nonzero_face_blocks(name, N, expect):
    _say(f"test: face copy {name} N={N}")
    import paper_1704_05001_amd as P
    S, k = make_config(name, N=N)
    G = P.Hierarchy(*to_dev(S.rowptr, S.colidx, S.vals), S.bs, P.Params(degree=k))
    assert check_face_copy(G, S.rowptr, S.colidx, S.vals) == expect
    # the transposed operator's copy is built with the transposes and used by solve_T
    G.solve_T(torch.from_numpy(S.rhs).cuda())
    off = P.Hierarchy(*to_dev(S.rowptr, S.colidx, S.vals), S.bs, P.Params(degree=k, faces=False))
    assert "face_meta" not in off.level(0)
    assert "face_meta" not in G.level(1)   # coarse operators are not face-shaped


@pytest.mark.parametrize("name,N,kw", [("dg_q2_256_curved", 20, {}), ("dg_q2_256_curved", 14, dict(relax=1)),
                                       ("dg_q1_32", None, dict(cycle="F")),
                                       ("dg_q2_256_curved", 14, dict(precision="fp32")),
                                       ("dg_q2_256_curved", 14, dict(gmres=10)),
                                       ("dg_q4_512_jitter", 6, {})])
def test_faces_change_no_bit(name, N, kw):
    _say(f"test: faces on/off {name} N={N} {kw}")
    S, k = make_config(name, N=N)
    on, off = pair_on_off(S.rowptr, S.colidx, S.vals, S.bs, degree=k, **kw)
    r = same_solves(on, off, S.rhs)
    rT = same_solves(on, off, np.random.default_rng(31).uniform(-1, 1, S.n), trans=True)
    _say(f"  {r.iters} / {rT.iters} iterations, identical")


def test_faces_irregular_patterns_against_the_oracle():
    """Face blocks with entries zeroed at random (fewer rows or columns per
    block, holes inside the rectangle, some blocks all zero): the copy still
    holds exactly the nonzeros, solves match the oracle and the uncompressed
    path bit for bit."""
    _say("test: irregular face patterns")
    S = small_dg(10, 2, seed=5)
    va = S.vals.copy()
    rows = np.repeat(np.arange(S.nb), np.diff(S.rowptr))
    off = np.flatnonzero(rows != S.colidx)
    rng = np.random.default_rng(8)
    for t in off:
        u = rng.uniform()
        if u < 0.1:
            va[t] = 0.0                                  # an empty coupling block
        elif u < 0.6:
            nz = np.argwhere(va[t] != 0)
            drop = nz[rng.uniform(size=len(nz)) < 0.4]
            va[t][drop[:, 0], drop[:, 1]] = 0.0
    on, offh = pair_on_off(S.rowptr, S.colidx, va, S.bs, degree=2, max_coarse_dofs=40)
    check_face_copy(on, S.rowptr, S.colidx, va)
    same_solves(on, offh, S.rhs)
    same_solves(on, offh, np.random.default_rng(32).uniform(-1, 1, S.n), trans=True)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, va, degree=2, max_coarse_dofs=40)
    check_solve(G, O, S.rhs)
    check_solve(G, O, np.random.default_rng(33).uniform(-1, 1, S.n), trans=True)


def test_no_copy_where_blocks_are_not_face_shaped():
    _say("test: no face copy for dense coupling blocks or the scalar form")
    import paper_1704_05001_amd as P
    rp, ci, va, _, _ = layered_block_triangular(300, 3, 12, deps=3, seed=7, zero_entries=0.3)
    G = P.Hierarchy(*to_dev(rp, ci, va), 3, P.Params(degree=2, max_coarse_dofs=30))
    assert "face_meta" not in G.level(0)
    S, k = make_config("dg_q1_32")
    G = P.Hierarchy(*to_dev(S.rowptr, S.colidx, S.vals), S.bs, P.Params(degree=k, form="scalar"))
    assert "face_meta" not in G.level(0)


def test_faces_batched_and_full_size():
    _say("test: faces batched and full size")
    import paper_1704_05001_amd as P
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(6, 9, 7), nang=4)
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    d = to_dev(rp, ci, va)
    on = P.Hierarchy(*d, systems[0].bs, P.Params(degree=k), sys_nb=sys_nb)
    offh = P.Hierarchy(*d, systems[0].bs, P.Params(degree=k, faces=False), sys_nb=sys_nb)
    check_face_copy(on, rp, ci, va)
    bt = torch.from_numpy(rhs).cuda()
    for trans in (False, True):
        x1, r1 = on.solve_batch(bt, trans=trans)
        x2, r2 = offh.solve_batch(bt, trans=trans)
        assert [r.iters for r in r1] == [r.iters for r in r2]
        assert torch.equal(x1, x2)
    S, k = make_config("dg_q2_256_curved")
    on, offh = pair_on_off(S.rowptr, S.colidx, S.vals, S.bs, degree=k)
    r = same_solves(on, offh, S.rhs)
    _say(f"  full size: {r.iters} iterations, identical")
