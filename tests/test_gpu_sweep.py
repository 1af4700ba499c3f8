"""Sweep copies (nair_params.sweep_copy): the F rows of each selected level
operator, in F-list order without their diagonal blocks, with D_F^{-1} in the
same order, read by the Jacobi F sweeps, and with them the row-compressed
copies of Z (restriction) and of the coarse levels' sweep blocks, whose row
masks come from the matrix-core kernels at 9x9 and 16x16 blocks and from a
pass over the blocks at 4x4 and 25x25.  The copy holds exactly the F rows'
off-diagonal blocks; with one lane group per row the solves are bit-identical
with and without copies (forward, transposed, FC, FP32-stored, batched, face
rectangles on level 0); with the default launch shapes they match the oracle
to the parity tolerances; the default rule selects the levels with at least
32768 lanes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config, make_batch, concat_systems
from test_gpu_parity import build_pair, to_dev, _say, np_, check_solve

pytestmark = pytest.mark.gpu

RELAX, RELAX_T = 0, 1


def one_group_table(levels=64):
    t = np.zeros((levels, 6), dtype=np.int8)
    t[:, RELAX] = 1
    t[:, RELAX_T] = 1
    return t


def off_diagonal_F_blocks(lv):
    rp = np_(lv["rowptr"]).astype(np.int64)
    ci = np_(lv["colidx"])
    cf = np_(lv["cf"])
    rows = np.repeat(np.arange(lv["nb"]), np.diff(rp))
    return int(((cf[rows] == 0) & (ci != rows)).sum())


def pair(rp, ci, va, bs, sys_nb=None, **kw):
    import paper_1704_05001_amd as P
    d = to_dev(rp, ci, va)
    on = P.Hierarchy(*d, bs, P.Params(sweep_copy="all", **kw), sys_nb=sys_nb)
    off = P.Hierarchy(*d, bs, P.Params(sweep_copy="off", **kw), sys_nb=sys_nb)
    return on, off


def same_solves(on, off, b, trans=False):
    bt = torch.from_numpy(b).cuda()
    f = (lambda H: H.solve_T) if trans else (lambda H: H.solve)
    x1, r1 = f(on)(bt, rtol=1e-10)
    h1 = on.history()
    x2, r2 = f(off)(bt, rtol=1e-10)
    h2 = off.history()
    assert r1.status == r2.status and r1.iters == r2.iters
    assert np.array_equal(h1, h2), "histories differ"
    assert torch.equal(x1, x2), "iterates differ"
    return r1


@pytest.mark.parametrize("name,N,kw", [("dg_q2_256_curved", 20, {}), ("dg_q2_256_curved", 14, dict(relax=1)),
                                       ("dg_q2_256_curved", 14, dict(precision="fp32")),
                                       ("dg_q2_256_curved", 14, dict(faces=False)),
                                       ("dg_q1_32", None, dict(cycle="F")),
                                       ("dg_q2_256_curved", 12, dict(gmres=8)),
                                       ("dg_q3_256_curved_sigma", 10, {}),
                                       ("dg_q3_256_curved_sigma", 8, dict(precision="fp32")),
                                       ("dg_q4_512_jitter", 6, {})])
def test_sweep_copy_changes_no_bit_at_one_group(name, N, kw):
    _say(f"test: sweep copy on/off {name} N={N} {kw}")
    S, k = make_config(name, N=N)
    on, off = pair(S.rowptr, S.colidx, S.vals, S.bs, degree=k, tuning=one_group_table(), **kw)
    for l in range(on.num_levels):
        lv = on.level(l, fields=("rowptr", "colidx", "cf"))
        if lv["coarsest"]:
            assert lv["sweep_nnzb"] == -1
            break
        assert lv["sweep_nnzb"] == off_diagonal_F_blocks(lv), l
        assert off.level(l, fields=())["sweep_nnzb"] == -1
    r = same_solves(on, off, S.rhs)
    rT = same_solves(on, off, np.random.default_rng(41).uniform(-1, 1, S.n), trans=True)
    _say(f"  {r.iters} / {rT.iters} iterations, identical")


def test_sweep_copy_batched_changes_no_bit():
    _say("test: sweep copy on/off, batch")
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(6, 9, 7), nang=4)
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    on, off = pair(rp, ci, va, systems[0].bs, sys_nb=sys_nb, degree=k, tuning=one_group_table())
    bt = torch.from_numpy(rhs).cuda()
    for trans in (False, True):
        x1, r1 = on.solve_batch(bt, trans=trans)
        x2, r2 = off.solve_batch(bt, trans=trans)
        assert [r.iters for r in r1] == [r.iters for r in r2]
        assert torch.equal(x1, x2)


def test_sweep_copy_default_rule_and_oracle():
    """64 x 64 Q2 cells: level 0 has 4096 rows x 9 = 36,864 lanes and gets a
    copy (face rectangles) by default, the smaller levels do not; the tuned
    and default launch shapes both match the oracle."""
    _say("test: sweep copy default rule, oracle parity")
    S, k = make_config("dg_q2_256_curved", N=64)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=k)
    lv0 = G.level(0, fields=("rowptr", "colidx", "cf"))
    assert lv0["face_rmax"] > 0
    assert lv0["sweep_nnzb"] == off_diagonal_F_blocks(lv0)
    for l in range(1, G.num_levels):
        lv = G.level(l, fields=())
        assert (lv["sweep_nnzb"] >= 0) == (not lv["coarsest"] and lv["nb"] * lv["bs"] >= 32768), l
    check_solve(G, O, S.rhs)
    check_solve(G, O, np.random.default_rng(43).uniform(-1, 1, S.n), trans=True)
    G.autotune(reps=2)
    check_solve(G, O, S.rhs)
