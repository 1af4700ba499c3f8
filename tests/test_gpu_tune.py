"""The lane-group autotuner changes launch shapes only: a tuned hierarchy (and
one built with a transferred tuning table) must still match the oracle's
iteration to the solve-phase bar."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nair_inputs import make_config, make_batch
from test_gpu_parity import build_pair, check_solve, compare_hierarchies, to_dev, _say
from test_gpu_batch import build_batch, check_batch_solve

import paper_1704_05001_amd as P

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,N,prec", [("dg_q2_256_curved", 24, "fp64"), ("dg_q4_512_jitter", 6, "fp64"),
                                         ("dg_q1_32", None, "fp64")])
def test_tuned_cycle_matches_oracle(name, N, prec):
    _say(f"test: autotune {name} N={N}")
    S, k = make_config(name, N=N)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=k)
    table = G.autotune(reps=3)
    assert table.shape == (G.num_levels, len(P.TUNE_KINDS))
    assert np.all((table == 0) | ((table > 0) & ((table & (table - 1)) == 0)))
    _say(f"  tuning table (levels x kinds):\n{table}")
    check_solve(G, O, S.rhs)
    g = np.random.default_rng(5).uniform(-1, 1, S.n)
    check_solve(G, O, g, trans=True)
    # the table carried over to a new hierarchy of the same matrix
    d_rp, d_ci, d_va = to_dev(S.rowptr, S.colidx, S.vals)
    G2 = P.Hierarchy(d_rp, d_ci, d_va, S.bs, P.Params(degree=k, tuning=table))
    compare_hierarchies(G2, O)
    check_solve(G2, O, S.rhs)


def test_tuned_batch_and_fp32():
    _say("test: autotune on a batch, FP32-stored")
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(6, 12, 9), nang=4)
    G, Os, rhs = build_batch(systems, gpu_kw=dict(precision="fp32"), degree=k)
    G.autotune(reps=3)
    check_batch_solve(G, Os, systems, rhs, fp32=True)
    check_batch_solve(G, Os, systems, rhs, trans=True, fp32=True)


def test_autotune_rejects_bad_reps():
    S, k = make_config("dg_q1_32", N=6)
    d_rp, d_ci, d_va = to_dev(S.rowptr, S.colidx, S.vals)
    G = P.Hierarchy(d_rp, d_ci, d_va, S.bs, P.Params(degree=k))
    with pytest.raises(P.NairError):
        G.autotune(reps=0)


def test_tuned_full_size_outer_residual():
    """Full-size Q2 256 x 256 system: every lane-group candidate of the outer
    residual (up to one block row per workgroup) writes its per-workgroup
    partial sums inside the buffer, and the tuned solve still converges like
    the untuned one."""
    _say("test: autotune full-size dg_q2_256_curved")
    S, k = make_config("dg_q2_256_curved")
    d_rp, d_ci, d_va = to_dev(S.rowptr, S.colidx, S.vals)
    b = torch.from_numpy(S.rhs).cuda()
    G0 = P.Hierarchy(d_rp, d_ci, d_va, S.bs, P.Params(degree=k))
    x0, r0 = G0.solve(b)
    table = G0.autotune(reps=3)
    x1, r1 = G0.solve(b)
    assert r0.status == r1.status == "OK" and abs(r0.iters - r1.iters) <= 1
    assert float((x1 - x0).abs().max() / x0.abs().max()) <= 1e-9
    G1 = P.Hierarchy(d_rp, d_ci, d_va, S.bs, P.Params(degree=k, tuning=table))
    x2, r2 = G1.solve(b)
    assert r2.iters == r1.iters and torch.equal(x2, x1)
