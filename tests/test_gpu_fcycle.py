"""F-cycles on the GPU against the oracle's F-cycles (cycle 1): the hierarchy
is the V-cycle's; solves and transposed solves to the solve-phase bar, with
F and FC relaxation, in FP32-stored, scalar-form and batched variants, and
the cycle complexity equal to the oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config, make_batch
from test_gpu_parity import build_pair, compare_hierarchies, check_solve, _say
from test_gpu_batch import build_batch, compare_batch, check_batch_solve
from test_gpu_fp32 import _fp32_vs_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,N,relax,form", [("dg_q2_256_curved", 16, 0, "block"),
                                               ("dg_q2_256_curved", 12, 1, "block"),
                                               ("dg_q1_32", None, 0, "scalar"),
                                               ("dg_q4_512_jitter", 5, 0, "block")])
def test_fcycle_matches_oracle(name, N, relax, form):
    _say(f"test: F-cycle {name} N={N} relax={relax} form={form}")
    S, k = make_config(name, N=N)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=dict(cycle="F", form=form), degree=k,
                      relax=relax)
    compare_hierarchies(G, O)
    check_solve(G, O, S.rhs)
    g = np.random.default_rng(9).uniform(-1, 1, S.n)
    check_solve(G, O, g, trans=True)
    oc, cc = O.complexity()
    info = G.info()
    assert abs(info["oc"] - oc) <= 1e-12 * oc and abs(info["cc"] - cc) <= 1e-12 * cc


def test_fcycle_fp32_and_batched():
    _say("test: F-cycle FP32-stored and batched")
    S, k = make_config("dg_q2_256_curved", N=14)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=dict(cycle="F", precision="fp32"), degree=k)
    _fp32_vs_oracle(G, O, S.rhs)
    _fp32_vs_oracle(G, O, np.random.default_rng(10).uniform(-1, 1, S.n), trans=True)
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(5, 10, 7), nang=4)
    G, Os, rhs = build_batch(systems, gpu_kw=dict(cycle="F"), degree=k)
    compare_batch(G, Os)
    check_batch_solve(G, Os, systems, rhs)
    check_batch_solve(G, Os, systems, np.random.default_rng(11).uniform(-1, 1, rhs.size), trans=True)
    check_batch_solve(G, Os, systems, rhs, graph=False)
