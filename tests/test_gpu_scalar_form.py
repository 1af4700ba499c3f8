"""Scalar nAIR of the system scaled by its block-diagonal inverse (the paper's
default form) on the GPU against the oracle's form 1: the scaled scalar
matrix and every level bit-exact, solves and transposed solves to the
solve-phase bar, in FP64, FP32-stored, tuned and batched variants."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config, make_batch
from test_gpu_parity import build_pair, compare_hierarchies, check_solve, _say
from test_gpu_batch import build_batch, compare_batch, check_batch_solve
from test_gpu_fp32 import _fp32_vs_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,N,relax", [("dg_q1_32", None, 0), ("dg_q2_256_curved", 16, 0),
                                          ("dg_q2_256_curved", 12, 1), ("dg_q3_256_curved_sigma", 8, 0),
                                          ("dg_q4_512_jitter", 5, 0)])
def test_scalar_form_matches_oracle(name, N, relax):
    _say(f"test: scalar form {name} N={N} relax={relax}")
    S, k = make_config(name, N=N)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=dict(form="scalar"), degree=k,
                      relax=relax)
    assert G.level(0, fields=("rowptr",))["bs"] == 1
    compare_hierarchies(G, O)
    check_solve(G, O, S.rhs)
    g = np.random.default_rng(6).uniform(-1, 1, S.n)
    check_solve(G, O, g, trans=True)


def test_scalar_form_fp32_and_tuned():
    _say("test: scalar form, FP32-stored, tuned")
    S, k = make_config("dg_q2_256_curved", N=20)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=dict(form="scalar", precision="fp32"),
                      degree=k)
    compare_hierarchies(G, O)
    G.autotune(reps=3)
    _fp32_vs_oracle(G, O, S.rhs)
    g = np.random.default_rng(7).uniform(-1, 1, S.n)
    _fp32_vs_oracle(G, O, g, trans=True)


def test_scalar_form_batched():
    _say("test: scalar form, batch of angles")
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(4, 9, 7), nang=4)
    G, Os, rhs = build_batch(systems, gpu_kw=dict(form="scalar"), degree=k)
    compare_batch(G, Os)
    check_batch_solve(G, Os, systems, rhs)
    g = np.random.default_rng(8).uniform(-1, 1, rhs.size)
    check_batch_solve(G, Os, systems, g, trans=True)
