"""FP32-stored hierarchy inside FP64 iterative refinement, against the FP64 oracle.

The setup (and every decision in it) is FP64 in both modes, so the hierarchy
must equal the oracle's exactly.  The cycle reads FP32 operators and vectors,
so iterates differ from the FP64 oracle's; what is fixed is that the FP64
outer iteration still reaches the requested relative residual, in about the
same number of iterations, and that the converged solution differs from the
oracle's by no more than the two residuals allow.  Each case reports its
error against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config
from test_gpu_parity import build_pair, compare_hierarchies, np_, _say

pytestmark = pytest.mark.gpu


def _fp32_vs_oracle(G, O, b, trans=False, rtol=1e-10):
    bt = torch.from_numpy(b).cuda()
    if trans:
        x, r = G.solve_T(bt, rtol=rtol)
        xo, ho, so = O.solve_T(b, rtol, 200)
    else:
        x, r = G.solve(bt, rtol=rtol)
        xo, ho, so = O.solve(b, rtol, 200)
    h = G.history()
    assert r.status == "OK" and so == "OK"
    assert r.relres <= rtol
    assert abs(r.iters - len(ho)) <= 2, (r.iters, len(ho))
    m = min(len(h), len(ho))
    # compare histories where the FP64 residual is above what an FP32 correction resolves
    sel = ho[:m] >= 1e-5
    hdev = float(np.max(np.abs(h[:m] - ho[:m])[sel] / ho[:m][sel])) if sel.any() else 0.0
    err = float(np.abs(np_(x) - xo).max() / np.abs(xo).max())
    _say(f"  fp32 hierarchy: {r.iters} iterations (oracle {len(ho)}), max |x - x_oracle| / max |x_oracle| = "
         f"{err:.2e}, max relative history deviation {hdev:.1e}")
    # the FP32 cycle perturbs each correction at single-precision level; above
    # that level the residual histories of the two iterations stay within 1e-3
    assert hdev <= 1e-3
    assert err <= 1e-8
    return err


@pytest.mark.parametrize("name,N", [("dg_q1_32", None), ("dg_q2_256_curved", 32), ("dg_q4_512_jitter", 8)])
def test_fp32_hierarchy_against_fp64_oracle(name, N):
    _say(f"test: fp32 hierarchy {name} N={N}")
    S, k = make_config(name, N=N)
    for relax in (0, 1):
        G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=dict(precision="fp32"), degree=k,
                          relax=relax)
        compare_hierarchies(G, O)
        _fp32_vs_oracle(G, O, S.rhs)
        g = np.random.default_rng(4).uniform(-1, 1, S.n)
        _fp32_vs_oracle(G, O, g, trans=True)


def test_fp32_hierarchy_full_bench_workload():
    _say("test: fp32 hierarchy, full dg_q2_256_curved")
    S, k = make_config("dg_q2_256_curved")
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=dict(precision="fp32"), degree=k)
    _fp32_vs_oracle(G, O, S.rhs)
