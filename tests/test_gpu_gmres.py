"""GMRES(m) preconditioned by the nAIR cycle on the GPU against the oracle's
GMRES (the section "Non-triangular matrices" uses one nAIR V-cycle per
GMRES iteration).

The GPU orthogonalises with classical Gram-Schmidt applied twice, the oracle
with modified Gram-Schmidt; the two are equal in exact arithmetic, so the
bar is the solve-phase one on status, iteration count and residual-estimate
history, and on x it is the level rounding leaves below the stopping
tolerance: both iterates solve to rtol = 1e-10, and their difference is the
rounding of the Hessenberg entries carried through the small least-squares
solves, far below that, so 1e-10 max|x| is the bar."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config, make_batch
from test_gpu_parity import build_pair, small_dg, to_dev, _say, np_
from test_gpu_batch import build_batch

pytestmark = pytest.mark.gpu

X_BAR = 1e-10


def check_gmres(G, O, b, trans=False, rtol=1e-10, max_iter=200):
    bt = torch.from_numpy(b).cuda()
    if trans:
        xg, rg = G.solve_T(bt, rtol=rtol, max_iter=max_iter)
        xo, ho, so = O.solve_T(b, rtol, max_iter)
    else:
        xg, rg = G.solve(bt, rtol=rtol, max_iter=max_iter)
        xo, ho, so = O.solve(b, rtol, max_iter)
    hg = G.history()
    xg = np_(xg)
    err = float(np.abs(xg - xo).max() / max(np.abs(xo).max(), 1e-300))
    # deviation of the history as a fraction of its bar 1e-12 + 1e-6 h_oracle
    hdev = float(np.max(np.abs(hg - ho) / (1e-12 + 1e-6 * ho))) if len(ho) and len(hg) == len(ho) else -1.0
    _say(f"  {'A^T' if trans else 'A'}: {rg.iters} iterations (oracle {len(ho)}), status {rg.status}/{so}, "
         f"history deviation {hdev:.2f} of its bar, max |x - x_oracle| / max |x_oracle| = {err:.1e}")
    assert rg.status == so, (rg.status, so)
    assert len(hg) == len(ho) == rg.iters
    assert np.all(np.abs(hg - ho) <= 1e-12 + 1e-6 * ho)
    assert err <= X_BAR
    return rg, hg


@pytest.mark.parametrize("name,N,m,kw", [("dg_q2_256_curved", 16, 30, {}),
                                         ("dg_q2_256_curved", 16, 4, {}),            # restarts
                                         ("dg_q2_256_curved", 12, 20, dict(relax=1)),
                                         ("dg_q1_32", None, 10, dict(form="scalar")),
                                         ("dg_q2_256_curved", 10, 15, dict(cycle="F")),
                                         ("dg_q4_512_jitter", 5, 25, {})])
def test_gmres_matches_oracle(name, N, m, kw):
    _say(f"test: GMRES({m}) {name} N={N} {kw}")
    S, k = make_config(name, N=N)
    kw = dict(kw)
    gpu_kw = {key: kw.pop(key) for key in ("form", "cycle") if key in kw}
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=gpu_kw, degree=k, gmres=m, **kw)
    check_gmres(G, O, S.rhs)
    g = np.random.default_rng(21).uniform(-1, 1, S.n)
    check_gmres(G, O, g, trans=True)


def test_gmres_minimal_residual_against_the_stationary_iteration():
    """Without a restart, GMRES minimises ||b - A x|| over the space the
    stationary iteration's iterates lie in, so its residual is never larger."""
    _say("test: GMRES residual <= stationary residual")
    import paper_1704_05001_amd as P
    S, k = make_config("dg_q2_256_curved", N=24)
    d = to_dev(S.rowptr, S.colidx, S.vals)
    b = torch.from_numpy(S.rhs).cuda()
    Gs = P.Hierarchy(*d, S.bs, P.Params(degree=k))
    _, rs = Gs.solve(b, rtol=1e-10)
    hs = Gs.history()
    Gk = P.Hierarchy(*d, S.bs, P.Params(degree=k, gmres=60))
    _, rk = Gk.solve(b, rtol=1e-10)
    hk = Gk.history()
    _say(f"  stationary {rs.iters} iterations, GMRES(60) {rk.iters}")
    assert rs.status == rk.status == "OK"
    assert rk.iters <= rs.iters
    # (GMRES's history is its estimate, the true residual up to rounding)
    assert np.all(hk <= hs[:len(hk)] * (1 + 1e-6) + 1e-13)


def test_gmres_fp32_hierarchy():
    """An FP32-stored cycle is a slightly different preconditioner each
    application; GMRES keeps the preconditioned directions, so x = Z y stays
    consistent with the residual estimate and the FP64 solve reaches rtol."""
    _say("test: GMRES with the FP32-stored hierarchy")
    S, k = make_config("dg_q2_256_curved", N=20)
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gpu_kw=dict(precision="fp32"), degree=k, gmres=30)
    for trans, b in ((False, S.rhs), (True, np.random.default_rng(22).uniform(-1, 1, S.n))):
        bt = torch.from_numpy(b).cuda()
        x, r = (G.solve_T if trans else G.solve)(bt, rtol=1e-10)
        xo, ho, so = (O.solve_T if trans else O.solve)(b, 1e-10, 200)
        err = float(np.abs(np_(x) - xo).max() / np.abs(xo).max())
        _say(f"  {'A^T' if trans else 'A'}: {r.iters} iterations (oracle FP64 {len(ho)}), error {err:.1e}")
        assert r.status == "OK" and so == "OK"
        assert abs(r.iters - len(ho)) <= 2
        assert err <= 1e-8


def test_gmres_edge_cases():
    _say("test: GMRES edge cases")
    import paper_1704_05001_amd as P
    S = small_dg(6, 1)
    d = to_dev(S.rowptr, S.colidx, S.vals)
    O_kw = dict(max_coarse_dofs=8)
    # zero right-hand side: x = 0 at once
    G, O = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gmres=5, **O_kw)
    x, r = G.solve(torch.zeros(S.n, dtype=torch.float64, device="cuda"))
    assert r.status == "OK" and r.iters == 0 and float(x.abs().max()) == 0.0
    # GMRES(1): a restart after every step
    G1, O1 = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gmres=1, **O_kw)
    check_gmres(G1, O1, S.rhs)
    # rtol 0 never stops early: max_iter inside the first cycle, at its end,
    # and across restarts
    for Gm, Om, mi in ((G, O, 3), (G, O, 5), (G1, O1, 4)):
        rg, _ = check_gmres(Gm, Om, S.rhs, rtol=0.0, max_iter=mi)
        assert rg.status == "ENOCONV" and rg.iters == mi
    # a hierarchy that is one dense solve: GMRES is exact after one step
    Gd, Od = build_pair(S.nb, S.bs, S.rowptr, S.colidx, S.vals, gmres=10, max_coarse_dofs=4096)
    assert Gd.info()["levels"] == 1
    rg, hg = check_gmres(Gd, Od, S.rhs)
    assert rg.iters == 1
    # a non-finite right-hand side
    b = torch.from_numpy(S.rhs).cuda()
    b[3] = float("nan")
    _, r = G.solve(b)
    assert r.status == "ENUMERIC"
    # parameter validation, and batched handles refuse GMRES
    for m in (-1, 201):
        with pytest.raises(P.NairError) as e:
            P.Hierarchy(*d, S.bs, P.Params(gmres=m))
        assert e.value.status == "EINVAL"
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(4, 5), nang=2)
    Gb, _, rhs = build_batch(systems, gpu_kw=dict(gmres=5), degree=k)
    with pytest.raises(P.NairError) as e:
        Gb.solve_batch(torch.from_numpy(rhs).cuda())
    assert e.value.status == "EINVAL"


def test_gmres_full_size():
    """The 256x256 Q2 curved-velocity workload (589,824 DOFs): GMRES(30)
    against the stationary solve on the GPU, both to rtol 1e-10."""
    _say("test: GMRES(30) full size")
    import paper_1704_05001_amd as P
    S, k = make_config("dg_q2_256_curved")
    d = to_dev(S.rowptr, S.colidx, S.vals)
    b = torch.from_numpy(S.rhs).cuda()
    xs, rs = P.Hierarchy(*d, S.bs, P.Params(degree=k)).solve(b, rtol=1e-10)
    G = P.Hierarchy(*d, S.bs, P.Params(degree=k, gmres=30))
    xk, rk = G.solve(b, rtol=1e-10)
    yk, rt = G.solve_T(b, rtol=1e-10)
    _say(f"  stationary {rs.iters}, GMRES {rk.iters}, transposed GMRES {rt.iters}")
    assert rs.status == rk.status == rt.status == "OK"
    assert rk.iters <= rs.iters
    diff = float((xk - xs).abs().max() / xs.abs().max())
    assert diff <= 1e-8, diff
