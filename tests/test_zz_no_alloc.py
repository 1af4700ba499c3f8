"""nair_solve_noalloc: the solve whose buffers live in the library's static
device scratch array, called through the C ABI and compared with nair_solve.

Both run the same kernels in the same order on the same hierarchy, so the
solutions must agree bit for bit and the iteration counts, statuses and
convergence figures exactly.  Each case makes two no-alloc calls in a row, the
second on a smaller system (the array keeps the first call's contents, so
everything the iteration reads must be set up again by the second), after a
call that stopped short of convergence.  A call must leave the device's free
memory unchanged.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config
from test_gpu_parity import to_dev, _need_gpu, _say

pytestmark = pytest.mark.gpu


def _hier(name, N, **kw):
    import paper_1704_05001_amd as P
    S, k = make_config(name, N=N)
    H = P.Hierarchy(*to_dev(S.rowptr, S.colidx, S.vals), S.bs, P.Params(degree=k, **kw))
    b = torch.from_numpy(np.ascontiguousarray(S.rhs, dtype=np.float64)).to("cuda:0")
    return H, b


def _bits(t):
    return t.detach().cpu().numpy().view(np.uint64)


def _same_result(r0, r1, what):
    assert (r0.status, r0.iters, r0.converged) == (r1.status, r1.iters, r1.converged), what
    for f in ("relres", "rho_avg", "rho_last5"):
        a, c = getattr(r0, f), getattr(r1, f)
        assert np.float64(a).view(np.uint64) == np.float64(c).view(np.uint64), f"{what}: {f} {a} vs {c}"


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


@pytest.mark.parametrize("kw", [dict(), dict(cycle="F"), dict(precision="fp32"), dict(form="scalar"),
                                dict(cycle="F", precision="fp32")],
                         ids=["V-fp64", "F-fp64", "V-fp32", "V-scalar", "F-fp32"])
def test_noalloc_matches_solve(kw):
    _need_gpu()
    _say(f"test: nair_solve_noalloc vs nair_solve {kw}")
    Hbig, bbig = _hier("dg_q2_256_curved", 32, **kw)
    Hsmall, bsmall = _hier("dg_q2_256_curved", 16, **kw)
    assert Hsmall.n < Hbig.n
    # the existing entry point
    xs_ref, rs_short = Hsmall.solve(bsmall, max_iter=2)
    xs_ref = xs_ref.clone()
    xb_ref, rb_ref = Hbig.solve(bbig)
    xb_ref = xb_ref.clone()
    x2_ref, r2_ref = Hsmall.solve(bsmall)
    x2_ref = x2_ref.clone()
    assert rb_ref.converged and r2_ref.converged and not rs_short.converged

    xs = torch.full_like(bsmall, float("nan"))
    xb = torch.full_like(bbig, float("nan"))
    x2 = torch.full_like(bsmall, float("nan"))
    free0 = _free()
    _, rs = Hsmall.solve_noalloc(bsmall, xs, max_iter=2)        # stops short: leaves state behind
    _, rb = Hbig.solve_noalloc(bbig, xb)
    _, r2 = Hsmall.solve_noalloc(bsmall, x2)                    # second call in a row, smaller system
    assert _free() == free0, "a no-alloc solve changed the device's free memory"

    _same_result(rs_short, rs, "short solve")
    _same_result(rb_ref, rb, "larger system")
    _same_result(r2_ref, r2, "smaller system after the larger")
    assert np.array_equal(_bits(xs), _bits(xs_ref))
    assert np.array_equal(_bits(xb), _bits(xb_ref))
    assert np.array_equal(_bits(x2), _bits(x2_ref))
    assert Hsmall.history().size == 0   # the no-alloc solve keeps no history


def test_noalloc_rejections():
    import paper_1704_05001_amd as P
    _need_gpu()
    _say("test: nair_solve_noalloc rejections")
    H, b = _hier("dg_q2_256_curved", 8)
    x = torch.zeros_like(b)
    cap = P.NOALLOC_SCRATCH_BYTES
    assert cap == 4 * 1024 * 1024
    too_many = cap // 8 + 1   # the residual history alone would overflow the array
    with pytest.raises(P.NairError) as e:
        H.solve_noalloc(b, x, max_iter=too_many)
    assert e.value.status == "EINVAL"
    assert "bytes of scratch" in str(e.value) and str(cap) in str(e.value)
    Hg, bg = _hier("dg_q2_256_curved", 8, gmres=10)
    with pytest.raises(P.NairError) as e:
        Hg.solve_noalloc(bg, torch.zeros_like(bg))
    assert e.value.status == "EINVAL" and "gmres" in str(e.value)
    # still usable, and equal to the allocating solve
    xr, rr = H.solve(b)
    xr = xr.clone()
    _, r = H.solve_noalloc(b, x)
    _same_result(rr, r, "after the rejections")
    assert np.array_equal(_bits(x), _bits(xr))
