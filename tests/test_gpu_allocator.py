"""Device memory from the caller (nair_params.allocator): every buffer of a
handle comes from the caller's allocator and goes back to it, and the results
equal those of the library's own pool bit for bit."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nair_inputs import make_config, make_batch, concat_systems
from test_gpu_parity import to_dev, _need_gpu, _say

pytestmark = pytest.mark.gpu


def _solves(H, b, g):
    x, r = H.solve(b)
    x = x.clone()
    y, rT = H.solve_T(g)
    return x, r, y.clone(), rT


def test_torch_allocator_matches_the_pool():
    import paper_1704_05001_amd as P
    _need_gpu()
    _say("test: torch caching allocator vs the library's pool")
    S, k = make_config("dg_q2_256_curved", N=24)
    d = to_dev(S.rowptr, S.colidx, S.vals)
    b = torch.from_numpy(S.rhs).cuda()
    g = torch.from_numpy(np.random.default_rng(7).uniform(-1, 1, S.n)).cuda()
    Hp = P.Hierarchy(*d, S.bs, P.Params(degree=k))
    ref = _solves(Hp, b, g)
    Hp.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    Ht = P.Hierarchy(*d, S.bs, P.Params(degree=k, allocator="torch"))
    after_setup = torch.cuda.memory_allocated()
    assert after_setup > before   # the hierarchy lives in torch's allocator
    got = _solves(Ht, b, g)
    assert torch.cuda.memory_allocated() >= after_setup   # (the transposes, built by solve_T, too)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[2], got[2])
    assert (ref[1].iters, ref[3].iters) == (got[1].iters, got[3].iters)
    del got   # (the test's own copies of the solutions)
    Ht.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before   # every block went back


def test_torch_allocator_batched():
    import paper_1704_05001_amd as P
    _need_gpu()
    _say("test: torch caching allocator, batched hierarchy")
    systems, k = make_batch("dg_q2_angles64_uneven", sizes=(6, 9, 7), nang=4)
    rp, ci, va, rhs, sys_nb = concat_systems(systems)
    d = to_dev(rp, ci, va)
    bt = torch.from_numpy(rhs).cuda()
    out = []
    for alloc in ("pool", "torch"):
        H = P.Hierarchy(*d, systems[0].bs, P.Params(degree=k, allocator=alloc), sys_nb=sys_nb)
        x, res = H.solve_batch(bt)
        out.append((x.clone(), [r.iters for r in res]))
        H.close()
    assert torch.equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_failing_allocator_is_reported_and_nothing_leaks():
    import paper_1704_05001_amd as P
    from paper_1704_05001_amd import nair as N
    _need_gpu()
    _say("test: an allocator that runs out during the setup")
    S, k = make_config("dg_q2_256_curved", N=12)
    d = to_dev(S.rowptr, S.colidx, S.vals)
    live = {}
    calls = {"alloc": 0}

    def alloc(nbytes, stream, ctx):
        calls["alloc"] += 1
        if calls["alloc"] > 40:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0))
        live[p] = nbytes
        return p

    def free(ptr, stream, ctx):
        live.pop(int(ptr))
        torch.cuda.caching_allocator_delete(int(ptr))

    keep = (N._ALLOC_FN(alloc), N._FREE_FN(free))
    a = N._Allocator()
    a.alloc, a.free, a.ctx = keep[0], keep[1], None
    p = N._Params()
    N.lib().nair_default_params(C.byref(p))
    p.degree = k
    p.allocator = C.addressof(a)
    h = C.c_void_p()
    st = N.lib().nair_setup(S.nb, S.bs, C.c_void_p(d[0].data_ptr()), C.c_void_p(d[1].data_ptr()),
                            C.c_void_p(d[2].data_ptr()), C.byref(p), None, C.byref(h))
    assert N.STATUS[st] == "ENOMEM"
    assert b"allocator returned no memory" in N.lib().nair_last_error(None)
    assert calls["alloc"] > 40 and not live   # what it had handed out came back
    # the library is still usable with its own pool
    H = P.Hierarchy(*d, S.bs, P.Params(degree=k))
    H.close()
