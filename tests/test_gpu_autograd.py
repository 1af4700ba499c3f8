"""Differentiable solve on the GPU: x = A^{-1} b as a torch autograd function.

The backward pass is the transposed-hierarchy solve A^T ybar = xbar plus the
pattern gradient -ybar_I x_J^T (a HIP kernel).  Checked against the oracle's
adjoint gradients (pinned by finite differences of dense solves), against
dense FP64 solves, by torch's gradcheck on a single-level system, and on the
sigma/q model of the Q3 workload (A(sigma) = A(0) + sigma_K M_K on diagonal
blocks, b = M q) by finite differences, up to the full 256 x 256 mesh.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nair_inputs import make_config, sigma_q_model
from nair_inputs.configs import CONFIGS
from nair_inputs.random_blocks import random_block_sparse
from test_gpu_parity import np_, _say

import paper_1704_05001_amd as P

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _model_torch(m, sigma, q):
    """vals(sigma) and b(q) as differentiable torch expressions."""
    S0 = m["system"]
    vals0 = _dev(S0.vals)
    mass = _dev(m["mass"])
    pos = _dev(m["diag_pos"].astype(np.int64))
    vals = vals0.index_add(0, pos, sigma[:, None, None] * mass)
    b = (mass * q.view(S0.nb, 1, S0.bs)).sum(-1).reshape(-1)
    return vals, b


@pytest.mark.parametrize("bs", [1, 3, 16])
def test_grad_vals_kernel_is_exact(bs):
    _say(f"test: grad_vals kernel bs={bs}")
    nb = 37
    rp, ci, va = random_block_sparse(nb, bs, 0.15, seed=bs)
    rng = np.random.default_rng(bs)
    y, x = rng.uniform(-1, 1, nb * bs), rng.uniform(-1, 1, nb * bs)
    g = np_(P.grad_vals(_dev(rp), _dev(ci), _dev(y), _dev(x), bs))
    ref = np.zeros_like(g)
    for I in range(nb):
        for t in range(rp[I], rp[I + 1]):
            ref[t] = -np.outer(y[I * bs:(I + 1) * bs], x[ci[t] * bs:(ci[t] + 1) * bs])
    assert np.array_equal(g, ref)


@pytest.mark.parametrize("name,N", [("dg_q3_256_curved_sigma", 8), ("dg_q2_256_curved", 12)])
def test_backward_matches_oracle_adjoint(name, N):
    _say(f"test: autograd vs oracle adjoint {name} N={N}")
    S, k = make_config(name, N=N)
    w = np.random.default_rng(7).uniform(-1, 1, S.n)
    O = oracle.Hierarchy(S.nb, S.bs, S.rowptr, S.colidx, S.vals, oracle.Params(degree=k))
    xo, yo, go = oracle.adjoint_gradients(O, S.rowptr, S.colidx, S.rhs, w, rtol=1e-12)
    vals = _dev(S.vals).requires_grad_(True)
    b = _dev(S.rhs).requires_grad_(True)
    x = P.solve(vals, b, _dev(S.rowptr), _dev(S.colidx), S.bs, P.Params(degree=k), rtol=1e-12)
    (x * _dev(w)).sum().backward()
    ex = np.abs(np_(x) - xo).max() / np.abs(xo).max()
    eb = np.abs(np_(b.grad) - yo).max() / np.abs(yo).max()
    ev = np.abs(np_(vals.grad) - go).max() / np.abs(go).max()
    _say(f"  rel. max diff: x {ex:.1e}, dL/db {eb:.1e}, dL/dvals {ev:.1e}")
    assert ex <= 1e-10 and eb <= 1e-10 and ev <= 1e-10
    # and against dense FP64 linear algebra
    D = S.to_dense()
    yd = np.linalg.solve(D.T, w)
    assert np.abs(np_(b.grad) - yd).max() <= 1e-10 * np.abs(yd).max()


def test_gradcheck_single_level():
    """A system below the coarsest-level size is solved directly; torch's
    gradcheck differentiates through forward and backward numerically."""
    _say("test: gradcheck single-level Q1 N=4")
    S, k = make_config("dg_q1_32", N=4)
    assert S.n <= P.Params().max_coarse_dofs
    rp, ci = _dev(S.rowptr), _dev(S.colidx)
    vals = _dev(S.vals).requires_grad_(True)
    b = _dev(S.rhs).requires_grad_(True)
    prm = P.Params(degree=k)
    fn = lambda v, r: P.solve(v, r, rp, ci, S.bs, prm, rtol=1e-13)
    assert torch.autograd.gradcheck(fn, (vals, b), eps=1e-6, atol=1e-6, rtol=1e-4)


def test_sigma_q_model_small_against_dense_fd():
    _say("test: sigma/q model Q3 N=8 against dense finite differences")
    flow = CONFIGS["dg_q3_256_curved_sigma"]["b"]
    m = sigma_q_model(8, 3, flow)
    S0 = m["system"]
    sigma = _dev(m["sigma"]).requires_grad_(True)
    q = _dev(m["q"]).requires_grad_(True)
    vals, b = _model_torch(m, sigma, q)
    x = P.solve(vals, b, _dev(S0.rowptr), _dev(S0.colidx), S0.bs, P.Params(degree=2), rtol=1e-12)
    xstar = _dev(m["xstar"])
    (0.5 * ((x - xstar) ** 2).sum()).backward()
    gs, gq = np_(sigma.grad), np_(q.grad)

    D0 = S0.to_dense()
    bs = S0.bs
    M = m["mass"]

    def loss(sig, qq):
        D = D0.copy()
        for K in range(S0.nb):
            D[K * bs:(K + 1) * bs, K * bs:(K + 1) * bs] += sig[K] * M[K]
        bb = np.einsum("kij,kj->ki", M, qq.reshape(S0.nb, bs)).reshape(-1)
        xx = np.linalg.solve(D, bb)
        return 0.5 * np.sum((xx - m["xstar"]) ** 2)

    rng = np.random.default_rng(3)
    h = 1e-5
    for K in rng.choice(S0.nb, 5, replace=False):
        e = np.zeros(S0.nb)
        e[K] = h
        fd = (loss(m["sigma"] + e, m["q"]) - loss(m["sigma"] - e, m["q"])) / (2 * h)
        assert abs(fd - gs[K]) <= 1e-6 * np.abs(gs).max(), (K, fd, gs[K])
    for i in rng.choice(S0.n, 5, replace=False):
        e = np.zeros(S0.n)
        e[i] = h
        fd = (loss(m["sigma"], m["q"] + e) - loss(m["sigma"], m["q"] - e)) / (2 * h)
        assert abs(fd - gq[i]) <= 1e-6 * np.abs(gq).max(), (i, fd, gq[i])


def test_sigma_q_model_full_size():
    """The Q3 256 x 256 workload (1,048,576 DOFs) forward and backward: both
    solves checked by FP64 residuals computed on the host, per-cell sigma
    gradients against -ybar_K^T M_K x_K, and a directional finite difference
    of the loss through two more GPU solves."""
    flow = CONFIGS["dg_q3_256_curved_sigma"]["b"]
    m = sigma_q_model(256, 3, flow)
    S0 = m["system"]
    _say(f"test: sigma/q model full size ({S0.n} DOFs)")
    bs = S0.bs
    rp, ci = _dev(S0.rowptr), _dev(S0.colidx)
    prm = P.Params(degree=2)
    sigma = _dev(m["sigma"]).requires_grad_(True)
    q = _dev(m["q"]).requires_grad_(True)
    vals, b = _model_torch(m, sigma, q)
    x = P.solve(vals, b, rp, ci, bs, prm, rtol=1e-11)
    xstar = _dev(m["xstar"])
    loss = 0.5 * ((x - xstar) ** 2).sum()
    loss.backward()
    gs = np_(sigma.grad)

    # host FP64 residuals of the forward and adjoint systems
    V = np_(vals.detach())
    xn, bn = np_(x.detach()), np_(b.detach())
    rows = np.repeat(np.arange(S0.nb), np.diff(S0.rowptr))
    Ax = np.zeros((S0.nb, bs))
    np.add.at(Ax, rows, np.einsum("tij,tj->ti", V, xn.reshape(S0.nb, bs)[S0.colidx]))
    rel = np.linalg.norm(Ax.reshape(-1) - bn) / np.linalg.norm(bn)
    # ybar from dL/dq = M^T ybar per cell
    gq = np_(q.grad).reshape(S0.nb, bs)
    ybar = np.linalg.solve(np.transpose(m["mass"], (0, 2, 1)), gq[:, :, None])[:, :, 0]
    ATy = np.zeros((S0.nb, bs))
    np.add.at(ATy, S0.colidx, np.einsum("tji,tj->ti", V, ybar[rows]))
    xbar = xn - m["xstar"]
    relT = np.linalg.norm(ATy.reshape(-1) - xbar) / np.linalg.norm(xbar)
    _say(f"  forward rel. residual {rel:.1e}, adjoint rel. residual {relT:.1e}")
    assert rel <= 1e-10 and relT <= 1e-9

    rng = np.random.default_rng(11)
    X = xn.reshape(S0.nb, bs)
    for K in rng.choice(S0.nb, 8, replace=False):
        ref = -ybar[K] @ m["mass"][K] @ X[K]
        assert abs(ref - gs[K]) <= 1e-8 * np.abs(gs).max(), (K, ref, gs[K])

    # directional derivative along a random sigma direction
    d = rng.uniform(-1, 1, S0.nb)
    h = 1e-3

    def loss_at(sig):
        with torch.no_grad():
            v, bb = _model_torch(m, _dev(sig), q.detach())
            H = P.Hierarchy(rp, ci, v, bs, prm)
            xx, r = H.solve(bb, rtol=1e-12)
            H.close()
            assert r.status == "OK"
            return float(0.5 * ((xx - xstar) ** 2).sum())

    fd = (loss_at(m["sigma"] + h * d) - loss_at(m["sigma"] - h * d)) / (2 * h)
    an = float(gs @ d)
    _say(f"  directional derivative: autograd {an:.10e}, central difference {fd:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
