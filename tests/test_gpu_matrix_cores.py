"""Setup block products on the FP64 matrix cores against the vector-unit kernels.

The setup's dense block products (the Neumann sparse products W_i = W_{i-1} T,
T = -D^-1 A_ff, Z = -S D^-1, and the Galerkin blocks of R A P) of 9x9, 16x16
and 25x25 blocks run on the matrix cores by default (nair_params.matrix_cores)
and on the vector units otherwise.  Both must give every entry as the fma chain
over the inner index in ascending order from +0 -- the oracle's order -- so the
two hierarchies are identical bit for bit (a zero may differ in sign: a padded
step adds fma(0, 0, -0) = +0) and equal to the oracle's.

The operands here are chosen to expose any other accumulation: with identity
diagonal blocks, D^-1 = I exactly and the products take the matrix's own entries
(T = -A_ff, W_1 = -A_cf A_ff, ...); those entries are drawn to produce exact
cancellations, subnormal and underflowing products, signed zeros and a wide
spread of exponents inside one dot product.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nair_inputs import make_config
from nair_inputs.random_blocks import layered_block_triangular

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(torch.device("cuda", 0))


def _hier(nb, bs, rp, ci, va, **kw):
    import paper_1704_05001_amd as P
    return P.Hierarchy(_dev(rp, np.int32), _dev(ci, np.int32), _dev(va, np.float64), bs, P.Params(**kw))


def _same(a, b, what):
    """Equal bit for bit, except that a zero may carry either sign."""
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    b = b.detach().cpu().numpy() if hasattr(b, "detach") else np.asarray(b)
    assert a.shape == b.shape, what
    if a.dtype != np.float64:
        assert np.array_equal(a, b), what
        return
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    ua, ub = a.view(np.uint64), b.view(np.uint64)
    diff = ua != ub
    if diff.any():
        bad = ~((a[diff] == 0) & (b[diff] == 0))
        if bad.any():
            ia = np.argwhere(diff)[bad][:5]
            ex = [(tuple(int(v) for v in i), float(a[tuple(i)]), float(b[tuple(i)])) for i in ia]
            raise AssertionError(f"{what}: {int(bad.sum())} of {a.size} entries differ, "
                                 f"max |diff| {float(np.abs(a - b).max()):.3e}; first: {ex}")


FIELDS = ("rowptr", "colidx", "vals", "dinv", "bnorm", "mask", "cf", "pmap", "z_rowptr", "z_colidx", "z_vals")


def _compare(Gm, Gv, O):
    lv = Gm.info()["levels"]
    assert lv == Gv.info()["levels"] == O.num_levels
    for l in range(lv):
        a, b, o = Gm.level(l), Gv.level(l), O.level(l)
        for f in FIELDS:
            if f in a or f in b:
                _same(a[f], b[f], f"level {l} {f}: matrix cores vs vector units")
        _same(a["vals"], o.vals, f"level {l} operator vs oracle")
        if not o.coarsest:
            _same(a["z_vals"], o.z_vals, f"level {l} Z vs oracle")
            _same(a["dinv"], o.dinv, f"level {l} D^-1 vs oracle")
            assert tuple(a["margin"]) == tuple(o.margin)


@pytest.mark.parametrize("name,N", [("dg_q2_256_curved", 20), ("dg_q3_256_curved_sigma", 10),
                                    ("dg_q4_512_jitter", 10)])
def test_dg_hierarchies_identical(name, N):
    _need_gpu()
    S, k = make_config(name, N=N)
    _say(f"test: matrix cores vs vector units, {name} N={N} (bs {S.bs})")
    Gm = _hier(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=k, matrix_cores=True)
    Gv = _hier(S.nb, S.bs, S.rowptr, S.colidx, S.vals, degree=k, matrix_cores=False)
    O = oracle.Hierarchy(S.nb, S.bs, S.rowptr, S.colidx, S.vals, oracle.Params(degree=k))
    _compare(Gm, Gv, O)


def _adversarial(bs, family, seed, nb=160):
    """Block-triangular pattern (hidden order) with identity diagonal blocks and
    off-diagonal entries of one adversarial family."""
    rp, ci, va, order, layer = layered_block_triangular(nb, bs, 8, deps=3, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    rows = np.repeat(np.arange(nb), np.diff(rp))
    va = va.copy()
    for t in range(len(ci)):
        if rows[t] == ci[t]:
            va[t] = np.eye(bs)
            continue
        if family == "cancel":
            # small integers and halves: many dot products cancel exactly to 0
            v = rng.integers(-2, 3, size=(bs, bs)) * 0.5
        elif family == "subnormal":
            # products around the smallest normal number (2^-1022): subnormal
            # partial sums, and products that underflow to a signed zero
            e = rng.integers(-545, -505, size=(bs, bs))
            v = np.ldexp(rng.choice([-1.0, 1.0], size=(bs, bs)) * rng.uniform(1, 2, size=(bs, bs)), e)
        elif family == "spread":
            # powers of two from 2^-60 to 2^60 with random signs and mantissas in one row
            e = rng.integers(-60, 61, size=(bs, bs))
            v = np.ldexp(rng.choice([-1.0, 1.0], size=(bs, bs)) * rng.uniform(1, 2, size=(bs, bs)), e)
        elif family == "zeros":
            # signed zeros and sparse entries
            v = rng.choice([0.0, -0.0, 1.0, -1.0, 0.25, -3.0], size=(bs, bs),
                           p=[0.35, 0.35, 0.1, 0.1, 0.05, 0.05])
        else:
            raise ValueError(family)
        va[t] = v
    return nb, bs, rp, ci, va


@pytest.mark.parametrize("bs", [9, 16, 25])
@pytest.mark.parametrize("family", ["cancel", "subnormal", "spread", "zeros"])
def test_adversarial_operands(bs, family):
    _need_gpu()
    nb, bs, rp, ci, va = _adversarial(bs, family, seed=11 * bs + len(family))
    _say(f"test: adversarial operands {family} bs {bs}")
    for degree in (1, 3):
        kw = dict(degree=degree, max_coarse_dofs=2 * bs, phi=0.0, drop=0.0)
        Gm = _hier(nb, bs, rp, ci, va, matrix_cores=True, **kw)
        Gv = _hier(nb, bs, rp, ci, va, matrix_cores=False, **kw)
        O = oracle.Hierarchy(nb, bs, rp, ci, va, oracle.Params(**kw))
        assert O.num_levels >= 2
        _compare(Gm, Gv, O)
