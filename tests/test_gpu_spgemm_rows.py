"""Sparse products with long rows: the per-workgroup symbolic path and its limits.

A block row of a sparse product whose candidate products (the summed lengths
of the right operand's rows it touches) exceed 1,024 leaves the per-wave LDS
hash for one workgroup with a larger table (k_symbolic_large) and has its pair
list built by k_pairs_large.  The matrices here make R A (R = [Z I]) produce
such a row: a "collector" C block depends on many F blocks, each of which
depends on the same few C blocks, so the collector's row of R A touches
thousands of candidate products that merge into a few hundred blocks.  The
hierarchy must equal the oracle's bit for bit (patterns, pair order, values).

Past 4,096 candidate products a row is refused (NAIR_ENOMEM, with the count in
the message), and so is a Galerkin row of R A with more than 1,024 blocks.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from test_gpu_parity import build_pair, compare_hierarchies, check_solve, to_dev, _need_gpu, _say

pytestmark = pytest.mark.gpu


def arrow(nf: int, nsrc: int, bs: int, seed: int = 0):
    """Block 0 (C) depends on F blocks 1..nf; every F block depends on the C
    blocks nf+1 .. nf+nsrc, which depend on nothing.  Block lower triangular in
    the order sources, F blocks, collector.  Returns (nb, rp, ci, va, cf)."""
    rng = np.random.default_rng(seed)
    nb = 1 + nf + nsrc
    src = list(range(nf + 1, nf + 1 + nsrc))
    rows = [[0] + list(range(1, nf + 1))]
    rows += [sorted([K] + src) for K in range(1, nf + 1)]
    rows += [[J] for J in src]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate([np.array(r) for r in rows]).astype(np.int32)
    va = rng.uniform(-1, 1, size=(len(ci), bs, bs)) / (nsrc + 1)
    rowid = np.repeat(np.arange(nb), np.diff(rp))
    d = rowid == ci
    va[d] += 2.0 * np.eye(bs)
    va[0] /= nf            # the collector's couplings: small enough for a stable coarse operator
    cf = np.zeros(nb, dtype=np.int8)
    cf[0] = 1
    cf[nf + 1:] = 1
    return nb, rp, ci, va, cf


@pytest.mark.parametrize("bs", [2, 9, 25])
def test_long_rows_match_the_oracle(bs):
    _need_gpu()
    nf, nsrc = 400, 5
    nb, rp, ci, va, cf = arrow(nf, nsrc, bs, seed=bs)
    # the collector's R A row: its own row (1 + nf blocks) plus, per F block, its row (1 + nsrc)
    candidates = (1 + nf) + nf * (1 + nsrc)
    assert 1024 < candidates <= 4096
    _say(f"test: long sparse-product row (bs {bs}, {candidates} candidate products)")
    G, O = build_pair(nb, bs, rp, ci, va, degree=1, cf_override=cf, max_coarse_dofs=8 * bs, drop=0.0)
    compare_hierarchies(G, O)
    assert O.level(0).z_rowptr[1] == nf   # the collector's Z row holds every F block
    b = np.random.default_rng(1).uniform(-1, 1, nb * bs)
    check_solve(G, O, b)


def test_row_past_the_product_limit_is_refused():
    import paper_1704_05001_amd as P
    _need_gpu()
    nf, nsrc = 800, 5
    nb, rp, ci, va, cf = arrow(nf, nsrc, 2)
    candidates = (1 + nf) + nf * (1 + nsrc)
    assert candidates > 4096
    _say(f"test: sparse-product row past the limit ({candidates} candidates)")
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(*to_dev(rp, ci, va), 2, P.Params(degree=1, cf_override=cf, max_coarse_dofs=16))
    assert e.value.status == "ENOMEM"
    assert f"{candidates} candidate blocks (limit 4096)" in str(e.value)
    # the library stays usable
    nb, rp, ci, va, cf = arrow(50, 2, 2)
    G, O = build_pair(nb, 2, rp, ci, va, degree=1, cf_override=cf, max_coarse_dofs=16)
    compare_hierarchies(G, O)


def test_galerkin_row_past_its_limit_is_refused():
    import paper_1704_05001_amd as P
    _need_gpu()
    nf, nsrc = 1100, 1
    nb, rp, ci, va, cf = arrow(nf, nsrc, 2)
    assert (1 + nf) + nf * (1 + nsrc) <= 4096   # the product itself fits; R A's row has 1 + nf + nsrc blocks
    _say("test: Galerkin row past 1024 blocks")
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(*to_dev(rp, ci, va), 2, P.Params(degree=1, cf_override=cf, max_coarse_dofs=16))
    assert e.value.status == "ENOMEM"
    assert f"Galerkin row has {1 + nf + nsrc} blocks (limit 1024)" in str(e.value)
