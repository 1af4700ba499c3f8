"""Sparse products with long rows: the per-workgroup symbolic path and its limits.

A block row of a sparse product whose candidate products (the summed lengths
of the right operand's rows it touches) exceed 1,024 leaves the per-wave LDS
hash for one workgroup with a larger table (k_symbolic_large) and has its pair
list built by k_pairs_large.  The matrices here make the coarse operator's
product R (A P) (R = [Z I]) produce such a row: a "collector" C block depends
on many F blocks, each of which depends on the same few C blocks, so the
collector's row touches thousands of candidate products that merge into a
few blocks.  The
hierarchy must equal the oracle's bit for bit (patterns, pair order, values).

Past 4,096 candidate products a row is refused (NAIR_ENOMEM, with the count in
the message), and so is an operator row of more than 1,024 blocks (the merge
of A's columns into A P).
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
    # the collector's row of R (A P): its own A P row (nsrc + 1 coarse columns) plus, per F
    # block of Z, that block's A P row (its nsrc sources)
    candidates = (nsrc + 1) + nf * nsrc
    assert 1024 < candidates <= 4096
    _say(f"test: long sparse-product row (bs {bs}, {candidates} candidate products)")
    G, O = build_pair(nb, bs, rp, ci, va, degree=1, cf_override=cf, max_coarse_dofs=8 * bs, drop=0.0)
    compare_hierarchies(G, O)
    assert O.level(0).z_rowptr[1] == nf   # the collector's Z row holds every F block
    b = np.random.default_rng(1).uniform(-1, 1, nb * bs)
    check_solve(G, O, b)


def test_row_past_the_product_limit_is_refused():
    """The collector's row of R (A P): nf F blocks of Z, each meeting an A P row
    with its nsrc source columns, so about nf * nsrc candidates."""
    import re
    import paper_1704_05001_amd as P
    _need_gpu()
    nf, nsrc = 1000, 5
    nb, rp, ci, va, cf = arrow(nf, nsrc, 2)
    assert nf * nsrc > 4096
    _say(f"test: sparse-product row past the limit (about {nf * nsrc} candidates)")
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(*to_dev(rp, ci, va), 2, P.Params(degree=1, cf_override=cf, max_coarse_dofs=16))
    assert e.value.status == "ENOMEM"
    m = re.search(r"sparse product row has (\d+) candidate blocks \(limit 4096\)", str(e.value))
    assert m and int(m.group(1)) > 4096
    # the library stays usable
    nb, rp, ci, va, cf = arrow(50, 2, 2)
    G, O = build_pair(nb, 2, rp, ci, va, degree=1, cf_override=cf, max_coarse_dofs=16)
    compare_hierarchies(G, O)


def test_operator_row_past_its_limit_is_refused():
    """A P merges an operator row in one wave's LDS hash: a row of more than
    1,024 blocks is refused (NAIR_ENOMEM, with the count in the message)."""
    import paper_1704_05001_amd as P
    _need_gpu()
    n = 1200
    nb = n + 1
    # block 0 depends on blocks 1..n (a long row); the others on nothing
    rows = [list(range(0, n + 1))] + [[J] for J in range(1, n + 1)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate([np.array(r) for r in rows]).astype(np.int32)
    rng = np.random.default_rng(5)
    va = rng.uniform(-1, 1, size=(len(ci), 2, 2)) / n
    rowid = np.repeat(np.arange(nb), np.diff(rp))
    va[rowid == ci] += 2.0 * np.eye(2)
    cf = np.ones(nb, dtype=np.int8)
    cf[0] = 0                       # the long row is an F row; its row of A keeps all 1 + n blocks
    _say("test: operator row past 1024 blocks")
    with pytest.raises(P.NairError) as e:
        P.Hierarchy(*to_dev(rp, ci, va), 2, P.Params(degree=1, cf_override=cf, max_coarse_dofs=16))
    assert e.value.status == "ENOMEM"
    assert f"operator row has {1 + n} blocks (limit 1024)" in str(e.value)
