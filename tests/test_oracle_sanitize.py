"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

gcc compiles the oracle's source together with a small driver
(`oracle_sanitize_main.c`) with -fsanitize=address,undefined and no recovery,
so any out-of-bounds access, use after free, leak or undefined operation in
setup, level views, complexities, both cycles and both solves ends the run
with a report.  The sanitized build must also give the same bits as the
oracle library the other tests load (same source, same -ffp-contract=off).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import Hierarchy, Params
from nair_inputs import dg_quad
from nair_inputs.random_blocks import random_block_sparse

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")

# degree, relax, cycle, gmres, form
VARIANTS = [(1, 0, 0, 0, 0), (2, 1, 0, 0, 0), (1, 0, 1, 0, 0), (1, 0, 0, 5, 0), (1, 1, 0, 0, 1), (3, 0, 1, 0, 1)]


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("asan")
    exe = str(d / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", ORACLE, os.path.join(HERE, "oracle_sanitize_main.c"), os.path.join(ORACLE, "nair_oracle.c"),
           "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


def _write(path, nb, bs, rp, ci, va, rhs):
    with open(path, "wb") as f:
        np.array([nb, bs, int(rp[-1]), len(VARIANTS)], dtype=np.int32).tofile(f)
        np.ascontiguousarray(rp, dtype=np.int32).tofile(f)
        np.ascontiguousarray(ci, dtype=np.int32).tofile(f)
        np.ascontiguousarray(va, dtype=np.float64).tofile(f)
        np.ascontiguousarray(rhs, dtype=np.float64).tofile(f)
        np.array(VARIANTS, dtype=np.int32).tofile(f)


def _systems():
    S1 = dg_quad(7, 1, (math.cos(0.4), math.sin(0.4)), seed_perm=3)
    S2 = dg_quad(5, 2, lambda x, y: (y + 0.25, -(x + 0.25)), sigma=0.5, seed_perm=5)
    rp, ci, va = random_block_sparse(40, 3, 0.08, seed=11)
    rhs = np.random.default_rng(11).uniform(-1, 1, 120)
    return [("dg_q1", S1.nb, S1.bs, S1.rowptr, S1.colidx, S1.vals, S1.rhs),
            ("dg_q2", S2.nb, S2.bs, S2.rowptr, S2.colidx, S2.vals, S2.rhs),
            ("random", 40, 3, rp, ci, va, rhs)]


@pytest.mark.parametrize("case", range(3))
def test_oracle_under_sanitizers_matches_library(sanitized, case):
    exe, d = sanitized
    name, nb, bs, rp, ci, va, rhs = _systems()[case]
    inp, out = str(d / f"{name}.in"), str(d / f"{name}.out")
    _write(inp, nb, bs, rp, ci, va, rhs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    n = nb * bs
    raw = open(out, "rb").read()
    off = 0
    for (deg, relax, cyc, gm, form) in VARIANTS:
        st, it, stT, itT, levels = np.frombuffer(raw, dtype=np.int32, count=5, offset=off)
        off += 20
        x = np.frombuffer(raw, dtype=np.float64, count=n, offset=off)
        off += 8 * n
        y = np.frombuffer(raw, dtype=np.float64, count=n, offset=off)
        off += 8 * n
        H = Hierarchy(nb, bs, rp, ci, va, Params(degree=deg, relax=relax, cycle=cyc, gmres=gm, form=form,
                                                 max_coarse_dofs=16))
        xl, hl, sl = H.solve(rhs, 1e-10, 200)
        yl, hTl, sTl = H.solve_T(rhs, 1e-10, 200)
        assert levels == H.num_levels and levels >= 2
        assert st == 0 and stT == 0 and sl == "OK" and sTl == "OK"
        assert it == len(hl) and itT == len(hTl)
        assert np.array_equal(x, xl) and np.array_equal(y, yl)
    assert off == len(raw)
