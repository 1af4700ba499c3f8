"""CPU checks of the C-ABI library: it loads and exports every entry point
that include/nair.h declares (no compute call: there may be no GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nair.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nair_[a-z_T0-9]+)\s*\(", src)))


def _lib_path():
    import paper_1704_05001_amd.nair as N
    if not os.path.exists(N.LIB_PATH):
        from paper_1704_05001_amd.build import build
        build()
    return N.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("nair_setup", "nair_solve", "nair_solve_T", "nair_destroy", "nair_get_level"):
        assert f in names


def test_library_exports_every_declared_symbol():
    path = _lib_path()
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (nair_\w+)", out))
    missing = [f for f in _declared() if f not in exported]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_1704_05001_amd as P
    assert sorted(P.EXPORTED) == _declared()
    L = P.lib()
    for f in P.EXPORTED:
        assert hasattr(L, f)


def test_allocator_field_defaults_to_the_pool():
    import ctypes as C
    import paper_1704_05001_amd as P
    from paper_1704_05001_amd import nair as N
    p = N._Params()
    assert P.lib().nair_default_params(C.byref(p)) == 0
    assert p.allocator is None
    src = open(os.path.join(ROOT, "include", "nair.h")).read()
    assert "const nair_allocator *allocator;" in src and "typedef struct nair_allocator" in src
    with pytest.raises(ValueError, match="allocator"):
        P.Hierarchy.__init__(object.__new__(P.Hierarchy), *_tiny_pattern(), 1, P.Params(allocator="bogus"))


def _tiny_pattern():
    import torch
    return (torch.tensor([0, 1], dtype=torch.int32), torch.tensor([0], dtype=torch.int32),
            torch.ones(1, dtype=torch.float64))


def test_noalloc_scratch_size_matches_header():
    import paper_1704_05001_amd as P
    src = open(os.path.join(ROOT, "include", "nair.h")).read()
    m = re.search(r"#define NAIR_NOALLOC_SCRATCH_BYTES (\d+)", src)
    assert m and int(m.group(1)) == P.NOALLOC_SCRATCH_BYTES


def test_default_params_and_host_side_errors():
    """Host-only entry points: defaults, and argument errors caught before any device work."""
    import ctypes as C
    import paper_1704_05001_amd.nair as N
    L = N.lib()
    p = N._Params()
    assert L.nair_default_params(C.byref(p)) == 0
    assert (p.degree, p.theta, p.phi, p.drop, p.relax, p.max_levels, p.max_coarse_dofs) == \
        (1, 0.75, 0.025, 1e-3, 0, 30, 128)
    h = C.c_void_p()
    # bs out of range, negative degree, theta outside [0,1): rejected on the host
    assert L.nair_setup(4, 0, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.byref(p), None, C.byref(h)) == 1
    p.degree = -1
    assert L.nair_setup(4, 2, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.byref(p), None, C.byref(h)) == 1
    L.nair_default_params(C.byref(p))
    p.theta = 1.5
    assert L.nair_setup(4, 2, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.byref(p), None, C.byref(h)) == 1
    assert b"theta" in L.nair_last_error(None)
    L.nair_default_params(C.byref(p))
    assert (p.precision, p.form, p.cycle, p.gmres, p.faces, p.sweep_copy) == (0, 0, 0, 0, 1, -1)
    p.gmres = 201   # longer than the largest GMRES restart cycle
    assert L.nair_setup(4, 2, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.byref(p), None, C.byref(h)) == 1
    assert b"gmres" in L.nair_last_error(None)
    L.nair_default_params(C.byref(p))
    p.faces = 2
    assert L.nair_setup(4, 2, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.byref(p), None, C.byref(h)) == 1
    assert b"faces" in L.nair_last_error(None)
    L.nair_default_params(C.byref(p))
    p.sweep_copy = 2
    assert L.nair_setup(4, 2, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.byref(p), None, C.byref(h)) == 1
    assert b"sweep_copy" in L.nair_last_error(None)
    assert h.value is None
    # NULL handle
    assert L.nair_solve(None, C.c_void_p(8), C.c_void_p(8), 1e-10, 5, None, None) == 1


def test_product_path_has_no_oracle_dependency():
    """The package never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1704_05001_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "nair_oracle" not in txt and "from oracle" not in txt, f
