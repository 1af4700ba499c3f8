"""The Python binding rejects tensors the library would misread, before any call.

The C ABI takes raw device pointers and reads or writes exactly nb * bs
doubles (or nnzb * bs * bs for the matrix); a float32, short, strided or
misplaced tensor would be read past its end.  The binding checks dtype,
contiguity, size and device first and raises ValueError, so these tests run
without a GPU: the check fires before the library is reached.
"""
import pytest
import torch

import paper_1704_05001_amd as P
from paper_1704_05001_amd import nair


def _fake_hierarchy(nb=4, bs=3):
    """A handle-less Hierarchy on the CPU device, enough for the argument checks."""
    H = P.Hierarchy.__new__(P.Hierarchy)
    H.nb, H.bs, H.nsys = nb, bs, 1
    H.device = torch.device("cpu")
    H._h = None
    return H


GOOD = lambda n: torch.zeros(n, dtype=torch.float64)


@pytest.mark.parametrize("method", ["solve", "solve_T", "solve_batch"])
@pytest.mark.parametrize("bad", ["float32", "short", "long", "strided", "list"])
def test_solve_rejects_bad_right_hand_side(method, bad):
    H = _fake_hierarchy()
    n = H.n
    b = {"float32": torch.zeros(n, dtype=torch.float32), "short": GOOD(n - 1), "long": GOOD(n + 3),
         "strided": torch.zeros(2 * n, dtype=torch.float64)[::2], "list": [0.0] * n}[bad]
    with pytest.raises(ValueError):
        getattr(H, method)(b)


@pytest.mark.parametrize("method", ["solve", "solve_T", "solve_batch"])
def test_solve_rejects_bad_output(method):
    H = _fake_hierarchy()
    n = H.n
    b = GOOD(n)
    for x in (torch.zeros(n, dtype=torch.float32), GOOD(n - 1), torch.zeros((n, 2), dtype=torch.float64)[:, 0],
              GOOD(n).requires_grad_()):
        with pytest.raises(ValueError):
            getattr(H, method)(b, x)
    with pytest.raises(ValueError):      # x aliasing b
        getattr(H, method)(b, b)


def test_vcycle_rejects_bad_vectors():
    H = _fake_hierarchy()
    with pytest.raises(ValueError):
        H.vcycle(torch.zeros(H.n, dtype=torch.float32))
    with pytest.raises(ValueError):
        H.vcycle_T(GOOD(H.n + 1))


def test_vector_on_another_device_is_rejected():
    H = _fake_hierarchy()
    H.device = torch.device("cuda", 0)      # the check compares devices before any launch
    with pytest.raises(ValueError):
        H.solve(GOOD(H.n))


def test_setup_rejects_bad_matrix_tensors():
    rp = torch.tensor([0, 1, 2], dtype=torch.int32)
    ci = torch.tensor([0, 1], dtype=torch.int32)
    va = torch.zeros((2, 3, 3), dtype=torch.float64)
    for args in ((rp.long(), ci, va), (rp, ci.long(), va), (rp, ci, va.float()),
                 (rp, ci, torch.zeros((3, 2, 3), dtype=torch.float64).transpose(0, 1))):
        with pytest.raises(ValueError):
            P.Hierarchy(*args, 3)
    with pytest.raises(ValueError):          # host tensors: the library takes device pointers
        P.Hierarchy(rp, ci, va, 3)


def test_block_sizes_follow_rowptr():
    """colidx and vals must hold exactly rowptr[-1] blocks of bs x bs."""
    nair._check_block_sizes(3, 3, 12, 2)                  # consistent: passes
    for args in ((3, 2, 12, 2), (3, 3, 8, 2), (3, 3, 12, 3), (3, 3, 0, 0), (0, 1, 0, 2)):
        with pytest.raises(ValueError):
            nair._check_block_sizes(*args)


def test_grad_vals_rejects_bad_vectors():
    rp = torch.tensor([0, 1, 2], dtype=torch.int32)
    ci = torch.tensor([0, 1], dtype=torch.int32)
    good = GOOD(6)
    for y, x in ((torch.zeros(6, dtype=torch.float32), good), (good, GOOD(5)), (GOOD(7), good)):
        with pytest.raises(ValueError):
            P.grad_vals(rp, ci, y, x, 3)
    with pytest.raises(ValueError):
        P.grad_vals(rp.long(), ci, good, good, 3)
