"""Argument checks of the batched-instance entry point that run before any
device work (no GPU needed: invalid descriptors are rejected on the host)."""
import os

import pytest

from paper_1909_13585_amd import _binding as B


def _lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libmlb.so is not built")
    return B.load()


def _create(nels, **kw):
    import ctypes as C
    lib = _lib()
    d = B.MlbBatchDesc()
    d.ninst = kw.get("ninst", len(nels))
    for i, (nx, ny) in enumerate(nels):
        d.nel[2 * i], d.nel[2 * i + 1] = nx, ny
    d.E1, d.E0, d.nu, d.penal = kw.get("E1", 1.0), kw.get("E0", 1e-6), kw.get("nu", 0.3), kw.get("penal", 3.0)
    d.precision = kw.get("precision", B.MLB_FP64)
    d.max_coarse_dofs = kw.get("max_coarse_dofs", 0)
    h = C.c_void_p()
    st = lib.mlb_batch_create(C.byref(d), C.byref(h))
    msg = lib.mlb_batch_last_error(h).decode() if h else ""
    if h:
        lib.mlb_batch_destroy(h)
    return st, msg


@pytest.mark.parametrize("nels,kw,needle", [
    ([], {}, "ninst"),
    ([(16, 9)], {}, "even"),
    ([(16, 0)], {}, "even"),
    ([(16, 8), (7, 8)], {}, "instance 1"),
    ([(2046, 2)], {}, "coarsest"),          # 1023 x 1 after one halving: 4096 DOFs
    ([(16, 8)], {"E0": 2.0}, "E0"),
    ([(16, 8)], {"nu": 0.5}, "Poisson"),
    ([(16, 8)], {"penal": 0.5}, "penalty"),
    ([(16, 8)], {"precision": 7}, "precision"),
])
def test_invalid_descriptors_are_rejected(nels, kw, needle):
    st, msg = _create(nels, **kw)
    assert st == B.MLB_EINVAL
    assert needle in msg, msg


def test_too_many_instances():
    st, msg = _create([(16, 8)] * 64, ninst=65)
    assert st == B.MLB_EINVAL and "ninst" in msg
