"""Many independent 2D static analyses advanced together (``include/mlb_batch.h``).

Argument marshalling only: every step runs in the library's HIP kernels.
Batched arrays are the instances' arrays concatenated in instance order
(``dof_off`` / ``elem_off`` give the offsets).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B
from ._binding import MLB_FP64, MlbError


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Batch:
    """Independent Q4 instances (grids ``nels``) solved by one set of launches."""

    def __init__(self, nels, E1=1.0, E0=1e-6, nu=0.3, penal=3.0, precision=MLB_FP64, device=0,
                 max_coarse_dofs=0):
        self.lib = B.load()
        d = B.MlbBatchDesc()
        d.ninst = len(nels)
        if not 1 <= d.ninst <= 64:
            raise ValueError("between 1 and 64 instances")
        for i, (nx, ny) in enumerate(nels):
            d.nel[2 * i], d.nel[2 * i + 1] = int(nx), int(ny)
        d.E1, d.E0, d.nu, d.penal = E1, E0, nu, penal
        d.precision, d.device, d.max_coarse_dofs = precision, device, max_coarse_dofs
        self.nels = [tuple(int(v) for v in nel) for nel in nels]
        self.ninst = d.ninst
        h = C.c_void_p()
        st = self.lib.mlb_batch_create(C.byref(d), C.byref(h))
        self.h = h
        if st != B.MLB_OK:
            msg = self.last_error()
            self.close()
            raise MlbError(st, msg)
        n = self.ninst
        dof = np.zeros(n + 1, dtype=np.int64)
        elem = np.zeros(n + 1, dtype=np.int64)
        lev = np.zeros(n, dtype=np.int32)
        self._check(self.lib.mlb_batch_layout(self.h, C.c_void_p(dof.ctypes.data), C.c_void_p(elem.ctypes.data),
                                              C.c_void_p(lev.ctypes.data)))
        self.dof_off, self.elem_off, self.levels = dof, elem, lev
        self.n, self.m = int(dof[-1]), int(elem[-1])

    def last_error(self):
        if not self.h:
            return ""
        return self.lib.mlb_batch_last_error(self.h).decode()

    def _check(self, st):
        if st != B.MLB_OK:
            raise MlbError(st, self.last_error())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mlb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_opts(self, smooth_steps=None, jacobi_omega=None, queue=None, graphs=None, check_every=None,
                 refine_steps=None):
        o = B.MlbBatchOpts()
        self._check(self.lib.mlb_batch_get_opts(self.h, C.byref(o)))
        if smooth_steps is not None:
            o.smooth_steps = smooth_steps
        if jacobi_omega is not None:
            o.jacobi_omega = jacobi_omega
        if queue is not None:
            o.queue = int(queue)
        if graphs is not None:
            o.graphs = int(graphs)
        if check_every is not None:
            o.check_every = check_every
        if refine_steps is not None:
            o.refine_steps = int(refine_steps)
        self._check(self.lib.mlb_batch_set_opts(self.h, C.byref(o)))

    def set_problem_dev(self, fixed, F, x):
        """fixed: uint8 [n], F: float64 [n], x: float64 [m] device tensors (batched layout)."""
        self._check(self.lib.mlb_batch_set_problem_dev(self.h, _dptr(fixed), _dptr(F), _dptr(x), _stream()))

    def solve_dev(self, U, tol=1e-8, max_it=2000):
        J = np.zeros(self.ninst)
        its = np.zeros(self.ninst, dtype=np.int32)
        info = B.MlbBatchInfo()
        self._check(self.lib.mlb_batch_solve_dev(self.h, tol, max_it, _dptr(U), C.c_void_p(J.ctypes.data),
                                                 C.c_void_p(its.ctypes.data), C.byref(info), _stream()))
        return J, its, {f: getattr(info, f) for f, _ in info._fields_}

    def residuals(self):
        """Per-instance true residuals of the returned u (double-double
        evaluation), FP64 floors, and residuals of the refined double-double
        solution, of the last solve."""
        res = np.zeros(self.ninst)
        floor = np.zeros(self.ninst)
        res_dd = np.zeros(self.ninst)
        self._check(self.lib.mlb_batch_residuals(self.h, C.c_void_p(res.ctypes.data), C.c_void_p(floor.ctypes.data),
                                                 C.c_void_p(res_dd.ctypes.data)))
        return res, floor, res_dd

    def compliance_sens_dev(self, dJ):
        self._check(self.lib.mlb_batch_compliance_sens_dev(self.h, _dptr(dJ), _stream()))

    # helpers for host arrays of the instances
    def concat(self, arrays, dtype):
        return np.concatenate([np.asarray(a, dtype=dtype).ravel() for a in arrays])

    def split_dofs(self, v):
        return [v[self.dof_off[i]:self.dof_off[i + 1]] for i in range(self.ninst)]

    def split_elems(self, v):
        return [v[self.elem_off[i]:self.elem_off[i + 1]] for i in range(self.ninst)]
