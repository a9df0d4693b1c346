"""MI355X multilevel linearized-buckling engine (Python binding).

Thin wrapper around the C ABI of ``include/mlb.h``: every call marshals
arguments and forwards to ``libmlb.so`` (hand-written HIP kernels for gfx950).
Host arrays are numpy float64 / uint8; device arrays are torch tensors on the
GPU (torch supplies device memory and the current stream only).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B
from ._binding import (MLB_ELEM_CONFORMING, MLB_ELEM_INCOMPATIBLE, MLB_FP64, MLB_MIXED, MLB_WARM_COARSE, MLB_WARM_NONE, MLB_WARM_STATIC, MlbError,
                       MlbEigInfo, MlbSolveInfo)

__all__ = ["Context", "MlbError", "MLB_FP64", "MLB_MIXED", "MLB_ELEM_CONFORMING", "MLB_ELEM_INCOMPATIBLE", "MLB_WARM_NONE", "MLB_WARM_COARSE",
           "MLB_WARM_STATIC", "load_library"]


def load_library():
    return B.load()


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _info_dict(info):
    return {f: getattr(info, f) for f, _ in info._fields_}


class Context:
    """One analysis context (``mlb_ctx``) for a fixed grid and material."""

    def __init__(self, nel, E1=1.0, E0=1e-6, nu=0.3, penal=3.0, mg_levels=3, eig_level=2,
                 precision=MLB_FP64, device=0, element=0):
        self.lib = B.load()
        d = B.MlbDesc()
        d.dim = len(nel)
        for i, v in enumerate(nel):
            d.nel[i] = int(v)
        d.E1, d.E0, d.nu, d.penal = E1, E0, nu, penal
        d.mg_levels, d.eig_level, d.precision, d.device = mg_levels, eig_level, precision, device
        d.element = element
        self.nel = tuple(int(v) for v in nel)
        self.dim = d.dim
        self.mg_levels, self.eig_level = mg_levels, eig_level
        h = C.c_void_p()
        st = self.lib.mlb_create(C.byref(d), C.byref(h))
        self.h = h
        if st != B.MLB_OK:
            msg = self.last_error()
            self.close()
            raise MlbError(st, msg)
        self.n, self.m = self.level_size(1)
        self.k = 0
        self.ncases = 0

    # -- plumbing
    def last_error(self):
        if not self.h:
            return ""
        return self.lib.mlb_last_error(self.h).decode()

    def _check(self, st):
        if st != B.MLB_OK:
            raise MlbError(st, self.last_error())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mlb_destroy(self.h)
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

    def level_size(self, level):
        n = C.c_int64()
        m = C.c_int64()
        self._check(self.lib.mlb_level_size(self.h, level, C.byref(n), C.byref(m)))
        return n.value, m.value

    def set_opts(self, smooth_steps=0, jacobi_omega=0.0, eig_guard=0, eig_max_it=0, check_every=0, seed=0,
                 cycle=0, block_cg=0, eig_sweeps=0, graphs=0, pinvit_steps=0, refine_sweeps=0, coarse_sweeps=0,
                 pinvit_shift=0, refine_fine=0):
        """Zero (the default of every argument) keeps the current value;
        pinvit_steps < 0 and refine_sweeps < 0 turn those steps off;
        pinvit_shift 1 = own Ritz values, 2 = the printed lam~_1;
        refine_fine 1 = the refinement also visits the fine grid, < 0 = not."""
        o = B.MlbOpts(smooth_steps, jacobi_omega, eig_guard, eig_max_it, check_every, seed, cycle, block_cg,
                      eig_sweeps, graphs, pinvit_steps, refine_sweeps, coarse_sweeps, pinvit_shift, refine_fine)
        self._check(self.lib.mlb_set_opts(self.h, C.byref(o)))

    def set_omegas(self, omegas):
        """Jacobi weights of levels 1 .. len(omegas) (until the next density)."""
        w = np.ascontiguousarray(omegas, dtype=np.float64)
        self._check(self.lib.mlb_set_omegas(self.h, len(w), _ptr(w)))

    def get_omegas(self, nlevels):
        w = np.zeros(nlevels)
        self._check(self.lib.mlb_get_omegas(self.h, nlevels, _ptr(w)))
        return w

    # -- problem data (host)
    def set_bc(self, fixed):
        f = np.ascontiguousarray(fixed, dtype=np.uint8)
        assert f.shape == (self.n,)
        self._check(self.lib.mlb_set_bc(self.h, _ptr(f)))

    def set_loads(self, F):
        F = np.asarray(F, dtype=np.float64)
        if F.ndim == 1:
            F = F[:, None]
        Fc = np.asfortranarray(F)
        assert Fc.shape[0] == self.n
        self.ncases = Fc.shape[1]
        self._check(self.lib.mlb_set_loads(self.h, self.ncases, C.c_void_p(Fc.ctypes.data)))

    def set_density(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.m,)
        self._check(self.lib.mlb_set_density(self.h, _ptr(x)))

    def set_warm_start(self, kind, data=None):
        if kind == MLB_WARM_NONE:
            self._check(self.lib.mlb_set_warm_start(self.h, kind, 0, None))
            return
        D = np.asfortranarray(np.asarray(data, dtype=np.float64))
        if D.ndim == 1:
            D = D[:, None]
        self._check(self.lib.mlb_set_warm_start(self.h, kind, D.shape[1], C.c_void_p(D.ctypes.data)))

    def set_warm_start_dev(self, kind, data):
        """Warm start from a float64 device tensor (n x ncols, column-major:
        pass the transpose of a contiguous (ncols, n) tensor, or one column)."""
        ncols = 1 if data.dim() == 1 else data.shape[1]
        self._check(self.lib.mlb_set_warm_start_dev(self.h, kind, ncols, _dptr(data), _stream()))

    # -- analysis (host outputs)
    def solve_static(self, tol=1e-8, max_it=1000):
        U = np.zeros((self.n, self.ncases), order="F")
        J = np.zeros(self.ncases)
        info = MlbSolveInfo()
        self._check(self.lib.mlb_solve_static(self.h, tol, max_it, C.c_void_p(U.ctypes.data), _ptr(J),
                                              C.byref(info)))
        return U, J, _info_dict(info)

    def buckling(self, k, ref_case=0, tol_eig=1e-10, want_modes=True):
        lam = np.zeros(k)
        Phi = np.zeros((self.n, k), order="F") if want_modes else None
        info = MlbEigInfo()
        self._check(self.lib.mlb_buckling(self.h, ref_case, k, tol_eig, _ptr(lam),
                                          C.c_void_p(Phi.ctypes.data) if want_modes else None, C.byref(info)))
        self.k = k
        return lam, Phi, _info_dict(info)

    def eig_residuals(self):
        r = np.zeros(self.k)
        self._check(self.lib.mlb_eig_residuals(self.h, _ptr(r)))
        return r

    def eig_residuals_dev(self, out):
        self._check(self.lib.mlb_eig_residuals_dev(self.h, _dptr(out), _stream()))

    def sensitivities(self, compliance=True, buckling=True):
        dJ = np.zeros((self.m, self.ncases), order="F") if compliance else None
        dl = np.zeros((self.m, self.k), order="F") if buckling else None
        info = MlbSolveInfo()
        self._check(self.lib.mlb_sensitivities(self.h, C.c_void_p(dJ.ctypes.data) if compliance else None,
                                               C.c_void_p(dl.ctypes.data) if buckling else None, C.byref(info)))
        return dJ, dl, _info_dict(info)

    # -- device variants (torch tensors on the GPU, current stream)
    def set_density_dev(self, x):
        self._check(self.lib.mlb_set_density_dev(self.h, _dptr(x), _stream()))

    def solve_static_dev(self, U, tol=1e-8, max_it=1000):
        J = np.zeros(self.ncases)
        info = MlbSolveInfo()
        self._check(self.lib.mlb_solve_static_dev(self.h, tol, max_it, _dptr(U), _ptr(J), C.byref(info),
                                                  _stream()))
        return J, _info_dict(info)

    def buckling_dev(self, k, Phi=None, ref_case=0, tol_eig=1e-10):
        lam = np.zeros(k)
        info = MlbEigInfo()
        self._check(self.lib.mlb_buckling_dev(self.h, ref_case, k, tol_eig, _ptr(lam), _dptr(Phi), C.byref(info),
                                              _stream()))
        self.k = k
        return lam, _info_dict(info)

    def sensitivities_dev(self, dJ=None, dlam=None):
        info = MlbSolveInfo()
        self._check(self.lib.mlb_sensitivities_dev(self.h, _dptr(dJ), _dptr(dlam), C.byref(info), _stream()))
        return _info_dict(info)

    def sensitivities_consistent(self):
        """Consistent buckling sensitivities (m, k) of the last buckling call (host)."""
        dl = np.zeros((self.m, self.k), order="F")
        info = MlbSolveInfo()
        self._check(self.lib.mlb_sensitivities_consistent(self.h, dl.ctypes.data_as(C.c_void_p), C.byref(info)))
        return dl, _info_dict(info)

    def sensitivities_consistent_dev(self, dlam):
        """Consistent buckling sensitivities into dlam (k, m) on the device."""
        info = MlbSolveInfo()
        self._check(self.lib.mlb_sensitivities_consistent_dev(self.h, _dptr(dlam), C.byref(info), _stream()))
        return _info_dict(info)

    def apply_K_dev(self, level, x, y):
        self._check(self.lib.mlb_apply_K_dev(self.h, level, x.shape[0] if x.dim() > 1 else 1,
                                             _dptr(x), _dptr(y), _stream()))

    def apply_G_dev(self, level, x, y):
        self._check(self.lib.mlb_apply_G_dev(self.h, level, x.shape[0] if x.dim() > 1 else 1,
                                             _dptr(x), _dptr(y), _stream()))

    def set_state_dev(self, u, stress_out=None):
        self._check(self.lib.mlb_set_state_dev(self.h, _dptr(u), _dptr(stress_out), _stream()))

    def prolong_dev(self, level, xc, yf):
        self._check(self.lib.mlb_prolong_dev(self.h, level, xc.shape[0] if xc.dim() > 1 else 1,
                                             _dptr(xc), _dptr(yf), _stream()))

    def restrict_dev(self, level, xf, yc):
        self._check(self.lib.mlb_restrict_dev(self.h, level, xf.shape[0] if xf.dim() > 1 else 1,
                                              _dptr(xf), _dptr(yc), _stream()))

    def coarse_modes_dev(self, k, Psi):
        """Copies the K^l-orthonormal coarse modes of the last buckling call into Psi (k, n_l)."""
        self._check(self.lib.mlb_coarse_modes_dev(self.h, k, _dptr(Psi), _stream()))

    def set_tiles(self, wht_zchunk=0, stencil_cols=0, wht_variant=-1):
        self._check(self.lib.mlb_set_tiles(self.h, wht_zchunk, stencil_cols, wht_variant))

    def autotune(self, ncols):
        """Times the candidate tiles on Jacobi sweeps of ncols columns and keeps the fastest."""
        info = B.MlbTuneInfo()
        self._check(self.lib.mlb_autotune(self.h, ncols, C.byref(info), _stream()))
        out = {}
        for f, _ in info._fields_:
            v = getattr(info, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out

    def adjoint_rhs_dev(self, k, B):
        """Copies the adjoint right-hand sides of the last sensitivities call into B (k, n)."""
        self._check(self.lib.mlb_adjoint_rhs_dev(self.h, k, _dptr(B), _stream()))

    def solve_block_dev(self, B, X, tol=1e-8, max_it=1000):
        """K X = B for the columns of B (ncols, n) as one block CG; returns the solve info."""
        info = MlbSolveInfo()
        self._check(self.lib.mlb_solve_block_dev(self.h, B.shape[0], _dptr(B), _dptr(X), tol, max_it, C.byref(info),
                                                 _stream()))
        return _info_dict(info)

    def _block(self, t, rows, width, name):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != rows * width:
            raise ValueError(f"{name}: contiguous float64 CUDA tensor of {rows} x {width} expected")

    def mac_dev(self, A, B, W):
        """C[j, r] = a_j^T K b_r (Sec. 5, modal energy correlation) for the rows of
        A (qa, n) and B (qb, n); W (qb, n) is overwritten with K B."""
        qa, qb = A.shape[0], B.shape[0]
        self._block(A, qa, self.n, "A")
        self._block(B, qb, self.n, "B")
        self._block(W, qb, self.n, "W")
        out = np.zeros(qa * qb)
        self._check(self.lib.mlb_mac_dev(self.h, qa, _dptr(A), qb, _dptr(B), _dptr(W),
                                         out.ctypes.data_as(C.c_void_p), _stream()))
        return out.reshape(qb, qa).T

    def sed_tv_dev(self, Phi, xbar, sed, gradn):
        """Strain energy density sed (q, m), its gradient magnitude on {x >= xbar}
        gradn (q, m) for the modes Phi (q, n); returns the total variations (q,)."""
        q = Phi.shape[0]
        self._block(Phi, q, self.n, "Phi")
        self._block(sed, q, self.m, "sed")
        self._block(gradn, q, self.m, "gradn")
        tv = np.zeros(q)
        self._check(self.lib.mlb_sed_tv_dev(self.h, q, _dptr(Phi), xbar, _dptr(sed), _dptr(gradn),
                                            tv.ctypes.data_as(C.c_void_p), _stream()))
        return tv

    def dilate_dev(self, gradn, rel_thr, r_th, x, xout):
        """xout = local dilation of x (m,) within r_th around the elements where a
        row of gradn (nsel, m) reaches rel_thr times its maximum."""
        nsel = gradn.shape[0] if gradn.dim() > 1 else 1
        self._block(gradn, nsel, self.m, "gradn")
        self._block(x, 1, self.m, "x")
        self._block(xout, 1, self.m, "xout")
        self._check(self.lib.mlb_dilate_dev(self.h, nsel, _dptr(gradn), rel_thr, r_th, _dptr(x), _dptr(xout),
                                            _stream()))

    def dilate_noalloc_dev(self, gradn, rel_thr, r_th, x, xout):
        """dilate_dev without any device allocation (fixed per-GPU scratch;
        calls that overlap on one GPU race)."""
        nsel = gradn.shape[0] if gradn.dim() > 1 else 1
        self._block(gradn, nsel, self.m, "gradn")
        self._block(x, 1, self.m, "x")
        self._block(xout, 1, self.m, "xout")
        self._check(self.lib.mlb_dilate_noalloc_dev(self.h, nsel, _dptr(gradn), rel_thr, r_th, _dptr(x),
                                                    _dptr(xout), _stream()))

    def set_penal(self, penal):
        """SIMP exponent for the following set_density* calls (continuation)."""
        self._check(self.lib.mlb_set_penal(self.h, float(penal)))

    def filter_project_dev(self, xhat, rmin, eta, beta, xtilde, x):
        """Density filter of radius rmin and Heaviside projection (eta, beta) of
        the design variables xhat (m,) into xtilde and x (m,) (Sec. 2)."""
        for t, name in ((xhat, "xhat"), (xtilde, "xtilde"), (x, "x")):
            self._block(t, 1, self.m, name)
        self._check(self.lib.mlb_filter_project_dev(self.h, _dptr(xhat), rmin, eta, beta, _dptr(xtilde), _dptr(x),
                                                    _stream()))

    def filter_chain_dev(self, xtilde, rmin, eta, beta, dfdx, work, dfdxhat):
        """Sensitivities dfdx (ncols, m) w.r.t. the physical densities taken back
        to the design variables into dfdxhat (ncols, m); work (ncols, m) scratch."""
        nc = dfdx.shape[0] if dfdx.dim() > 1 else 1
        self._block(xtilde, 1, self.m, "xtilde")
        for t, name in ((dfdx, "dfdx"), (work, "work"), (dfdxhat, "dfdxhat")):
            self._block(t, nc, self.m, name)
        self._check(self.lib.mlb_filter_chain_dev(self.h, nc, _dptr(xtilde), rmin, eta, beta, _dptr(dfdx),
                                                  _dptr(work), _dptr(dfdxhat), _stream()))

    def adjoints_dev(self, k, Z):
        """Copies the adjoint solutions of the last sensitivities call into Z (k, n)."""
        self._check(self.lib.mlb_adjoints_dev(self.h, k, _dptr(Z), _stream()))

    def sweep_dev(self, level, ncols, reps=1):
        """reps Jacobi sweeps of the cycle on its level work blocks (for timing)."""
        self._check(self.lib.mlb_sweep_dev(self.h, level, ncols, reps, _stream()))

    def vcycle_dev(self, level, r, z):
        self._check(self.lib.mlb_vcycle_dev(self.h, level, r.shape[0] if r.dim() > 1 else 1,
                                            _dptr(r), _dptr(z), _stream()))
