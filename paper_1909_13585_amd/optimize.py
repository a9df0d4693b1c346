"""Optimisation layer (binding of ``include/mlb_opt.h``; marshalling only).

``MMA`` wraps one ``mlb_mma`` handle (the method of moving asymptotes,
Svanberg 1987, with its per-variable work on the GPU); ``continuation``,
``p1_functions_dev`` and ``p2_functions_dev`` forward to the library's
continuation schedule and the problem functions of P1 (Sec. 3) and P2
(Sec. 6) with the bound formulation of the buckling constraint.
``p1_step_dev`` sequences one design step of P1 through the library's entry
points: filter and projection, analysis, sensitivities, problem functions,
chain rule, MMA update.  No arithmetic of the method runs here.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B
from ._binding import MlbError, MlbMmaInfo, MlbMmaOpts


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _hptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(t, numel, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= numel):
        raise ValueError(f"{name}: need a contiguous float64 CUDA tensor with at least {numel} entries")


def continuation(step, p0, dp, p_every, p_max, beta0=1.0, beta_every=0, beta_max=0.0):
    """(p, beta) at design step ``step`` (Secs. 3 and 6)."""
    lib = B.load()
    p, beta = C.c_double(), C.c_double()
    st = lib.mlb_continuation(int(step), float(p0), float(dp), int(p_every), float(p_max), float(beta0),
                              int(beta_every), float(beta_max), C.byref(p), C.byref(beta))
    if st != B.MLB_OK:
        raise MlbError(st, "invalid continuation parameters")
    return p.value, beta.value


def _functions(kind, x, J, dJ, lam, dlam, scale, lam_bar, f_bar, alpha, grad):
    lib = B.load()
    m = x.numel()
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    nb = lam.size
    _check_dev(x, m, "x")
    _check_dev(dJ, m, "dJ")
    _check_dev(dlam, nb * m, "dlam")
    _check_dev(grad, (2 + nb) * m, "grad")
    f0 = C.c_double()
    fval = np.zeros(1 + nb)
    if kind == 1:
        st = lib.mlb_p1_functions_dev(m, nb, _dptr(x), float(J), _dptr(dJ), _hptr(lam), _dptr(dlam), m, float(scale),
                                      float(lam_bar), float(f_bar), float(alpha), C.byref(f0), _hptr(fval),
                                      _dptr(grad), _stream())
    else:
        st = lib.mlb_p2_functions_dev(m, nb, _dptr(x), float(J), _dptr(dJ), _hptr(lam), _dptr(dlam), m, float(scale),
                                      float(lam_bar), float(alpha), C.byref(f0), _hptr(fval), _dptr(grad),
                                      _stream())
    if st != B.MLB_OK:
        raise MlbError(st, "problem functions")
    return f0.value, fval


def p1_functions_dev(x, J, dJ, lam, dlam, J0, lam_bar, f_bar, grad, alpha=0.99):
    """P1 (Sec. 3): returns (f0, fval); fills grad ((2 + nb), m) with the
    x-space gradient columns [objective, volume, bounds]."""
    return _functions(1, x, J, dJ, lam, dlam, J0, lam_bar, f_bar, alpha, grad)


def p2_functions_dev(x, J, dJ, lam, dlam, J_max, lam_bar, grad, alpha=0.99):
    """P2 (Sec. 6): returns (f0, fval); grad columns [objective (volume),
    compliance, bounds]."""
    return _functions(2, x, J, dJ, lam, dlam, J_max, lam_bar, 1.0, alpha, grad)


class MMA:
    """One ``mlb_mma`` handle for n variables and m constraints."""

    def __init__(self, n, m, xmin=0.0, xmax=1.0, move=0.2, asyinit=0.5, asyincr=1.2, asydecr=0.7, c=1000.0, d=1.0,
                 device=0):
        self.lib = B.load()
        o = MlbMmaOpts(xmin, xmax, move, asyinit, asyincr, asydecr, c, d)
        h = C.c_void_p()
        st = self.lib.mlb_mma_create(int(n), int(m), C.byref(o), int(device), C.byref(h))
        if st != B.MLB_OK:
            raise MlbError(st, "mlb_mma_create")
        self.h, self.n, self.m = h, int(n), int(m)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mlb_mma_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_dev(self, x, f0, df0, fval, dfdx):
        """x (n,) device in/out; df0 (n,) and dfdx (m, n) device; fval (m,) host.
        Returns the update's diagnostics."""
        _check_dev(x, self.n, "x")
        _check_dev(df0, self.n, "df0")
        _check_dev(dfdx, self.m * self.n, "dfdx")
        fv = np.ascontiguousarray(fval, dtype=np.float64)
        if fv.size != self.m:
            raise ValueError(f"fval: need {self.m} values")
        info = MlbMmaInfo()
        st = self.lib.mlb_mma_update_dev(self.h, _dptr(x), float(f0), _dptr(df0), _hptr(fv), _dptr(dfdx), self.n,
                                         C.byref(info), _stream())
        if st != B.MLB_OK:
            raise MlbError(st, self.lib.mlb_mma_last_error(self.h).decode())
        return dict(dual_iterations=info.dual_iterations, dual_evaluations=info.dual_evaluations,
                    proj_grad=info.proj_grad, dual_value=info.dual_value, lam=np.array(info.lam[:self.m]),
                    y=np.array(info.y[:self.m]), seconds=info.seconds)


class DesignStep:
    """Device buffers and settings of one design-step sequence on a context
    whose Dirichlet mask and loads are set: problem 1 = P1 (Sec. 3, minimum
    compliance; ``scale`` = J0 normalises the objective, ``f_bar`` the
    volume bound), problem 2 = P2 (Sec. 6, minimum volume; ``scale`` = J_max
    bounds the compliance).  ``step(xhat)`` runs one design step in place on
    the device design variables xhat (m,): filter and projection, analysis
    with q modes, sensitivities, problem functions with nb bounded factors,
    chain rule, MMA update.

    ``recycle``: each step's analysis starts from the previous step's
    solutions, the coarse buckling modes (a warm start of the coarse
    eigensolve, kept only if it beats the random start block) and the static
    displacement (scaled energy-optimally); answers stay within the solver
    tolerances, iteration counts drop as the design settles."""

    def __init__(self, ctx, problem, q, nb, rmin, eta, beta, scale, lam_bar, f_bar=1.0, alpha=0.99, tol=1e-8,
                 tol_eig=1e-8, max_it=3000, mma=None, recycle=False, **mma_opts):
        import torch
        if problem not in (1, 2):
            raise ValueError("problem must be 1 (P1) or 2 (P2)")
        self.ctx, self.problem, self.q, self.nb = ctx, problem, q, nb
        self.rmin, self.eta, self.beta = rmin, eta, beta
        self.scale, self.lam_bar, self.f_bar, self.alpha = scale, lam_bar, f_bar, alpha
        self.tol, self.tol_eig, self.max_it = tol, tol_eig, max_it
        m, n = ctx.m, ctx.n
        dev = dict(dtype=torch.float64, device="cuda")
        self.xt = torch.empty(m, **dev)
        self.x = torch.empty(m, **dev)
        self.U = torch.empty((1, n), **dev)
        self.dJ = torch.empty(m, **dev)
        self.dlam = torch.empty((q, m), **dev)
        self.gx = torch.empty((2 + nb, m), **dev)
        self.work = torch.empty((2 + nb, m), **dev)
        self.gh = torch.empty((2 + nb, m), **dev)
        self.mma = mma or MMA(m, 1 + nb, **mma_opts)
        self.recycle = bool(recycle)
        if self.recycle:
            self.Psi = torch.empty((q, ctx.level_size(ctx.eig_level)[0]), **dev)

    def step(self, xhat, penal=None, beta=None, timings=None):
        """One design step; ``penal`` / ``beta`` (optional) first move the SIMP
        exponent and the projection sharpness (continuation).  With a dict
        ``timings``, wall times of the analysis, the functions + chain rule
        and the MMA update are stored in it (the stream is synchronised
        between the parts)."""
        import time
        import torch
        c = self.ctx
        if penal is not None:
            c.set_penal(penal)
        if beta is not None:
            self.beta = float(beta)
        t0 = time.perf_counter()
        c.filter_project_dev(xhat, self.rmin, self.eta, self.beta, self.xt, self.x)
        c.set_density_dev(self.x)
        J, si = c.solve_static_dev(self.U, tol=self.tol, max_it=self.max_it)
        lam, ei = c.buckling_dev(self.q, None, tol_eig=self.tol_eig)
        c.sensitivities_dev(self.dJ, self.dlam)
        if self.recycle:
            # the next analysis starts from this one's solutions
            from . import MLB_WARM_COARSE, MLB_WARM_STATIC
            c.coarse_modes_dev(self.q, self.Psi)
            c.set_warm_start_dev(MLB_WARM_COARSE, self.Psi.t())
            c.set_warm_start_dev(MLB_WARM_STATIC, self.U.t())
        if timings is not None:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        if self.problem == 1:
            f0, fval = p1_functions_dev(self.x, J[0], self.dJ, lam[:self.nb], self.dlam, self.scale, self.lam_bar,
                                        self.f_bar, self.gx, self.alpha)
        else:
            f0, fval = p2_functions_dev(self.x, J[0], self.dJ, lam[:self.nb], self.dlam, self.scale, self.lam_bar,
                                        self.gx, self.alpha)
        c.filter_chain_dev(self.xt, self.rmin, self.eta, self.beta, self.gx, self.work, self.gh)
        if timings is not None:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        info = self.mma.update_dev(xhat, f0, self.gh[0], fval, self.gh[1:])
        if timings is not None:
            timings.update(analysis_s=t1 - t0, functions_chain_s=t2 - t1, mma_s=time.perf_counter() - t2)
        info.update(J=float(J[0]), lam=lam, f0=f0, fval=fval, static_iterations=si["iterations"],
                    coarse_iterations=ei["coarse_iterations"], coarse_warm_used=ei["coarse_warm_used"],
                    fine_iterations=ei["fine_iterations"])
        return info


class P1Step(DesignStep):
    """Design steps of P1 (Sec. 3): objective J / J0, volume fraction <= f_bar."""

    def __init__(self, ctx, q, nb, rmin, eta, beta, J0, lam_bar, f_bar, **kw):
        super().__init__(ctx, 1, q, nb, rmin, eta, beta, J0, lam_bar, f_bar, **kw)


class P2Step(DesignStep):
    """Design steps of P2 (Sec. 6): objective volume fraction, J <= J_max."""

    def __init__(self, ctx, q, nb, rmin, eta, beta, J_max, lam_bar, **kw):
        super().__init__(ctx, 2, q, nb, rmin, eta, beta, J_max, lam_bar, **kw)
