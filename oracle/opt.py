"""Optimisation layer of Secs. 3 and 6 (oracle; test infrastructure only).

Three pieces turn the buckling analysis into the paper's design problems
P1 (minimum compliance under a buckling and a volume constraint, Sec. 3) and
P2 (minimum volume under a buckling and a compliance constraint, Sec. 6):

* continuation of the SIMP exponent p and of the projection sharpness beta
  (Sec. 3: p from 1 to 6 in steps of 0.25 every 25 design steps, beta = 6
  fixed; Sec. 6: p from 3 the same way, then beta doubled every 50 steps
  from 1 up to 32);
* the bound formulation of the buckling constraint (Sec. 3): the minimum over
  the constrained set B of the buckling factors is replaced by one constraint
  per factor, with a small geometric gap alpha = 0.99 between their bounds;
* the method of moving asymptotes (MMA, Svanberg 1987, the method the paper
  names) that updates the design variables.

Readings (the paper is silent or garbled on these):
  (a) Continuation.  p_k = min(p0 + dp floor(k / p_every), p_max) at design
      step k = 0, 1, ...  Let k_p be the first step with p_k = p_max.  beta
      stays beta0 until k_p + beta_every and then doubles every beta_every
      steps: beta_k = min(beta0 2^floor((k - k_p) / beta_every), beta_max) for
      k >= k_p.  With Sec. 6's numbers p reaches 6 at step 300 and beta
      reaches 32 at step 550, inside the 600 steps run there.
  (b) Bound formulation.  The printed constraint has the factor in the
      numerator and reads as an upper bound, which would contradict the
      problem statement (lowest factor at least lambda_bar).  The reading
      consistent with both the stated purpose (a small gap that keeps the
      bounded factors from coalescing) and the coalescence measure delta_i
      of the same section (which vanishes when lambda_1 / lambda_i equals
      alpha^(i-1)) is the lower bound lambda~_i >= lambda_bar alpha^(-i):
          g_i = 1 - alpha^i lambda~_i / lambda_bar <= 0,   i = 1 .. |B|,
          dg_i/dx = -(alpha^i / lambda_bar) dlambda~_i/dx.
  (c) MMA.  Svanberg's approximations around the current point x^k,
          f~_i(x) = r_i + sum_j p_ij / (U_j - x_j) + q_ij / (x_j - L_j),
      with the later regularised coefficients (Svanberg's 2007 notes)
          p_ij = (U_j - x_j)^2 (1.001 g+ + 0.001 g- + 1e-5 / dx_j),
          q_ij = (x_j - L_j)^2 (0.001 g+ + 1.001 g- + 1e-5 / dx_j),
      g = df_i/dx_j, g+ = max(g, 0), g- = max(-g, 0), dx = x_max - x_min,
      and r_i such that f~_i(x^k) = f_i(x^k) (value and gradient are then
      exact at x^k).  Asymptotes: L = x - 0.5 dx, U = x + 0.5 dx on the first
      two iterations; afterwards each is moved out by 1.2 where x_j kept its
      direction over the last two steps, in by 0.7 where it reversed, and
      clamped to [0.01 dx, 10 dx] away from x_j.  Move limits: alpha_j =
      max(x_min, L + 0.1 (x - L), x - move dx), beta_j = min(x_max,
      U - 0.1 (U - x), x + move dx), move = 0.2.  Subproblem with elastic
      variables y >= 0 (a0 = 1, a_i = 0, c_i = 1000, d_i = 1, so z = 0):
          min f~_0(x) + sum_i (c_i y_i + d_i y_i^2 / 2)
          s.t. f~_i(x) - y_i <= 0,  alpha <= x <= beta,  y >= 0,
      strictly convex and separable, solved exactly through its dual (see
      ``MMA.solve_subproblem``).

Reading (b) and the MMA parameters are listed in the design notes.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- continuation
def continuation(k, p0, dp, p_every, p_max, beta0=1.0, beta_every=0, beta_max=None):
    """(p_k, beta_k) of reading (a); beta_every = 0 keeps beta fixed at beta0."""
    p = min(p0 + dp * (k // p_every), p_max)
    if beta_every <= 0:
        return p, beta0
    # first step at which p reaches p_max
    inc = int(np.ceil((p_max - p0) / dp - 1e-12))
    k_p = max(inc, 0) * p_every
    if k < k_p:
        return p, beta0
    beta = beta0 * 2.0 ** ((k - k_p) // beta_every)
    return p, min(beta, beta_max) if beta_max is not None else beta


def sec3_schedule(k):
    """Sec. 3 (problem P1): p 1 -> 6 by 0.25 every 25 steps, beta = 6."""
    return continuation(k, 1.0, 0.25, 25, 6.0, beta0=6.0)


def sec6_schedule(k):
    """Sec. 6 (problem P2): p 3 -> 6 by 0.25 every 25 steps, then beta doubled
    every 50 steps from 1 up to 32."""
    return continuation(k, 3.0, 0.25, 25, 6.0, beta0=1.0, beta_every=50, beta_max=32.0)


# ---------------------------------------------------------- bound formulation
def bound_constraints(lam, dlam, lam_bar, alpha=0.99):
    """g_i = 1 - alpha^i lam_i / lam_bar and its gradient rows (reading (b)).

    lam: (nb,) ascending buckling factors, dlam: (nb, m) their sensitivities.
    Returns g (nb,), dg (nb, m)."""
    lam = np.asarray(lam, dtype=np.float64)
    w = alpha ** np.arange(1, lam.size + 1, dtype=np.float64) / lam_bar
    g = 1.0 - w * lam
    dg = -w[:, None] * np.asarray(dlam, dtype=np.float64)
    return g, dg


# ------------------------------------------------------------------------ MMA
class MMA:
    """Method of moving asymptotes for min f_0(x) s.t. f_i(x) <= 0 (i = 1..m),
    x_min <= x <= x_max; one call of ``update`` per design step (reading (c)).
    """

    def __init__(self, n, m, xmin=0.0, xmax=1.0, move=0.2, asyinit=0.5, asyincr=1.2, asydecr=0.7,
                 c=1000.0, d=1.0):
        self.n, self.m = n, m
        self.xmin = np.full(n, float(xmin)) if np.isscalar(xmin) else np.asarray(xmin, dtype=np.float64)
        self.xmax = np.full(n, float(xmax)) if np.isscalar(xmax) else np.asarray(xmax, dtype=np.float64)
        self.move, self.asyinit, self.asyincr, self.asydecr = move, asyinit, asyincr, asydecr
        self.c = np.full(m, float(c))
        self.d = np.full(m, float(d))
        self.it = 0
        self.xold1 = None
        self.xold2 = None
        self.low = None
        self.upp = None

    # -- asymptotes and move limits
    def asymptotes(self, x):
        dx = self.xmax - self.xmin
        if self.it < 2:
            low = x - self.asyinit * dx
            upp = x + self.asyinit * dx
        else:
            trend = (x - self.xold1) * (self.xold1 - self.xold2)
            factor = np.where(trend > 0, self.asyincr, np.where(trend < 0, self.asydecr, 1.0))
            low = x - factor * (self.xold1 - self.low)
            upp = x + factor * (self.upp - self.xold1)
            low = np.clip(low, x - 10.0 * dx, x - 0.01 * dx)
            upp = np.clip(upp, x + 0.01 * dx, x + 10.0 * dx)
        alpha = np.maximum.reduce([self.xmin, low + 0.1 * (x - low), x - self.move * dx])
        beta = np.minimum.reduce([self.xmax, upp - 0.1 * (upp - x), x + self.move * dx])
        return low, upp, alpha, beta

    # -- the convex approximations
    @staticmethod
    def coefficients(x, low, upp, dx, fval, grad):
        """p, q (rows 0..m, row 0 the objective) and r with f~_i(x) = f_i(x)."""
        g = np.atleast_2d(np.asarray(grad, dtype=np.float64))
        gp, gm = np.maximum(g, 0.0), np.maximum(-g, 0.0)
        reg = 1e-5 / dx
        p = (upp - x) ** 2 * (1.001 * gp + 0.001 * gm + reg)
        q = (x - low) ** 2 * (0.001 * gp + 1.001 * gm + reg)
        r = np.asarray(fval, dtype=np.float64) - (p / (upp - x) + q / (x - low)).sum(axis=1)
        return p, q, r

    @staticmethod
    def approx(x, low, upp, p, q, r):
        """f~_i(x) for every row i."""
        return r + (p / (upp - x) + q / (x - low)).sum(axis=1)

    # -- the subproblem, through its dual
    def _x_of(self, lam, low, upp, alpha, beta, p, q):
        """Minimiser over alpha <= x <= beta of the Lagrangian's x-part: the
        stationary point P/(U-x)^2 = Q/(x-L)^2, clipped to the box."""
        w = np.concatenate(([1.0], lam))
        P = w @ p
        Q = w @ q
        sp, sq = np.sqrt(P), np.sqrt(Q)
        xs = (low * sp + upp * sq) / (sp + sq)
        return np.clip(xs, alpha, beta), P, Q

    def dual(self, lam, low, upp, alpha, beta, p, q, r):
        """Dual value W, gradient and Hessian at lam >= 0, plus x(lam), y(lam)."""
        x, P, Q = self._x_of(lam, low, upp, alpha, beta, p, q)
        y = np.maximum(0.0, (lam - self.c) / self.d)
        h = self.approx(x, low, upp, p, q, r)              # h[0] objective, h[1:] constraints
        W = h[0] + lam @ (h[1:] - y) + self.c @ y + 0.5 * self.d @ (y * y)
        g = h[1:] - y
        # Hessian: x_j moves with lam only where it is strictly inside its box
        free = (x > alpha) & (x < beta)
        a = p[1:] / (upp - x) ** 2 - q[1:] / (x - low) ** 2       # df~_i/dx_j
        curv = 2.0 * P / (upp - x) ** 3 + 2.0 * Q / (x - low) ** 3
        af = a[:, free]
        H = -(af / curv[free]) @ af.T
        H -= np.diag(np.where(lam > self.c, 1.0 / self.d, 0.0))
        return W, g, H, x, y

    def solve_subproblem(self, low, upp, alpha, beta, p, q, r, tol=1e-13, max_it=500):
        """Maximise the concave dual over lam >= 0 by projected Newton steps
        damped in the Levenberg-Marquardt way: the step (-H_FF + mu I)^-1 g_F
        on the free set F = {lam_i > 0 or g_i > 0} is taken only if the dual
        value does not drop (and the projected gradient shrinks when the value
        is flat to rounding); mu falls tenfold after a taken step and rises
        tenfold after a refused one.  The damping matters where every x_j
        sits on its box and the dual is piecewise linear.  Returns
        (x, y, lam, iterations)."""
        m = self.m
        lam = np.zeros(m)
        W, g, H, x, y = self.dual(lam, low, upp, alpha, beta, p, q, r)
        scale = 1.0 + np.abs(r).max()

        def proj_grad(lam, g):
            return np.abs(np.where(lam > 0, g, np.maximum(g, 0.0))).max()

        pgn = proj_grad(lam, g)
        mu = 1e-10 * (1.0 + np.trace(-H) / m)
        for it in range(max_it):
            if pgn <= tol * scale:
                return x, y, lam, it
            F = (lam > 0) | (g > 0)
            A = -H[np.ix_(F, F)]
            taken = False
            for _ in range(100):
                d = np.zeros(m)
                d[F] = np.linalg.solve(A + mu * np.eye(A.shape[0]), g[F])
                lt = np.maximum(0.0, lam + d)
                Wt, gt, Ht, xt, yt = self.dual(lt, low, upp, alpha, beta, p, q, r)
                pgt = proj_grad(lt, gt)
                if Wt > W or (Wt >= W - 1e-15 * abs(W) and pgt < pgn):
                    taken = True
                    break
                mu *= 10.0
            if not taken:
                return x, y, lam, it
            lam, W, g, H, x, y, pgn = lt, Wt, gt, Ht, xt, yt, pgt
            mu = max(mu * 0.1, 1e-300)
        return x, y, lam, max_it

    def update(self, x, f0, df0, fval, dfdx):
        """One MMA step from x; f0, df0 (n,): objective and gradient; fval (m,),
        dfdx (m, n): constraints f_i(x) <= 0 and their gradients.
        Returns the new x and a dict of diagnostics."""
        x = np.asarray(x, dtype=np.float64)
        dx = self.xmax - self.xmin
        low, upp, alpha, beta = self.asymptotes(x)
        grad = np.vstack([np.asarray(df0, dtype=np.float64)[None, :], np.atleast_2d(dfdx)])
        fv = np.concatenate(([float(f0)], np.asarray(fval, dtype=np.float64)))
        p, q, r = self.coefficients(x, low, upp, dx, fv, grad)
        xn, y, lam, its = self.solve_subproblem(low, upp, alpha, beta, p, q, r)
        self.xold2 = self.xold1
        self.xold1 = x.copy()
        self.low, self.upp = low, upp
        self.it += 1
        return xn, dict(low=low, upp=upp, alpha=alpha, beta=beta, p=p, q=q, r=r, y=y, lam=lam,
                        dual_iterations=its)


# ------------------------------------------------------------ design problems
def volume(x):
    """Volume fraction V(x) / |Omega_h| (unit elements)."""
    return float(np.mean(x))


def p1_functions(J, dJ, lam, dlam, x, J0, lam_bar, vol_frac, alpha=0.99):
    """Problem P1 (Sec. 3) in MMA form, all with respect to the physical
    densities x: objective J / J0; constraints V/(f_bar |Omega|) - 1 and the
    bound formulation of reading (b).  Returns (f0, df0, fval, dfdx)."""
    m = x.size
    g_b, dg_b = bound_constraints(lam, dlam.T, lam_bar, alpha)
    fval = np.concatenate(([volume(x) / vol_frac - 1.0], g_b))
    dfdx = np.vstack([np.full((1, m), 1.0 / (m * vol_frac)), dg_b])
    return J / J0, np.asarray(dJ, dtype=np.float64) / J0, fval, dfdx



def p2_functions(J, dJ, lam, dlam, x, J_max, lam_bar, alpha=0.99):
    """Problem P2 (Sec. 6) in MMA form, with respect to the physical
    densities x: objective V / |Omega| (the volume fraction); constraints
    J / J_max - 1 (J_max = 6 times the fully solid design's compliance in the
    paper) and the bound formulation of reading (b).
    Returns (f0, df0, fval, dfdx)."""
    m = x.size
    g_b, dg_b = bound_constraints(lam, dlam.T, lam_bar, alpha)
    fval = np.concatenate(([J / J_max - 1.0], g_b))
    dfdx = np.vstack([np.asarray(dJ, dtype=np.float64)[None, :] / J_max, dg_b])
    return volume(x), np.full(m, 1.0 / m), fval, dfdx

def p1_step(nel, xhat, F, fixed, mat, ell, q, nb, rmin, eta, beta, J0, lam_bar, vol_frac, mma, alpha=0.99):
    """One design step of problem P1 (Sec. 3) on the design variables xhat:
    density filter and projection (Sec. 2), the analysis of Sec. 2.1 with q
    modes from eigen level ell, compliance and buckling sensitivities of the
    lowest nb factors, the bound formulation, the chain rule back to xhat and
    one MMA update.  ``mat.p`` is the current SIMP exponent (continuation is
    the caller's).  Returns (xhat_new, diagnostics)."""
    from . import design, lba, sens
    xt = design.filter_density(nel, xhat, rmin)
    x = design.project(xt, eta, beta)
    an = lba.analysis(nel, x, F, fixed, mat, ell, q)
    J = float(an["J"][0])
    buck = an["buck"]
    lam = buck.lam[:nb]
    dJ = sens.compliance_sensitivity(nel, x, an["U"][:, :1], mat)[:, 0]
    dlam, _ = sens.buckling_sensitivity(nel, x, an["u"], lam, buck.phi[:, :nb], fixed, mat, an["solver"])
    f0, df0, fval, dfdx = p1_functions(J, dJ, lam, dlam, x, J0, lam_bar, vol_frac, alpha)
    cols = np.vstack([df0[None, :], dfdx]).T                  # (m, 1 + 1 + nb), x-space
    dhat = design.chain_rule(nel, xt, rmin, eta, beta, cols)  # xhat-space
    xnew, info = mma.update(xhat, f0, dhat[:, 0], fval, dhat[:, 1:].T)
    info.update(J=J, lam=buck.lam.copy(), x=x, xtilde=xt, f0=f0, fval=fval, grad_hat=dhat, grad_x=cols)
    return xnew, info


def p2_step(nel, xhat, F, fixed, mat, ell, q, nb, rmin, eta, beta, J_max, lam_bar, mma, alpha=0.99):
    """One design step of problem P2 (Sec. 6): as ``p1_step`` with the volume
    fraction as objective and the compliance bound J <= J_max as the first
    constraint.  Returns (xhat_new, diagnostics)."""
    from . import design, lba, sens
    xt = design.filter_density(nel, xhat, rmin)
    x = design.project(xt, eta, beta)
    an = lba.analysis(nel, x, F, fixed, mat, ell, q)
    J = float(an["J"][0])
    buck = an["buck"]
    lam = buck.lam[:nb]
    dJ = sens.compliance_sensitivity(nel, x, an["U"][:, :1], mat)[:, 0]
    dlam, _ = sens.buckling_sensitivity(nel, x, an["u"], lam, buck.phi[:, :nb], fixed, mat, an["solver"])
    f0, df0, fval, dfdx = p2_functions(J, dJ, lam, dlam, x, J_max, lam_bar, alpha)
    cols = np.vstack([df0[None, :], dfdx]).T
    dhat = design.chain_rule(nel, xt, rmin, eta, beta, cols)
    xnew, info = mma.update(xhat, f0, dhat[:, 0], fval, dhat[:, 1:].T)
    info.update(J=J, lam=buck.lam.copy(), x=x, xtilde=xt, f0=f0, fval=fval, grad_hat=dhat, grad_x=cols)
    return xnew, info
