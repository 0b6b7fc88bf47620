"""The paper's mixed-precision BiCGStab, emulated on the CPU (TEST INFRASTRUCTURE ONLY).

Sec. 4 of the paper keeps the solution x in 64-bit and everything else of BiCGStab in 32-bit:
the residual r, the shadow residual r^, the search directions p, s, their preconditioned forms
p^ = M p, s^ = M s and the products v = A p^, t = A s^; the global sums (dot products) are
accumulated in 64-bit; the iteration restarts from the 64-bit true residual b - A x every 150
iterations; and there is no outer refinement.  Here each 32-bit vector is a float32 array: every
vector operation is evaluated in float64 from the float32 operands and rounded once to float32,
the operator in that precision uses the coefficients rounded to float32, the preconditioner
(the column tridiagonal solve, or the red-black line SOR) is applied in float64 to the float32
vector and rounded, and the dot products are float64 sums of the float32 values.  x and the
true residual use the float64 operator.

``vec_dtype=np.float64`` turns every rounding off: the iteration is then the FP64 BiCGStab of
``oracle.bicgstab`` step for step (the same breakdown restarts, half-step exit, true-residual
check and periodic restart), which is how this emulation is pinned.  ``x_dtype=np.float32``
also rounds the solution to 32 bits after every update: the all-32-bit solver the paper
compares with the 64-bit one in its toy model (Sec. 4, Fig. 1), pinned by its representation
floor (its true residual stalls at that of the exact solution rounded to float32).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle

EPS_BD = 2.0 ** -52


@dataclass
class MpInfo:
    status: int            # 0 converged, 1 iteration limit, 3 true residual stuck above tol
    iterations: int
    restarts: int
    true_rel_residual: float
    history: np.ndarray    # recursive relative residual after each iteration


def bicgstab_mp(coef: np.ndarray, b: np.ndarray, tol: float = 1e-4, maxit: int = 5000, restart_every: int = 150,
                precond: str = "tri", sor_sweeps: int = 3, sor_omega: float = 1.5, vec_dtype=np.float32,
                x_dtype=np.float64, trace=None):
    """Solve A x = b from x = 0; returns (x (float64), MpInfo).  ``x_dtype=np.float32`` rounds
    the solution to float32 after every update as well: the all-32-bit solver of the paper's
    toy-model comparison (Sec. 4, Fig. 1; pass restart_every=0 for no periodic restarts).
    ``trace(it, state)``, if given, sees the iteration's vectors (r, rh, p, ph, v, s, sh, t, x)
    after every full iteration."""
    vd = np.dtype(vec_dtype)
    xd = np.dtype(x_dtype)

    def xr(v):                        # the solution's storage precision
        return v if xd == np.float64 else v.astype(xd).astype(np.float64)
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    coef_lo = coef.astype(vd).astype(np.float64) if vd != np.float64 else coef

    def lo(v):                        # one rounding to the vector precision
        return np.asarray(v, dtype=np.float64).astype(vd)

    def hi(v):
        return v.astype(np.float64)

    def op_lo(v):                     # A in the vector precision
        return lo(oracle.apply(coef_lo, hi(v)))

    def pc(v):                        # M in the vector precision
        if precond == "tri":
            return lo(oracle.thomas(coef_lo, hi(v)))
        if precond == "sor":
            return lo(oracle.rbsor(coef_lo, hi(v), sweeps=sor_sweeps, omega=sor_omega))
        raise ValueError(precond)

    def dot(u, v):                    # 64-bit sums, in index order as the C oracle sums
        return oracle.dot(hi(u), hi(v))

    def nrm(u):
        return float(np.sqrt(dot(u, u)))

    x = np.zeros(n)
    hist = []
    restarts = 0
    nb = nrm(b)
    if nb == 0.0:
        return x, MpInfo(0, 0, 0, 0.0, np.array(hist))
    r = lo(b - oracle.apply(coef, x))
    rnorm = nrm(r)
    if rnorm / nb <= tol:
        return x, MpInfo(0, 0, 0, rnorm / nb, np.array(hist))
    it, gap, fresh, status = 0, 0, True, 1
    rho_prev = alpha = omega = 1.0
    rh = p = v = None
    rhnorm = 0.0
    true_rel = rnorm / nb
    while it < maxit:
        if fresh:
            rh = r.copy()
            p = np.zeros(n, dtype=vd)
            v = np.zeros(n, dtype=vd)
            rho_prev = alpha = omega = 1.0
            rhnorm = nrm(rh)
            fresh = False
        it += 1
        rho = dot(rh, r)
        if abs(rho) <= EPS_BD * rhnorm * rnorm:          # r^ orthogonal to r: new shadow space
            rh = r.copy()
            p = np.zeros(n, dtype=vd)
            v = np.zeros(n, dtype=vd)
            rho_prev = alpha = omega = 1.0
            rhnorm = rnorm
            rho = dot(rh, r)
            restarts += 1
        beta = (rho / rho_prev) * (alpha / omega)
        p = lo(hi(r) + beta * (hi(p) - omega * hi(v)))
        ph = pc(p)
        v = op_lo(ph)
        sigma = dot(rh, v)
        if abs(sigma) <= EPS_BD * rhnorm * nrm(v):
            restarts += 1
            fresh = True
            hist.append(rnorm / nb)
            continue
        alpha = rho / sigma
        s = lo(hi(r) - alpha * hi(v))
        snorm = nrm(s)
        if snorm / nb <= tol:                              # converged at the half step
            x = xr(x + alpha * hi(ph))
            hist.append(snorm / nb)
            status = 0
        else:
            sh = pc(s)
            t = op_lo(sh)
            tt, ts = dot(t, t), dot(t, s)
            if tt == 0.0 or ts == 0.0:
                x = xr(x + alpha * hi(ph))
                r = s
                rnorm = snorm
                restarts += 1
                fresh = True
                hist.append(rnorm / nb)
                continue
            omega = ts / tt
            x = xr(x + alpha * hi(ph) + omega * hi(sh))
            r = lo(hi(s) - omega * hi(t))
            rho_prev = rho
            rnorm = nrm(r)
            hist.append(rnorm / nb)
            if trace is not None:
                trace(it, dict(r=r, rh=rh, p=p, ph=ph, v=v, s=s, sh=sh, t=t, x=x))
            if rnorm / nb <= tol:
                status = 0
        if status == 0:                                    # check the 64-bit true residual
            r64 = b - oracle.apply(coef, x)
            true_rel = nrm(r64) / nb
            if true_rel <= tol:
                break
            if gap >= 3:
                status = 3
                break
            gap += 1
            restarts += 1
            status = 1
            r = lo(r64)
            rnorm = nrm(r)
            fresh = True
            continue
        if restart_every > 0 and it % restart_every == 0:  # periodic restart from b - A x
            r = lo(b - oracle.apply(coef, x))
            rnorm = nrm(r)
            restarts += 1
            fresh = True
    if status != 0:
        true_rel = nrm(b - oracle.apply(coef, x)) / nb
    return x, MpInfo(status, it, restarts, true_rel, np.array(hist))
