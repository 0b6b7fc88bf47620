"""FP64 references of the Krylov methods that take a preconditioner which may change from one
application to the next (TEST INFRASTRUCTURE ONLY): restarted flexible GMRES and flexible
BiCGStab with the stall fallback of the learned preconditioner.

Restarted flexible GMRES.

The paper solves its Helmholtz problem with preconditioned BiCGStab (Sec. 2); a learned
preconditioner is not a fixed linear map, and the Krylov method that tolerates a preconditioner
that changes from one application to the next is flexible GMRES (Saad, SIAM J. Sci. Comput.
14 (1993)).  This is that textbook method, written out plainly:

    r0 = b - A x0,  beta = ||r0||,  v1 = r0 / beta
    for j = 1..m:   z_j = M_j(v_j),  w = A z_j,
                    h_ij = <w, v_i>, w -= h_ij v_i   (modified Gram-Schmidt, i = 1..j)
                    h_{j+1,j} = ||w||,  v_{j+1} = w / h_{j+1,j}
                    Givens rotations reduce H to upper triangular; |g_{j+1}| = ||b - A x_j||
    x = x0 + Z_k y_k with y_k the least-squares solution of min || beta e1 - H y ||
    restart from x until ||b - A x|| <= tol ||b|| or maxit inner steps.

M defaults to the exact column tridiagonal solve T^{-1} (``oracle.thomas``), the paper's
vertical line preconditioner.  ``history[k]`` is |g_{k+1}| / ||b|| after inner step k + 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle


@dataclass
class GmresInfo:
    iterations: int
    cycles: int
    status: int            # 0 converged, 1 maxit
    true_rel_residual: float
    history: np.ndarray


def fgmres(coef: np.ndarray, b: np.ndarray, x0: np.ndarray | None = None, tol: float = 1e-8, m: int = 30,
           maxit: int = 5000, precond=None):
    """Solve A x = b; returns (x, GmresInfo).  ``precond(j, v)`` may depend on the step j."""
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    if precond is None:
        precond = lambda j, v: oracle.thomas(coef, v)   # noqa: E731
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    nb = np.linalg.norm(b)
    hist, it, cycles = [], 0, 0
    if nb == 0.0:
        return np.zeros(n), GmresInfo(0, 0, 0, 0.0, np.zeros(0))
    while True:
        r = b - oracle.apply(coef, x)
        beta = np.linalg.norm(r)
        if beta <= tol * nb:
            return x, GmresInfo(it, cycles, 0, beta / nb, np.array(hist))
        if it >= maxit:
            return x, GmresInfo(it, cycles, 1, beta / nb, np.array(hist))
        cycles += 1
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = precond(it, V[j])
            w = oracle.apply(coef, Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
            rho = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / rho, H[j + 1, j] / rho) if rho > 0.0 else (1.0, 0.0)
            H[j, j], H[j + 1, j] = rho, 0.0
            g[j + 1], g[j] = -sn[j] * g[j], cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= tol * nb or it >= maxit or H[j + 1, j] == 0.0 and rho == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y


@dataclass
class FlexInfo:
    iterations: int
    restarts: int
    fallbacks: int         # switches from the given M to the fallback preconditioner
    status: int            # 0 converged, 1 maxit, 2 breakdown, 3 true residual stuck above tol
    true_rel_residual: float
    history: np.ndarray    # recursive relative residual after each iteration


def bicgstab_flex(coef: np.ndarray, b: np.ndarray, precond, x0: np.ndarray | None = None, tol: float = 1e-8,
                  maxit: int = 5000, fallback=None, stall_window: int = 20, eps_bd: float = 2.0 ** -52):
    """Right-preconditioned BiCGStab (van der Vorst 1992; the post-conditioned form of the
    paper's Sec. 2, Eq. 5, halted on the unpreconditioned residual of Sec. 3, Eq. 8-9) with a
    preconditioner ``precond(q)`` that may differ from call to call.  The recurrences are the
    fixed-M ones; what makes them flexible is that x is advanced with exactly the vectors
    p^ = M(p) and s^ = M(s) whose products v = A p^ and t = A s^ entered alpha and omega, so
    the recursive residual r stays b - A x.

    Steps of one iteration, as in the C oracle's BiCGStab (same operations, same order; inner
    products by the oracle's left-to-right sum):
        rho = <r^, r>;  beta = (rho / rho_prev)(alpha / omega);  p = r + beta (p - omega v)
        p^ = M(p);  v = A p^;  alpha = rho / <r^, v>;  s = r - alpha v
        stop with x += alpha p^ if ||s|| / ||b|| <= tol
        s^ = M(s);  t = A s^;  omega = <t, s> / <t, t>;  x += alpha p^ + omega s^;  r = s - omega t
    Breakdown guards (Sec. 4): |<r^, r>| or |<r^, v>| at most eps_bd times the product of the
    norms restarts the shadow space (r^ = r, p = v = 0, scalars 1); <t, t> = 0 or omega = 0 keeps
    the half step and restarts.  On convergence of the recursive residual the true residual is
    checked; up to three restarts from it, then status 3.

    Stall fallback (with ``fallback`` given, the learned preconditioner's rule): after each
    iteration that did not stop, with R the recursive relative residual, best the smallest R so
    far and an anchor that moves to R whenever R <= anchor / 2: when stall_window iterations
    pass without the anchor moving, or R > 1e3 best, or R is not finite, or the iteration broke
    down right after a restart, M becomes ``fallback`` for the rest of the solve and the
    iteration restarts from the true residual b - A x.  Without ``fallback`` a breakdown right
    after a restart ends the solve with status 2."""
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    M = precond
    nrm = lambda u: float(np.sqrt(oracle.dot(u, u)))   # noqa: E731
    hist, restarts, fallbacks, it = [], 0, 0, 0
    nb = nrm(b)
    if nb == 0.0:
        return np.zeros(n), FlexInfo(0, 0, 0, 0, 0.0, np.zeros(0))
    r = b - oracle.apply(coef, x)
    rnorm = nrm(r)
    if rnorm / nb <= tol:
        return x, FlexInfo(0, 0, 0, 0, rnorm / nb, np.zeros(0))
    status, gap, fresh, just_restarted = 1, 0, True, False
    best = anchor = rnorm / nb
    anchor_it = 0
    rho_prev = alpha = omega = 1.0
    rh = p = v = None
    rhnorm = 0.0

    def restart_from_true_residual():
        nonlocal r, rnorm
        r = b - oracle.apply(coef, x)
        rnorm = nrm(r)

    while it < maxit:
        if fresh:
            rh = r.copy()
            p = np.zeros(n)
            v = np.zeros(n)
            rho_prev = alpha = omega = 1.0
            rhnorm = nrm(rh)
            fresh = False
            just_restarted = True
        it += 1
        rho = oracle.dot(rh, r)
        if abs(rho) <= eps_bd * rhnorm * rnorm:
            rh = r.copy()
            p = np.zeros(n)
            v = np.zeros(n)
            rho_prev = alpha = omega = 1.0
            rhnorm = rnorm
            rho = oracle.dot(rh, r)
            restarts += 1
            just_restarted = True
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = M(p)
        v = oracle.apply(coef, ph)
        sigma = oracle.dot(rh, v)
        if abs(sigma) <= eps_bd * rhnorm * nrm(v):
            restarts += 1
            hist.append(rnorm / nb)
            if just_restarted:
                if fallback is None or M is fallback:
                    status = 2
                    break
                M = fallback               # breakdown right after a restart: hand over
                fallbacks += 1
                restarts += 1
                restart_from_true_residual()
            fresh = True
            continue
        just_restarted = False
        alpha = rho / sigma
        s = r - alpha * v
        snorm = nrm(s)
        if snorm / nb <= tol:
            x = x + alpha * ph
            hist.append(snorm / nb)
            status = 0
        else:
            sh = M(s)
            t = oracle.apply(coef, sh)
            tt, ts = oracle.dot(t, t), oracle.dot(t, s)
            if tt == 0.0 or ts == 0.0:
                x = x + alpha * ph
                r = s
                rnorm = snorm
                restarts += 1
                fresh = True
                hist.append(rnorm / nb)
                continue
            omega = ts / tt
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho_prev = rho
            rnorm = nrm(r)
            hist.append(rnorm / nb)
            if rnorm / nb <= tol:
                status = 0
        if status == 0:
            r64 = b - oracle.apply(coef, x)
            rt = nrm(r64)
            if rt / nb <= tol:
                return x, FlexInfo(it, restarts, fallbacks, 0, rt / nb, np.array(hist))
            if gap >= 3:
                return x, FlexInfo(it, restarts, fallbacks, 3, rt / nb, np.array(hist))
            gap += 1
            restarts += 1
            status = 1
            r, rnorm = r64, rt
            fresh = True
            continue
        if fallback is not None and M is not fallback:
            R = rnorm / nb
            best = min(best, R)
            if R <= 0.5 * anchor:
                anchor, anchor_it = R, it
            if it - anchor_it >= stall_window or R > 1e3 * best or not np.isfinite(R):
                M = fallback
                fallbacks += 1
                restarts += 1
                restart_from_true_residual()
                fresh = True
    true_rel = nrm(b - oracle.apply(coef, x)) / nb
    return x, FlexInfo(it, restarts, fallbacks, status, true_rel, np.array(hist))
