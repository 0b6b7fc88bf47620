"""FP64 reference of restarted flexible GMRES (TEST INFRASTRUCTURE ONLY).

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
