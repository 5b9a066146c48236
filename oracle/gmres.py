"""Oracle: right-preconditioned restarted GMRES(m), modified Gram-Schmidt, Givens.

The paper solves every Newton tangent system with preconditioned GMRES (§1;
§2 "Numerical approximation", eq. "tangent problem"). It does not state the
side, the orthogonalisation or the norm; the reading used throughout this
project is: right preconditioning (so the residual that is monitored is the
true, unpreconditioned 2-norm residual), x0 = 0, modified Gram-Schmidt,
stopping when the least-squares residual estimate drops below rtol * ||b||,
confirmed by the true residual (a failed confirmation restarts). The iteration
count is the number of Arnoldi steps (= preconditioner applications inside the
Krylov loop) summed over restarts.

Test infrastructure only; see the package docstring.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    restarts: int
    converged: bool
    rel_res_true: float
    rel_res_est: float
    history: list


def gmres(A, M, b: np.ndarray, rtol: float = 1e-8, restart: int = 30, max_it: int = 1000) -> GmresResult:
    """Solve A x = b with right preconditioner M (callables v -> A v, v -> M^-1 v)."""
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return GmresResult(x, 0, 0, True, 0.0, 0.0, hist)
    its = 0
    restarts = 0
    r = b - A(x)
    est = np.linalg.norm(r)
    while True:
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            return GmresResult(x, its, restarts, True, beta / bnorm, est / bnorm, hist)
        if its >= max_it:
            return GmresResult(x, its, restarts, False, beta / bnorm, est / bnorm, hist)
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            w = A(M(V[j]))
            its += 1
            for i in range(j + 1):               # modified Gram-Schmidt
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):                   # previous rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1])
            hist.append(est / bnorm)
            k = j + 1
            breakdown = np.linalg.norm(w) == 0.0
            if not breakdown:
                V[j + 1] = w / np.linalg.norm(w)
            if est <= rtol * bnorm or its >= max_it or breakdown:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):           # back substitution R y = g
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + M(V[:k].T @ y)
        r = b - A(x)
        restarts += 1
        if np.linalg.norm(r) > rtol * bnorm and its < max_it:
            continue
        beta = np.linalg.norm(r)
        return GmresResult(x, its, restarts - 1, beta <= rtol * bnorm, beta / bnorm, est / bnorm, hist)
