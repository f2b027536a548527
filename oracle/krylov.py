"""Plain FP64 Krylov solvers and block-Jacobi for the stage systems (oracle, test infrastructure).

The paper solves each implicit stage system, eq. (corelinear), with a
preconditioned Krylov method: CG for the SPD heat systems and GMRES for the
nonsymmetric advection systems (Section "Problem setting and solver design"),
stopping when the absolute or the relative residual falls below the tolerance
(Section "Linear solvers and setup of the numerical experiments").
These are the textbook algorithms, written plainly; they are used where a
sparse LU is too slow, and as the reference for solver-level checks.

Block-Jacobi (a Ginkgo preconditioner named in the Introduction, used here in
its fixed-precision form): consecutive blocks of `block` rows in lexicographic
order, the last one short when N is not a multiple; each diagonal block of
M is inverted densely.

Pins: dense direct solves on tiny systems, an eigenvector right-hand side
converging in one CG iteration, block size >= N converging in one iteration.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def block_jacobi_inverses(M: sp.csr_matrix, block: int):
    """List of dense inverses of the diagonal blocks M[I_b, I_b]."""
    N = M.shape[0]
    M = M.tocsr()
    out = []
    for start in range(0, N, block):
        stop = min(start + block, N)
        D = M[start:stop, start:stop].toarray()
        out.append(np.linalg.inv(D))
    return out


def block_jacobi_apply(inverses, r: np.ndarray, block: int) -> np.ndarray:
    """z_b = D_b^{-1} r_b for every block b."""
    z = np.empty_like(r)
    for bi, Dinv in enumerate(inverses):
        start = bi * block
        stop = start + Dinv.shape[0]
        z[start:stop] = Dinv @ r[start:stop]
    return z


def cg(M, b, precond=None, rtol=1e-13, atol=0.0, maxit=10000, x0=None):
    """Preconditioned conjugate gradients; stop when ||r|| <= max(rtol ||b||, atol).

    Returns (x, iterations, final residual norm)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - M @ x
    bnorm = np.linalg.norm(b)
    tol = max(rtol * bnorm, atol)
    if np.linalg.norm(r) <= tol:
        return x, 0, np.linalg.norm(r)
    z = precond(r) if precond is not None else r.copy()
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = M @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = np.linalg.norm(r)
        if rn <= tol:
            break
        z = precond(r) if precond is not None else r.copy()
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, np.linalg.norm(b - M @ x)


def gmres(M, b, precond=None, restart=30, rtol=1e-13, atol=0.0, maxit=10000, x0=None):
    """Right-preconditioned restarted GMRES(m), modified Gram-Schmidt Arnoldi,
    Givens rotations; stop when the true residual estimate
    <= max(rtol ||b||, atol).  Returns (x, iterations, final residual norm)."""
    P = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    tol = max(rtol * bnorm, atol)
    it = 0
    while True:
        r = b - M @ x
        beta = np.linalg.norm(r)
        if beta <= tol or it >= maxit:
            return x, it, beta
        m = restart
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            w = M @ P(V[j])
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
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
            it += 1
            j_end = j + 1
            if abs(g[j + 1]) <= tol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + P(V[:j_end].T @ y)
