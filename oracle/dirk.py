"""The diagonally implicit Runge--Kutta step with exact stage solves (oracle, test infrastructure).

eq. (RKstep): u_{n+1} = u_n + tau sum_i b_i k_i, k_i = f(u_n + tau sum_j a_ij k_j),
with lower-triangular A (a DIRK, Section "Runge--Kutta methods and mixed-precision").
For the linear f(u) = K u, stage i with a_ii != 0 is the linear system
    (I - tau a_ii K) y_i = rhs_i,   rhs_i = u_n + tau sum_{j<i} a_ij k_j,
(eq. (corelinear), written in the sign convention y = rhs + sigma K y), and
k_i = K y_i is the explicit evaluation of f (the high-precision correction of
Section "The implicit midpoint method and explicit corrector steps").
In exact arithmetic f^eps = f, so the A^(h)/A^(eps) split is immaterial: the
oracle applies the full A.

Stage solvers: 'dense' (LU of the dense stage matrix, N <= ~4096), 'splu'
(sparse LU), 'cg' / 'gmres' (the oracle's own FP64 Krylov to rtol 1e-13,
block-Jacobi preconditioned, or by the fast-diagonalisation inverse of eq. Pinvform).
Pins: closed-form modal evolution R(tau lambda)^N, dt-halving order, agreement
between the three solvers (tests/test_oracle_dirk.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fdm, krylov
from .operators import stage_matrix


class StageSolver:
    """Solves (I - sigma K) y = rhs; factorizations are cached per sigma.

    Krylov methods take block-Jacobi(block) as preconditioner, or with fdm_problem =
    (shape, bc, kind, diff, b) of K the fast-diagonalisation inverse of eq. Pinvform."""

    def __init__(self, K: sp.csr_matrix, method: str = 'splu', rtol: float = 1e-13,
                 block: int = 8, restart: int = 30, fdm_problem=None):
        self.K = K.tocsr()
        self.method = method
        self.rtol = rtol
        self.block = block
        self.restart = restart
        self.fdm_problem = fdm_problem
        self._cache = {}
        self.iterations = []

    def _factor(self, sigma: float):
        if sigma in self._cache:
            return self._cache[sigma]
        M = stage_matrix(self.K, sigma)
        if self.method == 'dense':
            f = ('dense', sla.lu_factor(M.toarray()))
        elif self.method == 'splu':
            f = ('splu', spla.splu(M.tocsc()))
        elif self.fdm_problem is not None:
            f = (self.method, (M, fdm.FDM(*self.fdm_problem, sigma)))
        else:
            inv = krylov.block_jacobi_inverses(M, self.block)
            f = (self.method, (M, inv))
        self._cache[sigma] = f
        return f

    def __call__(self, sigma: float, rhs: np.ndarray) -> np.ndarray:
        kind, f = self._factor(sigma)
        if kind == 'dense':
            return sla.lu_solve(f, rhs)
        if kind == 'splu':
            return f.solve(rhs)
        M, inv = f
        if self.fdm_problem is not None:
            prec = inv.apply
        else:
            prec = lambda r: krylov.block_jacobi_apply(inv, r, self.block)
        if kind == 'cg':
            y, it, _ = krylov.cg(M, rhs, prec, rtol=self.rtol, x0=rhs.copy())
        else:
            y, it, _ = krylov.gmres(M, rhs, prec, restart=self.restart, rtol=self.rtol,
                                    x0=rhs.copy())
        self.iterations.append(it)
        return y


def dirk_step(K, u: np.ndarray, tau: float, tab, solve, stage_hook=None, g=None) -> np.ndarray:
    """One step of eq. (RKstep) for du/dt = K u (+ g, a constant forcing) with the full tableau A.

    With forcing, f(y) = K y + g: stage i solves (I - tau a_ii K) y_i = rhs_i + tau a_ii g
    and k_i = K y_i + g.

    stage_hook(i, y) -> y, if given, replaces each implicit stage solution (used
    to model an inexact low-precision solve, e.g. for the corrector-divergence
    criterion of Section "The implicit midpoint method and explicit corrector steps")."""
    A, b = tab.A, tab.b
    ks = []
    for i in range(tab.s):
        rhs = u.copy()
        for j in range(i):
            if A[i, j] != 0.0:
                rhs += tau * A[i, j] * ks[j]
        if A[i, i] != 0.0:
            y = solve(tau * A[i, i], rhs if g is None else rhs + tau * A[i, i] * g)
            if stage_hook is not None:
                y = stage_hook(i, y)
        else:
            y = rhs
        ks.append(K @ y if g is None else K @ y + g)
    out = u.copy()
    for i in range(tab.s):
        if b[i] != 0.0:
            out += tau * b[i] * ks[i]
    return out


def integrate(K, u0: np.ndarray, tau: float, nsteps: int, tab, method: str = 'splu',
              g=None, **solver_kw) -> np.ndarray:
    """nsteps DIRK steps from u0 (a flat lexicographic vector), forcing g (flat) if given."""
    solve = StageSolver(K, method, **solver_kw)
    u = np.asarray(u0, dtype=np.float64).ravel().copy()
    gf = None if g is None else np.asarray(g, dtype=np.float64).ravel()
    for _ in range(nsteps):
        u = dirk_step(K, u, tau, tab, solve, g=gf)
    return u


def relative_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_2 / ||ref||_2 over all grid values."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
