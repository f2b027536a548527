"""DIRK steps for a semi-linear f with a pointwise polynomial reaction (oracle, test infrastructure).

The paper integrates linear problems du/dt = K u and names non-linear equations as the next
setting (Section "Summary and conclusions"); an implicit Runge--Kutta stage then is a non-linear
system (Section "Runge--Kutta methods and mixed-precision").  The problem class here is

    du/dt = f(u) = K u + g + R(u),   R(u)_p = r1 u_p + r2 u_p^2 + r3 u_p^3   (pointwise),

with K the operator of operators.py and g an optional constant forcing.  One step is eq. (RKstep)
with the full tableau A: stage i solves the non-linear system

    y_i - sigma f(y_i) = rhs_i,   sigma = tau a_ii,   rhs_i = u_n + tau sum_{j<i} a_ij k_j,

and k_i = f(y_i).  The oracle solves each stage by Newton's method in float64 with the exact
Jacobian I - sigma (K + diag(R'(y))), from the start value rhs_i, until the update is below
1e-15 relative (at most 30 iterations; failing that it raises).  Each Newton system is solved
by a sparse LU ('splu', small grids) or by the oracle's own GMRES with block-Jacobi(8) to
relative residual 1e-14 ('gmres', grids where the LU fill makes a factorisation per iteration
too slow).

The scalar form (scalar_integrate) is the same method for y' = lam y + R(y): the 3-D problem
with a spatially constant state on a periodic grid reduces to it, because K maps constants to 0.

Pins (tests/test_oracle_nonlinear.py): R = 0 reproduces the linear oracle; the two Newton
solvers agree; the scalar form
against the closed-form solutions of the Bernoulli equation y' = r1 y + r2 y^2 and of
y' = r1 y + r3 y^3 with the tableau's convergence order on dt halving; a constant periodic state
reproduces the scalar form at every point; each stage's residual is at rounding level and
Newton converges quadratically (few iterations); a small 3-D grid converges at the tableau's
order towards a tightly solved method-of-lines reference.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov

NEWTON_TOL = 1e-15
NEWTON_MAXIT = 30


def reaction(u, r):
    """R(u) = r1 u + r2 u^2 + r3 u^3, elementwise; r = (r1, r2, r3)."""
    r1, r2, r3 = r
    return r1 * u + r2 * u * u + r3 * u * u * u


def reaction_derivative(u, r):
    """R'(u) = r1 + 2 r2 u + 3 r3 u^2, elementwise."""
    r1, r2, r3 = r
    return r1 + 2.0 * r2 * u + 3.0 * r3 * u * u


def rhs_function(K, g, r):
    """f(y) = K y + g + R(y) of the semi-linear problem."""
    def f(y):
        out = K @ y + reaction(y, r)
        return out if g is None else out + g
    return f


def _newton_solve(J, b, method: str):
    if method == 'splu':
        return spla.splu(J.tocsc()).solve(b)
    inv = krylov.block_jacobi_inverses(J, 8)
    d, _, _ = krylov.gmres(J, b, lambda v: krylov.block_jacobi_apply(inv, v, 8), restart=30,
                           rtol=1e-14)
    return d


def newton_stage(K, sigma: float, rhs: np.ndarray, g, r, stats=None,
                 method: str = 'splu') -> np.ndarray:
    """Solves y - sigma f(y) = rhs by Newton's method with the exact Jacobian."""
    f = rhs_function(K, g, r)
    n = rhs.size
    eye = sp.identity(n, format='csr')
    y = rhs.copy()
    for it in range(1, NEWTON_MAXIT + 1):
        F = y - sigma * f(y) - rhs
        J = (eye - sigma * (K + sp.diags(reaction_derivative(y, r)))).tocsr()
        d = _newton_solve(J, -F, method)
        y = y + d
        if np.linalg.norm(d) <= NEWTON_TOL * max(np.linalg.norm(y), 1e-300):
            if stats is not None:
                stats.append(it)
            return y
    raise RuntimeError('Newton did not converge in the stage solve')


def dirk_step(K, u: np.ndarray, tau: float, tab, r, g=None, stats=None,
              method: str = 'splu') -> np.ndarray:
    """One step of eq. (RKstep) for du/dt = K u + g + R(u) with the full tableau A."""
    A, b = tab.A, tab.b
    f = rhs_function(K, g, r)
    ks = []
    for i in range(tab.s):
        rhs = u.copy()
        for j in range(i):
            if A[i, j] != 0.0:
                rhs += tau * A[i, j] * ks[j]
        y = newton_stage(K, tau * A[i, i], rhs, g, r, stats, method) if A[i, i] != 0.0 else rhs
        ks.append(f(y))
    out = u.copy()
    for i in range(tab.s):
        if b[i] != 0.0:
            out += tau * b[i] * ks[i]
    return out


def integrate(K, u0: np.ndarray, tau: float, nsteps: int, tab, r, g=None,
              stats=None, method: str = 'splu') -> np.ndarray:
    """nsteps steps from u0 (flat, lexicographic); stats collects Newton iteration counts;
    method: the Newton systems' solver, 'splu' or 'gmres'."""
    u = np.asarray(u0, dtype=np.float64).ravel().copy()
    K = sp.csr_matrix(K)
    gf = None if g is None else np.asarray(g, dtype=np.float64).ravel()
    for _ in range(nsteps):
        u = dirk_step(K, u, tau, tab, r, g=gf, stats=stats, method=method)
    return u


def stage_residuals(K, u: np.ndarray, tau: float, tab, r, g=None):
    """Relative residuals ||y - sigma f(y) - rhs|| / ||rhs|| of the implicit stages of one step."""
    A = tab.A
    K = sp.csr_matrix(K)
    f = rhs_function(K, g, r)
    ks, out = [], []
    for i in range(tab.s):
        rhs = u.copy()
        for j in range(i):
            if A[i, j] != 0.0:
                rhs += tau * A[i, j] * ks[j]
        if A[i, i] != 0.0:
            y = newton_stage(K, tau * A[i, i], rhs, g, r)
            out.append(float(np.linalg.norm(y - tau * A[i, i] * f(y) - rhs) / np.linalg.norm(rhs)))
        else:
            y = rhs
        ks.append(f(y))
    return out


def scalar_integrate(y0: float, tau: float, nsteps: int, tab, r, lam: float = 0.0,
                     g: float = 0.0) -> float:
    """The same DIRK for the scalar y' = lam y + g + R(y), scalar Newton per stage."""
    A, b = tab.A, tab.b

    def f(y):
        return lam * y + g + reaction(y, r)

    y = float(y0)
    for _ in range(nsteps):
        ks = []
        for i in range(tab.s):
            rhs = y
            for j in range(i):
                rhs += tau * A[i, j] * ks[j]
            z = rhs
            sigma = tau * A[i, i]
            if sigma != 0.0:
                for _it in range(NEWTON_MAXIT):
                    F = z - sigma * f(z) - rhs
                    d = -F / (1.0 - sigma * (lam + reaction_derivative(z, r)))
                    z += d
                    if abs(d) <= NEWTON_TOL * max(abs(z), 1e-300):
                        break
                else:
                    raise RuntimeError('scalar Newton did not converge')
            ks.append(f(z))
        for i in range(tab.s):
            y += tau * b[i] * ks[i]
    return y


def bernoulli_exact(y0: float, r1: float, r2: float, t: float) -> float:
    """Solution of y' = r1 y + r2 y^2 (r1 != 0): 1/y solves v' = -r1 v - r2."""
    v = (1.0 / y0 + r2 / r1) * np.exp(-r1 * t) - r2 / r1
    return 1.0 / v


def cubic_exact(y0: float, r1: float, r3: float, t: float) -> float:
    """Solution of y' = r1 y + r3 y^3 (r1 != 0, y0 > 0): 1/y^2 solves w' = -2 r1 w - 2 r3."""
    w = (1.0 / (y0 * y0) + r3 / r1) * np.exp(-2.0 * r1 * t) - r3 / r1
    return 1.0 / np.sqrt(w)
