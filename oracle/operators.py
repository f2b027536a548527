"""Semi-discrete operators K for du/dt = K u on the unit cube (oracle, test infrastructure).

Heat: the paper's heat test uses second-order central differences on [0,1]^3
with zero Dirichlet boundaries (Section "Heat equation").  Here K = kappa * Lap_h.
Advection-diffusion: K = nu * Lap_h - sum_d b_d D_d with D_d the first-order
upwind difference along axis d (backward when b_d >= 0, forward when b_d < 0)
and periodic wrap (the paper's advection boundary, Section "Advection equation").
Central advection(-diffusion), kind 2: D_d the second-order central difference
(u_{i+1} - u_{i-1}) / (2h), the paper's discretisation of its advection test (Section
"Test cases": second-order central stencils; the 1-D factor Tridiag(-1, 0, 1) / (2h) with
periodic corners of Section "Advection equation").

Grid spacing (reading of the paper's h = 1/(n-1), which counts boundary
nodes): Dirichlet uses n interior nodes and h = 1/(n+1); periodic uses
h = 1/n.  Unknowns are ordered x fastest, x_{ijk} = x[i + nx j + nx ny k]
(Section "Implementation of the Mixed-precision Runge--Kutta methods"), so the
3-D operator is the Kronecker sum I(x)I(x)Kx + I(x)Ky(x)I + Kz(x)I(x)I, the
same structure as the preconditioner form, eq. (preconbasic).

Pins (tests/test_oracle_operators.py): sine-mode eigenpairs (Dirichlet),
DFT eigenvalues (periodic), nnz counts, zero row sums (periodic), and a
brute-force pointwise stencil loop on tiny grids.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DIRICHLET = 0
PERIODIC = 1


def spacing(n: int, bc: int) -> float:
    """Grid spacing along an axis with n unknowns."""
    return 1.0 / (n + 1) if bc == DIRICHLET else 1.0 / n


def second_difference_1d(n: int, bc: int) -> sp.csr_matrix:
    """Unscaled 1-D second difference u_{i-1} - 2 u_i + u_{i+1}."""
    T = sp.lil_matrix((n, n))
    for i in range(n):
        T[i, i] += -2.0
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                T[i, j] += 1.0
            elif bc == PERIODIC:
                T[i, j % n] += 1.0
    return T.tocsr()


def upwind_difference_1d(n: int, bc: int, direction_positive: bool) -> sp.csr_matrix:
    """Unscaled 1-D first-order upwind difference.

    direction_positive: backward difference u_i - u_{i-1} (velocity >= 0);
    otherwise forward difference u_{i+1} - u_i (velocity < 0).
    """
    D = sp.lil_matrix((n, n))
    for i in range(n):
        if direction_positive:
            D[i, i] += 1.0
            j = i - 1
            if j >= 0:
                D[i, j] += -1.0
            elif bc == PERIODIC:
                D[i, j % n] += -1.0
        else:
            D[i, i] += -1.0
            j = i + 1
            if j < n:
                D[i, j] += 1.0
            elif bc == PERIODIC:
                D[i, j % n] += 1.0
    return D.tocsr()


def central_difference_1d(n: int, bc: int) -> sp.csr_matrix:
    """Unscaled 1-D central difference (u_{i+1} - u_{i-1}) / 2 (periodic wrap or zero ends)."""
    D = sp.lil_matrix((n, n))
    for i in range(n):
        for j, w in ((i + 1, 0.5), (i - 1, -0.5)):
            if 0 <= j < n:
                D[i, j] += w
            elif bc == PERIODIC:
                D[i, j % n] += w
    return D.tocsr()


def kron_sum(Kx, Ky, Kz) -> sp.csr_matrix:
    """I (x) I (x) Kx + I (x) Ky (x) I + Kz (x) I (x) I for x-fastest ordering."""
    nx, ny, nz = Kx.shape[0], Ky.shape[0], Kz.shape[0]
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(Iz, sp.kron(Iy, Kx)) + sp.kron(Iz, sp.kron(Ky, Ix))
            + sp.kron(Kz, sp.kron(Iy, Ix))).tocsr()


def laplacian(shape, bc: int) -> sp.csr_matrix:
    """7-point Lap_h on a grid of shape (nx, ny, nz)."""
    nx, ny, nz = shape
    T = [second_difference_1d(n, bc) / spacing(n, bc) ** 2 for n in (nx, ny, nz)]
    return kron_sum(*T)


def heat_operator(shape, bc: int, kappa: float) -> sp.csr_matrix:
    """K = kappa Lap_h (Section "Heat equation"; unforced)."""
    K = (kappa * laplacian(shape, bc)).tocsr()
    K.sum_duplicates()
    K.eliminate_zeros()
    return K


def advdiff_operator(shape, bc: int, nu: float, b, central: bool = False) -> sp.csr_matrix:
    """K = nu Lap_h - sum_d b_d D_d, D_d upwind (or central)."""
    nx, ny, nz = shape
    Z = [sp.csr_matrix((n, n)) for n in (nx, ny, nz)]
    K = nu * laplacian(shape, bc)
    for d, n in enumerate((nx, ny, nz)):
        if b[d] == 0.0:
            continue
        D1 = (central_difference_1d(n, bc) if central
              else upwind_difference_1d(n, bc, b[d] >= 0.0)) / spacing(n, bc)
        facs = list(Z)
        facs[d] = D1
        # kron_sum with only axis d non-zero
        K = K - b[d] * kron_sum(*facs)
    K = K.tocsr()
    K.sum_duplicates()
    K.eliminate_zeros()
    return K


def operator(shape, bc: int, kind: int, diff: float, b=(0.0, 0.0, 0.0)) -> sp.csr_matrix:
    """Dispatch: kind 0 = heat (kappa = diff), kind 1 = upwind advection-diffusion, kind 2 =
    central advection-diffusion (nu = diff)."""
    if kind == 0:
        return heat_operator(shape, bc, diff)
    return advdiff_operator(shape, bc, diff, b, central=kind == 2)


def stage_matrix(K: sp.csr_matrix, sigma: float) -> sp.csr_matrix:
    """M_sigma = I - sigma K, the implicit stage system of eq. (corelinear) in the sign
    convention y = rhs + sigma K y (sigma = tau a_ii)."""
    return (sp.identity(K.shape[0], format='csr') - sigma * K).tocsr()
