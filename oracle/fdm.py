"""Fast-diagonalisation preconditioner, FP64 (oracle; test infrastructure only).

The preconditioner of Section "Problem setting and solver design" (eq. preconbasic) is
P = I (x) I (x) A + I (x) B (x) I + C (x) I (x) I with n x n one-dimensional operators A, B, C
along x, y and z.  For a stage system (I - sigma K) y = rhs whose operator is a Kronecker sum
K = I (x) I (x) Kx + I (x) Ky (x) I + Kz (x) I (x) I (both operators of this repository are), the
paper's choice A = I - sigma Kx, B = -sigma Ky, C = -sigma Kz makes P the stage matrix itself,
so P^-1 is its exact inverse (Section "Test cases" gives these settings for the heat and
advection problems; the tensor kernels are in Section "Implementation of the Mixed-precision
Runge--Kutta methods").

Eq. Pinvform: with the spectral decompositions A = Q_A L_A Q_A^-1 (and B, C alike),
P^-1 = (Q_C (x) Q_B (x) Q_A) P_D^-1 (Q_C^-1 (x) Q_B^-1 (x) Q_A^-1),
P_D = I (x) I (x) L_A + I (x) L_B (x) I + L_C (x) I (x) I (diagonal), and by eq. TensorDecomp each
Kronecker factor is the product T_L T_M T_R of one-axis contractions, which in the paper's
0-based index notation (x_{ijk} = x[i + j nx + k nx ny]) read
    (T_R x)_{ijk} = sum_q Q_{iq} x_{qjk},  (T_M x)_{ijk} = sum_q Q_{jq} x_{iqk},
    (T_L x)_{ijk} = sum_q Q_{kq} x_{ijq}.
Every factor built here is a normal matrix (symmetric for the heat operator, circulant for the
periodic advection operators), so it has a unitary eigenbasis: the decompositions come from the
symmetric eigensolver (heat) or the complex Schur form A = Z T Z^H, whose triangular T is then
diagonal (checked; Q_A = Z, Q_A^-1 = Z^H).  A general eigensolver would also diagonalise these factors, but where pure
central advection repeats eigenvalues (the symbol sin(theta) takes each value twice) its bases
are ill-conditioned and their inverse loses digits; a non-normal factor (advection with
Dirichlet ends) is rejected rather than decomposed.  Arrays are held as (nz, ny, nx).

Pins (tests/test_oracle_fdm.py): P assembled from A, B, C equals the stage matrix; P^-1 r
equals a sparse direct solve to 1e-11 for every case, including pure central advection; the
bases are unitary; each contraction matches a brute-force loop on a non-cubic grid.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .operators import central_difference_1d, second_difference_1d, spacing, upwind_difference_1d


def one_d_factors(shape, bc: int, kind: int, diff: float, b=(0.0, 0.0, 0.0)):
    """Dense 1-D operators (Kx, Ky, Kz) whose Kronecker sum is the semi-discrete K (kind 1:
    upwind advection; kind 2: central, the factor Tridiag(-1, 0, 1) / (2h) with periodic corners
    of Section "Advection equation")."""
    out = []
    for d, n in enumerate(shape):
        h = spacing(n, bc)
        Kd = diff * second_difference_1d(n, bc).toarray() / h ** 2
        if kind == 1 and b[d] != 0.0:
            Kd = Kd - b[d] * upwind_difference_1d(n, bc, b[d] >= 0.0).toarray() / h
        elif kind == 2 and b[d] != 0.0:
            Kd = Kd - b[d] * central_difference_1d(n, bc).toarray() / h
        out.append(Kd)
    return tuple(out)


def preconditioner_factors(shape, bc: int, kind: int, diff: float, b, sigma: float):
    """A = I - sigma Kx, B = -sigma Ky, C = -sigma Kz (eq. preconbasic with the stage shift)."""
    Kx, Ky, Kz = one_d_factors(shape, bc, kind, diff, b)
    A = np.eye(shape[0]) - sigma * Kx
    return A, -sigma * Ky, -sigma * Kz


def assemble(A, B, C) -> sp.csr_matrix:
    """P of eq. preconbasic for x-fastest ordering."""
    Ia, Ib, Ic = (sp.identity(M.shape[0]) for M in (A, B, C))
    P = (sp.kron(Ic, sp.kron(Ib, sp.csr_matrix(A))) + sp.kron(Ic, sp.kron(sp.csr_matrix(B), Ia))
         + sp.kron(sp.csr_matrix(C), sp.kron(Ib, Ia)))
    return P.tocsr()


def unitary_eigenbasis(M):
    """(lam, Z) with M = Z diag(lam) Z^H, Z unitary, for a normal matrix M: the symmetric
    eigensolver for a symmetric M (real orthogonal Z), else the complex Schur form.  Raises
    ValueError when the Schur form is not diagonal (M not normal)."""
    M = np.asarray(M)
    if np.isrealobj(M) and np.array_equal(M, M.T):
        return sla.eigh(M)
    T, Z = sla.schur(M.astype(np.complex128), output='complex')
    scale = max(float(np.abs(M).max()), np.finfo(float).tiny)
    off = float(np.abs(np.triu(T, 1)).max(initial=0.0))
    if off > 1e-12 * scale:
        raise ValueError(f'factor is not normal (Schur off-diagonal {off / scale:.1e} of its '
                         'largest entry): no unitary eigenbasis')
    return np.diag(T).copy(), Z


def t_r(Q, x):
    """(T_R x)_{ijk} = sum_q Q_{iq} x_{qjk}; x has shape (nz, ny, nx)."""
    return np.einsum('iq,kjq->kji', Q, x)


def t_m(Q, x):
    """(T_M x)_{ijk} = sum_q Q_{jq} x_{iqk}."""
    return np.einsum('jq,kqi->kji', Q, x)


def t_l(Q, x):
    """(T_L x)_{ijk} = sum_q Q_{kq} x_{ijq}."""
    return np.einsum('kq,qji->kji', Q, x)


class FDM:
    """Inverse action of P (eq. Pinvform) for one stage shift sigma."""

    def __init__(self, shape, bc: int, kind: int, diff: float, b, sigma: float):
        self.shape = tuple(shape)
        A, B, C = preconditioner_factors(shape, bc, kind, diff, b, sigma)
        self.factors = (A, B, C)
        self.lam, self.Q, self.Qinv = [], [], []
        for M in (A, B, C):
            w, Q = unitary_eigenbasis(M)
            self.lam.append(w)
            self.Q.append(Q)
            self.Qinv.append(Q.conj().T)
        la, lb, lc = self.lam
        self.PD = lc[:, None, None] + lb[None, :, None] + la[None, None, :]

    def apply(self, r: np.ndarray) -> np.ndarray:
        nx, ny, nz = self.shape
        x = np.asarray(r, dtype=np.float64).reshape(nz, ny, nx)
        qa, qb, qc = self.Q
        ia, ib, ic = self.Qinv
        y = t_l(ic, t_m(ib, t_r(ia, x)))  # (Q_C^-1 (x) Q_B^-1 (x) Q_A^-1) x
        y = y / self.PD
        y = t_l(qc, t_m(qb, t_r(qa, y)))
        return (y.real if np.iscomplexobj(y) else y).ravel()  # real operator, real input
