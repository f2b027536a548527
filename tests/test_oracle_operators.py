"""Pins of oracle/operators.py against the mathematics of the 7-point operators."""
import numpy as np
import pytest

from oracle import operators as O
from oracle import closed_form as C


def brute_force_apply(u3, shape, bc, diff, b):
    """(K u) at every node straight from the finite-difference definition, by loops."""
    nx, ny, nz = shape
    h = [O.spacing(n, bc) for n in shape]
    out = np.zeros_like(u3)

    def val(i, j, k):
        idx = [i, j, k]
        for d, n in enumerate(shape):
            if idx[d] < 0 or idx[d] >= n:
                if bc == O.DIRICHLET:
                    return 0.0
                idx[d] %= n
        return u3[idx[2], idx[1], idx[0]]

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = u3[k, j, i]
                acc = 0.0
                for d in range(3):
                    e = [0, 0, 0]
                    e[d] = 1
                    up = val(i + e[0], j + e[1], k + e[2])
                    dn = val(i - e[0], j - e[1], k - e[2])
                    acc += diff * (up - 2.0 * c + dn) / h[d] ** 2
                    if b[d] > 0:
                        acc -= b[d] * (c - dn) / h[d]
                    elif b[d] < 0:
                        acc -= b[d] * (up - c) / h[d]
                out[k, j, i] = acc
    return out


@pytest.mark.parametrize("bc", [O.DIRICHLET, O.PERIODIC])
@pytest.mark.parametrize("b", [(0.0, 0.0, 0.0), (1.0, 0.5, 0.25), (-0.7, 0.3, -1.1)])
def test_kronecker_assembly_matches_pointwise_stencil(bc, b):
    shape = (4, 5, 3)
    rng = np.random.default_rng(11)
    u3 = rng.standard_normal((shape[2], shape[1], shape[0]))
    K = O.advdiff_operator(shape, bc, 0.37, b)
    ref = brute_force_apply(u3, shape, bc, 0.37, b)
    np.testing.assert_allclose(K @ u3.ravel(), ref.ravel(), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 8, 8)])
def test_heat_sine_modes_are_eigenvectors(shape):
    K = O.heat_operator(shape, O.DIRICHLET, 2.5)
    lam = C.heat_eigenvalues(shape, 2.5)
    for kvec in [(1, 1, 1), (2, 3, 1), (shape[0], 1, shape[2]), (3, 2, 4)]:
        phi = C.heat_sine_mode(shape, kvec).ravel()
        l = lam[kvec[2] - 1, kvec[1] - 1, kvec[0] - 1]
        err = np.linalg.norm(K @ phi - l * phi) / np.linalg.norm(l * phi)
        assert err < 1e-13


def test_heat_lowest_eigenvalue_tends_to_continuum():
    # The lowest Dirichlet mode decays at 3 pi^2 in the continuum (Section "Heat equation").
    prev = None
    for n in (8, 16, 32, 64):
        lam = C.heat_eigenvalues((n, n, n), 1.0)[0, 0, 0]
        gap = abs(lam + 3 * np.pi ** 2)
        if prev is not None:
            assert 3.5 < prev / gap < 4.5  # second-order in h
        prev = gap


def test_heat_operator_is_symmetric_negative_definite():
    K = O.heat_operator((4, 3, 5), O.DIRICHLET, 1.0).toarray()
    assert np.allclose(K, K.T)
    assert np.linalg.eigvalsh(K).max() < 0


@pytest.mark.parametrize("n", [3, 4, 16])
def test_nnz_counts(n):
    K = O.heat_operator((n, n, n), O.DIRICHLET, 1.0)
    assert K.nnz == 7 * n ** 3 - 6 * n ** 2
    Kp = O.advdiff_operator((n, n, n), O.PERIODIC, 1e-2, (1.0, 0.5, 0.25))
    assert Kp.nnz == 7 * n ** 3


def test_periodic_row_sums_vanish():
    K = O.advdiff_operator((6, 5, 4), O.PERIODIC, 0.3, (1.0, -0.5, 0.25))
    assert np.abs(np.asarray(K.sum(axis=1))).max() < 1e-10


@pytest.mark.parametrize("b", [(1.0, 0.5, 0.25), (-1.0, 0.5, -0.25)])
def test_periodic_fourier_modes_are_eigenvectors(b):
    shape = (6, 5, 4)
    K = O.advdiff_operator(shape, O.PERIODIC, 0.01, b)
    lam = C.periodic_eigenvalues(shape, 0.01, b)
    nx, ny, nz = shape
    ii = np.arange(nx)[None, None, :]
    jj = np.arange(ny)[None, :, None]
    kk = np.arange(nz)[:, None, None]
    for m in [(0, 0, 0), (1, 2, 3), (5, 4, 1)]:
        mode = np.exp(2j * np.pi * (m[0] * ii / nx + m[1] * jj / ny + m[2] * kk / nz)).ravel()
        # the mode e^{+i theta j} (theta = 2 pi m / n) sits at FFT index m
        l = lam[m[2], m[1], m[0]]
        assert np.linalg.norm(K @ mode - l * mode) <= 1e-10 * max(1.0, abs(l)) * np.linalg.norm(mode)


def test_upwind_direction_follows_velocity_sign():
    # b_d > 0 couples to the upstream (lower-index) neighbour only.
    K = O.advdiff_operator((5, 1, 1), O.PERIODIC, 0.0, (2.0, 0.0, 0.0)).toarray()
    h = 1 / 5
    assert K[2, 1] == pytest.approx(2.0 / h) and K[2, 3] == 0.0
    K = O.advdiff_operator((5, 1, 1), O.PERIODIC, 0.0, (-2.0, 0.0, 0.0)).toarray()
    assert K[2, 3] == pytest.approx(2.0 / h) and K[2, 1] == 0.0


def test_stage_matrix_sign_convention():
    K = O.heat_operator((3, 3, 3), O.DIRICHLET, 1.0)
    M = O.stage_matrix(K, 0.1).toarray()
    # y = rhs + sigma K y  <=>  (I - sigma K) y = rhs ; SPD with diagonal > 1
    assert np.all(np.diag(M) > 1.0)
    assert np.linalg.eigvalsh(M).min() > 1.0 - 1e-12
