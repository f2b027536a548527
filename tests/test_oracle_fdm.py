"""Pins of the oracle's fast-diagonalisation preconditioner (eqs. preconbasic, Pinvform,
TensorDecomp): P equals the stage matrix, P^-1 is the exact inverse, the contractions follow
their index definitions, and the heat factors have the analytic Dirichlet spectrum."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fdm, operators

CASES = [
    ((5, 4, 3), operators.DIRICHLET, 0, 1.3, (0.0, 0.0, 0.0), 2e-3),
    ((6, 5, 4), operators.PERIODIC, 1, 1e-2, (1.0, 0.5, -0.25), 2e-2),
    ((4, 6, 5), operators.PERIODIC, 0, 0.7, (0.0, 0.0, 0.0), 1e-2),
    ((6, 4, 5), operators.PERIODIC, 2, 0.0, (1.0, 1.0, 1.0), 3e-2),     # central advection
    ((5, 6, 4), operators.PERIODIC, 2, 2e-2, (1.0, -0.5, 0.7), 2e-2),
]


@pytest.mark.parametrize("case", CASES)
def test_preconditioner_equals_stage_matrix(case):
    shape, bc, kind, diff, b, sigma = case
    K = operators.operator(shape, bc, kind, diff, b)
    M = operators.stage_matrix(K, sigma).toarray()
    P = fdm.assemble(*fdm.preconditioner_factors(shape, bc, kind, diff, b, sigma)).toarray()
    assert np.max(np.abs(P - M)) <= 1e-12 * np.max(np.abs(M))


@pytest.mark.parametrize("case", CASES)
def test_inverse_action_is_a_direct_solve(case):
    shape, bc, kind, diff, b, sigma = case
    K = operators.operator(shape, bc, kind, diff, b)
    M = operators.stage_matrix(K, sigma)
    r = np.random.default_rng(7).standard_normal(M.shape[0])
    ref = spla.spsolve(M.tocsc(), r)
    F = fdm.FDM(shape, bc, kind, diff, b, sigma)
    z = F.apply(r)
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("case", CASES)
def test_bases_are_unitary_and_diagonalise_their_factor(case):
    shape, bc, kind, diff, b, sigma = case
    F = fdm.FDM(shape, bc, kind, diff, b, sigma)
    for M, Q, lam in zip(F.factors, F.Q, F.lam):
        n = M.shape[0]
        assert np.abs(Q.conj().T @ Q - np.eye(n)).max() <= 1e-13
        assert np.abs(M @ Q - Q * lam[None, :]).max() <= 1e-13 * max(1.0, np.abs(M).max())


def test_pure_central_advection_repeats_eigenvalues_and_still_inverts_exactly():
    # beta = (1, 1, 1), nu = 0 (the paper's advection test): the 1-D factor's eigenvalues
    # 1 - i sigma b sin(theta) / h repeat for theta and pi - theta; the inverse is still exact
    shape, sigma = (8, 8, 8), 3e-2
    F = fdm.FDM(shape, operators.PERIODIC, 2, 0.0, (1.0, 1.0, 1.0), sigma)
    lam = np.round(F.lam[0], 12)
    assert len(set(lam.tolist())) < shape[0]                   # repeated eigenvalues
    K = operators.operator(shape, operators.PERIODIC, 2, 0.0, (1.0, 1.0, 1.0))
    Mst = operators.stage_matrix(K, sigma)
    r = np.random.default_rng(8).standard_normal(Mst.shape[0])
    ref = spla.spsolve(Mst.tocsc(), r)
    assert np.linalg.norm(F.apply(r) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_non_normal_factor_is_rejected():
    # upwind advection with Dirichlet ends: a non-normal factor without a unitary eigenbasis
    with pytest.raises(ValueError):
        fdm.FDM((6, 5, 4), operators.DIRICHLET, 1, 1e-2, (1.0, 0.5, 0.25), 2e-2)


def test_contractions_follow_their_index_definitions():
    rng = np.random.default_rng(3)
    nx, ny, nz = 3, 4, 5
    x = rng.standard_normal((nz, ny, nx))
    Qa, Qb, Qc = rng.standard_normal((nx, nx)), rng.standard_normal((ny, ny)), rng.standard_normal((nz, nz))
    r = np.zeros_like(x)
    m = np.zeros_like(x)
    l = np.zeros_like(x)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r[k, j, i] = sum(Qa[i, q] * x[k, j, q] for q in range(nx))
                m[k, j, i] = sum(Qb[j, q] * x[k, q, i] for q in range(ny))
                l[k, j, i] = sum(Qc[k, q] * x[q, j, i] for q in range(nz))
    assert np.allclose(fdm.t_r(Qa, x), r, atol=1e-13)
    assert np.allclose(fdm.t_m(Qb, x), m, atol=1e-13)
    assert np.allclose(fdm.t_l(Qc, x), l, atol=1e-13)


def test_heat_factor_has_the_analytic_dirichlet_spectrum():
    n, kappa, sigma = 9, 2.0, 3e-3
    A, B, _ = fdm.preconditioner_factors((n, n, n), operators.DIRICHLET, 0, kappa, (0, 0, 0), sigma)
    h = 1.0 / (n + 1)
    mu = (4.0 / h ** 2) * np.sin(np.arange(1, n + 1) * np.pi * h / 2.0) ** 2
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(1.0 + sigma * kappa * mu), rtol=1e-13)
    assert np.allclose(np.sort(np.linalg.eigvalsh(B)), np.sort(sigma * kappa * mu), rtol=1e-12)


def test_fdm_preconditioned_cg_stage_solve_is_one_iteration_and_matches_splu():
    """CG with the exact inverse as preconditioner reaches the sparse-LU stage solution in one
    iteration (the preconditioned operator is the identity)."""
    from oracle import dirk
    shape, kappa, sigma = (10, 8, 7), 1.3, 4e-3
    K = operators.operator(shape, operators.DIRICHLET, 0, kappa, (0, 0, 0))
    rhs = np.random.default_rng(6).standard_normal(K.shape[0])
    s_fdm = dirk.StageSolver(K, 'cg', rtol=1e-12,
                             fdm_problem=(shape, operators.DIRICHLET, 0, kappa, (0, 0, 0)))
    y = s_fdm(sigma, rhs)
    ref = dirk.StageSolver(K, 'splu')(sigma, rhs)
    assert s_fdm.iterations == [1]
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
