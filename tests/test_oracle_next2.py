"""Pins of the oracle parts behind the paper's own test problems (Section "Test cases"): the
central-difference advection operator and the constant forcing of the heat test.

Central advection: brute-force pointwise stencil, skew-symmetry of the periodic central
difference, its Fourier eigenpairs against the sparse operator, and the FFT closed form of the
DIRK against sparse-LU time stepping.  Forcing: the DIRK with forcing (sparse solves) against
the independently derived scalar recursion for the forced sine mode, R(z) = 1 + z b^T(I-zA)^-1 e,
implicit Euler's forced recursion written out by hand, the method's order against the
semi-discrete exact amplitude, and the O(h^2) gap to the paper's continuum solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import closed_form, dirk, operators, tableaus
from oracle.tableaus import Tableau


def test_central_operator_matches_a_pointwise_stencil_loop():
    shape, nu, b = (5, 4, 3), 0.3, (1.0, -0.5, 0.25)
    K = operators.operator(shape, operators.PERIODIC, 2, nu, b).toarray()
    nx, ny, nz = shape
    h = [1.0 / n for n in shape]
    ref = np.zeros_like(K)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = i + nx * (j + ny * k)
                for d, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    ip = ((i + di) % nx) + nx * (((j + dj) % ny) + ny * ((k + dk) % nz))
                    im = ((i - di) % nx) + nx * (((j - dj) % ny) + ny * ((k - dk) % nz))
                    ref[r, ip] += nu / h[d] ** 2 - b[d] / (2 * h[d])
                    ref[r, im] += nu / h[d] ** 2 + b[d] / (2 * h[d])
                    ref[r, r] += -2.0 * nu / h[d] ** 2
    assert np.allclose(K, ref, atol=1e-12)


def test_periodic_central_advection_is_skew_symmetric():
    K = operators.operator((6, 5, 4), operators.PERIODIC, 2, 0.0, (1.0, 1.0, 1.0))
    assert abs(K + K.T).max() < 1e-12
    assert abs(K.diagonal()).max() == 0.0


def test_central_symbol_gives_fourier_eigenpairs_of_the_sparse_operator():
    shape, nu, b = (8, 6, 5), 0.05, (1.0, 0.7, -0.4)
    K = operators.operator(shape, operators.PERIODIC, 2, nu, b)
    lam = closed_form.periodic_eigenvalues(shape, nu, b, central=True)
    nx, ny, nz = shape
    rng = np.random.default_rng(1)
    for _ in range(5):
        m = [int(rng.integers(0, n)) for n in shape]
        x = [np.exp(2j * np.pi * m[d] * np.arange(n) / n) for d, n in enumerate(shape)]
        v = (x[2][:, None, None] * x[1][None, :, None] * x[0][None, None, :]).ravel()
        assert np.allclose(K @ v, lam[m[2], m[1], m[0]] * v, atol=1e-9)


@pytest.mark.parametrize("name", ['MID1', '4S3PA', '4S3PB', '4S3PC'])
def test_central_advection_closed_form_matches_sparse_time_stepping(name):
    shape, b, tau, nsteps = (8, 8, 8), (1.0, 1.0, 1.0), 1.0 / 40, 4
    tab = tableaus.by_name(name)
    rng = np.random.default_rng(2)
    u0 = rng.standard_normal(shape[::-1])
    K = operators.operator(shape, operators.PERIODIC, 2, 0.0, b)
    ref = dirk.integrate(K, u0.ravel(), tau, nsteps, tab).reshape(u0.shape)
    cf = closed_form.evolve(u0, 2, operators.PERIODIC, 0.0, b, tau, nsteps, tab)
    assert np.linalg.norm(cf - ref) <= 1e-11 * np.linalg.norm(ref)


def test_stability_function_is_one_plus_z_times_the_stage_sum():
    z = np.array([-0.3, -4.0, 2.5j, -1.0 + 0.5j])
    for name in ('SDIRK3', 'MID1', '4S3PB', '4S3PC'):
        tab = tableaus.by_name(name)
        assert np.allclose(tableaus.stability_function(tab, z),
                           1.0 + z * closed_form.stage_sum(tab, z), atol=1e-14)


@pytest.mark.parametrize("name", ['MID1', '4S3PB', '4S3PC', 'SDIRK3'])
def test_forced_dirk_matches_the_scalar_recursion_of_the_forced_mode(name):
    shape, kappa, tau, nsteps = (7, 6, 5), 1.0, 2e-3, 5
    tab = tableaus.by_name(name)
    g = closed_form.heat_sine_mode(shape, (1, 1, 1))
    K = operators.operator(shape, operators.DIRICHLET, 0, kappa)
    u = dirk.integrate(K, np.zeros(g.size), tau, nsteps, tab, g=g).reshape(g.shape)
    ref = closed_form.evolve_forced_heat(g, kappa, tau, nsteps, tab)
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)


def test_implicit_euler_forced_recursion_written_out():
    # a_{n+1} = (a_n + tau) / (1 - tau lambda) for a' = lambda a + 1 with implicit Euler
    ie = Tableau('IE', np.zeros((1, 1)), np.array([[1.0]]), np.array([1.0]))
    lam, tau, n = -7.0, 0.05, 9
    a = 0.0
    for _ in range(n):
        a = (a + tau) / (1.0 - tau * lam)
    assert abs(closed_form.forced_mode_amplitude(ie, lam, tau, n) - a) <= 1e-15


@pytest.mark.parametrize("name,order", [('MID1', 2), ('4S3PB', 3), ('SDIRK3', 3)])
def test_forced_amplitude_converges_at_the_method_order(name, order):
    tab = tableaus.by_name(name)
    lam, T = -3.0 * np.pi ** 2 * 1.1, 0.1
    exact = (np.exp(lam * T) - 1.0) / lam
    errs = [abs(closed_form.forced_mode_amplitude(tab, lam, T / n, n) - exact) for n in (40, 80)]
    assert 0.8 * 2 ** order <= errs[0] / errs[1] <= 1.3 * 2 ** order


def test_semi_discrete_forced_solution_approaches_the_continuum_at_second_order():
    t = 0.1
    gaps = []
    for n in (15, 31):
        g = closed_form.heat_sine_mode((n, n, n), (1, 1, 1))
        sd = closed_form.forced_heat_exact(g, 1.0, t)
        co = closed_form.forced_heat_exact(g, 1.0, t, continuum=True)
        gaps.append(np.max(np.abs(sd - co)))
    assert 3.5 <= gaps[0] / gaps[1] <= 4.5  # h halves: 1/16 -> 1/32


def test_cached_periodic_evolution_equals_the_direct_one():
    u0 = np.random.default_rng(9).standard_normal((6, 5, 8))
    ev = closed_form.PeriodicEvolution(u0, 0.0, (1.0, 1.0, 1.0), central=True)
    for name, tau, n in (('MID1', 0.05, 3), ('4S3PC', 0.02, 5)):
        tab = tableaus.by_name(name)
        ref = closed_form.evolve_periodic(u0, 0.0, (1.0, 1.0, 1.0), tau, n, tab, central=True)
        assert np.allclose(ev(tau, n, tab), ref, atol=1e-14)


def test_workload_continuum_solutions_match_the_oracle():
    """The continuum references the sweep reports against (workloads) agree with the oracle's:
    the forced heat amplitude and, for the advection test at t = 0, the initial Gaussian."""
    import workloads as W
    for n, t in ((9, 0.05), (16, 0.1)):
        g = closed_form.heat_sine_mode((n, n, n), (1, 1, 1))
        co = closed_form.forced_heat_exact(g, 1.0, t, continuum=True)
        assert np.allclose(W.paper_heat_exact(n, t), co, rtol=1e-14, atol=0.0)
    p = W.paper_advection(n=12, tableau='MID1', dt=0.1, t_end=0.1)
    assert np.allclose(W.translated_gaussian(12, (0.0, 0.0, 0.0)), p.u0, rtol=1e-14, atol=1e-300)
    # a shift by whole periods is the identity
    assert np.allclose(W.translated_gaussian(12, (1.0, -2.0, 3.0)), p.u0, rtol=1e-12, atol=1e-300)
