"""Pins of oracle/dirk.py, oracle/krylov.py and oracle/closed_form.py."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import closed_form as C
from oracle import dirk as D
from oracle import krylov as KR
from oracle import operators as O
from oracle import tableaus as T

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


def test_heat_sine_16_matches_modal_closed_form():
    # u0 is the lowest sine mode: u_N = R(tau lambda)^N u0 exactly.
    p = W.heat_sine_16()
    shape = (p.n,) * 3
    K = O.heat_operator(shape, O.DIRICHLET, p.diff)
    u = D.integrate(K, p.u0, p.dt, p.nsteps, T.sdirk2(), 'splu')
    lam = C.heat_eigenvalues(shape, p.diff)[0, 0, 0]
    R = T.stability_function(T.sdirk2(), np.array([p.dt * lam]))[0].real
    assert D.relative_l2(u, R ** p.nsteps * p.u0) < 1e-14
    # the sine mode factor itself, evaluated by hand from the SDIRK2 stage equations
    g = 1 - 1 / np.sqrt(2)
    z = p.dt * lam
    y1 = 1 / (1 - g * z)
    y2 = (1 + (1 - g) * z * y1) / (1 - g * z)
    assert abs(R - (1 + z * ((1 - g) * y1 + g * y2))) < 1e-15


def test_heat_sine_16_continuum_gap_is_spatial_error():
    # vs exp(-3 pi^2 kappa t) the gap is the O(h^2) spatial error; it falls ~4x per halving of h
    gaps = []
    for n in (8, 16, 32):
        u0 = W.sine_mode((n, n, n), (1, 1, 1))
        lam = C.heat_eigenvalues((n, n, n), 1.0)[0, 0, 0]
        R = T.stability_function(T.sdirk2(), np.array([1e-4 * lam]))[0].real
        uN = R ** 100 * u0
        gaps.append(D.relative_l2(uN, np.exp(-3 * np.pi ** 2 * 0.01) * u0))
    assert 3.3 < gaps[0] / gaps[1] < 4.5 and 3.3 < gaps[1] / gaps[2] < 4.5


@pytest.mark.parametrize("method", ["dense", "cg"])
def test_stage_solvers_agree_heat(method):
    shape = (6, 5, 7)
    K = O.heat_operator(shape, O.DIRICHLET, 1.3)
    rhs = np.random.default_rng(1).standard_normal(K.shape[0])
    ref = D.StageSolver(K, 'splu')(0.004, rhs)
    got = D.StageSolver(K, method)(0.004, rhs)
    assert D.relative_l2(got, ref) < 1e-12
    M = O.stage_matrix(K, 0.004)
    assert np.linalg.norm(M @ ref - rhs) < 1e-12 * np.linalg.norm(rhs)


@pytest.mark.parametrize("method", ["dense", "gmres"])
def test_stage_solvers_agree_advdiff(method):
    shape = (6, 6, 6)
    K = O.advdiff_operator(shape, O.PERIODIC, 1e-2, (1.0, 0.5, 0.25))
    rhs = np.random.default_rng(2).standard_normal(K.shape[0])
    ref = D.StageSolver(K, 'splu')(0.01, rhs)
    got = D.StageSolver(K, method)(0.01, rhs)
    assert D.relative_l2(got, ref) < 1e-12


@pytest.mark.parametrize("name", ["SDIRK2", "SDIRK3", "4s3pB", "4s3pC", "MID2"])
def test_dirk_matches_dst_closed_form_random_u0(name):
    n = 7
    tab = T.by_name(name)
    u0 = W.random_field(n, 5)
    K = O.heat_operator((n,) * 3, O.DIRICHLET, 0.8)
    u = D.integrate(K, u0, 2e-3, 4, tab, 'splu')
    ref = C.evolve_heat(u0, 0.8, 2e-3, 4, tab)
    assert D.relative_l2(u, ref) < 1e-12


@pytest.mark.parametrize("name", ["SDIRK3", "4s3pA", "4s3pB", "4s3pC"])
def test_dirk_matches_fft_closed_form_periodic(name):
    n = 6
    tab = T.by_name(name)
    u0 = W.random_field(n, 6)
    b = (1.0, -0.5, 0.25)
    K = O.advdiff_operator((n,) * 3, O.PERIODIC, 1e-2, b)
    u = D.integrate(K, u0, 5e-3, 3, tab, 'splu')
    ref = C.evolve_periodic(u0, 1e-2, b, 5e-3, 3, tab)
    assert D.relative_l2(u, ref) < 1e-12


def test_closed_form_periodic_equals_dft_of_dirk_for_the_advdiff_workload_on_16():
    # same physics as the 256^3 advection-diffusion workload, on 16^3
    p = W.advdiff_bump(n=16, nsteps=3)
    K = O.advdiff_operator((16,) * 3, O.PERIODIC, p.diff, p.b)
    u = D.integrate(K, p.u0, p.dt, p.nsteps, T.sdirk3(), 'splu')
    ref = C.evolve_periodic(p.u0, p.diff, p.b, p.dt, p.nsteps, T.sdirk3())
    assert D.relative_l2(u, ref) < 1e-12


def observed_orders(tab, errs_fn, taus):
    errs = [errs_fn(tab, t) for t in taus]
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def _heat_err(tab, tau, n=24, T_end=0.02):
    rng = np.random.default_rng(2)
    u0, _, _ = W.fourier_sine_modes(n, rng)
    steps = int(round(T_end / tau))
    u = C.evolve_heat(u0, 1.0, tau, steps, tab)
    return D.relative_l2(u, C.evolve_heat_exact(u0, 1.0, T_end))


@pytest.mark.parametrize("name,order", [("SDIRK2", 2), ("SDIRK3", 3), ("MID1", 2), ("4s3pB", 3)])
def test_dt_halving_order_closed_form(name, order):
    taus = [1e-3, 5e-4, 2.5e-4, 1.25e-4]
    q = observed_orders(T.by_name(name), _heat_err, taus)
    assert abs(q[-1] - order) < 0.15, q


@pytest.mark.parametrize("name,order", [("SDIRK2", 2), ("SDIRK3", 3), ("4s3pA", 3)])
def test_dt_halving_order_of_the_stepper(name, order):
    # the order of the DIRK stepping code itself, on a non-stiff periodic problem
    n = 8
    u0 = W.gaussian_bump(n, (0.5, 0.5, 0.5), 10.0)
    b = (1.0, 0.5, 0.25)
    K = O.advdiff_operator((n,) * 3, O.PERIODIC, 1e-2, b)
    T_end = 0.08
    ref = C.evolve_periodic_exact(u0, 1e-2, b, T_end)
    errs = []
    for steps in (8, 16, 32):
        u = D.integrate(K, u0, T_end / steps, steps, T.by_name(name), 'splu')
        errs.append(D.relative_l2(u, ref))
    q = np.log2(errs[1] / errs[2])
    assert abs(q - order) < 0.25, (errs, q)


def test_corrector_divergence_when_spectral_radius_exceeds_one():
    # Section "The implicit midpoint method and explicit corrector steps": an error e in the
    # low-precision stage is propagated by the corrector steps as (tau K / 2)^p e.
    n = 6
    K = O.heat_operator((n,) * 3, O.DIRICHLET, 1.0)
    u0 = W.random_field(n, 3).ravel()
    rng = np.random.default_rng(9)
    pert = 1e-6 * rng.standard_normal(u0.size)
    rho_unit = abs(C.heat_eigenvalues((n,) * 3, 1.0)).max() / 2

    def err(tau, p):
        tab = T.mid(p)
        solve = D.StageSolver(K, 'splu')
        exact = D.dirk_step(K, u0, tau, tab, solve)
        bad = D.dirk_step(K, u0, tau, tab, solve, stage_hook=lambda i, y: y + pert)
        return np.linalg.norm(bad - exact)

    tau_big = 3.0 / rho_unit      # rho(tau K / 2) = 3
    tau_small = 0.5 / rho_unit    # rho(tau K / 2) = 0.5
    big = [err(tau_big, p) for p in (1, 3, 5)]
    small = [err(tau_small, p) for p in (1, 3, 5)]
    assert big[2] > 20 * big[0]
    assert small[2] < small[0]


def test_krylov_special_cases():
    shape = (5, 5, 5)
    K = O.heat_operator(shape, O.DIRICHLET, 1.0)
    M = O.stage_matrix(K, 1e-3)
    phi = C.heat_sine_mode(shape, (2, 1, 3)).ravel()
    x, it, _ = KR.cg(M, phi, rtol=1e-12)
    assert it == 1                                   # eigenvector right-hand side
    rhs = np.random.default_rng(0).standard_normal(M.shape[0])
    inv = KR.block_jacobi_inverses(M, M.shape[0])    # one block covering everything
    x, it, _ = KR.cg(M, rhs, lambda r: KR.block_jacobi_apply(inv, r, M.shape[0]), rtol=1e-12)
    assert it == 1
    x, it, _ = KR.gmres(M, rhs, lambda r: KR.block_jacobi_apply(inv, r, M.shape[0]), rtol=1e-12)
    assert it == 1
    inv1 = KR.block_jacobi_inverses(M, 1)            # block size 1 is point Jacobi
    np.testing.assert_allclose([d[0, 0] for d in inv1], 1.0 / M.diagonal(), rtol=1e-15)


def test_block_jacobi_short_last_block():
    K = O.heat_operator((3, 3, 3), O.DIRICHLET, 1.0)   # N = 27 = 3*8 + 3
    M = O.stage_matrix(K, 1e-2)
    inv = KR.block_jacobi_inverses(M, 8)
    assert [d.shape[0] for d in inv] == [8, 8, 8, 3]
    for bi, d in enumerate(inv):
        s = bi * 8
        blk = M[s:s + d.shape[0], s:s + d.shape[0]].toarray()
        np.testing.assert_allclose(d @ blk, np.eye(d.shape[0]), atol=1e-14)


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith('#'):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_fp16_range_hazard():
    g = _golden('fp16_limits.txt')
    fi = np.finfo(np.float16)
    assert float(fi.max) == g['half_max_normal']
    assert float(fi.smallest_normal) == g['half_min_normal']
    assert 1.0 / g['example_h'] ** 2 > g['half_max_normal']
    # raw K of a kappa = 10, n = 96 heat problem overflows half precision...
    K = O.heat_operator((96, 1, 1), O.DIRICHLET, 10.0)
    with np.errstate(over='ignore'):
        assert not np.all(np.isfinite(K.data.astype(np.float16)))
    # ...while the tau-scaled stage matrix of the 256^3 advection-diffusion problem does not
    p = W.advdiff_bump(n=256)
    sigma = p.dt * T.sdirk3_gamma()
    Kp = O.advdiff_operator((256, 1, 1), O.PERIODIC, p.diff, p.b)
    row = O.stage_matrix(Kp, sigma).toarray()[5]
    assert np.all(np.isfinite(row.astype(np.float16)))


def test_relative_error_of_a_fully_decayed_state_is_roundoff_dominated():
    # A state that decays by ~1e-20 cannot be matched relative to its own norm, even by the
    # FP64 DIRK with exact (sparse LU) solves: roundoff seeds slowly decaying modes that the
    # exact state lacks.  Errors are therefore measured against max(|u_N|, 1e-6 |u_0|).
    n, kappa, dt, steps = 16, 10.0, 5e-4, 20
    u0 = W.sine_mode((n, n, n), (5, 5, 5))
    K = O.heat_operator((n,) * 3, O.DIRICHLET, kappa)
    u = D.integrate(K, u0, dt, steps, T.sdirk3(), 'splu')
    ref = C.evolve_heat(u0, kappa, dt, steps, T.sdirk3()).ravel()
    decay = np.linalg.norm(ref) / np.linalg.norm(u0)
    err = np.linalg.norm(u - ref)
    assert decay < 1e-15
    assert err / np.linalg.norm(ref) > 1.0                      # meaningless relative to |u_N|
    assert err / max(np.linalg.norm(ref), 1e-6 * np.linalg.norm(u0)) < 1e-12
