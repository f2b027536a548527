"""The paper's own test problems through the C ABI (Section "Test cases"): the forced heat
equation (constant source g = sin sin sin, u(0) = 0) and periodic advection with central
differences, for the methods of its experiments (implicit midpoint with a corrector, 4s3pA/B/C),
against the oracle's closed forms (the forced sine-mode recursion; the FFT evolution)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import closed_form, tableaus
from tests.gpu_util import log_case, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

# FP64: the all-FP64 bar (measured at most 1e-13 on these problems)
TOL = {'fp64': 1e-12, 'fp32': 1e-6, 'fp16': 1e-3}


def run(p, fmt=A.FMT_STENCIL, **over):
    st = M.from_problem(p, fmt=fmt, **over)
    stats = st.step(p.nsteps)
    u = st.get_u()
    st.close()
    return u, stats


def forced_ref(p):
    return closed_form.evolve_forced_heat(p.forcing, p.diff, p.dt, p.nsteps, tableaus.by_name(p.tableau))


def advection_ref(p):
    return closed_form.evolve(p.u0, 2, p.bc, p.diff, p.b, p.dt, p.nsteps, tableaus.by_name(p.tableau))


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("tab", ['MID1', '4S3PB', '4S3PC', 'SDIRK3'])
def test_forced_heat_fp64(tab, fmt):
    p = W.paper_heat(n=18, tableau=tab, dt=1.0 / 160, t_end=0.05, precision='fp64')
    log_case('paper_heat_18', tab=tab, fmt=fmt)
    u, stats = run(p, fmt, rtol=1e-12, outer_tol=1e-12)
    err = rel_l2(u, forced_ref(p))
    print(tab, fmt, 'rel-L2', err, stats['iters'])
    assert err <= TOL['fp64'], err


@pytest.mark.parametrize("storage", ['fp32', 'fp16'])
@pytest.mark.parametrize("tab", ['MID1', '4S3PC'])
def test_forced_heat_mixed(tab, storage):
    p = W.paper_heat(n=20, tableau=tab, dt=1.0 / 160, t_end=0.05, precision=storage)
    log_case('paper_heat_20', tab=tab, storage=storage)
    u, stats = run(p)
    err = rel_l2(u, forced_ref(p))
    assert err <= TOL[storage], err


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("tab", ['MID1', '4S3PA', '4S3PB', '4S3PC'])
def test_central_advection_fp64(tab, fmt):
    p = W.paper_advection(n=16, tableau=tab, dt=1.0 / 80, t_end=0.05, precision='fp64')
    log_case('paper_advection_16', tab=tab, fmt=fmt)
    u, stats = run(p, fmt, rtol=1e-12, outer_tol=1e-12)
    err = rel_l2(u, advection_ref(p))
    print(tab, fmt, 'rel-L2', err, stats['iters'])
    assert err <= TOL['fp64'], err


@pytest.mark.parametrize("storage", ['fp32', 'fp16'])
def test_central_advection_mixed(storage):
    p = W.paper_advection(n=24, tableau='4S3PC', dt=1.0 / 80, t_end=0.05, precision=storage)
    log_case('paper_advection_24', storage=storage)
    u, stats = run(p)
    err = rel_l2(u, advection_ref(p))
    assert err <= TOL[storage], err


def test_stage_solve_ignores_the_forcing_and_removal_restores_the_unforced_step():
    p = W.paper_heat(n=12, tableau='SDIRK3', dt=1e-2, t_end=0.02, precision='fp64')
    log_case('forcing_scope')
    st = M.from_problem(p, rtol=1e-12, outer_tol=1e-12)
    rhs = torch.from_numpy(W.random_field(12, 9).ravel()).cuda()
    x_forced, _ = st.solve(1, rhs)
    st.set_forcing(None)
    x_plain, _ = st.solve(1, rhs)
    assert torch.equal(x_forced, x_plain)  # mprk_solve solves (I - sigma K) x = rhs alone
    u0 = W.random_field(12, 10)
    st.set_u(u0)
    st.step(2)
    u = st.get_u()
    st.close()
    ref = closed_form.evolve_heat(u0, 1.0, p.dt, 2, tableaus.by_name('SDIRK3'))
    err = rel_l2(u, ref)
    assert err <= TOL['fp64'], err


@pytest.mark.parametrize("prob,tab,tau", [('heat', 'MID1', 1 / 10), ('heat', '4S3PC', 1 / 80),
                                          ('advection', '4S3PA', 1 / 10),
                                          ('advection', '4S3PC', 1 / 80)])
def test_sweep_reference_matches_the_oracle(prob, tab, tau):
    """The sweep's tight reference at its size (128^3, T = 0.1): the all-FP64 path with the
    fast-diagonalisation preconditioner and the FP64 residual loop to 1e-12.

    Stage derivatives are evaluated as K y + g in FP64, so a stage-solve error d (relative size
    up to the residual tolerance, in any mode) reaches the step result as tau b_i K d: the
    attainable accuracy is about rtol * tau * rho(K), rho(K) the spectral radius (12 (n+1)^2
    for the Dirichlet Laplacian, 3 n for central advection with beta = (1, 1, 1))."""
    n, rtol = 128, 1e-12
    mk = W.paper_heat if prob == 'heat' else W.paper_advection
    p = mk(n=n, tableau=tab, dt=tau, t_end=0.1, precision='fp64')
    p.precond = 'fdm'
    log_case(f'sweep_reference_{prob}_128', tab=tab, tau=tau)
    u, stats = run(p, rtol=rtol, outer_tol=rtol)
    err = rel_l2(u, forced_ref(p) if prob == 'heat' else advection_ref(p))
    rho = 12.0 * (n + 1) ** 2 if prob == 'heat' else 3.0 * n
    bound = TOL['fp64'] + 10.0 * rtol * tau * rho
    print(prob, tab, tau, 'rel-L2', err, 'bound', bound, stats['iters'])
    assert err <= bound, err
