"""GMRES with classical Gram-Schmidt and one re-orthogonalisation pass (CGS2, precisions.reorth
= 1) through the C ABI: stage solves against a sparse direct solve, time steps against the
oracle, and agreement with the one-pass variant where both are exact to rounding."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import workloads as W
from oracle import operators
from tests.gpu_util import log_case, reference_solution, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

# relative error bound of a stage solve vs sparse LU: kappa(M_sigma) (< 10 here) times the
# outer tolerance of the storage's defaults, with margin
SOLVE_BOUND = {'fp64': 1e-10, 'fp32': 1e-8, 'fp16': 1e-5}


def _solve(shape, kind, b, storage, fmt, reorth, precond='bj', compute=None, dt=5e-3):
    over = dict(reorth=reorth, precond=precond)
    if compute is not None:
        over['compute'] = compute
    prec = M.precisions(storage, 'gmres', **over)
    st = M.Stepper(shape, W.PERIODIC, kind, 1e-2, b, fmt, 'SDIRK3', prec, dt)
    rhs = np.random.default_rng(4).standard_normal(st.N)
    x, info = st.solve(1, torch.from_numpy(rhs).cuda())
    sigma = dt * (st.tab.a_lo[st.tab.s + 1] + st.tab.a_hi[st.tab.s + 1])
    st.close()
    Mx = operators.stage_matrix(operators.operator(shape, W.PERIODIC, kind, 1e-2, b), sigma)
    ref = spla.spsolve(Mx.tocsc(), rhs)
    return x.cpu().numpy(), ref, info


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("storage", ['fp64', 'fp32', 'fp16'])
def test_cgs2_stage_solve_matches_sparse_lu(storage, fmt):
    log_case('cgs2_solve', storage=storage, fmt=fmt)
    x, ref, info = _solve((16, 12, 10), W.ADVDIFF, (1.0, 0.5, 0.25), storage, fmt, 1)
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert info['converged'] == 1, info
    assert err <= SOLVE_BOUND[storage], (err, info)


@pytest.mark.parametrize("case", ['fdm', 'cb16', 'noprec'])
def test_cgs2_with_other_solver_options(case):
    log_case('cgs2_options', case=case)
    if case == 'fdm':      # complex fast-diagonalisation preconditioner, FP32
        x, ref, info = _solve((16, 12, 10), W.CENTRAL, (1.0, 1.0, 1.0), 'fp32', A.FMT_STENCIL, 1,
                              precond='fdm')
        bound = 1e-8
    elif case == 'cb16':   # FP16 storage, FP64 arithmetic
        x, ref, info = _solve((16, 12, 10), W.ADVDIFF, (1.0, 0.5, 0.25), 'fp16', A.FMT_STENCIL, 1,
                              compute=A.FP64)
        bound = 1e-5
    else:                  # no preconditioner: long Arnoldi cycles
        x, ref, info = _solve((20, 16, 12), W.ADVDIFF, (1.0, 0.5, 0.25), 'fp64', A.FMT_STENCIL, 1,
                              precond='none', dt=2e-2)
        bound = 1e-10
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert info['converged'] == 1, info
    assert err <= bound, (err, info)


def test_cgs2_and_cgs1_agree_in_fp64():
    log_case('cgs2_vs_cgs1')
    x2, ref, i2 = _solve((16, 12, 10), W.ADVDIFF, (1.0, 0.5, 0.25), 'fp64', A.FMT_STENCIL, 1)
    x1, _, i1 = _solve((16, 12, 10), W.ADVDIFF, (1.0, 0.5, 0.25), 'fp64', A.FMT_STENCIL, 0)
    assert np.linalg.norm(x2 - x1) <= 1e-10 * np.linalg.norm(ref)
    assert i2['iters'] <= i1['iters'] + 1


@pytest.mark.parametrize("storage", ['fp64', 'fp16'])
def test_cgs2_time_steps_match_the_oracle(storage):
    p = W.advdiff_bump(n=32, nsteps=4)
    p.precision = storage
    log_case('cgs2_steps', storage=storage)
    over = dict(reorth=1)
    if storage == 'fp64':
        over.update(rtol=1e-12, outer_tol=1e-12)
    st = M.from_problem(p, **over)
    stats = st.step(p.nsteps)
    u = st.get_u()
    st.close()
    err = rel_l2(u, reference_solution(p))
    assert err <= {'fp64': 1e-12, 'fp16': 1e-3}[storage], (err, stats)
    assert all(stats['converged'])
