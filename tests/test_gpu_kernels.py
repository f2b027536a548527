"""Kernel-level parity through the C ABI (mprk_apply / mprk_solve) against the FP64 oracle.

Bounds: for a product computed in precision u_c from inputs already rounded to the storage
type, |y - y_ref| <= 2 u_out |y_ref| + (c u_c + 2 u_val) sum_j |A_ij| |x_j|, with u_out the
rounding of the stored output and u_val that of stored matrix/inverse values.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import krylov, operators
from tests.gpu_util import log_case

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

U = {A.FP64: 2.0 ** -53, A.FP32: 2.0 ** -24, A.FP16: 2.0 ** -11}
# absolute rounding of a stored output that lands in the subnormal range of the storage type
TINY = {A.FP64: 0.0, A.FP32: 2.0 ** -150, A.FP16: 2.0 ** -25}
NP = {A.FP64: np.float64, A.FP32: np.float32, A.FP16: np.float16}

CASES = [
    # shape, bc, kind, diff, b
    ((16, 16, 16), W.DIRICHLET, W.HEAT, 1.0, (0.0, 0.0, 0.0)),
    ((13, 9, 7), W.DIRICHLET, W.HEAT, 2.5, (0.0, 0.0, 0.0)),           # nx % 4 != 0, N % 8 != 0
    ((32, 20, 12), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25)),
    ((12, 5, 3), W.PERIODIC, W.ADVDIFF, 0.3, (-1.0, 0.5, -0.25)),      # negative velocities
]


def _stepper(shape, bc, kind, diff, b, fmt, storage, krylov_name='gmres', dt=2e-3):
    prec = M.precisions(storage, krylov_name)
    return M.Stepper(shape, bc, kind, diff, b, fmt, 'SDIRK3', prec, dt)


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("case", CASES)
def test_apply_K64(case, fmt):
    shape, bc, kind, diff, b = case
    log_case('apply_K64', shape=shape, bc=bc, fmt=fmt)
    st = _stepper(shape, bc, kind, diff, b, fmt, 'fp64')
    rng = np.random.default_rng(1)
    x = rng.standard_normal(st.N)
    y = st.apply(A.APPLY_K64, torch.from_numpy(x).cuda()).cpu().numpy()
    K = operators.operator(shape, bc, kind, diff, b)
    ref = K @ x
    bound = 16 * 2.0 ** -53 * (abs(K) @ abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
    st.close()


@pytest.mark.parametrize("storage", ['fp64', 'fp32', 'fp16'])
@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("case", CASES)
def test_apply_M_lp(case, fmt, storage):
    shape, bc, kind, diff, b = case
    log_case('apply_M_lp', shape=shape, bc=bc, fmt=fmt, storage=storage)
    st = _stepper(shape, bc, kind, diff, b, fmt, storage)
    sd = st.prec.storage
    sigma = st.dt * st.tab.a_lo[0]
    rng = np.random.default_rng(2)
    x_lp = rng.standard_normal(st.N).astype(NP[sd])
    y = st.apply(A.APPLY_M_LP, torch.from_numpy(x_lp).cuda(), 0).cpu().numpy().astype(np.float64)
    Mx = operators.stage_matrix(operators.operator(shape, bc, kind, diff, b), sigma)
    xf = x_lp.astype(np.float64)
    ref = Mx @ xf
    u_c = U[A.FP64] if sd == A.FP64 else U[A.FP32]
    u_val = U[sd] if fmt == A.FMT_CSR else u_c
    bound = 2 * U[sd] * np.abs(ref) + (16 * u_c + 2 * u_val) * (abs(Mx) @ np.abs(xf)) + TINY[sd]
    assert np.all(np.abs(y - ref) <= bound + 1e-300), np.max(np.abs(y - ref) - bound)
    st.close()


@pytest.mark.parametrize("storage", ['fp64', 'fp32', 'fp16'])
@pytest.mark.parametrize("block", [1, 2, 4, 8])
@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("case", CASES[:3])
def test_block_jacobi_apply(case, fmt, block, storage):
    shape, bc, kind, diff, b = case
    log_case('bj_apply', shape=shape, fmt=fmt, block=block, storage=storage)
    prec = M.precisions(storage, 'gmres', block=block)
    st = M.Stepper(shape, bc, kind, diff, b, fmt, 'SDIRK3', prec, 2e-3)
    sd = st.prec.storage
    sigma = st.dt * st.tab.a_lo[0]
    rng = np.random.default_rng(3)
    x_lp = rng.standard_normal(st.N).astype(NP[sd])
    z = st.apply(A.APPLY_BJ_LP, torch.from_numpy(x_lp).cuda(), 0).cpu().numpy().astype(np.float64)
    Mx = operators.stage_matrix(operators.operator(shape, bc, kind, diff, b), sigma)
    inv = krylov.block_jacobi_inverses(Mx, block)
    xf = x_lp.astype(np.float64)
    ref = krylov.block_jacobi_apply(inv, xf, block)
    absd = krylov.block_jacobi_apply([np.abs(d) for d in inv], np.abs(xf), block)
    u_c = U[A.FP64] if sd == A.FP64 else U[A.FP32]
    bound = 2 * U[sd] * np.abs(ref) + (16 * u_c + 2 * U[sd]) * absd + TINY[sd]
    assert np.all(np.abs(z - ref) <= bound + 1e-300)
    st.close()


SOLVE_CASES = [
    # shape, bc, kind, diff, b, krylov, storage, rel-error bound vs sparse LU
    ((12, 12, 12), W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), 'cg', 'fp64', 1e-10),
    ((12, 12, 12), W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), 'cg', 'fp32', 1e-8),
    ((12, 12, 12), W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), 'cg', 'fp16', 1e-5),
    ((13, 11, 9), W.DIRICHLET, W.HEAT, 3.0, (0, 0, 0), 'cg', 'fp32', 1e-8),
    ((16, 16, 16), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25), 'gmres', 'fp64', 1e-10),
    ((16, 16, 16), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25), 'gmres', 'fp32', 1e-8),
    ((16, 16, 16), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25), 'gmres', 'fp16', 1e-5),
]


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("case", SOLVE_CASES)
def test_stage_solve_matches_sparse_lu(case, fmt):
    shape, bc, kind, diff, b, kr, storage, tol = case
    log_case('stage_solve', shape=shape, krylov=kr, storage=storage, fmt=fmt)
    prec = M.precisions(storage, kr)
    dt = 5e-3
    st = M.Stepper(shape, bc, kind, diff, b, fmt, 'SDIRK3', prec, dt)
    rng = np.random.default_rng(4)
    rhs = rng.standard_normal(st.N)
    x, info = st.solve(1, torch.from_numpy(rhs).cuda())
    K = operators.operator(shape, bc, kind, diff, b)
    Mx = operators.stage_matrix(K, dt * st.tab.a_lo[st.tab.s + 1])
    import scipy.sparse.linalg as spla
    ref = spla.spsolve(Mx.tocsc(), rhs)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert info['converged'] == 1
    assert err <= tol, (err, info)
    st.close()


def test_eigenvector_rhs_needs_one_cg_iteration():
    shape = (16, 16, 16)
    log_case('eigvec_cg')
    prec = M.precisions('fp64', 'cg', precond='none', rtol=1e-12, outer_tol=1e-11)
    st = M.Stepper(shape, W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), A.FMT_STENCIL, 'SDIRK2', prec, 1e-3)
    phi = W.sine_mode(shape, (2, 3, 1)).ravel()
    x, info = st.solve(0, torch.from_numpy(phi).cuda())
    assert info['iters'] == 1 and info['passes'] == 1
    st.close()


def test_block_covering_everything_needs_one_iteration():
    # 2x2x2 grid: N = 8 = one block-Jacobi block, so the preconditioner is the exact inverse
    log_case('bj_exact')
    prec = M.precisions('fp64', 'gmres', block=8, rtol=1e-12, outer_tol=1e-11)
    st = M.Stepper((4, 2, 1), W.PERIODIC, W.ADVDIFF, 0.1, (1.0, 0.5, 0.0), A.FMT_STENCIL,
                   'SDIRK3', prec, 1e-2)
    rhs = np.random.default_rng(0).standard_normal(st.N)
    x, info = st.solve(0, torch.from_numpy(rhs).cuda())
    assert info['iters'] == 1, info
    st.close()


@pytest.mark.parametrize("restart", [30, 10, 6])
def test_long_gmres_cycles_match_sparse_lu(restart):
    # unpreconditioned GMRES on a stiff advection-diffusion stage matrix: about 29 Arnoldi steps
    # per cycle to 1e-12, so every compiled bound on the basis size (4, 8, 16, 33) is used;
    # shorter cycles (restart 10, 6) need many outer passes
    shape = (16, 16, 16)
    log_case('gmres_long', restart=restart)
    prec = M.precisions('fp64', 'gmres', precond='none', rtol=1e-12, outer_tol=1e-11,
                        restart=restart, maxit=restart, refine_max=200)
    dt = 5e-2
    st = M.Stepper(shape, W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25), A.FMT_STENCIL, 'SDIRK3',
                   prec, dt)
    rhs = np.random.default_rng(4).standard_normal(st.N)
    x, info = st.solve(1, torch.from_numpy(rhs).cuda())
    K = operators.operator(shape, W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25))
    Mx = operators.stage_matrix(K, dt * st.tab.a_lo[st.tab.s + 1])
    import scipy.sparse.linalg as spla
    ref = spla.spsolve(Mx.tocsc(), rhs)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    st.close()
    assert info['converged'] == 1, info
    assert err <= 1e-9, (err, info)
    if restart == 30:
        assert info['iters'] >= 20, info
    else:
        assert info['passes'] >= 2, info
