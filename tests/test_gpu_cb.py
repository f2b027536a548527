"""Compressed-basis Krylov (FP64 arithmetic over FP16 / FP32 storage; the Ginkgo-style variant
the Introduction cites) through the C ABI, against the FP64 oracle.

Kernel bounds as in test_gpu_kernels.py with u_c the FP64 unit roundoff: the products are
computed in FP64 from inputs already rounded to the storage type, so only the stored output
(and stored matrix values) carry storage rounding."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import workloads as W
from oracle import closed_form, fdm, krylov, operators, tableaus
from tests.gpu_util import log_case, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

U = {A.FP32: 2.0 ** -24, A.FP16: 2.0 ** -11}
TINY = {A.FP32: 2.0 ** -150, A.FP16: 2.0 ** -25}
NP = {A.FP32: np.float32, A.FP16: np.float16}
DT = {'fp32': torch.float32, 'fp16': torch.float16}
U64 = 2.0 ** -53

CASES = [
    ((13, 9, 7), W.DIRICHLET, W.HEAT, 2.5, (0.0, 0.0, 0.0)),
    ((32, 20, 12), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25)),
    ((12, 10, 8), W.PERIODIC, W.CENTRAL, 0.0, (1.0, 1.0, 1.0)),
]


def cb(storage, krylov_name, **kw):
    return M.precisions(storage, krylov_name, compute=A.FP64, **kw)


@pytest.mark.parametrize("storage", ['fp32', 'fp16'])
@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("case", CASES)
def test_lp_operator_with_fp64_arithmetic(case, fmt, storage):
    shape, bc, kind, diff, b = case
    log_case('cb_apply_M', shape=shape, fmt=fmt, storage=storage)
    st = M.Stepper(shape, bc, kind, diff, b, fmt, 'SDIRK3', cb(storage, 'gmres'), 2e-3)
    sd = st.prec.storage
    sigma = st.dt * st.tab.a_lo[0]
    x_lp = np.random.default_rng(2).standard_normal(st.N).astype(NP[sd])
    y = st.apply(A.APPLY_M_LP, torch.from_numpy(x_lp).cuda(), 0).cpu().numpy().astype(np.float64)
    Mx = operators.stage_matrix(operators.operator(shape, bc, kind, diff, b), sigma)
    xf = x_lp.astype(np.float64)
    ref = Mx @ xf
    u_val = U[sd] if fmt == A.FMT_CSR else U64
    bound = 2 * U[sd] * np.abs(ref) + (16 * U64 + 2 * u_val) * (abs(Mx) @ np.abs(xf)) + TINY[sd]
    assert np.all(np.abs(y - ref) <= bound + 1e-300), np.max(np.abs(y - ref) - bound)
    st.close()


@pytest.mark.parametrize("storage", ['fp32', 'fp16'])
def test_block_jacobi_with_fp64_arithmetic(storage):
    shape, bc, kind, diff, b = CASES[1]
    log_case('cb_bj', storage=storage)
    st = M.Stepper(shape, bc, kind, diff, b, A.FMT_STENCIL, 'SDIRK3', cb(storage, 'gmres'), 2e-3)
    sd = st.prec.storage
    sigma = st.dt * st.tab.a_lo[0]
    x_lp = np.random.default_rng(3).standard_normal(st.N).astype(NP[sd])
    z = st.apply(A.APPLY_BJ_LP, torch.from_numpy(x_lp).cuda(), 0).cpu().numpy().astype(np.float64)
    Mx = operators.stage_matrix(operators.operator(shape, bc, kind, diff, b), sigma)
    inv = krylov.block_jacobi_inverses(Mx, 8)
    xf = x_lp.astype(np.float64)
    ref = krylov.block_jacobi_apply(inv, xf, 8)
    absd = krylov.block_jacobi_apply([np.abs(d) for d in inv], np.abs(xf), 8)
    bound = 2 * U[sd] * np.abs(ref) + (16 * U64 + 2 * U[sd]) * absd + TINY[sd]
    assert np.all(np.abs(z - ref) <= bound + 1e-300)
    st.close()


@pytest.mark.parametrize("storage,bound", [('fp32', 1e-8), ('fp16', 1e-5)])
@pytest.mark.parametrize("kr,case", [('cg', CASES[0]), ('gmres', CASES[1]), ('gmres', CASES[2])])
def test_stage_solve_matches_sparse_lu(kr, case, storage, bound):
    shape, bc, kind, diff, b = case
    log_case('cb_solve', krylov=kr, shape=shape, storage=storage)
    dt = 5e-3
    st = M.Stepper(shape, bc, kind, diff, b, A.FMT_STENCIL, 'SDIRK3', cb(storage, kr), dt)
    rhs = np.random.default_rng(4).standard_normal(st.N)
    x, info = st.solve(1, torch.from_numpy(rhs).cuda())
    Mx = operators.stage_matrix(operators.operator(shape, bc, kind, diff, b),
                                dt * (st.tab.a_lo[st.tab.s + 1] + st.tab.a_hi[st.tab.s + 1]))
    ref = spla.spsolve(Mx.tocsc(), rhs)
    st.close()
    assert info['converged'] == 1, info
    assert np.linalg.norm(x.cpu().numpy() - ref) <= bound * np.linalg.norm(ref)


@pytest.mark.parametrize("storage,tol", [('fp32', 1e-6), ('fp16', 1e-3)])
@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
def test_advdiff_steps(fmt, storage, tol):
    p = W.advdiff_bump(n=24, nsteps=6)
    p.precision = storage
    log_case('cb_advdiff_24', fmt=fmt, storage=storage)
    st = M.from_problem(p, fmt=fmt, compute=A.FP64)
    st.step(p.nsteps)
    u = st.get_u()
    st.close()
    ref = closed_form.evolve(p.u0, p.kind, p.bc, p.diff, p.b, p.dt, p.nsteps, tableaus.by_name(p.tableau))
    assert rel_l2(u, ref) <= tol


@pytest.mark.parametrize("storage,tol", [('fp32', 1e-6), ('fp16', 1e-3)])
def test_heat_steps(storage, tol):
    p = W.heat_modes(n=24, nsteps=8)
    p.precision = storage
    log_case('cb_heat_24', storage=storage)
    st = M.from_problem(p, compute=A.FP64)
    st.step(p.nsteps)
    u = st.get_u()
    st.close()
    ref = closed_form.evolve_heat(p.u0, p.diff, p.dt, p.nsteps, tableaus.by_name(p.tableau))
    assert rel_l2(u, ref) <= tol


@pytest.mark.parametrize("storage,tol", [('fp32', 1e-6), ('fp16', 3e-3)])
def test_fdm_apply_with_fp64_arithmetic(storage, tol):
    shape = (20, 12, 9)
    log_case('cb_fdm', storage=storage)
    prec = cb(storage, 'cg', precond='fdm')
    st = M.Stepper(shape, W.DIRICHLET, W.HEAT, 1.3, (0, 0, 0), A.FMT_STENCIL, 'SDIRK3', prec, 2e-3)
    sigma = st.dt * (st.tab.a_hi[0] + st.tab.a_lo[0])
    xd = torch.from_numpy(np.random.default_rng(11).standard_normal(st.N)).to('cuda', DT[storage])
    y = st.apply(A.APPLY_FDM_LP, xd, stage=0).double().cpu().numpy()
    ref = fdm.FDM(shape, W.DIRICHLET, 0, 1.3, (0, 0, 0), sigma).apply(xd.double().cpu().numpy())
    st.close()
    assert np.linalg.norm(y - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("storage,tol", [('fp32', 1e-6), ('fp16', 3e-3)])
def test_complex_fdm_apply_with_fp64_arithmetic(storage, tol):
    """The complex-basis contractions in FP64 (FP64 MFMA) over FP32 / FP16 storage, against the
    exact Fourier inverse of the periodic stage matrix."""
    shape, kind, diff, b = (16, 12, 10), W.ADVDIFF, 1e-2, (1.0, 0.5, -0.25)
    log_case('cb_fdm_cx', storage=storage)
    prec = cb(storage, 'gmres', precond='fdm')
    st = M.Stepper(shape, W.PERIODIC, kind, diff, b, A.FMT_STENCIL, 'SDIRK3', prec, 2e-3)
    sigma = st.dt * (st.tab.a_hi[0] + st.tab.a_lo[0])
    xd = torch.from_numpy(np.random.default_rng(14).standard_normal(st.N)).to('cuda', DT[storage])
    y = st.apply(A.APPLY_FDM_LP, xd, stage=0).double().cpu().numpy()
    lam = closed_form.periodic_eigenvalues(shape, diff, b)
    xr = xd.double().cpu().numpy().reshape(shape[::-1])
    ref = np.real(np.fft.ifftn(np.fft.fftn(xr) / (1.0 - sigma * lam))).ravel()
    st.close()
    assert np.linalg.norm(y - ref) <= tol * np.linalg.norm(ref)
