"""Degenerate grids through the C ABI: a single unknown, axes of length 1 and 2 (periodic axes
whose neighbours wrap onto the point itself or onto each other; CSR rows with merged duplicate
columns), a single x-column (one value per group), against the oracle's closed forms; and the
fast-diagonalisation applies on such axes."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import closed_form, fdm, tableaus
from tests.gpu_util import log_case, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

SHAPES = [(1, 1, 1), (1, 1, 17), (2, 1, 3), (3, 2, 1), (1, 5, 1)]
TOL = {'fp64': 1e-12, 'fp16': 1e-3}   # FP64: the all-FP64 bar (measured <= 5e-16 here)


def _run(shape, bc, kind, diff, b, krylov, storage, fmt, nsteps=3, dt=2e-3):
    prec = M.precisions(storage, krylov, **({'rtol': 1e-12, 'outer_tol': 1e-12} if storage == 'fp64' else {}))
    st = M.Stepper(shape, bc, kind, diff, b, fmt, 'SDIRK3', prec, dt)
    u0 = np.random.default_rng(sum(shape)).standard_normal(shape[::-1]) + 2.0
    st.set_u(u0)
    st.step(nsteps)
    u = st.get_u()
    st.close()
    return u0, u


@pytest.mark.parametrize("storage", ['fp64', 'fp16'])
@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("shape", SHAPES)
def test_dirichlet_heat_on_degenerate_grids(shape, fmt, storage):
    log_case('edge_heat', shape=shape, fmt=fmt, storage=storage)
    u0, u = _run(shape, W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), 'cg', storage, fmt)
    ref = closed_form.evolve_heat(u0, 1.0, 2e-3, 3, tableaus.by_name('SDIRK3'))
    err = rel_l2(u, ref)
    assert err <= TOL[storage], err


@pytest.mark.parametrize("storage", ['fp64', 'fp16'])
@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("shape", SHAPES)
def test_periodic_advection_diffusion_on_degenerate_grids(shape, fmt, storage):
    log_case('edge_advdiff', shape=shape, fmt=fmt, storage=storage)
    b = (1.0, 0.5, 0.25)
    u0, u = _run(shape, W.PERIODIC, W.ADVDIFF, 1e-2, b, 'gmres', storage, fmt)
    ref = closed_form.evolve(u0, W.ADVDIFF, W.PERIODIC, 1e-2, b, 2e-3, 3, tableaus.by_name('SDIRK3'))
    err = rel_l2(u, ref)
    assert err <= TOL[storage], err


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 2, 1), (1, 5, 2)])
def test_fdm_apply_on_degenerate_axes(shape):
    log_case('edge_fdm', shape=shape)
    prec = M.precisions('fp64', 'cg', precond='fdm')
    st = M.Stepper(shape, W.DIRICHLET, W.HEAT, 1.3, (0, 0, 0), A.FMT_STENCIL, 'SDIRK3', prec, 2e-3)
    sigma = st.dt * (st.tab.a_hi[0] + st.tab.a_lo[0])
    x = np.random.default_rng(3).standard_normal(st.N)
    y = st.apply(A.APPLY_FDM_LP, torch.from_numpy(x).cuda(), stage=0).cpu().numpy()
    ref = fdm.FDM(shape, W.DIRICHLET, 0, 1.3, (0, 0, 0), sigma).apply(x)
    st.close()
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


# nx < 4 keeps the full x spectrum; from nx = 4 on only frequencies 0 .. nx/2 (rounded up to
# 4) pass through the y and z contractions: even and odd nx at the edge of that rule
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 3), (1, 3, 2), (3, 2, 2), (4, 3, 2),
                                   (5, 2, 3), (6, 1, 1), (7, 2, 1)])
def test_complex_fdm_apply_on_degenerate_axes(shape):
    log_case('edge_fdm_cx', shape=shape)
    b = (1.0, 0.5, -0.25)
    prec = M.precisions('fp64', 'gmres', precond='fdm')
    st = M.Stepper(shape, W.PERIODIC, W.ADVDIFF, 1e-2, b, A.FMT_STENCIL, 'SDIRK3', prec, 2e-3)
    sigma = st.dt * (st.tab.a_hi[0] + st.tab.a_lo[0])
    x = np.random.default_rng(4).standard_normal(st.N)
    y = st.apply(A.APPLY_FDM_LP, torch.from_numpy(x).cuda(), stage=0).cpu().numpy()
    lam = closed_form.periodic_eigenvalues(shape, 1e-2, b)
    ref = np.real(np.fft.ifftn(np.fft.fftn(x.reshape(shape[::-1])) / (1.0 - sigma * lam))).ravel()
    st.close()
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
