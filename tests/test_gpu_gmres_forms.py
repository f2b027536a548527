"""The three kernel forms of the GMRES Arnoldi step (mprk_precisions.gm_form: gather kernels,
the product on z-marching tiles with the update kernel, the folded single launch per step) compute
the same method: each is checked through the C ABI against a sparse direct stage solve and the
oracle's time steps, on grids that exercise the tiles' edges (Dirichlet and periodic ends,
partial tiles in y and z, single planes, length-1 axes)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import workloads as W
from oracle import closed_form, operators, tableaus
from tests.gpu_util import log_case, reference_solution, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

FORMS = {'gather': A.GMFORM_GATHER, 'zsplit': A.GMFORM_ZSPLIT, 'folded': A.GMFORM_FOLDED}
SOLVE_BOUND = {'fp64': 1e-10, 'fp32': 1e-8, 'fp16': 1e-5}
STEP_TOL = {'fp64': 1e-12, 'fp32': 1e-6, 'fp16': 1e-3}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("storage", ['fp64', 'fp32', 'fp16'])
@pytest.mark.parametrize("case", [
    ((16, 12, 10), W.PERIODIC, (1.0, 0.5, 0.25), 'bj'),
    ((24, 9, 5), W.DIRICHLET, (1.0, -0.5, 0.25), 'bj'),    # partial tiles, Dirichlet ends
    ((32, 5, 1), W.PERIODIC, (0.7, 0.2, 0.1), 'none'),     # one plane, no preconditioner
])
def test_stage_solve_matches_sparse_lu(case, storage, form):
    shape, bc, b, precond = case
    log_case('gm_form_solve', shape=shape, bc=bc, storage=storage, form=form)
    prec = M.precisions(storage, 'gmres', precond=precond, gm_form=FORMS[form])
    st = M.Stepper(shape, bc, W.ADVDIFF, 1e-2, b, A.FMT_STENCIL, 'SDIRK3', prec, 5e-3)
    rhs = np.random.default_rng(4).standard_normal(st.N)
    x, info = st.solve(1, torch.from_numpy(rhs).cuda())
    sigma = 5e-3 * (st.tab.a_lo[st.tab.s + 1] + st.tab.a_hi[st.tab.s + 1])
    st.close()
    Mx = operators.stage_matrix(operators.operator(shape, bc, W.ADVDIFF, 1e-2, b), sigma)
    ref = spla.spsolve(Mx.tocsc(), rhs)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert info['converged'] == 1, info
    assert err <= SOLVE_BOUND[storage], (err, info)


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("storage", ['fp64', 'fp16'])
def test_time_steps_match_the_oracle(storage, form):
    p = W.advdiff_bump(n=32, nsteps=4)
    p.precision = storage
    log_case('gm_form_steps', storage=storage, form=form)
    over = dict(gm_form=FORMS[form])
    if storage == 'fp64':
        over.update(rtol=1e-12, outer_tol=1e-12)
    st = M.from_problem(p, **over)
    stats = st.step(p.nsteps)
    u = st.get_u()
    st.close()
    err = rel_l2(u, reference_solution(p))
    assert err <= STEP_TOL[storage], (err, stats)
    assert all(stats['converged'])


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("shape", [(8, 1, 1), (8, 1, 3), (16, 2, 1), (8, 3, 2)])
def test_degenerate_periodic_axes(shape, form):
    # length-1 and length-2 periodic axes: the tile's halo rows and planes wrap onto its own
    log_case('gm_form_edges', shape=shape, form=form)
    b = (1.0, 0.5, 0.25)
    prec = M.precisions('fp64', 'gmres', rtol=1e-12, outer_tol=1e-12, gm_form=FORMS[form])
    st = M.Stepper(shape, W.PERIODIC, W.ADVDIFF, 1e-2, b, A.FMT_STENCIL, 'SDIRK3', prec, 2e-3)
    u0 = np.random.default_rng(sum(shape)).standard_normal(shape[::-1]) + 2.0
    st.set_u(u0)
    st.step(3)
    u = st.get_u()
    st.close()
    ref = closed_form.evolve(u0, W.ADVDIFF, W.PERIODIC, 1e-2, b, 2e-3, 3, tableaus.by_name('SDIRK3'))
    err = rel_l2(u, ref)
    assert err <= 1e-12, err


def test_forms_the_problem_does_not_allow_are_rejected():
    # the folded form needs CGS1 and block-Jacobi or none; the tiled forms need the stencil format
    with pytest.raises(A.MprkError) as e:
        M.Stepper((16, 8, 8), W.PERIODIC, W.ADVDIFF, 1e-2, (1, 0, 0), A.FMT_STENCIL, 'SDIRK3',
                  M.precisions('fp32', 'gmres', reorth=1, gm_form=A.GMFORM_FOLDED), 2e-3)
    assert e.value.code == A.EUNSUPPORTED
    with pytest.raises(A.MprkError) as e:
        M.Stepper((16, 8, 8), W.PERIODIC, W.ADVDIFF, 1e-2, (1, 0, 0), A.FMT_CSR, 'SDIRK3',
                  M.precisions('fp32', 'gmres', gm_form=A.GMFORM_ZSPLIT), 2e-3)
    assert e.value.code == A.EUNSUPPORTED
