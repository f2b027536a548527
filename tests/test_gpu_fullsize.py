"""Parity at the full workload sizes, in the configuration bench.py times.

128^3 heat (8 seeded sine modes, SDIRK3, dt 5e-4, 50 steps, FP32 block-Jacobi CG) and 256^3
periodic upwind advection-diffusion (seeded Gaussian bump, SDIRK3, dt 2e-3, 20 steps, FP16
GMRES(30) + block-Jacobi) against the exact modal closed forms of the FP64 DIRK (DST-I / FFT),
which the oracle evaluates at any size.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log_case, reference_solution, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

_REF = {}


def _ref(key, p):
    if key not in _REF:
        _REF[key] = reference_solution(p)
    return _REF[key]


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
def test_heat_modes_128_fp32(fmt):
    p = W.heat_modes()
    log_case('heat_modes_128', fmt=fmt)
    st = M.from_problem(p, fmt=fmt)
    stats = st.step(p.nsteps)
    err = rel_l2(st.get_u(), _ref('heat128', p))
    st.close()
    print('heat 128^3 fp32 rel-L2', err, stats)
    assert stats['steps'] == 50
    assert err <= 1e-6


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
def test_advdiff_bump_256_fp16(fmt):
    p = W.advdiff_bump()
    log_case('advdiff_bump_256', fmt=fmt)
    st = M.from_problem(p, fmt=fmt)
    stats = st.step(p.nsteps)
    err = rel_l2(st.get_u(), _ref('advdiff256', p))
    st.close()
    print('advdiff 256^3 fp16 rel-L2', err, stats)
    assert stats['steps'] == 20
    assert err <= 1e-3


# ---- the configurations bench.py runs, with its tolerances ----
import bench  # noqa: E402


def _bench_problem(workload, precond, precision=None):
    p = bench.make_problem(workload, precond)
    if precision:
        p.precision = precision
    return p


@pytest.mark.parametrize("precond", ['bj', 'fdm'])
@pytest.mark.parametrize("workload", ['heat128', 'advdiff256'])
def test_fp64_reference_integration_matches_the_oracle(workload, precond):
    """The bench measures its errors against the all-FP64 path solved to rtol = outer_tol =
    1e-12; that path is pinned here to the exact-solve closed form at the full size."""
    p = _bench_problem(workload, precond, 'fp64')
    log_case(f'fp64_reference_{workload}', precond=precond)
    st = M.from_problem(p, rtol=bench.REF_TOL, outer_tol=bench.REF_TOL)
    stats = st.step(p.nsteps)
    err = rel_l2(st.get_u(), _ref(workload, p))
    st.close()
    print(workload, precond, 'fp64 reference rel-L2', err, stats['iters'])
    # the stated bar of the all-FP64 path (measured: 1.4e-13 heat with block-Jacobi, at most
    # 9e-15 in the three other cases)
    assert err <= 1e-12, (workload, precond, err, stats['iters'])


@pytest.mark.parametrize("precond", ['bj', 'fdm'])
@pytest.mark.parametrize("workload,bound", [('heat128', 1e-6), ('advdiff256', 1e-3)])
def test_mixed_path_at_the_bench_tolerances(workload, bound, precond):
    p = _bench_problem(workload, precond)
    log_case(f'mixed_bench_{workload}', precond=precond, storage=p.precision)
    st = M.from_problem(p, **bench.MIXED_TOL[workload])
    stats = st.step(p.nsteps)
    err = rel_l2(st.get_u(), _ref(workload, p))
    st.close()
    print(workload, precond, p.precision, 'rel-L2', err, stats['iters'])
    assert err <= bound
