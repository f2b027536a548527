"""Start values of the implicit stage solves (mprk_precisions.stage_start) through the C ABI.

The start value is the library's choice (the paper leaves it open): rhs, rhs + sigma k_{i-1}
for the stages after the first, additionally rhs + sigma f(u) for the first, or the slopes
extrapolated linearly in c (f(u) at c = 0).  Each is
iterated to the same tolerances, so every mode must match the FP64 oracle to the storage's
bound and the modes must agree with each other; a step depends on u alone, so the result does
not depend on how the steps are split into calls; AUTO is bitwise the mode it resolves to.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log_case, reference_nonlinear, reference_solution, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

TOL = {'fp64': 1e-12, 'fp32': 1e-6, 'fp16': 1e-3}
MODES = [A.START_RHS, A.START_SLOPE, A.START_SLOPE_EVAL, A.START_EXTRAP]


def _problem(name):
    if name == 'advdiff_fp16_gmres_bj':
        return W.advdiff_bump(n=32, nsteps=8), A.FMT_STENCIL
    if name == 'advdiff_fp16_gmres_bj_csr':
        return W.advdiff_bump(n=24, nsteps=6), A.FMT_CSR
    if name == 'advdiff_fp16_gmres_fdm':
        p = W.advdiff_bump(n=32, nsteps=8)
        p.precond = 'fdm'
        return p, A.FMT_STENCIL
    if name == 'heat_fp32_cg_bj':
        return W.heat_modes(n=24, nsteps=8), A.FMT_STENCIL
    if name == 'heat_fp32_gmres_4s3pc':
        p = W.heat_modes(n=20, nsteps=6)
        p.krylov = 'gmres'
        p.tableau = '4S3PC'
        return p, A.FMT_STENCIL
    if name == 'heat_fp64_gmres':
        p = W.heat_modes(n=16, nsteps=6)
        p.krylov = 'gmres'
        p.precision = 'fp64'
        return p, A.FMT_STENCIL
    raise KeyError(name)


def _run(p, fmt, calls=None, **over):
    if p.precision == 'fp64':
        over = {'rtol': 1e-12, 'outer_tol': 1e-12, **over}
    st = M.from_problem(p, fmt=fmt, **over)
    stats = None
    for n in (calls or [p.nsteps]):
        stats = st.step(n)
    u = st.get_u()
    info = st.launch_info()
    st.close()
    return u, stats, info


NAMES = ['advdiff_fp16_gmres_bj', 'advdiff_fp16_gmres_bj_csr', 'advdiff_fp16_gmres_fdm',
         'heat_fp32_cg_bj', 'heat_fp32_gmres_4s3pc', 'heat_fp64_gmres']


@pytest.mark.parametrize("name", NAMES)
def test_every_start_value_reaches_the_oracle(name):
    p, fmt = _problem(name)
    ref = reference_solution(p)
    us = []
    for mode in MODES:
        log_case('stage_start', case=name, mode=mode)
        u, stats, info = _run(p, fmt, stage_start=mode)
        err = rel_l2(u, ref)
        print(name, 'mode', mode, 'rel-L2', err, 'iters', stats['iters'], 'passes', stats['passes'])
        assert info['stage_start'] == mode
        assert stats['missed'] == 0
        assert err <= TOL[p.precision], (mode, err)
        us.append(u)
    # the modes agree to the tolerance each solve is iterated to
    for u in us[1:]:
        assert rel_l2(u, us[0]) <= 2 * TOL[p.precision]


@pytest.mark.parametrize("name", ['advdiff_fp16_gmres_bj', 'advdiff_fp16_gmres_fdm',
                                  'heat_fp32_cg_bj'])
def test_auto_is_bitwise_the_mode_it_resolves_to(name):
    p, fmt = _problem(name)
    log_case('stage_start_auto', case=name)
    ua, sa, ia = _run(p, fmt)
    assert ia['stage_start'] in MODES
    ub, sb, ib = _run(p, fmt, stage_start=ia['stage_start'])
    print(name, 'auto ->', ia['stage_start'], sa['iters'], sb['iters'])
    assert np.array_equal(ua, ub)
    assert sa['iters'] == sb['iters'] and sa['passes'] == sb['passes']


@pytest.mark.parametrize("mode", [A.START_SLOPE, A.START_SLOPE_EVAL, A.START_EXTRAP])
@pytest.mark.parametrize("name", ['advdiff_fp16_gmres_bj', 'advdiff_fp16_gmres_fdm',
                                  'heat_fp32_cg_bj'])
def test_result_does_not_depend_on_the_call_split(name, mode):
    # a step starts from values of its own stages (and f(u)), never from an earlier call
    p, fmt = _problem(name)
    log_case('stage_start_split', case=name, mode=mode)
    u1, _, _ = _run(p, fmt, calls=[p.nsteps], stage_start=mode)
    u2, _, _ = _run(p, fmt, calls=[1, 3, p.nsteps - 4], stage_start=mode)
    assert np.array_equal(u1, u2)


@pytest.mark.parametrize("mode", [A.START_SLOPE, A.START_EXTRAP])
def test_set_u_between_calls_restarts_cleanly(mode):
    # a new state between calls: the next step's first stage must not start from the old slopes
    p, fmt = _problem('advdiff_fp16_gmres_bj')
    log_case('stage_start_set_u', mode=mode)
    a = M.from_problem(p, fmt=fmt, stage_start=mode)
    a.step(3)
    a.set_u(p.u0)
    a.step(p.nsteps)
    ua = a.get_u()
    a.close()
    ub, _, _ = _run(p, fmt, stage_start=mode)
    assert np.array_equal(ua, ub)


def test_extrapolation_with_an_explicit_first_stage():
    # a first stage with a_11 = 0 computes f(u) as k_0 itself: the second stage starts from
    # k_0, the third extrapolates from k_0 and k_1
    p = W.heat_modes(n=16, nsteps=6)
    log_case('stage_start_explicit_first')
    us = []
    for mode in (A.START_RHS, A.START_EXTRAP):
        t = A.mprk_tableau_builtin(A.TAB_SDIRK3)
        s = t.s
        # a 4-stage tableau: an explicit first stage, then SDIRK3 (stiffly accurate, order 3)
        e = A.mprk_tableau()
        e.s = s + 1
        for i in range(s):
            for j in range(s):
                e.a_hi[(i + 1) * (s + 1) + (j + 1)] = t.a_hi[i * s + j]
                e.a_lo[(i + 1) * (s + 1) + (j + 1)] = t.a_lo[i * s + j]
        for i in range(s):
            e.b[i + 1] = t.b[i]
        prec = M.precisions('fp32', 'cg', stage_start=mode, rtol=1e-3, outer_tol=1e-10)
        st = M.Stepper(p.n, p.bc, p.kind, p.diff, p.b, A.FMT_STENCIL, e, prec, p.dt)
        st.set_u(p.u0)
        stats = st.step(p.nsteps)
        assert stats['missed'] == 0
        us.append(st.get_u())
        st.close()
    assert rel_l2(us[1], us[0]) <= 1e-8


@pytest.mark.parametrize("mode", MODES)
def test_start_values_with_a_reaction(mode):
    p = W.advdiff_fisher(n=32, nsteps=4)
    log_case('stage_start_reaction', mode=mode)
    u, stats, _ = _run(p, A.FMT_STENCIL, stage_start=mode, refine_max=30)
    err = rel_l2(u, reference_nonlinear(p, None))
    print('fisher mode', mode, 'rel-L2', err, stats['passes'])
    assert stats['missed'] == 0
    assert err <= TOL[p.precision], err
