"""Convergence-failure paths through the C ABI, forced from the host with iteration caps and
tolerances, so every kernel still ends normally.

* The one-solve mode (refine_max = 0, Section "Implementation of the Mixed-precision
  Runge--Kutta methods": one conversion, one low-precision solve) has no later pass that would
  absorb a solve cut short, so each solve must run to its own stopping rule even when a later
  step needs more iterations than the handle's history predicts.
* A solve stopped by its iteration cap is reported (converged = 0, counted in `missed`) and is
  not an error without strict, as the paper's runs keep stepping after a solve that did not
  converge (the "no convergence" entries of Table tbl:iterations).
* With strict, a missed stage in any step of the call returns MPRK_ENOTCONV and leaves u at the
  last step whose stages all met their tolerance; the next call starts afresh.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log_case

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi


def _smooth_and_rough(krylov, n=16):
    """A problem, a state whose stage systems are solved in one or two Krylov iterations
    without a preconditioner (an eigenvector of the stage matrix, or a pair of conjugate ones),
    and a random state that needs many more."""
    if krylov == 'cg':
        p = W.heat_modes(n=n, nsteps=1)
        smooth = W.sine_mode((n, n, n), (1, 1, 1))
    else:
        p = W.advdiff_bump(n=n, nsteps=1, dt=2e-2)
        x = W.axis_nodes(n, W.PERIODIC)
        smooth = np.broadcast_to(np.cos(2 * np.pi * x)[None, None, :], (n, n, n)).copy()
    p.krylov = krylov
    return p, smooth, W.random_field(n, 11)


@pytest.mark.parametrize('krylov', ['cg', 'gmres'])
def test_one_solve_mode_finishes_a_solve_longer_than_predicted(krylov):
    p, smooth, rough = _smooth_and_rough(krylov)
    log_case('one_solve_longer_than_predicted', krylov=krylov)
    over = dict(refine_max=0, rtol=1e-6)
    p.precision = 'fp32'
    p.precond = 'none'
    # handle A: a first step whose solves take 1-2 iterations sets the history, then a rough state
    a = M.from_problem(p, **over)
    a.set_u(smooth)
    s1 = a.step(1)
    a.set_u(rough)
    s2 = a.step(1)
    ua = a.get_u().copy()
    a.close()
    # handle B: the rough state on a fresh handle (no history: every solve is polled)
    b = M.from_problem(p, **over)
    b.set_u(rough)
    sb = b.step(1)
    ub = b.get_u().copy()
    b.close()
    print('smooth', s1['iters'], 'rough after history', s2['iters'], 'fresh', sb['iters'])
    assert max(s1['iters']) + 1 < min(s2['iters'])     # the prediction is exercised
    assert s2['iters'] == sb['iters']
    assert all(s2['converged']) and s2['missed'] == 0
    assert np.array_equal(ua, ub)


@pytest.mark.parametrize('krylov', ['cg', 'gmres'])
def test_solve_stopped_by_its_iteration_cap_is_reported_not_an_error(krylov):
    # tolerance 1e-9 with FP32 storage and at most 3 iterations: no solve can meet it
    p, _, rough = _smooth_and_rough(krylov)
    p.precision = 'fp32'
    log_case('capped_solve_reported', krylov=krylov)
    st = M.from_problem(p, refine_max=0, rtol=1e-9, maxit=3)
    st.set_u(rough)
    before = st.get_u().copy()
    rc, stats = st.step(3, check=False)
    after = st.get_u()
    st.close()
    print(rc, stats)
    assert rc == A.OK
    assert stats['steps'] == 3
    assert stats['converged'] == [0, 0, 0]
    assert stats['missed'] == 3 * 3          # every stage of every step of the call
    assert all(0 < it <= 3 for it in stats['iters'])
    assert not np.array_equal(before, after)  # stepping continued


def test_strict_miss_returns_enotconv_and_keeps_u_at_the_last_good_step():
    p, smooth, rough = _smooth_and_rough('cg')
    p.precision = 'fp64'
    p.precond = 'none'
    log_case('strict_miss')
    # one CG iteration per pass, two passes: exact for the sine mode, far from 1e-10 otherwise
    st = M.from_problem(p, strict=1, maxit=1, refine_max=2, rtol=1e-12, outer_tol=1e-10)
    st.set_u(smooth)
    st.step(2)                                # both steps meet the tolerance
    assert st.state()[1] == 2
    st.set_u(rough)
    rc, stats = st.step(3, check=False)
    print(rc, stats)
    assert rc == A.ENOTCONV
    assert np.array_equal(st.get_u(), rough)  # no step of this call was combined
    assert st.state()[1] == 2
    assert stats['missed'] >= 1
    # the halt belongs to the failed call: a later call steps again
    st.set_u(smooth)
    s = st.step(1)
    assert s['missed'] == 0 and st.state()[1] == 3
    st.close()


def test_strict_counts_every_step_of_the_call():
    # refine_max = 1 with FP32 storage: one pass per stage cannot reach outer_tol 1e-10, so every
    # stage misses; without strict the call reports all of them and keeps stepping
    p, _, rough = _smooth_and_rough('cg')
    p.precision = 'fp32'
    log_case('missed_counts')
    st = M.from_problem(p, refine_max=1, outer_tol=1e-10)
    st.set_u(rough)
    rc, stats = st.step(4, check=False)
    st.close()
    assert rc == A.OK and stats['steps'] == 4
    assert stats['missed'] == 4 * 3
