"""Batched form (one persistent launch per stage, hipGraph replay) vs the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log_case, reference_solution, rel_l2_floor

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi


def _run_batch(probs, prec, nsteps):
    b = M.Batch([{'shape': p.n, 'diff': p.diff, 'dt': p.dt} for p in probs], 'SDIRK3', prec)
    for i, p in enumerate(probs):
        b.set_u(i, p.u0)
    b.step(nsteps)
    us = [b.get_u(i) for i in range(len(probs))]
    st = [b.stats(i) for i in range(len(probs))]
    b.close()
    return us, st


def test_small_uneven_batch_matches_oracle():
    probs = W.heat_batch(count=6, nmin=13, nmax=40, nsteps=5)
    log_case('batch6', sizes=[p.n for p in probs])
    us, st = _run_batch(probs, M.precisions('fp32', 'cg'), 5)
    for p, u, s in zip(probs, us, st):
        p.nsteps = 5
        err = rel_l2_floor(u, reference_solution(p), p.u0)
        print(p.n, round(p.diff, 3), err, s['iters'], s['passes'])
        assert s['steps'] == 5
        assert err <= 1e-6


def test_batch_fp64_matches_oracle_tightly():
    probs = W.heat_batch(count=3, nmin=16, nmax=24, nsteps=3)
    log_case('batch3_fp64')
    us, st = _run_batch(probs, M.precisions('fp64', 'cg'), 3)
    for p, u in zip(probs, us):
        p.nsteps = 3
        assert rel_l2_floor(u, reference_solution(p), p.u0) <= 1e-12


def test_batch_is_deterministic():
    probs = W.heat_batch(count=4, nmin=16, nmax=48, nsteps=2)
    log_case('batch_repro')
    a, _ = _run_batch(probs, M.precisions('fp32', 'cg'), 2)
    b, _ = _run_batch(probs, M.precisions('fp32', 'cg'), 2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_batch_result_equals_single_problem_within_tolerance():
    probs = W.heat_batch(count=3, nmin=20, nmax=32, nsteps=4)
    log_case('batch_vs_alone')
    us, _ = _run_batch(probs, M.precisions('fp32', 'cg'), 4)
    for p, u in zip(probs, us):
        p.nsteps = 4
        st = M.from_problem(p)
        st.step(4)
        alone = st.get_u()
        st.close()
        assert rel_l2_floor(u, alone, p.u0) <= 1e-6


def test_full_batch_64_problems():
    # 64 heat problems, n uniform in [16, 96], kappa log-uniform in [0.1, 10], 20 steps
    probs = W.heat_batch()
    log_case('batch64', total_dof=sum(p.N for p in probs))
    us, st = _run_batch(probs, M.precisions('fp32', 'cg'), 20)
    worst = 0.0
    for i, (p, u, s) in enumerate(zip(probs, us, st)):
        err = rel_l2_floor(u, reference_solution(p), p.u0)
        if not err <= worst:
            print(f'problem {i}: n={p.n} kappa={p.diff:.3f} rel-L2={err:.3e} iters={s["iters"]} '
                  f'passes={s["passes"]}', flush=True)
        worst = max(worst, err)
        assert s['steps'] == 20
    print('batch64 worst rel-L2', worst)
    assert worst <= 1e-6


def test_autotune_restores_state_and_keeps_parity():
    probs = W.heat_batch(count=6, nmin=13, nmax=40, nsteps=3)
    log_case('batch_autotune', sizes=[p.n for p in probs])
    b = M.Batch([{'shape': p.n, 'diff': p.diff, 'dt': p.dt} for p in probs], 'SDIRK3',
                M.precisions('fp32', 'cg'))
    for i, p in enumerate(probs):
        b.set_u(i, p.u0)
    e, ru = b.autotune()
    assert e in (0.0, 0.25, 0.5, 0.75, 1.0) and ru in (1, 2, 4)
    assert sum(b.schedule) >= len(probs) and min(b.schedule) >= 1
    for i, p in enumerate(probs):  # autotuning leaves the states as they were
        assert np.array_equal(b.get_u(i), p.u0.reshape(b.get_u(i).shape))
        assert b.stats(i)['steps'] == 0
    b.step(3)
    for i, p in enumerate(probs):
        p.nsteps = 3
        assert b.stats(i)['steps'] == 3
        assert rel_l2_floor(b.get_u(i), reference_solution(p), p.u0) <= 1e-6
    b.close()


def test_autotune_refuses_a_fixed_schedule():
    probs = W.heat_batch(count=2, nmin=16, nmax=20, nsteps=1)
    log_case('batch_autotune_fixed')
    b = M.Batch([{'shape': p.n, 'diff': p.diff, 'dt': p.dt} for p in probs], 'SDIRK3',
                M.precisions('fp32', 'cg'), schedule=[2, 3])
    with pytest.raises(A.MprkError):
        b.autotune()
    b.close()


@pytest.mark.parametrize("mode", [A.START_RHS, A.START_SLOPE, A.START_SLOPE_EVAL, A.START_EXTRAP])
def test_batch_start_values_reach_the_oracle(mode):
    # every start value is iterated to the same tolerances: each problem within the FP32 bound
    probs = W.heat_batch(count=4, nmin=14, nmax=36, nsteps=4)
    log_case('batch_start', mode=mode, sizes=[p.n for p in probs])
    us, st = _run_batch(probs, M.precisions('fp32', 'cg', stage_start=mode), 4)
    for p, u, s in zip(probs, us, st):
        p.nsteps = 4
        err = rel_l2_floor(u, reference_solution(p), p.u0)
        print(mode, p.n, err, s['iters'], s['passes'])
        assert s['steps'] == 4
        assert err <= 1e-6


def test_batch_auto_start_is_the_extrapolation():
    probs = W.heat_batch(count=3, nmin=16, nmax=32, nsteps=3)
    log_case('batch_start_auto')
    a, _ = _run_batch(probs, M.precisions('fp32', 'cg'), 3)
    b, _ = _run_batch(probs, M.precisions('fp32', 'cg', stage_start=A.START_EXTRAP), 3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_batch_fp64_with_the_outer_stop_meets_the_outer_tolerance():
    # FP64 storage stopping its inner solves at the outer target: each problem within the outer
    # tolerance's reach of the oracle, and not more accurate than needed (the stop takes effect)
    probs = W.heat_batch(count=3, nmin=16, nmax=24, nsteps=3)
    log_case('batch3_fp64_outer_stop')
    tight, _ = _run_batch(probs, M.precisions('fp64', 'cg'), 3)
    loose, _ = _run_batch(probs, M.precisions('fp64', 'cg', inner_stop=A.STOP_OUTER), 3)
    for p, ut, ul in zip(probs, tight, loose):
        p.nsteps = 3
        ref = reference_solution(p)
        et, el = rel_l2_floor(ut, ref, p.u0), rel_l2_floor(ul, ref, p.u0)
        print(p.n, 'rtol stop', et, 'outer stop', el)
        assert et <= 1e-12 and el <= 1e-10
