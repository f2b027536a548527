"""Steps replayed from a captured hipGraph (mprk_set_step_graph) against steered stepping.

Two handles on the same problem: one replays whole steps from its graph once its stages have
solve histories, the other is steered by the host.  After every call (several replays each,
with the program's own eager GPU work and synchronisations in between) both states must agree
to the solve tolerances and both must match the FP64 oracle; replayed calls must report their
steps in stats.graph_steps.  A state change that makes the recorded iteration counts too small
must fall back to steered steps inside the call with the same result.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import log_case, reference_solution, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

TOL = {'fp64': 1e-12, 'fp32': 1e-6, 'fp16': 1e-3}
# agreement of the two handles: both solve every stage to the outer tolerance
AGREE = {'fp64': 1e-11, 'fp32': 1e-6, 'fp16': 1e-3}


def _eager_noise():
    x = torch.randn(1 << 16, device='cuda')
    y = (x * 2.0 + 1.0).sum()
    torch.cuda.synchronize()
    return float(y)


def _pair(p, fmt, **over):
    if p.precision == 'fp64':
        over = {'rtol': 1e-12, 'outer_tol': 1e-12, **over}
    a = M.from_problem(p, fmt=fmt, **over)
    b = M.from_problem(p, fmt=fmt, **over)
    a.set_step_graph(True)
    return a, b


CASES = [
    ('heat_fp32_cg', lambda: W.heat_modes(n=24, nsteps=22), A.FMT_STENCIL),
    ('heat_fp64_cg_csr', lambda: W.heat_modes(n=20, nsteps=22), A.FMT_CSR),
    ('advdiff_fp16_gmres', lambda: W.advdiff_bump(n=32, nsteps=22), A.FMT_STENCIL),
]


@pytest.mark.parametrize("name,make,fmt", CASES, ids=[c[0] for c in CASES])
def test_replayed_steps_match_steered_steps(name, make, fmt):
    p = make()
    if name == 'heat_fp64_cg_csr':
        p.precision = 'fp64'
    log_case('step_graph', case=name)
    a, b = _pair(p, fmt)
    # the first call is steered on both (it records the stage histories)
    sa = a.step(2)
    b.step(2)
    assert sa['graph_steps'] == 0
    replayed = 0
    for call in range(4):
        sa = a.step(5)
        sb = b.step(5)
        _eager_noise()
        ua, ub = a.get_u(), b.get_u()
        replayed += sa['graph_steps']
        assert sb['graph_steps'] == 0
        assert sa['steps'] == sb['steps'] == 2 + 5 * (call + 1)
        assert sa['missed'] == 0 and sb['missed'] == 0
        d = rel_l2(ua, ub)
        print(name, 'call', call, 'graph steps', sa['graph_steps'], 'diff', d, sa['iters'], sb['iters'])
        assert d <= AGREE[p.precision], (call, d)
    assert replayed >= 15, replayed
    ref = reference_solution(p)
    ea = rel_l2(a.get_u(), ref)
    eb = rel_l2(b.get_u(), ref)
    a.close()
    b.close()
    print(name, 'oracle rel-L2 graph', ea, 'steered', eb)
    assert ea <= TOL[p.precision] and eb <= TOL[p.precision]


@pytest.mark.parametrize("tab", ['4S3PC', 'MID2'])
def test_replays_with_split_and_corrected_tableaus(tab):
    p = W.heat_modes(n=16, nsteps=12)
    p.tableau = tab
    log_case('step_graph_tableau', tab=tab)
    a, b = _pair(p, A.FMT_STENCIL)
    a.step(2)
    b.step(2)
    sa = a.step(10)
    b.step(10)
    assert sa['graph_steps'] > 0
    d = rel_l2(a.get_u(), b.get_u())
    e = rel_l2(a.get_u(), reference_solution(p))
    a.close()
    b.close()
    print(tab, 'diff', d, 'oracle', e)
    assert d <= AGREE['fp32'] and e <= TOL['fp32']


def test_a_stage_needing_more_passes_falls_back_to_steered_steps():
    # histories recorded without a reaction (one or two passes per stage); a strong linear
    # reaction then makes each stage need ~25 simplified-Newton passes (contraction
    # dt a_ii r1 = 0.44), far more than the graph enqueues: the first replay holds its step, the
    # call finishes steered from the same state as the steered handle, and the results agree
    p = W.heat_modes(n=24, nsteps=10)
    log_case('step_graph_fallback')
    a, b = _pair(p, A.FMT_STENCIL, refine_max=60)
    a.step(3)
    b.step(3)
    for st in (a, b):
        st.set_reaction(2000.0, 0.0, 0.0)
    sa = a.step(6)
    sb = b.step(6)
    d = rel_l2(a.get_u(), b.get_u())
    print('fallback graph steps', sa['graph_steps'], 'diff', d, sa['passes'], sb['passes'])
    assert sa['steps'] == sb['steps'] == 9
    assert sa['missed'] == 0 and sb['missed'] == 0
    assert sa['graph_steps'] == 0
    assert d <= AGREE['fp32'], d
    # the next call replays again, captured from the new histories
    sa = a.step(4)
    sb = b.step(4)
    d = rel_l2(a.get_u(), b.get_u())
    a.close()
    b.close()
    print('after fallback graph steps', sa['graph_steps'], 'diff', d, sa['passes'], sb['passes'])
    assert sa['graph_steps'] > 0 and sa['missed'] == 0
    assert d <= AGREE['fp32'], d


def test_forcing_and_reaction_changes_rebuild_the_graph():
    p = W.heat_modes(n=16, nsteps=10)
    log_case('step_graph_rebuild')
    a, b = _pair(p, A.FMT_STENCIL, refine_max=30)
    a.step(2)
    b.step(2)
    a.step(3)
    b.step(3)
    g = np.random.default_rng(3).standard_normal(p.u0.shape)
    for st in (a, b):
        st.set_forcing(g)
        st.set_reaction(2.0, 0.0, -2.0)
    # (a's next call captures again and replays with the earlier histories; a stage that needs
    # more falls back to steered steps)
    a.step(2)
    b.step(2)
    sa = a.step(5)
    b.step(5)
    assert sa['graph_steps'] > 0
    d = rel_l2(a.get_u(), b.get_u())
    a.close()
    b.close()
    print('rebuild diff', d)
    assert d <= AGREE['fp32'], d


@pytest.mark.parametrize("workload", ['heat', 'advdiff'])
def test_replays_with_the_fdm_preconditioner(workload):
    if workload == 'heat':
        p = W.heat_modes(n=24, nsteps=12)
    else:
        p = W.advdiff_bump(n=32, nsteps=12)
    p.precond = 'fdm'
    log_case('step_graph_fdm', workload=workload)
    a, b = _pair(p, A.FMT_STENCIL)
    a.step(2)
    b.step(2)
    sa = a.step(10)
    b.step(10)
    assert sa['graph_steps'] > 0 and sa['missed'] == 0
    d = rel_l2(a.get_u(), b.get_u())
    e = rel_l2(a.get_u(), reference_solution(p))
    a.close()
    b.close()
    print(workload, 'fdm diff', d, 'oracle', e)
    assert d <= AGREE[p.precision] and e <= TOL[p.precision]


def test_strict_miss_inside_and_outside_the_graph_reports_enotconv():
    # a stage that cannot converge within refine_max even when steered: the graph holds the
    # step, the steered rerun misses too, the call returns MPRK_ENOTCONV and u stays at the last
    # step whose stages all converged -- as for a handle without the graph
    p = W.heat_modes(n=16, nsteps=6)
    log_case('step_graph_strict')
    a, b = _pair(p, A.FMT_STENCIL, refine_max=3, strict=1)
    a.step(2)
    b.step(2)
    ua0, ub0 = a.get_u(), b.get_u()
    for st in (a, b):
        st.set_reaction(2000.0, 0.0, 0.0)  # needs ~25 passes: 3 are not enough
    ra, sa = a.step(3, check=False)
    rb, sb = b.step(3, check=False)
    ua, ub = a.get_u(), b.get_u()
    a.close()
    b.close()
    print('strict rc', ra, rb, sa['steps'], sb['steps'], sa['missed'], sb['missed'])
    assert ra == A.ENOTCONV and rb == A.ENOTCONV
    assert sa['steps'] == sb['steps'] == 2
    assert np.array_equal(ua, ua0) and np.array_equal(ub, ub0)


def test_replays_with_fp64_arithmetic_over_fp16_storage():
    # the compressed-basis engine (FP64 arithmetic, FP16 basis) under the graph
    p = W.advdiff_bump(n=32, nsteps=12)
    log_case('step_graph_cb')
    a, b = _pair(p, A.FMT_STENCIL, compute=A.FP64)
    a.step(2)
    b.step(2)
    sa = a.step(10)
    b.step(10)
    assert sa['graph_steps'] > 0 and sa['missed'] == 0
    d = rel_l2(a.get_u(), b.get_u())
    e = rel_l2(a.get_u(), reference_solution(p))
    a.close()
    b.close()
    print('cb diff', d, 'oracle', e)
    assert d <= AGREE['fp16'] and e <= TOL['fp16']
