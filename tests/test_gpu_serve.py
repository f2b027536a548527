"""Serving on the GPU: jobs admitted while others run, overlapping on the device; each result
equals the same job run alone (same kernels, own handle and stream) within tolerance."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log_case, reference_solution, rel_l2_floor

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
from paper_2412_16638_amd import serve  # noqa: E402

TOL = {'fp64': 1e-12, 'fp32': 1e-6, 'fp16': 1e-3}


def test_mix_equals_alone():
    reqs = W.request_stream(count=8, rate=200.0, seed=11, nmin=16, nmax=28, smin=3, smax=6)
    log_case('serve_mix', n=len(reqs))
    be = serve.GpuBackend(keep_u=True, steps_per_call=2)
    out = serve.Server(be, max_active=4).run(reqs)
    assert out['n'] == 8 and out['failed'] == 0
    assert out['peak_active'] >= 2          # work overlapped on the device
    by_id = {r.rid: r for r in out['results']}
    for r in reqs:
        ok, _, alone = be.run(r.problem)
        mixed = by_id[r.rid].u
        tol = TOL[r.problem.precision]
        assert rel_l2_floor(mixed, alone, r.problem.u0) <= tol
        assert rel_l2_floor(mixed, reference_solution(r.problem), r.problem.u0) <= tol
    print('serve p50/p99', out['p50_s'], out['p99_s'], out['dof_steps_per_s'])
