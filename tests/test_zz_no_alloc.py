"""The allocation-free bind (mprk_bind_static) against the ordinary one, through the C ABI.

Two calls in a row on the device's one static scratch, the second with a smaller problem: each
result must equal, bit for bit, the same problem stepped with a caller-owned workspace (the
kernels and launch shapes are the same; only the workspace address differs).  A handle whose
static binding was taken over by a later bind must refuse to step.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import log_case, reference_solution, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi
S = M.stepper


def _handle(p, **over):
    prec = S.precisions(p.precision, p.krylov, precond=p.precond, **over)
    g = A.mprk_grid(p.n, p.n, p.n, p.bc)
    o = A.mprk_operator(p.kind, A.FMT_STENCIL, p.diff, (A.C.c_double * 3)(*p.b))
    stream = torch.cuda.current_stream()
    return A.mprk_create(g, o, S.tableau(p.tableau), prec, p.dt, stream.cuda_stream)


def _u(p):
    return torch.from_numpy(np.ascontiguousarray(p.u0, dtype=np.float64).ravel()).cuda()


def _run_static(p):
    h = _handle(p)
    assert A.mprk_workspace_bytes(h) <= A.STATIC_SCRATCH_BYTES
    u = _u(p)
    A.mprk_bind_static(h, u.data_ptr())
    rc, st = A.mprk_step(h, p.nsteps)
    A.check(rc, 'mprk_step')
    torch.cuda.synchronize()
    return h, u.cpu().numpy().reshape(p.u0.shape), st


def _run_caller_workspace(p):
    h = _handle(p)
    nb = A.mprk_workspace_bytes(h)
    ws = torch.empty(nb, dtype=torch.uint8, device='cuda')
    u = _u(p)
    A.mprk_bind(h, u.data_ptr(), ws.data_ptr(), nb)
    rc, st = A.mprk_step(h, p.nsteps)
    A.check(rc, 'mprk_step')
    torch.cuda.synchronize()
    A.mprk_destroy(h)
    return u.cpu().numpy().reshape(p.u0.shape), st


def test_static_bind_matches_the_caller_workspace_twice_second_smaller():
    first = W.advdiff_bump(n=32, nsteps=3)        # FP16 GMRES(30) + block-Jacobi(8)
    second = W.heat_modes(n=20, nsteps=4)         # FP32 CG + block-Jacobi(8), smaller
    log_case('static_bind', first=first.name, second=second.name)
    h1, u1, s1 = _run_static(first)
    r1, t1 = _run_caller_workspace(first)
    assert np.array_equal(u1, r1) and s1['iters'] == t1['iters']
    assert rel_l2(u1, reference_solution(first)) <= 1e-3
    h2, u2, s2 = _run_static(second)
    r2, t2 = _run_caller_workspace(second)
    assert np.array_equal(u2, r2) and s2['iters'] == t2['iters']
    assert rel_l2(u2, reference_solution(second)) <= 1e-6
    # the first handle's static binding was taken over by the second bind
    rc, _ = A.mprk_step(h1, 1)
    assert rc == A.ESTATE
    A.mprk_destroy(h1)
    A.mprk_destroy(h2)


def test_static_bind_rejects_a_workspace_beyond_the_scratch():
    p = W.advdiff_bump(n=160, nsteps=1)
    p.u0 = None
    h = _handle(p)
    try:
        assert A.mprk_workspace_bytes(h) > A.STATIC_SCRATCH_BYTES
        u = torch.zeros(p.N, dtype=torch.float64, device='cuda')
        with pytest.raises(A.MprkError) as e:
            A.mprk_bind_static(h, u.data_ptr())
        assert e.value.code == A.ENOMEM
    finally:
        A.mprk_destroy(h)
