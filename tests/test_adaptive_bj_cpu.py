"""The adaptive-precision block-Jacobi layout on the host (no device): the storage type the
library picks for every chunk of 64 lane groups equals the rule evaluated here from the oracle's
stage matrix -- the lowest of FP8 (E4M3), FP16, FP32, FP64 whose unit roundoff times the block's
1-norm condition number (for FP8 plus its flush of entries below 2^-9, n 2^-10 ||D||_1) is within
the tolerance and whose range holds the inverse (Ginkgo's adaptive block-Jacobi, cited in the
paper's Introduction; the rule's constants are this library's reading)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import operators

A = pytest.importorskip('paper_2412_16638_amd._abi')

U = [2.0 ** -4, 2.0 ** -11, 2.0 ** -24, 2.0 ** -53]  # FP8 (E4M3), FP16, FP32, FP64


def expected_chunk_types(shape, bc, kind, diff, b, sigma, bs, vec, tol):
    M = operators.stage_matrix(operators.operator(shape, bc, kind, diff, b), sigma).tocsr()
    N = M.shape[0]
    nblk = -(-N // bs)
    t_blk = []
    for s in range(0, N, bs):
        D = M[s:min(s + bs, N), s:min(s + bs, N)].toarray()
        Di = np.linalg.inv(D)
        n1 = np.abs(D).sum(axis=0).max()
        kappa = n1 * np.abs(Di).sum(axis=0).max()
        t = 3
        if U[0] * kappa + 2.0 ** -10 * D.shape[0] * n1 <= tol and np.abs(Di).max() <= 448.0:
            t = 0
        elif U[1] * kappa <= tol and np.abs(Di).max() < 6.0e4:
            t = 1
        elif U[2] * kappa <= tol:
            t = 2
        t_blk.append(t)
    groups = -(-nblk * bs // vec)
    nch = -(-groups // 64)
    tags = [0] * nch
    for bi, t in enumerate(t_blk):
        ch = (bi * bs // vec) // 64
        tags[ch] = max(tags[ch], t)
    return [tags.count(k) for k in range(4)]


def _launch_info(shape, bc, kind, diff, b, storage, krylov, tol, dt=2e-3):
    g = A.mprk_grid(*shape, bc)
    o = A.mprk_operator(kind, A.FMT_STENCIL, diff, (C.c_double * 3)(*b))
    t = A.mprk_tableau_builtin(A.TAB_SDIRK3)
    p = A.mprk_precisions_default(storage, krylov)
    p.bj_adapt_tol = tol
    h = A.mprk_create(g, o, t, p, dt, 0)
    try:
        return A.mprk_launch_info_get(h), t
    finally:
        A.mprk_destroy(h)


@pytest.mark.parametrize("tol", [5e-1, 1e-1, 1e-5, 1e-12])
@pytest.mark.parametrize("case", [
    ((16, 12, 10), W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), A.FP32, A.CG, 4),
    ((13, 9, 7), W.DIRICHLET, W.HEAT, 2.5, (0, 0, 0), A.FP64, A.CG, 1),
    ((32, 20, 12), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25), A.FP16, A.GMRES, 8),
])
def test_chunk_types_follow_the_condition_rule(case, tol):
    shape, bc, kind, diff, b, storage, krylov, vec = case
    li, t = _launch_info(shape, bc, kind, diff, b, storage, krylov, tol)
    sigma = 2e-3 * t.a_lo[0]
    want = expected_chunk_types(shape, bc, kind, diff, b, sigma, 8, vec, tol)
    assert li['bj_chunks'] == want


def test_a_tolerance_between_block_conditions_mixes_types():
    # 4s3pC has four distinct diagonal entries, so four stage matrices with block condition
    # numbers growing with tau a_ii; a tolerance between the smallest and the largest stores the
    # better-conditioned ones' inverses in FP16 and the others' in FP32 (the operator's blocks
    # are alike within one stage matrix, so the types differ between matrices, not chunks)
    shape, dt = (16, 12, 10), 2e-2
    t = A.mprk_tableau_builtin(A.TAB_4S3PC)
    s = t.s
    sigmas = sorted({dt * (t.a_hi[i * s + i] + t.a_lo[i * s + i]) for i in range(s)})
    kap = []
    for sg in sigmas:
        M = operators.stage_matrix(operators.operator(shape, W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0)),
                                   sg).tocsr()
        D = M[0:8, 0:8].toarray()
        kap.append(np.abs(D).sum(axis=0).max() * np.abs(np.linalg.inv(D)).sum(axis=0).max())
    tol = U[1] * np.sqrt(min(kap) * max(kap))
    g = A.mprk_grid(*shape, W.DIRICHLET)
    o = A.mprk_operator(W.HEAT, A.FMT_STENCIL, 1.0, (C.c_double * 3)(0, 0, 0))
    p = A.mprk_precisions_default(A.FP32, A.CG)
    p.bj_adapt_tol = tol
    h = A.mprk_create(g, o, t, p, dt, 0)
    li = A.mprk_launch_info_get(h)
    A.mprk_destroy(h)
    want = [0, 0, 0, 0]
    for sg in sigmas:
        c = expected_chunk_types(shape, W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), sg, 8, 4, tol)
        want = [a + b for a, b in zip(want, c)]
    assert li['bj_chunks'] == want
    assert want[1] > 0 and want[2] > 0


def test_a_loose_tolerance_stores_fp8_inverses():
    # advection-diffusion blocks on a small periodic grid: cond_1 about 1.09, so the FP8 bound
    # 2^-4 kappa + 8 2^-10 ||D||_1 (about 0.077) qualifies at 0.1 and not at 0.05
    case = ((32, 16, 8), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25))
    for tol, fp8 in ((0.1, True), (0.05, False)):
        li, t = _launch_info(*case, A.FP16, A.GMRES, tol)
        want = expected_chunk_types(*case, 2e-3 * t.a_lo[0], 8, 8, tol)
        assert li['bj_chunks'] == want
        assert (want[0] > 0) == fp8, (tol, want)


def test_adaptive_needs_one_inverse_per_block():
    g = A.mprk_grid(16, 16, 16, 0)
    o = A.mprk_operator(0, A.FMT_STENCIL, 1.0, (C.c_double * 3)(0, 0, 0))
    p = A.mprk_precisions_default(A.FP32, A.CG)
    p.bj_adapt_tol = 0.1
    p.bj_shared = 1
    with pytest.raises(A.MprkError) as e:
        A.mprk_create(g, o, A.mprk_tableau_builtin(A.TAB_SDIRK3), p, 1e-3, 0)
    assert e.value.code == A.EINVAL
