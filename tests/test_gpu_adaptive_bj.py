"""Adaptive-precision block-Jacobi (mprk_precisions.bj_adapt_tol > 0) through the C ABI: the
apply against the oracle's block inverses within the rounding of each chunk's storage type, and
time steps against the oracle's closed forms with inverses stored below, at and above the
vector storage precision."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import krylov, operators
from tests.gpu_util import log_case, reference_solution, rel_l2

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi

U = {A.FP64: 2.0 ** -53, A.FP32: 2.0 ** -24, A.FP16: 2.0 ** -11}
UT = [2.0 ** -4, 2.0 ** -11, 2.0 ** -24, 2.0 ** -53]  # chunk type 0 FP8 (E4M3), 1, 2, 3
TINY = {A.FP64: 0.0, A.FP32: 2.0 ** -150, A.FP16: 2.0 ** -25}
NP = {A.FP64: np.float64, A.FP32: np.float32, A.FP16: np.float16}
CASES = [
    ((16, 16, 16), W.DIRICHLET, W.HEAT, 1.0, (0.0, 0.0, 0.0)),
    ((13, 9, 7), W.DIRICHLET, W.HEAT, 2.5, (0.0, 0.0, 0.0)),          # nx % 4 != 0, N % 8 != 0
    ((32, 20, 12), W.PERIODIC, W.ADVDIFF, 1e-2, (1.0, 0.5, 0.25)),
]


def row_types(inv, N, bs, vec, tol):
    """Storage type of every row under the rule (lowest type with u * cond_1 <= tol, widest per
    chunk of 64 lane groups of vec rows)."""
    t_blk = []
    for bi, Di in enumerate(inv):
        s = bi * bs
        n1 = np.abs(np.linalg.inv(Di)).sum(axis=0).max()
        kappa = n1 * np.abs(Di).sum(axis=0).max()
        t = 3
        if UT[0] * kappa + 2.0 ** -10 * Di.shape[0] * n1 <= tol and np.abs(Di).max() <= 448.0:
            t = 0
        elif UT[1] * kappa <= tol and np.abs(Di).max() < 6.0e4:
            t = 1
        elif UT[2] * kappa <= tol:
            t = 2
        t_blk.append(t)
    nch = -(-(-(-len(inv) * bs // vec)) // 64)
    tags = [0] * nch
    for bi, t in enumerate(t_blk):
        tags[(bi * bs // vec) // 64] = max(tags[(bi * bs // vec) // 64], t)
    return np.array([tags[(r // vec) // 64] for r in range(N)])


@pytest.mark.parametrize("tol", [5e-1, 1e-1, 1e-5, 1e-13])
@pytest.mark.parametrize("storage", ['fp64', 'fp32', 'fp16'])
@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("case", CASES)
def test_adaptive_block_jacobi_apply(case, fmt, storage, tol):
    shape, bc, kind, diff, b = case
    log_case('bj_adaptive_apply', shape=shape, fmt=fmt, storage=storage, tol=tol)
    prec = M.precisions(storage, 'gmres', bj_adapt_tol=tol)
    st = M.Stepper(shape, bc, kind, diff, b, fmt, 'SDIRK3', prec, 2e-3)
    sd = st.prec.storage
    vec = st.launch_info()  # (the layout's lanes: 8 for FP16 with nx % 8 == 0, else 4 or 1)
    lanes = 8 if (sd == A.FP16 and shape[0] % 8 == 0) else (4 if shape[0] % 4 == 0 else 1)
    sigma = st.dt * st.tab.a_lo[0]
    rng = np.random.default_rng(3)
    x_lp = rng.standard_normal(st.N).astype(NP[sd])
    z = st.apply(A.APPLY_BJ_LP, torch.from_numpy(x_lp).cuda(), 0).cpu().numpy().astype(np.float64)
    Mx = operators.stage_matrix(operators.operator(shape, bc, kind, diff, b), sigma)
    inv = krylov.block_jacobi_inverses(Mx, 8)
    types = row_types(inv, st.N, 8, lanes, tol)
    counts = [int(np.sum(types[::1] == k)) for k in range(4)]
    st.close()
    assert sum(1 for c in vec['bj_chunks'] if c) == sum(1 for c in counts if c)
    xf = x_lp.astype(np.float64)
    ref = krylov.block_jacobi_apply(inv, xf, 8)
    absd = krylov.block_jacobi_apply([np.abs(d) for d in inv], np.abs(xf), 8)
    u_c = U[A.FP64] if sd == A.FP64 else U[A.FP32]
    u_inv = np.array(UT)[types]
    # FP8 entries: error at most max(2^-4 |x|, 2^-10) (spacing 2^-9 below the smallest normal)
    flush = np.where(types == 0, 2.0 ** -10, 0.0)
    absx_blk = krylov.block_jacobi_apply([np.ones_like(d) for d in inv], np.abs(xf), 8)
    bound = (2 * U[sd] * np.abs(ref) + (16 * u_c + 2 * u_inv) * absd + 2 * flush * absx_blk
             + TINY[sd])
    assert np.all(np.abs(z - ref) <= bound + 1e-300)


@pytest.mark.parametrize("fmt", [A.FMT_STENCIL, A.FMT_CSR])
@pytest.mark.parametrize("storage,tol", [('fp32', 1e-1), ('fp16', 1e-5), ('fp64', 1e-1),
                                         ('fp16', 5e-1), ('fp32', 5e-1), ('fp64', 5e-1)])
def test_adaptive_block_jacobi_heat_steps(storage, tol, fmt):
    # FP32 vectors with FP16 inverses, FP16 vectors with FP32 inverses, an all-FP64 solve with
    # FP16 inverses (the preconditioner's precision bounds only its quality, not the result)
    p = W.heat_modes(n=24, nsteps=6)
    p.precision = storage
    log_case('bj_adaptive_heat', storage=storage, tol=tol, fmt=fmt)
    over = dict(bj_adapt_tol=tol)
    if storage == 'fp64':
        over.update(rtol=1e-12, outer_tol=1e-12)
    st = M.from_problem(p, fmt=fmt, **over)
    stats = st.step(p.nsteps)
    u = st.get_u()
    chunks = st.launch_info()['bj_chunks']
    st.close()
    err = rel_l2(u, reference_solution(p))
    print(storage, tol, fmt, 'chunks', chunks, 'rel-L2', err)
    if tol == 5e-1:  # these blocks (cond_1 about 1.3) take FP8 at this tolerance
        assert chunks[0] > 0, chunks
    assert err <= {'fp64': 1e-12, 'fp32': 1e-6, 'fp16': 1e-3}[storage], (err, stats)
    assert all(stats['converged'])


@pytest.mark.parametrize("storage,tol", [('fp16', 1e-5), ('fp32', 1e-1), ('fp16', 2.5e-1)])
def test_adaptive_block_jacobi_advection_steps(storage, tol):
    p = W.advdiff_bump(n=32, nsteps=4)
    p.precision = storage
    log_case('bj_adaptive_adv', storage=storage, tol=tol)
    st = M.from_problem(p, bj_adapt_tol=tol)
    stats = st.step(p.nsteps)
    u = st.get_u()
    st.close()
    err = rel_l2(u, reference_solution(p))
    assert err <= {'fp32': 1e-6, 'fp16': 1e-3}[storage], (err, stats)
