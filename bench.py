#!/usr/bin/env python3
"""Benchmark: DOF-steps/s of mixed-precision DIRK time stepping on one MI355X.

Workload (default): 256^3 periodic upwind advection-diffusion (nu = 1e-2, b = (1, 0.5, 0.25)),
seeded Gaussian bump, SDIRK3, dt = 2e-3; implicit stages by GMRES(30) + block-Jacobi(8) with
FP16 storage / FP32 arithmetic inside the FP64 residual loop; FP64 explicit corrections and
step combination; matrix-free stencil.  One bench "step" is one Runge--Kutta time step of the
whole grid.  Also reported: the error of a full 20-step integration against the all-FP64 GPU
path solved to 1e-12 (the reference; the GPU tests pin that path to the oracle's exact-solve
closed form at this size), the all-FP64 GPU path at matched error, the dominant kernel
against the HBM roofline (HIP events on the library's stream), and the oracle's own time
stepping the method on the host (cpu_baseline, the only use of the oracle here).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-steps/s mixed vs FP64 at matched error; % peak HBM; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print('[bench]', *a, file=sys.stderr, flush=True)


def algorithmic_bytes(kc: str, N: int, s: int, m: int, bs: int, worked: int, units: int,
                      nv_total: int = 0, fdm: bool = False, cb: int = 4,
                      csr_nnz_row: float = 0.0, zstored: bool = False,
                      inv_entry: float = 0.0) -> float:
    """Bytes each kernel class must move per its definition (each array touched once; halos
    and reduction partials not counted).  s = LP storage bytes, m = LP matrix bytes, bs = block,
    cb = bytes of the arithmetic type; csr_nnz_row > 0: CSR format with that many nonzeros per
    row (values, int32 column indices and row pointers read once per SpMV); inv_entry > 0: mean
    bytes per block-Jacobi inverse entry (adaptive precision), else m."""
    inv = bs * (inv_entry or m)  # block-Jacobi inverse row per unknown
    pre = (inv + s) if bs else 0  # fused block-Jacobi: inverse row read + preconditioned write
    csr_lp = csr_nnz_row * (m + 4) + 4 if csr_nnz_row else 0.0    # LP matrix of one SpMV
    csr_64 = csr_nnz_row * (8 + 4) + 4 if csr_nnz_row else 0.0    # FP64 matrix of one SpMV
    if kc == 'gm_matvec':
        return N * (worked * (s + s + csr_lp) + units * s)
    if kc == 'gm_orth':
        return N * (worked * (s + s + pre) + units * s)
    if kc == 'gm_reorth':  # w read, w' written, the basis read once (its second read hits cache)
        return N * (worked * (s + s) + units * s)
    if kc == 'gm_step':  # folded step: w_{j-1} read, v_j and w_j written, block-Jacobi rows read,
        # the basis before v_j read once (units = j + 1 vectors in the products, v_j among them)
        return N * (worked * (3 * s + inv) + (units - worked) * s)
    if kc == 'gm_close':  # the cycle's last norm: w and the basis read
        return N * (worked * s + units * s)
    if kc == 'gm_finish':
        if fdm:  # t = sum_i y_i v_i in the arithmetic type; P^-1 t and y += s z come after
            return N * (worked * cb + units * s)
        if zstored:  # y += s sum_i y_i BJ(v_i) from the stored directions: no inverse read
            return N * (worked * 16 + units * s)
        return N * (worked * (inv + 16) + units * s)
    if kc == 'gm_begin':
        return N * worked * (8 + s + pre)
    if kc == 'residual':
        return N * worked * (32 + csr_64)
    if kc == 'cg_begin':
        return N * worked * (8 + s + (inv + s if bs else 0))
    if kc == 'cg_dir':
        return N * worked * (4 * s + csr_lp)
    if kc == 'cg_upd':
        return N * worked * ((6 if fdm else 7) * s + inv)
    if kc == 'cg_rz':
        return N * worked * 2 * s
    if kc == 'apply64':  # f(u): u read, k written (the stencil's neighbours gathered)
        return N * worked * (16 + csr_64)
    if kc == 'promote':
        return N * worked * (16 + s)
    if kc == 'stage_rhs':
        return N * 8 * (worked * 3 + nv_total)
    if kc == 'combine':
        return N * 8 * (worked * 2 + nv_total)
    return 0.0


# Solve tolerances of the mixed path per workload: the solve error is kept well below both the
# scheme's temporal truncation error (3.6e-4 for the 128^3 heat run, 1.3e-6 for the 256^3
# advection-diffusion run, both from modal closed forms) and the stated bounds for the
# mixed paths (1e-6 with FP32 inner solves, 1e-3 with FP16 storage).  Empty: library defaults.
MIXED_TOL = {'heat128': dict(rtol=1e-3, outer_tol=1e-6), 'advdiff256': {}}

# residual tolerance (inner and outer) of the all-FP64 reference integration
REF_TOL = 1e-12

# FP64 comparison runs stop their inner solves at the outer target too, as the mixed path does
# by default (the FP64 references solved to REF_TOL keep solving each pass to rtol)
FP64_CMP = {'inner_stop': 1}


def make_problem(name: str, precond: str = 'bj'):
    import workloads as W
    if name == 'advdiff256':
        p = W.advdiff_bump()
    elif name == 'heat128':
        p = W.heat_modes()
    else:
        raise SystemExit(f'unknown workload {name}')
    if precond == 'fdm':
        p.precond = 'fdm'
    return p


# dense matrix-core peaks of the FDM contractions' arithmetic (FP64 MFMA for FP64 storage, FP32
# MFMA otherwise), TFLOP/s
MFMA_PEAK = {'fp64': 78.6, 'fp32': 157.3, 'fp16': 157.3}


def fdm_apply_flops(p) -> float:
    """Algorithmic flops per unknown of one fast-diagonalisation apply (six dense contractions,
    2 flops per real multiply-add).  Real basis (heat): 2 n per contraction.  Complex DFT basis
    (periodic advection, real data): the x transforms keep H = nx/2 + 1 frequencies rounded up
    to 4 (all nx below nx = 4); forward x real x complex (4 H), y and z forward and back complex x
    complex on H of nx x-slices (8 n H / nx each), backward x only the real part (4 H).  The
    kernels execute 3 real products per complex one in the middle four, 3/4 of their count."""
    n = p.n
    if p.kind == 0:
        return 4.0 * 3 * n
    H = (n // 2 + 1 + 3) & ~3
    if H > n:
        H = n
    return 8.0 * H + 16.0 * (n + n) * H / n


def workload_name(args) -> str:
    """The configuration a step-mode line measures, named by what it is."""
    pc = 'fdm' if args.precond == 'fdm' else 'bj8'
    base = (f'advdiff_upwind_periodic_256^3_sdirk3_dt2e-3_gmres30_{pc}_fp16'
            if args.workload == 'advdiff256' else f'heat_dirichlet_128^3_sdirk3_dt5e-4_cg_{pc}_fp32')
    return base + ('_fp64arith' if args.compute == 'fp64' else '')


def cpu_oracle_rate(workload: str, precond: str = 'bj'):
    """The oracle stepping the method on the host: FP64 DIRK with its own Krylov stage solver
    (GMRES(30) or CG + block-Jacobi(8), rtol 1e-10), one thread, setup excluded.  The sample is
    two steps of the workload's PDE on a smaller grid (128^3 for the 256^3 advection-diffusion
    run, 96^3 for the 128^3 heat run), sized to 10-30 s of CPU work.  With the fast-
    diagonalisation preconditioner the oracle's Krylov solver uses its FDM inverse, and the
    sample is eight steps of the 128^3 heat workload itself, or three steps of the advection-
    diffusion problem on 96^3 (complex bases)."""
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import dirk, operators, tableaus
    fdm = precond == 'fdm'
    p = (W.advdiff_bump(n=96 if fdm else 128) if workload == 'advdiff256'
         else W.heat_modes(n=128 if fdm else 96))
    K = operators.operator((p.n,) * 3, p.bc, p.kind, p.diff, p.b)
    tab = tableaus.by_name(p.tableau)
    solve = dirk.StageSolver(K, 'gmres' if p.krylov == 'gmres' else 'cg', rtol=1e-10, block=8,
                             restart=30,
                             fdm_problem=((p.n,) * 3, p.bc, p.kind, p.diff, p.b) if fdm else None)
    # steps sized to 10-30 s of host work: the BJ samples take ~6-10 s per step on the GPU
    # box's host, the FDM ones ~1.3 s (heat, 128^3) and ~3 s (advection, 96^3)
    steps = (8 if workload != 'advdiff256' else 3) if fdm else 2
    u = np.asarray(p.u0, dtype=np.float64).ravel().copy()
    with threadpool_limits(limits=1):
        for i in range(tab.s):
            if tab.A[i, i] != 0.0:
                solve._factor(p.dt * tab.A[i, i])
        t0 = time.perf_counter()
        for _ in range(steps):
            u = dirk.dirk_step(K, u, p.dt, tab, solve)
        t = time.perf_counter() - t0
    sample = (f'{steps} {p.tableau} step{"s" if steps > 1 else ""} of the '
              f'{"advection-diffusion" if p.kind else "heat"} problem '
              f'on a {p.n}^3 grid ({p.N} unknowns), FP64 oracle DIRK with its '
              f'{p.krylov.upper()} + {"FDM" if fdm else "block-Jacobi(8)"} stage solver to rtol 1e-10 '
              f'({sum(solve.iterations)} iterations), one thread, setup excluded; {t:.1f} s')
    return p.N * steps / t, sample, t


def run_integration(M, p, fmt, **over):
    st = M.from_problem(p, fmt=fmt, **over)
    stats = st.step(p.nsteps)
    u = st.get_u()
    st.close()
    return u, stats


# outer-pass limit of the semi-linear runs (each pass contracts the stage error by about
# dt a_ii max|R'|: 0.02-0.05 for the two reaction workloads)
NONLINEAR_PASSES = 30


def make_reaction_problem(name: str, precond: str = 'bj'):
    """The workload with a pointwise reaction: Fisher-KPP 20 u (1 - u) on the advection-diffusion
    bump, Allen-Cahn 50 (u - u^3) on the heat modes (scaled to max |u0| = 1)."""
    import workloads as W
    p = W.advdiff_fisher() if name == 'advdiff256' else W.heat_allen_cahn()
    if precond == 'fdm':
        p.precond = 'fdm'
    return p


def nonlinear_leg(M, args, fmt, bjs, mixed_over, K: int, Wm: int) -> dict:
    """The semi-linear variant of the workload: the mixed path (the FP64 outer loop iterates the
    non-linear stage equation, LP solves with I - sigma K) timed over K steps, its error against
    the all-FP64 path solved to REF_TOL, and the FP64 path at the mixed path's tolerances."""
    q = make_reaction_problem(args.workload, args.precond)
    r64 = make_reaction_problem(args.workload, args.precond)
    r64.precision = 'fp64'
    # the non-linear stage needs more outer passes than the linear defaults allow
    mixed_over = dict(mixed_over, refine_max=NONLINEAR_PASSES)
    ref, st_ref = run_integration(M, r64, fmt, rtol=REF_TOL, outer_tol=REF_TOL, bj_shared=bjs,
                                  refine_max=NONLINEAR_PASSES)
    um, sm = run_integration(M, q, fmt, bj_shared=bjs, **mixed_over)
    err = float(np.linalg.norm(um - ref) / np.linalg.norm(ref))
    st = M.from_problem(q, fmt=fmt, bj_shared=bjs, **mixed_over)
    st.autotune()
    t, stats, _ = time_steps(st, q.u0, K, Wm)
    st.close()
    pm = M.precisions(q.precision, q.krylov, **MIXED_TOL[args.workload])
    over64 = dict(rtol=pm.rtol, outer_tol=pm.outer_tol, bj_shared=bjs, refine_max=NONLINEAR_PASSES,
                  **FP64_CMP)
    u64, _ = run_integration(M, r64, fmt, **over64)
    e64 = float(np.linalg.norm(u64 - ref) / np.linalg.norm(ref))
    st64 = M.from_problem(r64, fmt=fmt, **over64)
    st64.autotune()
    t64, _, _ = time_steps(st64, r64.u0, K, Wm)
    st64.close()
    out = {'problem': q.name, 'reaction': list(q.reaction), 'value': q.N * K / t,
           'ms_per_step': t * 1e3 / K, 'err_vs_fp64_reference': err,
           'passes_per_stage': stats['passes'], 'iters_per_stage': stats['iters'],
           'reference_passes_per_stage': st_ref['passes'],
           'fp64_at_mixed_tolerances': {'value': q.N * K / t64, 'ms_per_step': t64 * 1e3 / K,
                                        'err_vs_fp64_reference': e64}}
    log(f'semi-linear {q.name}: {out["value"]:.4e} DOF-steps/s, rel-L2 {err:.3e}, '
        f'passes/stage {stats["passes"]}; FP64 at the same tolerances {q.N * K / t64:.4e}')
    return out


def fdm_leg(M, K: int, Wm: int) -> dict:
    """Both workloads with the paper's fast-diagonalisation preconditioner instead of
    block-Jacobi (stencil format): the mixed path timed over K steps, its error against the
    all-FP64 FDM path solved to REF_TOL, and the FP64 path at the mixed path's tolerances."""
    out = {}
    for name in ('heat128', 'advdiff256'):
        p = make_problem(name, 'fdm')
        q = make_problem(name, 'fdm')
        q.precision = 'fp64'
        ref, _ = run_integration(M, q, 0, rtol=REF_TOL, outer_tol=REF_TOL)
        over = dict(MIXED_TOL[name])
        u, _ = run_integration(M, p, 0, **over)
        err = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
        st = M.from_problem(p, **over)
        st.autotune()
        t, stats, _ = time_steps(st, p.u0, K, Wm)
        st.close()
        pm = M.precisions(p.precision, p.krylov, **over)
        st64 = M.from_problem(q, rtol=pm.rtol, outer_tol=pm.outer_tol, **FP64_CMP)
        st64.autotune()
        t64, _, _ = time_steps(st64, q.u0, K, Wm)
        st64.close()
        out[name] = {'value': p.N * K / t, 'ms_per_step': t * 1e3 / K, 'err_vs_fp64_reference': err,
                     'iters_per_stage': stats['iters'], 'passes_per_stage': stats['passes'],
                     'fp64_at_mixed_tolerances': {'value': q.N * K / t64,
                                                  'ms_per_step': t64 * 1e3 / K},
                     'lp_storage': p.precision, 'krylov': p.krylov}
        log(f'fdm {name}: {out[name]["value"]:.4e} DOF-steps/s, rel-L2 {err:.3e}; FP64 at the same '
            f'tolerances {q.N * K / t64:.4e}')
    return out


def host_info() -> dict:
    """The host the oracle ran on: core count, CPU model, BLAS threads, OMP_NUM_THREADS."""
    model = None
    try:
        with open('/proc/cpuinfo') as fh:
            for line in fh:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = [{'api': d.get('internal_api'), 'threads': d.get('num_threads')}
                for d in threadpool_info()]
    except Exception:
        pass
    return {'os_cpu_count': os.cpu_count(), 'cpu_model': model, 'blas': blas,
            'OMP_NUM_THREADS': os.environ.get('OMP_NUM_THREADS')}


def time_steps(st, u0, K: int, W: int, profile: bool = False):
    import torch
    st.set_u(u0)
    st.set_state(0.0, 0)
    if W:
        st.step(W)
    torch.cuda.synchronize()
    from paper_2412_16638_amd import _abi as AB
    if profile:
        AB.mprk_profile(st.h, True)
    t0 = time.perf_counter()
    stats = st.step(K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile:
        AB.mprk_profile(st.h, False)
        prof = {name: AB.mprk_profile_read(st.h, i) for i, name in enumerate(AB.KC_NAMES)}
    return dt, stats, prof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=3)
    ap.add_argument('--workload', default='advdiff256', choices=['advdiff256', 'heat128'])
    ap.add_argument('--fmt', default='stencil', choices=['stencil', 'csr'])
    ap.add_argument('--no-fp64', action='store_true', help='skip the FP64 matched-error leg')
    ap.add_argument('--no-cpu', action='store_true', help='skip the oracle / cpu_baseline leg')
    ap.add_argument('--mode', default='step', choices=['step', 'batch', 'serve', 'sweep'],
                    help='step: the 256^3 / 128^3 single-problem line (default); batch: 64 heat '
                         'problems in one persistent launch per stage; serve: 512 Poisson '
                         'requests; sweep: the paper\'s time-step and tolerance experiments')
    ap.add_argument('--slots', type=int, default=8,
                    help='serve mode: jobs admitted concurrently (each on its own stream)')
    ap.add_argument('--requests', type=int, default=512,
                    help='serve mode: requests replayed (the first ones of the seeded stream)')
    ap.add_argument('--no-pool', action='store_true',
                    help='serve: a fresh handle per job instead of the pool of idle handles')
    ap.add_argument('--serve-requests', type=int, default=64,
                    help='step mode: requests of the serving side leg (0 = skip it)')
    ap.add_argument('--no-batch', action='store_true', help='step mode: skip the batched side leg')
    ap.add_argument('--gm-form', default='auto', choices=['auto', 'gather', 'zsplit', 'folded'],
                    help='GMRES Arnoldi step kernels (mprk_precisions.gm_form)')
    ap.add_argument('--bj-adapt', type=float, default=0.0, metavar='TOL',
                    help='adaptive-precision block-Jacobi inverses (mprk_precisions.bj_adapt_tol) '
                         'for the headline run; the default run also times TOL = 0.25 beside it')
    ap.add_argument('--stage-start', default='auto', choices=['auto', 'rhs', 'slope', 'eval', 'extrap'],
                    help='start value of the implicit stage solves (mprk_precisions.stage_start)')
    ap.add_argument('--n', type=int, default=128,
                    help='sweep mode: grid points per axis of the paper\'s test problems')
    ap.add_argument('--quick', action='store_true',
                    help='profiling runs: skip the full-integration error check and side legs')
    ap.add_argument('--bj', default='per-block', choices=['per-block', 'shared'],
                    help='block-Jacobi inverse storage of the headline run')
    ap.add_argument('--precond', default='bj', choices=['bj', 'fdm'],
                    help='stage-solve preconditioner: block-Jacobi(8) (the configurations) or the '
                         'paper\'s fast-diagonalisation one (real basis for heat, complex DFT '
                         'basis with GMRES for the periodic advection-diffusion)')
    ap.add_argument('--compute', default='fp32', choices=['fp32', 'fp64'],
                    help='arithmetic of the low-precision solves: fp32 (the configurations) or '
                         'fp64 over the same storage (compressed-basis Krylov)')
    ap.add_argument('--reps', type=int, default=5,
                    help='timed repetitions of the K steps (value = median)')
    ap.add_argument('--calib-copy', type=int, default=0, metavar='MIB',
                    help='first run a plain device copy of this many MiB (counter calibration)')
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) != 1:
        print('bench.py measures one GPU: the library has no multi-GPU path (each problem runs on '
              'one device; sharding is a design note only). Run with --gpus 1.', file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2412_16638_amd as M
    from paper_2412_16638_amd import _abi as AB

    assert torch.cuda.is_available(), 'bench.py needs a GPU'
    if args.mode == 'batch':
        return bench_batch(args)
    if args.mode == 'serve':
        return bench_serve(args)
    if args.mode == 'sweep':
        return bench_sweep(args)
    fmt = AB.FMT_STENCIL if args.fmt == 'stencil' else AB.FMT_CSR
    bjs = 1 if args.bj == 'shared' else 0
    if args.calib_copy:
        n = args.calib_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device='cuda')
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f'calibration copy: {args.calib_copy} MiB read + {args.calib_copy} MiB written')
        del src, dst
    p = make_problem(args.workload, args.precond)
    mixed_over = dict(MIXED_TOL[args.workload])
    if args.compute == 'fp64':
        mixed_over['compute'] = AB.FP64
    gmf = {'auto': AB.GMFORM_AUTO, 'gather': AB.GMFORM_GATHER, 'zsplit': AB.GMFORM_ZSPLIT,
           'folded': AB.GMFORM_FOLDED}[args.gm_form]
    if gmf != AB.GMFORM_AUTO:
        mixed_over['gm_form'] = gmf
    if args.bj_adapt > 0:
        mixed_over['bj_adapt_tol'] = args.bj_adapt
    if args.stage_start != 'auto':
        mixed_over['stage_start'] = {'rhs': AB.START_RHS, 'slope': AB.START_SLOPE,
                                     'eval': AB.START_SLOPE_EVAL,
                                     'extrap': AB.START_EXTRAP}[args.stage_start]
    N = p.N
    K, Wm = args.steps, args.warmup
    log(f'workload {args.workload}: N={N} ({p.n}^3), {p.tableau}, dt={p.dt}, {p.krylov}, '
        f'{p.precision} storage, fmt={args.fmt}')

    # ---- reference of the full integration: the all-FP64 GPU path solved to REF_TOL ----
    ref = None
    err_mixed = None
    if not args.quick:
        log(f'reference: all-FP64 full integration, rtol = outer_tol = {REF_TOL:.0e} ...')
        q = make_problem(args.workload, args.precond)
        q.precision = 'fp64'
        ref, st_ref = run_integration(M, q, fmt, rtol=REF_TOL, outer_tol=REF_TOL, bj_shared=bjs)
        log(f'reference iters/stage={st_ref["iters"]} passes/stage={st_ref["passes"]}')

        # ---- mixed path: the same full integration, compared with the reference ----
        log('mixed path: full integration for the error check ...')
        u_mixed, st_mixed = run_integration(M, p, fmt, bj_shared=bjs, **mixed_over)
        err_mixed = float(np.linalg.norm(u_mixed - ref) / np.linalg.norm(ref))
        log(f'mixed rel-L2 vs FP64 reference = {err_mixed:.3e}  iters/stage={st_mixed["iters"]} '
            f'passes/stage={st_mixed["passes"]}')

    # ---- timed mixed run ----
    st = M.from_problem(p, fmt=fmt, bj_shared=bjs, **mixed_over)
    tuned = st.autotune()
    launch = st.launch_info()
    log(f'autotuned groups per thread (vector, row) = {tuned}; launch shapes {launch}')
    reps = []
    for _ in range(max(1, args.reps)):
        t_rep, stats, _ = time_steps(st, p.u0, K, Wm)
        reps.append(t_rep)
    t_mixed = float(np.median(reps))
    value = N * K / t_mixed
    log(f'mixed: {K} steps in {t_mixed * 1e3:.2f} ms (median of {len(reps)}; '
        f'{min(reps) * 1e3:.2f}..{max(reps) * 1e3:.2f}) -> {value:.4e} DOF-steps/s')

    # ---- roofline pass (per-kernel HIP events on the library stream) ----
    t_prof, _, prof = time_steps(st, p.u0, K, 1, profile=True)
    s_bytes = {'fp64': 8, 'fp32': 4, 'fp16': 2}[p.precision]
    bs = st.prec.block if st.prec.precond == AB.PRECOND_BJ else 0
    nv = {'stage_rhs': 3, 'combine': 3}  # SDIRK3: sum over stages of rhs terms; b has 3 terms
    # start values: k_{i-1} and k_{i-2} are already terms of rhs_i (SDIRK3's A is full below
    # the diagonal), so only f(u) is a new read (first stage, or second under EXTRAP)
    slope_starts = 1 if launch['stage_start'] in (AB.START_SLOPE_EVAL, AB.START_EXTRAP) else 0
    rows = []
    nnz_row = 0.0
    if args.fmt == 'csr':  # 7-point rows; a zero-Dirichlet face row has one neighbour fewer
        n3 = (p.n, p.n, p.n)
        faces = 0 if p.bc == 1 else 2 * (n3[0] * n3[1] + n3[1] * n3[2] + n3[0] * n3[2])
        nnz_row = (7.0 * N - faces) / N
    # adaptive-precision inverses: chunks of FP8, FP16, FP32, FP64 entries (1, 2, 4, 8 bytes)
    chunks = launch.get('bj_chunks') or [0, 0, 0, 0]
    inv_entry = (sum(c << t for t, c in enumerate(chunks)) / sum(chunks)) if sum(chunks) else 0.0
    for kc, r in prof.items():
        if r['launches'] == 0:
            continue
        nv_total = 0
        if kc == 'stage_rhs':
            nv_total = r['worked'] // p_stages(p) * (nv['stage_rhs'] + slope_starts)
        if kc == 'combine':
            nv_total = r['worked'] * nv['combine']
        sv = s_bytes
        cbytes = 8 if args.compute == 'fp64' or p.precision == 'fp64' else 4
        if kc == 'promote' and args.precond == 'fdm' and p.krylov == 'gmres':
            sv = cbytes  # the GMRES correction P^-1 (V y) is formed in the arithmetic type
        # GMRES with block-Jacobi in the gather form stores each direction BJ(v_j)
        zst = (p.krylov == 'gmres' and bs > 0 and args.precond == 'bj' and launch.get('gm_form') == 1)
        b = algorithmic_bytes(kc, N, sv, s_bytes, bs, r['worked'], r['units'], nv_total,
                              fdm=args.precond == 'fdm', cb=cbytes, csr_nnz_row=nnz_row,
                              zstored=zst, inv_entry=inv_entry)
        rows.append((kc, r, b))
    total_ms = sum(r['ms'] for _, r, _ in rows)
    dom = max(rows, key=lambda x: x[1]['ms'])
    kc, r, b = dom
    # every launch counts (a launch whose phase had finished moves ~0 bytes in ~3 us), so the
    # average duration matches rocprofv3's per-kernel average
    avg_ms = r['ms'] / r['launches']
    bytes_per_launch = b / r['launches']
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    if 'fdm' in prof and prof['fdm']['launches']:
        fr = prof['fdm']
        fdm_tflops = fr['worked'] / 6.0 * N * fdm_apply_flops(p) / (fr['ms'] * 1e-3) / 1e12
        log(f'fdm contractions: {fdm_tflops:.2f} TFLOP/s over {fr["launches"]} launches')
    kernel_table = {k: {'launches': rr['launches'], 'worked': rr['worked'],
                        'ms': round(rr['ms'], 3),
                        'share': round(rr['ms'] / total_ms, 4) if total_ms else None,
                        'GBps': round(bb / (rr['ms'] * 1e-3) / 1e9, 1) if rr['ms'] else None}
                    for k, rr, bb in rows}
    log('per-kernel: ' + json.dumps(kernel_table))
    traffic = None
    tpath = os.path.join(ROOT, 'profiles', f'traffic_{kc}_{args.workload}.json')
    if os.path.exists(tpath):
        with open(tpath) as fh:
            tr = json.load(fh)
        from rocprof_summary import kernel_source_hash
        if tr.get("kernel_hash") == kernel_source_hash():
            # counters give bytes per working dispatch; spread over all launches like `achieved`
            traffic = tr['bytes_per_worked_launch'] * r['worked'] / r['launches']
    if kc == 'fdm':
        flops_per_launch = r['worked'] / 6.0 * N * fdm_apply_flops(p) / r['launches']
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        peak = MFMA_PEAK['fp64' if args.compute == 'fp64' else p.precision]
        roofline = {'bound': 'mfma', 'kernel': kc, 'achieved': round(achieved, 2), 'peak': peak,
                    'unit': 'TFLOP/s', 'frac': round(achieved / peak, 4), 'traffic': None,
                    'flops_per_launch': flops_per_launch, 'avg_launch_us': round(avg_ms * 1e3, 2),
                    'launches': r['launches'], 'worked': r['worked']}
    else:
        roofline = {'bound': 'hbm', 'kernel': kc, 'achieved': round(achieved, 1),
                    'peak': HBM_PEAK_GBS, 'unit': 'GB/s', 'frac': round(achieved / HBM_PEAK_GBS, 4),
                    'traffic': traffic, 'bytes_per_launch': bytes_per_launch,
                    'avg_launch_us': round(avg_ms * 1e3, 2), 'launches': r['launches'],
                    'worked': r['worked'],
                    'all_kernels_GBps': round(sum(bb for _, _, bb in rows) / (total_ms * 1e-3) / 1e9, 1)}
    st.close()

    # ---- FP64 path at matched error ----
    fp64 = None
    fp64_tight = None
    fp64_same = None
    sweep = {}
    if not args.no_fp64 and ref is not None:
        for tol in (1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8, 1e-8, 1e-9, 1e-10,
                    3e-11, 1e-11):
            over = dict(rtol=tol, outer_tol=tol, bj_shared=bjs, **FP64_CMP)
            q = make_problem(args.workload, args.precond)
            q.precision = 'fp64'
            u64, s64 = run_integration(M, q, fmt, **over)
            e64 = float(np.linalg.norm(u64 - ref) / np.linalg.norm(ref))
            log(f'fp64 rtol={tol:.0e}: rel-L2 {e64:.3e} iters/stage={s64["iters"]}')
            sweep[tol] = e64
            if e64 <= err_mixed:
                st64 = M.from_problem(q, fmt=fmt, **over)
                st64.autotune()
                t64, _, _ = time_steps(st64, q.u0, K, Wm)
                st64.close()
                v64 = N * K / t64
                fp64 = {'value': v64, 'rtol': tol, 'err_vs_fp64_reference': e64,
                        'ms_per_step': t64 * 1e3 / K}
                log(f'fp64 matched: {v64:.4e} DOF-steps/s; mixed speedup {value / v64:.2f}x')
                break
        # the FP64 path at the mixed path's own (inner, outer) tolerance pair: the other family
        # a matched-error comparison could use; it is the match when it is faster and as accurate
        pm = M.precisions(p.precision, p.krylov, **MIXED_TOL[args.workload])
        q = make_problem(args.workload, args.precond)
        q.precision = 'fp64'
        over = dict(rtol=pm.rtol, outer_tol=pm.outer_tol, bj_shared=bjs, **FP64_CMP)
        u64, s64 = run_integration(M, q, fmt, **over)
        e64 = float(np.linalg.norm(u64 - ref) / np.linalg.norm(ref))
        st64 = M.from_problem(q, fmt=fmt, **over)
        st64.autotune()
        t64, _, _ = time_steps(st64, q.u0, K, Wm)
        st64.close()
        fp64_same = {'value': N * K / t64, 'rtol': pm.rtol, 'outer_tol': pm.outer_tol,
                     'err_vs_fp64_reference': e64, 'ms_per_step': t64 * 1e3 / K,
                     'iters_per_stage': s64['iters']}
        log(f'fp64 at the mixed tolerances (inner {pm.rtol:.0e}, outer {pm.outer_tol:.0e}): '
            f'{fp64_same["value"]:.4e} DOF-steps/s, rel-L2 {e64:.3e}')
        if e64 <= err_mixed and (fp64 is None or fp64_same['value'] > fp64['value']):
            fp64 = dict(fp64_same, family='mixed tolerance pair')
        elif fp64 is not None:
            fp64['family'] = 'rtol = outer_tol sweep'
        # the FP64 path at a tight tolerance, for reference
        tight = 1e-10
        q = make_problem(args.workload, args.precond)
        q.precision = 'fp64'
        over = dict(rtol=tight, outer_tol=tight, bj_shared=bjs)
        if tight not in sweep:
            u64, _ = run_integration(M, q, fmt, **over)
            sweep[tight] = float(np.linalg.norm(u64 - ref) / np.linalg.norm(ref))
        st64 = M.from_problem(q, fmt=fmt, **over)
        st64.autotune()
        t64, _, _ = time_steps(st64, q.u0, K, Wm)
        st64.close()
        fp64_tight = {'value': N * K / t64, 'rtol': tight, 'err_vs_fp64_reference': sweep[tight],
                      'ms_per_step': t64 * 1e3 / K}
        log(f'fp64 at rtol {tight:.0e}: {fp64_tight["value"]:.4e} DOF-steps/s, '
            f'rel-L2 {sweep[tight]:.3e}')

    # ---- the other block-Jacobi storage (same values; per-block inverse stream or not) ----
    other = None
    if not args.no_fp64 and not args.quick and args.precond == 'bj' and args.bj_adapt == 0:
        st2 = M.from_problem(p, fmt=fmt, bj_shared=1 - bjs, **mixed_over)
        st2.autotune()
        t2, _, _ = time_steps(st2, p.u0, K, Wm)
        st2.close()
        other = {'bj': 'per-block' if bjs else 'shared', 'value': N * K / t2,
                 'ms_per_step': t2 * 1e3 / K}
        log(f'other block-Jacobi storage ({other["bj"]}): {other["value"]:.4e} DOF-steps/s')

    # ---- adaptive-precision block-Jacobi beside the headline storage ----
    adaptive = None
    if not args.no_fp64 and not args.quick and args.precond == 'bj' and args.bj_adapt == 0:
        tol_a = 0.25
        sta = M.from_problem(p, fmt=fmt, bj_shared=0, bj_adapt_tol=tol_a,
                             **{k: v for k, v in mixed_over.items() if k != 'bj_adapt_tol'})
        sta.autotune()
        ta, st_a, _ = time_steps(sta, p.u0, K, Wm)
        chunks = sta.launch_info()['bj_chunks']
        sta.close()
        ua, _ = run_integration(M, p, fmt, bj_shared=0, bj_adapt_tol=tol_a, **mixed_over) \
            if ref is not None else (None, None)
        ea = float(np.linalg.norm(ua - ref) / np.linalg.norm(ref)) if ua is not None else None
        adaptive = {'bj_adapt_tol': tol_a, 'value': N * K / ta, 'ms_per_step': ta * 1e3 / K,
                    'chunks_fp8_fp16_fp32_fp64': chunks, 'err_vs_fp64_reference': ea,
                    'iters_per_stage': st_a['iters']}
        log(f'adaptive block-Jacobi (tol {tol_a}): {adaptive["value"]:.4e} DOF-steps/s, '
            f'chunks {chunks}, rel-L2 {ea}')

    # ---- the semi-linear variant (pointwise reaction) of the same workload ----
    nonlin = None
    if not args.no_fp64 and not args.quick and args.fmt == 'stencil':
        nonlin = nonlinear_leg(M, args, fmt, bjs, mixed_over, K, Wm)

    # ---- the fast-diagonalisation preconditioner on both workloads ----
    fdm_side = None
    if not args.no_fp64 and not args.quick and args.precond == 'bj' and args.fmt == 'stencil':
        fdm_side = fdm_leg(M, K, Wm)

    # ---- side legs of the metric: batched problems and serving latency ----
    batch = None
    if not args.no_batch and not args.quick:
        batch = batch_leg(K, Wm, quick=True)
    serving = None
    if args.serve_requests > 0 and not args.quick:
        serving = serve_leg(args.serve_requests, args.slots)

    cpu = None
    if not args.no_cpu:
        log('cpu baseline: the oracle stepping the method on the host ...')
        v_cpu, sample, t_cpu = cpu_oracle_rate(args.workload, args.precond)
        log(f'cpu baseline: {v_cpu:.4e} DOF-steps/s ({t_cpu:.1f} s)')
        cpu = {'value': v_cpu, 'unit': 'DOF-steps/s', 'cores': 1, 'kind': 'oracle',
               'host': host_info(), 'sample': sample}

    out = {
        'metric': METRIC, 'value': value, 'unit': 'DOF-steps/s', 'n_gpus': 1, 'steps': K,
        'warmup': Wm, 'ms_per_step': t_mixed * 1e3 / K, 'higher_is_better': True,
        'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64' if args.compute == 'fp64' else 'f32',
        'data': 'synthetic',
        'config': {'workload': workload_name(args),
                   'N': N, 'format': args.fmt, 'lp_storage': p.precision,
                   'lp_compute': 'f64' if args.compute == 'fp64' else 'f32',
                   'explicit_parts': 'f64', 'krylov': p.krylov},
        'err_vs_fp64_reference': err_mixed,
        'reference': (f'all-FP64 GPU path, same problem and preconditioner, rtol = outer_tol = '
                      f'{REF_TOL:.0e}') if ref is not None else None,
        'iters_per_stage': stats['iters'], 'passes_per_stage': stats['passes'],
        'timed_reps_ms_per_step': [round(t * 1e3 / K, 4) for t in reps],
        'fp64_matched': fp64,
        'fp64_at_mixed_tolerances': fp64_same,
        'fp64_tight': fp64_tight,
        'bj_storage': args.bj if args.precond == 'bj' else None,
        'autotuned_groups_per_thread': list(tuned),
        'launch_shapes': launch,
        'other_bj_storage': other,
        'adaptive_bj': adaptive,
        'nonlinear': nonlin,
        'fdm': fdm_side,
        'speedup_vs_fp64_matched': (value / fp64['value']) if fp64 else None,
        'roofline': roofline,
        'cpu_baseline': cpu,
        'kernels': kernel_table,
        'p50_latency_s': serving['p50_latency_s'] if serving else None,
        'p99_latency_s': serving['p99_latency_s'] if serving else None,
        'serve': serving,
        'batch': batch,
    }
    prec = M.precisions(p.precision, p.krylov, **MIXED_TOL[args.workload])
    out['config']['outer_tol'] = prec.outer_tol
    out['config']['inner_rtol'] = prec.rtol
    out['config']['stage_start'] = {AB.START_RHS: 'rhs', AB.START_SLOPE: 'slope',
                                    AB.START_SLOPE_EVAL: 'slope_eval',
                                    AB.START_EXTRAP: 'extrap'}.get(launch['stage_start'])
    print(json.dumps(out), flush=True)


SWEEP_TAUS = (1 / 10, 1 / 20, 1 / 40, 1 / 80, 1 / 160, 1 / 320, 1 / 640, 1 / 1280)
SWEEP_METHODS = {'heat': ('MID1', '4S3PB', '4S3PC'),            # 4s3pA excluded for heat
                 'advection': ('MID1', '4S3PA', '4S3PB', '4S3PC')}


def bench_sweep(args):
    """The paper's experiments (Section "Linear solvers and setup of the numerical experiments",
    Figure CombinedErrors, Table iterations) on its two test problems: final-time error and
    wall time against tau in {1/10 .. 1/1280} to T = 1/10 for the methods M (implicit midpoint
    with one corrector), A, B, C, with FP32 and FP64 implicit solves in the paper's setting
    (one solve per stage to an absolute-or-relative residual tol = 1e-3, at most 40 Krylov
    iterations (GMRES: one cycle of at most 32, the longest built), the tableau's FP64
    corrector stages, no outer refinement); then the Krylov
    iterations per solve of method C against tol.  Both problems use the paper's fast-
    diagonalisation preconditioner: heat with CG (real sine basis), advection with GMRES (complex
    DFT basis); the iteration table also gives advection with block-Jacobi(8).
    Errors: relative L2 against the continuum solution (the paper's measure: spatial error
    included) and against the same DIRK with tight stage solves (the solver's own error): the
    all-FP64 path with the fast-diagonalisation preconditioner and the FP64 residual loop to
    1e-12, which the GPU tests pin to the oracle's exact-solve closed forms."""
    import torch
    import paper_2412_16638_amd as M
    from paper_2412_16638_amd import _abi as AB
    import workloads as W

    n, T = args.n, 0.1

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def make(prob, tab, tau, prec):
        if prob == 'heat':
            return W.paper_heat(n, tab, tau, T, prec)
        return W.paper_advection(n, tab, tau, T, prec)

    def run(p, tol, maxit=40, precond=None, **extra):
        p.precond = precond or 'fdm'
        over = {} if p.kind == W.HEAT else {'restart': 32}  # the longest GMRES cycle built
        st = M.from_problem(p, rtol=tol, atol=tol, maxit=maxit, refine_max=0, **over, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, stats = st.step(p.nsteps, check=False)  # a non-finite step is a result here
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        u = st.get_u()
        st.close()
        stats['rc'] = rc
        return u, stats, t

    def tight(prob, tab, tau):
        p = make(prob, tab, tau, 'fp64')
        p.precond = 'fdm'
        st = M.from_problem(p, rtol=REF_TOL, outer_tol=REF_TOL)
        st.step(p.nsteps)
        u = st.get_u()
        st.close()
        return u

    # warm-up (first launches, library initialisation)
    for prob in ('heat', 'advection'):
        for prec in ('fp32', 'fp64'):
            run(make(prob, '4S3PC', 1 / 10, prec), 1e-3)

    rows = []
    for prob, methods in SWEEP_METHODS.items():
        cont = W.paper_heat_exact(n, T) if prob == 'heat' else W.translated_gaussian(n, (T, T, T))
        for tab in methods:
            for tau in SWEEP_TAUS:
                p = make(prob, tab, tau, 'fp64')
                ref = tight(prob, tab, tau)
                row = {'problem': prob, 'method': tab, 'tau': tau, 'steps': p.nsteps}
                for prec in ('fp32', 'fp64'):
                    u, stats, t = run(make(prob, tab, tau, prec), 1e-3)
                    row[prec] = {'ms': round(t * 1e3, 3),
                                 'err_vs_continuum': rel(u, cont),
                                 'err_vs_tight_dirk': rel(u, ref),
                                 'iters_per_solve': round(stats['total_iters'] / max(1, stats['total_passes']), 2),
                                 'rc': stats['rc'], 'nonfinite': stats['nonfinite']}
                row['speedup'] = row['fp64']['ms'] / row['fp32']['ms']
                rows.append(row)
                log(f"sweep {prob:9s} {tab:5s} tau=1/{round(1 / tau):4d}: "
                    f"err fp32 {row['fp32']['err_vs_continuum']:.3e} fp64 {row['fp64']['err_vs_continuum']:.3e} "
                    f"(vs tight DIRK {row['fp32']['err_vs_tight_dirk']:.1e} / {row['fp64']['err_vs_tight_dirk']:.1e}); "
                    f"iters {row['fp32']['iters_per_solve']} / {row['fp64']['iters_per_solve']}; "
                    f"{row['fp32']['ms']:.1f} / {row['fp64']['ms']:.1f} ms -> {row['speedup']:.2f}x")
    # Krylov iterations per solve against the tolerance (method C, tau = 1/80)
    iters = []
    for prob in SWEEP_METHODS:
        for tol in (1e-3, 1e-4, 1e-5, 1e-6, 1e-8):
            rec = {'problem': prob, 'precond': 'fdm', 'tol': tol}
            for prec in ('fp32', 'fp64'):
                _, stats, t = run(make(prob, '4S3PC', 1 / 80, prec), tol)
                rec[prec] = round(stats['total_iters'] / max(1, stats['total_passes']), 2)
                rec[prec + '_ms'] = round(t * 1e3, 3)
            iters.append(rec)
            log(f"iterations {prob:9s} tol={tol:.0e}: fp32 {rec['fp32']} fp64 {rec['fp64']} per solve")
    # the advection problem with block-Jacobi(8) instead of the paper's preconditioner
    for tol in (1e-3, 1e-4, 1e-5, 1e-6, 1e-8):
        rec = {'problem': 'advection', 'precond': 'bj', 'tol': tol}
        for prec in ('fp32', 'fp64'):
            _, stats, t = run(make('advection', '4S3PC', 1 / 80, prec), tol, precond='bj')
            rec[prec] = round(stats['total_iters'] / max(1, stats['total_passes']), 2)
            rec[prec + '_ms'] = round(t * 1e3, 3)
        iters.append(rec)
        log(f"iterations advection+BJ tol={tol:.0e}: fp32 {rec['fp32']} fp64 {rec['fp64']} per solve")
    # FP16 storage with FP32 against FP64 arithmetic (compressed basis), same setting, method C,
    # tau = 1/80: the error of the one-solve-per-stage integration against the tight-solve DIRK
    cbrows = []
    for prob in SWEEP_METHODS:
        ref = tight(prob, '4S3PC', 1 / 80)
        for tol in (1e-3, 1e-5, 1e-8):
            rec = {'problem': prob, 'tol': tol}
            for lab, extra in (('fp16_fp32arith', {}), ('fp16_fp64arith', {'compute': AB.FP64})):
                u, stats, t = run(make(prob, '4S3PC', 1 / 80, 'fp16'), tol, **extra)
                rec[lab] = {'err_vs_tight_dirk': rel(u, ref), 'ms': round(t * 1e3, 3),
                            'iters_per_solve': round(stats['total_iters'] / max(1, stats['total_passes']), 2)}
            cbrows.append(rec)
            log(f"fp16 storage {prob:9s} tol={tol:.0e}: err vs tight DIRK fp32-arith "
                f"{rec['fp16_fp32arith']['err_vs_tight_dirk']:.2e} ({rec['fp16_fp32arith']['iters_per_solve']} it) "
                f"fp64-arith {rec['fp16_fp64arith']['err_vs_tight_dirk']:.2e} ({rec['fp16_fp64arith']['iters_per_solve']} it)")
    sp = np.array([r['speedup'] for r in rows])
    total_dof_steps = sum(n ** 3 * r['steps'] for r in rows)
    total_s = sum(r['fp32']['ms'] for r in rows) * 1e-3
    out = {'metric': 'paper experiments: final-time error and wall time vs tau, FP32 vs FP64 '
                     'implicit solves', 'mode': 'sweep',
           'value': total_dof_steps / total_s, 'unit': 'DOF-steps/s (all FP32 sweep runs)',
           'n_gpus': 1, 'higher_is_better': True, 'dtype': 'f32', 'data': 'synthetic',
           'vs_baseline': None,
           'config': {'workload': f'paper forced heat and central advection, {n}^3, T = 0.1, FDM, '
                                  f'tol 1e-3, maxit 40, one solve per stage',
                      'n': n, 'taus': list(SWEEP_TAUS)},
           'speedup_geomean': float(np.exp(np.mean(np.log(sp)))),
           'rows': rows, 'iterations_vs_tol': iters, 'fp16_storage_arithmetic': cbrows}
    print(json.dumps(out), flush=True)


def batch_leg(K: int, Wm: int, quick: bool) -> dict:
    """64 heat problems (n in [16, 96], kappa log-uniform in [0.1, 10]), SDIRK3, FP32 CG + BJ(8),
    one persistent launch per stage replayed as a hipGraph; DOF-steps/s over all problems."""
    import torch
    import paper_2412_16638_amd as M
    import workloads as W
    probs = W.heat_batch()
    b = M.Batch([{'shape': p.n, 'diff': p.diff, 'dt': p.dt} for p in probs], 'SDIRK3',
                M.precisions('fp32', 'cg'))
    dof = sum(p.N for p in probs)
    log(f'batch: {len(probs)} problems, {dof} unknowns, {sum(b.schedule)} workgroups')
    for i, p in enumerate(probs):
        b.set_u(i, p.u0)
    t0 = time.perf_counter()
    b.step(probs[0].nsteps)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    # each problem against the single-problem all-FP64 path solved to REF_TOL (pinned to the
    # oracle's closed forms by the GPU tests)
    worst = None
    if not quick:
        worst = 0.0
        for i, p in enumerate(probs):
            sref = M.from_problem(dataclasses.replace(p, precision='fp64'), rtol=REF_TOL,
                                  outer_tol=REF_TOL)
            sref.step(p.nsteps)
            ref = sref.get_u()
            sref.close()
            u = b.get_u(i)
            d = np.linalg.norm(u - ref) / max(np.linalg.norm(ref), 1e-6 * np.linalg.norm(p.u0))
            worst = max(worst, float(d))
        log(f'worst floored rel-L2 vs the FP64 reference over the batch: {worst:.3e}')

    def timed():
        for i, p in enumerate(probs):
            b.set_u(i, p.u0)
        b.step(Wm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(K)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    t_plan = timed()
    log(f'planned schedule (2 rows per thread, work model e = 0.5): {dof * K / t_plan:.4e} DOF-steps/s')
    for i, p in enumerate(probs):
        b.set_u(i, p.u0)
    expo, ru = b.autotune()
    model = 'measured work of the last step' if expo < 0 else f'work-model exponent {expo}'
    log(f'autotuned: {ru} rows per thread per CG sweep, {model}; workgroups '
        f'per problem {min(b.schedule)}..{max(b.schedule)}, total {sum(b.schedule)}')
    t = timed()
    st = [b.stats(i) for i in range(len(probs))]
    sched = list(b.schedule)
    wg = sum(sched)
    b.close()
    log(f'batch: {dof * K / t:.4e} DOF-steps/s')
    # where the time goes: the step's CG work (iterations x unknowns, from each problem's last
    # step) at the FP32 per-block BJ(8) bytes of one iteration (11 s + 8 m = 76 B), the FP64
    # outer passes (about 120 B per unknown each), stage right-hand sides and the combination
    # (about 136 B): an effective bandwidth; and the share of workgroup time that does work when
    # each problem's workgroups take N x iterations / workgroups and the stage ends with the
    # slowest (1 = every group finishes together)
    it_dofs = sum(p.N * sum(x['iters']) for p, x in zip(probs, st))
    pass_dofs = sum(p.N * sum(x['passes']) for p, x in zip(probs, st))
    bytes_step = 76.0 * it_dofs + 120.0 * pass_dofs + 136.0 * dof
    span = max(p.N * sum(x['iters']) / g for p, x, g in zip(probs, st, sched))
    balance = it_dofs / (wg * span) if span > 0 else None
    log(f'batch: {it_dofs / dof:.1f} CG iterations per unknown per step, effective '
        f'{bytes_step * K / t / 1e9:.0f} GB/s (byte model), workgroup balance {balance:.2f}')
    return {'value': dof * K / t, 'unit': 'DOF-steps/s', 'steps': K, 'warmup': Wm,
            'ms_per_step': t * 1e3 / K,
            'config': {'workload': 'batch_64_heat_n16-96_kappa0.1-10_sdirk3_dt5e-4_cg_bj8_fp32',
                       'problems': len(probs), 'N_total': dof,
                       'launch': 'one persistent kernel per stage, hipGraph per step'},
            'first_integration_s': t_full,
            'planned_schedule_value': dof * K / t_plan,
            'autotuned_work_exponent': expo,
            'autotuned_rows_per_thread': ru,
            'workgroups': wg,
            'worst_err_vs_fp64_reference': worst,
            'iters_per_stage_max': max(max(x['iters']) for x in st),
            'cg_iterations_per_unknown_per_step': it_dofs / dof,
            'effective_GBps_byte_model': bytes_step * K / t / 1e9,
            'workgroup_balance': balance}


def bench_batch(args):
    r = batch_leg(args.steps, args.warmup, args.quick)
    out = {'metric': METRIC, 'value': r['value'], 'unit': 'DOF-steps/s', 'n_gpus': 1,
           'steps': r['steps'], 'warmup': r['warmup'], 'ms_per_step': r['ms_per_step'],
           'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f32',
           'data': 'synthetic', 'config': r['config']}
    out.update({k: v for k, v in r.items() if k not in out})
    print(json.dumps(out), flush=True)


def serve_leg(count: int, slots: int, pool: bool = True) -> dict:
    """The first `count` requests of the seeded 512-request Poisson stream (50/s) replayed
    open-loop on the wall clock; p50/p99 latency (completion - arrival) and DOF-steps/s."""
    from paper_2412_16638_amd import serve
    import workloads as W
    reqs = W.request_stream(materialize_u0=False)[:count]
    be = serve.GpuBackend(u0_fn=W.initial_field, pool=pool)
    srv = serve.Server(be, max_active=slots)
    log(f'serve: {len(reqs)} requests over {reqs[-1].arrival:.1f} s, {slots} slots, '
        f'handle pool {"on" if pool else "off"}, budget {srv.budget / 2**30:.1f} GiB')
    seen = [0]

    def progress(msg):  # one line per 64 admissions
        seen[0] += 1
        if seen[0] % 64 == 0:
            log(f'serve progress: {seen[0]} admitted; {msg}')

    out = srv.run(reqs, log=progress)
    be.close()
    offered = sum(r.problem.N * r.problem.nsteps for r in reqs) / reqs[-1].arrival
    log(f'serve: p50 {out["p50_s"]:.3f} s, p99 {out["p99_s"]:.3f} s, served '
        f'{out["dof_steps_per_s"]:.3e} DOF-steps/s of {offered:.3e} offered, '
        f'{be.created} handles made for {len(reqs)} jobs')
    return {'requests': len(reqs), 'max_active': slots, 'handle_pool': pool,
            'handles_created': be.created,
            'p50_latency_s': out['p50_s'], 'p99_latency_s': out['p99_s'],
            'mean_latency_s': out['mean_s'], 'makespan_s': out['makespan_s'],
            'served_dof_steps_per_s': out['dof_steps_per_s'], 'offered_dof_steps_per_s': offered,
            'dof_steps': out['dof_steps'], 'failed': out['failed'],
            'peak_active': out['peak_active'], 'peak_resident_bytes': out['peak_resident_bytes'],
            'budget_bytes': srv.budget}


def bench_serve(args):
    """512 Poisson requests (50/s) replayed open-loop; p50/p99 latency and DOF-steps/s."""
    import paper_2412_16638_amd as M  # noqa: F401
    r = serve_leg(args.requests, args.slots, pool=not args.no_pool)
    res = {'metric': METRIC, 'value': r['served_dof_steps_per_s'], 'unit': 'DOF-steps/s',
           'n_gpus': 1, 'steps': None, 'warmup': 0, 'ms_per_step': None, 'higher_is_better': True,
           'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f32/f64 mix', 'data': 'synthetic',
           'config': {'workload': f'serve_{r["requests"]}_poisson50_heat-or-advdiff_n32-192_'
                                  f'steps10-100_fp64|fp32|fp16',
                      'max_active': r['max_active'], 'budget_bytes': r['budget_bytes'],
                      'handle_pool': r['handle_pool']},
           'p50_latency_s': r['p50_latency_s'], 'p99_latency_s': r['p99_latency_s']}
    res.update({k: v for k, v in r.items() if k not in res and k not in ('budget_bytes',)})
    print(json.dumps(res), flush=True)


def p_stages(p) -> int:
    return {'SDIRK2': 2, 'SDIRK3': 3}.get(p.tableau.upper(), 4)


if __name__ == '__main__':
    main()
