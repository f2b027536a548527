"""Helpers shared by the GPU tests (input preparation and oracle evaluation only)."""
import numpy as np

import workloads as W
from oracle import closed_form, dirk, nonlinear, operators, tableaus


def oracle_K(shape, bc, kind, diff, b):
    return operators.operator(shape, bc, kind, diff, b)


def oracle_tableau(name):
    return tableaus.by_name(name)


def reference_solution(p, method='closed'):
    """FP64 oracle u_N for a workloads.Problem (closed form where one exists)."""
    tab = tableaus.by_name(p.tableau)
    if method == 'closed':
        return closed_form.evolve(p.u0, p.kind, p.bc, p.diff, p.b, p.dt, p.nsteps, tab)
    K = oracle_K((p.n,) * 3, p.bc, p.kind, p.diff, p.b)
    return dirk.integrate(K, p.u0, p.dt, p.nsteps, tab, method).reshape(p.u0.shape)


def reference_nonlinear(p, shape=None):
    """FP64 oracle u_N (Newton stage solves) of a workloads.Problem with a reaction; the Newton
    systems go to the oracle's GMRES above 4096 unknowns (sparse LU fill grows too fast)."""
    shape = shape or (p.n,) * 3
    K = oracle_K(shape, p.bc, p.kind, p.diff, p.b)
    g = None if p.forcing is None else np.ravel(p.forcing)
    method = 'splu' if np.prod(shape) <= 4096 else 'gmres'
    return nonlinear.integrate(K, p.u0, p.dt, p.nsteps, tableaus.by_name(p.tableau), p.reaction,
                               g=g, method=method).reshape(np.shape(p.u0))


def reference_scalar(p, y0):
    """The oracle's scalar form y' = R(y) (+ a constant forcing value) over the same steps."""
    return nonlinear.scalar_integrate(y0, p.dt, p.nsteps, tableaus.by_name(p.tableau), p.reaction)


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def rel_l2_floor(a, ref, u0, floor=1e-6):
    """||a - ref|| / max(||ref||, floor ||u0||): relative L2 error of a state that may have decayed
    far below its initial norm (below the floor, roundoff seeded into slowly decaying modes absent
    from the exact state dominates -- see tests/test_oracle_dirk.py)."""
    d = np.linalg.norm(np.ravel(a) - np.ravel(ref))
    return float(d / max(np.linalg.norm(np.ravel(ref)), floor * np.linalg.norm(np.ravel(u0))))


def log_case(case_name, **kw):
    print(f'[gpu-case] {case_name} ' + ' '.join(f'{k}={v}' for k, v in kw.items()), flush=True)
