"""ctypes binding of include/mprk.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  All computation happens in
libmprk.so's HIP kernels; this module only converts Python values to the C structs.  Importing
it without a built library raises ImportError -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libmprk.so')

MAX_STAGES = 8
MAX_RESTART = 32
STATIC_SCRATCH_BYTES = 64 << 20   # MPRK_STATIC_SCRATCH_BYTES

# status codes
OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ENOTCONV, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
BC_DIRICHLET0, BC_PERIODIC = 0, 1
OP_HEAT, OP_ADVDIFF, OP_CENTRAL = 0, 1, 2
FMT_STENCIL, FMT_CSR = 0, 1
FP64, FP32, FP16 = 0, 1, 2
CG, GMRES = 0, 1
PRECOND_NONE, PRECOND_BJ, PRECOND_FDM = 0, 1, 2
GMFORM_AUTO, GMFORM_GATHER, GMFORM_ZSPLIT, GMFORM_FOLDED = 0, 1, 2, 3
START_AUTO, START_RHS, START_SLOPE, START_SLOPE_EVAL, START_EXTRAP = 0, 1, 2, 3, 4
STOP_AUTO, STOP_OUTER, STOP_RTOL = 0, 1, 2
TAB_SDIRK2, TAB_SDIRK3, TAB_MID, TAB_4S3PA, TAB_4S3PB, TAB_4S3PC = range(6)
APPLY_K64, APPLY_M_LP, APPLY_BJ_LP, APPLY_M64, APPLY_FDM_LP = range(5)
KC_NAMES = ('stage_rhs', 'residual', 'cg_begin', 'cg_dir', 'cg_upd', 'promote', 'gm_begin',
            'gm_prec', 'gm_matvec', 'gm_orth', 'gm_finish', 'keps', 'combine', 'apply', 'cg_rz',
            'fdm', 'gm_reorth', 'gm_step', 'gm_close')
KC = {n: i for i, n in enumerate(KC_NAMES)}

STATUS_NAMES = {OK: 'MPRK_OK', EINVAL: 'MPRK_EINVAL', ENOMEM: 'MPRK_ENOMEM', EDEVICE: 'MPRK_EDEVICE',
                ENONFINITE: 'MPRK_ENONFINITE', ENOTCONV: 'MPRK_ENOTCONV',
                EUNSUPPORTED: 'MPRK_EUNSUPPORTED', ESTATE: 'MPRK_ESTATE'}


class mprk_grid(C.Structure):
    _fields_ = [('nx', C.c_int32), ('ny', C.c_int32), ('nz', C.c_int32), ('bc', C.c_int32)]


class mprk_operator(C.Structure):
    _fields_ = [('kind', C.c_int32), ('format', C.c_int32), ('diff', C.c_double),
                ('b', C.c_double * 3)]


class mprk_tableau(C.Structure):
    _fields_ = [('s', C.c_int32), ('a_hi', C.c_double * (MAX_STAGES * MAX_STAGES)),
                ('a_lo', C.c_double * (MAX_STAGES * MAX_STAGES)), ('b', C.c_double * MAX_STAGES)]


class mprk_precisions(C.Structure):
    _fields_ = [('storage', C.c_int32), ('compute', C.c_int32), ('krylov', C.c_int32),
                ('restart', C.c_int32), ('precond', C.c_int32), ('block', C.c_int32),
                ('rtol', C.c_double), ('atol', C.c_double), ('maxit', C.c_int32),
                ('refine_max', C.c_int32), ('outer_tol', C.c_double), ('strict', C.c_int32),
                ('reorth', C.c_int32), ('bj_shared', C.c_int32), ('gm_form', C.c_int32),
                ('bj_adapt_tol', C.c_double), ('stage_start', C.c_int32),
                ('inner_stop', C.c_int32)]


class mprk_stats(C.Structure):
    _fields_ = [('steps', C.c_int64), ('t', C.c_double), ('stages', C.c_int32),
                ('iters', C.c_int32 * MAX_STAGES), ('passes', C.c_int32 * MAX_STAGES),
                ('resid', C.c_double * MAX_STAGES), ('converged', C.c_int32 * MAX_STAGES),
                ('total_iters', C.c_int64), ('total_passes', C.c_int64), ('nonfinite', C.c_int32),
                ('missed', C.c_int32), ('graph_steps', C.c_int32)]

    def as_dict(self):
        s = self.stages
        return {'steps': self.steps, 't': self.t, 'stages': s,
                'iters': list(self.iters[:s]), 'passes': list(self.passes[:s]),
                'resid': list(self.resid[:s]), 'converged': list(self.converged[:s]),
                'total_iters': self.total_iters, 'total_passes': self.total_passes,
                'nonfinite': self.nonfinite, 'missed': self.missed,
                'graph_steps': self.graph_steps}


class mprk_solve_info(C.Structure):
    _fields_ = [('iters', C.c_int32), ('passes', C.c_int32), ('converged', C.c_int32),
                ('resid', C.c_double)]


class mprk_launch_info(C.Structure):
    _fields_ = [('nit_vec', C.c_int32), ('nit_row', C.c_int32), ('nit_vec_red', C.c_int32),
                ('nit_row_red', C.c_int32), ('nit_lp', C.c_int32), ('nit_lp_red', C.c_int32),
                ('residual_planes', C.c_int32), ('gm_form', C.c_int32), ('gm_planes', C.c_int32),
                ('bj_chunks', C.c_int64 * 4), ('stage_start', C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d['bj_chunks'] = list(self.bj_chunks)
        return d


class mprk_problem(C.Structure):
    _fields_ = [('grid', mprk_grid), ('op', mprk_operator), ('dt', C.c_double)]


# One HIP runtime per process: torch ships its own libamdhip64, and libmprk.so must bind to
# that same instance (same device memory, same streams).  Loading torch first makes the
# dynamic linker resolve libmprk.so's HIP dependency to torch's copy.
try:
    import torch  # noqa: F401
except ImportError:  # a C-only caller without torch uses the system ROCm runtime
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError(f'{LIB_PATH} is missing: build the HIP library first '
                      '(python -c "import __graft_entry__ as g; g.build()")')

lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
_sig = {
    'mprk_tableau_builtin': (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(mprk_tableau)]),
    'mprk_precisions_default': (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(mprk_precisions)]),
    'mprk_create': (C.c_int32, [C.POINTER(mprk_grid), C.POINTER(mprk_operator),
                                C.POINTER(mprk_tableau), C.POINTER(mprk_precisions), C.c_double,
                                _P, C.POINTER(_P)]),
    'mprk_workspace_bytes': (C.c_int64, [_P]),
    'mprk_bind': (C.c_int32, [_P, _P, _P, C.c_int64]),
    'mprk_bind_static': (C.c_int32, [_P, _P]),
    'mprk_step': (C.c_int32, [_P, C.c_int32, C.POINTER(mprk_stats)]),
    'mprk_solve': (C.c_int32, [_P, C.c_int32, _P, _P, C.POINTER(mprk_solve_info)]),
    'mprk_apply': (C.c_int32, [_P, C.c_int32, C.c_int32, _P, _P]),
    'mprk_set_forcing': (C.c_int32, [_P, _P]),
    'mprk_set_reaction': (C.c_int32, [_P, C.c_double, C.c_double, C.c_double]),
    'mprk_set_step_graph': (C.c_int32, [_P, C.c_int32]),
    'mprk_get_state': (C.c_int32, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    'mprk_set_state': (C.c_int32, [_P, C.c_double, C.c_int64]),
    'mprk_stats_sync': (C.c_int32, [_P, C.POINTER(mprk_stats)]),
    'mprk_autotune': (C.c_int32, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    'mprk_profile': (C.c_int32, [_P, C.c_int32]),
    'mprk_launch_info_get': (C.c_int32, [_P, C.POINTER(mprk_launch_info)]),
    'mprk_profile_read': (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    'mprk_last_error': (C.c_char_p, []),
    'mprk_destroy': (None, [_P]),
    'mprk_batch_create': (C.c_int32, [C.c_int32, C.POINTER(mprk_problem), C.POINTER(mprk_tableau),
                                      C.POINTER(mprk_precisions), _P, C.POINTER(_P)]),
    'mprk_batch_set_schedule': (C.c_int32, [_P, C.POINTER(C.c_int32)]),
    'mprk_batch_get_schedule': (C.c_int32, [_P, C.POINTER(C.c_int32)]),
    'mprk_batch_autotune': (C.c_int32, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    'mprk_batch_workspace_bytes': (C.c_int64, [_P]),
    'mprk_batch_bind': (C.c_int32, [_P, C.POINTER(_P), _P, C.c_int64]),
    'mprk_batch_step': (C.c_int32, [_P, C.c_int32]),
    'mprk_batch_stats_sync': (C.c_int32, [_P, C.c_int32, C.POINTER(mprk_stats)]),
    'mprk_batch_destroy': (None, [_P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class MprkError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib.mprk_last_error().decode(errors='replace')
        super().__init__(f'{where}: {STATUS_NAMES.get(code, code)}: {msg}')


def check(code: int, where: str) -> int:
    if code != OK:
        raise MprkError(code, where)
    return code


# ---- thin wrappers with the C names -------------------------------------------------------

def mprk_tableau_builtin(tab_id: int, param: int = 0) -> mprk_tableau:
    t = mprk_tableau()
    check(lib.mprk_tableau_builtin(tab_id, param, C.byref(t)), 'mprk_tableau_builtin')
    return t


def mprk_precisions_default(storage: int, krylov: int) -> mprk_precisions:
    p = mprk_precisions()
    check(lib.mprk_precisions_default(storage, krylov, C.byref(p)), 'mprk_precisions_default')
    return p


def mprk_create(grid: mprk_grid, op: mprk_operator, tab: mprk_tableau, prec: mprk_precisions,
                dt: float, stream: int = 0) -> int:
    h = _P()
    check(lib.mprk_create(C.byref(grid), C.byref(op), C.byref(tab), C.byref(prec), dt,
                          _P(stream), C.byref(h)), 'mprk_create')
    return h.value


def mprk_workspace_bytes(h: int) -> int:
    n = lib.mprk_workspace_bytes(_P(h))
    if n < 0:
        raise MprkError(int(n), 'mprk_workspace_bytes')
    return int(n)


def mprk_bind(h: int, u_ptr: int, ws_ptr: int, nbytes: int) -> None:
    check(lib.mprk_bind(_P(h), _P(u_ptr), _P(ws_ptr), nbytes), 'mprk_bind')


def mprk_bind_static(h: int, u_ptr: int) -> None:
    check(lib.mprk_bind_static(_P(h), _P(u_ptr)), 'mprk_bind_static')


def mprk_step(h: int, nsteps: int, want_stats: bool = True):
    st = mprk_stats()
    rc = lib.mprk_step(_P(h), nsteps, C.byref(st) if want_stats else None)
    return rc, (st.as_dict() if want_stats else None)


def mprk_solve(h: int, stage: int, rhs_ptr: int, x_ptr: int):
    info = mprk_solve_info()
    rc = lib.mprk_solve(_P(h), stage, _P(rhs_ptr), _P(x_ptr), C.byref(info))
    return rc, {'iters': info.iters, 'passes': info.passes, 'converged': info.converged,
                'resid': info.resid}


def mprk_set_forcing(h: int, g_ptr: int) -> None:
    check(lib.mprk_set_forcing(_P(h), _P(g_ptr) if g_ptr else None), 'mprk_set_forcing')


def mprk_set_reaction(h: int, r1: float, r2: float, r3: float) -> None:
    check(lib.mprk_set_reaction(_P(h), float(r1), float(r2), float(r3)), 'mprk_set_reaction')


def mprk_set_step_graph(h: int, enable: bool) -> None:
    check(lib.mprk_set_step_graph(_P(h), 1 if enable else 0), 'mprk_set_step_graph')


def mprk_apply(h: int, op: int, stage: int, x_ptr: int, y_ptr: int) -> None:
    check(lib.mprk_apply(_P(h), op, stage, _P(x_ptr), _P(y_ptr)), 'mprk_apply')


def mprk_get_state(h: int):
    t = C.c_double()
    s = C.c_int64()
    check(lib.mprk_get_state(_P(h), C.byref(t), C.byref(s)), 'mprk_get_state')
    return t.value, s.value


def mprk_set_state(h: int, t: float, step: int) -> None:
    check(lib.mprk_set_state(_P(h), t, step), 'mprk_set_state')


def mprk_stats_sync(h: int) -> dict:
    st = mprk_stats()
    check(lib.mprk_stats_sync(_P(h), C.byref(st)), 'mprk_stats_sync')
    return st.as_dict()


def mprk_autotune(h: int):
    a, b = C.c_int32(), C.c_int32()
    check(lib.mprk_autotune(_P(h), C.byref(a), C.byref(b)), 'mprk_autotune')
    return a.value, b.value


def mprk_profile(h: int, enable: bool) -> None:
    check(lib.mprk_profile(_P(h), 1 if enable else 0), 'mprk_profile')


def mprk_launch_info_get(h: int) -> dict:
    li = mprk_launch_info()
    check(lib.mprk_launch_info_get(_P(h), C.byref(li)), 'mprk_launch_info_get')
    return li.as_dict()


def mprk_profile_read(h: int, kclass: int) -> dict:
    n, w, u, ms = C.c_int64(), C.c_int64(), C.c_int64(), C.c_double()
    check(lib.mprk_profile_read(_P(h), kclass, C.byref(n), C.byref(w), C.byref(u), C.byref(ms)),
          'mprk_profile_read')
    return {'launches': n.value, 'worked': w.value, 'units': u.value, 'ms': ms.value}


def mprk_last_error() -> str:
    return lib.mprk_last_error().decode(errors='replace')


def mprk_destroy(h: int) -> None:
    lib.mprk_destroy(_P(h))


def mprk_batch_create(problems, tab: mprk_tableau, prec: mprk_precisions, stream: int = 0) -> int:
    arr = (mprk_problem * len(problems))(*problems)
    h = _P()
    check(lib.mprk_batch_create(len(problems), arr, C.byref(tab), C.byref(prec), _P(stream),
                                C.byref(h)), 'mprk_batch_create')
    return h.value


def mprk_batch_set_schedule(b: int, wg_per_problem) -> None:
    if wg_per_problem is None:
        check(lib.mprk_batch_set_schedule(_P(b), None), 'mprk_batch_set_schedule')
        return
    arr = (C.c_int32 * len(wg_per_problem))(*wg_per_problem)
    check(lib.mprk_batch_set_schedule(_P(b), arr), 'mprk_batch_set_schedule')


def mprk_batch_get_schedule(b: int, count: int):
    arr = (C.c_int32 * count)()
    check(lib.mprk_batch_get_schedule(_P(b), arr), 'mprk_batch_get_schedule')
    return list(arr)


def mprk_batch_autotune(b: int):
    e = C.c_double(0.0)
    ru = C.c_int32(0)
    check(lib.mprk_batch_autotune(_P(b), C.byref(e), C.byref(ru)), 'mprk_batch_autotune')
    return e.value, ru.value


def mprk_batch_workspace_bytes(b: int) -> int:
    n = lib.mprk_batch_workspace_bytes(_P(b))
    if n < 0:
        raise MprkError(int(n), 'mprk_batch_workspace_bytes')
    return int(n)


def mprk_batch_bind(b: int, u_ptrs, ws_ptr: int, nbytes: int) -> None:
    arr = (_P * len(u_ptrs))(*[_P(p) for p in u_ptrs])
    check(lib.mprk_batch_bind(_P(b), arr, _P(ws_ptr), nbytes), 'mprk_batch_bind')


def mprk_batch_step(b: int, nsteps: int) -> int:
    return lib.mprk_batch_step(_P(b), nsteps)


def mprk_batch_stats_sync(b: int, idx: int) -> dict:
    st = mprk_stats()
    check(lib.mprk_batch_stats_sync(_P(b), idx, C.byref(st)), 'mprk_batch_stats_sync')
    return st.as_dict()


def mprk_batch_destroy(b: int) -> None:
    lib.mprk_batch_destroy(_P(b))
