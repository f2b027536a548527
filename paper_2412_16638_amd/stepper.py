"""Torch-memory plumbing around the C ABI: one problem = one handle + two device tensors.

PyTorch supplies only device memory (the FP64 state u and one workspace blob) and the HIP
stream; every arithmetic step runs in libmprk.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _abi as A

TABLEAUS = {'SDIRK2': (A.TAB_SDIRK2, 0), 'SDIRK3': (A.TAB_SDIRK3, 0), '4S3PA': (A.TAB_4S3PA, 0),
            '4S3PB': (A.TAB_4S3PB, 0), '4S3PC': (A.TAB_4S3PC, 0)}
STORAGE = {'fp64': A.FP64, 'fp32': A.FP32, 'fp16': A.FP16}
KRYLOV = {'cg': A.CG, 'gmres': A.GMRES}
LP_DTYPE = {A.FP64: torch.float64, A.FP32: torch.float32, A.FP16: torch.float16}


def tableau(name: str) -> A.mprk_tableau:
    name = name.upper()
    if name.startswith('MID'):
        return A.mprk_tableau_builtin(A.TAB_MID, int(name[3:] or 0))
    tid, param = TABLEAUS[name]
    return A.mprk_tableau_builtin(tid, param)


def precisions(storage: str = 'fp64', krylov: str = 'cg', **overrides) -> A.mprk_precisions:
    p = A.mprk_precisions_default(STORAGE[storage], KRYLOV[krylov])
    for k, v in overrides.items():
        if k == 'precond':
            v = {'none': A.PRECOND_NONE, 'bj': A.PRECOND_BJ, 'fdm': A.PRECOND_FDM}.get(v, v)
        setattr(p, k, v)
    return p


class Stepper:
    """One time-integration problem bound to torch-owned device memory."""

    def __init__(self, shape, bc: int, kind: int, diff: float, b=(0.0, 0.0, 0.0),
                 fmt: int = A.FMT_STENCIL, tab='SDIRK3', prec=None, dt: float = 1e-3,
                 device: str = 'cuda:0'):
        if not torch.cuda.is_available():
            raise RuntimeError('mprk needs a HIP device (torch.cuda.is_available() is False)')
        if isinstance(shape, int):
            shape = (shape, shape, shape)
        self.shape = tuple(int(s) for s in shape)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.device = torch.device(device)
        self.grid = A.mprk_grid(self.shape[0], self.shape[1], self.shape[2], bc)
        self.op = A.mprk_operator(kind, fmt, diff, (A.C.c_double * 3)(*b))
        self.tab = tableau(tab) if isinstance(tab, str) else tab
        self.prec = prec if prec is not None else precisions()
        self.dt = dt
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.h = A.mprk_create(self.grid, self.op, self.tab, self.prec, dt, self.stream.cuda_stream)
            self.ws_bytes = A.mprk_workspace_bytes(self.h)
            self.u = torch.zeros(self.N, dtype=torch.float64, device=self.device)
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            A.mprk_bind(self.h, self.u.data_ptr(), self.ws.data_ptr(), self.ws_bytes)

    @property
    def lp_dtype(self):
        return LP_DTYPE[self.prec.storage]

    def set_u(self, u) -> None:
        """Copy a host or device field into the state (on the handle's stream)."""
        if isinstance(u, np.ndarray):
            u = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float64).ravel())
        with torch.cuda.stream(self.stream):
            self.u.copy_(u.reshape(-1).to(self.device, torch.float64))
        self.stream.synchronize()

    def get_u(self) -> np.ndarray:
        self.stream.synchronize()
        with torch.cuda.stream(self.stream):
            out = self.u.detach().cpu().numpy()
        return out.reshape(self.shape[2], self.shape[1], self.shape[0])

    def set_forcing(self, g) -> None:
        """Constant forcing g of du/dt = K u + g (host or device field), or None to remove it.
        The device copy is kept alive here while the handle uses it."""
        if g is None:
            A.mprk_set_forcing(self.h, 0)
            self.g = None
            return
        if isinstance(g, np.ndarray):
            g = torch.from_numpy(np.ascontiguousarray(g, dtype=np.float64).ravel())
        self.g = g.reshape(-1).to(self.device, torch.float64).contiguous()
        torch.cuda.synchronize(self.device)
        A.mprk_set_forcing(self.h, self.g.data_ptr())

    def set_step_graph(self, enable: bool = True) -> None:
        """Replay whole steps from a captured hipGraph once the stage histories exist."""
        A.mprk_set_step_graph(self.h, enable)

    def set_reaction(self, r1: float = 0.0, r2: float = 0.0, r3: float = 0.0) -> None:
        """Pointwise reaction R(u) = r1 u + r2 u^2 + r3 u^3 of du/dt = K u + g + R(u); all zero
        removes it."""
        A.mprk_set_reaction(self.h, r1, r2, r3)

    def step(self, nsteps: int = 1, check: bool = True):
        rc, st = A.mprk_step(self.h, nsteps, True)
        if check:
            A.check(rc, 'mprk_step')
        return (rc, st) if not check else st

    def solve(self, stage: int, rhs: torch.Tensor):
        x = torch.empty_like(rhs)
        rc, info = A.mprk_solve(self.h, stage, rhs.data_ptr(), x.data_ptr())
        A.check(rc, 'mprk_solve')
        return x, info

    def apply(self, which: int, x: torch.Tensor, stage: int = 0) -> torch.Tensor:
        y = torch.empty_like(x)
        A.mprk_apply(self.h, which, stage, x.data_ptr(), y.data_ptr())
        return y

    def autotune(self):
        """Pick the launch shape (groups per thread) by timing candidates; returns (vec, row)."""
        return A.mprk_autotune(self.h)

    def launch_info(self) -> dict:
        """Launch shapes in use (groups per thread, tile depths, GMRES step form)."""
        return A.mprk_launch_info_get(self.h)

    def state(self):
        return A.mprk_get_state(self.h)

    def set_state(self, t: float, step: int) -> None:
        A.mprk_set_state(self.h, t, step)

    def close(self) -> None:
        if getattr(self, 'h', None):
            A.mprk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_problem(p, fmt: int = A.FMT_STENCIL, prec=None, device: str = 'cuda:0', **prec_overrides):
    """Stepper for a problem description with fields n, bc, kind, diff, b, tableau, dt,
    precision, krylov, precond (e.g. a workloads.Problem); u is initialised from p.u0."""
    if prec is None:
        prec = precisions(p.precision, p.krylov, precond=p.precond, **prec_overrides)
    s = Stepper(p.n, p.bc, p.kind, p.diff, p.b, fmt, p.tableau, prec, p.dt, device)
    if p.u0 is not None:
        s.set_u(p.u0)
    if getattr(p, 'forcing', None) is not None:
        s.set_forcing(p.forcing)
    if getattr(p, 'reaction', None) is not None:
        s.set_reaction(*p.reaction)
    return s


class Batch:
    """Many independent problems advanced together (one persistent launch per stage)."""

    def __init__(self, problems, tab='SDIRK3', prec=None, device: str = 'cuda:0', schedule=None):
        if not torch.cuda.is_available():
            raise RuntimeError('mprk needs a HIP device (torch.cuda.is_available() is False)')
        self.device = torch.device(device)
        self.tab = tableau(tab) if isinstance(tab, str) else tab
        self.prec = prec if prec is not None else precisions('fp32', 'cg')
        descs = []
        self.shapes = []
        for p in problems:
            sh = (p['shape'],) * 3 if isinstance(p['shape'], int) else tuple(p['shape'])
            self.shapes.append(sh)
            g = A.mprk_grid(sh[0], sh[1], sh[2], p.get('bc', A.BC_DIRICHLET0))
            o = A.mprk_operator(p.get('kind', A.OP_HEAT), A.FMT_STENCIL, p['diff'],
                                (A.C.c_double * 3)(*p.get('b', (0.0, 0.0, 0.0))))
            descs.append(A.mprk_problem(g, o, p['dt']))
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.h = A.mprk_batch_create(descs, self.tab, self.prec, self.stream.cuda_stream)
            if schedule is not None:
                A.mprk_batch_set_schedule(self.h, schedule)
            self.ws_bytes = A.mprk_batch_workspace_bytes(self.h)
            self.schedule = A.mprk_batch_get_schedule(self.h, len(descs))
            self.u = [torch.zeros(s[0] * s[1] * s[2], dtype=torch.float64, device=self.device)
                      for s in self.shapes]
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            A.mprk_batch_bind(self.h, [t.data_ptr() for t in self.u], self.ws.data_ptr(),
                              self.ws_bytes)

    def set_u(self, i: int, u) -> None:
        if isinstance(u, np.ndarray):
            u = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float64).ravel())
        self.u[i].copy_(u.reshape(-1).to(self.device, torch.float64))
        torch.cuda.synchronize(self.device)

    def get_u(self, i: int) -> np.ndarray:
        torch.cuda.synchronize(self.device)
        s = self.shapes[i]
        return self.u[i].cpu().numpy().reshape(s[2], s[1], s[0])

    def step(self, nsteps: int = 1) -> None:
        A.check(A.mprk_batch_step(self.h, nsteps), 'mprk_batch_step')

    def autotune(self):
        """Pick rows per thread and the CTA-group schedule by timing one step per candidate;
        returns (work-model exponent, rows per thread)."""
        e, ru = A.mprk_batch_autotune(self.h)
        self.schedule = A.mprk_batch_get_schedule(self.h, len(self.shapes))
        return e, ru

    def stats(self, i: int) -> dict:
        return A.mprk_batch_stats_sync(self.h, i)

    def close(self) -> None:
        if getattr(self, 'h', None):
            A.mprk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
