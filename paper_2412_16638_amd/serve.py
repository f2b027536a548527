"""Continuous-batching request loop for time-integration jobs on one GPU.

Requests arrive over time (open loop).  A request is admitted as soon as a slot is free and its
device footprint (the library's exact workspace size plus the FP64 state) fits the memory
budget; admitted jobs run concurrently, each on its own HIP stream with its own handle and
resident workspace, so their kernels overlap on the device, and a job leaves (freeing slot and
memory) when its last step is done.  Latency = completion - arrival.

The scheduler is independent of the device: `GpuBackend` runs jobs through libmprk.so;
`FakeBackend` (deterministic durations, virtual clock) exercises admission, footprint
accounting and the latency statistics on a CPU.
"""
from __future__ import annotations

import dataclasses
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np


@dataclasses.dataclass
class JobResult:
    rid: int
    arrival: float
    admitted: float
    finished: float
    dof_steps: float
    footprint: int
    ok: bool
    stats: dict | None = None
    u: np.ndarray | None = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class GpuBackend:
    """Runs a job as one handle on its own stream; the footprint comes from the library.

    Handles are pooled: a finished job's handle, with its workspace (block-Jacobi inverses
    included) and its iteration history, waits idle for the next job with the same operator,
    grid, tableau and precisions, which then only resets the state and the step counters.  Idle
    handles keep their device memory; the server counts it (idle_bytes) and evicts the least
    recently used ones when an admission needs the room."""

    def __init__(self, device: str = 'cuda:0', keep_u: bool = False, u0_fn=None,
                 pool: bool = True, steps_per_call: int = 0):
        import torch
        from . import _abi as A
        from .stepper import Stepper, precisions
        self.torch, self.A, self.Stepper, self.precisions = torch, A, Stepper, precisions
        self.device = torch.device(device)
        self.keep_u = keep_u
        self.u0_fn = u0_fn  # builds a job's initial field when the job starts (if p.u0 is None)
        self.pool = pool
        self.steps_per_call = steps_per_call  # 0: all of a job's steps in one library call
        self._idle = {}        # key -> idle Steppers (most recently used last)
        self._idle_order = []  # (key, stepper) from least to most recently used
        self._idle_bytes = 0
        self._lock = threading.Lock()
        self.created = 0       # handles made (the rest of the jobs reused a pooled one)

    def _args(self, p):
        A = self.A
        kind = A.OP_HEAT if p.kind == 0 else A.OP_ADVDIFF
        prec = self.precisions(p.precision, p.krylov, precond=p.precond)
        return kind, prec

    @staticmethod
    def _key(p):
        return (p.kind, p.n, p.bc, p.diff, tuple(p.b), p.tableau, p.dt, p.precision, p.krylov,
                p.precond)

    def footprint(self, p) -> int:
        A = self.A
        kind, prec = self._args(p)
        from .stepper import tableau
        g = A.mprk_grid(p.n, p.n, p.n, p.bc)
        o = A.mprk_operator(kind, A.FMT_STENCIL, p.diff, (A.C.c_double * 3)(*p.b))
        h = A.mprk_create(g, o, tableau(p.tableau), prec, p.dt, 0)
        try:
            return A.mprk_workspace_bytes(h) + 8 * p.N
        finally:
            A.mprk_destroy(h)

    def memory_budget(self, fraction: float = 0.8) -> int:
        free, _total = self.torch.cuda.mem_get_info(self.device)
        return int(free * fraction)

    # ---------------- handle pool ----------------
    def idle_bytes(self) -> int:
        return self._idle_bytes

    def has_idle(self, p) -> bool:
        with self._lock:
            return bool(self._idle.get(self._key(p)))

    def evict(self, nbytes: int, keep=None) -> int:
        """Close least recently used idle handles (not of job `keep`'s kind) until at least
        nbytes are released; returns the bytes released."""
        freed = 0
        kk = self._key(keep) if keep is not None else None
        with self._lock:
            i = 0
            while freed < nbytes and i < len(self._idle_order):
                key, st = self._idle_order[i]
                if key == kk:
                    i += 1
                    continue
                self._idle_order.pop(i)
                self._idle[key].remove(st)
                fp = st.ws_bytes + 8 * st.N
                self._idle_bytes -= fp
                freed += fp
                st.close()
        return freed

    def _acquire(self, p):
        key = self._key(p)
        with self._lock:
            lst = self._idle.get(key)
            if self.pool and lst:
                st = lst.pop()
                self._idle_order.remove((key, st))
                self._idle_bytes -= st.ws_bytes + 8 * st.N
                return st
        torch = self.torch
        kind, prec = self._args(p)
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            st = self.Stepper(p.n, p.bc, kind, p.diff, p.b, self.A.FMT_STENCIL, p.tableau, prec,
                              p.dt, str(self.device))
        self.created += 1
        return st

    def _release(self, p, st, ok: bool):
        if not (self.pool and ok):
            st.close()
            return
        key = self._key(p)
        with self._lock:
            self._idle.setdefault(key, []).append(st)
            self._idle_order.append((key, st))
            self._idle_bytes += st.ws_bytes + 8 * st.N

    def close(self):
        self.evict(1 << 62)

    def run(self, p):
        """Advance job p to its last step on its handle's stream; returns (ok, stats, u)."""
        st = self._acquire(p)
        ok = False
        try:
            st.set_u(p.u0 if p.u0 is not None else self.u0_fn(p))
            st.set_state(0.0, 0)
            left = p.nsteps
            stats = None
            ok = True
            chunk = self.steps_per_call or left
            while left > 0:
                n = min(chunk, left)
                rc, stats = st.step(n, check=False)
                if rc != self.A.OK:
                    ok = False
                    break
                left -= n
            u = st.get_u().copy() if self.keep_u else None
        finally:
            self._release(p, st, ok)
        return ok, stats, u


class FakeBackend:
    """Deterministic stand-in: a job takes `sec_per_dof_step * N * steps` of virtual time."""

    def __init__(self, sec_per_dof_step: float = 1e-9, bytes_per_dof: int = 200,
                 budget: int = 1 << 30):
        self.sec_per_dof_step = sec_per_dof_step
        self.bytes_per_dof = bytes_per_dof
        self.budget = budget

    def footprint(self, p) -> int:
        return self.bytes_per_dof * p.N

    def memory_budget(self, fraction: float = 0.8) -> int:
        return self.budget

    def duration(self, p) -> float:
        return self.sec_per_dof_step * p.N * p.nsteps

    def run(self, p):
        """Wall-clock stand-in for Server.run: sleeps the job's duration."""
        time.sleep(self.duration(p))
        return True, None, None


class Server:
    def __init__(self, backend, max_active: int = 8, budget: int | None = None):
        self.backend = backend
        self.max_active = max_active
        self.budget = budget if budget is not None else backend.memory_budget()

    def _admissible(self, fp: int, used: int, active: int) -> bool:
        return active < self.max_active and used + fp <= self.budget

    def _admit_pooled(self, r, fp: int, used: int, active: int) -> bool:
        """Admission with the backend's idle handles counted as resident: a job whose kind
        has an idle handle reuses its memory; otherwise idle handles are evicted (least
        recently used first) when the job would not fit beside them."""
        be = self.backend
        if active >= self.max_active:
            return False
        idle_fn = getattr(be, 'idle_bytes', None)
        if idle_fn is None:
            return used + fp <= self.budget
        reuse = be.has_idle(r.problem)
        idle = idle_fn() - (fp if reuse else 0)
        over = used + fp + idle - self.budget
        if over > 0:
            over -= be.evict(over, keep=r.problem)
        return over <= 0

    # ---------------- virtual-clock simulation (FakeBackend) ----------------
    def simulate(self, requests):
        """Event-driven replay with a virtual clock (no threads).  Concurrent jobs share the
        device: with k jobs running each progresses at 1/k of its solo speed."""
        be = self.backend
        pending = sorted(requests, key=lambda r: r.arrival)
        fps = {r.rid: be.footprint(r.problem) for r in pending}
        for r in pending:
            if fps[r.rid] > self.budget:
                raise ValueError(f'request {r.rid} can never fit the memory budget')
        t = 0.0
        queue = []            # arrived, waiting (FIFO)
        running = {}          # rid -> [remaining work (s), request, admitted time]
        used = 0
        peak_used = 0
        peak_active = 0
        results = []
        i = 0
        while i < len(pending) or queue or running:
            # admit in arrival order while it fits (FIFO: no overtaking)
            while queue and self._admissible(fps[queue[0].rid], used, len(running)):
                r = queue.pop(0)
                running[r.rid] = [be.duration(r.problem), r, t]
                used += fps[r.rid]
                peak_used = max(peak_used, used)
                peak_active = max(peak_active, len(running))
            k = len(running)
            t_next_arrival = pending[i].arrival if i < len(pending) else float('inf')
            t_next_finish = float('inf')
            if k:
                rem = min(v[0] for v in running.values())
                t_next_finish = t + rem * k
            t_new = min(t_next_arrival, t_next_finish)
            if k:
                dt = t_new - t
                for v in running.values():
                    v[0] -= dt / k
            t = t_new
            if t_next_arrival <= t_next_finish and i < len(pending):
                queue.append(pending[i])
                i += 1
            else:
                done = [rid for rid, v in running.items() if v[0] <= 1e-15]
                for rid in sorted(done):
                    rem, r, t_adm = running.pop(rid)
                    used -= fps[rid]
                    results.append(JobResult(rid, r.arrival, t_adm, t, r.problem.N * r.problem.nsteps,
                                             fps[rid], True))
        out = summarize(results, self.budget)
        out['peak_resident_bytes'] = peak_used
        out['peak_active'] = peak_active
        return out

    # ---------------- real run (GpuBackend) ----------------
    def run(self, requests, time_scale: float = 1.0, log=None):
        """Open-loop replay on the wall clock (arrival times scaled by time_scale)."""
        be = self.backend
        pending = sorted(requests, key=lambda r: r.arrival)
        fps = {r.rid: be.footprint(r.problem) for r in pending}
        for r in pending:
            if fps[r.rid] > self.budget:
                raise ValueError(f'request {r.rid} can never fit the memory budget')
        lock = threading.Condition()
        state = {'used': 0, 'active': 0, 'peak_used': 0, 'peak_active': 0}
        results = []
        t0 = time.perf_counter()

        def work(r, t_adm):
            # the slot and the footprint are released whatever the job does: a job that raises
            # (device memory exhausted, a rejected problem) is recorded as failed with its error
            ok, stats, u, err = False, None, None, None
            try:
                ok, stats, u = be.run(r.problem)
            except Exception as e:  # noqa: BLE001 -- any failure of one job is that job's result
                err = f'{type(e).__name__}: {e}'
            finally:
                t_fin = time.perf_counter() - t0
                with lock:
                    state['used'] -= fps[r.rid]
                    state['active'] -= 1
                    results.append(JobResult(r.rid, r.arrival * time_scale, t_adm, t_fin,
                                             r.problem.N * r.problem.nsteps, fps[r.rid], ok, stats,
                                             u, err))
                    lock.notify_all()

        queue = []
        i = 0
        with ThreadPoolExecutor(self.max_active) as ex:
            while i < len(pending) or queue:
                with lock:
                    now = time.perf_counter() - t0
                    while i < len(pending) and pending[i].arrival * time_scale <= now:
                        queue.append(pending[i])
                        i += 1
                    while queue and self._admit_pooled(queue[0], fps[queue[0].rid], state['used'],
                                                       state['active']):
                        r = queue.pop(0)
                        state['used'] += fps[r.rid]
                        state['active'] += 1
                        state['peak_used'] = max(state['peak_used'],
                                                 state['used'] + getattr(be, 'idle_bytes', lambda: 0)())
                        state['peak_active'] = max(state['peak_active'], state['active'])
                        ex.submit(work, r, now)
                        if log:
                            log(f'admit {r.rid} n={r.problem.n} steps={r.problem.nsteps} '
                                f'{r.problem.precision} active={state["active"]}')
                    if i < len(pending) or queue:
                        wait = 0.05
                        if i < len(pending):
                            wait = max(0.0, min(wait, pending[i].arrival * time_scale - now))
                        lock.wait(timeout=wait if wait > 0 else 0.001)
        out = summarize(results, self.budget)
        out['peak_resident_bytes'] = state['peak_used']
        out['peak_active'] = state['peak_active']
        return out


def summarize(results, budget):
    lat = np.array([r.latency for r in results]) if results else np.zeros(0)
    makespan = max((r.finished for r in results), default=0.0)
    first = min((r.arrival for r in results), default=0.0)
    dof = sum(r.dof_steps for r in results)
    return {
        'n': len(results),
        'failed': sum(0 if r.ok else 1 for r in results),
        'p50_s': float(np.percentile(lat, 50)) if lat.size else None,
        'p99_s': float(np.percentile(lat, 99)) if lat.size else None,
        'mean_s': float(lat.mean()) if lat.size else None,
        'makespan_s': makespan,
        'dof_steps': dof,
        'dof_steps_per_s': dof / (makespan - first) if makespan > first else None,
        'budget_bytes': budget,
        'results': sorted(results, key=lambda r: r.rid),
    }
