"""Serving scheduler on the CPU: admission, footprint accounting, latency statistics
(deterministic fake backend with a virtual clock)."""
import importlib.util
import os
import sys

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# load serve.py without importing the package (which needs the built library)
_spec = importlib.util.spec_from_file_location(
    'mprk_serve', os.path.join(ROOT, 'paper_2412_16638_amd', 'serve.py'))
S = importlib.util.module_from_spec(_spec)
sys.modules['mprk_serve'] = S
_spec.loader.exec_module(S)


def _req(rid, t, n, steps):
    p = W.Problem(f'r{rid}', n, W.DIRICHLET, W.HEAT, 1.0, (0, 0, 0), 'SDIRK3', 1e-3, steps, None)
    return W.Request(rid, t, p)


def test_single_slot_is_a_fifo_queue():
    be = S.FakeBackend(sec_per_dof_step=1e-6, bytes_per_dof=1, budget=10 ** 9)
    reqs = [_req(0, 0.0, 10, 1), _req(1, 0.1, 10, 1), _req(2, 0.2, 10, 1)]   # 1 ms each
    reqs[0].problem.nsteps = 1000  # 1 s
    out = S.Server(be, max_active=1).simulate(reqs)
    res = out['results']
    assert [round(r.finished, 9) for r in res] == [1.0, 1.001, 1.002]
    assert [round(r.admitted, 9) for r in res] == [0.0, 1.0, 1.001]
    assert out['peak_active'] == 1


def test_processor_sharing_and_latency_percentiles():
    be = S.FakeBackend(sec_per_dof_step=1e-5, bytes_per_dof=1, budget=10 ** 9)
    # two equal jobs arriving together share the device: both finish at 2x their solo time
    reqs = [_req(0, 0.0, 10, 100), _req(1, 0.0, 10, 100)]   # 1000 DOF x 100 steps: solo 1 s
    out = S.Server(be, max_active=4).simulate(reqs)
    assert all(abs(r.finished - 2.0) < 1e-12 for r in out['results'])
    assert abs(out['p50_s'] - 2.0) < 1e-12 and abs(out['p99_s'] - 2.0) < 1e-12
    assert abs(out['dof_steps_per_s'] - 2 * 1000 * 100 / 2.0) < 1e-6


def test_memory_budget_limits_concurrency():
    be = S.FakeBackend(sec_per_dof_step=1e-6, bytes_per_dof=100, budget=250_000)
    reqs = [_req(i, 0.0, 10, 10) for i in range(6)]   # footprint 100 * 1000 = 100 kB each
    out = S.Server(be, max_active=8).simulate(reqs)
    assert out['peak_active'] == 2
    assert out['peak_resident_bytes'] <= 250_000
    assert out['n'] == 6 and out['failed'] == 0


def test_request_that_never_fits_is_rejected():
    be = S.FakeBackend(bytes_per_dof=100, budget=1000)
    with pytest.raises(ValueError):
        S.Server(be).simulate([_req(0, 0.0, 10, 1)])


def test_seeded_request_mix_statistics():
    reqs = W.request_stream(materialize_u0=False)
    assert len(reqs) == 512
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) >= 0)
    assert 8.0 < arr[-1] < 12.5                       # ~512 / 50 s
    ns = np.array([r.problem.n for r in reqs])
    assert ns.min() >= 32 and ns.max() <= 192
    kinds = np.array([r.problem.kind for r in reqs])
    assert 0.4 < kinds.mean() < 0.6
    be = S.FakeBackend(sec_per_dof_step=2e-10, bytes_per_dof=120, budget=64 << 30)
    out = S.Server(be, max_active=16).simulate(reqs)
    assert out['n'] == 512
    lat = np.array([r.latency for r in out['results']])
    assert out['p50_s'] == pytest.approx(np.percentile(lat, 50))
    assert out['p99_s'] >= out['p50_s']


class _RaisingBackend(S.FakeBackend):
    """Wall-clock fake whose job `bad` raises, as a job does when its device memory runs out."""

    def __init__(self, bad, **kw):
        super().__init__(**kw)
        self.bad = bad

    def run(self, p):
        if p.name == f'r{self.bad}':
            raise MemoryError('workspace allocation failed')
        return super().run(p)


def test_a_job_that_raises_releases_its_slot_and_is_reported_failed():
    # one slot: if the raising job kept it, the three jobs queued behind it would never start
    be = _RaisingBackend(1, sec_per_dof_step=1e-6, bytes_per_dof=1, budget=10 ** 9)
    reqs = [_req(i, 0.0, 10, 2) for i in range(5)]            # 2 ms each
    out = S.Server(be, max_active=1).run(reqs)
    assert out['n'] == 5 and out['failed'] == 1
    res = {r.rid: r for r in out['results']}
    assert not res[1].ok and 'MemoryError' in res[1].error
    assert all(res[i].ok and res[i].error is None for i in (0, 2, 3, 4))
    assert out['peak_active'] == 1


class _PoolBackend(S.FakeBackend):
    """Fake with the pooled backend's accounting: idle handles hold memory until evicted."""

    def __init__(self, idle, **kw):
        super().__init__(**kw)
        self.idle = dict(idle)        # key (n) -> bytes held by an idle handle of that kind
        self.evicted = []

    def idle_bytes(self):
        return sum(self.idle.values())

    def has_idle(self, p):
        return p.n in self.idle

    def evict(self, nbytes, keep=None):
        freed = 0
        for k in sorted(self.idle):
            if freed >= nbytes:
                break
            if keep is not None and k == keep.n:
                continue
            freed += self.idle.pop(k)
            self.evicted.append(k)
        return freed


def test_pooled_admission_counts_idle_memory_and_evicts_it_when_needed():
    # budget 1000 B, footprint = n bytes; idle handles of n = 300 and n = 400 hold 700 B
    be = _PoolBackend({300: 300, 400: 400}, bytes_per_dof=1, budget=1000)
    srv = S.Server(be, max_active=4)
    r_same = _req(0, 0.0, 1, 1)
    r_same.problem.n = 400                     # reuses the idle n = 400 handle: no eviction
    assert srv._admit_pooled(r_same, 400, used=0, active=0)
    assert be.evicted == []
    r_new = _req(1, 0.0, 1, 1)
    r_new.problem.n = 500                      # 500 + 700 idle > 1000: evicts n = 300 only
    assert srv._admit_pooled(r_new, 500, used=0, active=0)
    assert be.evicted == [300]
    r_big = _req(2, 0.0, 1, 1)
    r_big.problem.n = 800                      # 300 used + 800 > 1000 even with no idle memory
    assert not srv._admit_pooled(r_big, 800, used=300, active=1)
    assert be.evicted == [300, 400]            # (what could be evicted was)
    assert not srv._admit_pooled(r_same, 400, used=0, active=4)   # no free slot
