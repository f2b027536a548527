"""The largest grid the int32 indexing admits (659^3 = 286 M unknowns, 7N < 2^31; the
block-Jacobi table of 8N entries is indexed in 64 bits): two SDIRK3 steps of the heat problem
from one sine mode, FP32 block-Jacobi CG stage solves, checked at sampled points against the
oracle's modal closed form R(tau lambda)^N phi (a value the oracle computes point by point)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import tableaus
from tests.gpu_util import log_case

pytestmark = pytest.mark.gpu

M = pytest.importorskip('paper_2412_16638_amd')
A = M._abi


def test_heat_sine_mode_at_the_int32_size_limit():
    if torch.cuda.get_device_properties(0).total_memory < 64 * 2 ** 30:
        pytest.skip('needs about 40 GB of device memory')
    n, kvec, kappa, dt, nsteps = 659, (1, 2, 3), 1.0, 5e-4, 2
    log_case('maxsize_heat', n=n)
    prec = M.precisions('fp32', 'cg')
    st = M.Stepper((n, n, n), W.DIRICHLET, W.HEAT, kappa, (0, 0, 0), A.FMT_STENCIL, 'SDIRK3', prec, dt)
    # u0 = phi, built on the device from its separable factors
    h = 1.0 / (n + 1)
    x = torch.arange(1, n + 1, dtype=torch.float64, device='cuda') * h
    f = [torch.sin(k * np.pi * x) for k in kvec]
    st.u.copy_((f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]).reshape(-1))
    del f
    torch.cuda.synchronize()
    st.step(nsteps)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    idx = rng.integers(0, n ** 3, 4096)
    u = st.u[torch.from_numpy(idx).cuda()].cpu().numpy()
    st.close()
    i, j, k = idx % n, (idx // n) % n, idx // (n * n)
    phi = (np.sin(kvec[0] * np.pi * (i + 1) * h) * np.sin(kvec[1] * np.pi * (j + 1) * h)
           * np.sin(kvec[2] * np.pi * (k + 1) * h))
    lam = -kappa * sum((4.0 / h ** 2) * np.sin(kk * np.pi * h / 2.0) ** 2 for kk in kvec)
    amp = np.real(tableaus.stability_function(tableaus.by_name('SDIRK3'), dt * lam)) ** nsteps
    ref = amp * phi
    assert np.linalg.norm(u - ref) <= 1e-6 * np.linalg.norm(ref), np.linalg.norm(u - ref) / np.linalg.norm(ref)
