"""Modal closed forms of the semi-discrete problems (oracle, test infrastructure).

For du/dt = K u with a diagonalisable K = Q diag(lambda) Q^{-1}, one step of a
Runge--Kutta method with exact stage solves multiplies each mode by R(tau lambda),
R the stability function of Section "Method stability in the context of mixed
precision".  Hence u_N = Q diag(R(tau lambda)^N) Q^{-1} u_0 exactly, at any size.

  * Dirichlet heat: the sine modes phi_k(x) = prod_d sin(k_d pi x_d), k_d = 1..n_d,
    are eigenvectors of the 7-point Laplacian with
    lambda_k = -kappa sum_d (4/h_d^2) sin^2(k_d pi h_d / 2); the transform is the
    type-I discrete sine transform.  (The paper's heat solution is a sine mode,
    Section "Heat equation".)
  * Periodic advection-diffusion: the DFT diagonalises K, with, per axis,
    nu (2 cos theta - 2)/h^2 - b (1 - e^{-i theta})/h for b >= 0 (backward
    upwind difference) and - b (e^{i theta} - 1)/h for b < 0, theta = 2 pi m / n
    (numpy's FFT sign convention); with central differences - i b sin(theta) / h.
  * Constant forcing g along the lowest Dirichlet sine mode (the paper's forced heat test,
    Section "Heat equation", u(0) = 0): the solution stays a(t) g.  For a' = lambda a + 1
    one DIRK step with exact stage solves has stage values Y = (I - zA)^{-1}(a e + tau A e),
    z = tau lambda, so a_{n+1} = a_n + tau b^T (lambda Y + e) = R(z) a_n + tau b^T (I - zA)^{-1} e
    (using z (I - zA)^{-1} A e + e = (I - zA)^{-1} e); the semi-discrete exact amplitude is
    (e^{lambda t} - 1) / lambda, and the continuum one (1 - e^{-3 pi^2 kappa t}) / (3 pi^2 kappa).
The continuum decay of the lowest heat mode is exp(-3 pi^2 kappa t) (Section
"Heat equation": the analytic solution decays at rate 3 pi^2).
Fields are arrays of shape (nz, ny, nx) (x fastest when flattened).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .tableaus import stability_function


def _spacing(n: int, periodic: bool) -> float:
    return 1.0 / n if periodic else 1.0 / (n + 1)


def heat_eigenvalues(shape, kappa: float) -> np.ndarray:
    """lambda[kz-1, ky-1, kx-1] of kappa Lap_h with zero Dirichlet, shape = (nx, ny, nz)."""
    lam1 = []
    for n in shape:
        h = _spacing(n, False)
        k = np.arange(1, n + 1)
        lam1.append(-(4.0 / h ** 2) * np.sin(k * np.pi * h / 2.0) ** 2)
    lx, ly, lz = lam1
    return kappa * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :])


def heat_sine_mode(shape, kvec) -> np.ndarray:
    """prod_d sin(k_d pi x_d), x_d = (i+1) h_d, as an array (nz, ny, nx)."""
    f = []
    for n, k in zip(shape, kvec):
        h = _spacing(n, False)
        f.append(np.sin(k * np.pi * h * np.arange(1, n + 1)))
    fx, fy, fz = f
    return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]


def periodic_eigenvalues(shape, nu: float, b, central: bool = False) -> np.ndarray:
    """DFT symbol of nu Lap_h - sum_d b_d D_d (upwind, or central), as an array (nz, ny, nx)."""
    parts = []
    for d, n in enumerate(shape):
        h = _spacing(n, True)
        theta = 2.0 * np.pi * np.arange(n) / n
        lam = nu * (2.0 * np.cos(theta) - 2.0) / h ** 2
        if central:
            lam = lam - 1j * b[d] * np.sin(theta) / h
        elif b[d] >= 0.0:
            lam = lam - b[d] * (1.0 - np.exp(-1j * theta)) / h
        else:
            lam = lam - b[d] * (np.exp(1j * theta) - 1.0) / h
        parts.append(lam)
    lx, ly, lz = parts
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def evolve_heat(u0: np.ndarray, kappa: float, tau: float, nsteps: int, tab) -> np.ndarray:
    """u_N of the DIRK with exact solves for Dirichlet heat, via DST-I."""
    nz, ny, nx = u0.shape
    lam = heat_eigenvalues((nx, ny, nz), kappa)
    amp = np.real(stability_function(tab, tau * lam)) ** nsteps
    c = sfft.dstn(u0, type=1)
    return sfft.idstn(c * amp, type=1)


def evolve_heat_exact(u0: np.ndarray, kappa: float, t: float) -> np.ndarray:
    """Semi-discrete exact solution exp(t K) u0 for Dirichlet heat."""
    nz, ny, nx = u0.shape
    lam = heat_eigenvalues((nx, ny, nz), kappa)
    c = sfft.dstn(u0, type=1)
    return sfft.idstn(c * np.exp(t * lam), type=1)


def evolve_periodic(u0: np.ndarray, nu: float, b, tau: float, nsteps: int, tab,
                    central: bool = False) -> np.ndarray:
    """u_N of the DIRK with exact solves for periodic advection-diffusion, via FFT."""
    nz, ny, nx = u0.shape
    lam = periodic_eigenvalues((nx, ny, nz), nu, b, central)
    amp = stability_function(tab, tau * lam) ** nsteps
    return np.real(sfft.ifftn(sfft.fftn(u0) * amp))


class PeriodicEvolution:
    """evolve_periodic for one initial state and many (tableau, tau, nsteps): the forward
    transform of u0 and the DFT symbol are computed once."""

    def __init__(self, u0: np.ndarray, nu: float, b, central: bool = False):
        nz, ny, nx = u0.shape
        self.lam = periodic_eigenvalues((nx, ny, nz), nu, b, central)
        self.u0_hat = sfft.fftn(u0)

    def __call__(self, tau: float, nsteps: int, tab) -> np.ndarray:
        amp = stability_function(tab, tau * self.lam) ** nsteps
        return np.real(sfft.ifftn(self.u0_hat * amp))


def evolve_periodic_exact(u0: np.ndarray, nu: float, b, t: float,
                          central: bool = False) -> np.ndarray:
    """Semi-discrete exact solution exp(t K) u0 for periodic advection-diffusion."""
    nz, ny, nx = u0.shape
    lam = periodic_eigenvalues((nx, ny, nz), nu, b, central)
    return np.real(sfft.ifftn(sfft.fftn(u0) * np.exp(t * lam)))


def evolve(u0: np.ndarray, kind: int, bc: int, diff: float, b, tau: float, nsteps: int, tab):
    """Dispatch to the closed form matching (kind, bc); kind 0 heat, bc 0 Dirichlet."""
    if kind == 0 and bc == 0:
        return evolve_heat(u0, diff, tau, nsteps, tab)
    if bc == 1:
        bb = (0.0, 0.0, 0.0) if kind == 0 else b
        return evolve_periodic(u0, diff, bb, tau, nsteps, tab, central=kind == 2)
    raise ValueError('no closed form for Dirichlet advection-diffusion')


def stage_sum(tab, z):
    """b^T (I - z A)^{-1} e for an array of complex z (forward substitution per stage)."""
    z = np.asarray(z, dtype=np.complex128)
    A, b = tab.A, tab.b
    X = []
    for i in range(tab.s):
        acc = np.ones_like(z)
        for j in range(i):
            acc = acc + z * A[i, j] * X[j]
        X.append(acc / (1.0 - z * A[i, i]))
    return sum(b[i] * X[i] for i in range(tab.s))


def forced_mode_amplitude(tab, lam: float, tau: float, nsteps: int) -> float:
    """a_N of the DIRK for a' = lambda a + 1, a_0 = 0 (exact stage solves)."""
    z = tau * lam
    R = complex(stability_function(tab, z))
    beta = complex(stage_sum(tab, z))
    a = 0.0
    for _ in range(nsteps):
        a = (R * a + tau * beta).real
    return a


def forced_heat_lowest_eigenvalue(shape, kappa: float) -> float:
    """lambda of the (1, 1, 1) sine mode of kappa Lap_h (zero Dirichlet)."""
    return float(heat_eigenvalues(shape, kappa)[0, 0, 0])


def evolve_forced_heat(g: np.ndarray, kappa: float, tau: float, nsteps: int, tab) -> np.ndarray:
    """u_N of the DIRK for du/dt = K u + g, u_0 = 0, g the lowest sine mode (array (nz,ny,nx))."""
    nz, ny, nx = g.shape
    lam = forced_heat_lowest_eigenvalue((nx, ny, nz), kappa)
    return forced_mode_amplitude(tab, lam, tau, nsteps) * g


def forced_heat_exact(g: np.ndarray, kappa: float, t: float, continuum: bool = False) -> np.ndarray:
    """Exact solution at t: semi-discrete (e^{lambda t} - 1)/lambda g, or the continuum
    (1 - e^{-3 pi^2 kappa t}) / (3 pi^2 kappa) g."""
    if continuum:
        c = 3.0 * np.pi ** 2 * kappa
        return (1.0 - np.exp(-c * t)) / c * g
    nz, ny, nx = g.shape
    lam = forced_heat_lowest_eigenvalue((nx, ny, nz), kappa)
    return (np.exp(lam * t) - 1.0) / lam * g
