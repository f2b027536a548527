"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side tests.

This module holds no arithmetic of the time-stepping method: no operators, no
tableaus, no solves.  It only draws the seeded random numbers of each workload
and evaluates the initial fields (sine modes, a Gaussian bump) at the grid
nodes.  Both the oracle and the GPU path receive its arrays as inputs.

Grid conventions (the paper's unit cube, Section "Test cases"):
  * zero Dirichlet: n interior nodes per axis, spacing h = 1/(n+1), nodes at
    x_i = (i+1) h for i = 0..n-1;
  * periodic: spacing h = 1/n, nodes at x_i = i h for i = 0..n-1.
Global vectors are lexicographic with x fastest: x_{ijk} = x[i + n_x j + n_x n_y k]
(Section "Implementation of the Mixed-precision Runge--Kutta methods").
A 3-D field is returned as a float64 array of shape (nz, ny, nx); ``.ravel()``
gives the lexicographic vector.
"""
from __future__ import annotations

import dataclasses
import numpy as np

DIRICHLET = 0
PERIODIC = 1

HEAT = 0
ADVDIFF = 1
CENTRAL = 2   # advection(-diffusion) with central differences (the paper's advection test)


def axis_nodes(n: int, bc: int) -> np.ndarray:
    """Node coordinates along one axis (see the module docstring)."""
    if bc == DIRICHLET:
        return (np.arange(n, dtype=np.float64) + 1.0) / (n + 1)
    return np.arange(n, dtype=np.float64) / n


def sine_mode(shape, kvec, bc: int = DIRICHLET) -> np.ndarray:
    """prod_d sin(k_d pi x_d) at the nodes; shape = (nx, ny, nz), kvec = (kx, ky, kz)."""
    nx, ny, nz = shape
    sx = np.sin(kvec[0] * np.pi * axis_nodes(nx, bc))
    sy = np.sin(kvec[1] * np.pi * axis_nodes(ny, bc))
    sz = np.sin(kvec[2] * np.pi * axis_nodes(nz, bc))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def fourier_sine_modes(n: int, rng: np.random.Generator, nmodes: int = 8, kmax: int = 8):
    """The 'sum of seeded random Fourier sine modes' initial state.

    Draw order (fixed): k = rng.integers(1, kmax+1, (nmodes, 3)), then
    a = rng.standard_normal(nmodes) / |k|^2 with |k|^2 = k1^2 + k2^2 + k3^2.
    Returns (u0 of shape (n, n, n), k, a).
    """
    k = rng.integers(1, kmax + 1, (nmodes, 3))
    a = rng.standard_normal(nmodes) / (k ** 2).sum(axis=1)
    u = np.zeros((n, n, n))
    for m in range(nmodes):
        u += a[m] * sine_mode((n, n, n), k[m], DIRICHLET)
    return u, k, a


def gaussian_bump(n: int, center, width: float = 100.0, bc: int = PERIODIC) -> np.ndarray:
    """exp(-width * |x - center|^2) at the nodes (the advection initial state shape)."""
    x = axis_nodes(n, bc)
    gx = np.exp(-width * (x - center[0]) ** 2)
    gy = np.exp(-width * (x - center[1]) ** 2)
    gz = np.exp(-width * (x - center[2]) ** 2)
    return gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


@dataclasses.dataclass
class Problem:
    """One time-integration job: grid, physics, initial state and step control."""
    name: str
    n: int
    bc: int
    kind: int                  # HEAT, ADVDIFF or CENTRAL
    diff: float                # kappa (heat) or nu (advection-diffusion)
    b: tuple                   # advection velocity (0,0,0) for heat
    tableau: str               # 'SDIRK2' | 'SDIRK3' | ...
    dt: float
    nsteps: int
    u0: np.ndarray             # shape (n, n, n), float64
    precision: str = 'fp64'    # 'fp64' | 'fp32' | 'fp16' (storage of the implicit solve)
    krylov: str = 'cg'         # 'cg' | 'gmres'
    precond: str = 'bj'        # 'none' | 'bj' | 'fdm'
    meta: dict = dataclasses.field(default_factory=dict)
    forcing: np.ndarray = None # constant source g of du/dt = K u + g, shape (n, n, n), or None
    reaction: tuple = None     # (r1, r2, r3) of du/dt = K u + g + r1 u + r2 u^2 + r3 u^3, or None

    @property
    def N(self) -> int:
        return self.n ** 3


def heat_sine_16() -> Problem:
    """16^3 interior grid heat problem, u0 = sin(pi x) sin(pi y) sin(pi z)."""
    n = 16
    u0 = sine_mode((n, n, n), (1, 1, 1), DIRICHLET)
    return Problem('heat_sine_16', n, DIRICHLET, HEAT, 1.0, (0.0, 0.0, 0.0), 'SDIRK2',
                   1e-3, 10, u0, precision='fp64', krylov='cg', precond='none')


def heat_modes(n: int = 128, seed: int = 2, nsteps: int = 50, dt: float = 5e-4,
               kappa: float = 1.0) -> Problem:
    """Heat problem with u0 = sum of 8 seeded sine modes (amplitudes N(0,1)/|k|^2)."""
    rng = np.random.default_rng(seed)
    u0, k, a = fourier_sine_modes(n, rng)
    return Problem(f'heat_modes_{n}', n, DIRICHLET, HEAT, kappa, (0.0, 0.0, 0.0), 'SDIRK3',
                   dt, nsteps, u0, precision='fp32', krylov='cg', precond='bj',
                   meta={'k': k, 'a': a, 'seed': seed})


def advdiff_bump(n: int = 256, seed: int = 3, nsteps: int = 20, dt: float = 2e-3,
                 nu: float = 1e-2, b=(1.0, 0.5, 0.25)) -> Problem:
    """Periodic upwind advection-diffusion with a seeded Gaussian bump."""
    rng = np.random.default_rng(seed)
    c = 0.5 + rng.uniform(-0.1, 0.1, 3)
    u0 = gaussian_bump(n, c, 100.0, PERIODIC)
    return Problem(f'advdiff_bump_{n}', n, PERIODIC, ADVDIFF, nu, tuple(b), 'SDIRK3',
                   dt, nsteps, u0, precision='fp16', krylov='gmres', precond='bj',
                   meta={'center': c, 'seed': seed})


def heat_allen_cahn(n: int = 128, seed: int = 2, nsteps: int = 20, dt: float = 5e-4,
                    rho: float = 50.0) -> Problem:
    """heat_modes' state and solver with the Allen-Cahn reaction rho (u - u^3), amplitudes
    scaled so that the cubic term matters (max |u0| = 1)."""
    p = heat_modes(n, seed, nsteps, dt)
    p.u0 = p.u0 / np.max(np.abs(p.u0))
    p.name = f'heat_allen_cahn_{n}'
    p.reaction = (rho, 0.0, -rho)
    p.meta['rho'] = rho
    return p


def advdiff_fisher(n: int = 256, seed: int = 3, nsteps: int = 20, dt: float = 2e-3,
                   rho: float = 20.0) -> Problem:
    """advdiff_bump's state and solver with the Fisher-KPP reaction rho u (1 - u)."""
    p = advdiff_bump(n, seed, nsteps, dt)
    p.name = f'advdiff_fisher_{n}'
    p.reaction = (rho, -rho, 0.0)
    p.meta['rho'] = rho
    return p


def uniform_state(n: int, value: float) -> np.ndarray:
    """A spatially constant field, shape (n, n, n)."""
    return np.full((n, n, n), float(value))


def paper_heat(n: int = 128, tableau: str = 'MID1', dt: float = 1.0 / 80, t_end: float = 0.1,
               precision: str = 'fp32') -> Problem:
    """The paper's heat test (Section "Heat equation"): du/dt = Lap u + g on the unit cube,
    zero Dirichlet, g = sin(pi x) sin(pi y) sin(pi z) at the nodes, u(0) = 0, to t_end."""
    g = sine_mode((n, n, n), (1, 1, 1), DIRICHLET)
    return Problem(f'paper_heat_{n}', n, DIRICHLET, HEAT, 1.0, (0.0, 0.0, 0.0), tableau, dt,
                   int(round(t_end / dt)), np.zeros((n, n, n)), precision=precision,
                   krylov='cg', precond='bj', forcing=g)


def paper_advection(n: int = 128, tableau: str = 'MID1', dt: float = 1.0 / 80,
                    t_end: float = 0.1, precision: str = 'fp32') -> Problem:
    """The paper's advection test (Section "Advection equation"): du/dt + div(beta u) = 0,
    beta = (1, 1, 1), periodic, u(0) = exp(-100 |x - 1/2|^2) at the nodes, to t_end;
    central differences."""
    u0 = gaussian_bump(n, (0.5, 0.5, 0.5), 100.0, PERIODIC)
    return Problem(f'paper_advection_{n}', n, PERIODIC, CENTRAL, 0.0, (1.0, 1.0, 1.0), tableau,
                   dt, int(round(t_end / dt)), u0, precision=precision, krylov='gmres',
                   precond='bj')


def paper_heat_exact(n: int, t: float) -> np.ndarray:
    """The continuum solution of the paper's heat test at time t, at the nodes: with u(0) = 0
    and g the lowest Dirichlet sine mode (Laplacian eigenvalue -3 pi^2) the solution stays
    along g, u(t) = (1 - exp(-3 pi^2 t)) / (3 pi^2) g."""
    c = 3.0 * np.pi ** 2
    return (1.0 - np.exp(-c * t)) / c * sine_mode((n, n, n), (1, 1, 1), DIRICHLET)


def translated_gaussian(n: int, shift, width: float = 100.0) -> np.ndarray:
    """exp(-width |x - 1/2 - shift|^2) at the periodic nodes with the nearest periodic image:
    the exact solution of the constant-velocity advection test at time t (shift = beta t)."""
    x = axis_nodes(n, PERIODIC)
    parts = []
    for d in range(3):
        r = x - 0.5 - shift[d]
        r = r - np.round(r)
        parts.append(np.exp(-width * r ** 2))
    gx, gy, gz = parts
    return gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


def random_field(n: int, seed: int) -> np.ndarray:
    """Standard-normal field of shape (n, n, n) (a generic, non-modal test input)."""
    return np.random.default_rng(seed).standard_normal((n, n, n))


def heat_batch(count: int = 64, seed: int = 4, nmin: int = 16, nmax: int = 96,
               nsteps: int = 20, dt: float = 5e-4):
    """Batch of independent heat problems of uneven sizes.

    Draw order: for each problem p in turn: n_p = rng.integers(nmin, nmax+1),
    kappa_p = 10**rng.uniform(-1, 1), then the 8-mode u0 draws.
    """
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        kappa = float(10.0 ** rng.uniform(-1.0, 1.0))
        u0, k, a = fourier_sine_modes(n, rng)
        out.append(Problem(f'batch{p}_heat_{n}', n, DIRICHLET, HEAT, kappa, (0.0, 0.0, 0.0),
                           'SDIRK3', dt, nsteps, u0, precision='fp32', krylov='cg',
                           precond='bj', meta={'k': k, 'a': a}))
    return out


@dataclasses.dataclass
class Request:
    """One serving request: arrival time (s) and the job."""
    rid: int
    arrival: float
    problem: Problem


def request_stream(count: int = 512, rate: float = 50.0, seed: int = 5,
                   nmin: int = 32, nmax: int = 192, smin: int = 10, smax: int = 100,
                   materialize_u0: bool = True):
    """Poisson-arrival request mix.

    Draw order per request: inter-arrival rng.exponential(1/rate); kind (heat or
    advection-diffusion, probability 1/2 each); n ~ U{nmin..nmax}; steps ~ U{smin..smax};
    precision uniform over fp64/fp32/fp16; then the u0 draws of that kind.
    Heat: kappa = 1, dt = 5e-4, zero Dirichlet, 8 sine modes, CG.
    Advection-diffusion: nu = 1e-2, b = (1, 0.5, 0.25), dt = 2e-3, periodic,
    Gaussian bump, GMRES(30).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    precs = ('fp64', 'fp32', 'fp16')
    reqs = []
    for r in range(count):
        t += float(rng.exponential(1.0 / rate))
        kind = HEAT if rng.random() < 0.5 else ADVDIFF
        n = int(rng.integers(nmin, nmax + 1))
        steps = int(rng.integers(smin, smax + 1))
        prec = precs[int(rng.integers(0, 3))]
        if kind == HEAT:
            kk = rng.integers(1, 9, (8, 3))
            aa = rng.standard_normal(8) / (kk ** 2).sum(axis=1)
            u0 = None
            if materialize_u0:
                u0 = np.zeros((n, n, n))
                for m in range(8):
                    u0 += aa[m] * sine_mode((n, n, n), kk[m], DIRICHLET)
            p = Problem(f'req{r}_heat_{n}', n, DIRICHLET, HEAT, 1.0, (0.0, 0.0, 0.0), 'SDIRK3',
                        5e-4, steps, u0, precision=prec, krylov='cg', precond='bj',
                        meta={'k': kk, 'a': aa})
        else:
            c = 0.5 + rng.uniform(-0.1, 0.1, 3)
            u0 = gaussian_bump(n, c, 100.0, PERIODIC) if materialize_u0 else None
            p = Problem(f'req{r}_adv_{n}', n, PERIODIC, ADVDIFF, 1e-2, (1.0, 0.5, 0.25), 'SDIRK3',
                        2e-3, steps, u0, precision=prec, krylov='gmres', precond='bj',
                        meta={'center': c})
        reqs.append(Request(r, t, p))
    return reqs


def initial_field(p: Problem) -> np.ndarray:
    """Rebuild a request's initial field from its recorded draws (requests made with
    materialize_u0=False keep only the seeds' outcomes in p.meta)."""
    if p.u0 is not None:
        return p.u0
    if p.kind == HEAT:
        u = np.zeros((p.n, p.n, p.n))
        for m in range(len(p.meta['a'])):
            u += p.meta['a'][m] * sine_mode((p.n, p.n, p.n), p.meta['k'][m], DIRICHLET)
        return u
    return gaussian_bump(p.n, p.meta['center'], 100.0, PERIODIC)
