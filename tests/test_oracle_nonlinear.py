"""Pins of oracle/nonlinear.py: the DIRK with Newton stage solves for du/dt = K u + g + R(u)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import dirk as D
from oracle import nonlinear as NL
from oracle import operators as O
from oracle import tableaus as T


def _field(shape, seed, scale=0.5):
    return scale * np.random.default_rng(seed).standard_normal(int(np.prod(shape)))


@pytest.mark.parametrize("kind,bc,shape", [(0, O.DIRICHLET, (6, 5, 7)), (1, O.PERIODIC, (5, 6, 4))])
def test_zero_reaction_is_the_linear_oracle(kind, bc, shape):
    K = O.operator(shape, bc, kind, 0.7, (0.5, -0.3, 0.2))
    u0 = _field(shape, 11)
    lin = D.integrate(K, u0, 0.01, 5, T.sdirk3(), 'splu')
    got = NL.integrate(K, u0, 0.01, 5, T.sdirk3(), (0.0, 0.0, 0.0))
    assert D.relative_l2(got, lin) < 1e-13


@pytest.mark.parametrize("kind,bc,shape", [(0, O.DIRICHLET, (7, 6, 5)), (1, O.PERIODIC, (6, 5, 6))])
def test_newton_solvers_agree(kind, bc, shape):
    K = O.operator(shape, bc, kind, 0.5, (0.9, 0.4, -0.3))
    u0 = _field(shape, 14)
    r = (2.0, -1.0, -3.0)
    a = NL.integrate(K, u0, 0.01, 4, T.sdirk3(), r, method='splu')
    b = NL.integrate(K, u0, 0.01, 4, T.sdirk3(), r, method='gmres')
    assert D.relative_l2(b, a) < 1e-13


def _order_errors(tab, exact, r, y0, t_end, taus):
    return [abs(NL.scalar_integrate(y0, tau, int(round(t_end / tau)), tab, r) - exact)
            for tau in taus]


@pytest.mark.parametrize("name,order", [("SDIRK2", 2), ("SDIRK3", 3), ("4S3PA", 3), ("4S3PC", 3)])
def test_scalar_bernoulli_converges_at_the_tableau_order(name, order):
    # logistic growth y' = y - y^2 from 0.1 to t = 1
    r = (1.0, -1.0, 0.0)
    exact = NL.bernoulli_exact(0.1, 1.0, -1.0, 1.0)
    errs = _order_errors(T.by_name(name), exact, r, 0.1, 1.0, [0.1, 0.05, 0.025])
    for a, b in zip(errs, errs[1:]):
        assert 2 ** order * 0.8 < a / b < 2 ** order * 1.25, (name, errs)


def test_scalar_cubic_converges_at_third_order():
    # y' = 2 y - 3 y^3 (the Allen-Cahn reaction) from 0.2 to t = 1
    r = (2.0, 0.0, -3.0)
    exact = NL.cubic_exact(0.2, 2.0, -3.0, 1.0)
    errs = _order_errors(T.sdirk3(), exact, r, 0.2, 1.0, [0.025, 0.0125, 0.00625])
    for a, b in zip(errs, errs[1:]):
        assert 6.4 < a / b < 10.0, errs
    assert errs[-1] < 1e-8


@pytest.mark.parametrize("g", [None, 0.4])
def test_constant_periodic_state_follows_the_scalar_equation(g):
    # K maps constants to zero on a periodic grid, so every point follows y' = g + R(y)
    shape = (6, 5, 4)
    K = O.operator(shape, O.PERIODIC, 1, 0.3, (0.8, -0.6, 0.4))
    r = (2.0, -1.5, -0.7)
    n = int(np.prod(shape))
    u0 = np.full(n, 0.3)
    gv = None if g is None else np.full(n, g)
    got = NL.integrate(K, u0, 0.02, 6, T.sdirk3(), r, g=gv)
    want = NL.scalar_integrate(0.3, 0.02, 6, T.sdirk3(), r, g=0.0 if g is None else g)
    assert np.max(np.abs(got - want)) < 1e-13 * abs(want)


def test_stage_residuals_vanish_and_newton_is_quadratic():
    shape = (6, 5, 7)
    K = O.heat_operator(shape, O.DIRICHLET, 0.4)
    r = (1.0, -2.0, -3.0)
    u0 = _field(shape, 12)
    res = NL.stage_residuals(K, u0, 0.01, T.sdirk3(), r)
    assert len(res) == 3 and max(res) < 1e-14
    its = []
    NL.integrate(K, u0, 0.01, 4, T.sdirk3(), r, stats=its)
    # quadratic convergence: a handful of iterations to 1e-15 (a wrong Jacobian needs many)
    assert len(its) == 12 and max(its) <= 5, its


def test_small_grid_converges_to_the_method_of_lines_solution():
    shape = (4, 3, 5)
    K = O.heat_operator(shape, O.DIRICHLET, 0.05)
    r = (1.0, 0.5, -2.0)
    u0 = _field(shape, 13, 0.8)
    f = NL.rhs_function(K, None, r)
    Kd = K.toarray()

    def jac(t, y):
        return Kd + np.diag(NL.reaction_derivative(y, r))

    ref = solve_ivp(lambda t, y: f(y), (0.0, 0.4), u0, method='Radau', jac=jac,
                    rtol=1e-13, atol=1e-15).y[:, -1]
    # (the ratio approaches 8 from below as the stiff components resolve)
    errs = [np.linalg.norm(NL.integrate(K, u0, tau, int(round(0.4 / tau)), T.sdirk3(), r) - ref)
            for tau in (0.01, 0.005, 0.0025)]
    for a, b in zip(errs, errs[1:]):
        assert 6.4 < a / b < 10.0, errs
