"""Pins of oracle/tableaus.py: order conditions, stability functions, printed digits."""
import os

import numpy as np
import pytest

from oracle import tableaus as T

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


def order_residuals(tab):
    A, b, c = tab.A, tab.b, tab.c
    e = np.ones(tab.s)
    return {
        1: [b @ e - 1.0],
        2: [b @ c - 0.5],
        3: [b @ c ** 2 - 1.0 / 3.0, b @ A @ c - 1.0 / 6.0],
    }


def order_of(tab, tol=1e-13):
    r = order_residuals(tab)
    p = 0
    for q in (1, 2, 3):
        if max(abs(x) for x in r[q]) < tol:
            p = q
        else:
            break
    return p


@pytest.mark.parametrize("name,order", [("SDIRK2", 2), ("SDIRK3", 3), ("4s3pA", 3),
                                        ("4s3pB", 3), ("4s3pC", 3), ("MID0", 2),
                                        ("MID1", 2), ("MID4", 2)])
def test_order_conditions(name, order):
    assert order_of(T.by_name(name)) == order


def test_printed_4s3pB_is_not_second_order_and_fix_restores_structure():
    printed = T.s4p3b(printed_a42_eps=True)
    assert abs(order_residuals(printed)[2][0]) > 1.0     # printed digits break order 2
    fixed = T.s4p3b()
    # the fixed full matrix is the L-stable base method, stiffly accurate (last row = b)
    base = np.array([[0.5, 0, 0, 0], [1 / 6, 0.5, 0, 0], [-0.5, 0.5, 0.5, 0], [1.5, -1.5, 0.5, 0.5]])
    np.testing.assert_allclose(fixed.A, base, atol=2e-15)
    np.testing.assert_allclose(fixed.A[-1], fixed.b, atol=2e-15)
    # perturbation condition b^T A^(eps) e = 0
    assert abs(fixed.b @ fixed.A_lo @ np.ones(4)) < 1e-13


def test_4s3pA_low_precision_part_is_invisible_to_b():
    tab = T.s4p3a()
    assert np.abs(tab.b @ tab.A_lo).max() < 1e-15


def test_c_row_sums_and_diagonals_match_the_printed_tables():
    # Table ButchertabA: a11 = a33 = 0.788675134594813 and a21 = 0.211324865405187 (so c1 and c2
    # are these, c3 the sum of the third row); Table ButchertabC: the diagonal as printed
    np.testing.assert_allclose(T.s4p3a().c, [0.788675134594813, 0.211324865405187,
                                             0.684800648252415, 0.788675134594813], atol=1e-14)
    np.testing.assert_allclose(np.diag(T.s4p3c().A), [0.511243008730995, 1.957161067302390,
                                                      0.128283796414019, 1.484688928981990])


@pytest.mark.parametrize("p", [0, 1, 2, 3, 7])
def test_midpoint_with_correctors_has_closed_form_R(p):
    # Appendix A: R(z) = (z + 2) / (2 - z) for any number of corrector steps.
    z = np.array([-0.5, -3.0, -40.0, 2j, -1 + 1j, 0.3 - 0.2j])
    R = T.stability_function(T.mid(p), z)
    exact = (z + 2) / (2 - z)
    # each corrector multiplies a rounding error by z/2 (the fixed-point iteration of
    # Section "The implicit midpoint method and explicit corrector steps"), so the
    # attainable accuracy is ~ eps * max(1, |z/2|)^p
    tol = 1e-14 * np.maximum(1.0, np.abs(z / 2)) ** p
    assert np.all(np.abs(R - exact) <= tol * np.abs(exact))


def test_corrector_rounding_amplification_follows_spectral_radius():
    # rho(z/2) > 1: the error grows with p; rho < 1: it stays at rounding level.
    z = np.array([-40.0])
    errs = [abs(T.stability_function(T.mid(p), z)[0] - (z[0] + 2) / (2 - z[0])) for p in range(2, 8)]
    assert errs[-1] > 1e3 * max(errs[0], 1e-17)
    z = np.array([-1.5])
    errs = [abs(T.stability_function(T.mid(p), z)[0] - (z[0] + 2) / (2 - z[0])) for p in range(2, 8)]
    assert max(errs) < 1e-15


@pytest.mark.parametrize("name", ["SDIRK2", "SDIRK3", "4s3pA", "4s3pB", "4s3pC", "MID2"])
def test_forward_substitution_equals_dense_solve(name):
    tab = T.by_name(name)
    for z in (-0.7, -12.0 + 3j, 0.2 + 1.5j):
        assert abs(T.stability_function(tab, np.array([z]))[0]
                   - T.stability_function_dense(tab, z)) < 1e-12 * max(1, abs(z))


@pytest.mark.parametrize("name", ["SDIRK2", "SDIRK3", "4s3pB", "4s3pC", "MID0", "MID3"])
def test_A_stable_on_imaginary_axis(name):
    tab = T.by_name(name)
    y = np.concatenate([-np.logspace(-3, 4, 400), np.logspace(-3, 4, 400)])
    R = T.stability_function(tab, 1j * y)
    # MID(p) evaluated in floating point carries rounding amplified by |z/2|^p
    p = tab.s - 1 if name.startswith('MID') else 0
    tol = 1e-10 * np.maximum(1.0, np.abs(y / 2)) ** p
    assert np.all(np.abs(R) <= 1.0 + tol)


def test_4s3pA_is_not_A_stable():
    # Section "Method 4s3pA": not A-stable.  Search the left half-plane for |R| > 1.
    # R grows without bound along the negative real axis (stiff heat modes), which is
    # why the paper leaves 4s3pA out of the heat tests (Section "Heat equation").
    x = -np.logspace(-2, 6, 300)
    y = np.linspace(-50, 50, 201)
    Z = x[:, None] + 1j * y[None, :]
    assert np.abs(T.stability_function(T.s4p3a(), Z)).max() > 1.0


def test_L_stability_limits():
    big = np.array([-1e12])
    for name in ("SDIRK2", "SDIRK3", "4s3pB"):
        assert abs(T.stability_function(T.by_name(name), big)[0]) < 1e-9
    rc = abs(T.stability_function(T.s4p3c(), big)[0])
    assert 0.1 < rc < 1.0          # A-stable but not L-stable


def test_sdirk3_gamma_is_the_cubic_root():
    g = T.sdirk3_gamma()
    assert abs(g ** 3 - 3 * g ** 2 + 1.5 * g - 1 / 6) < 1e-15
    assert 1 / 6 < g < 0.5
    assert abs(g - 0.435866521508459) < 1e-14


def test_sdirk2_gamma():
    tab = T.sdirk2()
    assert tab.A[0, 0] == pytest.approx(1 - 1 / np.sqrt(2), abs=1e-16)
    np.testing.assert_allclose(tab.c, [tab.A[0, 0], 1.0], atol=1e-15)


def _read_golden():
    rows = []
    with open(os.path.join(GOLDEN, 'paper_tableaus.txt')) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith('#'):
                continue
            m, e, v = line.split()
            rows.append((m, e, float(v)))
    return rows


def test_oracle_tableaus_carry_the_printed_digits():
    tabs = {'4s3pA': T.s4p3a(), '4s3pB': T.s4p3b(), '4s3pC': T.s4p3c(),
            'MID1': T.mid(1), 'MID2': T.mid(2)}
    printed_b = T.s4p3b(printed_a42_eps=True)
    n = 0
    for m, e, v in _read_golden():
        tab = tabs[m]
        if e.startswith('b'):
            got = tab.b[int(e[1]) - 1]
        else:
            i, j = int(e[1]) - 1, int(e[2]) - 1
            if e.endswith('eps_printed'):
                got = printed_b.A_lo[i, j]
            elif e.endswith('eps'):
                got = tab.A_lo[i, j]
            else:
                got = tab.A_hi[i, j]
        assert got == v, (m, e)
        n += 1
    assert n > 60
