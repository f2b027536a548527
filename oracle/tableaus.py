"""Butcher tableaus with the high/low-precision split A = A^(h) + A^(eps) (oracle, test infrastructure).

The split follows Section "Method stability in the context of mixed precision":
entries carrying the (eps) superscript belong to A^(eps) (stages solved or
evaluated in low precision); the others, and b, are high precision.  c is the
row sum of the full A (stated under Table ButchertabA).

Tableaus:
  * MID(p): implicit midpoint with p explicit corrector steps (Figure
    fig_Aq_rat; general form in Appendix A): A^(eps)_{11} = 1/2,
    A^(h)_{i,i-1} = 1/2 for i = 2..p+1, b = e_{p+1}.  MID(0) is the plain rule.
  * 4s3pA (Table ButchertabA), 4s3pC (Table ButchertabC): digits as printed.
  * 4s3pB (Table ButchertabB): digits as printed except a42^(eps).  The printed
    a42^(eps) repeats 4s3pA's a31^(eps); with it the method is not even second
    order.  Reading used here: a42^(eps) = -3/2 - a42, so the full matrix is the
    L-stable base method with last row equal to b (stiffly accurate) and the
    perturbation condition b^T A^(eps) e = 0 holds.
  * SDIRK2: Alexander's two-stage L-stable SDIRK, gamma = 1 - 1/sqrt(2).
  * SDIRK3: Alexander's three-stage L-stable SDIRK of order 3, gamma the root in
    (1/6, 1/2) of x^3 - 3x^2 + 3x/2 - 1/6.
    For the two SDIRKs (not in the paper) the mixed reading puts the diagonal
    in A^(eps) and the strictly lower part in A^(h), mirroring the mixed midpoint
    rule where the implicit stage is the low-precision one.

R(z) = 1 + z b^T (I - z A)^{-1} e is the stability function of Section
"Method stability in the context of mixed precision".

Pins (tests/test_oracle_tableaus.py): order conditions up to 3, R(z) of MID(p)
equals (2+z)/(2-z) (Appendix A), A-stability on the imaginary axis, R(-inf),
the printed digits (tests/golden/paper_tableaus.txt), the cubic for gamma.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class Tableau:
    name: str
    A_hi: np.ndarray
    A_lo: np.ndarray
    b: np.ndarray

    @property
    def A(self) -> np.ndarray:
        return self.A_hi + self.A_lo

    @property
    def c(self) -> np.ndarray:
        return self.A.sum(axis=1)

    @property
    def s(self) -> int:
        return len(self.b)


def mid(p: int) -> Tableau:
    """Implicit midpoint rule with p corrector steps (Figure fig_Aq_rat, Appendix A)."""
    s = p + 1
    A_hi = np.zeros((s, s))
    A_lo = np.zeros((s, s))
    A_lo[0, 0] = 0.5
    for i in range(1, s):
        A_hi[i, i - 1] = 0.5
    b = np.zeros(s)
    b[-1] = 1.0
    return Tableau(f'MID{p}', A_hi, A_lo, b)


def s4p3a() -> Tableau:
    """4s3pA, Table ButchertabA, as printed."""
    A_hi = np.zeros((4, 4))
    A_lo = np.zeros((4, 4))
    A_lo[0, 0] = 0.788675134594813
    A_hi[1, 0] = 0.211324865405187
    A_lo[2, 0] = 0.051944240459852
    A_hi[2, 0] = 0.709495523817170
    A_hi[2, 1] = -0.86531425061942
    A_lo[2, 2] = 0.788675134594813
    A_hi[3, 0] = 0.705123240545107
    A_hi[3, 1] = 0.943370088535775
    A_hi[3, 2] = -0.859818194486069
    b = np.array([0.0, 0.5, 0.0, 0.5])
    return Tableau('4s3pA', A_hi, A_lo, b)


def s4p3b(printed_a42_eps: bool = False) -> Tableau:
    """4s3pB, Table ButchertabB; a42^(eps) corrected unless printed_a42_eps is set."""
    A_hi = np.zeros((4, 4))
    A_lo = np.zeros((4, 4))
    for i in range(4):
        A_lo[i, i] = 0.5
    A_lo[1, 0] = -2.376349376129689
    A_hi[1, 0] = 2.543016042796356
    A_lo[2, 0] = -2.951484396921318
    A_hi[2, 0] = 2.451484396921318
    A_lo[2, 1] = 0.475891038758779
    A_hi[2, 1] = 0.024108961241221
    A_lo[3, 0] = -0.573861819468268
    A_hi[3, 0] = 2.073861819468268
    A_hi[3, 1] = 2.367724727682735
    A_lo[3, 1] = 0.051944240459852 if printed_a42_eps else -1.5 - 2.367724727682735
    A_lo[3, 2] = -1.211868223075524
    A_hi[3, 2] = 1.711868223075524
    b = np.array([1.5, -1.5, 0.5, 0.5])
    return Tableau('4s3pB' + ('-printed' if printed_a42_eps else ''), A_hi, A_lo, b)


def s4p3c() -> Tableau:
    """4s3pC, Table ButchertabC, as printed."""
    A_hi = np.zeros((4, 4))
    A_lo = np.zeros((4, 4))
    A_lo[0, 0] = 0.511243008730995
    A_lo[1, 0] = -1.999347282862640
    A_hi[1, 0] = -0.050470366527530
    A_lo[1, 1] = 1.957161067302390
    A_lo[2, 0] = 0.443312893511937
    A_hi[2, 0] = 0.368613367355336
    A_lo[2, 1] = -0.573131033672219
    A_hi[2, 1] = 0.273504374252976
    A_lo[2, 2] = 0.128283796414019
    A_lo[3, 0] = -2.0
    A_hi[3, 0] = 1.803794668975043
    A_lo[3, 1] = -0.160330320741428
    A_hi[3, 1] = 0.097485042980759
    A_lo[3, 2] = 0.579597314161362
    A_hi[3, 2] = -1.895660952342050
    A_lo[3, 3] = 1.484688928981990
    b = np.array([0.002837446974069, 0.336264433650450, 0.806376720267787,
                  -0.145478600892306])
    return Tableau('4s3pC', A_hi, A_lo, b)


def sdirk2() -> Tableau:
    """Two-stage L-stable SDIRK of order 2, gamma = 1 - 1/sqrt(2)."""
    g = 1.0 - 1.0 / np.sqrt(2.0)
    A_lo = np.diag([g, g])
    A_hi = np.array([[0.0, 0.0], [1.0 - g, 0.0]])
    return Tableau('SDIRK2', A_hi, A_lo, np.array([1.0 - g, g]))


def sdirk3_gamma() -> float:
    """Root in (1/6, 1/2) of x^3 - 3x^2 + 3x/2 - 1/6."""
    r = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    r = np.real(r[np.abs(np.imag(r)) < 1e-12])
    g = float(r[(r > 1.0 / 6.0) & (r < 0.5)][0])
    # one Newton step in float64 to remove root-finder rounding
    f = g ** 3 - 3 * g ** 2 + 1.5 * g - 1.0 / 6.0
    df = 3 * g ** 2 - 6 * g + 1.5
    return g - f / df


def sdirk3() -> Tableau:
    """Three-stage L-stable, stiffly accurate SDIRK of order 3."""
    g = sdirk3_gamma()
    b1 = -1.5 * g * g + 4.0 * g - 0.25
    b2 = 1.5 * g * g - 5.0 * g + 1.25
    A_lo = np.diag([g, g, g])
    A_hi = np.array([[0.0, 0.0, 0.0], [(1.0 - g) / 2.0, 0.0, 0.0], [b1, b2, 0.0]])
    return Tableau('SDIRK3', A_hi, A_lo, np.array([b1, b2, g]))


def by_name(name: str) -> Tableau:
    name = name.upper()
    if name.startswith('MID'):
        return mid(int(name[3:] or 0))
    table = {'SDIRK2': sdirk2, 'SDIRK3': sdirk3, '4S3PA': s4p3a, '4S3PB': s4p3b, '4S3PC': s4p3c}
    return table[name]()


def stability_function(tab: Tableau, z):
    """R(z) = 1 + z b^T (I - z A)^{-1} e, evaluated for an array of complex z.

    (I - zA) X = e is lower triangular for a DIRK and is solved by forward
    substitution, one stage at a time, elementwise in z.
    """
    z = np.asarray(z, dtype=np.complex128)
    A, b = tab.A, tab.b
    X = []
    for i in range(tab.s):
        acc = np.ones_like(z)
        for j in range(i):
            acc = acc + z * A[i, j] * X[j]
        X.append(acc / (1.0 - z * A[i, i]))
    R = np.ones_like(z)
    for i in range(tab.s):
        R = R + z * b[i] * X[i]
    return R


def stability_function_dense(tab: Tableau, z: complex) -> complex:
    """The same R(z) through a dense solve of (I - zA) x = e (for a single z)."""
    s = tab.s
    x = np.linalg.solve(np.eye(s) - z * tab.A, np.ones(s))
    return 1.0 + z * tab.b @ x
