"""Pins of the oracle's smoothing functions against high-precision evaluation.

The reference values are the paper's four formulas for s_k (section
"High-order regularization of kernels on the surface") evaluated with
mpmath at 80-200 significant digits, where the cancellation at small rho
is harmless.  This checks both branches of the oracle (Taylor series for
small rho, direct formula above) and its derivative functions.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O

P = {1: 1, 2: 3, 3: 3, 4: 5}


def s_hp(k, r):
    c = 2 / mp.sqrt(mp.pi)
    r = mp.mpf(r)
    E = mp.e ** (-r * r)
    ef = mp.erf(r)
    if k == 1:
        return ef - (c / 3) * r * (2 * r**2 - 5) * E
    if k == 2:
        return ef + (c / 3) * r * (2 * r**2 - 3) * E
    if k == 3:
        return ef - (c / 3) * r * (4 * r**4 - 14 * r**2 + 3) * E
    return ef - (c / 9) * r * (8 * r**6 - 36 * r**4 + 6 * r**2 + 9) * E


def F_hp(k, r):
    with mp.workdps(200):
        if r == 0:
            r = mp.mpf("1e-40")  # F_k is even and entire: F(1e-40) = F(0) to 1e-80
        return s_hp(k, r) / mp.mpf(r) ** P[k]


RHOS = [0.0, 1e-12, 1e-6, 1e-3, 0.01, 0.05, 0.1, 0.25, 0.4, 0.55, 0.599, 0.6, 0.601,
        0.75, 0.99, 1.0, 1.01, 1.3, 2.0, 3.0, 4.5, 5.3, 6.0, 7.1, 9.0, 15.0]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_F_matches_high_precision(k):
    got = O.F(k, RHOS)
    ref = np.array([float(F_hp(k, r)) for r in RHOS])
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() < 2e-15, (k, RHOS[int(rel.argmax())], rel.max())


def test_F_zero_limits(golden):
    c = 1.0 / math.sqrt(math.pi)
    ref = {1: 16 * c / 3, 2: 8 * c / 3, 3: 32 * c / 3, 4: 128 * c / 15}
    for k in range(1, 5):
        assert abs(O.F(k, 0.0)[0] - ref[k]) < 1e-15 * ref[k]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_F_far_field_is_inverse_power(k):
    # s_k -> 1 so F_k -> rho^-p; |1 - s_k| < 1e-20 beyond rho = 7.5
    for r in [7.5, 10.0, 30.0]:
        assert abs(O.F(k, r)[0] * r ** P[k] - 1.0) < 1e-15


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_G_is_minus_dF_over_rho(k):
    rhos = [1e-4, 0.05, 0.3, 0.7, 0.99, 1.0, 1.01, 1.7, 3.0, 5.0, 8.0]
    got = O.G(k, rhos)
    with mp.workdps(80):
        ref = np.array([float(-mp.diff(lambda t: F_hp(k, t), mp.mpf(r)) / r) for r in rhos])
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() < 3e-15, (k, rel.max())


def test_smoothing_structure_identities():
    # s3 = s1 - rho s1' and s4 = s3 - rho s3'/3: the relations that make the
    # Stokeslet and stresslet smoothings consistent with the Laplace ones.
    with mp.workdps(60):
        for r in [0.3, 1.0, 2.2]:
            r = mp.mpf(r)
            d1 = mp.diff(lambda t: s_hp(1, t), r)
            d3 = mp.diff(lambda t: s_hp(3, t), r)
            assert abs(s_hp(3, r) - (s_hp(1, r) - r * d1)) < mp.mpf("1e-40")
            assert abs(s_hp(4, r) - (s_hp(3, r) - r * d3 / 3)) < mp.mpf("1e-40")


def test_s_is_paper_formula():
    # the oracle's direct formula reproduces the printed s_k; s_k(0) = 0 and
    # s_k -> 1 in the far field
    rr = np.linspace(0.0, 8.0, 81)
    for k in range(1, 5):
        v = O.s(k, rr)
        ref = np.array([float(s_hp(k, r)) for r in rr])
        assert np.max(np.abs(v - ref)) < 1e-15
        assert v[0] == 0.0 and abs(v[-1] - 1.0) < 1e-16
