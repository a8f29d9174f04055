"""Pins for oracle/tableau.py: order conditions and Pade stability functions."""
from math import factorial

import numpy as np
import pytest

from oracle.tableau import stability_function, tableau

# (family, r) -> (quadrature order p, stage order q, Pade numerator degree, R(inf))
EXPECT = {
    ("radauIIA", 1): (1, 1, 0, 0.0),
    ("radauIIA", 2): (3, 2, 1, 0.0),
    ("radauIIA", 3): (5, 3, 2, 0.0),
    ("gauss", 1): (2, 1, 1, -1.0),
    ("gauss", 2): (4, 2, 2, 1.0),
    ("gauss", 3): (6, 3, 3, -1.0),
    ("lobattoIIIC", 2): (2, 1, 0, 0.0),
    ("lobattoIIIC", 3): (4, 2, 1, 0.0),
}


def pade(k, j, z):
    """(k, j) Pade approximant of exp(z) from its closed-form coefficients."""
    num = sum(factorial(k + j - i) * factorial(k) / (factorial(k + j) * factorial(i) * factorial(k - i)) * z**i for i in range(k + 1))
    den = sum(factorial(k + j - i) * factorial(j) / (factorial(k + j) * factorial(i) * factorial(j - i)) * (-z) ** i for i in range(j + 1))
    return num / den


@pytest.mark.parametrize("key", sorted(EXPECT))
def test_consistency(key):
    A, b, c = tableau(*key)
    assert abs(b.sum() - 1) < 1e-15
    assert np.allclose(A.sum(axis=1), c, atol=1e-15)


@pytest.mark.parametrize("key", sorted(EXPECT))
def test_quadrature_and_stage_order(key):
    A, b, c = tableau(*key)
    p, q, _, _ = EXPECT[key]
    for k in range(1, p + 1):
        assert abs(b @ c ** (k - 1) - 1 / k) < 1e-14, k
    assert abs(b @ c**p - 1 / (p + 1)) > 1e-8  # order is exactly p
    for k in range(1, q + 1):
        assert np.allclose(A @ c ** (k - 1), c**k / k, atol=1e-14), k
    assert not np.allclose(A @ c**q, c ** (q + 1) / (q + 1), atol=1e-10)


@pytest.mark.parametrize("key", sorted(EXPECT))
def test_stability_function_is_pade(key):
    A, b, c = tableau(*key)
    r = len(b)
    _, _, knum, rinf = EXPECT[key]
    for z in (-0.7, 0.3 + 0.4j, -3.0 + 2.0j, -25.0):
        assert abs(stability_function(A, b, z) - pade(knum, r, z)) < 1e-12 * max(1, abs(pade(knum, r, z)))
    assert abs(stability_function(A, b, -1e9) - rinf) < 1e-6
