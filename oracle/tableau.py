"""Butcher tableaux of the fully implicit RK families used in Sec. 5 (Gauss, RadauIIA,
LobattoIIIC), in closed form.

TEST INFRASTRUCTURE ONLY (oracle).

Sec. 2 (eq. "general RK") defines an r-stage method by its tableau (A, b, c) with the
consistency conditions sum(b) = 1 and A 1 = c.  Sec. 5 names the three families and
their orders 2r (Gauss), 2r-1 (RadauIIA) and 2r-2 (LobattoIIIC); the coefficients are
the standard textbook ones, typed here from their closed forms.

Pinned by tests/test_oracle_tableau.py against: the consistency conditions; the
simplifying order conditions B(p) and C(q) at the stated orders; the stability
function equal to the Pade approximant of exp(z) of the right degree (computed from
the Pade formula, not from the tableau); R(inf) = 0 for the L-stable families.
"""
from __future__ import annotations

import numpy as np

FAMILIES = ("radauIIA", "gauss", "lobattoIIIC")


def tableau(family: str, r: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Return (A, b, c) as float64 arrays."""
    s6, s3, s15 = np.sqrt(6.0), np.sqrt(3.0), np.sqrt(15.0)
    if family == "radauIIA":
        if r == 1:  # backward Euler
            A = [[1.0]]
            c = [1.0]
        elif r == 2:
            A = [[5 / 12, -1 / 12], [3 / 4, 1 / 4]]
            c = [1 / 3, 1.0]
        elif r == 3:
            A = [
                [(88 - 7 * s6) / 360, (296 - 169 * s6) / 1800, (-2 + 3 * s6) / 225],
                [(296 + 169 * s6) / 1800, (88 + 7 * s6) / 360, (-2 - 3 * s6) / 225],
                [(16 - s6) / 36, (16 + s6) / 36, 1 / 9],
            ]
            c = [(4 - s6) / 10, (4 + s6) / 10, 1.0]
        else:
            raise ValueError(r)
        A = np.array(A)
        b = A[-1].copy()  # stiffly accurate
    elif family == "gauss":
        if r == 1:  # implicit midpoint
            A = [[0.5]]
            b = [1.0]
            c = [0.5]
        elif r == 2:
            A = [[1 / 4, 1 / 4 - s3 / 6], [1 / 4 + s3 / 6, 1 / 4]]
            b = [1 / 2, 1 / 2]
            c = [1 / 2 - s3 / 6, 1 / 2 + s3 / 6]
        elif r == 3:
            A = [
                [5 / 36, 2 / 9 - s15 / 15, 5 / 36 - s15 / 30],
                [5 / 36 + s15 / 24, 2 / 9, 5 / 36 - s15 / 24],
                [5 / 36 + s15 / 30, 2 / 9 + s15 / 15, 5 / 36],
            ]
            b = [5 / 18, 4 / 9, 5 / 18]
            c = [1 / 2 - s15 / 10, 1 / 2, 1 / 2 + s15 / 10]
        else:
            raise ValueError(r)
        A, b = np.array(A), np.array(b)
    elif family == "lobattoIIIC":
        if r == 2:
            A = [[1 / 2, -1 / 2], [1 / 2, 1 / 2]]
            b = [1 / 2, 1 / 2]
            c = [0.0, 1.0]
        elif r == 3:
            A = [[1 / 6, -1 / 3, 1 / 6], [1 / 6, 5 / 12, -1 / 12], [1 / 6, 2 / 3, 1 / 6]]
            b = [1 / 6, 2 / 3, 1 / 6]
            c = [0.0, 1 / 2, 1.0]
        else:
            raise ValueError(r)
        A, b = np.array(A), np.array(b)
    else:
        raise ValueError(family)
    return np.array(A, dtype=np.float64), np.array(b, dtype=np.float64), np.array(c, dtype=np.float64)


def stability_function(A: np.ndarray, b: np.ndarray, z: complex) -> complex:
    """R(z) = 1 + z b^T (I - z A)^{-1} 1: the map u^{n+1} = R(lambda dt) u^n of the
    Dahlquist test problem (Sec. 2)."""
    r = len(b)
    return 1.0 + z * (b @ np.linalg.solve(np.eye(r) - z * A, np.ones(r)))
