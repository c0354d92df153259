"""Pins of the oracle's Pade [13/13] scaling-and-squaring exponential
against closed forms and an independent library routine."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import expm_pade13, pade13_coefficients


def test_pade_coefficients_are_the_pade_approximant():
    # [13/13] Pade of e^x: p(x)/p(-x) = e^x + O(x^27); check at several x.
    b = pade13_coefficients()
    assert b[13] == 1.0
    assert all(float(c).is_integer() for c in b)
    for x in (0.05, 0.3, 1.0, -0.7):
        p = sum(c * x**j for j, c in enumerate(b))
        q = sum(c * (-x)**j for j, c in enumerate(b))
        assert abs(p / q - math.exp(x)) <= 4e-16 * math.exp(x)


@pytest.mark.parametrize("lam", [[0.0, -1.0, 2.0], [-300.0, -1e-3, 5.0, 40.0]])
def test_diagonal_closed_form(lam):
    lam = np.array(lam)
    for t in (0.0, 0.1, 1.0, 3.0):
        E = expm_pade13(np.diag(lam * t))
        np.testing.assert_allclose(np.diag(E), np.exp(lam * t), rtol=1e-13, atol=1e-300)
        assert np.all(E - np.diag(np.diag(E)) == 0.0)


@pytest.mark.parametrize("t", [0.0, math.pi / 4, 3 * math.pi / 4, 10.0, 123.4])
def test_rotation_closed_form(t):
    R = expm_pade13(np.array([[0.0, 1.0], [-1.0, 0.0]]) * t)
    exact = np.array([[math.cos(t), math.sin(t)], [-math.sin(t), math.cos(t)]])
    np.testing.assert_allclose(R, exact, atol=1e-13 * max(1.0, t))


def test_nilpotent_jordan_polynomial():
    n = 7
    J = np.diag(np.ones(n - 1), 1)
    for t in (0.5, 2.0, 7.0):
        E = expm_pade13(J * t)
        exact = np.zeros((n, n))
        for i in range(n):
            for j in range(i, n):
                exact[i, j] = t ** (j - i) / math.factorial(j - i)
        np.testing.assert_allclose(E, exact, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("scale", [1e-3, 0.5, 5.0, 60.0, 900.0])
def test_against_library_expm(scale):
    rng = np.random.default_rng(3)
    for k in (1, 4, 17, 40):
        M = rng.normal(size=(k, k))
        M = -M @ M.T * scale / k    # symmetric negative semidefinite: stable, like heat
        np.testing.assert_allclose(expm_pade13(M), scipy.linalg.expm(M), rtol=1e-12,
                                   atol=1e-14 * np.abs(scipy.linalg.expm(M)).max())
        G = rng.normal(size=(k, k)) * scale / k ** 0.5 * 0.05
        ref = scipy.linalg.expm(G)
        np.testing.assert_allclose(expm_pade13(G), ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())


def test_empty_and_zero():
    assert expm_pade13(np.zeros((0, 0))).shape == (0, 0)
    np.testing.assert_allclose(expm_pade13(np.zeros((3, 3))), np.eye(3), rtol=0, atol=4e-16)
