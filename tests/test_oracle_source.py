"""Pins of the oracle's relaxation source step (Sec. 4).

The source step integrates the purely algebraic right-hand side of
eq. (HSGN), a linear ODE in (hw, h sigma, hp, h p_b) with h fixed, by the
two-stage, second-order, L-stable SDIRK(2,2) method.  Pinned here by:
  * second-order agreement with the exact flow exp(tau M / h) (scipy expm):
    the one-step error shrinks by ~2^3 per halving of tau;
  * L-stability: a huge step damps every auxiliary variable to ~0;
  * the ODE's spectrum is purely imaginary, so the exact flow is neutral and
    the scheme must not amplify (spectral radius of the step <= 1);
  * h, hu, hv are untouched.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import oracle as O


def rhs_matrix(c2):
    """d/dt (hw, h sigma, hp, h p_b) = M (w, sigma, p, p_b) from eq. (HSGN)."""
    return np.array([
        [0.0, 0.0, 0.0, 1.0],            # d(hw)/dt = p_b
        [0.0, 0.0, 12.0, -6.0],          # d(h sigma)/dt = -6 p_b + 12 p
        [0.0, -c2, 0.0, 0.0],            # d(hp)/dt = -c^2 sigma
        [-6.0 * c2, 3.0 * c2, 0.0, 0.0],  # d(h p_b)/dt = -6 c^2 (w - sigma/2)
    ])


def step_matrix(h, c2, tau):
    """4x4 matrix of the oracle's one-step map, column by column."""
    S = np.zeros((4, 4))
    for c in range(4):
        q = np.zeros(7)
        q[0] = h
        q[3 + c] = 1.0
        S[:, c] = O.source_cell(q, c2, tau)[3:]
    return S


def test_second_order_against_exact_flow():
    rng = np.random.default_rng(21)
    for _ in range(5):
        h = rng.uniform(0.5, 2.0)
        c2 = rng.uniform(1.0, 100.0)
        Y = rng.normal(size=4)
        M = rhs_matrix(c2) / h
        errs = []
        omega = np.abs(np.linalg.eigvals(M)).max()
        for k in range(4):
            tau = 0.2 / omega / 2 ** k
            exact = expm(tau * M) @ Y
            q = np.concatenate([[h, 0.3, -0.2], Y])
            got = O.source_cell(q, c2, tau)
            assert got[0] == h and got[1] == 0.3 and got[2] == -0.2
            errs.append(np.abs(got[3:] - exact).max())
        ratios = np.array(errs[:-1]) / np.array(errs[1:])
        assert np.all(ratios > 6.0), (errs, ratios)
        assert errs[-1] < 1e-4 * np.abs(Y).max()


def test_spectrum_neutral_and_scheme_not_amplifying():
    h, c2 = 1.3, 40.0
    lam = np.linalg.eigvals(rhs_matrix(c2) / h)
    assert np.abs(lam.real).max() < 1e-9 * np.abs(lam).max()
    # eigenvalues +- i sqrt(6 (3 +- sqrt 7)) c / h
    expect = np.sort(np.sqrt(6 * (3 + np.array([-1, 1]) * np.sqrt(7))) * np.sqrt(c2) / h)
    got = np.sort(np.unique(np.round(np.abs(lam.imag), 9)))
    np.testing.assert_allclose(got, expect, rtol=1e-8)
    for tau in (1e-3, 1e-1, 1.0, 10.0, 1e3):
        rho = np.abs(np.linalg.eigvals(step_matrix(h, c2, tau))).max()
        assert rho <= 1.0 + 1e-12


def test_l_stability():
    h, c2 = 1.0, 50.0
    q = np.array([h, 0, 0, 0.3, -0.4, 0.2, 0.5])
    out = O.source_cell(q, c2, 1e9)
    assert np.abs(out[3:]).max() < 1e-6
