"""Pins of oracle/chebyshev.py against closed forms of the Chebyshev
polynomials (paper Sec. 2.1-2.2)."""
import math

import numpy as np
import pytest

from oracle import chebyshev as ch

# textbook expansions of the first Chebyshev polynomials (not the cos/cosh form)
EXPANSIONS = {
    0: lambda t: 1.0,
    1: lambda t: t,
    2: lambda t: 2 * t**2 - 1,
    3: lambda t: 4 * t**3 - 3 * t,
    4: lambda t: 8 * t**4 - 8 * t**2 + 1,
    5: lambda t: 16 * t**5 - 20 * t**3 + 5 * t,
    6: lambda t: 32 * t**6 - 48 * t**4 + 18 * t**2 - 1,
}


@pytest.mark.parametrize("m", sorted(EXPANSIONS))
@pytest.mark.parametrize("t", [-3.5, -1.7, -1.0, -0.3, 0.0, 0.42, 1.0, 1.3, 4.0])
def test_closed_form_matches_expansion(m, t):
    ref = EXPANSIONS[m](t)
    assert ch.cheb_closed(m, t) == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_integer_values_at_two():
    # C_n(2) = 1, 2, 7, 26, 97, 362, 1351, 5042, 18817 (integer sequence)
    seq = [1, 2, 7, 26, 97, 362, 1351, 5042, 18817]
    for n, v in enumerate(seq):
        assert ch.cheb_closed(n, 2.0) == pytest.approx(v, rel=1e-13)
        assert ch.cheb_closed(n, -2.0) == pytest.approx((-1) ** n * v, rel=1e-13)


@pytest.mark.parametrize("t", [1.01, 1.5, 2.0, 7.3, -1.2, -4.0])
@pytest.mark.parametrize("m", [1, 2, 5, 13, 36])
def test_rho_asymptotic_identity(t, m):
    # the rho form of C_m in Sec. 2.1: C_m(t) = (|rho|^m + |rho|^-m)/2 for |t| > 1 (|C_m|, sign by parity)
    rho = ch.rho_abs(t, 0.0, 1.0)
    assert rho > 1.0
    lhs = abs(ch.cheb_closed(m, t))
    assert lhs == pytest.approx(0.5 * (rho**m + rho ** (-m)), rel=1e-12)


def test_rho_inside_interval_is_one():
    for x in np.linspace(-1.0, 3.0, 17):  # interval [c-e, c+e] = [-1, 3]
        assert ch.rho_abs(float(x), 1.0, 2.0) == 1.0


def test_rho_golden_ratio():
    # t = 1.5 -> |rho| = 1.5 + sqrt(1.25) = phi^2
    phi = (1 + math.sqrt(5)) / 2
    assert ch.rho_abs(-1.5, 0.0, 1.0) == pytest.approx(phi**2, rel=1e-15)
    assert ch.rho_abs(2.0, 0.0, 1.0) == pytest.approx(2 + math.sqrt(3), rel=1e-15)


@pytest.mark.parametrize("c,e,gamma", [(0.0, 1.0, -2.0), (0.063, 0.936, -0.999), (24.5, 25.5, -2.0), (500.0, 500.5, -1.0)])
def test_sigma_is_ratio_of_polynomials(c, e, gamma):
    # Sec. 2.2: sigma_{m+1} = eta_m / eta_{m+1}, eta_m = C_m((gamma-c)/e)
    tg = (gamma - c) / e
    s = ch.sigma_sequence(30, c, e, gamma)
    for m in range(1, 31):
        ref = ch.cheb_closed(m - 1, tg) / ch.cheb_closed(m, tg)
        assert s[m] == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("m", [1, 2, 3, 10, 20, 36, 60])
def test_scaled_recurrence_matches_closed_form(m):
    c, e, gamma = 0.3, 1.2, -1.4
    for x in [-1.4, -1.1, -0.9, 0.0, 0.7, 1.5]:
        r = ch.scaled_poly_recurrence(m, x, c, e, gamma)
        ref = ch.scaled_poly_closed(m, x, c, e, gamma)
        assert r == pytest.approx(ref, rel=1e-11, abs=1e-14)
    # normalisation p_m(gamma) = 1
    assert ch.scaled_poly_recurrence(m, gamma, c, e, gamma) == pytest.approx(1.0, rel=1e-12)


def test_filter_optimality_bound():
    # inside [alpha, beta] |p_m| <= 1/|C_m(t_gamma)| (Thm. in Sec. 2.1)
    c, e, gamma, m = 0.0, 1.0, -1.3, 12
    bound = 1.0 / abs(ch.cheb_closed(m, (gamma - c) / e))
    for x in np.linspace(-1, 1, 101):
        assert abs(ch.scaled_poly_recurrence(m, float(x), c, e, gamma)) <= bound * (1 + 1e-10)
