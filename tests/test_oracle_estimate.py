"""Pins of oracle/estimate.py (estimate (1.1), estimate (1.2), Alg. 3)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import estimate as est
from oracle import solver

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
PHI = (1 + math.sqrt(5)) / 2


def test_hand_evaluated_simple_estimate():
    # c = 0, e = 1, gamma = -2: |rho_1| = 2 + sqrt(3); (2+sqrt3)^5 = 2*C_5(2) - (2-sqrt3)^5
    v = est.cond_estimate(-2.0, 5, 5, -2.0, 0.0, 1.0)
    assert v == pytest.approx(2 * 362 - (2 - math.sqrt(3)) ** 5, rel=1e-13)


def test_hand_evaluated_full_estimate():
    # theta_{k+1} = -1.5 -> |rho| = phi^2; m_{k+1} = 3, m_l = 5, gamma = -2:
    # est = phi^6 (2+sqrt3)^2 = (9 + 4 sqrt5)(7 + 4 sqrt3)
    v = est.cond_estimate(-1.5, 3, 5, -2.0, 0.0, 1.0)
    assert v == pytest.approx((9 + 4 * math.sqrt(5)) * (7 + 4 * math.sqrt(3)), rel=1e-13)
    assert PHI**6 == pytest.approx(9 + 4 * math.sqrt(5), rel=1e-14)


@pytest.mark.parametrize("m_next,m_max", [(1, 20), (20, 20), (7, 36)])
def test_full_reduces_to_simple_without_locking(m_next, m_max):
    # estimate (1.2) with theta_{k+1} = lambda_1 (nothing locked) is estimate (1.1) with m -> m_l
    c, e, g = 0.063, 0.936, -0.999
    full = est.cond_estimate(g, m_next, m_max, g, c, e)
    simple = est.cond_estimate(g, m_max, m_max, g, c, e)
    assert full == pytest.approx(simple, rel=1e-12)


def test_no_opt_reduces_to_single_ratio():
    # fixed degree: the estimate is |rho_{k+1}|^m (Sec. 4.3)
    c, e, g, th, m = 0.0, 1.0, -2.0, -1.5, 20
    assert est.cond_estimate(th, m, m, g, c, e) == pytest.approx(PHI ** (2 * m), rel=1e-12)


def test_locking_never_raises_estimate():
    c, e, g = 0.0, 1.0, -2.0
    top = est.cond_estimate(g, 36, 36, g, c, e)
    for th in np.linspace(-2.0, -1.0, 11):
        for mn in [1, 10, 36]:
            assert est.cond_estimate(float(th), mn, 36, g, c, e) <= top * (1 + 1e-12)


def test_overflow_is_infinite_not_error():
    assert est.cond_estimate(-1e6, 200, 400, -1e6, 0.0, 1.0) == float("inf")
    assert est.log_cond_estimate(-1e6, 200, 400, -1e6, 0.0, 1.0) > 709


def test_variant_thresholds_from_paper():
    hi, lo = GOLD["alg3_thresholds"]["hi"], GOLD["alg3_thresholds"]["lo"]
    assert (est.EST_HI, est.EST_LO) == (hi, lo)
    assert est.select_variant(1.0000001e8) == "shifted"
    assert est.select_variant(1e8) == "chol2"
    assert est.select_variant(20.0) == "chol2"
    assert est.select_variant(19.999) == "chol1"
    assert est.select_variant(float("inf")) == "shifted"


@pytest.mark.parametrize("deg_opt", [False, True])
def test_estimate_bounds_exact_condition_number(deg_opt):
    """Empirical property reported in Sec. 4.3: the estimate stays above the
    exact kappa_2 (by SVD) of [Y, filtered] at every iteration."""
    N, nev, nex = 400, 16, 10
    H, lam = synth.planted_numpy(N, "uniform", 21)
    V0 = synth.start_block(N, nev + nex, 22)
    r = solver.chase_solve(H, nev, nex, 20, 1e-10, V0=V0, deg_opt=deg_opt,
                           bounds=(lam[0], lam[nev + nex - 1], lam[-1]), exact_cond=True)
    assert r.converged == nev
    for rec in r.log:
        assert rec["cond_est"] >= rec["cond_exact"], rec


@pytest.mark.parametrize("cplx", [False, True])
def test_deflation_theorem_brute_force(cplx):
    """Theorem 3.4 (Sec. 3.3), the step that lets the locked block drop out
    of the estimate: for A (n x q) and B (n x p) with A^H B = 0,
    kappa_2([A B]) <= (sigma_1(A) + sigma_1(B)) / min(sigma_q(A), sigma_p(B)).
    Checked on random pairs with spread singular values, including pairs
    where the bound is nearly tight (one singular value per block)."""
    rng = np.random.default_rng(41)
    for trial in range(200):
        n = int(rng.integers(8, 60))
        q = int(rng.integers(1, n // 2))
        p = int(rng.integers(1, n - q))
        G = rng.standard_normal((n, q + p)) + (1j * rng.standard_normal((n, q + p)) if cplx else 0)
        U = np.linalg.qr(G)[0]
        sa = 10.0 ** rng.uniform(-4, 4, q)
        sb = 10.0 ** rng.uniform(-4, 4, p)
        Wa = np.linalg.qr(rng.standard_normal((q, q)))[0]
        Wb = np.linalg.qr(rng.standard_normal((p, p)))[0]
        A = (U[:, :q] * sa) @ Wa
        B = (U[:, q:] * sb) @ Wb
        assert np.linalg.norm(A.conj().T @ B) <= 1e-10 * np.linalg.norm(A) * np.linalg.norm(B)
        s = np.linalg.svd(np.hstack([A, B]), compute_uv=False)
        bound = (sa.max() + sb.max()) / min(sa.min(), sb.min())
        assert s[0] / s[-1] <= bound * (1 + 1e-9), (trial, s[0] / s[-1], bound)


@pytest.mark.parametrize("m", [1, 5, 20])
def test_filtered_eigenvectors_condition_closed_form(m):
    """Lemma 3.1, statement 1 (Sec. 3.1): filtering the wanted eigenvectors
    themselves gives kappa_2 = |C_m(t_1)| / |C_m(t_l)| with t = (lambda - c)/e,
    computed here by SVD of the oracle's filtered block and by cosh/arccosh;
    it never exceeds estimate (1.1) = |rho(lambda_1)|^m."""
    N, L = 300, 24
    lam = np.sort(np.concatenate([np.linspace(-2.0, -1.2, L), np.linspace(-1.0, 5.0, N - L)]))
    H = np.diag(lam)
    c, e = 0.5 * (-1.0 + 5.0), 0.5 * (5.0 + 1.0)
    from oracle import filter as ofilter
    X = np.eye(N)[:, :L]
    Y = ofilter.chebyshev_filter(H, X, np.full(L, m), c, e, lam[0])
    s = np.linalg.svd(Y, compute_uv=False)
    t = (lam[:L] - c) / e
    cm = np.cosh(m * np.arccosh(np.abs(t)))  # |C_m(t)| for |t| >= 1
    closed = cm.max() / cm.min()
    assert s[0] / s[-1] == pytest.approx(closed, rel=1e-10)
    assert closed <= est.cond_estimate(lam[0], m, m, lam[0], c, e) * (1 + 1e-12)
