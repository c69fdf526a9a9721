"""Pins of oracle/qr.py on blocks with planted singular values (Table 1,
Alg. 2, Alg. 3)."""
import json
import os

import numpy as np
import pytest

from oracle import qr

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
U = 2.0**-53


def planted_block(N, L, kappa, seed, cplx=False):
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((N, L)) + (1j * rng.standard_normal((N, L)) if cplx else 0)
    G2 = rng.standard_normal((L, L)) + (1j * rng.standard_normal((L, L)) if cplx else 0)
    Uo, _ = np.linalg.qr(G1)
    Wo, _ = np.linalg.qr(G2)
    s = np.logspace(0, -np.log10(kappa), L)
    return (Uo * s) @ Wo.conj().T


def orth_err(Q):
    return np.linalg.norm(Q.conj().T @ Q - np.eye(Q.shape[1]))


def span_err(Q, X):
    # residual of X projected on range(Q), relative
    return np.linalg.norm(X - Q @ (Q.conj().T @ X)) / np.linalg.norm(X)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("kappa", [1e1, 1e4, 1e7])
def test_cholqr2_orthogonal_within_its_range(kappa, cplx):
    X = planted_block(600, 40, kappa, 1, cplx)
    Q = qr.cholqr(X, 2)
    assert orth_err(Q) < 100 * 40 * U
    assert span_err(Q, X) < 1e-12


def test_cholqr1_loses_orthogonality_like_kappa_squared():
    errs = []
    for kappa in [1e2, 1e4, 1e6]:
        errs.append(orth_err(qr.cholqr(planted_block(600, 40, kappa, 2), 1)))
    # O(kappa^2 u): each factor 100 in kappa costs ~1e4 in orthogonality
    assert errs[0] < 1e-10 and errs[1] > 1e-10 and errs[2] > 1e-6
    assert errs[2] / errs[0] > 1e6


@pytest.mark.parametrize("kappa", [1e10, 1e12])
def test_shifted_extends_range(kappa):
    X = planted_block(600, 40, kappa, 3)
    with pytest.raises(qr.CholeskyFailure):
        qr.cholqr(X, 2)
    Q, failed = qr.dynamic_caqr(X, "shifted")
    assert not failed
    assert orth_err(Q) < 100 * 40 * U
    assert span_err(Q, X) < 1e-9


def test_fallback_to_householder_beyond_shifted_range():
    X = planted_block(600, 40, 1e17, 4)
    Q, failed = qr.dynamic_caqr(X, "shifted")
    assert failed
    assert orth_err(Q) < 100 * 40 * U
    Q2, failed2 = qr.dynamic_caqr(X, "chol2")
    assert failed2 and orth_err(Q2) < 100 * 40 * U


def test_table1_ordering():
    """Table 1: the kappa each variant tolerates grows CholQR < CholQR2 <
    shifted CholQR2 < Householder; the exponents of u are the paper's."""
    lim = GOLD["table1_kappa_limits_log10u"]
    assert lim["cholqr"] > lim["cholqr2"] > lim["shifted_cholqr2"]
    ok = {"chol2": [], "shifted": []}
    for kappa in [1e6, 1e9, 1e11, 1e13, 1e16]:
        X = planted_block(400, 30, kappa, 5)
        for v in ok:
            Q, failed = qr.dynamic_caqr(X, v)
            if not failed and orth_err(Q) < 1e-12:
                ok[v].append(kappa)
    assert max(ok["chol2"]) <= 1e9 < max(ok["shifted"])
    # u^-1/2 ~ 9.5e7: CholQR2 works well below it
    assert 1e6 in ok["chol2"]


def test_householder_reconstructs():
    X = planted_block(300, 25, 1e20, 6, True)
    Q = qr.householder_qr(X)
    assert orth_err(Q) < 1e-13
    R = Q.conj().T @ X
    assert np.linalg.norm(np.tril(R, -1)) < 1e-12 * np.linalg.norm(X)


def test_shift_scales_with_frobenius_norm_squared():
    X = planted_block(200, 10, 10.0, 7)
    s1 = qr.shift_value(X)
    s2 = qr.shift_value(3.0 * X)
    assert s2 == pytest.approx(9.0 * s1, rel=1e-13, abs=0)
    assert 0 < s1 < 1e-9


def test_shift_hand_evaluated():
    """Alg. 3's shift s = 11 (m n + n (n + 1)) u ||X||^2 (reading: m rows,
    n columns, u = 2^-53, squared Frobenius norm), evaluated by hand on
    X = [e_1, 2 e_2] in R^{4 x 2}: m n = 8, n (n + 1) = 6, ||X||_F^2 = 1 + 4 = 5,
    so s = 11 * 14 * 5 * 2^-53 = 770 * 2^-53.  A slip in any factor (the 11,
    u = 2^-52, n (n - 1), m (m + 1), an unsquared norm, a stray scale) changes
    the value by far more than the tolerance."""
    X = np.zeros((4, 2))
    X[0, 0] = 1.0
    X[1, 1] = 2.0
    assert qr.shift_value(X) == pytest.approx(8.548717289613705e-14, rel=1e-15, abs=0)
    assert 770.0 * 2.0 ** -53 == pytest.approx(8.548717289613705e-14, rel=1e-15, abs=0)
    # complex entries: |x|^2 enters the norm (||X||_F^2 = 1 + |1 + 2i|^2 = 6)
    Xc = np.zeros((3, 1), dtype=complex)
    Xc[0, 0] = 1.0
    Xc[2, 0] = 1.0 + 2.0j
    # m n = 3, n (n + 1) = 2: s = 11 * 5 * 6 * 2^-53 = 330 * 2^-53
    assert qr.shift_value(Xc) == pytest.approx(330.0 * 2.0 ** -53, rel=1e-15, abs=0)


def test_shifted_pass_adds_the_shift_to_the_gram_diagonal():
    """The shifted pass factors X^H X + s I: on X = [e_1, 2 e_2] that matrix is
    diag(1 + s, 4 + s), so R = diag(sqrt(1 + s), sqrt(4 + s)) and the
    output columns are e_1 / sqrt(1 + s) and 2 e_2 / sqrt(4 + s)."""
    X = np.zeros((4, 2))
    X[0, 0] = 1.0
    X[1, 1] = 2.0
    s = 770.0 * 2.0 ** -53
    Q = qr.shifted_cholqr_pass(X)
    assert Q[0, 0] == pytest.approx(1.0 / np.sqrt(1.0 + s), rel=1e-16, abs=0)
    assert Q[1, 1] == pytest.approx(2.0 / np.sqrt(4.0 + s), rel=1e-16, abs=0)
    assert 1.0 - Q[0, 0] == pytest.approx(0.5 * s, rel=1e-2, abs=0)
