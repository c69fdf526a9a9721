"""Pins of oracle/filter.py: on a planted H = Q diag(lambda) Q^H the filtered
block has the closed form Q diag(p_{m_a}(lambda)) Q^H v_a column by column
(the spectral form of p(A)V in Sec. 2.3), computed here from cos/cosh without the recurrence."""
import numpy as np
import pytest

import synth
from oracle import chebyshev as ch
from oracle import filter as flt


def _closed_form(Q, lam, V, degrees, c, e, gamma):
    out = np.empty_like(V)
    S = Q.conj().T @ V
    for a, m in enumerate(degrees):
        p = ch.scaled_poly_closed_vec(int(m), lam, c, e, gamma)
        out[:, a] = Q @ (p * S[:, a])
    return out


def _planted_with_q(N, cplx, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, N)) + (1j * rng.standard_normal((N, N)) if cplx else 0)
    Q, _ = np.linalg.qr(G)
    lam = np.sort(rng.uniform(-1, 1, N))
    H = (Q * lam) @ Q.conj().T
    return 0.5 * (H + H.conj().T), Q, lam


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("degrees", [[20] * 12, [1, 2, 3, 5, 8, 13, 21, 34, 36], [7, 3, 12, 1, 36, 5]])
def test_filter_matches_spectral_closed_form(cplx, degrees):
    N = 160
    H, Q, lam = _planted_with_q(N, cplx, 5)
    V = synth.start_block(N, len(degrees), 6, cplx)
    alpha, beta = lam[len(degrees) + 4], lam[-1]
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    gamma = lam[0]
    got = flt.chebyshev_filter(H, V, degrees, c, e, gamma)
    ref = _closed_form(Q, lam, V, degrees, c, e, gamma)
    for a in range(len(degrees)):
        err = np.linalg.norm(got[:, a] - ref[:, a]) / np.linalg.norm(ref[:, a])
        assert err < 1e-11, (a, degrees[a], err)


def test_filter_matvec_count():
    assert flt.matvecs([1, 2, 3, 36]) == 42


def test_filter_rejects_bad_degrees():
    H = np.eye(4)
    with pytest.raises(ValueError):
        flt.chebyshev_filter(H, np.ones((4, 2)), [0, 1], 0.0, 1.0, -2.0)
    with pytest.raises(ValueError):
        flt.chebyshev_filter(H, np.ones((4, 2)), [1], 0.0, 1.0, -2.0)


def test_filter_empty_block():
    H = np.eye(4)
    out = flt.chebyshev_filter(H, np.ones((4, 0)), [], 0.0, 1.0, -2.0)
    assert out.shape == (4, 0)


def test_planted_mistake_is_caught(monkeypatch):
    """A plausible slip (dropping the sigma_{i-1} sigma_i term's sign) must
    fail the closed-form pin."""
    import oracle.chebyshev as chm
    N = 80
    H, Q, lam = _planted_with_q(N, False, 7)
    V = synth.start_block(N, 4, 8)
    c, e, gamma = 0.5 * (lam[10] + lam[-1]), 0.5 * (lam[-1] - lam[10]), lam[0]
    degrees = [3, 4, 5, 6]
    ref = _closed_form(Q, lam, V, degrees, c, e, gamma)
    good = flt.chebyshev_filter(H, V, degrees, c, e, gamma)
    assert np.linalg.norm(good - ref) / np.linalg.norm(ref) < 1e-11

    orig = chm.sigma_sequence

    def wrong(mmax, c_, e_, g_):
        s = orig(mmax, c_, e_, g_)
        return [-x for x in s]  # wrong sign convention of sigma_1

    monkeypatch.setattr(flt, "sigma_sequence", wrong)
    bad = flt.chebyshev_filter(H, V, degrees, c, e, gamma)
    assert np.linalg.norm(bad - ref) / np.linalg.norm(ref) > 1e-3
