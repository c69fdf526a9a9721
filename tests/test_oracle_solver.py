"""Pins of oracle/rr.py, oracle/solver.py, oracle/lanczos.py and
oracle/degrees.py: planted eigenvalues, full diagonalisation, the residual
bound, the HHQR-versus-CholQR invariant of Table 3, and the Lanczos
estimate's Gauss weights, top Ritz pair and upper-bound property."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import degrees, lanczos, rr, solver
from oracle import filter as ofilter

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_rr_on_exact_eigenvectors():
    N = 120
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    lam = np.sort(rng.uniform(-3, 3, N))
    H = (Q * lam) @ Q.conj().T
    H = 0.5 * (H + H.conj().T)
    sub = Q[:, [5, 2, 9, 0]]
    W, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    theta, V, HV = rr.rayleigh_ritz(H, sub @ W)  # rotated basis of an invariant subspace
    assert np.allclose(theta, np.sort(lam[[5, 2, 9, 0]]), atol=1e-13)
    r = rr.residual_norms(HV, V, theta)
    assert np.all(r < 1e-13)


def test_residual_definition_on_known_vector():
    H = np.diag([1.0, 2.0, 3.0])
    v = np.array([[1.0], [1.0], [0.0]])
    theta = np.array([1.0])
    # ||H v - v|| / ||v|| = ||(0, 1, 0)|| / sqrt(2)
    assert rr.residual_norms(H @ v, v, theta)[0] == pytest.approx(1 / np.sqrt(2), rel=1e-15)


@pytest.mark.parametrize("cplx,family,seed", [(False, "uniform", 1), (True, "dft", 2)])
def test_solver_finds_planted_eigenvalues(cplx, family, seed):
    N, nev, nex = (1000, 40, 20) if not cplx else (600, 30, 12)
    H, lam = synth.planted_numpy(N, family, seed, cplx)
    V0 = synth.start_block(N, nev + nex, seed + 10, cplx)
    max_deg = 36
    res = solver.chase_solve(H, nev, nex, 20, 1e-10, V0=V0,
                             bounds=(lam[0], lam[nev + nex - 1], lam[-1]), max_deg=max_deg)
    assert res.converged == nev
    scale = np.max(np.abs(lam))
    assert np.max(np.abs(res.evals - lam[:nev])) <= 1e-10 * scale
    assert np.all(res.resid < 1e-10)
    # residual bound: a true eigenvalue within r of every Ritz value
    for th, r in zip(res.evals, res.resid):
        assert np.min(np.abs(lam - th)) <= r + 1e-15
    Y = res.evecs[:, :nev]
    assert np.linalg.norm(Y.conj().T @ Y - np.eye(nev)) < 1e-12
    assert 2 <= res.iters <= 12


def test_solver_matches_full_diagonalisation_small():
    N, nev, nex = 200, 10, 6
    rng = np.random.default_rng(3)
    A = rng.standard_normal((N, N))
    H = 0.5 * (A + A.T)  # not planted: compare with LAPACK full eigh
    w = sla.eigh(H, eigvals_only=True)
    v0 = synth.lanczos_start(N, 4)
    V0 = synth.start_block(N, nev + nex, 5)
    res = solver.chase_solve(H, nev, nex, 20, 1e-10, V0=V0, lanczos_v0=v0, lanczos_steps=40)
    assert res.converged == nev
    assert np.max(np.abs(res.evals - w[:nev])) < 1e-10 * np.max(np.abs(w))


def test_householder_vs_dynamic_same_convergence():
    """Table 3: the QR variant leaves the iteration count unchanged and the
    MatVecs within a few per cent."""
    rows = GOLD["table3_cholqr_vs_hhqr"]["rows"]
    paper_spread = max(abs(r["hh_matvecs"] - r["chol_matvecs"]) / r["hh_matvecs"] for r in rows)
    assert all(r["hh_iters"] == r["chol_iters"] for r in rows)
    N, nev, nex = 500, 20, 10
    H, lam = synth.planted_numpy(N, "uniform", 7)
    V0 = synth.start_block(N, nev + nex, 8)
    b = (lam[0], lam[nev + nex - 1], lam[-1])
    auto = solver.chase_solve(H, nev, nex, 20, 1e-10, V0=V0, bounds=b)
    hh = solver.chase_solve(H, nev, nex, 20, 1e-10, V0=V0, bounds=b, qr_policy="householder")
    assert auto.iters == hh.iters
    assert abs(auto.matvecs - hh.matvecs) / hh.matvecs <= max(paper_spread, 0.04) + 1e-12
    assert np.max(np.abs(auto.evals - hh.evals)) < 1e-12


def test_upper_bound_check_is_inert_for_a_true_bound():
    theta = np.array([-1.0, -0.5, 0.2])
    r = np.array([1e-3, 1e-2, 0.3])
    assert solver.upper_bound_check(theta, r, 0.2) == 0.2  # equal: still a bound
    assert solver.upper_bound_check(theta, r, 5.0) == 5.0
    # above it: theta_max + 2 r_max + 1e-3 (theta_max - theta_min)
    assert solver.upper_bound_check(theta, r, 0.1) == pytest.approx(0.2 + 0.6 + 1.2e-3, rel=1e-15)
    assert solver.upper_bound_check(theta, np.zeros(3), 0.1) > 0.2  # r = 0: interval stays open


@pytest.mark.parametrize("beta", [0.5, 0.0])
def test_wrong_upper_bound_is_detected_and_raised(beta):
    """Sec. 1.2 needs beta >= lambda_n.  Given a beta inside the spectrum,
    the first Rayleigh-Ritz step shows a Ritz value above it (Ritz values
    never exceed lambda_n), beta is raised, every later damped interval is
    non-empty (e > 0), and the solve still finds the planted eigenvalues."""
    N, nev, nex = 300, 20, 10
    H, lam = synth.planted_numpy(N, "uniform", 11)
    V0 = synth.start_block(N, nev + nex, 12)
    res = solver.chase_solve(H, nev, nex, 20, 1e-10, V0=V0, bounds=(-1.0, -0.8, beta))
    assert res.converged == nev
    assert np.max(np.abs(res.evals - lam[:nev])) < 1e-12
    assert all(x["e"] > 0 for x in res.log)
    assert any(x["c"] + x["e"] > beta + 1e-9 for x in res.log[1:])


def test_search_space_must_exceed_nev():
    H, lam = synth.planted_numpy(20, "uniform", 1)
    with pytest.raises(ValueError):
        solver.chase_solve(H, 3, 0, V0=synth.start_block(20, 3, 2), bounds=(lam[0], lam[2], lam[-1]))


def test_not_converged_reports_partial():
    N, nev, nex = 300, 12, 6
    H, lam = synth.planted_numpy(N, "uniform", 9)
    V0 = synth.start_block(N, nev + nex, 10)
    res = solver.chase_solve(H, nev, nex, 4, 1e-10, V0=V0, deg_opt=False,
                             bounds=(lam[0], lam[nev + nex - 1], lam[-1]), max_iter=1)
    assert res.converged < nev and res.iters == 1
    assert res.evals.shape == (nev,)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("family", ["dft", "uniform", "stress"])
def test_lanczos_upper_bound(seed, cplx, family):
    """Four runs (the library's default): the estimate bounds lambda_n."""
    N = 400
    H, lam = synth.planted_numpy(N, family, seed, cplx, **({"n_low": 20} if family == "stress" else {}))
    V0 = synth.lanczos_starts(N, 4, seed + 100, cplx)
    low, mid, up = lanczos.lanczos_bounds(H, 30, V0, 40)
    assert up >= lam[-1]
    assert low >= lam[0] - 1e-12  # Ritz values lie inside the spectrum
    assert low < mid < up
    # and it is tight: the top of the spectrum converges first
    assert up - lam[-1] <= 0.03 * (lam[-1] - lam[0])


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("family", ["dft", "uniform"])
def test_lanczos_upper_bound_single_run(seed, family):
    """One run of 40 steps on a small matrix can miss a nearly isolated top
    eigenvalue that its start vector hardly sees (seed 2 of the dft family
    here); the miss stays a tiny part of the spectrum's width, where the
    filter's growth is modest."""
    N = 400
    H, lam = synth.planted_numpy(N, family, seed, False)
    low, mid, up = lanczos.lanczos_bounds(H, 30, synth.lanczos_starts(N, 1, seed + 100), 40)
    span = lam[-1] - lam[0]
    assert lam[-1] - 1e-3 * span <= up <= lam[-1] + 0.03 * span


def test_lanczos_single_vector_equals_block_of_one():
    N = 300
    H, _ = synth.planted_numpy(N, "dft", 5, True)
    v = synth.lanczos_start(N, 6, True)
    assert lanczos.lanczos_bounds(H, 20, v, 30) == lanczos.lanczos_bounds(H, 20, v[:, None], 30)


def test_lanczos_gauss_weights_three_eigenvalues():
    """H with three distinct eigenvalues: three Lanczos steps span an
    invariant Krylov space, the Ritz values are the eigenvalues and the
    spectral-density weights are N times the squared norms of the start
    vector's projections on the eigenspaces (Gauss quadrature of the
    spectral measure)."""
    N = 90
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    vals = np.array([-1.5] * 7 + [0.25] * 20 + [2.0] * (N - 27))
    H = (Q * vals) @ Q.T
    H = 0.5 * (H + H.T)
    v0 = rng.standard_normal(N)
    a, b = lanczos.lanczos_tridiag(H, v0, 3)
    theta, w, top_r = lanczos.lanczos_dos(a, b, N)
    assert np.allclose(theta, [-1.5, 0.25, 2.0], atol=1e-12)
    vhat = v0 / np.linalg.norm(v0)
    c = Q.T @ vhat
    proj = np.array([np.sum(c[:7] ** 2), np.sum(c[7:27] ** 2), np.sum(c[27:] ** 2)])
    assert np.allclose(w, N * proj, rtol=1e-10)
    assert np.isclose(w.sum(), N)
    assert top_r <= 1e-12  # the top Ritz pair is exact
    # the l estimate counts whole eigenspaces: l = 7 falls on -1.5 when the
    # start vector's weight there reaches it
    low, mid, up = lanczos.bounds_from_runs([(a, b)], N, 1)
    assert low == pytest.approx(-1.5, abs=1e-12) and up == pytest.approx(2.0, abs=1e-12)


def test_lanczos_density_count_tracks_eigenvalue_count():
    """The lambda_l estimate reads the run-averaged count (1/nvec) sum_r
    sum_{theta_rj <= x} N |e_1^T s_rj|^2, an unbiased estimate of the
    number of eigenvalues <= x (E N |q_i^H v|^2 = 1 for a random unit v).
    With 32 full-length runs the estimate lands within a few eigenvalues of
    lambda_l; with 40 steps, within the coarser quadrature resolution."""
    N = 200
    H, lam = synth.planted_numpy(N, "uniform", 9)
    V0 = synth.lanczos_starts(N, 32, 10)
    full = [lanczos.lanczos_tridiag(H, V0[:, r], N) for r in range(32)]
    short = [lanczos.lanczos_tridiag(H, V0[:, r], 40) for r in range(32)]
    for L in (20, 60, 120):
        j_full = int(np.sum(lam <= lanczos.bounds_from_runs(full, N, L)[1] + 1e-12))
        j_short = int(np.sum(lam <= lanczos.bounds_from_runs(short, N, L)[1] + 1e-12))
        assert abs(j_full - L) <= 4, (L, j_full)
        assert abs(j_short - L) <= 0.1 * L + 2, (L, j_short)


@pytest.mark.parametrize("cplx", [False, True])
def test_lanczos_top_pair_against_krylov_rayleigh_ritz(cplx):
    """The largest Ritz value of T_k and |beta_k||e_k^T s_max| equal the
    largest Rayleigh-Ritz value, and its residual norm, on an orthonormal
    basis of the Krylov space built by QR of the power sequence."""
    N, k = 200, 6
    H, _ = synth.planted_numpy(N, "uniform", 8, cplx)
    v0 = synth.lanczos_start(N, 9, cplx)
    K = np.empty((N, k), dtype=H.dtype)
    x = v0 / np.linalg.norm(v0)
    for j in range(k):
        K[:, j] = x
        x = H @ x
        x = x / np.linalg.norm(x)
    Qk, _ = np.linalg.qr(K)
    th, Z = np.linalg.eigh(Qk.conj().T @ H @ Qk)
    y = Qk @ Z[:, -1]
    r_direct = np.linalg.norm(H @ y - th[-1] * y)
    a, b = lanczos.lanczos_tridiag(H, v0, k)
    theta, w, top_r = lanczos.lanczos_dos(a, b, N)
    assert theta[-1] == pytest.approx(th[-1], abs=1e-10)
    assert top_r == pytest.approx(r_direct, rel=1e-6, abs=1e-12)


def test_lanczos_tridiagonal_reproduces_krylov_basis():
    # T_k = V^H H V for the Lanczos basis; its eigenvalues interlace the spectrum
    N = 150
    H, lam = synth.planted_numpy(N, "uniform", 4)
    a, b = lanczos.lanczos_tridiag(H, synth.lanczos_start(N, 5), N)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    # a full run (k = N) has the whole spectrum
    assert np.allclose(np.sort(sla.eigvalsh(T)), lam, atol=1e-10)


@pytest.mark.parametrize("lam1", [-1.5, -1.1, -3.0])
@pytest.mark.parametrize("delta", [1e-2, 1e-4, 1e-6])
def test_degree_rule_reaches_tol(lam1, delta):
    """What the degree rule predicts: a vector with residual r whose unwanted
    components lie in the damped interval loses a factor |rho(theta)| per
    filter step (Chebyshev growth outside [-1, 1], Sec. 2.1), so the
    predicted degree brings its residual to tol.  Diagonal H, wanted
    eigenvalue lam1 below the damped interval [0, 2]; the filtered vector's
    residual is recomputed from its own Rayleigh quotient."""
    rng = np.random.default_rng(int(abs(lam1) * 10) + int(-np.log10(delta)))
    N, tol = 300, 1e-10
    lam = np.concatenate([[lam1], np.sort(rng.uniform(0.0, 2.0, N - 1))])
    H = np.diag(lam)

    def resid(x):
        x = x / np.linalg.norm(x)
        th = float(x @ (H @ x))
        return th, float(np.linalg.norm(H @ x - th * x))

    w = rng.standard_normal(N)
    w[0] = 0.0
    v = np.zeros(N)
    v[0] = 1.0
    v = v + delta * w / np.linalg.norm(w)
    th, r = resid(v)
    c, e = 1.0, 1.0
    m = int(degrees.optimised_degrees(np.array([th]), np.array([r]), tol, c, e, 1, 200)[0])
    r_at = {mm: resid(ofilter.chebyshev_filter(H, v[:, None], np.array([mm]), c, e, th)[:, 0])[1]
            for mm in (m - 3, m - 2, m)}
    assert r_at[m] <= tol                 # the rule with its margin of 2
    assert r_at[m - 2] <= 2.0 * tol       # the bare prediction: tol within T_m ~ |rho|^m / 2
    assert r_at[m - 3] > 0.1 * tol        # and not more than one degree to spare


def test_degrees_rule():
    c, e = 0.0, 1.0
    tol = 1e-10
    th = np.array([-2.0, -1.5, -1.2, 0.5, -3.0])
    r = np.array([1e-2, 1e-4, 1e-3, 1e-2, 1e-11])
    m = degrees.optimised_degrees(th, r, tol, c, e, 1, 36)
    assert m[4] == 1            # already converged
    assert m[3] == 36           # inside the damped interval
    assert 1 <= m[0] <= m[2] <= 36
    d0 = int(np.ceil(np.log(1e-2 / tol) / np.log(2 + np.sqrt(3)))) + 2
    assert m[0] == d0
    gold = GOLD["experiment_settings"]
    assert gold["max_degree"] == 36 and gold["initial_degree"] == 20
