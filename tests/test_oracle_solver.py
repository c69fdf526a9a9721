"""Pins of oracle/rr.py, oracle/solver.py, oracle/lanczos.py and
oracle/degrees.py: planted eigenvalues, full diagonalisation, the residual
bound, the HHQR-versus-CholQR invariant of Table 3 and the upper-bound
property of the Lanczos estimate."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import degrees, lanczos, rr, solver

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


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("cplx", [False, True])
def test_lanczos_upper_bound(seed, cplx):
    N = 400
    H, lam = synth.planted_numpy(N, "dft", seed, cplx)
    low, mid, up = lanczos.lanczos_bounds(H, 30, synth.lanczos_start(N, seed + 100, cplx), 40)
    assert up >= lam[-1]
    assert low >= lam[0] - 1e-12  # Ritz values lie inside the spectrum
    assert low < mid < up


def test_lanczos_tridiagonal_reproduces_krylov_basis():
    # T_k = V^H H V for the Lanczos basis; its eigenvalues interlace the spectrum
    N = 150
    H, lam = synth.planted_numpy(N, "uniform", 4)
    a, b = lanczos.lanczos_tridiag(H, synth.lanczos_start(N, 5), N)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    # a full run (k = N) has the whole spectrum
    assert np.allclose(np.sort(sla.eigvalsh(T)), lam, atol=1e-10)


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
