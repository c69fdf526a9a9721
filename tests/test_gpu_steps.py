"""GPU parity of the individual steps (filter, QR variants, Rayleigh-Ritz,
residuals, Lanczos) against the oracle, called through the C ABI."""
import numpy as np
import pytest

import synth
from oracle import filter as ofilter
from oracle import lanczos as olanczos
from oracle import qr as oqr
from oracle import rr as orr

from gpu_util import U32, U64, col_rel_err, phase_align, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P(gpu):
    import paper_2603_10514_amd as P
    return P


def _interval(lam, L):
    alpha, beta = lam[min(L + 4, lam.size - 2)], lam[-1]
    return 0.5 * (alpha + beta), 0.5 * (beta - alpha), lam[0]


FILTER_CASES = [
    # N, ncols, cplx, degrees kind
    (1000, 60, False, "mixed"),
    (1000, 60, False, "const20"),
    (1000, 61, True, "mixed"),
    (129, 7, False, "mixed"),
    (70, 3, True, "mixed"),
    (517, 1, False, "one"),
    (300, 40, True, "spread"),
]


def _degrees(kind, n, rng):
    if kind == "const20":
        return np.full(n, 20)
    if kind == "one":
        return np.array([1])
    if kind == "spread":
        return np.sort(rng.integers(1, 37, n))
    return np.sort(np.concatenate([[1, 2, 3], rng.integers(1, 37, n - 3)]))


@pytest.mark.parametrize("N,ncols,cplx,kind", FILTER_CASES)
def test_filter_fp64_matches_oracle(P, gpu, N, ncols, cplx, kind):
    print("filter case", N, ncols, cplx, kind, flush=True)
    H, lam = synth.planted_numpy(N, "uniform" if not cplx else "dft", 3, cplx)
    V = synth.start_block(N, ncols, 4, cplx)
    deg = _degrees(kind, ncols, np.random.default_rng(5))
    c, e, g = _interval(lam, ncols)
    ref = ofilter.chebyshev_filter(H, V, deg, c, e, g)
    out = to_host(P.chase_filter(to_dev(H, gpu), to_dev(V, gpu), deg, c, e, g))
    # bound: each of the m steps adds about N u relative to the column scale
    tol = 4.0 * int(deg.max()) * N * U64
    assert col_rel_err(out, ref) <= tol


@pytest.mark.parametrize("N,cplx", [(1000, False), (1000, True), (1100, True), (777, True)])
def test_filter_fp32_matches_oracle(P, gpu, N, cplx):
    """Complex FP32 runs the direct-load loop when rows are 16-byte aligned
    (even N; N = 1100 leaves a partial last K chunk of 12) and the
    register-prefetch loop otherwise (N = 777)."""
    print("fp32 filter case", N, cplx, flush=True)
    ncols = 60
    H, lam = synth.planted_numpy(N, "dft", 6, cplx)
    V = synth.start_block(N, ncols, 7, cplx)
    deg = _degrees("mixed", ncols, np.random.default_rng(8))
    c, e, g = _interval(lam, ncols)
    ref = ofilter.chebyshev_filter(H, V, deg, c, e, g)
    out = to_host(P.chase_filter(to_dev(H, gpu), to_dev(V, gpu), deg, c, e, g,
                                 precision=P.PREC_MIXED))
    # FP32 storage and accumulation: a rounding error of u32 per step and per
    # operand, accumulated over sqrt(N) terms and m steps
    tol = 8.0 * int(deg.max()) * np.sqrt(N) * U32
    err = col_rel_err(out, ref)
    assert err <= tol, (err, tol)


def planted_block(N, L, kappa, seed, cplx):
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((N, L)) + (1j * rng.standard_normal((N, L)) if cplx else 0)
    G2 = rng.standard_normal((L, L)) + (1j * rng.standard_normal((L, L)) if cplx else 0)
    Uo, _ = np.linalg.qr(G1)
    Wo, _ = np.linalg.qr(G2)
    s = np.logspace(0, -np.log10(kappa), L)
    return np.asfortranarray((Uo * s) @ Wo.conj().T)


QR_CASES = [
    ("chol1", 10.0), ("chol2", 10.0), ("chol2", 1e4), ("chol2", 1e7), ("shifted", 1e7),
    ("shifted", 1e11), ("householder", 1e11),
]


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("variant,kappa", QR_CASES)
def test_qr_variant_matches_oracle(P, gpu, variant, kappa, cplx):
    N, L = 1000, 130  # several 64-wide panels, ragged last panel
    print("qr case", variant, kappa, cplx, flush=True)
    X = planted_block(N, L, kappa, 11, cplx)
    Qref, failed_ref = oqr.dynamic_caqr(X, variant)
    Xd = to_dev(X, gpu)
    failed, (fro2, shift) = P.chase_qr_factor(Xd, variant, return_shift=True)
    Q = to_host(Xd)
    assert failed == failed_ref
    if variant == "shifted":
        # the shift the library added (Alg. 3) against the oracle's, and the
        # squared Frobenius norm it was formed from
        assert fro2 == pytest.approx(float(np.sum(np.abs(X) ** 2)), rel=1e-14, abs=0)
        assert shift == pytest.approx(oqr.shift_value(X), rel=1e-14, abs=0)
    else:
        assert np.isnan(fro2) and np.isnan(shift)
    orth = np.linalg.norm(Q.conj().T @ Q - np.eye(L))
    if variant == "chol1":
        assert orth <= 10 * L * kappa**2 * U64
    else:
        assert orth <= 100 * L * U64
    # Q = X R^{-1} is unique up to column phases.  A relative perturbation of
    # X by a few u moves the oracle's own Q by about kappa u (kappa^2 u for a
    # single CholeskyQR pass); the bound allows ten times that, plus L u for
    # the well-conditioned cases
    diff = col_rel_err(phase_align(Q, Qref), Qref)
    amp = kappa**2 if variant == "chol1" else kappa
    print("qr %s kappa %.0e cplx %d: Q diff %.2e = %.2f kappa u" % (
        variant, kappa, cplx, diff, diff / (kappa * U64)), flush=True)
    assert diff <= 10 * (amp + L) * U64
    # span: X - Q Q^H X = (X - Q R) - Q (Q^H Q - I) R, so its relative size is
    # the backward error (a few u) plus the loss of orthogonality; this is
    # what still binds at kappa = 1e11, where the Q comparison above allows
    # 0.1 (the variants' span is exact to rounding whatever kappa is)
    span = np.linalg.norm(X - Q @ (Q.conj().T @ X)) / np.linalg.norm(X)
    print("qr %s kappa %.0e cplx %d: span %.2e orth %.2e" % (variant, kappa, cplx, span, orth),
          flush=True)
    assert span <= orth + 10 * L * U64


@pytest.mark.parametrize("cplx", [False, True])
def test_qr_fallback_to_householder(P, gpu, cplx):
    N, L = 600, 70
    X = planted_block(N, L, 1e17, 12, cplx)
    for variant in ["chol2", "shifted"]:
        Qref, failed_ref = oqr.dynamic_caqr(X, variant)
        Xd = to_dev(X, gpu)
        failed = P.chase_qr_factor(Xd, variant)
        Q = to_host(Xd)
        assert failed and failed_ref
        assert np.linalg.norm(Q.conj().T @ Q - np.eye(L)) <= 100 * L * U64


HH_SHAPES = [
    # N, L, cplx: one column, two one-column panels, N == L, ragged panels,
    # several row blocks of the panel kernel, 254 rows per block (near its
    # LDS limit), and more rows than its 256 blocks hold (one launch per
    # column step instead)
    (300, 1, False), (257, 2, True), (64, 64, False), (96, 96, True), (257, 33, True),
    (1100, 97, False), (5000, 200, True), (65000, 40, True), (70000, 40, False),
    (80000, 40, True),
]


@pytest.mark.parametrize("N,L,cplx", HH_SHAPES)
def test_householder_matches_lapack_convention(P, gpu, N, L, cplx):
    """The blocked Householder QR follows geqrf/orgqr's convention (beta =
    -sign(Re alpha) ||x||, real R diagonal), so its Q equals numpy's
    (LAPACK) Q column by column to rounding, with no phase alignment; two
    runs on the same input are bit-identical (fixed-order reductions)."""
    print("householder case", N, L, cplx, flush=True)
    X = planted_block(N, L, 1e6, 31, cplx)
    Qref = oqr.householder_qr(X)
    Xd = to_dev(X, gpu)
    assert not P.chase_qr_factor(Xd, "householder")
    Q = to_host(Xd)
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(L)) <= 100 * L * U64
    assert col_rel_err(Q, Qref) <= 100 * L * 1e6 * U64
    Xd2 = to_dev(X, gpu)
    P.chase_qr_factor(Xd2, "householder")
    assert np.array_equal(to_host(Xd2), Q)


def test_householder_panel_wait_timeout_is_reported(P, gpu):
    """The failure path of the panel kernel's grid barrier, forced from the
    host: with a one-tick limit the waits give up at once (every block still
    finishes), the QR reports a device error instead of returning a wrong
    Q, and with the limit restored the next factorisation is correct."""
    N, L = 5000, 64  # 40 blocks per panel launch
    print("householder wait time-out case", N, L, flush=True)
    X = planted_block(N, L, 1e3, 33, True)
    try:
        P.chase_set_panel_wait_limit(1)
        Xd = to_dev(X, gpu)
        with pytest.raises(P.ChaseError) as exc:
            P.chase_qr_factor(Xd, "householder")
        assert "timed out" in str(exc.value)
    finally:
        P.chase_set_panel_wait_limit(0)
    Xd = to_dev(X, gpu)
    assert not P.chase_qr_factor(Xd, "householder")
    Q = to_host(Xd)
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(L)) <= 100 * L * U64
    assert col_rel_err(Q, oqr.householder_qr(X)) <= 100 * L * 1e3 * U64


@pytest.mark.parametrize("cplx", [False, True])
def test_householder_rank_deficient(P, gpu, cplx):
    """Zero and repeated columns: the reflector of a zero column is the
    identity (tau = 0); Q stays orthonormal and spans X."""
    N, L = 500, 70
    X = planted_block(N, L, 10.0, 32, cplx)
    X[:, 5] = 0
    X[:, 40] = X[:, 3]
    X[:, 41] = 2 * X[:, 40] - X[:, 7]
    Xd = to_dev(np.asfortranarray(X), gpu)
    P.chase_qr_factor(Xd, "householder")
    Q = to_host(Xd)
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(L)) <= 100 * L * U64
    assert np.linalg.norm(X - Q @ (Q.conj().T @ X)) <= 1e-13 * np.linalg.norm(X)


def _subspace_gap(A, B):
    """sin of the largest principal angle between the column spans of the
    orthonormal A and B (equal widths): ||B - A (A^H B)||_2."""
    return float(np.linalg.norm(B - A @ (A.conj().T @ B), 2))


def _clustered_spectrum(kind, N, rng):
    if kind == "repeated":   # eigenvalues of multiplicity 4 and 7
        lam = np.sort(rng.uniform(-1, 1, N))
        lam[:4] = -1.2
        lam[10:17] = 0.3
        return np.sort(lam)
    if kind == "cluster":    # a dense low cluster with gaps near 1e-9
        lam = np.concatenate([-1.5 + 1e-9 * np.arange(N // 2), rng.uniform(-1, 50, N - N // 2)])
        return np.sort(lam)
    raise ValueError(kind)


@pytest.mark.parametrize("L,cplx,kind", [(40, False, "repeated"), (64, True, "repeated"),
                                         (33, True, "cluster"), (64, False, "cluster")])
def test_rayleigh_ritz_clustered_small(P, gpu, L, cplx, kind):
    """The one-work-group eigensolver (up to 64 columns) on projected
    matrices with repeated and tightly clustered eigenvalues: Ritz values
    against the planted ones, eigenvectors compared by invariant subspace
    (unique only as a subspace inside a cluster), and the library's
    convergence flag (a non-converged solve raises)."""
    print("rr clustered case", L, cplx, kind, flush=True)
    N = 400
    rng = np.random.default_rng(51)
    lam_small = _clustered_spectrum(kind, L, rng)
    # H with an exact invariant subspace Q of dimension L carrying lam_small
    Qf, _ = np.linalg.qr(synth.start_block(N, N, 52, cplx))
    lam = np.concatenate([lam_small, rng.uniform(60, 70, N - L)])
    H = (Qf * lam[None, :]) @ Qf.conj().T
    H = np.asfortranarray(0.5 * (H + H.conj().T))
    # Q spans the same subspace as Qf[:, :L] in a random basis
    W, _ = np.linalg.qr(synth.start_block(L, L, 53, cplx))
    Q = np.asfortranarray(Qf[:, :L] @ W)
    th, V, HV = P.chase_rayleigh_ritz(to_dev(H, gpu), to_dev(Q, gpu))
    scale = float(np.max(np.abs(lam)))
    assert np.max(np.abs(th - lam_small)) <= 100 * N * U64 * scale
    Vh = to_host(V)
    assert np.linalg.norm(Vh.conj().T @ Vh - np.eye(L)) <= 1e-12
    # each group of (numerically) equal eigenvalues spans its planted
    # subspace, to within the perturbation bound u ||H|| / gap (Davis-Kahan)
    # times a factor 1e3 for the rounding of the projection and the solver
    groups = np.split(np.arange(L), np.where(np.diff(lam_small) > 1e-6)[0] + 1)
    for g in groups:
        others = np.delete(lam, g)
        gap = float(np.min(np.abs(others[:, None] - lam_small[g][None, :])))
        assert _subspace_gap(Vh[:, g], Qf[:, g]) <= 1e3 * U64 * scale / gap, (g, gap)
    R = H @ Vh - Vh * th[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-12 * scale


EIG_CASES = [
    # L (order of the projected problem), cplx, spectrum of H
    (25, True, "uniform"), (48, False, "cluster"), (65, True, "uniform"), (65, False, "uniform"),
    (129, False, "uniform"), (300, False, "uniform"),
    (300, True, "repeated"), (700, True, "cluster"), (1300, True, "dft"),
    (1300, False, "cluster"), (1900, True, "dft"),
]


@pytest.mark.parametrize("L,cplx,kind", EIG_CASES)
def test_rayleigh_ritz_eigensolver_large(P, gpu, L, cplx, kind):
    """The library's own eigensolver of the projected matrix above 64 columns
    (Householder reduction to tridiagonal form, divide and conquer, back
    transform) against the oracle's Rayleigh-Ritz (LAPACK eigh): Ritz values
    to 1e-12 ||A||, the projected eigen-residual Q^H (HV - V Theta) and the
    orthogonality of V to a few hundred u, and the invariant subspaces of
    well-separated groups to within the perturbation bound.  The DFT-like
    spectra put most Ritz values in a dense cluster (deflation); the
    repeated one has eigenvalues of multiplicity 5 and 9."""
    print("eigensolver case", L, cplx, kind, flush=True)
    N = L + 100
    rng = np.random.default_rng(61)
    exact = None
    if kind == "cluster":
        # Q spans an exact invariant subspace whose eigenvalues hold a cluster
        # of L / 2 values 1e-9 apart (the deflation of the merges)
        Qf, _ = np.linalg.qr(synth.start_block(N, N, 63, cplx))
        exact = np.sort(np.concatenate([-1.5 + 1e-9 * np.arange(L // 2),
                                        rng.uniform(-1.0, 0.0, L - L // 2)]))
        lam = np.concatenate([exact, rng.uniform(1.0, 50.0, N - L)])
        H = (Qf * lam) @ Qf.conj().T
        H = np.asfortranarray(0.5 * (H + H.conj().T))
        W, _ = np.linalg.qr(synth.start_block(L, L, 65, cplx))
        Q = np.asfortranarray(Qf[:, :L] @ W)
    elif kind == "repeated":
        H, lam = synth.planted_numpy(N, "uniform", 62, cplx)
        Qf, _ = np.linalg.qr(synth.start_block(N, N, 63, cplx))
        lam = np.sort(lam)
        lam[3:8] = lam[3]
        lam[100:109] = lam[100]
        H = np.asfortranarray(0.5 * ((Qf * lam) @ Qf.conj().T + ((Qf * lam) @ Qf.conj().T).conj().T))
    else:
        H, lam = synth.planted_numpy(N, kind, 62, cplx)
    if exact is None:
        Q, _ = np.linalg.qr(synth.start_block(N, L, 64, cplx))
        Q = np.asfortranarray(Q)
    th_ref, V_ref, HV_ref = orr.rayleigh_ritz(H, Q)
    th, V, HV = P.chase_rayleigh_ritz(to_dev(H, gpu), to_dev(Q, gpu))
    Vh, HVh = to_host(V), to_host(HV)
    scale = float(np.max(np.abs(lam)))
    err = float(np.max(np.abs(th - th_ref)))
    resid = float(np.max(np.linalg.norm(Q.conj().T @ (HVh - Vh * th[None, :]), axis=0)))
    orth = float(np.linalg.norm(Vh.conj().T @ Vh - np.eye(L)))
    print("  eig err %.2e resid %.2e orth %.2e (||A|| %.1f)" % (err, resid, orth, scale), flush=True)
    assert err <= 1e-12 * scale
    if exact is not None:
        assert np.max(np.abs(th - exact)) <= 1e-12 * scale
    assert resid <= 300 * L * U64 * scale / 10
    assert orth <= 300 * L * U64
    # invariant subspaces of groups separated by more than 1e-6 ||A||
    groups = np.split(np.arange(L), np.where(np.diff(th_ref) > 1e-6 * scale)[0] + 1)
    worst = 0.0
    for g in groups[:: max(1, len(groups) // 40)]:
        others = np.delete(th_ref, g)
        gap = float(np.min(np.abs(others[:, None] - th_ref[g][None, :]))) if others.size else scale
        worst = max(worst, _subspace_gap(Vh[:, g], V_ref[:, g]) / (1e3 * U64 * scale / gap))
    print("  worst subspace ratio to bound %.3f" % worst, flush=True)
    assert worst <= 1.0


@pytest.mark.parametrize("N,L,cplx", [(1000, 60, False), (600, 37, True), (200, 130, False),
                                      (500, 64, True), (300, 1, False), (400, 65, True)])
def test_rayleigh_ritz_and_residuals(P, gpu, N, L, cplx):
    """Up to 64 columns the projected eigenproblem is solved in one
    work-group (the matrix in LDS), above by the multi-launch solver."""
    H, lam = synth.planted_numpy(N, "uniform", 13, cplx)
    Q, _ = np.linalg.qr(synth.start_block(N, L, 14, cplx))
    Q = np.asfortranarray(Q)
    th_ref, V_ref, HV_ref = orr.rayleigh_ritz(H, Q)
    Hd = to_dev(H, gpu)
    th, V, HV = P.chase_rayleigh_ritz(Hd, to_dev(Q, gpu))
    scale = np.max(np.abs(lam))
    assert np.max(np.abs(th - th_ref)) <= 100 * N * U64 * scale
    Vh = to_host(V)
    # eigenvectors: unique up to phase for the (simple) Ritz values here
    ov = np.abs(np.sum(Vh.conj() * V_ref, axis=0))
    assert np.all(ov >= 1 - 1e-8)
    # residual kernel on identical inputs: element by element
    r_ref = orr.residual_norms(HV_ref, V_ref, th_ref)
    r = P.chase_residuals(to_dev(HV_ref, gpu), to_dev(V_ref, gpu), th_ref)
    assert np.max(np.abs(r - r_ref) / r_ref) <= 1e-12
    # and on the GPU's own RR output
    r2 = P.chase_residuals(HV, V, th)
    assert np.max(np.abs(r2 - r_ref)) <= 1e-10 * scale


@pytest.mark.parametrize("N,cplx,nvec", [(1000, False, 1), (700, True, 1), (1000, False, 4),
                                         (1537, True, 4), (333, False, 3), (2100, True, 8),
                                         (4096, False, 2), (4097, True, 2)])
def test_lanczos_matches_oracle(P, gpu, N, cplx, nvec):
    """nvec runs advanced as one block (the N x N product streams H once for
    all of them) against the oracle's runs one by one; sizes span one and
    several row blocks and column splits of the product, with ragged ends,
    and both forms of the step after the product (one work-group per run up
    to order 4096, wide launches above)."""
    print("lanczos case", N, cplx, nvec, flush=True)
    H, lam = synth.planted_numpy(N, "dft", 15, cplx)
    V0 = synth.lanczos_starts(N, nvec, 16, cplx)
    runs = [olanczos.lanczos_tridiag(H, V0[:, r], 40) for r in range(nvec)]
    bounds_ref = olanczos.lanczos_bounds(H, 60, V0, 40)
    a, b, bounds = P.chase_lanczos(to_dev(H, gpu), to_dev(V0, gpu), 40, 60)
    scale = np.max(np.abs(lam))
    assert a.shape == (nvec, 40) and b.shape == (nvec, 40)
    for r, (a_ref, b_ref) in enumerate(runs):
        # Lanczos with full reorthogonalisation is forward stable here; the
        # coefficients drift by a few ulps per step
        assert np.max(np.abs(a[r] - a_ref)) <= 1e-9 * scale, r
        assert np.max(np.abs(b[r] - b_ref)) <= 1e-9 * scale, r
    assert np.allclose(bounds, bounds_ref, rtol=1e-8, atol=1e-9 * scale)
    assert bounds[2] >= lam[-1]


@pytest.mark.parametrize("N,cplx", [(20000, True), (10000, False)])
def test_lanczos_first_step_full_size(P, gpu, N, cplx):
    """At full size: the first coefficients of each run against torch's own
    matrix product, alpha_0 = v^H H v and beta_0 = ||H v - alpha_0 v|| for
    the normalised start vector v, and the upper-bound property."""
    import torch
    print("lanczos full-size case", N, cplx, flush=True)
    Hd, lam = synth.planted_torch(N, "dft", 41, cplx, gpu)
    V0 = synth.start_block_torch(N, 4, 42, cplx, gpu)
    a, b, bounds = P.chase_lanczos(Hd, V0, 3, int(0.065 * N))
    torch.cuda.synchronize()
    v = V0 / torch.linalg.vector_norm(V0, dim=0, keepdim=True)
    Hv = Hd @ v
    a0 = torch.real(torch.sum(v.conj() * Hv, dim=0))
    b0 = torch.linalg.vector_norm(Hv - v * a0, dim=0)
    scale = float(np.max(np.abs(lam)))
    assert np.max(np.abs(a[:, 0] - a0.cpu().numpy())) <= 1e-12 * scale
    assert np.max(np.abs(b[:, 0] - b0.cpu().numpy())) <= 1e-12 * scale
    assert bounds[0] >= lam[0] - 1e-9 * scale


@pytest.mark.parametrize("N,ncols,cplx,maxdeg", [(3000, 1300, True, 6), (2500, 700, False, 5),
                                                 (20000, 64, True, 3), (9000, 200, True, 4),
                                                 (6000, 250, False, 3), (6000, 300, False, 3),
                                                 (4101, 1030, False, 2)])
def test_filter_remainder_split_shapes(P, gpu, N, ncols, cplx, maxdeg):
    """Shapes whose tile count leaves a partial last wave (or less than one
    wave): the remainder tiles run split along K plus a reduce kernel; the
    result must still match the oracle column by column.  The real cases at
    N >= 4096 cover both real tile sizes of the direct-load path (250
    columns: 128 x 128; 300 columns: 64 x 64) and, with the odd leading
    dimension of N = 4101, the register-prefetch path it falls back to."""
    import torch
    print("remainder-split case", N, ncols, cplx, flush=True)
    rng = np.random.default_rng(31)
    if N <= 3000:
        H, lam = synth.planted_numpy(N, "dft", 32, cplx)
        Hd = to_dev(H, gpu)
    else:
        Hd, lam = synth.planted_torch(N, "dft", 32, cplx, gpu)
        H = np.ascontiguousarray(Hd.T.cpu().numpy()).T
    V = synth.start_block(N, ncols, 33, cplx)
    deg = np.sort(rng.integers(1, maxdeg + 1, ncols))
    c, e, g = _interval(lam, ncols)
    out = to_host(P.chase_filter(Hd, to_dev(V, gpu), deg, c, e, g))
    cols = np.unique(np.linspace(0, ncols - 1, 12).astype(int))
    ref = ofilter.chebyshev_filter(H, V[:, cols], deg[cols], c, e, g)
    assert col_rel_err(out[:, cols], ref) <= 4.0 * maxdeg * N * U64


def test_lanczos_wait_timeout_is_reported(P, gpu):
    """The failure path of the one-launch Lanczos's grid barriers, forced
    from the host: with a one-tick limit the waits give up at once (every
    block still finishes its bounded steps), the call reports a device error
    instead of returning wrong coefficients, and with the limit restored the
    next run matches the oracle."""
    N, nvec = 1000, 4  # one launch of 63 blocks
    print("lanczos wait time-out case", N, nvec, flush=True)
    H, lam = synth.planted_numpy(N, "dft", 15, False)
    V0 = synth.lanczos_starts(N, nvec, 16, False)
    try:
        P.chase_set_panel_wait_limit(1)
        with pytest.raises(P.ChaseError) as exc:
            P.chase_lanczos(to_dev(H, gpu), to_dev(V0, gpu), 40, 60)
        assert "timed out" in str(exc.value)
    finally:
        P.chase_set_panel_wait_limit(0)
    a, b, _ = P.chase_lanczos(to_dev(H, gpu), to_dev(V0, gpu), 40, 60)
    a_ref, b_ref = olanczos.lanczos_tridiag(H, V0[:, 0], 40)
    scale = np.max(np.abs(lam))
    assert np.max(np.abs(a[0] - a_ref)) <= 1e-9 * scale
    assert np.max(np.abs(b[0] - b_ref)) <= 1e-9 * scale


def test_lanczos_long_runs_take_the_per_step_launches(P, gpu):
    """Bases too large for one block's LDS (8 complex runs of 100 steps: 16
    rows x 101 vectors x 8 runs) leave the one-launch form for one launch
    per step; the coefficients must still match the oracle's runs."""
    N, nvec, steps = 600, 8, 100
    print("lanczos per-step case", N, nvec, steps, flush=True)
    H, lam = synth.planted_numpy(N, "dft", 15, True)
    V0 = synth.lanczos_starts(N, nvec, 16, True)
    a, b, _ = P.chase_lanczos(to_dev(H, gpu), to_dev(V0, gpu), steps, 60)
    scale = np.max(np.abs(lam))
    for r in range(nvec):
        a_ref, b_ref = olanczos.lanczos_tridiag(H, V0[:, r], steps)
        assert np.max(np.abs(a[r] - a_ref)) <= 1e-9 * scale, r
        assert np.max(np.abs(b[r] - b_ref)) <= 1e-9 * scale, r
