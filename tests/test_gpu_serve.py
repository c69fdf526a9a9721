"""Serving form: continuous batching of correlated eigenproblem sequences on
asynchronous handles.  Each result must be the same alone and in the mix;
eigenvalues are checked against a CPU full diagonalisation of every H_j and,
step by step, against the oracle's solve of the same H_j from the same
(warm) start block and bounds; the scheduler must never admit beyond its HBM
budget, and a request that fits may overtake one that does not only a
bounded number of times."""
import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu


def _requests(gpu, Ns, steps=3, arrival_gap=0.0):
    from paper_2603_10514_amd import serve
    import synth
    out = []
    for i, N in enumerate(Ns):
        nev, nex = serve.request_shape(N)
        H0, lam = synth.planted_torch(N, "dft", 500 + i, True, gpu)
        out.append(serve.Request(rid=i, arrival=i * arrival_gap, N=N, nev=nev, nex=nex, H0=H0,
                                 lam=lam, steps=steps, seed=40 + i))
    return out


def _fresh(r):
    from paper_2603_10514_amd import serve
    return serve.Request(rid=r.rid, arrival=0.0, N=r.N, nev=r.nev, nex=r.nex, H0=r.H0, lam=r.lam,
                         steps=r.steps, eps=r.eps, seed=r.seed)


def test_alone_equals_mix_and_matches_dense_eigensolver(gpu):
    import torch
    from paper_2603_10514_amd import serve
    Ns = [420, 640, 880, 530]
    reqs = _requests(gpu, Ns)
    srv = serve.Server(n_slots=3, N_max=900, device=gpu)
    mix = srv.run(reqs)
    srv.close()
    for r in mix:
        assert all(st == 0 for st in r.status), r.status
        assert len(r.evals) == r.steps
    # every step against a dense eigensolver of the same H_j (CPU)
    for r in mix:
        H = r.H0.clone()
        for j in range(r.steps):
            if j > 0:
                H += serve.perturbation(r.N, r.seed, j, r.eps, H.dtype, gpu)
            w = sla.eigh(H.cpu().numpy(), eigvals_only=True, subset_by_index=[0, r.nev - 1])
            scale = float(np.max(np.abs(r.lam)))
            assert np.max(np.abs(r.evals[j] - w)) <= 1e-10 * scale, (r.rid, j)
            assert np.all(r.resid[j] < 1e-10)
        # warm steps are cheaper than the cold one
        assert r.infos[-1]["matvecs"] < r.infos[0]["matvecs"]
    # each request alone, one slot, same inputs
    for r in mix:
        srv1 = serve.Server(n_slots=1, N_max=900, device=gpu)
        (alone,) = srv1.run([_fresh(r)])
        srv1.close()
        for j in range(r.steps):
            assert np.max(np.abs(alone.evals[j] - r.evals[j])) <= 1e-12 * float(np.max(np.abs(r.lam)))
            assert alone.infos[j]["iters"] == r.infos[j]["iters"]
    torch.cuda.synchronize()


def test_admission_respects_hbm_budget(gpu):
    from paper_2603_10514_amd import serve
    Ns = [700, 760, 820]
    reqs = _requests(gpu, Ns, steps=2)
    big = max(serve.data_bytes(r.N, r.nev, r.nex) for r in reqs)
    # room for one request at a time although three slots are free
    srv = serve.Server(n_slots=3, N_max=900, hbm_budget=int(1.5 * big), device=gpu)
    done = srv.run(reqs)
    srv.close()
    assert srv.peak_used <= srv.budget
    order = sorted(done, key=lambda r: r.t_admit)
    for a, b in zip(order, order[1:]):
        assert b.t_admit >= a.t_done - 1e-6
    assert all(all(st == 0 for st in r.status) for r in done)


def test_warm_started_steps_match_oracle(gpu):
    """Two small sequences, every step against the oracle: the server keeps
    a host copy of each step's start block (the Gaussian block of step 0,
    the previous step's subspace afterwards) and bounds (step 0: the
    library's Lanczos bounds; afterwards the previous ones widened by the
    perturbation bound), and the oracle solves the same H_j from them (Alg. 1
    with its optional start block and bounds, the warm start of Sec. 1.2).
    The server filters in FP32, the oracle in FP64: eigenvalues agree to
    1e-10 and iteration counts to within one."""
    import torch
    from paper_2603_10514_amd import serve
    from oracle import solver as osolver
    reqs = _requests(gpu, [360, 520], steps=3)
    srv = serve.Server(n_slots=2, N_max=600, device=gpu, capture=True)
    done = srv.run(reqs)
    srv.close()
    for r in done:
        assert len(r.captured) == r.steps
        H = r.H0.clone()
        scale = float(np.max(np.abs(r.lam)))
        for j in range(r.steps):
            if j > 0:
                H += serve.perturbation(r.N, r.seed, j, r.eps, H.dtype, gpu)
            torch.cuda.synchronize()
            Hn = np.ascontiguousarray(H.T.cpu().numpy()).T
            V0, b = r.captured[j]
            print("serve oracle case rid %d N %d step %d bounds %s" % (r.rid, r.N, j, b), flush=True)
            ref = osolver.chase_solve(Hn, r.nev, r.nex, 20, 1e-10, V0=V0, bounds=b, min_deg=10,
                                      max_deg=36)
            assert ref.converged == r.nev and r.status[j] == 0
            assert np.max(np.abs(r.evals[j] - ref.evals)) <= 1e-10 * scale, (r.rid, j)
            assert np.max(np.abs(r.evals[j] - ref.evals) / np.abs(ref.evals)) <= 1e-10
            assert abs(r.infos[j]["iters"] - ref.iters) <= 1, (r.infos[j]["iters"], ref.iters)
            if j > 0:  # warm steps start from the previous subspace and bounds
                assert b[0] < r.evals[j][0] and b[2] > b[1]


def test_bypass_admission_is_bounded(gpu):
    """A large request that does not fit next to a running one is overtaken
    by smaller ones at most max_bypass times; then it is admitted before
    any later request, as soon as the memory frees up."""
    from paper_2603_10514_amd import serve
    Ns = [700, 880, 400, 420, 440, 460, 480]
    reqs = _requests(gpu, Ns, steps=1, arrival_gap=0.0)
    big = serve.data_bytes(880, *serve.request_shape(880))
    first = serve.data_bytes(700, *serve.request_shape(700))
    small = max(serve.data_bytes(n, *serve.request_shape(n)) for n in Ns[2:])
    # the 880 request fits only alone; the small ones fit beside the 700 one
    budget = max(big, first + small) + small // 2
    assert first + big > budget
    srv = serve.Server(n_slots=2, N_max=900, hbm_budget=budget, device=gpu, max_bypass=2)
    done = srv.run(reqs)
    srv.close()
    assert srv.peak_used <= srv.budget
    assert all(all(st == 0 for st in r.status) for r in done)
    by_rid = {r.rid: r for r in done}
    big_req = by_rid[1]
    assert big_req.bypassed <= 2
    overtook = [r for r in done if r.rid > 1 and r.t_admit < big_req.t_admit]
    assert len(overtook) == big_req.bypassed
    # nothing that arrived after it was admitted once its bypass budget ran out
    later = [r for r in done if r.rid > 1 and r.t_admit > big_req.t_admit]
    assert len(overtook) + len(later) == len(Ns) - 2
