"""Serving form: continuous batching of correlated eigenproblem sequences on
asynchronous handles.  Each result must be the same alone and in the mix;
eigenvalues are checked against a CPU full diagonalisation of every H_j; the
scheduler must never admit beyond its HBM budget."""
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
