"""Continuous-batching serving loop over asynchronous solver handles.

A request is a correlated sequence of Hermitian eigenproblems
H_{j+1} = H_j + eps * E_j (E_j Hermitian Gaussian, E|g|^2 = 1, scaled by
1/(2 sqrt(N))), each solved for the nev lowest pairs and warm-started from the
previous problem's subspace, which stays in device memory (the warm start of
Sec. 1.2 of the paper).  The scheduler:

* keeps a queue of arrived requests (arrival order) and a fixed set of
  slots, each owning a library handle (own stream, workspace sized for the
  largest problem, host worker thread), so solves of different requests
  overlap on the device;
* admits into a free slot the oldest waiting request whose device memory
  (working matrix, perturbation scratch, search block) fits the HBM budget:
  a later request may overtake an older one that does not fit, but only
  `max_bypass` times, after which the oldest one is admitted first (no
  starvation);
* keeps an admitted request in its slot for all its steps (continuous
  batching: a slot frees, the next request enters while the others run);
* records, per request, arrival-to-completion latency and every step's
  eigenvalues, residuals and timings.

Only the eigensolver's work runs in the HIP library; torch provides the
device buffers, the perturbation matrices and the stream for the update.
"""
import math
import time
from dataclasses import dataclass, field

import numpy as np

import paper_2603_10514_amd as P

GIB = 1 << 30


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    N: int
    nev: int
    nex: int
    H0: object              # column-major device tensor (complex128 or float64)
    lam: np.ndarray         # planted spectrum of H0 (for checks)
    steps: int = 5
    eps: float = 1e-3
    seed: int = 0
    # results
    bypassed: int = 0       # times a later request was admitted before this one
    captured: list = field(default_factory=list)  # (V0, bounds) per step, capture mode
    t_admit: float = None
    t_done: float = None
    evals: list = field(default_factory=list)
    resid: list = field(default_factory=list)
    infos: list = field(default_factory=list)
    status: list = field(default_factory=list)


def request_shape(N):
    """nev = 5% of N, nex = max(20, 1.5% of N)."""
    return max(1, int(round(0.05 * N))), max(20, int(round(0.015 * N)))


def data_bytes(N, nev, nex, cplx=True):
    es = 16 if cplx else 8
    return es * (3 * N * N + N * (nev + nex))  # H_j, E_j and its Gaussian, block


class Slot:
    """One concurrent execution slot: a library handle and a torch stream."""

    def __init__(self, idx, handle, ws_bytes, stream):
        self.idx = idx
        self.handle = handle
        self.ws_bytes = ws_bytes
        self.stream = stream
        self.req = None
        self.step = 0
        self.need = 0
        self.pending = None
        self.Hk = None
        self.evecs = None
        self.bounds = None
        self.t_step = 0.0


class Server:
    def __init__(self, n_slots=4, N_max=25000, nev_max=None, nex_max=None, precision=P.PREC_MIXED,
                 hbm_budget=None, reserve=16 * GIB, degree=20, tol=1e-10, min_deg=10, max_deg=36,
                 device="cuda:0", cplx=True, max_bypass=4, capture=False):
        import torch
        self.device = torch.device(device)
        self.cplx = cplx
        nev_d, nex_d = request_shape(N_max)
        nev_max = nev_max or nev_d
        nex_max = nex_max or nex_d
        self.opts_tmpl = dict(precision=precision, min_deg=min_deg, max_deg=max_deg)
        o = P.opts_default(**self.opts_tmpl)
        o.dtype = P.COMPLEX128 if cplx else P.REAL64
        self.slots = [Slot(i, P.Handle(N_max, nev_max, nex_max, o),
                           P.chase_workspace_bytes(N_max, nev_max, nex_max, o.dtype, o.precision),
                           torch.cuda.Stream(device=self.device)) for i in range(n_slots)]
        free, total = torch.cuda.mem_get_info(self.device)
        # the slots' workspaces are already allocated: the budget covers
        # request data on top of them
        self.budget = hbm_budget if hbm_budget is not None else max(0, free - reserve)
        self.used = 0
        self.peak_used = 0
        self.degree, self.tol = degree, tol
        self.N_max, self.nev_max, self.nex_max = N_max, nev_max, nex_max
        self.max_bypass = max_bypass
        # capture: keep a host copy of every step's start block and bounds
        # (for checking the steps one by one against a reference solver)
        self.capture = capture
        self.log = []

    # ------------------------------------------------------------------ API
    def run(self, requests, clock=None, progress=None):
        """Serve requests (sorted by arrival) until all have finished.
        Returns the list of requests with their results filled in;
        progress(msg), if given, is called as each request finishes."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if r.N > self.N_max or r.nev > self.nev_max or r.nex > self.nex_max:
                raise ValueError("request %d larger than the server's maximum shape" % r.rid)
            if data_bytes(r.N, r.nev, r.nex, self.cplx) > self.budget:
                raise ValueError("request %d can never fit the HBM budget" % r.rid)
        import torch
        torch.cuda.synchronize(self.device)  # inputs generated on other streams
        t0 = time.perf_counter() if clock is None else clock
        waiting = []
        nxt = 0
        done = 0
        while done < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            progressed = False
            # completions
            for s in self.slots:
                if s.pending is None:
                    continue
                st = s.handle.query()
                if st == P.CHASE_EBUSY:
                    continue
                r = s.req
                self._finish_step(s, st, time.perf_counter() - t0)
                progressed = True
                if s.req is None:
                    done += 1
                    if progress:
                        progress("request %d done (N=%d): latency %.2f s, %d/%d finished"
                                 % (r.rid, r.N, r.t_done - r.arrival, done, len(reqs)))
                elif progress:
                    progress("request %d (N=%d) step %d done" % (r.rid, r.N, s.step))
            # admission: the oldest request that fits, with bounded bypass
            for s in self.slots:
                if s.req is not None or not waiting:
                    continue
                pick = self._pick(waiting)
                if pick is None:
                    break
                r = waiting.pop(pick)
                for older in waiting[:pick]:
                    older.bypassed += 1
                self._admit(s, r, data_bytes(r.N, r.nev, r.nex, self.cplx),
                            time.perf_counter() - t0)
                progressed = True
            if not progressed:
                if nxt < len(reqs) and not waiting and all(s.req is None for s in self.slots):
                    time.sleep(max(0.0, min(0.01, reqs[nxt].arrival - now)))
                else:
                    time.sleep(0.0005)
        return reqs

    def close(self):
        for s in self.slots:
            s.handle.close()

    def _pick(self, waiting):
        """Index of the request to admit next, or None.  The oldest waiting
        request goes first when it fits; a later one that fits may overtake
        it unless the oldest has already been overtaken max_bypass times."""
        for i, r in enumerate(waiting):
            if self.used + data_bytes(r.N, r.nev, r.nex, self.cplx) <= self.budget:
                return i
            if r.bypassed >= self.max_bypass:
                return None  # hold the memory that frees up for this one
        return None

    # ------------------------------------------------------------- internals
    def _admit(self, s, r, need, now):
        import torch
        r.t_admit = now
        s.req = r
        s.step = 0
        s.need = need
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        with torch.cuda.stream(s.stream):
            s.Hk = torch.empty_strided(r.H0.shape, r.H0.stride(), dtype=r.H0.dtype,
                                       device=self.device)
            s.Hk.copy_(r.H0)
            # Gaussian start block of the first problem (Alg. 1's random
            # V0): real N(0,1), complex (N(0,1) + i N(0,1)) / sqrt(2)
            g = torch.Generator(device=self.device)
            g.manual_seed(int(r.seed) * 7919 + 1)
            s.evecs = torch.randn((r.nev + r.nex, r.N), dtype=r.H0.dtype, device=self.device,
                                  generator=g).T
        s.bounds = None
        self._launch(s)

    def _perturb(self, s):
        """H_{j+1} = H_j + eps * E_j on the slot's torch stream."""
        import torch
        r = s.req
        with torch.cuda.stream(s.stream):
            E = perturbation(r.N, r.seed, s.step, r.eps, r.H0.dtype, self.device)
            s.Hk.add_(E)
            del E

    def _launch(self, s):
        import torch
        r = s.req
        if s.step > 0:
            self._perturb(s)
        s.stream.synchronize()  # the handle's stream starts after the update
        o = P.opts_default(**self.opts_tmpl)
        o.seed = r.seed * 7919 + 1
        o.warm_start = 1  # step 0: the Gaussian block drawn at admission
        if s.step > 0:
            # warm start: the previous subspace and bounds widened by a bound
            # on ||eps E||_2 (eigenvalues move by at most that, Weyl); the
            # Gaussian E of the perturbation has ||E||_2 close to sqrt(2),
            # taken four times over
            o.have_bounds = 1
            o.lambda_1, o.lambda_l, o.lambda_max = P.chase_sequence_bounds(
                s.bounds, 4.0 * r.eps * math.sqrt(2.0))
        if self.capture:
            V0 = np.ascontiguousarray(s.evecs.T.cpu().numpy()).T
            r.captured.append([V0, (o.lambda_1, o.lambda_l, o.lambda_max)
                               if s.step > 0 else None])
        s.pending = s.handle.solve_async(s.Hk, r.nev, r.nex, self.degree, self.tol, s.evecs, o)
        s.t_step = time.perf_counter()

    def _finish_step(self, s, status, now):
        r = s.req
        evals, resid, info = s.pending
        s.pending = None
        inf = P._info_dict(info)
        inf["wall"] = time.perf_counter() - s.t_step
        r.evals.append(evals.copy())
        r.resid.append(resid.copy())
        r.infos.append(inf)
        r.status.append(status)
        if self.capture and r.captured[-1][1] is None:
            # the first problem's bounds came from the library's Lanczos runs
            r.captured[-1][1] = (inf["lambda_1"], inf["lambda_l"], inf["lambda_max"])
        # bounds for the next problem: lowest and largest Ritz values of the
        # search space and the upper bound of this one
        s.bounds = (float(evals[0]), float(inf["ritz_max"]), float(inf["lambda_max"]))
        s.step += 1
        if s.step < r.steps and status in (P.CHASE_OK, P.CHASE_NOT_CONVERGED):
            self._launch(s)
            return
        r.t_done = now
        s.req = None
        s.Hk = None
        s.evecs = None
        self.used -= s.need


def make_stream(n_requests, rate, N_lo, N_hi, seed, device, cplx=True, steps=5, eps=1e-3,
                progress=None):
    """Poisson arrivals at `rate` per second with N log-uniform in
    [N_lo, N_hi]; the first matrix of each request is generated up front in
    device memory (DFT-like planted spectrum, scaled to N)."""
    import synth
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        N = int(round(math.exp(rng.uniform(math.log(N_lo), math.log(N_hi)))))
        nev, nex = request_shape(N)
        H0, lam = synth.planted_torch(N, "dft", 10_000 + i, cplx, device)
        out.append(Request(rid=i, arrival=t, N=N, nev=nev, nex=nex, H0=H0, lam=lam, steps=steps,
                           eps=eps, seed=100 + i))
        if progress:
            progress("generated request %d: N=%d nev=%d nex=%d" % (i, N, nev, nex))
    return out


def perturbation(N, seed, step, eps, dtype, device):
    """The E_j that the server adds at `step` (for checks outside it)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000 + step)
    G = torch.randn((N, N), dtype=dtype, device=device, generator=g)
    return (G + G.conj().T) * (eps / (2.0 * math.sqrt(N)))


def latency_stats(reqs):
    lat = np.array([r.t_done - r.arrival for r in reqs])
    return dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                mean=float(lat.mean()), max=float(lat.max()))
