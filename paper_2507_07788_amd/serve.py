"""Serving loop: many resident bases (model-order-reduction sessions) on one GPU.

Each session keeps its basis Q (m x cap) and R (cap x cap) in HBM between
requests.  A request either orthogonalises a new matrix for its session
(sqr_orth, which replaces the session's basis) or appends a block of columns
to the session's basis (sqr_append, Algorithm 2 / Prop. 2.1).

Scheduling (continuous, not a queue drained in order):
  * worker threads, each with its own HIP stream, take the oldest request that
    has arrived, whose input is ready, whose session has no request in flight
    (a session's requests run in arrival order) and whose new memory fits the
    HBM budget;
  * with batch = B, a worker takes up to B such requests at once and runs them
    as one sqr_batch call: the passes of all of them advance together and each
    kernel launch covers every request of the batch (uneven m, n and p);
  * a request that arrives while others run is admitted as soon as a worker and
    memory are free, and its kernels then run on the device concurrently with
    the kernels of the requests already in flight;
  * between requests a session's handle is parked (sqr_park): its scratch
    workspace goes back to the library pool and only Q and R stay resident.

Inputs are produced ahead of their arrival times by a generator thread on its
own stream (bounded look-ahead).  Latency is measured from the request's
arrival to the point where the request's stream has finished its work; an
input that was not ready at arrival is charged to the latency (and counted in
the summary as a late input).

Only the scheduling lives here; every step of the numerical method runs in the
HIP kernels behind the C ABI.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import sys
import threading
import time

import numpy as np
import torch

from . import Basis, colmajor, sqr_append, sqr_batch, sqr_default_opts, sqr_free, sqr_orth, sqr_park


@dataclasses.dataclass
class Request:
    rid: int
    session: int
    kind: str            # "orth" or "append"
    m: int
    cols: int            # n for "orth", p for "append"
    cap: int             # "orth": columns to reserve for the appends that follow
    kappa: float
    arrival: float = 0.0  # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    session: int
    kind: str
    status: int
    passes: int
    arrival: float
    ready: float
    start: float
    end: float
    bytes: float          # algorithmic HBM bytes of the request

    @property
    def latency(self) -> float:
        return self.end - self.arrival


def request_bytes(kind: str, m: int, q: int, p: int, passes: int) -> float:
    """Algorithmic bytes: CholQR with x passes moves (1 + 2x) m n words; an
    append with x iterations moves m [(q + p) + x (q + 2p)] words."""
    if kind == "orth":
        return 8.0 * m * p * (1 + 2 * passes)
    return 8.0 * m * ((q + p) + passes * (q + 2 * p))


_V_CACHE: dict = {}


def _rotation(k: int, device) -> torch.Tensor:
    """V of the input recipe for width k: the Q factor of a k x k Gaussian
    drawn from a fixed seed per k, formed once and kept (a small QR per
    request would cap the rate at which inputs can be synthesised)."""
    key = (k, str(device))
    V = _V_CACHE.get(key)
    if V is None:
        gen = torch.Generator(device=device)
        gen.manual_seed(7919 * 1000 + k)
        V, _ = torch.linalg.qr(torch.randn((k, k), generator=gen, device=device, dtype=torch.float64))
        _V_CACHE[key] = V
    return V


def make_input(req: Request, seed: int, device="cuda") -> torch.Tensor:
    """Seeded synthetic input of a request: G diag(s) V^T / sqrt(m) with G
    Gaussian (m x k, from the request's seed), V the Q factor of a Gaussian
    k x k matrix (one per width k) and s log-spaced from 1 to 1/kappa, FP64,
    column-major (k = n or p).  G / sqrt(m) has orthonormal columns up to
    O(sqrt(k/m)), so cond(A) is kappa to that accuracy."""
    k = req.cols
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    V = _rotation(k, device)
    s = torch.logspace(0.0, -math.log10(req.kappa), k, device=device, dtype=torch.float64) \
        if k > 1 else torch.ones(1, device=device, dtype=torch.float64)
    SVt = (s[:, None] * V.t()).contiguous() / math.sqrt(req.m)
    out = colmajor(req.m, k, device=device)
    G = torch.randn((k, req.m), generator=gen, device=device, dtype=torch.float64).t()
    torch.matmul(G, SVt, out=out)
    return out


def synthetic_workload(n_requests: int, n_sessions: int, seed: int = 4,
                       m_range=(10_000, 2_000_000), n_range=(8, 256), p_range=(1, 16),
                       kappa_range=(1e2, 1e12), orth_share: float = 0.25,
                       max_cols: int = 512):
    """Requests of the serving workload (arrival times filled in later).

    Sessions draw m log-uniform in m_range; a session's first request is an
    orthogonalisation, later ones are orthogonalisations with probability
    orth_share (n uniform in n_range) and appends otherwise (p uniform in
    p_range); an append that would take the basis past max_cols columns
    becomes an orthogonalisation.  Requests of the sessions interleave in a
    seeded random order; each orthogonalisation reserves room for exactly the
    appends that follow it."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, n_requests, n_sessions])))
    lo, hi = np.log10(m_range[0]), np.log10(m_range[1])
    ms = [int(10 ** g.uniform(lo, hi)) for _ in range(n_sessions)]
    per = [n_requests // n_sessions + (1 if i < n_requests % n_sessions else 0) for i in range(n_sessions)]
    plans = []
    for sidx in range(n_sessions):
        ops, width = [], 0
        for j in range(per[sidx]):
            kappa = 10 ** g.uniform(np.log10(kappa_range[0]), np.log10(kappa_range[1]))
            if j == 0 or g.uniform() < orth_share:
                n = int(min(g.integers(n_range[0], n_range[1] + 1), ms[sidx]))
                ops.append(["orth", n, kappa])
                width = n
            else:
                p = int(g.integers(p_range[0], p_range[1] + 1))
                if width + p > min(max_cols, ms[sidx]):
                    n = int(min(g.integers(n_range[0], n_range[1] + 1), ms[sidx]))
                    ops.append(["orth", n, kappa])
                    width = n
                else:
                    ops.append(["append", p, kappa])
                    width += p
        plans.append(ops)
    # capacity of each orth = its n plus the appends up to the next orth
    order = []
    for sidx, ops in enumerate(plans):
        caps = [0] * len(ops)
        for j in range(len(ops) - 1, -1, -1):
            if ops[j][0] == "orth":
                extra, k = 0, j + 1
                while k < len(ops) and ops[k][0] == "append":
                    extra += ops[k][1]
                    k += 1
                caps[j] = ops[j][1] + extra
        for j, (kind, c, kappa) in enumerate(ops):
            order.append((sidx, kind, c, caps[j], kappa))
    keys = g.permutation(len(order))
    # keep each session's requests in plan order while interleaving sessions
    by_session = collections.defaultdict(list)
    for item in order:
        by_session[item[0]].append(item)
    slots = sorted(range(len(order)), key=lambda i: keys[i])
    seq_sessions = [order[i][0] for i in slots]
    reqs, nxt = [], collections.Counter()
    for rid, sidx in enumerate(seq_sessions):
        item = by_session[sidx][nxt[sidx]]
        nxt[sidx] += 1
        reqs.append(Request(rid=rid, session=sidx, kind=item[1], m=ms[sidx], cols=item[2],
                            cap=item[3], kappa=item[4]))
    return reqs


def poisson_arrivals(reqs, rate_per_s: float, seed: int = 5):
    """Fill in Poisson arrival times (exponential gaps at the given rate)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, len(reqs)])))
    t = 0.0
    for r in reqs:
        t += g.exponential(1.0 / rate_per_s)
        r.arrival = t
    return reqs


class _Session:
    def __init__(self, sid: int):
        self.sid = sid
        self.basis: Basis | None = None
        self.bytes = 0
        self.busy = False
        self.queue = collections.deque()


class Server:
    """Runs a list of requests with `workers` concurrent streams under an HBM
    budget; returns one Result per request.  `batch` > 0 runs up to that many
    requests per library call (sqr_batch).  `keep` maps a session id to a
    callback that receives (Q, R) on the host after the session's last request
    (used by tests)."""

    def __init__(self, workers: int = 4, budget_bytes: float | None = None,
                 lookahead_bytes: float = 8e9, opts=None, keep=None, progress: int = 0,
                 batch: int = 0):
        self.workers = workers
        self.batch = batch         # 0: one library call per request; B: up to B per sqr_batch
        self.progress = progress   # print a line to stderr every `progress` results
        if budget_bytes is None:
            # resident bases may take 80 % of the memory that is free now (the
            # caching allocator's idle blocks returned first), less a reserve
            # for inputs in flight, the library's workspaces and the runtime's
            # scratch: a dispatch whose scratch cannot be allocated aborts the
            # queue (HSA_STATUS_ERROR_OUT_OF_RESOURCES)
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = 0.8 * free - lookahead_bytes - 8e9
        self.budget = budget_bytes
        self.lookahead = lookahead_bytes
        self.opts = opts if opts is not None else sqr_default_opts()
        self.keep = keep or {}

    # -- generator -----------------------------------------------------------
    def _generate(self, reqs, seeds):
        stream = torch.cuda.Stream()
        for r in reqs:
            need = 8.0 * r.m * r.cols
            with self.cv:
                while not self.stop and self.inflight_inputs + need > self.lookahead \
                        and self.inflight_inputs > 0:
                    self.cv.wait(0.05)
                if self.stop:
                    return
                self.inflight_inputs += need
            with torch.cuda.stream(stream):
                X = make_input(r, seeds[r.rid])
                ev = torch.cuda.Event()
                ev.record(stream)
            ev.synchronize()
            with self.cv:
                self.inputs[r.rid] = (X, time.perf_counter() - self.t0)
                self.cv.notify_all()

    # -- scheduling ----------------------------------------------------------
    def _pick(self, now):
        """Oldest arrived request with its input ready, an idle session and
        memory to spare; None if there is none."""
        for s in self.waiting_sessions():
            sess = self.sessions[s]
            if sess.busy or not sess.queue:
                continue
            r = sess.queue[0]
            if r.arrival > now or r.rid not in self.inputs:
                continue
            grow = 0                   # an append needs no new resident memory
            if r.kind == "orth":
                grow = 8 * (r.m * r.cap + r.cap * r.cap) - sess.bytes
            # admit when it fits, and always when nothing is in flight (progress)
            if grow > 0 and self.resident + grow > self.budget and self.in_flight > 0:
                continue
            sess.queue.popleft()
            sess.busy = True
            self.resident += grow
            self.in_flight += 1
            return r, grow
        return None

    def waiting_sessions(self):
        # sessions in the order of their head request's arrival
        heads = [(self.sessions[s].queue[0].arrival, s) for s in self.active
                 if self.sessions[s].queue]
        heads.sort()
        return [s for _, s in heads]

    def _take(self, now):
        """Up to `batch` admissible requests (one per session), oldest first."""
        got = []
        while len(got) < max(1, self.batch):
            g = self._pick(now)
            if not g:
                break
            got.append(g)
        return got

    def _work(self):
        stream = torch.cuda.Stream()
        while True:
            with self.cv:
                while True:
                    if self.stop or self.remaining == 0:
                        return
                    now = time.perf_counter() - self.t0
                    got = self._take(now)
                    if got:
                        break
                    self.cv.wait(0.0005)
                work = [(r, grow) + self.inputs.pop(r.rid) for r, grow in got]
            start = time.perf_counter() - self.t0
            outs = []   # (request, info, q) per request
            with torch.cuda.stream(stream):
                calls, qs = [], []
                for r, grow, X, ready in work:
                    sess = self.sessions[r.session]
                    if r.kind == "orth":
                        if sess.basis is not None:
                            sqr_free(sess.basis)
                            sess.basis = None
                        Q = colmajor(r.m, r.cap)
                        R = colmajor(r.cap, r.cap)
                        calls.append(("orth", X, r.cap, Q, R))
                        qs.append(0)
                    else:
                        calls.append(("append", sess.basis, X))
                        qs.append(sess.basis.n)
                if self.batch:
                    # one batched call: the passes of all requests advance
                    # together, each launch covering every request
                    res = sqr_batch(calls, opts=self.opts, stream=stream)
                    for (r, grow, X, ready), call, q, d in zip(work, calls, qs, res):
                        if d["rc"] < 0:
                            raise RuntimeError(f"request {r.rid}: sqr_batch item failed with code {d['rc']}")
                        if r.kind == "orth":
                            self.sessions[r.session].basis = d["basis"]
                        outs.append((r, d["info"], q))
                else:
                    for (r, grow, X, ready), call, q in zip(work, calls, qs):
                        if r.kind == "orth":
                            _, A, cap, Q, R = call
                            b, info = sqr_orth(A, cap=cap, opts=self.opts, Q=Q, R=R, stream=stream)
                            self.sessions[r.session].basis = b
                        else:
                            info = sqr_append(call[1], call[2], stream=stream)
                        outs.append((r, info, q))
                for r, _, _ in outs:
                    sqr_park(self.sessions[r.session].basis)   # waits for the stream; frees scratch
            end = time.perf_counter() - self.t0
            with self.cv:
                for (r, info, q), (_, grow, X, ready) in zip(outs, work):
                    sess = self.sessions[r.session]
                    res = Result(r.rid, r.session, r.kind, info["status"], info["passes"],
                                 r.arrival, ready, start, end,
                                 request_bytes(r.kind, r.m, q, r.cols, info["passes"]))
                    if r.kind == "orth":
                        sess.bytes = 8 * (r.m * r.cap + r.cap * r.cap)
                    self.inflight_inputs -= 8.0 * r.m * r.cols
                    self.results.append(res)
                    self.remaining -= 1
                    if self.progress and len(self.results) % self.progress == 0:
                        print(f"served {len(self.results)} requests, {end:.1f} s",
                              file=sys.stderr, flush=True)
                    last = not sess.queue
                    if last:
                        if r.session in self.keep and sess.basis is not None:
                            bb = sess.basis
                            self.keep[r.session](bb.q().cpu(), bb.r().cpu())
                        if sess.basis is not None:
                            sqr_free(sess.basis)
                        sess.basis = None
                        self.resident -= sess.bytes
                        sess.bytes = 0
                        self.active.discard(r.session)
                    sess.busy = False
                    self.in_flight -= 1
                del work, outs
                self.cv.notify_all()

    def run(self, reqs, seeds=None):
        """Serve `reqs` (arrival times relative to the start); returns the
        results in completion order."""
        if seeds is None:
            seeds = {r.rid: 1_000_003 * (r.rid + 1) for r in reqs}
        self.cv = threading.Condition()
        self.sessions = {}
        for r in sorted(reqs, key=lambda r: r.rid):
            self.sessions.setdefault(r.session, _Session(r.session)).queue.append(r)
        for s in self.sessions.values():
            s.queue = collections.deque(sorted(s.queue, key=lambda r: r.rid))
        self.active = set(self.sessions)
        self.inputs = {}
        self.results = []
        self.resident = 0
        self.in_flight = 0
        self.inflight_inputs = 0.0
        self.remaining = len(reqs)
        self.stop = False
        arrival_order = sorted(reqs, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        gen = threading.Thread(target=self._generate, args=(arrival_order, seeds), daemon=True)
        gen.start()
        threads = [threading.Thread(target=self._work, daemon=True) for _ in range(self.workers)]
        for t in threads:
            t.start()
        try:
            for t in threads:
                t.join()
        finally:
            with self.cv:
                self.stop = True
                self.cv.notify_all()
            gen.join()
        torch.cuda.synchronize()
        return self.results


def summarize(results):
    """p50 / p99 latency (ms), throughput (requests/s), aggregate GB/s."""
    lat = sorted(r.latency for r in results)
    if not lat:
        return {}
    t_first = min(r.arrival for r in results)
    t_last = max(r.end for r in results)
    span = max(t_last - t_first, 1e-9)

    def pct(p):
        return lat[min(len(lat) - 1, int(math.ceil(p / 100.0 * len(lat))) - 1)] * 1e3

    return {"p50_ms": round(pct(50), 3), "p99_ms": round(pct(99), 3),
            "mean_ms": round(1e3 * sum(lat) / len(lat), 3),
            "requests": len(results), "makespan_s": round(span, 3),
            "req_per_s": round(len(results) / span, 2),
            "GBs": round(sum(r.bytes for r in results) / span / 1e9, 1),
            "ok": sum(r.status == 0 for r in results),
            "late_inputs": sum(r.ready > r.arrival for r in results)}
