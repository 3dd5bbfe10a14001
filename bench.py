"""Benchmark: iterative basis growth with the Cholesky QR block append.

Headline workload (one step): m = 1,000,000 rows; a CholQR3 of a 10-column
start block, then 19 appends of p = 10 columns (Algorithm 2) up to n = 200.
Block k is U_k diag(s_k) V_k^T + 1e-3 [U_0..U_{k-1}] G_k with kappa_k
log-uniform in [1e2, 1e12] (seeded, synthetic).  All inputs are resident in
HBM before the timed region; the outputs Q (m x 200) and R (200 x 200) are
reused buffers.

value = algorithmic HBM bytes of the step / time, where a CholQR pass count x
costs (1 + 2x) m n 8 bytes and an append with x iterations costs
8 m [(q + p) + x (q + 2p)] bytes (x = the passes the device executed).

Beside the headline, the same JSON line carries bounded sub-runs ("sub"):
the 20000 x 20 CholQR3 (kappa 1e6), the 4e6 x {16, 64, 128} CholQR3 at kappa
1e4 in FP64 and in the mixed FP32/FP64 form (with the speedup of the mixed
form), and a serving run (Poisson arrivals, p50/p99 latency from arrival).
Each sub-run has the roofline of its dominant kernel and an oracle CPU
baseline.  The CPU baselines run last, pinned to the physical cores of NUMA
node 0 (at most 16 threads, the host share of one GPU), median of repeats.

Other workloads: --workload orth (one orthogonalisation), serve (the full
serving run), sweep (the m- and n-sweeps of Fig. 3b/3c at kappa 1e20), panel
(the panel scheme against Algorithm 1, Fig. 4's shape up to n = 4096).

Prints one JSON line (sweep: one line per point, then a summary line).
--gpus N > 1 is refused: this program runs on one GPU.
"""
from __future__ import annotations

import argparse
import contextlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TF = 78.6
METRIC = ("CholQR3/append GB/s (% HBM roofline) at ‖QᵀQ−I‖≤1e-12; "
          "served p50/p99 ms")


def orth_bytes(m, n, x):
    return 8.0 * m * n * (1 + 2 * x)


def orth_flops(m, n, x):
    return (2 * x + 1) * m * n * n


def orth_moved_bytes(m, n, x, precision):
    """HBM bytes a CholQR3 call of x passes actually moves.  The one-block
    route (n <= 16, FP64 and mixed) recomputes the input of passes 2 and 3 from A and
    writes only from pass 3 on (the first pass that can end the call), so
    passes 1 and 2 read m n words and write none: (2x - 1) m n words for
    x >= 3 instead of the (1 + 2x) m n of the algorithmic count.  Every
    other route moves the algorithmic bytes."""
    if n <= 16:
        words = 1 + sum(1 if k < 3 else 2 for k in range(1, x + 1))
        return 8.0 * m * n * words
    return orth_bytes(m, n, x)


def append_bytes(m, q, p, x):
    return 8.0 * m * ((q + p) + x * (q + 2 * p))


def step_bytes(m, n0, p, infos):
    total = orth_bytes(m, n0, infos[0]["passes"])
    q = n0
    for inf in infos[1:]:
        total += append_bytes(m, q, p, inf["passes"])
        q += p
    return total


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "block_pass_apply_growth_m1e6_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2507_07788_amd", "csrc", "sqr_kernels.hip")


def measured_traffic(alg_bytes_per_launch):
    """HBM bytes per apply launch of the streaming kernel, from the committed
    FETCH_SIZE / WRITE_SIZE summary (scaled by a plain-copy calibration), as
    measured/algorithmic ratio times this run's algorithmic bytes per launch.
    None when the summary is missing or the kernel source changed since."""
    import hashlib
    try:
        kv = dict(line.split(":", 1) for line in open(TRAFFIC_FILE)
                  if ":" in line and not line.startswith("#"))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if kv.get("kernel_source_sha256", "").strip() != sha:
            return None
        return round(float(kv["measured_over_algorithmic"]) * alg_bytes_per_launch)
    except (OSError, KeyError, ValueError):
        return None


# --------------------------------------------------------------------------
# host cores for the CPU baseline
# --------------------------------------------------------------------------
def _cpulist(text):
    out = set()
    for part in text.strip().split(","):
        if not part:
            continue
        if "-" in part:
            a, b = part.split("-")
            out.update(range(int(a), int(b) + 1))
        else:
            out.add(int(part))
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


@contextlib.contextmanager
def pinned_host(max_threads=16):
    """Pin every thread of this process to the physical cores of NUMA node 0
    that it may run on (one hardware thread per core, at most max_threads: the
    host share of one GPU) and limit the BLAS pool to as many threads.
    Yields a description {cores, cpus, model, node}."""
    allowed = os.sched_getaffinity(0)
    try:
        node0 = _cpulist(open("/sys/devices/system/node/node0/cpulist").read())
    except OSError:
        node0 = set(allowed)
    cand = sorted(allowed & node0) or sorted(allowed)
    phys, seen = [], set()
    for c in cand:
        try:
            sib = min(_cpulist(open(f"/sys/devices/system/cpu/cpu{c}/topology/thread_siblings_list").read()))
        except OSError:
            sib = c
        if sib in seen:
            continue
        seen.add(sib)
        phys.append(c)
    cpus = set(phys[:max_threads]) or set(cand[:max_threads])
    tids = [int(t) for t in os.listdir("/proc/self/task")]
    old = {}
    for t in tids:
        try:
            old[t] = os.sched_getaffinity(t)
            os.sched_setaffinity(t, cpus)
        except OSError:
            pass
    desc = {"cores": len(cpus), "cpus": ",".join(str(c) for c in sorted(cpus)),
            "model": _cpu_model(), "node": 0 if node0 & cpus else None}
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(len(cpus))
    except Exception:  # pragma: no cover
        limiter = contextlib.nullcontext()
    try:
        with limiter:
            yield desc
    finally:
        for t, a in old.items():
            try:
                os.sched_setaffinity(t, a)
            except OSError:
                pass


def _median_time(fn, reps):
    ts = []
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), out


# --------------------------------------------------------------------------
# GPU runs
# --------------------------------------------------------------------------
def growth_gpu(args):
    import numpy as np
    import torch
    import paper_2507_07788_amd as sq
    import synth

    m, n0, p, nb = args.m, 10, 10, args.blocks
    cap = n0 + p * nb
    t0 = time.time()
    A0, Ws, kappas = synth.growth_blocks(m, n0, p, nb, 1e2, 1e12)
    gen_s = time.time() - t0
    log(f"growth: inputs generated in {gen_s:.1f} s")

    def to_dev(X):
        t = torch.empty((X.shape[1], X.shape[0]), dtype=torch.float64, device="cuda").t()
        t.copy_(torch.from_numpy(np.ascontiguousarray(X)))
        return t

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        del src, dst

    A0d = to_dev(A0)
    Wd = [to_dev(W) for W in Ws]
    Q = sq.colmajor(m, cap)
    R = sq.colmajor(cap, cap)
    torch.cuda.synchronize()

    def step():
        b, info = sq.sqr_orth(A0d, cap=cap, Q=Q, R=R)
        infos = [info]
        for W in Wd:
            infos.append(sq.sqr_append(b, W))
        return b, infos

    for _ in range(args.warmup):
        b, infos = step()
        sq.sqr_free(b)
    torch.cuda.synchronize()

    # The streaming launches of the last timed step are bracketed by HIP
    # events (the roofline's kernel times); each event is a marker packet on
    # the stream that delays the next kernel by a few microseconds, so the
    # other steps run without them.
    sq.sqr_prof_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_infos = []
    for _ in range(args.steps):
        if _ == args.steps - 1:
            sq.sqr_prof_enable(True)
        b, infos = step()
        all_infos.append(infos)
        if _ != args.steps - 1:
            sq.sqr_free(b)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = sq.sqr_prof_read()
    sq.sqr_prof_enable(False)
    log(f"growth: {args.steps} steps in {dt:.3f} s")

    statuses = [i["status"] for infos in all_infos for i in infos]
    bytes_total = sum(step_bytes(m, n0, p, infos) for infos in all_infos)
    value = bytes_total / dt / 1e9
    # accuracy of the final basis (outside the timed region)
    Qf = b.q()
    G = Qf.t() @ Qf
    loo = float(torch.linalg.norm(G - torch.eye(cap, dtype=G.dtype, device=G.device)))
    sq.sqr_free(b)
    del A0d, Wd, Q, R, Qf, G
    torch.cuda.empty_cache()

    nl, ms, by = prof["apply"]
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    traffic = measured_traffic(by / max(nl, 1))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "apply launches: block_pass (narrow_pass for the 10-column start)",
                "launches": nl,
                "avg_launch_us": round(ms * 1e3 / max(nl, 1), 2),
                "algorithmic_bytes_per_launch": round(by / max(nl, 1))}
    ng, msg, byg = prof["gram"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"basis growth: CholQR3 of {m}x{n0}, then {nb} appends of "
                               f"p={p} (block kappa log-uniform 1e2..1e12)",
                   "m": m, "n0": n0, "p": p, "blocks": nb, "final_n": cap},
        "frac_of_hbm_peak": round(value / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "gram_only_launches": {"launches": ng, "avg_launch_us": round(msg * 1e3 / max(ng, 1), 2),
                               "GBs": round(byg / (msg * 1e-3) / 1e9, 1) if msg > 0 else None},
        "cpu_baseline": None,
        "loo": loo, "ok": all(s == 0 for s in statuses) and loo <= 1e-12,
        "passes": [i["passes"] for i in all_infos[-1]],
        "gen_s": round(gen_s, 1),
    }
    return out, (A0, Ws)


def _orth_invariants(A, Q, R, m, n):
    import torch
    G = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    res = nrm = 0.0
    Rt = torch.triu(R).contiguous()
    # row blocks of 2^16 rows: the evaluation's own rounding (a library GEMM
    # summing over the block's rows) stays below the quantity it measures
    for r0 in range(0, m, 1 << 16):
        r1 = min(m, r0 + (1 << 16))
        Qb, Ab = Q[r0:r1].contiguous(), A[r0:r1].contiguous()
        G += Qb.t() @ Qb
        D = Ab - Qb @ Rt
        res += float((D * D).sum())
        nrm += float((Ab * Ab).sum())
    loo = float(torch.linalg.norm(G - torch.eye(n, dtype=G.dtype, device=G.device)))
    return loo, math.sqrt(res / nrm)


def _dominant_roofline(prof, m, n, precision, x=0):
    """Roofline object of the kernel kind with the larger total time among
    the timed launches: HBM bytes per launch below 80 columns, FP64 MFMA
    flops from 80 columns on (a pass moves 16 m n bytes for 2 m n^2 flops, so
    its intensity n / 8 passes the ridge of 78.6 TFLOP/s over 8 TB/s near
    n = 79).  Flops: m n^2 per apply or Gramian of a pass, 2 m n^2 where one
    launch does both.  The mixed form is measured on its FP64 apply
    launches."""
    na, msa, bya = prof["apply"]
    ng, msg, byg = prof["gram"]
    kind = "apply" if (msa >= msg or precision == 1) else "gram"
    nl, ms, by = (na, msa, bya) if kind == "apply" else (ng, msg, byg)
    if nl == 0 or ms <= 0:
        return None
    # fused: an apply launch also forms the next Gramian (2 m n^2 flops)
    if precision == 0 and n > 256:
        names, fused = {"apply": "block_pass apply", "gram": "block_pass Gram"}, True
    elif n > 112:
        names, fused = {"apply": "wide_apply", "gram": "gram_pass"}, False
    elif n <= 16:
        names, fused = {"apply": "narrow_pass (apply + Gramian)", "gram": "narrow_pass (Gramian)"}, True
    elif n <= 128:
        names, fused = {"apply": "wide_pass (apply + Gramian)", "gram": "wide_pass (Gramian)"}, True
    else:
        names, fused = {"apply": "wide_apply", "gram": "gram_pass"}, False
    if n >= 80:
        fpl = m * n * n * (2 if (fused and kind == "apply") else 1)
        if n > 256 and precision == 0:
            # one block_pass launch per 16-column block: a pass's flops are
            # spread over ceil(n / 16) launches
            fpl = fpl / ((n + 15) // 16)
        achieved = nl * fpl / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_PEAK_TF,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TF, 4), "traffic": None,
                "kernel": names[kind], "launches": nl, "avg_launch_us": round(ms * 1e3 / nl, 2),
                "algorithmic_flops_per_launch": float(fpl)}
    achieved = by / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": names[kind],
           "launches": nl, "avg_launch_us": round(ms * 1e3 / nl, 2),
           "algorithmic_bytes_per_launch": round(by / nl)}
    if n <= 16 and kind == "apply" and x:
        # passes 1 and 2 read A and write nothing (m n words, not 2 m n)
        moved = sum(1 if k < 3 else 2 for k in range(1, x + 1)) / x * 8.0 * m * n
        out["moved_bytes_per_launch"] = round(moved)
        out["moved_GBs"] = round(moved * nl / (ms * 1e-3) / 1e9, 1)
    return out


def orth_gpu(m, n, kappa, precision, steps, warmup, seed=(3,), A=None):
    """CholQR3 of a seeded m x n matrix U diag(s) V^T (formed on the device).
    Returns a dict: ms per call, algorithmic GB/s and GFLOP/s, passes,
    invariants, roofline of the dominant kernel."""
    import torch
    import paper_2507_07788_amd as sq
    import synth

    if A is None:
        A = synth.test_matrix_device(m, n, kappa, seed)
    Q = sq.colmajor(m, n)
    R = sq.colmajor(n, n)
    opts = sq.sqr_default_opts(precision=precision)
    for _ in range(warmup):
        b, info = sq.sqr_orth(A, opts=opts, Q=Q, R=R)
        sq.sqr_free(b)
    torch.cuda.synchronize()
    sq.sqr_prof_enable(False)
    t0 = time.perf_counter()
    for i in range(steps):
        if i == steps - 1:   # events around the last call's streaming launches only
            sq.sqr_prof_enable(True)
        b, info = sq.sqr_orth(A, opts=opts, Q=Q, R=R)
        sq.sqr_free(b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = sq.sqr_prof_read()
    sq.sqr_prof_enable(False)
    x = info["passes"]
    loo, rrr = _orth_invariants(A, Q, R, m, n)
    res = {"m": m, "n": n, "kappa": kappa, "precision": precision,
           "ms": round(dt * 1e3, 4), "GBs": round(orth_bytes(m, n, x) / dt / 1e9, 1),
           "GFLOPs": round(orth_flops(m, n, x) / dt / 1e9, 1),
           "frac_of_hbm_peak": round(orth_bytes(m, n, x) / dt / 1e9 / HBM_PEAK_GBS, 4),
           "frac_of_fp64_mfma_peak": round(orth_flops(m, n, x) / dt / 1e12 / FP64_PEAK_TF, 4),
           "moved_GBs": round(orth_moved_bytes(m, n, x, precision) / dt / 1e9, 1),
           "passes": x, "status": info["status"], "loo": loo, "rrr": rrr,
           "ok": info["status"] == 0 and loo <= 1e-12 and rrr <= 1e-13,
           "roofline": _dominant_roofline(prof, m, n, precision, x)}
    del Q, R
    return res


def serve_gpu(requests, sessions, workers, rate, batch=0):
    """Serving run: returns (summary dict, saturated summary, rate, requests).
    batch > 0: up to that many requests per batched library call."""
    import gc
    import torch
    from paper_2507_07788_amd import serve

    gc.collect()
    torch.cuda.empty_cache()   # earlier runs' idle blocks back to the device

    reqs = serve.synthetic_workload(requests, sessions)
    # saturated rate: a calibration batch of whole sessions, all arriving at once
    cal_sessions = set(range(min(16, sessions)))
    cal = [serve.Request(**{**r.__dict__, "arrival": 0.0}) for r in reqs if r.session in cal_sessions]
    cres = serve.Server(workers=workers, batch=batch, progress=500).run(cal)
    csum = serve.summarize(cres)
    del cres
    gc.collect()
    torch.cuda.empty_cache()
    rate = rate if rate > 0 else 0.8 * csum["req_per_s"]
    serve.poisson_arrivals(reqs, rate)
    torch.cuda.synchronize()
    res = serve.Server(workers=workers, batch=batch, progress=1000).run(reqs)
    summ = serve.summarize(res)
    return summ, csum, rate, reqs


# --------------------------------------------------------------------------
# CPU baselines (the oracle as it stands, on the host)
# --------------------------------------------------------------------------
def cpu_growth(A0, Ws, m, n0, p, reps):
    from oracle import cholqr as O

    def run():
        Qo, Ro, io = O.orth(A0)
        oinfos = [io]
        for W in Ws:
            Qo, Ro, io = O.append(Qo, Ro, W)
            oinfos.append(io)
        return oinfos

    t, oinfos = _median_time(run, reps)
    return step_bytes(m, n0, p, oinfos) / t / 1e9, t


def cpu_orth(m, n, kappa, precision, reps, seed=(3,)):
    import synth
    from oracle import cholqr as O
    A = synth.test_matrix(m, n, kappa, seed=seed)
    t, res = _median_time(lambda: O.orth(A, precision=precision), reps)
    x = res[2]["passes"]
    return orth_bytes(m, n, x) / t / 1e9, t, x


def cpu_serve(reqs, budget_s):
    from paper_2507_07788_amd import serve
    from oracle import cholqr as O
    # the requests of the four sessions with the fewest rows, in order
    small = sorted({r.session: r.m for r in reqs}.items(), key=lambda kv: kv[1])[:4]
    keep = {sid for sid, _ in small}
    sample = sorted((r for r in reqs if r.session in keep), key=lambda r: r.rid)
    byt, done, cdt = 0.0, 0, 0.0
    state = {}
    for r in sample:
        if cdt > budget_s:
            break
        X = serve.make_input(r, 1_000_003 * (r.rid + 1)).cpu().numpy()   # not timed
        ts = time.perf_counter()
        if r.kind == "orth":
            Qo, Ro, io = O.orth(X)
            state[r.session] = Qo, Ro
            q = 0
        else:
            Qi, Ri = state[r.session]
            q = Qi.shape[1]
            Qo, Ro, io = O.append(Qi, Ri, X)
            if io["status"] == 0:
                state[r.session] = Qo, Ro
        cdt += time.perf_counter() - ts
        byt += serve.request_bytes(r.kind, r.m, q, r.cols, io["passes"])
        done += 1
    return byt / cdt / 1e9, cdt, done


def _cpu_obj(value, unit, host, sample):
    return {"value": round(value, 3), "unit": unit, "cores": host["cores"], "kind": "oracle",
            "sample": sample, "host": {"model": host["model"], "numa_node": host["node"],
                                       "cpus": host["cpus"]}}


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
C3_SAMPLE_ROWS = 250_000


def main_growth(args):
    out, (A0, Ws) = growth_gpu(args)
    subs = {}
    if not args.no_sub:
        c1 = orth_gpu(20000, 20, 1e6, 0, steps=200, warmup=20, seed=(1,))
        c1["us"] = round(c1["ms"] * 1e3, 2)
        subs["C1_orth_20000x20_k1e6"] = c1
        log(f"sub C1: {c1['us']} us")
        for n in (16, 64, 128):
            import synth
            A = synth.test_matrix_device(4_000_000, n, 1e4, (3,))
            for prec in (0, 1):
                # 20 timed calls below 1 ms per call keep the events of the last
                # one and the spread between calls from moving the mean
                r = orth_gpu(4_000_000, n, 1e4, prec, steps=20 if n <= 64 else 5, warmup=3, A=A)
                subs[f"C3_orth_4e6x{n}_k1e4_{'mixed' if prec else 'fp64'}"] = r
                log(f"sub C3 n={n} prec={prec}: {r['ms']} ms")
            f64 = subs[f"C3_orth_4e6x{n}_k1e4_fp64"]
            mix = subs[f"C3_orth_4e6x{n}_k1e4_mixed"]
            mix["speedup_vs_fp64"] = round(f64["ms"] / mix["ms"], 3)
            del A
        # both modes at the same offered load: 0.8 x the batched mode's
        # saturated rate, measured on a calibration batch of whole sessions
        rate = 0.0
        for key, workers, batch in (("C4_serve", args.batch_workers, args.batch),
                                    ("C4_serve_unbatched", args.workers, 0)):
            summ, csum, rate, reqs = serve_gpu(args.sub_requests, args.sub_sessions, workers, rate, batch)
            subs[key] = {"requests": args.sub_requests, "sessions": args.sub_sessions,
                         "workers": workers, "batch": batch, "rate_per_s": round(rate, 2),
                         "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"],
                         "mean_ms": summ["mean_ms"], "req_per_s": summ["req_per_s"],
                         "GBs": summ["GBs"], "ok": summ["ok"], "late_inputs": summ["late_inputs"],
                         "saturated": csum,
                         "latency": "from arrival to the end of the request's stream work"}
            log(f"sub {key}: p50 {summ['p50_ms']} ms, p99 {summ['p99_ms']} ms")
    if not args.no_cpu_baseline:
        with pinned_host() as host:
            v, t = cpu_growth(A0, Ws, args.m, 10, 10, reps=3)
            out["cpu_baseline"] = _cpu_obj(v, "GB/s", host, f"the full step (m={args.m}, 10->"
                                           f"{10 + 10 * args.blocks} columns), median of 3: {t:.1f} s")
            log(f"cpu growth: {t:.1f} s")
            if subs:
                v, t, _ = cpu_orth(20000, 20, 1e6, 0, reps=10, seed=(1,))
                c1 = subs["C1_orth_20000x20_k1e6"]
                c1["cpu_baseline"] = _cpu_obj(v, "GB/s", host, f"the same 20000x20 CholQR3, median of 10: "
                                              f"{t * 1e3:.2f} ms")
                for n in (16, 64, 128):
                    for prec in (0, 1):
                        v, t, x = cpu_orth(C3_SAMPLE_ROWS, n, 1e4, prec, reps=3)
                        subs[f"C3_orth_4e6x{n}_k1e4_{'mixed' if prec else 'fp64'}"]["cpu_baseline"] = \
                            _cpu_obj(v, "GB/s", host, f"{C3_SAMPLE_ROWS}x{n} rows of the same recipe "
                                     f"({x} passes), median of 3: {t:.2f} s; GB/s scales with m")
                log("cpu C1/C3 done")
                v, t, done = cpu_serve(reqs, budget_s=8.0)
                subs["C4_serve"]["cpu_baseline"] = _cpu_obj(
                    v, "GB/s", host, f"{done} requests of the 4 sessions with the fewest rows, "
                    f"in order: {t:.1f} s")
    if subs:
        out["sub"] = subs
    print(json.dumps(out))


def main_orth(args):
    r = orth_gpu(args.m, args.n, args.kappa, args.precision, args.steps, args.warmup)
    out = {
        "metric": METRIC, "value": r["GBs"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"orth {args.m}x{args.n}, kappa {args.kappa:g}, "
                               f"{'mixed FP32/FP64' if args.precision else 'FP64'}",
                   "m": args.m, "n": args.n, "kappa": args.kappa, "precision": args.precision},
        "GFLOPs": r["GFLOPs"], "moved_GBs": r["moved_GBs"], "roofline": r["roofline"], "passes": r["passes"],
        "status": r["status"], "loo": r["loo"], "rrr": r["rrr"], "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        with pinned_host() as host:
            ms = min(args.m, C3_SAMPLE_ROWS)
            v, t, x = cpu_orth(ms, args.n, args.kappa, args.precision, reps=3)
            out["cpu_baseline"] = _cpu_obj(v, "GB/s", host, f"{ms}x{args.n} rows of the same recipe "
                                           f"({x} passes), median of 3: {t:.2f} s")
    print(json.dumps(out))


def main_serve(args):
    workers = args.batch_workers if args.batch else args.workers
    summ, csum, rate, reqs = serve_gpu(args.requests, args.sessions, workers, args.rate, args.batch)
    out = {
        "metric": METRIC, "value": summ["GBs"], "unit": "GB/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(summ["makespan_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} requests from {args.sessions} sessions, "
                               f"Poisson arrivals at {rate:.1f}/s, {workers} streams, "
                               f"batches of up to {args.batch}",
                   "requests": args.requests, "sessions": args.sessions,
                   "workers": workers, "batch": args.batch, "rate_per_s": round(rate, 2)},
        "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"], "mean_ms": summ["mean_ms"],
        "req_per_s": summ["req_per_s"], "ok": summ["ok"], "saturated": csum,
        "roofline": None, "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        with pinned_host() as host:
            v, t, done = cpu_serve(reqs, budget_s=20.0)
            out["cpu_baseline"] = _cpu_obj(v, "GB/s", host, f"{done} requests of the 4 sessions "
                                           f"with the fewest rows, in order: {t:.1f} s")
    print(json.dumps(out))


SWEEP_M = [10_000, 31_623, 100_000, 316_228, 1_000_000, 3_162_278, 10_000_000]
SWEEP_N = [50, 100, 150, 200, 250, 300, 350, 400, 450, 500]


def main_sweep(args):
    """Fig. 3b (n = 100, m = 1e4 .. 1e7) and Fig. 3c (m = 1e6, n = 50 .. 500)
    at nominal kappa 1e20, FP64 CholQR3: one JSON line per point (runtime per
    row for the m-sweep, as the figure plots it), then a summary line."""
    import torch
    pts = [("m", m, 100) for m in SWEEP_M] + [("n", 1_000_000, n) for n in SWEEP_N]
    rows = []
    for kind, m, n in pts:
        r = orth_gpu(m, n, 1e20, 0, steps=args.steps, warmup=args.warmup, seed=(30,))
        r["sweep"] = kind
        r["s_per_row"] = r["ms"] * 1e-3 / m
        rows.append(r)
        print(json.dumps(r), flush=True)
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "CholQR3 sweeps of Fig. 3b/3c (kappa 1e20)", "points": len(rows),
                      "ok": all(r["ok"] for r in rows)}))


PANEL_N = [128, 256, 384, 512, 1024, 2048, 4096]


def main_panel(args):
    """Fig. 4's comparison at m = 1e6, kappa = 1e5: Algorithm 1 as printed
    (rsCholQR: no first-pass shift, stopping test from the first pass), the
    CholQR3 start, and the panel scheme with r = 2..5 panels, for the n of
    --panel-n.  One JSON line per point (ms per call), then a summary."""
    import torch
    import paper_2507_07788_amd as sq
    import synth
    m = 1_000_000
    rows = []
    ns = [int(v) for v in args.panel_n.split(",")] if args.panel_n else PANEL_N
    for n in ns:
        t0 = time.perf_counter()
        A = synth.test_matrix_device(m, n, 1e5, (50,))
        torch.cuda.synchronize()
        print(f"panel: n = {n} input in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        Q, R = sq.colmajor(m, n), sq.colmajor(n, n)
        variants = [("rsCholQR", None), ("CholQR3", None)] + [(f"pnCholQR({r})", r) for r in range(2, 6)]
        for name, r in variants:
            def call():
                if r is None:
                    kw = dict(first_pass_shift=0, min_passes=0) if name == "rsCholQR" else {}
                    return sq.sqr_orth(A, Q=Q, R=R, opts=sq.sqr_default_opts(**kw))
                return sq.sqr_panel(A, r, Q=Q, R=R)
            for _ in range(args.warmup):
                b, info = call()
                sq.sqr_free(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                b, info = call()
                sq.sqr_free(b)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            loo, rrr = _orth_invariants(A, Q, R, m, n)
            row = {"variant": name, "m": m, "n": n, "kappa": 1e5, "ms": round(dt * 1e3, 3),
                   "status": info["status"], "loo": loo, "rrr": rrr,
                   "ok": info["status"] == 0 and loo <= 1e-12 and rrr <= 1e-13}
            rows.append(row)
            print(json.dumps(row), flush=True)
        del A, Q, R
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "panel scheme vs Algorithm 1 (Fig. 4 shape, m = 1e6, kappa 1e5)",
                      "points": len(rows), "ok": all(r["ok"] for r in rows)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--blocks", type=int, default=19)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sub", action="store_true", help="growth: skip the sub-runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of 1 GiB first (counter calibration)")
    ap.add_argument("--workload", choices=["growth", "serve", "orth", "sweep", "panel"], default="growth",
                    help="growth: the basis-growth step and the sub-runs (default); serve: the "
                         "serving loop; orth: one CholQR3 of an m x n matrix (--m, --n, --kappa, "
                         "--precision); sweep: the m- and n-sweeps of Fig. 3b/3c; panel: the panel "
                         "scheme against Algorithm 1 (Fig. 4 shape)")
    ap.add_argument("--n", type=int, default=128, help="orth: columns")
    ap.add_argument("--panel-n", type=str, default="", help="panel: comma-separated n (default 128..4096)")
    ap.add_argument("--kappa", type=float, default=1e12, help="orth: condition number")
    ap.add_argument("--precision", type=int, default=0, help="orth: 0 FP64, 1 mixed")
    ap.add_argument("--requests", type=int, default=10000, help="serve: requests")
    ap.add_argument("--sessions", type=int, default=256, help="serve: sessions")
    ap.add_argument("--sub-requests", type=int, default=2000, help="growth: serving sub-run requests")
    ap.add_argument("--sub-sessions", type=int, default=64, help="growth: serving sub-run sessions")
    ap.add_argument("--workers", type=int, default=4, help="serve: concurrent streams (unbatched)")
    ap.add_argument("--batch", type=int, default=8,
                    help="serve: requests per batched library call (0: one call per request)")
    ap.add_argument("--batch-workers", type=int, default=2, help="serve: concurrent streams (batched)")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serve: arrivals per second (0: 0.8 x the measured saturated rate)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this program runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    {"growth": main_growth, "serve": main_serve, "orth": main_orth,
     "sweep": main_sweep, "panel": main_panel}[args.workload](args)


if __name__ == "__main__":
    main()
