"""Benchmark: iterative basis growth with the Cholesky QR block append.

Workload (one step): m = 1,000,000 rows; a CholQR3 of a 10-column start
block, then 19 appends of p = 10 columns (Algorithm 2) up to n = 200.  Block
k is U_k diag(s_k) V_k^T + 1e-3 [U_0..U_{k-1}] G_k with kappa_k log-uniform in
[1e2, 1e12] (seeded, synthetic).  All inputs are resident in HBM before the
timed region; the outputs Q (m x 200) and R (200 x 200) are reused buffers.

value = algorithmic HBM bytes of the step / time, where a CholQR pass count x
costs (1 + 2x) m n 8 bytes and an append with x iterations costs
8 m [(q + p) + x (q + 2p)] bytes (x = the passes the device executed).

Prints one JSON line.  --gpus N > 1 is refused: this program runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("CholQR3/append GB/s (% HBM roofline) at ‖QᵀQ−I‖≤1e-12; "
          "served p50/p99 ms")


def orth_bytes(m, n, x):
    return 8.0 * m * n * (1 + 2 * x)


def append_bytes(m, q, p, x):
    return 8.0 * m * ((q + p) + x * (q + 2 * p))


def step_bytes(m, n0, p, infos):
    total = orth_bytes(m, n0, infos[0]["passes"])
    q = n0
    for inf in infos[1:]:
        total += append_bytes(m, q, p, inf["passes"])
        q += p
    return total


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--blocks", type=int, default=19)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of 1 GiB first (counter calibration)")
    ap.add_argument("--workload", choices=["growth", "serve", "orth"], default="growth",
                    help="growth: the basis-growth step (default); serve: the serving loop; "
                         "orth: one CholQR3 of an m x n matrix (--m, --n, --kappa, --precision)")
    ap.add_argument("--n", type=int, default=128, help="orth: columns")
    ap.add_argument("--kappa", type=float, default=1e12, help="orth: condition number")
    ap.add_argument("--precision", type=int, default=0, help="orth: 0 FP64, 1 mixed")
    ap.add_argument("--requests", type=int, default=10000, help="serve: requests")
    ap.add_argument("--sessions", type=int, default=256, help="serve: sessions")
    ap.add_argument("--workers", type=int, default=4, help="serve: concurrent streams")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serve: arrivals per second (0: 0.8 x the measured saturated rate)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this program runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "serve":
        return serve_main(args)
    if args.workload == "orth":
        return orth_main(args)

    import numpy as np
    import torch
    import paper_2507_07788_amd as sq
    import synth

    m, n0, p, nb = args.m, 10, 10, args.blocks
    cap = n0 + p * nb
    t0 = time.time()
    A0, Ws, kappas = synth.growth_blocks(m, n0, p, nb, 1e2, 1e12)
    gen_s = time.time() - t0

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

    sq.sqr_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_infos = []
    for _ in range(args.steps):
        b, infos = step()
        all_infos.append(infos)
        if _ != args.steps - 1:
            sq.sqr_free(b)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = sq.sqr_prof_read()
    sq.sqr_prof_enable(False)

    statuses = [i["status"] for infos in all_infos for i in infos]
    bytes_total = sum(step_bytes(m, n0, p, infos) for infos in all_infos)
    value = bytes_total / dt / 1e9
    # accuracy of the final basis (outside the timed region)
    Qf = b.q()
    G = Qf.t() @ Qf
    loo = float(torch.linalg.norm(G - torch.eye(cap, dtype=G.dtype, device=G.device)))
    sq.sqr_free(b)

    nl, ms, by = prof["apply"]
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    traffic = measured_traffic(by / max(nl, 1))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "apply launches: block_pass (narrow_pass for the 10-column start)",
                "launches": nl,
                "avg_launch_us": round(ms * 1e3 / max(nl, 1), 2),
                "algorithmic_bytes_per_launch": round(by / max(nl, 1))}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import cholqr as O
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            cores = os.cpu_count()
        t0 = time.perf_counter()
        Qo, Ro, io = O.orth(A0)
        oinfos = [io]
        for W in Ws:
            Qo, Ro, io = O.append(Qo, Ro, W)
            oinfos.append(io)
        cdt = time.perf_counter() - t0
        cpu = {"value": round(step_bytes(m, n0, p, oinfos) / cdt / 1e9, 3), "unit": "GB/s",
               "cores": cores, "kind": "oracle",
               "sample": f"one full step (m={m}, 10->{cap} columns), {cdt:.1f} s"}

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
        "cpu_baseline": cpu,
        "loo": loo, "ok": all(s == 0 for s in statuses) and loo <= 1e-12,
        "passes": [i["passes"] for i in all_infos[-1]],
        "gen_s": round(gen_s, 1),
    }
    print(json.dumps(out))


def orth_main(args):
    """One orthogonalisation (Algorithm 1 with the CholQR3 start) of a seeded
    m x n matrix U diag(s) V^T with the given condition number, formed on the
    device.  value = algorithmic GB/s of the call ((1 + 2x) m n words for x
    passes); GFLOP/s counts (2x + 1) m n^2.  Invariants evaluated afterwards."""
    import torch
    import paper_2507_07788_amd as sq
    import synth

    m, n = args.m, args.n
    A = synth.test_matrix_device(m, n, args.kappa, (3,))
    Q = sq.colmajor(m, n)
    R = sq.colmajor(n, n)
    opts = sq.sqr_default_opts(precision=args.precision)
    for _ in range(args.warmup):
        b, info = sq.sqr_orth(A, opts=opts, Q=Q, R=R)
        sq.sqr_free(b)
    torch.cuda.synchronize()
    sq.sqr_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b, info = sq.sqr_orth(A, opts=opts, Q=Q, R=R)
        sq.sqr_free(b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    prof = sq.sqr_prof_read()
    sq.sqr_prof_enable(False)
    x = info["passes"]
    byt = 8.0 * m * n * (1 + 2 * x)
    fl = (2 * x + 1) * m * n * n
    # invariants, in row blocks
    G = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    res = nrm = 0.0
    Rt = torch.triu(R).contiguous()
    for r0 in range(0, m, 1 << 22):
        r1 = min(m, r0 + (1 << 22))
        Qb, Ab = Q[r0:r1].contiguous(), A[r0:r1].contiguous()
        G += Qb.t() @ Qb
        D = Ab - Qb @ Rt
        res += float((D * D).sum())
        nrm += float((Ab * Ab).sum())
    loo = float(torch.linalg.norm(G - torch.eye(n, dtype=G.dtype, device=G.device)))
    mfma = n >= 128
    achieved = fl / dt / 1e12 if mfma else byt / dt / 1e9
    peak = 78.6 if mfma else HBM_PEAK_GBS
    out = {
        "metric": METRIC, "value": round(byt / dt / 1e9, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"orth {m}x{n}, kappa {args.kappa:g}, "
                               f"{'mixed FP32/FP64' if args.precision else 'FP64'}",
                   "m": m, "n": n, "kappa": args.kappa, "precision": args.precision},
        "GFLOPs": round(fl / dt / 1e9, 1),
        "roofline": {"bound": "mfma" if mfma else "hbm", "achieved": round(achieved, 2 if mfma else 1),
                     "peak": peak, "unit": "TFLOP/s" if mfma else "GB/s",
                     "frac": round(achieved / peak, 4), "traffic": None,
                     "scope": "whole call (all kernels)"},
        "passes": x, "status": info["status"], "loo": loo, "rrr": math.sqrt(res / nrm),
        "kernels": {"apply": prof["apply"], "gram": prof["gram"]},
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def serve_main(args):
    """Serving workload: Poisson arrivals of orthogonalise / append requests
    from many resident sessions (m log-uniform 1e4..2e6, n 8..256, p 1..16,
    kappa log-uniform 1e2..1e12).  value = aggregate algorithmic GB/s over the
    makespan; p50 / p99 latency beside it."""
    import torch
    from paper_2507_07788_amd import serve

    reqs = serve.synthetic_workload(args.requests, args.sessions)
    # saturated rate: a calibration batch of whole sessions, all arriving at once
    cal_sessions = set(range(min(16, args.sessions)))
    cal = [serve.Request(**{**r.__dict__, "arrival": 0.0}) for r in reqs if r.session in cal_sessions]
    cres = serve.Server(workers=args.workers, progress=500).run(cal)
    csum = serve.summarize(cres)
    rate = args.rate if args.rate > 0 else 0.8 * csum["req_per_s"]
    serve.poisson_arrivals(reqs, rate)
    torch.cuda.synchronize()
    res = serve.Server(workers=args.workers, progress=1000).run(reqs)
    summ = serve.summarize(res)

    cpu = None
    if not args.no_cpu_baseline:
        import numpy as np
        from oracle import cholqr as O
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            cores = os.cpu_count()
        # a sample: the requests of the four sessions with the fewest rows, in
        # order, about 20 s of oracle work
        small = sorted({r.session: r.m for r in reqs}.items(), key=lambda kv: kv[1])[:4]
        keep = {sid for sid, _ in small}
        sample = sorted((r for r in reqs if r.session in keep), key=lambda r: r.rid)
        byt, done, cdt = 0.0, 0, 0.0
        state = {}
        for r in sample:
            if cdt > 20.0:
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
            print(f"cpu baseline: request {done} ({r.kind} m={r.m}) {cdt:.1f} s",
                  file=sys.stderr, flush=True)
        cpu = {"value": round(byt / cdt / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
               "sample": f"{done} requests of the 4 sessions with the fewest rows, in order, "
                         f"on the host, {cdt:.1f} s"}

    out = {
        "metric": METRIC, "value": summ["GBs"], "unit": "GB/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(summ["makespan_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} requests from {args.sessions} sessions, "
                               f"Poisson arrivals at {rate:.1f}/s (0.8 x saturated), "
                               f"{args.workers} streams",
                   "requests": args.requests, "sessions": args.sessions,
                   "workers": args.workers, "rate_per_s": round(rate, 2)},
        "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"], "mean_ms": summ["mean_ms"],
        "req_per_s": summ["req_per_s"], "ok": summ["ok"],
        "saturated": csum,
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
