#!/usr/bin/env python3
"""Benchmark of the sketching hot path on one MI355X.

Workload (the paper's sketch-and-solve least squares, eq. 4.2, at the
synthetic heavy-leverage shape): A is 2^20 x 256 fp32 (rows g_i |t_i|, g_i ~
N(0, I), t_i Student-t with 2 degrees of freedom), b = A x* + N(0, 1e-3),
sketch size s = 4096.

One step = for each sketch family (CountSketch, SRHT, Gaussian) the whole
path of the library: the sketch C = S^T [A | b] (one pass over A), the FP64
CholeskyQR2 solve of the s x 256 sketched system, and the FP64 residual
||A x~ - b|| (a second pass over A).  Inputs are resident in HBM before the
timed region.  `value` is GB/s of A: (number of sketches) x bytes of [A | b]
per second of step time.

Prints one JSON line.  Extra keys: per-family sketch time and roofline,
sketch-and-solve p50/p99 latency next to the plain FP64 normal-equation
solve, rsvd solves/s on the 2048 x 512 fp64 problem, the 65536 x 8192 rsvd
(sigma_i = 1/i) in fp32, BF16 and FP8 with its error against the known
spectrum, Nystrom on 200,000 points (c = 1024), the serving workload
(plain one-at-a-time against the grouped, budgeted server), and the CPU
oracle timed on a bounded row sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6

# kernel source behind each sketch family (traffic counters are void once it changes)
KERNEL_SRC = {
    "countsketch": "paper_1505_07570_amd/csrc/countsketch.hip",
    "srht": "paper_1505_07570_amd/csrc/srht.hip",
    "gaussian": "paper_1505_07570_amd/csrc/gauss_sketch.hip",
}


def src_sha(path):
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# main kernel of each sketch family (the one the counters are read for)
KERNEL_NAME = {
    "countsketch": "countsketch_sched_kernel",
    "srht": "srht_kernel",
    "gaussian": "gauss_sketch_kernel",
}
COPY_ELEMS = 1 << 28  # fp32 elements of the calibration copy (1 GiB read, 1 GiB written)


def measured_traffic(kind):
    """HBM bytes per launch of a family's main kernel from committed counters.

    profiles/traffic.json holds, per sketch family, the FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) of its main kernel, the factors that map
    each counter onto the bytes of a plain copy of known size, and the sha
    of the kernel source they were taken on; stale entries give null.
    """
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f).get(kind)
    if not t or t.get("src_sha") != src_sha(KERNEL_SRC[kind]):
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def traffic_workload(h, Ad, bd, C, s, seed, kinds):
    """The dispatches the counter runs read: a plain copy of known size, then
    two sketches per family (the second one is the measured dispatch)."""
    import torch
    x = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    for k in kinds:
        for _ in range(2):
            h.sketch(Ad, s, k, seed, b=bd, out=C[k])
        torch.cuda.synchronize()


def summarize_traffic(fetch_csv, write_csv, kinds):
    """profiles/traffic.json from the counter CSVs of the two runs."""
    import csv

    def per_dispatch(path, counter):
        rows = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name", counter) != counter:
                    continue
                d = int(r["Dispatch_Id"])
                rows.setdefault(d, [r["Kernel_Name"], 0.0])
                rows[d][1] += float(r["Counter_Value"])
        return [rows[d] for d in sorted(rows)]

    out = {}
    fetch = per_dispatch(fetch_csv, "FETCH_SIZE")
    write = per_dispatch(write_csv, "WRITE_SIZE")
    kib = COPY_ELEMS * 4 / 1024.0

    def last(rows, needle):
        hits = [v for n, v in rows if needle in n]
        return hits[-1] if hits else None

    # the calibration copy is the largest copy dispatch of the run
    cf = max((v for n, v in fetch if "copy" in n), default=None)
    cw = max((v for n, v in write if "copy" in n), default=None)
    for k in kinds:
        fk, wk = last(fetch, KERNEL_NAME[k]), last(write, KERNEL_NAME[k])
        if None in (fk, wk, cf, cw):
            continue
        out[k] = {"kernel": KERNEL_NAME[k], "fetch_kib": fk, "write_kib": wk,
                  "fetch_scale": kib / cf, "write_scale": kib / cw,
                  "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_kib_each_way": kib,
                  "src_sha": src_sha(KERNEL_SRC[k])}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def cpu_baseline(A, b, s, kinds, seed, rows):
    """The FP64 oracle's sketch-and-solve on the first `rows` rows."""
    import numpy as np
    from oracle import lsr as olsr, sketch as osk
    codes = {"countsketch": osk.COUNTSKETCH, "srht": osk.SRHT, "gaussian": osk.GAUSSIAN}
    As = np.asarray(A[:rows], dtype=np.float64)
    bs = np.asarray(b[:rows], dtype=np.float64)
    t0 = time.perf_counter()
    for k in kinds:
        olsr.sketched_lsr(As, bs, s, codes[k], seed, fp64=False)
    dt = time.perf_counter() - t0
    nbytes = len(kinds) * rows * (A.shape[1] + 1) * 4
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    # the same oracle on one core (BLAS limited to one thread), on an eighth
    # of the sample
    from threadpoolctl import threadpool_limits
    rows1 = max(s, rows // 8)
    A1, b1 = As[:rows1], bs[:rows1]
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        for k in kinds:
            olsr.sketched_lsr(A1, b1, s, codes[k], seed, fp64=False)
        dt1 = time.perf_counter() - t1
    return {
        "value": nbytes / dt / 1e9,
        "unit": "GB/s",
        "cores": min(cores, threads),
        "kind": "oracle",
        "sample": f"first {rows} rows of [A|b] (m={rows}, d={A.shape[1]}), s={s}, "
                  f"sketch-and-solve for {','.join(kinds)} in fp64 numpy with explicit S; "
                  f"{dt:.1f} s wall",
        "single_core": {"value": len(kinds) * rows1 * (A.shape[1] + 1) * 4 / dt1 / 1e9, "unit": "GB/s",
                        "cores": 1, "sample": f"first {rows1} rows, the same calls; {dt1:.1f} s wall"},
    }


def rsvd_spectrum(h, reps, lat):
    """Randomized SVD of A = U diag(1/i) V^T (65536 x 8192 fp32), k=100, p=28, q=2,
    in fp32 and with BF16 / FP8 operands: time per solve and the error against
    the exactly known spectrum."""
    import numpy as np
    import torch

    import synth
    import paper_1505_07570_amd as rmm
    m, n, k, p, q = 65536, 8192, 100, 28, 2
    sig = 1.0 / np.arange(1, n + 1)
    A = synth.spectrum_matrix(synth.data_seed(3), m, n, sig, backend="torch", device="cuda")
    torch.cuda.synchronize()
    a_bytes = m * n * 4
    opt = float(np.sqrt((sig[k:] ** 2).sum()))        # ||A - A_k||_F
    seed = synth.sketch_seed(3)
    out = {"m": m, "n": n, "k": k, "p": p, "q": q, "sigma": "1/i", "opt_resid_fro": opt}
    for name, prec in (("fp32", rmm.PREC_NATIVE), ("bf16", rmm.PREC_BF16), ("fp8", rmm.PREC_FP8)):
        h.set_autotune(True)  # the dense products get their tuned launch plans
        U, s, V, st = h.rsvd(A, k, p, q, seed, prec=prec)
        h.set_autotune(False)
        ts = lat(lambda: h.rsvd(A, k, p, q, seed, prec=prec), reps)
        s64 = s.double().cpu().numpy()
        # ||A - U diag(s) V^T||_F in row blocks
        acc = 0.0
        for r0 in range(0, m, 8192):
            blk = A[r0:r0 + 8192] - (U[r0:r0 + 8192] * s[None, :]) @ V.t()
            acc += float(torch.linalg.vector_norm(blk.double()) ** 2)
        eb = {"fp32": 4, "bf16": 2, "fp8": 1}[name]
        # algorithmic bytes: fp32 reads A in each of the 2q+2 products; the mixed
        # paths read A once to quantize it, write two quantized copies and read one
        # quantized copy per product
        nb = (2 * q + 2) * a_bytes if eb == 4 else a_bytes * (1 + 2 * eb / 4 + (2 * q + 2) * eb / 4)
        p50 = percentile(ts, 50)
        out[name] = {"p50_ms": p50, "p99_ms": percentile(ts, 99), "solves_per_s": 1e3 / float(np.mean(ts)),
                     "hbm_gbs_algorithmic": nb / (p50 * 1e-3) / 1e9, "status": int(st.item()),
                     "max_sigma_err_rel_sigma1": float(np.abs(s64 - sig[:k]).max() / sig[0]),
                     "max_sigma_rel_err": float((np.abs(s64 - sig[:k]) / sig[:k]).max()),
                     "resid_fro_over_opt": float(np.sqrt(acc)) / opt}
        del U, s, V
    # the faster randomized k-SVD of Alg. 5.3 on the same A (two passes):
    # s = 128 (> k), composite row sketch to p_cs = 4096 then SRHT to p = 1024
    fs, fpcs, fp = 128, 4096, 1024
    h.set_autotune(True)
    U, s, V, st = h.rsvd_faster(A, k, fs, fpcs, fp, seed, "srht")
    h.set_autotune(False)
    ts = lat(lambda: h.rsvd_faster(A, k, fs, fpcs, fp, seed, "srht"), reps)
    s64 = s.double().cpu().numpy()
    acc = 0.0
    for r0 in range(0, m, 8192):
        blk = A[r0:r0 + 8192] - (U[r0:r0 + 8192] * s[None, :]) @ V.t()
        acc += float(torch.linalg.vector_norm(blk.double()) ** 2)
    p50 = percentile(ts, 50)
    out["faster_ksvd_fp32"] = {"s": fs, "p_cs": fpcs, "p": fp, "kind2": "srht", "p50_ms": p50,
                               "p99_ms": percentile(ts, 99), "solves_per_s": 1e3 / float(np.mean(ts)),
                               "hbm_gbs_algorithmic": 2 * a_bytes / (p50 * 1e-3) / 1e9,
                               "status": int(st.item()),
                               "max_sigma_err_rel_sigma1": float(np.abs(s64 - sig[:k]).max() / sig[0]),
                               "resid_fro_over_opt": float(np.sqrt(acc)) / opt}
    del U, s, V
    del A
    torch.cuda.empty_cache()
    return out


def serving_leg(count, factors=(1.0,)):
    """Serving workload: `count` requests (half rsvd, half CountSketch LSR,
    m log-uniform in [4096, 262144], n in [32, 512], matrices generated on
    the device from per-request seeds, inside both paths' latency).  First
    the plain comparator (one request at a time, same library calls) with
    all requests arriving at once gives its saturation throughput; then both
    are run with Poisson arrivals at each factor times that rate.  The memory
    budget is 200 GB scaled by count / 10000 (the share of a 10,000-request
    run); it covers the server's stream workspaces (reserved at start) and
    the admitted requests.  Results leave the device as they complete."""
    import numpy as np

    import synth
    from paper_1505_07570_amd import serve
    reqs = synth.serving_mix(count)
    make = synth.serving_request
    # warm up workspaces and code paths
    h0 = serve.Handle()
    for q in reqs[:4]:
        A, b = make(q)
        serve._solve_one(h0, q, A, b)
    del h0
    import torch
    torch.cuda.synchronize()

    def drop(rid, o):
        pass

    _, _, wall_sat = serve.run_plain(reqs, np.zeros(count), make, on_done=drop)
    rate = count / wall_sat
    print(f"serving: plain saturation {rate:.1f} solves/s", file=sys.stderr, flush=True)
    budget = int(200e9 * count / 10000)
    req_bytes = sum(4 * q["m"] * q["n"] for q in reqs)

    def summary(lat, wall):
        v = [lat[i] * 1e3 for i in sorted(lat)]
        return {"p50_ms": serve.percentile(v, 50), "p99_ms": serve.percentile(v, 99),
                "solves_per_s": len(v) / wall, "hbm_gbs_of_A": req_bytes / wall / 1e9}

    out = {"requests": count, "saturation_solves_per_s_plain": rate, "budget_bytes": budget,
           "latency_includes": "on-device generation of each request's matrix", "by_arrival_rate": {}}
    for f in factors:
        arrivals = synth.poisson_arrivals(count, f * rate)
        _, lat_p, wall_p = serve.run_plain(reqs, arrivals, make, on_done=drop)
        print(f"serving: {f:g}x plain done ({wall_p:.1f} s)", file=sys.stderr, flush=True)
        srv = serve.Server(budget, streams=4)
        _, lat_s, wall_s = srv.run(reqs, arrivals, make, on_done=drop)
        print(f"serving: {f:g}x served done ({wall_s:.1f} s)", file=sys.stderr, flush=True)
        out["by_arrival_rate"][f"{f:g}x"] = {
            "arrival_rate_per_s": f * rate, "plain_one_at_a_time": summary(lat_p, wall_p),
            "served": summary(lat_s, wall_s), "peak_admitted_bytes": srv.peak_bytes,
            "reserved_workspace_bytes": srv.reserved, "rejected": len(srv.rejected)}
        del srv
        torch.cuda.empty_cache()
    return out


def nystrom_leg(h, reps):
    """Nystrom on 200,000 Gaussian-mixture points in 32 dimensions with
    c = 1024 sampled columns (k = 820): time and the relative error of L L^T
    against K on 10^6 sampled entries."""
    import numpy as np
    import torch

    import synth
    from paper_1505_07570_amd import serve
    n, c = 200000, 1024
    X, sigma = synth.gmm_points(n=n)
    Xd = torch.from_numpy(X).cuda()
    h.nystrom(Xd, sigma, c, synth.sketch_seed(4))
    ts = []
    for _ in range(reps):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        L, idx, C, ev, st = h.nystrom(Xd, sigma, c, synth.sketch_seed(4))
        z.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(z))
    g = np.random.default_rng(17)
    i = torch.from_numpy(g.integers(0, n, 10 ** 6)).cuda()
    j = torch.from_numpy(g.integers(0, n, 10 ** 6)).cuda()
    Xi, Xj = Xd[i].double(), Xd[j].double()
    K = torch.exp(-((Xi - Xj) ** 2).sum(1) / (2 * sigma * sigma))
    A = (L[i].double() * L[j].double()).sum(1)
    err = float(torch.linalg.vector_norm(K - A) / torch.linalg.vector_norm(K))
    out = {"n": n, "d": 32, "c": c, "k": L.shape[1], "p50_ms": serve.percentile(ts, 50),
           "rel_err_LLt_vs_K_sampled_1e6": err, "status": int(st.item()),
           "C_bytes": n * c * 4}
    del L, C
    # Gaussian-projection variant: C = K Omega over the implicit 200,000^2 K
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    Lg, Cg, evg, stg = h.nystrom_gaussian(Xd, sigma, c, synth.sketch_seed(4))
    z.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(z)
    Ag = (Lg[i].double() * Lg[j].double()).sum(1)
    out["gaussian_variant"] = {
        "ms": ms, "status": int(stg.item()),
        "rel_err_LLt_vs_K_sampled_1e6": float(torch.linalg.vector_norm(K - Ag) / torch.linalg.vector_norm(K)),
        "mfma_tflops": 2.0 * n * n * c / (ms * 1e-3) / 1e12}
    del Lg, Cg
    # faster SPSD sketching (Alg. 6.1) on the same points: s = 1024 uniform
    # columns, p = 4 s leverage-score draws joined with S; error of
    # Q_C Z Q_C^T on the same sampled entries
    s_, p_ = 1024, 4096
    h.spsd_faster(Xd, sigma, s_, p_, synth.sketch_seed(4))
    ts = []
    for _ in range(reps):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        Qc, Z, S, P, st = h.spsd_faster(Xd, sigma, s_, p_, synth.sketch_seed(4))
        z.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(z))
    As = ((Qc[i] @ Z) * Qc[j]).sum(1)
    out["spsd_faster"] = {"s": s_, "p": p_, "P_len": int(P.numel()), "p50_ms": serve.percentile(ts, 50),
                          "status": int(st.item()),
                          "rel_err_vs_K_sampled_1e6": float(torch.linalg.vector_norm(K - As) /
                                                            torch.linalg.vector_norm(K))}
    del Qc, Z
    # faster CUR (Sec. 6.6.3) of K(Xtest, Xtrain): the first 20,000 points as
    # test points, the other 180,000 as training points; c = r = 512,
    # p_c = p_r = 2 (c + r) as in the listing; uniform and leverage P_C, P_R
    mt = 20000
    Xte, Xtr = Xd[:mt], Xd[mt:]
    ci = torch.from_numpy(g.integers(0, mt, 10 ** 6)).cuda()
    cj = torch.from_numpy(g.integers(0, n - mt, 10 ** 6)).cuda()
    Kc = torch.exp(-((Xte[ci].double() - Xtr[cj].double()) ** 2).sum(1) / (2 * sigma * sigma))
    cc = rr = 512
    pcr = 2 * (cc + rr)
    out["cur_faster"] = {"m": mt, "n": n - mt, "c": cc, "r": rr, "p_c": pcr, "p_r": pcr}
    for mode in ("uniform", "leverage"):
        h.cur_faster(Xte, Xtr, sigma, cc, rr, pcr, pcr, synth.sketch_seed(4), mode)
        ts = []
        for _ in range(reps):
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            C, U, R, SC, SR, PC, PR, st = h.cur_faster(Xte, Xtr, sigma, cc, rr, pcr, pcr,
                                                       synth.sketch_seed(4), mode)
            z.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(z))
        Ac = ((C[ci].double() @ U) * R.t()[cj].double()).sum(1)
        out["cur_faster"][mode] = {"p50_ms": serve.percentile(ts, 50), "status": int(st.item()),
                                   "rel_err_vs_K_sampled_1e6": float(torch.linalg.vector_norm(Kc - Ac) /
                                                                     torch.linalg.vector_norm(Kc))}
        del C, U, R
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kinds", default="countsketch,srht,gaussian")
    ap.add_argument("--latency-reps", type=int, default=20)
    ap.add_argument("--cpu-rows", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip latency / rsvd side measurements")
    ap.add_argument("--rsvd-reps", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serving-sweep", type=int, default=0, metavar="N",
                    help="run only the serving workload on N requests at 0.5, 1, 2 and 4 times "
                         "the plain path's saturation rate")
    ap.add_argument("--only-rsvd-spectrum", action="store_true",
                    help="run only the 65536 x 8192 rsvd leg (for profiling)")
    ap.add_argument("--only-extras", action="store_true",
                    help="run only the Nystrom and serving legs")
    ap.add_argument("--traffic-run", action="store_true",
                    help="run only the dispatches read by the FETCH_SIZE / WRITE_SIZE counter runs")
    ap.add_argument("--traffic-summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from the two counter-collection CSVs")
    args = ap.parse_args()
    if args.traffic_summarize:
        kinds = [k.strip() for k in args.kinds.split(",") if k.strip()]
        print(json.dumps(summarize_traffic(*args.traffic_summarize, kinds)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs the sketching path on a single "
              "MI355X (the multi-GPU sharding is a design, not a measured configuration).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1505_07570_amd as rmm
    if not os.path.exists(rmm.LIB_PATH):
        from paper_1505_07570_amd import build as _b
        _b.build()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)

    def lat(fn, reps):
        ts = []
        for _ in range(reps):
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            z.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(z))
        return ts

    h = rmm.handle()

    def tune(fn):
        """One untimed call with the GEMM autotuner on (plans kept per shape)."""
        h.set_autotune(True)
        fn()
        torch.cuda.synchronize()
        h.set_autotune(False)

    if args.serving_sweep > 0:
        print(json.dumps({"serving": serving_leg(args.serving_sweep, (0.5, 1.0, 2.0, 4.0))}), flush=True)
        return
    if args.only_rsvd_spectrum:
        print(json.dumps({"rsvd_65536x8192": rsvd_spectrum(h, args.rsvd_reps, lat)}), flush=True)
        return
    if args.only_extras:
        ex = {"nystrom_200000x32_c1024": nystrom_leg(h, args.rsvd_reps)}
        if args.serve_requests > 0:
            ex["serving"] = serving_leg(args.serve_requests)
        print(json.dumps(ex), flush=True)
        return

    kinds = [k.strip() for k in args.kinds.split(",") if k.strip()]
    s, seed = 4096, synth.sketch_seed(2)
    t0 = time.perf_counter()
    A, b, xs = synth.lsr_fp32()
    gen_s = time.perf_counter() - t0
    m, d = A.shape
    Ad = torch.from_numpy(A.T.copy()).cuda().t()   # column-major, lda = m
    bd = torch.from_numpy(b).cuda()
    C = {k: torch.empty(d + 1, s, dtype=torch.float32, device="cuda").t() for k in kinds}
    res = {k: torch.empty(1, dtype=torch.float64, device="cuda") for k in kinds}
    xsol = {}
    ab_bytes = (m * (d + 1)) * 4
    if args.traffic_run:
        traffic_workload(h, Ad, bd, C, s, seed, kinds)
        return

    def step(ev=None):
        for k in kinds:
            if ev is not None:
                ev[k][0].record()
            h.sketch(Ad, s, k, seed, b=bd, out=C[k])
            if ev is not None:
                ev[k][1].record()
            x, st = h.lsr_solve(C[k], d)
            h.residual(Ad, bd, x, out=res[k])
            xsol[k] = x

    tune(step)  # the solves' dense products get their tuned plans
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for k in kinds} for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for i in range(args.steps):
        step(evs[i])
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    sketch_ms = {k: float(np.mean([ev[k][0].elapsed_time(ev[k][1]) for ev in evs])) for k in kinds}
    value = len(kinds) * ab_bytes / (ms_step * 1e-3) / 1e9

    # each family's main sketch kernel alone: HIP events that the library
    # records on its stream right around that launch (same workload and
    # launch configuration as the steps; rmm_set_kernel_timing)
    h.set_kernel_timing(True)
    kernel_ms = {}
    for k in kinds:
        ts = []
        for _ in range(args.steps):
            h.sketch(Ad, s, k, seed, b=bd, out=C[k])
            ts.append(h.kernel_time())
        kernel_ms[k] = float(np.mean(ts))
    h.set_kernel_timing(False)

    # practical HBM read ceiling: one streaming read of [A | b]'s bytes
    # (rmm_stream_read: the sketches' 16-byte nontemporal load pattern, no arithmetic)
    probe = torch.empty(ab_bytes // 16 * 4, dtype=torch.float32, device="cuda")
    sink = torch.empty(4096, dtype=torch.float32, device="cuda")
    h.stream_read(probe, sink)
    read_ms = float(np.median(lat(lambda: h.stream_read(probe, sink), 20)))
    read_gbs = probe.numel() * 4 / (read_ms * 1e-3) / 1e9
    del probe

    # roofline of every sketch kernel; the dominant one is reported as "roofline"
    rl = {}
    for k in kinds:
        t = kernel_ms[k] * 1e-3
        if k == "gaussian":
            flops = 2.0 * s * m * (d + 1)
            rl[k] = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": FP32_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / t / 1e12 / FP32_MFMA_PEAK_TFLOPS,
                     "traffic": measured_traffic(k)}
        else:
            nb = ab_bytes + s * (d + 1) * 4
            rl[k] = {"bound": "hbm", "achieved": nb / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": nb / t / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic(k),
                     "call_frac": nb / (sketch_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "frac_of_read_reference": nb / t / 1e9 / read_gbs}
        rl[k]["kernel_ms"] = kernel_ms[k]
    dominant = max(kinds, key=lambda k: kernel_ms[k])

    out = {
        "metric": "sketch GB/s of A & % roofline; rsvd/LSR solves/sec; p50/p99 latency vs plain",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sketch-and-solve LSR, A 1048576x256 fp32 (Student-t leverage) "
                               f"+ b, s={s}, families={','.join(kinds)}; per family: sketch, "
                               "fp64 CholeskyQR2 solve, fp64 residual",
                   "m": m, "d": d, "s": s, "parallelism": "single GPU"},
        "roofline": dict(rl[dominant], kernel=f"{dominant} sketch"),
        "roofline_by_kernel": rl,
        "sketch_ms": sketch_ms,
        "kernel_ms": kernel_ms,
        "sketch_gbs": {k: ab_bytes / (sketch_ms[k] * 1e-3) / 1e9 for k in kinds},
        "hbm_read_reference": {"GB/s": read_gbs, "frac_of_peak": read_gbs / HBM_PEAK_GBS,
                               "what": "rmm_stream_read of the bytes of [A | b]: 16-byte "
                                       "nontemporal loads, no arithmetic"},
        "data_gen_s": gen_s,
    }

    if not args.no_extras:
        R = args.latency_reps
        lsr_lat = {}
        for k in kinds:
            ts = lat(lambda: h.sketched_lsr(Ad, bd, s, k, seed), R)
            lsr_lat[k] = {"p50_ms": percentile(ts, 50), "p99_ms": percentile(ts, 99),
                          "solves_per_s": 1e3 / float(np.mean(ts))}
        tune(lambda: h.plain_lsr(Ad, bd))
        ts = lat(lambda: h.plain_lsr(Ad, bd), R)
        xp, rp, _ = h.plain_lsr(Ad, bd)
        out["lsr_latency"] = lsr_lat
        out["plain_lsr"] = {"p50_ms": percentile(ts, 50), "p99_ms": percentile(ts, 99),
                            "method": "fp64 normal equations on the GPU"}
        out["objective_ratio"] = {k: (float(res[k].item()) / float(rp.item())) ** 2 for k in kinds}
        # composite sketch (Sec. 3.2.4): CountSketch to s1 = 4 s rows, then a
        # Gaussian projection or SRHT to s; the same sketch-and-solve after it
        comp = {}
        s1 = 4 * s
        Cc = torch.empty(d + 1, s, dtype=torch.float32, device="cuda").t()
        for k2 in ("gaussian", "srht"):
            fn = lambda: h.sketch_composite(Ad, s1, s, k2, seed, b=bd, out=Cc)
            fn()
            ts = lat(fn, R)
            xc, _ = h.lsr_solve(Cc, d)
            rc = h.residual(Ad, bd, xc)
            p50 = percentile(ts, 50)
            comp["countsketch+" + k2] = {"s1": s1, "p50_ms": p50, "p99_ms": percentile(ts, 99),
                                         "gbs_of_A": ab_bytes / (p50 * 1e-3) / 1e9,
                                         "objective_ratio": (float(rc.item()) / float(rp.item())) ** 2}
        out["composite_sketch"] = comp
        # machine-precision LSR (Alg. 4.1): sketch-and-solve start, 20 CG steps
        # (one fused FP64 pass over A each); objective ratio against the
        # normal-equation solve, and per-step time from the 0- and 20-step runs
        prec = {}
        for k in ("countsketch", "srht"):
            tune(lambda: h.precise_lsr(Ad, bd, s, k, seed, 1))
            ts0 = lat(lambda: h.precise_lsr(Ad, bd, s, k, seed, 0), R)
            ts = lat(lambda: h.precise_lsr(Ad, bd, s, k, seed, 20), R)
            _, rr, _ = h.precise_lsr(Ad, bd, s, k, seed, 20)
            step_ms = (percentile(ts, 50) - percentile(ts0, 50)) / 20
            prec[k] = {"iters": 20, "p50_ms": percentile(ts, 50), "p99_ms": percentile(ts, 99),
                       "ms_per_step": step_ms,
                       "step_hbm_gbs": m * d * 4 / (step_ms * 1e-3) / 1e9,
                       "objective_ratio": (float(rr.item()) / float(rp.item())) ** 2}
        out["precise_lsr"] = prec
        A1, _ = synth.rsvd_fp64()
        A1d = torch.from_numpy(A1.T.copy()).cuda().t()
        tune(lambda: h.rsvd(A1d, 20, 10, 2, synth.sketch_seed(1)))
        ts = lat(lambda: h.rsvd(A1d, 20, 10, 2, synth.sketch_seed(1)), R)
        # the same with the 256 MB Infinity Cache flushed before each solve
        # (a 512 MB write, outside the timed region): A (8.4 MB) then comes
        # from HBM on the first pass
        flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        tsf = []
        for _ in range(R):
            flush.fill_(1)
            torch.cuda.synchronize()
            tsf += lat(lambda: h.rsvd(A1d, 20, 10, 2, synth.sketch_seed(1)), 1)
        del flush
        out["rsvd_2048x512_fp64"] = {"k": 20, "p": 10, "q": 2, "p50_ms": percentile(ts, 50),
                                     "p99_ms": percentile(ts, 99),
                                     "solves_per_s": 1e3 / float(np.mean(ts)),
                                     "cache": "back-to-back solves, A resident in the Infinity Cache",
                                     "p50_ms_cache_flushed": percentile(tsf, 50)}
        # the same config by block Lanczos (Alg. 5.1): 3 Krylov blocks of width
        # 30, next to the prototype's q = 2 (the same 2q + 2 = 6 passes over A)
        # and the projection error of each against the truncated SVD
        seed1 = synth.sketch_seed(1)
        tune(lambda: h.rsvd_lanczos(A1d, 20, 30, 3, seed1))
        tsl = lat(lambda: h.rsvd_lanczos(A1d, 20, 30, 3, seed1), R)
        sv1 = np.linalg.svd(A1, compute_uv=False)
        opt1 = float(np.sqrt((sv1[20:] ** 2).sum()))
        errs = {}
        for nm, fn in (("prototype_q2", lambda: h.rsvd(A1d, 20, 10, 2, seed1)),
                       ("lanczos_3x30", lambda: h.rsvd_lanczos(A1d, 20, 30, 3, seed1))):
            U1, s1, V1, _ = fn()
            R1 = A1 - (U1.double().cpu().numpy() * s1.double().cpu().numpy()) @ V1.double().cpu().numpy().T
            errs[nm] = {"resid_fro_over_opt": float(np.linalg.norm(R1)) / opt1,
                        "max_sigma_rel_err": float((np.abs(s1.double().cpu().numpy() - sv1[:20]) / sv1[:20]).max())}
        out["rsvd_lanczos_2048x512_fp64"] = {"k": 20, "s": 30, "q_blocks": 3,
                                             "p50_ms": percentile(tsl, 50), "p99_ms": percentile(tsl, 99),
                                             "solves_per_s": 1e3 / float(np.mean(tsl)), "errors": errs}
        del A1d
        out["rsvd_65536x8192"] = rsvd_spectrum(h, args.rsvd_reps, lat)
        out["nystrom_200000x32_c1024"] = nystrom_leg(h, args.rsvd_reps)
        if args.serve_requests > 0:
            out["serving"] = serving_leg(args.serve_requests)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, b, s, kinds, seed, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
