"""Throughput benchmark of the N-FHMM variational-inference loop on one MI355X.

A step is one complete fit of a batch of J independent jobs of the paper-typical
shape (S=2 sources, N=40 dictionaries of K=10 elements, F=513 bins, T=1000
frames, 50 iterations): packing, the default start, every iteration (both
dictionary contractions, the forward-backward of every chain, Eq. 6 / Eq. 8 and
the bound) and the separation, with the inputs already resident in HBM.

value = J * T * iterations / seconds per step (frame-iterations/s), FP32
contraction.  The BF16-contraction form and a single job are measured beside it.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12     # MI355X dense FP32 matrix, FLOP/s
PEAK_BF16_MFMA = 2.5e15       # MI355X dense BF16 matrix, FLOP/s
PEAK_HBM = 8.0e12             # B/s
PEAK_FP32_VALU = 157.3e12     # MI355X FP32 vector, FLOP/s


def _traffic_record(record):
    """A committed counter record (rocprofv3 FETCH_SIZE + WRITE_SIZE per kernel,
    scaled by a plain copy), if it was taken on the current sources of the kernels
    it covers; else None."""
    from paper_1206_6468_amd.rocprof_summary import KERNEL_SOURCES, kernel_source_hash
    path = os.path.join(ROOT, "profiles", record)
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash(tuple(d.get("kernel_sources", KERNEL_SOURCES))):
        return None
    return d


def _traffic_for(kernel, workload, record="hbm_traffic.json"):
    """Measured HBM bytes per launch of `kernel` (its FP32 instantiation when the
    record names template arguments) on this workload, from a current record; else None."""
    d = _traffic_record(record)
    if d is None:
        return None
    for name, e in d.get("kernels", {}).items():
        if (name == kernel or name.startswith(kernel + "<false")) and e.get("workload") == workload:
            return e.get("bytes_per_launch")
    return None


def bf16_bytes_per_frame_iteration(S, N, K, F, T):
    """Algorithmic HBM bytes per frame-iteration of the BF16-contraction form: the
    least that must cross each iteration's boundary -- V read once (4 F), the
    carried alpha-hat read and written in float32 (8 M), the chain rows (evidence
    and marginals, 8 S N) and one bfloat16 copy of the dictionary read once per
    iteration and shared by the T frames (2 F M / T)."""
    M = S * N * K
    return 4.0 * F + 8.0 * M + 8.0 * S * N + 2.0 * F * M / T


def bf16_measured_bytes(J, T, iters, record="hbm_traffic_bf16.json"):
    """HBM bytes per frame-iteration that the BF16 form's iteration kernels move by
    counter, from a current record of one fit of the same batch (bench.py --bf16-only
    --steps 1 --warmup 0: every dispatch of these kernels belongs to its `iters`
    iterations, plus the default start's one launch of each contraction); else None."""
    d = _traffic_record(record)
    if d is None:
        return None
    per_iter = ("k_spectrum", "k_counts", "k_counts_bf16", "k_update", "k_fb_round", "k_fb_fixup", "k_posterior",
                "k_chain_exact")
    tot = sum(e["bytes_per_launch"] * e["dispatches"] for name, e in d.get("kernels", {}).items()
              if name.split("<")[0] in per_iter)
    return tot / (iters * J * T)


def make_jobs(cfg, n, iters=None):
    from gen import make_problem
    probs = []
    for j in range(n):
        p = make_problem(cfg, j)
        if iters is not None:
            p = dict(p, iters=iters)
        probs.append(p)
    return probs


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_batch(L, ctx, jobs, precision, steps, warmup, profile=False, kinds=None):
    """Seconds per fit of `jobs`; with `profile`, HIP-event times of the kernel
    kinds `kinds` (None: all) recorded over the same timed steps."""
    import torch
    log(f"{len(jobs)} jobs, {precision}: {warmup} warm-up + {steps} timed steps")
    for _ in range(warmup):
        L.fit_batch_device(ctx, jobs, precision)
    torch.cuda.synchronize()
    if profile:
        L.profile_select(ctx, kinds)
        L.profile_enable(ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        L.fit_batch_device(ctx, jobs, precision)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = None
    if profile:
        prof = {k: L.profile_read(ctx, k)
                for k in (kinds or ("spectrum", "counts", "chains", "posterior", "update"))}
        L.profile_enable(ctx, False)
        L.profile_select(ctx, None)
    return dt, prof


def serving_problems(n_jobs):
    """The serving-mix problems, drawn on host threads (no child processes: the
    bench process holds GPU state once it has run a fit)."""
    from concurrent.futures import ThreadPoolExecutor

    from gen import make_problem
    log(f"serving: generating {n_jobs} serving-mix problems")
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda j: make_problem(4, j), range(n_jobs)))


def serving(L, probs, budget_bytes, max_slots, load=0.8, seed=4):
    """Serving form: n_jobs serving-mix jobs (S in {2,3}, T in [200, 4000], 50
    iterations, BF16 contraction) through nfhmm_submit / nfhmm_wait on a context
    with a device-memory budget.  First all jobs at once (saturated throughput),
    then Poisson arrivals at `load` x the saturated job rate (latency from the
    scheduled arrival to the outputs in host memory), then the same jobs one at a
    time with nfhmm_fit in FP32 as the sequential baseline."""
    import threading

    import numpy as np

    n_jobs = len(probs)
    work = sum(p["T"] * p["iters"] for p in probs)
    ctx = L.Context(0, hbm_budget_bytes=budget_bytes, max_slots=max_slots)
    try:
        L.wait(ctx, L.submit(ctx, dict(probs[0], iters=2), "bf16"))    # warm-up

        log("serving: saturated (all jobs queued at once)")
        t0 = time.perf_counter()
        subs = [L.submit(ctx, p, "bf16") for p in probs]
        lat_sat = [L.wait(ctx, s)[1] for s in subs]
        t_sat = time.perf_counter() - t0
        rate = load * n_jobs / t_sat

        # the same into pinned output arrays, which the library copies into
        # directly (no pass through its pinned ring and host copy pool)
        log("serving: saturated, outputs into pinned host arrays")
        # pinning memory is slow the first time: the same arrays once beforehand,
        # released to torch's caching host allocator, which hands them back below
        warm = []
        for p in probs:
            L._alloc_outputs(p, warm, L.OUTPUTS, True)
        del warm
        t0 = time.perf_counter()
        subs = [L.submit(ctx, p, "bf16", pinned=True) for p in probs]
        for sb in subs:
            L.wait(ctx, sb)
        t_pin = time.perf_counter() - t0
        del subs

        # the same, bringing back only the posteriors and the separations (not
        # alpha-hat, 40 % of the bytes): how much of the saturated time is the
        # host<->device copies
        log("serving: saturated, posteriors and separations only")
        t0 = time.perf_counter()
        subs = [L.submit(ctx, p, "bf16", outputs=("post", "sep", "elbo")) for p in probs]
        for sb in subs:
            L.wait(ctx, sb)
        t_sep = time.perf_counter() - t0

        log(f"serving: Poisson arrivals at {rate:.1f} jobs/s")
        rng = np.random.default_rng(seed)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_jobs))
        lags, subs = [None] * n_jobs, [None] * n_jobs
        ready = [threading.Event() for _ in range(n_jobs)]

        def submitter(t_start):
            for j, a in enumerate(arrivals):
                d = t_start + a - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                subs[j] = L.submit(ctx, probs[j], "bf16")
                lags[j] = time.perf_counter() - (t_start + a)
                ready[j].set()

        t_start = time.perf_counter()
        th = threading.Thread(target=submitter, args=(t_start,))
        th.start()
        lat = []
        for j in range(n_jobs):
            ready[j].wait()
            lat.append(lags[j] + L.wait(ctx, subs[j])[1])
        t_end = time.perf_counter()
        th.join()
        lat_ms = np.array(lat) * 1e3
    finally:
        ctx.close()

    # the same mix as one blocking BF16 batch: with host arrays (the copies of
    # serving, but no admission, rounds or overlap), then with the inputs resident
    # (the device-side rate of this mix, which serving's rounds approach when the
    # copies are free)
    log("serving: the same jobs as one blocking BF16 batch, host arrays / resident inputs")
    import torch
    ctx = L.Context(0)
    try:
        L.fit_batch(ctx, [dict(p, iters=2) for p in probs[:4]], "bf16")
        t0 = time.perf_counter()
        L.fit_batch(ctx, probs, "bf16")
        t_bh = time.perf_counter() - t0

        # the same with the caller's input and output arrays in pinned host
        # memory: the library copies them directly (no ring, no copy pool)
        log("serving: the same blocking batch, inputs and outputs in pinned host arrays")

        def _pin(x):
            t = torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
            t.numpy()[...] = x
            return t.numpy()
        pprobs = [dict(p, **{k: _pin(p[k]) for k in ("V", "W", "A", "pi")}) for p in probs]
        warm = []
        for p in probs:
            L._alloc_outputs(p, warm, L.OUTPUTS, True)
        del warm
        t0 = time.perf_counter()
        L.fit_batch(ctx, pprobs, "bf16", pinned=True)
        t_bp = time.perf_counter() - t0
        del pprobs
        djobs = [L.DeviceJob(p) for p in probs]
        L.fit_batch_device(ctx, djobs, "bf16")          # warm: arenas and tables for these shapes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.fit_batch_device(ctx, djobs, "bf16")
        torch.cuda.synchronize()
        t_bd = time.perf_counter() - t0
        del djobs

        log("serving: sequential FP32 baseline (one job at a time)")
        L.fit(ctx, dict(probs[0], iters=2), "fp32")
        t0 = time.perf_counter()
        for p in probs:
            L.fit(ctx, p, "fp32")
        t_seq = time.perf_counter() - t0
    finally:
        ctx.close()
    return {
        "jobs": n_jobs, "precision": "bf16", "budget_bytes": budget_bytes, "max_slots": max_slots,
        "frame_iterations": work,
        "saturated": {"seconds": t_sat, "jobs_per_s": n_jobs / t_sat, "frame_iterations_per_s": work / t_sat,
                      "p50_ms": float(np.percentile(np.array(lat_sat) * 1e3, 50)),
                      "p99_ms": float(np.percentile(np.array(lat_sat) * 1e3, 99))},
        "saturated_pinned_outputs": {"seconds": t_pin, "frame_iterations_per_s": work / t_pin,
                                     "note": "output arrays in pinned host memory, copied into directly"},
        "saturated_without_alpha": {"seconds": t_sep, "frame_iterations_per_s": work / t_sep,
                                    "note": "the same jobs bringing back d-hat, V* and the bound only"},
        "copied_gb": {"in": sum(p["V"].nbytes + p["W"].nbytes + p["A"].nbytes + p["pi"].nbytes for p in probs) / 1e9,
                      "out": sum(p["T"] * p["S"] * p["N"] * p["K"] * 4 + p["S"] * p["T"] * (p["N"] + p["F"]) * 4
                                 for p in probs) / 1e9},
        "poisson": {"load": load, "rate_jobs_per_s": rate, "seconds": t_end - t_start,
                    "frame_iterations_per_s": work / (t_end - t_start),
                    "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                    "mean_ms": float(lat_ms.mean()), "max_submit_lag_ms": float(max(lags) * 1e3)},
        "blocking_bf16_host_arrays": {"seconds": t_bh, "frame_iterations_per_s": work / t_bh,
                                      "saturated_serving_over_this": t_bh / t_sat},
        "blocking_bf16_pinned_arrays": {"seconds": t_bp, "frame_iterations_per_s": work / t_bp,
                                        "note": "inputs and outputs in pinned host memory, copied directly"},
        "blocking_bf16_resident": {"seconds": t_bd, "frame_iterations_per_s": work / t_bd,
                                   "saturated_serving_over_this": t_bd / t_sat},
        "sequential_fp32": {"seconds": t_seq, "frame_iterations_per_s": work / t_seq,
                            "mean_job_ms": t_seq / n_jobs * 1e3},
        "note": "latency = scheduled arrival -> outputs in host memory (includes host<->device copies)",
    }


def stft_bench(L, ctx, jobs=32, sources=2, frames=1000, nfft=1024, hop=256, reps=5):
    """The time-frequency front and back end at the paper's analysis (16 kHz,
    64 ms windows, 16 ms hop): the STFT of `jobs` mixtures of `frames` frames in
    one call, then the inverse of `sources` masked spectrograms per mixture with
    its phase, all mixtures in one call, on device-resident data, timed with HIP
    events on the stream the calls use.  Algorithmic bytes: the forward reads
    every sample once and writes |X| and arg X; the inverse reads the magnitudes
    and each mixture's phase once and writes the signals."""
    import torch
    F = nfft // 2 + 1
    n = (frames - 1) * hop + nfft
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(7)
    x = torch.randn((jobs, n), generator=g, device=dev)
    mag = torch.empty((jobs, frames, F), device=dev)
    phase = torch.empty_like(mag)
    src = torch.rand((jobs, sources, frames, F), generator=g, device=dev)
    y = torch.empty((jobs, sources, n), device=dev)
    torch.cuda.synchronize()
    # a stream of its own: torch's default stream has the handle 0, which the
    # library reads as "no stream" (its own), and the events would not bracket it
    st = torch.cuda.Stream()
    L.stft_device(ctx, x, mag, phase, nfft, hop, stream=st)
    L.istft_device(ctx, src, phase, y, nfft, hop, stream=st)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(st)
    for _ in range(reps):
        L.stft_device(ctx, x, mag, phase, nfft, hop, stream=st)
    e[1].record(st)
    for _ in range(reps):
        L.istft_device(ctx, src, phase, y, nfft, hop, stream=st)
    e[2].record(st)
    torch.cuda.synchronize()
    ms_f = e[0].elapsed_time(e[1]) / reps
    ms_i = e[1].elapsed_time(e[2]) / reps
    bytes_f = jobs * n * 4 + 2 * jobs * frames * F * 4
    bytes_i = jobs * sources * frames * F * 4 + jobs * frames * F * 4 + jobs * sources * n * 4
    rec, wl = f"stft_hbm_traffic_T{frames}-nfft{nfft}-hop{hop}_x{jobs}.json", \
        f"stft-T{frames}-nfft{nfft}-hop{hop}-x{jobs}-S{sources}"

    def roof(kernel, nbytes, ms):
        # HBM-bound in principle; LDS and barriers bound it in practice
        return {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": nbytes / (ms * 1e-3) / PEAK_HBM, "algorithmic_bytes_per_launch": nbytes,
                "traffic": _traffic_for(kernel, wl, rec)}
    return {
        "roofline": {"k_stft": roof(f"k_stft<{nfft}>", bytes_f, ms_f),
                     "k_istft": roof(f"k_istft<{nfft}>", bytes_i, ms_i)},
        "workload": f"{jobs} mixtures of {n} samples (T={frames}, nfft={nfft}, hop={hop}), {sources} sources each",
        "stft_ms": ms_f, "stft_frames_per_s": jobs * frames / (ms_f * 1e-3),
        "stft_gbps": bytes_f / (ms_f * 1e-3) / 1e9, "stft_frac_hbm": bytes_f / (ms_f * 1e-3) / PEAK_HBM,
        "istft_ms": ms_i, "istft_frames_per_s": jobs * sources * frames / (ms_i * 1e-3),
        "istft_gbps": bytes_i / (ms_i * 1e-3) / 1e9, "istft_frac_hbm": bytes_i / (ms_i * 1e-3) / PEAK_HBM,
    }


def em_bench(L, ctx, iters=20, reps=3, sources=32):
    """EM learning of one source's N-HMM (Section 2.1) at the separation's source
    shapes (N=40 states of K=10 elements, F=513, T=1000), inputs resident on the
    device, `iters` iterations per call, timed over `reps` calls.  Algorithmic work
    per frame-iteration: the three (F x K) by (K x N)-per-state products of an
    iteration -- P = theta beta in the E-step (double), and the theta and beta
    updates' sums (float) -- 6 N K F flops, against the FP32 vector peak.  Then
    `sources` such problems (one model per speaker) in one batched call."""
    import torch

    from gen import make_nhmm_problem
    p = make_nhmm_problem(1, 0, iters=iters)
    job = L.DeviceNhmm(p)
    L.learn_nhmm_device(ctx, job)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        L.learn_nhmm_device(ctx, job)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    N, K, F, T = p["N"], p["K"], p["F"], p["T"]
    v = T * iters / dt
    fl = 6.0 * N * K * F
    tr = job.loglik.cpu().numpy()
    del job

    # one model per speaker: `sources` such problems in one batched run (host
    # arrays, so the copies in and out are inside the timed call)
    probs = [make_nhmm_problem(1, j, iters=iters) for j in range(sources)]
    L.learn_nhmm_batch(ctx, probs[:2], iters=1)
    t0 = time.perf_counter()
    for _ in range(max(reps - 1, 1)):
        L.learn_nhmm_batch(ctx, probs)
    dtb = (time.perf_counter() - t0) / max(reps - 1, 1)
    vb = sources * T * iters / dtb
    return {"workload": f"N{N}-K{K}-F{F}-T{T}", "iterations": iters, "ms_per_call": dt * 1e3,
            "em_iterations_per_s": iters / dt, "frame_iterations_per_s": v,
            "roofline": {"bound": "alu", "achieved": v * fl / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                         "unit": "TFLOP/s", "frac": v * fl / PEAK_FP32_VALU, "flops_per_frame_iteration": fl},
            "loglik_first_last": [float(tr[0]), float(tr[-1])],
            "batch": {"sources": sources, "ms_per_call": dtb * 1e3,
                      "source_iterations_per_s": sources * iters / dtb, "frame_iterations_per_s": vb,
                      "over_one_source": vb / v,
                      "roofline": {"bound": "alu", "achieved": vb * fl / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                                   "unit": "TFLOP/s", "frac": vb * fl / PEAK_FP32_VALU},
                      "note": "host arrays: copies in and out inside the timed call"}}


def measured_peaks():
    """What library code reaches on this GPU, beside the nominal peaks: a plain
    FP32 GEMM through torch (the vendor BLAS) at 8192^3 and on the shape of one
    k_counts launch, and a 1 GiB device copy, each timed with events after a
    warm-up."""
    import torch
    out = {}
    n = 8192
    a = torch.rand((n, n), device="cuda")
    b = torch.rand((n, n), device="cuda")
    torch.matmul(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        torch.matmul(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["fp32_gemm_vendor_tflops"] = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
    out["fp32_gemm_vendor_frac"] = out["fp32_gemm_vendor_tflops"] * 1e12 / PEAK_FP32_MFMA
    del a, b
    # the same library on the shape of one k_counts launch: 16 jobs, each an
    # (M = 800) x (F = 512) by (F x T = 1000) product (plain GEMM, no epilogue)
    a = torch.rand((16, 800, 512), device="cuda")
    b = torch.rand((16, 512, 1000), device="cuda").contiguous()
    torch.bmm(a, b)
    e0.record()
    for _ in range(reps):
        torch.bmm(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["fp32_gemm_vendor_counts_shape_tflops"] = 2.0 * 16 * 800 * 512 * 1000 / (ms * 1e-3) / 1e12
    out["fp32_gemm_vendor_counts_shape_frac"] = out["fp32_gemm_vendor_counts_shape_tflops"] * 1e12 / PEAK_FP32_MFMA
    del a, b
    src = torch.empty((1 << 28,), device="cuda")   # 1 GiB of float32
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["hbm_copy_gbps"] = 2.0 * src.numel() * 4 / (ms * 1e-3) / 1e9   # read + write
    out["hbm_copy_frac"] = out["hbm_copy_gbps"] * 1e9 / PEAK_HBM
    del src, dst
    # the host link: 256 MiB each way, from pinned and from pageable host memory
    # (what bounds the copies of serving and of the host-array calls)
    dev = torch.empty((1 << 26,), device="cuda")
    for kind, pin in (("pinned", True), ("pageable", False)):
        host = torch.empty((1 << 26,), pin_memory=pin)
        host.fill_(1.0)
        for name, (dst, src) in (("h2d", (dev, host)), ("d2h", (host, dev))):
            dst.copy_(src)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                dst.copy_(src)
            torch.cuda.synchronize()
            out[f"{name}_{kind}_gbps"] = reps * host.numel() * 4 / (time.perf_counter() - t0) / 1e9
        del host
    del dev
    torch.cuda.empty_cache()
    return out


def cpu_baseline(seconds_target=15.0, one_thread=False, config=1):
    """The FP64 oracle on the host cores: job 0 of the given workload (1 =
    paper-typical), one warm-up iteration, then iterations until about
    `seconds_target` seconds have passed (all BLAS threads, or one)."""
    import contextlib

    import numpy as np

    from gen import make_problem
    from oracle import nfhmm_oracle as O
    limit = contextlib.nullcontext()
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
        if one_thread:
            limit, threads = threadpool_limits(limits=1, user_api="blas"), 1
    except Exception:
        threads = 1 if one_thread else os.cpu_count()
    with limit:
        return _cpu_run(make_problem(config, 0), seconds_target, threads, O, np)


def _cpu_run(p, seconds_target, threads, O, np):
    S, N, K = p["S"], p["N"], p["K"]
    V, beta, A, pi = O.paper_arrays(p)
    B = O.mask_B(S, N, K)
    alpha = O.init_alpha(V, beta, B, 1.0, N)
    alpha = O.one_iteration(alpha, V, beta, A, pi, B, 1.0, S, N, K)["alpha"]   # warm-up
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds_target:
        alpha = O.one_iteration(alpha, V, beta, A, pi, B, 1.0, S, N, K)["alpha"]
        n += 1
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(alpha))
    shape = f"S={S},N={N},K={K},F={p['F']},T={p['T']}"
    return {"value": p["T"] * n / dt, "unit": "frame-iterations/s", "cores": int(threads), "kind": "oracle",
            "sample": f"job 0 ({shape}): 1 warm-up + {n} timed FP64 iterations, {dt:.1f} s, "
                      f"{threads} BLAS thread(s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--jobs", type=int, default=32, help="concurrent paper-typical jobs (S=2, N=40, K=10, F=513, T=1000) per step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the BF16 and single-job forms")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-one-lane", action="store_true", help="skip the one-lane roofline pass")
    ap.add_argument("--serving-jobs", type=int, default=256)
    ap.add_argument("--serving-budget-gib", type=float, default=4.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy three times (the reference "
                         "kernel for scaling HBM byte counters) and exit")
    ap.add_argument("--stft-only", action="store_true",
                    help="only time the time-frequency front and back end (STFT of 32 mixtures of "
                         "1000 frames, inverse of 2 sources each) and print its figures")
    ap.add_argument("--em-only", action="store_true",
                    help="only the EM learning of one source model (one JSON line)")
    ap.add_argument("--bf16-only", action="store_true",
                    help="only time the BF16-contraction form of the batch (for a profiler run of its "
                         "kernels) and print its figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no "
              "multi-GPU path (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 64 << 20                       # float32 elements: 256 MiB per buffer
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)
        return

    from paper_1206_6468_amd import nfhmm as L
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.stft_only:
        ctx = L.Context(0)
        print(json.dumps(stft_bench(L, ctx, reps=max(args.steps, 1))), flush=True)
        ctx.close()
        return
    if args.em_only:
        ctx = L.Context(0)
        print(json.dumps(em_bench(L, ctx)), flush=True)
        ctx.close()
        return
    if args.bf16_only:
        probs = make_jobs(1, args.jobs)
        ctx = L.Context(0)
        jobs = [L.DeviceJob(p) for p in probs]
        dtb, profb = time_batch(L, ctx, jobs, "bf16", args.steps, args.warmup, profile=True)
        p0 = probs[0]
        print(json.dumps({"workload": f"S{p0['S']}-N{p0['N']}-K{p0['K']}-F{p0['F']}-T{p0['T']}-x{len(jobs)}",
                          "precision": "bf16", "ms_per_step": dtb * 1e3,
                          "value": len(jobs) * p0["T"] * p0["iters"] / dtb,
                          "kernels_ms_per_launch": {k: v[1] / max(v[0], 1) for k, v in profb.items()}}), flush=True)
        ctx.close()
        return
    # host-side inputs first, before anything touches the GPU
    serving_probs = None if args.no_serving else serving_problems(args.serving_jobs)
    log(f"generating {args.jobs} paper-typical problems")
    probs = make_jobs(1, args.jobs)
    S, N, K, F, T, iters = (probs[0][k] for k in ("S", "N", "K", "F", "T", "iters"))
    M = S * N * K
    ctx = L.Context(0)
    jobs = [L.DeviceJob(p) for p in probs]
    torch.cuda.synchronize()

    # A fully profiled pass (every launch bracketed by events) gives the per-kernel
    # breakdown and names the kernel with the largest summed time; the timed steps
    # then bracket only the two contractions, so that the step time is barely
    # perturbed, and the contract's roofline is that of the dominant one.
    dt_all, prof = time_batch(L, ctx, jobs, "fp32", args.steps, args.warmup, profile=True)
    # the dominant kernel: "chains" times three kernels together (two rounds and the
    # fix-up), so it is not a candidate; of the single kernels the spectrum leads
    dom = max((k for k in prof if k != "chains"), key=lambda k: prof[k][1])
    dt, prof_c = time_batch(L, ctx, jobs, "fp32", args.steps, 1, profile=True, kinds=("spectrum", "counts"))
    J = len(jobs)
    value = J * T * iters / dt

    # achieved = algorithmic flops per launch (2 F M T per job and iteration, times
    # the jobs of the launch) / average launch duration over the timed steps
    flops_per_job_iter = {"spectrum": 2.0 * F * M * T, "counts": 2.0 * F * M * T}
    rows = {}
    for k, (n, ms) in prof.items():
        rows[k] = {"launches": n, "avg_ms": ms / max(n, 1), "total_ms": ms}
        if k in flops_per_job_iter:
            rows[k]["achieved_tflops"] = flops_per_job_iter[k] * J * iters * args.steps / (ms * 1e-3) / 1e12
    workload = f"S{S}-N{N}-K{K}-F{F}-T{T}-x{J}"   # the paper-typical job, J of them in one batch

    def gemm_roof(kname):
        n_g, ms_g = prof_c[kname]
        fl = flops_per_job_iter[kname] * J * iters * args.steps / max(n_g, 1)
        ach = fl / (ms_g / max(n_g, 1) * 1e-3)
        return {"bound": "mfma", "kernel": f"k_{kname}", "achieved": ach / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_MFMA, "traffic": _traffic_for(f"k_{kname}", workload),
                "algorithmic_flops_per_launch": fl, "avg_launch_ms": ms_g / max(n_g, 1)}
    gemm = dom if dom in flops_per_job_iter else "spectrum"
    roofline = dict(gemm_roof(gemm), largest_summed_time=f"k_{dom}", kernels=rows,
                    kernels_note="from a separate, fully profiled pass of the same steps "
                                 f"({dt_all * 1e3:.2f} ms per step with every launch timed); the jobs run in two "
                                 "stream lanes of 16, whose launches overlap, so each launch shares the chip; "
                                 "'chains' is three kernels (two rounds and the fix-up) per launch")
    other = "counts" if gemm == "spectrum" else "spectrum"
    # the whole loop against the FP32 MFMA peak: both contractions' 4 F M flops per
    # frame-iteration at the measured frame-iterations/s
    loop = {"achieved": value * 4.0 * F * M / 1e12, "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
            "frac": value * 4.0 * F * M / PEAK_FP32_MFMA, "flops_per_frame_iteration": 4.0 * F * M,
            "note": "frame-iterations/s x the two contractions' flops per frame-iteration (2 F M each)"}

    extra = {"roofline_" + other: gemm_roof(other), "roofline_loop": loop}
    # the same steps on one stream lane: every launch then has the chip to itself,
    # so this is the contraction's own rate (the two-lane schedule above overlaps
    # one lane's launches with the other's)
    if not args.no_one_lane:
        L.set_lanes(ctx, 1)
        dt1l, prof1 = time_batch(L, ctx, jobs, "fp32", args.steps, 1, profile=True, kinds=("counts",))
        L.set_lanes(ctx, 2)
        n1, ms1 = prof1["counts"]
        fl1 = flops_per_job_iter["counts"] * J * iters * args.steps / max(n1, 1)
        a1 = fl1 / (ms1 / max(n1, 1) * 1e-3)
        extra["roofline_one_lane"] = {"value": J * T * iters / dt1l, "ms_per_step": dt1l * 1e3,
                                      "kernel": "k_counts", "achieved": a1 / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                                      "unit": "TFLOP/s", "frac": a1 / PEAK_FP32_MFMA,
                                      "algorithmic_flops_per_launch": fl1}
    if not args.no_extra:
        # BF16 contraction operands: HBM-bound by its algorithmic bytes per
        # frame-iteration (V read, alpha-hat's w / c round trip in bf16 / f32, the
        # chain rows, the dictionary's bf16 copies once per iteration)
        dtb_all, profb = time_batch(L, ctx, jobs, "bf16", args.steps, 1, profile=True)
        dtb, profb_c = time_batch(L, ctx, jobs, "bf16", args.steps, 0, profile=True, kinds=("counts",))
        vb = J * T * iters / dtb
        bytes_fi = bf16_bytes_per_frame_iteration(S, N, K, F, T)
        tb = flops_per_job_iter["counts"] * J * iters * args.steps / (profb_c["counts"][1] * 1e-3)
        extra["bf16"] = {"value": vb, "ms_per_step": dtb * 1e3,
                         "roofline_loop": {"bound": "hbm", "achieved": vb * bytes_fi / 1e9, "peak": PEAK_HBM / 1e9,
                                           "unit": "GB/s", "frac": vb * bytes_fi / PEAK_HBM,
                                           "algorithmic_bytes_per_frame_iteration": bytes_fi},
                         "k_counts_tflops": tb / 1e12, "k_counts_frac_of_bf16_peak": tb / PEAK_BF16_MFMA,
                         "measured_bytes_per_frame_iteration": bf16_measured_bytes(J, T, iters),
                         "kernels_ms_per_launch": {k: v[1] / max(v[0], 1) for k, v in profb.items()},
                         "dominant": max(profb, key=lambda k: profb[k][1])}
        # three sources (S=3, N=40, K=10, F=513, T=1000): the cost is linear in S
        log("three-source jobs")
        p3s = make_jobs(2, J)
        j3s = [L.DeviceJob(p) for p in p3s]
        del p3s
        dts3, prof3 = time_batch(L, ctx, j3s, "fp32", max(2, args.steps // 2), 1, profile=True,
                                 kinds=("spectrum", "counts"))
        M3 = 3 * N * K
        v3 = J * T * iters / dts3
        extra["three_sources_fp32"] = {
            "workload": f"S3-N{N}-K{K}-F{F}-T{T}-x{J}", "value": v3, "ms_per_step": dts3 * 1e3,
            "roofline_loop": {"achieved": v3 * 4.0 * F * M3 / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                              "unit": "TFLOP/s", "frac": v3 * 4.0 * F * M3 / PEAK_FP32_MFMA},
            "time_ratio_vs_two_sources": dts3 / dt, "work_ratio_vs_two_sources": 1.5}
        del j3s
        dt1, _ = time_batch(L, ctx, jobs[:1], "fp32", max(2, args.steps), 1)
        extra["single_job_fp32"] = {"value": T * iters / dt1, "ms_per_fit": dt1 * 1e3}
        # batch sizes around the headline one (same per-job workload)
        sweep = {}
        for nj in (8, 128):
            if nj <= J:
                sub = jobs[:nj]
            else:
                from gen import make_problem
                sub = jobs + [L.DeviceJob(make_problem(1, j)) for j in range(J, nj)]
            dts, _ = time_batch(L, ctx, sub, "fp32", 2, 1)
            sweep[str(nj)] = nj * T * iters / dts
            del sub
        sweep["1"] = extra["single_job_fp32"]["value"]
        sweep[str(J)] = value
        extra["jobs_sweep_fp32"] = dict(sorted(sweep.items(), key=lambda kv: int(kv[0])))
        # the long precision-form job (S=2, N=60, K=20, F=1025, T=4000), one job, timed over 10 iterations
        p3 = dict(make_jobs(3, 1)[0], iters=10)
        j3 = [L.DeviceJob(p3)]
        c3 = {"iterations_timed": 10}
        for prec in ("fp32", "bf16"):
            dt3, pr3 = time_batch(L, ctx, j3, prec, 2, 1, profile=True)
            c3[prec] = {"value": p3["T"] * 10 / dt3, "ms_per_10_iterations": dt3 * 1e3,
                        "kernels_ms": {k: v[1] / 2 for k, v in pr3.items()}}
        extra["precision_form_single_job"] = c3
        del j3
        # the host-buffer form: nfhmm_fit_batch on host arrays, so the copies of V and
        # W in and of the outputs back are inside the time (never the headline value)
        log("host-buffer fit of the batch")
        import numpy as np
        hp = [{k: (np.ascontiguousarray(v, dtype=np.float32) if isinstance(v, np.ndarray) and v.dtype.kind == "f"
                   else v) for k, v in p.items()} for p in probs]
        L.fit_batch(ctx, hp, "fp32")
        th = []
        for _ in range(2):
            t0 = time.perf_counter()
            L.fit_batch(ctx, hp, "fp32")
            th.append(time.perf_counter() - t0)
        dth = min(th)
        extra["host_buffer_fit_fp32"] = {"value": J * T * iters / dth, "ms_per_fit": dth * 1e3,
                                         "copied_mb": sum(p["V"].nbytes + p["W"].nbytes for p in hp) / 1e6,
                                         "note": "nfhmm_fit_batch on host arrays (V, W in; alpha, posteriors, "
                                                 "separated spectrograms, bounds out), best of 2"}
        del hp
        log("EM learning of one source's N-HMM")
        extra["nhmm_em"] = em_bench(L, ctx)
        log("time-frequency front and back end")
        extra["stft"] = stft_bench(L, ctx)
        log("library GEMM and copy on this GPU")
        extra["measured_peaks"] = measured_peaks()

    out = {
        "metric": "VI frame-iterations/s at S=2,N=40,F=513 (FP32 contraction)",
        "value": value,
        "unit": "frame-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "jobs": J, "S": S, "N": N, "K": K, "F": F, "T": T,
                   "iterations": iters, "contraction": "fp32", "stream_lanes": 2},
        "roofline": roofline,
    }
    out.update(extra)
    if not args.no_serving:
        out["serving"] = serving(L, serving_probs, int(args.serving_budget_gib * (1 << 30)), 64)
    if not args.no_cpu:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline_1thread"] = cpu_baseline(10.0, one_thread=True)
        # the oracle on the small and the long workloads too, each a bounded sample
        out["cpu_baseline_other_workloads"] = {"S2-N5-K8-F129-T100": cpu_baseline(3.0, config=0),
                                               "S2-N60-K20-F1025-T4000": cpu_baseline(10.0, config=3)}
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
