#!/usr/bin/env python3
"""Frames/s of compress + two-time correlation (compressed vs raw) on one MI355X.

One step = compress_frames (basis from the data, randomized subspace
iteration) + correlate_two_time for every q-ROI with the full C written in
FP32 and g2 fused into the same pass, on the 512 x 512 px x 10,000-frame,
36-annulus workload (uint16 counts, k = 64 by default).  The raw path
(exact int8 Gram of the same frames, same C and g2 outputs) is timed beside
it.  Inputs are generated on the device before timing; nothing is copied
from the host inside the timed region.

Prints one JSON line: the metric and its value (frames/s of the compressed
step), the roofline object of the dominant kernel, the CPU oracle baseline, and
the raw path, stream, serving, precision and g2-without-C measurements.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/sec compress+two-time C (compressed vs raw, 1 GPU) at 1e-3 rel err; p99 latency"
PEAK_HBM_GBS = 8000.0
PEAK_I8_TOPS = 5000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def roi_counts_and_sums(labels, n_roi, F=None):
    """|R| per ROI and, for host frames F (n x M), the exact per-frame ROI photon sums
    (plain NumPy bookkeeping for the spot checks and operation counts)."""
    import numpy as np
    lab = np.asarray(labels)
    npix = np.bincount(lab[lab >= 0], minlength=n_roi)[:n_roi].astype(np.int64)
    if F is None:
        return npix, None
    S = np.stack([np.asarray(F)[:, lab == r].astype(np.int64).sum(axis=1) for r in range(n_roi)])
    return npix, S


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frames_host, labels, n_roi, k, seed, n_sample):
    """Time the FP64 oracle on the first n_sample frames: basis + C~ + g2 for every ROI."""
    import numpy as np
    import oracle as O
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        info = [p for p in threadpool_info() if p.get("user_api") == "blas"] or threadpool_info()
        threads = max([int(p.get("num_threads", 1)) for p in info] or [1])
        blas = ", ".join(sorted({f"{p.get('internal_api', '?')} {p.get('version', '')}".strip() for p in info}))
    except Exception:
        threads = os.cpu_count() or 1
    F = np.ascontiguousarray(frames_host[:n_sample])
    t0 = time.perf_counter()
    U, s, V = O.randomized_basis(F, k, 16, 1, seed=seed)
    W = O.encode(F, U)
    S = O.roi_frame_sums(F, labels, n_roi)
    npix = O.roi_pixel_counts(labels, n_roi)
    for r in range(n_roi):
        C = O.compressed_two_time_from_factors(W, O.roi_basis_gram(U, labels, r), S[r], int(npix[r]))
        O.g2_from_two_time(C)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "blas": blas, "host_cpus": os.cpu_count(),
            "sample": f"first {n_sample} frames of the same series ({F.shape[1]} px, {n_roi} ROIs, k={k}): "
                      f"FP64 randomized basis + compressed C and g2 for every ROI, {dt:.1f} s",
            "seconds": dt}


def stream_latency(api, torch, dev, n_blocks):
    """Per-push device time of an online stream at the largest serving shape:
    1024 x 512 px, 36 ROIs, uint8, k = 64, 256-frame blocks, a 4096-frame window
    (lags), band rows written.  The basis is a fixed orthonormal one (the cost does
    not depend on it); pushes after the window has filled are the steady state."""
    import numpy as np
    import synth
    H, Wd, n_roi, k, nb, window = 1024, 512, 36, 64, 256, 4096
    M = H * Wd
    labels = torch.from_numpy(synth.annular_labels(H, Wd, n_roi)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(52000)
    Q, _ = torch.linalg.qr(torch.randn(M, k, device=dev, generator=g, dtype=torch.float32))
    basis = Q.T.contiguous()
    pool = [synth.speckle_frames_torch(M, nb, 0.05, 0.2, 50.0, "u8", seed=52001 + i, device=dev) for i in range(4)]
    ctx = api.Context(0)
    s = api.Stream(ctx, labels, n_roi, basis, window=window, max_block=nb)
    band = torch.empty((n_roi, nb, window), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    times = []
    for i in range(n_blocks):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.push(pool[i % len(pool)], band=band)
        b.record(stream)
        times.append((a, b))
    torch.cuda.synchronize()
    ctx.sync()
    ms = [a.elapsed_time(b) for a, b in times]
    steady = ms[window // nb + 1:] or ms
    g2, npairs = s.g2()
    torch.cuda.synchronize()
    ok = bool(torch.isfinite(g2[:, :window - nb]).all().item())
    s.close()
    ctx.close()
    p50 = percentile(steady, 50)
    return {"workload": "stream_1024x512_36roi_k64_w4096", "block_frames": nb, "pushes": n_blocks,
            "steady_pushes": len(steady), "push_p50_ms": p50, "push_p99_ms": percentile(steady, 99),
            "frames_per_s_one_stream": nb / (p50 / 1e3), "band_bytes_per_push": n_roi * nb * window * 4,
            "frames_pushed": int(n_blocks * nb), "g2_finite": ok}


def serving_run(api, torch, dev, n_streams, life_lo, life_hi, lanes, budget_bytes=0, seed=4000):
    """Many online streams served at once (the serving workload): detectors drawn
    from {256x256, 512x512, 1024x512} px, 8..36 annular ROIs, uint8 counts
    (mean 0.05, beta 0.2, tau_c 50), k = 64 with each stream's basis compressed
    from its first 4 blocks, a 4096-lag window, 256-frame blocks arriving every
    256 / 52,000 s per stream with a random phase, stream starts as Poisson
    arrivals, lifetimes of life_lo..life_hi blocks.  One run pushes the blocks back
    to back (the rate the server sustains); the next pushes every block at its
    arrival time (latency = push call to the end of the block's work, by device
    events, plus how late the host issued the push)."""
    import numpy as np
    import synth
    rng = np.random.default_rng(seed)
    shapes = [(256, 256), (512, 512), (1024, 512)]
    nb, window, k, period = 256, 4096, 64, 256 / 52000.0
    streams = []
    ctx = api.Context(0)
    for i in range(n_streams):
        H, Wd = shapes[rng.integers(len(shapes))]
        n_roi = int(rng.integers(8, 37))
        M = H * Wd
        labels = torch.from_numpy(synth.annular_labels(H, Wd, n_roi)).to(dev)
        pool = synth.speckle_frames_torch(M, 4 * nb, 0.05, 0.2, 50.0, "u8", seed=seed + 1 + i, device=dev)
        f = api.compress_frames(ctx, pool, labels, n_roi, k=k, seed=seed + 100 + i)
        basis = f.U.contiguous()
        band = torch.empty((n_roi, nb, window), dtype=torch.float32, device=dev)
        streams.append(dict(M=M, shape=(H, Wd), n_roi=n_roi, labels=labels, pool=pool, basis=basis, band=band,
                            life=int(rng.integers(life_lo, life_hi + 1))))
    ctx.sync()
    ctx.close()
    torch.cuda.synchronize()
    starts = np.cumsum(rng.exponential(2 * period, size=n_streams))
    events = []
    for i, st in enumerate(streams):
        phase = rng.uniform(0, period)
        for b in range(st["life"]):
            events.append((starts[i] + phase + b * period, i, b))
    events.sort()

    def run(paced, budget=0):
        """Push every block at its arrival time (paced) or back to back.  A stream
        closes once its last block is reported, which frees its memory for waiting
        requests; a request that does not fit the budget waits, and its blocks are
        pushed once it is admitted (their latency then includes the wait)."""
        from collections import deque
        srv = api.Server(0, hbm_budget_bytes=budget, lanes=lanes, max_streams=n_streams)
        ids, lat, lag, opens, arrival_to_done = {}, [], {}, [], []
        seen = {i: 0 for i in range(n_streams)}
        held = {i: deque() for i in range(n_streams)}       # blocks of a waiting stream
        admitted, closing, closed = set(), set(), set()
        max_admitted, queued_opens, admit_wait = 0, 0, []
        t_open = {}
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def push(i, ta, b):
            st = streams[i]
            lag[(i, b)] = max(0.0, (now() - ta) * 1e3) if paced else 0.0
            srv.push(ids[i], st["pool"][(b % 4) * nb:(b % 4 + 1) * nb], band=st["band"])
            if b == st["life"] - 1:
                closing.add(i)

        def collect(i):
            for ms, _ in srv.poll(ids[i]):
                lat.append(ms)
                arrival_to_done.append(lag[(i, seen[i])] + ms)
                seen[i] += 1

        def service():
            nonlocal max_admitted
            for j in list(admitted):
                collect(j)
            for j in list(closing):
                if seen[j] == streams[j]["life"]:
                    srv.close(ids[j])
                    closing.discard(j)
                    admitted.discard(j)
                    closed.add(j)
            for j in list(ids):
                if j not in admitted and j not in closed and srv.state(ids[j]) == 2:
                    admitted.add(j)
                    admit_wait.append((now() - t_open[j]) * 1e3)
                    while held[j]:
                        push(j, *held[j].popleft())
            max_admitted = max(max_admitted, len(admitted))

        for (ta, i, b) in events:
            if paced:
                while now() < ta:
                    pass
            if b == 0:
                to = time.perf_counter()
                ids[i], state = srv.open(streams[i]["labels"], streams[i]["n_roi"], streams[i]["basis"], window, nb)
                opens.append((time.perf_counter() - to) * 1e3)
                t_open[i] = now()
                if state == 2:
                    admitted.add(i)
                    admit_wait.append(0.0)
                else:
                    queued_opens += 1
            if i in admitted:
                push(i, ta, b)
            else:
                held[i].append((ta, b))
            service()
        while len(closed) < n_streams:
            before = (len(closed), len(admitted))
            srv.wait()
            service()
            if (len(closed), len(admitted)) == before and not admitted:
                raise RuntimeError("a serving request can never be admitted under the budget")
        wall = now()
        srv.destroy()
        return dict(lat=lat, a2d=arrival_to_done, opens=opens, wall=wall, max_admitted=max_admitted,
                    queued=queued_opens, admit_wait=admit_wait)

    run(False)                                   # loads every kernel; not timed
    sat = run(False)
    pac = run(True)
    total_frames = sum(st["life"] for st in streams) * nb
    out = {"workload": f"serve_{n_streams}streams_u8_k64_w4096_b256",
           "streams": [{"px": f"{st['shape'][0]}x{st['shape'][1]}", "n_roi": st["n_roi"], "blocks": st["life"]}
                       for st in streams],
           "lanes": lanes, "blocks": len(events), "frames": total_frames,
           "block_latency_p50_ms": percentile(pac["lat"], 50), "block_latency_p99_ms": percentile(pac["lat"], 99),
           "arrival_to_done_p50_ms": percentile(pac["a2d"], 50), "arrival_to_done_p99_ms": percentile(pac["a2d"], 99),
           "open_ms_p50": percentile(pac["opens"], 50), "open_ms_max": max(pac["opens"]),
           "paced_wall_s": pac["wall"], "arrival_frames_per_s": total_frames / (events[-1][0] + period),
           "saturated_frames_per_s": total_frames / sat["wall"], "saturated_wall_s": sat["wall"],
           "saturated_block_latency_p50_ms": percentile(sat["lat"], 50),
           "max_admitted_at_once": pac["max_admitted"]}
    if budget_bytes:
        b = run(True, budget_bytes)
        out["budget"] = {"hbm_budget_bytes": budget_bytes, "requests_that_waited": b["queued"],
                         "max_admitted_at_once": b["max_admitted"],
                         "admission_wait_ms_p50": percentile(b["admit_wait"], 50),
                         "admission_wait_ms_max": max(b["admit_wait"]),
                         "block_latency_p50_ms": percentile(b["lat"], 50),
                         "block_latency_p99_ms": percentile(b["lat"], 99),
                         "arrival_to_done_p99_ms": percentile(b["a2d"], 99), "wall_s": b["wall"],
                         "frames_per_s": total_frames / b["wall"]}
    return out


def precision_table(api, torch, dev, steps=3, raw_steps=5):
    """BF16 vs FP8 subspace passes on the precision workload: 1024 x 1024 px x
    20,000 frames, uint8 counts <= 127 (mean 0.02, beta 0.15, tau_c 50), 36 ROIs,
    k = 128 (q = 1).  Per precision: compress time, the basis' orthonormality and
    W = X^T U on 16 sampled frames against FP64 (the encoding pass is split-bf16 in
    both); between the two: singular values, the subspaces (cosine of the largest
    principal angle over the top 32 and over all k directions) and g2 (fused)."""
    import numpy as np
    import synth
    spec = synth.WORKLOADS["det1024_20k_precision"]
    M, N, n_roi, k = spec.n_pixels, spec.n_frames, spec.n_roi, spec.ranks[0]
    labels = synth.workload_labels(spec)
    frames = synth.speckle_frames_torch(M, N, spec.mu, spec.beta, synth.workload_tau(spec, labels), spec.dtype,
                                        seed=3000, device=dev, max_count=spec.max_count)
    labels_d = torch.from_numpy(labels).to(dev)
    ts = np.sort(np.random.default_rng(11).choice(N, size=16, replace=False))
    Fs = frames[torch.from_numpy(ts).to(dev)].cpu().numpy().astype(np.float64)
    ctx = api.Context(0)
    res, U, sig, g2 = {}, {}, {}, {}
    for prec in ("bf16", "fp8"):
        f = api.compress_frames(ctx, frames, labels_d, n_roi, k=k, seed=7, precision=prec)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f = api.compress_frames(ctx, frames, labels_d, n_roi, k=k, seed=7, precision=prec)
        ctx.sync()
        ms = (time.perf_counter() - t0) / steps * 1e3
        _, g, _ = api.correlate_two_time(ctx, f, want_c=False)
        ctx.sync()
        Uh = f.U.T.contiguous()
        U[prec], sig[prec], g2[prec] = Uh, f.sigma.cpu().numpy(), g.cpu().numpy()
        Un = Uh.double().cpu().numpy()
        Ws = Fs @ Un
        Wg = (f.V.T.double().cpu().numpy() * sig[prec])[ts]
        # compression's bound: four passes over the frames (the sketch, the power pass's two
        # products and the encoding pass) at peak HBM bandwidth
        x4 = 4 * M * N * frames.element_size()
        res[prec] = {"compress_ms": ms, "frames_per_s": N / (ms / 1e3),
                     "compress_algorithmic_bytes": x4,
                     "compress_hbm_frac": x4 / (PEAK_HBM_GBS * 1e9) * 1e3 / ms,
                     "u_orthonormality": float((Uh.double().T @ Uh.double() - torch.eye(k, device=dev,
                                                                                          dtype=torch.float64))
                                               .abs().max().item()),
                     "w_rel_err": float(np.linalg.norm(Wg - Ws) / np.linalg.norm(Ws)),
                     "sigma_first": float(sig[prec][0]), "sigma_last": float(sig[prec][-1])}
        del f
    # the raw path on the same frames: exact int8 Gram of every ROI, C in FP32 (57.6 GB) + fused g2
    C = api.empty_two_time(dev, n_roi, N)
    g2r = torch.empty((n_roi, N), dtype=torch.float64, device=dev)
    npr = torch.empty((n_roi, N), dtype=torch.int64, device=dev)
    raw_step = lambda: api.correlate_two_time_raw(ctx, frames, labels_d, n_roi, C=C, g2=g2r, npairs=npr)
    ctx.phase_filter(["raw_gram_tiles"])              # events around the Gram only in the timed steps
    ctx.enable_phase_timing(True)
    per, wall = timed_steps(torch, ctx, raw_step, raw_steps, 1)
    ph = ctx.phase_times()
    ctx.enable_phase_timing(False)
    ctx.phase_filter(None)
    ctx.enable_phase_timing(True)                     # the breakdown from one more step, untimed
    raw_step()
    ctx.sync()
    ph_all = ctx.phase_times()
    ctx.enable_phase_timing(False)
    tot_ms, cnt = ph.get("raw_gram_tiles", (float("nan"), 1))
    ops = 2.0 * N * N * float(roi_counts_and_sums(labels, n_roi)[0].sum())
    raw = {"ms_per_step": 1e3 * wall / raw_steps, "frames_per_s": N / (wall / raw_steps),
           "p50_ms": percentile(per, 50), "p99_ms": percentile(per, 99), "steps": raw_steps, "warmup": 1,
           "gram_ms": tot_ms / cnt, "gram_int8_TOPs": ops / (tot_ms / cnt / 1e3) / 1e12,
           "gram_frac_of_int8_peak": ops / (tot_ms / cnt / 1e3) / 1e12 / PEAK_I8_TOPS,
           # the Gram is symmetric and the kernel forms one triangle: on the symmetric
           # product's count N (N + 1) sum|R| the same time is this fraction of peak
           "gram_symmetric_frac_of_int8_peak": ops * (N + 1) / (2.0 * N) / (tot_ms / cnt / 1e3) / 1e12 / PEAK_I8_TOPS,
           "phases_ms": {kk: round(v[0] / v[1], 4) for kk, v in ph_all.items()}}
    del C, g2r, npr
    cross = (U["bf16"].double().T @ U["fp8"].double())
    cos_all = float(torch.linalg.svdvals(cross).min().item())
    cos_top = float(torch.linalg.svdvals(cross[:32, :32]).min().item())
    ok = np.isfinite(g2["bf16"]) & np.isfinite(g2["fp8"])
    ctx.close()
    del frames
    torch.cuda.empty_cache()
    return {"workload": "det1024_20k_precision (1024x1024 px x 20000 frames, u8 <= 127, 36 ROIs, k=128)",
            "bf16": res["bf16"], "fp8": res["fp8"],
            "sigma_max_rel_diff": float(np.max(np.abs(sig["fp8"] - sig["bf16"]) / sig["bf16"])),
            "subspace_cos_min_top32": cos_top, "subspace_cos_min_all": cos_all,
            "g2_max_rel_diff": float(np.max(np.abs(g2["fp8"][ok] - g2["bf16"][ok]) / np.abs(g2["bf16"][ok]))),
            "raw": raw, "speedup_bf16_vs_raw": raw["ms_per_step"] / res["bf16"]["compress_ms"]}


def timed_steps(torch, ctx, fn, steps, warmup):
    """Device time of each of `steps` calls of fn after `warmup` untimed ones (events
    on the current stream), and the host wall time of the timed ones."""
    for _ in range(warmup):
        fn()
    ctx.sync()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    w0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.sync()
    return [a.elapsed_time(b) for a, b in evs], wall


def tiny_line(api, torch, dev, steps, warmup):
    """The tiny workload (64 x 64 px x 1,000 frames, uint8, one ROI, k = 32): the
    compressed step (basis + C in FP32 + fused g2) and the raw step (exact Gram, C in
    FP64 + fused g2) in absolute microseconds (launch- and latency-bound sizes)."""
    import synth
    spec = synth.WORKLOADS["tiny_64x64x1000"]
    M, N, k = spec.n_pixels, spec.n_frames, spec.ranks[0]
    labels = torch.from_numpy(synth.workload_labels(spec)).to(dev)
    frames = synth.speckle_frames_torch(M, N, spec.mu, spec.beta, spec.tau_c, spec.dtype, seed=1001, device=dev)
    ctx = api.Context(0)
    f = api.Factors.empty(M, N, k, 1, dev)
    C = api.empty_two_time(dev, 1, N)
    C64 = api.empty_two_time(dev, 1, N, torch.float64)
    g2 = torch.empty((1, N), dtype=torch.float64, device=dev)
    npairs = torch.empty((1, N), dtype=torch.int64, device=dev)

    def comp():
        api.compress_frames(ctx, frames, labels, 1, k=k, seed=7, out=f)
        api.correlate_two_time(ctx, f, C=C, g2=g2, npairs=npairs)

    def raw():
        api.correlate_two_time_raw(ctx, frames, labels, 1, C=C64, g2=g2, npairs=npairs)

    pc, wc = timed_steps(torch, ctx, comp, steps, warmup)
    pr, wr = timed_steps(torch, ctx, raw, steps, warmup)
    ctx.close()
    return {"workload": "tiny_64x64x1000 (4096 px x 1000 frames, u8, 1 ROI, k=32)",
            "compressed_us_p50": 1e3 * percentile(pc, 50), "compressed_us_p99": 1e3 * percentile(pc, 99),
            "compressed_frames_per_s": N / (wc / steps),
            "raw_us_p50": 1e3 * percentile(pr, 50), "raw_us_p99": 1e3 * percentile(pr, 99),
            "raw_frames_per_s": N / (wr / steps), "steps": steps, "warmup": warmup}


def k128_line(api, torch, ctx, frames, labels_d, n_roi, steps, warmup):
    """The benchmark workload's compressed step at k = 128 (same frames, C and g2)."""
    N, M = frames.shape
    k = 128
    f = api.Factors.empty(M, N, k, n_roi, frames.device)
    C = api.empty_two_time(frames.device, n_roi, N)
    g2 = torch.empty((n_roi, N), dtype=torch.float64, device=frames.device)
    npairs = torch.empty((n_roi, N), dtype=torch.int64, device=frames.device)

    def comp():
        api.compress_frames(ctx, frames, labels_d, n_roi, k=k, seed=7, out=f)
        api.correlate_two_time(ctx, f, C=C, g2=g2, npairs=npairs)

    per, wall = timed_steps(torch, ctx, comp, steps, warmup)
    del C
    torch.cuda.empty_cache()
    ms = 1e3 * wall / steps
    # the step's bound as for the benchmark step: four passes over the frames and C once
    step_bytes = 4 * M * N * frames.element_size() + n_roi * N * N * 4
    return {"workload": "det512_10k_36roi at k=128", "ms_per_step": ms,
            "frames_per_s": N / (wall / steps), "p50_ms": percentile(per, 50), "p99_ms": percentile(per, 99),
            "steps": steps, "warmup": warmup, "step_algorithmic_bytes": step_bytes,
            "step_hbm_frac": step_bytes / (PEAK_HBM_GBS * 1e9) * 1e3 / ms}


def g2_only(api, torch, ctx, f, reps=5):
    """g2 of every ROI without C: the tile pass with C = NULL against the FFT form,
    on the factors of the benchmark step (times from events on the context's stream)."""
    import numpy as np
    stream = torch.cuda.current_stream()

    def run(fn):
        fn()
        ctx.sync()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            out = fn()
            b.record(stream)
        torch.cuda.synchronize()
        ctx.sync()
        return sorted(a.elapsed_time(b) for a, b in evs)[reps // 2], out

    t_tile, (_, g_tile, n_tile) = run(lambda: api.correlate_two_time(ctx, f, want_c=False))
    t_fft, (g_fft, n_fft) = run(lambda: api.g2_from_factors(ctx, f))
    t_stats, (m_s, s_s, _) = run(lambda: api.two_time_stats(ctx, f))
    gt, gf = g_tile.cpu().numpy(), g_fft.cpu().numpy()
    ok = n_tile.cpu().numpy() > 0
    return {"tile_ms": t_tile, "fft_ms": t_fft, "ttc_stats_ms": t_stats,
            "ttc_mean_roi0": float(m_s[0]), "ttc_std_roi0": float(s_s[0]),
            "npairs_equal": bool(torch.equal(n_tile, n_fft)),
            "g2_max_rel_diff": float(np.max(np.abs(gf[ok] - gt[ok]) / np.abs(gt[ok])))}


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summaries.

    A summary carries a line <!-- traffic: kernel=K fetch_bytes=F write_bytes=W
    sources=a,b sha256=H --> written from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE, already scaled by the copy-kernel factor).  The figure is used
    only while the kernel's sources still hash to H; otherwise it is stale and
    None is returned.
    """
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for m in re.finditer(r"<!-- traffic: (.*?) -->", open(path).read()):
            kv = dict(item.split("=", 1) for item in m.group(1).split())
            if kv.get("kernel") != kernel:
                continue
            h = hashlib.sha256()
            try:
                for src in kv["sources"].split(","):
                    h.update(open(os.path.join(ROOT, src), "rb").read())
            except OSError:
                continue
            if h.hexdigest() != kv.get("sha256"):
                continue
            return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="det512_10k_36roi")
    ap.add_argument("--k", type=int, default=64)
    ap.add_argument("--raw-steps", type=int, default=20)
    ap.add_argument("--no-raw", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-frames", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--no-stream", action="store_true", help="skip the online-stream latency measurement")
    ap.add_argument("--stream-blocks", type=int, default=40)
    ap.add_argument("--no-serve", action="store_true", help="skip the many-stream serving measurement")
    ap.add_argument("--serve-streams", type=int, default=16)
    ap.add_argument("--serve-life", type=int, nargs=2, default=[64, 512], metavar=("LO", "HI"),
                    help="stream lifetimes in blocks")
    ap.add_argument("--serve-budget-mib", type=int, default=1024,
                    help="HBM budget of the extra serving run that exercises admission (0: skip it)")
    ap.add_argument("--serve-lanes", type=int, default=4)
    ap.add_argument("--no-g2only", action="store_true", help="skip the g2-without-C comparison")
    ap.add_argument("--no-k128", action="store_true", help="skip the k = 128 line of the benchmark workload")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny workload's microsecond line")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16 vs FP8 table on the 1024 x 1024 x 20,000 uint8 workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (the reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is "
              "a design only and not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2407_20356_amd import api

    spec = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1, out=dst)     # an elementwise kernel: reads and writes nbytes each
        torch.cuda.synchronize()
        log(f"copy calibration: 3 elementwise copies of {nbytes} bytes")
        del src, dst
    M, N, n_roi, k = spec.n_pixels, spec.n_frames, spec.n_roi, args.k
    labels = synth.workload_labels(spec)
    tau = synth.workload_tau(spec, labels)
    log(f"generating {args.workload}: {N} frames x {M} px ({spec.dtype}) on {dev}")
    t = time.perf_counter()
    frames = synth.speckle_frames_torch(M, N, spec.mu, spec.beta, tau, spec.dtype, seed=args.seed,
                                        device=dev, max_count=spec.max_count)
    labels_d = torch.from_numpy(labels).to(dev)
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t:.1f} s")

    ctx = api.Context(0)
    f = api.Factors.empty(M, N, k, n_roi, dev)
    C = api.empty_two_time(dev, n_roi, N)          # rows padded to whole 128-byte lines (ldc = 10016)
    g2 = torch.empty((n_roi, N), dtype=torch.float64, device=dev)
    npairs = torch.empty((n_roi, N), dtype=torch.int64, device=dev)

    def step_compressed():
        api.compress_frames(ctx, frames, labels_d, n_roi, k=k, seed=7, out=f)
        api.correlate_two_time(ctx, f, C=C, g2=g2, npairs=npairs)

    def step_raw():
        api.correlate_two_time_raw(ctx, frames, labels_d, n_roi, C=C, g2=g2, npairs=npairs)

    def timed(fn, steps, warmup, name, key_phase):
        """The timed steps record HIP events around the dominant kernel only (its
        launch times feed the roofline); the per-phase breakdown comes from as many
        further steps with every phase recorded, outside the timed region."""
        for i in range(warmup):
            fn()
        ctx.sync()
        torch.cuda.synchronize()
        ctx.phase_filter([key_phase])
        ctx.enable_phase_timing(True)
        stream = torch.cuda.current_stream(dev)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ctx.sync()
        per = [a.elapsed_time(b) for a, b in evs]
        key = ctx.phase_times()
        ctx.enable_phase_timing(False)
        ctx.phase_filter(None)
        ctx.enable_phase_timing(True)
        for _ in range(steps):
            fn()
        ctx.sync()
        phases = ctx.phase_times()
        ctx.enable_phase_timing(False)
        phases.update(key)
        log(f"{name}: {steps} steps, mean {sum(per) / len(per):.3f} ms, wall {1e3 * wall / steps:.3f} ms/step")
        return per, wall, phases

    log("compressed path: warmup + timed steps")
    per_c, wall_c, ph_c = timed(step_compressed, args.steps, args.warmup, "compressed", "lowrank_tiles")
    ms_c = 1e3 * wall_c / args.steps
    log("compressed phases (ms per launch x launches per step): " + ", ".join(
        f"{kk} {v[0] / v[1]:.3f}x{v[1] // args.steps}" for kk, v in sorted(ph_c.items(), key=lambda kv: -kv[1][0])))

    # light parity spot checks on this run (sampled frames; the full checks are in tests/)
    rng = np.random.default_rng(0)
    ts = np.sort(rng.choice(N, size=16, replace=False))
    idx = torch.from_numpy(ts).to(dev)
    if spec.dtype == "u16":      # torch has no uint16 gather on the device: gather the int16 view
        Fs = frames.view(torch.int16)[idx].cpu().numpy().view(np.uint16)
    else:
        Fs = frames[idx].cpu().numpy()
    U = f.U.cpu().numpy().T.astype(np.float64)
    Ws = Fs.astype(np.float64) @ U
    Wg = (f.V.cpu().numpy().T.astype(np.float64) * f.sigma.cpu().numpy())[ts]
    npix, S_host = roi_counts_and_sums(labels, n_roi, Fs)
    S_ok = bool(np.array_equal(f.roi_sum.cpu().numpy()[:, ts], S_host))
    w_err = float(np.linalg.norm(Wg - Ws) / np.linalg.norm(Ws))
    orth = float(np.abs(U.T @ U - np.eye(k)).max())
    Cs = C[:, torch.from_numpy(ts).to(dev)][:, :, torch.from_numpy(ts).to(dev)].cpu().numpy()
    Sg = S_host.astype(np.float64)
    c_err = 0.0
    for r in range(n_roi):
        Ur = U[labels == r]
        Cr = npix[r] * (Ws @ (Ur.T @ Ur) @ Ws.T) / np.outer(Sg[r], Sg[r])
        ok = np.isfinite(Cr)
        c_err = max(c_err, float(np.max(np.abs(Cs[r][ok] - Cr[ok]) / np.maximum(np.abs(Cr[ok]), 0.1))))
    parity = {"roi_sum_exact": S_ok, "w_rel_err": w_err, "u_orthonormality": orth,
              "c_identity_max_rel_err": c_err, "sampled_frames": int(len(ts))}
    log(f"parity spot checks: {parity}")

    raw = None
    if not args.no_raw:
        log("raw path: warmup + timed steps")
        per_r, wall_r, ph_r = timed(step_raw, args.raw_steps, args.warmup, "raw", "raw_gram_tiles")
        ms_r = 1e3 * wall_r / args.raw_steps
        log("raw phases (ms per launch x launches per step): " + ", ".join(
            f"{kk} {v[0] / v[1]:.3f}x{v[1] // args.raw_steps}" for kk, v in sorted(ph_r.items(), key=lambda kv: -kv[1][0])))
        raw = {"frames_per_s": N / (ms_r / 1e3), "ms_per_step": ms_r, "p50_ms": percentile(per_r, 50),
               "p99_ms": percentile(per_r, 99), "steps": args.raw_steps,
               "phases_ms": {kk: round(v[0] / v[1], 4) for kk, v in ph_r.items()}}

    # per-kernel achieved rates from the HIP events recorded around each phase
    esz = 1 if spec.dtype == "u8" else 2
    x_bytes = N * M * esz
    kp = (k + 31) // 32 * 32
    nb = (N + 127) // 128
    algo = {
        # bytes each launch must move: the frames it reads / the matrix it writes
        "sketch": (x_bytes, "hbm"),
        "proj_frames": (x_bytes, "hbm"),
        "proj_pixels": (x_bytes, "hbm"),
        "lowrank_tiles": (n_roi * N * N * 4 + 2 * n_roi * N * kp * 2, "hbm"),
    }
    kernels = {}
    for name, (bytes_per_launch, bound) in algo.items():
        if name in ph_c:
            tot_ms, cnt = ph_c[name]
            avg_ms = tot_ms / cnt
            kernels[name] = {"avg_ms": avg_ms, "launches_per_step": cnt / args.steps,
                             "achieved_GBs": bytes_per_launch / (avg_ms / 1e3) / 1e9,
                             "bytes_per_launch": bytes_per_launch}
    dom = max(kernels, key=lambda kk: kernels[kk]["avg_ms"] * kernels[kk]["launches_per_step"])
    dk = kernels[dom]
    traffic = pmc_traffic(dom) if args.workload == "det512_10k_36roi" and k == 64 else None
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(dk["achieved_GBs"], 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(dk["achieved_GBs"] / PEAK_HBM_GBS, 4),
                "traffic": traffic, "algorithmic_bytes": dk["bytes_per_launch"]}
    # the whole step against its bound: four passes over the frames (the sketch, the power
    # pass's two products and the encoding pass) plus writing C once, at peak HBM bandwidth
    step_bytes = 4 * x_bytes + n_roi * N * N * 4
    ideal_ms = step_bytes / (PEAK_HBM_GBS * 1e9) * 1e3
    step_roofline = {"bound": "hbm", "algorithmic_bytes": step_bytes, "ideal_ms": ideal_ms, "ms_per_step": ms_c,
                     "frac": ideal_ms / ms_c}
    if raw is not None and "raw_gram_tiles" in ph_r:
        tot_ms, cnt = ph_r["raw_gram_tiles"]
        ops = 2.0 * N * N * float(npix.sum())
        raw["gram_int8_TOPs"] = ops / (tot_ms / cnt / 1e3) / 1e12
        raw["gram_frac_of_int8_peak"] = raw["gram_int8_TOPs"] / PEAK_I8_TOPS
        # on the symmetric product's op count N (N + 1) sum|R| (the kernel forms one triangle)
        raw["gram_symmetric_frac_of_int8_peak"] = raw["gram_frac_of_int8_peak"] * (N + 1) / (2.0 * N)

    k128 = None
    if not args.no_k128 and args.workload == "det512_10k_36roi" and k != 128:
        log("compressed step at k = 128 on the same frames")
        k128 = k128_line(api, torch, ctx, frames, labels_d, n_roi, args.steps, args.warmup)
        log(f"k = 128: {k128['ms_per_step']:.3f} ms per step, {k128['frames_per_s']:.0f} frames/s")

    g2o = None
    if not args.no_g2only:
        log("g2 without C, every ROI: tile pass (C = NULL) vs FFT form")
        g2o = g2_only(api, torch, ctx, f)
        log(f"g2 without C: tile {g2o['tile_ms']:.3f} ms, FFT {g2o['fft_ms']:.3f} ms, "
            f"max rel diff {g2o['g2_max_rel_diff']:.2e}, npairs equal {g2o['npairs_equal']}")

    serving = None
    if not args.no_stream:
        log("online stream: per-push latency at 1024 x 512 px, 36 ROIs, k = 64, window 4096")
        serving = stream_latency(api, torch, dev, args.stream_blocks)
        log(f"online stream: push p50 {serving['push_p50_ms']:.3f} ms, p99 {serving['push_p99_ms']:.3f} ms")
    served = None
    if not args.no_serve:
        log(f"serving: {args.serve_streams} streams, lifetimes {args.serve_life} blocks, {args.serve_lanes} lanes")
        served = serving_run(api, torch, dev, args.serve_streams, args.serve_life[0], args.serve_life[1],
                             args.serve_lanes, budget_bytes=args.serve_budget_mib << 20)
        log(f"serving: block latency p50 {served['block_latency_p50_ms']:.3f} ms, "
            f"p99 {served['block_latency_p99_ms']:.3f} ms; arrival to done p99 "
            f"{served['arrival_to_done_p99_ms']:.3f} ms; open max {served['open_ms_max']:.1f} ms; "
            f"saturated {served['saturated_frames_per_s']:.0f} frames/s")

    prec_table = None
    if not args.no_precision:
        log("precision table: BF16 vs FP8 subspace passes, 1024 x 1024 px x 20,000 uint8 frames, k = 128")
        prec_table = precision_table(api, torch, dev)
        log(f"precision table: compress bf16 {prec_table['bf16']['compress_ms']:.2f} ms, "
            f"fp8 {prec_table['fp8']['compress_ms']:.2f} ms; sigma diff {prec_table['sigma_max_rel_diff']:.2e}; "
            f"g2 diff {prec_table['g2_max_rel_diff']:.2e}")

    tiny = None
    if not args.no_tiny:
        log("tiny workload: compressed and raw steps in microseconds")
        tiny = tiny_line(api, torch, dev, args.steps, args.warmup)
        log(f"tiny: compressed {tiny['compressed_us_p50']:.1f} us, raw {tiny['raw_us_p50']:.1f} us (p50)")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on the first {args.cpu_sample_frames} frames")
        host = frames[:args.cpu_sample_frames].cpu().numpy()
        cpu = cpu_baseline(host, labels, n_roi, k, 7, args.cpu_sample_frames)
        log(f"cpu baseline: {cpu['value']:.1f} frames/s in {cpu['seconds']:.1f} s on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": N / (ms_c / 1e3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_c,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": args.workload, "pixels": M, "frames": N, "count_dtype": spec.dtype,
                   "n_roi": n_roi, "k": k, "oversample": 16, "power_iters": 1, "c_dtype": "f32",
                   "g2": "fused"},
        "p50_ms": percentile(per_c, 50),
        "p99_ms": percentile(per_c, 99),
        "raw": raw,
        "speedup_vs_raw": (raw["ms_per_step"] / ms_c) if raw else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stream": serving,
        "serving": served,
        "precision": prec_table,
        "k128": k128,
        "tiny": tiny,
        "step_roofline": step_roofline,
        "g2_without_c": g2o,
        "kernels": kernels,
        "phases_ms": {kk: round(v[0] / v[1], 4) for kk, v in ph_c.items()},
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
