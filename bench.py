#!/usr/bin/env python3
"""Benchmark of the X-engine correlation hot path on one MI355X.

A step is one integration period of one CHIME-shaped channel: correlate
N=2048 inputs x T=32768 samples of 4+4-bit data into the device-resident
int32 accumulators, then dump the N(N+1)/2 visibilities with reset.  The
metric is the paper's cost unit, complex multiply-accumulates per second
(Sec. 2.2, eta counts N(N+1)/2 products per sample), on one GPU.

Prints one JSON line.  Inputs are synthetic (seeded) and resident in HBM
before the timed region starts.  Before the W warm-up steps, untimed steps
run for --settle-ms of wall time: the GPU's clock takes tens of
milliseconds of sustained load to ramp up, longer than a few steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0          # MI355X dense int8, TOP/s (5.0 POP/s)
HBM_PEAK_GBS = 8000.0


def measured_traffic():
    """HBM bytes per correlation launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if the kernel source
    has changed since those counters were taken."""
    import hashlib
    rec = os.path.join(ROOT, "profiles", "xcorr_dma_n2048_t32768_traffic.txt")
    src = os.path.join(ROOT, "paper_2005_09481_amd", "csrc", "xeng_kernel_dma.hip")
    try:
        fields = {}
        for line in open(rec):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields["kernel_source_sha256"]:
            return None
        return int(fields["fetch_bytes_per_launch"]) + int(fields["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(x, n, target_s=12.0):
    """The oracle, as it stands, timed on this host: compiled here with -O3
    -march=native, every host thread, on a bounded time sample of the same
    input; plus one thread on the small N=64, T=4096 channel."""
    import tempfile

    import numpy as np

    import oracle
    import synth
    tmp = tempfile.mkdtemp(prefix="xeng_oracle_")
    lib = oracle.load_library(oracle.build_native(tmp))
    tri = n * (n + 1) // 2
    t_probe = 64
    t0 = time.perf_counter()
    oracle.correlate(np.ascontiguousarray(x[:t_probe]), _lib_override=lib)
    dt = time.perf_counter() - t0
    rate = t_probe * tri / max(dt, 1e-6)
    t_s = int(min(x.shape[0], max(t_probe, target_s * rate / tri)))
    t_s = max(32, (t_s // 32) * 32)
    t0 = time.perf_counter()
    oracle.correlate(np.ascontiguousarray(x[:t_s]), _lib_override=lib)
    dt = time.perf_counter() - t0
    threads = int(lib.xo_num_threads())
    # one thread, small channel
    small = synth.uniform_bytes(64, 4096, seed=1)
    lib.xo_set_threads(1)
    t1 = time.perf_counter()
    oracle.correlate(small, _lib_override=lib)
    dt1 = time.perf_counter() - t1
    lib.xo_set_threads(threads)
    return {"value": t_s * tri / dt / 1e12, "unit": "TCMAC/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {t_s} of {x.shape[0]} samples of the N={n} channel "
                      f"({t_s * tri:.3e} CMAC in {dt:.1f} s), gcc -O3 -march=native, OpenMP",
            "one_thread_n64_t4096_tcmacs": round(4096 * 2080 / dt1 / 1e12, 6)}


def bench_many_channels(args, xeng, synth, torch, np, n, t):
    """An HBM-bound channel size run the way a deployment runs it: many
    frequency channels (one slot each) correlated by one persistent launch
    of a prepared batch (so that no per-job host work sits in the timed
    region).  Returns the launch time and its rate against HBM peak."""
    dev = torch.device("cuda:0")
    c = args.many_channels
    x = torch.from_numpy(synth.uniform_bytes(n, t * c, seed=5)).to(dev).view(c, t, n)
    corr = xeng.Correlator(n, c, device=0)
    jobs = [(corr, k, x[k]) for k in range(c)]
    stream = torch.cuda.current_stream(dev)
    batch = xeng.Batch(jobs)
    reps = max(5, args.steps)
    for _ in range(3):
        batch.launch(stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        batch.launch(stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    t_launch = float(np.median([a.elapsed_time(b) for a, b in ev])) / 1e3
    batch.close()
    tri = n * (n + 1) // 2
    gbs = c * (n * t + 8 * tri) / t_launch / 1e9
    return {"channels": c, "launch_us": round(t_launch * 1e6, 2),
            "tcmacs": round(c * t * tri / t_launch / 1e12, 3),
            "achieved_gbs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def bench_serve(args, xeng, synth, torch, np):
    """Streaming: K channels of N=2048 each release a 256-sample frame every
    655.36 us (390625 samples/s); exports every 128 frames (83.886 ms).  K is
    real-time when every released frame is integrated (no drops, no growing
    backlog) and the p99 frame latency stays below the export period."""
    n, frame_len, dump = 2048, 256, 128
    period_ms = dump * frame_len / 390625 * 1e3
    # distinct frames per source, cycled: a device source holds 64 frames
    # (32 MiB: a server running behind may take up to that many frames of a
    # channel in one launch), a pinned host source 16
    n_src_dev, n_src_host = 64, 16
    base = synth.stream_frames(n, n_src_dev, seed=5)
    base_dev = torch.from_numpy(base).cuda()
    results = []
    # shader clock stamped by workgroup 0 of the last correlation launch of a trial
    clock_buf = None if args.no_clock_probe else torch.zeros(4, dtype=torch.int64, device="cuda")

    def trial(k, host):
        srv = xeng.Server(n, max_channels=k, dump_frames=dump, launch_period_us=args.serve_launch_us,
                          ring_frames=64, max_inflight=2, stagger_exports=bool(args.serve_stagger))
        srcs = []
        for c in range(k):
            if host:                                 # distinct bytes per channel
                f = torch.from_numpy(np.roll(base[:n_src_host], c, axis=2).copy()).pin_memory()
            else:
                f = torch.roll(base_dev, c, dims=2)
            srcs.append(f)
            srv.admit(f, start_s=0.05 + 655.36e-6 * c / k)
        if host:
            # a long-lived ingest buffer has been read by the copy engines
            # before: one untimed copy of each source maps its pinned pages
            # for the device, outside the run
            scratch = torch.empty(srcs[0].shape, dtype=torch.uint8, device="cuda")
            for f in srcs:
                scratch.copy_(f, non_blocking=True)
            torch.cuda.synchronize()
            del scratch
        if clock_buf is not None:
            xeng.clock_probe(clock_buf)
        st = srv.run(args.serve_seconds)
        sclk = None
        if clock_buf is not None:
            torch.cuda.synchronize()
            sclk = round(xeng.sclk_ghz(clock_buf), 3)
            xeng.clock_probe(None)
        srv.close()
        # real time: nothing dropped, p99 below the export period, and the
        # frames still queued at the end no more than arrive within the p99
        # latency plus two launch periods (a server that falls behind sees
        # its latency grow past the export period within the run)
        frame_ms = 655.36e-3
        launch_ms = args.serve_launch_us / 1e3
        ok = (st["frames_dropped"] == 0 and st["p99_ms"] < period_ms and
              st["backlog_frames"] <= k * (st["p99_ms"] + 2 * launch_ms) / frame_ms)
        r = {"k": k, "source": "host" if host else "device", "real_time": bool(ok),
             "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
             "max_pass_ms": round(st["max_pass_ms"], 3), "max_launch_call_ms": round(st["max_launch_call_ms"], 3),
             "max_copy_call_ms": round(st["max_copy_call_ms"], 3), "frames_gathered": st["frames_gathered"],
             "max_ms": round(st["max_ms"], 3), "tcmacs": round(st["tcmacs"], 2),
             "frames_done": st["frames_done"], "dropped": st["frames_dropped"],
             "backlog": st["backlog_frames"], "launches": st["launches"], "dumps": st["dumps"],
             "sclk_ghz": sclk}
        print(json.dumps(r), flush=True)
        return r

    for host, ks in ((False, args.serve_k), (True, args.serve_host_k)):
        for k in [int(v) for v in ks.split(",") if int(v) > 0]:
            r = trial(k, host)
            results.append(r)
            if not r["real_time"]:
                break
    best = {src: max([r["k"] for r in results if r["source"] == src and r["real_time"]], default=0)
            for src in ("device", "host")}
    rt = [r for r in results if r["real_time"] and r["source"] == "device"]
    res = {"metric": "real-time channels/GPU, p99 latency", "value": best["device"],
           "unit": "channels (N=2048, 390625 samples/s)", "n_gpus": 1, "higher_is_better": True,
           "dtype": "int8", "data": "synthetic",
           "config": {"workload": "streaming serve, N=2048, 256-sample frames, export every 128 frames",
                      "seconds_per_trial": args.serve_seconds,
                      "launch_period_us": args.serve_launch_us,
                      "staggered_exports": bool(args.serve_stagger)},
           "max_k_host_frames": best["host"],
           "p99_ms_at_max_k": rt[-1]["p99_ms"] if rt else None,
           "export_period_ms": round(period_ms, 3)}
    print(json.dumps(res), flush=True)


def bench_batch(args, xeng, synth, torch, np):
    """Many jobs in one persistent launch (and as a prepared batch replayed
    from a hipGraph) against the same jobs launched one by one."""
    if args.workload == "channels16":
        xs = synth.batched_channels(n_channels=16, n_inputs=2048, seed=3)
        label = "16 channels x N=2048, T uniform in [2048,16384], 5% of inputs flagged"
    else:
        xs = synth.subarray_batch(n_instances=64, seed=4)
        label = "64 sub-arrays, N in {256,512,1024,2048}, T in {4096,8192,16384}"
    dev = torch.device("cuda:0")
    bufs = [torch.from_numpy(x).to(dev) for x in xs]
    cs = [xeng.Correlator(x.shape[1], 1, device=0) for x in xs]
    jobs = [(c, 0, b) for c, b in zip(cs, bufs)]
    cmac = sum(x.shape[0] * x.shape[1] * (x.shape[1] + 1) // 2 for x in xs)
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        for c in cs:
            c.reset(0)
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            for c in cs:
                c.reset(0)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) / 1e3)
        return float(np.median(times))

    def plain():
        for c, b in zip(cs, bufs):
            c.correlate(0, b, stream=stream)

    def batched():
        xeng.correlate_batch(jobs, stream=stream)

    t_settle = time.perf_counter() + args.settle_ms / 1e3
    while time.perf_counter() < t_settle:
        batched()
        torch.cuda.synchronize()
        for c in cs:
            c.reset(0)
    t_plain = timed(plain, args.steps)
    t_batch = timed(batched, args.steps)
    prepared = xeng.Batch(jobs)
    t_prep = timed(lambda: prepared.launch(stream=stream), args.steps)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        prepared.launch(stream=side)
    t_graph = timed(g.replay, args.steps)
    res = {
        "metric": "Tera-CMAC/s, batched persistent launch vs per-job launches",
        "value": round(cmac / t_batch / 1e12, 3), "unit": "TCMAC/s", "n_gpus": 1,
        "steps": args.steps, "higher_is_better": True, "dtype": "int8", "data": "synthetic",
        "config": {"workload": label, "jobs": len(xs), "cmac": cmac},
        "batched_ms": round(t_batch * 1e3, 4), "plain_ms": round(t_plain * 1e3, 4),
        "prepared_ms": round(t_prep * 1e3, 4), "graph_replay_ms": round(t_graph * 1e3, 4),
        "plain_tcmacs": round(cmac / t_plain / 1e12, 3),
        "graph_tcmacs": round(cmac / t_graph / 1e12, 3),
        "speedup_vs_plain": round(t_plain / t_batch, 3),
    }
    print(json.dumps(res), flush=True)


def bench_flagged(args, xeng, synth, torch, np):
    """RFI excision + flag-aware correlation of one CHIME-shaped channel with
    injected interference: per step, spectral-kurtosis flags over blocks of
    256 samples, the flag-aware correlation (masked copy, wide kernel,
    per-pair counts), then the count and visibility exports.  Each part is
    timed with HIP events on the stream it runs on."""
    n, t, bl = args.n, args.t, 256
    tri = n * (n + 1) // 2
    x = torch.from_numpy(synth.rfi_channel(n, t, seed=6, block_len=bl)).cuda()
    corr = xeng.Correlator(n, 1, device=0, counts=True)
    out = torch.empty((tri, 2), dtype=torch.int32, device="cuda")
    cnt = torch.empty(tri, dtype=torch.int32, device="cuda")
    fl = torch.empty(((t + bl - 1) // bl, n), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        xeng.rfi_flags(x, block_len=bl, out=fl, stream=stream)
        if ev:
            ev[1].record(stream)
        corr.correlate_flagged(0, x, fl, bl, stream=stream)
        if ev:
            ev[2].record(stream)
        corr.dump_counts(0, out=cnt, stream=stream)
        corr.dump(0, out=out, reset=True, stream=stream)

    t_settle = time.perf_counter() + args.settle_ms / 1e3
    while time.perf_counter() < t_settle:
        step()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rfi_s = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) / 1e3
    corr_s = float(np.mean([e[1].elapsed_time(e[2]) for e in evs])) / 1e3
    ms_per_step = wall / args.steps * 1e3
    cmac = t * tri
    flagged = float(fl.float().mean())
    res = {"metric": "Tera-CMAC/s, RFI excision + flag-aware correlation at N=2048",
           "value": round(cmac / (ms_per_step / 1e3) / 1e12, 3), "unit": "TCMAC/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "dtype": "int8", "data": "synthetic",
           "config": {"workload": f"CHIME-shaped channel with injected carriers and bursts, N={n}, T={t}, "
                                  f"flag blocks of {bl} samples", "flagged_fraction": round(flagged, 4)},
           # the excision kernel reads every sample once and writes one flag per (block, input)
           "rfi_flags_us": round(rfi_s * 1e6, 2),
           "rfi_flags_gbs": round((n * t + n * ((t + bl - 1) // bl)) / rfi_s / 1e9, 1),
           "correlate_flagged_us": round(corr_s * 1e6, 2),
           "correlate_flagged_tcmacs": round(cmac / corr_s / 1e12, 3)}
    print(json.dumps(res), flush=True)


def bench_presum(args, xeng, synth, torch, np):
    """The unsigned-nibble form with pre-sums (xeng_correlate_presum) on the
    CHIME-shaped channel: the wide kernel's unsigned instance on the stored
    nibbles, which also adds up the pre-sums; the O(N) correction runs in
    the next export.  Timed with HIP events on its stream, next to
    xeng_correlate on the same data: the call alone, and the call with its
    export (which then carries the correction of its one call)."""
    n, t = args.n, args.t
    tri = n * (n + 1) // 2
    x = torch.from_numpy(synth.chime_channel(n, t, seed=2)).cuda()
    corr = xeng.Correlator(n, 1, device=0)
    out = torch.empty((tri, 2), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn):
        t_settle = time.perf_counter() + args.settle_ms / 1e3
        while time.perf_counter() < t_settle:
            fn()
            corr.dump(0, out=out, stream=stream)
            torch.cuda.synchronize()
        evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
        for a, b, c in evs:
            a.record(stream)
            fn()
            b.record(stream)
            corr.dump(0, out=out, stream=stream)
            c.record(stream)
        torch.cuda.synchronize()
        return (float(np.mean([a.elapsed_time(b) for a, b, _ in evs])) / 1e3,
                float(np.mean([a.elapsed_time(c) for a, _, c in evs])) / 1e3)

    t_presum, s_presum = timed(lambda: corr.correlate_presum(0, x, stream=stream))
    t_plain, s_plain = timed(lambda: corr.correlate(0, x, stream=stream))
    cmac = t * tri
    res = {"metric": "Tera-CMAC/s at N=2048, unsigned-nibble form with pre-sums",
           "value": round(cmac / t_presum / 1e12, 3), "unit": "TCMAC/s", "n_gpus": 1, "steps": args.steps,
           "higher_is_better": True, "dtype": "int8", "data": "synthetic",
           "config": {"workload": f"CHIME-shaped single channel N={n}, T={t}, xeng_correlate_presum"},
           "presum_call_us": round(t_presum * 1e6, 2), "correlate_call_us": round(t_plain * 1e6, 2),
           "presum_step_us": round(s_presum * 1e6, 2), "correlate_step_us": round(s_plain * 1e6, 2),
           "roofline": {"bound": "mfma", "achieved": round(8.0 * cmac / t_presum / 1e12, 2),
                        "peak": INT8_PEAK_TOPS, "unit": "TFLOP/s",
                        "frac": round(8.0 * cmac / t_presum / 1e12 / INT8_PEAK_TOPS, 4), "traffic": None}}
    print(json.dumps(res), flush=True)


def bench_beamform(args, xeng, synth, torch, np):
    """Phased-array beamforming of the CHIME-shaped channel: 10 beams of
    complex int8 weights, exact int32 beams; HBM-bound (every sample byte
    read once, about 10 complex MACs per byte), so the roofline is GB/s."""
    n, t, nb = args.n, args.t, 10
    x = torch.from_numpy(synth.chime_channel(n, t, seed=2)).cuda()
    beams = xeng.Beams(synth.beam_weights(nb, n, seed=8))
    out = torch.empty((t, nb, 2), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    t_settle = time.perf_counter() + args.settle_ms / 1e3
    while time.perf_counter() < t_settle:
        beams.form(x, out=out, stream=stream)
        torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        beams.form(x, out=out, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_s = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
    nbytes = n * t + t * nb * 8
    gbs = nbytes / k_s / 1e9
    res = {"metric": "beamformed samples/s, 10 beams at N=2048", "value": round(t / k_s / 1e6, 3),
           "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps, "ms_per_step": round(wall / args.steps * 1e3, 4),
           "higher_is_better": True, "dtype": "int8", "data": "synthetic",
           "config": {"workload": f"CHIME-shaped channel N={n}, T={t}, {nb} beams, int32 output"},
           "beamform_us": round(k_s * 1e6, 2), "tcmacs": round(t * n * nb / k_s / 1e12, 3),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--t", type=int, default=32768)
    ap.add_argument("--settle-ms", type=float, default=300.0,
                    help="untimed steps for this long before the warm-up steps (clock ramp)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ceiling-ms", type=int, default=400,
                    help="after the timed steps, run the matrix-core ceiling loop (xeng_mfma_ceiling) this "
                         "long and report it beside the kernel (0: skip)")
    ap.add_argument("--no-clock-probe", action="store_true",
                    help="do not stamp the shader clock of the timed launches")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", default="channel",
                    choices=["channel", "channels16", "subarrays64", "serve", "flagged", "presum", "beamform"],
                    help="channel: the one-channel step (default, the JSON contract line); "
                         "channels16 / subarrays64: batched launches against plain launches; "
                         "serve: streaming channels, largest real-time K")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of each streaming trial (real time)")
    ap.add_argument("--serve-launch-us", type=float, default=4000.0,
                    help="launch period of the streaming server (frames per launch per channel)")
    ap.add_argument("--serve-stagger", type=int, choices=(0, 1), default=0,
                    help="1: each slot exports at its own phase of the export period "
                         "(XENG_SERVER_STAGGER_EXPORTS); 0: every channel exports in the same launch")
    ap.add_argument("--serve-k", default="256,288,320,336,352,368,384",
                    help="channel counts to try (device-sourced frames)")
    ap.add_argument("--serve-host-k", default="40,48,56,64",
                    help="channel counts to try with pinned-host frames (0 to skip)")
    ap.add_argument("--data", default="auto", choices=["auto", "uniform", "chime"],
                    help="channel workload data: uniform nibbles (default below N=256) "
                         "or the CHIME-shaped sky + tones + noise")
    ap.add_argument("--many-channels", type=int, default=1024,
                    help="HBM-bound N: also time this many channels of the same size "
                         "in one batched launch (0: skip)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "dma4", "general", "fp8"],
                    help="correlation kernel: the eight-wave DMA kernel (auto), its four-wave "
                         "instance, the general 128 x 128 kernel, or its exact FP8 instance")
    ap.add_argument("--plan-order", default="xcd", choices=["xcd", "linear"],
                    help="work order of the single-channel launch (xeng_set_plan_order; never changes results)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this many MiB "
                         "(reference kernel for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: only one GPU is used by this build (got --gpus {args.gpus}); "
              "channels shard across GPUs with no exchange, so run one process per GPU.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2005_09481_amd import xeng

    xeng.set_plan_order({"xcd": xeng.XENG_PLAN_XCD, "linear": xeng.XENG_PLAN_LINEAR}[args.plan_order])
    xeng.set_tuning(0, 0, {"auto": xeng.XENG_KERNEL_AUTO, "dma4": xeng.XENG_KERNEL_DMA4,
                           "general": xeng.XENG_KERNEL_GENERAL, "fp8": xeng.XENG_KERNEL_FP8}[args.kernel])
    if args.workload == "serve":
        return bench_serve(args, xeng, synth, torch, np)
    if args.workload == "flagged":
        return bench_flagged(args, xeng, synth, torch, np)
    if args.workload == "presum":
        return bench_presum(args, xeng, synth, torch, np)
    if args.workload == "beamform":
        return bench_beamform(args, xeng, synth, torch, np)
    if args.workload != "channel":
        return bench_batch(args, xeng, synth, torch, np)

    n, t = args.n, args.t
    tri = n * (n + 1) // 2
    data = args.data if args.data != "auto" else ("uniform" if n < 256 else "chime")
    x_np = synth.uniform_bytes(n, t, seed=1) if data == "uniform" else synth.chime_channel(n, t, seed=2)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(x_np).to(dev)
    corr = xeng.Correlator(n, 1, device=0)
    out = torch.empty((tri, 2), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        corr.correlate(0, x, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        corr.dump(0, out=out, reset=True, stream=stream)

    t_settle = time.perf_counter() + args.settle_ms / 1e3
    while time.perf_counter() < t_settle:
        for _ in range(10):
            step()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    # shader clock of the timed launches (the wide kernel's workgroup 0
    # stamps its start and end; the last launch's stamps remain)
    clk = torch.zeros(4, dtype=torch.int64, device=dev)
    if not args.no_clock_probe:
        xeng.clock_probe(clk, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not args.no_clock_probe:
        xeng.clock_probe(None, 0)
    sclk = xeng.sclk_ghz(clk) if int(clk[0]) != 0 else None
    kern_ms = [a.elapsed_time(b) for a, b in events]
    kern_s = float(np.mean(kern_ms)) / 1e3

    ms_per_step = wall / args.steps * 1e3
    cmac = t * tri
    value = cmac / (ms_per_step / 1e3) / 1e12
    achieved = 8.0 * cmac / kern_s / 1e12            # int8 ops: 4 MAC per CMAC, 2 ops per MAC
    # 2(N+1) int8 MACs per input byte against the chip's balance of
    # 2.5e15 MAC/s / 8e12 B/s: below it (N < ~155) the kernel is HBM-bound
    hbm_bound = 2 * (n + 1) < INT8_PEAK_TOPS / 2 / HBM_PEAK_GBS * 1e3
    if hbm_bound:
        gbs = (n * t + 8 * tri) / kern_s / 1e9       # samples in, one export's worth out
        roofline = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
        many = bench_many_channels(args, xeng, synth, torch, np, n, t) if args.many_channels > 0 else None
    else:
        roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / INT8_PEAK_TOPS, 4),
                    "traffic": measured_traffic() if (n, t) == (2048, 32768) and args.kernel == "auto"
                    and args.plan_order == "xcd" else None}
    res = {
        "metric": "Tera-CMAC/s at N=2048 (int8 MFMA util %)",
        "value": round(value, 3),
        "unit": "TCMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp8-e4m3" if args.kernel == "fp8" else "int8",
        "data": "synthetic",
        "config": {"workload": (f"CHIME-shaped single channel N={n}, T={t}, 4+4-bit, "
                                if data == "chime" else
                                f"single channel N={n}, T={t}, 4+4-bit, uniform nibbles, ")
                               + "correlate + dump/reset per step",
                   "n_inputs": n, "n_samples": t, "parallelism": "single GPU",
                   "plan_order": args.plan_order, "kernel": args.kernel},
        "roofline": roofline,
        "mfma_util_pct": round(100 * achieved / INT8_PEAK_TOPS, 2),
        # the int8 peak assumes 2.4 GHz; under this load the chip runs slower
        "sclk_ghz": round(sclk, 3) if sclk else None,
        "mfma_util_at_sclk_pct": round(100 * achieved / (INT8_PEAK_TOPS * sclk / 2.4), 2) if sclk else None,
        "correlate_kernel_ms": round(kern_s * 1e3, 4),
        "correlate_tcmacs": round(cmac / kern_s / 1e12, 3),
    }
    if hbm_bound and many is not None:
        res["many_channels_one_launch"] = many
    if not hbm_bound and args.ceiling_ms > 0:
        # the same chip in the same state, running nothing but int8 MFMAs: the
        # rate its power limit allows any int8 kernel (context for the line:
        # a failure here is reported, not fatal)
        try:
            mac_s, ceil_ghz = xeng.mfma_ceiling(args.ceiling_ms, 0)
            ceil_frac = 2.0 * mac_s / 1e12 / INT8_PEAK_TOPS
            res["mfma_ceiling"] = {"tops": round(2.0 * mac_s / 1e12, 1), "frac_of_peak": round(ceil_frac, 4),
                                   "sclk_ghz": round(ceil_ghz, 3), "ms": args.ceiling_ms}
            res["frac_of_ceiling"] = round(achieved / INT8_PEAK_TOPS / ceil_frac, 4) if ceil_frac > 0 else None
        except xeng.XengError as e:
            res["mfma_ceiling"] = {"error": str(e)}
    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(x_np, n, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
