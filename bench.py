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


def cpu_baseline(x, n, target_s=12.0):
    """The oracle, as it stands, on a bounded time sample of the same input."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    tri = n * (n + 1) // 2
    t_probe = 64
    t0 = time.perf_counter()
    oracle.correlate(np.ascontiguousarray(x[:t_probe]))
    dt = time.perf_counter() - t0
    rate = t_probe * tri / max(dt, 1e-6)
    t_s = int(min(x.shape[0], max(t_probe, target_s * rate / tri)))
    t_s = max(32, (t_s // 32) * 32)
    t0 = time.perf_counter()
    oracle.correlate(np.ascontiguousarray(x[:t_s]))
    dt = time.perf_counter() - t0
    return {"value": t_s * tri / dt / 1e12, "unit": "TCMAC/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {t_s} of {x.shape[0]} samples of the N={n} channel "
                      f"({t_s * tri:.3e} CMAC in {dt:.1f} s)"}


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
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
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

    n, t = args.n, args.t
    tri = n * (n + 1) // 2
    x_np = synth.chime_channel(n, t, seed=2)
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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in events]
    kern_s = float(np.mean(kern_ms)) / 1e3

    ms_per_step = wall / args.steps * 1e3
    cmac = t * tri
    value = cmac / (ms_per_step / 1e3) / 1e12
    achieved = 8.0 * cmac / kern_s / 1e12            # int8 ops: 4 MAC per CMAC, 2 ops per MAC
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
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": f"CHIME-shaped single channel N={n}, T={t}, 4+4-bit, "
                               "correlate + dump/reset per step",
                   "n_inputs": n, "n_samples": t, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / INT8_PEAK_TOPS, 4),
                     "traffic": None},
        "mfma_util_pct": round(100 * achieved / INT8_PEAK_TOPS, 2),
        "correlate_kernel_ms": round(kern_s * 1e3, 4),
        "correlate_tcmacs": round(cmac / kern_s / 1e12, 3),
    }
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
