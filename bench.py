"""Throughput and latency of the first-match classifier on one MI355X.

One step classifies the whole batch of the 10,000-rule x 16,777,216-packet
workload (skewed prefix lengths) once, with inputs already resident in HBM.
The headline value is the learned-index path's Mpps when the index can be
built, next to the plain scans (packet split, rule split with 16 partitions)
timed the same way on the same batch; p50/p99 are closed-loop batch latencies
(one batch in flight, sizes log-uniform in 64..65,536).  Prints one JSON line
on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--seed S]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks used for the roofline: HBM3E bandwidth, and the int32
# vector-ALU lane-op rate 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
HBM_PEAK_GBS = 8000.0
VALU_INT32_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic cost of one rule check: the destination test every check makes
# (one subtract, one unsigned compare); deeper field tests are not counted.
OPS_PER_CHECK = 2
BYTES_PER_PACKET = 13 + 5          # 5-tuple in (4+4+2+2+1), index + action out (4+1)


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def time_steps(fn, steps: int, warmup: int, stream):
    """Run fn() `warmup` times, then time exactly `steps` calls with events on `stream`."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def closed_loop_latency(rs, dp, mode_kw, seed: int, n_batches: int, stream):
    """p50/p99 of host-enqueue-to-completion over batches of log-uniform size."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed + 31337))
    sizes = np.clip(np.round(np.exp(rng.uniform(math.log(64), math.log(65536), n_batches))),
                    64, 65536).astype(np.int64)
    starts = rng.integers(0, (len(dp) - 65536) // 16, n_batches) * 16   # 16-byte aligned
    n = len(dp)
    out_i = torch.empty(65536, dtype=torch.int32, device="cuda")
    out_a = torch.empty(65536, dtype=torch.uint8, device="cuda")
    for i in range(20):                           # warm the path
        rs.classify(dp.slice(0, 4096), stream=stream, out_idx=out_i, out_act=out_a, **mode_kw)
    stream.synchronize()
    lat = np.empty(n_batches)
    for b in range(n_batches):
        s, k = int(starts[b]), int(sizes[b])
        sub = dp.slice(s, min(n, s + k))
        t0 = time.perf_counter()
        rs.classify(sub, stream=stream, out_idx=out_i, out_act=out_a, **mode_kw)
        stream.synchronize()
        lat[b] = time.perf_counter() - t0
    return float(np.percentile(lat, 50) * 1e6), float(np.percentile(lat, 99) * 1e6)


def cpu_baseline(rules, pk, n_sample: int):
    """The CPU oracle, as it stands, on a bounded sample of the same batch."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    sub = pk.subset(slice(0, n_sample))
    t0 = time.perf_counter()
    oracle.classify(rules, sub, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt / 1e6, "unit": "Mpps", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sample} packets of the timed batch, {threads} threads, "
                      f"{dt:.2f} s wall"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", default="learned_10000x16M")
    ap.add_argument("--latency-batches", type=int, default=2000)
    ap.add_argument("--cpu-sample", type=int, default=4_194_304)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the packet-split "
              "path shards by packets with no exchange, so the one-GPU figure is per GPU.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from synth import gen
    from paper_1312_4188_amd import fw

    log(f"generating {args.workload} seed {args.seed}")
    rules, pk = gen.workload(args.workload, seed=args.seed)
    n, R = len(pk), len(rules)
    dp = fw.DevicePackets.from_host(pk)
    stream = torch.cuda.current_stream()
    out_i = torch.empty(n, dtype=torch.int32, device="cuda")
    out_a = torch.empty(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    rs = fw.Ruleset(rules)
    modes = {"packet_split": dict(mode="packet_split"),
             "rule_split_p16": dict(mode="rule_split", partitions=16)}
    results = {}
    ref = None
    for name, kw in modes.items():
        log(f"timing {name}")
        ms, wall = time_steps(lambda: rs.classify(dp, stream=stream, out_idx=out_i,
                                                  out_act=out_a, **kw),
                              args.steps, args.warmup, stream)
        idx = out_i.cpu().numpy()
        if ref is None:
            ref = idx.copy()
        agree = bool(np.array_equal(idx, ref))
        checks = int(np.where(idx < 0, R, idx.astype(np.int64) + 1).sum())
        results[name] = {"ms": ms, "mpps": n / ms / 1e3,
                         "rule_checks_per_s": checks / (ms * 1e-3),
                         "same_as_packet_split": agree, "wall_s": wall}
        log(f"  {name}: {ms:.3f} ms/step, {n / ms / 1e3:.1f} Mpps")

    checks = int(np.where(ref < 0, R, ref.astype(np.int64) + 1).sum())
    full = ((rules.src_plen == 0) & (rules.dst_plen == 0) & (rules.proto_any != 0) &
            (rules.sport_lo == 0) & (rules.sport_hi == 65535) &
            (rules.dport_lo == 0) & (rules.dport_hi == 65535))
    k_star = int(np.argmax(full)) if full.any() else None   # first catch-all rule

    latency = {}
    for name, kw in modes.items():
        log(f"latency {name}")
        p50, p99 = closed_loop_latency(rs, dp, kw, args.seed, args.latency_batches, stream)
        latency[name] = {"p50_us": p50, "p99_us": p99}

    head = "packet_split"
    ms = results[head]["ms"]
    achieved_tops = checks * OPS_PER_CHECK / (ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved_tops, "peak": VALU_INT32_PEAK_TOPS,
                "unit": "Tops/s", "frac": achieved_tops / VALU_INT32_PEAK_TOPS,
                "traffic": None, "kernel": "k_packet_split<4>",
                "hbm_gbs": n * BYTES_PER_PACKET / (ms * 1e-3) / 1e9}

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(rules, pk, min(args.cpu_sample, n))

    line = {
        "metric": "Mpps (bit-exact first-match) at 10k rules: learned-index vs scan; p99 latency",
        "value": results[head]["mpps"], "unit": "Mpps", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded generators)",
        "config": {"workload": args.workload, "rules": R, "packets": n, "seed": args.seed,
                   "path": head, "k_star": k_star},
        "modes": results, "latency": latency,
        "rule_checks_per_s": checks / (ms * 1e-3),
        "roofline": roofline, "cpu_baseline": cpu,
    }
    rs.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
