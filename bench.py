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
RECORD_BYTES = 32                  # one compiled rule record


def kernel_sources_sha256() -> str:
    """Hash of every .hip and .h kernel source (name + bytes, sorted)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1312_4188_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def committed_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or {} when
    that summary is for another workload or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_sha256():
        return {}
    return {k.split(".")[0]: float(v) for k, v in vals.items() if k.endswith(".traffic_bytes")}


def _list_checks(B, off, L, keys, ans):
    """Per packet: entries of its interval's list up to and including its answer."""
    M = len(B)
    j = np.searchsorted(B, keys, side="right") - 1
    owner = np.repeat(np.arange(M, dtype=np.int64), np.diff(off))
    key = owner * (1 << 41) + L
    return np.searchsorted(key, j * (1 << 41) + ans, side="right") - off[j]


def learned_work(rs, pk, idx, hidden: int = 32):
    """Exact algorithmic work of the learned path for every packet of the batch.

    Candidate checks of packet p: the entries of its destination interval's
    list, of its source interval's list (destination-wildcard rules that
    specify a source) and of the fully wildcard shared list, each up to and
    including p's first match (all of them when nothing matches).  Lane-ops:
    2 per candidate check (one subtract, one compare: the first field test),
    6H per packet for the two networks (per hidden unit a multiply-add, a max
    and a multiply-add, in each stage) and 2 per binary-search probe (the mean
    error window, plus the source-interval search).  Bytes: the packet in, the
    result out, and a 32-byte record gathered per check of a per-lane list.
    """
    e = lambda w: rs.export(w).astype(np.int64)
    B, off, L, err = e(0), e(1), e(2), rs.export(4).astype(np.float64)
    Bs, soff, S, Gw = e(6), e(7), e(8), e(9)
    ans = np.where(idx < 0, 1 << 40, idx.astype(np.int64))
    n_l = _list_checks(B, off, L, pk.dst_ip.astype(np.int64), ans)
    n_s = _list_checks(Bs, soff, S, pk.src_ip.astype(np.int64), ans)
    n_g = np.searchsorted(Gw, ans, side="right")
    checks = int(n_l.sum() + n_s.sum() + n_g.sum())
    probes = (math.ceil(math.log2(2.0 * float(err.mean()) + 1.0)) + 1
              + math.ceil(math.log2(max(len(Bs), 1))) + 1)
    ops = 2 * checks + len(pk) * (6 * hidden + 2 * probes)
    gathered = int(n_l.sum() + n_s.sum())
    nbytes = len(pk) * BYTES_PER_PACKET + gathered * RECORD_BYTES
    return {"candidate_checks": checks, "list_checks": gathered, "lane_ops": ops,
            "bytes": nbytes, "probes_per_packet": probes}


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
    ap.add_argument("--modes", default="",
                    help="comma list of modes to time (default: all); the first is the headline")
    ap.add_argument("--serving-requests", type=int, default=600,
                    help="requests per offered load in the serving leg (0 = skip it)")
    ap.add_argument("--no-multichain", action="store_true", help="skip the 64-chain leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for scaling HBM counters)")
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
    log("building the learned index (trained)")
    t0 = time.perf_counter()
    index_stats = rs.build_learned_index(seed=args.seed)
    index_stats["build_s"] = time.perf_counter() - t0
    rs_un = fw.Ruleset(rules)
    log("building the learned index (untrained network)")
    untrained_stats = rs_un.build_learned_index(seed=args.seed, train=False)
    modes = {"learned": (rs, dict(mode="learned")),
             "learned_binary_search": (rs, dict(mode="learned", lookup=1)),
             "learned_untrained": (rs_un, dict(mode="learned")),
             "learned_k1": (rs, dict(mode="learned", packets_per_lane=1)),
             "learned_k4": (rs, dict(mode="learned", packets_per_lane=4)),
             "packet_split": (rs, dict(mode="packet_split")),
             "packet_split_k1": (rs, dict(mode="packet_split", packets_per_lane=1)),
             "packet_split_k2": (rs, dict(mode="packet_split", packets_per_lane=2)),
             "rule_split_p16": (rs, dict(mode="rule_split", partitions=16)),
             "hybrid_p16": (rs, dict(mode="hybrid", partitions=16))}
    if args.modes:
        keep = args.modes.split(",")
        modes = {k: modes[k] for k in keep}
    results = {}
    ref = None
    for name, (ruleset, kw) in modes.items():
        log(f"timing {name}")
        ms, wall = time_steps(lambda: ruleset.classify(dp, stream=stream, out_idx=out_i,
                                                       out_act=out_a, **kw),
                              args.steps, args.warmup, stream)
        idx = out_i.cpu().numpy()
        act = out_a.cpu().numpy()
        if ref is None:
            ref = (idx.copy(), act.copy())
        agree = bool(np.array_equal(idx, ref[0]) and np.array_equal(act, ref[1]))
        results[name] = {"ms": ms, "mpps": n / ms / 1e3, "same_as_learned": agree,
                         "wall_s": wall}
        if kw["mode"] == "learned":
            _, _, miss = ruleset.classify(dp, stream=stream, out_idx=out_i, out_act=out_a,
                                          count_misses=True, **kw)
            results[name]["window_misses"] = miss
        log(f"  {name}: {ms:.3f} ms/step, {n / ms / 1e3:.1f} Mpps")
    ref = ref[0]
    checks = int(np.where(ref < 0, R, ref.astype(np.int64) + 1).sum())
    for name in [m for m in ("packet_split", "rule_split_p16", "hybrid_p16") if m in results]:
        results[name]["rule_checks_per_s"] = checks / (results[name]["ms"] * 1e-3)
    full = ((rules.src_plen == 0) & (rules.dst_plen == 0) & (rules.proto_any != 0) &
            (rules.sport_lo == 0) & (rules.sport_hi == 65535) &
            (rules.dport_lo == 0) & (rules.dport_hi == 65535))
    k_star = int(np.argmax(full)) if full.any() else None   # first catch-all rule

    latency = {}
    for name in [m for m in ("learned", "packet_split", "rule_split_p16", "hybrid_p16")
                 if m in modes and args.latency_batches > 0]:
        ruleset, kw = modes[name]
        log(f"latency {name}")
        p50, p99 = closed_loop_latency(ruleset, dp, kw, args.seed, args.latency_batches, stream)
        latency[name] = {"p50_us": p50, "p99_us": p99}

    head = next(iter(modes))
    ms = results[head]["ms"]
    work = learned_work(rs, pk, ref)
    achieved_tops = work["lane_ops"] / (ms * 1e-3) / 1e12
    traffic = committed_traffic(args.workload)
    roofline = {"bound": "alu", "achieved": achieved_tops, "peak": VALU_INT32_PEAK_TOPS,
                "unit": "Tops/s", "frac": achieved_tops / VALU_INT32_PEAK_TOPS,
                "traffic": traffic.get("k_learned"), "kernel": "k_learned<true,2>",
                "algorithmic_lane_ops": work["lane_ops"], "algorithmic_bytes": work["bytes"],
                "hbm_gbs": work["bytes"] / (ms * 1e-3) / 1e9,
                "hbm_frac": work["bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    scan_roofline = None
    if "packet_split" in results:
        scan_ms = results["packet_split"]["ms"]
        scan_ops = checks * OPS_PER_CHECK
        scan_roofline = {"bound": "alu", "kernel": "k_packet_split<4>",
                         "traffic": traffic.get("k_packet_split"),
                         "achieved": scan_ops / (scan_ms * 1e-3) / 1e12,
                         "frac": scan_ops / (scan_ms * 1e-3) / 1e12 / VALU_INT32_PEAK_TOPS,
                         "hbm_gbs": n * BYTES_PER_PACKET / (scan_ms * 1e-3) / 1e9}
    if args.copy_calibration:
        log("copy calibration: 256 MiB device-to-device")
        a = torch.empty(64 << 20, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()

    serving = None
    if args.serving_requests > 0:
        log("serving leg")
        serving = serving_leg(args.seed, args.serving_requests,
                              (0.1, 0.3, 0.5, 0.7, 0.9, 1.0, 1.2), log)

    multichain = None
    if not args.no_multichain:
        log("multi-chain leg")
        multichain = multichain_leg(args.seed, max(3, args.steps // 2), log)

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
        "scan_mpps": results["packet_split"]["mpps"] if "packet_split" in results else None,
        "speedup_vs_scan": (results["packet_split"]["ms"] / ms
                            if "packet_split" in results else None),
        "p99_us": latency.get(head, {}).get("p99_us"),
        "p50_us": latency.get(head, {}).get("p50_us"),
        "modes": results, "latency": latency,
        "scan_rule_checks": checks, "learned_candidate_checks": work["candidate_checks"],
        "index": index_stats, "index_untrained": untrained_stats,
        "roofline": roofline, "scan_roofline": scan_roofline, "serving": serving,
        "multichain": multichain,
        "cpu_baseline": cpu,
    }
    rs.close()
    rs_un.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
