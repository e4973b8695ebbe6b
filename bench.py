"""Throughput and latency of the first-match classifier on one MI355X.

One step classifies the whole batch of the 10,000-rule x 16,777,216-packet
workload (skewed prefix lengths) once, with inputs already resident in HBM.
The headline value is the learned-index path's Mpps when the index can be
built, next to the plain scans (packet split, rule split with 16 partitions)
timed the same way on the same batch; p50/p99 are closed-loop batch latencies
(one batch in flight, sizes log-uniform in 64..65,536), enqueue to completion through
the library's C interface (fw_closed_loop); the same batches driven from Python, one
binding call each, are reported beside them.  Prints one JSON line
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
# A fuller pricing of a learned-path candidate check: every field test, the select of the
# answer and the list step, about 7 lane-ops; reported beside the lower bound above.
OPS_PER_CHECK_FULL = 7
BYTES_PER_PACKET = 13 + 5          # 5-tuple in (4+4+2+2+1), index + action out (4+1)
RECORD_BYTES = 32                  # one compiled rule record
SETTLE_MS = 50.0                   # minimum warm-up of the secondary legs' timings


# The sources the profiled kernels (k_learned, k_lookup, k_packet_split) are compiled from:
# their two translation units and every header under csrc/ that those include (the public
# header include/fw.h, also included, is left out: its edits are mostly documentation).
PROFILED_SOURCES = ("device_util.h", "fw_internal.h", "host_types.h", "index.h",
                    "learned_core.h", "rmi.hip", "scan.hip", "scan_core.h")


def kernel_sources_sha256() -> str:
    """Hash of the profiled kernels' sources (name + bytes, in the order above)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1312_4188_amd", "csrc")
    for name in PROFILED_SOURCES:
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as f:
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


def committed_valu_counters(workload: str):
    """Executed VALU lane-ops per launch (SQ_INSTS_VALU x 64) from the committed counter summary,
    or {} when it is for another workload or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"valu_counters_{workload}.txt")
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
    return {k.rsplit(".", 1)[0]: 64.0 * float(v) for k, v in vals.items()
            if k.endswith(".SQ_INSTS_VALU")}


def _list_checks(B, off, L, keys, ans):
    """Per packet: entries of its interval's list up to and including its answer."""
    M = len(B)
    j = np.searchsorted(B, keys, side="right") - 1
    owner = np.repeat(np.arange(M, dtype=np.int64), np.diff(off))
    key = owner * (1 << 41) + L
    return np.searchsorted(key, j * (1 << 41) + ans, side="right") - off[j]


def learned_work(rs, pk, idx, hidden: int = 32, network: bool = True):
    """Exact algorithmic work of the learned path for every packet of the batch.

    Candidate checks of packet p: the entries of its destination interval's
    list, of its source interval's list (destination-wildcard rules that
    specify a source) and of the address-wildcard rules past the first 64 (the
    grouped scan), each up to and including p's first match (all of them when
    nothing matches).  Lane-ops: 2 per candidate check (one subtract, one
    compare: the first field test); 6H per packet for the two networks (per
    hidden unit a multiply-add, a max and a multiply-add, in each stage); 2 per
    binary-search probe of the mean error window and 2 per probe of the
    source-interval lookup (bucket-table read plus its walk steps, or a
    binary search when the index has no bucket table); without the network (``network`` false),
    no 6H and the probes of the full binary search over B instead of the window; for the
    port/protocol table of the first 64 address-wildcard
    rules, 2 per table read (the two high-byte tables, the walk steps, three
    masks, the rule entry) and 3 for combining the masks (two ANDs, one bit
    scan).  Bytes: the packet in, the result out, and a 32-byte record
    gathered per check of a per-lane list.
    """
    e = lambda w: rs.export(w).astype(np.int64)
    B, off, L, err = e(0), e(1), e(2), rs.export(4).astype(np.float64)
    Bs, soff, S, Gw = e(6), e(7), e(8), e(9)
    pt_count, steps_s, steps_d, bs_bits, bs_steps = (int(x) for x in rs.export(11))
    rest = Gw[pt_count:]                 # the table holds the first pt_count entries
    ans = np.where(idx < 0, 1 << 40, idx.astype(np.int64))
    n_l = _list_checks(B, off, L, pk.dst_ip.astype(np.int64), ans)
    n_s = _list_checks(Bs, soff, S, pk.src_ip.astype(np.int64), ans)
    n_g = np.searchsorted(rest, ans, side="right")
    checks = int(n_l.sum() + n_s.sum() + n_g.sum())
    src_probes = (1 + bs_steps) if bs_bits else math.ceil(math.log2(max(len(Bs), 1))) + 1
    if network:
        probes = math.ceil(math.log2(2.0 * float(err.mean()) + 1.0)) + 1 + src_probes
    else:            # the full binary search over B instead of the network and its window
        probes = math.ceil(math.log2(max(len(B), 1))) + 1 + src_probes
    table_ops = (2 * (2 + steps_s + steps_d + 4) + 3) if pt_count else 0
    ops = 2 * checks + len(pk) * ((6 * hidden if network else 0) + 2 * probes + table_ops)
    gathered = int(n_l.sum() + n_s.sum())
    nbytes = len(pk) * BYTES_PER_PACKET + gathered * RECORD_BYTES
    return {"candidate_checks": checks, "list_checks": gathered, "lane_ops": ops,
            "bytes": nbytes, "probes_per_packet": probes, "table_ops_per_packet": table_ops}


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def time_steps(fn, steps: int, warmup: int, stream, settle_ms: float = 0.0):
    """Run fn() `warmup` times, then time exactly `steps` calls with events on `stream`.
    With settle_ms, the warm-up continues until it has kept the GPU busy that long (the
    clocks settle after about 20 ms of sustained work; the secondary legs use this, the
    headline loop takes exactly `warmup` steps)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if settle_ms > 0:
        t0 = time.perf_counter()
        while (time.perf_counter() - t0) * 1e3 < settle_ms:
            for _ in range(8):
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
    # the same batches through the library's own closed loop (no Python per batch)
    counts = np.minimum(sizes, n - starts)
    rs.closed_loop(dp, starts[:20], counts[:20], stream=stream, **mode_kw)   # warm
    nat = rs.closed_loop(dp, starts, counts, stream=stream, **mode_kw)[0]
    pct = lambda a, q: float(np.percentile(a, q) * 1e6)
    return {"p50_us": pct(nat, 50), "p99_us": pct(nat, 99),
            "python_p50_us": pct(lat, 50), "python_p99_us": pct(lat, 99)}


def serving_oracle(chains, chain, offset, sizes, pool):
    """The CPU oracle's answer for every request of a serving trace, at the request's offset
    in the pool (requests of one chain classified together)."""
    import oracle
    from synth import gen
    total = int(pool[0].shape[0])
    want_i = np.full(total, -7, dtype=np.int32)
    want_a = np.zeros(total, dtype=np.uint8)
    u = lambda a, dt: a.view(dt)
    for c in range(len(chains)):
        ks = np.nonzero(chain == c)[0]
        if ks.size == 0:
            continue
        pos = np.concatenate([np.arange(int(offset[k]), int(offset[k] + sizes[k])) for k in ks])
        pk = gen.Packets(u(pool[0], np.uint32)[pos], u(pool[1], np.uint32)[pos],
                         u(pool[2], np.uint16)[pos], u(pool[3], np.uint16)[pos], pool[4][pos])
        i, a = oracle.classify(chains[c], pk, threads=max(1, min(16, os.cpu_count() or 1)))
        want_i[pos] = i
        want_a[pos] = a
    return want_i, want_a


def serving_leg(seed: int, n_req: int, loads, log_fn):
    """Open-loop serving: 3 resident chains, Poisson arrivals of log-uniform batches.

    The same trace of request sizes and chains is replayed at each offered
    load (a fraction of the saturated throughput measured first), through the
    native load generator; latency is done - scheduled arrival.
    """
    import torch
    from synth import gen
    from paper_1312_4188_amd import fw
    chains = gen.serving_chains(seed)
    rsets = [fw.Ruleset(c) for c in chains]
    build = []
    for rs in rsets:
        t0 = time.perf_counter()
        st = rs.build_learned_index(seed=seed)
        build.append({"rules": rs.n_rules, "build_s": time.perf_counter() - t0,
                      "err_mean": st["err_mean"], "boundaries": st["n_boundaries"]})
    _, sizes, chain = gen.serving_arrivals(seed, n_req, 1.0, n_chains=len(chains))
    sizes = (sizes + 15) // 16 * 16                     # 16-byte aligned slices
    offset = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.uint64)
    total = int(sizes.sum())

    def pinned(n, dt):
        t = torch.empty(n, dtype=dt, pin_memory=True)
        return t, t.numpy()
    keep, pool = [], []
    for n_bytes, dt, field in ((4, torch.int32, "src_ip"), (4, torch.int32, "dst_ip"),
                               (2, torch.int16, "sport"), (2, torch.int16, "dport"),
                               (1, torch.uint8, "proto")):
        t, a = pinned(total, dt)
        keep.append(t)
        pool.append(a)
    for k in range(n_req):
        pk = gen.make_packets(chains[chain[k]], int(sizes[k]), seed * 7919 + k)
        o, e = int(offset[k]), int(offset[k] + sizes[k])
        pool[0][o:e] = pk.src_ip.view(np.int32)
        pool[1][o:e] = pk.dst_ip.view(np.int32)
        pool[2][o:e] = pk.sport.view(np.int16)
        pool[3][o:e] = pk.dport.view(np.int16)
        pool[4][o:e] = pk.proto
    ti, out_i = pinned(total, torch.int32)
    ta, out_a = pinned(total, torch.uint8)
    want_i, want_a = serving_oracle(chains, chain, offset, sizes, pool)
    out = {"chains": build, "requests": n_req, "packets": total, "modes": {},
           "host": {"logical_cpus": os.cpu_count(),
                    "usable_cpus": len(os.sched_getaffinity(0))
                    if hasattr(os, "sched_getaffinity") else None}}
    mean_batch = total / n_req
    for name, mode, slots, ingest in (("learned_copy", "auto", 4, "copy"),
                                      ("learned_mapped", "auto", 4, "mapped"),
                                      ("learned_copy_1slot", "auto", 1, "copy"),
                                      ("packet_split_copy", "packet_split", 4, "copy"),
                                      ("packet_split_mapped", "packet_split", 4, "mapped")):
        with fw.Server(rsets, slots=slots, mode=mode, ingest=ingest) as sv:
            zero = np.zeros(n_req)
            sv.replay(zero[:32], chain[:32], offset[:32], sizes[:32], pool, out_i, out_a)
            t = sv.replay(zero, chain, offset, sizes, pool, out_i, out_a)
            peak = total / (t[:, 2].max() - t[:, 0].min()) / 1e6
            res = {"peak_mpps": peak, "loads": [], "slots": slots, "ingest": ingest,
                   "mode": mode}
            log_fn(f"  serving {name}: saturated {peak:.0f} Mpps")
            for frac in loads:
                rate = frac * peak * 1e6 / mean_batch          # requests per second
                rng = np.random.Generator(np.random.PCG64(seed + int(frac * 1000)))
                arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
                t = sv.replay(arr, chain, offset, sizes, pool, out_i, out_a)
                lat = (t[:, 2] - t[:, 0]) * 1e6
                span = t[:, 2].max() - t[:, 0].min()
                res["loads"].append({"offered_frac": frac, "offered_mpps": frac * peak,
                                     "achieved_mpps": total / span / 1e6,
                                     "p50_us": float(np.percentile(lat, 50)),
                                     "p99_us": float(np.percentile(lat, 99))})
                log_fn(f"  serving {name} load {frac:.0%}: "
                       f"p50 {res['loads'][-1]['p50_us']:.0f} us "
                       f"p99 {res['loads'][-1]['p99_us']:.0f} us")
            # the last replay wrote every request's results: each one against the oracle
            res["bit_exact"] = bool(np.array_equal(out_i, want_i) and
                                    np.array_equal(out_a, want_a))
            log_fn(f"  serving {name}: every request bit-exact vs the oracle: {res['bit_exact']}")
            out["modes"][name] = res
    for rs in rsets:
        rs.close()
    return out


def ingest_leg(rs, pk, ref_idx, chunk: int, log_fn):
    """The whole batch from pinned host memory through the serving runtime: submitted in
    chunks of `chunk` packets at once, copied in, classified and copied out (copy ingest), or
    read and written in place by the kernel (mapped ingest).  One chunk per group lets the
    slots overlap one chunk's copies with another's classification; the default lets a slot
    take as many chunks as its share of the budget holds.  PCIe-inclusive rate, reported
    beside the headline (which starts from HBM-resident packets)."""
    import torch
    from paper_1312_4188_amd import fw
    n = len(pk)
    pool, keep = [], []
    for a, dt in ((pk.src_ip, torch.int32), (pk.dst_ip, torch.int32), (pk.sport, torch.int16),
                  (pk.dport, torch.int16), (pk.proto, torch.uint8)):
        t = torch.empty(n, dtype=dt, pin_memory=True)
        v = t.numpy().view(a.dtype)
        v[:] = a
        keep.append(t)
        pool.append(v)
    ti = torch.empty(n, dtype=torch.int32, pin_memory=True)
    ta = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    out_i, out_a = ti.numpy(), ta.numpy()
    sizes = np.full((n + chunk - 1) // chunk, chunk, dtype=np.uint64)
    sizes[-1] = n - chunk * (len(sizes) - 1)
    offset = np.arange(len(sizes), dtype=np.uint64) * np.uint64(chunk)
    chain = np.zeros(len(sizes), dtype=np.uint32)
    zero = np.zeros(len(sizes))
    out = {"packets": n, "chunk": chunk, "bytes_per_packet": BYTES_PER_PACKET}
    for slots, ingest, group in ((1, "copy", 1), (2, "copy", 1), (4, "copy", 1),
                                 (4, "copy", 0), (1, "mapped", 1), (4, "mapped", 1),
                                 (4, "mapped", 0)):
        with fw.Server([rs], slots=slots, mem_budget=1 << 30, ingest=ingest,
                       max_group=group) as sv:
            sv.replay(zero[:2], chain[:2], offset[:2], sizes[:2], pool, out_i, out_a)  # warm
            out_i[:] = -2
            t = sv.replay(zero, chain, offset, sizes, pool, out_i, out_a)
            span = float(t[:, 2].max() - t[:, 0].min())
            name = f"{ingest}_slots_{slots}" + ("_chunk_per_group" if group == 1 else "")
            out[name] = {"s": span, "mpps": n / span / 1e6,
                         "pcie_gbs": n * BYTES_PER_PACKET / span / 1e9,
                         "same_as_device": bool(np.array_equal(out_i, ref_idx))}
            log_fn(f"  ingest {name}: {n / span / 1e6:.0f} Mpps "
                   f"({n * BYTES_PER_PACKET / span / 1e9:.1f} GB/s over PCIe), "
                   f"same as device-resident: {out[name]['same_as_device']}")
    return out


def scan_configs_leg(seed: int, steps: int, log_fn):
    """The two plain-scan configurations side by side: 100 rules x 10,000 packets and 1,000
    rules x 1,048,576 packets, packet split and rule split (16 partitions), each checked bit for
    bit against the CPU oracle.  Rule-checks/s count the scan's algorithmic work (first-match
    index + 1, or R, per packet); the VALU fraction prices each check at 2 lane-ops against the
    39.3 T peak; GB/s counts 18 bytes per packet (13 in, 5 out)."""
    import torch
    import oracle
    from synth import gen
    from paper_1312_4188_amd import fw
    out = {}
    for wl in ("scan_100x10k", "scan_1000x1M"):
        rules, pk = gen.workload(wl, seed=seed)
        n, R = len(pk), len(rules)
        want_idx, want_act = oracle.classify(rules, pk, threads=16)
        checks = int(np.where(want_idx < 0, R, want_idx.astype(np.int64) + 1).sum())
        dp = fw.DevicePackets.from_host(pk)
        oi = torch.empty(n, dtype=torch.int32, device="cuda")
        oa = torch.empty(n, dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream()
        res = {"rules": R, "packets": n, "rule_checks": checks}
        with fw.Ruleset(rules) as rs:
            for name, kw in (("packet_split", dict(mode="packet_split")),
                             ("rule_split_p16", dict(mode="rule_split", partitions=16))):
                ms, _ = time_steps(lambda: rs.classify(dp, stream=stream, out_idx=oi, out_act=oa,
                                                       **kw), max(steps, 20), 3, stream,
                                   settle_ms=SETTLE_MS)
                exact = bool(np.array_equal(oi.cpu().numpy(), want_idx) and
                             np.array_equal(oa.cpu().numpy(), want_act))
                t = ms * 1e-3
                res[name] = {"ms": ms, "mpps": n / t / 1e6, "rule_checks_per_s": checks / t,
                             "valu_frac": OPS_PER_CHECK * checks / t / 1e12 / VALU_INT32_PEAK_TOPS,
                             "hbm_gbs": n * BYTES_PER_PACKET / t / 1e9, "bit_exact": exact}
                log_fn(f"  {wl} {name}: {ms:.4f} ms, {n / t / 1e6:.0f} Mpps, exact={exact}")
        out[wl] = res
    return out


def multichain_leg(seed: int, steps: int, log_fn):
    """64 independent chains (32..8,192 rules, 4,096..1,048,576 packets, log-uniform) in one
    persistent launch, autotuned, against one packet-split launch per chain; then the same
    chains with a learned index each (the default placement routes them through the learned
    lookup), autotuned again.  Every configuration's time, the tuned launch's run-to-run
    spread, and every chain against the oracle in both phases."""
    import torch
    import oracle
    from synth import gen
    from paper_1312_4188_amd import fw
    work = gen.multichain_workload(seed=seed)
    items, rss = [], []
    for rules, pk in work:
        rs = fw.Ruleset(rules)
        rss.append(rs)
        n = len(pk)
        items.append((rs, fw.DevicePackets.from_host(pk),
                      torch.empty(n, dtype=torch.int32, device="cuda"),
                      torch.empty(n, dtype=torch.uint8, device="cuda")))
    total = sum(len(it[1]) for it in items)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    threads = max(1, min(16, os.cpu_count() or 1))
    want = [oracle.classify(r, p, threads=threads) for r, p in work]
    # the scan's algorithmic work: first-match index + 1 per packet, else the chain's length
    checks = int(sum(np.where(w[0] < 0, len(r), w[0].astype(np.int64) + 1).sum()
                     for w, (r, _) in zip(want, work)))
    out = {"chains": len(items), "packets": total,
           "rules_total": int(sum(len(r) for r, _ in work)), "rule_checks": checks}

    call = fw.MultiBatch(items)        # marshalled once: the timed calls are the library's

    def phase(name, variants):
        best, tuned_ms = fw.autotune_multi(items)
        log_fn(f"  multichain {name}: autotuned {best} ({tuned_ms:.3f} ms)")
        res = {"tuned": best, "autotune_best_ms": tuned_ms, "configs": {}}
        for cname, kw in variants.items():
            ms, _ = time_steps(lambda: call.run(stream=stream, **kw), steps, 2, stream,
                               settle_ms=SETTLE_MS)
            res["configs"][cname] = {"ms": ms, "mpps": total / ms / 1e3}
            if name == "scan":
                res["configs"][cname]["rule_checks_per_s"] = checks / (ms * 1e-3)
                res["configs"][cname]["valu_frac"] = (checks * OPS_PER_CHECK / (ms * 1e-3)
                                                      / 1e12 / VALU_INT32_PEAK_TOPS)
        reps = sorted([res["configs"]["tuned"]["ms"]] +
                      [time_steps(lambda: call.run(stream=stream), steps, 1, stream,
                                  settle_ms=SETTLE_MS)[0]
                       for _ in range(5)])
        res["tuned_ms_spread"] = {"min": reps[0], "median": reps[len(reps) // 2],
                                  "max": reps[-1], "runs": len(reps)}
        log_fn(f"  multichain {name} tuned: {reps[0]:.3f} / {reps[len(reps) // 2]:.3f} / "
               f"{reps[-1]:.3f} ms (min / median / max of {len(reps)} runs)")
        torch.cuda.synchronize()
        res["bit_exact"] = bool(all(
            np.array_equal(it[2].cpu().numpy(), w[0]) and np.array_equal(it[3].cpu().numpy(), w[1])
            for it, w in zip(items, want)))
        log_fn(f"  multichain {name}: every chain bit-exact vs the oracle: {res['bit_exact']}")
        return res

    variants = {"tuned": {}}
    for K in (1, 2, 4):
        variants[f"plan_k{K}"] = dict(packets_per_lane=K, placement=4)
        variants[f"scalar_k{K}"] = dict(packets_per_lane=K, placement=1)
        variants[f"vector_k{K}"] = dict(packets_per_lane=K, placement=3)
        variants[f"lds1024_k{K}"] = dict(packets_per_lane=K, placement=2, rule_tile=1024)
    out["scan"] = phase("scan", variants)

    def per_chain():
        for rs, dp, oi, oa in items:
            rs.classify(dp, mode="packet_split", stream=stream, out_idx=oi, out_act=oa)
    ms, _ = time_steps(per_chain, steps, 2, stream, settle_ms=SETTLE_MS)
    out["scan"]["configs"]["one_launch_per_chain"] = {
        "ms": ms, "mpps": total / ms / 1e3, "rule_checks_per_s": checks / (ms * 1e-3),
        "valu_frac": checks * OPS_PER_CHECK / (ms * 1e-3) / 1e12 / VALU_INT32_PEAK_TOPS}
    tuned = out["scan"]["configs"]["tuned"]
    log_fn(f"  multichain scan: {checks} rule checks, tuned {tuned['rule_checks_per_s'] / 1e12:.2f} "
           f"T checks/s, {tuned['valu_frac']:.3f} of the VALU peak at {OPS_PER_CHECK} ops per check")

    t0 = time.perf_counter()
    for k, rs in enumerate(rss):
        rs.build_learned_index(seed=seed + k)
    out["index_build_s"] = time.perf_counter() - t0
    out["learned"] = phase("learned", {"tuned": {}, **{f"plan_k{K}": dict(packets_per_lane=K,
                                                                          placement=4)
                                                       for K in (1, 2, 4)}})

    def per_chain_learned():
        for rs, dp, oi, oa in items:
            rs.classify(dp, mode="learned", stream=stream, out_idx=oi, out_act=oa)
    ms, _ = time_steps(per_chain_learned, steps, 2, stream, settle_ms=SETTLE_MS)
    out["learned"]["configs"]["one_launch_per_chain"] = {"ms": ms, "mpps": total / ms / 1e3}
    for rs in rss:
        rs.close()
    return out


def network_gain_leg(seed: int, steps: int, n_packets: int, log_fn):
    """What the trained network gains (trained / untrained network / no network / plain scan)
    on indexes of other sizes than the headline's: the 50,000-rule serving chain as generated
    (it reaches a rule matching every packet early, so its index is small) and the same
    chain with every rule's destination specified (no such rule: the boundary array, tens
    of thousands of entries, is searched in global memory).  Per variant: mean window,
    interval lookup ns per key, end-to-end Mpps; every variant's output equals the plain
    scan's on the whole batch and the oracle's on a 200,000-packet sample."""
    import torch
    import oracle
    from synth import gen
    from paper_1312_4188_amd import fw
    out = {}
    stream = torch.cuda.current_stream()
    for name, all_dst in (("50000_rules_as_generated", False),
                          ("50000_rules_every_destination", True)):
        rules = gen.serving_chains(seed)[2]
        if all_dst:
            rules.dst_plen[rules.dst_plen == 0] = 16
        pk = gen.make_packets(rules, n_packets, seed)
        n = len(pk)
        rng = np.random.Generator(np.random.PCG64(seed + 5))
        sample = np.sort(rng.choice(n, min(n, 200_000), replace=False))
        want = oracle.classify(rules, pk.subset(sample), threads=max(1, min(16, os.cpu_count() or 1)))
        dp = fw.DevicePackets.from_host(pk)
        oi = torch.empty(n, dtype=torch.int32, device="cuda")
        oa = torch.empty(n, dtype=torch.uint8, device="cuda")
        res = {"rules": len(rules), "packets": n}
        with fw.Ruleset(rules) as rs, fw.Ruleset(rules) as rs_un:
            st = rs.build_learned_index(seed=seed)
            st_un = rs_un.build_learned_index(seed=seed, train=False)
            M = st["n_boundaries"]
            res["boundaries"] = M
            res["boundaries_in_lds"] = M * 4 <= 80 * 1024
            ms_scan, _ = time_steps(lambda: rs.classify(dp, mode="packet_split", stream=stream,
                                                        out_idx=oi, out_act=oa), steps, 2, stream,
                                    settle_ms=SETTLE_MS)
            ref = (oi.cpu().numpy(), oa.cpu().numpy())
            exact = bool(np.array_equal(ref[0][sample], want[0]) and
                         np.array_equal(ref[1][sample], want[1]))
            res["scan"] = {"mpps": n / ms_scan / 1e3, "bit_exact": exact}
            for vname, ruleset, lookup, stats in (("trained", rs, 0, st),
                                                  ("untrained", rs_un, 0, st_un),
                                                  ("no_network", rs, 1, st)):
                ms, _ = time_steps(lambda: ruleset.classify(dp, mode="learned", lookup=lookup,
                                                            stream=stream, out_idx=oi, out_act=oa),
                                   steps, 2, stream, settle_ms=SETTLE_MS)
                same = bool(np.array_equal(oi.cpu().numpy(), ref[0]) and
                            np.array_equal(oa.cpu().numpy(), ref[1]))
                ms_l, _ = time_steps(lambda: ruleset.lookup_intervals(dp.dst_ip, lookup=lookup,
                                                                      stream=stream),
                                     steps, 2, stream)
                res[vname] = {"mean_window": (2 * stats["err_mean"] + 1) if lookup == 0 else M,
                              "lookup_ns_per_packet": ms_l * 1e6 / n, "mpps": n / ms / 1e3,
                              "bit_exact": bool(same and exact)}
                log_fn(f"  gain {name} {vname}: window {res[vname]['mean_window']:.1f}, "
                       f"lookup {ms_l * 1e6 / n:.4f} ns/key, {n / ms / 1e3:.0f} Mpps, "
                       f"exact {res[vname]['bit_exact']}")
            log_fn(f"  gain {name} scan: {n / ms_scan / 1e3:.0f} Mpps (|B| = {M})")
        out[name] = res
    return out


def host_cpu_model() -> str:
    """The host's CPU model name, as the kernel reports it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_peak_gbs(torch, stream, reps: int = 10) -> float:
    """Measured HBM ceiling: a plain 256 MiB device-to-device copy (bytes read plus bytes
    written per copy), median over `reps` event-timed copies on `stream`."""
    a = torch.empty(64 << 20, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    times = []
    with torch.cuda.stream(stream):
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.copy_(a)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
    times.sort()
    return 2 * a.numel() * 4 / times[len(times) // 2] / 1e9


def cpu_baseline(rules, pk, n_sample: int, n_single: int = 1_048_576):
    """The CPU oracle, as it stands, on a bounded sample of the same batch: with up to 16
    worker threads (the headline figure), and on one core over a smaller sample.  Returns the
    report and the oracle's (rule index, action) for the first n_sample packets, which the
    caller compares with the GPU's output."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    n_sample = min(n_sample, len(pk))
    sub = pk.subset(slice(0, n_sample))
    t0, c0 = time.perf_counter(), time.process_time()
    want = oracle.classify(rules, sub, threads=threads)
    dt, cpu = time.perf_counter() - t0, time.process_time() - c0
    n_single = min(n_single, len(pk))
    t1 = time.perf_counter()
    oracle.classify(rules, pk.subset(slice(0, n_single)), threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": n_sample / dt / 1e6, "unit": "Mpps", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sample} packets of the timed batch, {threads} threads, "
                      f"{dt:.2f} s wall, {cpu:.1f} s CPU",
            "single_core": {"value": n_single / dt1 / 1e6, "unit": "Mpps",
                            "sample": f"first {n_single} packets, 1 thread, {dt1:.2f} s"},
            "host": {"cpu": host_cpu_model(), "logical_cpus": os.cpu_count()}}, want


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=300,
                    help="untimed steps before each timed mode: the GPU reaches its steady "
                         "clocks after about 20 ms of sustained work (with 3, the headline's "
                         "timed steps ran about 13%% slower)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", default="learned_10000x16M")
    ap.add_argument("--latency-batches", type=int, default=2000)
    ap.add_argument("--cpu-sample", type=int, default=16_777_216)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--modes", default="",
                    help="comma list of modes to time (default: all); the first is the headline")
    ap.add_argument("--serving-requests", type=int, default=600,
                    help="requests per offered load in the serving leg (0 = skip it)")
    ap.add_argument("--no-multichain", action="store_true", help="skip the 64-chain leg")
    ap.add_argument("--no-gain", action="store_true",
                    help="skip the network-gain leg on the 50,000-rule indexes")
    ap.add_argument("--no-scan-configs", action="store_true",
                    help="skip the 100x10k and 1000x1M plain-scan leg")
    ap.add_argument("--no-ingest", action="store_true",
                    help="skip the PCIe-inclusive leg (whole batch from pinned host memory)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for scaling HBM counters)")
    ap.add_argument("--probe-batch", type=int, default=0,
                    help="profiling aid: classify the first N packets 25 times in each scan mode "
                         "named by --modes (packet_split, rule_split_p16, rule_split_p64, "
                         "hybrid_p16), print a short JSON line and exit")
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
    if args.probe_batch:
        table = {"packet_split": dict(mode="packet_split"),
                 "rule_split_p16": dict(mode="rule_split", partitions=16),
                 "rule_split_p64": dict(mode="rule_split", partitions=64),
                 "hybrid_p16": dict(mode="hybrid", partitions=16)}
        names = args.modes.split(",") if args.modes else list(table)
        sub = dp.slice(0, min(args.probe_batch, n))
        for name in names:
            for _ in range(25):
                rs.classify(sub, stream=stream, out_idx=out_i, out_act=out_a, **table[name])
            torch.cuda.synchronize()
            log(f"probe {name}: 25 calls of {len(sub)} packets")
        rs.close()
        print(json.dumps({"probe_batch": len(sub), "modes": names, "workload": args.workload}),
              flush=True)
        return
    log("building the learned index (trained)")
    t0 = time.perf_counter()
    index_stats = rs.build_learned_index(seed=args.seed)
    index_stats["build_s"] = time.perf_counter() - t0
    rs_plain = fw.Ruleset(rules)          # no index: mode AUTO picks a scan form by batch size
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
             "hybrid_p16": (rs, dict(mode="hybrid", partitions=16)),
             "auto_no_index": (rs_plain, dict(mode="auto"))}
    if args.modes:
        keep = args.modes.split(",")
        unknown = [k for k in keep if k not in modes]
        if unknown:
            raise SystemExit(f"unknown mode(s) {', '.join(unknown)}; known: {', '.join(modes)}")
        modes = {k: modes[k] for k in keep}
    results = {}
    ref = None
    ref_act = None
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
        del idx, act
        results[name] = {"ms": ms, "mpps": n / ms / 1e3, "same_as_learned": agree,
                         "wall_s": wall}
        if kw["mode"] == "learned":
            _, _, miss = ruleset.classify(dp, stream=stream, out_idx=out_i, out_act=out_a,
                                          count_misses=True, **kw)
            results[name]["window_misses"] = miss
        log(f"  {name}: {ms:.3f} ms/step, {n / ms / 1e3:.1f} Mpps")
    ref, ref_act = ref

    # what the trained network gains: window width, interval lookup alone, end to end
    gain = {}
    if "learned" in results:
        M = index_stats["n_boundaries"]
        variants = (("trained", rs, 0, index_stats, "learned"),
                    ("untrained", rs_un, 0, untrained_stats, "learned_untrained"),
                    ("no_network", rs, 1, index_stats, "learned_binary_search"))
        for name, ruleset, lookup, st, mode in variants:
            ms_l, _ = time_steps(lambda: ruleset.lookup_intervals(dp.dst_ip, lookup=lookup,
                                                                  stream=stream),
                                 args.steps, args.warmup, stream)
            gain[name] = {"mean_window": (2 * st["err_mean"] + 1) if lookup == 0 else M,
                          "lookup_ns_per_packet": ms_l * 1e6 / n,
                          "mpps": results.get(mode, {}).get("mpps")}
            log(f"  lookup {name}: {ms_l * 1e6 / n:.4f} ns/packet")
        gain["scan"] = {"mpps": results.get("packet_split", {}).get("mpps")}
    checks = int(np.where(ref < 0, R, ref.astype(np.int64) + 1).sum())
    for name in [m for m in ("packet_split", "rule_split_p16", "hybrid_p16") if m in results]:
        results[name]["rule_checks_per_s"] = checks / (results[name]["ms"] * 1e-3)
    full = ((rules.src_plen == 0) & (rules.dst_plen == 0) & (rules.proto_any != 0) &
            (rules.sport_lo == 0) & (rules.sport_hi == 65535) &
            (rules.dport_lo == 0) & (rules.dport_hi == 65535))
    k_star = int(np.argmax(full)) if full.any() else None   # first catch-all rule

    latency = {}
    for name in [m for m in ("learned", "packet_split", "rule_split_p16", "hybrid_p16",
                             "auto_no_index")
                 if m in modes and args.latency_batches > 0]:
        ruleset, kw = modes[name]
        log(f"latency {name}")
        latency[name] = closed_loop_latency(ruleset, dp, kw, args.seed, args.latency_batches,
                                            stream)

    head = next(iter(modes))
    ms = results[head]["ms"]
    copy_gbs = copy_peak_gbs(torch, stream)
    log(f"  device copy (256 MiB, median of 10): {copy_gbs:.0f} GB/s")
    traffic = committed_traffic(args.workload)
    counters = committed_valu_counters(args.workload)

    def alu_roofline(kernel, mode, work, profile_key):
        """VALU roofline of one timed mode: algorithmic lane-ops per step over its time; HBM
        from the committed counter traffic when it is current, else 18 B per packet."""
        t = results[mode]["ms"] * 1e-3
        tr = traffic.get(profile_key)
        hbm = tr if tr is not None else n * BYTES_PER_PACKET
        r = {"bound": "alu", "achieved": work["lane_ops"] / t / 1e12,
             "peak": VALU_INT32_PEAK_TOPS, "unit": "Tops/s",
             "frac": work["lane_ops"] / t / 1e12 / VALU_INT32_PEAK_TOPS,
             "traffic": tr, "kernel": kernel, "algorithmic_lane_ops": work["lane_ops"],
             "ops_per_check": OPS_PER_CHECK,
             "algorithmic_hbm_bytes": n * BYTES_PER_PACKET,
             "hbm_gbs": hbm / t / 1e9, "hbm_frac": hbm / t / 1e9 / HBM_PEAK_GBS,
             "hbm_copy_gbs": copy_gbs, "hbm_frac_of_copy": hbm / t / 1e9 / copy_gbs,
             "hbm_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE" if tr is not None
                           else "algorithmic, 18 B per packet"}
        if "candidate_checks" in work:
            # the fuller pricing of a candidate check: ~7 lane-ops (all field tests, select, step)
            ops7 = work["lane_ops"] + (OPS_PER_CHECK_FULL - OPS_PER_CHECK) * work["candidate_checks"]
            r["frac_at_7_ops_per_check"] = ops7 / t / 1e12 / VALU_INT32_PEAK_TOPS
            # records gathered from the per-lane lists: served by L2 and LDS, not HBM
            r["gather_bytes"] = work["list_checks"] * RECORD_BYTES
            r["gather_gbs"] = r["gather_bytes"] / t / 1e9
        ex = counters.get(profile_key)
        if ex:
            r["executed_lane_ops"] = ex
            r["useful_over_executed"] = work["lane_ops"] / ex
        return r

    roofline = roofline_bs = None
    if "learned" in results:
        work = learned_work(rs, pk, ref)
        roofline = alu_roofline("k_learned<true,2,false>", "learned", work, "k_learned")
    if "learned_binary_search" in results:
        work_bs = learned_work(rs, pk, ref, network=False)
        roofline_bs = alu_roofline("k_learned<true,2,false> (lookup=1)", "learned_binary_search",
                                   work_bs, "k_learned_binary_search")
    scan_roofline = None
    if "packet_split" in results:
        scan_roofline = alu_roofline("k_packet_split<4>", "packet_split",
                                     {"lane_ops": checks * OPS_PER_CHECK}, "k_packet_split")
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

    ingest = None
    if not args.no_ingest:
        log("ingest leg: whole batch from pinned host memory")
        ingest = ingest_leg(rs, pk, ref, 1 << 20, log)

    scan_configs = None
    if not args.no_scan_configs:
        log("plain-scan configurations")
        scan_configs = scan_configs_leg(args.seed, args.steps, log)

    multichain = None
    if not args.no_multichain:
        log("multi-chain leg")
        multichain = multichain_leg(args.seed, max(3, args.steps // 2), log)

    gain_configs = None
    if not args.no_gain:
        log("network gain on the 50,000-rule indexes")
        gain_configs = network_gain_leg(args.seed, max(3, args.steps // 2), 4_194_304, log)

    cpu = None
    oracle_exact, checked = None, 0
    if not args.no_cpu:
        log("cpu baseline (the oracle over the timed batch)")
        cpu, (want_i, want_a) = cpu_baseline(rules, pk, min(args.cpu_sample, n))
        checked = int(want_i.shape[0])
        # the timed output (every mode agreed with the first one) against the oracle
        oracle_exact = bool(np.array_equal(ref[:checked], want_i) and
                            np.array_equal(ref_act[:checked], want_a))
        for r in results.values():
            r["bit_exact"] = bool(r["same_as_learned"] and oracle_exact)
        log(f"  timed output vs the oracle over {checked} packets: bit-exact {oracle_exact}")
        del want_i, want_a

    line = {
        "metric": "Mpps (bit-exact first-match) at 10k rules: learned-index vs scan; p99 latency",
        "value": results[head]["mpps"], "unit": "Mpps", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded generators)",
        "config": {"workload": args.workload, "rules": R, "packets": n, "seed": args.seed,
                   "path": head, "k_star": k_star},
        "bit_exact": oracle_exact, "bit_exact_packets": checked,
        "scan_mpps": results["packet_split"]["mpps"] if "packet_split" in results else None,
        "speedup_vs_scan": (results["packet_split"]["ms"] / ms
                            if "packet_split" in results else None),
        "p99_us": latency.get(head, {}).get("p99_us"),
        "p50_us": latency.get(head, {}).get("p50_us"),
        "modes": results, "latency": latency,
        "scan_rule_checks": checks,
        "learned_candidate_checks": work["candidate_checks"] if roofline else None,
        "index": index_stats, "index_untrained": untrained_stats, "network_gain": gain,
        "network_gain_other_indexes": gain_configs,
        "roofline": roofline, "roofline_binary_search": roofline_bs,
        "scan_roofline": scan_roofline, "serving": serving,
        "multichain": multichain, "ingest": ingest, "scan_configs": scan_configs,
        "cpu_baseline": cpu,
    }
    rs.close()
    rs_un.close()
    rs_plain.close()
    for name, lat in latency.items():
        log(f"closed-loop latency {name}: p50 {lat['p50_us']:.1f} us, p99 {lat['p99_us']:.1f} us")
    if serving:
        for name, m in serving["modes"].items():
            by = {ld["offered_frac"]: ld for ld in m["loads"]}
            p = lambda f: by.get(f, {}).get("p99_us", float("nan"))
            log(f"serving {name}: peak {m['peak_mpps']:.0f} Mpps, bit-exact {m.get('bit_exact')}, "
                f"p99 at 70% / 100% / 120% load {p(0.7):.0f} / {p(1.0):.0f} / {p(1.2):.0f} us")
    log(f"headline {head}: {line['value']:.0f} Mpps, bit-exact vs oracle {oracle_exact} "
        f"({checked} packets)")
    print(json.dumps(line), flush=True)
    if oracle_exact is False:
        sys.exit("the timed output differs from the oracle")


if __name__ == "__main__":
    main()
