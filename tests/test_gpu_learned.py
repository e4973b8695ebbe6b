"""GPU tests of the learned destination index.

The index structure is checked against the oracle's set definitions
(oracle.intervals), the interval lookup against the textbook upper_bound,
classifications against the sequential oracle bit for bit, and the training
kernels' gradients and Adam step against the float64 reference
(oracle.rmi).
"""

import numpy as np
import pytest

import oracle
from oracle import intervals as iv
from oracle import rmi
from synth import gen
from tests.gpu_util import assert_same, fwmod, say

pytestmark = pytest.mark.gpu

FAST = dict(epochs1=300, epochs2=600)


def _check_half_rounding(rs, st, hidden=32):
    """The lookup stores each expert's w1 and w2 as IEEE half after scaling hidden unit
    (w1, b1, w2) to (w1 2^-k, b1 2^-k, w2 2^k) with 2^k > |w1| + |b1| (so ReLU becomes a
    clamp to [0, 1]); among the first 24 such k it takes the smallest that half rounds the
    fewest of (w2, and w1 when w2 is not zero).  Recomputed here from the exported bf16
    weights of the experts: the index's count must agree, and every weight half rounds must
    lie below half's normal range (2^-14), so none overflows and each moves by at most
    2^-25."""
    H, P = hidden, 3 * hidden + 1
    nets = rs.export(5).astype(np.float32).reshape(-1, P)[1:]   # the experts (stage 2)

    def exact(x):
        with np.errstate(over="ignore"):
            h = np.float16(x)
        return bool(np.isfinite(h)) and np.float32(h) == np.float32(x)

    count, worst = 0, 0.0
    for net in nets:
        for i in range(H):
            a, b, c = (np.float32(net[i]), np.float32(net[H + i]), np.float32(net[2 * H + i]))
            m = np.float32(abs(a) + abs(b))
            if not (m > 0) or not np.isfinite(m):
                continue
            k0 = int(np.frexp(m)[1])
            best = None
            for k in range(k0, k0 + 24):
                a2, b2, c2 = np.ldexp(a, -k), np.ldexp(b, -k), np.ldexp(c, k)
                if not (np.ldexp(a2, k) == a and np.ldexp(b2, k) == b and np.ldexp(c2, -k) == c
                        and np.isfinite(c2)
                        and all(x == 0 or abs(x) >= np.finfo(np.float32).tiny
                                for x in (a2, b2, c2))):
                    continue
                bad = [c2] if not exact(c2) else []
                if c2 != 0 and not exact(a2):
                    bad.append(a2)
                if best is None or len(bad) < len(best):
                    best = bad
                if not bad:
                    break
            if best is None:   # no scaling round-trips: the unit is stored unscaled
                best = [c] if not exact(c) else []
                if c != 0 and not exact(a):
                    best.append(a)
            for x in best:
                count += 1
                worst = max(worst, abs(float(x)))
    assert st["weights_rounded"] == count, (st["weights_rounded"], count)
    assert worst < 2.0 ** -14, worst


def _learned_np(rules, pk, build_kw=None, **kw):
    import torch
    fw = fwmod()
    with fw.Ruleset(rules) as rs:
        stats = rs.build_learned_index(**(build_kw or FAST))
        dp = fw.DevicePackets.from_host(pk)
        idx, act, miss = rs.classify(dp, mode="learned", count_misses=True, **kw)
        torch.cuda.synchronize()
        return (idx.cpu().numpy(), act.cpu().numpy()), miss, stats


@pytest.mark.parametrize("seed,skew,R", [(1, False, 100), (2, True, 300), (3, True, 1000)])
def test_index_structure_matches_definition(seed, skew, R):
    fw = fwmod()
    rules = gen.make_rules(R, seed, skew=skew)
    say(f"structure seed={seed} R={R}")
    with fw.Ruleset(rules) as rs:
        st = rs.build_learned_index(**FAST)
        B = rs.export(0)
        off = rs.export(1)
        L = rs.export(2)
        G = rs.export(3)
    want_B = iv.boundaries(rules)
    np.testing.assert_array_equal(B, want_B)
    assert st["n_boundaries"] == len(B)
    assert off[0] == 0 and off[-1] == len(L) and np.all(np.diff(off.astype(np.int64)) >= 0)
    C = iv.candidates(rules, want_B)
    full = iv.full_match_in_interval(rules)
    Gs = set(G.tolist())
    assert list(G) == sorted(G)
    for j in range(len(B)):
        U = Gs | set(L[off[j]:off[j + 1]].tolist())
        Cj = set(C[j].tolist())
        Tj = set(iv.truncated(C[j], full).tolist())
        assert Tj <= U <= Cj, j
        lj = L[off[j]:off[j + 1]]
        assert np.all(np.diff(lj.astype(np.int64)) > 0)


@pytest.mark.parametrize("lookup", [0, 1])
def test_interval_lookup_matches_upper_bound(lookup):
    import torch
    fw = fwmod()
    rules = gen.make_rules(2000, 4, skew=True)
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(**FAST)
        B = rs.export(0).astype(np.int64)
        rng = np.random.Generator(np.random.PCG64(4))
        probe = np.concatenate([B - 1, B, B + 1, rng.integers(0, 2**32, 50_000), [0, 2**32 - 1]])
        probe = probe[(probe >= 0) & (probe < 2**32)].astype(np.uint32)
        keys = torch.from_numpy(probe.view(np.int32)).cuda()
        say(f"interval lookup {lookup} n={len(probe)}")
        got = rs.lookup_intervals(keys, lookup=lookup)
        torch.cuda.synchronize()
        want = np.searchsorted(B, probe.astype(np.int64), side="right") - 1
        np.testing.assert_array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("wl,seed", [("scan_100x10k", 1), ("scan_100x10k", 2),
                                     ("scan_1000x1M", 1), ("scan_1000x1M", 3)])
def test_learned_classify_matches_oracle(wl, seed):
    rules, pk = gen.workload(wl, seed=seed)
    say(f"learned {wl} seed={seed}")
    want = oracle.classify(rules, pk, threads=16)
    for lookup, ppl in ((0, 0), (1, 0), (0, 1), (0, 4)):
        got, miss, st = _learned_np(rules, pk, lookup=lookup, packets_per_lane=ppl)
        assert_same(got, want, f"learned {wl} seed {seed} lookup {lookup} ppl {ppl}")
        if lookup == 1:
            assert miss == 0


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_learned_10000_rules_whole_batch(seed):
    """10,000 skewed rules x 16,777,216 packets, seeds 1-5: every packet of the batch against
    the oracle, through the learned index (network + window, and the full binary search) and
    the packet-split scan."""
    import torch
    fw = fwmod()
    rules, pk = gen.workload("learned_10000x16M", seed=seed)
    want = oracle.classify(rules, pk, threads=16)
    dp = fw.DevicePackets.from_host(pk)
    with fw.Ruleset(rules) as rs:
        say(f"learned 10000x16M seed={seed} build")
        st = rs.build_learned_index()
        say(f"  stats {st}")
        _check_half_rounding(rs, st)
        for lookup in (0, 1):
            idx, act, miss = rs.classify(dp, mode="learned", lookup=lookup, count_misses=True)
            torch.cuda.synchronize()
            assert_same((idx.cpu().numpy(), act.cpu().numpy()), want,
                        f"learned 10000x16M seed {seed} lookup {lookup}")
            say(f"  lookup {lookup}: window misses {miss} of {len(pk)}")
        si, sa = rs.classify(dp, mode="packet_split")
        torch.cuda.synchronize()
        assert_same((si.cpu().numpy(), sa.cpu().numpy()), want,
                    f"packet split 10000x16M seed {seed}")


@pytest.mark.parametrize("seed,all_dst", [(1, False), (2, False), (1, True)])
def test_learned_50000_rule_chain(seed, all_dst):
    """The largest resident serving chain (50,000 skewed rules) through its learned index and
    the scans, every packet of a 4,194,304-packet batch against the oracle, at the library's
    default and at 1 and 4 packets per lane.  As generated, the chain reaches a rule matching
    every packet early, so its index is small; with every rule's destination specified
    (all_dst) there is none, and the boundary array (about 75,000 entries) is searched in
    global memory."""
    import torch
    fw = fwmod()
    rules = gen.serving_chains(seed)[2]
    assert len(rules) == 50_000
    if all_dst:
        rules.dst_plen[rules.dst_plen == 0] = 16
    pk = gen.make_packets(rules, 4_194_304, seed)
    want = oracle.classify(rules, pk, threads=16)
    dp = fw.DevicePackets.from_host(pk)
    with fw.Ruleset(rules) as rs:
        say(f"learned 50000-rule chain seed={seed} all_dst={all_dst} build")
        st = rs.build_learned_index(seed=seed)
        say(f"  stats {st}")
        _check_half_rounding(rs, st)
        if all_dst:
            assert st["n_boundaries"] * 4 > 80 * 1024
        for kw in (dict(), dict(packets_per_lane=1), dict(packets_per_lane=4),
                   dict(lookup=1)):
            say(f"  learned {kw}")
            idx, act = rs.classify(dp, mode="learned", **kw)[:2]
            torch.cuda.synchronize()
            assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, f"learned 50k {kw}")
        for mode in ("packet_split", "hybrid"):
            say(f"  {mode}")
            si, sa = rs.classify(dp, mode=mode)[:2]
            torch.cuda.synchronize()
            assert_same((si.cpu().numpy(), sa.cpu().numpy()), want, f"{mode} 50k")


@pytest.mark.parametrize("n", [1, 63, 65, 1000, 4097])
def test_learned_ragged_and_edge_rulesets(n):
    for R, seed in ((0, 1), (1, 2), (7, 3), (300, 4)):
        rules = gen.make_rules(R, seed, skew=True)
        pk = gen.make_packets(gen.make_rules(20, seed + 50), n, seed)
        say(f"learned ragged n={n} R={R}")
        want = oracle.classify(rules, pk)
        for ppl in (1, 2, 4):
            got, _, _ = _learned_np(rules, pk, packets_per_lane=ppl)
            assert_same(got, want, f"learned n={n} R={R} ppl={ppl}")


def test_forced_window_miss_stays_exact():
    """Error bounds forced to 0, and an untrained network: every answer still exact."""
    rules, pk = gen.workload("scan_1000x1M", seed=5, n_packets=200_000)
    want = oracle.classify(rules, pk, threads=16)
    got, miss, st = _learned_np(rules, pk, build_kw=dict(FAST, zero_error_bounds=True))
    assert_same(got, want, "zero error bounds")
    assert st["err_max"] == 0 and miss > len(pk) // 4
    got, miss2, st2 = _learned_np(rules, pk, build_kw=dict(FAST, train=False))
    assert_same(got, want, "untrained network")


def test_small_network_shapes():
    """Fewer hidden units and experts than the defaults (padded inference layout)."""
    rules, pk = gen.workload("scan_1000x1M", seed=2, n_packets=100_000)
    want = oracle.classify(rules, pk, threads=16)
    for hidden, experts in ((7, 5), (1, 1), (32, 200)):
        say(f"learned hidden={hidden} experts={experts}")
        got, _, st = _learned_np(rules, pk, build_kw=dict(FAST, hidden=hidden, experts=experts))
        assert_same(got, want, f"hidden={hidden} experts={experts}")


def test_network_gain():
    """What training buys: narrower windows than the untrained network and than a full search."""
    fw = fwmod()
    rules = gen.make_rules(10_000, 1, skew=True)
    with fw.Ruleset(rules) as rs:
        tr = rs.build_learned_index(seed=3)
        un = rs.build_learned_index(seed=3, train=False)
    M = tr["n_boundaries"]
    say(f"gain: trained err mean {tr['err_mean']:.1f} max {tr['err_max']}; "
        f"untrained mean {un['err_mean']:.1f} max {un['err_max']}; M = {M}")
    assert tr["err_mean"] * 4 < un["err_mean"]
    # binary-search steps in the mean window against a search over all M boundaries
    assert np.log2(2 * tr["err_mean"] + 1) < 0.6 * np.log2(M)


@pytest.mark.parametrize("E,H,n", [(1, 32, 1000), (3, 7, 777), (64, 32, 5000), (5, 32, 0)])
@pytest.mark.parametrize("mfma", [False, True])
def test_gradients_match_float64(E, H, n, mfma):
    fw = fwmod()
    rng = np.random.Generator(np.random.PCG64(E * 100 + H))
    params = rng.normal(0, 1, (E, 3 * H + 1)).astype(np.float32)
    u = rng.random(n).astype(np.float32)
    t = rng.random(n).astype(np.float32)
    ex = rng.integers(0, E, n).astype(np.uint32)
    if E == 64:
        ex[ex == 7] = 8               # an expert with no samples
    say(f"gradients E={E} H={H} n={n} mfma={mfma}")
    g, loss = fw.rmi_gradients(params, u, t, ex, H, use_mfma=mfma)
    want = rmi.stage_grad(params.astype(np.float64), u, t, ex, H)
    scale = max(np.max(np.abs(want)), 1e-30)
    tol = 2e-2 if mfma else 1e-4
    assert np.max(np.abs(g - want)) / scale <= tol
    want_loss = np.array([rmi.loss(params[e].astype(np.float64), u[ex == e], t[ex == e], H)
                          for e in range(E)])
    np.testing.assert_allclose(loss, want_loss, rtol=tol, atol=1e-6)
    if E == 64:
        assert np.all(g[7] == 0)


def test_adam_step_matches_float64():
    fw = fwmod()
    rng = np.random.Generator(np.random.PCG64(8))
    p = rng.normal(size=500)
    g = rng.normal(size=500)
    m = rng.normal(size=500) * 0.1
    v = rng.random(500) * 0.1
    for step in (1, 2, 50):
        got = fw.rmi_adam_step(p, g, m, v, step, 0.01)
        want = rmi.adam(p, g, m, v, step, 0.01)
        for a, b in zip(got, want):
            np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6)


def test_memory_budget_leaves_scan_usable():
    import torch
    fw = fwmod()
    rules, pk = gen.workload("scan_100x10k", seed=6)
    want = oracle.classify(rules, pk)
    dp = fw.DevicePackets.from_host(pk)
    with fw.Ruleset(rules) as rs:
        with pytest.raises(fw.FwError) as ei:
            rs.build_learned_index(mem_budget=1024)
        assert ei.value.status == fw.E_NOMEM
        with pytest.raises(fw.FwError) as ei:
            rs.classify(dp, mode="learned")
        assert ei.value.status == fw.E_NOINDEX
        idx, act = rs.classify(dp)          # AUTO falls back to the scan
        torch.cuda.synchronize()
        assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, "auto after failed build")


@pytest.mark.parametrize("seed,R", [(2, 300), (3, 1000), (1, 10_000)])
def test_source_lists_match_definition(seed, R):
    """The destination-wildcard candidates, split by source: for every source interval i of
    those that specify a source, the entries of S_i together with the fully wildcard list
    Gw hold every candidate reachable for a packet whose source lies in interval i."""
    fw = fwmod()
    rules = gen.make_rules(R, seed, skew=True)
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(**FAST)
        G = rs.export(3)
        Bs, soff, S, Gw = rs.export(6), rs.export(7), rs.export(8), rs.export(9)
    wild_src = rules.src_plen[G] == 0
    np.testing.assert_array_equal(Gw, G[wild_src])
    sub = rules.subset(G[~wild_src])
    np.testing.assert_array_equal(Bs, iv.boundaries(sub, "src"))
    C = iv.candidates(sub, Bs, "src")
    # within a source interval every candidate's source test passes: it matches every
    # packet there once ports and protocol are unspecified
    full = ((sub.sport_lo == 0) & (sub.sport_hi == 65535) & (sub.dport_lo == 0)
            & (sub.dport_hi == 65535) & (sub.proto_any != 0))
    mapped = G[~wild_src]
    for i in range(len(Bs)):
        got = S[soff[i]:soff[i + 1]]
        want = mapped[iv.truncated(C[i], full)]
        assert set(want.tolist()) <= set(got.tolist()) <= set(mapped[C[i]].tolist()), i
        assert np.all(np.diff(got.astype(np.int64)) > 0)


_PT_DTYPE = np.dtype([("mask_p", "<u8", 256), ("mask_s", "<u8", 130), ("mask_d", "<u8", 130),
                      ("b_s", "<u4", 132), ("b_d", "<u4", 132), ("rule", "<u4", 68),
                      ("bucket_s", "u1", 256), ("bucket_d", "u1", 256)])


def _address_wildcard_heavy(R, seed, frac):
    """Random rules with a fraction made address-wildcard (both prefixes /0); those are kept
    from being catch-alls so the wildcard list stays long."""
    rules = gen.make_rules(R, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 99))
    pick = rng.random(R) < frac
    rules.src_plen[pick] = 0
    rules.dst_plen[pick] = 0
    catch = (pick & (rules.sport_lo == 0) & (rules.sport_hi == 65535) & (rules.dport_lo == 0)
             & (rules.dport_hi == 65535) & (rules.proto_any != 0))
    rules.proto_any[catch] = 0
    rules.proto[catch] = 6
    return rules


def _wildcard_list(rules):
    """Address-wildcard rules up to and including the first catch-all (definition)."""
    wild = (rules.src_plen == 0) & (rules.dst_plen == 0)
    catch = (wild & (rules.sport_lo == 0) & (rules.sport_hi == 65535) & (rules.dport_lo == 0)
             & (rules.dport_hi == 65535) & (rules.proto_any != 0))
    idx = np.nonzero(wild)[0]
    if catch.any():
        idx = idx[idx <= np.argmax(catch)]
    return idx, catch


@pytest.mark.parametrize("seed,R,frac", [(1, 10000, 0.0), (4, 600, 0.3), (5, 300, 1.0),
                                         (6, 40, 0.5)])
def test_port_table_matches_definition(seed, R, frac):
    """The port/protocol table of the first 64 address-wildcard candidates against the
    oracle's masks, and the high-byte walk against the interval of every port value."""
    fw = fwmod()
    rules = (gen.make_rules(R, seed, skew=True) if frac == 0.0
             else _address_wildcard_heavy(R, seed, frac))
    say(f"port table seed={seed} R={R} frac={frac}")
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(**FAST)
        Gw, raw, shape = rs.export(9), rs.export(10), rs.export(11)
    gw_def, catch = _wildcard_list(rules)
    np.testing.assert_array_equal(Gw, gw_def)
    sel = np.array([r for r in gw_def if not catch[r]][:64], dtype=np.int64)
    t = np.frombuffer(raw.tobytes(), dtype=_PT_DTYPE, count=1)[0]
    assert int(shape[0]) == len(sel)
    want_rule = [int(r) | (int(rules.action[r]) << 24) for r in sel]
    assert [int(x) for x in t["rule"][:len(sel)]] == want_rule
    assert np.all(t["rule"][len(sel):] == 0xFFFFFFFF)
    assert [int(x) for x in t["mask_p"]] == iv.proto_masks(rules.proto[sel], rules.proto_any[sel])
    ports = np.arange(65536, dtype=np.int64)
    for name, lo, hi, steps in (("s", rules.sport_lo[sel], rules.sport_hi[sel], int(shape[1])),
                                ("d", rules.dport_lo[sel], rules.dport_hi[sel], int(shape[2]))):
        B, masks = iv.port_masks(lo, hi) if len(sel) else (np.zeros(1, np.int64), [0])
        b = t[f"b_{name}"].astype(np.int64)
        np.testing.assert_array_equal(b[:len(B)], B)
        assert np.all(b[len(B):] == 0x10000)
        assert [int(x) for x in t[f"mask_{name}"][:len(B)]] == masks
        # the kernel's walk: high-byte table, then `steps` forward steps
        i = t[f"bucket_{name}"].astype(np.int64)[ports >> 8]
        for _ in range(steps):
            i = i + (b[i + 1] <= ports)
        np.testing.assert_array_equal(i, np.searchsorted(B, ports, side="right") - 1)


@pytest.mark.parametrize("seed,R,frac", [(7, 400, 0.5), (8, 1500, 0.2), (9, 64, 1.0),
                                         (10, 65, 1.0)])
def test_learned_with_many_address_wildcard_rules(seed, R, frac):
    """Long address-wildcard lists: more than 64 such candidates put the rest on the grouped
    scan after the port/protocol table.  Every packet against the oracle."""
    rules = _address_wildcard_heavy(R, seed, frac)
    pk = gen.make_packets(rules, 50_000, seed)
    say(f"learned, address-wildcard heavy seed={seed} R={R} frac={frac}")
    want = oracle.classify(rules, pk)
    for ppl in (1, 2, 4):
        got, _, _ = _learned_np(rules, pk, packets_per_lane=ppl)
        assert_same(got, want, f"seed={seed} R={R} K={ppl}")


@pytest.mark.parametrize("seed,R", [(1, 10000), (2, 3000), (3, 200)])
def test_source_bucket_table(seed, R):
    """The source-address bucket table plus its walk gives the interval of every key the
    textbook upper_bound gives: at every boundary and its neighbours, at every bucket start,
    and at random keys."""
    fw = fwmod()
    rules = gen.make_rules(R, seed, skew=True)
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(**FAST)
        Bs, shape, table = rs.export(6), rs.export(11), rs.export(12)
    bits, steps = int(shape[3]), int(shape[4])
    if bits == 0:
        assert table.size == 0
        return
    assert table.size == 1 << bits and steps <= 8
    B = Bs.astype(np.int64)
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.unique(np.concatenate([B, B - 1, B + 1, np.arange(1 << bits) << (32 - bits),
                                     rng.integers(0, 1 << 32, 100_000), [0, (1 << 32) - 1]]))
    keys = keys[(keys >= 0) & (keys < (1 << 32))]
    i = table.astype(np.int64)[keys >> (32 - bits)]
    for _ in range(steps):
        nxt = np.minimum(i + 1, len(B) - 1)
        i = i + ((i + 1 < len(B)) & (B[nxt] <= keys))
    np.testing.assert_array_equal(i, np.searchsorted(B, keys, side="right") - 1)


def test_large_index_global_boundaries():
    """A destination index too large for LDS (about 45,000 boundaries): the kernels search the
    boundary array in global memory.  Every packet against the oracle, at 1, 2 and 4 packets
    per lane."""
    rules = gen.make_rules(30_000, 12, skew=True)
    rules.dst_plen[rules.dst_plen == 0] = 24          # every rule specifies a destination
    pk = gen.make_packets(rules, 200_000, 12)
    say("learned, 30000 rules with specified destinations (boundaries in global memory)")
    want = oracle.classify(rules, pk, threads=16)
    for ppl in (1, 2, 4):
        got, miss, st = _learned_np(rules, pk, packets_per_lane=ppl)
        assert st["n_boundaries"] * 4 > 80 * 1024
        assert_same(got, want, f"large index K={ppl}")


def test_source_bucket_fallback_to_binary_search():
    """Source prefixes crowded into one bucket of the top-bits table (more than 8 boundaries
    in one /12) make the index fall back to a binary search over source intervals."""
    rules = gen.make_rules(400, 13)
    rng = np.random.Generator(np.random.PCG64(13))
    pick = np.arange(0, 400, 10)                       # 40 destination-wildcard rules
    rules.dst_plen[pick] = 0
    rules.src_plen[pick] = 32
    rules.src_ip[pick] = (0x0A000000 + rng.integers(0, 1 << 20, len(pick))).astype(np.uint32)
    pk = gen.make_packets(rules, 50_000, 13)
    fw = fwmod()
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(**FAST)
        shape = rs.export(11)
    assert int(shape[3]) == 0, "expected no bucket table"
    want = oracle.classify(rules, pk)
    for ppl in (1, 2, 4):
        got, _, _ = _learned_np(rules, pk, packets_per_lane=ppl)
        assert_same(got, want, f"binary-search sources K={ppl}")


def test_long_candidate_lists():
    """Wide destination prefixes with specified sources: few intervals (the boundary arrays
    fit in LDS easily), but every interval's list is long, more than 65,535 records in all.
    Every packet against the oracle at 1, 2 and 4 packets per lane."""
    rng = np.random.Generator(np.random.PCG64(14))
    rules = gen.make_rules(4000, 14)
    rules.dst_plen[:] = rng.integers(1, 9, 4000).astype(np.uint8)
    rules.src_plen[:] = rng.integers(16, 25, 4000).astype(np.uint8)
    pk = gen.make_packets(rules, 100_000, 14)
    fw = fwmod()
    with fw.Ruleset(rules) as rs:
        st = rs.build_learned_index(**FAST)
        n_list = int(rs.export(1)[-1])
    say(f"long lists: {n_list} records, {st['n_boundaries']} boundaries")
    assert n_list > 0xFFFF and st["n_boundaries"] * 4 < 16 * 1024
    want = oracle.classify(rules, pk, threads=16)
    for ppl in (1, 2, 4):
        got, _, _ = _learned_np(rules, pk, packets_per_lane=ppl)
        assert_same(got, want, f"long lists K={ppl}")


def test_positions_identical_across_packets_per_lane():
    """190 experts on a small ruleset, one index classified with 1, 2 and 4 packets per lane
    (different kernels and LDS budgets).  With error bounds forced to zero every window miss
    depends on the exact predicted position, so equal miss counts show that all of them
    predict alike; every answer against the oracle."""
    import torch
    rules = gen.make_rules(200, 15, skew=True)
    pk = gen.make_packets(rules, 60_000, 15)
    want = oracle.classify(rules, pk)
    fw = fwmod()
    misses = {}
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(**dict(FAST, experts=190, zero_error_bounds=True))
        dp = fw.DevicePackets.from_host(pk)
        for ppl in (1, 2, 4):
            say(f"row formats K={ppl}")
            idx, act, misses[ppl] = rs.classify(dp, mode="learned", count_misses=True,
                                                packets_per_lane=ppl)
            torch.cuda.synchronize()
            assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, f"190 experts K={ppl}")
    assert misses[1] == misses[2] == misses[4] > 0


def test_rebuild_waits_for_work_in_flight():
    """A classification still running on another stream when the index is rebuilt: the
    rebuild waits for it before freeing the old index, so its results stay exact."""
    import torch
    rules, pk = gen.workload("scan_1000x1M", seed=16, n_packets=2_000_000)
    sample = np.arange(0, len(pk), 97)
    want = oracle.classify(rules, pk.subset(sample), threads=16)
    fw = fwmod()
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(**FAST)
        dp = fw.DevicePackets.from_host(pk)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())     # the packets' upload
        say("classify on a side stream, then rebuild the index at once")
        idx, act = rs.classify(dp, mode="learned", stream=side)[:2]
        rs.build_learned_index(**dict(FAST, seed=2))
        side.synchronize()
        assert_same((idx.cpu().numpy()[sample], act.cpu().numpy()[sample]), want,
                    "classified while the index was rebuilt")
        again = rs.classify(dp, mode="learned")[:2]
        torch.cuda.synchronize()
        assert np.array_equal(again[0].cpu().numpy(), idx.cpu().numpy())
