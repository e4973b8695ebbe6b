"""GPU parity of the scan modes against the CPU oracle, bit for bit.

Packet split (paper Section IV-A), rule split (Section IV-B) and the hybrid
(Section IV-C) must all give exactly the oracle's first-match index and
action for every packet.
"""

import numpy as np
import pytest

import oracle
from synth import gen
from tests import golden_io
from tests.gpu_util import assert_same, classify_np, fwmod, say

pytestmark = pytest.mark.gpu

SCAN_MODES = [
    dict(mode="packet_split", packets_per_lane=4),
    dict(mode="packet_split", packets_per_lane=2),
    dict(mode="packet_split", packets_per_lane=1),
    dict(mode="rule_split", partitions=16),
    dict(mode="rule_split", partitions=1),
    dict(mode="rule_split", partitions=3),
    dict(mode="rule_split", partitions=64),
    dict(mode="rule_split", partitions=100),
    dict(mode="hybrid", partitions=4),
    dict(mode="hybrid", partitions=16),
    dict(mode="hybrid", partitions=4, packets_per_lane=2),
    dict(mode="hybrid", partitions=16, packets_per_lane=4),
]


def _id(kw):
    return "-".join(f"{v}" for v in kw.values())


@pytest.mark.parametrize("kw", SCAN_MODES, ids=_id)
@pytest.mark.parametrize("name", golden_io.names())
def test_golden(name, kw):
    say(f"golden {name} {kw}")
    rs, pk, ei, ea = golden_io.load(name)
    assert_same(classify_np(rs, pk, **kw), (ei, ea), f"{name} {kw}")


@pytest.mark.parametrize("kw", SCAN_MODES, ids=_id)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_small_config_all_modes(seed, kw):
    """100 rules x 10,000 packets (every packet checked)."""
    say(f"scan_100x10k seed={seed} {kw}")
    rules, pk = gen.workload("scan_100x10k", seed=seed)
    want = oracle.classify(rules, pk, threads=8)
    assert_same(classify_np(rules, pk, **kw), want, f"seed {seed} {kw}")


@pytest.mark.parametrize("kw", [dict(mode="packet_split"), dict(mode="rule_split", partitions=16),
                                dict(mode="rule_split", partitions=1000),
                                dict(mode="hybrid", partitions=8)], ids=_id)
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_1000_rules_full_batch(seed, kw):
    """1,000 rules x 1,048,576 packets, seeds 1-5, every packet against the oracle."""
    say(f"scan_1000x1M seed={seed} {kw}")
    rules, pk = gen.workload("scan_1000x1M", seed=seed)
    want = oracle.classify(rules, pk, threads=16)
    assert_same(classify_np(rules, pk, **kw), want, f"1000x1M seed {seed} {kw}")


def test_rule_split_launch_chunks():
    """Rule split over 10,000 rules with no catch-all, asked for 156 partitions: 65 rules each,
    so 154 non-empty partitions and 64 * 154 / 16 = 616 work-items per packet (a wave per
    partition and 16 packets); one launch holds fewer than 2^32, so 7,200,000 packets go in two
    launches (the first covers 6,972,288).
    Packets around the launch edge and a random sample against the oracle; the whole batch
    against the packet-split scan."""
    import torch
    fw = fwmod()
    rules = gen.make_rules(10_000, 31)
    catch = ((rules.src_plen == 0) & (rules.dst_plen == 0) & (rules.sport_lo == 0)
             & (rules.sport_hi == 65535) & (rules.dport_lo == 0) & (rules.dport_hi == 65535)
             & (rules.proto_any != 0))
    rules.proto_any[catch] = 0                  # no catch-all: every rule stays reachable
    n = 7_200_000
    pk = gen.make_packets(rules, n, 31)
    edge = 6_972_288                            # the first launch's last packet + 1
    rng = np.random.Generator(np.random.PCG64(31))
    sample = np.unique(np.concatenate([np.arange(edge - 1000, edge + 1000),
                                       rng.integers(0, n, 20_000)]))
    want = oracle.classify(rules, pk.subset(sample), threads=16)
    say(f"rule split, 156 partitions, {n} packets (two launches)")
    with fw.Ruleset(rules) as rs:
        dp = fw.DevicePackets.from_host(pk)
        got = rs.classify(dp, mode="rule_split", partitions=156)
        ref = rs.classify(dp, mode="packet_split")
        torch.cuda.synchronize()
        gi, ga = got[0].cpu().numpy(), got[1].cpu().numpy()
        np.testing.assert_array_equal(gi, ref[0].cpu().numpy())
        np.testing.assert_array_equal(ga, ref[1].cpu().numpy())
    assert_same((gi[sample], ga[sample]), want, "rule split P=156 sample")


def test_rule_split_short_partitions_share_waves():
    """Partitions shorter than 64 rules are grouped per wave; results are those of the
    oracle for every partition count around the grouping thresholds."""
    rules = gen.make_rules(700, 32)
    pk = gen.make_packets(rules, 30_000, 32)
    want = oracle.classify(rules, pk)
    for P in (1, 10, 11, 12, 13, 63, 64, 65, 127, 700, 5000):
        assert_same(classify_np(rules, pk, mode="rule_split", partitions=P), want, f"P={P}")


def test_hybrid_launch_chunks():
    """Hybrid with 16 partitions and one packet per lane takes 16 work-items per packet, so one
    launch covers 268,435,392 packets; a batch just above that runs in two launches.  The batch tiles
    1,048,576 distinct packets, so every output is checked against the oracle's answer for
    its tile position."""
    import torch
    fw = fwmod()
    rules = gen.make_rules(100, 41)
    base = gen.make_packets(rules, 1 << 20, 41)
    want_idx, want_act = oracle.classify(rules, base, threads=16)
    n = 268_435_392 + 10_000
    reps = -(-n // (1 << 20))
    small = fw.DevicePackets.from_host(base)
    dp = fw.DevicePackets(*(t.repeat(reps)[:n] for t in (small.src_ip, small.dst_ip,
                                                          small.sport, small.dport,
                                                          small.proto)))
    say(f"hybrid P=16 over {n} packets (two launches)")
    with fw.Ruleset(rules) as rs:
        idx, act = rs.classify(dp, mode="hybrid", partitions=16, packets_per_lane=1)
        torch.cuda.synchronize()
    wi = torch.from_numpy(want_idx).cuda().repeat(reps)[:n]
    wa = torch.from_numpy(want_act).cuda().repeat(reps)[:n]
    bad = torch.nonzero((idx != wi) | (act != wa))
    assert bad.numel() == 0, f"{bad.numel()} mismatches, first at {int(bad[0])}"


@pytest.mark.parametrize("n", [0, 1, 3, 63, 64, 65, 255, 257, 1023, 4099])
@pytest.mark.parametrize("kw", SCAN_MODES[:5] + SCAN_MODES[8:9], ids=_id)
def test_ragged_sizes(n, kw):
    say(f"ragged n={n} {kw}")
    rules = gen.make_rules(37, 9)
    pk = gen.make_packets(rules, max(n, 1), 9).subset(slice(0, n))
    want = oracle.classify(rules, pk)
    assert_same(classify_np(rules, pk, **kw), want, f"n={n} {kw}")


@pytest.mark.parametrize("R", [0, 1, 2, 15, 16, 17])
def test_tiny_rulesets_every_partition_count(R):
    """R < P, R = 1, R = 0, and P not dividing R."""
    rules = gen.make_rules(R, 21)
    rules.default_action = 1
    pk = gen.make_packets(gen.make_rules(5, 22), 777, 21)
    want = oracle.classify(rules, pk)
    for kw in ([dict(mode="packet_split")] +
               [dict(mode="rule_split", partitions=p) for p in (1, 2, 5, 16, 33, 64, 65, 200)] +
               [dict(mode="hybrid", partitions=p) for p in (1, 3, 16)]):
        say(f"R={R} {kw}")
        assert_same(classify_np(rules, pk, **kw), want, f"R={R} {kw}")


@pytest.mark.parametrize("wild", [False, True])
def test_boundary_packets(wild):
    """Packets at every rule's lo-1, lo, hi, hi+1 in each field; /0 and /32; ports 0 and 65535.
    Every scan mode and the learned path (whose interval, port-table and source-bucket lookups
    all turn on these values); with `wild`, a third of the rules leave both addresses
    unspecified, so the port/protocol table's edges are probed as well."""
    rules = gen.make_rules(64, 31)
    rules.src_plen[::7] = 32
    rules.dst_plen[::5] = 0
    rules.dport_lo[::6] = 0
    rules.dport_hi[::6] = 65535
    if wild:
        rules.src_plen[1::3] = 0
        rules.dst_plen[1::3] = 0
        catch = ((rules.src_plen == 0) & (rules.dst_plen == 0) & (rules.sport_lo == 0)
                 & (rules.sport_hi == 65535) & (rules.dport_lo == 0) & (rules.dport_hi == 65535))
        rules.proto_any[catch] = 0                 # no catch-all: every rule stays reachable
    rng = np.random.Generator(np.random.PCG64(31))
    from tests.boxes import rule_box
    pts = []
    for r in range(len(rules)):
        box = rule_box(rules, r)
        for f in range(5):
            lo, hi = box[f]
            top = [2**32 - 1, 2**32 - 1, 65535, 65535, 255][f]
            for v in (lo - 1, lo, hi, hi + 1):
                if 0 <= v <= top:
                    p = [int(rng.integers(a, b + 1)) for a, b in box]
                    p[f] = v
                    pts.append(p)
    from tests.boxes import points_to_packets
    pk = points_to_packets(pts)
    want = oracle.classify(rules, pk)
    for kw in SCAN_MODES:
        say(f"boundary wild={wild} {kw}")
        assert_same(classify_np(rules, pk, **kw), want, f"boundary {kw}")
    import torch
    fw = fwmod()
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(epochs1=300, epochs2=600)
        dp = fw.DevicePackets.from_host(pk)
        for ppl in (1, 2, 4):
            say(f"boundary wild={wild} learned K={ppl}")
            idx, act = rs.classify(dp, mode="learned", packets_per_lane=ppl)[:2]
            torch.cuda.synchronize()
            assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, f"boundary learned K={ppl}")


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_10000_rules_16M_packets_whole_batch(seed):
    """10,000 skewed rules x 16,777,216 packets, seeds 1-5: packet split, rule split and hybrid,
    every packet against the oracle."""
    import torch
    fw = fwmod()
    rules, pk = gen.workload("learned_10000x16M", seed=seed)
    want = oracle.classify(rules, pk, threads=16)
    dp = fw.DevicePackets.from_host(pk)
    with fw.Ruleset(rules) as rs:
        for kw in (dict(mode="packet_split"), dict(mode="rule_split", partitions=16),
                   dict(mode="hybrid", partitions=16)):
            say(f"10000x16M seed={seed} {kw}")
            idx, act = rs.classify(dp, **kw)
            torch.cuda.synchronize()
            assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, f"10000x16M seed {seed} {kw}")


@pytest.mark.parametrize("wl,seed", [("learned_10000x16M", 1), ("scan_1000x1M", 2),
                                     ("scan_100x10k", 3)])
def test_auto_without_index_every_batch_size(wl, seed):
    """Mode AUTO without an index picks rule split, the hybrid or packet split by batch size
    (and reachable rules): batches on both sides of every threshold, each against the oracle,
    and each equal to packet split on the same batch."""
    import torch
    fw = fwmod()
    rules, pk = gen.workload(wl, seed=seed, n_packets=300_000)
    want = oracle.classify(rules, pk, threads=16)
    dp = fw.DevicePackets.from_host(pk)
    with fw.Ruleset(rules) as rs:
        for n in (1, 63, 64, 1000, 4096, 4097, 16384, 32768, 32769, 65536, 262143, 262144,
                  300_000):
            say(f"auto {wl} seed={seed} n={n}")
            sub = dp.slice(0, n)
            idx, act = rs.classify(sub)
            ps = rs.classify(sub, mode="packet_split")
            torch.cuda.synchronize()
            got = (idx.cpu().numpy(), act.cpu().numpy())
            assert_same(got, (want[0][:n], want[1][:n]), f"auto {wl} n={n}")
            assert_same(got, (ps[0].cpu().numpy(), ps[1].cpu().numpy()), f"auto vs scan n={n}")


def test_determinism_and_streams():
    """Repeated runs are byte-identical, on the null stream and on a side stream."""
    import torch
    fw = fwmod()
    rules, pk = gen.workload("scan_1000x1M", seed=2, n_packets=200_000)
    dp = fw.DevicePackets.from_host(pk)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with fw.Ruleset(rules) as rs:
        outs = []
        for kw in (dict(mode="packet_split"), dict(mode="rule_split", partitions=16),
                   dict(mode="rule_split", partitions=256), dict(mode="hybrid", partitions=16)):
            for stream in (None, s):
                idx, act = rs.classify(dp, stream=stream, **kw)
                torch.cuda.synchronize()
                outs.append((idx.cpu().numpy(), act.cpu().numpy()))
        for o in outs[1:]:
            np.testing.assert_array_equal(o[0], outs[0][0])
            np.testing.assert_array_equal(o[1], outs[0][1])


def test_plain_entry_point_and_errors():
    import torch
    fw = fwmod()
    rules, pk = gen.workload("scan_100x10k", seed=4, n_packets=1000)
    want = oracle.classify(rules, pk)
    dp = fw.DevicePackets.from_host(pk)
    with fw.Ruleset(rules) as rs:
        assert rs.size() == 100
        idx, act = rs.classify_plain(dp)
        torch.cuda.synchronize()
        assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, "fw_classify")
        # misaligned packet array
        bad = fw.DevicePackets(dp.src_ip[1:], dp.dst_ip[1:], dp.sport[1:], dp.dport[1:],
                               dp.proto[1:])
        with pytest.raises(fw.FwError) as ei:
            rs.classify(bad)
        assert ei.value.status == fw.E_ALIGN
        with pytest.raises(fw.FwError) as ei:
            rs.classify(dp, mode=9)
        assert ei.value.status == fw.E_INVAL
        with pytest.raises(fw.FwError) as ei:
            rs.classify(dp, mode="learned")
        assert ei.value.status == fw.E_NOINDEX
        with pytest.raises(fw.FwError) as ei:
            rs.classify(dp, mode="hybrid", partitions=17)
        assert ei.value.status == fw.E_INVAL
        # n == 0 is accepted and writes nothing
        rs.classify(dp.slice(0, 0))
        # fields of unequal length, and outputs too short, never reach a kernel
        with pytest.raises(ValueError):
            rs.classify(fw.DevicePackets(dp.src_ip, dp.dst_ip, dp.sport[:-16], dp.dport,
                                         dp.proto))
        with pytest.raises(ValueError):
            rs.classify(dp, out_idx=torch.empty(len(dp) - 1, dtype=torch.int32, device="cuda"))
        with pytest.raises(ValueError):
            rs.closed_loop(dp, [0], [len(dp) + 16])


@pytest.mark.parametrize("catch_all_at", [None, 0, 150, 299])
def test_every_first_test_kind(catch_all_at):
    """Rules whose most selective field is each of destination, source, ports and protocol,
    with and without a catch-all (rules after it can never match)."""
    rng = np.random.Generator(np.random.PCG64(77))
    R = 300
    rules = gen.make_rules(R, 77, skew=True)
    kind = rng.integers(0, 4, R)
    rules.src_plen[kind == 0] = 0                      # destination only (or both narrow)
    rules.dst_plen[kind == 1] = 0                      # source only
    for k in (2, 3):
        rules.src_plen[kind == k] = 0
        rules.dst_plen[kind == k] = 0
    rules.proto_any[kind == 2] = 1                     # ports only
    rules.sport_lo[kind == 3] = 0                      # protocol only
    rules.sport_hi[kind == 3] = 65535
    rules.dport_lo[kind == 3] = 0
    rules.dport_hi[kind == 3] = 65535
    rules.proto_any[kind == 3] = 0
    if catch_all_at is not None:
        c = catch_all_at
        rules.src_plen[c] = rules.dst_plen[c] = 0
        rules.sport_lo[c] = rules.dport_lo[c] = 0
        rules.sport_hi[c] = rules.dport_hi[c] = 65535
        rules.proto_any[c] = 1
    pk = gen.make_packets(rules, 50_000, 78)
    want = oracle.classify(rules, pk, threads=8)
    for kw in SCAN_MODES + [dict(mode="learned")]:
        say(f"kinds catch_all_at={catch_all_at} {kw}")
        if kw["mode"] == "learned":
            import torch
            fw = fwmod()
            with fw.Ruleset(rules) as rs:
                rs.build_learned_index(epochs1=200, epochs2=400)
                idx, act = rs.classify(fw.DevicePackets.from_host(pk), mode="learned")
                torch.cuda.synchronize()
                got = (idx.cpu().numpy(), act.cpu().numpy())
        else:
            got = classify_np(rules, pk, **kw)
        assert_same(got, want, f"kinds {catch_all_at} {kw}")


def _address_filter_case(seed: int):
    """Rules built so that many lanes pass one address while every lane fails the next test,
    with the matching rules only in the last third of the list (long scans through them):
    destination-first rules whose source (a /8 no packet uses) fails, source-first rules whose
    destination fails, rules passing both addresses but failing on ports or on protocol, and
    rules that match packets of one destination /24 on one port and protocol."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, R = 20_000, 600
    src_nets = (0x0A010000 + (np.arange(8, dtype=np.uint32) << 8)).astype(np.uint32)
    dst_nets = (0xAC100000 + (np.arange(8, dtype=np.uint32) << 8)).astype(np.uint32)
    ports = np.array([53, 80, 443, 8080], dtype=np.uint16)
    pk = gen.Packets(
        src_ip=(src_nets[rng.integers(0, 8, n)] | rng.integers(0, 256, n).astype(np.uint32)),
        dst_ip=(dst_nets[rng.integers(0, 8, n)] | rng.integers(0, 256, n).astype(np.uint32)),
        sport=rng.integers(1024, 65536, n).astype(np.uint16),
        dport=ports[rng.integers(0, 4, n)],
        proto=np.array([6, 17], dtype=np.uint8)[rng.integers(0, 2, n)])
    kind = rng.integers(0, 4, R)
    kind[2 * R // 3:] = rng.integers(0, 5, R - 2 * R // 3)      # matching rules: the last third
    z8 = np.zeros(R, np.uint8)
    rules = gen.Ruleset(
        src_ip=src_nets[rng.integers(0, 8, R)].copy(), src_plen=np.full(R, 16, np.uint8),
        dst_ip=dst_nets[rng.integers(0, 8, R)].copy(), dst_plen=np.full(R, 24, np.uint8),
        sport_lo=np.zeros(R, np.uint16), sport_hi=np.full(R, 65535, np.uint16),
        dport_lo=np.zeros(R, np.uint16), dport_hi=np.full(R, 65535, np.uint16),
        proto=z8.copy(), proto_any=np.ones(R, np.uint8),
        action=rng.integers(0, 2, R).astype(np.uint8))
    d = kind == 0                                   # destination /24 passes, source /8 fails
    rules.src_ip[d] = 0xC0000000
    rules.src_plen[d] = 8
    s_ = kind == 1                                  # source /24 passes, destination /8 fails
    rules.src_plen[s_] = 24
    rules.dst_ip[s_] = 0xC0000000
    rules.dst_plen[s_] = 8
    p_ = kind == 2                                  # both addresses pass, ports fail
    rules.dport_lo[p_] = 1
    rules.dport_hi[p_] = 52
    q_ = kind == 3                                  # addresses and ports pass, protocol fails
    rules.proto_any[q_] = 0
    rules.proto[q_] = 1
    m_ = kind == 4                                  # matches a destination /24, port, protocol
    rules.dport_lo[m_] = rules.dport_hi[m_] = ports[rng.integers(0, 4, int(m_.sum()))]
    rules.proto_any[m_] = 0
    rules.proto[m_] = 6
    return rules, pk


@pytest.mark.parametrize("seed", [5, 6])
def test_second_field_rejections(seed):
    """Every path against the oracle where a rule's first address passes in many lanes and a
    later field fails in all of them (the rule is left after that field's test)."""
    import torch
    fw = fwmod()
    rules, pk = _address_filter_case(seed)
    want = oracle.classify(rules, pk, threads=8)
    assert (want[0] >= 0).mean() > 0.3 and (want[0] < 0).any()
    for kw in SCAN_MODES:
        say(f"second-field seed={seed} {kw}")
        assert_same(classify_np(rules, pk, **kw), want, f"second-field {seed} {kw}")
    with fw.Ruleset(rules) as rs:
        dp = fw.DevicePackets.from_host(pk)
        for K in (1, 2, 4):
            for placement, tile in ((1, 0), (2, 256), (2, 1024), (3, 0), (4, 0)):
                say(f"second-field seed={seed} multi K={K} placement={placement} tile={tile}")
                oi = torch.full((len(pk),), 7, dtype=torch.int32, device="cuda")
                oa = torch.full((len(pk),), 9, dtype=torch.uint8, device="cuda")
                fw.classify_multi([(rs, dp, oi, oa)], packets_per_lane=K, placement=placement,
                                  rule_tile=tile)
                torch.cuda.synchronize()
                assert_same((oi.cpu().numpy(), oa.cpu().numpy()), want,
                            f"second-field {seed} multi K={K} placement={placement} tile={tile}")
        say(f"second-field seed={seed} learned")
        rs.build_learned_index(epochs1=200, epochs2=400)
        idx, act = rs.classify(dp, mode="learned")
        torch.cuda.synchronize()
        assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, f"second-field {seed} learned")


def test_closed_loop_probe():
    """fw_closed_loop classifies each batch like fw_classify_ex (checked on its last batch,
    whose results are left in the output arrays), reports a positive time per batch, and
    rejects a batch start that breaks 16-byte alignment."""
    import torch
    fw = fwmod()
    rules = gen.make_rules(300, 41)
    pk = gen.make_packets(rules, 20_000, 41)
    with fw.Ruleset(rules) as rs:
        dp = fw.DevicePackets.from_host(pk)
        rs.build_learned_index(epochs1=200, epochs2=400)
        for mode in ("packet_split", "rule_split", "hybrid", "learned"):
            starts = np.array([0, 16, 4096, 8000], dtype=np.uint64)
            counts = np.array([64, 1000, 3, 5000], dtype=np.uint64)
            sec, idx, act = rs.closed_loop(dp, starts, counts, mode=mode, partitions=4)
            torch.cuda.synchronize()
            assert sec.shape == (4,) and np.all(sec > 0)
            want = oracle.classify(rules, pk.subset(slice(8000, 13000)))
            assert_same((idx[:5000].cpu().numpy(), act[:5000].cpu().numpy()), want,
                        f"closed loop {mode}")
        with pytest.raises(fw.FwError) as ei:
            rs.closed_loop(dp, np.array([8]), np.array([10]))
        assert ei.value.status == fw.E_ALIGN


def test_permutation_and_batch_size_invariance():
    """Invariants of a per-packet result (the oracle's own tests pin them on the CPU): permuting
    the packets permutes the outputs, and any 16-aligned slice of a batch, of any length,
    classifies exactly as the same packets inside the whole batch, in every mode (the library
    picks packets per lane and launch shapes by batch size, so this crosses those choices)."""
    import torch
    fw = fwmod()
    rules, pk = gen.workload("scan_1000x1M", seed=17, n_packets=300_000)
    rng = np.random.Generator(np.random.PCG64(17))
    perm = rng.permutation(len(pk))
    dp = fw.DevicePackets.from_host(pk)
    dperm = fw.DevicePackets.from_host(pk.subset(perm))
    cuts = [(0, 1), (16, 63), (4096, 65), (160_000, 9_999), (32, 300_000 - 32)]
    with fw.Ruleset(rules) as rs:
        rs.build_learned_index(epochs1=300, epochs2=600)
        modes = SCAN_MODES[:4] + [dict(mode="hybrid", partitions=16)] + \
            [dict(mode="learned", packets_per_lane=k) for k in (0, 1, 2, 4)]
        for kw in modes:
            say(f"invariance {kw}")
            full = [t.cpu().numpy() for t in rs.classify(dp, **kw)[:2]]
            got = [t.cpu().numpy() for t in rs.classify(dperm, **kw)[:2]]
            torch.cuda.synchronize()
            assert np.array_equal(got[0], full[0][perm]) and np.array_equal(got[1], full[1][perm]), \
                f"permutation {kw}"
            for a, m in cuts:
                part = [t.cpu().numpy() for t in rs.classify(dp.slice(a, a + m), **kw)[:2]]
                assert np.array_equal(part[0], full[0][a:a + m]), f"slice {a}+{m} {kw}"
                assert np.array_equal(part[1], full[1][a:a + m]), f"slice {a}+{m} {kw}"
