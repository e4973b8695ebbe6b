"""Seeded random sweep: many small rulesets of mixed shape through every path, each result
against the CPU oracle bit for bit.  Shapes vary rule count (0, 1, 2, 64 and 65 rules pinned
for the first seeds), prefix skew, address-wildcard density and where (if anywhere) a
catch-all rule sits; one seed classifies a single packet."""

import numpy as np
import pytest

import oracle
from synth import gen
from tests.gpu_util import assert_same, fwmod, say

pytestmark = pytest.mark.gpu


def _ruleset(seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    R = (0, 1, 2, 64, 65)[seed] if seed < 5 else int(rng.integers(0, 400))
    rules = gen.make_rules(R, 2000 + seed, skew=bool(seed % 2))
    if R:
        wild = rng.random(R) < rng.choice([0.0, 0.1, 0.5])
        rules.src_plen[wild] = 0
        rules.dst_plen[wild] = 0
        catch = ((rules.src_plen == 0) & (rules.dst_plen == 0) & (rules.sport_lo == 0)
                 & (rules.sport_hi == 65535) & (rules.dport_lo == 0)
                 & (rules.dport_hi == 65535) & (rules.proto_any != 0))
        rules.proto_any[catch] = 0          # place catch-alls explicitly below
        if rng.random() < 0.5:
            k = int(rng.integers(0, R))
            for f, v in (("src_plen", 0), ("dst_plen", 0), ("sport_lo", 0), ("sport_hi", 65535),
                         ("dport_lo", 0), ("dport_hi", 65535), ("proto_any", 1)):
                getattr(rules, f)[k] = v
    rules.default_action = int(rng.integers(0, 2))
    return rules, rng


@pytest.mark.parametrize("seed", range(30))
def test_random_rulesets_every_path(seed):
    import torch
    fw = fwmod()
    rules, rng = _ruleset(seed)
    n = 1 if seed == 5 else int(rng.integers(1, 6000))
    pk = gen.make_packets(rules if len(rules) else gen.make_rules(5, seed), n, 3000 + seed)
    want = oracle.classify(rules, pk)
    P = int(rng.integers(1, 40))
    say(f"random seed={seed} R={len(rules)} n={n} P={P}")
    with fw.Ruleset(rules) as rs:
        dp = fw.DevicePackets.from_host(pk)
        runs = [dict(mode="packet_split", packets_per_lane=k) for k in (1, 2, 4)]
        runs += [dict(mode="rule_split", partitions=P), dict(mode="hybrid",
                                                             partitions=1 + P % 16)]
        if len(rules):
            rs.build_learned_index(epochs1=150, epochs2=300, seed=seed)
            runs += [dict(mode="learned", packets_per_lane=k) for k in (1, 2, 4)]
            runs += [dict(mode="learned", lookup=1)]
        for kw in runs:
            idx, act = rs.classify(dp, **kw)[:2]
            torch.cuda.synchronize()
            assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, f"seed={seed} {kw}")


@pytest.mark.parametrize("seed", range(8))
def test_random_large_rulesets(seed):
    """Larger seeded rulesets (1,000-30,000 rules, mostly skewed prefixes, some with every
    destination specified so that tens of thousands of boundaries sit in global memory) and
    batches of 100,000-1,000,000 packets: every learned variant, AUTO, packet split and the
    hybrid against the oracle, and the index's half-storage rounding count."""
    import torch
    fw = fwmod()
    rng = np.random.Generator(np.random.PCG64(77 + seed))
    R = int(rng.integers(1000, 30000))
    rules = gen.make_rules(R, 5000 + seed, skew=bool(rng.random() < 0.7))
    if rng.random() < 0.3:
        rules.dst_plen[rules.dst_plen == 0] = int(rng.choice([8, 16, 24]))
    n = int(rng.integers(100_000, 1_000_000))
    pk = gen.make_packets(rules, n, 6000 + seed)
    want = oracle.classify(rules, pk, threads=16)
    say(f"random large seed={seed} R={R} n={n}")
    with fw.Ruleset(rules) as rs:
        dp = fw.DevicePackets.from_host(pk)
        st = rs.build_learned_index(seed=seed)
        say(f"  |B|={st['n_boundaries']} err_mean={st['err_mean']:.1f}")
        assert st["weights_rounded"] == 0
        runs = [dict(mode="learned", packets_per_lane=k) for k in (1, 2, 4)]
        runs += [dict(mode="learned", lookup=1), dict(mode="auto"), dict(mode="packet_split"),
                 dict(mode="hybrid", partitions=16)]
        for kw in runs:
            idx, act = rs.classify(dp, **kw)[:2]
            torch.cuda.synchronize()
            assert_same((idx.cpu().numpy(), act.cpu().numpy()), want, f"seed={seed} {kw}")
