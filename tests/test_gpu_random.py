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
