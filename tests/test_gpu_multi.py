"""Many chains in one persistent launch: every chain bit-exact against the oracle."""

import numpy as np
import pytest

import oracle
from synth import gen
from tests.gpu_util import fwmod, say

pytestmark = pytest.mark.gpu


def _setup(scale, seed=1, extra_edge=True):
    import torch
    fw = fwmod()
    work = gen.multichain_workload(seed=seed, scale=scale)
    if extra_edge:
        work.append((gen.make_rules(0, 5), gen.make_packets(gen.make_rules(3, 6), 300, 5)))
        work.append((gen.make_rules(50, 7), gen.make_packets(gen.make_rules(50, 7), 1, 7)))
        empty = gen.make_packets(gen.make_rules(3, 8), 1, 8).subset(slice(0, 0))
        work.append((gen.make_rules(20, 9), empty))
    items, rss = [], []
    for rules, pk in work:
        rs = fw.Ruleset(rules)
        rss.append(rs)
        n = len(pk)
        dp = fw.DevicePackets.from_host(pk) if n else fw.DevicePackets.from_host(
            gen.make_packets(rules if len(rules) else gen.make_rules(1, 1), 1, 1)).slice(0, 0)
        items.append((rs, dp, torch.full((max(n, 1),), 7, dtype=torch.int32, device="cuda")[:n],
                      torch.full((max(n, 1),), 9, dtype=torch.uint8, device="cuda")[:n]))
    torch.cuda.synchronize()
    return work, items, rss


def _check(work, items, what):
    import torch
    torch.cuda.synchronize()
    for c, ((rules, pk), (_, _, oi, oa)) in enumerate(zip(work, items)):
        want_i, want_a = oracle.classify(rules, pk, threads=8)
        np.testing.assert_array_equal(oi.cpu().numpy(), want_i, err_msg=f"{what} chain {c} idx")
        np.testing.assert_array_equal(oa.cpu().numpy(), want_a, err_msg=f"{what} chain {c} act")


@pytest.mark.parametrize("placement,tile", [(4, 0), (1, 0), (3, 0), (2, 256), (2, 1024)])
@pytest.mark.parametrize("K", [1, 2, 4])
def test_every_configuration(K, placement, tile):
    fw = fwmod()
    work, items, rss = _setup(scale=0.02)
    say(f"multi K={K} placement={placement} tile={tile} chains={len(items)}")
    for _, _, oi, oa in items:
        oi.fill_(7)
        oa.fill_(9)
    fw.classify_multi(items, packets_per_lane=K, placement=placement, rule_tile=tile)
    _check(work, items, f"K={K} placement={placement} tile={tile}")
    for rs in rss:
        rs.close()


def test_autotuned_full_shape_sampled():
    """64 chains at full batch sizes (log-uniform 4,096..1,048,576 packets); a sample per chain."""
    import torch
    fw = fwmod()
    work, items, rss = _setup(scale=1.0, seed=2, extra_edge=False)
    say(f"multi autotune over {sum(len(p) for _, p in work)} packets")
    best, ms = fw.autotune_multi(items)
    say(f"  best {best} {ms:.3f} ms")
    assert best["packets_per_lane"] in (1, 2, 4) and best["placement"] in (1, 2, 3, 4)
    for _, _, oi, oa in items:
        oi.fill_(7)
    fw.classify_multi(items)                    # tuned options
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(3))
    for c, ((rules, pk), (_, _, oi, oa)) in enumerate(zip(work, items)):
        sel = np.sort(rng.choice(len(pk), min(len(pk), 2000), replace=False))
        want_i, want_a = oracle.classify(rules, pk.subset(sel), threads=8)
        np.testing.assert_array_equal(oi.cpu().numpy()[sel], want_i, err_msg=f"chain {c}")
        np.testing.assert_array_equal(oa.cpu().numpy()[sel], want_a, err_msg=f"chain {c}")
    for rs in rss:
        rs.close()


@pytest.mark.parametrize("big_index", [False, True])
@pytest.mark.parametrize("K", [1, 2, 4])
def test_learned_and_scanned_chains_in_one_launch(K, big_index):
    """Placement 4 routes chains with a learned index through the learned lookup (their LDS
    images staged as work-groups move between chains) and the rest through the grouped-plan
    scan, in one launch.  With big_index one chain's boundary array is too large for LDS, so
    that index is searched in global memory while the others keep theirs in LDS, in the same
    launch.  Each chain against the oracle, and again on a second call with fewer chains."""
    import torch
    fw = fwmod()
    work = []
    for c, (R, n, skew) in enumerate([(10_000, 150_000, True), (2_000, 40_000, True),
                                      (300, 9_000, False), (5_000, 70_000, True),
                                      (40, 1_000, False), (1_500, 33_000, False)]):
        rules = gen.make_rules(R, 300 + c, skew=skew)
        work.append((rules, gen.make_packets(rules, n, 300 + c)))
    if big_index:
        rules = gen.make_rules(30_000, 399, skew=True)
        rules.dst_plen[rules.dst_plen == 0] = 24
        work.append((rules, gen.make_packets(rules, 60_000, 399)))
    items, rss = [], []
    for c, (rules, pk) in enumerate(work):
        rs = fw.Ruleset(rules)
        if c % 2 == 0 or (big_index and c == len(work) - 1):
            rs.build_learned_index(epochs1=300, epochs2=600, seed=c)
        rss.append(rs)
        n = len(pk)
        items.append((rs, fw.DevicePackets.from_host(pk),
                      torch.full((n,), 7, dtype=torch.int32, device="cuda"),
                      torch.full((n,), 9, dtype=torch.uint8, device="cuda")))
    torch.cuda.synchronize()
    for what, pick in (("all chains", list(range(len(items)))), ("three chains", [1, 2, 3])):
        say(f"multi learned+scan K={K} big_index={big_index}: {what}")
        sub = [items[i] for i in pick]
        for _, _, oi, oa in sub:
            oi.fill_(7)
            oa.fill_(9)
        fw.classify_multi(sub, packets_per_lane=K, placement=4)
        _check([work[i] for i in pick], sub, f"K={K} {what}")
    for rs in rss:
        rs.close()


@pytest.mark.parametrize("K", [1, 2, 4])
def test_every_chain_indexed_boundary_placements(K):
    """Every chain with a learned index (the launch without scan items): the boundary arrays of
    all chains in LDS, of none (one index too large for LDS alone), and of some (that index
    beside small ones); each chain against the oracle."""
    import torch
    fw = fwmod()
    work = []
    for c, (R, n) in enumerate([(3_000, 60_000), (800, 20_000), (6_000, 90_000)]):
        rules = gen.make_rules(R, 700 + c, skew=True)
        work.append((rules, gen.make_packets(rules, n, 700 + c)))
    big = gen.make_rules(30_000, 799, skew=True)
    big.dst_plen[big.dst_plen == 0] = 24
    work.append((big, gen.make_packets(big, 50_000, 799)))
    items = []
    for c, (rules, pk) in enumerate(work):
        rs = fw.Ruleset(rules)
        rs.build_learned_index(epochs1=300, epochs2=600, seed=c)
        n = len(pk)
        items.append((rs, fw.DevicePackets.from_host(pk),
                      torch.full((n,), 7, dtype=torch.int32, device="cuda"),
                      torch.full((n,), 9, dtype=torch.uint8, device="cuda")))
    torch.cuda.synchronize()
    for what, pick in (("all in LDS", [0, 1, 2]), ("none in LDS", [3]), ("mixed", [0, 1, 2, 3])):
        say(f"every chain indexed K={K}: {what}")
        sub = [items[i] for i in pick]
        for _, _, oi, oa in sub:
            oi.fill_(7)
            oa.fill_(9)
        fw.classify_multi(sub, packets_per_lane=K, placement=4)
        _check([work[i] for i in pick], sub, f"K={K} {what}")
    for rs, _, _, _ in items:
        rs.close()
