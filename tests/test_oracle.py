"""Pins for the CPU first-match oracle (no GPU).

The oracle is checked against things other than itself: hand-derived answers
(tests/golden), packets constructed inside exactly one leading box, invariants
of first match, and an exhaustive painter's-algorithm brute force.
"""

import numpy as np
import pytest

import oracle
from synth import gen
from tests import boxes, golden_io


@pytest.mark.parametrize("name", golden_io.names())
def test_golden_fixtures(name):
    rs, pk, exp_i, exp_a = golden_io.load(name)
    idx, act = oracle.classify(rs, pk)
    np.testing.assert_array_equal(idx, exp_i)
    np.testing.assert_array_equal(act, exp_a)


@pytest.mark.parametrize("seed,skew", [(1, False), (2, True), (3, False)])
def test_box_construction_gives_k(seed, skew):
    """A packet inside rule k's box and outside every earlier box has first match k."""
    rules = gen.make_rules(60, seed, skew=skew)
    rng = np.random.Generator(np.random.PCG64(seed))
    pts, ks = [], []
    for k in range(len(rules)):
        p = boxes.point_inside_only(rules, k, rng)
        if p is not None:          # k fully shadowed by earlier rules: skip it
            pts.append(p)
            ks.append(k)
    assert len(ks) > 30
    idx, act = oracle.classify(rules, boxes.points_to_packets(pts))
    np.testing.assert_array_equal(idx, np.array(ks, np.int32))
    np.testing.assert_array_equal(act, rules.action[np.array(ks)])


def test_painter_bruteforce_tiny_domain():
    """Every cell of a dense grid agrees with painting the boxes in reverse order."""
    rng = np.random.Generator(np.random.PCG64(11))
    base = 0xC0A80100                      # 192.168.1.0/27 holds every address used
    R = 40
    def pfx():
        plen = int(rng.choice([27, 28, 29, 30, 31, 32]))
        return base + int(rng.integers(0, 32)), plen   # host bits left set
    cols = {k: [] for k in ("src_ip", "src_plen", "dst_ip", "dst_plen", "sport_lo",
                            "sport_hi", "dport_lo", "dport_hi", "proto", "proto_any",
                            "action")}
    for _ in range(R):
        for f in ("src", "dst"):
            if rng.random() < 0.15:
                b, l = int(rng.integers(0, 2**32)), 0
            else:
                b, l = pfx()
            cols[f + "_ip"].append(b)
            cols[f + "_plen"].append(l)
        for f in ("sport", "dport"):
            if rng.random() < 0.3:
                lo, hi = 0, 65535
            else:
                lo = int(rng.integers(0, 8))
                hi = int(rng.integers(lo, 8))
            cols[f + "_lo"].append(lo)
            cols[f + "_hi"].append(hi)
        pk = int(rng.integers(0, 3))
        cols["proto"].append([0, 6, 17][pk] if rng.random() < 0.7 else 0)
        cols["proto_any"].append(int(rng.random() >= 0.7))
        cols["action"].append(int(rng.integers(0, 2)))
    dts = dict(src_ip=np.uint32, dst_ip=np.uint32, src_plen=np.uint8, dst_plen=np.uint8,
               sport_lo=np.uint16, sport_hi=np.uint16, dport_lo=np.uint16,
               dport_hi=np.uint16, proto=np.uint8, proto_any=np.uint8, action=np.uint8)
    rules = gen.Ruleset(**{k: np.array(v, dtype=dts[k]) for k, v in cols.items()})
    ips = base + np.arange(32)
    pk, want = boxes.painter(rules, ips, ips, np.arange(8), np.arange(8), [0, 6, 17, 200])
    idx, act = oracle.classify(rules, pk, threads=4)
    np.testing.assert_array_equal(idx, want)
    exp_act = np.where(want < 0, rules.default_action, rules.action[np.maximum(want, 0)])
    np.testing.assert_array_equal(act, exp_act)


def _perm_tail(rules, start, rng):
    order = np.concatenate([np.arange(start), start + rng.permutation(len(rules) - start)])
    return rules.subset(order)


@pytest.mark.parametrize("seed", [1, 4])
def test_invariants(seed):
    rules, pk = gen.workload("scan_100x10k", seed=seed, n_packets=4000)
    idx, act = oracle.classify(rules, pk)
    rng = np.random.Generator(np.random.PCG64(seed))
    # permuting the rules after the last first-match changes nothing
    m = int(idx.max())
    if m + 1 < len(rules):
        i2, a2 = oracle.classify(_perm_tail(rules, m + 1, rng), pk)
        np.testing.assert_array_equal(i2, idx)
        np.testing.assert_array_equal(a2, act)
    # appending rules only changes packets that had no match
    extra = gen.make_rules(50, seed + 100)
    i3, _ = oracle.classify(gen.concat_rulesets([rules, extra]), pk)
    np.testing.assert_array_equal(i3[idx >= 0], idx[idx >= 0])
    assert np.all((i3[idx < 0] == -1) | (i3[idx < 0] >= len(rules)))
    # unmatched packets get (-1, default)
    assert np.all(act[idx < 0] == rules.default_action)
    # packet permutation permutes the results; batch size does not matter
    p = rng.permutation(len(pk))
    i4, a4 = oracle.classify(rules, pk.subset(p))
    np.testing.assert_array_equal(i4, idx[p])
    np.testing.assert_array_equal(a4, act[p])
    i5, _ = oracle.classify(rules, pk.subset(slice(123, 777)))
    np.testing.assert_array_equal(i5, idx[123:777])
    # thread count does not matter
    i6, a6 = oracle.classify(rules, pk, threads=7)
    np.testing.assert_array_equal(i6, idx)
    np.testing.assert_array_equal(a6, act)


def test_catch_all_first_and_empty_ruleset():
    rules, pk = gen.workload("scan_100x10k", seed=2, n_packets=1000)
    catch = gen.Ruleset(np.zeros(1, np.uint32), np.zeros(1, np.uint8),
                        np.zeros(1, np.uint32), np.zeros(1, np.uint8),
                        np.zeros(1, np.uint16), np.full(1, 65535, np.uint16),
                        np.zeros(1, np.uint16), np.full(1, 65535, np.uint16),
                        np.zeros(1, np.uint8), np.ones(1, np.uint8), np.ones(1, np.uint8))
    idx, act = oracle.classify(gen.concat_rulesets([catch, rules]), pk)
    assert np.all(idx == 0) and np.all(act == 1)
    empty = rules.subset(slice(0, 0))
    empty.default_action = 1
    idx, act = oracle.classify(empty, pk)
    assert np.all(idx == -1) and np.all(act == 1)


def test_check_counts():
    """Rule checks = first-match index + 1, or the rule count when unmatched."""
    rules, pk = gen.workload("scan_100x10k", seed=3, n_packets=3000)
    idx, _, (checks, tests) = oracle.classify(rules, pk, threads=3, with_stats=True)
    want = np.where(idx < 0, len(rules), idx.astype(np.int64) + 1).sum()
    assert checks == int(want)
    assert checks <= tests <= 4 * checks
