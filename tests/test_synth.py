"""The seeded workload generators against the stated input recipe (no GPU).

Rules: prefix lengths uniform over {0, 8, 16, 24, 32} (skewed: {24, 32} with probability
0.6, else {0, 8, 16}); each port field 40% wildcard, 30% exact, 30% a range of width
clamp(floor(2^(12u)), 1, 4096); protocol uniform over {TCP, UDP, any}; action 50/50.
Packets: half inside a uniformly chosen rule's box, half uniform.  Proportions are checked
within about five standard deviations of their sampling error.
"""

import math

import numpy as np
import pytest

import oracle
from synth import gen

N = 200_000


def _close(frac, p, n, what):
    sd = math.sqrt(p * (1 - p) / n)
    assert abs(frac - p) < 5 * sd, f"{what}: {frac:.4f} against {p:.4f} (sd {sd:.4f})"


@pytest.mark.parametrize("skew", [False, True])
def test_prefix_lengths(skew):
    r = gen.make_rules(N, 11, skew=skew)
    for plen in (r.src_plen, r.dst_plen):
        want = ({24: 0.3, 32: 0.3, 0: 0.4 / 3, 8: 0.4 / 3, 16: 0.4 / 3} if skew
                else {k: 0.2 for k in (0, 8, 16, 24, 32)})
        assert set(np.unique(plen)) == set(want)
        for k, p in want.items():
            _close(float((plen == k).mean()), p, N, f"plen {k} skew {skew}")


def test_ports_protocol_action():
    r = gen.make_rules(N, 12)
    for lo, hi in ((r.sport_lo, r.sport_hi), (r.dport_lo, r.dport_hi)):
        lo = lo.astype(np.int64)
        hi = hi.astype(np.int64)
        assert (lo <= hi).all()
        wild = (lo == 0) & (hi == 65535)
        exact = lo == hi
        rng_ = ~wild & ~exact
        # a range draw of width 1 (probability 1/12) is an exact port, so exact ports and
        # ranges are checked together; a range (width at most 4,096) is never a wildcard
        _close(float(wild.mean()), 0.4, N, "wildcard ports")
        _close(float((exact | rng_).mean()), 0.6, N, "specified ports")
        assert ((hi - lo + 1)[rng_] <= 4096).all()
        # log-uniform widths: the median width of the ranges is near 2^6
        med = float(np.median((hi - lo + 1)[rng_]))
        assert 40 <= med <= 100, med
    any_ = r.proto_any != 0
    _close(float(any_.mean()), 1 / 3, N, "any protocol")
    _close(float((~any_ & (r.proto == 6)).mean()), 1 / 3, N, "TCP")
    _close(float((~any_ & (r.proto == 17)).mean()), 1 / 3, N, "UDP")
    _close(float((r.action == 1).mean()), 0.5, N, "ACCEPT")


def test_packets_half_in_a_box():
    rules = gen.make_rules(100, 13)
    pk = gen.make_packets(rules, 40_000, 13)
    idx, _ = oracle.classify(rules, pk, threads=4)
    matched = float((idx >= 0).mean())
    # every in-box packet matches at least its own rule; a uniform packet rarely matches
    assert 0.49 <= matched <= 0.65, matched
    # the uniform half spans the header space: protocol values well beyond TCP and UDP
    assert len(np.unique(pk.proto)) > 200


def test_named_sizes_and_multichain_ranges():
    for name, (R, n, skew) in gen.WORKLOADS.items():
        if n > 2_000_000:
            continue
        rules, pk = gen.workload(name, seed=1)
        assert (len(rules), len(pk)) == (R, n)
    assert gen.WORKLOADS["learned_10000x16M"] == (10_000, 16_777_216, True)
    work = gen.multichain_workload(seed=1, scale=0.01)
    assert len(work) == 64
    rules_n = np.array([len(r) for r, _ in work])
    assert rules_n.min() >= 32 and rules_n.max() <= 8192
    # log-uniform over 32..8192: the median near sqrt(32 * 8192) = 512
    assert 150 <= np.median(rules_n) <= 1700


def test_seeded():
    a = gen.workload("scan_100x10k", seed=4)
    b = gen.workload("scan_100x10k", seed=4)
    c = gen.workload("scan_100x10k", seed=5)
    assert np.array_equal(a[0].dst_ip, b[0].dst_ip) and np.array_equal(a[1].src_ip, b[1].src_ip)
    assert not np.array_equal(a[0].dst_ip, c[0].dst_ip)
