"""Pins for the interval / candidate-list oracle and the float64 network oracle (no GPU)."""

import bisect

import numpy as np
import pytest

import oracle
from oracle import intervals as iv
from oracle import rmi
from synth import gen
from tests import boxes


def _covers(rules, r, x):
    lo, hi = boxes.prefix_range(int(rules.dst_ip[r]), int(rules.dst_plen[r]))
    return lo <= x <= hi


@pytest.mark.parametrize("seed,skew,R", [(1, False, 40), (2, True, 60), (5, True, 25)])
def test_candidate_lemma(seed, skew, R):
    """For addresses around every boundary, the covering rules are exactly C_j of x's interval."""
    rules = gen.make_rules(R, seed, skew=skew)
    B = iv.boundaries(rules)
    C = iv.candidates(rules, B)
    assert B[0] == 0 and np.all(np.diff(B.astype(np.int64)) > 0)
    probes = set()
    for b in B.tolist():
        probes.update(v for v in (b - 1, b, b + 1) if 0 <= v < 2**32)
    probes.update([0, 2**32 - 1])
    Bl = B.tolist()
    for x in sorted(probes):
        j = int(iv.interval_of(B, [x])[0])
        assert j == bisect.bisect_right(Bl, x) - 1            # textbook upper_bound - 1
        assert Bl[j] <= x and (j + 1 == len(Bl) or x < Bl[j + 1])
        want = [r for r in range(R) if _covers(rules, r, x)]
        assert list(C[j]) == want


def test_boundary_set_by_hand():
    """Three destination prefixes whose boundary set can be listed by hand."""
    rules = gen.make_rules(3, 1)
    rules.dst_ip[:] = [0x0A000000, 0x0A010000, 0xFFFFFF00]   # 10/8, 10.1/16, 255.255.255.0/24
    rules.dst_plen[:] = [8, 16, 24]
    B = iv.boundaries(rules)
    want = [0, 0x0A000000, 0x0A010000, 0x0A020000, 0x0B000000, 0xFFFFFF00]
    assert B.tolist() == want                  # 2**32 (end of the /24) does not fit: omitted
    C = iv.candidates(rules, B)
    assert [list(c) for c in C] == [[], [0], [0, 1], [0], [], [2]]


def test_dst_only_ruleset_is_a_stabbing_query():
    """With source, ports and protocol wildcarded, first match = lowest index whose range holds x."""
    rules = gen.make_rules(50, 7, skew=True)
    rules.src_plen[:] = 0
    rules.sport_lo[:] = 0
    rules.sport_hi[:] = 65535
    rules.dport_lo[:] = 0
    rules.dport_hi[:] = 65535
    rules.proto_any[:] = 1
    pk = gen.make_packets(rules, 2000, 7)
    idx, _ = oracle.classify(rules, pk)
    lo, hi = iv.dst_ranges(rules)
    x = pk.dst_ip.astype(np.uint64)
    inside = (lo[None, :] <= x[:, None]) & (x[:, None] <= hi[None, :])
    stab = np.where(inside.any(axis=1), inside.argmax(axis=1), -1)
    np.testing.assert_array_equal(idx, stab)


@pytest.mark.parametrize("seed,skew", [(1, False), (3, True)])
def test_first_match_via_candidates_equals_scan(seed, skew):
    rules = gen.make_rules(80, seed, skew=skew)
    pk = gen.make_packets(rules, 1500, seed)
    B = iv.boundaries(rules)
    C = iv.candidates(rules, B)
    want, _ = oracle.classify(rules, pk)
    np.testing.assert_array_equal(iv.first_match_via_candidates(rules, B, C, pk), want)
    # truncating each list after its first full-match entry changes nothing
    full = iv.full_match_in_interval(rules)
    Ct = [iv.truncated(c, full) for c in C]
    np.testing.assert_array_equal(iv.first_match_via_candidates(rules, B, Ct, pk), want)


# ---------------------------------------------------------------- network oracle

H = 32


def _theta(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, 1.0, rmi.n_params(H))


def test_grad_matches_central_differences():
    rng = np.random.Generator(np.random.PCG64(3))
    th = _theta(3)
    u = rng.random(200)
    t = rng.random(200) * 3
    g = rmi.grad(th, u, t, H)
    h = 1e-6
    fd = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        fd[i] = (rmi.loss(th + e, u, t, H) - rmi.loss(th - e, u, t, H)) / (2 * h)
    assert np.max(np.abs(fd - g)) / np.max(np.abs(g)) <= 1e-6


def test_grad_closed_form_constant_network():
    """With w1 = 0 the network is a constant c; dL/db2 = 2 mean(c - t) and the rest follow."""
    rng = np.random.Generator(np.random.PCG64(4))
    th = _theta(4)
    th[:H] = 0.0                                   # w1 = 0
    u = rng.random(64)
    t = rng.random(64)
    w1, b1, w2, b2 = rmi.split(th, H)
    c = float(np.maximum(b1, 0) @ w2 + b2)
    dc = 2.0 * np.mean(c - t)
    g = rmi.grad(th, u, t, H)
    np.testing.assert_allclose(g[3 * H], dc, rtol=1e-12)
    np.testing.assert_allclose(g[2 * H:3 * H], np.maximum(b1, 0) * dc, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(g[H:2 * H], (b1 > 0) * w2 * dc, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(g[:H], (b1 > 0) * w2 * 2.0 * np.mean((c - t) * u),
                               rtol=1e-12, atol=1e-15)


def test_stage_grad_splits_by_expert():
    rng = np.random.Generator(np.random.PCG64(5))
    th = np.stack([_theta(10 + e) for e in range(4)])
    u = rng.random(300)
    t = rng.random(300)
    ex = rng.integers(0, 4, 300)
    g = rmi.stage_grad(th, u, t, ex, H)
    for e in range(4):
        np.testing.assert_allclose(g[e], rmi.grad(th[e], u[ex == e], t[ex == e], H))
    # an expert with no samples gets a zero gradient
    g2 = rmi.stage_grad(th, u, t, np.zeros(300, int), H)
    assert np.all(g2[1:] == 0)


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2: the step is lr * g / (|g| + eps)."""
    rng = np.random.Generator(np.random.PCG64(6))
    th = rng.normal(size=20)
    g = rng.normal(size=20)
    new, m, v = rmi.adam(th, g, np.zeros(20), np.zeros(20), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_port_masks_against_every_port():
    """Port masks pinned by brute force: for every port value p, the mask of p's interval
    holds exactly the rules whose range contains p (the covering argument on 16 bits)."""
    rng = np.random.Generator(np.random.PCG64(11))
    lo = rng.integers(0, 65536, 40)
    hi = np.minimum(lo + rng.integers(0, 3000, 40), 65535)
    lo[:3] = [0, 0, 65535]
    hi[:3] = [65535, 0, 65535]                      # wildcard, [0,0], [65535,65535]
    B, masks = iv.port_masks(lo, hi)
    assert B[0] == 0 and np.all(np.diff(B) > 0) and B[-1] <= 65535
    ports = np.arange(65536)
    j = np.searchsorted(B, ports, side="right") - 1
    want = np.zeros(65536, dtype=object)
    for k in range(len(lo)):
        inside = (ports >= lo[k]) & (ports <= hi[k])
        want[inside] = want[inside] + (1 << k)
    got = np.array([masks[i] for i in j], dtype=object)
    assert np.array_equal(got, want)


def test_proto_masks_definition():
    pm = iv.proto_masks(np.array([6, 17, 0, 6]), np.array([0, 0, 0, 1]))
    assert pm[6] == 0b1001 and pm[17] == 0b1010 and pm[0] == 0b1100 and pm[1] == 0b1000
