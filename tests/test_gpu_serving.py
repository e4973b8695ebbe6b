"""The serving loop: continuous batching over resident chains.

Each request's result must be identical whether it runs alone or in the mix
with others in flight, and identical to the CPU oracle (tolerance 0:
classification is exact).
"""

import numpy as np
import pytest

import oracle
from synth import gen
from tests.gpu_util import fwmod, say

pytestmark = pytest.mark.gpu


def _pinned(a):
    import torch
    t = torch.empty(a.shape[0], dtype={1: torch.uint8, 2: torch.int16, 4: torch.int32}[a.itemsize],
                    pin_memory=True)
    v = t.numpy().view(a.dtype)
    v[:] = a
    return t, v


def _requests(chains, n_req, seed, max_batch=20_000):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_req):
        c = int(rng.integers(0, len(chains)))
        n = int(np.clip(np.exp(rng.uniform(np.log(64), np.log(max_batch))), 64, max_batch))
        pk = gen.make_packets(chains[c], n, seed * 1000 + k)
        out.append((c, pk))
    return out


def _run(server, reqs):
    """Prepare every request's pinned buffers first (results too: mapped ingest writes them
    in place), then submit them back to back."""
    keep = []
    for c, pk in reqs:
        bufs = [_pinned(a) for a in (pk.src_ip, pk.dst_ip, pk.sport, pk.dport, pk.proto)]
        oi = _pinned(np.full(len(pk), -7, np.int32))
        oa = _pinned(np.full(len(pk), 9, np.uint8))
        bufs += [oi, oa]
        keep.append((c, bufs[:5], oi[1], oa[1]))
    tickets = [server.submit(c, *[b[1] for b in bufs], oi, oa) for c, bufs, oi, oa in keep]
    times = [server.wait(t) for t in tickets]
    return [(k[2], k[3]) for k in keep], times


@pytest.mark.parametrize("ingest,slots,max_group", [("copy", 1, 0), ("copy", 4, 0),
                                                    ("mapped", 4, 0), ("mapped", 3, 5),
                                                    ("copy", 16, 2)])
def test_mix_equals_alone_equals_oracle(ingest, slots, max_group):
    fw = fwmod()
    chains = [gen.make_rules(n, 70 + i, skew=True) for i, n in enumerate((200, 1000, 3000))]
    rs = [fw.Ruleset(c) for c in chains]
    rs[1].build_learned_index(epochs1=300, epochs2=600)
    reqs = _requests(chains, 48, 5)
    say(f"serving: mix of 48 requests over 3 chains, {slots} slots, ingest={ingest}, "
        f"max_group={max_group}")
    with fw.Server(rs, slots=slots, ingest=ingest, max_group=max_group) as sv:
        mix, times = _run(sv, reqs)
    say("serving: the same requests one at a time")
    with fw.Server(rs, slots=1) as sv:
        alone = []
        for r in reqs:
            res, _ = _run(sv, [r])
            alone.append(res[0])
    for k, ((c, pk), m, a) in enumerate(zip(reqs, mix, alone)):
        want = oracle.classify(chains[c], pk)
        np.testing.assert_array_equal(m[0], a[0], err_msg=f"request {k} idx mix vs alone")
        np.testing.assert_array_equal(m[1], a[1], err_msg=f"request {k} action mix vs alone")
        np.testing.assert_array_equal(m[0], want[0], err_msg=f"request {k} vs oracle")
        np.testing.assert_array_equal(m[1], want[1], err_msg=f"request {k} action vs oracle")
    # work overlapped: some request was admitted before an earlier one finished
    spans = sorted((t[1], t[2]) for t in times)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert all(t[0] <= t[1] <= t[2] for t in times)
    for r in rs:
        r.close()


def test_memory_budget_admission():
    fw = fwmod()
    chains = [gen.make_rules(500, 81)]
    rs = [fw.Ruleset(chains[0])]
    reqs = _requests(chains, 20, 6, max_batch=8192)
    budget = 8192 * 18 + 8 * 256        # room for about one of the largest requests
    say("serving: tight memory budget")
    with fw.Server(rs, slots=4, mem_budget=budget) as sv:
        res, times = _run(sv, reqs)
        big = gen.make_packets(chains[0], 20_000, 3)
        oi = np.empty(20_000, np.int32)
        oa = np.empty(20_000, np.uint8)
        with pytest.raises(fw.FwError) as ei:
            sv.submit(0, big.src_ip, big.dst_ip, big.sport, big.dport, big.proto, oi, oa)
        assert ei.value.status == fw.E_NOMEM
    # admitted groups never held more than the budget at once
    for (c, pk), (i, a) in zip(reqs, res):
        want = oracle.classify(chains[c], pk)
        np.testing.assert_array_equal(i, want[0])
        np.testing.assert_array_equal(a, want[1])
    rs[0].close()


def test_empty_request_and_bad_chain():
    fw = fwmod()
    rs = [fw.Ruleset(gen.make_rules(10, 1))]
    with fw.Server(rs, slots=2) as sv:
        e = np.empty(0, np.uint32)
        t = sv.submit(0, e, e, np.empty(0, np.uint16), np.empty(0, np.uint16),
                      np.empty(0, np.uint8), np.empty(0, np.int32), np.empty(0, np.uint8))
        sv.wait(t)
        with pytest.raises(fw.FwError) as ei:
            sv.submit(3, e, e, np.empty(0, np.uint16), np.empty(0, np.uint16),
                      np.empty(0, np.uint8), np.empty(0, np.int32), np.empty(0, np.uint8))
        assert ei.value.status == fw.E_INVAL
        # buffers of unequal length or the wrong element size never reach the library
        a = np.zeros(64, np.uint32)
        with pytest.raises(ValueError):
            sv.submit(0, a, a, np.zeros(63, np.uint16), np.zeros(64, np.uint16),
                      np.zeros(64, np.uint8), np.zeros(64, np.int32), np.zeros(64, np.uint8))
        with pytest.raises(ValueError):
            sv.submit(0, a, a, np.zeros(64, np.uint16), np.zeros(64, np.uint16),
                      np.zeros(64, np.uint8), np.zeros(64, np.int64), np.zeros(64, np.uint8))
        pool = [a, a, np.zeros(64, np.uint16), np.zeros(64, np.uint16), np.zeros(64, np.uint8)]
        with pytest.raises(ValueError):   # a request past the end of the pool
            sv.replay([0.0], [0], [32], [64], pool, np.zeros(64, np.int32), np.zeros(64, np.uint8))
    rs[0].close()


def test_serving_chains_of_2k_10k_50k_rules():
    """The serving chains of 2,000, 10,000 and 50,000 skewed rules, each with its learned
    index: 40 requests of log-uniform size (64..65,536 packets) give, request by request,
    the same results in the mix (four slots) as alone (one slot), and the oracle's."""
    fw = fwmod()
    chains = gen.serving_chains(1)
    rs = [fw.Ruleset(c) for c in chains]
    for r in rs:
        r.build_learned_index(seed=1)
    reqs = _requests(chains, 40, 11, max_batch=65_536)
    say("serving: 40 requests over the 2k/10k/50k-rule chains, 4 slots")
    with fw.Server(rs, slots=4) as sv:
        mix, _ = _run(sv, reqs)
    say("serving: the same requests one at a time")
    with fw.Server(rs, slots=1) as sv:
        alone = [_run(sv, [r])[0][0] for r in reqs]
    for k, ((c, pk), m, a) in enumerate(zip(reqs, mix, alone)):
        want = oracle.classify(chains[c], pk, threads=16)
        np.testing.assert_array_equal(m[0], a[0], err_msg=f"request {k} idx mix vs alone")
        np.testing.assert_array_equal(m[1], a[1], err_msg=f"request {k} action mix vs alone")
        np.testing.assert_array_equal(m[0], want[0], err_msg=f"request {k} vs oracle")
        np.testing.assert_array_equal(m[1], want[1], err_msg=f"request {k} action vs oracle")
    for r in rs:
        r.close()


def test_server_options_and_modes():
    """Packet-split mode ignores built indexes, learned mode needs one on every chain, and the
    split forms are refused (groups run as one multi-chain launch); mapped ingest refuses
    buffers that are not 16-byte aligned.  Results against the oracle."""
    fw = fwmod()
    chains = [gen.make_rules(n, 90 + i, skew=True) for i, n in enumerate((500, 2000))]
    rs = [fw.Ruleset(c) for c in chains]
    rs[0].build_learned_index(epochs1=300, epochs2=600)
    reqs = _requests(chains, 12, 7, max_batch=5000)
    for mode in ("packet_split", "auto"):
        say(f"serving mode {mode}")
        with fw.Server(rs, mode=mode) as sv:
            res, _ = _run(sv, reqs)
        for (c, pk), (i, a) in zip(reqs, res):
            want = oracle.classify(chains[c], pk)
            np.testing.assert_array_equal(i, want[0])
            np.testing.assert_array_equal(a, want[1])
    with pytest.raises(fw.FwError) as ei:
        fw.Server(rs, mode="learned")
    assert ei.value.status == fw.E_NOINDEX
    rs[1].build_learned_index(epochs1=300, epochs2=600)
    say("serving mode learned")
    with fw.Server(rs, mode="learned", ingest="mapped", slots=2) as sv:
        res, _ = _run(sv, reqs)
    for (c, pk), (i, a) in zip(reqs, res):
        want = oracle.classify(chains[c], pk)
        np.testing.assert_array_equal(i, want[0])
        np.testing.assert_array_equal(a, want[1])
    for mode in ("rule_split", "hybrid"):
        with pytest.raises(fw.FwError) as ei:
            fw.Server(rs, mode=mode)
        assert ei.value.status == fw.E_INVAL
    with fw.Server(rs, ingest="mapped") as sv:
        t, a = _pinned(np.zeros(80, np.uint32))
        b = a[1:65]                                  # 4 bytes past an aligned start
        with pytest.raises(fw.FwError) as ei:
            sv.submit(0, b, a[:64], np.zeros(64, np.uint16), np.zeros(64, np.uint16),
                      np.zeros(64, np.uint8), np.zeros(64, np.int32), np.zeros(64, np.uint8))
        assert ei.value.status == fw.E_ALIGN
    for r in rs:
        r.close()
