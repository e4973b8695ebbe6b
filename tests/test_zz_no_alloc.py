"""fw_classify_multi_noalloc: the multi-chain launch with its descriptors in the library's
static device array.  Called through the C interface, its results must equal
fw_classify_multi's (and the oracle's) on two calls in a row, the second with a smaller
input, so whatever the first call left in the shared array cannot leak into the second."""

import ctypes

import numpy as np
import pytest

import oracle
from synth import gen
from tests.gpu_util import fwmod, say

pytestmark = pytest.mark.gpu


def _items(work):
    import torch
    fw = fwmod()
    items, rss = [], []
    for rules, pk in work:
        rs = fw.Ruleset(rules)
        rss.append(rs)
        n = len(pk)
        items.append((rs, fw.DevicePackets.from_host(pk),
                      torch.full((n,), 7, dtype=torch.int32, device="cuda"),
                      torch.full((n,), 9, dtype=torch.uint8, device="cuda")))
    return items, rss


def _launch(items, no_alloc, stream_ptr, **kw):
    """Both entry points through the C interface with the same options."""
    fw = fwmod()
    arr = fw._chain_array(items)
    opts = fw.MultiOpts(stream_ptr, int(kw.get("packets_per_lane", 0)),
                        int(kw.get("placement", 0)), int(kw.get("rule_tile", 0)), 0)
    lib = fw.load_library()
    fn = lib.fw_classify_multi_noalloc if no_alloc else lib.fw_classify_multi
    st = fn(arr, len(items), ctypes.byref(opts))
    assert st == fw.OK, lib.fw_last_error().decode()


def _results(items):
    return [(oi.cpu().numpy().copy(), oa.cpu().numpy().copy()) for _, _, oi, oa in items]


@pytest.mark.parametrize("kw", [dict(), dict(packets_per_lane=1, placement=1),
                                dict(packets_per_lane=4, placement=2, rule_tile=256),
                                dict(packets_per_lane=2, placement=3)])
def test_noalloc_matches_allocating_entry_point(kw):
    import torch
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    # first call: 40 chains; second call: 6 smaller chains (fewer descriptors, fewer items)
    big = gen.multichain_workload(seed=3, n_chains=40, scale=0.05)
    small = [(r, p.subset(slice(0, max(1, len(p) // 5)))) for r, p in big[5:11]]
    for what, work in (("40 chains", big), ("6 smaller chains", small)):
        items, rss = _items(work)
        torch.cuda.synchronize()
        say(f"no-alloc multi {kw}: {what}, {sum(len(p) for _, p in work)} packets")
        _launch(items, False, sp, **kw)
        torch.cuda.synchronize()
        ref = _results(items)
        for _, _, oi, oa in items:
            oi.fill_(7)
            oa.fill_(9)
        _launch(items, True, sp, **kw)
        torch.cuda.synchronize()
        got = _results(items)
        for c, ((rules, pk), (ri, ra), (gi, ga)) in enumerate(zip(work, ref, got)):
            np.testing.assert_array_equal(gi, ri, err_msg=f"{what} chain {c} idx")
            np.testing.assert_array_equal(ga, ra, err_msg=f"{what} chain {c} act")
            wi, wa = oracle.classify(rules, pk, threads=8)
            np.testing.assert_array_equal(gi, wi, err_msg=f"{what} chain {c} vs oracle")
            np.testing.assert_array_equal(ga, wa, err_msg=f"{what} chain {c} act vs oracle")
        for rs in rss:
            rs.close()


def test_noalloc_rejects_too_many_chains_on_device():
    fw = fwmod()
    lib = fw.load_library()
    arr = (fw.ChainBatch * 1025)()
    assert lib.fw_classify_multi_noalloc(arr, 1025, None) == fw.E_INVAL
    assert "1024" in lib.fw_last_error().decode()


def test_noalloc_with_learned_chains():
    """The no-allocation entry point on chains with learned indexes (the default placement
    routes them through the learned lookup): equal to fw_classify_multi and the oracle, on two
    calls in a row, the second with fewer and smaller chains."""
    import torch
    fw = fwmod()
    stream_ptr = torch.cuda.current_stream().cuda_stream
    work = []
    for c, (R, n) in enumerate([(3000, 60_000), (800, 20_000), (5000, 90_000), (120, 3_000)]):
        rules = gen.make_rules(R, 500 + c, skew=True)
        work.append((rules, gen.make_packets(rules, n, 500 + c)))
    small = [(r, p.subset(slice(0, len(p) // 3))) for r, p in work[1:3]]
    for what, w in (("four chains", work), ("two smaller chains", small)):
        items, rss = _items(w)
        for k, rs in enumerate(rss):
            if k % 2 == 0:
                rs.build_learned_index(epochs1=300, epochs2=600, seed=k)
        torch.cuda.synchronize()
        say(f"no-alloc multi with learned chains: {what}")
        _launch(items, False, stream_ptr)
        torch.cuda.synchronize()
        ref = _results(items)
        for _, _, oi, oa in items:
            oi.fill_(7)
            oa.fill_(9)
        _launch(items, True, stream_ptr)
        torch.cuda.synchronize()
        for c, ((rules, pk), (ri, ra), (gi, ga)) in enumerate(zip(w, ref, _results(items))):
            np.testing.assert_array_equal(gi, ri, err_msg=f"{what} chain {c} idx")
            np.testing.assert_array_equal(ga, ra, err_msg=f"{what} chain {c} act")
            wi, wa = oracle.classify(rules, pk, threads=8)
            np.testing.assert_array_equal(gi, wi, err_msg=f"{what} chain {c} vs oracle")
            np.testing.assert_array_equal(ga, wa, err_msg=f"{what} chain {c} act vs oracle")
        for rs in rss:
            rs.close()
