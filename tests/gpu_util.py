"""Shared helpers for the GPU tests: device transfer and one-call classification."""

from __future__ import annotations

import sys

import numpy as np


def say(msg: str):
    """Print and flush a line naming the case before a GPU step."""
    print(msg, flush=True)
    sys.stdout.flush()


def fwmod():
    from paper_1312_4188_amd import fw
    return fw


def classify_np(rules, pk, **kw):
    """Load `rules`, classify host packets `pk` on cuda:0, return numpy (idx, act)."""
    import torch
    fw = fwmod()
    with fw.Ruleset(rules) as rs:
        dp = fw.DevicePackets.from_host(pk)
        idx, act = rs.classify(dp, **kw)[:2]
        torch.cuda.synchronize()
        return idx.cpu().numpy(), act.cpu().numpy()


def assert_same(got, want, what=""):
    gi, ga = got
    wi, wa = want
    bad = np.nonzero((gi != wi) | (ga != wa))[0]
    if bad.size:
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} mismatches; first at {i}: "
                             f"got ({gi[i]}, {ga[i]}) want ({wi[i]}, {wa[i]})")
