"""Reader for the hand-built ruleset fixtures under tests/golden/."""

from __future__ import annotations

import os

import numpy as np

from synth.gen import Packets, Ruleset

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_ACT = {"DROP": 0, "ACCEPT": 1}


def ip(s: str) -> int:
    a, b, c, d = (int(x) for x in s.split("."))
    assert all(0 <= v <= 255 for v in (a, b, c, d))
    return (a << 24) | (b << 16) | (c << 8) | d


def _pfx(s: str):
    base, plen = s.split("/")
    return ip(base), int(plen)


def _range(s: str):
    lo, hi = s.split("-")
    return int(lo), int(hi)


def load(name: str):
    """Return (Ruleset, Packets, expected_idx, expected_action) of a fixture."""
    rules, pkts, exp_i, exp_a = [], [], [], []
    default = 0
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "rule":
                s, sl = _pfx(tok[1])
                d, dl = _pfx(tok[2])
                spl, sph = _range(tok[3])
                dpl, dph = _range(tok[4])
                anyp = tok[5] == "any"
                rules.append((s, sl, d, dl, spl, sph, dpl, dph,
                              0 if anyp else int(tok[5]), int(anyp), _ACT[tok[6]]))
            elif tok[0] == "default":
                default = _ACT[tok[1]]
            elif tok[0] == "packet":
                arrow = tok.index("->")
                s, d, sp, dp, pr = tok[1:arrow]
                pkts.append((ip(s), ip(d), int(sp), int(dp), int(pr)))
                exp_i.append(int(tok[arrow + 1]))
                exp_a.append(_ACT[tok[arrow + 2]])
            else:
                raise ValueError(f"{name}: bad line {line!r}")
    cols = list(zip(*rules)) if rules else [[]] * 11
    dt = [np.uint32, np.uint8, np.uint32, np.uint8, np.uint16, np.uint16, np.uint16,
          np.uint16, np.uint8, np.uint8, np.uint8]
    arr = [np.array(c, dtype=t) for c, t in zip(cols, dt)]
    rs = Ruleset(*arr, default_action=default)
    pc = list(zip(*pkts))
    pk = Packets(np.array(pc[0], np.uint32), np.array(pc[1], np.uint32),
                 np.array(pc[2], np.uint16), np.array(pc[3], np.uint16),
                 np.array(pc[4], np.uint8))
    return rs, pk, np.array(exp_i, np.int32), np.array(exp_a, np.uint8)


def names():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))
