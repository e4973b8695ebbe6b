"""Independent helpers for building and brute-forcing test cases.

These restate the rule semantics in a third form (integer ranges computed with
Python ints, and a painter's algorithm over a dense grid) so that the oracle
is checked against something other than itself.
"""

from __future__ import annotations

import numpy as np

from synth.gen import Packets


def prefix_range(base: int, plen: int):
    """[first, last] address of a prefix, by counting: 2**(32-plen) addresses in the block."""
    size = 1 << (32 - plen)
    first = (base // size) * size
    return first, first + size - 1


def rule_box(rules, r: int):
    """The rule as five inclusive integer ranges (src, dst, sport, dport, proto)."""
    s = prefix_range(int(rules.src_ip[r]), int(rules.src_plen[r]))
    d = prefix_range(int(rules.dst_ip[r]), int(rules.dst_plen[r]))
    sp = (int(rules.sport_lo[r]), int(rules.sport_hi[r]))
    dp = (int(rules.dport_lo[r]), int(rules.dport_hi[r]))
    pr = (0, 255) if rules.proto_any[r] else (int(rules.proto[r]),) * 2
    return (s, d, sp, dp, pr)


def in_box(box, point) -> bool:
    return all(lo <= v <= hi for (lo, hi), v in zip(box, point))


def point_inside_only(rules, k: int, rng, tries: int = 200):
    """A header inside rule k's box and outside every earlier box, or None if none was found."""
    boxes = [rule_box(rules, r) for r in range(k + 1)]
    for _ in range(tries):
        p = tuple(int(rng.integers(lo, hi + 1)) for lo, hi in boxes[k])
        if not any(in_box(boxes[r], p) for r in range(k)):
            return p
    return None


def points_to_packets(points) -> Packets:
    c = list(zip(*points))
    return Packets(np.array(c[0], np.uint32), np.array(c[1], np.uint32),
                   np.array(c[2], np.uint16), np.array(c[3], np.uint16),
                   np.array(c[4], np.uint8))


def painter(rules, src_vals, dst_vals, sport_vals, dport_vals, proto_vals):
    """First-match map of a dense grid by painting boxes from the last rule to the first.

    Each later paint overwrites, so after rule 0 is painted each cell holds the
    lowest index whose box contains it; unpainted cells keep -1.  The grid is
    the Cartesian product of the given value lists, in that axis order.
    """
    axes = [np.asarray(v, dtype=np.int64) for v in
            (src_vals, dst_vals, sport_vals, dport_vals, proto_vals)]
    grid = np.full(tuple(len(a) for a in axes), -1, dtype=np.int32)
    for r in range(len(rules) - 1, -1, -1):
        box = rule_box(rules, r)
        sel = [np.nonzero((a >= lo) & (a <= hi))[0] for a, (lo, hi) in zip(axes, box)]
        if any(s.size == 0 for s in sel):
            continue
        grid[np.ix_(*sel)] = r
    mesh = np.meshgrid(*axes, indexing="ij")
    pk = Packets(mesh[0].ravel().astype(np.uint32), mesh[1].ravel().astype(np.uint32),
                 mesh[2].ravel().astype(np.uint16), mesh[3].ravel().astype(np.uint16),
                 mesh[4].ravel().astype(np.uint8))
    return pk, grid.ravel()
