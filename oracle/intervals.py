"""Elementary address intervals and exact candidate lists.  TEST INFRASTRUCTURE.

Not in the paper: the learned index is this project's addition on top of the
paper's scan.  Everything here is written from set definitions, with no
blocking, splitting or truncation tricks, so a reader can check it by eye
(written for the destination field; `field="src"` applies the same to sources):

* a rule's destination prefix (base, len) covers the addresses whose top
  ``len`` bits equal the base's: the range [lo, hi] with
  lo = base with its low 32-len bits cleared and hi = lo + 2**(32-len) - 1;
* the boundary set B is {0} together with every lo and every hi + 1 that
  still fits in 32 bits, sorted and de-duplicated;
* elementary interval j is [B[j], B[j+1] - 1] (the last ends at 2**32 - 1),
  and an address x lies in the interval j with B[j] <= x < B[j+1];
* the candidate list C_j holds, in ascending rule order, every rule whose
  destination range contains the whole interval j.

Because every lo and every hi + 1 is a boundary, each destination range is a
union of whole intervals, so a packet whose destination lies in interval j
matches rule r's destination field exactly when r is in C_j.  The first match
over C_j therefore equals the first match over the whole list.
"""

from __future__ import annotations

import numpy as np

TOP = 2**32 - 1


def dst_ranges(rules, field: str = "dst"):
    """Per-rule address range [lo, hi] (uint64 arrays) of the `field` ("dst" or "src") prefix."""
    base = np.asarray(getattr(rules, f"{field}_ip"), dtype=np.uint64)
    plen = np.asarray(getattr(rules, f"{field}_plen"), dtype=np.uint64)
    span = np.left_shift(np.uint64(1), np.uint64(32) - plen)        # 2**(32-len)
    lo = (base // span) * span                                       # clear low bits
    hi = lo + span - np.uint64(1)
    return lo, hi


def boundaries(rules, field: str = "dst") -> np.ndarray:
    """Sorted unique boundary set B (uint32) of the `field` prefixes."""
    lo, hi = dst_ranges(rules, field)
    ends = hi[hi < TOP] + np.uint64(1)
    b = np.unique(np.concatenate([np.zeros(1, np.uint64), lo, ends]))
    return b.astype(np.uint32)


def interval_of(B: np.ndarray, x) -> np.ndarray:
    """Index j of the interval holding each address: the largest j with B[j] <= x."""
    return np.searchsorted(B.astype(np.uint64), np.asarray(x, dtype=np.uint64),
                           side="right") - 1


def interval_end(B: np.ndarray) -> np.ndarray:
    """Last address of each interval (uint64)."""
    b = B.astype(np.uint64)
    return np.concatenate([b[1:] - np.uint64(1), np.array([TOP], np.uint64)])


def candidates(rules, B: np.ndarray, field: str = "dst"):
    """C_j for every interval j: list of int64 arrays of rule indices, ascending."""
    lo, hi = dst_ranges(rules, field)
    start = B.astype(np.uint64)
    end = interval_end(B)
    out = []
    for j in range(B.shape[0]):
        cover = (lo <= start[j]) & (end[j] <= hi)
        out.append(np.nonzero(cover)[0])
    return out


def full_match_in_interval(rules) -> np.ndarray:
    """Rules that match every packet whose destination they cover.

    Such a rule leaves source, both ports and protocol unspecified (source
    prefix length 0, both port ranges [0, 65535], any protocol).  Once a
    candidate list reaches one, later entries can never be a first match.
    """
    return ((np.asarray(rules.src_plen) == 0)
            & (np.asarray(rules.sport_lo) == 0) & (np.asarray(rules.sport_hi) == 65535)
            & (np.asarray(rules.dport_lo) == 0) & (np.asarray(rules.dport_hi) == 65535)
            & (np.asarray(rules.proto_any) != 0))


def truncated(cand: np.ndarray, full: np.ndarray) -> np.ndarray:
    """The list up to and including its first full-match entry (the rest is unreachable)."""
    hit = np.nonzero(full[cand])[0]
    return cand if hit.size == 0 else cand[: hit[0] + 1]


def _field_match(rules, r, src, sport, dport, proto) -> bool:
    """Source, port and protocol tests of rule r (destination is implied by the list)."""
    plen = int(rules.src_plen[r])
    if plen and ((int(src) ^ int(rules.src_ip[r])) >> (32 - plen)) != 0:
        return False
    if not (int(rules.sport_lo[r]) <= int(sport) <= int(rules.sport_hi[r])):
        return False
    if not (int(rules.dport_lo[r]) <= int(dport) <= int(rules.dport_hi[r])):
        return False
    return bool(rules.proto_any[r]) or int(rules.proto[r]) == int(proto)


def first_match_via_candidates(rules, B, cand, packets):
    """Per packet: locate its interval, then the first rule of C_j whose other fields match.

    Pure-Python loops: for small inputs only.
    """
    j = interval_of(B, packets.dst_ip)
    out = np.full(len(j), -1, dtype=np.int32)
    for i in range(len(j)):
        for r in cand[j[i]]:
            if _field_match(rules, r, packets.src_ip[i], packets.sport[i],
                            packets.dport[i], packets.proto[i]):
                out[i] = r
                break
    return out


# ---- port/protocol masks of address-wildcard rules (TEST INFRASTRUCTURE)
#
# A rule that leaves both addresses unspecified matches a packet exactly when
# the packet's source port, destination port and protocol pass its tests.  For
# a port field, the same boundary construction as above over [0, 65535] gives
# elementary port intervals, and interval i's mask has bit k set when the k-th
# rule's port range contains the whole interval.  Written from that definition.

PORT_TOP = 65535


def port_boundaries(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """{0} together with every lo and every hi + 1 <= 65535, sorted and de-duplicated."""
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    ends = hi[hi < PORT_TOP] + 1
    return np.unique(np.concatenate([np.zeros(1, np.int64), lo, ends]))


def port_masks(lo: np.ndarray, hi: np.ndarray):
    """Boundaries of one port field and, per interval, the bit mask (python int) of the rules
    (bit k = k-th rule) whose range [lo_k, hi_k] contains the whole interval."""
    B = port_boundaries(lo, hi)
    end = np.concatenate([B[1:] - 1, [PORT_TOP]])
    masks = []
    for i in range(len(B)):
        m = 0
        for k in range(len(lo)):
            if int(lo[k]) <= int(B[i]) and int(end[i]) <= int(hi[k]):
                m |= 1 << k
        masks.append(m)
    return B, masks


def proto_masks(proto: np.ndarray, proto_any: np.ndarray):
    """Per protocol value 0..255, the bit mask of the rules whose protocol test it passes."""
    out = []
    for p in range(256):
        m = 0
        for k in range(len(proto)):
            if int(proto_any[k]) != 0 or int(proto[k]) == p:
                m |= 1 << k
        out.append(m)
    return out
