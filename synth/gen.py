"""Random rules and packet headers with the paper's 5-tuple shape.

The paper (Section IV) describes each rule as a 5-tuple of source/destination
IPv4 address, source/destination port and protocol plus an action, where an
unspecified field matches every value, and the list is consulted in insertion
order with first match and default deny (Section I).  It gives no rule or
traffic distribution (its traffic came from a live HPING3 stream, Section IV
Results), so the distributions below are the ones the workload definitions of
this project fix:

* IP fields are CIDR prefixes: a uniform 32-bit base stored *unmasked* (host
  bits below the prefix are left as drawn) and a prefix length uniform over
  {0, 8, 16, 24, 32}; with ``skew=True`` each length is drawn from {24, 32}
  with probability 0.6, else from {0, 8, 16}, uniform within each set.
* Each port field independently: 40% wildcard [0, 65535], 30% exact [a, a],
  30% range [a, min(a + w - 1, 65535)] with a uniform and
  w = clamp(floor(2 ** (12 u)), 1, 4096), u ~ U[0, 1) (log-uniform 1..4096).
* Protocol uniform over {TCP=6, UDP=17, any}; action ACCEPT/DROP 50/50;
  default action DROP (default deny).
* Packets: half are drawn uniformly inside the box of a uniformly chosen rule
  (so their first match is at or before that rule), half uniformly over the
  whole header space (protocol over 0..255).

All values are host-order integers (10.0.0.1 == 0x0A000001).  Randomness comes
from ``numpy.random.Generator(PCG64(seed))`` only; draws happen in a fixed
order so a (size, seed) pair always yields the same arrays.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

#: Seeds declared before any measurement; benchmarks and tests draw from these.
SEEDS = (1, 2, 3, 4, 5)

DROP = 0
ACCEPT = 1
TCP = 6
UDP = 17

_PLENS = np.array([0, 8, 16, 24, 32], dtype=np.uint8)


@dataclasses.dataclass
class Ruleset:
    """An ordered rule list, one numpy array per field (index = priority)."""

    src_ip: np.ndarray      # uint32 base, host bits left as drawn
    src_plen: np.ndarray    # uint8, 0..32, 0 = wildcard
    dst_ip: np.ndarray
    dst_plen: np.ndarray
    sport_lo: np.ndarray    # uint16, inclusive
    sport_hi: np.ndarray
    dport_lo: np.ndarray
    dport_hi: np.ndarray
    proto: np.ndarray       # uint8, meaningful when proto_any == 0
    proto_any: np.ndarray   # uint8, nonzero = any protocol
    action: np.ndarray      # uint8, DROP=0 / ACCEPT=1
    default_action: int = DROP

    def __len__(self) -> int:
        return int(self.src_ip.shape[0])

    def subset(self, index) -> "Ruleset":
        f = {k.name: getattr(self, k.name)[index] for k in dataclasses.fields(self)
             if k.name != "default_action"}
        return Ruleset(default_action=self.default_action, **f)

    def as_records(self) -> np.ndarray:
        """Pack into a numpy structured array with the 24-byte C rule layout."""
        rec = np.zeros(len(self), dtype=RULE_DTYPE)
        for name in ("src_ip", "dst_ip", "src_plen", "dst_plen", "proto", "proto_any",
                     "sport_lo", "sport_hi", "dport_lo", "dport_hi", "action"):
            rec[name] = getattr(self, name)
        return rec


#: Byte layout of one rule as the C interface takes it (24 bytes, host order).
RULE_DTYPE = np.dtype([
    ("src_ip", "<u4"), ("dst_ip", "<u4"),
    ("src_plen", "u1"), ("dst_plen", "u1"), ("proto", "u1"), ("proto_any", "u1"),
    ("sport_lo", "<u2"), ("sport_hi", "<u2"), ("dport_lo", "<u2"), ("dport_hi", "<u2"),
    ("action", "u1"), ("_pad", "u1", (3,)),
])
assert RULE_DTYPE.itemsize == 24


@dataclasses.dataclass
class Packets:
    """A batch of packet headers, structure-of-arrays."""

    src_ip: np.ndarray   # uint32
    dst_ip: np.ndarray   # uint32
    sport: np.ndarray    # uint16
    dport: np.ndarray    # uint16
    proto: np.ndarray    # uint8

    def __len__(self) -> int:
        return int(self.src_ip.shape[0])

    def subset(self, index) -> "Packets":
        return Packets(self.src_ip[index], self.dst_ip[index], self.sport[index],
                       self.dport[index], self.proto[index])


def _draw_plen(rng: np.random.Generator, n: int, skew: bool) -> np.ndarray:
    if not skew:
        return _PLENS[rng.integers(0, 5, size=n)]
    long_ = rng.random(n) < 0.6
    hi = np.where(rng.integers(0, 2, size=n) == 0, 24, 32)
    lo = np.array([0, 8, 16])[rng.integers(0, 3, size=n)]
    return np.where(long_, hi, lo).astype(np.uint8)


def _draw_ports(rng: np.random.Generator, n: int):
    kind = rng.random(n)                      # <0.4 wildcard, <0.7 exact, else range
    a = rng.integers(0, 65536, size=n)
    u = rng.random(n)
    w = np.clip(np.floor(np.exp2(12.0 * u)), 1, 4096).astype(np.int64)
    lo = np.where(kind < 0.4, 0, a)
    hi = np.where(kind < 0.4, 65535, np.where(kind < 0.7, a, np.minimum(a + w - 1, 65535)))
    return lo.astype(np.uint16), hi.astype(np.uint16)


def make_rules(n_rules: int, seed: int, skew: bool = False,
               default_action: int = DROP) -> Ruleset:
    """Draw ``n_rules`` rules.  ``skew`` selects the /24-/32-heavy prefix mix."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(n_rules)
    src_ip = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    src_plen = _draw_plen(rng, n, skew)
    dst_ip = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    dst_plen = _draw_plen(rng, n, skew)
    sport_lo, sport_hi = _draw_ports(rng, n)
    dport_lo, dport_hi = _draw_ports(rng, n)
    pk = rng.integers(0, 3, size=n)           # 0 -> TCP, 1 -> UDP, 2 -> any
    proto = np.where(pk == 0, TCP, np.where(pk == 1, UDP, 0)).astype(np.uint8)
    proto_any = (pk == 2).astype(np.uint8)
    action = rng.integers(0, 2, size=n).astype(np.uint8)
    return Ruleset(src_ip, src_plen, dst_ip, dst_plen, sport_lo, sport_hi,
                   dport_lo, dport_hi, proto, proto_any, action, default_action)


def _uniform_in_prefix(rng, base: np.ndarray, plen: np.ndarray) -> np.ndarray:
    """Uniform address inside the prefix (base, plen): the generator's own view of a box."""
    size = np.left_shift(np.uint64(1), (32 - plen.astype(np.uint64)))
    first = base.astype(np.uint64) & ~(size - np.uint64(1)) & np.uint64(0xFFFFFFFF)
    off = rng.integers(0, size, dtype=np.uint64)
    return (first + off).astype(np.uint32)


def make_packets(rules: Ruleset, n_packets: int, seed: int,
                 box_fraction: float = 0.5) -> Packets:
    """Draw ``n_packets`` headers: ``box_fraction`` inside a random rule's box, the rest uniform."""
    rng = np.random.Generator(np.random.PCG64(seed + 0x9E3779B9))
    n = int(n_packets)
    R = len(rules)
    in_box = (rng.random(n) < box_fraction) if R > 0 else np.zeros(n, dtype=bool)
    # uniform part
    src = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    dst = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    sport = rng.integers(0, 65536, size=n).astype(np.uint16)
    dport = rng.integers(0, 65536, size=n).astype(np.uint16)
    proto = rng.integers(0, 256, size=n).astype(np.uint8)
    idx = np.nonzero(in_box)[0]
    if idx.size:
        k = rng.integers(0, R, size=idx.size)
        src[idx] = _uniform_in_prefix(rng, rules.src_ip[k], rules.src_plen[k])
        dst[idx] = _uniform_in_prefix(rng, rules.dst_ip[k], rules.dst_plen[k])
        sport[idx] = rng.integers(rules.sport_lo[k].astype(np.int64),
                                  rules.sport_hi[k].astype(np.int64) + 1).astype(np.uint16)
        dport[idx] = rng.integers(rules.dport_lo[k].astype(np.int64),
                                  rules.dport_hi[k].astype(np.int64) + 1).astype(np.uint16)
        any_ = rules.proto_any[k] != 0
        pr = rules.proto[k].copy()
        pr[any_] = rng.integers(0, 256, size=int(any_.sum())).astype(np.uint8)
        proto[idx] = pr
    return Packets(src, dst, sport, dport, proto)


#: Named single-chain workloads: (rules, packets, skewed prefix lengths).
WORKLOADS = {
    "scan_100x10k": (100, 10_000, False),
    "scan_1000x1M": (1_000, 1_048_576, False),
    "learned_10000x16M": (10_000, 16_777_216, True),
}


def workload(name: str, seed: int = 1, n_packets: int | None = None):
    """Return (Ruleset, Packets) of a named workload; ``n_packets`` overrides the batch size."""
    n_rules, n_pk, skew = WORKLOADS[name]
    rules = make_rules(n_rules, seed, skew=skew)
    pk = make_packets(rules, n_pk if n_packets is None else n_packets, seed)
    return rules, pk


def _log_uniform_int(rng, lo: int, hi: int, size: int) -> np.ndarray:
    v = np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))
    return np.clip(np.round(v), lo, hi).astype(np.int64)


def multichain_workload(seed: int = 1, n_chains: int = 64,
                        rules_range=(32, 8192), packets_range=(4096, 1_048_576),
                        scale: float = 1.0):
    """Many independent chains of uneven size: a list of (Ruleset, Packets).

    Rule counts and batch sizes are log-uniform over the given ranges; ``scale``
    shrinks every batch (for quick tests) without changing the rule counts.
    """
    rng = np.random.Generator(np.random.PCG64(seed + 7777))
    nr = _log_uniform_int(rng, *rules_range, n_chains)
    npk = _log_uniform_int(rng, *packets_range, n_chains)
    out = []
    for c in range(n_chains):
        rs = make_rules(int(nr[c]), seed * 1000 + c)
        pk = make_packets(rs, max(1, int(npk[c] * scale)), seed * 1000 + c)
        out.append((rs, pk))
    return out


def serving_chains(seed: int = 1, sizes=(2_000, 10_000, 50_000)):
    """Resident chains for the serving loop."""
    return [make_rules(n, seed * 100 + i, skew=True) for i, n in enumerate(sizes)]


def serving_arrivals(seed: int, n_requests: int, rate_per_s: float,
                     batch_range=(64, 65_536), n_chains: int = 3):
    """Poisson arrival times (s), batch sizes (log-uniform) and target chain per request."""
    rng = np.random.Generator(np.random.PCG64(seed + 4242))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    sizes = _log_uniform_int(rng, *batch_range, n_requests)
    chain = rng.integers(0, n_chains, size=n_requests)
    return t, sizes, chain


def concat_rulesets(parts) -> Ruleset:
    f = {}
    for k in dataclasses.fields(Ruleset):
        if k.name == "default_action":
            continue
        f[k.name] = np.concatenate([getattr(p, k.name) for p in parts])
    return Ruleset(default_action=parts[0].default_action, **f)
