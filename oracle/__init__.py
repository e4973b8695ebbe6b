"""CPU oracle for the first-match classifier.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the classifier itself never does.  Nothing here shares
code with the GPU library (``paper_1312_4188_amd``), and nothing there is
imported here.

* :func:`classify` -- the sequential first-match scan (``fwref.c``), the
  definition from the paper's Section I (first match, default deny) and
  Section IV (5-tuple rules with wildcard fields).
* :mod:`oracle.intervals` -- destination-address elementary intervals and
  exact per-interval candidate lists, written from their set definitions.
* :mod:`oracle.rmi` -- float64 forward/backward of the two-stage index
  network and the Adam update, for checking the GPU training kernels.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfwref.so")
_lib = None


class _Rules(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("src_ip", ctypes.c_void_p), ("dst_ip", ctypes.c_void_p),
        ("src_plen", ctypes.c_void_p), ("dst_plen", ctypes.c_void_p),
        ("sport_lo", ctypes.c_void_p), ("sport_hi", ctypes.c_void_p),
        ("dport_lo", ctypes.c_void_p), ("dport_hi", ctypes.c_void_p),
        ("proto", ctypes.c_void_p), ("proto_any", ctypes.c_void_p),
        ("action", ctypes.c_void_p),
        ("default_action", ctypes.c_uint8),
    ]


class _Packets(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("src_ip", ctypes.c_void_p), ("dst_ip", ctypes.c_void_p),
        ("sport", ctypes.c_void_p), ("dport", ctypes.c_void_p),
        ("proto", ctypes.c_void_p),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.ref_classify.argtypes = [ctypes.POINTER(_Rules), ctypes.POINTER(_Packets),
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p]
        lib.ref_classify.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def classify(rules, packets, threads: int = 1, with_stats: bool = False):
    """Sequential first match of every packet.

    ``rules`` needs the per-field arrays ``src_ip, src_plen, dst_ip, dst_plen,
    sport_lo, sport_hi, dport_lo, dport_hi, proto, proto_any, action`` and
    ``default_action``; ``packets`` needs ``src_ip, dst_ip, sport, dport,
    proto``.  Returns ``(rule_idx int32, action uint8)`` and, with
    ``with_stats``, also ``(rule checks, field tests)`` summed over packets.
    """
    lib = _load()
    keep = []

    def ptr(a, dt):
        a = _c(a, dt)
        keep.append(a)
        return a.ctypes.data

    n_rules = int(np.asarray(rules.src_ip).shape[0])
    r = _Rules(n_rules,
               ptr(rules.src_ip, np.uint32), ptr(rules.dst_ip, np.uint32),
               ptr(rules.src_plen, np.uint8), ptr(rules.dst_plen, np.uint8),
               ptr(rules.sport_lo, np.uint16), ptr(rules.sport_hi, np.uint16),
               ptr(rules.dport_lo, np.uint16), ptr(rules.dport_hi, np.uint16),
               ptr(rules.proto, np.uint8), ptr(rules.proto_any, np.uint8),
               ptr(rules.action, np.uint8), int(rules.default_action))
    n = int(np.asarray(packets.src_ip).shape[0])
    p = _Packets(n, ptr(packets.src_ip, np.uint32), ptr(packets.dst_ip, np.uint32),
                 ptr(packets.sport, np.uint16), ptr(packets.dport, np.uint16),
                 ptr(packets.proto, np.uint8))
    idx = np.empty(n, dtype=np.int32)
    act = np.empty(n, dtype=np.uint8)
    stats = np.zeros(2, dtype=np.uint64)
    rc = lib.ref_classify(ctypes.byref(r), ctypes.byref(p), idx.ctypes.data,
                          act.ctypes.data, int(threads), stats.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle: could not start worker threads")
    if with_stats:
        return idx, act, (int(stats[0]), int(stats[1]))
    return idx, act
