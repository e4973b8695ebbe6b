"""ctypes binding of ``libfw.so`` (see ``include/fw.h``) over torch device tensors.

Argument marshalling only: every step of classification, index lookup and
network training runs in the library's HIP kernels.  torch supplies device
memory and streams.  There is no CPU fallback: if the library is missing or
a call fails, an exception is raised.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch  # loaded first so libfw.so binds to the HIP runtime torch already uses

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfw.so")

OK, E_INVAL, E_ALIGN, E_NOMEM, E_DEVICE, E_NOINDEX = 0, -1, -2, -3, -4, -5
DROP, ACCEPT = 0, 1
MODE_AUTO, MODE_PACKET_SPLIT, MODE_RULE_SPLIT, MODE_LEARNED, MODE_HYBRID = 0, 1, 2, 3, 4
MODES = {"auto": MODE_AUTO, "packet_split": MODE_PACKET_SPLIT, "rule_split": MODE_RULE_SPLIT,
         "learned": MODE_LEARNED, "hybrid": MODE_HYBRID}

#: The 24-byte rule record of the C interface (fw_rule), as a numpy dtype.
RULE_DTYPE = np.dtype([
    ("src_ip", "<u4"), ("dst_ip", "<u4"),
    ("src_plen", "u1"), ("dst_plen", "u1"), ("proto", "u1"), ("proto_any", "u1"),
    ("sport_lo", "<u2"), ("sport_hi", "<u2"), ("dport_lo", "<u2"), ("dport_hi", "<u2"),
    ("action", "u1"), ("_pad", "u1", (3,)),
])


class Packets(ctypes.Structure):
    _fields_ = [("src_ip", ctypes.c_void_p), ("dst_ip", ctypes.c_void_p),
                ("src_port", ctypes.c_void_p), ("dst_port", ctypes.c_void_p),
                ("proto", ctypes.c_void_p)]


class ClassifyOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("partitions", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("lookup", ctypes.c_uint32),
                ("packets_per_lane", ctypes.c_uint32),
                ("window_misses", ctypes.POINTER(ctypes.c_uint64))]


class IndexOpts(ctypes.Structure):
    _fields_ = [("experts", ctypes.c_uint32), ("hidden", ctypes.c_uint32),
                ("epochs1", ctypes.c_uint32), ("epochs2", ctypes.c_uint32),
                ("lr", ctypes.c_float), ("seed", ctypes.c_uint32), ("train", ctypes.c_uint32),
                ("use_mfma", ctypes.c_uint32), ("zero_error_bounds", ctypes.c_uint32),
                ("mem_budget", ctypes.c_uint64),
                ("stream", ctypes.c_void_p)]


class IndexStats(ctypes.Structure):
    _fields_ = [("n_boundaries", ctypes.c_uint32), ("n_global", ctypes.c_uint32),
                ("n_list_entries", ctypes.c_uint64), ("max_list", ctypes.c_uint32),
                ("err_max", ctypes.c_uint32), ("err_mean", ctypes.c_float),
                ("loss1", ctypes.c_float), ("loss2", ctypes.c_float),
                ("train_ms", ctypes.c_float), ("weights_rounded", ctypes.c_uint32),
                ("device_bytes", ctypes.c_uint64)]


class ChainBatch(ctypes.Structure):
    _fields_ = [("rs", ctypes.c_void_p), ("pk", Packets), ("n", ctypes.c_size_t),
                ("out_rule_idx", ctypes.c_void_p), ("out_action", ctypes.c_void_p)]


class MultiOpts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("packets_per_lane", ctypes.c_uint32),
                ("placement", ctypes.c_uint32), ("rule_tile", ctypes.c_uint32),
                ("_reserved", ctypes.c_uint32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("max_group", ctypes.c_uint32), ("ingest", ctypes.c_uint32),
                ("mem_budget", ctypes.c_uint64), ("max_group_packets", ctypes.c_uint64)]


class HostPackets(ctypes.Structure):
    _fields_ = [("src_ip", ctypes.c_void_p), ("dst_ip", ctypes.c_void_p),
                ("src_port", ctypes.c_void_p), ("dst_port", ctypes.c_void_p),
                ("proto", ctypes.c_void_p)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("submit", ctypes.c_double), ("admit", ctypes.c_double),
                ("done", ctypes.c_double)]


#: Every symbol include/fw.h declares, with (restype, argtypes).
_VP, _SZ, _U32, _U8 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint8
SIGNATURES = {
    "fw_load_ruleset": (ctypes.c_int, [_VP, _U32, _U8, ctypes.POINTER(_VP)]),
    "fw_free_ruleset": (ctypes.c_int, [_VP]),
    "fw_ruleset_size": (_U32, [_VP]),
    "fw_classify": (ctypes.c_int, [_VP, ctypes.POINTER(Packets), _SZ, _VP, _VP]),
    "fw_classify_ex": (ctypes.c_int, [_VP, ctypes.POINTER(Packets), _SZ, _VP, _VP,
                                      ctypes.POINTER(ClassifyOpts)]),
    "fw_build_learned_index": (ctypes.c_int, [_VP, ctypes.POINTER(IndexOpts),
                                              ctypes.POINTER(IndexStats)]),
    "fw_index_lookup": (ctypes.c_int, [_VP, _VP, _SZ, _VP, _U32, _VP]),
    "fw_index_export": (ctypes.c_int, [_VP, _U32, _VP, _SZ, ctypes.POINTER(_SZ)]),
    "fw_rmi_gradients": (ctypes.c_int, [_U32, _U32, _VP, _SZ, _VP, _VP, _VP, _U32, _VP, _VP]),
    "fw_rmi_adam_step": (ctypes.c_int, [_SZ, _VP, _VP, _VP, _VP, _U32, ctypes.c_float,
                                        ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "fw_classify_multi": (ctypes.c_int, [ctypes.POINTER(ChainBatch), _U32,
                                         ctypes.POINTER(MultiOpts)]),
    "fw_classify_multi_noalloc": (ctypes.c_int, [ctypes.POINTER(ChainBatch), _U32,
                                                 ctypes.POINTER(MultiOpts)]),
    "fw_autotune_multi": (ctypes.c_int, [ctypes.POINTER(ChainBatch), _U32, _VP,
                                         ctypes.POINTER(MultiOpts),
                                         ctypes.POINTER(ctypes.c_float)]),
    "fw_server_create": (ctypes.c_int, [ctypes.POINTER(_VP), _U32, ctypes.POINTER(ServerOpts),
                                        ctypes.POINTER(_VP)]),
    "fw_server_submit": (ctypes.c_int, [_VP, _U32, ctypes.POINTER(HostPackets), _SZ, _VP, _VP,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "fw_server_wait": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(RequestTimes)]),
    "fw_server_destroy": (ctypes.c_int, [_VP]),
    "fw_server_replay": (ctypes.c_int, [_VP, _U32, _VP, _VP, _VP, _VP,
                                        ctypes.POINTER(HostPackets), _VP, _VP, _VP]),
    "fw_closed_loop": (ctypes.c_int, [_VP, ctypes.POINTER(Packets), _U32, _VP, _VP, _VP, _VP,
                                      ctypes.POINTER(ClassifyOpts), _VP]),
    "fw_last_error": (ctypes.c_char_p, []),
}

_lib = None


class FwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fw status {status}: {message}")
        self.status = status


def load_library():
    """Load libfw.so once; raises FileNotFoundError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with "
                "python paper_1312_4188_amd/build_lib.py")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != OK:
        raise FwError(status, load_library().fw_last_error().decode())


def rules_to_records(rules) -> np.ndarray:
    """Pack a rule list (an object with per-field arrays, or a RULE_DTYPE array) into fw_rule records."""
    if isinstance(rules, np.ndarray) and rules.dtype == RULE_DTYPE:
        return np.ascontiguousarray(rules)
    n = int(np.asarray(rules.src_ip).shape[0])
    rec = np.zeros(n, dtype=RULE_DTYPE)
    for name in ("src_ip", "dst_ip", "src_plen", "dst_plen", "proto", "proto_any",
                 "sport_lo", "sport_hi", "dport_lo", "dport_hi", "action"):
        rec[name] = np.asarray(getattr(rules, name))
    return rec


def _check_outputs(out_idx: torch.Tensor, out_act: torch.Tensor, n: int, dev):
    """Result buffers: n entries each, contiguous, on the packets' device."""
    for name, t, size in (("out_idx", out_idx, 4), ("out_act", out_act, 1)):
        if t.device != dev or t.dim() != 1 or not t.is_contiguous() or t.shape[0] < n \
                or t.element_size() != size:
            raise ValueError(f"{name} must be a contiguous 1-D tensor of at least {n} "
                             f"{size}-byte elements on {dev}")


def _record_on(stream, tensors):
    """Work enqueued on a side stream uses these tensors: tell torch's allocator, so that
    memory freed by the caller is not handed out again before that work is done."""
    if isinstance(stream, torch.cuda.Stream) and stream != torch.cuda.current_stream():
        for t in tensors:
            t.record_stream(stream)


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


@dataclasses.dataclass
class DevicePackets:
    """Five device tensors, one per header field (bit patterns of uint32/uint16/uint8)."""

    src_ip: torch.Tensor   # int32 storage of uint32 addresses
    dst_ip: torch.Tensor
    sport: torch.Tensor    # int16 storage of uint16 ports
    dport: torch.Tensor
    proto: torch.Tensor    # uint8

    def __len__(self):
        return int(self.src_ip.shape[0])

    @staticmethod
    def from_host(pk, device="cuda") -> "DevicePackets":
        """Copy host arrays (attributes src_ip, dst_ip, sport, dport, proto) to the device."""
        def t(a, view):
            return torch.from_numpy(np.ascontiguousarray(a).view(view)).to(device)
        return DevicePackets(t(pk.src_ip, np.int32), t(pk.dst_ip, np.int32),
                             t(pk.sport, np.int16), t(pk.dport, np.int16),
                             t(pk.proto, np.uint8))

    def slice(self, start: int, stop: int) -> "DevicePackets":
        return DevicePackets(self.src_ip[start:stop], self.dst_ip[start:stop],
                             self.sport[start:stop], self.dport[start:stop],
                             self.proto[start:stop])

    def c_struct(self) -> Packets:
        return Packets(self.src_ip.data_ptr(), self.dst_ip.data_ptr(), self.sport.data_ptr(),
                       self.dport.data_ptr(), self.proto.data_ptr())

    def fields(self):
        return (self.src_ip, self.dst_ip, self.sport, self.dport, self.proto)

    def check(self) -> int:
        """The kernels read len(self) entries of each field: validate that before any launch."""
        n = len(self)
        dev = self.src_ip.device
        for name, t, size in zip(("src_ip", "dst_ip", "sport", "dport", "proto"), self.fields(),
                                 (4, 4, 2, 2, 1)):
            if t.device != dev or dev.type != "cuda":
                raise ValueError(f"packet field {name} must be on {dev} (a CUDA device)")
            if t.dim() != 1 or t.shape[0] != n or not t.is_contiguous():
                raise ValueError(f"packet field {name} must be a contiguous 1-D tensor of {n}")
            if t.element_size() != size:
                raise ValueError(f"packet field {name} must have {size}-byte elements")
        return n


class Ruleset:
    """A device-resident ruleset (fw_load_ruleset) and its optional learned index."""

    def __init__(self, rules, default_action: int | None = None):
        lib = load_library()
        rec = rules_to_records(rules)
        if default_action is None:
            default_action = int(getattr(rules, "default_action", DROP))
        h = ctypes.c_void_p()
        _check(lib.fw_load_ruleset(rec.ctypes.data if rec.size else None, rec.shape[0],
                                   int(default_action), ctypes.byref(h)))
        self._h = h
        self.n_rules = int(rec.shape[0])
        self.default_action = int(default_action)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().fw_free_ruleset(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def size(self) -> int:
        return int(load_library().fw_ruleset_size(self._h))

    def classify(self, pk: DevicePackets, mode="auto", partitions: int = 0, stream=None,
                 out_idx: torch.Tensor | None = None, out_act: torch.Tensor | None = None,
                 lookup: int = 0, packets_per_lane: int = 0, count_misses: bool = False):
        """Enqueue first-match classification; returns (rule_idx int32, action uint8[, misses])."""
        n = pk.check()
        dev = pk.src_ip.device
        if out_idx is None:
            out_idx = torch.empty(n, dtype=torch.int32, device=dev)
        if out_act is None:
            out_act = torch.empty(n, dtype=torch.uint8, device=dev)
        _check_outputs(out_idx, out_act, n, dev)
        _record_on(stream, pk.fields() + (out_idx, out_act))
        misses = ctypes.c_uint64(0)
        opts = ClassifyOpts(MODES[mode] if isinstance(mode, str) else int(mode),
                            int(partitions), _stream_ptr(stream), int(lookup),
                            int(packets_per_lane),
                            ctypes.pointer(misses) if count_misses else None)
        c = pk.c_struct()
        _check(load_library().fw_classify_ex(self._h, ctypes.byref(c), n, out_idx.data_ptr(),
                                             out_act.data_ptr(), ctypes.byref(opts)))
        if count_misses:
            return out_idx, out_act, int(misses.value)
        return out_idx, out_act

    def classify_plain(self, pk: DevicePackets, out_idx=None, out_act=None):
        """fw_classify: mode AUTO on the null stream."""
        n = pk.check()
        dev = pk.src_ip.device
        out_idx = torch.empty(n, dtype=torch.int32, device=dev) if out_idx is None else out_idx
        out_act = torch.empty(n, dtype=torch.uint8, device=dev) if out_act is None else out_act
        _check_outputs(out_idx, out_act, n, dev)
        c = pk.c_struct()
        _check(load_library().fw_classify(self._h, ctypes.byref(c), n, out_idx.data_ptr(),
                                          out_act.data_ptr()))
        return out_idx, out_act

    def build_learned_index(self, experts=0, hidden=0, epochs1=0, epochs2=0, lr=0.0, seed=1,
                            train=True, use_mfma=True, mem_budget=0, stream=None,
                            zero_error_bounds=False) -> dict:
        opts = IndexOpts(experts, hidden, epochs1, epochs2, lr, seed, int(bool(train)),
                         int(bool(use_mfma)), int(bool(zero_error_bounds)), int(mem_budget),
                         _stream_ptr(stream))
        st = IndexStats()
        _check(load_library().fw_build_learned_index(self._h, ctypes.byref(opts),
                                                     ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in IndexStats._fields_}

    def closed_loop(self, pk: DevicePackets, starts, counts, mode="auto", partitions: int = 0,
                    stream=None, packets_per_lane: int = 0, lookup: int = 0) -> np.ndarray:
        """fw_closed_loop: batches [starts[k], starts[k] + counts[k]) one after another, each
        waited for; returns (native enqueue-to-completion seconds per batch, rule_idx, action),
        the outputs holding the last batch's results at their front."""
        n = pk.check()
        st = np.ascontiguousarray(starts, dtype=np.uint64)
        ct = np.ascontiguousarray(counts, dtype=np.uint64)
        if st.shape != ct.shape or (st.size and int((st + ct).max()) > n):
            raise ValueError("every batch [start, start + count) must lie inside the packets")
        cap = int(ct.max()) if ct.size else 1
        dev = pk.src_ip.device
        oi = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        oa = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
        opts = ClassifyOpts(MODES[mode] if isinstance(mode, str) else int(mode), int(partitions),
                            _stream_ptr(stream), int(lookup), int(packets_per_lane), None)
        sec = np.zeros(len(st), dtype=np.float64)
        c = pk.c_struct()
        _check(load_library().fw_closed_loop(self._h, ctypes.byref(c), len(st), st.ctypes.data,
                                             ct.ctypes.data, oi.data_ptr(), oa.data_ptr(),
                                             ctypes.byref(opts), sec.ctypes.data))
        return sec, oi, oa

    def lookup_intervals(self, keys: torch.Tensor, lookup: int = 0, stream=None) -> torch.Tensor:
        if keys.device.type != "cuda" or keys.dim() != 1 or not keys.is_contiguous() \
                or keys.element_size() != 4:
            raise ValueError("keys must be a contiguous 1-D CUDA tensor of 32-bit values")
        out = torch.empty(keys.shape[0], dtype=torch.int32, device=keys.device)
        _record_on(stream, (keys, out))
        _check(load_library().fw_index_lookup(self._h, keys.data_ptr(), keys.shape[0],
                                              out.data_ptr(), int(lookup), _stream_ptr(stream)))
        return out

    _EXPORT = {0: np.uint32, 1: np.uint32, 2: np.uint32, 3: np.uint32, 4: np.uint32,
               5: np.float32, 6: np.uint32, 7: np.uint32, 8: np.uint32, 9: np.uint32,
               10: np.uint8, 11: np.uint32, 12: np.uint16}

    def export(self, what: int) -> np.ndarray:
        lib = load_library()
        size = ctypes.c_size_t(0)
        _check(lib.fw_index_export(self._h, int(what), None, 0, ctypes.byref(size)))
        dt = self._EXPORT[int(what)]
        out = np.empty(size.value // np.dtype(dt).itemsize, dtype=dt)
        _check(lib.fw_index_export(self._h, int(what), out.ctypes.data if out.size else None,
                                   out.nbytes, ctypes.byref(size)))
        return out


def rmi_gradients(params: np.ndarray, u, t, expert, hidden: int, use_mfma: bool = True):
    """Gradient (E, 3H+1) and per-network loss (E,) from the library's training kernels."""
    params = np.ascontiguousarray(params, dtype=np.float32)
    E = params.shape[0]
    u = np.ascontiguousarray(u, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    ex = np.ascontiguousarray(expert, dtype=np.uint32)
    grad = np.zeros_like(params)
    loss = np.zeros(E, dtype=np.float32)
    _check(load_library().fw_rmi_gradients(E, int(hidden), params.ctypes.data, u.shape[0],
                                           u.ctypes.data, t.ctypes.data, ex.ctypes.data,
                                           int(bool(use_mfma)), grad.ctypes.data,
                                           loss.ctypes.data))
    return grad, loss


def rmi_adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One library Adam step; returns new (params, m, v) float32 arrays."""
    p = np.array(params, dtype=np.float32)
    g = np.ascontiguousarray(grad, dtype=np.float32)
    m = np.array(m, dtype=np.float32)
    v = np.array(v, dtype=np.float32)
    _check(load_library().fw_rmi_adam_step(p.size, p.ctypes.data, g.ctypes.data, m.ctypes.data,
                                           v.ctypes.data, int(step), lr, beta1, beta2, eps))
    return p, m, v


def _chain_array(items):
    """items: list of (Ruleset, DevicePackets, out_idx tensor, out_act tensor)."""
    arr = (ChainBatch * len(items))()
    for k, (rs, pk, oi, oa) in enumerate(items):
        n = pk.check()
        _check_outputs(oi, oa, n, pk.src_ip.device)
        arr[k] = ChainBatch(rs.handle.value, pk.c_struct(), n, oi.data_ptr(), oa.data_ptr())
    return arr


def classify_multi(items, stream=None, packets_per_lane=0, placement=0, rule_tile=0,
                   no_alloc=False):
    """One persistent launch over many chains; items as for _chain_array (outputs preallocated).
    ``no_alloc`` calls fw_classify_multi_noalloc (descriptors in the library's static device
    array instead of memory allocated for the call)."""
    arr = _chain_array(items)
    for _, pk, oi, oa in items:
        _record_on(stream, pk.fields() + (oi, oa))
    opts = MultiOpts(_stream_ptr(stream), int(packets_per_lane), int(placement), int(rule_tile), 0)
    lib = load_library()
    fn = lib.fw_classify_multi_noalloc if no_alloc else lib.fw_classify_multi
    _check(fn(arr, len(items), ctypes.byref(opts)))


class MultiBatch:
    """A multi-chain call prepared once: the chains' tensors are checked and the C array of
    fw_chain_batch entries built at construction, so repeated calls marshal only the
    options (the items must stay alive and unchanged while the object is used)."""

    def __init__(self, items):
        self.items = list(items)
        self.arr = _chain_array(self.items)

    def run(self, stream=None, packets_per_lane=0, placement=0, rule_tile=0, no_alloc=False):
        for _, pk, oi, oa in self.items:
            _record_on(stream, pk.fields() + (oi, oa))
        opts = MultiOpts(_stream_ptr(stream), int(packets_per_lane), int(placement),
                         int(rule_tile), 0)
        lib = load_library()
        fn = lib.fw_classify_multi_noalloc if no_alloc else lib.fw_classify_multi
        _check(fn(self.arr, len(self.items), ctypes.byref(opts)))


def autotune_multi(items, stream=None):
    """Time the configuration grid on these chains; returns (options dict, best ms)."""
    arr = _chain_array(items)
    best = MultiOpts()
    ms = ctypes.c_float(0)
    _check(load_library().fw_autotune_multi(arr, len(items), _stream_ptr(stream),
                                            ctypes.byref(best), ctypes.byref(ms)))
    return ({"packets_per_lane": best.packets_per_lane, "placement": best.placement,
             "rule_tile": best.rule_tile}, float(ms.value))


# element sizes of src_ip, dst_ip, sport, dport, proto, rule index and action
_SERVER_ITEMSIZES = (4, 4, 2, 2, 1, 4, 1)


class Server:
    """Continuous-batching server over resident rulesets (fw_server_*).

    ``submit`` takes host arrays (numpy; with ``ingest="mapped"`` they must be views of
    pinned torch tensors, 16-byte aligned) that must stay alive until ``wait`` returns for
    the ticket; it returns the ticket at once.  ``wait`` returns the request's (submit,
    admit, done) times in seconds.
    """

    INGEST = {"copy": 0, "mapped": 1}

    def __init__(self, rulesets, slots: int = 0, mode="auto", mem_budget: int = 0,
                 ingest="copy", max_group: int = 0, max_group_packets: int = 0):
        lib = load_library()
        self._chains = list(rulesets)
        arr = (ctypes.c_void_p * len(self._chains))(*[r.handle.value for r in self._chains])
        opts = ServerOpts(int(slots), MODES[mode] if isinstance(mode, str) else int(mode),
                          int(max_group), self.INGEST[ingest] if isinstance(ingest, str)
                          else int(ingest), int(mem_budget), int(max_group_packets))
        h = ctypes.c_void_p()
        _check(lib.fw_server_create(arr, len(self._chains), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, chain: int, src_ip, dst_ip, sport, dport, proto, out_idx, out_act) -> int:
        arrays = (src_ip, dst_ip, sport, dport, proto, out_idx, out_act)
        for a in arrays:
            if not (isinstance(a, np.ndarray) and a.flags.c_contiguous):
                raise TypeError("server buffers must be C-contiguous numpy arrays")
        n = int(src_ip.shape[0])
        for a, size in zip(arrays, _SERVER_ITEMSIZES):
            if a.ndim != 1 or a.shape[0] != n or a.itemsize != size:
                raise ValueError(f"server buffers must be 1-D arrays of {n} entries with "
                                 "4, 4, 2, 2, 1, 4 and 1-byte elements")
        pk = HostPackets(*(a.ctypes.data for a in arrays[:5]))
        t = ctypes.c_uint64(0)
        _check(load_library().fw_server_submit(self._h, int(chain), ctypes.byref(pk), n,
                                               out_idx.ctypes.data, out_act.ctypes.data,
                                               ctypes.byref(t)))
        self._keep[t.value] = arrays
        return int(t.value)

    def wait(self, ticket: int):
        times = RequestTimes()
        try:
            _check(load_library().fw_server_wait(self._h, int(ticket), ctypes.byref(times)))
        finally:
            self._keep.pop(int(ticket), None)
        return times.submit, times.admit, times.done

    def replay(self, arrival_s, chain, offset, n, pool, out_idx, out_act):
        """Replay an arrival trace (fw_server_replay); returns an (n_req, 3) array of
        (scheduled arrival, admit, done) times in seconds."""
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        ch = np.ascontiguousarray(chain, dtype=np.uint32)
        off = np.ascontiguousarray(offset, dtype=np.uint64)
        cnt = np.ascontiguousarray(n, dtype=np.uint64)
        pool = [np.ascontiguousarray(a) for a in pool]   # kept alive through the call
        total = int(pool[0].shape[0])
        for a, size in zip(list(pool) + [out_idx, out_act], _SERVER_ITEMSIZES):
            if a.ndim != 1 or a.shape[0] != total or a.itemsize != size:
                raise ValueError(f"pool and result arrays must be 1-D with {total} entries and "
                                 "4, 4, 2, 2, 1, 4 and 1-byte elements")
        if not (out_idx.flags.c_contiguous and out_act.flags.c_contiguous):
            raise TypeError("result arrays must be C-contiguous")
        if not (len(arr) == len(ch) == len(off) == len(cnt)) or \
                (len(off) and int((off + cnt).max()) > total):
            raise ValueError("every request [offset, offset + n) must lie inside the pool")
        pk = HostPackets(*(a.ctypes.data for a in pool))
        times = np.zeros((len(arr), 3), dtype=np.float64)
        _check(load_library().fw_server_replay(self._h, len(arr), arr.ctypes.data, ch.ctypes.data,
                                               off.ctypes.data, cnt.ctypes.data, ctypes.byref(pk),
                                               out_idx.ctypes.data, out_act.ctypes.data,
                                               times.ctypes.data))
        return times

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().fw_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
