"""The C interface on the CPU: the library loads, exports what include/fw.h declares,
and rejects bad arguments before touching a device."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "fw.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fw_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def fw():
    from paper_1312_4188_amd import fw as m
    m.load_library()
    return m


def test_exports_every_declared_symbol(fw):
    lib = fw.load_library()
    names = _declared()
    assert "fw_classify" in names and "fw_load_ruleset" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(fw.SIGNATURES)


def _c_layout(tmp_path, structs):
    """sizeof/offsetof of header structs, from a C program compiled against include/fw.h."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fw.h"', 'int main(void){']
    for name, fields in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return dict((k, int(v)) for k, v in (ln.split() for ln in out.splitlines()))


def test_struct_layouts_match_header(fw, tmp_path):
    structs = {"fw_packets": fw.Packets, "fw_classify_opts": fw.ClassifyOpts,
               "fw_index_opts": fw.IndexOpts, "fw_index_stats": fw.IndexStats,
               "fw_server_opts": fw.ServerOpts, "fw_host_packets": fw.HostPackets,
               "fw_request_times": fw.RequestTimes, "fw_chain_batch": fw.ChainBatch,
               "fw_multi_opts": fw.MultiOpts}
    c = _c_layout(tmp_path, {k: [f for f, _ in v._fields_] for k, v in structs.items()} |
                  {"fw_rule": [n for n in fw.RULE_DTYPE.names if n != "_pad"]})
    for name, cls in structs.items():
        assert c[name] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert c[f"{name}.{f}"] == getattr(cls, f).offset, (name, f)
    assert c["fw_rule"] == fw.RULE_DTYPE.itemsize == 24
    for f in fw.RULE_DTYPE.names:
        if f != "_pad":
            assert c[f"fw_rule.{f}"] == fw.RULE_DTYPE.fields[f][1], f


def _rule(**kw):
    r = np.zeros(1, dtype=__import__("paper_1312_4188_amd.fw", fromlist=["x"]).RULE_DTYPE)
    r["sport_hi"] = 65535
    r["dport_hi"] = 65535
    r["proto_any"] = 1
    for k, v in kw.items():
        r[k] = v
    return r


@pytest.mark.parametrize("bad", [dict(src_plen=33), dict(dst_plen=40), dict(sport_lo=5, sport_hi=4),
                                 dict(dport_lo=65535, dport_hi=0), dict(action=2)])
def test_invalid_rules_rejected(fw, bad):
    lib = fw.load_library()
    rec = _rule(**bad)
    h = ctypes.c_void_p(1234)
    st = lib.fw_load_ruleset(rec.ctypes.data, 1, 0, ctypes.byref(h))
    assert st == fw.E_INVAL
    assert h.value is None
    assert lib.fw_last_error().decode()


def test_argument_errors(fw):
    lib = fw.load_library()
    rec = _rule()
    assert lib.fw_load_ruleset(rec.ctypes.data, 1, 0, None) == fw.E_INVAL
    h = ctypes.c_void_p()
    assert lib.fw_load_ruleset(None, 3, 0, ctypes.byref(h)) == fw.E_INVAL
    assert lib.fw_load_ruleset(rec.ctypes.data, 1, 2, ctypes.byref(h)) == fw.E_INVAL
    assert lib.fw_load_ruleset(rec.ctypes.data, (1 << 24) + 1, 0, ctypes.byref(h)) == fw.E_INVAL
    assert lib.fw_classify(None, None, 5, None, None) == fw.E_INVAL
    assert "NULL" in lib.fw_last_error().decode()
    assert lib.fw_ruleset_size(None) == 0
    assert lib.fw_free_ruleset(None) == fw.OK
    assert lib.fw_build_learned_index(None, None, None) == fw.E_INVAL
    assert lib.fw_index_lookup(None, None, 0, None, 0, None) == fw.E_INVAL
    assert lib.fw_index_export(None, 0, None, 0, None) == fw.E_INVAL
    out = ctypes.c_void_p()
    assert lib.fw_server_create(None, 0, None, ctypes.byref(out)) == fw.E_INVAL
    assert out.value is None
    # options are validated before any device work (the chain handle is never touched)
    fake = (ctypes.c_void_p * 1)(1)
    for opts in (fw.ServerOpts(17, 0, 0, 0, 0), fw.ServerOpts(4, 9, 0, 0, 0),
                 fw.ServerOpts(4, 2, 0, 0, 0), fw.ServerOpts(4, 4, 0, 0, 0),
                 fw.ServerOpts(4, 0, 1025, 0, 0), fw.ServerOpts(4, 0, 0, 2, 0)):
        assert lib.fw_server_create(fake, 1, ctypes.byref(opts), ctypes.byref(out)) == fw.E_INVAL
        assert out.value is None
    assert lib.fw_server_submit(None, 0, None, 0, None, None, None) == fw.E_INVAL
    assert lib.fw_server_wait(None, 1, None) == fw.E_INVAL
    assert lib.fw_server_destroy(None) == fw.OK
    assert lib.fw_server_replay(None, 0, None, None, None, None, None, None, None, None) == fw.E_INVAL
    bad = (fw.ChainBatch * 1)()
    assert lib.fw_classify_multi(bad, 1, None) == fw.E_INVAL       # NULL ruleset
    assert lib.fw_classify_multi_noalloc(bad, 1, None) == fw.E_INVAL
    many = (fw.ChainBatch * 1025)()
    assert lib.fw_classify_multi_noalloc(many, 1025, None) == fw.E_INVAL   # over the array
    assert "1024" in lib.fw_last_error().decode()
    assert lib.fw_classify_multi(None, 0, None) == fw.OK           # nothing to do
    assert lib.fw_autotune_multi(None, 3, None, None, None) == fw.E_INVAL
    # closed loop: NULL packet fields are caught before the slices are offset
    # (the ruleset handle is never touched)
    starts = (ctypes.c_size_t * 1)(16)
    counts = (ctypes.c_size_t * 1)(64)
    secs = (ctypes.c_double * 1)()
    assert lib.fw_closed_loop(fake, ctypes.byref(fw.Packets()), 1, starts, counts, None, None,
                              None, secs) == fw.E_INVAL
    assert lib.fw_closed_loop(None, None, 1, starts, counts, None, None, None, secs) == fw.E_INVAL


def test_binding_checks_shapes_before_any_launch(fw):
    """The binding validates what the kernels will read and write (lengths, element sizes,
    contiguity, device) and raises before calling into the library."""
    import torch
    n = 32
    good = [torch.zeros(n, dtype=d) for d in (torch.int32, torch.int32, torch.int16,
                                                torch.int16, torch.uint8)]
    with pytest.raises(ValueError, match="CUDA"):
        fw.DevicePackets(*good).check()               # host tensors
    short = list(good)
    short[3] = torch.zeros(n - 1, dtype=torch.int16)
    with pytest.raises(ValueError):
        fw.DevicePackets(*short).check()
    wide = list(good)
    wide[4] = torch.zeros(n, dtype=torch.int32)
    with pytest.raises(ValueError):
        fw.DevicePackets(*wide).check()
    dev = torch.device("cpu")
    with pytest.raises(ValueError, match="out_idx"):
        fw._check_outputs(torch.zeros(n - 1, dtype=torch.int32), torch.zeros(n, dtype=torch.uint8),
                          n, dev)
    with pytest.raises(ValueError, match="out_act"):
        fw._check_outputs(torch.zeros(n, dtype=torch.int32), torch.zeros(n, dtype=torch.int32),
                          n, dev)
    fw._check_outputs(torch.zeros(n, dtype=torch.int32), torch.zeros(n, dtype=torch.uint8), n, dev)
