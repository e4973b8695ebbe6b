"""The benchmark's algorithmic work count (CPU): checks against a brute-force count."""

import numpy as np

import oracle
from oracle import intervals as iv
from synth import gen
import bench


class _FakeIndex:
    """Exports shaped like the library's learned index, built from the oracle's definitions."""

    def __init__(self, rules):
        wild_dst = np.asarray(rules.dst_plen) == 0
        wild_src = np.asarray(rules.src_plen) == 0
        B = iv.boundaries(rules.subset(np.nonzero(~wild_dst)[0]))
        C = iv.candidates(rules.subset(np.nonzero(~wild_dst)[0]), B)
        dsel = np.nonzero(~wild_dst)[0]
        self.L = [dsel[c] for c in C]
        gsel = np.nonzero(wild_dst & ~wild_src)[0]
        Bs = iv.boundaries(rules.subset(gsel), "src")
        Cs = iv.candidates(rules.subset(gsel), Bs, "src")
        self.S = [gsel[c] for c in Cs]
        self.Gw = np.nonzero(wild_dst & wild_src)[0]
        self.B, self.Bs = B, Bs
        catch = ((np.asarray(rules.sport_lo) == 0) & (np.asarray(rules.sport_hi) == 65535)
                 & (np.asarray(rules.dport_lo) == 0) & (np.asarray(rules.dport_hi) == 65535)
                 & (np.asarray(rules.proto_any) != 0))
        if (catch[self.Gw]).any():                  # the list ends at its first catch-all
            self.Gw = self.Gw[: np.argmax(catch[self.Gw]) + 1]
        self.table = min(64, int((~catch[self.Gw]).sum()))

    def export(self, what):
        off = lambda lists: np.concatenate([[0], np.cumsum([len(x) for x in lists])])
        cat = lambda lists: (np.concatenate(lists) if lists else np.zeros(0, np.int64))
        return {0: self.B, 1: off(self.L), 2: cat(self.L), 4: np.array([3.0, 5.0]),
                6: self.Bs, 7: off(self.S), 8: cat(self.S), 9: self.Gw,
                11: np.array([self.table, 2, 3, 0, 0])}[what]


def test_candidate_checks_match_brute_force():
    rules = gen.make_rules(150, 3, skew=True)
    pk = gen.make_packets(rules, 2000, 3)
    idx, _ = oracle.classify(rules, pk)
    fake = _FakeIndex(rules)
    work = bench.learned_work(fake, pk, idx)
    j = iv.interval_of(fake.B, pk.dst_ip)
    i = iv.interval_of(fake.Bs, pk.src_ip)
    brute = 0
    for p in range(len(pk)):
        for lst in (fake.L[j[p]], fake.S[i[p]], fake.Gw[fake.table:]):
            lst = np.asarray(lst)
            brute += int(np.sum(lst <= idx[p])) if idx[p] >= 0 else len(lst)
    assert work["candidate_checks"] == brute
    assert work["lane_ops"] > 2 * brute


def test_every_global_name_in_bench_resolves():
    """Every module-level name the benchmark's functions read is defined (a missing helper
    would only show at run time on the GPU)."""
    import builtins
    import symtable
    src = open(bench.__file__).read()
    top = symtable.symtable(src, bench.__file__, "exec")
    defined = set(vars(bench))
    missing = []

    def walk(t):
        for s in t.get_symbols():
            if s.is_global() and s.is_referenced() and s.get_name() not in defined \
                    and not hasattr(builtins, s.get_name()):
                missing.append((t.get_name(), s.get_name()))
        for c in t.get_children():
            walk(c)
    for child in top.get_children():
        walk(child)
    assert not missing, missing


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
