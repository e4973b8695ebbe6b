"""The CPU oracle and the library's host-only code built with the address and
undefined-behaviour sanitizers, run on seeded random inputs and edge cases.

tests/sanitize/oracle_checks.c drives oracle/fwref.c (empty rule list, empty and one-packet
batches, 1-17 worker threads, prefix lengths 0-32); tests/sanitize/host_checks.cpp drives the
serving arena, the learned index's candidate lists, port/protocol table and source bucket
table, and the scan plan's grouping (csrc/arena.h, csrc/lists.cpp), each against a
brute-force definition.  Any sanitizer report aborts the program (no recovery)."""

import os
import shutil
import subprocess

import pytest

from tests.conftest import ROOT

SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror"]


def _run(exe):
    # the sanitizer runtime need not be first among preloaded libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_checks"
    subprocess.run(["gcc", "-std=c11", *SAN, "-pthread",
                    os.path.join(ROOT, "tests", "sanitize", "oracle_checks.c"), "-o", str(exe)],
                   check=True)
    assert "oracle checks passed" in _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_sanitizers(tmp_path):
    exe = tmp_path / "host_checks"
    csrc = os.path.join(ROOT, "paper_1312_4188_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", *SAN,
                    os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
                    os.path.join(csrc, "lists.cpp"), "-o", str(exe)], check=True)
    assert "host checks passed" in _run(exe)
