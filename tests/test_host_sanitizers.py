"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two small driver programs are built with gcc/g++ and -fsanitize=address,
undefined (any report aborts the program):
  * the C oracle (seeding, every request kind on several threads, the x-part
    stepping, Berlekamp-Massey, primitivity, polynomial jump-ahead);
  * libxg's host-only sources (the batch planner and the jump polynomials,
    which include no HIP header), whose jump polynomials must also equal the
    oracle's z^J mod P;
  * the request server's output pool, fuzzed against a brute-force model;
  * the tuning cache's file reader on thousands of damaged files, and its
    put / get from several threads;
  * the jump polynomials' lazy initialisation under ThreadSanitizer.
"""
import os
import shutil
import subprocess

import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1108_0486_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _run(cmd, tmp_path, *args):
    exe = str(tmp_path / "a.out")
    subprocess.run(cmd + ["-o", exe], check=True, cwd=ROOT)
    p = subprocess.run([exe, *args], capture_output=True, text=True, timeout=120, env=ENV)
    assert p.returncode == 0 and p.stdout.rstrip().endswith("OK"), p.stdout + p.stderr
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr
    return p.stdout


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    cmd = ["gcc", "-std=gnu11", "-mpclmul", "-msse4.1", *SAN, os.path.join(HERE, "sanitize", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "xorgens_oracle.c"), os.path.join(ROOT, "oracle", "gf2.c"),
           "-lpthread", "-lm"]
    _run(cmd, tmp_path)


def test_host_library_code_under_sanitizers(tmp_path):
    _need("g++")
    cmd = ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "sanitize", "host_driver.cpp"), os.path.join(CSRC, "xg_plan.cpp"),
           os.path.join(CSRC, "xg_jump.cpp")]
    Js = [1, 63, 2047, 2048, 4095, 4096, 4097, 123456789, 10**12, (1 << 64) - 1]
    members = {0: O.PAPER, 1: O.R64, 2: O.W64}               # XG_FAMILY_* -> the oracle's parameters
    out = _run(cmd, tmp_path, *["%d:%d" % (f, J) for f in members for J in Js])
    got = {(int(t[1]), int(t[2])): int(t[3], 16) for t in (l.split() for l in out.splitlines()) if t and t[0] == "J"}
    assert sorted(got) == sorted((f, J) for f in members for J in Js)
    for f, p in members.items():
        P = O.charpoly(p)
        for J in Js:
            assert got[(f, J)] == O.z_pow_mod(J, P), (f, J)


def test_server_pool_under_sanitizers(tmp_path):
    """The server's output pool against a brute-force occupancy model."""
    _need("g++")
    cmd = ["g++", "-std=c++17", *SAN, "-I", CSRC, os.path.join(HERE, "sanitize", "pool_driver.cpp")]
    _run(cmd, tmp_path)


def test_tune_cache_under_sanitizers(tmp_path):
    """The tuning cache's JSON reader on damaged files (each loads or is
    refused whole) and concurrent put / get, under ASan and UBSan."""
    _need("g++")
    cmd = ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "sanitize", "tune_driver.cpp"), os.path.join(CSRC, "xg_tune.cpp"), "-lpthread"]
    _run(cmd, tmp_path, str(tmp_path))


def test_tune_cache_under_thread_sanitizer(tmp_path):
    _need("g++")
    exe = str(tmp_path / "tt")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, os.path.join(HERE, "sanitize", "tune_driver.cpp"), os.path.join(CSRC, "xg_tune.cpp"),
                    "-o", exe, "-lpthread"], check=True, cwd=ROOT)
    p = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert p.returncode == 0 and p.stdout.strip().endswith("OK"), p.stdout + p.stderr
    assert "ThreadSanitizer" not in p.stderr, p.stderr


def test_jump_polynomials_under_thread_sanitizer(tmp_path):
    """Eight threads make the first calls for every member at once (the moduli
    are built lazily, once per process); ThreadSanitizer must stay silent and
    every thread's z^J mod P must equal a later single-threaded one."""
    _need("g++")
    exe = str(tmp_path / "jt")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, os.path.join(HERE, "sanitize", "jump_threads.cpp"), os.path.join(CSRC, "xg_jump.cpp"),
                    "-o", exe, "-lpthread"], check=True, cwd=ROOT)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert p.returncode == 0 and p.stdout.strip().endswith("OK"), p.stdout + p.stderr
    assert "ThreadSanitizer" not in p.stderr, p.stderr
