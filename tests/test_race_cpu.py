"""Alg. 4 by host threads with std::atomic CAS, under ThreadSanitizer: the
tree equals the oracle's, and the sanitizer finds no race in the box
merge; moving the box publication after the CAS is reported."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "race", "alg4_threads.cpp")


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("race") / "alg4_threads")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                        "-o", out, SRC], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("ThreadSanitizer build unavailable: " + r.stderr[-300:])
    return out


def run(binary, t, racy=False):
    n = t.n
    lines = [str(n)] + [str(int(d)) for d in t.delta]
    leaves = t.aabb[n - 1:]
    lines += [repr(float(x)) for x in leaves.reshape(-1)]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([binary] + (["--racy"] if racy else []), input="\n".join(lines),
                       capture_output=True, text=True, env=env, timeout=120)
    return r


@pytest.mark.parametrize("n,dup", [(1, False), (2, False), (7, False), (200, True), (3000, False),
                                   (3000, True)])
def test_threaded_alg4_matches_oracle_without_races(binary, n, dup):
    rng = np.random.default_rng([40, n, dup])
    pts = rng.random((n, 3), dtype=np.float32)
    if dup:
        pts = (np.floor(pts * 4) / 4).astype(np.float32)   # many equal codes
    t = oracle.build(0, pts, 30)
    r = run(binary, t)
    assert r.returncode == 0, r.stderr[-2000:]
    vals = r.stdout.split()
    ni, nt = n - 1, 2 * n - 1
    left = np.array(vals[:ni], np.int64)
    rope = np.array(vals[ni:ni + nt], np.int64)
    boxes = np.array(vals[ni + nt:], np.float32).reshape(nt, 6)
    assert np.array_equal(left, t.left.astype(np.int64))
    assert np.array_equal(rope, t.rope.astype(np.int64))
    assert np.array_equal(boxes, t.aabb)


def test_sanitizer_reports_box_published_after_cas(binary):
    rng = np.random.default_rng(41)
    t = oracle.build(0, rng.random((200, 3), dtype=np.float32), 30)
    r = run(binary, t, racy=True)
    assert r.returncode == 66 and "data race" in r.stderr, r.stderr[-1000:]
