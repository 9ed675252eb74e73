"""The host's chunk rule for enqueueing iterations (next_chunk in
csrc/common.hpp), compiled into a host program and checked on the CPU: the
chunk never exceeds twice the previous one nor the cap, falls back to
doubling while the residual history says nothing, is capped by the
iterations the residual's mean rate still needs (10% margin, one more) less
those in flight, and is 0 exactly when the iterations in flight should
finish the solve.  No GPU is used: the program only calls the inline rule."""
import math
import os
import shutil
import subprocess

import pytest

pytestmark = pytest.mark.cpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = [  # chunk, cap, rnorm, r0norm, target, seen, in_flight
    (2, 64, 1.0, 1.0, 1e-8, 0, 0),
    (2, 64, 0.5, 1.0, 1e-8, 1, 2),
    (32, 64, 2.0, 1.0, 1e-8, 50, 10),
    (32, 64, 1e-4, 1.0, 1e-8, 100, 0),
    (64, 64, 1e-7, 1.0, 1e-8, 100, 20),
    (64, 64, 1.1e-8, 1.0, 1e-8, 100, 64),
    (8, 16, 1e-3, 1.0, 1e-9, 30, 8),
    (16, 16, 5e-9, 1.0, 1e-8, 40, 0),
    (4, 64, 1e-6, 1e-2, 1e-10, 10, 4),
]


def reference(chunk, cap, rnorm, r0norm, target, seen, in_flight):
    grown = min(2 * chunk, cap)
    if not (seen >= 2 and target > 0 and target < rnorm < r0norm):
        return grown
    rate = math.log(rnorm / r0norm) / seen
    need = math.ceil(1.1 * math.log(target / rnorm) / rate) + 1
    left = need - in_flight
    return 0 if left <= 0 else min(int(left), grown)


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("next_chunk")
    src = d / "probe.cpp"
    lines = ['#include "common.hpp"', "#include <cstdio>", "int main() {"]
    for c in CASES:
        lines.append('    printf("%%d\\n", fvpcg::next_chunk(%d, %d, %r, %r, %r, %d, %d));' % c)
    lines += ["    return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = d / "probe"
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", f"-I{ROOT}/include",
                        f"-I{ROOT}/paper_1505_07630_amd/csrc", str(src), "-o", str(exe)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0
    return [int(v) for v in out.stdout.split()]


def test_next_chunk_rule(probe):
    assert len(probe) == len(CASES)
    for c, got in zip(CASES, probe):
        chunk, cap = c[0], c[1]
        assert 0 <= got <= min(2 * chunk, cap), c
        assert got == reference(*c), (c, got)
    # no history, or a residual not below its start: plain doubling
    assert probe[0] == 4 and probe[2] == 64
    # a long way to go: the cap
    assert probe[3] == 64
    # the chunk in flight finishes the solve: wait for it
    assert probe[4] == 0 and probe[5] == 0
    # nothing in flight and the target not met: at least one more iteration
    assert probe[7] >= 1
