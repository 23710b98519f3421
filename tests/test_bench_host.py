"""Host-only checks of bench.py: the one-GPU rule, the FP32 operation counts
of the vertex programs, the counter-summary lookup and the host fields of the
CPU baseline (no device work)."""
import os
import subprocess
import sys

import bench
from paper_1805_08893_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_shader_flops_of_the_written_programs():
    # fma = 2, sqrt and divide = 1: MVP 49, Phong-L 80 + 48 L, Offset-K 60 + 9 K
    assert bench.shader_flops(W.make_shader(W.SHADER_MVP, 1)) == 49
    for L in (1, 4, 8, 16):
        assert bench.shader_flops(W.make_shader(W.SHADER_PHONG, 1, num_lights=L)) == 80 + 48 * L
    for K in (1, 64):
        assert bench.shader_flops(W.make_shader(W.SHADER_OFFSET, 1, iterations=K)) == 60 + 9 * K


def test_traffic_lookup_ignores_unknown_kernels():
    assert bench.committed_traffic("no_such_kernel") is None


def test_kernel_source_hash_is_stable():
    a, b = bench.kernel_source_sha(), bench.kernel_source_sha()
    assert a == b and len(a) == 16


def test_host_cpu_model_is_text_or_none():
    m = bench.host_cpu_model()
    assert m is None or (isinstance(m, str) and m)
