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


def _sources_hash(tmp_path, kernel, header, monkeypatch):
    (tmp_path / "paper_1805_08893_amd" / "csrc").mkdir(parents=True, exist_ok=True)
    (tmp_path / "include").mkdir(exist_ok=True)
    (tmp_path / "paper_1805_08893_amd" / "csrc" / "k.h").write_text(kernel)
    (tmp_path / "include" / "vr.h").write_text(header)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return bench.kernel_source_sha()


def test_kernel_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    """Counters stay valid across comment edits and become stale on any code edit."""
    code = "int f(int x) {\n    return x + 1;\n}\n"
    base = _sources_hash(tmp_path, code, "int g(void);\n", monkeypatch)
    commented = "// adds one\n/* a block\n   comment */\nint f(int x) {   // trailing\n\n    return x + 1;\n}\n"
    assert _sources_hash(tmp_path, commented, "/* api */\nint g(void);\n", monkeypatch) == base
    assert _sources_hash(tmp_path, code.replace("+ 1", "+ 2"), "int g(void);\n", monkeypatch) != base
    assert _sources_hash(tmp_path, code, "int g(int);\n", monkeypatch) != base


def test_comment_stripping_keeps_literals():
    src = 'const char *u = "http://x/*y*/"; // note\nchar c = \'/\'; /* a\n b */ int k = 1; // "q"\n'
    out = bench.strip_c_comments(src)
    assert '"http://x/*y*/"' in out and "'/'" in out and "int k = 1;" in out
    assert "note" not in out and "a\n b" not in out and '"q"' not in out


def test_host_cpu_model_is_text_or_none():
    m = bench.host_cpu_model()
    assert m is None or (isinstance(m, str) and m)


def test_unit_chunks_cut_only_at_unit_starts():
    cuts = [0, 5, 9, 30, 31, 60]
    ch = bench.unit_chunks(70, cuts, 4)
    assert ch[0][0] == 0 and ch[-1][1] == 70
    assert all(a < b for a, b in ch)
    assert all(ch[i][1] == ch[i + 1][0] for i in range(len(ch) - 1))
    assert {b for _, b in ch[:-1]} <= set(cuts)
    assert bench.unit_chunks(10, [0], 8) == [(0, 10)]


def test_all_threads_oracle_leg_adds_up_to_the_whole_draws():
    # every strategy family on a small icosphere: the chunked runs must give
    # the whole draw's invocations (checked inside the leg), and the FIFO
    # comparison point lies between the unique count and 3T
    from paper_1805_08893_amd import vr
    mesh = W.icosphere_mesh(4, 2, "hilbert", swap_frac=0.05)
    sp = W.shader_for_mesh(mesh, W.SHADER_PHONG, 2, num_lights=2)
    strategies = [("naive", vr.VR_NAIVE, 1, 0), ("static_ballot", vr.VR_STATIC_BALLOT, 64, 0),
                  ("static_sort", vr.VR_STATIC_SORT, 64, 0), ("dyn_hash", vr.VR_DYN_HASH, 341, 256),
                  ("dyn_ballot", vr.VR_DYN_BALLOT, 85, 64)]
    r = bench.cpu_oracle_baseline(mesh, sp, strategies, 1, 1)
    assert r["cores"] >= 1 and r["value"] > 0 and r["single_thread"]["cores"] == 1
    U = len(set(mesh.indices.tolist()))
    for k in ("fifo16", "fifo32"):
        m = r["fifo_post_transform_cache"][k]["invocations"]
        assert U <= m <= 3 * mesh.num_tris
    assert set(r["plan_ms_one_thread"]) == {"dyn_hash", "dyn_ballot"}
