"""CPU checks of bench.py's host logic: the one-GPU guard, the algorithmic
byte counts behind the roofline line, and the source hash that keys the
measured traffic (insensitive to comments, sensitive to code)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_per_launch():
    # 2-D: 60 B per particle + 4 B per stored neighbour entry; the 512^2
    # Taylor-Green rows at 1.6h hold 12 entries
    n = 512 * 512
    assert bench.stage_bytes_2d(n, 12 * n) == 60 * n + 48 * n == 28311552
    # 3-D: 92 B per particle + 4 B per entry (200^3 at 1.6h: 32 entries)
    m = 200 ** 3
    assert bench.stage_bytes_3d(m, 32 * m) == 1.76e9


def test_source_hash_ignores_comments_not_code(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text('int f(int x) {\n    return x + 1;  // one more\n}\nconst char* s = "a // b";\n')
    b.write_text('// header comment\nint f(int x) {\n\n    return x + 1;\n}\nconst char* s = "a // b";  // tail\n')
    c.write_text('int f(int x) {\n    return x + 2;\n}\nconst char* s = "a // b";\n')
    assert bench.source_sha(str(a)) == bench.source_sha(str(b))
    assert bench.source_sha(str(a)) != bench.source_sha(str(c))
    # a "//" inside a string literal is code
    assert bench._code_lines('const char* s = "x // y";') == ['const char* s = "x // y";']


def test_measured_traffic_is_keyed_by_the_current_stage_sources():
    """Every stored traffic figure names the hash of the code it was measured
    on; the figures are bytes per launch."""
    for key, v in bench.TRAFFIC.items():
        assert len(key) == 64 and set(v) == {"2d", "3d"}
        assert all(isinstance(x, int) and x > 0 for x in v.values())
    sha = bench.source_sha(*bench.STAGE_SOURCES)
    assert len(sha) == 64
