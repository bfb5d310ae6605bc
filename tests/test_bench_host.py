"""Host-side logic of bench.py, on the CPU.

- The one-GPU rule: any request for more than one GPU, by flag or by a
  launcher's WORLD_SIZE, ends with exit code 2 and a message, before torch
  or the library is loaded.
- The algorithmic bytes per cell behind the roofline: every field a stage
  must read or write once, 8 bytes each (FP64 state U = (h, q, m, W), the bed
  b where there is one).
- The source hash that keys the stored counter traffic: blind to comments
  and blank lines, sensitive to any change of code.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402  (stdlib imports only at module level)


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                          capture_output=True, text=True, env=env, timeout=120)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None),
                                      (["--gpus", "8", "--steps", "3"], None),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = _run(args, env)
    assert r.returncode == 2, (r.returncode, r.stdout, r.stderr)
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_algorithmic_bytes_per_cell():
    # stage 1 reads U^n (4 fields) and the bed, writes U^(1): 9 doubles
    assert bench.bytes_per_cell("win1", True) == 72
    # stage 2 reads U^n, U^(1) and the bed, writes U^{n+1}: 13 doubles
    assert bench.bytes_per_cell("win2", True) == 104
    assert bench.bytes_per_cell("win2", False) == 96
    # the two-pass reduce passes read only
    assert bench.bytes_per_cell("reduce2", True) == 72
    # explicit Heun: 8 and 12 doubles; SGN phi solve: h, q in, phi out
    assert bench.bytes_per_cell("ex1", False) == 64
    assert bench.bytes_per_cell("ex2", False) == 96
    assert bench.bytes_per_cell("sgn_solve", False) == 24
    assert bench.bytes_per_cell("no such kernel", True) == 0


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2510_07539_amd" / "csrc"
    csrc.mkdir(parents=True)
    f = csrc / "k.hpp"
    f.write_text("int a = 1;  // one\n\n// note\nint b = 2;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.src_hash(["k.hpp"])
    f.write_text("// header\nint a = 1;  // changed comment\nint b = 2;\n\n")
    assert bench.src_hash(["k.hpp"]) == h0
    f.write_text("int a = 1;\nint b = 3;\n")
    assert bench.src_hash(["k.hpp"]) != h0


def test_stored_traffic_entries_name_existing_sources():
    csrc = os.path.join(ROOT, "paper_2510_07539_amd", "csrc")
    for e in bench.TRAFFIC:
        for s in e["sources"]:
            assert os.path.isfile(os.path.join(csrc, s)), (e["kernel"], s)
        # the stored total is the sum of the two scaled counter passes
        assert abs(e["bytes_per_launch"] - e["fetch_bytes"] - e["write_bytes"]) <= 1, e
