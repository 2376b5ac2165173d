"""Host-side checks of bench.py: the one-GPU contract, the roofline
arithmetic and the committed HBM traffic record (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_valu_roofline_arithmetic():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert abs(bench.PEAK_VALU_TOPS - 39.3216) < 1e-9
    faces, ms = 1024256, 0.0582
    r = bench._alu(faces, ms)
    want = faces * bench.VALU_OPS_PER_FACE / (ms / 1e3) / 1e12
    assert r["bound"] == "alu" and abs(r["achieved"] - want) < 1e-9
    assert abs(r["frac"] - want / bench.PEAK_VALU_TOPS) < 1e-12
    # the training roofline's algorithmic work: forward 3104 MAC, deltas of
    # layers 5..2 (the input needs none), weight gradients 3104 MAC
    macs = 6 * 64 + 64 * 32 + 32 * 16 + 16 * 8 + 8 * 4
    assert macs == 3104
    assert bench.TRAIN_FLOP_PER_SAMPLE == 2 * (macs + (macs - 6 * 64) + macs)


def test_traffic_record_is_consistent():
    """The committed FETCH/WRITE record parses; its bytes per launch cover at
    least the algorithmic bytes of a launch (state in, right-hand side out,
    FP32, on the 4096-problem batch) and stay within a few times of them;
    when its source hash matches the tree, bench.py reports it."""
    import json

    from paper_2207_08500_amd import inputs
    line = [ln for ln in open(bench.TRAFFIC_RECORD) if ln.startswith("traffic-record:")][0]
    rec = json.loads(line.split(":", 1)[1])
    scaled = (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024
    assert abs(scaled - rec["bytes_per_launch"]) / rec["bytes_per_launch"] < 1e-3
    cells = int(inputs.uneven_sizes(inputs.BASE_SEED, 4096, 256, 16384).sum())
    assert rec["cells"] == cells
    alg = 2 * 3 * cells * 4
    assert alg <= rec["bytes_per_launch"] < 4 * alg
    got = bench._traffic_record()
    assert got is None or got["bytes_per_launch"] == rec["bytes_per_launch"]


def test_code_digest_ignores_comments_only():
    """The traffic record's digest: comments and layout do not change it,
    code (including string and character literals) does."""
    import bench
    base = 'int f(int a) {\n  return a + 1;  // one\n}\nconst char* s = "// kept";\n'
    same = '/* header */\nint f(int a) { return a + 1; }\n// note\nconst char* s = "// kept";'
    code = 'int f(int a) {\n  return a - 1;  // one\n}\nconst char* s = "// kept";\n'
    lit = 'int f(int a) {\n  return a + 1;  // one\n}\nconst char* s = "// kepT";\n'
    d = {k: bench.code_digest(["x"], read=lambda _, t=t: t)
         for k, t in [("base", base), ("same", same), ("code", code), ("lit", lit)]}
    assert d["base"] == d["same"]
    assert d["base"] != d["code"] and d["base"] != d["lit"]
    assert bench._strip_comments("char c = '\\''; // q") == "char c = '\\'';"


def test_perturbed_half_batch():
    """The benchmark's second 4096-problem batch: problems of even index are
    those of the plain Riemann batch, those of odd index those of the fully
    perturbed one (same draws)."""
    import numpy as np
    import pytest

    from paper_2207_08500_amd import inputs
    sizes = np.array([300, 257, 1000, 64, 5])
    a, off, _ = inputs.riemann1d_batch(9, sizes)
    b, _, _ = inputs.riemann1d_batch(9, sizes, perturb=True)
    c, _, _ = inputs.riemann1d_batch(9, sizes, perturb="odd")
    for i in range(sizes.size):
        want = (b if i % 2 else a)[:, off[i]:off[i + 1]]
        assert np.array_equal(c[:, off[i]:off[i + 1]], want)
        assert not np.array_equal(a[:, off[i]:off[i + 1]], b[:, off[i]:off[i + 1]])
    with pytest.raises(ValueError):
        inputs.riemann1d_batch(9, sizes, perturb="even")
