"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, and the algorithmic byte counts per pass follow the
pass formulas (one evaluation of the 64^3 scan system)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_pass_bytes_follow_the_three_pass_model():
    """Per grid point of one FP64 evaluation with four fields: pass A
    8 (phi) + 32 (half spectra), pass B 64 + 8 (V_loc), pass C 32 + 16 --
    160 B in all, 168 with the trial direction d -- up to the Nyquist
    column (33 of 64 complex columns per half spectrum); FP32 half."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2601_23002_amd import workloads as W
    s = W.config_scan(64)[0]
    M, H = 64 ** 3, 64 * 64 * 33
    spec = 2 * 8 * H
    a, b, c = bench.pass_bytes(s, 8, 4, True, False)
    assert a == 8 * M + 4 * spec
    assert b == 2 * 4 * spec + spec
    assert c == 4 * spec + 2 * 8 * M
    at, bt, ct = bench.pass_bytes(s, 8, 4, True, True)
    assert at == a + 8 * M and bt == b and ct == c
    # 160 B per point plus the Nyquist column of the 17 half-spectrum crossings
    assert a + b + c == 160 * M + 17 * 16 * 64 * 64
    a4, b4, c4 = bench.pass_bytes(s, 4, 4, True, False)
    assert 2 * (a4 + b4 + c4) == a + b + c


def test_unknown_leg_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--legs", "nope"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
