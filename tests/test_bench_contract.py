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


def test_pass_bytes_of_the_scan_system():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2601_23002_amd import workloads as W
    s = W.config_scan(64)[0]
    M, H = 64 ** 3, 64 * 64 * 33
    point, a, b, c = bench.pass_bytes(s, 8, 4, True, False)
    spec = 2 * 8 * H
    assert point == 8 * M + 5 * 8 * M            # phi in; phi_t, v0, c_P, n^a, c_Q out
    assert a == 2 * 8 * M + 4 * spec              # phi_t and n^a in, 4 half spectra out
    assert b == 2 * 4 * spec + spec               # 4 spectra in and out, V_loc in
    assert c == 4 * spec + 4 * 8 * M + 8 * M      # spectra, phi_t, v0, c_P, c_Q in; dE/dphi out
