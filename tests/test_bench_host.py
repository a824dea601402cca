"""Host-side logic of bench.py (no GPU): the trailing-update launch schedule
its roofline figures are computed over, the keying of the committed
HBM-counter summaries, and the single-GPU guard."""
import os
import subprocess
import sys

import pytest

import bench


def _groups_with_trailing_columns(n, nb, g):
    # the same schedule from its definition: groups of g block columns (the
    # last one possibly short); a group updates the columns to its right
    groups, k0 = [], 0
    while k0 < n:
        w = min(g * nb, n - k0)
        groups.append((k0, w))
        k0 += w
    return [(k0, w) for k0, w in groups if k0 + w < n]


@pytest.mark.parametrize("m,n,nb", [(88320, 65536, 256), (3744, 1600, 128), (700, 300, 64), (517, 517, 256),
                                    (88320, 65536, 96), (777, 300, 96)])
def test_trailing_launches_schedule(m, n, nb):
    g = 4 if 512 % nb == 0 else 1
    got = bench.trailing_launches(m, n, nb)
    want = [(m - k0, n - k0 - w, w) for k0, w in _groups_with_trailing_columns(n, nb, g)]
    assert got == want
    # the inner dimensions partition the columns left of the last group
    assert sum(k for _, _, k in got) + min(g * nb, n - sum(k for _, _, k in got)) == n


def test_trailing_launches_counts():
    assert len(bench.trailing_launches(88320, 65536, 256)) == 63       # 64 groups of 1024 columns
    assert len(bench.trailing_launches(88320, 65536, 96)) == 682       # 683 blocks of 96 (the last 64 wide)
    assert bench.trailing_launches(100, 64, 256) == []                 # one block: no trailing columns


def _traffic_file(tmp_path, launches, key):
    p = tmp_path / "traffic.txt"
    p.write_text("# comment line\nworkload=ct256\nlaunches=%d\ngemm_hip_sha256=%s\nbytes_per_launch=1.5e+10\n"
                 % (launches, key))
    return str(p)


def test_measured_traffic_keys(tmp_path, monkeypatch):
    key = bench.gemm_source_hash()
    monkeypatch.setitem(bench.TRAFFIC_FILES, "bf16x3", _traffic_file(tmp_path, 63, key))
    assert bench.measured_traffic("ct256", "bf16x3", 63) == 1.5e10
    assert bench.measured_traffic("ct256", "bf16x3", 127) is None      # another launch schedule
    assert bench.measured_traffic("ct512", "bf16x3", 63) is None       # another workload
    monkeypatch.setitem(bench.TRAFFIC_FILES, "bf16x3", _traffic_file(tmp_path, 63, "0" * 16))
    assert bench.measured_traffic("ct256", "bf16x3", 63) is None       # the kernel source changed
    monkeypatch.setitem(bench.TRAFFIC_FILES, "bf16x3", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("ct256", "bf16x3", 63) is None


def test_source_hash_ignores_comments_and_split_rule():
    import hashlib
    import re
    path = os.path.join(bench.ROOT, "paper_1907_01891_amd", "csrc", "gemm.hip")
    src = open(path).read()
    assert "\nint gemm_tn_splits(int M, int N, int K)\n{" in src
    body = re.sub(r"\nint gemm_tn_splits\(int M, int N, int K\)\n\{.*?\n\}\n", "\n", src, count=1, flags=re.S)
    assert len(body) < len(src) and "gemm_tn_splits(int M, int N, int K)\n{" not in body
    code = re.sub(r"[ \t]*//[^\n]*", "", body)
    code = "\n".join(line.strip() for line in code.splitlines() if line.strip())
    assert bench.gemm_source_hash() == hashlib.sha256(code.encode()).hexdigest()[:16]
    # comment, blank-line and indentation edits keep the key; a code edit does not
    edited = src.replace("\n{", "\n\n  {  // note", 1)
    assert edited != src and bench.gemm_source_hash(edited) == bench.gemm_source_hash(src)
    assert bench.gemm_source_hash(src.replace("BIGT", "BIGT2")) != bench.gemm_source_hash(src)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
