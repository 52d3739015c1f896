"""The host's vectorised dependency test against the pairwise definition of
Algorithm 1 applied both ways (Section III-C), on random kernels, at
misaligned table placements and with every instruction set the host has."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_segment_table_equals_pairwise_definition(tmp_path):
    exe = str(tmp_path / "segtable_check")
    src = os.path.join(ROOT, "tests", "hostsan", "segtable_check.cpp")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2401_12377_amd", "csrc")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"] + inc +
                   [src, "-o", exe], check=True)
    out = subprocess.run([exe, "40000"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok"), out.stdout
