"""The block-tile kernel divides the pivot row by one reciprocal and a
one-FMA correction per entry (Markstein's theorem); the same sequence in C
must give exactly x / b on random, adversarial and workload-like operands in
the range where the kernel uses it."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_markstein_quotient_equals_division(tmp_path):
    exe = str(tmp_path / "division_check")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe, os.path.join(HERE, "division_check.c"), "-lm"],
                   check=True)
    out = subprocess.run([exe, "20000000"], capture_output=True, text=True, check=True).stdout.split()
    checked, bad = int(out[0]), int(out[1])
    assert checked > 15_000_000 and bad == 0, (checked, bad)
