"""The node-index division magic of the kernels (host computed multiplier and
shift) equals integer division at the values where a wrong magic would show
first (every small quotient of divisors up to 3000; just below and above
multiples of divisors up to 2^21; the largest index below 2^31); built with
the host compiler."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_divmagic_exact(tmp_path):
    exe = tmp_path / "divmagic_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe),
                    os.path.join(HERE, "divmagic_check.cpp")], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "0 mismatches" in r.stdout
