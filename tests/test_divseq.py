"""The FP64 division sequence of the WENO weights (Newton-Raphson refinement
of a reciprocal estimate, Markstein's final correction; hj_divseq.h) returns
the correctly rounded quotient and reciprocal over the operands the weights
produce, for reciprocal estimates with a relative error up to 2^-14 (the
hardware reciprocal is far closer), built with the host compiler.  The one
exception, the largest double below a power of two as denominator (its
reciprocal within 2^-106 above a rounding tie), is counted apart; a weight
denominator is such a number with probability about 2^-52."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    path = tmp_path_factory.mktemp("divseq") / "divseq_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-o", str(path),
                    os.path.join(HERE, "divseq_check.cpp")], check=True)
    return str(path)


@pytest.mark.parametrize("e", [23, 20, 14])
def test_division_sequence_correctly_rounded(exe, e):
    r = subprocess.run([exe, str(e), "1000000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:]
    assert " 0 mismatches" in r.stdout


def test_a_coarse_estimate_is_caught(exe):
    """With estimates only 2^-6 accurate two Newton steps are not enough: the
    check sees it (so it would see a broken sequence)."""
    r = subprocess.run([exe, "6", "200000"], capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
