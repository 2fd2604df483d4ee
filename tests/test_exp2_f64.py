"""The double-precision exp2 of the QMC_FP64 per-point exponentials (csrc/exp2_f64.hpp)
and of the MDI-LR recurrence seeds (csrc/exp2_seed.hpp), compiled for the host with
g++ and checked against the C library's long-double exp2l: within one unit in the last
place over the range |x| <= 1000, exact at integers (powers of two) and at 0; the
seeds' short form within one unit in the last place over |x| <= 1/16, and the seeds'
dispatch between the two forms over the whole range; and the table form of log2
(csrc/log2_tab.hpp) against log2l in absolute error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("exp2") / "exp2_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2404_08867_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "exp2_check.cpp"), "-o", str(out), "-lm"],
                   check=True)
    return str(out)


def _max_ulp(checker, n, lo, hi, form=None):
    r = subprocess.run([checker, str(n), repr(lo), repr(hi)] + ([form] if form else []),
                       capture_output=True, text=True, check=True)
    ulp, x = r.stdout.split()
    return float(ulp), float(x)


@pytest.mark.parametrize("lo,hi,n", [(-1000.0, 1000.0, 2_000_000), (-1.0, 1.0, 1_000_000),
                                     (-0.5, 0.5, 1_000_000), (-64.0, -63.0, 200_000),
                                     (999.0, 1000.0, 100_000), (-1000.0, -999.0, 100_000)])
def test_within_one_ulp(checker, lo, hi, n):
    ulp, x = _max_ulp(checker, n, lo, hi)
    assert ulp <= 1.0, (ulp, x)


@pytest.mark.parametrize("x", [0.0, 1.0, -1.0, 7.0, -300.0, 1000.0, -1000.0])
def test_exact_at_integers(checker, x):
    # one point, the end points lo = hi = x: a power of two is exact
    ulp, _ = _max_ulp(checker, 0, x, x)
    assert ulp == 0.0


@pytest.mark.parametrize("lo,hi,n", [(-0.0625, 0.0625, 2_000_000), (-1e-3, 1e-3, 500_000),
                                     (0.06, 0.0625, 200_000), (-0.0625, -0.06, 200_000)])
def test_seed_small_within_one_ulp(checker, lo, hi, n):
    ulp, x = _max_ulp(checker, n, lo, hi, form="small")
    assert ulp <= 1.0, (ulp, x)


@pytest.mark.parametrize("lo,hi,n", [(-1000.0, 1000.0, 1_000_000), (-1.0, 1.0, 1_000_000),
                                     (-0.07, 0.07, 500_000), (999.0, 1000.0, 100_000),
                                     (-1000.0, -999.0, 100_000)])
def test_seed_within_one_ulp(checker, lo, hi, n):
    ulp, x = _max_ulp(checker, n, lo, hi, form="seed")
    assert ulp <= 1.0, (ulp, x)


@pytest.mark.parametrize("form", ["small", "seed"])
def test_seed_exact_at_zero(checker, form):
    ulp, _ = _max_ulp(checker, 0, 0.0, 0.0, form=form)
    assert ulp == 0.0


@pytest.mark.parametrize("lo,hi,n", [(-0.0434, 0.0434, 200000), (-1e-6, 1e-6, 20000), (1e-12, 0.0434, 20000)])
def test_expm1_small_within_two_ulp(checker, lo, hi, n):
    """e^t - 1 for the double-double ratio step of the FP64 MDI-LR recurrence: relative to
    its (small) result, within two units in the last place over |t| <= 0.0434."""
    ulp, x = _max_ulp(checker, n, lo, hi, form="expm1")
    assert ulp <= 2.0, (ulp, x)


def test_expm1_small_exact_at_zero(checker):
    ulp, _ = _max_ulp(checker, 0, 0.0, 0.0, form="expm1")
    assert ulp == 0.0


@pytest.fixture(scope="module")
def log2_checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("log2") / "log2_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2404_08867_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "log2_check.cpp"), "-o", str(out), "-lm"],
                   check=True)
    return str(out)


@pytest.mark.parametrize("lo,hi,n,bound", [(2.2250738585072014e-308, 1.7e308, 2_000_000, 3.5e-13),
                                           (0.25, 4.0, 1_000_000, 2.7e-13),
                                           (1.0, 202.0, 1_000_000, 2.7e-13)])
def test_log2_table_form_absolute_error(log2_checker, lo, hi, n, bound):
    """The table form of log2 (csrc/log2_tab.hpp) that the FP32c power of the coordinate
    sum takes: the series' first omitted term t^5 / (5 ln 2) <= 2.6e-13 at the table's
    interval edges, plus the rounding of e + log2 T_j (half a unit of 1022 at the range's
    ends), against log2l; (1, 202) spans b + c s of the power sets up to d = 200."""
    r = subprocess.run([log2_checker, str(n), repr(lo), repr(hi)], capture_output=True, text=True, check=True)
    err, x = (float(v) for v in r.stdout.split())
    assert err <= bound, (err, x)


@pytest.mark.parametrize("lo,hi,n", [(2.2250738585072014e-308, 1.7e308, 2_000_000), (0.25, 4.0, 1_000_000),
                                     (0.999, 1.001, 500_000), (1.0, 202.0, 1_000_000)])
def test_log2_table_two_part_form(log2_checker, lo, hi, n):
    """The two-part form hi + lo of the FP64 power: the series to t^6 and the exact split
    of e + r leave only the roundings of the table entries and of r, below 2.5e-16."""
    r = subprocess.run([log2_checker, str(n), repr(lo), repr(hi), "dd"], capture_output=True, text=True,
                       check=True)
    err, x = (float(v) for v in r.stdout.split())
    assert err <= 2.5e-16, (err, x)
