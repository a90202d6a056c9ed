"""Host check of the kernels' table-driven exponential (exp_tab in csrc/stage.h).

The function's source is taken from stage.h as it stands, compiled for the host
with g++ (its builtins -- fma, rint, ldexp, fmax -- round as the GPU's
instructions do) and compared with long-double expl on seeded arguments over
[-700, 700] and near the ends of the range.  The 64-entry table 2^(j/64) is
built here with exp2l rounded to double (the kernels build theirs with the
device exp2).  No GPU needed.
"""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <random>
#define __device__
#define __forceinline__ inline
%s
static double ulp_err(double got, long double want)
{
    const double w = (double)want;
    const double u = std::nextafter(std::fabs(w), INFINITY) - std::fabs(w);
    return (double)(std::fabs((long double)got - want) / (long double)u);
}
int main()
{
    double t64[64];
    for (int j = 0; j < 64; ++j) t64[j] = (double)exp2l((long double)j / 64.0L);
    std::mt19937_64 rng(20240611);
    std::uniform_real_distribution<double> U(-700.0, 700.0), S(-1.0, 1.0);
    double worst = 0.0, worst_x = 0.0;
    auto check = [&](double x) {
        const double e = ulp_err(exp_tab(x, t64), expl((long double)x));
        if (e > worst) { worst = e; worst_x = x; }
    };
    for (int i = 0; i < 2000000; ++i) check(U(rng));
    for (int i = 0; i < 200000; ++i) check(S(rng));           // |x| < 1
    for (int i = 0; i < 200000; ++i) check(1e-6 * S(rng));    // near 0
    for (int i = 0; i < 100000; ++i) check(-700.0 - 8.0 * std::fabs(S(rng)));  // -708 .. -700
    for (int i = 0; i < 100000; ++i) check(700.0 + 9.0 * std::fabs(S(rng)));   // 700 .. 709
    std::printf("%%.6f %%.17g\n", worst, worst_x);
    std::printf("%%.17g %%.17g %%.17g\n", exp_tab(0.0, t64), exp_tab(-800.0, t64), exp_tab(710.0, t64));
    return 0;
}
"""


def exp_tab_source():
    src = open(os.path.join(ROOT, "paper_1706_07413_amd", "csrc", "stage.h")).read()
    m = re.search(r"__device__ __forceinline__ double exp_tab\(double x, const double\* t64\)\n\{.*?\n\}\n",
                  src, re.S)
    assert m, "exp_tab not found in stage.h"
    return m.group(0)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_exp_tab_within_1_5_ulp(tmp_path):
    c = tmp_path / "exp_tab_check.cpp"
    c.write_text(DRIVER % exp_tab_source())
    exe = tmp_path / "exp_tab_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    worst, worst_x = (float(v) for v in out[0].split())
    assert worst <= 1.5, "exp_tab: %.3f ulp at x = %r" % (worst, worst_x)
    e0, lo, hi = (float(v) for v in out[1].split())
    assert e0 == 1.0           # e^0 exactly
    assert lo == 0.0           # arguments below -746 give 0
    assert np.isinf(hi)        # past the largest double
