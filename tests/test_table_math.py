"""Host-side check of the table builder's FP64 sine and cosine (no GPU needed).

The multiplier tables convert each angle with sincos_quarter() of
csrc/hygt_table.h (Taylor series of sin h and cos h for |h| <= pi/4, the half
angle after the reduction to |phi| <= pi/2). The function is pure arithmetic,
so its text is compiled here with the host compiler and compared with the C
library's sin and cos over the whole range: within 2 units in the last place
of FP64, far below the FP32 rounding that the tables apply afterwards.
"""

import os
import re
import shutil
import subprocess

import pytest

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_2505_21728_amd", "csrc", "hygt_table.h")

MAIN = r"""
#include <cmath>
#include <cstdio>
int main() {
    double worst_s = 0.0, worst_c = 0.0, worst_t = 0.0;
    const int steps = 200000;
    for (int i = -steps; i <= steps; ++i) {
        const double h = (M_PI / 4.0) * i / steps;
        double s, c;
        sincos_quarter(h, &s, &c);
        if (h != 0.0) worst_s = std::fmax(worst_s, std::fabs(s - std::sin(h)) / std::fabs(std::sin(h)));
        worst_c = std::fmax(worst_c, std::fabs(c - std::cos(h)) / std::fabs(std::cos(h)));
        if (h != 0.0) worst_t = std::fmax(worst_t, std::fabs(s / c - std::tan(h)) / std::fabs(std::tan(h)));
    }
    std::printf("%.6e %.6e %.6e\n", worst_s, worst_c, worst_t);
    return 0;
}
"""


def _extract(text, start):
    i = text.index(start)
    depth, j = 0, text.index("{", i)
    while True:
        if text[j] == "{":
            depth += 1
        elif text[j] == "}":
            depth -= 1
            if depth == 0:
                return text[i:j + 1]
        j += 1


def test_sincos_quarter_against_libm(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    text = open(HEADER).read()
    fact = _extract(text, "constexpr double inv_factorial(int n)")
    sc = _extract(text, "__device__ __forceinline__ void sincos_quarter(")
    sc = re.sub(r"__device__ __forceinline__ ", "inline ", sc)
    src = tmp_path / "sc.cpp"
    src.write_text("#include <cmath>\nusing std::fma;\n" + fact + "\n" + sc + "\n" + MAIN)
    exe = tmp_path / "sc"
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    ws, wc, wt = (float(v) for v in out)
    ulp = 2.0 ** -52
    assert ws <= 2 * ulp and wc <= 2 * ulp, (ws, wc)
    assert wt <= 4 * ulp, wt
