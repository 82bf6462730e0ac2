"""Floating-point operation count of the oracle's law evaluation — TEST
INFRASTRUCTURE (part of the oracle package).

Counts the additions, subtractions, multiplications, divisions, square roots
and powers that ``oracle_law_eval`` (Section 2.1, eqs. 1-3: residual and
exact Jacobian of the Norton and Norton + Armstrong-Frederick laws) executes
on data that depends on the point, by compiling that function's own source
text, taken from ``lupp_oracle.c`` at run time, against a counting number
type (C++, g++). Arithmetic on the law parameters alone (Lame constants,
dt * A, 2/3 C) is done in plain doubles and not counted: a kernel computes it
once per launch. Sign changes and comparisons are not counted.

    python -m oracle.law_flops      # prints the counts as JSON
"""
from __future__ import annotations

import json
import os
import subprocess
import tempfile

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lupp_oracle.c")

_PRELUDE = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <cstddef>
#include "lupp_oracle.h"

static long g_add, g_mul, g_div, g_sqrt, g_pow;

struct counted {
    double v;
    counted() : v(0.0) {}
    counted(double x) : v(x) {}
};
static inline counted operator+(counted a, counted b) { ++g_add; return counted(a.v + b.v); }
static inline counted operator-(counted a, counted b) { ++g_add; return counted(a.v - b.v); }
static inline counted operator*(counted a, counted b) { ++g_mul; return counted(a.v * b.v); }
static inline counted operator/(counted a, counted b) { ++g_div; return counted(a.v / b.v); }
static inline counted operator-(counted a) { return counted(-a.v); }
static inline counted &operator+=(counted &a, counted b) { a = a + b; return a; }
static inline counted &operator-=(counted &a, counted b) { a = a - b; return a; }
static inline counted &operator*=(counted &a, counted b) { a = a * b; return a; }
static inline bool operator>(counted a, counted b) { return a.v > b.v; }
static inline bool operator<(counted a, counted b) { return a.v < b.v; }
static inline bool operator>=(counted a, counted b) { return a.v >= b.v; }
static inline bool operator<=(counted a, counted b) { return a.v <= b.v; }
static inline bool operator==(counted a, counted b) { return a.v == b.v; }
static inline bool operator!=(counted a, counted b) { return a.v != b.v; }
static inline counted sqrt(counted a) { ++g_sqrt; return counted(std::sqrt(a.v)); }
static inline counted pow(counted a, counted b) { ++g_pow; return counted(std::pow(a.v, b.v)); }

#define oracle_lame counted_lame
#define oracle_law_eval counted_law_eval
#define double counted
"""

_MAIN = r"""
#undef double
#undef oracle_lame
#undef oracle_law_eval

static void run(int kind, int with_j, long out[5])
{
    oracle_law law = {kind, 200000.0, 0.3, 1e-6, 5.0, 20000.0, 200.0, 1.0};
    counted deps[6], st[13], y[13], F[13], J[169], sig[6];
    for (int i = 0; i < 6; ++i) deps[i] = counted(1e-3 * (i + 1) * (i % 2 ? -1.0 : 1.0));
    for (int i = 0; i < 13; ++i) { st[i] = counted(1e-4 * (i + 1)); y[i] = counted(2e-4 * (13 - i)); }
    g_add = g_mul = g_div = g_sqrt = g_pow = 0;
    counted_law_eval(&law, deps, st, y, F, with_j ? J : NULL, sig);
    out[0] = g_add; out[1] = g_mul; out[2] = g_div; out[3] = g_sqrt; out[4] = g_pow;
}

int main()
{
    const int kinds[2] = {7, 13};
    printf("{");
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j) {
            long c[5];
            run(kinds[k], j, c);
            printf("%s\"%d_%s\": {\"add\": %ld, \"mul\": %ld, \"div\": %ld, \"sqrt\": %ld, \"pow\": %ld}",
                   (k || j) ? ", " : "", kinds[k], j ? "residual_jacobian" : "residual", c[0], c[1],
                   c[2], c[3], c[4]);
        }
    printf("}\n");
    return 0;
}
"""


def _extract() -> str:
    """The source text of oracle_lame and oracle_law_eval, as in lupp_oracle.c."""
    src = open(_SRC).read()
    start = src.index("static void oracle_lame(")
    body = src.index("void oracle_law_eval(", start)
    i = src.index("{", body)
    depth = 0
    for j in range(i, len(src)):
        if src[j] == "{":
            depth += 1
        elif src[j] == "}":
            depth -= 1
            if depth == 0:
                return src[start:j + 1]
    raise RuntimeError("unbalanced braces in oracle_law_eval")


def counts() -> dict:
    """{'<kind>_residual' | '<kind>_residual_jacobian': {add, mul, div, sqrt,
    pow, flops}} for kind 7 and 13 (flops = add + mul + div + sqrt + pow:
    each operation counted once)."""
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, "law_flops.cpp")
        exe = os.path.join(d, "law_flops")
        with open(cpp, "w") as f:
            f.write(_PRELUDE + _extract() + _MAIN)
        subprocess.run(["g++", "-O1", "-std=c++17", "-I", _HERE, "-o", exe, cpp], check=True)
        out = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    for v in out.values():
        v["flops"] = v["add"] + v["mul"] + v["div"] + v["sqrt"] + v["pow"]
    return out


if __name__ == "__main__":
    print(json.dumps(counts(), indent=1))
