"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU),
builds it, and runs the pin tests against that build: they must fail.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lupp_oracle.c")

MUTANTS = {
    "tie_break_highest_row": ("if (v > best) {", "if (v >= best) {"),
    "update_sign": ("return use_fma ? fma(-l, u, a) : a - l * u;",
                    "return use_fma ? fma(-l, u, a) : a + l * u;"),
    "fma_update_sign": ("return use_fma ? fma(-l, u, a) : a - l * u;",
                        "return use_fma ? fma(l, u, a) : a - l * u;"),
    "update_transposed": ("a[k + (int64_t)j * lda], use_fma);",
                          "a[j + (int64_t)k * lda], use_fma);"),
    "swap_trailing_only": ("for (int j = 0; j < n; ++j) {\n                double t = a[k + (int64_t)j * lda];",
                           "for (int j = k; j < n; ++j) {\n                double t = a[k + (int64_t)j * lda];"),
    "no_rhs_interchange": ("int p = ipiv[k] - 1;", "int p = k;"),
    "forward_sub_skips_first": ("for (int j = 0; j < n; ++j)\n        for (int i = j + 1; i < n; ++i)",
                                "for (int j = 1; j < n; ++j)\n        for (int i = j + 1; i < n; ++i)"),
    "norton_sign": ("F[6] = dp - law->dt", "F[6] = dp + law->dt"),
    "von_mises_factor": ("double seq = sqrt(1.5 * xx);", "double seq = sqrt(xx);"),
    "jacobian_drops_dFp_deel": ("JAC(6, a) = -gdot * 2.0 * mu * KN[a];", "JAC(6, a) = 0.0;"),
    "af_recall_sign": ("+ law->D * dp * alpha[i];", "- law->D * dp * alpha[i];"),
    "lame_mu": ("*mu = law->E / (2.0 * (1.0 + law->nu));", "*mu = law->E / (1.0 + law->nu);"),
    "tangent_transposed": ("tan[6 * r + c] =", "tan[6 * c + r] ="),
    "tangent_drops_lambda": ("(r < 3 ? lam * tr : 0.0)", "0.0"),
    "tangent_wrong_rhs": ("x[i] = (i == c) ? 1.0 : 0.0;", "x[i] = (i == c + 1) ? 1.0 : 0.0;"),
    "tiled_no_fallback": ("if (fabs(col[p]) < thresh) {", "if (0) {"),
    "tiled_threshold_inverted": ("if (fabs(col[p]) < thresh) {", "if (fabs(col[p]) > thresh) {"),
    "tiled_tile_end": ("int k1 = (k / ts + 1) * ts;", "int k1 = (k / ts + 1) * ts + 1;"),
    "stop_rule_off_by_one": ("if (k == maxit) {", "if (k + 1 >= maxit) {"),
    "reciprocal_multipliers": (
        "a[i + (int64_t)k * lda] = a[i + (int64_t)k * lda] / a[k + (int64_t)k * lda];",
        "a[i + (int64_t)k * lda] = a[i + (int64_t)k * lda] * (1.0 / a[k + (int64_t)k * lda]);"),
    "fma_forward_substitution_unfused": (
        "for (int i = j + 1; i < n; ++i)\n            b[i] = oracle_msub(b[i], lu[i + (int64_t)j * lda], b[j], use_fma);",
        "for (int i = j + 1; i < n; ++i)\n            b[i] = oracle_msub(b[i], lu[i + (int64_t)j * lda], b[j], 0);"),
    "fma_back_substitution_unfused": (
        "for (int i = 0; i < j; ++i)\n            b[i] = oracle_msub(b[i], lu[i + (int64_t)j * lda], b[j], use_fma);",
        "for (int i = 0; i < j; ++i)\n            b[i] = oracle_msub(b[i], lu[i + (int64_t)j * lda], b[j], 0);"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-I", os.path.dirname(SRC), "-o", str(so), str(mut),
                    "-lm", "-lpthread"], check=True)
    env = dict(os.environ, ORACLE_SO=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_lupp.py"),
                        os.path.join(ROOT, "tests", "test_oracle_newton.py"),
                        os.path.join(ROOT, "tests", "test_oracle_tiled.py"),
                        os.path.join(ROOT, "tests", "test_oracle_fma.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
