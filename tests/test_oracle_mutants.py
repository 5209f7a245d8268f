"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake in a copy of oracle/oracle.c (a dropped
term, a wrong sign, a transposed operand, a wrong threshold, a different
reduction order, a wrong stop rule, ...), builds it on the CPU, points the
`oracle` module at it and runs tests/test_oracle.py in a subprocess: at least
one pin must fail.  The unmodified oracle passes the same run.  The
hand-worked fixtures (tests/test_golden.py) run alongside the pins.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "operand order of SUB": ("case 1: return a - b;", "case 1: return b - a;"),
    "ADD becomes SUB": ("case 0: return a + b;", "case 0: return a - b;"),
    "protected threshold compared in double": ("(fabsf(b) < 1e-6f)", "(fabs((double)b) < 1e-6)"),
    "protection returns 0": ("? 1.0f : a / b", "? 0.0f : a / b"),
    "no protection": ("(fabsf(b) < 1e-6f) ? 1.0f : a / b", "a / b"),
    "stack pops right before left": ("float l = stack[--sp];\n            float r = stack[--sp];",
                                     "float r = stack[--sp];\n            float l = stack[--sp];"),
    "fitness sums left to right": ("for (int64_t h = P / 2; h >= 1; h /= 2)\n        for (int64_t i = 0; i < h; ++i) s[i] = s[i] + s[i + h];",
                                   "for (int64_t i = 1; i < P; ++i) s[0] = s[0] + s[i];"),
    "fitness drops the last case": ("for (int64_t t = 0; t < T; ++t) {\n        float e = out[t] - y[t];",
                                    "for (int64_t t = 0; t + 1 < T; ++t) {\n        float e = out[t] - y[t];"),
    "fitness without abs": ("s[t] = (double)fabsf(e);", "s[t] = (double)e;"),
    "NAND computed as AND": ("case 2: return ~(a & b);", "case 2: return a & b;"),
    "NOR computed as OR": ("default: return ~(a | b);", "default: return a | b;"),
    "Boolean fitness counts mismatches": ("uint64_t m = ~(out[w] ^ target[w]) & valid_mask(w, T);",
                                          "uint64_t m = (out[w] ^ target[w]) & valid_mask(w, T);"),
    "equality merges +0 and -0": ("return ua == ub;", "return a == b;"),
    "level 0 not checked": ("int32_t level = agreed ? 0 : -1;\n\n    for (int64_t k = 1; k < len; ++k) {\n        int64_t a = path[len - 1 - k];           /* ancestor k levels above c */",
                            "int32_t level = -1;\n\n    for (int64_t k = 1; k < len; ++k) {\n        int64_t a = path[len - 1 - k];           /* ancestor k levels above c */"),
    "walk swaps the path operand side": ("float v = (below == l) ? op_f32(f, child[t], sib[t]) : op_f32(f, sib[t], child[t]);",
                                         "float v = (below == l) ? op_f32(f, sib[t], child[t]) : op_f32(f, child[t], sib[t]);"),
    "interpreted count omits the donor": ("int64_t interp = nd;\n\n    int agreed = 1;", "int64_t interp = 0;\n\n    int agreed = 1;"),
    "splice keeps the removed subtree": ("memcpy(child + c + nd, P + e, (size_t)(n - e));",
                                         "memcpy(child + c + nd, P + c, (size_t)(n - e));"),
    "validation only checks the final count": ("if (i < n - 1 && s < 0) return ORC_EINVAL;", "(void)0;"),
    "Philox with nine rounds": ("for (int r = 0; r < 10; ++r) {", "for (int r = 0; r < 9; ++r) {"),
    "uniform by modulo": ("return ((uint64_t)u * n) >> 32;", "return u % n;"),
    "draw counter without blocks": ("(uint32_t)s, (uint32_t)(j / 4)}", "(uint32_t)s, (uint32_t)j}"),
    "tournament ties keep the later draw": ("if (!isnan(a) && (isnan(b) || a < b)) best = c;",
                                            "if (!isnan(a) && (isnan(b) || a <= b)) best = c;"),
    "Boolean tournament prefers fewer hits": ("if (fit[c] > fit[best]) best = c;", "if (fit[c] < fit[best]) best = c;"),
    "parent is the function that opened the earliest slot": ("parent[j] = sp > 0 ? st[sp - 1] : -1;",
                                                              "parent[j] = sp > 0 ? st[0] : -1;"),
    "a function takes three children": ("left[sp] = 2;", "left[sp] = 3;"),
    "Strahler adds one for unequal children": ("v = l == r ? l + 1 : (l > r ? l : r);", "v = (l > r ? l : r) + 1;"),
    "Strahler takes the smaller child": ("v = l == r ? l + 1 : (l > r ? l : r);", "v = l == r ? l + 1 : (l < r ? l : r);"),
}


def run_pins(lib_path):
    env = dict(os.environ)
    env["GPE_ORACLE_LIB"] = lib_path
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py"), os.path.join(ROOT, "tests", "test_golden.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return r.returncode


def build_variant(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-o", str(lib), str(src), "-lm"])
    return str(lib)


def test_unmodified_oracle_passes(tmp_path):
    lib = build_variant(tmp_path, "orig", open(SRC).read())
    assert run_pins(lib) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation anchor not found: {name}"
    lib = build_variant(tmp_path, "m", text.replace(old, new, 1))
    assert run_pins(lib) != 0, f"no pin caught: {name}"
