"""The oracle's pins are strong enough: every planted mistake fails one.

Each case copies the oracle's C source, plants one plausible mistake (a
dropped step, a wrong sign, index or comparison, a transposed operand, the
paper's intermediate-vertex matrix in place of successors), builds the copy on
the CPU and runs the pin suite of test_oracle on it.  The real oracle passes
the same suite (test_oracle.py).
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests import oracle_pins as P
from tests.test_oracle import check_all_pins_i32

INF = P.INF
SRC = os.path.join(os.path.dirname(oracle.__file__), "fw_oracle.c")
VAL = os.path.join(os.path.dirname(oracle.__file__), "validate.c")
GRAD = os.path.join(os.path.dirname(oracle.__file__), "grad.c")

MUTANTS = {
    "non-strict compare (Fig. 1 as printed)": ("if (s < (int64_t)Di[j])", "if (s <= (int64_t)Di[j])"),
    "wrong column index": ("int64_t s = dik + (int64_t)Dk[j];", "int64_t s = dik + (int64_t)Dk[i];"),
    "wrong sign": ("int64_t s = dik + (int64_t)Dk[j];", "int64_t s = dik - (int64_t)Dk[j];"),
    "transposed operand": ("const int64_t dik = Di[k];", "const int64_t dik = D[k * ld + i];"),
    "dropped last step": ("for (int64_t k = 0; k < n; ++k) {\n        const int32_t *Dk",
                          "for (int64_t k = 0; k < n - 1; ++k) {\n        const int32_t *Dk"),
    "dropped first step": ("for (int64_t k = 0; k < n; ++k) {\n        const int32_t *Dk",
                           "for (int64_t k = 1; k < n; ++k) {\n        const int32_t *Dk"),
    "intermediate instead of successor": ("                    if (Ni) Ni[j] = nik;\n                }\n            }\n        }\n    }\n    return 0;\n}\n\n/* ------------------------------------------------------------ FW, float64",
                                          "                    if (Ni) Ni[j] = (int32_t)k;\n                }\n            }\n        }\n    }\n    return 0;\n}\n\n/* ------------------------------------------------------------ FW, float64"),
    "successor initialised to source": ("if (NX) NX[i * ld + j] = (i == j) ? (int32_t)i : (d < ORACLE_INF_I32 ? (int32_t)j : -1);",
                                        "if (NX) NX[i * ld + j] = (i == j) ? (int32_t)i : (d < ORACLE_INF_I32 ? (int32_t)i : -1);"),
    "diagonal kept from input": ("int32_t d = (i == j) ? 0 : (w >= ORACLE_INF_I32 ? ORACLE_INF_I32 : w);",
                                 "int32_t d = (w >= ORACLE_INF_I32 ? ORACLE_INF_I32 : w);"),
    "INF not normalised": ("int32_t d = (i == j) ? 0 : (w >= ORACLE_INF_I32 ? ORACLE_INF_I32 : w);",
                           "int32_t d = (i == j) ? 0 : w;"),
}


def graphs():
    yield synth.graph_i32(30, 7, 0.2, 1, 5)             # sparse, many ties
    yield synth.graph_i32(64, 8, 0.6, 1, 1000)
    W = synth.graph_i32(25, 9, 0.3, 1, 50)
    np.fill_diagonal(W, 3)                                # self-loops to ignore
    W[W >= INF] = np.iinfo(np.int32).max                  # absent written as INT_MAX
    yield W
    W = synth.graph_i32(30, 10, 0.04, 1, 9)              # many unreachable pairs
    W[W >= INF] = INF + 12345                              # absent written above 2^30
    yield W
    w = np.arange(1, 20)
    yield P.chain(20, w)[0].astype(np.int32)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name!r} not found"
    mutated = src.replace(old, new, 1)
    cfile = tmp_path / "fw_oracle_mut.c"
    cfile.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           str(cfile), VAL, GRAD, "-o", str(so), "-lm"])
    lib = oracle.load_library(str(so))
    caught = []
    for W in graphs():
        try:
            fails, _, _ = check_all_pins_i32(W, lib=lib)
        except ValueError as e:                          # negative weight paths etc.
            fails = [str(e)]
        caught += fails
    assert caught, f"planted mistake {name!r} passed every pin"


def _in_function(src, fn_start, fn_end, old, new):
    """Replace `old` by `new` only inside the source between two markers."""
    a = src.index(fn_start)
    b = src.index(fn_end, a)
    body = src[a:b]
    assert body.count(old) >= 1, f"mutation site {old!r} not found in {fn_start!r}"
    return src[:a] + body.replace(old, new, 1) + src[b:]


def _build(tmp_path, fw_src, val_src):
    fdir = tmp_path / "src"
    fdir.mkdir()
    (fdir / "fw_oracle.c").write_text(fw_src)
    (fdir / "validate.c").write_text(val_src)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           str(fdir / "fw_oracle.c"), str(fdir / "validate.c"), GRAD, "-o", str(so), "-lm"])
    return oracle.load_library(str(so))


F32_VAL = ("int64_t validate_walk_f32(", "int64_t validate_walk_f64(")
VALIDATOR_MUTANTS = {
    "f32 validator never checks the sum": ("if (fabs(sum - dd) > rtol * scale) reason = 4;", "(void)scale;"),
    # (dropping "h == u" alone is an equivalent mutant: the hop bound still
    # ends a walk that stays put, with the same reason code)
    "f32 validator ends a walk that stays put": ("if (h < 0 || h >= n || h == u || hops >= n - 1)",
                                                 "if (h == u) break;\n                    if (h < 0 || h >= n || hops >= n - 1)"),
    "f32 validator ignores an INF / -1 mismatch": ("if (!(isinf(d) && d > 0 && h0 == -1)) reason = 2;", ";"),
    "f32 validator does not check the diagonal": ("if (d != 0.0f || h0 != (int32_t)i) reason = 1;", ";"),
    "f32 validator walks over absent edges": ("if (isinf(w) || isnan(w) || w < 0.0f) { reason = 3; break; }", ";"),
    "f32 validator accepts any negative infinity": ("if (!(isinf(d) && d > 0 && h0 == -1)) reason = 2;",
                                                    "if (!(isinf(d) && h0 == -1)) reason = 2;"),
    "f32 validator takes the first hop only": ("                    u = h;\n                    ++hops;",
                                               "                    u = j;\n                    ++hops;"),
}


@pytest.mark.parametrize("name", sorted(VALIDATOR_MUTANTS))
def test_validator_mutant_is_caught(name, tmp_path):
    """A lenient (or otherwise wrong) float32 walk validator fails a pin."""
    from tests.test_oracle import check_validator_pins
    old, new = VALIDATOR_MUTANTS[name]
    val = _in_function(open(VAL).read(), F32_VAL[0], F32_VAL[1], old, new)
    lib = _build(tmp_path, open(SRC).read(), val)
    fails = check_validator_pins("f32", lib=lib)
    assert fails, f"planted mistake {name!r} passed every validator pin"


F32_FW = ("int oracle_fw_f32(", "void oracle_sssp_i32(")
F32_ORACLE_MUTANTS = {
    "f32 non-strict compare": ("if (s < Di[j]) {", "if (s <= Di[j]) {"),
    "f32 successor not updated": ("                    if (Ni) Ni[j] = nik;", "                    ;"),
    "f32 intermediate instead of successor": ("if (Ni) Ni[j] = nik;", "if (Ni) Ni[j] = (int32_t)k;"),
    "f32 successor of the wrong operand": ("const int32_t nik = Ni ? Ni[k] : 0;",
                                           "const int32_t nik = Ni ? NX[k * ld + i] : 0;"),
    "f32 dropped last step": ("for (int64_t k = 0; k < n; ++k) {\n        const float *Dk",
                              "for (int64_t k = 0; k < n - 1; ++k) {\n        const float *Dk"),
    "f32 transposed operand": ("float s = dik + Dk[j];", "float s = dik + D[j * ld + k];"),
}


@pytest.mark.parametrize("name", sorted(F32_ORACLE_MUTANTS))
def test_f32_oracle_mutant_is_caught(name, tmp_path):
    """A plausible mistake in the float32 oracle fails a float32 pin."""
    from tests.test_oracle import check_f32_oracle_pins
    old, new = F32_ORACLE_MUTANTS[name]
    src = _in_function(open(SRC).read(), F32_FW[0], F32_FW[1], old, new)
    lib = _build(tmp_path, src, open(VAL).read())
    try:
        fails = check_f32_oracle_pins(lib=lib)
    except ValueError as e:
        fails = [str(e)]
    assert fails, f"planted mistake {name!r} passed every float32 pin"
