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
