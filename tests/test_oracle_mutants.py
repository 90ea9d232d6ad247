"""Plant plausible mistakes in a copy of the oracle's C source and check that the
pins of test_oracle.py reject every one (all on the CPU)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle as pins

MUTANTS = {
    "drop_bias": ("z += (double)b[j];", ""),
    "no_relu": ("double y = z > 0.0 ? z : 0.0;", "double y = z;"),
    "no_clamp": ("if (y > clamp) y = clamp;", ""),
    "slot_index_reversed": ("double t = (double)wj[k] * yi[ij[k]];", "double t = (double)wj[k] * yi[ij[K - 1 - k]];"),
    "mask_inclusive": ("double g = (y > 0.0 && y < clamp)", "double g = (y >= 0.0 && y <= clamp)"),
    "dw_transposed_operand": ("dwj[k] += g * yi[ij[k]];", "dwj[k] += g * yi[j];"),
    "dw_wrong_sign": ("dwj[k] += g * yi[ij[k]];", "dwj[k] -= g * yi[ij[k]];"),
    "dy_missing_weight": ("di[ij[k]] += g * (double)wj[k];", "di[ij[k]] += g;"),
    "db_missing": ("sb += g;", ""),
    "bound_no_propagation": ("eo[j] = (1.0 + g) * prop + g * s;", "eo[j] = g * s;"),
}


def _checks(orc):
    yield lambda: pins.test_hand_computed_net(orc)
    yield lambda: pins.test_forward_matches_dense_bruteforce(orc, 40, 8, 5, 17, 1.5, False)
    yield lambda: pins.test_backward_matches_dense_chain_rule(orc, 48, 8, 4, 9, 1.0)
    yield lambda: pins.test_first_layer_closed_form_on_binary_inputs(orc)
    yield lambda: pins.test_fp32_evaluations_stay_within_the_propagated_bound(orc, "S2", 1024, 12, 120)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, name
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", str(mut), "-o", so, "-lm"])
    oracle._use_library(so)
    try:
        failed = 0
        for check in _checks(oracle):
            try:
                check()
            except AssertionError:
                failed += 1
        assert failed >= 1, f"planted mistake {name} passed every pin"
    finally:
        oracle._use_library(None)
