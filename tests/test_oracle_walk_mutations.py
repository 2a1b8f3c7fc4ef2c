"""Planted mistakes in the oracle's C walk simulator must be caught by its pins.

Each case compiles a copy of oracle/walks.c with one plausible slip (a
wrong word, a wrong decay, a biased index, a miscounted meeting, a broken
key schedule), loads it in place of the built library, and checks that at
least one pin then fails.
"""
import os
import shutil
import subprocess

import pytest

import test_oracle_lde as lde_pins
import test_oracle_pins as pins
from oracle import build as obuild
from oracle import exactsim as ox

SRC = os.path.join(os.path.dirname(obuild.__file__), "walks.c")

MUTANTS = [
    # walk y steps with walk x's word: the two walks coincide
    ("y_uses_x_word", "y = (uint64_t)in_idx[in_off[y] + (int64_t)oracle_mulhi64(wy, dy)];",
     "y = (uint64_t)in_idx[in_off[y] + (int64_t)oracle_mulhi64(wx, dy)];",
     [pins.test_walks_meet_probability_three_sources, pins.test_walks_match_exact_diagonal]),
    # lifetime thresholds of one sqrt(c)-walk instead of the pair's c
    ("lifetime_of_one_walk", "    p = p * c;\n", "    p = p * __builtin_sqrt(c);\n",
     [pins.test_walks_match_exact_diagonal, pins.test_walks_cycle_meet_at_step_one]),
    # index map that never picks the last in-neighbour
    ("index_skips_last", "x = (uint64_t)in_idx[in_off[x] + (int64_t)oracle_mulhi64(wx, dx)];",
     "x = (uint64_t)in_idx[in_off[x] + (int64_t)oracle_mulhi64(wx, dx > 1 ? dx - 1 : dx)];",
     [pins.test_walks_meet_probability_three_sources, pins.test_walks_match_exact_diagonal]),
    # a meeting during the non-stop phase counted
    ("nonstop_meeting_counted", "if (x == y) return t > nonstop ? 1 : 0;", "if (x == y) return 1;",
     [lambda: lde_pins.test_nonstop_pairs_meet_at_the_tail_probability(1)]),
    # key schedule bumps only the first key word
    ("philox_key_half_bumped", "      k1 += PHILOX_W1;\n", "",
     [lambda: pins.test_philox_matches_numpy((1, 2), (3, 4, 5, 6))]),
]


@pytest.mark.parametrize("name,old,new,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_walk_pins_catch_planted_mistake(name, old, new, checks, tmp_path, monkeypatch):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "walks_mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"liboraclewalks_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           str(path), "-o", str(lib), "-lm"])
    monkeypatch.setattr(obuild, "LIB", str(lib))
    monkeypatch.setattr(ox, "_walk_lib", None)
    caught = 0
    for check in checks:
        try:
            check()
        except AssertionError:
            caught += 1
    assert caught >= 1, f"no pin caught the mutant {name}"
