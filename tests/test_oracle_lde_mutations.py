"""Planted mistakes in Algorithm 3's level rule must be caught by its pins.

The rule exists twice in the oracle: the printed loops in Python
(lde.printed_exploitation, small graphs) and the C edge counter
(oracle/lde_count.c, any graph).  Each case plants one plausible slip in one
of them (walks counted instead of supports, the stopping round off by one, a
strict comparison, a dropped table, no end when nothing is left to
traverse, the wrong decay power in Lemma 4) and checks that a pin fails.
"""
import inspect
import os
import shutil
import subprocess
import textwrap

import pytest

import test_oracle_lde as pins
from oracle import build as obuild
from oracle import lde

C_SRC = os.path.join(os.path.dirname(obuild.__file__), "lde_count.c")

GOLDEN = [lambda name=name: pins.test_edge_counts_hand_counted(name) for name in pins.GOLDEN_GRAPHS]
LEVELS = [lambda T=T, w=w: pins.test_level_is_the_round_where_the_budget_is_reached(T, w)
          for T, w in [(2.0, 0), (6.0, 1), (6.25, 2), (15.5, 4)]]
RANDOM = [lambda seed=seed: pins.test_c_counter_matches_printed_loops_and_sets(seed) for seed in (1, 2)]

C_MUTANTS = [
    # every walk counted: a node reached twice in one step is kept twice
    ("walks_not_supports", "if (s->mark[q] != st) {", "if (1) {", GOLDEN + RANDOM),
    # the level one past the round that reached the budget
    ("level_one_late", "          if (costs) costs[l] = cost;\n          return l;",
     "          if (costs) costs[l] = cost;\n          return l + 1;", LEVELS + RANDOM),
    # the budget must be exceeded, not reached
    ("strict_budget", "if ((double)(E + cost) >= T) {", "if ((double)(E + cost) > T) {", LEVELS),
    # the table of v_k itself never extended
    ("source_table_dropped", "for (int32_t lp = 0; lp <= l; ++lp) {", "for (int32_t lp = 0; lp < l; ++lp) {",
     GOLDEN + RANDOM),
    # nothing left to traverse does not end the rounds
    ("no_exhaustion_end", "    if (cost == 0) return l; /* no walk from v_k survives l + 1 steps */\n", "",
     [pins.test_exhausted_exploitation_is_exact] + GOLDEN),
    # in-degree of the origin instead of its table's support at step l'
    ("origin_degree_only", "cost += edges_from_level(s, n, in_off, in_idx, s->lev[d][i], lp);",
     "cost += edges_from_level(s, n, in_off, in_idx, s->lev[d][i], 0);", GOLDEN + RANDOM),
]


def _caught(checks):
    caught = 0
    for check in checks:
        try:
            check()
        except AssertionError:
            caught += 1
    return caught


@pytest.mark.parametrize("name,old,new,checks", C_MUTANTS, ids=[m[0] for m in C_MUTANTS])
def test_c_counter_pins_catch_planted_mistake(name, old, new, checks, tmp_path, monkeypatch):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(C_SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "lde_mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"liboraclelde_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(path), "-o", str(lib)])
    monkeypatch.setattr(obuild, "LDE_LIB", str(lib))
    monkeypatch.setattr(lde, "_lib", None)
    assert _caught(checks) >= 1, f"no pin caught the mutant {name}"


PY_MUTANTS = [
    ("py_strict_budget", "if E + cost >= T:", "if E + cost > T:", LEVELS),
    ("py_level_one_late", "                            costs.append(cost)\n                            return l, Z, costs",
     "                            costs.append(cost)\n                            return l + 1, Z, costs", LEVELS),
    ("py_source_table_dropped", "for lp in range(l + 1):", "for lp in range(l):", GOLDEN),
    ("py_no_exhaustion_end", "        if cost == 0:\n            return l, Z, costs\n", "",
     [pins.test_exhausted_exploitation_is_exact]),
    ("py_lemma4_decay_not_powered", "z -= (c ** lp) * t * t * z2", "z -= c * t * t * z2",
     [lambda: pins.test_printed_rounds_give_lemma4_and_enumeration("random8a"),
      lambda: pins.test_printed_rounds_give_lemma4_and_enumeration("complete4")]),
    ("py_transition_not_divided", "nxt[int(q)] = nxt.get(int(q), 0.0) + px / din[x]",
     "nxt[int(q)] = nxt.get(int(q), 0.0) + px", [lambda: pins.test_printed_rounds_give_lemma4_and_enumeration("complete4")]),
]


@pytest.mark.parametrize("name,old,new,checks", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_printed_loop_pins_catch_planted_mistake(name, old, new, checks, monkeypatch):
    src = textwrap.dedent(inspect.getsource(lde.printed_exploitation))
    assert src.count(old) == 1, name
    ns = dict(vars(lde))
    exec(compile(src.replace(old, new), f"<{name}>", "exec"), ns)
    monkeypatch.setattr(lde, "printed_exploitation", ns["printed_exploitation"])
    assert _caught(checks) >= 1, f"no pin caught the mutant {name}"
