"""Planted mistakes: each one must fail a pin of ``test_oracle_pins.py``.

A mutant oracle is the oracle's C source with one line changed, compiled on
the CPU into a temporary library and loaded next to the real one.  Every
mutation is a plausible slip in the part of the oracle that a pin is meant to
fix (Sec. II-A rules, Sec. II-B credit, the value leaf); the test passes when
the pin catches it, i.e. raises an assertion error on the mutant.
"""
import importlib.util
import os
import shutil

import pytest

import test_oracle_pins as PINS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

MUTATIONS = {
    # a node's W credited with the searching player's wins instead of its chooser's
    "credit_root_player": ("mcts.c", "if (x->chooser >= 0) x->W += vals[x->chooser];",
                           "if (x->chooser >= 0) x->W += vals[root->mover];",
                           PINS.check_search_trees),
    # a guessed value held by the guesser counted as a candidate
    "candidates_ignore_own_row": ("mcts.c", "if (x <= lo || x >= hi || mine[x] || revd[x]) continue;",
                                  "if (x <= lo || x >= hi || revd[x]) continue;",
                                  PINS.check_candidates),
    # a wrong guess in the tree reveals a random own tile instead of the drawn one
    "wrong_guess_ignores_drawn_tile": ("mcts.c", "} else if (s->drawn >= 0) {",
                                       "} else if (0 && s->drawn >= 0) {",
                                       PINS.check_in_tree_step),
    # the next player's draw taken with word 0 of the chance block
    "draw_with_word_0": ("mcts.c", "    end_turn(s, m, w[1]);\n    return 0;\n}",
                         "    end_turn(s, m, w[0]);\n    return 0;\n}",
                         PINS.check_in_tree_step),
    # a value leaf credits every seat with the searching player's value
    "value_leaf_root_value": ("mcts.c",
                              "vals[k] = (float)mp->fallback_playouts * (float)v[k];",
                              "vals[k] = (float)mp->fallback_playouts * (float)v[root_mover];",
                              PINS.check_value_trees),
    # a pipelined pass credited at once instead of after the next pass's descents
    "pipeline_credited_at_once": ("mcts.c", "if (mp->pipeline) {", "if (0) {",
                                  PINS.check_pass_trees),
    # the fallback decided on the leaf's player to move instead of the searching player
    "fallback_on_leaf_mover": ("mcts.c", "float vm = (float)v[root_mover];",
                               "float vm = (float)v[S->mover];",
                               PINS.check_value_trees),
}


def _mutant(tmp_path, name, fname, old, new):
    src = tmp_path / name
    src.mkdir()
    for f in os.listdir(ORACLE):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(ORACLE, f), src / f)
    text = (src / fname).read_text()
    assert text.count(old) == 1, f"mutation site of {name} not found exactly once"
    (src / fname).write_text(text.replace(old, new))
    from oracle import build as obuild
    so = obuild.build(src_dir=str(src), out=str(src / "liboracle_mutant.so"))
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}",
                                                  os.path.join(ORACLE, "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.LIB_PATH = so
    mod._lib = None
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pin_catches_planted_mistake(tmp_path, name):
    fname, old, new, check = MUTATIONS[name]
    mutant = _mutant(tmp_path, name, fname, old, new)
    with pytest.raises(AssertionError):
        check(mutant)


def test_unchanged_copy_passes_every_pin(tmp_path):
    """Control: the same loading path with no change passes all the checks."""
    plain = _mutant(tmp_path, "control", "mcts.c", "int oracle_mcts_search(",
                    "int oracle_mcts_search(")
    for check in (PINS.check_candidates, PINS.check_in_tree_step, PINS.check_search_trees,
                  PINS.check_value_trees):
        check(plain)
