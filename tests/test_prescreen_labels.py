"""The pre-screen label fixture agrees with the oracle (CPU).

tests/golden/prescreen_labels.txt is written by make_prescreen_labels.py from
the float64 oracle; a few of its rows are recomputed here from the recipe in
its header, and the positive rate is checked against what the recipe implies
(noise alone marks a block with probability 1 - (1 - 1e-8)^(85*4096) ~ 0.35 %).
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_prescreen_labels as mk  # noqa: E402

PATH = os.path.join(HERE, "golden", "prescreen_labels.txt")


def _rows():
    with open(PATH) as f:
        lines = f.read().splitlines()
    recipe = json.loads(next(l for l in lines if l.startswith("# recipe: "))[len("# recipe: "):])
    rows = {int(a): b for a, b in (l.split() for l in lines if l and not l.startswith("#"))}
    return recipe, rows


def test_recipe_matches_generator():
    recipe, rows = _rows()
    assert recipe == mk.RECIPE
    assert sorted(rows) == list(range(len(rows)))
    assert all(len(b) == recipe["n"] // recipe["block"] for b in rows.values())


def test_rows_recomputed_from_the_oracle():
    _, rows = _rows()
    for i in (0, 1, 2, 3, 101):
        j, bits = mk.label(i)
        assert bits == rows[i], i


def test_noise_only_rows_are_mostly_negative():
    recipe, rows = _rows()
    noise = [b for i, b in rows.items() if i % 4 == 0]  # i % 4 pulsars: row i % 4 == 0 has none
    rate = np.mean([c == "1" for b in noise for c in b])
    p_block = 1.0 - (1.0 - recipe["p_label"]) ** (85 * recipe["block"])
    assert rate <= 5 * p_block + 0.002, rate
