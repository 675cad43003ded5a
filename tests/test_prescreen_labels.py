"""The pre-screen label fixtures agree with the oracle (CPU).

tests/golden/prescreen_labels.txt (2^16-bin spectra) and
prescreen_labels_2p20.txt (2^20-bin spectra, block labels as hex digits) are
written by make_prescreen_labels.py from the float64 oracle; a few of their
rows are recomputed here from the recipe in the header, and the positive rate
of noise-only rows is checked against what the recipe implies (noise alone
marks a block with probability 1 - (1 - 1e-8)^(85*4096) ~ 0.35 %).
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_prescreen_labels as mk  # noqa: E402

PATH = os.path.join(HERE, "golden", "prescreen_labels.txt")
PATH_2P20 = os.path.join(HERE, "golden", "prescreen_labels_2p20.txt")


def _rows(path=PATH):
    with open(path) as f:
        lines = f.read().splitlines()
    recipe = json.loads(next(l for l in lines if l.startswith("# recipe: "))[len("# recipe: "):])
    nb = recipe["n"] // recipe["block"]
    rows = {}
    for a, b in (l.split() for l in lines if l and not l.startswith("#")):
        rows[int(a)] = b if len(b) == nb else mk.from_hex(b, nb)
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


def test_2p20_fixture_recipe_and_size():
    recipe, rows = _rows(PATH_2P20)
    assert recipe == mk.RECIPE_2P20
    assert sorted(rows) == list(range(10240))
    assert all(len(b) == 256 for b in rows.values())


def test_2p20_rows_recomputed_from_the_oracle():
    # about 10 CPU seconds per 2^20-bin spectrum: two rows with pulsars
    _, rows = _rows(PATH_2P20)
    for i in (1, 4099):
        j, bits = mk.label(i, mk.RECIPE_2P20)
        assert bits == rows[i], i


def test_2p20_noise_only_rows_are_mostly_negative():
    recipe, rows = _rows(PATH_2P20)
    noise = [b for i, b in rows.items() if i % 4 == 0]
    rate = np.mean([c == "1" for b in noise for c in b])
    p_block = 1.0 - (1.0 - recipe["p_label"]) ** (85 * recipe["block"])
    assert rate <= 5 * p_block + 0.002, rate
