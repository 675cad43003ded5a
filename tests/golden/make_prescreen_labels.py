"""Write prescreen_labels.txt: oracle labels for training the block pre-screen.

Each training spectrum (2^16 bins, seed SEED0 + i, i % 4 random pulsars drawn
by the input generator) is convolved by the float64 oracle; a 4096-bin block
is labelled 1 when some template's power in its columns exceeds T_1(P_LABEL),
the single-cell threshold at a per-cell false-alarm probability P_LABEL (a
signal visible in the block itself; noise alone labels ~0.35 % of blocks).
Significant harmonic-sum candidates elsewhere that such a signal causes (at
multiples of its frequency, under the stretch index map) are reached by
searching the flagged blocks' harmonic multiples, so they are not labels.
Only oracle/ and the input generator are used.

Usage: python tests/golden/make_prescreen_labels.py [count]
"""

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fop as ofop  # noqa: E402
from oracle import harmonic as oh  # noqa: E402
from paper_1806_01556_amd import synth  # noqa: E402

RECIPE = {"n": 1 << 16, "seed0": 5_000_000, "pulsars": "i % 4", "r_range": [1000.0, 30000.0],
          "z_range": [-42.0, 42.0], "snr_range": [5.0, 20.0], "harm_range": [1, 8], "block": 4096,
          "p_label": 1e-8, "p_sig": 1e-12, "n_harm": 8}


def spectrum(i):
    r = RECIPE
    return synth.make_spectrum(r["n"], r["seed0"] + i, n_random=i % 4, r_range=tuple(r["r_range"]),
                               z_range=tuple(r["z_range"]), snr_range=tuple(r["snr_range"]),
                               harm_range=tuple(r["harm_range"]))[0]


def label(i):
    r = RECIPE
    spec = spectrum(i)
    plane = ofop.fop(spec.astype(np.complex128), workers=1)
    t1 = oh.thresholds(1, r["p_label"])[0]
    hot = (plane > t1).any(axis=0)
    blocks = hot.reshape(-1, r["block"]).any(axis=1).astype(int)
    return i, "".join(str(v) for v in blocks)


def main():
    count = int(sys.argv[1]) if len(sys.argv) > 1 else 384
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        rows = sorted(ex.map(label, range(count)))
    path = os.path.join(HERE, "prescreen_labels.txt")
    with open(path, "w") as f:
        f.write("# oracle labels for the block pre-screen (tests/golden/make_prescreen_labels.py)\n")
        f.write("# recipe: " + json.dumps(RECIPE) + "\n")
        f.write("# one line per spectrum i: i, then one 0/1 per 4096-bin block\n")
        for i, bits in rows:
            f.write(f"{i} {bits}\n")
    pos = sum(b.count("1") for _, b in rows)
    print(f"wrote {path}: {count} spectra, {pos} positive blocks of {count * 16}")


if __name__ == "__main__":
    main()
