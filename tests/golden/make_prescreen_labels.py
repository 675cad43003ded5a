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

Two fixtures: prescreen_labels.txt (RECIPE, 2^16-bin spectra, one 0/1 per
block) and prescreen_labels_2p20.txt (RECIPE_2P20, 2^20-bin spectra, the 256
block labels of a spectrum as 64 hex digits, block 0 in the leading bit).
The 2^20 labels take about 10 CPU seconds per spectrum; finished rows are
appended to <fixture>.part as they come, so an interrupted run resumes.

Usage: python tests/golden/make_prescreen_labels.py [count] [--2p20] [--workers W]
                                                    [--range A B --part PATH]
With --range only spectra A <= i < B are labelled, into the partial file PATH
(rows of several such runs are merged by appending them to <fixture>.part).
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

RECIPE_2P20 = {"n": 1 << 20, "seed0": 7_000_000, "pulsars": "i % 4", "r_range": [2500.0, 500000.0],
               "z_range": [-42.0, 42.0], "snr_range": [5.0, 20.0], "harm_range": [1, 8], "block": 4096,
               "p_label": 1e-8, "p_sig": 1e-12, "n_harm": 8}


def spectrum(i, r=RECIPE):
    return synth.make_spectrum(r["n"], r["seed0"] + i, n_random=i % 4, r_range=tuple(r["r_range"]),
                               z_range=tuple(r["z_range"]), snr_range=tuple(r["snr_range"]),
                               harm_range=tuple(r["harm_range"]))[0]


def label(i, r=RECIPE):
    spec = spectrum(i, r)
    plane = ofop.fop(spec.astype(np.complex128), workers=1)
    t1 = oh.thresholds(1, r["p_label"])[0]
    hot = (plane > t1).any(axis=0)
    blocks = hot.reshape(-1, r["block"]).any(axis=1).astype(int)
    return i, "".join(str(v) for v in blocks)


def to_hex(bits):
    """block labels (0/1 string) -> hex digits, block 0 in the leading bit"""
    return format(int(bits, 2), "0%dx" % (len(bits) // 4))


def from_hex(h, blocks):
    return format(int(h, 16), "0%db" % blocks)


def _label_2p20(i):
    return label(i, RECIPE_2P20)


def main():
    args = sys.argv[1:]
    big = "--2p20" in args
    workers = min(8, os.cpu_count() or 1)
    if "--workers" in args:
        workers = int(args[args.index("--workers") + 1])
        del args[args.index("--workers"):args.index("--workers") + 2]
    lo, hi, part = None, None, None
    if "--range" in args:
        k = args.index("--range")
        lo, hi = int(args[k + 1]), int(args[k + 2])
        del args[k:k + 3]
    if "--part" in args:
        k = args.index("--part")
        part = args[k + 1]
        del args[k:k + 2]
    args = [a for a in args if a != "--2p20"]
    count = int(args[0]) if args else (10240 if big else 384)
    recipe = RECIPE_2P20 if big else RECIPE
    path = os.path.join(HERE, "prescreen_labels_2p20.txt" if big else "prescreen_labels.txt")
    part = part or path + ".part"
    done = {}
    if big and os.path.exists(part):
        with open(part) as f:
            for line in f:
                a, b = line.split()
                done[int(a)] = b
    span = range(count) if lo is None else range(lo, hi)
    todo = [i for i in span if i not in done]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        if big:
            with open(part, "a") as f:
                for i, bits in ex.map(_label_2p20, todo, chunksize=4):
                    done[i] = bits
                    f.write(f"{i} {bits}\n")
                    f.flush()
        else:
            for i, bits in ex.map(label, todo):
                done[i] = bits
    if lo is not None:
        print(f"labelled spectra {lo}..{hi - 1} into {part}")
        return
    rows = sorted((i, done[i]) for i in range(count))
    with open(path, "w") as f:
        f.write("# oracle labels for the block pre-screen (tests/golden/make_prescreen_labels.py%s)\n"
                % (" --2p20" if big else ""))
        f.write("# recipe: " + json.dumps(recipe) + "\n")
        if big:
            f.write("# one line per spectrum i: i, then its block labels as hex digits (block 0 in the leading bit)\n")
        else:
            f.write("# one line per spectrum i: i, then one 0/1 per 4096-bin block\n")
        for i, bits in rows:
            f.write(f"{i} {to_hex(bits) if big else bits}\n")
    pos = sum(b.count("1") for _, b in rows)
    nb = recipe["n"] // recipe["block"]
    print(f"wrote {path}: {count} spectra, {pos} positive blocks of {count * nb}")


if __name__ == "__main__":
    main()
