"""Test-side references for the block-restricted search (no library code).

``closure_reference`` is the harmonic closure of a block list under the
stretched index map, written by brute force over columns: a signal at column
j raises the stretched harmonic sums HP_m at columns m*j .. m*j + m - 1
(floor(j'/m) = j exactly there), so a flagged block also needs the blocks that
hold those columns searched.
"""

import numpy as np

BLOCK = 4096


def closure_reference(blocks, n, n_harm):
    nblk = (int(n) + BLOCK - 1) // BLOCK
    out = set(int(b) for b in blocks)
    for b in blocks:
        j = np.arange(BLOCK * int(b), min(int(n), BLOCK * (int(b) + 1)), dtype=np.int64)
        for m in range(2, n_harm + 1):
            for e in range(m):
                c = m * j + e
                out.update(np.unique(c[c < n] // BLOCK).tolist())
    return np.array(sorted(b for b in out if b < nblk), dtype=np.int32)
