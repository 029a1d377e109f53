"""Writes fixed_saturation_n2048.txt: 2048 int8 channel values on which the fixed-point
decoder's path metric saturates (reading R18: the metric is an int16 that saturates at
32767).

The values come from a seeded local search that calls only the oracle: starting from
uniformly random values in [-127, 127], it changes one value at a time and keeps the change
when the total penalty of the all-frozen SC path does not fall.  The penalty is eq. (PMupd)
summed in Python integers over the leaf LLRs that the fixed-point oracle's SC decoder
reports (every leaf frozen but the last, the PC(2048, 1) information set), so it is the
metric the decoder would reach without saturation.

Run from the repository root:  python tests/golden/make_fixed_saturation.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

N, SEED, STEPS = 2048, 20241, 12000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fixed_saturation_n2048.txt")


def penalty(info, y):
    _, leaf = oracle.sc_decode(oracle.FIX, info, y)
    lf = leaf.astype(np.int64)
    return int(np.maximum(0, -lf[info == 0]).sum())


def main():
    info = oracle.construct(N, 1, 2.0)
    rng = np.random.default_rng(SEED)
    y = rng.integers(-127, 128, N).astype(np.int8)
    cur = penalty(info, y)
    for _ in range(STEPS):
        j = int(rng.integers(N))
        old = y[j]
        y[j] = np.int8(rng.integers(-127, 128))
        v = penalty(info, y)
        if v >= cur:
            cur = v
        else:
            y[j] = old
    with open(OUT, "w") as f:
        f.write("# int8 channel values (one frame, N = 2048) on which the fixed-point path metric\n")
        f.write("# saturates; written by make_fixed_saturation.py (seed %d, %d steps).\n" % (SEED, STEPS))
        f.write("# unsaturated penalty of the all-frozen SC path: %d\n" % cur)
        for r in range(0, N, 32):
            f.write(" ".join("%d" % v for v in y[r:r + 32]) + "\n")
    print("penalty", cur, "->", OUT)


if __name__ == "__main__":
    main()
