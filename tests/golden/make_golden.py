"""Write oracle_tiny.txt: a regression fixture of the FP64 oracle.

The paper prints no worked example (its figures carry no numbers), so the
stored values here are the oracle's own output on a tiny seeded case; the
oracle itself is pinned by the closed forms and brute-force checks in
tests/test_oracle_pins.py.  This script calls only oracle/.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402


def tiny_case():
    """8x7x6 volume of integers/8 (exact in float32), n = 4, s = 1, six
    neighbours at offset 2, adapted weights against a fixed desired map."""
    rng = np.random.default_rng(20260)
    V = (rng.integers(-16, 17, size=(8, 7, 6)) / 8.0).astype(np.float32)
    D = (rng.integers(0, 2, size=(8, 7, 6))).astype(np.float32)
    off = np.array([[2, 0, 0], [-2, 0, 0], [0, 2, 0], [0, -2, 0], [0, 0, 2], [0, 0, -2]], np.int32)
    p = orc.Params(n=4, s=1, window="hann", offsets=off, fusion="adapt_ls", D=D, delta=1e-6)
    return V, p


def main():
    V, p = tiny_case()
    r = orc.forward(V, p)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_tiny.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle output for tiny_case() in make_golden.py (regression fixture, not a paper value)\n")
        f.write("# E, Sm: planar [3][8][7][6] flattened; W: adapted fusion weights (Eq. 4)\n")
        for k in ("E", "Sm", "W"):
            f.write("%s = %s\n" % (k, " ".join("%.17g" % v for v in np.asarray(r[k]).reshape(-1))))


if __name__ == "__main__":
    main()
