"""Writes tiny_energyscape.txt: a small fixed case evaluated by the FP64 oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The fixture freezes the oracle's output so that a later change to its
arithmetic shows up as a failing test and has to be justified.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402


def tiny_case():
    rng = np.random.default_rng(20220823)
    M, N, L = 4, 96, 16
    x = rng.standard_normal((M, N))
    t = np.arange(L) / 450e3
    s = 0.5 * (1 - np.cos(2 * np.pi * np.arange(L) / L)) * np.sin(2 * np.pi * (60e3 * t + 2e9 * t * t))
    pos = np.zeros((M, 3))
    pos[:, :2] = rng.uniform(-0.0175, 0.0175, size=(M, 2))
    dirs = np.array([[0.0, 0.0, 1.0], [0.5, 0.0, np.sqrt(0.75)], [0.0, -0.6, 0.8]])
    return dict(x=x, chirp=s, mic_pos=pos, dirs=dirs, fs=450e3, c=343.0, P=128, R=4,
                band=(20e3, 150e3))


def main():
    c = tiny_case()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_energyscape.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle output for tests/golden/make_golden.py:tiny_case(); rows td then fd\n")
        for mode in ("td", "fd"):
            E = oracle.energyscape(c["x"], c["chirp"], c["mic_pos"], c["dirs"], fs=c["fs"], c=c["c"],
                                   P=c["P"], R=c["R"], band=c["band"], mode=mode)
            for row in E:
                f.write(" ".join(f"{v:.17e}" for v in row) + "\n")


if __name__ == "__main__":
    main()
