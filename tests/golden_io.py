"""Readers for the hand-derived fixtures in tests/golden/."""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_fixture(name):
    pts, edges, cuts = [], [], []
    mode = None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line == "points":
                mode = "p"
                continue
            if line.startswith("edges"):
                mode = "e"
                continue
            if line.startswith("cut5"):
                mode = "c5"
                continue
            if line.startswith("cut"):
                mode = "c"
                continue
            tok = line.split()
            if mode == "p":
                pts.append([float(t) for t in tok])
            elif mode == "e":
                edges.append((int(tok[0]), int(tok[1]), float(tok[2])))
            elif mode == "c":
                kl1, kl4 = int(tok[0]), int(tok[1])
                dmax = math.inf if tok[2] == "inf" else float(tok[2])
                cuts.append((kl1, kl4, dmax, [int(t) for t in tok[3:]]))
            elif mode == "c5":
                # all five settings: dict of keyword arguments, labels
                kw = dict(kl1=int(tok[0]), kl2=int(tok[1]), kl3=int(tok[2]), kl4=int(tok[3]),
                          dmax=math.inf if tok[4] == "inf" else float(tok[4]))
                cuts.append((kw, [int(t) for t in tok[5:]]))
    X = np.array(pts, dtype=np.float32)
    return X, edges, cuts
