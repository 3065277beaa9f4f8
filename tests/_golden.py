"""Reader for the text fixtures under tests/golden (exact rationals)."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                out.append([float(Fraction(t)) for t in line.split()])
    return out


def matrix(name):
    return np.array(rows(name), dtype=np.float64)
