"""Reader for the small text fixtures under tests/golden/ (values from the paper)."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(tok):
    return Fraction(tok)


def load(name):
    """Parse 'key: v v v ; v v v' lines; returns {key: list of rows of Fractions}."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(":")
            rows = [[_num(t) for t in r.split()] for r in rest.split(";")]
            out[key.strip()] = rows
    return out


def matrix(d, key="A"):
    rows = d[key]
    scale = d["scale"][0][0] if "scale" in d else Fraction(1)
    return [[v * scale for v in r] for r in rows]


def vector(d, key):
    return d[key][0]


def as_float(m):
    return np.array([[float(v) for v in r] for r in m]) if isinstance(m[0], list) \
        else np.array([float(v) for v in m])
