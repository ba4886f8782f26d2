"""Reader for the hand-worked fixtures in tests/golden/ (key: value lines)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.split()
    return out


def ints(v):
    return [int(t, 0) for t in v]


def floats(v):
    return [float(t) for t in v]
