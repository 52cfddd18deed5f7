"""Reader of tests/golden/paper_values.txt: numbers the paper prints, each with its citation."""
import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")


def load():
    """name -> tuple of floats (the citation column is for the reader)."""
    out = {}
    with open(_PATH) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, values, cite = (p.strip() for p in line.split("|", 2))
            assert cite, name
            out[name] = tuple(float(v) for v in values.split())
    return out


PAPER = load()


def value(name):
    """a single-valued entry"""
    (v,) = PAPER[name]
    return v
