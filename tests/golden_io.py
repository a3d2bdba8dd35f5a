"""Readers for the hand-traced text fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line


def records(name):
    """`lhs : rhs` records as (list of lhs tokens, list of rhs tokens)."""
    out = []
    for line in _lines(name):
        lhs, rhs = line.split(":", 1)
        out.append((lhs.split(), rhs.split()))
    return out


def fields(name):
    """`key: values` records as a dict of token lists."""
    return {lhs[0]: rhs for lhs, rhs in records(name)}
