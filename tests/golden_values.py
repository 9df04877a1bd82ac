"""Loader of the text fixtures under tests/golden/: values the paper prints, one file per
passage (each file's header cites it). Lines are whitespace-separated fields; '#' starts
a comment."""
from __future__ import annotations

import os

_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rows(name: str) -> dict[str, list[float]]:
    """{first field: remaining fields as floats} of tests/golden/<name>.txt."""
    out = {}
    with open(os.path.join(_DIR, name + ".txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = [float(v) for v in line[1:]]
    return out


def scalars(name: str) -> dict[str, float]:
    return {k: v[0] for k, v in rows(name).items()}
