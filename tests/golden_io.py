"""Readers for the text fixtures under tests/golden/ (values printed in the
paper, each file citing its figure)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
INF = -1  # "infinity" cells are returned as -1


def table(name: str) -> np.ndarray:
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append([INF if v == "inf" else int(v) for v in line])
    return np.array(rows, dtype=np.int64)


def keyed(name: str) -> dict:
    """Lines 'key v1 v2 ...' (or 'key ... : v1 v2 ...') as a dict of lists."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if ":" in line:
                head, tail = line.split(":", 1)
                out[tuple(head.split())] = tail.split()
            else:
                parts = line.split()
                out[parts[0]] = parts[1:]
    return out
