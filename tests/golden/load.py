"""Reader for the small text fixtures in this folder (sections of numbers)."""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load_sections(name: str) -> dict[str, np.ndarray]:
    out: dict[str, list[list[float]]] = {}
    cur = None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                out[cur] = []
                continue
            out[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in out.items()}
