"""The five workload configurations, read from ``configs/cfg{c}.json``.

Each file holds the shapes, sizes, distributions and seeds of one workload:
0 the tiny parity case, 1 the 1080p frame, 2 the codec fit, 3 serving, 4 the
4K stress frame.  The generators in this package and the benchmark take
their parameters from here, so a file is the one place a workload is defined;
callers override fields with keyword arguments or command-line flags.
"""

from __future__ import annotations

import copy
import functools
import json
from pathlib import Path

_DIR = Path(__file__).with_name("configs")


@functools.lru_cache(maxsize=None)
def _load(c: int) -> dict:
    path = _DIR / f"cfg{c}.json"
    if not path.is_file():
        raise ValueError(f"no workload configuration {c} ({path.name})")
    with open(path) as f:
        return json.load(f)


def config(c: int) -> dict:
    """Workload configuration c (a fresh copy, safe to modify)."""
    return copy.deepcopy(_load(int(c)))
