"""Per-measurement energies of a correlated pair as JSON lines.

A trace from `pair_step` / `pair_batch_step` holds one row (E_A, E_B, dE) per
measurement (Eq. 7 for each system, dE = E_B - E_A); `trace_records` turns it
into one record per measurement with the step at which it was taken, and
`write_jsonl` writes records one JSON object per line.
"""
from __future__ import annotations

import json
from typing import Iterable, Iterator

import numpy as np


def trace_records(trace, first_step: int, measure_every: int, **extra) -> Iterator[dict]:
    """Records of a trace whose run started after step `first_step`: the k-th
    measurement falls at step first_step + (k + 1) * measure_every."""
    tr = np.asarray(trace, dtype=float).reshape(-1, 3)
    for k, (ea, eb, de) in enumerate(tr):
        yield {"step": int(first_step + (k + 1) * measure_every), "E_A": float(ea),
               "E_B": float(eb), "dE": float(de), **extra}


def write_jsonl(path: str, records: Iterable[dict]) -> int:
    """Write the records one per line; returns how many were written."""
    n = 0
    with open(path, "w") as f:
        for r in records:
            f.write(json.dumps(r) + "\n")
            n += 1
    return n
