"""JSONL run metrics: one JSON object per line, appended, each with the time
and the host; the benchmark, the trainer and the batch driver write their
per-step, per-epoch and per-group records through it."""
from __future__ import annotations

import json
import os
import socket
import time


def append(path: str | None, kind: str, **record) -> None:
    """Append {"kind": kind, "time": ..., "host": ..., **record} to `path` (no-op for None)."""
    if not path:
        return
    rec = {"kind": kind, "time": time.strftime("%Y-%m-%dT%H:%M:%S"), "host": socket.gethostname(), **record}
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(path, "a") as f:
        f.write(json.dumps(rec, default=float) + "\n")
