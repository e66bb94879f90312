"""Per-run records as JSON lines.

``append(record)`` adds one line to the file named by ``path`` or, if that is None,
by the environment variable ``LBM_RUN_LOG`` (unset: nothing is written).  The line is
the record with the time (UTC), the host (name, CPU count), the command line and a
digest of the library file beside this module (so a result can be tied to the build
that produced it).  ``bench.py``, the batch benchmark, the studies and the surrogate
study append their result lines here.
"""
from __future__ import annotations

import datetime
import functools
import hashlib
import json
import os
import platform
import sys

ENV = "LBM_RUN_LOG"


@functools.lru_cache(maxsize=None)
def library_digest() -> str | None:
    """sha256 (first 16 hex digits) of the built library, None if it is not built."""
    from . import lbm

    try:
        with open(lbm.LIB_PATH, "rb") as fh:
            return hashlib.sha256(fh.read()).hexdigest()[:16]
    except OSError:
        return None


def append(record: dict, path: str | None = None) -> str | None:
    """Append ``record`` (JSON-serialisable) as one line; returns the file written, or
    None when no log file is configured."""
    path = path or os.environ.get(ENV)
    if not path:
        return None
    line = dict(time=datetime.datetime.now(datetime.timezone.utc).isoformat(timespec="seconds"),
                host=dict(name=platform.node(), cpus=os.cpu_count()), argv=list(sys.argv),
                library=library_digest())
    line.update(record)
    with open(path, "a") as fh:
        fh.write(json.dumps(line, default=str) + "\n")
    return path
