"""The benchmark and study workloads as data (``workloads.json`` beside this file):
the FP64 droplet, the 200 x 200 Laplace sweep, the 4096^2 throughput lattice, the
uneven droplet batch and the surrogate study.  ``bench.py``, the batch benchmark,
the Laplace sweep, the surrogate study and the seeded input generators take their
sizes, parameter grids and ranges from here, so a workload is changed in one place.

    from paper_1412_7228_amd import workloads
    w = workloads.get("lattice_4096_spinodal")
"""
from __future__ import annotations

import copy
import functools
import json
import os

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")


@functools.lru_cache(maxsize=None)
def _all() -> dict:
    with open(PATH) as fh:
        return json.load(fh)


def names() -> list[str]:
    return sorted(_all())


def get(name: str) -> dict:
    """A copy of the named workload (KeyError for an unknown name)."""
    return copy.deepcopy(_all()[name])


def lattice_config(name: str, **overrides) -> dict:
    """The library configuration (nx, ny, EOS and its parameters) of a single-lattice
    workload, with ``overrides`` applied."""
    w = _all()[name]
    nx, ny = w["lattice"]
    return dict(nx=nx, ny=ny, **w["params"], **overrides)
