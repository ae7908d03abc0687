"""The (theta, degree) settings and leaf sizes the benchmark and the full-size
tests run, per workload, kernel and precision.

workloads/settings.json holds the cheapest setting of the benchmark's parameter
sweep (`python bench.py --sweep --workload atom|benzene --write-settings`) that
keeps the relative L2 and maximum error within 1e-6 at 10,000 seeded targets
for every orbital; DEFAULT_SETTINGS fills in what the file lacks.
"""
from __future__ import annotations

import json
import os

SETTINGS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "settings.json")

DEFAULT_SETTINGS = {
    "benzene": {"leaf_size": 2000,
                "yukawa_ss": {"fp64": [0.7, 8], "mixed": [0.8, 10]}},
    "atom": {"leaf_size": 2000,
             "yukawa_ss": {"fp64": [0.75, 8]}, "coulomb_ss": {"fp64": [0.8, 8]}},
}


def load_settings() -> dict:
    """{workload: {"leaf_size": N_L, kernel: {precision: [theta, degree]}}}."""
    s = json.loads(json.dumps(DEFAULT_SETTINGS))
    if os.path.exists(SETTINGS):
        with open(SETTINGS) as fh:
            stored = json.load(fh)
        for wl, v in stored.items():
            if wl not in s:
                continue
            for k, vv in v.items():
                if isinstance(vv, dict):
                    s[wl].setdefault(k, {}).update(
                        {p: list(x["setting"]) if isinstance(x, dict) else list(x)
                         for p, x in vv.items()})
                elif k == "leaf_size":
                    s[wl][k] = vv
    return s
