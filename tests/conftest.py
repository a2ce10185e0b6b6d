import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def read_golden(name):
    """Parse a golden fixture: '#' comments; each line 'label v v v ...' where a
    value is 're,im' (complex) or a plain number.  Returns dict label -> list."""
    out = {}
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            toks = line.split()
            vals = []
            label = None
            for i, t in enumerate(toks):
                try:
                    if "," in t:
                        re_, im_ = t.split(",")
                        vals.append(complex(float(re_), float(im_)))
                    else:
                        vals.append(float(t))
                except ValueError:
                    if i == 0:
                        label = t
                        continue
                    raise
            if label is None:
                rows.append(vals)
            else:
                out[label] = vals
    if rows:
        out["_rows"] = rows
    return out
