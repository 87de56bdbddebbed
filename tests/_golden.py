"""Reader for the integer fixtures in tests/golden/ (see tests/golden/make_golden.py)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    out, key, rows, want = {}, None, [], 0
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if key is None or len(rows) == want:
                if key is not None:
                    out[key] = np.array(rows, dtype=np.float64)
                key, want, rows = parts[0], int(parts[1]), []
                continue
            rows.append([float(v) for v in parts])
    out[key] = np.array(rows, dtype=np.float64)
    return out
