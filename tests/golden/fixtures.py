"""Reader for the worked-example fixtures (values printed in the paper)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    """Returns dict with 'p' and the matrices/rows listed in the fixture file."""
    out, key, rows = {}, None, []
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "p":
                out["p"] = float(parts[1])
            elif len(parts) == 1 and parts[0].isalpha():
                if key is not None:
                    out[key] = np.array(rows, dtype=np.float64)
                key, rows = parts[0], []
            else:
                rows.append([float(x) for x in parts])
    if key is not None:
        out[key] = np.array(rows, dtype=np.float64)
    return out
