"""Reader for the hand-worked fixtures in tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    d = {"edges": [], "level": {}, "parent_choices": {}}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            vals = [int(x) for x in vals]
            if key == "edge":
                d["edges"].append(vals)
            elif key == "level":
                d["level"][vals[0]] = vals[1]
            elif key == "parent_choices":
                d["parent_choices"][vals[0]] = vals[1:]
            elif key in ("n", "root"):
                d[key] = vals[0]
            else:
                d[key] = np.array(vals, dtype=np.int64)
    d["edges"] = np.array(d["edges"], dtype=np.int64).reshape(-1, 2)
    return d
