"""Reader of the stored oracle states under tests/golden/."""
import os

import numpy as np

GOLDEN_CONFIG2 = os.path.join(os.path.dirname(__file__), "golden", "config2_2048_1e4.txt")


def load_golden(path=GOLDEN_CONFIG2):
    """(observables, flat cell indices, values (cells, 4) complex128)."""
    obs, idx, vals = None, [], []
    with open(path) as f:
        for line in f:
            if line.startswith("obs "):
                obs = np.array([float(v) for v in line.split()[1:]])
            elif line.startswith("cell "):
                parts = line.split()
                idx.append(int(parts[1]))
                re_im = np.array([float(v) for v in parts[2:]])
                vals.append(re_im[0::2] + 1j * re_im[1::2])
    return obs, np.array(idx), np.array(vals)
