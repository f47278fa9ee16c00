"""Shared helpers of the GPU tests (system construction and list comparison)."""
import sys

import numpy as np


def say(msg: str) -> None:
    """Print a progress line that names the case before each GPU step."""
    print(msg, flush=True)
    sys.stdout.flush()


def make_system(at, hp, params, sur_hp=None, sur_params=None, cap_radial=160, cap_angular=96, skin=1.0,
                build=True):
    from paper_2604_24816_amd import nep
    full = nep.NEPModel(hp, params)
    sur = nep.NEPModel(sur_hp, sur_params) if sur_hp is not None else None
    s = nep.NEPSystem(full, at.n, at.box, surrogate=sur, cap_radial=cap_radial, cap_angular=cap_angular)
    s.set_state(at.x, at.types, at.masses, at.v)
    if build:
        s.build_neighbors(skin)
    return s


def lists_equal(offsets, idx, counts, oidx):
    """GPU CSR lists against oracle (counts, [N][cap]) lists, row by row."""
    n = counts.size
    if not np.array_equal(np.diff(offsets), counts):
        bad = np.nonzero(np.diff(offsets) != counts)[0]
        return False, f"count mismatch at {bad[:5]}"
    for i in range(n):
        a = idx[offsets[i]: offsets[i + 1]]
        b = oidx[i, : counts[i]]
        if not np.array_equal(a, b):
            return False, f"row {i}: {a[:8]} vs {b[:8]}"
    return True, ""


def min_image_diff(a, b, box):
    d = a - b
    return d - box * np.round(d / box)
