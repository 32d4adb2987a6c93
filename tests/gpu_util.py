"""Shared helpers of the GPU tests (compare the HIP path with the oracle)."""
import math
import sys

import numpy as np


def rel_errors(u, v, ur, vr):
    """(relative max, relative L2) velocity error against a reference field;
    the L2 norm sums both components (relative L2 error of Sec. III)."""
    scale = max(np.max(np.abs(ur)), np.max(np.abs(vr)))
    emax = max(np.max(np.abs(u - ur)), np.max(np.abs(v - vr))) / scale
    el2 = math.sqrt((np.sum((u - ur) ** 2) + np.sum((v - vr) ** 2)) /
                    (np.sum(ur ** 2) + np.sum(vr ** 2)))
    return emax, el2


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}


W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]


def stored_state(f, storage, mask=None):
    """The pre-collision state a periodic or walled lattice holds after
    set_populations(f): f itself in FP64 storage, f - w rounded to nearest
    even in FP32 / FP16 storage plus w (computed on the host from the seeded
    state; solid nodes 0)."""
    f = np.asarray(f, dtype=np.float64)
    if storage == "f64":
        out = f.copy()
    else:
        dt = np.float32 if storage == "f32" else np.float16
        out = (f - W9).astype(dt).astype(np.float64) + W9
    if mask is not None:
        out[:, np.asarray(mask) != 0] = 0.0
    return out
