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
