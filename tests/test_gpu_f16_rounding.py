"""FP16 storage, population by population: one sweep rounds each stored
value once.

The sweep stores g_i = f*_i - w_i (the shifted form; the weights w_i of
Sec. II.B) in FP16 and computes in FP32.  Starting from a state that is
exactly representable in the storage (the seeded state rounded to FP16 (f - w)
on the host, which is exactly what set_populations stores), the
FP64 oracle's post-collision g_i is the exact value up to FP64 rounding; the
stored g_i must then lie within half an FP16 unit in the last place of it,
plus a margin for the FP32 arithmetic before the final rounding (terms of
order 0.1 at 2^-24 relative: 2e-7 absolute, against half-ulps near 1e-5 for
the typical |g_i| ~ 0.01 here).  A wrong weight, sign or half in the FP16
output path misses this by orders of magnitude.  Nearly every value also
equals the FP16 rounding of the oracle's value exactly (only values within
the FP32 margin of a rounding tie may differ): at least 99%.

Cases: open even and odd widths (two columns per lane, moments summed from
the stored halves; the odd width's last column takes column 0 as its right
edge), a width of 1 mod 128 (one column per lane), and walls with obstacles
and a body force (link map), even and odd.  Solid nodes are excluded (the oracle
outputs 0 there; the sweep leaves them untouched).
"""
import numpy as np
import pytest

import f16_harness
import oracle
from gpu_util import say
from paper_2312_10318_amd import inputs

pytestmark = pytest.mark.gpu

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
MARGIN = 2e-7


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_10318_amd import lattice
    return lattice


def _half_ulp(x):
    """Half the FP16 spacing of the binade of |x| (subnormal spacing below
    2^-14)."""
    a = np.abs(x)
    _, e = np.frexp(np.where(a > 0, a, 1.0))
    return 0.5 * np.maximum(np.ldexp(1.0, e - 11), 2.0 ** -24)


def _case(seed, nx, ny, walls):
    rng = np.random.default_rng(seed)
    f = inputs.random_populations(rng, (ny, nx), amp=0.1)
    mask = None
    g = (0.0, 0.0)
    if walls:
        mask = np.zeros((ny, nx), np.uint8)
        mask[0] = mask[-1] = 1
        for _ in range(nx * ny // 150):
            mask[rng.integers(1, ny - 1), rng.integers(0, nx)] = 1
        f[:, mask.astype(bool)] = 0.0
        g = tuple(rng.uniform(-1e-4, 1e-4, 2))
    tau1 = float(rng.uniform(0.52, 2.0))
    tau2 = float(rng.uniform(0.5, 3.0))
    return f, mask, g, tau1, tau2


@pytest.mark.parametrize("nx, ny, walls, cols", [(322, 41, False, 2), (131, 37, False, 2),
                                                (129, 37, False, 1), (322, 41, True, 2),
                                                (131, 41, True, 2)])
def test_fp16_one_step_rounds_each_population_once(L, nx, ny, walls, cols):
    f, mask, g, tau1, tau2 = _case(17 + nx + int(walls), nx, ny, walls)
    lat = L.Lattice(nx, ny, tau1, tau2, g=g, mask=mask, storage="f16").set_populations(f)
    assert lat.tuning()[3] == cols
    f0 = f16_harness.to_f16_storage(f, mask)
    lat.step(1)
    f1 = lat.get_populations().cpu().numpy()
    lat.close()
    ref = oracle.step(f0, tau1, tau2, g[0], g[1], mask)
    fluid = np.ones((ny, nx), bool) if mask is None else ~mask.astype(bool)
    gr = (ref - W[:, None, None])[:, fluid]
    gg = (f1 - W[:, None, None])[:, fluid]
    err = np.abs(gg - gr)
    bound = _half_ulp(gr) + MARGIN
    worst = float(np.max(err / bound))
    exact = float(np.mean(gg.astype(np.float16) == gr.astype(np.float16)))
    say("case: FP16 one step %dx%d walls=%s cols=%d: max |g - g_oracle| / (half-ulp + %.0e) = "
        "%.3f, equal to the rounded oracle value: %.4f" % (nx, ny, walls, cols, MARGIN, worst, exact))
    assert worst <= 1.0
    assert exact >= 0.99
