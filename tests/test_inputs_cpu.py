"""Synthetic input generators (no GPU)."""
import numpy as np

from paper_2312_10318_amd import inputs


def test_taylor_green_device_path_gives_the_host_bits():
    """Fields built with torch from the per-axis factors equal the numpy
    fields exactly (same operations in the same order)."""
    for n, kw in ((16, {}), (257, {"seed": 5}), (128, {"nu": 0.03, "t": 100.0, "seed": 2}),
                  (32, {"seed": None})):
        host = inputs.taylor_green(n, 0.01, **kw)
        dev = inputs.taylor_green(n, 0.01, device="cpu", **kw)
        for h, d in zip(host, dev):
            assert h.shape == tuple(d.shape) == (n, n)
            assert np.array_equal(h, d.numpy())


def test_taylor_green_is_the_stated_field():
    """Spot values of the closed form: u_x = -u0 cos(2 pi x) sin(2 pi y),
    u_y = u0 cos(2 pi y) sin(2 pi x), rho = 1 - 3 u0^2/4 (cos 4 pi x + cos 4 pi y)."""
    n, u0 = 8, 0.02
    rho, ux, uy = inputs.taylor_green(n, u0, seed=None)
    for j, i in ((0, 0), (1, 2), (5, 3)):
        x, y = i / n, j / n
        assert abs(ux[j, i] + u0 * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)) < 1e-17
        assert abs(uy[j, i] - u0 * np.cos(2 * np.pi * y) * np.sin(2 * np.pi * x)) < 1e-17
        r = 1 - 3 * u0 ** 2 / 4 * (np.cos(4 * np.pi * x) + np.cos(4 * np.pi * y))
        assert abs(rho[j, i] - r) < 1e-15
