"""Measurements on fields shared by the oracle and GPU physics tests."""
import numpy as np


def cap_angle(rho, rl, rv):
    """Contact angle (liquid side) of a circular cap sitting on the bottom
    wall: base width w on row 1 (the first fluid row) and apex height h above
    it, tan(theta/2) = 2h/w, with the interface located by linear
    interpolation at the mean of the two densities."""
    mid = 0.5 * (rl + rv)
    nx = rho.shape[1]
    c = rho[:, nx // 2]
    j = np.where(c > mid)[0].max()
    top = j + (c[j] - mid) / (c[j] - c[j + 1])
    r1 = rho[1]
    idx = np.where(r1 > mid)[0]
    i0, i1 = idx.min(), idx.max()
    assert 0 < i0 and i1 < nx - 1, "drop touches the periodic seam"
    w = (i1 - i0) + (r1[i0] - mid) / (r1[i0] - r1[i0 - 1]) + (r1[i1] - mid) / (r1[i1] - r1[i1 + 1])
    return 2 * np.degrees(np.arctan(2 * (top - 1) / w))
