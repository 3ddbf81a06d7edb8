"""Seeded synthetic inputs and the named workloads.

This module holds no arithmetic of the model itself: it only draws seeded
noise, lays out initial density fields and heater profiles from numbers the
caller supplies, and names the workload sizes and parameters.  Both the GPU
library's tests and the CPU oracle take their inputs from here.

Initial state (Sec. 3.1 of arXiv:1501.03857): liquid below its vapour at the
coexistence densities, uniform saturation temperature, small random density
fluctuations to seed bubble formation (Sec. 3.2).  The fluctuation is
additive uniform noise in [-A, A) from SplitMix64 (Steele, Lea and Flood,
OOPSLA 2014; reference code by S. Vigna), used as a counter-based generator:
the value of cell c = j*nx + i is the (c+1)-th output of the generator seeded
with ``seed``, mapped to [0, 1) by its top 53 bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """The (counter+1)-th SplitMix64 output for a generator seeded with seed."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (np.asarray(counter, dtype=np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) from the top 53 bits of SplitMix64 outputs 1..n."""
    bits = splitmix64(seed, np.arange(n, dtype=np.uint64)) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)


def layered_density(nx: int, ny: int, rho_L: float, rho_V: float, liquid_rows: int,
                    noise_amp: float, seed: int) -> np.ndarray:
    """rho0[j, i] = (rho_L if j < liquid_rows else rho_V) + A (2u - 1)."""
    u = uniform01(seed, nx * ny).reshape(ny, nx)
    base = np.where(np.arange(ny)[:, None] < liquid_rows, rho_L, rho_V) * np.ones((1, nx))
    return base + noise_amp * (2.0 * u - 1.0)


def layered_density3(nx: int, ny: int, nz: int, rho_L: float, rho_V: float, liquid_rows: int,
                     noise_amp: float, seed: int) -> np.ndarray:
    """Three-dimensional lattices: rho0[k, j, i] = (rho_L if j < liquid_rows
    else rho_V) + A (2u - 1), u from counter (k ny + j) nx + i."""
    u = uniform01(seed, nx * ny * nz).reshape(nz, ny, nx)
    base = np.where(np.arange(ny)[None, :, None] < liquid_rows, rho_L, rho_V) * np.ones((nz, 1, nx))
    return base + noise_amp * (2.0 * u - 1.0)


def smooth_layered_density(nx: int, ny: int, rho_L: float, rho_V: float, liquid_rows: int, width: float,
                           noise_amp: float, seed: int) -> np.ndarray:
    """The liquid layer with a tanh interface of half-width `width` at
    y = liquid_rows - 1/2: rho0[j, i] = rho_V + (rho_L - rho_V)(1 - tanh((j +
    1/2 - liquid_rows)/width))/2 + A (2u - 1).  At density ratios far above
    the paper's, the force of a one-row jump empties the vapour row next to
    it in the first steps; a smooth start avoids that."""
    u = uniform01(seed, nx * ny).reshape(ny, nx)
    j = np.arange(ny, dtype=np.float64)[:, None]
    base = rho_V + (rho_L - rho_V) * 0.5 * (1.0 - np.tanh((j + 0.5 - liquid_rows) / width))
    return base * np.ones((1, nx)) + noise_amp * (2.0 * u - 1.0)


def smooth_layered_density3(nx: int, ny: int, nz: int, rho_L: float, rho_V: float, liquid_rows: int,
                            width: float, noise_amp: float, seed: int) -> np.ndarray:
    """smooth_layered_density on three-dimensional lattices (u from counter
    (k ny + j) nx + i)."""
    u = uniform01(seed, nx * ny * nz).reshape(nz, ny, nx)
    j = np.arange(ny, dtype=np.float64)[None, :, None]
    base = rho_V + (rho_L - rho_V) * 0.5 * (1.0 - np.tanh((j + 0.5 - liquid_rows) / width))
    return base * np.ones((nz, 1, nx)) + noise_amp * (2.0 * u - 1.0)


def heater_profile(nx: int, T_s: float, T_heater: float, lo: int = 0, hi: Optional[int] = None) -> np.ndarray:
    """Bottom-wall temperature: T_heater on cells [lo, hi), T_s elsewhere."""
    hi = nx if hi is None else hi
    Tb = np.full(nx, T_s, dtype=np.float64)
    Tb[lo:hi] = T_heater
    return Tb


@dataclass(frozen=True)
class Workload:
    """A named lattice workload.  Temperatures are in units of T_c (the
    caller converts with the T_c of the same EOS parameters)."""
    name: str
    nx: int
    ny: int
    precision: str                 # "fp64" or "fp32"
    steps: int
    a: float = 2.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    omega: float = 0.344
    Ts_over_Tc: float = 0.86
    sigma: float = 1.2
    g: float = 3e-5
    Gw_bottom: float = 0.0
    dT_over_Tc: float = 0.05
    heater: Tuple[int, int] = (0, -1)  # [lo, hi); hi = -1 means the full width
    liquid_frac: float = 0.6
    noise_amp: float = 1e-3
    seed: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def liquid_rows(self) -> int:
        return int(np.floor(self.liquid_frac * self.ny))

    @property
    def heater_range(self) -> Tuple[int, int]:
        lo, hi = self.heater
        return lo, (self.nx if hi < 0 else hi)

    def heater_T(self, Tc: float) -> np.ndarray:
        lo, hi = self.heater_range
        T_s = self.Ts_over_Tc * Tc
        return heater_profile(self.nx, T_s, T_s + self.dT_over_Tc * Tc, lo, hi)

    def density(self, rho_L: float, rho_V: float) -> np.ndarray:
        return layered_density(self.nx, self.ny, rho_L, rho_V, self.liquid_rows, self.noise_amp, self.seed)

    def resized(self, nx: int, ny: int, **kw) -> "Workload":
        return replace(self, nx=nx, ny=ny, **kw)


def scaled_gravity(ny: int, a: float, g_paper: float = 3e-5, ny_paper: int = 150, a_paper: float = 3.0 / 49.0) -> float:
    """Gravity for a lattice of height ny that keeps the paper's ratio of the
    hydrostatic load to the saturation pressure (600x150, a = 3/49, g = 3e-5,
    Sec. 3.1).  Buoyancy is measured against the domain-mean density
    (Eq. (9)), so the vapour layer is pushed up with (rho_ave - rho_V) g per
    node; over a tall layer that load exceeds p_sat (which scales with a) and
    the vapour next to the interface empties.  Scaling g with
    (ny_paper / ny) (a / a_paper) keeps the load at the paper's fraction."""
    return g_paper * (ny_paper / ny) * (a / a_paper)


# Wall strengths of the contact-angle labels at a = 2/49 (the workloads'
# EOS), measured by the sessile-drop calibration on the GPU path
# (experiments.calibrate_wall_strength: 160x60 drops of radius 22, FP64, 5000
# steps, G_w grid step 0.05, linear interpolation): theta(G_w) = 33.7, 43.1,
# 58.4, 85.6, 131.5 deg at G_w = -0.1, 0, 0.1, 0.2, 0.3; above about 0.33 the
# drop leaves the wall.  The same harness at a = 3/49 gives 50 and 55.5 deg at
# G_w = 0.062 and 0.103, against the paper's 0.065 and 0.105 (Sec. 3.3).
CONTACT_ANGLE_GW = {40: -0.030, 60: 0.107, 90: 0.211, 120: 0.278}

# Small plain case: 128x64, FP64, a 32-cell heater at 0.05 T_c, 1000 steps.
PLAIN_128x64 = Workload("plain_128x64_fp64", 128, 64, "fp64", 1000, dT_over_Tc=0.05,
                        heater=(48, 80), Gw_bottom=0.0, seed=1)
# Single large instance: 1024x512, FP32 storage, full-width heater at 0.10 T_c,
# contact angle ~60 deg, 20000 steps; gravity scaled to the lattice height
# (with g = 3e-5 the 205-row vapour layer carries a buoyant load above p_sat
# and empties within ~1000 steps).
LARGE_1024x512 = Workload("large_1024x512_fp32", 1024, 512, "fp32", 20000, dT_over_Tc=0.10,
                          heater=(0, -1), Gw_bottom=CONTACT_ANGLE_GW[60], seed=2,
                          g=scaled_gravity(512, 2.0 / 49.0))
# Bandwidth-truth supplement: the same physics on a lattice far larger than
# the 256 MB last-level cache.
LARGE_4096x2048 = Workload("large_4096x2048_fp32", 4096, 2048, "fp32", 2000, dT_over_Tc=0.10,
                           heater=(0, -1), Gw_bottom=CONTACT_ANGLE_GW[60], seed=2,
                           g=scaled_gravity(2048, 2.0 / 49.0))
# Adjoint case: 256x128, heater i in [96, 160) at 0.10 T_c, G_w = 0.065, 400 steps.
ADJOINT_256x128 = Workload("adjoint_256x128", 256, 128, "fp64", 400, dT_over_Tc=0.10,
                           heater=(96, 160), Gw_bottom=0.065, seed=4)

SWEEP_SIZES = ((256, 128), (384, 192), (512, 256))


def sweep_workloads(steps: int = 10000):
    """48 boiling-curve instances: 12 superheats x 4 contact-angle labels, sizes
    drawn from SWEEP_SIZES by SplitMix64(3, i) mod 3, seeds 1000 + i."""
    out = []
    pick = splitmix64(3, np.arange(48, dtype=np.uint64)) % np.uint64(3)
    i = 0
    for k in range(1, 13):
        for ang in (40, 60, 90, 120):
            nx, ny = SWEEP_SIZES[int(pick[i])]
            out.append(Workload(f"sweep_{i:02d}", nx, ny, "fp32", steps, dT_over_Tc=0.02 * k,
                                heater=(0, -1), Gw_bottom=CONTACT_ANGLE_GW[ang], seed=1000 + i,
                                g=scaled_gravity(ny, 2.0 / 49.0), extra={"angle": ang}))
            i += 1
    return out


def batch_adjoint_workloads(steps: int = 600):
    """16 lattices of 384x192 (FP32) for the batched adjoint: superheats
    0.04, 0.08, 0.12, 0.16 T_c times the four contact-angle labels, full-width
    heaters, seeds 2000 + i, gravity scaled to the lattice height."""
    out = []
    i = 0
    for dT in (0.04, 0.08, 0.12, 0.16):
        for ang in (40, 60, 90, 120):
            out.append(Workload(f"badj_{i:02d}", 384, 192, "fp32", steps, dT_over_Tc=dT, heater=(0, -1),
                                Gw_bottom=CONTACT_ANGLE_GW[ang], seed=2000 + i,
                                g=scaled_gravity(192, 2.0 / 49.0), extra={"angle": ang}))
            i += 1
    return out
