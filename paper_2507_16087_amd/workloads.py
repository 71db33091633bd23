"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws media (sound speed c, density rho, absorption alpha),
source lists, receiver lattices and request streams.  It holds none of the
solver's arithmetic, so both the CPU oracle tests and the GPU path may use it.

Workloads (all SI units; alpha in Np/m):

* ``disc2d``     -- 2-D 128x128 water grid at 1 MHz, dx = 0.25 mm, with one
  circular inclusion (c 1800, rho 1500) of radius 32 cells at the centre and a
  unit point source at cell (32, 64); 16-cell absorbing layer.
* ``random3d``   -- 3-D N^3 grid at dx = lambda/6, Gaussian-filtered random
  fields (sigma 4 cells) uniform-mapped to c in [1400, 1700], rho in
  [900, 1200], alpha in [0, 0.5] dB/cm/MHz; unit point source at the centre.
* ``shell3d``    -- 3-D 256^3 skull-like case at 500 kHz, dx = 0.5 mm: a
  spherical shell (radii 64-70 mm) of bone-like material modulated by porosity
  noise, insonified by a focused bowl (64 mm radius of curvature, 60 mm
  aperture) rasterised as a surface of point sources.  It stands in for the
  paper's transcranial benchmark, whose skull mesh is not used here.
* ``disks2d``    -- the paper's 2-D disks example (256^2, 0.5 mm, 500 kHz,
  inclusions of c 3500, rho 3000, alpha 10 dB/cm, line source at the top).
* ``requests``   -- a Poisson stream of mixed-size random3d solves.
* ``inversion``  -- the random3d medium with 8 shots on one face, 128
  receivers on the opposite face and a smooth +/-3 % bump for the data model.

Cell centres sit at integer indices times dx; arrays are C-ordered with the
last axis contiguous.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np
from scipy.special import erf

WATER_C = 1500.0
WATER_RHO = 1000.0
PML_CELLS = 16
DB_PER_NEPER = 20.0 / math.log(10.0)  # 8.6859 dB per neper


def db_cm_mhz_to_np_m(a_db, f_hz):
    """Absorption in dB/(cm MHz) at frequency f -> Np/m."""
    return np.asarray(a_db) * (f_hz / 1e6) * 100.0 / DB_PER_NEPER


@dataclasses.dataclass
class Problem:
    """One solve: grid, medium and a sparse pressure source."""

    name: str
    ndim: int
    shape: Tuple[int, ...]
    dx: float
    omega: float
    c: np.ndarray
    rho: np.ndarray
    alpha: np.ndarray
    src_idx: np.ndarray          # flat cell indices of pressure sources
    src_val: np.ndarray          # complex source values s_p at those cells
    pml_cells: int = PML_CELLS

    @property
    def ncell(self) -> int:
        return int(np.prod(self.shape))

    def dense_source(self) -> np.ndarray:
        """Dense complex pressure source s_p on the grid."""
        s = np.zeros(self.ncell, dtype=np.complex128)
        np.add.at(s, self.src_idx, self.src_val)
        return s.reshape(self.shape)


def uniform_mapped_field(shape, sigma_cells, lo, hi, seed) -> np.ndarray:
    """White noise -> periodic Gaussian filter -> standardise -> normal CDF ->
    affine map to [lo, hi].  The result is marginally uniform on [lo, hi]."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    axes = tuple(range(len(shape)))
    wh = np.fft.rfftn(w, axes=axes)
    filt = np.ones(wh.shape)
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = 2.0 * np.pi * np.fft.rfftfreq(n)
        else:
            k = 2.0 * np.pi * np.fft.fftfreq(n)
        bshape = [1] * len(shape)
        bshape[ax] = k.size
        filt = filt * np.exp(-0.5 * (sigma_cells * k.reshape(bshape)) ** 2)
    f = np.fft.irfftn(wh * filt, s=shape, axes=axes)
    z = (f - f.mean()) / f.std()
    u = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    return lo + (hi - lo) * u


def disc2d(n: int = 128) -> Problem:
    """2-D disc inclusion at 1 MHz, dx = 0.25 mm (lambda/6 in water)."""
    f = 1e6
    dx = 0.25e-3
    shape = (n, n)
    c = np.full(shape, WATER_C)
    rho = np.full(shape, WATER_RHO)
    alpha = np.zeros(shape)
    ctr = n // 2
    rad = n // 4
    i0, i1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    inside = (i0 - ctr) ** 2 + (i1 - ctr) ** 2 < rad ** 2   # strictly inside
    c[inside] = 1800.0
    rho[inside] = 1500.0
    src = np.array([(n // 4) * n + n // 2], dtype=np.int64)   # cell (32, 64)
    return Problem("disc2d", 2, shape, dx, 2 * np.pi * f, c, rho, alpha, src,
                   np.array([1.0 + 0j]))


def disks2d(n: int = 256) -> Problem:
    """2-D example of the paper's first experiment: 256 x 256 grid, 0.5 mm,
    500 kHz, water background, circular inclusions of c 3500 m/s, rho 3000
    kg/m^3 and alpha 10 dB/cm, and a planar line source near the top edge.
    The paper gives no positions or sizes; here one disc of each property
    (radius 16 mm) sits on the axis below the source and the three overlap
    pairwise in lens-shaped regions."""
    f = 5e5
    dx = 0.5e-3
    shape = (n, n)
    c = np.full(shape, WATER_C)
    rho = np.full(shape, WATER_RHO)
    a_db = np.zeros(shape)
    i0, i1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s = n / 256.0
    rad = 32 * s
    centres = {"c": (112 * s, 96 * s), "rho": (112 * s, 160 * s), "alpha": (160 * s, 128 * s)}
    for key, (y, x) in centres.items():
        inside = (i0 - y) ** 2 + (i1 - x) ** 2 < rad ** 2
        if key == "c":
            c[inside] = 3500.0
        elif key == "rho":
            rho[inside] = 3000.0
        else:
            a_db[inside] = 10.0
    alpha = a_db * 100.0 / DB_PER_NEPER          # 10 dB/cm at 500 kHz -> Np/m
    row = int(round(40 * s))
    cols = np.arange(int(48 * s), int(208 * s))
    idx = np.ravel_multi_index((np.full(cols.size, row), cols), shape).astype(np.int64)
    return Problem(f"disks2d_{n}", 2, shape, dx, 2 * np.pi * f, c, rho, alpha, idx,
                   np.ones(idx.size, dtype=np.complex128))


def random_medium(shape, seed: int, f_hz: float, sigma: float = 4.0):
    """c, rho, alpha of the random heterogeneous workload (three seeds)."""
    c = uniform_mapped_field(shape, sigma, 1400.0, 1700.0, seed)
    rho = uniform_mapped_field(shape, sigma, 900.0, 1200.0, seed + 1)
    a_db = uniform_mapped_field(shape, sigma, 0.0, 0.5, seed + 2)
    return c, rho, db_cm_mhz_to_np_m(a_db, f_hz)


def random3d(n: int = 128, f_hz: float = 1e6, seed: int = 2507,
             src: Optional[Tuple[int, int, int]] = None) -> Problem:
    """3-D random heterogeneous medium, dx = lambda/6 at f in water."""
    shape = (n, n, n)
    dx = WATER_C / (6.0 * f_hz)
    c, rho, alpha = random_medium(shape, seed, f_hz)
    if src is None:
        src = (n // 2, n // 2, n // 2)
    idx = np.array([np.ravel_multi_index(src, shape)], dtype=np.int64)
    return Problem(f"random3d_{n}", 3, shape, dx, 2 * np.pi * f_hz, c, rho,
                   alpha, idx, np.array([1.0 + 0j]))


def shell3d(n: int = 256, seed: int = 2507) -> Problem:
    """Skull-like shell at 500 kHz, dx = 0.5 mm, with a focused-bowl source.

    Geometry (mm, domain n*0.5 mm on a side): the shell sphere is centred at
    (100, 64, 64) * (n/256) with radii 64-70 mm, so it crosses the domain as a
    curved plate.  The bowl axis is +x with focus at (76, 64, 64) mm, radius of
    curvature 64 mm and aperture diameter 60 mm; its rim lies outside the shell.
    Shell material: c = 3200 - 400 phi, rho = 2000 - 150 phi,
    alpha = 2 + 6 phi dB/cm/MHz with porosity phi uniform-mapped (sigma 1 mm).
    """
    f = 5e5
    dx = 0.5e-3
    shape = (n, n, n)
    s = n / 256.0
    mm = 1e-3
    ctr = np.array([100.0, 64.0, 64.0]) * s * mm
    r_in, r_out = 64.0 * mm * s, 70.0 * mm * s
    phi = uniform_mapped_field(shape, 2.0, 0.0, 1.0, seed + 10)
    ax = np.arange(n) * dx
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    r = np.sqrt((X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + (Z - ctr[2]) ** 2)
    shell = (r >= r_in) & (r <= r_out)
    del X, Y, Z, r
    c = np.full(shape, WATER_C)
    rho = np.full(shape, WATER_RHO)
    a_db = np.zeros(shape)
    c[shell] = 3200.0 - 400.0 * phi[shell]
    rho[shell] = 2000.0 - 150.0 * phi[shell]
    a_db[shell] = 2.0 + 6.0 * phi[shell]
    alpha = db_cm_mhz_to_np_m(a_db, f)
    idx = bowl_cells(shape, dx, focus=np.array([76.0, 64.0, 64.0]) * s * mm,
                     roc=64.0 * mm * s, aperture=60.0 * mm * s)
    return Problem(f"shell3d_{n}", 3, shape, dx, 2 * np.pi * f, c, rho, alpha,
                   idx, np.ones(idx.size, dtype=np.complex128))


def bowl_cells(shape, dx, focus, roc, aperture) -> np.ndarray:
    """Flat indices of cells whose centre lies within dx/2 of a spherical cap.

    The cap is the part of the sphere of radius ``roc`` about ``focus`` whose
    polar angle from the -x axis is at most asin(aperture / (2 roc)); its apex
    is at focus - roc * e_x."""
    n0 = shape[0]
    theta_max = math.asin(aperture / (2.0 * roc))
    out = []
    ax = np.arange(shape[1]) * dx
    Y, Z = np.meshgrid(ax, ax, indexing="ij")
    for i in range(n0):
        x = i * dx
        dxv = x - focus[0]
        if dxv > 0:
            continue
        d = np.sqrt(dxv ** 2 + (Y - focus[1]) ** 2 + (Z - focus[2]) ** 2)
        cosang = -dxv / np.maximum(d, 1e-30)
        sel = (np.abs(d - roc) <= 0.5 * dx) & (cosang >= math.cos(theta_max))
        jj, kk = np.nonzero(sel)
        out.append(np.ravel_multi_index((np.full(jj.size, i), jj, kk), shape))
    return np.sort(np.concatenate(out)).astype(np.int64)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    problem: Problem


def request_stream(count: int = 64, rate_hz: float = 4.0, seed: int = 4242,
                   sizes=(64, 96, 128, 192)) -> List[Request]:
    """Poisson arrivals of random3d solves of mixed size and frequency."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        n = int(rng.choice(sizes))
        f = float(rng.uniform(0.25e6, 1.0e6))
        lo, hi = PML_CELLS, n - PML_CELLS
        src = tuple(int(v) for v in rng.integers(lo, hi, size=3))
        prob = random3d(n, f, seed=1000 + 3 * i, src=src)
        prob.name = f"req{i}_{n}"
        out.append(Request(i, t, prob))
    return out


def lattice(lo: int, hi: int, count: int) -> np.ndarray:
    """``count`` evenly spaced integer positions in [lo, hi)."""
    return np.array([int(lo + (hi - lo) * (j + 0.5) / count) for j in range(count)])


@dataclasses.dataclass
class Inversion:
    model: Problem               # medium used for the forward model
    true_c: np.ndarray
    true_rho: np.ndarray
    shots: List[np.ndarray]      # flat source index per shot (one cell each)
    receivers: np.ndarray        # flat receiver indices


def inversion(n: int = 128, seed: int = 2507, shots_yz=(2, 4),
              receivers_yz=(16, 8), pml: int = PML_CELLS) -> Inversion:
    """8 single-cell shots at x index ~n*20/128, 128 receivers at ~n*107/128
    (kept two cells clear of the absorbing layer), and a true medium with a
    smooth bump: c*(1+0.03 b), rho*(1-0.03 b)."""
    base = random3d(n, 1e6, seed)
    base.pml_cells = pml
    shape = base.shape
    lo, hi = pml, n - pml
    xs = max(pml + 2, int(round(20 * n / 128)))
    xr = min(n - pml - 3, int(round(107 * n / 128)))
    shots = []
    for jy in lattice(lo, hi, shots_yz[0]):
        for jz in lattice(lo, hi, shots_yz[1]):
            shots.append(np.array([np.ravel_multi_index((xs, jy, jz), shape)]))
    rec = []
    for jy in lattice(lo, hi, receivers_yz[0]):
        for jz in lattice(lo, hi, receivers_yz[1]):
            rec.append(np.ravel_multi_index((xr, jy, jz), shape))
    i = np.arange(n) - n / 2
    I0, I1, I2 = np.meshgrid(i, i, i, indexing="ij")
    b = np.exp(-(I0 ** 2 + I1 ** 2 + I2 ** 2) / (2.0 * (10.0 * n / 128) ** 2))
    return Inversion(base, base.c * (1 + 0.03 * b), base.rho * (1 - 0.03 * b),
                     shots, np.array(rec, dtype=np.int64))


def smooth_direction(shape, seed: int, sigma: float = 4.0) -> np.ndarray:
    """Zero-mean smooth random field with unit max-abs (for directional tests)."""
    v = uniform_mapped_field(shape, sigma, -1.0, 1.0, seed)
    v = v - v.mean()
    return v / np.abs(v).max()


def small_random(shape, seed: int, f_hz: float = 1e6, contrast: float = 1.0):
    """Small heterogeneous media for quick parity cases (any ndim)."""
    rng = np.random.default_rng(seed)
    c = WATER_C * (1.0 + 0.2 * contrast * rng.uniform(-1, 1, shape))
    rho = WATER_RHO * (1.0 + 0.3 * contrast * rng.uniform(-1, 1, shape))
    alpha = db_cm_mhz_to_np_m(rng.uniform(0.0, 0.5, shape), f_hz)
    return c, rho, alpha


def random_complex(count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(count) + 1j * rng.standard_normal(count)
