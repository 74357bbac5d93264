"""Seeded synthetic inputs and workload recipes.

This module is the only code shared by the product path and the CPU oracle's
tests. It holds no arithmetic of the ocean method itself: it builds the inputs
the method is given -- layer thicknesses, the wet-layer count of every column
(bathymetry), the initial temperature, wind stress and the restoring target --
from a counter-based random generator, and it lists the workloads.

Stand-ins. The paper's realistic runs use ECCO2 forcing and real bathymetry and
its aqua-planet runs an idealised two-ridge geometry (paper Sec. 6); neither is
available here. The generators below give inputs of the same shapes and sizes:
near-global lat-lon grids periodic in longitude, seamount-and-ridge bathymetry
up to 5.5 km deep with two ridges that split the ocean into two basins north of
50S, exponential stratification with small seeded noise, a zonal wind stress
that varies as cos(latitude), and surface temperature restoring.

Random numbers: splitmix64 (Steele, Lea and Flood, 2014) evaluated at a counter,
so any element can be drawn independently of the others. A draw is
mix64(base(seed, stream) + (n + 1) * GOLDEN) with base = mix64(seed ^ (stream << 32)).
Uniforms take the top 53 bits; normals use Box-Muller (cosine branch) on the
uniform pair drawn at counters 2n and 2n+1. Streams: 0 temperature noise,
1 bathymetry, 2 ensemble-member parameters, 3 salinity noise.
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import math
import os
from typing import Dict, Optional

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_TEMPERATURE = 0
STREAM_BATHYMETRY = 1
STREAM_MEMBERS = 2
STREAM_SALINITY = 3


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _base(seed: int, stream: int) -> np.uint64:
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (np.uint64(stream) << np.uint64(32))
    return _mix64(np.array([s], dtype=np.uint64))[0]


def draw_u64(seed: int, stream: int, counters: np.ndarray) -> np.ndarray:
    """Raw 64-bit splitmix64 outputs at the given counters."""
    n = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _base(seed, stream) + (n + np.uint64(1)) * GOLDEN
    return _mix64(z)


def uniform(seed: int, stream: int, counters: np.ndarray) -> np.ndarray:
    """Uniform deviates in [0, 1) from the top 53 bits."""
    return (draw_u64(seed, stream, counters) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, counters: np.ndarray) -> np.ndarray:
    """Standard normal deviates, Box-Muller cosine branch on draws 2n and 2n+1."""
    n = np.asarray(counters, dtype=np.uint64)
    u1 = uniform(seed, stream, n * np.uint64(2))
    u2 = uniform(seed, stream, n * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


def _parallel_blocks(n: int, fn, block: int = 64):
    """Run fn(start, stop) over [0, n) in blocks on a thread pool (numpy releases
    the GIL in its array loops); blocks are disjoint, so the result does not
    depend on scheduling."""
    spans = [(a, min(a + block, n)) for a in range(0, n, block)]
    if len(spans) <= 1:
        for a, b in spans:
            fn(a, b)
        return
    workers = min(len(spans), os.cpu_count() or 1, 16)
    with _cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(fn, a, b) for a, b in spans]:
            f.result()


@dataclasses.dataclass(frozen=True)
class Workload:
    """A synthetic basin: grid, constants, forcing recipe and stepping parameters."""

    name: str
    nx: int
    ny: int
    nz: int
    coords: str = "cartesian"          # "cartesian" beta-plane or "latlon"
    periodic_x: bool = False
    periodic_y: bool = False
    x0: float = 0.0                     # Cartesian: m. lat-lon: longitude of the west edge (deg)
    y0: float = 0.0                     # lat-lon: latitude of the south edge (deg)
    dx: float = 50e3                    # Cartesian: m. lat-lon: degrees of longitude
    dy: float = 50e3                    # Cartesian: m. lat-lon: degrees of latitude
    depth: float = 4000.0
    bathymetry: str = "flat"            # "flat" or "seamounts"
    halo: int = 3
    f0: float = 1e-4
    beta: float = 2e-11
    radius: float = 6.371e6
    omega: float = 7.292115e-5
    g: float = 9.81
    alpha: float = 2e-4
    rho0: float = 1025.0
    t_ref: float = 0.0
    kappa: float = 1e-5
    dt: float = 1200.0
    n_substeps: int = 30
    chi: float = 0.1                    # AB2 offset (quasi-second-order form)
    pgf_weight: float = 0.75            # pressure gradient from T^n + pgf_weight dt Ghat_T
    tau0: float = 0.1                   # wind-stress amplitude, N/m^2
    restore_days: float = 0.0           # <= 0: no restoring
    strat_t0: float = 20.0              # T = strat_t0 * exp(z / strat_scale) + noise
    strat_scale: float = 1000.0
    noise_std: float = 0.01
    seed: int = 0
    # salinity and the nonlinear equation of state (off in the benchmarked
    # configurations, which are temperature-only with a linear equation of state)
    salinity: bool = False
    # S = sal_s0 - sal_ds exp(z / strat_scale) + noise_std_s N(0, 1): fresher at the surface
    sal_s0: float = 35.0
    sal_ds: float = 1.0
    noise_std_s: float = 0.01
    # (a0, b0, lambda1, lambda2, mu1, mu2, nu, t0, s0) of the simplified seawater
    # equation of state (Roquet et al. 2015 form): kg/m^3/K, kg/m^3/(g/kg), 1/K,
    # 1/(g/kg), 1/(K m), 1/((g/kg) m), kg/m^3/(K g/kg), degC, g/kg
    eos: tuple = (1.6550e-1, 7.6554e-1, 5.9520e-2, 5.4914e-4, 1.4970e-4, 1.1090e-5, 2.4341e-3, 10.0, 35.0)
    # momentum advection: "flux" (flux form, the benchmarked configurations) or
    # "vector_invariant"
    momentum_form: str = "flux"

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# Closed beta-plane basin, 64x64x16, dx = dy = 50 km, 4 km flat bottom, 30 substeps.
BETA_BASIN_64 = Workload(name="beta_basin_64x64x16", nx=64, ny=64, nz=16)

# Near-global lat-lon at 1/4 degree: 1440x600x50 over 80S-80N, periodic in longitude,
# seamount-and-ridge bathymetry to 5.5 km, restoring, dt = 600 s, 60 substeps.
LATLON_QUARTER = Workload(
    name="latlon_1440x600x50", nx=1440, ny=600, nz=50, coords="latlon", periodic_x=True,
    x0=0.0, y0=-80.0, dx=0.25, dy=160.0 / 600.0, depth=5500.0, bathymetry="seamounts",
    dt=600.0, n_substeps=60, restore_days=30.0)

# One GPU's share at 1/12 degree: 4320x1800x100 over 75S-75N, 5-point halos,
# dt = 300 s, 60 substeps.
LATLON_TWELFTH = Workload(
    name="latlon_4320x1800x100", nx=4320, ny=1800, nz=100, coords="latlon", periodic_x=True,
    x0=0.0, y0=-75.0, dx=1.0 / 12.0, dy=1.0 / 12.0, depth=5500.0, bathymetry="seamounts",
    halo=5, dt=300.0, n_substeps=60, restore_days=30.0)

WORKLOADS = {w.name: w for w in (BETA_BASIN_64, LATLON_QUARTER, LATLON_TWELFTH)}


def ensemble_members(n: int = 64, seed: int = 0, precision_note: str = "fp32"):
    """Members of a batched ensemble of closed beta-plane basins.

    Member m draws five uniforms at counters 5m..5m+4 of the member stream:
    nx in {128, 160, ..., 512}, ny in {128, 160, ..., 256}, nz in {32, 40, ..., 64},
    wind amplitude tau0 ~ U(0.05, 0.2) N/m^2 and stratification scale ~ U(500, 1500) m.
    Every basin has dx = dy = 50 km, a 4 km flat bottom, dt = 1200 s and 30
    substeps; member m takes seed + m for its temperature noise.
    """
    u = uniform(seed, STREAM_MEMBERS, np.arange(5 * n, dtype=np.uint64)).reshape(n, 5)
    out = []
    for m in range(n):
        nx = 128 + 32 * int(u[m, 0] * 13)
        ny = 128 + 32 * int(u[m, 1] * 5)
        nz = 32 + 8 * int(u[m, 2] * 5)
        out.append(BETA_BASIN_64.replace(
            name=f"member{m:02d}_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, tau0=0.05 + 0.15 * float(u[m, 3]),
            strat_scale=500.0 + 1000.0 * float(u[m, 4]), seed=seed + m))
    return out


def layer_thickness(w: Workload) -> np.ndarray:
    """Uniform layers over the full depth, bottom to top."""
    return np.full(w.nz, w.depth / w.nz, dtype=np.float64)


def layer_centre_z(w: Workload) -> np.ndarray:
    """Height of every layer centre (m, negative below the surface), bottom to top."""
    dz = layer_thickness(w)
    top = np.cumsum(dz) - w.depth
    return top - 0.5 * dz


def _centres_deg(w: Workload):
    lon = w.x0 + (np.arange(w.nx) + 0.5) * w.dx
    lat = w.y0 + (np.arange(w.ny) + 0.5) * w.dy
    return lon, lat


def seafloor_depth(w: Workload) -> np.ndarray:
    """Sea-floor depth D(lon, lat) in metres, [ny, nx].

    D = depth - sum over 200 seamounts h exp(-r^2 / (2 sigma^2))
              - sum over two ridges depth exp(-dlon^2 / (2 * 2deg^2)) north of 50S,
    clipped to [0, depth]. Seamount heights U(1000, 5000) m, widths U(1, 4) deg,
    longitudes U(0, 360), latitudes U(-70, 70); r^2 = (dlon cos(lat_s))^2 + dlat^2
    in degrees with dlon wrapped to [-180, 180). Ridges sit at 0 and 90 deg E.
    """
    lon, lat = _centres_deg(w)
    d = np.full((w.ny, w.nx), w.depth, dtype=np.float64)
    if w.bathymetry == "flat":
        return d
    if w.coords != "latlon":
        raise ValueError("seamount bathymetry needs a lat-lon grid")
    n_mounts = 200
    u = uniform(w.seed, STREAM_BATHYMETRY, np.arange(4 * n_mounts, dtype=np.uint64)).reshape(n_mounts, 4)
    h = 1000.0 + 4000.0 * u[:, 0]
    sig = 1.0 + 3.0 * u[:, 1]
    lon_s = 360.0 * u[:, 2]
    lat_s = -70.0 + 140.0 * u[:, 3]
    north = (lat > -50.0).astype(np.float64)

    def rows(j0, j1):
        # every row block runs the same per-element arithmetic in the same order
        for s in range(n_mounts):
            dl = (lon - lon_s[s] + 180.0) % 360.0 - 180.0
            ex = np.exp(-((dl * math.cos(math.radians(lat_s[s]))) ** 2) / (2.0 * sig[s] ** 2))
            ey = np.exp(-((lat[j0:j1] - lat_s[s]) ** 2) / (2.0 * sig[s] ** 2))
            d[j0:j1] -= h[s] * np.outer(ey, ex)
        for lon_r in (0.0, 90.0):
            dl = (lon - lon_r + 180.0) % 360.0 - 180.0
            d[j0:j1] -= w.depth * np.outer(north[j0:j1], np.exp(-dl ** 2 / (2.0 * 2.0 ** 2)))

    _parallel_blocks(w.ny, rows)
    return np.clip(d, 0.0, w.depth)


def wet_layers(w: Workload) -> np.ndarray:
    """Number of wet layers per column counted from the surface, int32 [ny, nx].

    Full cells: K = floor(D / dz + 1/2); columns with fewer than two wet layers
    are land.
    """
    if w.bathymetry == "flat":
        return np.full((w.ny, w.nx), w.nz, dtype=np.int32)
    dz = w.depth / w.nz
    k = np.floor(seafloor_depth(w) / dz + 0.5).astype(np.int32)
    k = np.clip(k, 0, w.nz)
    k[k < 2] = 0
    return k


def initial_temperature(w: Workload, levels: Optional[range] = None) -> np.ndarray:
    """T = strat_t0 exp(z / strat_scale) + noise_std N(0, 1), [nz, ny, nx] (or the given levels).

    The noise of cell (i, j, k) is the normal deviate at counter i + nx (j + ny k)
    of the temperature stream.
    """
    zc = layer_centre_z(w)
    ks = list(range(w.nz) if levels is None else levels)
    out = np.empty((len(ks), w.ny, w.nx), dtype=np.float64)
    plane = np.arange(w.nx * w.ny, dtype=np.uint64)

    def level(q):
        k = ks[q]
        base = w.strat_t0 * math.exp(zc[k] / w.strat_scale)
        if w.noise_std != 0.0:
            n = normal(w.seed, STREAM_TEMPERATURE, plane + np.uint64(k * w.nx * w.ny))
            out[q] = base + w.noise_std * n.reshape(w.ny, w.nx)
        else:
            out[q] = base

    _parallel_blocks(len(ks), lambda a, b: [level(q) for q in range(a, b)], block=1)
    return out


def wind_stress(w: Workload):
    """Zonal stress at u-points and meridional stress at v-points, each [ny, nx] (N/m^2).

    Lat-lon: tau_x = tau0 cos(lat of the row). Beta-plane: tau_x = tau0 cos(pi (y - Ly/2) / Ly),
    the basin mapped onto latitudes -90..90. tau_y = 0.
    """
    if w.coords == "latlon":
        _, lat = _centres_deg(w)
        prof = w.tau0 * np.cos(np.radians(lat))
    else:
        ly = w.ny * w.dy
        y = (np.arange(w.ny) + 0.5) * w.dy
        prof = w.tau0 * np.cos(math.pi * (y - 0.5 * ly) / ly)
    taux = np.repeat(prof[:, None], w.nx, axis=1).astype(np.float64)
    return taux, np.zeros_like(taux)


def restoring_target(w: Workload) -> np.ndarray:
    """Surface restoring temperature T* = 20 cos(lat) degC, [ny, nx] (zero when restoring is off)."""
    if w.restore_days <= 0.0:
        return np.zeros((w.ny, w.nx), dtype=np.float64)
    if w.coords == "latlon":
        _, lat = _centres_deg(w)
        prof = 20.0 * np.cos(np.radians(lat))
    else:
        ly = w.ny * w.dy
        y = (np.arange(w.ny) + 0.5) * w.dy
        prof = 20.0 * np.cos(math.pi * (y - 0.5 * ly) / ly)
    return np.repeat(prof[:, None], w.nx, axis=1).astype(np.float64)


def initial_salinity(w: Workload) -> np.ndarray:
    """S = sal_s0 - sal_ds exp(z / strat_scale) + noise_std_s N(0, 1), [nz, ny, nx]:
    fresher water at the surface (stabilising, like the temperature profile).

    The noise of cell (i, j, k) is the normal deviate at counter i + nx (j + ny k)
    of the salinity stream.
    """
    zc = layer_centre_z(w)
    out = np.empty((w.nz, w.ny, w.nx), dtype=np.float64)
    plane = np.arange(w.nx * w.ny, dtype=np.uint64)
    for k in range(w.nz):
        base = w.sal_s0 - w.sal_ds * math.exp(zc[k] / w.strat_scale)
        n = normal(w.seed, STREAM_SALINITY, plane + np.uint64(k * w.nx * w.ny)) if w.noise_std_s else 0.0
        out[k] = base + w.noise_std_s * np.reshape(n, (w.ny, w.nx)) if w.noise_std_s else base
    return out


def salinity_target(w: Workload) -> np.ndarray:
    """Surface restoring salinity S* = 34 + 2 cos^2(lat) g/kg (sphere; the basin
    mapped onto latitudes -90..90 on the beta-plane), [ny, nx]."""
    if w.coords == "latlon":
        _, lat = _centres_deg(w)
        phi = np.radians(lat)
    else:
        ly = w.ny * w.dy
        phi = math.pi * ((np.arange(w.ny) + 0.5) * w.dy - 0.5 * ly) / ly
    prof = 34.0 + 2.0 * np.cos(phi) ** 2
    return np.repeat(prof[:, None], w.nx, axis=1).astype(np.float64)


def make_inputs(w: Workload) -> Dict[str, np.ndarray]:
    """All inputs of a workload: dz, kbottom, T0, taux, tauy, tstar (and S0,
    sstar with salinity)."""
    taux, tauy = wind_stress(w)
    out = {
        "dz": layer_thickness(w),
        "kbottom": wet_layers(w),
        "T0": initial_temperature(w),
        "taux": taux,
        "tauy": tauy,
        "tstar": restoring_target(w),
    }
    if w.salinity:
        out["S0"] = initial_salinity(w)
        out["sstar"] = salinity_target(w)
    return out
