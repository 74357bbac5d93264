"""Shared test helpers: small workloads and oracle construction."""
import numpy as np

import oracle
from paper_2309_06662_amd import inputs


def small_latlon(nx=36, ny=20, nz=6, **kw):
    """A coarse near-global lat-lon basin with seamounts and ridges (periodic in x)."""
    base = dict(name=f"latlon_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, coords="latlon", periodic_x=True,
                x0=0.0, y0=-70.0, dx=360.0 / nx, dy=140.0 / ny, depth=5500.0, bathymetry="seamounts",
                dt=1800.0, n_substeps=60, restore_days=30.0)
    base.update(kw)
    return inputs.Workload(**base)


def make_oracle(w, **overrides):
    inp = inputs.make_inputs(w)
    inp.update(overrides)
    return oracle.OracleModel.from_inputs(w, inp), inp


def rel_l2(a, b, mask=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if mask is not None:
        a, b = a[mask], b[mask]
    nb = np.linalg.norm(b.ravel())
    if nb < 1e-300:
        return np.linalg.norm((a - b).ravel())
    return np.linalg.norm((a - b).ravel()) / nb


def masks(w, kb):
    """Wet masks (c, u, v) built from the wet-layer counts in plain numpy."""
    nz = w.nz
    k = np.arange(nz)[:, None, None]
    wet = (k >= nz - kb[None, :, :])
    west = np.roll(wet, 1, axis=2)
    south = np.roll(wet, 1, axis=1)
    if not w.periodic_x:
        west[:, :, 0] = False
    if not w.periodic_y:
        south[:, 0, :] = False
    return wet, wet & west, wet & south


def metrics(w):
    """Row metrics (dxc, dxv at south faces 0..ny, dy, area) in plain numpy."""
    j = np.arange(w.ny + 1)
    if w.coords == "latlon":
        lat_c = np.radians(w.y0 + (j[:-1] + 0.5) * w.dy)
        lat_s = np.radians(w.y0 + j * w.dy)
        dl = np.radians(w.dx)
        dxc = w.radius * np.cos(lat_c) * dl
        dxv = w.radius * np.cos(lat_s) * dl
        dy = w.radius * np.radians(w.dy)
    else:
        dxc = np.full(w.ny, w.dx)
        dxv = np.full(w.ny + 1, w.dx)
        dy = w.dy
    return dxc, dxv, dy, dxc * dy
