"""Host-side pieces of the closure's training data: coarse-graining, the eddy
heat flux, the diffusivity target and the mixed-layer depth, on arrays with
closed-form answers."""
import math

import numpy as np

from paper_2309_06662_amd import closure_train as ct
from paper_2309_06662_amd import inputs


def _pair(factor=2):
    coarse, fine = ct.regional_pair(factor=factor, nx=4, ny=3, nz=5, lon0=10.0, lat0=-10.0, res=1.0,
                                    depth=1000.0)
    coarse = coarse.replace(bathymetry="flat")
    fine = fine.replace(bathymetry="flat")
    kb_c = np.full((coarse.ny, coarse.nx), coarse.nz, np.int32)
    kb_f = np.full((fine.ny, fine.nx), fine.nz, np.int32)
    return coarse, fine, ct.CoarseGrainer(coarse, fine, kb_f, kb_c, factor)


def test_pair_shares_the_box():
    c, f = ct.regional_pair(factor=4)
    assert f.nx == 4 * c.nx and f.ny == 4 * c.ny and f.nz == c.nz
    assert math.isclose(f.dx * f.nx, c.dx * c.nx) and f.x0 == c.x0 and f.y0 == c.y0
    assert math.isclose(f.dt * 4, c.dt)


def test_block_means_are_area_weighted():
    coarse, fine, cg = _pair()
    a = np.ones((fine.nz, fine.ny, fine.nx)) * 3.0
    assert np.allclose(cg.cells(a), 3.0)
    lat = fine.y0 + (np.arange(fine.ny) + 0.5) * fine.dy
    b = np.broadcast_to(lat[None, :, None], a.shape)
    w = np.cos(np.radians(lat))
    exp = np.array([(lat[2 * j:2 * j + 2] * w[2 * j:2 * j + 2]).sum() / w[2 * j:2 * j + 2].sum()
                    for j in range(coarse.ny)])
    assert np.allclose(cg.cells(b)[0, :, 0], exp, rtol=1e-14)


def test_faces_take_the_fine_faces_on_the_coarse_face_line():
    coarse, fine, cg = _pair()
    u = np.random.default_rng(0).normal(size=(fine.nz, fine.ny, fine.nx))
    uc = cg.u_faces(u)
    assert uc.shape == (coarse.nz, coarse.ny, coarse.nx)
    assert np.allclose(uc[:, 1, 2], 0.5 * (u[:, 2, 4] + u[:, 3, 4]))
    vc = cg.v_faces(u)
    assert np.allclose(vc[:, 2, 1], 0.5 * (u[:, 4, 2] + u[:, 4, 3]))


def test_eddy_flux_of_correlated_and_uncorrelated_fields():
    coarse, fine, cg = _pair()
    nz = fine.nz
    T = np.broadcast_to(np.arange(nz, dtype=float)[:, None, None], (nz, fine.ny, fine.nx)).copy()
    W = np.zeros((nz + 1, fine.ny, fine.nx))
    W[:nz] = 0.3                                  # uniform w: no eddy flux
    assert np.allclose(ct.eddy_flux(cg, T, W)[1:], 0.0, atol=1e-14)
    # w and T both carry the same zero-mean checkerboard x' inside each block
    x = np.where((np.arange(fine.nx)[None, :] + np.arange(fine.ny)[:, None]) % 2 == 0, 1.0, -1.0)
    T2 = T + 0.5 * x[None]
    W2 = np.zeros_like(W)
    W2[:nz] = 2.0 * x[None]
    fl = ct.eddy_flux(cg, T2, W2)
    assert np.allclose(fl[1:], 2.0 * 0.5, rtol=1e-12)   # <w'T'> = a b <x'^2> with T at faces = mean of two layers


def test_kappa_target():
    nz = 4
    dz = np.full(nz, 10.0)
    Tc = np.broadcast_to((0.1 * np.arange(nz))[:, None, None], (nz, 1, 1)).copy()   # dT/dz = 0.01 K/m
    flux = np.zeros((nz, 1, 1))
    y = ct.kappa_target(flux, Tc, dz, 1e-5)
    assert np.allclose(y, math.log10(1e-5))           # no flux: the background on every face
    flux[1:] = -2e-5                              # down-gradient flux: kappa0 + 2e-5 / 0.01
    y = ct.kappa_target(flux, Tc, dz, 1e-5)
    assert np.allclose(10 ** y[1:], 1e-5 + 2e-3, rtol=1e-12) and np.allclose(10 ** y[0], 1e-5)
    flux[1:] = -100.0                             # clipped above (slot 0, the bottom face, stays background)
    assert np.allclose(10 ** ct.kappa_target(flux, Tc, dz, 1e-5)[1:], 1.0)


def test_mixed_layer_depth():
    dz = np.full(6, 10.0)                         # centres at 5, 15, ..., 55 m below the top
    T = np.array([1.0, 2.0, 3.0, 9.95, 9.9, 10.0])[:, None, None]   # bottom first
    assert ct.mixed_layer_depth(T, dz)[0, 0] == 35.0    # layer index 2 (T = 3) is the first 0.2 K colder
    T2 = np.full((6, 1, 1), 5.0)
    assert ct.mixed_layer_depth(T2, dz)[0, 0] == 55.0   # no such layer: the deepest centre
    assert np.isclose(ct.heat_content(T2, dz)[0, 0], 300.0)


def test_subgrid_flux_includes_mixing_beyond_the_background():
    coarse, fine, cg = _pair()
    nz = fine.nz
    dz = np.full(nz, 10.0)
    T = np.broadcast_to((0.02 * np.arange(nz))[:, None, None], (nz, fine.ny, fine.nx)).copy()  # dT/dz = 0.002
    W = np.zeros((nz + 1, fine.ny, fine.nx))
    kap = np.full((nz, fine.ny, fine.nx), 1e-5)
    kap[3] = 0.5                                  # one mixed face
    fl = ct.eddy_flux(cg, T, W, kap, 1e-5, dz)
    assert np.allclose(fl[3], -(0.5 - 1e-5) * 0.002, rtol=1e-12)
    assert np.allclose(np.delete(fl, 3, axis=0), 0.0, atol=1e-18)


def test_kappa_target_counts_unstable_down_gradient_flux():
    """Cold over warm (dT/dz < 0) with an upward heat flux is down-gradient:
    the target diffusivity is positive, not the background."""
    nz = 3
    dz = np.full(nz, 10.0)
    Tc = np.array([5.0, 4.9, 4.8])[:, None, None]       # dT/dz = -0.01 K/m
    flux = np.zeros((nz, 1, 1))
    flux[1:] = 2e-4                                    # upward
    k = 10 ** ct.kappa_target(flux, Tc, dz, 1e-5)
    assert np.allclose(k[1:], 1e-5 + 2e-4 / 0.01, rtol=1e-12)
    flux[1:] = -2e-4                                   # counter-gradient: background only
    assert np.allclose(10 ** ct.kappa_target(flux, Tc, dz, 1e-5), 1e-5)
