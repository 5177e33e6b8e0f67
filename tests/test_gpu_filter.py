"""GPU parity of the mask walls: wall functions of arbitrary geometry by the
recursive filter of Appendix A (eq. iteration) computed on the device at
creation, then the update on them, against the FP64 oracle (its own filter,
orc_filter_walls, and its own step).

Bars: FP64 storage within 1e-13 after one step and 1e-10 after hundreds
(the two filters differ only in rounding order); binary32 within 1e-5.
"""
import numpy as np
import pytest

import oracle as O
from paper_1202_6130_amd import inputs as I
from paper_1202_6130_amd import lbm

pytestmark = pytest.mark.gpu


def to_orc(fg):
    return np.ascontiguousarray(np.moveaxis(fg, 0, -1))


def from_orc(fo):
    return np.ascontiguousarray(np.moveaxis(fo, -1, 0))


def geometry(nx, ny, seed):
    """A bottom solid band with a bump and a free-floating solid disc; the
    band's lowest row is the held outer boundary."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y, x = np.mgrid[0:ny, 0:nx]
    H = np.zeros((ny, nx))
    H[:3, :] = 1.0
    H[((x - nx * 0.3) ** 2 + (y - 2) ** 2) < (0.15 * min(nx, ny) + 1) ** 2] = 1.0
    cx, cy = rng.uniform(0.5, 0.8) * nx, rng.uniform(0.5, 0.8) * ny
    H[((x - cx) ** 2 + (y - cy) ** 2) < (0.1 * min(nx, ny) + 1) ** 2] = 1.0
    B = np.zeros_like(H)
    B[0, :] = 1.0
    return H, B


def fluid(lat):
    return (dict(lattice=21, psi_kind=1, G=-1.0), 0.08, 1.1) if lat == 21 else (dict(lattice=9, psi_kind=0, G=-5.0),
                                                                                0.2, 1.8)


@pytest.mark.parametrize("lat", [9, 21])
@pytest.mark.parametrize("nx,ny", [(7, 9), (40, 30), (131, 70)])
def test_mask_walls_one_step_f64(lat, nx, ny):
    fl, lo, hi = fluid(lat)
    kw = dict(tau=0.9, G_R=0.6, G_A=0.3, eps=1.3, F_ext=(1e-4, 0.0), **fl)
    H, B = geometry(nx, ny, nx + ny)
    walls = O.Walls.filtered(H, B, lat, 5, 22)
    po = O.make_params(nx, ny, **kw)
    rho, ux, uy = I.random_state_field(nx, ny, 5 + nx, lo=lo, hi=hi)
    rng = np.random.Generator(np.random.PCG64(ny))
    f = O.init(po, rho, ux, uy) * (1 + 0.05 * rng.uniform(-1, 1, (ny, nx, O.nq(po))))
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=lbm.STORE_F64, wall_kind=lbm.WALL_MASK, **kw)
    L = lbm.Lattice(p, np.ones((ny, nx)), wall_fields=np.stack([H, B]))
    L.set_state(from_orc(f), 0)
    L.step(1)
    assert np.abs(to_orc(L.get_state()) - O.step(po, walls, f)).max() < 1e-13
    L.close()


@pytest.mark.parametrize("lat", [9, 21])
def test_mask_walls_drop_multi_step(lat):
    """A drop resting on the bump of the geometry, 400 steps, FP64 and binary32."""
    fl, _, _ = fluid(lat)
    nx, ny = 96, 64
    rl, rg = (1.0, 0.1) if lat == 21 else (1.93, 0.156)
    kw = dict(tau=1.0, G_R=0.5, G_A=0.3, eps=1.0, **fl)
    H, B = geometry(nx, ny, 3)
    walls = O.Walls.filtered(H, B, lat)
    y, x = np.mgrid[0:ny, 0:nx]
    r = np.hypot(x - 0.6 * nx, y - 12.0)
    rho0 = rg + (rl - rg) * 0.5 * (1 - np.tanh((r - 10.0) / 2.0))
    po = O.make_params(nx, ny, **kw)
    fo = O.run(po, walls, O.init(po, rho0), 400)
    r_o, ux_o, uy_o, tot_o = O.macros(po, walls, fo)
    for storage in (lbm.STORE_F64, lbm.STORE_F32):
        p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage, wall_kind=lbm.WALL_MASK, **kw)
        L = lbm.Lattice(p, rho0, wall_fields=np.stack([H, B]))
        L.step(400)
        rho, ux, uy, tot = L.moments()
        if storage == lbm.STORE_F64:
            assert np.abs(to_orc(L.get_state()) - fo).max() < 1e-10
        else:
            cs = np.sqrt(2.0 / 3.0) if lat == 21 else 1.0 / np.sqrt(3.0)
            r_err = np.abs(rho - r_o).max() / np.abs(r_o).max()
            u_err = np.hypot(ux - ux_o, uy - uy_o).max() / cs
            print(f"mask walls D2Q{lat} drop t=400 FP32: rho {r_err:.2e}, u/c_s {u_err:.2e}")
            assert r_err < 1e-5 and u_err < 1e-5
        L.close()


def test_mask_walls_reject_bad_input():
    p = lbm.lbm_params_default(nx=8, ny=8, wall_kind=lbm.WALL_MASK)
    H = np.zeros((8, 8))
    with pytest.raises(lbm.LbmError):
        lbm.Lattice(p, np.ones((8, 8)), wall_fields=np.stack([H + 0.5, H]))
    with pytest.raises(lbm.LbmError):
        lbm.Lattice(p, np.ones((8, 8)))
