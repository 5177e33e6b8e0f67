"""GPU runs at the largest lattices the C ABI accepts (tests/max_lattices.py:
each population buffer just below 4 GiB, so the last planes' offsets reach
just below 2^32 bytes).  After 10 steps from a smooth two-phase field on a
lattice with a flat solid band, one more GPU step is checked at sampled
nodes, including the first and last rows and columns, against the oracle's
one-step update of a patch of the same GPU state (the update of a node
depends on its radius-2 neighbourhood for D2Q9, radius 6 for D2Q21).  For
binary32 D2Q21 the step is taken by the marching and by the one-row tile
variants from the same state, which must agree bit for bit; for binary32
D2Q9 two further steps are taken one per launch and, from the same state,
in one two-step launch, which must also agree bit for bit.

Bars: FP64 storage 1e-12; binary32 2e-6 (one step of binary32 arithmetic);
FP16 deviations: half of one binary16 unit of the stored deviation
h = f / w - rho_ref, times w, plus the binary32 bar.
"""
import numpy as np
import pytest

import oracle as O
from max_lattices import MAX_LATTICES
from paper_1202_6130_amd import lbm

pytestmark = pytest.mark.gpu

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
SLAB = 8
G_R, G_A = 0.5, 0.3


def smooth_two_phase(nx, ny, lo, hi):
    """rho between lo and hi: tanh of a product of sines (interfaces a few
    nodes wide, periods 197 and 173 nodes)."""
    sx = np.sin(2 * np.pi * np.arange(nx) / 197.0)
    sy = np.sin(2 * np.pi * np.arange(ny) / 173.0)
    f = np.multiply.outer(sy, sx)
    f *= 2.0
    np.tanh(f, out=f)
    f *= 0.5 * (hi - lo)
    f += 0.5 * (hi + lo)
    return f


def oracle_node(q, po_kw, walls_col, f0, y, x, r):
    """Oracle one-step result at (y, x) from the (2r+1)^2 patch of f0
    ([Q, ny, nx]); walls_col holds the flat-slab wall functions per row."""
    _, ny, nx = f0.shape
    ys = np.arange(y - r, y + r + 1) % ny
    xs = np.arange(x - r, x + r + 1) % nx
    n = 2 * r + 1
    patch = np.ascontiguousarray(np.moveaxis(f0[:, ys][:, :, xs], 0, -1))
    w = O.Walls(*(np.ascontiguousarray(np.repeat(a[ys, :1], n, axis=1)) for a in walls_col))
    po = O.make_params(n, n, **po_kw)
    return O.step(po, w, patch)[r, r]


@pytest.mark.parametrize("case", sorted(MAX_LATTICES))
def test_max_lattice_sampled_one_step(case):
    q, st, nx, ny = MAX_LATTICES[case]
    storage = {"f32": lbm.STORE_F32, "f16dev": lbm.STORE_F16DEV, "f64": lbm.STORE_F64}[st]
    if q == 21:
        fluid = dict(lattice=lbm.D2Q21, psi_kind=lbm.PSI_EOS, G=-1.0)
        po_kw = dict(tau=1.0, G=-1.0, G_R=G_R, G_A=G_A, eps=1.0, lattice=21, psi_kind=1)
        rho0 = smooth_two_phase(nx, ny, 0.1, 1.0)
        r = 7
    else:
        fluid = dict(G=-5.0)
        po_kw = dict(tau=1.0, G=-5.0, G_R=G_R, G_A=G_A, eps=1.0)
        rho0 = smooth_two_phase(nx, ny, 0.15, 1.93)
        r = 4
    rho_ref = float(rho0.mean())
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage, wall_kind=lbm.WALL_FLAT_SLAB, slab_rows=SLAB,
                               G_R=G_R, G_A=G_A, rho_ref=rho_ref, **fluid)
    print(f"{case}: {nx}x{ny} D2Q{q} {st}, creating", flush=True)
    L = lbm.Lattice(p, rho0)
    del rho0
    print(f"{case}: variant/shape {L.tile_shape}, 10 steps", flush=True)
    L.step(10)
    f0 = L.get_state()
    L.step(1)
    f1 = L.get_state()
    if q == 21 and st == "f32":
        # the same step by the one-row tiles from the same state
        shape = L.tile_shape
        L.set_state(f0, 10)
        L.tile_shape = 2
        print(f"{case}: one step by variant 2 (default {shape})", flush=True)
        L.step(1)
        assert np.array_equal(L.get_state(), f1)
    if q == 9 and st == "f32":
        # steps 12 and 13 one at a time, then again as one two-step launch
        # (64 x 24 blocks) from the same state: bitwise the same
        L.step(2)
        f3 = L.get_state()
        L.set_state(f1, 11)
        L.two_step = 8
        print(f"{case}: two steps in one launch (variant 8)", flush=True)
        L.step(2)
        assert np.array_equal(L.get_state(), f3)
        del f3
    L.close()
    rng = np.random.Generator(np.random.PCG64(nx + ny))
    ys = np.concatenate([rng.integers(0, ny, 24), [0, 1, ny - 1, ny - SLAB, ny - SLAB - 1, 0, ny - 1]])
    xs = np.concatenate([rng.integers(0, nx, 24), [0, nx - 1, 63, 64, nx - 1, nx - 1, 0]])
    walls_col = O.Walls.flat_slab(1, ny, SLAB, 2.0, 1.0, 3.0)
    walls_col = (walls_col.phi, walls_col.psiR, walls_col.psiA)
    worst = 0.0
    for y, x in zip(ys, xs):
        want = oracle_node(q, po_kw, walls_col, f0, int(y), int(x), r)
        got = f1[:, int(y), int(x)]
        err = np.abs(got - want)
        if st == "f64":
            bar = np.full(q, 1e-12)
        elif st == "f32":
            bar = np.full(q, 2e-6)
        else:                                     # 16-bit deviations (units of 2^-12): D2Q9 only
            bar = W9 * 2.0 ** -13 * (1 + 1e-6) + 2e-6
        worst = max(worst, float((err / bar).max()))
        assert np.all(err <= bar), (case, int(y), int(x), err.max())
    print(f"{case}: worst error / bar over {len(ys)} nodes = {worst:.3f}", flush=True)
