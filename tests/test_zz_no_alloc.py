"""lbm_diagnostics_noalloc against lbm_diagnostics through the C ABI.

Two contexts are created from the same inputs and stepped alike; one is
queried with lbm_diagnostics (partial sums in its workspace), the other with
lbm_diagnostics_noalloc (partial sums in the library's static device array).
The passes run the same kernels over the same state, so every result must
agree bit for bit.  Two calls in a row, the second on a smaller lattice (and
a third on the first size again, after the array held the smaller one's
partials), plus the size limit and the non-finite report.
"""
import numpy as np
import pytest

from paper_1202_6130_amd import inputs as I
from paper_1202_6130_amd import lbm

pytestmark = pytest.mark.gpu


def pair(nx, ny, storage, K=0, lattice=lbm.D2Q9, psi=lbm.PSI_EXP, seed=3):
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage, wall_kind=lbm.WALL_FLAT_SLAB, G_R=0.4, G_A=0.2,
                               diag_interval=K, lattice=lattice, psi_kind=psi,
                               G=-1.0 if psi == lbm.PSI_EOS else -5.0)
    rho, ux, uy = I.random_state_field(nx, ny, seed)
    if psi == lbm.PSI_EOS:
        rho = 0.1 + 0.45 * rho
    return lbm.Lattice(p, rho, ux, uy), lbm.Lattice(p, rho, ux, uy)


def same(a, b):
    return np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("storage", [lbm.STORE_F32, lbm.STORE_F64])
def test_noalloc_matches_diagnostics_two_calls(storage):
    sizes = [(300, 200), (70, 45), (300, 200)]     # second call smaller, third back to the first size
    for nx, ny in sizes:
        A, B = pair(nx, ny, storage)
        for steps in (0, 37, 100):
            A.step(steps)
            B.step(steps)
            da, ca = lbm.lbm_diagnostics(A.ctx, check=False)
            db, cb = lbm.lbm_diagnostics_noalloc(B.ctx, check=False)
            assert ca == cb == lbm.LBM_OK
            assert same(da, db), (nx, ny, steps, da, db)
            # a repeated query at the same step reports the same pass
            assert same(lbm.lbm_diagnostics_noalloc(B.ctx)[0], db)
        A.close()
        B.close()


def check_pair(A, B):
    da, ca = lbm.lbm_diagnostics(A.ctx, check=False)
    db, cb = lbm.lbm_diagnostics_noalloc(B.ctx, check=False)
    assert ca == cb and same(da, db), (ca, cb, da, db)


def test_noalloc_with_scheduled_passes_and_d2q21():
    A, B = pair(128, 96, lbm.STORE_F32, K=25)
    for steps in (50, 30):
        A.step(steps)
        B.step(steps)
        check_pair(A, B)
    A.close()
    B.close()
    A, B = pair(96, 64, lbm.STORE_F32, lattice=lbm.D2Q21, psi=lbm.PSI_EOS)
    A.step(20)
    B.step(20)
    check_pair(A, B)
    A.close()
    B.close()


def test_noalloc_reports_non_finite():
    A, B = pair(64, 32, lbm.STORE_F32)
    f = B.get_state()
    f[2, 5, 7] = np.nan
    A.set_state(f, 0)
    B.set_state(f, 0)
    da, ca = lbm.lbm_diagnostics(A.ctx, check=False)
    db, cb = lbm.lbm_diagnostics_noalloc(B.ctx, check=False)
    assert ca == cb == lbm.LBM_EUNSTABLE and db[5] >= 1 and same(da, db)
    A.close()
    B.close()


def test_noalloc_rejects_lattices_beyond_the_array():
    # 1 x 270000 nodes: one strip, segments of 8 rows -> 33750 partial rows > 32768
    p = lbm.lbm_params_default(nx=1, ny=270000, seg_rows=8)
    L = lbm.Lattice(p, np.ones((270000, 1)))
    out, code = lbm.lbm_diagnostics_noalloc(L.ctx, check=False)
    assert code == lbm.LBM_EINVAL and "32768" in L.last_error
    # the workspace path still serves it (binary32 populations of a uniform
    # fluid at rho = 1 sum to 1 within the rounding of the weights)
    assert lbm.lbm_diagnostics(L.ctx)[0][1] == pytest.approx(270000.0, rel=1e-7)
    L.close()
