"""GPU checks of the C-ABI contract that involve device work:

  - lbm_step(ctx, n, residual_out): the residual it reports equals
    lbm_diagnostics' and the oracle's; it stops with LBM_EUNSTABLE at the
    first diagnostic pass that sees a planted non-finite population;
  - lbm_last_error(ctx) keeps each context's own message;
  - lbm_create takes the initial velocity as one [2][ny][nx] array.

Bars: FP64 storage, residuals within 1e-10 relative of the oracle's (the
residual is a ratio of sums over the same fields); the initial populations
within 1e-15 of the oracle's equilibrium.
"""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1202_6130_amd import inputs as I
from paper_1202_6130_amd import lbm

pytestmark = pytest.mark.gpu


def drop(storage=lbm.STORE_F64, K=0):
    nx, ny = 64, 32
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage, wall_kind=lbm.WALL_FLAT_SLAB, G_R=0.5, G_A=0.3,
                               diag_interval=K)
    po = O.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=0.3, eps=1.0)
    w = O.Walls.flat_slab(nx, ny, 8, 2.0, 1.0, 3.0)
    return p, po, w, I.drop_field(nx, ny, 12.0)


def oracle_residual(po, w, rho0, t_prev, t):
    fa = O.run(po, w, O.init(po, rho0), t_prev)
    fb = O.run(po, w, fa, t - t_prev)
    _, ax, ay, _ = O.macros(po, w, fb)
    _, bx, by, _ = O.macros(po, w, fa)
    return O.residual(ax, ay, bx, by)


def test_step_residual_out_scheduled_passes():
    """diag_interval K = 50: every pass is checked, the last one reported."""
    p, po, w, rho0 = drop(K=50)
    L = lbm.Lattice(p, rho0)
    assert L.step(30, residual=True) == np.inf          # no pass yet
    r = L.step(70, residual=True)                         # passes at 50 and 100
    assert L.step_index == 100
    want = oracle_residual(po, w, rho0, 50, 100)
    assert abs(r - want) < 1e-10 * want, (r, want)
    d = L.diagnostics()
    assert d[0] == 100 and d[4] == r
    # a call that crosses no multiple of K reports the latest pass
    assert L.step(20, residual=True) == r
    L.close()


def test_step_residual_out_without_interval():
    """diag_interval 0: a pass runs after the last step of the call."""
    p, po, w, rho0 = drop(K=0)
    L = lbm.Lattice(p, rho0)
    assert L.step(40, residual=True) == np.inf          # the first pass has nothing to compare with
    r = L.step(60, residual=True)
    want = oracle_residual(po, w, rho0, 40, 100)
    assert abs(r - want) < 1e-10 * want, (r, want)
    L.close()


@pytest.mark.parametrize("storage", [lbm.STORE_F64, lbm.STORE_F32])
def test_step_unstable_on_planted_nan(storage):
    """A non-finite population planted at t = 100 is found by the first pass
    after it (t = 110): lbm_step returns LBM_EUNSTABLE there and takes no
    further step; the message stays with that context only."""
    p, po, w, rho0 = drop(storage, K=10)
    L = lbm.Lattice(p, rho0)
    other = lbm.Lattice(p, rho0)
    L.step(100)
    f = L.get_state()
    f[5, 12, 30] = np.nan
    L.set_state(f, 100)
    r = ctypes.c_double(-1.0)
    code = lbm.lib().lbm_step(L.ctx, 200, ctypes.byref(r))
    assert code == lbm.LBM_EUNSTABLE
    assert L.step_index == 110
    assert "non-finite" in lbm.lbm_last_error(L.ctx) and "110" in lbm.lbm_last_error(L.ctx)
    assert lbm.lbm_last_error(other.ctx) == ""
    # without residual_out the call only enqueues and does not stop
    code = lbm.lib().lbm_step(L.ctx, 20, None)
    assert code == lbm.LBM_OK and L.step_index == 130
    # the other context is unaffected
    assert np.isfinite(other.step(20, residual=True))
    L.close()
    other.close()


def test_last_error_is_per_context():
    p, po, w, rho0 = drop()
    a = lbm.Lattice(p, rho0)
    b = lbm.Lattice(p, rho0)
    with pytest.raises(lbm.LbmError):
        a.tile_shape = 99
    with pytest.raises(lbm.LbmError):
        b.two_step = 99
    assert "tile shape 99" in a.last_error and "variant 99" in b.last_error
    assert "variant 99" in lbm.lbm_last_error(None)   # the thread's last message
    a.close()
    b.close()


@pytest.mark.parametrize("storage", [lbm.STORE_F64, lbm.STORE_F32])
def test_create_takes_stacked_velocity(storage):
    """u0 is [2][ny][nx]: plane 0 is u_x, plane 1 u_y (random per node)."""
    nx, ny = 24, 16
    rho, ux, uy = I.random_state_field(nx, ny, 7)
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage)
    L = lbm.Lattice(p, rho, ux, uy)
    fg = L.get_state()
    L.close()
    po = O.make_params(nx, ny)
    fo = np.moveaxis(O.init(po, rho, ux, uy), -1, 0)
    tol = 1e-15 if storage == lbm.STORE_F64 else 6e-8
    assert np.abs(fg - fo).max() <= tol * np.abs(fo).max()


def test_f16dev_saturation_counts_as_unstable():
    """16-bit storage holds no non-finite values: a NaN and a population far
    outside the encodable range (|f/w - rho_ref| >= 8) are stored at the
    int16 bounds, read back as the bound's value, and the diagnostic pass
    counts both nodes, as it counts non-finite nodes of the floating-point
    storages (LBM_EUNSTABLE)."""
    p, po, w, rho0 = drop(lbm.STORE_F16DEV, K=0)
    p.rho_ref = 1.0
    L = lbm.Lattice(p, rho0)
    L.step(10)
    f = L.get_state()
    f[5, 12, 30] = np.nan
    f[2, 20, 7] = 1e3
    L.set_state(f, 10)
    g = L.get_state()
    w5, w2 = 1.0 / 36.0, 1.0 / 9.0
    bounds5 = {np.float32(w5) * np.float32(1.0 - 8.0), np.float32(w5) * np.float32(1.0 + 8.0 - 2.0 ** -12)}
    assert any(abs(g[5, 12, 30] - b) < 1e-6 for b in bounds5), g[5, 12, 30]
    assert abs(g[2, 20, 7] - w2 * (1.0 + 8.0 - 2.0 ** -12)) < 1e-6
    out = np.zeros(6)
    code = lbm.lib().lbm_diagnostics(L.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert code == lbm.LBM_EUNSTABLE and out[5] == 2, (code, out)
    # the rest of the lattice is untouched
    ok = np.ones(f.shape, bool)
    ok[5, 12, 30] = ok[2, 20, 7] = False
    assert np.abs(g[ok] - f[ok]).max() < 1e-12
    L.close()


@pytest.mark.parametrize("storage", [lbm.STORE_F32, lbm.STORE_F16DEV])
def test_zero_and_negative_step_counts(storage):
    """lbm_step with nsteps = 0 leaves the state and the step index as they
    were (with or without a residual request); a negative count is
    LBM_EINVAL and changes nothing.  The batch call likewise, and rejects an
    odd graph chunk."""
    p, _, _, rho0 = drop(storage, K=10)
    L = lbm.Lattice(p, rho0)
    L.step(7)
    f = L.get_state()
    L.step(0)
    assert L.step_index == 7 and np.array_equal(L.get_state(), f)
    r = ctypes.c_double(-1.0)
    assert lbm.lib().lbm_step(L.ctx, 0, ctypes.byref(r)) == lbm.LBM_OK
    assert L.step_index == 7 and np.array_equal(L.get_state(), f)
    assert lbm.lib().lbm_step(L.ctx, -1, None) == lbm.LBM_EINVAL
    assert "nsteps" in lbm.lib().lbm_last_error(L.ctx).decode()
    assert L.step_index == 7 and np.array_equal(L.get_state(), f)
    L.close()
    if storage != lbm.STORE_F32:
        return
    ps = [lbm.lbm_params_default(nx=64, ny=32, wall_kind=lbm.WALL_FLAT_SLAB, G_R=0.5, G_A=0.3),
          lbm.lbm_params_default(nx=96, ny=64, wall_kind=lbm.WALL_FLAT_SLAB, G_R=0.2, G_A=0.1)]
    rhos = [I.drop_field(64, 32, 12.0), I.drop_field(96, 64, 18.0)]
    B = lbm.Batch(ps, rhos)
    B.step(4)
    before = [B.lattice(k).get_state() for k in range(2)]
    B.step(0)
    for bad in ((-2, 0), (4, 3)):
        with pytest.raises(lbm.LbmError) as e:
            B.step(*bad)
        assert e.value.code == lbm.LBM_EINVAL
    for k in range(2):
        assert np.array_equal(B.lattice(k).get_state(), before[k])
    B.close()
