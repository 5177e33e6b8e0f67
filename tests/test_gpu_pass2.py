"""GPU tests of two time steps per pass (temporal blocking): every variant
gives bitwise the fields of single steps, for both storages it supports, both
wall kinds, both collisions and tau = 1, on ragged, tiny and one-row lattices;
diagnostics keep their schedule; the variants agree with the FP64 oracle on
the small drop to the single step's tolerance."""
import numpy as np
import pytest

from paper_1202_6130_amd import inputs as I
from paper_1202_6130_amd import lbm

pytestmark = pytest.mark.gpu
VARIANTS = [(1, 8, 4), (1, 8, 8), (2, 8, 8), (1, 12, 6), (1, 12, 12), (1, 16, 8), (1, 16, 16), (1, 24, 8),
            (1, 24, 12)]


def _fields(nx, ny, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 0.5, (ny, nx))])


def _run(nx, ny, storage, wall, variant, steps, rho0, fields=None, tau=0.9, collision=lbm.COLL_BGK,
         diag_interval=0):
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage, wall_kind=wall, G_R=0.5, G_A=0.3, eps=1.3,
                               tau=tau, collision=collision, F_ext=(1e-5, 0.0), rho_ref=float(rho0.mean()),
                               diag_interval=diag_interval)
    L = lbm.Lattice(p, rho0, wall_fields=fields)
    L.two_step = variant
    assert L.two_step == variant
    L.step(steps)
    assert L.step_index == steps
    s = L.get_state()
    d = L.diagnostics()
    L.close()
    return s, d


def test_variant_table():
    assert lbm.lbm_two_step_variants() == VARIANTS


@pytest.mark.parametrize("storage", [lbm.STORE_F32, lbm.STORE_F16DEV, lbm.STORE_F64])
@pytest.mark.parametrize("nx,ny", [(200, 96), (130, 71), (64, 15), (5, 6), (70, 1), (1, 40)])
def test_every_variant_same_update(storage, nx, ny):
    wall = lbm.WALL_FLAT_SLAB if ny > 9 else lbm.WALL_NONE
    rho0 = I.drop_field(nx, ny, 0.3 * min(nx, ny) + 1) if ny > 9 and nx > 9 else I.random_state_field(nx, ny, 3)[0]
    ref, _ = _run(nx, ny, storage, wall, -1, 25, rho0)
    for v in range(len(VARIANTS)):
        print(f"two-step variant {v} storage {storage} lattice {nx}x{ny}", flush=True)
        got, _ = _run(nx, ny, storage, wall, v, 25, rho0)
        assert np.array_equal(got, ref), (storage, nx, ny, v)


@pytest.mark.parametrize("storage", [lbm.STORE_F32, lbm.STORE_F64])
@pytest.mark.parametrize("tau,collision", [(1.0, lbm.COLL_BGK), (0.7, lbm.COLL_PROJECTED), (0.9, lbm.COLL_BGK)])
def test_every_variant_node_fields(storage, tau, collision):
    nx, ny = 150, 77
    rho0 = I.random_state_field(nx, ny, 4)[0]
    fields = _fields(nx, ny, 5)
    ref, _ = _run(nx, ny, storage, lbm.WALL_FIELDS, -1, 20, rho0, fields, tau=tau, collision=collision)
    for v in range(len(VARIANTS)):
        print(f"two-step variant {v} node fields storage {storage} tau {tau}", flush=True)
        got, _ = _run(nx, ny, storage, lbm.WALL_FIELDS, v, 20, rho0, fields, tau=tau, collision=collision)
        assert np.array_equal(got, ref), v


def test_diagnostic_schedule_kept():
    # diag_interval 7 is odd: pairs never straddle a diagnostic step, odd
    # remainders take single steps; residual bookkeeping equals single steps
    nx, ny = 256, 96
    rho0 = I.drop_field(nx, ny, 30.0)
    ref_s, ref_d = _run(nx, ny, lbm.STORE_F32, lbm.WALL_FLAT_SLAB, -1, 71, rho0, diag_interval=7)
    for v in (1, 7):
        s, d = _run(nx, ny, lbm.STORE_F32, lbm.WALL_FLAT_SLAB, v, 71, rho0, diag_interval=7)
        assert np.array_equal(s, ref_s)
        assert np.array_equal(d, ref_d)


def test_refused_where_not_built():
    nx, ny = 64, 32
    rho0 = I.drop_field(nx, ny, 12.0)
    for storage in (lbm.STORE_F32X,):
        L = lbm.Lattice(lbm.lbm_params_default(nx=nx, ny=ny, storage=storage), rho0)
        with pytest.raises(lbm.LbmError):
            L.two_step = 0
        assert L.two_step == -1
        L.close()
    L = lbm.Lattice(lbm.lbm_params_default(nx=nx, ny=ny), rho0)
    with pytest.raises(lbm.LbmError):
        L.two_step = len(VARIANTS)
    L.close()


def test_tune_two_step_is_plain_stepping():
    nx, ny = 384, 160
    rho0 = I.drop_field(nx, ny, 48.0)
    p = lbm.lbm_params_default(nx=nx, ny=ny, wall_kind=lbm.WALL_FLAT_SLAB, G_R=0.4, G_A=0.2, diag_interval=10)
    L = lbm.Lattice(p, rho0)
    v, ms = L.tune_two_step(3)
    assert -1 <= v < len(VARIANTS) and L.two_step == v
    assert ms.shape == (len(VARIANTS) + 1,) and np.all(np.isfinite(ms)) and np.all(ms > 0)
    assert ms[v] == ms.min()
    n = L.step_index
    assert n == (6 * 3 + 2) * (len(VARIANTS) + 1)
    ref = lbm.Lattice(p, rho0)
    ref.step(n)
    assert np.array_equal(L.get_state(), ref.get_state())
    L.step(13)
    ref.step(13)
    assert np.array_equal(L.get_state(), ref.get_state())
    assert np.array_equal(L.diagnostics(), ref.diagnostics())
    L.close()
    ref.close()


def test_tune_two_step_single_only_where_not_built():
    nx, ny = 96, 48
    rho0 = I.drop_field(nx, ny, 14.0)
    L = lbm.Lattice(lbm.lbm_params_default(nx=nx, ny=ny, storage=lbm.STORE_F32X), rho0)
    v, ms = L.tune_two_step(2)
    assert v == -1 and L.two_step == -1
    assert np.all(np.isinf(ms[:-1])) and np.isfinite(ms[-1])
    assert L.step_index == 6 * 2 + 2
    L.close()


def test_oracle_parity_small_drop_two_step():
    """The 64x32 drop of the small configuration, 2000 steps, binary32 storage
    with two steps per pass (every variant), against the FP64 oracle at the
    single step's bar: max|rho - rho_o| / max|rho_o| <= 1e-5 and
    max|u - u_o| / c_s <= 1e-5."""
    import oracle as O
    nx, ny = 64, 32
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=lbm.STORE_F32, wall_kind=lbm.WALL_FLAT_SLAB, G_R=0.5, G_A=0.3)
    po = O.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=0.3, eps=1.0)
    w = O.Walls.flat_slab(nx, ny, 8, 2.0, 1.0, 3.0)
    rho0 = I.drop_field(nx, ny, 12.0)
    fo = O.run(po, w, O.init(po, rho0), 2000)
    r_o, ux_o, uy_o, _ = O.macros(po, w, fo)
    cs = 1.0 / np.sqrt(3.0)
    for v in range(len(VARIANTS)):
        L = lbm.Lattice(p, rho0)
        L.two_step = v
        L.step(2000)
        rho, ux, uy, _ = L.moments()
        L.close()
        e_rho = np.abs(rho - r_o).max() / np.abs(r_o).max()
        e_u = max(np.abs(ux - ux_o).max(), np.abs(uy - uy_o).max()) / cs
        print(f"two-step variant {v}, FP32 drop 64x32 t=2000: rho {e_rho:.3e}, u/c_s {e_u:.3e}", flush=True)
        assert e_rho <= 1e-5 and e_u <= 1e-5


def _ensemble(seed, count):
    cases = I.ensemble_cases(seed=seed, count=count)
    ps = [lbm.lbm_params_default(nx=c.nx, ny=c.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=c.G, G_R=c.G_R, G_A=c.G_A)
          for c in cases]
    return ps, [I.drop_field(c.nx, c.ny, c.radius) for c in cases]


def _alone(p, rho, steps):
    L = lbm.Lattice(lbm.lbm_params_default(nx=p.nx, ny=p.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=p.G, G_R=p.G_R,
                                           G_A=p.G_A), rho)
    L.step(steps)
    s = L.get_state()
    L.close()
    return s


@pytest.mark.parametrize("variant", [0, 3, 7])
def test_batch_two_step_bitwise(variant):
    # graph chunks of 6 steps (3 passes: the buffer parity flips per replay)
    # and of 4 (2 passes), odd remainders as single steps, plain launches
    ps, rhos = _ensemble(31, 5)
    B = lbm.Batch(ps, rhos)
    B.two_step = variant
    assert B.two_step == variant
    B.step(12, chunk=6)
    B.step(7, chunk=4)
    B.step(5)
    for k, (p, r) in enumerate(zip(ps, rhos)):
        print(f"batch two-step variant {variant}, lattice {k} {p.nx}x{p.ny}", flush=True)
        assert np.array_equal(B.lattice(k).get_state(), _alone(p, r, 24)), k
    B.two_step = -1
    B.step(6, chunk=6)
    for k, (p, r) in enumerate(zip(ps, rhos)):
        assert np.array_equal(B.lattice(k).get_state(), _alone(p, r, 30)), k
    B.close()


def test_batch_tune_two_step_is_plain_stepping():
    ps, rhos = _ensemble(32, 4)
    B = lbm.Batch(ps, rhos)
    v, ms = B.tune_two_step(2)
    assert -1 <= v < len(VARIANTS) and B.two_step == v
    assert ms.shape == (len(VARIANTS) + 1,) and np.all(np.isfinite(ms)) and ms[v] == ms.min()
    n = (6 * 2 + 2) * (len(VARIANTS) + 1)
    B.step(10, chunk=10)
    for k, (p, r) in enumerate(zip(ps, rhos)):
        assert np.array_equal(B.lattice(k).get_state(), _alone(p, r, n + 10)), k
    B.close()
