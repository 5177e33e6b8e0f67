"""GPU tests of the step tile shapes and the autotuner: every shape computes
bitwise the same update, for every storage mode and wall kind, on lattices
with ragged edges; tuning (single and batched) leaves states bitwise equal to
plain stepping; padded population planes round-trip."""
import numpy as np
import pytest

from paper_1202_6130_amd import inputs as I
from paper_1202_6130_amd import lbm

pytestmark = pytest.mark.gpu
SHAPES = [(16, 2, 1), (8, 2, 1), (8, 4, 1), (16, 3, 1), (16, 2, 2), (8, 4, 2), (16, 4, 2), (16, 4, 4), (16, 3, 2)]


def _fields(nx, ny, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 0.5, (ny, nx))])


def _run(nx, ny, storage, wall, shape, steps, rho0, fields=None):
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage, wall_kind=wall, G_R=0.5, G_A=0.3, eps=1.3,
                               tau=0.9, F_ext=(1e-5, 0.0), rho_ref=float(rho0.mean()))
    L = lbm.Lattice(p, rho0, wall_fields=fields)
    L.tile_shape = shape
    assert L.tile_shape == shape
    L.step(steps)
    s = L.get_state()
    L.close()
    return s


@pytest.mark.parametrize("storage", [lbm.STORE_F32, lbm.STORE_F16DEV, lbm.STORE_F64, lbm.STORE_F32X])
@pytest.mark.parametrize("nx,ny", [(200, 96), (130, 71), (64, 15), (5, 6), (70, 1)])
def test_every_shape_same_update(storage, nx, ny):
    wall = lbm.WALL_FLAT_SLAB if ny > 9 else lbm.WALL_NONE
    rho0 = I.drop_field(nx, ny, 0.3 * min(nx, ny) + 1) if ny > 9 else I.random_state_field(nx, ny, 3)[0]
    ref = _run(nx, ny, storage, wall, 0, 25, rho0)
    for s in range(1, len(SHAPES)):
        assert np.array_equal(_run(nx, ny, storage, wall, s, 25, rho0), ref), (storage, nx, ny, s)


def test_every_shape_same_update_node_fields():
    nx, ny = 150, 77
    rho0 = I.random_state_field(nx, ny, 4)[0]
    fields = _fields(nx, ny, 5)
    ref = _run(nx, ny, lbm.STORE_F32, lbm.WALL_FIELDS, 0, 20, rho0, fields)
    for s in range(1, len(SHAPES)):
        assert np.array_equal(_run(nx, ny, lbm.STORE_F32, lbm.WALL_FIELDS, s, 20, rho0, fields), ref)


def test_shape_table():
    assert lbm.lbm_tile_shapes() == SHAPES


def test_tune_single_is_plain_stepping():
    nx, ny = 384, 160
    rho0 = I.drop_field(nx, ny, 48.0)
    p = lbm.lbm_params_default(nx=nx, ny=ny, wall_kind=lbm.WALL_FLAT_SLAB, G_R=0.4, G_A=0.2, diag_interval=10)
    L = lbm.Lattice(p, rho0)
    shape, ms = L.tune(4)
    assert 0 <= shape < len(SHAPES) and L.tile_shape == shape
    assert np.all(np.isfinite(ms)) and np.all(ms > 0) and ms[shape] == ms.min()
    n = L.step_index
    assert n == (3 * 4 + 1) * len(SHAPES)
    ref = lbm.Lattice(p, rho0)
    ref.step(n)
    assert np.array_equal(L.get_state(), ref.get_state())
    L.step(7)
    ref.step(7)
    assert np.array_equal(L.get_state(), ref.get_state())
    # the residual bookkeeping of the built-in diagnostic pass is unaffected
    assert np.array_equal(L.diagnostics(), ref.diagnostics())
    L.close()
    ref.close()


def _ensemble(seed, count):
    cases = I.ensemble_cases(seed=seed, count=count)
    ps = [lbm.lbm_params_default(nx=c.nx, ny=c.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=c.G, G_R=c.G_R, G_A=c.G_A)
          for c in cases]
    rhos = [I.drop_field(c.nx, c.ny, c.radius) for c in cases]
    return ps, rhos


def _alone(p, rho, steps):
    L = lbm.Lattice(lbm.lbm_params_default(nx=p.nx, ny=p.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=p.G, G_R=p.G_R,
                                           G_A=p.G_A), rho)
    L.step(steps)
    s = L.get_state()
    L.close()
    return s


def test_batch_mixed_shapes_bitwise():
    ps, rhos = _ensemble(8, 6)
    B = lbm.Batch(ps, rhos)
    B.tile_shapes = [k % len(SHAPES) for k in range(len(ps))]
    assert list(B.tile_shapes) == [k % len(SHAPES) for k in range(len(ps))]
    B.step(20, chunk=10)
    B.tile_shapes = [(k + 1) % len(SHAPES) for k in range(len(ps))]   # drops the recorded graphs
    B.step(21, chunk=10)
    for k, (p, rho) in enumerate(zip(ps, rhos)):
        assert np.array_equal(B.lattice(k).get_state(), _alone(p, rho, 41)), k
    B.close()


def test_batch_tune_is_plain_stepping():
    ps, rhos = _ensemble(9, 12)
    B = lbm.Batch(ps, rhos)
    shapes, ms = B.tune(3)
    nshape = len(SHAPES)
    assert len(shapes) == len(ps) and all(0 <= s < nshape for s in shapes)
    assert list(B.tile_shapes) == list(shapes)
    assert np.all(np.isfinite(ms[:nshape]))
    tuned_steps = (nshape + (0 if np.isnan(ms[nshape]) else 1)) * (3 * 3 + 1)
    B.step(10, chunk=10)
    for k, (p, rho) in enumerate(zip(ps, rhos)):
        assert np.array_equal(B.lattice(k).get_state(), _alone(p, rho, tuned_steps + 10)), k
    B.close()


def test_attached_keeps_context_shapes():
    ps, rhos = _ensemble(10, 3)
    import torch
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    lats = [lbm.Lattice(p, r, stream=st) for p, r in zip(ps, rhos)]
    for k, L in enumerate(lats):
        L.tile_shape = 2 * k + 1
    A = lbm.Attached(lats)
    assert list(A.tile_shapes) == [1, 3, 5]
    A.tile_shapes = [6, 2, 4]
    A.step(10, chunk=10)
    A.close()
    assert [L.tile_shape for L in lats] == [6, 2, 4]
    for L, p, r in zip(lats, ps, rhos):
        assert np.array_equal(L.get_state(), _alone(p, r, 10))
        L.close()


@pytest.mark.parametrize("storage", [lbm.STORE_F32, lbm.STORE_F16DEV, lbm.STORE_F64])
def test_padded_planes_state_roundtrip(storage):
    """Lattices above 1 MiB per plane use a padded plane stride."""
    nx, ny = 1024, 640
    rng = np.random.Generator(np.random.PCG64(21))
    p = lbm.lbm_params_default(nx=nx, ny=ny, storage=storage, rho_ref=1.0)
    L = lbm.Lattice(p, np.ones((ny, nx)))
    f = 0.1 + 0.01 * rng.uniform(-1, 1, (9, ny, nx))
    if storage == lbm.STORE_F32:
        f = f.astype(np.float32).astype(np.float64)
    L.set_state(f, 0)
    g = L.get_state()
    tol = {lbm.STORE_F32: 0.0, lbm.STORE_F64: 0.0, lbm.STORE_F16DEV: 1e-3}[storage]
    assert np.abs(g - f).max() <= tol
    L.close()
