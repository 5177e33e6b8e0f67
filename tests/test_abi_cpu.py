"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point include/lbm.h declares, and validates arguments before any
device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from max_lattices import MAX_LATTICES, STORAGE_BYTES, buffer_bytes
from paper_1202_6130_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_library_built_from_current_sources():
    """The library that the tests load is newer than every source it is built
    from (a stale library would hide a source that no longer compiles)."""
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("library not built")
    csrc = os.path.join(ROOT, "paper_1202_6130_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in os.listdir(csrc)] + [HEADER]
    built = os.path.getmtime(lbm.LIB_PATH)
    newer = [os.path.relpath(f, ROOT) for f in srcs if os.path.getmtime(f) > built]
    assert not newer, f"rebuild (python -m paper_1202_6130_amd.build): newer sources {newer}"


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(lbm.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 26
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_tile_shape_table_and_null_context():
    shapes = lbm.lbm_tile_shapes()
    assert len(shapes) >= 2 and shapes[0] == (16, 2, 1)
    assert all(w in (4, 8, 16) and 1 <= r <= 4 and s in (1, 2, 4) and w % s == 0 for w, r, s in shapes)
    L = lbm.lib()
    assert L.lbm_get_tile_shape(None) == -1
    assert L.lbm_set_tile_shape(None, 0) == lbm.LBM_EINVAL
    assert L.lbm_tune(None, 1, None, None) == lbm.LBM_EINVAL
    assert L.lbm_batch_tune(None, 1, None, None) == lbm.LBM_EINVAL
    assert L.lbm_batch_set_tile_shapes(None, None) == lbm.LBM_EINVAL


def test_two_step_table_and_null_context():
    """Two-steps-per-pass variants (strips, output rows, waves per workgroup)
    and the NULL-argument errors of their calls (no GPU needed)."""
    v = lbm.lbm_two_step_variants()
    assert v == [(1, 8, 4), (1, 8, 8), (2, 8, 8), (1, 12, 6), (1, 12, 12), (1, 16, 8), (1, 16, 16), (1, 24, 8),
                 (1, 24, 12)]
    # every block's rows split evenly over the waves of a strip, at most 1024 threads
    assert all(r % (w // s) == 0 and w * 64 <= 1024 for s, r, w in v)
    L = lbm.lib()
    assert L.lbm_get_two_step(None) == -2
    assert L.lbm_set_two_step(None, 0) == lbm.LBM_EINVAL
    assert L.lbm_tune_two_step(None, 1, None, None) == lbm.LBM_EINVAL
    assert L.lbm_batch_get_two_step(None) == -2
    assert L.lbm_batch_set_two_step(None, 0) == lbm.LBM_EINVAL
    assert L.lbm_batch_tune_two_step(None, 1, None, None) == lbm.LBM_EINVAL


def test_params_struct_matches_header():
    # field order of lbm_params in the header must match the ctypes mirror
    text = open(HEADER).read()
    body = text[text.index("typedef struct {"):text.index("} lbm_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b([A-Za-z_]+)(?:\[\d+\])?\s*[,;]", body)
    assert fields == [f for f, _ in lbm.lbm_params._fields_]


def test_defaults():
    p = lbm.lbm_params_default()
    assert p.tau == 1.0 and p.G == -5.0 and p.eps == 1.0
    assert p.wall_width == 2.0 and p.core_range == 1.0 and p.tail_range == 3.0
    assert p.slab_rows == 8 and p.storage == lbm.STORE_F32 and p.wall_kind == lbm.WALL_NONE


@pytest.mark.parametrize("field,value,msg", [
    ("tau", 0.5, "tau"), ("eps", 0.9, "eps"), ("nx", 0, "nx"), ("storage", 7, "storage"),
    ("wall_kind", 9, "wall_kind"), ("reserved", 1, "reserved"), ("seg_rows", -1, "seg_rows"),
    ("G", float("nan"), "non-finite"),
])
def test_validation_errors(field, value, msg):
    p = lbm.lbm_params_default(nx=16, ny=8)
    setattr(p, field, value)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes(p)
    assert e.value.code == lbm.LBM_EINVAL and msg in str(e.value)


def test_slab_validation():
    p = lbm.lbm_params_default(nx=16, ny=8, wall_kind=lbm.WALL_FLAT_SLAB, slab_rows=8)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(p)
    p.slab_rows = 3
    assert lbm.lbm_workspace_bytes(p) > 0


def test_too_large_lattice_rejected():
    p = lbm.lbm_params_default(nx=65536, ny=65536)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes(p)
    assert "too large" in str(e.value)


@pytest.mark.parametrize("case", sorted(MAX_LATTICES))
def test_largest_lattice_accepted_one_more_row_rejected(case):
    q, st, nx, ny = MAX_LATTICES[case]
    assert buffer_bytes(q, st, nx, ny) < 1 << 32 <= buffer_bytes(q, st, nx, ny + 1)
    kw = dict(storage={"f32": lbm.STORE_F32, "f16dev": lbm.STORE_F16DEV, "f64": lbm.STORE_F64}[st],
              lattice=lbm.D2Q21 if q == 21 else lbm.D2Q9)
    if q == 21:
        kw.update(psi_kind=lbm.PSI_EOS, G=-1.0)
    assert lbm.lbm_workspace_bytes(lbm.lbm_params_default(nx=nx, ny=ny, **kw)) > 2 * q * nx * ny * STORAGE_BYTES[st]
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes(lbm.lbm_params_default(nx=nx, ny=ny + 1, **kw))
    assert "too large" in str(e.value)


def test_workspace_bytes_scale_with_storage():
    sizes = {}
    for st in (lbm.STORE_F16DEV, lbm.STORE_F32, lbm.STORE_F64):
        sizes[st] = lbm.lbm_workspace_bytes(lbm.lbm_params_default(nx=1024, ny=512, storage=st))
    N = 1024 * 512
    # two population buffers dominate: 18 N * bytes
    assert sizes[lbm.STORE_F16DEV] < sizes[lbm.STORE_F32] < sizes[lbm.STORE_F64]
    assert sizes[lbm.STORE_F32] >= 18 * N * 4
    assert sizes[lbm.STORE_F32] < 18 * N * 4 * 1.6


def test_create_rejects_bad_host_inputs_before_device_work():
    p = lbm.lbm_params_default(nx=8, ny=8)
    rho = np.ones((8, 8))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None, None, None, 0, 0, 0)
    assert e.value.code == lbm.LBM_EINVAL
    bad = rho.copy(); bad[3, 3] = -1
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, bad, None, None, 0, 0, 0)
    assert "rho0" in str(e.value)
    u0 = np.zeros((2, 8, 8)); u0[1, 2, 5] = np.inf
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, rho, u0, None, 0, 0, 0)
    assert "u0 at 85" in str(e.value)          # [2][ny][nx]: plane 1 starts at 64, + 2 * 8 + 5
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, rho, None, np.zeros((3, 8, 8)), 0, 0, 0)
    assert "wall_fields" in str(e.value)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, rho, None, None, 0, 0, 0)
    assert "workspace" in str(e.value)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, rho, None, None, 256, 16, 0)
    assert e.value.code == lbm.LBM_ENOMEM
    # no context exists: the message is the thread's
    assert "workspace too small" in lbm.lbm_last_error(None)


def test_binding_stacks_initial_velocity():
    ux, uy = np.full((3, 4), 0.1), np.full((3, 4), -0.2)
    u0 = lbm._u0(ux, uy)
    assert u0.shape == (2, 3, 4) and u0.flags["C_CONTIGUOUS"]
    assert (u0[0] == 0.1).all() and (u0[1] == -0.2).all()
    assert lbm._u0(None, None) is None
    with pytest.raises(ValueError):
        lbm._u0(ux, None)


def test_null_context_calls_fail_cleanly():
    L = lbm.lib()
    out = (ctypes.c_double * 6)()
    r = ctypes.c_double()
    assert L.lbm_step(None, 1, None) == lbm.LBM_EINVAL
    assert L.lbm_step(None, 1, ctypes.byref(r)) == lbm.LBM_EINVAL
    assert "ctx is NULL" in lbm.lbm_last_error(None)
    assert L.lbm_diagnostics(None, out) == lbm.LBM_EINVAL
    assert L.lbm_step_index(None) == -1


def test_batch_validation():
    ps = [lbm.lbm_params_default(nx=64, ny=32, wall_kind=lbm.WALL_FLAT_SLAB) for _ in range(3)]
    assert lbm.lbm_batch_workspace_bytes(ps) > 3 * lbm.lbm_workspace_bytes(ps[0]) * 0.9
    ps[1].storage = lbm.STORE_F64
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_workspace_bytes(ps)
    assert "F32" in str(e.value)


def test_mask_wall_parameters_validated():
    from paper_1202_6130_amd import lbm
    ok = lbm.lbm_params_default(nx=16, ny=16, wall_kind=lbm.WALL_MASK)
    assert ok.filter_core == 5 and ok.filter_wall == 22
    assert lbm.lbm_workspace_bytes(ok) > 0
    for core, wall in ((6, 5), (-1, 22), (0, 0), (5, 1001)):
        bad = lbm.lbm_params_default(nx=16, ny=16, wall_kind=lbm.WALL_MASK, filter_core=core, filter_wall=wall)
        with pytest.raises(lbm.LbmError):
            lbm.lbm_workspace_bytes(bad)


@pytest.mark.parametrize("src,dst,nbytes,msg", [
    (0, 4096, 16, "NULL"), (4096, 0, 16, "NULL"), (4100, 8192, 16, "multiples of 16"),
    (4096, 8200, 16, "multiples of 16"), (4096, 8192, 24, "multiples of 16"), (4096, 4112, 32, "overlap"),
    (4112, 4096, 32, "overlap"),
])
def test_device_copy_rejects_bad_arguments(src, dst, nbytes, msg):
    # validated on the host before any launch: the addresses are never touched
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_device_copy(src, dst, nbytes, 0)
    assert e.value.code == lbm.LBM_EINVAL and msg in str(e.value)
