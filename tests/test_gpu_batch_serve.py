"""GPU tests of batched stepping over existing contexts and of the server."""
import numpy as np
import pytest

from paper_1202_6130_amd import inputs as I
from paper_1202_6130_amd import lbm
from paper_1202_6130_amd import serve

pytestmark = pytest.mark.gpu


def _stream():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.Stream()


def _drop_lattice(case, stream, seg=0):
    p = lbm.lbm_params_default(nx=case.nx, ny=case.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=case.G, G_R=case.G_R,
                               G_A=case.G_A, seg_rows=seg)
    return lbm.Lattice(p, I.drop_field(case.nx, case.ny, case.radius), stream=stream), p


def test_attach_matches_alone_bitwise():
    """Contexts at different step parities, attached into one batch and
    stepped with graph replays, end bitwise where they end alone."""
    cases = I.ensemble_cases(seed=5, count=4)
    st = _stream()
    lats, params = [], []
    for k, c in enumerate(cases):
        L, p = _drop_lattice(c, st)
        L.step(k)          # parities 0, 1, 0, 1
        lats.append(L)
        params.append(p)
    A = lbm.Attached(lats)
    A.step(30, chunk=10)
    A.step(1, chunk=0)
    with pytest.raises(lbm.LbmError) as e:
        lats[0].step(1)
    assert e.value.code == lbm.LBM_ESTATE
    A.close()
    for k, (c, L) in enumerate(zip(cases, lats)):
        assert L.step_index == k + 31
        ref, _ = _drop_lattice(c, st)
        ref.step(k + 31)
        assert np.array_equal(L.get_state(), ref.get_state())
        L.step(5)          # usable alone again after the batch is gone
        ref.step(5)
        assert np.array_equal(L.get_state(), ref.get_state())
        ref.close()
        L.close()


def test_attach_rejects_mixed_streams():
    cases = I.ensemble_cases(seed=6, count=2)
    a, _ = _drop_lattice(cases[0], _stream())
    b, _ = _drop_lattice(cases[1], _stream())
    with pytest.raises(ValueError):
        lbm.Attached([a, b])
    a.close()
    b.close()


def _small_requests(n, seed=0):
    reqs = I.request_stream(seed=seed, rate=200.0, count=n, nx_range=(64, 192), ny_range=(64, 160))
    return reqs


def test_server_alone_equals_mix():
    """Each request's result is the same served alone and in the mix."""
    reqs = _small_requests(5, seed=1)
    srv = serve.Server(max_steps=600, diag_every=100, tol=0.0)
    mix = srv.run(reqs, realtime=False)
    assert all(not r.error for r in mix), [r.error for r in mix]
    for req, got in zip(reqs, mix):
        alone = serve.Server(max_steps=600, diag_every=100, tol=0.0).run([req], realtime=False)[0]
        assert alone.steps == got.steps == 600
        assert np.array_equal(np.array(alone.value), np.array(got.value)), (req.kind, alone.value, got.value)


def test_server_admission_by_footprint():
    reqs = _small_requests(4, seed=2)
    srv = serve.Server(max_steps=200, diag_every=100, tol=0.0)
    fps = [srv.footprint(r) for r in reqs]
    budget = max(fps)
    srv = serve.Server(budget_bytes=budget, max_steps=200, diag_every=100, tol=0.0)
    res = srv.run(reqs, realtime=False)
    assert srv.max_seen_used <= budget
    # the largest request can never share the budget with another one
    assert srv.max_seen_resident < len(reqs)
    assert all(not r.error and r.steps == 200 for r in res)
    # admission order follows arrival order
    admitted = [r.admitted for r in sorted(res, key=lambda r: r.arrival)]
    assert admitted == sorted(admitted)


def test_server_isolates_failed_request():
    reqs = _small_requests(3, seed=3)
    bad = reqs[1].rid

    def plant_nan(req, lat):
        if req.rid == bad:
            f = lat.get_state()
            f[0, 3, 3] = np.nan
            lat.set_state(f, 0)

    srv = serve.Server(max_steps=300, diag_every=100, tol=0.0, on_admit=plant_nan)
    res = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert "non-finite" in res[bad].error
    assert all(not r.error and r.steps == 300 for k, r in res.items() if k != bad)


def test_sequential_baseline_same_results():
    reqs = _small_requests(3, seed=4)
    a = serve.Server(max_steps=300, diag_every=100, tol=0.0).run(reqs, realtime=False)
    b = serve.Server(max_steps=300, diag_every=100, tol=0.0, batched=False, max_resident=1).run(reqs,
                                                                                                realtime=False)
    for x, y in zip(a, b):
        assert x.steps == y.steps
        assert np.array_equal(np.array(x.value), np.array(y.value))
