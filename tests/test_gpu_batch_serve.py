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


# ------------------------------------------------------------ against the oracle
CS = 1.0 / np.sqrt(3.0)


def _oracle_drop(nx, ny, radius, G, G_R, G_A, steps):
    import oracle as O
    po = O.make_params(nx, ny, tau=1.0, G=G, G_R=G_R, G_A=G_A, eps=1.0)
    w = O.Walls.flat_slab(nx, ny, I.SLAB_ROWS, 2.0, 1.0, 3.0)
    fo = O.run(po, w, O.init(po, I.drop_field(nx, ny, radius)), steps)
    return O.macros(po, w, fo)[:3], (po, w, fo)


@pytest.mark.parametrize("two_step", [-1, 7])
def test_batch_lattices_match_oracle(two_step):
    """Four sessile drops of uneven size with different G, G_R and G_A stepped
    together in one batch (graph replays of 10 steps, then plain launches to
    an odd total), with one and with two time steps per launch: every lattice
    against the FP64 oracle run of the same drop alone, at the FP32 bar
    (density within 1e-5 of its maximum, velocity within 1e-5 of c_s and of
    the largest oracle velocity)."""
    cases = [I.DropCase(96, 64, 18.0, -5.0, 0.5, 0.3), I.DropCase(160, 64, 19.2, -4.6, 0.9, 0.1),
             I.DropCase(64, 96, 19.2, -5.4, 0.2, 0.55), I.DropCase(128, 128, 38.4, -4.9, 0.7, 0.4)]
    steps = 301
    ps = [lbm.lbm_params_default(nx=c.nx, ny=c.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=c.G, G_R=c.G_R, G_A=c.G_A)
          for c in cases]
    B = lbm.Batch(ps, [I.drop_field(c.nx, c.ny, c.radius) for c in cases])
    B.two_step = two_step
    B.step(300, chunk=10)
    B.step(1)
    for k, c in enumerate(cases):
        rho, ux, uy, _ = B.lattice(k).moments()
        (r_o, ux_o, uy_o), _ = _oracle_drop(c.nx, c.ny, c.radius, c.G, c.G_R, c.G_A, steps)
        e_rho = np.abs(rho - r_o).max() / np.abs(r_o).max()
        du = max(np.abs(ux - ux_o).max(), np.abs(uy - uy_o).max())
        umax = max(np.abs(ux_o).max(), np.abs(uy_o).max())
        print(f"batch lattice {k} ({c.nx}x{c.ny}, G {c.G}), two-step {two_step}: rho {e_rho:.2e}, "
              f"u/c_s {du / CS:.2e}, u/max|u| {du / umax:.2e}")
        assert e_rho <= 1e-5 and du / CS <= 1e-5 and du / umax <= 1e-5
    B.close()


def test_served_results_match_oracle():
    """Two small requests, a contact-angle query (sessile drop) and a slip
    query (body-force channel), served together for 600 steps: the reported
    angle and slip length against the oracle's on the same lattice after the
    same number of steps."""
    import oracle as O
    reqs = [I.Request(0, 0.0, "angle", 96, 64, -5.0, 0.6, 0.2, 1.0),
            I.Request(1, 0.0, "slip", 32, 96, -5.0, 0.6, 0.2, 1.3)]
    srv = serve.Server(max_steps=600, diag_every=100, tol=0.0, tile_costs=None, two_step=-1)
    got = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert all(not r.error and r.steps == 600 for r in got.values())
    for req in reqs:
        p, rho0 = serve.request_params(req)
        u0 = serve.initial_velocity(req, p)
        po = O.make_params(req.nx, req.ny, tau=1.0, G=req.G, G_R=req.G_R, G_A=req.G_A, eps=req.eps,
                           F_ext=tuple(p.F_ext))
        w = O.Walls.flat_slab(req.nx, req.ny, I.SLAB_ROWS, 2.0, 1.0, 3.0)
        f0 = O.init(po, rho0) if u0 is None else O.init(po, rho0, u0[0], u0[1])
        fo = O.run(po, w, f0, 600)
        if req.kind == "angle":
            want = O.contact_angle(po, w, fo, I.ISO, 0.0)
            print("served angle", got[0].value[:2], "oracle", want[:2])
            assert abs(got[0].value[0] - want[0]) < 1e-3 and abs(got[0].value[1] - want[1]) < 1e-3
        else:
            want = O.slip_length(po, w, fo, I.SLAB_ROWS, 2.0)
            print("served slip", got[1].value, "oracle", want)
            assert abs(got[1].value[0] - want[0]) < 1e-2 * abs(want[0])
            assert abs(got[1].value[1] - want[1]) < 1e-2 * abs(want[1])


def test_server_staggered_admission_equals_alone():
    """Continuous batching with lattices joining a running batch: at most two
    resident, requests retiring at different steps by the residual criterion,
    so the later ones are attached while others are mid-run (at other step
    indices and buffer parities).  Every result equals, bit for bit, the same
    request served alone."""
    reqs = _small_requests(5, seed=7)
    kw = dict(max_steps=3000, diag_every=100, tol=2e-3, tile_costs=None, two_step=7)
    srv = serve.Server(max_resident=2, **kw)
    mix = srv.run(reqs, realtime=False)
    assert all(not r.error for r in mix), [r.error for r in mix]
    admitted = sorted(r.admitted for r in mix)
    assert srv.max_seen_resident == 2 and admitted[-1] > admitted[0]
    assert len({r.steps for r in mix}) > 1          # retired at different steps
    for req, got in zip(reqs, mix):
        alone = serve.Server(**kw).run([req], realtime=False)[0]
        assert alone.steps == got.steps and alone.converged == got.converged
        assert np.array_equal(np.array(alone.value), np.array(got.value)), (req.kind, alone.value, got.value)
