"""Host logic of the server that needs no GPU: the binary32 residual-floor
detector, the stalled-noise signal of the rest rule, the warm start of slip
queries and the JSON-safe summary."""
import json
import math

import numpy as np

from paper_1202_6130_amd import inputs as I
from paper_1202_6130_amd import serve


def test_floor_detected_on_plateau():
    f = serve.Floor(window=20)
    r = np.concatenate([np.geomspace(1e-2, 3e-6, 60), 3e-6 * (1 + 0.2 * np.sin(np.arange(200)))])
    hits = [f.add(v) for v in r]
    first = hits.index(True)
    # not before the decay has flattened out for a full window
    assert first >= 60 + 20
    assert all(hits[first:])


def test_floor_not_detected_while_decaying():
    # a slow channel: the residual halves every 700 passes (70000 steps)
    f = serve.Floor(window=200)
    r = 1e-4 * 0.5 ** (np.arange(3000) / 700.0)
    assert not any(f.add(v) for v in r)


def test_floor_not_detected_above_ceiling():
    f = serve.Floor(window=10, ceiling=1e-4)
    assert not any(f.add(2e-4) for _ in range(100))


def test_noise_residual_marks_stalled_not_floor():
    """Residuals of two independent noise fields hover about sqrt(2): the
    detector reports a stall at that level (the server then checks |u|), and
    never a floor (above the ceiling)."""
    rng = np.random.default_rng(3)
    f = serve.Floor(window=50)
    floors = [f.add(v) for v in np.sqrt(2) * (1 + 0.05 * rng.standard_normal(100))]
    assert not any(floors)
    assert f.stalled and f.level >= serve.NOISE_RESIDUAL


def test_slow_motion_is_not_noise():
    """A coherent slow flow (residual 1e-3, stalled) stays below the noise
    level, so the rest rule does not apply to it."""
    f = serve.Floor(window=50)
    for _ in range(100):
        f.add(1e-3)
    assert f.stalled and f.level < serve.NOISE_RESIDUAL


def test_summary_is_json():
    res = [serve.Result(0, "angle", 8, 8, 0.0, 0.0, 1.0, 100, np.bool_(True), np.bool_(True), False, 1e-5),
           serve.Result(1, "slip", 8, 8, 0.5, 0.5, 2.0, 200, True, False, True, 1.4)]
    d = serve.summarize(res, 2.0)
    json.dumps(d)
    assert d["converged"] == 2 and d["converged_at_floor"] == 1 and d["converged_at_rest"] == 1


def test_slip_warm_start_is_the_no_slip_profile():
    req = I.Request(0, 0.0, "slip", 32, 136, -5.0, 0.5, 0.2, 1.0)
    p, rho0 = serve.request_params(req)
    u0 = serve.initial_velocity(req, p)
    assert u0.shape == (2, 136, 32) and not u0[1].any()
    prof = u0[0, :, 0]
    assert np.array_equal(u0[0], np.repeat(prof[:, None], 32, axis=1))
    H, yw, nu = 136 - 8, 2.0 * math.atanh(0.98), 1.0 / 6.0
    # zero at and outside the hydrodynamic boundaries, maximum at mid-gap
    assert (prof[:5] == 0).all() and (prof[H - 4:] == 0).all()
    mid = H / 2
    umax = p.F_ext[0] * (mid - yw) ** 2 / (2 * serve.CHANNEL_RHO * nu)
    assert abs(prof[int(mid)] - umax) < 1e-12
    # curvature -F / (rho nu) (the Poiseuille pin of the oracle)
    assert abs(np.diff(prof[10:H - 10], 2).mean() + p.F_ext[0] / (serve.CHANNEL_RHO * nu)) < 1e-15
    assert serve.initial_velocity(I.Request(1, 0.0, "angle", 64, 64, -5.0, 0.5, 0.2, 1.0), p) is None
