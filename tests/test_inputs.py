"""CPU checks of the seeded input generators."""
import numpy as np

from paper_1202_6130_amd import inputs as I


def test_spinodal_half_liquid_and_seeded():
    a = I.spinodal_field(64, seed=3)
    b = I.spinodal_field(64, seed=3)
    c = I.spinodal_field(64, seed=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert (a == I.RHO_L).sum() == 64 * 64 // 2
    assert set(np.unique(a)) == {I.RHO_G, I.RHO_L}


def test_drop_field_shape():
    r = I.drop_field(128, 64, 20.0)
    assert r.shape == (64, 128)
    assert abs(r[0, 64] - I.RHO_L) < 1e-6 and abs(r[40, 5] - I.RHO_G) < 1e-6
    assert np.all(r[64 - 8 + 1:] == I.RHO_G)
    # centred on the lower face: mirror symmetric about x = 64
    assert np.allclose(r[:, 1:], r[:, 1:][:, ::-1])


def test_ensemble_and_requests():
    cs = I.ensemble_cases(seed=0, count=256)
    assert len(cs) == 256
    assert all(c.nx % 32 == 0 and 128 <= c.nx <= 1024 and c.ny % 32 == 0 and 64 <= c.ny <= 512 for c in cs)
    assert all(-5.5 <= c.G <= -4.5 and 0 <= c.G_R <= 1 and 0 <= c.G_A <= 0.6 for c in cs)
    rs = I.request_stream(seed=0, rate=20.0, count=300)
    t = np.array([r.arrival for r in rs])
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
    assert abs(300 / t[-1] - 20.0) < 4.0          # Poisson rate
    assert {r.kind for r in rs} == {"angle", "slip"}
