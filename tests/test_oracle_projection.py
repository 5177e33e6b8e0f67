"""Pins of the oracle's projection step (Sec. II.A, after eq. f2) and of the
collision that uses it.

The projection replaces a node's populations by the truncated Hermite form
of eq. f2 built from their own M0, M1 and M2.  Two properties determine it
without restating its formula: it keeps those six moments, and its output is
w_i times a polynomial of degree two in c_i (the functional form of eq. f2);
on a quadrature of degree >= 4 exactly one such set of populations has given
M0, M1, M2.  The rest follow: ghost components vanish, the map is idempotent,
equilibria are fixed points, and at tau = 1 the collision is unchanged.
"""
import numpy as np
import pytest

from paper_1202_6130_amd import inputs as I

LATTICES = [9, 21]


def moments(f, cx, cy):
    return np.array([f.sum(), (f * cx).sum(), (f * cy).sum(), (f * cx * cx).sum(), (f * cx * cy).sum(),
                     (f * cy * cy).sum()])


def quad_basis(cx, cy):
    cx = cx.astype(float)
    cy = cy.astype(float)
    return np.stack([np.ones_like(cx), cx, cy, cx * cx, cx * cy, cy * cy], axis=1)


@pytest.mark.parametrize("lat", LATTICES)
def test_projection_keeps_moments_and_has_the_form_of_f2(orc, lat):
    """Catches a dropped or doubled second-order term, a theta of the other
    lattice, or a wrong weight: any of them breaks the moments or the form."""
    cx, cy, w, th = orc.lattice_tables(lat)
    rng = np.random.Generator(np.random.PCG64(lat))
    B = quad_basis(cx, cy)
    for _ in range(20):
        f = w * rng.uniform(0.5, 1.5, len(w)) * rng.uniform(0.1, 2.0)
        g = orc.project(f, lat)
        assert np.abs(moments(g, cx, cy) - moments(f, cx, cy)).max() < 1e-15
        coef, res, *_ = np.linalg.lstsq(B, g / w, rcond=None)
        assert np.abs(B @ coef - g / w).max() < 1e-12


@pytest.mark.parametrize("lat", LATTICES)
def test_projection_removes_ghosts_and_is_idempotent(orc, lat):
    """A population vector with zero M0, M1, M2 (a pure ghost mode) projects
    to zero; projecting twice equals projecting once; an equilibrium (eq. f2
    with M2 = rho u u + rho theta I) is a fixed point."""
    cx, cy, w, th = orc.lattice_tables(lat)
    rng = np.random.Generator(np.random.PCG64(10 + lat))
    B = quad_basis(cx, cy)
    # null space of the six moment functionals
    _, _, vt = np.linalg.svd(B.T)
    null = vt[6:]
    for k in range(null.shape[0]):
        gh = null[k] * 1e-2
        assert np.abs(moments(gh, cx, cy)).max() < 1e-15
        assert np.abs(orc.project(gh, lat)).max() < 1e-16
    f = w * rng.uniform(0.5, 1.5, len(w))
    g = orc.project(f, lat)
    assert np.abs(orc.project(g, lat) - g).max() < 4e-16
    feq = orc.equilibrium(1.3, 0.05, -0.03, lat)
    assert np.abs(orc.project(feq, lat) - feq).max() < 4e-16


@pytest.mark.parametrize("lat", LATTICES)
def test_projected_collision_conserves_and_is_bgk_at_tau_one(orc, lat):
    """Mass conserved and momentum raised by exactly F for any tau; at tau = 1
    the post-collision state is feq(u*) with or without the projection."""
    nx, ny = 10, 8
    psi_kind = 1 if lat == 21 else 0
    G = -1.0 if lat == 21 else -5.0
    rng = np.random.Generator(np.random.PCG64(20 + lat))
    walls = orc.Walls(rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 0.4, (ny, nx)))
    rho, ux, uy = I.random_state_field(nx, ny, 3, lo=0.1, hi=1.2)
    cx, cy, w, th = orc.lattice_tables(lat)
    for tau in (0.7, 1.0, 1.4):
        kw = dict(tau=tau, G=G, G_R=0.4, G_A=0.2, eps=1.3, F_ext=(1e-3, -2e-3), lattice=lat, psi_kind=psi_kind)
        pb = orc.make_params(nx, ny, **kw)
        pp = orc.make_params(nx, ny, collision=1, **kw)
        f = orc.init(pb, rho, ux, uy) * (1 + 0.05 * rng.uniform(-1, 1, (ny, nx, len(w))))
        F = orc.forces(pp, walls, f)["F"]
        g = orc.collide(pp, walls, f)
        assert np.abs(g.sum(-1) - f.sum(-1)).max() < 1e-14
        assert np.abs((g * cx).sum(-1) - (f * cx).sum(-1) - F[..., 0]).max() < 1e-14
        assert np.abs((g * cy).sum(-1) - (f * cy).sum(-1) - F[..., 1]).max() < 1e-14
        gb = orc.collide(pb, walls, f)
        if tau == 1.0:
            assert np.abs(g - gb).max() < 1e-15
        else:
            assert np.abs(g - gb).max() > 1e-6      # the ghost content of f differs


@pytest.mark.parametrize("lat", LATTICES)
def test_projected_shear_wave_viscosity(orc, lat):
    """The projection keeps the hydrodynamics: a decaying shear wave still has
    nu = theta (tau - 1/2) at tau = 0.8."""
    nx, ny, tau = 4, 64, 0.8
    p = orc.make_params(nx, ny, tau=tau, G=0.0, lattice=lat, collision=1)
    k = 2 * np.pi / ny
    y = np.arange(ny)
    ux0 = (1e-4 * np.sin(k * y))[:, None] * np.ones((1, nx))
    wl = orc.Walls.none(nx, ny)
    f = orc.run(p, wl, orc.init(p, np.ones((ny, nx)), ux0, np.zeros((ny, nx))), 400)
    _, ux, _, _ = orc.macros(p, wl, f)
    amp = (ux[:, 0] * np.sin(k * y)).sum() / (np.sin(k * y) ** 2).sum()
    nu_meas = -np.log(amp / 1e-4) / (k * k * 400)
    th = orc.lattice_tables(lat)[3]
    assert abs(nu_meas - th * (tau - 0.5)) / (th * (tau - 0.5)) < 5e-3
