"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the plausible oracle mistake it would expose.  None of these
tests retypes the oracle's own formulas: they check conservation laws, closed
forms, fixed points, thermodynamic coexistence computed by quadrature, the
Laplace law, symmetry, geometric fits on exact curves, and the paper's
qualitative trends for the wall model (Sec. III).
"""
import ctypes
import os

import numpy as np
import pytest
from scipy import integrate, optimize

from paper_1202_6130_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def walls_random(orc, nx, ny, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return orc.Walls(rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 1, (ny, nx)),
                     rng.uniform(-0.3, 0.5, (ny, nx)))


def random_f(orc, p, seed):
    rho, ux, uy = I.random_state_field(p.nx, p.ny, seed)
    f = orc.init(p, rho, ux, uy)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    # a non-equilibrium part so the collision has something to relax
    return f * (1.0 + 0.05 * rng.uniform(-1, 1, f.shape))


def lattice_tables(orc):
    L = orc.lib()
    cx = np.array((ctypes.c_int * 9).in_dll(L, "ORC_CX")[:])
    cy = np.array((ctypes.c_int * 9).in_dll(L, "ORC_CY")[:])
    w = np.array((ctypes.c_double * 9).in_dll(L, "ORC_W")[:])
    th = ctypes.c_double.in_dll(L, "ORC_THETA").value
    return cx, cy, w, th


# ---------------------------------------------------------------- lattice
def test_d2q9_quadrature_isotropy(orc):
    """Lattice of Sec. II.A (here D2Q9): weights must integrate the Gaussian
    weight's moments up to fourth order.  Catches a wrong weight or velocity."""
    cx, cy, w, th = lattice_tables(orc)
    assert abs(th - 1.0 / 3.0) < 1e-16
    assert abs(w.sum() - 1) < 1e-15
    assert abs((w * cx).sum()) < 1e-15 and abs((w * cy).sum()) < 1e-15
    assert abs((w * cx * cx).sum() - th) < 1e-15
    assert abs((w * cy * cy).sum() - th) < 1e-15
    assert abs((w * cx * cy).sum()) < 1e-15
    assert abs((w * cx ** 4).sum() - 3 * th ** 2) < 1e-15
    assert abs((w * cx ** 2 * cy ** 2).sum() - th ** 2) < 1e-15
    assert abs((w * cx ** 3).sum()) < 1e-15
    # opposite pairs present
    pairs = {(a, b) for a, b in zip(cx, cy)}
    assert all((-a, -b) in pairs for a, b in pairs)


def test_equilibrium_moments(orc):
    """Eqs. M0-M2 with eq. f2: the equilibrium carries mass rho, momentum
    rho u and momentum flux rho u u + rho theta I.  Catches a dropped u^2 term,
    a wrong 1/theta factor or a sign error."""
    cx, cy, w, th = lattice_tables(orc)
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(50):
        rho = rng.uniform(0.1, 3)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        f = orc.equilibrium(rho, ux, uy)
        assert abs(f.sum() - rho) < 1e-14 * rho
        assert abs((f * cx).sum() - rho * ux) < 1e-15
        assert abs((f * cy).sum() - rho * uy) < 1e-15
        assert abs((f * cx * cx).sum() - (rho * ux * ux + rho * th)) < 1e-14
        assert abs((f * cy * cy).sum() - (rho * uy * uy + rho * th)) < 1e-14
        assert abs((f * cx * cy).sum() - rho * ux * uy) < 1e-15
    # at rest the equilibrium is rho * w
    assert np.allclose(orc.equilibrium(1.3, 0, 0), 1.3 * w, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- collision
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_collision_conserves_mass_and_adds_force(orc, tau):
    """Sec. II.B (exact difference method): the collision keeps mass and adds
    exactly the force F to the momentum, for any tau and any wall fields."""
    nx, ny = 12, 10
    cx, cy, w, th = lattice_tables(orc)
    p = orc.make_params(nx, ny, tau=tau, G=-5.0, G_R=0.7, G_A=0.4, eps=1.3,
                        U_wall=(0.01, -0.02), F_ext=(1e-4, -2e-4))
    walls = walls_random(orc, nx, ny, 3)
    f = random_f(orc, p, 5)
    fp = orc.collide(p, walls, f)
    fr = orc.forces(p, walls, f)
    assert np.abs(fp.sum(-1) - f.sum(-1)).max() < 1e-14
    jx0, jy0 = (f * cx).sum(-1), (f * cy).sum(-1)
    jx1, jy1 = (fp * cx).sum(-1), (fp * cy).sum(-1)
    assert np.abs(jx1 - jx0 - fr["F"][..., 0]).max() < 1e-14
    assert np.abs(jy1 - jy0 - fr["F"][..., 1]).max() < 1e-14


def test_tau_one_edm_equals_shifted_equilibrium(orc):
    """At tau = 1 the EDM collision returns f^eq(rho, u*) (Sec. II.B)."""
    nx, ny = 8, 6
    p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=0.3)
    walls = walls_random(orc, nx, ny, 7)
    f = random_f(orc, p, 9)
    fp = orc.collide(p, walls, f)
    fr = orc.forces(p, walls, f)
    for y in range(ny):
        for x in range(nx):
            feq = orc.equilibrium(fr["rho"][y, x], fr["usx"][y, x], fr["usy"][y, x])
            assert np.abs(fp[y, x] - feq).max() < 1e-15


def test_rest_state_is_fixed_point(orc):
    """A uniform fluid at rest with no solid feels no force (sum_i w_i c_i = 0)
    and is an exact fixed point of the whole step."""
    p = orc.make_params(16, 8, tau=0.9, G=-5.0)
    walls = orc.Walls.none(16, 8)
    f = orc.init(p, I.uniform_field(16, 8, 0.7))
    g = orc.run(p, walls, f, 5)
    assert np.abs(g - f).max() < 1e-15


def test_periodic_conservation(orc):
    """Periodic, no solid, no external force: the fluid-fluid force sums to zero
    by the i <-> -i antisymmetry, so total mass and momentum are conserved."""
    nx, ny = 24, 20
    cx, cy, w, th = lattice_tables(orc)
    p = orc.make_params(nx, ny, tau=0.8, G=-5.0)
    walls = orc.Walls.none(nx, ny)
    f0 = random_f(orc, p, 11)
    f = orc.run(p, walls, f0, 300)
    m0, m1 = f0.sum(), f.sum()
    assert abs(m1 - m0) < 1e-12 * m0
    for c in (cx, cy):
        assert abs((f * c).sum() - (f0 * c).sum()) < 1e-11


def test_external_force_momentum_budget(orc):
    """Without solid, total momentum grows by N * F_ext per step (F_ext enters
    the force sum once per node, Sec. III.A body force)."""
    nx, ny = 10, 12
    cx, cy, w, th = lattice_tables(orc)
    F = (3e-5, -1e-5)
    p = orc.make_params(nx, ny, tau=1.2, G=-4.0, F_ext=F)
    walls = orc.Walls.none(nx, ny)
    f0 = random_f(orc, p, 13)
    f = orc.run(p, walls, f0, 40)
    for c, Fc in zip((cx, cy), F):
        assert abs((f * c).sum() - (f0 * c).sum() - 40 * nx * ny * Fc) < 1e-12


@pytest.mark.parametrize("lattice,tau", [(9, 1.0), (9, 0.7), (21, 1.0), (21, 0.8)])
def test_reported_velocity_uniform_acceleration(orc, lattice, tau):
    """Reported velocity of the exact difference method (Sec. II.B: u* = u +
    g dt, the velocity over a step being the average of the pre- and
    post-force velocities).  A uniform fluid (G = 0, no solid, periodic) from
    u0 under a uniform force density F gains F per step at every node, so
    after t steps the momentum is rho u0 + t F and the reported velocity must
    be u0 + F (t + 1/2) / rho exactly.  Reporting j / rho would give
    u0 + F t / rho and (j + F) / rho would give u0 + F (t + 1) / rho, both
    off by F / (2 rho) = 1.9e-5 here, far above the 1e-12 bar."""
    nx, ny, rho0, u0 = 6, 5, 1.37, (2e-3, -1e-3)
    F = (5.2e-5, -3.1e-5)
    p = orc.make_params(nx, ny, tau=tau, G=0.0, F_ext=F, lattice=lattice)
    walls = orc.Walls.none(nx, ny)
    f = orc.init(p, np.full((ny, nx), rho0), np.full((ny, nx), u0[0]), np.full((ny, nx), u0[1]))
    t = 0
    for t_next in (0, 1, 7, 40):
        f = orc.run(p, walls, f, t_next - t)
        t = t_next
        rho, ux, uy, _ = orc.macros(p, walls, f)
        assert np.abs(rho - rho0).max() < 1e-13
        assert np.abs(ux - (u0[0] + F[0] * (t + 0.5) / rho0)).max() < 1e-12, t
        assert np.abs(uy - (u0[1] + F[1] * (t + 0.5) / rho0)).max() < 1e-12, t


def test_reported_velocity_vanishes_at_rest(orc):
    """At a converged flat interface (periodic liquid slab, G = -5, no solid)
    nothing flows: the reported velocity (j + F/2)/rho (Sec. II.B) must
    vanish to well below the force scale, while the pre-force velocity j/rho
    and the post-force one (j + F)/rho are -F/(2 rho) and +F/(2 rho) there
    (|F| reaches 0.2 at the interface).  Pins the half-force convention on a
    state with a strongly non-uniform force."""
    nx, ny = 4, 128
    p = orc.make_params(nx, ny, tau=1.0, G=-5.0)
    walls = orc.Walls.none(nx, ny)
    f = orc.run(p, walls, orc.init(p, I.slab_field(nx, ny)), 10000)
    d = orc.forces(p, walls, f)
    rho, ux, uy, _ = orc.macros(p, walls, f)
    half = (np.abs(d["F"][..., 1]) / (2 * d["rho"])).max()
    assert half > 0.05
    assert np.abs(uy).max() < 1e-2 * half and np.abs(ux).max() < 1e-12
    # the pre- and post-force velocities are half a force step away
    assert np.abs(d["uy"] + 0.5 * d["F"][..., 1] / d["rho"] - uy).max() < 1e-14
    assert np.abs(d["uy"]).max() > 0.9 * half


def test_mass_conserved_with_walls(orc):
    """Wall forces exchange momentum but never mass."""
    nx, ny = 20, 24
    p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.8, G_A=0.4, eps=1.3,
                        F_ext=(1e-5, 0))
    walls = orc.Walls.flat_slab(nx, ny, 8)
    f0 = orc.init(p, I.drop_field(nx, ny, 6.0))
    f = orc.run(p, walls, f0, 200)
    assert abs(f.sum() - f0.sum()) < 1e-12 * f0.sum()


def test_center_of_mass_moves_with_momentum(orc):
    """Streaming direction (Sec. II.A): after one step the mass centre moves by
    exactly the post-collision momentum over the mass.  A reversed stream
    would move it backwards."""
    nx, ny = 40, 40
    cx, cy, w, th = lattice_tables(orc)
    p = orc.make_params(nx, ny, tau=1.0, G=0.0)
    walls = orc.Walls.none(nx, ny)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    bump = np.exp(-((x - 20) ** 2 + (y - 20) ** 2) / 8.0)
    rho = 1.0 + 0.5 * bump
    # moving bump in a resting, uniform background: nothing crosses the
    # periodic seam except rest-equilibrium populations, which cancel there
    f = orc.init(p, rho, 0.05 * bump, -0.03 * bump)
    g = orc.step(p, walls, f)
    M = f.sum()
    X0 = ((f.sum(-1)) * x).sum() / M
    Y0 = ((f.sum(-1)) * y).sum() / M
    X1 = ((g.sum(-1)) * x).sum() / M
    Y1 = ((g.sum(-1)) * y).sum() / M
    fp = orc.collide(p, walls, f)
    assert abs((X1 - X0) - (fp * cx).sum() / M) < 1e-12
    assert abs((Y1 - Y0) - (fp * cy).sum() / M) < 1e-12
    assert X1 - X0 > 5e-4 and Y1 - Y0 < -3e-4


def test_mirror_symmetry(orc):
    """An x-mirror-symmetric drop on the wall stays symmetric: catches any
    x-bias (wrong index, asymmetric stencil)."""
    nx, ny = 48, 32
    p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=0.3)
    walls = orc.Walls.flat_slab(nx, ny, 8)
    f = orc.run(p, walls, orc.init(p, I.drop_field(nx, ny, 10.0)), 400)
    rho, ux, uy, _ = orc.macros(p, walls, f)
    mirror = (-np.arange(nx)) % nx
    assert np.abs(rho - rho[:, mirror]).max() < 1e-12
    assert np.abs(ux + ux[:, mirror]).max() < 1e-12
    assert np.abs(uy - uy[:, mirror]).max() < 1e-12


# ---------------------------------------------------------------- closed forms
def test_taylor_green_decay(orc):
    """Ideal-gas BGK (G = 0, no solid): a Taylor-Green vortex decays as
    exp(-2 nu k^2 t) with nu = theta (tau - 1/2) (eq. BE-BGK, tau sets the
    viscosity).  Catches a wrong tau relation, weights or streaming."""
    n, tau, U0 = 64, 0.8, 1e-3
    k = 2 * np.pi / n
    p = orc.make_params(n, n, tau=tau, G=0.0)
    walls = orc.Walls.none(n, n)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    sx = np.sin(k * x) * np.cos(k * y)
    f = orc.init(p, np.ones((n, n)), U0 * sx, -U0 * np.cos(k * x) * np.sin(k * y))
    T = 400
    f = orc.run(p, walls, f, T)
    _, ux, _, _ = orc.macros(p, walls, f)
    amp = (ux * sx).sum() / (sx * sx).sum() / U0
    nu = (tau - 0.5) / 3.0
    assert abs(amp / np.exp(-2 * nu * k * k * T) - 1) < 5e-3


@pytest.mark.slow
def test_poiseuille_curvature(orc):
    """Body-force driven channel without wall interaction (G = G_R = G_A = 0,
    walls from phi only; Sec. III.A): in the hydrodynamic region the steady
    profile is a parabola of curvature -F/(rho nu)."""
    nx, ny, P, F = 4, 64, 8, 1e-6
    p = orc.make_params(nx, ny, tau=1.0, G=0.0, G_R=0.0, G_A=0.0, F_ext=(F, 0))
    walls = orc.Walls.flat_slab(nx, ny, P)
    f = orc.run(p, walls, orc.init(p, np.ones((ny, nx))), 30000)
    rho, ux, _, _ = orc.macros(p, walls, f)
    y = np.arange(ny)
    core = walls.phi[:, 0] < 1e-6   # far from both faces
    c = np.polyfit(y[core], ux[core, 0], 2)
    nu = (1.0 - 0.5) / 3.0
    assert abs(2 * c[0] / (-F / (rho[core, 0].mean() * nu)) - 1) < 5e-3
    # no flow inside the solid band (phi -> 1 pins u to U_wall = 0)
    assert abs(ux[ny - P // 2, 0]) < 1e-3 * ux.max()


def shan_chen_coexistence(G):
    """Bulk densities from the mechanical-stability rule of the pseudo-potential
    model: equal pressures and int (p0 - p) psi'/psi^2 drho = 0, with
    p = rho theta + G theta psi^2 / 2 for this lattice (theta = 1/3)."""
    psi = lambda r: 1 - np.exp(-r)
    dpsi = lambda r: np.exp(-r)
    pr = lambda r: r / 3 + G / 6 * psi(r) ** 2

    def eqs(v):
        g, l = v
        p0 = pr(g)
        return [pr(l) - p0, integrate.quad(lambda r: (p0 - pr(r)) * dpsi(r) / psi(r) ** 2, g, l)[0]]

    return optimize.fsolve(eqs, [0.15, 1.9], xtol=1e-13)


def test_coexistence_reference_values():
    g, l = shan_chen_coexistence(-5.0)
    assert abs(g - 0.1564) < 1e-4 and abs(l - 1.9324) < 1e-4


@pytest.mark.parametrize("normal", ["y", "x"])
def test_flat_interface_coexistence(orc, normal):
    """A periodic liquid slab (G = -5, no solid) becomes stationary with bulk
    densities at the pseudo-potential coexistence values (within the D2Q9
    stencil's ~1% discreteness).  Run with the slab normal along y and along x
    to catch a transposed force component."""
    g, l = shan_chen_coexistence(-5.0)
    n, m = 128, 4
    if normal == "y":
        nx, ny = m, n
        rho0 = I.slab_field(nx, ny)
    else:
        nx, ny = n, m
        rho0 = np.ascontiguousarray(I.slab_field(ny, nx).T)
    p = orc.make_params(nx, ny, tau=1.0, G=-5.0)
    walls = orc.Walls.none(nx, ny)
    f = orc.run(p, walls, orc.init(p, rho0), 10000)
    rho, ux, uy, _ = orc.macros(p, walls, f)
    assert abs(rho.min() / g - 1) < 0.015
    assert abs(rho.max() / l - 1) < 0.005
    assert max(np.abs(ux).max(), np.abs(uy).max()) < 1e-3


@pytest.mark.slow
def test_laplace_law(orc):
    """Free discs in a periodic box: the pressure jump, with the bulk pressure
    p = rho/3 + (G/6) psi^2, is linear in 1/R with a small intercept and a
    positive slope (the surface tension)."""
    G, n = -5.0, 64
    psi = lambda r: 1 - np.exp(-r)
    pr = lambda r: r / 3 + G / 6 * psi(r) ** 2
    inv_r, dp = [], []
    for R in (8, 10, 12, 14):
        p = orc.make_params(n, n, tau=1.0, G=G)
        walls = orc.Walls.none(n, n)
        f = orc.run(p, walls, orc.init(p, I.disc_field(n, n, R)), 3000)
        rho, _, _, _ = orc.macros(p, walls, f)
        rl, rg = rho[n // 2, n // 2], rho[0, 0]
        Req = np.sqrt((rho.sum() - rg * n * n) / (rl - rg) / np.pi)
        inv_r.append(1 / Req)
        dp.append(pr(rl) - pr(rg))
    inv_r, dp = np.array(inv_r), np.array(dp)
    slope, icpt = np.polyfit(inv_r, dp, 1)
    fit = slope * inv_r + icpt
    assert slope > 0
    assert np.abs(fit - dp).max() < 0.02 * dp.min()
    assert abs(icpt) < 0.1 * dp.min()


# ---------------------------------------------------------------- wall model
def test_wall_functions_flat_slab(orc):
    """Appendix A conditions on the wall functions: phi = 1/2 on both faces,
    -> 1 deep in the solid, -> 0 in the fluid bulk; region III (phi < 0.01)
    starts 5 nodes from a face; psi_A vanishes on the face."""
    nx, ny, P = 4, 40, 8
    w = orc.Walls.flat_slab(nx, ny, P)
    phi = w.phi[:, 0]
    assert abs(phi[0] - 0.5) < 1e-15 and abs(phi[ny - P] - 0.5) < 1e-15
    assert phi[ny - P // 2] > 0.98
    assert np.all(np.diff(phi[:(ny - P) // 2 + 1]) < 0)
    assert phi[4] > 0.01 > phi[5]
    assert abs(w.psiA[0, 0]) < 1e-15
    assert np.all(w.psiA[1:(ny - P) // 2, 0] > 0)
    assert np.all(w.psiR[:, 0] >= 0) and np.all(w.psiR[:, 0] <= 1)
    # mirror symmetric about the gap centre and the band centre
    gap = phi[:ny - P + 1]
    assert np.abs(gap - gap[::-1]).max() < 1e-15


def test_solid_bulk_takes_wall_velocity(orc):
    """Eq. wall_shift read with the velocity shift in velocity units: at
    phi = 1 the shifted velocity is U_wall plus only the long-range wall force
    and the external force, u* = U_wall + (F_LR + F_ext)/rho."""
    nx, ny = 10, 8
    p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.6, G_A=0.3, eps=1.3,
                        U_wall=(0.02, -0.01), F_ext=(2e-4, 1e-4))
    rng = np.random.Generator(np.random.PCG64(4))
    phi = np.ones((ny, nx))
    walls = orc.Walls(phi, rng.uniform(0, 1, (ny, nx)), rng.uniform(0, 0.4, (ny, nx)))
    f = random_f(orc, p, 21)
    fr = orc.forces(p, walls, f)
    ex = 0.02 + (fr["Flr"][..., 0] + 2e-4) / fr["rho"]
    ey = -0.01 + (fr["Flr"][..., 1] + 1e-4) / fr["rho"]
    assert np.abs(fr["usx"] - ex).max() < 1e-14
    assert np.abs(fr["usy"] - ey).max() < 1e-14
    # and phi = 0 leaves the fluid alone: no short-range exchange
    walls0 = orc.Walls(np.zeros((ny, nx)), walls.psiR, walls.psiA)
    assert np.abs(orc.forces(p, walls0, f)["dFs"]).max() == 0.0


@pytest.mark.slow
def test_trend_adsorption_falls_with_core(orc):
    """Sec. III (region I): the vapour adsorbed inside the solid decreases as
    the repulsive amplitude G_R rises.  Fixes the sign of the core force."""
    nx, ny, P = 4, 48, 8
    band = []
    for GR in (0.2, 0.6, 1.0):
        p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=GR, G_A=0.0)
        walls = orc.Walls.flat_slab(nx, ny, P)
        f = orc.run(p, walls, orc.init(p, I.uniform_field(nx, ny, 1.93)), 4000)
        rho, _, _, _ = orc.macros(p, walls, f)
        band.append(rho[ny - P // 2, 0])
    assert band[0] > band[1] > band[2]
    assert band[2] < 0.1


@pytest.mark.slow
def test_trend_angle_falls_with_tail(orc):
    """Sec. III.B (Fig. 8): at fixed G_R the contact angle decreases as the
    attractive amplitude G_A rises.  Fixes the sign of the tail force."""
    nx, ny = 128, 48
    ang = []
    for GA in (0.0, 0.3, 0.6):
        p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=GA)
        walls = orc.Walls.flat_slab(nx, ny, 8)
        f = orc.run(p, walls, orc.init(p, I.drop_field(nx, ny, 20.0)), 3000)
        out = orc.contact_angle(p, walls, f, 1.07, 0.0)
        assert out is not None
        ang.append(out[0])
    assert ang[0] > 120 and ang[0] > ang[1] > ang[2]


@pytest.mark.slow
def test_trend_slip_grows_with_eps(orc):
    """Sec. III.A: a 'smooth' wall (eps = 1.3) slips more than a 'rough' one
    (eps = 1.0) at the same G_R, G_A.  Fixes how eps enters eq. wall_shift."""
    nx, ny, P = 4, 64, 8
    b = []
    for eps in (1.0, 1.3):
        p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=0.3, eps=eps,
                            F_ext=(1e-6, 0))
        walls = orc.Walls.flat_slab(nx, ny, P)
        f = orc.run(p, walls, orc.init(p, I.uniform_field(nx, ny, 1.93)), 20000)
        out = orc.slip_length(p, walls, f, P, 2.0)
        b.append(out[0])
    assert b[1] > 1.3 * b[0] > 0


# ---------------------------------------------------------------- diagnostics
def test_circle_fit_exact_arc(orc):
    """A least-squares circle through points on an exact arc returns it."""
    t = np.linspace(0.3, 2.6, 40)
    xc, yc, R = 31.3, -7.2, 17.5
    out = orc.circle_fit(xc + R * np.cos(t), yc + R * np.sin(t))
    assert np.allclose(out, [xc, yc, R], atol=1e-9)
    assert orc.circle_fit(np.arange(10.0), np.zeros(10)) is None  # collinear


def test_circle_fit_noisy_is_geometric(orc):
    """Gauss-Newton refinement: on noisy points the result is a stationary
    point of the geometric residual sum (gradient ~ 0)."""
    rng = np.random.Generator(np.random.PCG64(2))
    t = np.linspace(0.2, 2.9, 60)
    px = 10 + 5 * np.cos(t) + rng.normal(0, 0.05, t.size)
    py = 3 + 5 * np.sin(t) + rng.normal(0, 0.05, t.size)
    xc, yc, R = orc.circle_fit(px, py)
    d = np.hypot(px - xc, py - yc)
    r = d - R
    grad = [np.sum(r * -(px - xc) / d), np.sum(r * -(py - yc) / d), -np.sum(r)]
    assert np.abs(grad).max() < 1e-10


def test_isoline_points_linear_profile(orc):
    """Crossings of a density that is linear along x fall exactly where the
    linear interpolation puts them; region filtering drops rows with phi >= cut."""
    nx, ny = 8, 6
    x = np.arange(nx, dtype=float)
    rho = np.tile(0.1 + 0.3 * x, (ny, 1))        # crosses 1.07 between x=3 and 4
    phi = np.zeros((ny, nx)); phi[0] = 0.5
    px, py = orc.isoline_points(rho, phi, 1.07, 0.01)
    # wrap edge nx-1 -> 0 also crosses (2.2 -> 0.1)
    xs = sorted(set(np.round(px, 12)))
    assert np.allclose(xs, [3 + (1.07 - 1.0) / 0.3, 7 + (2.2 - 1.07) / 2.1])
    assert set(py) == {1, 2, 3, 4, 5}


def test_contact_angle_synthetic_drop(orc):
    """Sec. III.B: theta = acos(1 - h/R) with h measured from y_ref.  For a
    tanh disc whose centre sits at height yc, the fit returns R and
    cos(theta) = (y_ref - yc)/R; a centre on y_ref gives 90 degrees."""
    nx, ny, R = 160, 80, 30.0
    for yc, y_ref in ((0.0, 0.0), (-10.0, 0.0), (12.0, 0.0), (0.0, 6.0)):
        y, x = np.mgrid[0:ny, 0:nx].astype(float)
        rho = 0.15 + 1.85 * 0.5 * (1 - np.tanh((np.hypot(x - 80, y - yc) - R) / 2))
        p = orc.make_params(nx, ny, tau=1.0, G=0.0)
        walls = orc.Walls.flat_slab(nx, ny, 8)
        f = orc.init(p, rho)
        out = orc.contact_angle(p, walls, f, 1.07, y_ref)
        assert out is not None
        assert abs(out[1] - R) < 0.1
        expect = np.degrees(np.arccos(np.clip((y_ref - yc) / R, -1, 1)))
        assert abs(out[0] - expect) < 0.3
    # a flat film has no circle: not enough curvature -> degenerate or no points
    p = orc.make_params(nx, ny, tau=1.0, G=0.0)
    walls = orc.Walls.flat_slab(nx, ny, 8)
    assert orc.contact_angle(p, walls, orc.init(p, np.full((ny, nx), 0.15)), 1.07, 0) is None


def test_slip_fit_parabola(orc):
    """Slip measurement of Sec. III.A on a synthetic parabolic profile: the fit
    recovers the parabola's value and slope at y_w (phi(y_w) = 0.01)."""
    nx, ny, P = 4, 48, 8
    top = ny - P
    a, U = 0.5 * top, 1e-3
    y = np.arange(ny, dtype=float)
    prof = U * (1 - ((y - a) / a) ** 2) + 2e-4
    ux = np.tile(prof[:, None], (1, nx))
    # a large eps makes the short-range exchange vanish in region III, so the
    # reported velocity there is the imposed one
    p = orc.make_params(nx, ny, tau=1.0, G=0.0, eps=20.0)
    walls = orc.Walls.flat_slab(nx, ny, P)
    f = orc.init(p, np.ones((ny, nx)), ux, np.zeros((ny, nx)))
    b, us, c2 = orc.slip_length(p, walls, f, P, 2.0)
    yw = 2.0 * np.arctanh(0.98)
    u_w = U * (1 - ((yw - a) / a) ** 2) + 2e-4
    g_w = abs(-2 * U * (yw - a) / a ** 2)
    assert abs(us - u_w) < 1e-15 + 1e-12 * U
    assert abs(b - u_w / g_w) < 1e-9
    assert abs(c2 + 2 * U / a ** 2) < 1e-15 + 1e-12 * U


def test_residual(orc):
    a = np.array([1.0, -2.0]); b = np.array([0.5, 0.5])
    assert orc.residual(a, b, a, b) == 0.0
    assert abs(orc.residual(a, b, a + 0.1, b) - 0.2 / 4.0) < 1e-15


# ---------------------------------------------------------------- brute force
def brute_force_step(nx, ny, tau, G, GR, GA, eps, U, Fext, phi, psiR, psiA, f):
    """Independent dense formulation of one step on a tiny lattice: streaming
    and the neighbour sums as explicit index matrices, the equilibrium as the
    second-order Hermite expansion written with Hermite tensors."""
    N = nx * ny
    c = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    w = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1]) / 36.0
    th = 1.0 / 3.0
    nb = np.zeros((9, N, N))            # nb[i] @ v = v(x + c_i)
    for yy in range(ny):
        for xx in range(nx):
            for i in range(9):
                nb[i, yy * nx + xx, ((yy + c[i, 1]) % ny) * nx + (xx + c[i, 0]) % nx] = 1
    F_ = f.reshape(N, 9)
    rho = F_.sum(1)
    j = F_ @ c
    u = j / rho[:, None]
    psi = 1 - np.exp(-rho)
    fs = GA * psiA.ravel() - GR * psiR.ravel()
    grad_psi = sum(w[i] * np.outer(nb[i] @ psi, c[i]) for i in range(9))
    grad_fs = sum(w[i] * np.outer(nb[i] @ fs, c[i]) for i in range(9))
    Fff = -G * psi[:, None] * grad_psi
    Flr = rho[:, None] * grad_fs
    pe = phi.ravel() ** eps
    dFs = pe[:, None] * (rho[:, None] * (np.asarray(U)[None, :] - u) - Fff)
    Ftot = Fff + Flr + dFs + np.asarray(Fext)[None, :]
    us = u + Ftot / rho[:, None]
    H2 = np.einsum("ia,ib->iab", c, c) - th * np.eye(2)[None]

    def feq(r, v):
        a2 = r[:, None, None] * np.einsum("na,nb->nab", v, v)
        return w[None, :] * (r[:, None] + (r[:, None] * v) @ c.T / th
                             + np.einsum("nab,iab->ni", a2, H2) / (2 * th * th))

    fe_u, fe_s = feq(rho, u), feq(rho, us)
    post = F_ - (F_ - fe_u) / tau + fe_s - fe_u
    out = np.zeros_like(post)
    for i in range(9):
        out[:, i] = nb[i].T @ post[:, i]   # value at x lands on x + c_i
    return out.reshape(ny, nx, 9)


def test_brute_force_4x4(orc):
    nx, ny = 4, 4
    args = dict(tau=0.85, G=-5.0, G_R=0.6, G_A=0.35, eps=1.3,
                U_wall=(0.01, 0.02), F_ext=(1e-3, -2e-3))
    p = orc.make_params(nx, ny, **args)
    walls = walls_random(orc, nx, ny, 17)
    walls.psiA = np.ascontiguousarray(np.abs(walls.psiA))
    f = random_f(orc, p, 19)
    g = orc.step(p, walls, f)
    h = brute_force_step(nx, ny, 0.85, -5.0, 0.6, 0.35, 1.3, (0.01, 0.02), (1e-3, -2e-3),
                         walls.phi, walls.psiR, walls.psiA, f)
    assert np.abs(g - h).max() < 1e-14


def test_parallel_build_is_bitwise_serial(orc, tmp_path):
    """The OpenMP build of the oracle (long reference runs) gives bitwise the
    serial build's result."""
    import subprocess
    import sys
    nx, ny = 40, 24
    p = orc.make_params(nx, ny, tau=0.9, G=-5.0, G_R=0.5, G_A=0.3, eps=1.3, F_ext=(1e-4, 0.0))
    w = orc.Walls.flat_slab(nx, ny, 6)
    f = orc.run(p, w, orc.init(p, I.drop_field(nx, ny, 8.0)), 30)
    out = tmp_path / "f_omp.npy"
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r)\n"
        "import oracle as O; O.use_threads(3)\n"
        "from paper_1202_6130_amd import inputs as I\n"
        "p = O.make_params(40, 24, tau=0.9, G=-5.0, G_R=0.5, G_A=0.3, eps=1.3, F_ext=(1e-4, 0.0))\n"
        "w = O.Walls.flat_slab(40, 24, 6)\n"
        "np.save(%r, O.run(p, w, O.init(p, I.drop_field(40, 24, 8.0)), 30))\n"
    ) % (ROOT, str(out))
    subprocess.check_call([sys.executable, "-c", code])
    assert np.array_equal(np.load(out), f)
