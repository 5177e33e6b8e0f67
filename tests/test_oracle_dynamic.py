"""Pins of the oracle's dynamic contact angles (Sec. III.C): two circles fitted
to the rear and front parts of a drop's region-III isoline, joined at the
apex, and the drop's mean speed U.

A synthetic drop is built from two arcs that meet at a common apex: the rear
arc of a circle of radius 30 centred 10.13 below the wall face, the front arc
of a circle of radius 25 centred 5.13 below it, so theta_R = acos(10.13/30)
and theta_A = acos(5.13/25) are known in closed form (centres off the lattice
so that no node lies exactly on the iso level).  Populations are the equilibrium at a
uniform liquid velocity U0 with every force off in the fluid, so U = U0
exactly.
"""
import numpy as np
import pytest

NX, NY, P = 160, 72, 8
RHO_L, RHO_G = 1.9, 0.16
ISO = 0.5 * (RHO_L + RHO_G)


def two_arc_drop(orc, U0, xap=70.37, shift=0, mirror=False):
    y, x = np.mgrid[0:NY, 0:NX].astype(float)
    xs = (x - shift) % NX
    rear = xs <= xap
    yc = np.where(rear, -10.13, -5.13)
    R = np.where(rear, 30.0, 25.0)
    s = np.hypot(xs - xap, y - yc) - R
    rho = RHO_G + (RHO_L - RHO_G) * 0.5 * (1 - np.tanh(s / 2.0))
    rho[NY - P:, :] = RHO_G
    if mirror:                                  # exact lattice mirror x -> NX - 1 - x
        rho = np.ascontiguousarray(rho[:, ::-1])
    ux = np.where(rho >= ISO, U0, 0.0)
    p = orc.make_params(NX, NY, tau=1.0, G=0.0)
    phi = np.zeros((NY, NX))
    phi[NY - P:, :] = 1.0                        # solid band: rows y < 0 by wrap
    walls = orc.Walls(phi, np.zeros_like(phi), np.zeros_like(phi))
    f = orc.init(p, rho, ux, np.zeros_like(ux))
    return p, walls, f, rho


def test_two_arc_drop_recovers_both_circles(orc):
    U0 = 3e-3
    p, w, f, rho = two_arc_drop(orc, U0)
    out = orc.dynamic_angles(p, w, f, ISO, 0.0)
    assert out is not None
    thA, thR, U, RA, RR, xa, ya, rl = out
    assert abs(RA - 25.0) < 0.3 and abs(RR - 30.0) < 0.3
    assert abs(thA - np.degrees(np.arccos(5.13 / 25))) < 1.0
    assert abs(thR - np.degrees(np.arccos(10.13 / 30))) < 1.0
    assert abs(xa - 70.37) < 1.0 and abs(ya - 19.87) < 0.5
    assert abs(U - U0) < 1e-14
    liquid = (w.phi < 0.01) & (rho >= ISO)
    assert abs(rl - rho[liquid].mean()) < 1e-12


def test_direction_swaps_advancing_and_receding(orc):
    p, w, f, _ = two_arc_drop(orc, 3e-3)
    a = orc.dynamic_angles(p, w, f, ISO, 0.0)
    p, w, f, _ = two_arc_drop(orc, -3e-3)
    b = orc.dynamic_angles(p, w, f, ISO, 0.0)
    assert np.abs(b[[0, 1, 3, 4]] - a[[1, 0, 4, 3]]).max() < 1e-9
    assert b[2] == -a[2]


def test_drop_across_the_periodic_boundary(orc):
    """Rolling the lattice along x (the drop then straddles x = 0) changes
    nothing but the apex position."""
    p, w, f, _ = two_arc_drop(orc, 3e-3)
    a = orc.dynamic_angles(p, w, f, ISO, 0.0)
    for shift in (95, 123):
        p, w, f, _ = two_arc_drop(orc, 3e-3, shift=shift)
        b = orc.dynamic_angles(p, w, f, ISO, 0.0)
        assert np.abs(b[[0, 1, 3, 4, 6]] - a[[0, 1, 3, 4, 6]]).max() < 1e-9
        assert abs(((b[5] - a[5] - shift + NX / 2) % NX) - NX / 2) < 1e-9


def test_mirror_image_swaps_the_arcs(orc):
    """The mirrored drop moving the other way has the same advancing and
    receding arcs."""
    p, w, f, _ = two_arc_drop(orc, 3e-3)
    a = orc.dynamic_angles(p, w, f, ISO, 0.0)
    p, w, f, _ = two_arc_drop(orc, -3e-3, mirror=True)
    b = orc.dynamic_angles(p, w, f, ISO, 0.0)
    assert np.abs(b[[0, 1, 3, 4]] - a[[0, 1, 3, 4]]).max() < 1e-9


def test_no_drop_no_fit(orc):
    p = orc.make_params(NX, NY, tau=1.0, G=0.0)
    w = orc.Walls.none(NX, NY)
    f = orc.init(p, np.full((NY, NX), RHO_G))
    assert orc.dynamic_angles(p, w, f, ISO, 0.0) is None
