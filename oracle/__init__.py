"""ctypes front-end of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain C implementation of the wetting-model lattice-Boltzmann
update of arXiv:1202.6130 (Sec. II; Appendix A for the wall functions).  Only
the test-suite, the smoke check and the benchmark's CPU-baseline leg may use
it; the HIP library never does.  Arrays are numpy float64, populations in the
oracle's node-major layout f[y, x, i] (post-streaming state).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")
LIB_OMP_PATH = os.path.join(HERE, "liblbm_oracle_omp.so")

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("tau", ctypes.c_double), ("G", ctypes.c_double),
                ("G_R", ctypes.c_double), ("G_A", ctypes.c_double),
                ("eps", ctypes.c_double),
                ("U_wall", ctypes.c_double * 2), ("F_ext", ctypes.c_double * 2),
                ("lattice", ctypes.c_int), ("psi_kind", ctypes.c_int),
                ("eos", ctypes.c_double * 5), ("collision", ctypes.c_int)]


# eq. EOS parameters of the paper: theta_V/theta, theta_U/theta, theta_L/theta,
# rho_1, rho_2 (Sec. II.B)
EOS_PAPER = (0.25, -0.25, 1.0, 0.222, 0.869)


_lib = None
_path = LIB_PATH


def use_threads(n):
    """Switch to the OpenMP build of the same source with n threads (long
    reference runs; bitwise the same results).  Call before the first use."""
    global _lib, _path
    if _lib is not None:
        raise RuntimeError("use_threads must be called before the oracle is loaded")
    os.environ["OMP_NUM_THREADS"] = str(int(n))
    _path = LIB_OMP_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_path):
            from . import build as _b
            _b.build(parallel=_path == LIB_OMP_PATH)
        L = ctypes.CDLL(_path)
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(Params)
        L.orc_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_equilibrium_q.argtypes = [ctypes.c_int] + [ctypes.c_double] * 3 + [dp]
        L.orc_project_q.argtypes = [ctypes.c_int, dp, dp]
        L.orc_filter_walls.argtypes = [ctypes.c_int] * 3 + [dp, dp] + [ctypes.c_int] * 2 + [dp] * 3
        L.orc_psi.argtypes = [P, ctypes.c_double]
        L.orc_psi.restype = ctypes.c_double
        L.orc_p_eos.argtypes = [P, ctypes.c_double]
        L.orc_p_eos.restype = ctypes.c_double
        L.orc_stream_q.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_flat_slab_walls.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, dp, dp, dp]
        L.orc_init.argtypes = [P, dp, dp, dp, dp]
        L.orc_forces.argtypes = [P, dp, dp, dp, dp] + [dp] * 9
        L.orc_collide.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_stream.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_step.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_run.argtypes = [P, dp, dp, dp, dp, ctypes.c_long]
        L.orc_run.restype = ctypes.c_int
        L.orc_macros.argtypes = [P, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_isoline_points.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp,
                                         ctypes.c_double, ctypes.c_double, dp, dp,
                                         ctypes.c_long]
        L.orc_isoline_points.restype = ctypes.c_long
        L.orc_circle_fit.argtypes = [ctypes.c_long, dp, dp, dp]
        L.orc_circle_fit.restype = ctypes.c_int
        L.orc_contact_angle.argtypes = [P, dp, dp, dp, dp, ctypes.c_double,
                                        ctypes.c_double, dp]
        L.orc_contact_angle.restype = ctypes.c_int
        L.orc_dynamic_angles.argtypes = [P, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_dynamic_angles.restype = ctypes.c_int
        L.orc_slip_length.argtypes = [P, dp, dp, dp, dp, ctypes.c_int,
                                      ctypes.c_double, dp]
        L.orc_slip_length.restype = ctypes.c_int
        L.orc_residual.argtypes = [ctypes.c_long, dp, dp, dp, dp]
        L.orc_residual.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.0, G_A=0.0, eps=1.0,
                U_wall=(0.0, 0.0), F_ext=(0.0, 0.0), lattice=9, psi_kind=0, eos=EOS_PAPER, collision=0):
    p = Params()
    p.nx, p.ny = int(nx), int(ny)
    p.tau, p.G, p.G_R, p.G_A, p.eps = tau, G, G_R, G_A, eps
    p.U_wall[0], p.U_wall[1] = U_wall
    p.F_ext[0], p.F_ext[1] = F_ext
    p.lattice, p.psi_kind = int(lattice), int(psi_kind)
    p.collision = int(collision)
    for k, v in enumerate(eos):
        p.eos[k] = v
    return p


def nq(p):
    """Populations per node of the parameters' lattice."""
    return 21 if p.lattice == 21 else 9


def lattice_tables(lattice=9):
    """(cx, cy, w, theta) of the oracle's velocity set."""
    L = lib()
    q = 21 if lattice == 21 else 9
    pre = "ORC21_" if q == 21 else "ORC_"
    cx = np.array((ctypes.c_int * q).in_dll(L, pre + "CX")[:])
    cy = np.array((ctypes.c_int * q).in_dll(L, pre + "CY")[:])
    w = np.array((ctypes.c_double * q).in_dll(L, pre + "W")[:])
    th = ctypes.c_double.in_dll(L, pre + "THETA").value
    return cx, cy, w, th


def psi(p, rho):
    return lib().orc_psi(ctypes.byref(p), float(rho))


def p_eos(p, rho):
    return lib().orc_p_eos(ctypes.byref(p), float(rho))


class Walls:
    """Per-node wall functions (phi_S, psi_R bar, psi_A bar), shape [ny, nx]."""

    def __init__(self, phi, psiR, psiA):
        self.phi = np.ascontiguousarray(phi, dtype=np.float64)
        self.psiR = np.ascontiguousarray(psiR, dtype=np.float64)
        self.psiA = np.ascontiguousarray(psiA, dtype=np.float64)

    @staticmethod
    def none(nx, ny):
        z = np.zeros((ny, nx))
        return Walls(z, z.copy(), z.copy())

    @staticmethod
    def filtered(solid, bnd, lattice=9, n_core=5, n_wall=22):
        """Appendix A: recursive filter of the solid indicator (orc_filter_walls)."""
        solid = np.ascontiguousarray(solid, dtype=np.float64)
        bnd = np.ascontiguousarray(bnd, dtype=np.float64)
        ny, nx = solid.shape
        phi = np.zeros((ny, nx)); psiR = np.zeros((ny, nx)); psiA = np.zeros((ny, nx))
        lib().orc_filter_walls(lattice, nx, ny, _p(solid), _p(bnd), n_core, n_wall, _p(phi), _p(psiR), _p(psiA))
        return Walls(phi, psiR, psiA)

    @staticmethod
    def flat_slab(nx, ny, P=8, width=2.0, core=1.0, tail=3.0):
        phi = np.zeros((ny, nx)); psiR = np.zeros((ny, nx)); psiA = np.zeros((ny, nx))
        lib().orc_flat_slab_walls(nx, ny, P, width, core, tail, _p(phi), _p(psiR), _p(psiA))
        return Walls(phi, psiR, psiA)


def project(f, lattice=9):
    """Projection of one node's populations onto eq. f2 (Sec. II.A)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    lib().orc_project_q(lattice, _p(f), _p(out))
    return out


def equilibrium(rho, ux, uy, lattice=9):
    out = np.zeros(21 if lattice == 21 else 9)
    lib().orc_equilibrium_q(lattice, rho, ux, uy, _p(out))
    return out


def init(p, rho0, ux0=None, uy0=None):
    f = np.zeros((p.ny, p.nx, nq(p)))
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
    uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
    lib().orc_init(ctypes.byref(p), _p(rho0), _p(ux0), _p(uy0), _p(f))
    return f


def forces(p, walls, f):
    ny, nx = p.ny, p.nx
    out = {k: np.zeros((ny, nx)) for k in ("rho", "ux", "uy", "usx", "usy")}
    for k in ("Fff", "Flr", "dFs", "F"):
        out[k] = np.zeros((ny, nx, 2))
    lib().orc_forces(ctypes.byref(p), _p(walls.phi), _p(walls.psiR), _p(walls.psiA),
                     _p(f), _p(out["rho"]), _p(out["ux"]), _p(out["uy"]),
                     _p(out["Fff"]), _p(out["Flr"]), _p(out["dFs"]), _p(out["F"]),
                     _p(out["usx"]), _p(out["usy"]))
    return out


def collide(p, walls, f):
    g = np.zeros_like(f)
    lib().orc_collide(ctypes.byref(p), _p(walls.phi), _p(walls.psiR), _p(walls.psiA),
                      _p(f), _p(g))
    return g


def stream(nx, ny, fpost, lattice=9):
    g = np.zeros_like(fpost)
    lib().orc_stream_q(lattice, nx, ny, _p(np.ascontiguousarray(fpost)), _p(g))
    return g


def step(p, walls, f):
    g = np.zeros_like(f)
    lib().orc_step(ctypes.byref(p), _p(walls.phi), _p(walls.psiR), _p(walls.psiA),
                   _p(f), _p(g))
    return g


def run(p, walls, f, nsteps):
    f = np.array(f, dtype=np.float64, copy=True, order="C")
    rc = lib().orc_run(ctypes.byref(p), _p(walls.phi), _p(walls.psiR), _p(walls.psiA),
                       _p(f), int(nsteps))
    if rc != 0:
        raise MemoryError("oracle: cannot allocate scratch lattice")
    return f


def macros(p, walls, f):
    ny, nx = p.ny, p.nx
    rho = np.zeros((ny, nx)); ux = np.zeros((ny, nx)); uy = np.zeros((ny, nx))
    tot = np.zeros(3)
    lib().orc_macros(ctypes.byref(p), _p(walls.phi), _p(walls.psiR), _p(walls.psiA),
                     _p(f), _p(rho), _p(ux), _p(uy), _p(tot))
    return rho, ux, uy, tot


def isoline_points(rho, phi, iso, phi_max=0.01):
    ny, nx = rho.shape
    cap = 2 * nx * ny
    px = np.zeros(cap); py = np.zeros(cap)
    n = lib().orc_isoline_points(nx, ny, _p(np.ascontiguousarray(rho)),
                                 _p(np.ascontiguousarray(phi)), iso, phi_max,
                                 _p(px), _p(py), cap)
    return px[:n].copy(), py[:n].copy()


def circle_fit(px, py):
    out = np.zeros(3)
    rc = lib().orc_circle_fit(len(px), _p(np.ascontiguousarray(px, dtype=np.float64)),
                              _p(np.ascontiguousarray(py, dtype=np.float64)), _p(out))
    return None if rc != 0 else out


def contact_angle(p, walls, f, iso=1.07, y_ref=0.0):
    out = np.zeros(4)
    rc = lib().orc_contact_angle(ctypes.byref(p), _p(walls.phi), _p(walls.psiR),
                                 _p(walls.psiA), _p(f), iso, y_ref, _p(out))
    return None if rc != 0 else out


def dynamic_angles(p, walls, f, iso=1.07, y_ref=0.0):
    out = np.zeros(8)
    rc = lib().orc_dynamic_angles(ctypes.byref(p), _p(walls.phi), _p(walls.psiR),
                                  _p(walls.psiA), _p(f), iso, y_ref, _p(out))
    return None if rc != 0 else out


def slip_length(p, walls, f, P=8, width=2.0):
    out = np.zeros(3)
    rc = lib().orc_slip_length(ctypes.byref(p), _p(walls.phi), _p(walls.psiR),
                               _p(walls.psiA), _p(f), P, width, _p(out))
    return None if rc != 0 else out


def residual(uxa, uya, uxb, uyb):
    a = [np.ascontiguousarray(v, dtype=np.float64).ravel() for v in (uxa, uya, uxb, uyb)]
    return lib().orc_residual(a[0].size, *[_p(v) for v in a])
