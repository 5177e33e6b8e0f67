"""Seeded synthetic inputs shared by the HIP path, its tests and the benchmark.

This module holds no arithmetic of the lattice-Boltzmann method itself: it only
builds initial density fields, draws parameters and generates request streams.
Every field is float64 and row-major [ny, nx] (index y*nx + x).  Random draws use
numpy's PCG64 generator with an explicit seed.

Workload shapes follow the paper's cases: a sessile drop on a flat wall
(Sec. III.B), a pressure-driven channel (Sec. III.A), plus a periodic
phase-separation lattice, a batched ensemble and a served request stream.
"""
import dataclasses

import numpy as np

RHO_L = 2.0      # liquid density of the initial drop
RHO_G = 0.15     # gas density of the initial drop
ISO = 1.07       # density isoline used for the contact-angle fit
SLAB_ROWS = 8    # rows of the solid band at the top of the periodic domain


def _step_profile(s, width):
    # smooth step, 1 for s << 0 and 0 for s >> 0
    return 0.5 * (1.0 - np.tanh(s / width))


def drop_field(nx, ny, radius, rho_l=RHO_L, rho_g=RHO_G, width=2.0,
               slab_rows=SLAB_ROWS, xc=None):
    """Half-disc drop of the given radius centred on the lower wall face (row 0).

    Rows 0..ny-slab_rows carry rho_g + (rho_l - rho_g) * step(r - radius); the
    rows of the solid band above start at rho_g.
    """
    xc = nx / 2.0 if xc is None else xc
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - xc) ** 2 + y ** 2)
    rho = rho_g + (rho_l - rho_g) * _step_profile(r - radius, width)
    if slab_rows > 0:
        rho[ny - slab_rows + 1:, :] = rho_g
    return np.ascontiguousarray(rho)


def uniform_field(nx, ny, rho):
    return np.full((ny, nx), float(rho))


def slab_field(nx, ny, rho_l=RHO_L, rho_g=RHO_G, width=2.0):
    """Periodic liquid slab occupying the middle half of the rows."""
    y = np.arange(ny, dtype=np.float64)[:, None]
    d = np.abs(y - (ny - 1) / 2.0) - ny / 4.0
    rho = rho_g + (rho_l - rho_g) * _step_profile(d, width)
    return np.ascontiguousarray(np.broadcast_to(rho, (ny, nx)))


def disc_field(nx, ny, radius, rho_l=RHO_L, rho_g=RHO_G, width=2.0):
    """Free disc centred in a periodic box."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - (nx - 1) / 2.0) ** 2 + (y - (ny - 1) / 2.0) ** 2)
    return np.ascontiguousarray(rho_g + (rho_l - rho_g) * _step_profile(r - radius, width))


def spinodal_field(n, seed=0, sigma=4.0, rho_l=RHO_L, rho_g=RHO_G, ny=None):
    """Periodic n x ny lattice, exactly half liquid.

    White N(0,1) noise is smoothed with a periodic Gaussian of std sigma nodes
    (FFT) and the upper half of its values (by rank) becomes liquid.
    """
    ny = n if ny is None else ny
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((ny, n))
    ky = 2 * np.pi * np.fft.fftfreq(ny)[:, None]
    kx = 2 * np.pi * np.fft.rfftfreq(n)[None, :]
    smooth = np.fft.irfft2(np.fft.rfft2(noise) * np.exp(-0.5 * sigma ** 2 * (kx ** 2 + ky ** 2)),
                           s=(ny, n))
    order = np.argsort(smooth, axis=None, kind="stable")
    liquid = np.zeros(ny * n, dtype=bool)
    liquid[order[(ny * n) // 2:]] = True
    return np.ascontiguousarray(np.where(liquid.reshape(ny, n), rho_l, rho_g))


def random_state_field(nx, ny, seed=0, lo=0.2, hi=1.8, umax=0.05):
    """Random (rho, ux, uy) for parity tests of a single step."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rng.uniform(lo, hi, (ny, nx))
    ux = rng.uniform(-umax, umax, (ny, nx))
    uy = rng.uniform(-umax, umax, (ny, nx))
    return rho, ux, uy


def draw_wall_amplitudes(seed, n=1):
    """(G_R, G_A) pairs: core amplitude ~ U[0,1], tail amplitude ~ U[0,0.6]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gr = rng.uniform(0.0, 1.0, n)
    ga = rng.uniform(0.0, 0.6, n)
    return gr, ga


@dataclasses.dataclass
class DropCase:
    nx: int
    ny: int
    radius: float
    G: float
    G_R: float
    G_A: float


def ensemble_cases(seed=0, count=256):
    """Sessile drops of uneven size: nx in {128..1024}, ny in {64..512}
    (multiples of 32), radius 0.3*min(nx, ny), G ~ U[-5.5, -4.5], wall
    amplitudes as in draw_wall_amplitudes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nxs = rng.integers(128 // 32, 1024 // 32 + 1, count) * 32
    nys = rng.integers(64 // 32, 512 // 32 + 1, count) * 32
    G = rng.uniform(-5.5, -4.5, count)
    gr = rng.uniform(0.0, 1.0, count)
    ga = rng.uniform(0.0, 0.6, count)
    return [DropCase(int(a), int(b), 0.3 * min(int(a), int(b)), float(g), float(r), float(t))
            for a, b, g, r, t in zip(nxs, nys, G, gr, ga)]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    kind: str               # "angle" or "slip"
    nx: int
    ny: int
    G: float
    G_R: float
    G_A: float
    eps: float


def request_stream(seed=0, rate=20.0, count=300, nx_range=(128, 2048),
                   ny_range=(128, 1024)):
    """Poisson arrivals at `rate` per second; sizes uniform over multiples of 32;
    half contact-angle queries (sessile drop), half slip queries (channel)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    nxs = rng.integers(nx_range[0] // 32, nx_range[1] // 32 + 1, count) * 32
    nys = rng.integers(ny_range[0] // 32, ny_range[1] // 32 + 1, count) * 32
    G = rng.uniform(-5.5, -4.5, count)
    gr = rng.uniform(0.0, 1.0, count)
    ga = rng.uniform(0.0, 0.6, count)
    kinds = np.where(rng.uniform(size=count) < 0.5, "angle", "slip")
    eps = np.where(rng.uniform(size=count) < 0.5, 1.0, 1.3)
    return [Request(i, float(t[i]), str(kinds[i]), int(nxs[i]), int(nys[i]), float(G[i]),
                    float(gr[i]), float(ga[i]), float(eps[i])) for i in range(count)]
