"""Continuous-batching server for contact-angle and slip-length queries.

Each request is one lattice (sessile drop -> static contact angle, Sec. III.B;
body-force channel -> slip length, Sec. III.A).  Requests are admitted in
arrival order while their device footprint fits the memory budget, a slot is
free and the resident lattice nodes stay under `max_nodes` (enough to fill the
GPU: more resident work only delays every request without raising
throughput); all resident lattices advance together, one kernel launch per time
step (lbm_batch_attach), replayed from a HIP graph in chunks of `diag_every`
steps.  After every chunk the velocity residual of each lattice is read; a
lattice whose residual falls below `tol`, or reaches its binary32 floor
(Floor), or is at rest (its residual stalled at the O(1) level of rounding
noise, every |u| below REST_SPEED), or reaches `max_steps`, is measured and
retired, and its slot and memory go to the next request.  The
batch is rebuilt whenever membership changes; resident lattices keep their
state across rebuilds.  A request whose lattice turns non-finite fails alone.

Tile shapes: at start-up the batch autotuner measures a per-tile step cost
for every tile shape on a small calibration ensemble; each admitted lattice
then gets the shape of least predicted cost (tile count x per-tile cost).
Two steps per launch: on the same calibration ensemble the batch's two-step
autotuner chooses between single steps and the two-step variants, and every
batch (and, in the sequential baseline, every lattice) uses that choice.
Shapes and step variants change speed only, never results.

`Server(batched=False, max_resident=1)` is the plain sequential baseline.
"""
import collections
import dataclasses
import math
import time

import numpy as np

from . import inputs as I
from . import lbm

CHANNEL_FORCE = 1e-6      # body force density of the slip queries
CHANNEL_RHO = 2.0         # liquid filling the channel


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    nx: int
    ny: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    steps: int = 0
    converged: bool = False
    floor: bool = False       # converged at the binary32 floor of the residual, not below tol
    rest: bool = False        # converged at rest: the residual is rounding noise of a fluid at rest
    residual: float = float("inf")
    value: tuple = ()
    error: str = ""

    @property
    def latency(self):
        return self.finished - self.arrival


def tile_count(nx, ny, shape):
    """Workgroups of one step of an nx x ny lattice with this tile shape."""
    w, r, s = lbm.lbm_tile_shapes()[shape]
    return math.ceil(math.ceil(nx / 64) / s) * math.ceil(ny / (w // s * r - 2))


def calibrate_tile_costs(seed=0, count=16, steps=3, device="cuda:0"):
    """Per-tile step time (ms) of every tile shape, from the batch autotuner's
    uniform-shape timings on a calibration ensemble of sessile drops."""
    cases = I.ensemble_cases(seed=seed, count=count)
    ps = [lbm.lbm_params_default(nx=c.nx, ny=c.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=c.G, G_R=c.G_R, G_A=c.G_A)
          for c in cases]
    B = lbm.Batch(ps, [I.drop_field(c.nx, c.ny, c.radius) for c in cases], device=device)
    _, ms = B.tune(steps)
    B.close()
    nshape = len(lbm.lbm_tile_shapes())
    return [float(ms[s]) / sum(tile_count(c.nx, c.ny, s) for c in cases) for s in range(nshape)]


def calibrate_two_step(seed=0, count=16, steps=2, device="cuda:0"):
    """Two-step variant (or -1 for single steps) the batch two-step autotuner
    keeps on the calibration ensemble of calibrate_tile_costs."""
    cases = I.ensemble_cases(seed=seed, count=count)
    ps = [lbm.lbm_params_default(nx=c.nx, ny=c.ny, wall_kind=lbm.WALL_FLAT_SLAB, G=c.G, G_R=c.G_R, G_A=c.G_A)
          for c in cases]
    B = lbm.Batch(ps, [I.drop_field(c.nx, c.ny, c.radius) for c in cases], device=device)
    B.tune(3)
    v, _ = B.tune_two_step(steps)
    B.close()
    return v


def pick_tile_shape(nx, ny, costs):
    return min(range(len(costs)), key=lambda s: tile_count(nx, ny, s) * costs[s])


def lattice_params(req, seg_rows=0):
    """Lattice parameters of one request."""
    common = dict(nx=req.nx, ny=req.ny, storage=lbm.STORE_F32, wall_kind=lbm.WALL_FLAT_SLAB, G=req.G,
                  G_R=req.G_R, G_A=req.G_A, eps=req.eps, seg_rows=seg_rows)
    if req.kind == "angle":
        return lbm.lbm_params_default(**common)
    return lbm.lbm_params_default(F_ext=(CHANNEL_FORCE, 0.0), **common)


def request_params(req, seg_rows=0):
    """Lattice parameters and initial density of one request."""
    if req.kind == "angle":
        rho0 = I.drop_field(req.nx, req.ny, 0.3 * min(req.nx, req.ny))
    else:
        rho0 = I.uniform_field(req.nx, req.ny, CHANNEL_RHO)
    return lattice_params(req, seg_rows), rho0


def initial_velocity(req, p):
    """Initial velocity [2, ny, nx] of a request, or None (at rest).  A slip
    query starts from the no-slip Poiseuille profile between its hydrodynamic
    boundaries (phi = 0.01, Sec. III.A), u_x = F (y - y_w)(H - y_w - y) /
    (2 rho nu), so that the run only has to settle the wall region and the
    slip instead of building the whole profile up from rest (a viscous time
    H^2 / nu of up to 6e6 steps on the largest channels).  The steady state
    does not depend on this choice."""
    if req.kind != "slip":
        return None
    nx, ny, P = p.nx, p.ny, p.slab_rows
    H = ny - P                                       # gap between the two faces
    yw = p.wall_width * math.atanh(0.98)             # phi(y_w) = 0.01
    nu = (p.tau - 0.5) / 3.0
    y = np.arange(ny, dtype=np.float64)
    prof = p.F_ext[0] * (y - yw) * (H - yw - y) / (2.0 * CHANNEL_RHO * nu)
    prof[(y < yw) | (y > H - yw)] = 0.0
    u0 = np.zeros((2, ny, nx))
    u0[0] = prof[:, None]
    return u0


class Floor:
    """Detects that a lattice's residual has stopped falling.

    Storage rounding keeps the residual of a binary32 lattice from falling
    below a floor that depends on the lattice (measured 5e-7 to 4e-5 on served
    drops and channels); a tolerance below it would never be met.  The
    residual has stalled once the median of the last `window` passes is no
    smaller than `ratio` times the median of the `window` passes before (a
    slowly relaxing channel, its residual halving over ~70000 steps, improves
    by more than 10% over 200 passes of 100 steps).  Below `ceiling` a stalled
    residual is the floor (`add` returns True); above it the server checks
    whether the lattice is at rest (`stalled`)."""

    def __init__(self, window=200, ratio=0.9, ceiling=1e-4):
        self.window, self.ratio, self.ceiling = int(window), float(ratio), float(ceiling)
        self.hist = collections.deque(maxlen=2 * self.window)
        self.stalled = False
        self.level = float("inf")     # median of the last window

    def add(self, r):
        self.hist.append(r)
        if len(self.hist) < 2 * self.window:
            return False
        h = list(self.hist)
        old, new = float(np.median(h[:self.window])), float(np.median(h[self.window:]))
        self.stalled = bool(new >= self.ratio * old)
        self.level = new
        return self.stalled and r < self.ceiling


# A lattice at rest: its residual stalled at NOISE_RESIDUAL or above (two
# independent noise fields give sqrt(2)) and every |u| below REST_SPEED.
NOISE_RESIDUAL = 0.5
REST_SPEED = 1e-5


class Server:
    def __init__(self, budget_bytes=96 << 30, max_resident=64, diag_every=100, max_steps=1000000, tol=1e-5,
                 batched=True, device="cuda:0", seg_rows=0, on_admit=None, tile_costs="calibrate",
                 max_nodes=16 << 20, two_step="calibrate", floor_window=200):
        import torch
        if diag_every % 2:
            raise ValueError("diag_every must be even (graph replays keep the buffer parity)")
        self.budget = int(budget_bytes)
        self.max_resident = int(max_resident)
        self.max_nodes = int(max_nodes)
        self.K = int(diag_every)
        self.max_steps = int(max_steps)
        self.tol = float(tol)
        self.floor_window = floor_window
        self.batched = bool(batched)
        self.device = device
        self.seg_rows = seg_rows
        self.on_admit = on_admit          # called as on_admit(request, lattice) after creation
        self._footprints = {}
        self.max_seen_resident = 0
        self.max_seen_used = 0            # largest sum of resident footprints (bytes)
        # per-tile cost of every tile shape: measured, given, or None (shape 0)
        self.tile_costs = calibrate_tile_costs(device=device) if tile_costs == "calibrate" else tile_costs
        # two-step variant of every batch (-1: single steps): measured or given
        self.two_step = calibrate_two_step(device=device) if two_step == "calibrate" else int(two_step)
        torch.cuda.synchronize(device)
        self.stream = torch.cuda.Stream(device)

    def footprint(self, req):
        fp = self._footprints.get(req.rid)
        if fp is None:
            fp = self._footprints[req.rid] = lbm.lbm_workspace_bytes(lattice_params(req, self.seg_rows))
        return fp

    @staticmethod
    def _at_rest(lat):
        _, ux, uy, _ = lat.moments()
        return bool(max(np.abs(ux).max(), np.abs(uy).max()) < REST_SPEED)

    def _measure(self, req, lat):
        if req.kind == "angle":
            out = lat.contact_angle(I.ISO, 0.0)
            return tuple(out) if out is not None else ()
        return tuple(lat.slip_length())

    def run(self, requests, realtime=True, log=None):
        """Serve `requests` (inputs.Request, arrival in seconds from the start).
        Returns the list of Result in request order.  log: a file to which
        one line per retired request is written (progress of long runs)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        results = {r.rid: Result(r.rid, r.kind, r.nx, r.ny, r.arrival) for r in requests}
        waiting = collections.deque()
        resident = []            # [(req, Lattice, footprint)]
        floors = {}              # rid -> Floor detector
        used = 0
        nodes = 0
        batch = None
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        if not realtime:
            # every request is present from time zero
            for r in requests:
                results[r.rid].arrival = 0.0
        while pending or waiting or resident:
            now = clock()
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            changed = False
            while waiting and len(resident) < self.max_resident:
                req = waiting[0]
                fp = self.footprint(req)
                if fp > self.budget:
                    waiting.popleft()
                    res = results[req.rid]
                    res.error = f"footprint {fp} B exceeds the budget"
                    res.finished = clock()
                    continue
                if used + fp > self.budget:
                    break
                if resident and nodes + req.nx * req.ny > self.max_nodes:
                    break
                waiting.popleft()
                t_adm = clock()
                p, rho0 = request_params(req, self.seg_rows)
                u0 = initial_velocity(req, p)
                lat = lbm.Lattice(p, rho0, None if u0 is None else u0[0], None if u0 is None else u0[1],
                                  device=self.device, stream=self.stream)
                if self.tile_costs is not None:
                    lat.tile_shape = pick_tile_shape(req.nx, req.ny, self.tile_costs)
                if not self.batched:
                    lat.two_step = self.two_step
                if self.on_admit is not None:
                    self.on_admit(req, lat)
                resident.append((req, lat, fp))
                floors[req.rid] = Floor(self.floor_window) if self.floor_window else None
                self.max_seen_resident = max(self.max_seen_resident, len(resident))
                used += fp
                nodes += req.nx * req.ny
                self.max_seen_used = max(self.max_seen_used, used)
                results[req.rid].admitted = t_adm
                changed = True
            if not resident:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - clock()))
                continue
            if self.batched:
                if changed or batch is None:
                    if batch is not None:
                        batch.close()
                    batch = lbm.Attached([lat for _, lat, _ in resident], device=self.device)
                    batch.two_step = self.two_step
                batch.step(self.K, chunk=self.K)
                diag, code = batch.diagnostics(check=False)
            else:
                diag = []
                for _, lat, _ in resident:
                    lat.step(self.K)
                    d, _ = lbm.lbm_diagnostics(lat.ctx, check=False)
                    diag.append(d)
                diag = np.array(diag)
            retire = []
            for k, (req, lat, fp) in enumerate(resident):
                res = results[req.rid]
                res.steps = int(diag[k][0])
                res.residual = float(diag[k][4])
                bad = diag[k][5] > 0
                fl = floors[req.rid]
                at_floor = fl is not None and fl.add(res.residual)
                at_rest = False
                if fl is not None and fl.stalled and fl.level >= NOISE_RESIDUAL and not bad:
                    # a residual stalled at O(1): successive velocity fields are
                    # uncorrelated, as rounding noise of a fluid at rest is
                    at_rest = self._at_rest(lat)
                    fl.hist.clear()
                    fl.stalled = False
                below = bool(res.residual < self.tol)
                done = below or at_floor or at_rest or res.steps >= self.max_steps
                if bad:
                    res.error = "non-finite state"
                    retire.append(k)
                elif done:
                    res.converged = below or at_floor or at_rest
                    res.floor = at_floor and not below
                    res.rest = at_rest and not below
                    try:
                        res.value = self._measure(req, lat)
                    except lbm.LbmError as e:
                        res.error = str(e)
                    retire.append(k)
            if retire:
                if batch is not None:
                    batch.close()
                    batch = None
                now = clock()
                for k in sorted(retire, reverse=True):
                    req, lat, fp = resident.pop(k)
                    results[req.rid].finished = now
                    if log is not None:
                        r = results[req.rid]
                        print(f"t={now:8.2f}s done {r.rid} {r.kind} {r.nx}x{r.ny} steps {r.steps} "
                              f"residual {r.residual:.2e} converged {r.converged} floor {r.floor} rest {r.rest} "
                              f"latency {r.latency:.2f}s {r.error}", file=log, flush=True)
                    lat.close()
                    used -= fp
                    nodes -= req.nx * req.ny
        if batch is not None:
            batch.close()
        self.elapsed = clock()
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summarize(results, elapsed):
    lat = np.array([r.latency for r in results if not r.error])
    done = [r for r in results if not r.error]
    return {
        "requests": len(results),
        "completed": len(done),
        "failed": len(results) - len(done),
        "converged": int(sum(bool(r.converged) for r in done)),
        "converged_below_tol": int(sum(bool(r.converged and not (r.floor or r.rest)) for r in done)),
        "converged_at_floor": int(sum(bool(r.floor) for r in done)),
        "converged_at_rest": int(sum(bool(r.rest) for r in done)),
        "at_step_cap": int(sum(not r.converged for r in done)),
        "solves_per_s": len(done) / elapsed if elapsed > 0 else 0.0,
        "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
        "elapsed_s": float(elapsed),
        "lattice_updates": int(sum(r.steps * r.nx * r.ny for r in done)),
    }
