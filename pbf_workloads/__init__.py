"""Seeded synthetic inputs for the powder-bed-fusion thermal step.

This module only *describes* problems: box meshes, material tables, laser paths,
probe points and targets, all drawn from fixed seeds.  It contains none of the
method's arithmetic (no shape functions, no quadrature, no material law, no time
step rule), so that both the CPU oracle and the GPU library can be driven from
the same numbers without sharing any computation.

Workload shapes follow the paper's setting: a box of metal with a Dirichlet
base (heat equation with Dirichlet bottom, insulated elsewhere), a Gaussian beam
of radius 50 um scanning tracks on the top surface, a powder layer on top
(phase-dependent conductivity, consolidated fraction history), and
piecewise-linear temperature-dependent conductivity and heat capacity with an
apparent-capacity latent-heat bump between solidus and liquidus.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# face bits of the box boundary: x-, x+, y-, y+, z-, z+
FACE_XM, FACE_XP, FACE_YM, FACE_YP, FACE_ZM, FACE_ZP = 1, 2, 4, 8, 16, 32
ALL_FACES = 63

LASER_OFF, LASER_SURFACE, LASER_VOLUME = -1, 0, 1


@dataclass
class Problem:
    name: str
    degree: int
    nx: int
    ny: int
    nz: int
    L: tuple
    dirichlet_mask: int
    T_D: float
    T0: float
    T_bp: np.ndarray
    k_bp: np.ndarray
    cp_bp: np.ndarray
    rho: float
    T_s: float
    T_l: float
    latent: float
    powder_k_factor: float
    powder_depth: float
    laser_kind: int
    radius: float
    absorptivity: float
    h_powder: float
    t_start: float
    tracks: np.ndarray  # (n_tracks, 8): x0 y0 z0 x1 y1 z1 speed power
    steps: int = 0
    dt_factor: float = 0.5  # fraction of the explicit stability limit
    seed: int = 0
    probes: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    targets: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # octree meshes: nx, ny, nz are the coarse (level 0) cells; leaves (n, 4) hold
    # (level, ix, iy, iz) with the origin in units of the finest cell size
    max_level: int = 0
    refine_radius: float = 0.0
    refine_ahead: float = 0.0   # path length refined ahead of the beam
    refine_trail: float = 0.0   # path length refined behind the beam (window schedules)
    scan_start: float = 0.0     # arc length of the beam when a window schedule starts
    remesh_every: int = 0
    leaves: np.ndarray = None
    implicit_steps: int = 0
    implicit_dt: float = 0.0
    # radiation and evaporation on the free top surface (off by default); the
    # constants default to the stainless-steel values of the paper's Table 2
    # (T_inf is the ambient temperature; None: T_D)
    emissivity: float = 0.0
    T_inf: float = None
    evap_on: bool = False
    T_v: float = 3000.0
    C_P: float = 54.0e3
    C_T: float = 5.0e4
    C_M: float = 1.0e-3
    h_v: float = 6.0e6
    T_h0: float = 663.0
    dT_max: float = 1000.0

    # --- counting helpers (mesh bookkeeping only) ---
    @property
    def nodes_per_dim(self):
        p = self.degree
        return (p * self.nx + 1, p * self.ny + 1, p * self.nz + 1)

    @property
    def ambient(self) -> float:
        return self.T_D if self.T_inf is None else self.T_inf

    @property
    def n_dofs(self) -> int:
        a, b, c = self.nodes_per_dim
        return a * b * c

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_qp_per_cell(self) -> int:
        return (self.degree + 1) ** 3

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _material_tables(seed: int):
    """8 breakpoints: 293 K, 3000 K and 6 sorted interior points; k in [15,35] W/mK,
    cp in [450,750] J/kgK, all drawn uniformly from one seed."""
    rng = np.random.default_rng(seed)
    interior = np.sort(rng.uniform(293.0, 3000.0, size=6))
    T_bp = np.concatenate([[293.0], interior, [3000.0]])
    k_bp = rng.uniform(15.0, 35.0, size=8)
    cp_bp = rng.uniform(450.0, 750.0, size=8)
    return T_bp, k_bp, cp_bp


def zigzag(seed: int, centre, z_top: float, n_tracks=10, length=1.0e-3, hatch=100e-6,
           speed=0.8, power=200.0) -> np.ndarray:
    """Serpentine scan: n_tracks tracks along +-x of the given length, hatch spacing
    in y, centred on `centre`; the start corner comes from the seed; turnarounds are
    instantaneous (the next track starts where the last one ended, one hatch over)."""
    rng = np.random.default_rng(seed + 7)
    sx = 1.0 if rng.integers(0, 2) == 0 else -1.0   # first track direction
    sy = 1.0 if rng.integers(0, 2) == 0 else -1.0   # hatch direction
    cx, cy = centre
    tr = np.zeros((n_tracks, 8))
    for j in range(n_tracks):
        y = cy + sy * (j - 0.5 * (n_tracks - 1)) * hatch
        d = sx if j % 2 == 0 else -sx
        x0 = cx - d * 0.5 * length
        x1 = cx + d * 0.5 * length
        tr[j] = [x0, y, z_top, x1, y, z_top, speed, power]
    return tr


def _base_nonlinear(name, seed, nx, ny, nz, L, steps, track_length=1.0e-3, n_tracks=10,
                    hatch=100e-6):
    T_bp, k_bp, cp_bp = _material_tables(seed)
    tracks = zigzag(seed, (0.5 * L[0], 0.5 * L[1]), L[2], n_tracks=n_tracks,
                    length=track_length, hatch=hatch)
    return Problem(
        name=name, degree=2, nx=nx, ny=ny, nz=nz, L=tuple(L),
        dirichlet_mask=FACE_ZM, T_D=293.0, T0=293.0,
        T_bp=T_bp, k_bp=k_bp, cp_bp=cp_bp,
        rho=7900.0, T_s=1563.0, T_l=1623.0, latent=2.7e5,
        powder_k_factor=0.01, powder_depth=40e-6,
        laser_kind=LASER_VOLUME, radius=50e-6, absorptivity=0.35, h_powder=40e-6,
        t_start=0.0, tracks=tracks, steps=steps, dt_factor=0.5, seed=seed)


def cfg1() -> Problem:
    """Q1 16x16x8 box of 1x1x0.5 mm, constant k=20, rho=7900, cp=500, Dirichlet
    293 K at the bottom, Gaussian *surface* flux P=200 W, A=0.35, R=50 um, moving
    +x at 0.8 m/s from (0, 0.5 mm); 200 steps at half the stability limit."""
    tracks = np.array([[0.0, 0.5e-3, 0.5e-3, 1.0e-3, 0.5e-3, 0.5e-3, 0.8, 200.0]])
    return Problem(
        name="cfg1_q1_16x16x8", degree=1, nx=16, ny=16, nz=8, L=(1e-3, 1e-3, 0.5e-3),
        dirichlet_mask=FACE_ZM, T_D=293.0, T0=293.0,
        T_bp=np.array([293.0, 3000.0]), k_bp=np.array([20.0, 20.0]),
        cp_bp=np.array([500.0, 500.0]),
        rho=7900.0, T_s=1563.0, T_l=1623.0, latent=0.0,
        powder_k_factor=1.0, powder_depth=0.0,
        laser_kind=LASER_SURFACE, radius=50e-6, absorptivity=0.35, h_powder=40e-6,
        t_start=0.0, tracks=tracks, steps=200, dt_factor=0.5, seed=0)


def cfg2() -> Problem:
    """Q2 128x128x64 box of 4x4x2 mm (8,520,321 DoFs), seeded nonlinear law,
    powder in the top 40 um, zigzag of 10 tracks, 5000 explicit steps."""
    return _base_nonlinear("cfg2_q2_128x128x64", 2302, 128, 128, 64, (4e-3, 4e-3, 2e-3), 5000)


def cfg4() -> Problem:
    """cfg2's law and scan on the same box at 160x160x80 Q2 (16,589,601 DoFs)."""
    return _base_nonlinear("cfg4_q2_160x160x80", 2302, 160, 160, 80, (4e-3, 4e-3, 2e-3), 5000)


def cfg5() -> Problem:
    """Q2 48x48x24 box of 1.5x1.5x0.75 mm (461,041 DoFs), cfg2's law, zigzag of 10
    tracks of 0.6 mm so that the whole path is scanned within 3000 steps; 64 probes
    seeded on the top face over the scanned area, targets seeded in [T0, 2000 K]."""
    p = _base_nonlinear("cfg5_q2_48x48x24", 2302, 48, 48, 24, (1.5e-3, 1.5e-3, 0.75e-3), 3000,
                        track_length=0.6e-3)
    return with_probes(p, 64, seed=2305)


def with_probes(p: Problem, n: int, seed: int, t_lo=None, t_hi=2000.0) -> Problem:
    rng = np.random.default_rng(seed)
    tr = p.tracks
    xlo, xhi = tr[:, [0, 3]].min(), tr[:, [0, 3]].max()
    ylo, yhi = tr[:, [1, 4]].min(), tr[:, [1, 4]].max()
    pts = np.zeros((n, 3))
    pts[:, 0] = rng.uniform(xlo, xhi, n)
    pts[:, 1] = rng.uniform(ylo, yhi, n)
    pts[:, 2] = p.L[2]
    lo = p.T0 if t_lo is None else t_lo
    targets = rng.uniform(lo, t_hi, n)
    return p.replace(probes=pts, targets=targets)


def small_nonlinear(nx=20, ny=18, nz=10, steps=200, seed=2302, h=31.25e-6, track_length=None,
                    n_tracks=4, hatch=100e-6) -> Problem:
    """cfg2's physics at a size the oracle runs in seconds; the cell counts are chosen
    so that they are not multiples of the GPU tile and leave ragged tails."""
    L = (nx * h, ny * h, nz * h)
    if track_length is None:
        track_length = 0.6 * L[0]
    return _base_nonlinear(f"small_q2_{nx}x{ny}x{nz}", seed, nx, ny, nz, L, steps,
                           track_length=track_length, n_tracks=n_tracks, hatch=hatch)


def active_part(p: Problem, nz_active: int) -> Problem:
    """The bottom nz_active cell layers of a box as a problem of their own (the
    active part of a growing box: same cells, top face at nz_active hz)."""
    hz = p.L[2] / p.nz
    return p.replace(nz=nz_active, L=(p.L[0], p.L[1], nz_active * hz))


def with_surface_losses(p: Problem, emissivity=0.7, evap=True) -> Problem:
    """The same problem with radiation (emissivity of the paper's Table 2) and
    evaporation on the top surface."""
    return p.replace(name=p.name + "_re", emissivity=emissivity, evap_on=evap)


def convergence_box(degree=2, h=40e-6, power=200.0, absorptivity=0.35) -> Problem:
    """The two-layer example of the paper's temporal-convergence appendix: a
    1.0 x 0.2 x 0.2 mm base plate with two 40 um powder layers on top (cells of h,
    the top two cell layers are the powder layers when h = 40 um), the material of
    Table 2 (k = 20 W/mK in melt and solid, 0.2 in powder, rho = 7430, c = 965,
    T_s = 1500 K, T_l = 1900 K, T_0 = 303 K, no latent heat, radiation and
    evaporation on), the scan of Table 4 (v = 0.96 m/s, R = 60 um); one track per
    layer along +x from (0, 0) at the top of that layer.  The laser power is not
    given in the paper: 200 W with absorptivity 0.35 as in the other workloads.
    `tracks` holds both tracks (layer 1, layer 2); a run scans them one per layer."""
    L = (1.0e-3, 0.2e-3, 0.28e-3)
    nx, ny, nz = round(L[0] / h), round(L[1] / h), round(L[2] / h)
    tracks = np.array([[0.0, 0.0, 0.24e-3, 1.0e-3, 0.0, 0.24e-3, 0.96, power],
                       [0.0, 0.0, 0.28e-3, 1.0e-3, 0.0, 0.28e-3, 0.96, power]])
    p = Problem(
        name=f"convergence_q{degree}_{nx}x{ny}x{nz}", degree=degree, nx=nx, ny=ny, nz=nz, L=L,
        dirichlet_mask=FACE_ZM, T_D=303.0, T0=303.0,
        T_bp=np.array([303.0, 3000.0]), k_bp=np.array([20.0, 20.0]), cp_bp=np.array([965.0, 965.0]),
        rho=7430.0, T_s=1500.0, T_l=1900.0, latent=0.0, powder_k_factor=0.01, powder_depth=40e-6,
        laser_kind=LASER_VOLUME, radius=60e-6, absorptivity=absorptivity, h_powder=40e-6,
        t_start=0.0, tracks=tracks, steps=0, dt_factor=0.5, seed=0)
    return with_surface_losses(p)


def sine_mode(degree: int, n: int, k=20.0, rho=7900.0, cp=500.0) -> Problem:
    """Unit cube, all faces Dirichlet, constant coefficients, laser off: the setting of
    the decaying eigenmode T = T_D + A sin(pi x) sin(pi y) sin(pi z)."""
    return Problem(
        name=f"sine_q{degree}_{n}", degree=degree, nx=n, ny=n, nz=n, L=(1.0, 1.0, 1.0),
        dirichlet_mask=ALL_FACES, T_D=293.0, T0=293.0,
        T_bp=np.array([0.0, 1.0e9]), k_bp=np.array([k, k]), cp_bp=np.array([cp, cp]),
        rho=rho, T_s=1.0e8, T_l=2.0e8, latent=0.0, powder_k_factor=1.0, powder_depth=0.0,
        laser_kind=LASER_OFF, radius=50e-6, absorptivity=0.35, h_powder=40e-6,
        t_start=0.0, tracks=np.zeros((0, 8)), steps=0, dt_factor=0.5, seed=0)


def hot_spot_state(p: Problem, seed: int, peak=2600.0, width=120e-6, noise=5.0):
    """A seeded temperature field on a box with a melt pool: T0 plus a Gaussian
    bump of height peak - T0 and 1/e radius `width`, centred on the top surface
    0.1 mm along the first track (a quarter as deep as wide), plus uniform noise
    of +-noise K; Dirichlet nodes at T_D.  Returns (T, t) with t the time at
    which the beam is at the bump's centre.  (Input data only: a field shape and
    random numbers.)"""
    rng = np.random.default_rng(seed)
    NX, NY, NZ = p.nodes_per_dim
    tr = p.tracks[0]
    a, b = np.asarray(tr[0:3]), np.asarray(tr[3:6])
    d = (b - a) / np.linalg.norm(b - a)
    c = a + 0.1e-3 * d
    x = np.linspace(0.0, p.L[0], NX)
    y = np.linspace(0.0, p.L[1], NY)
    z = np.linspace(0.0, p.L[2], NZ)
    ex = np.exp(-((x - c[0]) / width) ** 2)
    ey = np.exp(-((y - c[1]) / width) ** 2)
    ez = np.exp(-((z - p.L[2]) / (0.25 * width)) ** 2)
    T = (p.T0 + (peak - p.T0) * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]).reshape(-1)
    T += rng.uniform(-noise, noise, T.size)
    m = p.dirichlet_mask
    k, j, i = (np.arange(NZ)[:, None, None], np.arange(NY)[None, :, None], np.arange(NX)[None, None, :])
    dmask = np.zeros((NZ, NY, NX), dtype=bool)
    for bit, cond in ((1, i == 0), (2, i == NX - 1), (4, j == 0), (8, j == NY - 1), (16, k == 0),
                      (32, k == NZ - 1)):
        if m & bit:
            dmask |= np.broadcast_to(cond, dmask.shape)
    T[dmask.reshape(-1)] = p.T_D
    return T, float(p.t_start + 0.1e-3 / tr[6])


def seeded_vector(n: int, seed: int) -> np.ndarray:
    """Uniform(-1, 1) numbers: start vectors for power iterations and random fields."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


# ---------------------------------------------------------------------------
# octree meshes
# ---------------------------------------------------------------------------
def path_points(p: Problem, s_lo: float, s_hi: float, spacing: float) -> np.ndarray:
    """Beam centres along the scan path between arc lengths s_lo and s_hi
    (tracks in order, arc length measured from the first track's start), sampled
    at most `spacing` apart, shape (m, 3)."""
    out = []
    s0 = 0.0
    for tr in p.tracks:
        a, b = np.asarray(tr[0:3]), np.asarray(tr[3:6])
        length = float(np.linalg.norm(b - a))
        lo, hi = max(s_lo, s0), min(s_hi, s0 + length)
        if hi >= lo:
            n = max(2, int(np.ceil((hi - lo) / spacing)) + 1)
            u = (np.linspace(lo, hi, n) - s0) / length
            out.append(a[None, :] + u[:, None] * (b - a)[None, :])
        s0 += length
    return np.concatenate(out) if out else np.zeros((0, 3))


def beam_arc_length(p: Problem, t: float) -> float:
    """Arc length of the beam position at time t along the scan path."""
    s, tk = 0.0, p.t_start
    for tr in p.tracks:
        length = float(np.linalg.norm(np.asarray(tr[3:6]) - np.asarray(tr[0:3])))
        dur = length / tr[6]
        if t < tk + dur:
            return s + max(0.0, t - tk) * tr[6]
        s += length
        tk += dur
    return s


def _morton(ix, iy, iz):
    key = np.zeros(len(ix), dtype=np.int64)
    for b in range(21):
        key |= ((ix >> b) & 1) << (3 * b) | ((iy >> b) & 1) << (3 * b + 1) | ((iz >> b) & 1) << (3 * b + 2)
    return key


def octree_leaves(p: Problem, s_hi: float, s_lo: float = 0.0) -> np.ndarray:
    """Leaves (level, ix, iy, iz) of an octree over p's coarse box, origins in
    units of the finest cell: a level-l cell is split when its distance to the
    sampled beam path between arc lengths s_lo and s_hi is below R_{l+1}, with
    R_max = p.refine_radius and R_l = R_{l+1} + (diagonal of a level-l cell).
    The graded radii make the tree 2:1 balanced across faces, edges and
    vertices (a leaf touching a leaf two levels finer would be closer to the
    path than its own radius).  Leaves are returned in Morton order."""
    L = np.asarray(p.L, dtype=np.float64)
    n0 = np.array([p.nx, p.ny, p.nz])
    maxl = p.max_level
    h0 = L / n0
    unit = h0 / 2 ** maxl
    R = np.zeros(maxl + 1)
    R[maxl] = p.refine_radius
    for l in range(maxl - 1, -1, -1):
        R[l] = R[l + 1] + float(np.linalg.norm(h0 / 2 ** l))
    pts = path_points(p, s_lo, s_hi, spacing=0.5 * float(unit.min()))
    g = np.stack(np.meshgrid(np.arange(p.nx), np.arange(p.ny), np.arange(p.nz), indexing="ij"),
                 -1).reshape(-1, 3).astype(np.int64) * 2 ** maxl
    out = []
    for l in range(maxl + 1):
        size = 2 ** (maxl - l)
        split = np.zeros(len(g), dtype=bool)
        if l < maxl and len(pts) and len(g):
            lo, hi = g * unit, (g + size) * unit
            d2 = np.full(len(g), np.inf)
            for c0 in range(0, len(pts), 256):
                q = pts[c0:c0 + 256]
                e = np.maximum(np.maximum(lo[:, None, :] - q[None], 0.0), q[None] - hi[:, None, :])
                d2 = np.minimum(d2, (e * e).sum(-1).min(1))
            split = d2 < R[l + 1] ** 2
        keep = g[~split]
        out.append(np.concatenate([np.full((len(keep), 1), l, dtype=np.int64), keep], 1))
        half = size // 2
        par = g[split]
        if l < maxl and len(par):
            off = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], dtype=np.int64) * half
            g = (par[:, None, :] + off[None]).reshape(-1, 3)
        else:
            g = np.zeros((0, 3), dtype=np.int64)
    leaves = np.concatenate(out)
    order = np.argsort(_morton(leaves[:, 1], leaves[:, 2], leaves[:, 3]), kind="stable")
    return np.ascontiguousarray(leaves[order])


def with_leaves(p: Problem, s_hi: float, s_lo: float = 0.0) -> Problem:
    return p.replace(leaves=octree_leaves(p, s_hi, s_lo))


def cfg3() -> Problem:
    """Q2 octree over a 10x10x5 mm part: coarse 20x20x10 cells (0.5 mm) refined to
    level 6 (7.8 um) within 200 um of the window [s - 8 mm, s + 100 um] of the
    scan path around the beam's arc length s, cfg2's law, a 10-track zigzag of
    1 mm tracks at the centre of the top face.  The schedule starts with the
    beam at the start of the tenth track (s = 9 mm, about 5.2M dofs) and runs
    2000 explicit steps with a remesh every 100, then 50 backward-Euler steps of
    1 ms with the laser off.  The leaves are built at run time by the library
    (the window at this size takes a minute in octree_leaves)."""
    p = _base_nonlinear("cfg3_q2_octree", 2302, 20, 20, 10, (10e-3, 10e-3, 5e-3), 2000)
    return p.replace(max_level=6, refine_radius=200e-6, refine_ahead=100e-6, refine_trail=8.0e-3,
                     scan_start=9.0e-3, remesh_every=100, implicit_steps=50, implicit_dt=1e-3)


def cfg3_reduced(max_level=2, trail=0.3e-3, start=0.45e-3) -> Problem:
    """cfg3's schedule on a 1x0.75x0.5 mm part (coarse 4x3x2 cells of 0.25 mm)
    refined to `max_level` within 60 um of a short path window, a zigzag of
    0.4 mm tracks: sizes the octree oracle runs in seconds."""
    p = _base_nonlinear("cfg3_reduced", 2302, 4, 3, 2, (1.0e-3, 0.75e-3, 0.5e-3), 40,
                        track_length=0.4e-3, n_tracks=4, hatch=60e-6)
    return p.replace(max_level=max_level, refine_radius=60e-6, refine_ahead=40e-6, refine_trail=trail,
                     scan_start=start, remesh_every=10, implicit_steps=2, implicit_dt=2e-4)


def growing_octree_build(max_level=2, n_layers=6) -> Problem:
    """A growing build on an octree (Section 4.1): coarse cells of
    2^max_level powder layers (h_powder = 40 um, eq. coarse_fine_relation) over
    a 4x3 coarse-cell chamber three coarse cells tall; the part starts as one
    coarse layer of substrate whose top 40 um are the first powder layer, and
    every further layer is activated on top; one track per layer (a zigzag of
    0.4 mm tracks), cfg2's law."""
    hc = 40e-6 * (1 << max_level)
    p = _base_nonlinear("growing_octree", 2306, 4, 3, 3, (4 * hc, 3 * hc, 3 * hc), 60,
                        track_length=0.4e-3, n_tracks=n_layers, hatch=60e-6)
    return p.replace(max_level=max_level, remesh_every=0)


def small_octree(degree=2, max_level=2, seed=2302, ahead=60e-6, radius=40e-6) -> Problem:
    """cfg3's physics on a 3x2x2-cell coarse box of 0.375x0.25x0.25 mm refined to
    level `max_level` around the start of the scan (sizes the oracle runs in
    seconds)."""
    h = 125e-6
    p = _base_nonlinear(f"small_octree_q{degree}", seed, 3, 2, 2, (3 * h, 2 * h, 2 * h), 0,
                        track_length=0.2e-3, n_tracks=2, hatch=60e-6)
    p = p.replace(degree=degree, max_level=max_level, refine_radius=radius, refine_ahead=ahead)
    return with_leaves(p, ahead)


CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4, "cfg5": cfg5}
