"""Seeded synthetic inputs for the radar ray-tracing hot path.

This module builds scenes (triangle meshes with per-object material and
velocity, plus point reflectors), MIMO array geometries, FMCW chirp
parameters and trace parameters.  It is the only code shared by the CPU
oracle tests and the GPU path: it holds geometry construction and random
draws only, none of the method's arithmetic (no ray tracing, no bounce, no
phase or synthesis).

Conventions (both sides rely on them):
  * metres, seconds, hertz; x = boresight, y = left, z = up; arrays lie in
    the plane x = 0.
  * vertices are float32 [nv][3]; triangles int32 [nt][3]; tri_obj int32 [nt]
    names the object of each triangle; object 0 is the ground when present.
  * obj_alpha float32 [nobj] is the material mix of the paper's Eq. 3
    (0 = specular, 1 = diffuse), obj_vel float64 [nobj][3] is a constant
    velocity; an optional tri_alpha float32 [nt] gives every face its own
    mix instead of its object's.
  * point reflectors: pt_pos / pt_vel float64 [np][3], pt_aperture float64 [np]
    (m^2).
  * Tx / Rx positions float64 [n][3]; virtual channel c = t * n_rx + r.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C0 = 299792458.0          # speed of light, m/s (exact by definition)
F77 = 77e9
LAMBDA77 = C0 / F77       # 3.8934 mm

MODE_PER_TX = 0           # rays launched from every Tx element, N/n_tx each
MODE_SHARED = 1           # rays launched once from the Tx phase centre


@dataclass
class Scene:
    verts: np.ndarray                 # float32 [nv][3]
    tris: np.ndarray                  # int32 [nt][3]
    tri_obj: np.ndarray               # int32 [nt]
    obj_alpha: np.ndarray             # float32 [nobj]
    obj_vel: np.ndarray               # float64 [nobj][3]
    pt_pos: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    pt_vel: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    pt_aperture: np.ndarray = field(default_factory=lambda: np.zeros((0,)))
    tri_alpha: np.ndarray | None = None   # float32 [nt] per-face alpha (None: the object's)

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_obj(self) -> int:
        return int(self.obj_alpha.shape[0])

    @property
    def n_pts(self) -> int:
        return int(self.pt_pos.shape[0])

    def checked(self) -> "Scene":
        self.verts = np.ascontiguousarray(self.verts, dtype=np.float32).reshape(-1, 3)
        self.tris = np.ascontiguousarray(self.tris, dtype=np.int32).reshape(-1, 3)
        self.tri_obj = np.ascontiguousarray(self.tri_obj, dtype=np.int32).reshape(-1)
        self.obj_alpha = np.ascontiguousarray(self.obj_alpha, dtype=np.float32).reshape(-1)
        self.obj_vel = np.ascontiguousarray(self.obj_vel, dtype=np.float64).reshape(-1, 3)
        self.pt_pos = np.ascontiguousarray(self.pt_pos, dtype=np.float64).reshape(-1, 3)
        self.pt_vel = np.ascontiguousarray(self.pt_vel, dtype=np.float64).reshape(-1, 3)
        self.pt_aperture = np.ascontiguousarray(self.pt_aperture, dtype=np.float64).reshape(-1)
        if self.tri_alpha is not None:
            self.tri_alpha = np.ascontiguousarray(self.tri_alpha, dtype=np.float32).reshape(-1)
            assert self.tri_alpha.shape[0] == self.tris.shape[0]
        assert self.tri_obj.shape[0] == self.tris.shape[0]
        assert self.obj_vel.shape[0] == self.obj_alpha.shape[0]
        assert self.pt_vel.shape[0] == self.pt_pos.shape[0] == self.pt_aperture.shape[0]
        return self


@dataclass
class Array:
    tx: np.ndarray                    # float64 [n_tx][3]
    rx: np.ndarray                    # float64 [n_rx][3]
    rx_radius: float = 0.25           # reception-sphere radius (m)
    mode: int = MODE_PER_TX

    @property
    def n_tx(self) -> int:
        return int(self.tx.shape[0])

    @property
    def n_rx(self) -> int:
        return int(self.rx.shape[0])

    @property
    def n_ch(self) -> int:
        return self.n_tx * self.n_rx

    def checked(self) -> "Array":
        self.tx = np.ascontiguousarray(self.tx, dtype=np.float64).reshape(-1, 3)
        self.rx = np.ascontiguousarray(self.rx, dtype=np.float64).reshape(-1, 3)
        return self


@dataclass
class Chirp:
    f0: float = F77
    bandwidth: float = 1e9
    t_chirp: float = 50e-6
    t_rep: float = 50e-6
    n_samples: int = 64
    n_chirps: int = 16


def chirp_sfcw(f_start: float = 72e9, f_stop: float = 82e9, n_steps: int = 128) -> Chirp:
    """A stepped-frequency sweep f_n = f_start + n (f_stop - f_start) / (n_steps - 1),
    n = 0 .. n_steps - 1 (both ends included), as one chirp of n_steps samples:
    f0 + B k / K with B = (f_stop - f_start) n_steps / (n_steps - 1)."""
    bw = (f_stop - f_start) * n_steps / (n_steps - 1)
    return Chirp(f0=f_start, bandwidth=bw, t_chirp=1e-3, t_rep=1e-3, n_samples=n_steps,
                 n_chirps=1)


@dataclass
class TraceParams:
    n_rays: int = 100_000            # total launched rays (split over Tx in PER_TX mode)
    max_bounces: int = 2
    seed: int = 0
    az_min: float = -math.pi / 2
    az_max: float = math.pi / 2
    el_min: float = -math.pi / 2
    el_max: float = math.pi / 2
    rays_per_tri: int = 0            # > 0: cast this many rays (a perfect square) towards
                                     # every triangle from every source instead of n_rays
    tri_omega_max: float = 0.0       # > 0: first cut triangles into pieces of at most this
                                     # solid angle (sr) from the Tx phase centre
    tri_depth_max: int = 8           # at most 4^depth pieces per triangle


@dataclass
class Workload:
    name: str
    scene: Scene
    array: Array
    chirp: Chirp
    trace: TraceParams
    path_cap: int | None = None      # keep only the first path_cap paths (ray, bounce order)


# ----------------------------------------------------------------------------
# mesh primitives (geometry only)
# ----------------------------------------------------------------------------

class _MeshBuilder:
    def __init__(self):
        self.v: list[np.ndarray] = []
        self.t: list[np.ndarray] = []
        self.o: list[np.ndarray] = []
        self.nv = 0

    def add(self, verts: np.ndarray, tris: np.ndarray, obj: int):
        verts = np.asarray(verts, dtype=np.float64).reshape(-1, 3)
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3) + self.nv
        self.v.append(verts)
        self.t.append(tris)
        self.o.append(np.full(tris.shape[0], obj, dtype=np.int32))
        self.nv += verts.shape[0]

    def grid_quad(self, origin, e1, e2, n1: int, n2: int, obj: int):
        """Parallelogram origin + a*e1 + b*e2, a,b in [0,1], split n1 x n2 cells."""
        origin, e1, e2 = (np.asarray(x, dtype=np.float64) for x in (origin, e1, e2))
        a = np.linspace(0.0, 1.0, n1 + 1)
        b = np.linspace(0.0, 1.0, n2 + 1)
        A, B = np.meshgrid(a, b, indexing="ij")
        verts = origin + A[..., None] * e1 + B[..., None] * e2
        idx = np.arange((n1 + 1) * (n2 + 1)).reshape(n1 + 1, n2 + 1)
        i00 = idx[:-1, :-1].ravel()
        i10 = idx[1:, :-1].ravel()
        i01 = idx[:-1, 1:].ravel()
        i11 = idx[1:, 1:].ravel()
        tris = np.concatenate([np.stack([i00, i10, i11], 1), np.stack([i00, i11, i01], 1)])
        self.add(verts.reshape(-1, 3), tris, obj)

    def box(self, lo, hi, step: float | None, obj: int, yaw: float = 0.0):
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        ext = hi - lo
        n = [1, 1, 1] if step is None else [max(1, int(round(e / step))) for e in ext]
        ex, ey, ez = np.diag(ext)
        faces = [
            (lo, ey, ex, n[1], n[0]),                 # bottom z = lo
            (lo + ez, ex, ey, n[0], n[1]),            # top z = hi
            (lo, ex, ez, n[0], n[2]),                 # y = lo
            (lo + ey, ez, ex, n[2], n[0]),            # y = hi
            (lo, ez, ey, n[2], n[1]),                 # x = lo
            (lo + ex, ey, ez, n[1], n[2]),            # x = hi
        ]
        start = len(self.v)
        for o, a, b, na, nb in faces:
            self.grid_quad(o, a, b, na, nb, obj)
        if yaw != 0.0:
            c = 0.5 * (lo + hi)
            cs, sn = math.cos(yaw), math.sin(yaw)
            for i in range(start, len(self.v)):
                d = self.v[i] - c
                x = cs * d[:, 0] - sn * d[:, 1]
                y = sn * d[:, 0] + cs * d[:, 1]
                self.v[i] = np.stack([x + c[0], y + c[1], self.v[i][:, 2]], 1)

    def cylinder(self, base, radius: float, height: float, facets: int, segs: int, obj: int):
        base = np.asarray(base, dtype=np.float64)
        ang = np.arange(facets) * (2 * math.pi / facets)
        ring = np.stack([radius * np.cos(ang), radius * np.sin(ang)], 1)
        zs = np.linspace(0.0, height, segs + 1)
        verts = np.concatenate([
            np.column_stack([ring[:, 0] + base[0], ring[:, 1] + base[1],
                             np.full(facets, base[2] + z)]) for z in zs])
        tris = []
        for s in range(segs):
            for f in range(facets):
                a = s * facets + f
                b = s * facets + (f + 1) % facets
                c = (s + 1) * facets + f
                d = (s + 1) * facets + (f + 1) % facets
                tris.append((a, b, d))
                tris.append((a, d, c))
        nv = verts.shape[0]
        centres = np.array([[base[0], base[1], base[2]], [base[0], base[1], base[2] + height]])
        verts = np.concatenate([verts, centres])
        for f in range(facets):
            tris.append((nv, (f + 1) % facets, f))
            top = segs * facets
            tris.append((nv + 1, top + f, top + (f + 1) % facets))
        self.add(verts, np.array(tris), obj)

    def build(self, obj_alpha, obj_vel, pt_pos=None, pt_vel=None, pt_ap=None) -> Scene:
        verts = np.concatenate(self.v) if self.v else np.zeros((0, 3))
        tris = np.concatenate(self.t) if self.t else np.zeros((0, 3), dtype=np.int64)
        tri_obj = np.concatenate(self.o) if self.o else np.zeros((0,), dtype=np.int32)
        npt = 0 if pt_pos is None else len(pt_pos)
        return Scene(
            verts=verts.astype(np.float32), tris=tris.astype(np.int32), tri_obj=tri_obj,
            obj_alpha=np.asarray(obj_alpha, dtype=np.float32),
            obj_vel=np.asarray(obj_vel, dtype=np.float64).reshape(-1, 3),
            pt_pos=np.zeros((0, 3)) if pt_pos is None else np.asarray(pt_pos, dtype=np.float64),
            pt_vel=np.zeros((npt, 3)) if pt_vel is None else np.asarray(pt_vel, dtype=np.float64),
            pt_aperture=np.zeros((npt,)) if pt_ap is None else np.asarray(pt_ap, dtype=np.float64),
        ).checked()


# ----------------------------------------------------------------------------
# arrays
# ----------------------------------------------------------------------------

def array_c1() -> Array:
    """1 Tx at (0, -2 lambda, 0.5); 4 Rx half-wavelength ULA centred on y = 0."""
    lam = LAMBDA77
    tx = np.array([[0.0, -2 * lam, 0.5]])
    rx = np.array([[0.0, (r - 1.5) * lam / 2, 0.5] for r in range(4)])
    return Array(tx, rx, 0.25, MODE_PER_TX).checked()


def array_square(n_side: int = 47, pitch: float = 3e-3, mode: int = MODE_SHARED,
                 rx_radius: float = 0.07) -> Array:
    """Square MIMO frame in the y-z plane centred on the origin: n_side
    elements at `pitch` on each side; Tx on the two sides y = -+L/2, Rx on the
    two sides z = -+L/2 (L = n_side * pitch), so 2 n_side x 2 n_side channels
    (94 x 94 for n_side = 47: a 14.1 cm aperture)."""
    s = (np.arange(n_side) - (n_side - 1) / 2) * pitch
    h = n_side * pitch / 2
    z = np.zeros(n_side)
    tx = np.concatenate([np.stack([z, np.full(n_side, -h), s], 1),
                         np.stack([z, np.full(n_side, h), s], 1)])
    rx = np.concatenate([np.stack([z, s, np.full(n_side, -h)], 1),
                         np.stack([z, s, np.full(n_side, h)], 1)])
    return Array(tx, rx, rx_radius, mode).checked()


def array_ula(n_tx: int, n_rx: int, mode: int = MODE_PER_TX, height: float = 0.5) -> Array:
    """Rx: n_rx ULA at lambda/2 along y; Tx: n_tx ULA at n_rx*lambda/2 (a filled
    virtual ULA), lifted by 2 lambda in z so that Tx and Rx elements do not coincide."""
    lam = LAMBDA77
    rx = np.array([[0.0, (r - (n_rx - 1) / 2) * lam / 2, height] for r in range(n_rx)])
    tx = np.array([[0.0, (t - (n_tx - 1) / 2) * n_rx * lam / 2, height + 2 * lam]
                   for t in range(n_tx)])
    return Array(tx, rx, 0.25, mode).checked()


def array_sparse_grid(n_tx: int, n_rx: int, seed: int, grid: int = 64,
                      mode: int = MODE_SHARED, height: float = 0.5) -> Array:
    """Tx and Rx drawn without replacement (disjoint) from a grid x grid lattice
    at lambda/2 in the y-z plane centred on (0, 0, height)."""
    lam = LAMBDA77
    rng = np.random.default_rng(seed)
    cells = rng.choice(grid * grid, size=n_tx + n_rx, replace=False)
    iy, iz = cells // grid, cells % grid
    pos = np.stack([np.zeros(len(cells)),
                    (iy - (grid - 1) / 2) * lam / 2,
                    (iz - (grid - 1) / 2) * lam / 2 + height], 1)
    return Array(pos[:n_tx], pos[n_tx:], 0.25, mode).checked()


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def _reflectors(rng, n, r_lo=5.0, r_hi=30.0, az_deg=30.0, z=0.5, keep_out=None):
    pts = []
    while len(pts) < n:
        r = rng.uniform(r_lo, r_hi)
        az = math.radians(rng.uniform(-az_deg, az_deg))
        p = np.array([r * math.cos(az), r * math.sin(az), z])
        if keep_out is not None and keep_out(p):
            continue
        pts.append(p)
    return np.array(pts)


def scene_c1(seed: int = 0) -> Scene:
    """Ground square +-100 m (2 triangles), a 1 m box centred at (10, 0, 0.5)
    moving +x at 5 m/s (12 triangles), 3 point reflectors at range U[5, 30] m,
    azimuth U[-30, 30] deg, height 0.5 m.  alpha = 0.5 everywhere."""
    rng = np.random.default_rng(seed)
    mb = _MeshBuilder()
    mb.grid_quad((-100.0, -100.0, 0.0), (200.0, 0.0, 0.0), (0.0, 200.0, 0.0), 1, 1, 0)
    mb.box((9.5, -0.5, 0.0), (10.5, 0.5, 1.0), None, 1)
    inside = lambda p: (9.3 < p[0] < 10.7) and (-0.7 < p[1] < 0.7)
    pts = _reflectors(rng, 3, keep_out=inside)
    return mb.build([0.5, 0.5], [[0, 0, 0], [5.0, 0, 0]], pts, np.zeros((3, 3)),
                    np.full(3, 0.01))


def scene_box_family(seed: int) -> Scene:
    """Scene family of the learned-proposal experiment: the tiny scene with the
    box at range U[5, 30] m, azimuth U[-30, 30] deg, yaw U[0, 90] deg and radial
    speed U[-5, 5] m/s, plus 3 reflectors as in the tiny scene."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(5.0, 30.0)
    az = math.radians(rng.uniform(-30.0, 30.0))
    yaw = math.radians(rng.uniform(0.0, 90.0))
    v = rng.uniform(-5.0, 5.0)
    cx, cy = r * math.cos(az), r * math.sin(az)
    mb = _MeshBuilder()
    mb.grid_quad((-100.0, -100.0, 0.0), (200.0, 0.0, 0.0), (0.0, 200.0, 0.0), 1, 1, 0)
    mb.box((cx - 0.5, cy - 0.5, 0.0), (cx + 0.5, cy + 0.5, 1.0), None, 1, yaw=yaw)
    inside = lambda p: math.hypot(p[0] - cx, p[1] - cy) < 1.0
    pts = _reflectors(rng, 3, keep_out=inside)
    vel = [[0, 0, 0], [v * math.cos(az), v * math.sin(az), 0.0]]
    return mb.build([0.5, 0.5], vel, pts, np.zeros((3, 3)), np.full(3, 0.01))


def scene_street(seed: int = 0, scale: float = 1.0, n_cars: int = 20, n_poles: int = 40) -> Scene:
    """Procedural street: ground x in [-10, 90] m, y in [-25, 25] m as a grid
    (500 x 200 cells at scale 1); n_cars box cars 4.5 x 1.8 x 1.5 m (0.2 m
    ground clearance, faces subdivided at 0.1 m) at seeded positions in
    x in [5, 65], y in [-7.5, 7.5] with v_x ~ U[-15, 15] m/s; n_poles
    cylinders r = 0.1 m, h = 4 m, 64 facets x 32 segments on the curbs
    y = +-8 m.  alpha ~ U[0, 1] per object.  At scale 1 this is 509 360
    triangles; `scale` multiplies the triangle count (mesh resolution) so the
    same generator spans 1e4..1e6 triangles."""
    rng = np.random.default_rng(seed)
    f = math.sqrt(scale)
    mb = _MeshBuilder()
    nx, ny = max(1, int(round(500 * f))), max(1, int(round(200 * f)))
    mb.grid_quad((-10.0, -25.0, 0.0), (100.0, 0.0, 0.0), (0.0, 50.0, 0.0), nx, ny, 0)
    alphas = [rng.uniform(0.0, 1.0)]
    vels = [[0.0, 0.0, 0.0]]
    placed: list[tuple[float, float]] = []
    obj = 1
    step = 0.1 / f
    while len(placed) < n_cars:
        x = rng.uniform(5.0, 65.0)
        y = rng.uniform(-7.5, 7.5)
        if any(abs(x - px) < 5.0 and abs(y - py) < 2.2 for px, py in placed):
            continue
        placed.append((x, y))
        mb.box((x - 2.25, y - 0.9, 0.2), (x + 2.25, y + 0.9, 1.7), step, obj)
        alphas.append(rng.uniform(0.0, 1.0))
        vels.append([rng.uniform(-15.0, 15.0), 0.0, 0.0])
        obj += 1
    facets = max(8, int(round(64 * f)))
    segs = max(1, int(round(32 * f)))
    for i in range(n_poles):
        side = 8.0 if i % 2 == 0 else -8.0
        x = rng.uniform(0.0, 80.0)
        mb.cylinder((x, side, 0.0), 0.1, 4.0, facets, segs, obj)
        alphas.append(rng.uniform(0.0, 1.0))
        vels.append([0.0, 0.0, 0.0])
        obj += 1
    return mb.build(alphas, vels)


def random_soup(n: int, seed: int, size: float = 0.2) -> Scene:
    """n random small triangles in the unit cube [1, 2]^3 (one object each,
    alpha = 0), for brute-force versus BVH checks."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 2.0, size=(n, 1, 3))
    v = c + rng.uniform(-size, size, size=(n, 3, 3))
    verts = v.reshape(-1, 3)
    tris = np.arange(3 * n).reshape(n, 3)
    return Scene(verts.astype(np.float32), tris.astype(np.int32), np.zeros(n, np.int32),
                 np.zeros(1, np.float32), np.zeros((1, 3))).checked()


def plate(distance: float, half: float, alpha: float = 0.0, normal_axis: int = 0) -> Scene:
    """A square plate of half-width `half` normal to +x at x = distance (2 triangles)."""
    mb = _MeshBuilder()
    mb.grid_quad((distance, -half, -half + 0.5), (0.0, 2 * half, 0.0), (0.0, 0.0, 2 * half), 1, 1, 0)
    return mb.build([alpha], [[0.0, 0.0, 0.0]])


def point_only(pos, vel=None, aperture=0.01) -> Scene:
    """A scene with no triangles and point reflectors only."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    vel = np.zeros_like(pos) if vel is None else np.asarray(vel, dtype=np.float64).reshape(-1, 3)
    ap = np.full(pos.shape[0], aperture) if np.isscalar(aperture) else np.asarray(aperture)
    return Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), np.zeros(0, np.int32),
                 np.zeros(1, np.float32), np.zeros((1, 3)), pos, vel, ap).checked()


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def workload_tiny(seed: int = 0) -> Workload:
    """Ground + 1 m box at 10 m moving 5 m/s + 3 reflectors; 77 GHz, 1 GHz,
    50 us, 64 samples x 16 chirps; 1 Tx x 4 Rx; 1e5 uniform rays, 2 bounces."""
    return Workload("tiny", scene_c1(seed), array_c1(), Chirp(n_samples=64, n_chirps=16),
                    TraceParams(n_rays=100_000, max_bounces=2, seed=seed))


def workload_street(seed: int = 0, n_rays: int = 10_000_000) -> Workload:
    """Street (~5.1e5 triangles); 12 Tx x 16 Rx ULA (192 channels); 256 samples
    x 128 chirps; 1e7 rays, 3 bounces."""
    return Workload("street", scene_street(seed), array_ula(12, 16),
                    Chirp(n_samples=256, n_chirps=128),
                    TraceParams(n_rays=n_rays, max_bounces=3, seed=seed))


LARGE_MIMO_RAYS = 4_000_000
LARGE_MIMO_PATHS = 100_000


def workload_large_mimo(seed: int = 0, n_rays: int = LARGE_MIMO_RAYS,
                        path_cap: int = LARGE_MIMO_PATHS) -> Workload:
    """Street, 48 Tx x 64 Rx sparse array on a 64 x 64 lambda/2 grid (3072
    channels), shared launch from the Tx phase centre, 512 samples x 256
    chirps, the first ~1e5 returned paths."""
    return Workload("large_mimo", scene_street(seed), array_sparse_grid(48, 64, seed + 17),
                    Chirp(n_samples=512, n_chirps=256),
                    TraceParams(n_rays=n_rays, max_bounces=3, seed=seed), path_cap)


def workload_batch(n_scenes: int = 64, seed0: int = 2000, rays: int = 1_000_000,
                   tri_lo: float = 1e4, tri_hi: float = 1e6, ch_hi: int = 3072) -> list[Workload]:
    """Uneven batch: triangle counts log-uniform in [tri_lo, tri_hi], channel
    counts log-uniform in [4, ch_hi] (n_rx = min(64, ceil(sqrt C)),
    n_tx = ceil(C / n_rx)), samples in {128, 256, 512}, chirps in {64, 128, 256}."""
    out = []
    for i in range(n_scenes):
        s = seed0 + i
        rng = np.random.default_rng(s)
        tris = math.exp(rng.uniform(math.log(tri_lo), math.log(tri_hi)))
        ch = math.exp(rng.uniform(math.log(4), math.log(ch_hi)))
        n_rx = min(64, int(math.ceil(math.sqrt(ch))))
        n_tx = max(1, int(math.ceil(ch / n_rx)))
        K = int(rng.choice([128, 256, 512]))
        M = int(rng.choice([64, 128, 256]))
        scale = tris / 509_360.0
        n_cars = 20 if scale > 0.05 else 5
        n_poles = 40 if scale > 0.05 else 10
        scene = scene_street(s, scale=scale, n_cars=n_cars, n_poles=n_poles)
        arr = array_sparse_grid(n_tx, n_rx, s + 17, mode=MODE_SHARED)
        out.append(Workload(f"batch{i}", scene, arr, Chirp(n_samples=K, n_chirps=M),
                            TraceParams(n_rays=rays, max_bounces=3, seed=s)))
    return out


def _hand_builder(seed: int, step: float, rng_x: float):
    """Mesh builder of the hand proxy and the vertex range of each part
    (palm, four fingers, thumb)."""
    rng = np.random.default_rng(seed)
    mb = _MeshBuilder()
    t = 0.015
    parts = []

    def part(lo, hi):
        a = mb.nv
        mb.box(lo, hi, step, 0)
        parts.append((a, mb.nv))

    part((rng_x, -0.04, -0.05), (rng_x + t, 0.04, 0.04))
    for i in range(4):
        y0 = -0.038 + i * 0.0195
        w = 0.016 + 0.002 * rng.random()
        ln = 0.06 + 0.025 * rng.random()
        part((rng_x + 0.002, y0, 0.04), (rng_x + t - 0.002, y0 + w, 0.04 + ln))
    ln = 0.05 + 0.015 * rng.random()
    part((rng_x + 0.002, 0.04, -0.03), (rng_x + t - 0.002, 0.04 + ln, -0.012))
    return mb, parts


def scene_hand_proxy(seed: int = 0, step: float = 2e-3, rng_x: float = 0.30,
                     alpha: float = 0.3) -> Scene:
    """A static open hand facing the array: a palm (8 cm wide, 9 cm tall,
    1.5 cm thick) at range rng_x and five fingers (1.6-1.8 cm wide) above it,
    lengths and spread drawn from `seed`, the thumb to the side; faces
    subdivided at `step`.  One object, material alpha."""
    mb, _ = _hand_builder(seed, step, rng_x)
    return mb.build([alpha], [[0.0, 0.0, 0.0]])


def hand_motion(seed: int = 0, n_frames: int = 32, step: float = 2e-3, rng_x: float = 0.30,
                alpha: float = 0.3, curl_deg: float = 70.0, drift: float = 0.01):
    """The hand proxy moving: over n_frames (one period), finger i curls
    towards the array about its knuckle line (the y axis through the finger's
    base at the palm's mid-thickness) by curl_deg (1 - cos(2 pi f / n + i pi / 4)) / 2,
    the thumb swings about its base (the z axis) by half that, and the whole
    hand drifts by drift sin(2 pi f / n) along y.  Returns (scene at frame 0,
    [float32 vertex arrays of frames 0..n-1]); the topology never changes."""
    mb, parts = _hand_builder(seed, step, rng_x)
    scene = mb.build([alpha], [[0.0, 0.0, 0.0]])
    base = np.concatenate(mb.v).astype(np.float64)
    cx = rng_x + 0.0075
    frames = []
    for f in range(n_frames):
        v = base.copy()
        ph = 2 * math.pi * f / n_frames
        for i in range(4):
            a, b = parts[1 + i]
            th = math.radians(curl_deg) * (1 - math.cos(ph + i * math.pi / 4)) / 2
            dx, dz = v[a:b, 0] - cx, v[a:b, 2] - 0.04
            v[a:b, 0] = cx + dx * math.cos(th) - dz * math.sin(th)
            v[a:b, 2] = 0.04 + dz * math.cos(th) + dx * math.sin(th)
        a, b = parts[5]
        th = 0.5 * math.radians(curl_deg) * (1 - math.cos(ph)) / 2
        dx, dy = v[a:b, 0] - cx, v[a:b, 1] - 0.04
        v[a:b, 0] = cx + dx * math.cos(th) - dy * math.sin(th)
        v[a:b, 1] = 0.04 + dy * math.cos(th) + dx * math.sin(th)
        v[:, 1] += drift * math.sin(ph)
        frames.append(v.astype(np.float32))
    return with_verts(scene, frames[0]), frames


def with_verts(scene: Scene, verts) -> Scene:
    """The same scene (topology, objects, materials) with new vertex positions."""
    return Scene(np.asarray(verts, np.float32), scene.tris, scene.tri_obj, scene.obj_alpha,
                 scene.obj_vel, scene.pt_pos, scene.pt_vel, scene.pt_aperture,
                 scene.tri_alpha).checked()


def workload_hand(seed: int = 0, n_rays: int = 10_000_000) -> Workload:
    """The paper's imaging set-up with a synthetic hand: the 94 x 94 square
    array (shared launch from its centre, reception sphere 7 cm), a
    72-82 GHz stepped-frequency sweep of 128 steps, rays within +-25 degrees
    of boresight, 2 bounces."""
    deg = math.pi / 180.0
    return Workload("hand", scene_hand_proxy(seed), array_square(), chirp_sfcw(),
                    TraceParams(n_rays=n_rays, max_bounces=2, seed=seed, az_min=-25 * deg,
                                az_max=25 * deg, el_min=-25 * deg, el_max=25 * deg))


def with_alpha(scene: Scene, alpha: float) -> Scene:
    """The same scene with every object (and no face override) at one alpha."""
    return Scene(scene.verts, scene.tris, scene.tri_obj,
                 np.full(scene.n_obj, alpha, dtype=np.float32), scene.obj_vel, scene.pt_pos,
                 scene.pt_vel, scene.pt_aperture).checked()


def alpha_sweep(lo: float = 0.0, hi: float = 1.0, step: float = 0.1) -> list[float]:
    """Alpha values lo, lo + step, ..., hi (the paper's sweep: 0 to 1 by 0.1),
    each rounded to float32 as the scene stores it."""
    n = int(round((hi - lo) / step)) + 1
    return [float(np.float32(lo + i * step)) for i in range(n)]


def vary_alpha(scene: Scene, seed: int, spread: float = 0.2) -> Scene:
    """Per-face alpha for data diversity: each face draws its own mix
    uniformly within +-spread of its object's, clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    base = scene.obj_alpha[scene.tri_obj].astype(np.float64)
    ta = np.clip(base + rng.uniform(-spread, spread, scene.n_tris), 0.0, 1.0)
    return Scene(scene.verts, scene.tris, scene.tri_obj, scene.obj_alpha, scene.obj_vel,
                 scene.pt_pos, scene.pt_vel, scene.pt_aperture,
                 ta.astype(np.float32)).checked()


def imaging_grid(x_lo: float = 0.26, x_hi: float = 0.34, half: float = 0.10,
                 step: float = 1e-3):
    """Voxel grid of the imaging volume: range x in [x_lo, x_hi], y and z in
    [-half, half], spacing `step`; returns (origin, step, (nx, ny, nz))."""
    nx = int(round((x_hi - x_lo) / step)) + 1
    ny = nz = int(round(2 * half / step)) + 1
    return (x_lo, -half, -half), step, (nx, ny, nz)


def workload_box_mimo(seed: int, n_rays: int) -> Workload:
    """A box-family scene (no point reflectors) seen by the large-MIMO array
    (48 Tx x 64 Rx from the 64 x 64 grid, shared launch) moved so that its Tx
    and Rx phase centres sit where the tiny array's Tx and Rx centre are;
    512 samples x 256 chirps, 2 bounces."""
    c1 = array_c1()
    big = array_sparse_grid(48, 64, seed + 17)
    tx = big.tx - big.tx.mean(axis=0) + c1.tx.mean(axis=0)
    rx = big.rx - big.rx.mean(axis=0) + c1.rx.mean(axis=0)
    sc = scene_box_family(seed)
    sc = Scene(sc.verts, sc.tris, sc.tri_obj, sc.obj_alpha, sc.obj_vel).checked()
    return Workload(f"boxmimo{seed}", sc, Array(tx, rx, c1.rx_radius, MODE_SHARED).checked(),
                    Chirp(n_samples=512, n_chirps=256),
                    TraceParams(n_rays=n_rays, max_bounces=2, seed=seed))


def workload_box_family(seed: int, n_rays: int, points: bool = True) -> Workload:
    """One scene of the learned-proposal family with the tiny scene's array
    and chirp, 2 bounces (points=False drops the point reflectors, leaving
    only the traced part of the cube)."""
    sc = scene_box_family(seed)
    if not points:
        sc = Scene(sc.verts, sc.tris, sc.tri_obj, sc.obj_alpha, sc.obj_vel).checked()
    return Workload(f"box{seed}", sc, array_c1(), Chirp(n_samples=64, n_chirps=16),
                    TraceParams(n_rays=n_rays, max_bounces=2, seed=seed))
