"""Seeded synthetic scenes and sensor models for the S-BKI map update.

This module produces *inputs only*: labelled hit points (float32 xyz, int32
class id), sensor origins and the hyper-parameters each workload runs with.
It holds none of the mapping method's arithmetic (no free-space sampling, no
kernel, no cell keys); both the CPU oracle and the GPU library consume what it
returns.  The paper's own datasets (KITTI stereo, SemanticKITTI LiDAR, a
town-scale map) are not available, so every workload here is a ray-cast
synthetic scene that only takes the *shape* of those workloads: sensor
geometry, point counts, range cuts, noise and class count.

Class id 0 is reserved for the free-space class; hits carry occupied class ids
1..K-1.  Label -1 marks a point the caller wants dropped.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Params", "Scan", "Scene", "World",
    "tiny_scene", "lidar_scan_scene", "stereo_sequence_scene",
    "batched_town_scene", "differentiable_scene", "random_points_scene",
    "make_config", "CONFIG_NAMES",
]


# ---------------------------------------------------------------------------
# containers
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Params:
    """Map and kernel hyper-parameters (all binary32 on the library boundary)."""
    res: float = 0.1          # voxel edge [m]
    block_size: int = 8       # voxels per block edge
    l: float = 0.3            # kernel length-scale [m]
    sigma0: float = 0.1       # kernel scale
    alpha0: float = 0.001     # Dirichlet prior concentration (every class)
    K: int = 20               # classes, including the free class
    free_class: int = 0       # index of the free-space class
    free_step: float = 0.3    # spacing of free-space samples along a beam [m]

    def f32(self) -> "Params":
        """Round every real parameter to binary32 (the boundary's precision)."""
        q = dataclasses.replace(self)
        for name in ("res", "l", "sigma0", "alpha0", "free_step"):
            setattr(q, name, float(np.float32(getattr(self, name))))
        return q


@dataclasses.dataclass
class Scan:
    xyz: np.ndarray        # float32 [N, 3], world frame, metres
    label: np.ndarray      # int32 [N]
    origin: np.ndarray     # float32 [3], sensor origin of every beam of the scan


@dataclasses.dataclass
class Scene:
    name: str
    params: Params
    scans: List[Scan]
    query_ijk: Optional[np.ndarray] = None     # int32 [M, 3] voxel indices to read out
    holdout: Optional[Scan] = None             # held-out labelled hits (differentiable form)
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_hits(self) -> int:
        return int(sum(s.xyz.shape[0] for s in self.scans))

    def concat(self):
        """Concatenate scans: (xyz, label, offsets int64[S+1], origins f32[S,3])."""
        xyz = np.concatenate([s.xyz for s in self.scans]).astype(np.float32)
        lab = np.concatenate([s.label for s in self.scans]).astype(np.int32)
        off = np.zeros(len(self.scans) + 1, dtype=np.int64)
        off[1:] = np.cumsum([s.xyz.shape[0] for s in self.scans])
        org = np.stack([s.origin for s in self.scans]).astype(np.float32)
        return xyz, lab, off, org


# ---------------------------------------------------------------------------
# geometry: a tiny ray caster over planes, boxes, vertical cylinders, ellipsoids
# ---------------------------------------------------------------------------
class World:
    """A set of labelled primitives that rays can be cast against."""

    def __init__(self):
        self.planes = []      # (height z, class-or-callable)
        self.boxes = []       # (lo[3], hi[3], class)
        self.cyls = []        # (cx, cy, r, z0, z1, class)
        self.ellipsoids = []  # (centre[3], radii[3], class)

    def add_plane(self, z, cls):
        self.planes.append((float(z), cls))

    def add_box(self, lo, hi, cls):
        self.boxes.append((np.asarray(lo, np.float64), np.asarray(hi, np.float64), int(cls)))

    def add_cylinder(self, cx, cy, r, z0, z1, cls):
        self.cyls.append((float(cx), float(cy), float(r), float(z0), float(z1), int(cls)))

    def add_ellipsoid(self, c, radii, cls):
        self.ellipsoids.append((np.asarray(c, np.float64), np.asarray(radii, np.float64), int(cls)))

    def near(self, o, radius: float) -> "World":
        """The primitives that can be hit from o within `radius` (planes kept):
        casting from o with tmax <= radius against this subset gives the same
        result as against the whole world."""
        o = np.asarray(o, np.float64)
        w = World()
        w.planes = list(self.planes)

        def close(lo, hi):
            q = np.clip(o, lo, hi)
            return float(np.linalg.norm(q - o)) <= radius

        w.boxes = [b for b in self.boxes if close(b[0], b[1])]
        w.cyls = [c for c in self.cyls
                  if close(np.array([c[0] - c[2], c[1] - c[2], c[3]]),
                           np.array([c[0] + c[2], c[1] + c[2], c[4]]))]
        w.ellipsoids = [e for e in self.ellipsoids if close(e[0] - e[1], e[0] + e[1])]
        return w

    def cast(self, o: np.ndarray, d: np.ndarray, tmax: float = np.inf):
        """Nearest hit along rays o + t d (o [3] or [R,3], d [R,3] unit).

        Returns (t [R] float64, cls [R] int32); t = inf / cls = -1 where nothing
        is hit before tmax.
        """
        d = np.asarray(d, np.float64)
        R = d.shape[0]
        o = np.broadcast_to(np.asarray(o, np.float64), (R, 3))
        best_t = np.full(R, np.inf)
        best_c = np.full(R, -1, dtype=np.int32)
        eps = 1e-9

        def take(t, cls):
            nonlocal best_t, best_c
            better = (t > eps) & (t < best_t) & (t <= tmax)
            best_t = np.where(better, t, best_t)
            if callable(cls):
                p = o + np.where(np.isfinite(t), t, 0.0)[:, None] * d
                c = cls(p)
                best_c = np.where(better, c, best_c)
            else:
                best_c = np.where(better, cls, best_c)

        for z, cls in self.planes:
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (z - o[:, 2]) / d[:, 2]
            t = np.where(np.isfinite(t) & (t > 0), t, np.inf)
            take(t, cls)

        for lo, hi, cls in self.boxes:
            with np.errstate(divide="ignore", invalid="ignore"):
                inv = 1.0 / d
                t0 = (lo - o) * inv
                t1 = (hi - o) * inv
            tn = np.nanmax(np.minimum(t0, t1), axis=1)
            tf = np.nanmin(np.maximum(t0, t1), axis=1)
            hit = (tf >= tn) & (tf > eps)
            t = np.where(hit, np.where(tn > eps, tn, np.inf), np.inf)
            take(t, cls)

        for cx, cy, r, z0, z1, cls in self.cyls:
            ox = o[:, 0] - cx
            oy = o[:, 1] - cy
            a = d[:, 0] ** 2 + d[:, 1] ** 2
            b = 2 * (ox * d[:, 0] + oy * d[:, 1])
            c = ox ** 2 + oy ** 2 - r * r
            disc = b * b - 4 * a * c
            ok = (disc >= 0) & (a > 1e-12)
            sq = np.sqrt(np.where(ok, disc, 0))
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (-b - sq) / (2 * a)
            z = o[:, 2] + t * d[:, 2]
            t = np.where(ok & (z >= z0) & (z <= z1) & (t > eps), t, np.inf)
            take(t, cls)
            # top cap
            with np.errstate(divide="ignore", invalid="ignore"):
                tc = (z1 - o[:, 2]) / d[:, 2]
            px = ox + tc * d[:, 0]
            py = oy + tc * d[:, 1]
            tc = np.where(np.isfinite(tc) & (tc > eps) & (px * px + py * py <= r * r), tc, np.inf)
            take(tc, cls)

        for cen, rad, cls in self.ellipsoids:
            oo = (o - cen) / rad
            dd = d / rad
            a = np.sum(dd * dd, axis=1)
            b = 2 * np.sum(oo * dd, axis=1)
            c = np.sum(oo * oo, axis=1) - 1
            disc = b * b - 4 * a * c
            ok = disc >= 0
            sq = np.sqrt(np.where(ok, disc, 0))
            t = (-b - sq) / (2 * a)
            t = np.where(ok & (t > eps), t, np.inf)
            take(t, cls)

        return best_t, best_c


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _flip_labels(rng, lab, frac, k_lo, k_hi):
    """Replace a fraction of labels by a different uniform class in [k_lo, k_hi]."""
    lab = lab.copy()
    m = rng.random(lab.shape[0]) < frac
    n = int(m.sum())
    span = k_hi - k_lo + 1
    shift = rng.integers(1, span, size=n)
    lab[m] = (lab[m] - k_lo + shift) % span + k_lo
    return lab


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def tiny_scene(seed: int = 0, n_hits: int = 2000) -> Scene:
    """Ground plane + 3 boxes inside a 3.2 m cube, 3 occupied classes + free.

    Shape of the paper's three-class toy example (ground / wall / obstacle),
    scaled to a cube the CPU oracle maps in seconds: origin (0, 0, 1.5),
    seeded uniform beam directions, the first `n_hits` beams whose first
    return lies inside [-1.6, 1.6]^2 x [0, 3.2].  K = 4, free step 0.1 m,
    0.1 m voxels, query grid 32^3 (i, j in [-16, 15], k in [0, 31]),
    l = 0.3 m, sigma0 = 1.0, alpha0 = 0.001.
    """
    rng = np.random.default_rng(seed)
    w = World()
    w.add_plane(0.0, 1)
    # three boxes well clear of the sensor at (0, 0, 1.5)
    centres = [(-0.95, -0.7), (0.9, 0.35), (-0.1, 1.05)]
    classes = [2, 2, 3]
    for (cx, cy), cls in zip(centres, classes):
        jx, jy = rng.uniform(-0.12, 0.12, size=2)
        hx, hy = rng.uniform(0.22, 0.4, size=2)
        h = rng.uniform(0.8, 2.6)
        w.add_box((cx + jx - hx, cy + jy - hy, 0.0), (cx + jx + hx, cy + jy + hy, h), cls)
    origin = np.array([0.0, 0.0, 1.5])
    pts, labs = [], []
    need = n_hits
    while need > 0:
        m = 4 * need + 64
        d = rng.normal(size=(m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        t, c = w.cast(origin, d)
        p = origin + t[:, None] * d
        inside = (np.isfinite(t) & (np.abs(p[:, 0]) <= 1.6) & (np.abs(p[:, 1]) <= 1.6)
                  & (p[:, 2] >= 0.0) & (p[:, 2] <= 3.2))
        p, c = p[inside], c[inside]
        pts.append(p[:need])
        labs.append(c[:need])
        need -= min(need, p.shape[0])
    xyz = _f32(np.concatenate(pts))
    lab = np.concatenate(labs).astype(np.int32)
    params = Params(res=0.1, block_size=8, l=0.3, sigma0=1.0, alpha0=0.001, K=4,
                    free_class=0, free_step=0.1)
    g = np.arange(-16, 16)
    k = np.arange(0, 32)
    I, J, Kk = np.meshgrid(g, g, k, indexing="ij")
    q = np.stack([I.ravel(), J.ravel(), Kk.ravel()], axis=1).astype(np.int32)
    return Scene("tiny", params, [Scan(xyz, lab, _f32(origin))], query_ijk=q,
                 info={"seed": seed})


def _street_world(rng, length=120.0, n_classes=19):
    """A street along x: road, raised sidewalks, two building rows, cars, poles,
    vegetation (canopies on trunks and shrubs).  Class ids 1..n_classes."""
    w = World()
    # class map (ids are only labels; which id goes to which primitive kind is arbitrary)
    ROAD, SIDEWALK, TERRAIN, BUILDING, CAR, POLE, VEG, TRUNK, SIGN, FENCE = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10
    # further vehicle / object classes (with 10 classes, cars and signs stand in)
    extra = list(range(11, n_classes + 1)) or [CAR, SIGN]

    def ground_cls(p):
        ay = np.abs(p[:, 1])
        return np.where(ay < 5.0, ROAD, TERRAIN).astype(np.int32)

    w.add_plane(0.0, ground_cls)
    L = length
    for side in (-1, 1):
        # sidewalk slab
        y0, y1 = sorted((side * 5.0, side * 8.0))
        w.add_box((-L, y0, 0.0), (L, y1, 0.15), SIDEWALK)
        # buildings
        x = -L
        while x < L:
            blen = rng.uniform(8.0, 25.0)
            back = rng.uniform(8.0, 15.0)
            depth = rng.uniform(8.0, 14.0)
            h = rng.uniform(4.0, 20.0)
            ya, yb = sorted((side * back, side * (back + depth)))
            cls = BUILDING if rng.random() < 0.8 else FENCE
            w.add_box((x, ya, 0.0), (x + blen, yb, h if cls == BUILDING else 1.8), cls)
            x += blen + rng.uniform(1.0, 6.0)
        # parked cars / other vehicles
        x = -L + rng.uniform(0, 6)
        while x < L:
            clen = rng.uniform(3.8, 5.2)
            yc = side * rng.uniform(3.4, 4.2)
            cls = CAR if rng.random() < 0.7 else int(rng.choice(extra))
            w.add_box((x, yc - 0.9, 0.0), (x + clen, yc + 0.9, rng.uniform(1.3, 1.8)), cls)
            x += clen + rng.uniform(1.5, 12.0)
        # poles and signs
        x = -L + rng.uniform(0, 10)
        while x < L:
            yp = side * rng.uniform(6.0, 7.5)
            w.add_cylinder(x, yp, rng.uniform(0.08, 0.2), 0.0, rng.uniform(4.0, 8.0), POLE)
            if rng.random() < 0.4:
                w.add_box((x - 0.35, yp - 0.05, 2.2), (x + 0.35, yp + 0.05, 2.9), SIGN)
            x += rng.uniform(8.0, 20.0)
        # trees: trunk + canopy, and shrubs
        x = -L + rng.uniform(0, 8)
        while x < L:
            yt = side * rng.uniform(7.0, 9.5)
            th = rng.uniform(2.0, 3.5)
            w.add_cylinder(x, yt, rng.uniform(0.12, 0.3), 0.0, th, TRUNK)
            w.add_ellipsoid((x, yt, th + 1.2), (rng.uniform(1.2, 2.5), rng.uniform(1.2, 2.5),
                                                 rng.uniform(1.0, 2.0)), VEG)
            if rng.random() < 0.5:
                w.add_ellipsoid((x + rng.uniform(-3, 3), side * rng.uniform(8.2, 9.8), 0.4),
                                (rng.uniform(0.5, 1.2), rng.uniform(0.4, 0.8), 0.6), VEG)
            x += rng.uniform(6.0, 16.0)
    # a few people / bikes on the sidewalks
    for _ in range(12):
        x = rng.uniform(-L * 0.5, L * 0.5)
        y = rng.choice([-1, 1]) * rng.uniform(5.5, 7.5)
        w.add_cylinder(x, y, 0.25, 0.0, rng.uniform(1.5, 1.9), int(rng.choice(extra)))
    return w


def _lidar_dirs(n_beams=64, n_az=2048, el_lo=-25.0, el_hi=3.0, yaw=0.0):
    el = np.deg2rad(np.linspace(el_lo, el_hi, n_beams))
    az = yaw + np.arange(n_az) * (2 * np.pi / n_az)
    E, A = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1)
    return d.reshape(-1, 3)


def _lidar_returns(rng, world, origin, dirs, rmin=2.0, rmax=50.0, sigma=0.02, chunk=1 << 16):
    ts, cs = [], []
    world = world.near(origin, rmax + 1.0)
    for i in range(0, dirs.shape[0], chunk):
        t, c = world.cast(origin, dirs[i:i + chunk], tmax=rmax + 1.0)
        ts.append(t)
        cs.append(c)
    t = np.concatenate(ts)
    c = np.concatenate(cs)
    t = t + rng.normal(0.0, sigma, size=t.shape)
    keep = np.isfinite(t) & (t >= rmin) & (t <= rmax) & (c >= 0)
    p = origin + t[keep, None] * dirs[keep]
    return p, c[keep].astype(np.int32)


def lidar_scan_scene(seed: int = 1, flip: float = 0.10) -> Scene:
    """One spinning-LiDAR-shaped scan over a street.

    64 beams uniform in elevation [-25, +3] deg, 2048 azimuth steps, sensor at
    (0, 0, 1.73), returns kept for 2 <= range <= 50 m, Gaussian range noise
    sigma = 2 cm; 19 occupied classes + free (K = 20) with 10 % uniform label
    flips among occupied classes (stand-in for network label noise); free
    step 0.3 m; 0.1 m voxels in 8^3 blocks; l = 0.3 m, sigma0 = 0.1,
    alpha0 = 0.001.  About 1.2e5 hits.
    """
    rng = np.random.default_rng(seed)
    w = _street_world(rng)
    origin = np.array([0.0, 0.0, 1.73])
    p, c = _lidar_returns(rng, w, origin, _lidar_dirs())
    c = _flip_labels(rng, c, flip, 1, 19)
    params = Params(res=0.1, block_size=8, l=0.3, sigma0=0.1, alpha0=0.001, K=20,
                    free_class=0, free_step=0.3)
    return Scene("lidar", params, [Scan(_f32(p), c.astype(np.int32), _f32(origin))],
                 info={"seed": seed})


_STEREO = {}   # the sequence being generated (read by forked workers)


def _stereo_scan(s: int) -> Scan:
    c = _STEREO
    origin = np.array([c["x0"] + s * c["step"], 0.0, 1.65])
    rng = np.random.default_rng([c["seed"], s])   # scan s is reproducible on its own
    zmax = c["zmax"]
    dirs_u, norms = c["dirs_u"], c["norms"]
    ws = c["world"].near(origin, zmax * 1.5)
    t, cl = [], []
    for i in range(0, dirs_u.shape[0], 1 << 16):
        ti, ci = ws.cast(origin, dirs_u[i:i + (1 << 16)], tmax=zmax * 1.5)
        t.append(ti)
        cl.append(ci)
    t = np.concatenate(t)
    cl = np.concatenate(cl)
    with np.errstate(invalid="ignore"):
        z = t / norms                      # depth along the optical axis
        z = z + rng.normal(0.0, 1.0, size=z.shape) * 5e-4 * z * z
    keep = np.isfinite(z) & (z > 0.5) & (z <= zmax) & (cl >= 0)
    p = origin + (z[keep] * norms[keep])[:, None] * dirs_u[keep]
    lab = _flip_labels(rng, cl[keep].astype(np.int32), c["flip"], 1, 10)
    return Scan(_f32(p), lab, _f32(origin))


def stereo_sequence_scene(seed: int = 2, n_scans: int = 100, width: int = 1242,
                          height: int = 375, focal: float = 720.0, zmax: float = 25.0,
                          step: float = 1.0, flip: float = 0.10, first: int = None,
                          workers: int = 1) -> Scene:
    """Stereo-shaped dense scans along a street, one persistent map.

    Pinhole camera width x height, focal length `focal` px, centred principal
    point, 1.65 m high, looking along +x; depth from ray casting with noise
    sigma_z = 5e-4 z^2 (growing quadratically with depth), cut at 25 m;
    10 occupied classes + free (K = 11); `n_scans` poses 1 m apart along +x;
    0.1 m voxels, l = 0.3, sigma0 = 0.1, free step 0.3 m.  Only the first
    `first` scans of the sequence are generated when it is given (each scan has
    its own seeded generator, so they equal those of the whole sequence);
    `workers` > 1 casts scans in forked worker processes.
    """
    rng = np.random.default_rng(seed)
    w = _street_world(rng, length=max(120.0, n_scans * step + 60.0), n_classes=10)
    u = np.arange(width) + 0.5
    v = np.arange(height) + 0.5
    U, V = np.meshgrid(u, v, indexing="xy")
    cam = np.stack([(U - width / 2) / focal, (V - height / 2) / focal, np.ones_like(U)], axis=-1)
    cam = cam.reshape(-1, 3)
    # camera frame (x right, y down, z forward) -> world (x forward, y left, z up)
    dirs = np.stack([cam[:, 2], -cam[:, 0], -cam[:, 1]], axis=1)
    norms = np.linalg.norm(dirs, axis=1)
    _STEREO.clear()
    _STEREO.update(world=w, dirs_u=dirs / norms[:, None], norms=norms, zmax=zmax, step=step,
                   x0=-0.5 * n_scans * step, seed=seed, flip=flip)
    todo = list(range(n_scans if first is None else min(first, n_scans)))
    if workers > 1 and len(todo) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(todo))) as pool:
            scans = pool.map(_stereo_scan, todo, chunksize=1)
    else:
        scans = [_stereo_scan(s) for s in todo]
    _STEREO.clear()
    params = Params(res=0.1, block_size=8, l=0.3, sigma0=0.1, alpha0=0.001, K=11,
                    free_class=0, free_step=0.3)
    return Scene("stereo", params, scans, info={"seed": seed, "n_scans": n_scans})


def _town_world(rng, size=200.0, height=10.0):
    """A size x size town: a grid of streets with buildings, cars, poles, trees."""
    w = World()

    def ground_cls(p):
        gx = np.mod(p[:, 0], 40.0)
        gy = np.mod(p[:, 1], 40.0)
        street = (gx < 10.0) | (gy < 10.0)
        return np.where(street, 1, 3).astype(np.int32)

    w.add_plane(0.0, ground_cls)
    half = size / 2
    for bx in np.arange(-half, half, 40.0):
        for by in np.arange(-half, half, 40.0):
            # one lot per 40 m cell, streets along its low x / y edges
            x0, y0 = bx + 10.0, by + 10.0
            n = rng.integers(1, 4)
            for _ in range(n):
                lx, ly = rng.uniform(6, 14, size=2)
                ox, oy = rng.uniform(0, 30 - lx), rng.uniform(0, 30 - ly)
                w.add_box((x0 + ox, y0 + oy, 0.0), (x0 + ox + lx, y0 + oy + ly,
                                                    rng.uniform(3.0, height)), 4)
            for _ in range(rng.integers(2, 6)):
                cx = bx + rng.uniform(0, 40)
                cy = by + rng.uniform(1.0, 9.0)
                w.add_box((cx, cy, 0.0), (cx + 4.5, cy + 1.8, 1.5), int(rng.choice([5, 11, 12, 13])))
            for _ in range(rng.integers(1, 4)):
                px, py = bx + rng.uniform(0, 40), by + rng.uniform(8.5, 9.8)
                w.add_cylinder(px, py, 0.15, 0.0, rng.uniform(4, 7), 6)
            for _ in range(rng.integers(1, 4)):
                tx, ty = bx + rng.uniform(10, 40), by + rng.uniform(10, 40)
                w.add_cylinder(tx, ty, 0.25, 0.0, 2.5, 8)
                w.add_ellipsoid((tx, ty, 3.5), (2.0, 2.0, 1.5), 7)
            for _ in range(rng.integers(0, 3)):
                w.add_cylinder(bx + rng.uniform(0, 40), by + rng.uniform(0, 10), 0.25, 0.0, 1.8,
                               int(rng.choice([14, 15, 16, 17, 18, 19])))
    return w


def batched_town_scene(seed: int = 3, n_scans: int = 64, n_lo: int = 10_000,
                       n_hi: int = 130_000, flip: float = 0.10) -> Scene:
    """`n_scans` LiDAR scans of uneven size from random street poses in a
    200 x 200 x 10 m town.  Per scan N ~ U[n_lo, n_hi] returns are kept by
    seeded subsampling of the spinning-LiDAR model; random yaw.  K = 20,
    0.2 m voxels, 8^3 blocks, l = 0.3, sigma0 = 0.1, free step 0.3 m."""
    rng = np.random.default_rng(seed)
    w = _town_world(rng)
    scans = []
    for s in range(n_scans):
        # pose on a street (street cells are the low 10 m of each 40 m period)
        if rng.random() < 0.5:
            x = rng.uniform(-100, 100)
            y = -100 + 40 * rng.integers(0, 5) + rng.uniform(2, 8)
        else:
            y = rng.uniform(-100, 100)
            x = -100 + 40 * rng.integers(0, 5) + rng.uniform(2, 8)
        origin = np.array([x, y, 1.73])
        dirs = _lidar_dirs(yaw=rng.uniform(0, 2 * np.pi))
        p, c = _lidar_returns(rng, w, origin, dirs)
        n = int(rng.integers(n_lo, n_hi + 1))
        if p.shape[0] > n:
            idx = np.sort(rng.choice(p.shape[0], size=n, replace=False))
            p, c = p[idx], c[idx]
        c = _flip_labels(rng, c, flip, 1, 19)
        scans.append(Scan(_f32(p), c.astype(np.int32), _f32(origin)))
    params = Params(res=0.2, block_size=8, l=0.3, sigma0=0.1, alpha0=0.001, K=20,
                    free_class=0, free_step=0.3)
    return Scene("batched", params, scans, info={"seed": seed})


def differentiable_scene(seed: int = 4, holdout: float = 0.2, base: Scene = None) -> Scene:
    """The tiny scene (or `base`, e.g. the LiDAR scan) with a seeded 20 % of its
    labelled hits held out.

    The held-out hits (and their beams) are removed from the training scan and
    returned as `holdout`: they are the query points of the predictive loss."""
    base = tiny_scene(seed=0) if base is None else base
    rng = np.random.default_rng(seed)
    s = base.scans[0]
    n = s.xyz.shape[0]
    perm = rng.permutation(n)
    n_h = int(round(holdout * n))
    held = np.sort(perm[:n_h])
    keep = np.sort(perm[n_h:])
    train = Scan(s.xyz[keep].copy(), s.label[keep].copy(), s.origin.copy())
    hold = Scan(s.xyz[held].copy(), s.label[held].copy(), s.origin.copy())
    return Scene("differentiable", base.params, [train], holdout=hold,
                 info={"seed": seed, "base": base.name})


def random_points_scene(seed: int, n: int, K: int = 4, extent: float = 1.0,
                        centre=(0.0, 0.0, 0.0), res: float = 0.1, l: float = 0.3,
                        sigma0: float = 1.0, alpha0: float = 0.001, free_step: float = 0.0,
                        block_size: int = 8, origin=(0.0, 0.0, 0.0)) -> Scene:
    """Uniform random labelled points in a cube (small property / brute-force cases)."""
    rng = np.random.default_rng(seed)
    c = np.asarray(centre, np.float64)
    xyz = _f32(c + rng.uniform(-extent, extent, size=(n, 3)))
    lab = rng.integers(1 if K > 1 else 0, K, size=n).astype(np.int32)
    params = Params(res=res, block_size=block_size, l=l, sigma0=sigma0, alpha0=alpha0, K=K,
                    free_class=0, free_step=free_step)
    return Scene("random", params, [Scan(xyz, lab, _f32(origin))], info={"seed": seed})


def soft_measurements(label, K, seed=0, top=3, peak=3.0, dropped=0.02):
    """Pseudo-probability vectors shaped like a semantic classifier's output, one
    per hit: softmax of N(0, 1) logits with +peak on the hit's label, truncated
    to its `top` largest entries (the rest 0, not renormalised), float32.  Hits
    with label -1 and a `dropped` fraction of the others get all-zero rows.
    Seeded; the free class (0) is never a measured class."""
    rng = np.random.default_rng(seed)
    lab = np.asarray(label)
    n = lab.shape[0]
    z = rng.standard_normal((n, K))
    z[:, 0] = -np.inf                                   # a hit never measures free space
    ok = lab >= 0
    z[np.nonzero(ok)[0], lab[ok]] += peak
    z -= z.max(axis=1, keepdims=True)
    e = np.exp(z)
    pr = e / e.sum(axis=1, keepdims=True)
    if top < K:
        cut = np.sort(pr, axis=1)[:, K - top][:, None]
        pr = np.where(pr >= cut, pr, 0.0)
    pr[~ok] = 0.0
    pr[rng.random(n) < dropped] = 0.0
    return pr.astype(np.float32)


CONFIG_NAMES = ["tiny", "lidar", "stereo", "batched", "differentiable"]


def make_config(n: int, **kw) -> Scene:
    """Workload n (0-based): 0 tiny, 1 lidar scan, 2 stereo sequence, 3 batched
    town, 4 differentiable split of the tiny scene.  The seed of workload n is n
    unless given."""
    fns = [tiny_scene, lidar_scan_scene, stereo_sequence_scene, batched_town_scene,
           differentiable_scene]
    kw.setdefault("seed", n)
    return fns[n](**kw)
