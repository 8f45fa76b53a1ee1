"""Seeded synthetic inputs shaped like the paper's LiDAR workloads.

The paper evaluates on KITTI, MulRan and racing recordings, none of which are
available here; these generators stand in for them.  This module holds none of
the registration method's arithmetic (no voxel keys, covariances, matching or
optimisation): only scene geometry, a spinning-LiDAR ray caster, ground-truth
poses and random sampling.  Both the GPU library's tests and the FP64 oracle
consume what it produces.

Every generator takes an integer seed and draws from
numpy.random.Generator(PCG64(seed)); per-scan draws use the sub-seed
seed * 1000 + scan.  Points are returned SoA float32 [3, n]; poses are
row-major float64 [4, 4] mapping sensor coordinates into the map frame.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Poses
# ---------------------------------------------------------------------------
def pose(R: np.ndarray, t) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def pose_inverse(T: np.ndarray) -> np.ndarray:
    R = T[:3, :3]
    return pose(R.T, -R.T @ T[:3, 3])


def unit_vector(g: np.random.Generator) -> np.ndarray:
    v = g.normal(size=3)
    return v / np.linalg.norm(v)


def random_offset(g: np.random.Generator, trans: float, angle_deg: float,
                  exact: bool = True) -> np.ndarray:
    """Rigid offset with rotation angle_deg about a random axis and translation
    of norm trans along a random direction (exact=True), or uniform in the ball
    and angle (exact=False)."""
    axis = unit_vector(g)
    ang = math.radians(angle_deg) * (1.0 if exact else g.uniform())
    tr = trans * (1.0 if exact else g.uniform() ** (1.0 / 3.0))
    return pose(Rotation.from_rotvec(axis * ang).as_matrix(), unit_vector(g) * tr)


def apply(T: np.ndarray, xyz: np.ndarray) -> np.ndarray:
    """Transform SoA points by T in float64 and round to float32."""
    p = T[:3, :3] @ xyz.astype(np.float64) + T[:3, 3:4]
    return p.astype(np.float32)


# ---------------------------------------------------------------------------
# Tiny scene: ground, two walls, two vertical cylinders
# ---------------------------------------------------------------------------
def _sample_rect(g, n, origin, u, v):
    a, b = g.uniform(size=n), g.uniform(size=n)
    return (np.asarray(origin)[:, None] + np.outer(u, a) + np.outer(v, b))


def _sample_cyl(g, n, cx, cy, r, h):
    th = g.uniform(0, 2 * math.pi, size=n)
    z = g.uniform(0, h, size=n)
    return np.stack([cx + r * np.cos(th), cy + r * np.sin(th), z])


def tiny_scene_samples(g: np.random.Generator, n: int) -> np.ndarray:
    """n area-uniform samples of: ground z=0 over [-20,20]^2, wall x=16 and wall
    y=16 (40 m long, 5 m high) and cylinders r=0.5 m, h=4 m at (-3,2), (4,-5)."""
    parts = [
        (1600.0, lambda m: _sample_rect(g, m, (-20, -20, 0), (40, 0, 0), (0, 40, 0))),
        (200.0, lambda m: _sample_rect(g, m, (16, -20, 0), (0, 40, 0), (0, 0, 5))),
        (200.0, lambda m: _sample_rect(g, m, (-20, 16, 0), (40, 0, 0), (0, 0, 5))),
        (2 * math.pi * 0.5 * 4, lambda m: _sample_cyl(g, m, -3.0, 2.0, 0.5, 4.0)),
        (2 * math.pi * 0.5 * 4, lambda m: _sample_cyl(g, m, 4.0, -5.0, 0.5, 4.0)),
    ]
    w = np.array([a for a, _ in parts])
    which = g.choice(len(parts), size=n, p=w / w.sum())
    out = np.empty((3, n))
    for j, (_, f) in enumerate(parts):
        idx = np.nonzero(which == j)[0]
        if idx.size:
            out[:, idx] = f(idx.size)
    return out.astype(np.float32)


@dataclass
class TinyCase:
    """Plain GICP case: map batches, a noisy moved source and its ground truth."""
    map_batches: list
    source: np.ndarray
    T_gt: np.ndarray
    voxel_size: float = 1.0
    max_pts_per_voxel: int = 20
    min_spacing: float = 1.0 / math.sqrt(20.0)
    k: int = 5
    tau: float = 1.0
    kappa: float = 1.0 / 9.0
    max_iters: int = 10


def make_tiny(seed: int = 1, n_batches: int = 11, batch: int = 5000,
              n_source: int = 5000, noise: float = 0.02, trans: float = 0.3,
              angle_deg: float = 2.0) -> TinyCase:
    g = rng(seed)
    batches = [tiny_scene_samples(g, batch) for _ in range(n_batches)]
    x = tiny_scene_samples(g, n_source).astype(np.float64)
    x += g.normal(scale=noise, size=x.shape)
    T_gt = random_offset(g, trans, angle_deg)
    src = apply(pose_inverse(T_gt), x)
    return TinyCase(batches, src, T_gt)


# ---------------------------------------------------------------------------
# Corridor scene and spinning-LiDAR ray caster
# ---------------------------------------------------------------------------
@dataclass
class Corridor:
    length: float = 1000.0
    half_width: float = 15.0
    wall_height: float = 10.0
    pole_radius: float = 0.2
    pole_height: float = 6.0
    pole_spacing: float = 20.0
    pole_inset: float = 3.0
    pillar_spacing: float = 10.0   # wall pillars (0: none), jittered +-1.5 m
    pillar_width: float = 1.0
    pillar_depth: float = 0.6
    seed: int = 7
    poles: np.ndarray = field(default=None, repr=False)    # [P, 2] centres
    pillars: np.ndarray = field(default=None, repr=False)  # [Q, 4] x0, x1, y0, y1

    def __post_init__(self):
        g = rng(self.seed)
        if self.poles is None:
            xs = np.arange(self.pole_spacing / 2, self.length, self.pole_spacing)
            ys = self.half_width - self.pole_inset
            left = np.stack([xs + g.uniform(-2, 2, xs.size), np.full(xs.size, ys)], 1)
            right = np.stack([xs + g.uniform(-2, 2, xs.size), np.full(xs.size, -ys)], 1)
            self.poles = np.concatenate([left, right])
        if self.pillars is None:
            rows = []
            if self.pillar_spacing > 0:
                W, w, dp = self.half_width, self.pillar_width / 2, self.pillar_depth
                for xc in np.arange(self.pillar_spacing / 2, self.length, self.pillar_spacing):
                    a = xc + g.uniform(-1.5, 1.5)
                    b = xc + g.uniform(-1.5, 1.5)
                    rows.append((a - w, a + w, W - dp, W))
                    rows.append((b - w, b + w, -W, -W + dp))
            self.pillars = np.array(rows, dtype=np.float64).reshape(-1, 4)

    def _pillar_face_areas(self):
        H = self.wall_height
        fw = (self.pillars[:, 1] - self.pillars[:, 0]) * H       # face toward the corridor
        sd = (self.pillars[:, 3] - self.pillars[:, 2]) * H       # each side face
        return fw, sd

    def surface_area(self):
        fw, sd = self._pillar_face_areas()
        return (self.length * 2 * self.half_width + 2 * self.length * self.wall_height
                + len(self.poles) * 2 * math.pi * self.pole_radius * self.pole_height
                + float(np.sum(fw + 2 * sd)))

    def surface_samples(self, g: np.random.Generator, n: int) -> np.ndarray:
        L, W, H = self.length, self.half_width, self.wall_height
        pa = 2 * math.pi * self.pole_radius * self.pole_height
        fw, sd = self._pillar_face_areas()
        w = np.array([L * 2 * W, L * H, L * H, pa * len(self.poles), float(np.sum(fw + 2 * sd))])
        which = g.choice(5, size=n, p=w / w.sum())
        out = np.empty((3, n))
        for j in range(5):
            idx = np.nonzero(which == j)[0]
            m = idx.size
            if not m:
                continue
            if j == 0:
                pts = _sample_rect(g, m, (0, -W, 0), (L, 0, 0), (0, 2 * W, 0))
            elif j == 1:
                pts = _sample_rect(g, m, (0, W, 0), (L, 0, 0), (0, 0, H))
            elif j == 2:
                pts = _sample_rect(g, m, (0, -W, 0), (L, 0, 0), (0, 0, H))
            elif j == 3:
                k = g.integers(0, len(self.poles), size=m)
                th = g.uniform(0, 2 * math.pi, size=m)
                pts = np.stack([self.poles[k, 0] + self.pole_radius * np.cos(th),
                                self.poles[k, 1] + self.pole_radius * np.sin(th),
                                g.uniform(0, self.pole_height, size=m)])
            else:
                # pillar faces: the one toward the corridor and the two sides
                areas = np.concatenate([fw, sd, sd])
                f = g.choice(areas.size, size=m, p=areas / areas.sum())
                q = len(self.pillars)
                P = self.pillars[f % q]
                u, z = g.uniform(size=m), g.uniform(0, H, size=m)
                # toward-corridor face: y = inner side of the pillar
                inner = np.where(P[:, 3] > 0, P[:, 2], P[:, 3])
                x = np.where(f < q, P[:, 0] + u * (P[:, 1] - P[:, 0]),
                             np.where(f < 2 * q, P[:, 0], P[:, 1]))
                y = np.where(f < q, inner, P[:, 2] + u * (P[:, 3] - P[:, 2]))
                pts = np.stack([x, y, z])
            out[:, idx] = pts
        return out.astype(np.float32)

    def cast(self, origin: np.ndarray, dirs: np.ndarray, max_range: float) -> np.ndarray:
        """First-hit distance of rays origin + t*dir (dirs [3, m], unit); inf = none.
        origin is one point [3] or one per ray [3, m]."""
        ox, oy, oz = origin
        lo, hi = np.min(ox), np.max(ox)
        dx, dy, dz = dirs
        best = np.full(dirs.shape[1], np.inf)
        with np.errstate(divide="ignore", invalid="ignore"):
            # ground z = 0 inside the corridor footprint
            t = -oz / dz
            x, y = ox + t * dx, oy + t * dy
            ok = (t > 0) & (x >= 0) & (x <= self.length) & (np.abs(y) <= self.half_width)
            best = np.where(ok & (t < best), t, best)
            for ywall in (self.half_width, -self.half_width):
                t = (ywall - oy) / dy
                x, z = ox + t * dx, oz + t * dz
                ok = (t > 0) & (x >= 0) & (x <= self.length) & (z >= 0) & (z <= self.wall_height)
                best = np.where(ok & (t < best), t, best)
            # axis-aligned pillar boxes (slab test in x and y, z in [0, H])
            px = self.pillars[:, 0]
            for x0, x1, y0, y1 in self.pillars[(px > lo - max_range - 2) & (px < hi + max_range + 2)]:
                tx0, tx1 = (x0 - ox) / dx, (x1 - ox) / dx
                ty0, ty1 = (y0 - oy) / dy, (y1 - oy) / dy
                tmin = np.maximum(np.minimum(tx0, tx1), np.minimum(ty0, ty1))
                tmax = np.minimum(np.maximum(tx0, tx1), np.maximum(ty0, ty1))
                z = oz + tmin * dz
                ok = (tmax >= tmin) & (tmin > 0) & (z >= 0) & (z <= self.wall_height)
                best = np.where(ok & (tmin < best), tmin, best)
            if np.ndim(ox) == 0:
                near = self.poles[np.hypot(self.poles[:, 0] - ox, self.poles[:, 1] - oy)
                                  < max_range + 1.0]
            else:
                cx = self.poles[:, 0]
                near = self.poles[(cx > lo - max_range - 1.0) & (cx < hi + max_range + 1.0)]
            a = dx * dx + dy * dy
            for cx, cy in near:
                fx, fy = ox - cx, oy - cy
                bq = 2 * (fx * dx + fy * dy)
                cq = fx * fx + fy * fy - self.pole_radius ** 2
                disc = bq * bq - 4 * a * cq
                t = (-bq - np.sqrt(np.maximum(disc, 0))) / (2 * a)
                z = oz + t * dz
                ok = (disc >= 0) & (t > 0) & (z >= 0) & (z <= self.pole_height)
                best = np.where(ok & (t < best), t, best)
        return best


@dataclass
class Lidar:
    beams: int = 128
    azimuths: int = 1024
    elev_min_deg: float = -22.5
    elev_max_deg: float = 22.5
    min_range: float = 1.0
    max_range: float = 120.0
    range_noise: float = 0.03
    drop: float = 0.1

    def directions(self) -> np.ndarray:
        el = np.radians(np.linspace(self.elev_min_deg, self.elev_max_deg, self.beams))
        az = np.linspace(0, 2 * math.pi, self.azimuths, endpoint=False)
        # azimuth-major firing order: one column of all beams per azimuth step
        A, E = np.meshgrid(az, el, indexing="ij")
        A, E = A.ravel(), E.ravel()
        return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)])


def scan(scene: Corridor, lidar: Lidar, T_world_sensor: np.ndarray,
         g: np.random.Generator) -> np.ndarray:
    """One instantaneous spinning-LiDAR scan, returned in the sensor frame."""
    d_s = lidar.directions()
    R, t = T_world_sensor[:3, :3], T_world_sensor[:3, 3]
    rng_ = scene.cast(t, R @ d_s, lidar.max_range)
    rng_ = rng_ + g.normal(scale=lidar.range_noise, size=rng_.shape)
    keep = np.isfinite(rng_) & (rng_ >= lidar.min_range) & (rng_ <= lidar.max_range)
    keep &= g.uniform(size=rng_.shape) >= lidar.drop
    return (d_s[:, keep] * rng_[keep]).astype(np.float32)


def trajectory_pose(t: float, speed: float = 70.0, amp: float = 3.0,
                    period: float = 8.0, height: float = 2.0, x0: float = 5.0,
                    accel: float = 0.0) -> np.ndarray:
    """Smooth path along the corridor: x = x0 + speed t + accel t^2 / 2,
    y = amp sin(2 pi t / period), heading along the velocity."""
    x = x0 + speed * t + 0.5 * accel * t * t
    y = amp * math.sin(2 * math.pi * t / period)
    vx = speed + accel * t
    vy = amp * 2 * math.pi / period * math.cos(2 * math.pi * t / period)
    yaw = math.atan2(vy, vx)
    return pose(Rotation.from_euler("z", yaw).as_matrix(), (x, y, height))


def trajectory_twist(t: float, speed: float = 70.0, amp: float = 3.0,
                     period: float = 8.0, accel: float = 0.0) -> np.ndarray:
    """Body-frame velocity (vx, vy, vz, wx, wy, wz) of trajectory_pose at time t,
    from its derivatives: the heading follows the planar velocity, so the linear
    part is (|v|, 0, 0) and the angular part (0, 0, d yaw / dt)."""
    w = 2 * math.pi / period
    vx, vy = speed + accel * t, amp * w * math.cos(w * t)
    ax, ay = accel, -amp * w * w * math.sin(w * t)
    return np.array([math.hypot(vx, vy), 0.0, 0.0, 0.0, 0.0,
                     (vx * ay - vy * ax) / (vx * vx + vy * vy)])


def scan_moving(scene: Corridor, lidar: Lidar, pose_at, t0: float, period: float,
                g: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """A spinning-LiDAR scan taken while the sensor moves: azimuth column j fires
    at t0 + period j / azimuths from the pose pose_at(time), and each return is
    expressed in the sensor frame of its own firing time.  Returns the points
    [3, n] float32 and their times relative to t0 [n] float32, in firing order."""
    d_s = lidar.directions()
    B, A = lidar.beams, lidar.azimuths
    tcol = period * np.arange(A) / A
    Ts = [pose_at(t0 + tc) for tc in tcol]
    R = np.stack([T[:3, :3] for T in Ts])                        # [A, 3, 3]
    org = np.repeat(np.stack([T[:3, 3] for T in Ts]), B, axis=0).T   # [3, A B]
    d_w = np.einsum("aij,jab->iab", R, d_s.reshape(3, A, B)).reshape(3, A * B)
    rng_ = scene.cast(org, d_w, lidar.max_range)
    rng_ = rng_ + g.normal(scale=lidar.range_noise, size=rng_.shape)
    keep = np.isfinite(rng_) & (rng_ >= lidar.min_range) & (rng_ <= lidar.max_range)
    keep &= g.uniform(size=rng_.shape) >= lidar.drop
    times = np.repeat(tcol, B)[keep].astype(np.float32)
    return (d_s[:, keep] * rng_[keep]).astype(np.float32), times


@dataclass
class SequenceCase:
    scans: list
    poses: list
    scene: Corridor
    voxel_size: float = 1.0
    max_pts_per_voxel: int = 20
    min_spacing: float = 1.0 / math.sqrt(20.0)
    downsample: float = 0.5
    k: int = 5
    map_capacity: int = 2_000_000
    sigma0: float = 1.0 / 3.0
    r_max: float = 120.0


def make_sequence(seed: int = 2, n_scans: int = 100, rate_hz: float = 10.0,
                  lidar: Lidar | None = None) -> SequenceCase:
    """Spinning-LiDAR sequence: 128 x 1024 rays per scan along a 70 m/s path."""
    lidar = lidar or Lidar()
    scene = Corridor()
    poses, scans = [], []
    for s in range(n_scans):
        T = trajectory_pose(s / rate_hz)
        poses.append(T)
        scans.append(scan(scene, lidar, T, rng(seed * 1000 + s)))
    return SequenceCase(scans, poses, scene)


@dataclass
class DeskewCase:
    """A sequence scanned while moving: per scan the points in firing order,
    their times, velocity samples on the same clock (relative to the scan's
    start) and the ground-truth pose at each scan's last point time."""
    scans: list
    times: list          # [n] float32 per scan, seconds after the scan start
    vel_t: list          # [m] float64 per scan, sample times on the same clock
    vel: list            # [m, 6] float64 per scan, body-frame (vx vy vz wx wy wz)
    poses: list          # pose at each scan's largest point time
    starts: list         # scan start times (sequence clock)
    traj: dict
    scene: Corridor
    voxel_size: float = 1.0
    max_pts_per_voxel: int = 20
    min_spacing: float = 1.0 / math.sqrt(20.0)
    downsample: float = 0.5
    k: int = 5
    map_capacity: int = 2_000_000
    sigma0: float = 1.0 / 3.0
    r_max: float = 120.0


RACING = dict(speed=70.0, amp=4.0, period=2.5, accel=5.0)


def make_deskew(seed: int = 6, n_scans: int = 40, rate_hz: float = 10.0,
                lidar: Lidar | None = None, imu_hz: float = 200.0,
                noise_v: float = 0.05, noise_w: float = 0.002,
                traj: dict | None = None) -> DeskewCase:
    """Sequence along an accelerating, weaving racing line (70 m/s, 5 m/s^2,
    +-4 m at 0.4 Hz): each scan spans one rotation period, so uncorrected
    points are smeared by up to 7 m and 2 degrees.  Velocity samples at imu_hz
    from 10 ms before the scan start to its end, with Gaussian noise (noise_v
    m/s on the linear, noise_w rad/s on the angular part), stand in for the
    sensor fusion's velocity history."""
    lidar = lidar or Lidar()
    traj = dict(RACING if traj is None else traj)
    scene = Corridor()
    period = 1.0 / rate_hz
    pose_at = lambda t: trajectory_pose(t, **traj)
    out = dict(scans=[], times=[], vel_t=[], vel=[], poses=[], starts=[])
    for s in range(n_scans):
        g = rng(seed * 1000 + s)
        t0 = s * period
        xyz, tt = scan_moving(scene, lidar, pose_at, t0, period, g)
        vt = np.arange(-0.01, period + 1e-9, 1.0 / imu_hz)
        v = np.stack([trajectory_twist(t0 + x, **traj) for x in vt])
        v[:, :3] += g.normal(scale=noise_v, size=(vt.size, 3))
        v[:, 3:] += g.normal(scale=noise_w, size=(vt.size, 3))
        out["scans"].append(xyz)
        out["times"].append(tt)
        out["vel_t"].append(vt)
        out["vel"].append(v)
        out["poses"].append(pose_at(t0 + float(tt.max())))
        out["starts"].append(t0)
    return DeskewCase(traj=traj, scene=scene, **out)


@dataclass
class BatchCase:
    """Independent scans of uneven size against one prebuilt map."""
    map_batches: list
    map_capacity: int
    scans: list           # sensor-frame SoA float32 [3, n_s]
    T_gt: list            # ground-truth poses
    T0: list              # initial guesses (ground truth times a random offset)
    scene: Corridor
    voxel_size: float = 1.0
    max_pts_per_voxel: int = 20
    min_spacing: float = 1.0 / math.sqrt(20.0)
    k: int = 5
    tau: float = 1.0
    kappa: float = 1.0 / 9.0
    max_iters: int = 10


def make_batch(seed: int = 3, n_scans: int = 64, n_min: int = 8000, n_max: int = 130000,
               map_points: int = 2_000_000, map_batch: int = 1_000_000,
               n_map_batches: int = 8, max_offset_m: float = 0.5,
               max_offset_deg: float = 3.0, scene: Corridor | None = None) -> BatchCase:
    """64 scans at random ground-truth poses along a widened corridor (the map
    needs about 2e5 m^2 of surface to hold 2M points at the default spacing),
    each subsampled without replacement to n_s ~ U{n_min..n_max} (clamped to the
    hits of its 128 x 1024 rays) and given its own initial offset."""
    scene = scene or Corridor(half_width=50.0, wall_height=50.0, pole_height=20.0,
                              pole_inset=10.0)
    g = rng(seed)
    map_batches = [scene.surface_samples(rng(seed * 1000 + 900 + b), map_batch)
                   for b in range(n_map_batches)]
    lidar = Lidar()
    scans, T_gt, T0 = [], [], []
    for s in range(n_scans):
        gs = rng(seed * 1000 + s)
        x = gs.uniform(60.0, scene.length - 60.0)
        y = gs.uniform(-0.5, 0.5) * scene.half_width
        yaw = gs.uniform(-math.pi, math.pi)
        T = pose(Rotation.from_euler("z", yaw).as_matrix(), (x, y, 2.0))
        pts = scan(scene, lidar, T, gs)
        n_s = int(gs.integers(n_min, n_max + 1))
        n_s = min(n_s, pts.shape[1])
        sel = np.sort(gs.choice(pts.shape[1], size=n_s, replace=False))
        scans.append(np.ascontiguousarray(pts[:, sel]))
        T_gt.append(T)
        T0.append(T @ random_offset(gs, max_offset_m, max_offset_deg, exact=False))
    del g
    return BatchCase(map_batches, map_points, scans, T_gt, T0, scene)


def random_cloud(seed: int, n: int, extent: float = 4.0, dup_frac: float = 0.0,
                 on_faces: float = 0.0, v: float = 1.0) -> np.ndarray:
    """Uniform random cloud in [-extent, extent]^3 with optional exact duplicates
    and points snapped onto voxel faces (multiples of v) for tie and boundary
    cases."""
    g = rng(seed)
    p = g.uniform(-extent, extent, size=(3, n))
    if on_faces > 0:
        m = g.uniform(size=(3, n)) < on_faces
        p[m] = np.round(p[m] / v) * v
    p = p.astype(np.float32)
    if dup_frac > 0:
        nd = int(n * dup_frac)
        src = g.integers(0, n, size=nd)
        dst = g.integers(0, n, size=nd)
        p[:, dst] = p[:, src]
    return np.ascontiguousarray(p)


def line_cloud(seed: int, n_lines: int = 300, per_line: int = 12, extent: float = 8.0,
               step: float = 0.125) -> np.ndarray:
    """Points on straight lines (edges and thin poles in a scan): per line
    per_line points step apart from a random start; two thirds of the lines
    run along a coordinate axis with exactly representable coordinates, so
    their neighbourhoods are exactly collinear (the sample covariance's
    smallest eigenvalue is double), the rest along random directions."""
    g = rng(seed)
    out = []
    for i in range(n_lines):
        start = np.round(g.uniform(-extent, extent, size=3) * 8.0) / 8.0
        if i % 3 != 2:
            d = np.zeros(3)
            d[i % 3] = 1.0
        else:
            d = g.normal(size=3)
            d /= np.linalg.norm(d)
        t = step * np.arange(per_line)
        out.append(start[:, None] + d[:, None] * t[None, :])
    return np.ascontiguousarray(np.concatenate(out, axis=1).astype(np.float32))


# ---------------------------------------------------------------------------
# Precision stress: exact planes (near-degenerate neighbourhoods) and rough
# surfaces, fine voxels
# ---------------------------------------------------------------------------
def make_diff(seed: int = 4, n_scans: int = 16, n_points: int = 32768,
              map_points: int = 1_000_000) -> BatchCase:
    """Differentiation workload: n_scans scans of exactly n_points points from
    the spinning-LiDAR simulator against a map of map_points points (the
    batched-scans scene and map recipe at these sizes)."""
    return make_batch(seed, n_scans=n_scans, n_min=n_points, n_max=n_points,
                      map_points=map_points, n_map_batches=4)


@dataclass
class PrecisionCase:
    map_batches: list
    map_capacity: int
    scan: np.ndarray       # sensor frame, SoA float32 [3, n]
    T_gt: np.ndarray
    T0: np.ndarray
    planar_frac: float
    voxel_size: float = 0.25
    max_pts_per_voxel: int = 30
    min_spacing: float = 0.25 / math.sqrt(30.0)
    k: int = 5
    tau: float = 0.25
    kappa: float = 0.25 / 9.0
    max_iters: int = 10


def _site_samples(g, n, size, planar):
    """Area-uniform samples of a size x size site.  planar=True: the exact
    planes (floor z = 0 and four 20 m facades) with N(0, 1e-5^2) noise;
    planar=False: rough surfaces with N(0, 0.03^2) noise - a rolling terrain
    patch, boxes and vertical cylinders."""
    if planar:
        w = np.array([size * size, 4 * size * 20.0])
        which = g.choice(2, size=n, p=w / w.sum())
        out = np.empty((3, n))
        i0 = np.nonzero(which == 0)[0]
        out[:, i0] = _sample_rect(g, i0.size, (0, 0, 0), (size, 0, 0), (0, size, 0))
        i1 = np.nonzero(which == 1)[0]
        side = g.integers(0, 4, i1.size)
        u, h = g.uniform(0, size, i1.size), g.uniform(0, 20.0, i1.size)
        out[0, i1] = np.where(side == 0, 0.0, np.where(side == 1, size, u))
        out[1, i1] = np.where(side == 2, 0.0, np.where(side == 3, size, u))
        out[2, i1] = h
        return out + g.normal(scale=1e-5, size=out.shape)
    gs = rng(11)  # fixed clutter layout
    boxes = np.concatenate([gs.uniform(10, size - 10, (60, 2)), gs.uniform(1.5, 4.0, (60, 2)),
                            gs.uniform(1.0, 6.0, (60, 1))], 1)
    cyl = np.concatenate([gs.uniform(10, size - 10, (80, 2)), gs.uniform(0.3, 1.0, (80, 1)),
                          gs.uniform(2.0, 8.0, (80, 1))], 1)
    a_terr = (size / 2) ** 2
    a_box = boxes[:, 2] * boxes[:, 3] + 2 * (boxes[:, 2] + boxes[:, 3]) * boxes[:, 4]
    a_cyl = 2 * math.pi * cyl[:, 2] * cyl[:, 3]
    w = np.array([a_terr, a_box.sum(), a_cyl.sum()])
    which = g.choice(3, size=n, p=w / w.sum())
    out = np.empty((3, n))
    i = np.nonzero(which == 0)[0]
    x, y = g.uniform(0, size / 2, i.size), g.uniform(size / 2, size, i.size)
    out[:, i] = np.stack([x, y, 0.4 * np.sin(x / 3.0) * np.cos(y / 4.0) + 0.5])
    i = np.nonzero(which == 1)[0]
    b = boxes[g.choice(len(boxes), size=i.size, p=a_box / a_box.sum())]
    face = g.integers(0, 5, i.size)
    u, v = g.uniform(size=i.size), g.uniform(size=i.size)
    x = np.where(face == 1, b[:, 0], np.where(face == 2, b[:, 0] + b[:, 2], b[:, 0] + u * b[:, 2]))
    y = np.where(face == 3, b[:, 1], np.where(face == 4, b[:, 1] + b[:, 3], b[:, 1] + v * b[:, 3]))
    z = np.where(face == 0, b[:, 4], v * b[:, 4])
    out[:, i] = np.stack([x, y, z])
    i = np.nonzero(which == 2)[0]
    cc = cyl[g.choice(len(cyl), size=i.size, p=a_cyl / a_cyl.sum())]
    th = g.uniform(0, 2 * math.pi, i.size)
    out[:, i] = np.stack([cc[:, 0] + cc[:, 2] * np.cos(th), cc[:, 1] + cc[:, 2] * np.sin(th),
                          g.uniform(0, 1, i.size) * cc[:, 3]])
    return out + g.normal(scale=0.03, size=out.shape)


def make_precision(seed: int = 5, map_points: int = 20_000_000, map_batch: int = 5_000_000,
                   n_map_batches: int = 12, n_scan: int = 1_000_000, planar_frac: float = 0.3,
                   site: float = 250.0, scan_radius: float = 40.0) -> PrecisionCase:
    """Precision stress: map of fine voxels (v = 0.25 m, N_max = 30) over a
    site of exact planes and rough clutter; one scan of n_scan points within
    scan_radius of a sensor near a corner of the site, a fraction planar_frac
    of them on the exact planes (near-degenerate neighbourhoods), moved by a
    0.05 m / 0.25 deg initial offset from the ground truth."""
    g = rng(seed)
    batches = []
    for b in range(n_map_batches):
        gb = rng(seed * 1000 + 500 + b)
        m_pl = int(map_batch * 0.5)
        pts = np.concatenate([_site_samples(gb, m_pl, site, True),
                              _site_samples(gb, map_batch - m_pl, site, False)], 1)
        batches.append(pts[:, gb.permutation(pts.shape[1])].astype(np.float32))
    centre = np.array([35.0, 35.0, 2.0])

    def near(planar, want):
        got = []
        while sum(x.shape[1] for x in got) < want:
            x = _site_samples(g, max(4 * want, 1000), site, planar)
            got.append(x[:, np.linalg.norm(x[:2] - centre[:2, None], axis=0) < scan_radius])
        return np.concatenate(got, 1)[:, :want]

    n_pl = int(n_scan * planar_frac)
    x = np.concatenate([near(True, n_pl), near(False, n_scan - n_pl)], 1)
    x = x[:, g.permutation(x.shape[1])]
    T_gt = pose(Rotation.from_euler("z", g.uniform(-math.pi, math.pi)).as_matrix(), centre)
    scan_ = apply(pose_inverse(T_gt), x)
    T0 = T_gt @ random_offset(g, 0.05, 0.25)
    return PrecisionCase(batches, map_points, scan_, T_gt, T0, planar_frac)
