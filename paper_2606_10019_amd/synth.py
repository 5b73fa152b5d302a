"""Seeded synthetic point-cloud pairs for registration tests and benchmarks.

This module only builds inputs: surfaces, ray casts, voxel grids and the
ground-truth rigid motion of each pair.  It holds none of the registration
method's arithmetic (no kernels, no covariances, no gradients), so both the
GPU path and the CPU oracle can consume its output without sharing code.

Every generator is a pure function of ``(config, instance)``: instance ``i`` of
configuration ``c`` draws from ``numpy.random.default_rng(1_000_003 * c + i)``
in a fixed order.  Clouds are returned as C-contiguous float32 ``[n, 3]``
arrays; the float64 view of those exact values is what the oracle receives.

Pose convention (Notation section of the paper): a pose T acts on points as
``T p = R p + t`` and the objective compares target points x_i with
``T^{-1} z_j``.  When the target is generated as ``x = G p`` from the same
surface as the source ``z = p``, the registration should return ``T = G^{-1}``.
Each pair records ``G`` and ``T_true = G^{-1}``; truth is informational, the
accuracy gate compares the GPU against the oracle.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

SEED_STRIDE = 1_000_003


def rng_for(config: int, instance: int) -> np.random.Generator:
    return np.random.default_rng(SEED_STRIDE * config + instance)


def rigid(R: np.ndarray, t) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = np.asarray(t, dtype=np.float64)
    return T


def transform_points(T: np.ndarray, P: np.ndarray) -> np.ndarray:
    return P @ T[:3, :3].T + T[:3, 3]


def random_unit(rng: np.random.Generator) -> np.ndarray:
    while True:
        v = rng.normal(size=3)
        n = np.linalg.norm(v)
        if n > 1e-12:
            return v / n


def rotation_about(axis: np.ndarray, angle_rad: float) -> np.ndarray:
    return Rotation.from_rotvec(np.asarray(axis, dtype=np.float64) * angle_rad).as_matrix()


def cloud_digest(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def voxel_centroids(P: np.ndarray, voxel: float) -> np.ndarray:
    """Replace the points of every occupied voxel by their centroid (float64).

    Output order is the lexicographic order of the integer voxel keys, so it is
    deterministic for a given input.
    """
    keys = np.floor(P / voxel).astype(np.int64)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    cnt = np.bincount(inv, minlength=len(uniq)).astype(np.float64)
    out = np.empty((len(uniq), 3))
    for d in range(3):
        out[:, d] = np.bincount(inv, weights=P[:, d], minlength=len(uniq)) / cnt
    return out


@dataclass
class PairSpec:
    """One registration problem: target X, source Z and its solver settings."""
    name: str
    target: np.ndarray          # float32 [n_x, 3]
    source: np.ndarray          # float32 [n_z, 3]
    G: np.ndarray               # float64 4x4 generator motion
    length_scale: float
    length_scale_min: float
    anneal_factor: float = 0.5
    cutoff_scale: float = 3.0
    knn: int = 10
    eig_ratio_min: float = 0.01
    sigma2: float = 1.0
    max_iters: int = 30
    max_iters_per_stage: int = 30
    tol: float = 1e-6
    stage_tol: float = 1e-4
    extra: dict = field(default_factory=dict)

    @property
    def T_true(self) -> np.ndarray:
        return np.linalg.inv(self.G)

    def digest(self) -> str:
        return cloud_digest(self.target, self.source)

    def params(self) -> dict:
        return dict(length_scale=self.length_scale, length_scale_min=self.length_scale_min,
                    anneal_factor=self.anneal_factor, cutoff_scale=self.cutoff_scale,
                    knn=self.knn, eig_ratio_min=self.eig_ratio_min, sigma2=self.sigma2,
                    max_iters=self.max_iters, max_iters_per_stage=self.max_iters_per_stage,
                    tol=self.tol, stage_tol=self.stage_tol)


# --------------------------------------------------------------------------
# Configuration 1: three orthogonal 4x4 m planes and a 1 m hemisphere cap.
# --------------------------------------------------------------------------

def _sample_planes_and_cap(rng: np.random.Generator, n: int, noise: float) -> np.ndarray:
    plane_area = 16.0
    cap_area = 2.0 * np.pi * 1.0 ** 2
    areas = np.array([plane_area, plane_area, plane_area, cap_area])
    which = rng.choice(4, size=n, p=areas / areas.sum())
    u = rng.uniform(0.0, 4.0, size=n)
    v = rng.uniform(0.0, 4.0, size=n)
    zc = rng.uniform(0.0, 1.0, size=n)            # uniform height => uniform on the sphere
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    P = np.empty((n, 3))
    m = which == 0
    P[m] = np.stack([u[m], v[m], np.zeros(m.sum())], 1)      # z = 0
    m = which == 1
    P[m] = np.stack([u[m], np.zeros(m.sum()), v[m]], 1)      # y = 0
    m = which == 2
    P[m] = np.stack([np.zeros(m.sum()), u[m], v[m]], 1)      # x = 0
    m = which == 3
    rho = np.sqrt(np.maximum(0.0, 1.0 - zc[m] ** 2))
    P[m] = np.stack([2.0 + rho * np.cos(phi[m]), 2.0 + rho * np.sin(phi[m]), zc[m]], 1)
    return P + rng.normal(0.0, noise, size=P.shape)


def make_config1(instance: int = 0, n: int = 2000, noise: float = 0.01,
                 angle_deg: float = 5.0, trans_m: float = 0.2) -> PairSpec:
    rng = rng_for(1, instance)
    src = _sample_planes_and_cap(rng, n, noise)
    tgt_p = _sample_planes_and_cap(rng, n, noise)
    G = rigid(rotation_about(random_unit(rng), np.deg2rad(angle_deg)), trans_m * random_unit(rng))
    tgt = transform_points(G, tgt_p)
    return PairSpec(name=f"c1_planes_cap_{instance}", target=np.ascontiguousarray(tgt, np.float32),
                    source=np.ascontiguousarray(src, np.float32), G=G,
                    length_scale=0.3, length_scale_min=0.3, max_iters=30, max_iters_per_stage=30)


# --------------------------------------------------------------------------
# Configuration 2: spinning 64 x 1024 LiDAR over a ground plane with boxes
# and vertical cylinders, voxel-downsampled at 0.3 m.
# --------------------------------------------------------------------------

@dataclass
class LidarScene:
    box_lo: np.ndarray   # [nb, 3]
    box_hi: np.ndarray   # [nb, 3]
    cyl_c: np.ndarray    # [nc, 2]
    cyl_r: np.ndarray    # [nc]
    cyl_h: np.ndarray    # [nc]


def _annulus(rng, r0, r1):
    r = np.sqrt(rng.uniform(r0 * r0, r1 * r1))
    a = rng.uniform(0.0, 2.0 * np.pi)
    return np.array([r * np.cos(a), r * np.sin(a)])


BOX_ANNULUS_M = (35.0, 70.0)
CYLINDER_ANNULUS_M = (20.0, 60.0)
SENSOR_HEIGHT_M = 2.7
# Eigenvalue floor of the LiDAR pairs' shapes: with flatter ground kernels the
# rings that each scan draws around its sensor make the objective peak near the
# identity at the first length scale, a wrong basin for a forward motion.
LIDAR_RHO = 0.2


def make_lidar_scene(rng: np.random.Generator, keep_clear: np.ndarray,
                     n_boxes: int = 40, n_cyl: int = 30, box_annulus=BOX_ANNULUS_M,
                     cylinder_annulus=CYLINDER_ANNULUS_M) -> LidarScene:
    """Boxes rest on z = 0 with sides U[1, 10] m and centres uniform in an
    annulus (35-70 m); cylinders have r U[0.2, 0.5] m, height U[2, 6] m,
    centres in an annulus (20-60 m).  Objects far out hide little ground and
    catch the near-horizontal rays, which is what brings a 0.3 m voxelised scan
    to about 30k points (nearer placements give fewer).  Objects whose
    footprint comes within 2 m of a sensor position in ``keep_clear`` ([k, 2]
    xy) are redrawn, so no sensor sits inside a solid."""
    lo, hi = [], []
    while len(lo) < n_boxes:
        side = rng.uniform(1.0, 10.0, size=3)
        c = _annulus(rng, *box_annulus)
        blo = np.array([c[0] - side[0] / 2, c[1] - side[1] / 2, 0.0])
        bhi = np.array([c[0] + side[0] / 2, c[1] + side[1] / 2, side[2]])
        d = np.maximum(0.0, np.maximum(blo[None, :2] - keep_clear, keep_clear - bhi[None, :2]))
        if np.min(np.linalg.norm(d, axis=1)) < 2.0:
            continue
        lo.append(blo)
        hi.append(bhi)
    cc, cr, ch = [], [], []
    while len(cc) < n_cyl:
        r = rng.uniform(0.2, 0.5)
        h = rng.uniform(2.0, 6.0)
        c = _annulus(rng, *cylinder_annulus)
        if np.min(np.linalg.norm(keep_clear - c[None], axis=1)) - r < 2.0:
            continue
        cc.append(c)
        cr.append(r)
        ch.append(h)
    return LidarScene(np.array(lo), np.array(hi), np.array(cc), np.array(cr), np.array(ch))


def raycast(scene: LidarScene, origin: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Distance to the nearest hit along each unit ray (inf when nothing is hit)."""
    n = len(dirs)
    best = np.full(n, np.inf)
    dz = dirs[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(dz < -1e-12, -origin[2] / dz, np.inf)
    best = np.minimum(best, np.where(tg > 0, tg, np.inf))
    inv = np.where(np.abs(dirs) > 1e-15, 1.0 / np.where(np.abs(dirs) > 1e-15, dirs, 1.0), np.inf)
    for lo, hi in zip(scene.box_lo, scene.box_hi):
        with np.errstate(invalid="ignore"):
            t0 = (lo[None] - origin[None]) * inv
            t1 = (hi[None] - origin[None]) * inv
        # Rays parallel to a slab: inside it => (-inf, inf), outside => empty.
        par = ~np.isfinite(inv)
        inside = (origin[None] >= lo[None]) & (origin[None] <= hi[None])
        t0 = np.where(par, np.where(inside, -np.inf, np.inf), t0)
        t1 = np.where(par, np.where(inside, np.inf, -np.inf), t1)
        tn = np.max(np.minimum(t0, t1), axis=1)
        tf = np.min(np.maximum(t0, t1), axis=1)
        hit = (tf >= tn) & (tf > 0)
        th = np.where(tn > 0, tn, tf)
        best = np.where(hit & (th < best), th, best)
    ox, oy, oz = origin
    dx, dy = dirs[:, 0], dirs[:, 1]
    a = dx * dx + dy * dy
    for c, r, h in zip(scene.cyl_c, scene.cyl_r, scene.cyl_h):
        px, py = ox - c[0], oy - c[1]
        b = 2.0 * (px * dx + py * dy)
        cq = px * px + py * py - r * r
        disc = b * b - 4.0 * a * cq
        ok = (disc >= 0) & (a > 1e-15)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        with np.errstate(divide="ignore", invalid="ignore"):
            t_in = np.where(ok, (-b - sq) / (2.0 * a), np.inf)
        zh = oz + t_in * dz
        side_hit = ok & (t_in > 0) & (zh >= 0) & (zh <= h)
        best = np.where(side_hit & (t_in < best), t_in, best)
        with np.errstate(divide="ignore", invalid="ignore"):
            tc = np.where(np.abs(dz) > 1e-12, (h - oz) / dz, np.inf)
        xc = ox + tc * dx - c[0]
        yc = oy + tc * dy - c[1]
        cap_hit = (tc > 0) & (xc * xc + yc * yc <= r * r)
        best = np.where(cap_hit & (tc < best), tc, best)
    return best


def lidar_directions(n_rings: int = 64, n_az: int = 1024, elev_lo: float = -25.0,
                     elev_hi: float = 3.0) -> np.ndarray:
    el = np.deg2rad(np.linspace(elev_lo, elev_hi, n_rings))
    az = 2.0 * np.pi * np.arange(n_az) / n_az
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1).reshape(-1, 3)


def lidar_scan(scene: LidarScene, pose: np.ndarray, rng: np.random.Generator,
               range_noise: float = 0.02, max_range: float = 80.0) -> np.ndarray:
    """Points of one spin in the sensor frame (float64, before voxelisation)."""
    d_s = lidar_directions()
    d_w = d_s @ pose[:3, :3].T
    t = raycast(scene, pose[:3, 3], d_w)
    t = t + rng.normal(0.0, range_noise, size=t.shape)
    keep = np.isfinite(t) & (t > 0.0) & (t <= max_range)
    return d_s[keep] * t[keep, None]


def make_config2(instance: int = 0, voxel: float = 0.3, forward_m: float = 1.0,
                 yaw_deg: float = 2.0, sensor_height: float = SENSOR_HEIGHT_M) -> PairSpec:
    """LiDAR frame-to-frame pair: X = scan 1, Z = scan 2 taken after the ego
    motion M (forward along the sensor x axis, then yaw).  Expected T = M^{-1}."""
    rng = rng_for(2, instance)
    S1 = rigid(np.eye(3), [0.0, 0.0, sensor_height])
    M = rigid(rotation_about(np.array([0.0, 0.0, 1.0]), np.deg2rad(yaw_deg)), [forward_m, 0.0, 0.0])
    S2 = S1 @ M
    scene = make_lidar_scene(rng, np.array([S1[:2, 3], S2[:2, 3]]))
    x = voxel_centroids(lidar_scan(scene, S1, rng), voxel)
    z = voxel_centroids(lidar_scan(scene, S2, rng), voxel)
    # G maps the source surface into the target frame: x = M z for a static point.
    return PairSpec(name=f"c2_lidar_{instance}", target=np.ascontiguousarray(x, np.float32),
                    source=np.ascontiguousarray(z, np.float32), G=M,
                    length_scale=1.0, length_scale_min=0.1, anneal_factor=0.5,
                    eig_ratio_min=LIDAR_RHO, max_iters=200, max_iters_per_stage=60,
                    extra=dict(voxel=voxel))


C5_EVAL_OFFSET = 500_000


def make_config5(instance: int = 0, split: str = "train", max_trans_m: float = 3.0,
                 max_yaw_deg: float = 15.0, voxel: float = 0.3, sensor_height: float = SENSOR_HEIGHT_M) -> PairSpec:
    """LiDAR pair with a large ego motion (warm-start workload): the config-2
    scene and scanner, scan 2 after a yaw of U[-15, 15] deg and a planar
    translation of U[0, 3] m in a uniform direction.  Training and evaluation
    instances draw from disjoint seeds.  Expected T = M^{-1}."""
    rng = rng_for(5, instance + (C5_EVAL_OFFSET if split == "eval" else 0))
    S1 = rigid(np.eye(3), [0.0, 0.0, sensor_height])
    yaw = np.deg2rad(rng.uniform(-max_yaw_deg, max_yaw_deg))
    phi = rng.uniform(0.0, 2.0 * np.pi)
    d = rng.uniform(0.0, max_trans_m)
    M = rigid(rotation_about(np.array([0.0, 0.0, 1.0]), yaw), [d * np.cos(phi), d * np.sin(phi), 0.0])
    S2 = S1 @ M
    scene = make_lidar_scene(rng, np.array([S1[:2, 3], S2[:2, 3]]))
    x = voxel_centroids(lidar_scan(scene, S1, rng), voxel)
    z = voxel_centroids(lidar_scan(scene, S2, rng), voxel)
    return PairSpec(name=f"c5_{split}_{instance}", target=np.ascontiguousarray(x, np.float32),
                    source=np.ascontiguousarray(z, np.float32), G=M,
                    length_scale=1.0, length_scale_min=0.1, anneal_factor=0.5,
                    eig_ratio_min=LIDAR_RHO, max_iters=200, max_iters_per_stage=60,
                    extra=dict(voxel=voxel, yaw_deg=float(np.rad2deg(yaw)), trans_m=float(d)))


# --------------------------------------------------------------------------
# Configuration 3: 640x480 pinhole depth camera in a 6 x 5 x 3 m room with
# boxes and spheres, depth noise 0.0015 z^2, voxel size bisected to ~20k points.
# --------------------------------------------------------------------------

@dataclass
class RoomScene:
    box_lo: np.ndarray
    box_hi: np.ndarray
    sph_c: np.ndarray
    sph_r: np.ndarray


def make_room_scene(rng: np.random.Generator, keep_clear: np.ndarray, n_boxes: int = 20,
                    n_spheres: int = 20) -> RoomScene:
    """Boxes (sides U[0.2, 1] m) rest on the floor, spheres (r U[0.1, 0.5] m)
    float at random heights; objects within 0.5 m of a camera are redrawn."""
    lo, hi = [], []
    while len(lo) < n_boxes:
        side = rng.uniform(0.2, 1.0, size=3)
        c = rng.uniform([0.0, 0.0], [6.0, 5.0])
        blo = np.array([c[0] - side[0] / 2, c[1] - side[1] / 2, 0.0])
        bhi = np.array([c[0] + side[0] / 2, c[1] + side[1] / 2, side[2]])
        d = np.maximum(0.0, np.maximum(blo[None] - keep_clear, keep_clear - bhi[None]))
        if np.min(np.linalg.norm(d, axis=1)) < 0.5:
            continue
        lo.append(blo)
        hi.append(bhi)
    cc, rr = [], []
    while len(cc) < n_spheres:
        r = rng.uniform(0.1, 0.5)
        c = rng.uniform([r, r, r], [6.0 - r, 5.0 - r, 3.0 - r])
        if np.min(np.linalg.norm(keep_clear - c[None], axis=1)) - r < 0.5:
            continue
        cc.append(c)
        rr.append(r)
    return RoomScene(np.array(lo), np.array(hi), np.array(cc), np.array(rr))


def _slab_hits(lo, hi, origin, dirs, inv):
    t0 = (lo[None] - origin[None]) * inv
    t1 = (hi[None] - origin[None]) * inv
    tn = np.max(np.minimum(t0, t1), axis=1)
    tf = np.min(np.maximum(t0, t1), axis=1)
    return tn, tf


def room_depth_rays(scene: RoomScene, origin: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Distance along unit rays from a camera inside the room to the first surface."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(np.abs(dirs) > 1e-15, 1.0 / np.where(np.abs(dirs) > 1e-15, dirs, 1.0), 1e30)
    # room interior: exit distance through the walls, floor and ceiling
    _, best = _slab_hits(np.zeros(3), np.array([6.0, 5.0, 3.0]), origin, dirs, inv)
    for lo, hi in zip(scene.box_lo, scene.box_hi):
        tn, tf = _slab_hits(lo, hi, origin, dirs, inv)
        hit = (tf >= tn) & (tn > 0)
        best = np.where(hit & (tn < best), tn, best)
    for c, r in zip(scene.sph_c, scene.sph_r):
        oc = origin - c
        b = dirs @ oc
        disc = b * b - (oc @ oc - r * r)
        ok = disc >= 0
        t = -b - np.sqrt(np.where(ok, disc, 0.0))
        hit = ok & (t > 0)
        best = np.where(hit & (t < best), t, best)
    return best


def depth_view(scene: RoomScene, cam_pose: np.ndarray, rng: np.random.Generator, width: int = 640,
               height: int = 480, f: float = 525.0, noise_k: float = 0.0015) -> np.ndarray:
    """Back-projected depth image in the camera frame (x right, y down, z forward)."""
    u, v = np.meshgrid(np.arange(width, dtype=np.float64), np.arange(height, dtype=np.float64))
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    d_c = np.stack([(u - cx) / f, (v - cy) / f, np.ones_like(u)], -1).reshape(-1, 3)
    norm = np.linalg.norm(d_c, axis=1)
    d_w = (d_c / norm[:, None]) @ cam_pose[:3, :3].T
    t = room_depth_rays(scene, cam_pose[:3, 3], d_w)
    z = t / norm                                   # depth along the optical axis
    z = z + rng.normal(0.0, 1.0, size=z.shape) * noise_k * z * z
    keep = np.isfinite(z) & (z > 0.1)
    return d_c[keep] * z[keep, None]


def voxel_to_count(P: np.ndarray, target: int, lo: float = 0.002, hi: float = 0.5) -> float:
    """Voxel size (bisection) whose centroid downsampling leaves about `target` points."""
    for _ in range(30):
        mid = np.sqrt(lo * hi)
        if len(voxel_centroids(P, mid)) > target:
            lo = mid
        else:
            hi = mid
    return np.sqrt(lo * hi)


def make_config3(instance: int = 0, target_points: int = 20000, trans_m: float = 0.05,
                 angle_deg: float = 3.0) -> PairSpec:
    """RGB-D pair: X = view 1, Z = view 2 after motion M (camera frame); T = M^{-1}."""
    rng = rng_for(3, instance)
    R_wc = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])   # camera z -> world +x
    C1 = rigid(R_wc, [1.0, 2.5, 1.5])
    M = rigid(rotation_about(random_unit(rng), np.deg2rad(angle_deg)), trans_m * random_unit(rng))
    C2 = C1 @ M
    scene = make_room_scene(rng, np.array([C1[:3, 3], C2[:3, 3]]))
    P1 = depth_view(scene, C1, rng)
    P2 = depth_view(scene, C2, rng)
    vox = voxel_to_count(P1, target_points)
    x = voxel_centroids(P1, vox)
    z = voxel_centroids(P2, vox)
    return PairSpec(name=f"c3_rgbd_{instance}", target=np.ascontiguousarray(x, np.float32),
                    source=np.ascontiguousarray(z, np.float32), G=M, length_scale=0.2,
                    length_scale_min=0.025, anneal_factor=0.5, eig_ratio_min=0.01, max_iters=150,
                    max_iters_per_stage=40, extra=dict(voxel=vox))




# --------------------------------------------------------------------------
# Configuration 4: object-scale pairs (unions of 1-4 primitives), uneven sizes.
# --------------------------------------------------------------------------

PRIMITIVES = ("box", "cylinder", "torus", "ellipsoid")


def _uniform_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    return Rotation.from_quat(q / np.linalg.norm(q)).as_matrix()


def _primitive_area(kind: str, dims: np.ndarray) -> float:
    if kind == "box":
        a, b, c = dims
        return 2.0 * (a * b + b * c + a * c)
    if kind == "cylinder":
        r, h = dims[:2]
        return 2.0 * np.pi * r * (r + h)
    if kind == "torus":
        R, r = dims[:2]
        return 4.0 * np.pi ** 2 * R * r
    a, b, c = dims                                          # ellipsoid: Monte-Carlo area
    n = np.random.default_rng(0).normal(size=(20000, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    g = np.sqrt((b * c * n[:, 0]) ** 2 + (a * c * n[:, 1]) ** 2 + (a * b * n[:, 2]) ** 2)
    return 4.0 * np.pi * float(np.mean(g))


def _sample_primitive(rng: np.random.Generator, kind: str, dims: np.ndarray, n: int) -> np.ndarray:
    """n area-uniform points on the closed surface of a primitive in its own frame."""
    if n == 0:
        return np.zeros((0, 3))
    if kind == "box":
        ext = dims
        face_area = np.array([ext[1] * ext[2], ext[0] * ext[2], ext[0] * ext[1]])
        face = rng.choice(6, size=n, p=np.repeat(face_area, 2) / (2.0 * face_area.sum()))
        P = (rng.uniform(size=(n, 3)) - 0.5) * ext
        ax = face // 2
        P[np.arange(n), ax] = np.where(face % 2 == 1, 0.5, -0.5) * ext[ax]
        return P
    if kind == "cylinder":
        r, h = dims[:2]
        side = rng.uniform(size=n) < h / (h + r)                 # lateral 2 pi r h vs caps 2 pi r^2
        th = rng.uniform(0.0, 2.0 * np.pi, size=n)
        rad = np.where(side, r, r * np.sqrt(rng.uniform(size=n)))
        zc = np.where(rng.uniform(size=n) < 0.5, -h / 2, h / 2)
        z = np.where(side, rng.uniform(-h / 2, h / 2, size=n), zc)
        return np.stack([rad * np.cos(th), rad * np.sin(th), z], 1)
    if kind == "torus":
        R, r = dims[:2]
        out = []
        while sum(len(o) for o in out) < n:
            m = 2 * n
            phi = rng.uniform(0.0, 2.0 * np.pi, size=m)
            keep = rng.uniform(size=m) * (R + r) <= R + r * np.cos(phi)
            th = rng.uniform(0.0, 2.0 * np.pi, size=m)
            w = R + r * np.cos(phi)
            out.append(np.stack([w * np.cos(th), w * np.sin(th), r * np.sin(phi)], 1)[keep])
        return np.concatenate(out)[:n]
    a, b, c = dims
    gmax = max(b * c, a * c, a * b)
    out = []
    while sum(len(o) for o in out) < n:
        m = 2 * n
        u = rng.normal(size=(m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        g = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = rng.uniform(size=m) * gmax <= g
        out.append((u * np.array([a, b, c]))[keep])
    return np.concatenate(out)[:n]


@dataclass
class ObjectScene:
    kinds: list
    dims: list
    poses: list
    areas: np.ndarray


def make_object_scene(rng: np.random.Generator) -> ObjectScene:
    """1-4 primitives, characteristic size s ~ U[0.2, 1] m, uniformly random
    orientation, centre uniform in the unit cube."""
    k = int(rng.integers(1, 5))
    kinds, dims, poses = [], [], []
    for _ in range(k):
        kind = PRIMITIVES[int(rng.integers(0, 4))]
        s = rng.uniform(0.2, 1.0)
        if kind == "box":
            d = s * rng.uniform(0.3, 1.0, size=3)
        elif kind == "cylinder":
            d = np.array([s * rng.uniform(0.15, 0.5), s * rng.uniform(0.5, 1.0), 0.0])
        elif kind == "torus":
            R = s * rng.uniform(0.3, 0.5)
            d = np.array([R, R * rng.uniform(0.2, 0.5), 0.0])
        else:
            d = 0.5 * s * rng.uniform(0.3, 1.0, size=3)
        kinds.append(kind)
        dims.append(d)
        poses.append(rigid(_uniform_rotation(rng), rng.uniform(0.0, 1.0, size=3)))
    areas = np.array([_primitive_area(kd, d) for kd, d in zip(kinds, dims)])
    return ObjectScene(kinds, dims, poses, areas)


def sample_object_cloud(scene: ObjectScene, rng: np.random.Generator, n: int, noise: float,
                        outlier_frac: float) -> np.ndarray:
    """n points: area-weighted surface samples of the union with iid Gaussian
    noise, of which a fraction is replaced by uniform outliers in the cloud's
    bounding box; rows in random order."""
    n_out = int(round(outlier_frac * n))
    counts = rng.multinomial(n - n_out, scene.areas / scene.areas.sum())
    parts = [transform_points(T, _sample_primitive(rng, kd, d, int(c)))
             for kd, d, T, c in zip(scene.kinds, scene.dims, scene.poses, counts)]
    P = np.concatenate(parts) + rng.normal(0.0, noise, size=(n - n_out, 3))
    lo, hi = P.min(0), P.max(0)
    P = np.concatenate([P, rng.uniform(lo, hi, size=(n_out, 3))])
    return P[rng.permutation(n)]


def median_nn_spacing(P: np.ndarray) -> float:
    from scipy.spatial import cKDTree
    d, _ = cKDTree(P).query(P, k=2)
    return float(np.median(d[:, 1]))


def make_config4(instance: int = 0, n: int | None = None, n_lo: int = 1000, n_hi: int = 50000,
                 noise: float = 0.005, outlier_frac: float = 0.1, max_angle_deg: float = 30.0,
                 max_trans_m: float = 0.2) -> PairSpec:
    """Object pair `instance` of the batch: independent source/target samples of
    one random union of primitives, N ~ U{n_lo..n_hi} (same N for both clouds);
    target x = G p with G a rotation of U[0, 30] deg about a uniform axis through
    the unit cube's centre followed by a translation of U[0, 0.2] m."""
    rng = rng_for(4, instance)
    scene = make_object_scene(rng)
    N = int(rng.integers(n_lo, n_hi + 1))
    N = N if n is None else int(n)
    angle = np.deg2rad(rng.uniform(0.0, max_angle_deg))
    Rg = rotation_about(random_unit(rng), angle)
    tg = rng.uniform(0.0, max_trans_m) * random_unit(rng)
    c0 = np.full(3, 0.5)
    G = rigid(Rg, c0 - Rg @ c0 + tg)
    z = sample_object_cloud(scene, rng, N, noise, outlier_frac)
    x = transform_points(G, sample_object_cloud(scene, rng, N, noise, outlier_frac))
    x32 = np.ascontiguousarray(x, np.float32)
    ell_min = max(0.01, 2.0 * median_nn_spacing(x32.astype(np.float64)))
    return PairSpec(name=f"c4_objects_{instance}" + ("" if n is None else f"_n{N}"), target=x32,
                    source=np.ascontiguousarray(z, np.float32), G=G, length_scale=0.2,
                    length_scale_min=min(0.2, ell_min), anneal_factor=0.5, eig_ratio_min=0.01,
                    max_iters=200, max_iters_per_stage=40,
                    extra=dict(kinds=list(scene.kinds), angle_deg=float(np.rad2deg(angle))))


def config4_sizes(n_pairs: int = 256, n_lo: int = 1000, n_hi: int = 50000) -> list:
    """Point counts of the first n_pairs object pairs without building clouds
    (replays each pair's scene draws, then its size draw)."""
    out = []
    for i in range(n_pairs):
        rng = rng_for(4, i)
        make_object_scene(rng)
        out.append(int(rng.integers(n_lo, n_hi + 1)))
    return out


# --------------------------------------------------------------------------
# Per-point labels (intensity / colour channels or semantic classes) for the
# labelled objective.  A label is a function of the point's position on the
# underlying surface, so corresponding target and source points carry the same
# label up to the sampling: source points are surface points, target points are
# mapped back by T_true first.
# --------------------------------------------------------------------------

def label_field(P: np.ndarray, dim: int, kind: str, seed: int = 0) -> np.ndarray:
    """float32 [n, dim] labels at surface points P [n, 3].

    kind "colour": channel c is 0.5 + 0.4 sin(w_c . p + phase_c) with |w_c| = 2 rad/m
    (smooth, in (0.1, 0.9)); kind "class": one-hot of the channel with the largest
    such value (a partition into dim regions)."""
    rng = np.random.default_rng(9_000_001 + seed)
    W = np.stack([2.0 * random_unit(rng) for _ in range(dim)])
    phase = rng.uniform(0.0, 2.0 * np.pi, size=dim)
    L = 0.5 + 0.4 * np.sin(np.asarray(P, np.float64) @ W.T + phase)
    if kind == "class":
        L = np.eye(dim)[np.argmax(L, axis=1)]
    elif kind != "colour":
        raise ValueError(f"unknown label kind {kind!r}")
    return np.ascontiguousarray(L, np.float32)


def pair_labels(spec: PairSpec, dim: int, kind: str, seed: int = 0):
    """(target labels, source labels) of a pair, both float32 [n, dim]."""
    surf_t = transform_points(spec.T_true, spec.target.astype(np.float64))
    return (label_field(surf_t, dim, kind, seed), label_field(spec.source.astype(np.float64), dim, kind, seed))


def make_pair(config: int, instance: int = 0) -> PairSpec:
    return CONFIGS[config](instance)


CONFIGS = {1: make_config1, 2: make_config2, 3: make_config3, 4: make_config4, 5: make_config5}
