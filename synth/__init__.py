"""Seeded synthetic inputs shaped like the paper's workloads (Sec. IV: a 10 Hz spinning
multi-beam LiDAR in urban and campus scenes, submaps of consecutive scans, thousands of
matching-cost factors). The datasets themselves are not available; these scenes stand in for
their shapes.

This module only makes inputs: point clouds (FP32 SoA, xyz (3, n) and covariances (6, n) as xx,
xy, xz, yy, yz, zz), world-from-local poses (FP64, row-major 3x4) and factor lists. It holds
none of the registration arithmetic and is shared by the oracle side and the GPU side.

Workloads:
  room()          single 5k-vs-5k unary factor in a 10 x 8 x 3 m box room, res 1.0 m
  urban(scene)    one 32-beam scan (~20k points after a 0.25 m voxel-grid filter) against 8
                  keyframes (union of 3 such scans, ~57k points), binary factors at
                  res 0.25 / 0.5 / 1.0 m
  diff_set()      32 urban scenes x 8 keyframes = 256 factors at res 0.5 m
  global_batch()  400 submaps (10 scans each, 10k-120k points, log-uniform) along a 2 km loop,
                  ~8,000 binary factors between submaps whose origins are within 50 m
  precision_batch()  the same loop moved 4.3-5.0 km away from the world origin

Seeding: numpy.random.SeedSequence(220200242, spawn_key=(workload, item, role)).
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

BASE_SEED = 220200242
W_ROOM, W_URBAN, W_DIFF, W_GLOBAL, W_PRECISION = 0, 1, 2, 3, 4
R_TARGET, R_SOURCE, R_POSE, R_SCENE, R_TRAJ, R_NOISE, R_SUBSAMPLE, R_SIZE = range(8)
GENERATOR_VERSION = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_synth.cpp")
_LIB = os.path.join(_HERE, "libsynth.so")

# LiDAR model (32 beams, -25..+15 deg, 1,800 azimuth steps, 80 m, 1.8 m above the ground)
N_BEAMS = 32
ELEVATIONS = np.deg2rad(np.linspace(-25.0, 15.0, N_BEAMS))
N_AZIMUTH = 1800
MAX_RANGE = 80.0
SENSOR_HEIGHT = 1.8
RANGE_SIGMA = 0.02
DOWNSAMPLE = 0.25
KNN = 10
COV_SCALE = 0.01      # m^2
SCAN_PERIOD = 0.1     # s: one sweep at 10 Hz
COV_FLAT = 1e-3       # eigenvalues (1, 1, 1e-3) * COV_SCALE around the local surface


def rng_for(workload: int, item: int, role: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(BASE_SEED,
                                                        spawn_key=(workload, item, role)))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ------------------------------------------------------------------------------ native part

def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _native():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.synth_raycast.argtypes = [P, I, P, I, P, I, P, I, I, D, P, P, P, I]
        L.synth_downsample.argtypes = [P, I64, D, P]
        L.synth_downsample.restype = I64
        L.synth_plane_cov.argtypes = [P, I64, P, I, D, D, P, I]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def raycast(boxes, cyls, sensors, noise, nthreads=0, return_rays=False):
    """Sensor-frame hit points of every ray of every sensor: list of (m, 3) float64 (and, with
    return_rays, the ray index beam * N_AZIMUTH + azimuth column of each hit)."""
    boxes = np.ascontiguousarray(boxes, np.float64).reshape(-1, 6)
    cyls = np.ascontiguousarray(cyls, np.float64).reshape(-1, 5)
    sensors = np.ascontiguousarray(sensors, np.float64).reshape(-1, 4)
    ns = sensors.shape[0]
    nr = N_BEAMS * N_AZIMUTH
    noise = np.ascontiguousarray(noise, np.float64).reshape(ns, nr)
    out = np.empty((ns, nr, 3))
    valid = np.empty((ns, nr), np.uint8)
    elev = np.ascontiguousarray(ELEVATIONS)
    _native().synth_raycast(_ptr(boxes), boxes.shape[0], _ptr(cyls), cyls.shape[0],
                            _ptr(sensors), ns, _ptr(elev), N_BEAMS, N_AZIMUTH, MAX_RANGE,
                            _ptr(noise), _ptr(out), _ptr(valid), int(nthreads))
    if return_rays:
        return [(out[s][valid[s].astype(bool)], np.flatnonzero(valid[s])) for s in range(ns)]
    return [out[s][valid[s].astype(bool)] for s in range(ns)]


def downsample(pts, res):
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 3)
    out = np.empty_like(pts)
    m = _native().synth_downsample(_ptr(pts), pts.shape[0], float(res), _ptr(out))
    return out[:m].copy()


def plane_covariances(pts, k=KNN, nthreads=0):
    """(6, n) FP32 covariances from each point's k nearest neighbours (itself included)."""
    from scipy.spatial import cKDTree

    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 3)
    n = pts.shape[0]
    kk = min(k, n)
    if n == 0:
        return np.zeros((6, 0), np.float32)
    _, idx = cKDTree(pts).query(pts, k=kk, workers=nthreads if nthreads > 0 else -1)
    idx = np.ascontiguousarray(np.asarray(idx).reshape(n, kk), np.int64)
    out = np.empty((6, n), np.float32)
    _native().synth_plane_cov(_ptr(pts), n, _ptr(idx), kk, COV_SCALE, COV_FLAT, _ptr(out),
                              int(nthreads))
    return out


# ------------------------------------------------------------------------------ geometry

def rot_z(yaw):
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def axis_angle(v):
    v = np.asarray(v, np.float64)
    th = np.linalg.norm(v)
    if th < 1e-15:
        return np.eye(3)
    k = v / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def pose(R, t):
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def inv(T):
    R, t = T[:3, :3], T[:3, 3]
    return pose(R.T, -R.T @ t)


def to12(T):
    return np.ascontiguousarray(np.asarray(T, np.float64)[:3, :4].reshape(12))


def unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def transform(T, pts):
    """pts (m, 3) -> (m, 3)."""
    return pts @ T[:3, :3].T + T[:3, 3]


def soa(pts):
    return np.ascontiguousarray(np.asarray(pts, np.float64).T.astype(np.float32))


# ------------------------------------------------------------------------------ room (C0)

_ROOM_HALF = np.array([5.0, 4.0, 1.5])


def _room_samples(rng, n):
    """Uniform samples on the 6 faces of the room (area-weighted) plus N(0, 0.01^2) noise."""
    hx, hy, hz = _ROOM_HALF
    faces = [  # (axis, sign, area)
        (2, -1, 4 * hx * hy), (2, 1, 4 * hx * hy), (0, -1, 4 * hy * hz), (0, 1, 4 * hy * hz),
        (1, -1, 4 * hx * hz), (1, 1, 4 * hx * hz)]
    areas = np.array([f[2] for f in faces])
    which = rng.choice(len(faces), size=n, p=areas / areas.sum())
    u = rng.uniform(-1.0, 1.0, size=(n, 3)) * _ROOM_HALF
    normals = np.zeros((n, 3))
    for i, (ax, sg, _) in enumerate(faces):
        sel = which == i
        u[sel, ax] = sg * _ROOM_HALF[ax]
        normals[sel, ax] = 1.0
    u += rng.normal(scale=0.01, size=(n, 3))
    return u, normals


def _plane_cov_from_normals(normals):
    n = normals
    g = 1.0 - COV_FLAT
    c6 = np.stack([1 - g * n[:, 0] ** 2, -g * n[:, 0] * n[:, 1], -g * n[:, 0] * n[:, 2],
                   1 - g * n[:, 1] ** 2, -g * n[:, 1] * n[:, 2], 1 - g * n[:, 2] ** 2])
    return np.ascontiguousarray((COV_SCALE * c6).astype(np.float32))


def room(item: int = 0, n: int = 5000):
    """Single unary factor in a 10 x 8 x 3 m room (res 1.0: the walls at x = +-5 m and
    y = +-4 m lie on voxel faces). The target pose is the identity; the source cloud is a fresh
    sample moved by a random G (angle <= 5 deg, translation <= 0.3 m). Linearization poses:
    'identity', 'truth' (= G), 'perturbed' (= G Exp(xi), |omega| = 0.5 deg, |rho| = 5 cm)."""
    rt, rs, rp = rng_for(W_ROOM, item, R_TARGET), rng_for(W_ROOM, item, R_SOURCE), \
        rng_for(W_ROOM, item, R_POSE)
    tp, tn = _room_samples(rt, n)
    sp, sn = _room_samples(rs, n)
    G = pose(axis_angle(unit(rp) * math.radians(rp.uniform(0, 5.0))),
             unit(rp) * rp.uniform(0, 0.3))
    Gi = inv(G)
    sp_local = transform(Gi, sp)
    sn_local = sn @ Gi[:3, :3].T
    xi_w = unit(rp) * math.radians(0.5)
    xi_t = unit(rp) * 0.05
    P = pose(axis_angle(xi_w), xi_t)
    return {
        "res": 1.0,
        "target": (soa(tp), _plane_cov_from_normals(tn)),
        "source": (soa(sp_local), _plane_cov_from_normals(sn_local)),
        "T_target": to12(np.eye(4)),
        "T_source": {"identity": to12(np.eye(4)), "truth": to12(G), "perturbed": to12(G @ P)},
        "G": G,
    }


# ------------------------------------------------------------------------------ urban scenes

def _poly_dist(points, poly):
    """Distance from each of points (m, 2) to the densely sampled polyline poly (k, 2)."""
    d = np.full(points.shape[0], np.inf)
    for s in range(0, poly.shape[0], 512):
        seg = poly[s:s + 512]
        dd = np.sqrt(((points[:, None, :] - seg[None, :, :]) ** 2).sum(-1)).min(1)
        d = np.minimum(d, dd)
    return d


def _rect_dist(cx, cy, hx, hy, poly):
    dx = np.maximum(np.abs(poly[:, 0] - cx) - hx, 0.0)
    dy = np.maximum(np.abs(poly[:, 1] - cy) - hy, 0.0)
    return float(np.sqrt(dx * dx + dy * dy).min())


def _densify(path, step=0.25):
    out = [path[:1]]
    for a, b in zip(path[:-1], path[1:]):
        L = np.linalg.norm(b - a)
        k = max(1, int(math.ceil(L / step)))
        out.append(a + (b - a) * (np.arange(1, k + 1)[:, None] / k))
    return np.concatenate(out)


def make_scene(rng, path, n_boxes, n_poles):
    """Boxes (footprint sides and height U(10, 40) m, centres 15-80 m from the path) and poles
    (radius U(0.1, 0.3) m, height U(4, 8) m, 5-60 m from the path), all clear of an 8 m road
    corridor around the path."""
    poly = _densify(np.asarray(path)[:, :2])
    lo = poly.min(0) - 80.0
    hi = poly.max(0) + 80.0
    boxes, poles = [], []
    tries = 0
    while len(boxes) < n_boxes and tries < 200 * n_boxes:
        tries += 1
        c = rng.uniform(lo, hi)
        hx, hy = rng.uniform(10, 40, size=2) / 2
        h = rng.uniform(10, 40)
        dc = _poly_dist(c[None], poly)[0]
        if not (15.0 <= dc <= 80.0) or _rect_dist(c[0], c[1], hx, hy, poly) < 4.0:
            continue
        boxes.append([c[0] - hx, c[1] - hy, 0.0, c[0] + hx, c[1] + hy, h])
    tries = 0
    while len(poles) < n_poles and tries < 200 * n_poles:
        tries += 1
        c = rng.uniform(lo + 20.0, hi - 20.0)
        r = rng.uniform(0.1, 0.3)
        h = rng.uniform(4, 8)
        dc = _poly_dist(c[None], poly)[0]
        if not (5.0 <= dc <= 60.0) or dc - r < 4.0:
            continue
        poles.append([c[0], c[1], r, 0.0, h])
    return np.array(boxes).reshape(-1, 6), np.array(poles).reshape(-1, 5)


def scan_pose(x, y, yaw):
    return pose(rot_z(yaw), [x, y, SENSOR_HEIGHT])


def _scan_points(boxes, poles, xyyaw, workload, scan_ids, nthreads):
    sensors = np.array([[x, y, SENSOR_HEIGHT, yaw] for x, y, yaw in xyyaw])
    nr = N_BEAMS * N_AZIMUTH
    noise = np.stack([rng_for(workload, int(s), R_NOISE).normal(scale=RANGE_SIGMA, size=nr)
                      for s in scan_ids])
    return raycast(boxes, poles, sensors, noise, nthreads=nthreads)


def _urban_setup(scene, workload):
    rtraj = rng_for(workload, scene, R_TRAJ)
    n_frames = 11                    # frames 0..10; source = 10; keyframes 9..2 use k-2..k
    yaw = rtraj.uniform(0, 2 * math.pi)
    xyyaw = []
    x = y = 0.0
    for f in range(n_frames):
        xyyaw.append((x, y, yaw))
        x += math.cos(yaw)
        y += math.sin(yaw)
        yaw += math.radians(rtraj.uniform(-2.0, 2.0))
    path = np.array([[a, b] for a, b, _ in xyyaw])
    boxes, poles = make_scene(rng_for(workload, scene, R_SCENE), path, 20, 50)
    scan_ids = [scene * 1000 + f for f in range(n_frames)]
    return boxes, poles, xyyaw, scan_ids


def raw_scan(scene: int = 0, frame: int = 10, workload: int = W_URBAN):
    """One raw sweep of an urban scene (the frames of `urban`) in its sensor frame, before any
    downsampling: (3, n) float32 points and (n,) float32 timestamps in [0, SCAN_PERIOD), the
    time at which the spinning sensor's azimuth column of each ray fired."""
    boxes, poles, xyyaw, scan_ids = _urban_setup(scene, workload)
    x, y, yaw = xyyaw[frame]
    sensors = np.array([[x, y, SENSOR_HEIGHT, yaw]])
    nr = N_BEAMS * N_AZIMUTH
    noise = rng_for(workload, scan_ids[frame], R_NOISE).normal(scale=RANGE_SIGMA, size=(1, nr))
    pts, rays = raycast(boxes, poles, sensors, noise, return_rays=True)[0]
    t = (rays % N_AZIMUTH) * (SCAN_PERIOD / N_AZIMUTH)
    return soa(pts), np.ascontiguousarray(t.astype(np.float32))


def urban(scene: int = 0, workload: int = W_URBAN, resolutions=(0.25, 0.5, 1.0),
          nthreads: int = 0):
    """One odometry step: the newest scan (source) against 8 keyframes (targets). Each
    keyframe cloud is the union of 3 consecutive scans in the keyframe's frame. The trajectory
    advances 1 m per frame with a yaw increment U(-2, 2) deg per frame. Returns clouds, poses
    and one binary factor per (keyframe, resolution)."""
    boxes, poles, xyyaw, scan_ids = _urban_setup(scene, workload)
    n_frames = len(xyyaw)
    scans = _scan_points(boxes, poles, xyyaw, workload, scan_ids, nthreads)
    T = [scan_pose(*p) for p in xyyaw]
    scans = [downsample(sc, DOWNSAMPLE) for sc in scans]   # each scan on its own
    src_pts = scans[-1]
    source = (soa(src_pts), plane_covariances(src_pts, nthreads=nthreads))
    targets, T_key = [], []
    for k in range(n_frames - 2, n_frames - 10, -1):
        pts = np.concatenate([transform(inv(T[k]) @ T[j], scans[j]) for j in (k - 2, k - 1, k)])
        targets.append((soa(pts), plane_covariances(pts, nthreads=nthreads)))
        T_key.append(to12(T[k]))
    rp = rng_for(workload, scene, R_POSE)
    P = pose(axis_angle(rp.normal(scale=math.radians(1.0), size=3)), rp.normal(scale=0.1, size=3))
    factors = []  # (keyframe index, resolution)
    for ki in range(len(targets)):
        for res in resolutions:
            factors.append((ki, float(res)))
    return {
        "source": source,
        "targets": targets,
        "T_targets": np.array(T_key),
        "T_source_truth": to12(T[-1]),
        "T_source": to12(T[-1] @ P),
        "factors": factors,
    }


def diff_set(n_scenes: int = 32, res: float = 0.5):
    """256 factors = 32 urban scenes x 8 keyframes, res 0.5 m (scenes built in parallel)."""
    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        return list(ex.map(lambda s: urban(s, workload=W_DIFF, resolutions=(res,), nthreads=1),
                           range(n_scenes)))


# ------------------------------------------------------------------------------ global loop

LOOP_RADIUS = 50.0
LOOP_STRAIGHT_X = 600.0
LOOP_STRAIGHT_Y = (2000.0 - 2 * math.pi * LOOP_RADIUS - 2 * LOOP_STRAIGHT_X) / 2  # 2 km total
N_SCANS = 4000
SCANS_PER_SUBMAP = 10
SUBMAP_MIN, SUBMAP_MAX = 10_000, 120_000
FACTOR_RADIUS = 50.0


def loop_point(s):
    """Position and heading at arc length s on the rounded rectangle, counter-clockwise from
    the left end of its lower straight."""
    r, a, b = LOOP_RADIUS, LOOP_STRAIGHT_X, LOOP_STRAIGHT_Y
    q = math.pi * r / 2
    segs = [("line", (-a / 2, -b / 2 - r), 0.0, a), ("arc", (a / 2, -b / 2), -math.pi / 2, q),
            ("line", (a / 2 + r, -b / 2), math.pi / 2, b), ("arc", (a / 2, b / 2), 0.0, q),
            ("line", (a / 2, b / 2 + r), math.pi, a), ("arc", (-a / 2, b / 2), math.pi / 2, q),
            ("line", (-a / 2 - r, b / 2), -math.pi / 2, b),
            ("arc", (-a / 2, -b / 2), math.pi, q)]
    s = s % sum(g[3] for g in segs)
    for i, (kind, p, ang, length) in enumerate(segs):
        if s <= length or i == len(segs) - 1:
            if kind == "line":
                return p[0] + s * math.cos(ang), p[1] + s * math.sin(ang), ang
            th = ang + s / r
            return p[0] + r * math.cos(th), p[1] + r * math.sin(th), th + math.pi / 2
        s -= length
    raise AssertionError("unreachable")


def _submap(boxes, poles, scans_xyyaw, scan_ids, sm, workload, nthreads):
    pts_scans = _scan_points(boxes, poles, scans_xyyaw, workload, scan_ids, nthreads)
    T = [scan_pose(*p) for p in scans_xyyaw]
    origin = T[SCANS_PER_SUBMAP // 2]
    pts = np.concatenate([transform(inv(origin) @ Tj, downsample(P, DOWNSAMPLE))
                          for Tj, P in zip(T, pts_scans)])
    rs = rng_for(W_GLOBAL, sm, R_SIZE)
    size = int(round(math.exp(rs.uniform(math.log(SUBMAP_MIN), math.log(SUBMAP_MAX)))))
    keep = np.sort(rng_for(W_GLOBAL, sm, R_SUBSAMPLE).permutation(pts.shape[0])[:size])
    sub = pts[keep]
    cov = plane_covariances(sub, nthreads=nthreads)
    return soa(sub), cov, origin, size, pts.shape[0]


def _cache_path(name):
    d = os.environ.get("VGICP_SYNTH_CACHE", os.path.join("/tmp", "vgicp_synth_cache"))
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, name)


def global_batch(n_submaps: int = N_SCANS // SCANS_PER_SUBMAP, factor_radius=FACTOR_RADIUS,
                 cache: bool = True, progress=None):
    """400 submaps of 10 consecutive scans along a 2 km loop (scan spacing 0.5 m), origin =
    pose of the centre scan; each scan downsampled at 0.25 m, the 10 unioned in the submap
    frame (~190k points), a uniform subsample to a log-uniform size in [10k, 120k] points,
    then covariances from each point's neighbours in the subsampled cloud. Factors: all ordered pairs
    (i, j), i != j, with origins within factor_radius metres; target map = j, source = i.
    Linearization poses: truth perturbed by N(0, 0.5 deg) and N(0, 0.2 m) per submap."""
    key = hashlib.sha1(repr((GENERATOR_VERSION, n_submaps, float(factor_radius),
                             BASE_SEED)).encode()).hexdigest()[:16]
    path = _cache_path(f"global_{key}.npz")
    if cache and os.path.exists(path):
        z = np.load(path)
        clouds = [(z[f"xyz{i}"], z[f"cov{i}"]) for i in range(n_submaps)]
        return {"clouds": clouds, "T_truth": z["T_truth"], "T": z["T"],
                "factors": z["factors"], "union_sizes": z["union_sizes"],
                "target_sizes": z["target_sizes"]}
    n_scans = n_submaps * SCANS_PER_SUBMAP
    spacing = 0.5
    xyyaw = [loop_point(i * spacing) for i in range(n_scans)]
    path_xy = np.array([[a, b] for a, b, _ in xyyaw] + [list(xyyaw[0][:2])])
    # scene density of the urban scenes, spread along the loop's band
    L = n_scans * spacing
    n_boxes = int(round(20 * L * 160.0 / (math.pi * 80.0 ** 2 + 2 * 80.0 * 10.0)))
    n_poles = int(round(50 * L * 120.0 / (math.pi * 60.0 ** 2 + 2 * 60.0 * 10.0)))
    boxes, poles = make_scene(rng_for(W_GLOBAL, 0, R_SCENE), path_xy, n_boxes, n_poles)
    workers = _threads()

    def one(sm):
        ids = list(range(sm * SCANS_PER_SUBMAP, (sm + 1) * SCANS_PER_SUBMAP))
        out = _submap(boxes, poles, [xyyaw[i] for i in ids], ids, sm, W_GLOBAL, 1)
        if progress:
            progress(sm)
        return out

    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, range(n_submaps)))
    clouds = [(r[0], r[1]) for r in res]
    T_truth = np.stack([to12(r[2]) for r in res])
    centres = T_truth.reshape(-1, 3, 4)[:, :, 3]
    factors = []
    for i in range(n_submaps):
        for j in range(n_submaps):
            if i != j and np.linalg.norm(centres[i] - centres[j]) <= factor_radius:
                factors.append((j, i, j, i, 1))   # map j, cloud i, target pose j, source pose i
    factors = np.array(factors, np.int32).reshape(-1, 5)
    rp = rng_for(W_GLOBAL, 0, R_POSE)
    T = []
    for i in range(n_submaps):
        P = pose(axis_angle(rp.normal(scale=math.radians(0.5), size=3)),
                 rp.normal(scale=0.2, size=3))
        T.append(to12(np.vstack([T_truth[i].reshape(3, 4), [0, 0, 0, 1]]) @ P))
    out = {"clouds": clouds, "T_truth": T_truth, "T": np.stack(T), "factors": factors,
           "union_sizes": np.array([r[4] for r in res]),
           "target_sizes": np.array([r[3] for r in res])}
    if cache:
        tmp = path + f".tmp{os.getpid()}.npz"
        arrs = {f"xyz{i}": c[0] for i, c in enumerate(clouds)}
        arrs.update({f"cov{i}": c[1] for i, c in enumerate(clouds)})
        np.savez(tmp, T_truth=out["T_truth"], T=out["T"], factors=factors,
                 union_sizes=out["union_sizes"], target_sizes=out["target_sizes"], **arrs)
        os.replace(tmp, path)
    return out


PRECISION_OFFSET = np.array([4650.0, 0.0, 0.0])


def precision_batch(**kw):
    """The global loop moved so that submap origins lie about 4.3-5.0 km from the world
    origin. Points stay submap-local FP32; only the FP64 poses move."""
    g = global_batch(**kw)
    out = dict(g)
    for k in ("T_truth", "T"):
        T = g[k].reshape(-1, 3, 4).copy()
        T[:, :, 3] += PRECISION_OFFSET
        out[k] = T.reshape(-1, 12)
    return out


def subset(batch, n_factors, stride=None):
    """A deterministic subset of a batch's factors (every stride-th), for oracle checks."""
    F = batch["factors"].shape[0]
    stride = stride or max(1, F // n_factors)
    return batch["factors"][::stride][:n_factors]
