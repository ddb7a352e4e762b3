"""Seeded synthetic inputs: scenes of Gaussian primitives, cameras and rays.

This module only builds inputs.  It holds none of the rendering method's
arithmetic (no ray integral, transmittance, sampling or shading); both the GPU
library and the CPU oracle consume what it returns.  Every generator takes a
seed and uses numpy's PCG64, so a workload is reproduced exactly from its name.

Scene dictionaries hold float32 / int32 numpy arrays:
  mean [n,3], scale [n,3] (>0), rotation [n,4] (w,x,y,z quaternion, any norm),
  density [n] (peak value of the Gaussian), albedo [n,3], roughness [n],
  emission [n,3] (radiance, 0 = not emissive), material [n] (0 diffuse, 1 glossy,
  2 / 3 SGGX microflakes with a Lambertian / Disney-style base) and, where
  material 2 or 3 occurs, sggx [n,6] (the SGGX matrix: xx, yy, zz, xy, xz, yz)
  and optionally metallic [n] (material 3)
and a "bounds" entry (lo, hi) used by camera set-up and the cache's position
normalisation.

The workloads stand in for the paper's scenes, whose assets are not available:
  tiny_random  -- 1,000 random Gaussians in the unit cube (the shape of the
                  paper's random-scene convergence experiment, Sec. 5.2),
  mixed_100k   -- 70% flat surface Gaussians on spheres and planes, 30% a
                  volumetric cloud,
  room_5p5m    -- a room of boxes and planes tiled with flat Gaussians plus 40
                  clusters of elongated Gaussians and two emissive panels, at
                  the primitive count of the paper's largest scene (~5.5M).
Flat primitives follow the paper's mesh-conversion rule (Sec. 7.1): tangent
scale sqrt(eps*k*A/N) with eps = 0.01, k = 16, thin axis 1/100 of it along the
surface normal, centres on a jittered grid.  Each one's density is set from an
opacity alpha ~ U[0.6, 1]: half the ray integral through its centre at normal
incidence equals alpha.  The cover of such a tiling (k eps times the
truncated kernel's footprint) is 0.98, so the mean F of a surface at normal
incidence is about 0.8: most such rays pass it partially, and it saturates
across its several overlapping layers at oblique incidence.
"""
from __future__ import annotations

import math

import numpy as np

EPS = 0.01
K_COVER = 16.0
# ray integral through the centre of an untruncated-at-r normal-incidence flat
# Gaussian is d * sqrt(2 pi) * s_n * erf(r / sqrt 2); this constant turns a
# chosen normal-incidence opacity alpha (= half that integral) into a density.
_R_CUT = math.sqrt(-2.0 * math.log(EPS))
_CENTRE_INTEGRAL = math.sqrt(2.0 * math.pi) * math.erf(_R_CUT / math.sqrt(2.0))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _random_quat(rng, n):
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _quat_from_frames(t1, t2, nrm):
    """Unit quaternions (w,x,y,z) of rotations whose columns are (t1, t2, nrm)."""
    R = np.stack([t1, t2, nrm], axis=2)  # [n,3,3], columns
    m00, m11, m22 = R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]
    tr = m00 + m11 + m22
    q = np.zeros((R.shape[0], 4))
    # Shepperd's method, choosing the largest diagonal term for stability
    c0 = tr > 0
    s = np.sqrt(np.maximum(tr + 1.0, 1e-30)) * 2
    q[c0, 0] = 0.25 * s[c0]
    q[c0, 1] = (R[c0, 2, 1] - R[c0, 1, 2]) / s[c0]
    q[c0, 2] = (R[c0, 0, 2] - R[c0, 2, 0]) / s[c0]
    q[c0, 3] = (R[c0, 1, 0] - R[c0, 0, 1]) / s[c0]
    c1 = (~c0) & (m00 > m11) & (m00 > m22)
    s = np.sqrt(np.maximum(1.0 + m00 - m11 - m22, 1e-30)) * 2
    q[c1, 0] = (R[c1, 2, 1] - R[c1, 1, 2]) / s[c1]
    q[c1, 1] = 0.25 * s[c1]
    q[c1, 2] = (R[c1, 0, 1] + R[c1, 1, 0]) / s[c1]
    q[c1, 3] = (R[c1, 0, 2] + R[c1, 2, 0]) / s[c1]
    c2 = (~c0) & (~c1) & (m11 > m22)
    s = np.sqrt(np.maximum(1.0 + m11 - m00 - m22, 1e-30)) * 2
    q[c2, 0] = (R[c2, 0, 2] - R[c2, 2, 0]) / s[c2]
    q[c2, 1] = (R[c2, 0, 1] + R[c2, 1, 0]) / s[c2]
    q[c2, 2] = 0.25 * s[c2]
    q[c2, 3] = (R[c2, 1, 2] + R[c2, 2, 1]) / s[c2]
    c3 = (~c0) & (~c1) & (~c2)
    s = np.sqrt(np.maximum(1.0 + m22 - m00 - m11, 1e-30)) * 2
    q[c3, 0] = (R[c3, 1, 0] - R[c3, 0, 1]) / s[c3]
    q[c3, 1] = (R[c3, 0, 2] + R[c3, 2, 0]) / s[c3]
    q[c3, 2] = (R[c3, 1, 2] + R[c3, 2, 1]) / s[c3]
    q[c3, 3] = 0.25 * s[c3]
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _tangent_frame(nrm, angle):
    """Two unit tangents orthogonal to unit normals, rotated in-plane by angle."""
    helper = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    a = np.cross(nrm, helper)
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(nrm, a)
    c, s = np.cos(angle)[:, None], np.sin(angle)[:, None]
    return c * a + s * b, -s * a + c * b


def _flat(rng, centres, normals, s_t, thin, alpha_lo=0.6, alpha_hi=1.0):
    """Flat primitives at given centres with normals; returns partial scene."""
    n = centres.shape[0]
    t1, t2 = _tangent_frame(normals, rng.uniform(0, 2 * np.pi, n))
    q = _quat_from_frames(t1, t2, normals)
    s_t = np.broadcast_to(np.asarray(s_t, dtype=np.float64), (n,))
    s_n = s_t * thin
    scale = np.stack([s_t, s_t, s_n], axis=1)
    alpha = rng.uniform(alpha_lo, alpha_hi, n)
    dens = 2.0 * alpha / (_CENTRE_INTEGRAL * s_n)
    return centres, scale, q, dens


def _grid_on_rect(rng, origin, eu, ev, w, h, cell, jitter=0.5):
    """Jittered-grid points on the rectangle origin + [0,w] eu + [0,h] ev."""
    nu = max(1, int(round(w / cell)))
    nv = max(1, int(round(h / cell)))
    iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    iu = iu.ravel().astype(np.float64)
    iv = iv.ravel().astype(np.float64)
    fu = (iu + 0.5 + jitter * rng.uniform(-0.5, 0.5, iu.shape)) / nu * w
    fv = (iv + 0.5 + jitter * rng.uniform(-0.5, 0.5, iv.shape)) / nv * h
    return origin[None, :] + fu[:, None] * eu[None, :] + fv[:, None] * ev[None, :]


def _sphere_points(rng, centre, radius, n):
    """Quasi-uniform points on a sphere (golden-angle spiral, jittered)."""
    i = np.arange(n) + 0.5 + 0.25 * rng.uniform(-1, 1, n)
    z = 1.0 - 2.0 * i / n
    phi = np.pi * (3.0 - np.sqrt(5.0)) * np.arange(n) + rng.uniform(0, 2 * np.pi)
    rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    nrm = np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)
    return centre[None, :] + radius * nrm, nrm


def _finish(parts, rng, *, albedo_lo, albedo_hi, rough_lo, rough_hi, glossy_frac):
    mean = np.concatenate([p[0] for p in parts])
    scale = np.concatenate([p[1] for p in parts])
    rot = np.concatenate([p[2] for p in parts])
    dens = np.concatenate([p[3] for p in parts])
    n = mean.shape[0]
    albedo = rng.uniform(albedo_lo, albedo_hi, (n, 3))
    rough = rng.uniform(rough_lo, rough_hi, n)
    material = (rng.uniform(0, 1, n) < glossy_frac).astype(np.int32)
    return {
        "mean": mean.astype(np.float32),
        "scale": scale.astype(np.float32),
        "rotation": rot.astype(np.float32),
        "density": dens.astype(np.float32),
        "albedo": albedo.astype(np.float32),
        "roughness": rough.astype(np.float32),
        "emission": np.zeros((n, 3), np.float32),
        "material": material,
    }


def tiny_random(seed: int = 0, n: int = 1000, n_emit: int = 10, emit: float = 5.0) -> dict:
    """1,000 random Gaussians in the unit cube: means U[0,1]^3, per-axis scales
    log-uniform in [0.005, 0.05], random rotations, peak density U[0.5, 5],
    diffuse albedo U[0.2, 0.8]^3, n_emit of them emissive with radiance emit."""
    rng = _rng(seed)
    mean = rng.uniform(0, 1, (n, 3))
    scale = _loguniform(rng, 0.005, 0.05, (n, 3))
    q = _random_quat(rng, n)
    dens = rng.uniform(0.5, 5.0, n)
    sc = _finish([(mean, scale, q, dens)], rng, albedo_lo=0.2, albedo_hi=0.8, rough_lo=0.5,
                 rough_hi=0.5, glossy_frac=0.0)
    idx = rng.choice(n, size=min(n_emit, n), replace=False)
    sc["emission"][idx] = emit
    sc["bounds"] = (np.zeros(3, np.float32), np.ones(3, np.float32))
    return sc


def needles(seed: int = 4, n: int = 3000, n_emit: int = 30, emit: float = 5.0) -> dict:
    """A ball of long thin Gaussians (long scale 5-20x the two equal short
    ones, short scale log-uniform in [0.003, 0.01]), means N(0.5, 0.12^2) per
    axis, random rotations, peak density U[5, 50]: the shape of the elongated
    clusters of the room workload, small enough for the oracle.  The BVH cuts
    these primitives into slabs along their long axis."""
    rng = _rng(seed)
    mean = rng.normal(0.5, 0.12, (n, 3))
    short = _loguniform(rng, 0.003, 0.01, n)
    ratio = rng.uniform(5.0, 20.0, n)
    scale = np.stack([short * ratio, short, short], 1)
    q = _random_quat(rng, n)
    dens = rng.uniform(5.0, 50.0, n)
    sc = _finish([(mean, scale, q, dens)], rng, albedo_lo=0.2, albedo_hi=0.8, rough_lo=0.1,
                 rough_hi=1.0, glossy_frac=0.5)
    idx = rng.choice(n, size=min(n_emit, n), replace=False)
    sc["emission"][idx] = emit
    sc["bounds"] = (np.zeros(3, np.float32), np.ones(3, np.float32))
    return sc


def overlap_pile(seed: int = 5, n: int = 40, dens_lo: float = 0.02, dens_hi: float = 0.25) -> dict:
    """n large, faint Gaussians piled on one point: means N(0.5, 0.02^2) per
    axis, scales log-uniform in [0.15, 0.3] per axis, random rotations, peak
    density U[dens_lo, dens_hi].  Every ray through the middle overlaps all
    of them at once, the case that needs more than the sweep's 16-entry
    buffer; some rays saturate inside the pile, others cross it."""
    rng = _rng(seed)
    mean = rng.normal(0.5, 0.02, (n, 3))
    scale = _loguniform(rng, 0.15, 0.3, 3 * n).reshape(n, 3)
    q = _random_quat(rng, n)
    dens = rng.uniform(dens_lo, dens_hi, n)
    sc = _finish([(mean, scale, q, dens)], rng, albedo_lo=0.2, albedo_hi=0.8, rough_lo=0.1,
                 rough_hi=1.0, glossy_frac=0.5)
    sc["emission"][: max(1, n // 10)] = 5.0
    sc["bounds"] = (np.zeros(3, np.float32), np.ones(3, np.float32))
    return sc


def mixed_100k(seed: int = 1, n_flat: int = 70_000, n_cloud: int = 30_000,
               n_emit: int = 1_000, emit: float = 5.0) -> dict:
    """70% flat Gaussians (one axis 100x thinner, opacity U[0.6, 1]) on 10
    spheres and 10 square planes, 30% a volumetric cloud; half diffuse, half
    glossy (roughness U[0.05, 1]); 1% emissive."""
    rng = _rng(seed)
    shapes = []
    for _ in range(10):
        shapes.append(("sphere", rng.uniform(0.2, 0.8, 3), rng.uniform(0.05, 0.2)))
    for _ in range(10):
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        shapes.append(("plane", rng.uniform(0.2, 0.8, 3), nrm, rng.uniform(0.2, 0.6)))
    areas = np.array([4 * np.pi * s[2] ** 2 if s[0] == "sphere" else s[3] ** 2 for s in shapes])
    cell = math.sqrt(areas.sum() / n_flat)
    s_t = math.sqrt(EPS * K_COVER) * cell
    parts = []
    for s in shapes:
        if s[0] == "sphere":
            m = int(round(4 * np.pi * s[2] ** 2 / cell ** 2))
            pts, nrm = _sphere_points(rng, s[1], s[2], m)
        else:
            c, nrm1, side = s[1], s[2], s[3]
            t1, t2 = _tangent_frame(nrm1[None, :], rng.uniform(0, 2 * np.pi, 1))
            o = c - 0.5 * side * (t1[0] + t2[0])
            pts = _grid_on_rect(rng, o, t1[0], t2[0], side, side, cell)
            nrm = np.broadcast_to(nrm1, pts.shape).copy()
        parts.append(_flat(rng, pts, nrm, s_t, 0.01))
    # volumetric cloud: a ball of small random Gaussians
    centre = rng.uniform(0.3, 0.7, 3)
    d = rng.normal(size=(n_cloud, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = 0.2 * rng.uniform(0, 1, n_cloud) ** (1.0 / 3.0)
    cmean = centre[None, :] + rad[:, None] * d
    cscale = _loguniform(rng, 0.002, 0.006, (n_cloud, 3))
    parts.append((cmean, cscale, _random_quat(rng, n_cloud), rng.uniform(1.0, 10.0, n_cloud)))
    sc = _finish(parts, rng, albedo_lo=0.2, albedo_hi=0.8, rough_lo=0.05, rough_hi=1.0,
                 glossy_frac=0.5)
    n = sc["mean"].shape[0]
    idx = rng.choice(n, size=min(n_emit, n), replace=False)
    sc["emission"][idx] = emit
    sc["bounds"] = (np.zeros(3, np.float32), np.ones(3, np.float32))
    return sc


ROOM = np.array([8.0, 3.0, 8.0])


def room_5p5m(seed: int = 2, n_surface: int = 4_300_000, n_clusters: int = 40,
              per_cluster: int = 30_000, panel_radiance: float = 158.0, panel_size: float = 1.0) -> dict:
    """An 8 x 3 x 8 m room (6 walls), 60 boxes on the floor, 12 free planes and
    two 1 x 1 m emissive ceiling panels, all tiled with flat Gaussians
    (n_surface in total, thin axis 1/100 of the tangent scale, opacity
    U[0.6, 1]), plus n_clusters clusters of elongated Gaussians
    (20:1:1, short scale log-uniform [0.5, 2] mm, spread 0.15 m, peak density
    U[8, 80] /m).  Albedo U[0.1, 0.9]^3, roughness U[0.02, 1], 50/50 diffuse /
    glossy.  The panel radiance was set once so that the mean pixel of a
    16-spp 1920x1080 render at depth 12, clamped to [0, 1], is 0.25
    (transport is linear in emission: one render at radiance 1200 had a
    clamped mean of 0.563, and scaling that image by 0.1313 gives 0.25)."""
    rng = _rng(seed)
    X, Y, Z = ROOM
    rects = []  # (origin, eu, ev, w, h, normal, emissive)

    def add(o, eu, ev, w, h, emissive=False):
        o, eu, ev = np.asarray(o, float), np.asarray(eu, float), np.asarray(ev, float)
        nrm = np.cross(eu, ev)
        nrm /= np.linalg.norm(nrm)
        rects.append((o, eu, ev, w, h, nrm, emissive))

    ex, ey, ez = np.eye(3)
    add([0, 0, 0], ex, ez, X, Z)            # floor
    # ceiling, with an opening above each emissive panel (a closed ceiling
    # 1 cm above a two-sided emitter traps light in the gap)
    P_ = panel_size
    panels = ((2.5 - P_ / 2, 4.0 - P_ / 2), (5.5 - P_ / 2, 4.0 - P_ / 2))  # (x, z) corners
    z0, z1 = 4.0 - P_ / 2, 4.0 + P_ / 2
    add([0, Y, 0], ex, ez, X, z0)
    add([0, Y, z1], ex, ez, X, Z - z1)
    xs = [0.0, panels[0][0], panels[0][0] + P_, panels[1][0], panels[1][0] + P_, X]
    for a, b in ((xs[0], xs[1]), (xs[2], xs[3]), (xs[4], xs[5])):
        if b > a:
            add([a, Y, z0], ex, ez, b - a, P_)
    add([0, 0, 0], ex, ey, X, Y)            # wall z = 0
    add([0, 0, Z], ex, ey, X, Y)            # wall z = Z
    add([0, 0, 0], ez, ey, Z, Y)            # wall x = 0
    add([X, 0, 0], ez, ey, Z, Y)            # wall x = X
    for _ in range(60):
        w, h, d = rng.uniform(0.3, 1.5, 3)
        cx, cz = rng.uniform(0.8, X - 0.8), rng.uniform(0.8, Z - 0.8)
        yaw = rng.uniform(0, 2 * np.pi)
        u = np.array([np.cos(yaw), 0.0, np.sin(yaw)])
        v = np.array([-np.sin(yaw), 0.0, np.cos(yaw)])
        base = np.array([cx, 0.0, cz]) - 0.5 * w * u - 0.5 * d * v
        add(base, u, ey, w, h)
        add(base + d * v, u, ey, w, h)
        add(base, v, ey, d, h)
        add(base + w * u, v, ey, d, h)
        add(base + h * ey, u, v, w, d)       # top
    for _ in range(12):
        side = rng.uniform(0.5, 1.5)
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        t1, t2 = _tangent_frame(nrm[None, :], rng.uniform(0, 2 * np.pi, 1))
        c = np.array([rng.uniform(1, X - 1), rng.uniform(0.6, Y - 0.6), rng.uniform(1, Z - 1)])
        add(c - 0.5 * side * (t1[0] + t2[0]), t1[0], t2[0], side, side)
    for (px, pz) in panels:  # emissive panels hang 1 cm under the openings
        add([px, Y - 0.01, pz], ex, ez, P_, P_, emissive=True)
    area = sum(r[3] * r[4] for r in rects)
    cell = math.sqrt(area / n_surface)
    s_t = math.sqrt(EPS * K_COVER) * cell
    parts, emissive_mask = [], []
    for (o, eu, ev, w, h, nrm, em) in rects:
        pts = _grid_on_rect(rng, o, eu, ev, w, h, cell)
        nn = np.broadcast_to(nrm, pts.shape).copy()
        parts.append(_flat(rng, pts, nn, s_t, 0.01))
        emissive_mask.append(np.full(pts.shape[0], em))
    centres = np.stack([rng.uniform(0.5, X - 0.5, n_clusters), rng.uniform(0.5, Y - 0.5, n_clusters),
                        rng.uniform(0.5, Z - 0.5, n_clusters)], axis=1)
    for c in centres:
        m = c[None, :] + rng.normal(0, 0.15, (per_cluster, 3))
        short = _loguniform(rng, 0.0005, 0.002, per_cluster)
        sc = np.stack([20 * short, short, short], axis=1)
        parts.append((m, sc, _random_quat(rng, per_cluster), rng.uniform(8.0, 80.0, per_cluster)))
        emissive_mask.append(np.zeros(per_cluster, bool))
    sc = _finish(parts, rng, albedo_lo=0.1, albedo_hi=0.9, rough_lo=0.02, rough_hi=1.0,
                 glossy_frac=0.5)
    em = np.concatenate(emissive_mask)
    sc["emission"][em] = panel_radiance
    sc["bounds"] = (np.zeros(3, np.float32), ROOM.astype(np.float32))
    return sc


# ---------------------------------------------------------------------------
# cameras and render settings of the workloads
# ---------------------------------------------------------------------------
def camera(name: str) -> dict:
    if name in ("tiny_random", "mixed_100k", "needles"):
        w = 512 if name == "mixed_100k" else 128
        return {"origin": (0.5, 0.5, -1.0), "target": (0.5, 0.5, 0.5), "up": (0.0, 1.0, 0.0),
                "vfov_deg": 45.0, "width": w, "height": w}
    if name == "room_5p5m":
        return {"origin": (1.0, 1.6, 1.0), "target": (7.0, 1.0, 7.0), "up": (0.0, 1.0, 0.0),
                "vfov_deg": 60.0, "width": 1920, "height": 1080}
    raise KeyError(name)


def ring_cameras(centre, radius: float, n: int = 8, size: int = 256, height: float = 0.3,
                 vfov_deg: float = 40.0) -> list:
    """n pinhole cameras on a ring around `centre` (tilted `height` x radius
    up), all looking at it: the views of a transmittance fit."""
    c = np.asarray(centre, np.float64)
    cams = []
    for k in range(n):
        a = 2 * np.pi * k / n
        o = c + radius * np.array([np.cos(a), height, np.sin(a)])
        cams.append({"origin": tuple(float(x) for x in o), "target": tuple(float(x) for x in c),
                     "up": (0.0, 1.0, 0.0), "vfov_deg": vfov_deg, "width": size, "height": size})
    return cams


def perturbed(sc: dict, seed: int = 0, pos: float = 0.5, scale: float = 0.25, dens: float = 0.5,
              rot: float = 0.2) -> dict:
    """A start for a transmittance fit: the primitives of `sc` with means moved
    by N(0, (pos * smallest scale)^2) per axis, scales multiplied by
    exp(U[-scale, scale]), densities by U[1 - dens, 1 + dens] and rotations
    turned by a quaternion perturbation of size `rot`."""
    rng = _rng(seed)
    n = sc["mean"].shape[0]
    out = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    smin = np.min(sc["scale"], axis=1, keepdims=True)
    out["mean"] = (sc["mean"] + rng.normal(size=(n, 3)) * pos * smin).astype(np.float32)
    out["scale"] = (sc["scale"] * np.exp(rng.uniform(-scale, scale, (n, 3)))).astype(np.float32)
    out["density"] = (sc["density"] * rng.uniform(1 - dens, 1 + dens, n)).astype(np.float32)
    q = sc["rotation"] + rot * rng.normal(size=(n, 4))
    out["rotation"] = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    return out


def _quat_axes(q):
    """columns of the rotation matrices of unit quaternions (w, x, y, z) [n,4] -> [n,3,3]"""
    w, x, y, z = (q[:, i] for i in range(4))
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - w * z); R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y); R[:, 2, 1] = 2 * (y * z + w * x); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def with_sggx(sc: dict, seed: int = 0, frac: float = 0.5, base: str = "lambert") -> dict:
    """A copy of `sc` in which a random `frac` of the primitives are SGGX
    microflake primitives (material 2 with base "lambert"; material 3 with
    base "disney", whose primitives then get roughness U[0.05, 1] and every
    primitive a metallic U[0, 1]) and every primitive carries an SGGX
    matrix ("sggx" [n,6] = xx, yy, zz, xy, xz, yz).  The matrices are
    S = V diag(l1, l2, l3) V^T in the primitive's own frame (V = its rotation,
    axes sorted by scale), of three kinds drawn with equal probability, the
    three configurations of the paper's phase-function figure:
      surface-like: normals about the axis of the smallest scale,
                    eigenvalue 1 there and r^2 on the other two, r ~ U[0.05, 0.5];
      isotropic   : S = I (a sphere of flakes);
      fibre-like  : normals orthogonal to the axis of the largest scale,
                    eigenvalue r^2 there and 1 on the other two, r ~ U[0.05, 0.3].
    Primitives that keep materials 0 / 1 hold the isotropic matrix."""
    rng = _rng(seed)
    n = sc["mean"].shape[0]
    out = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    q = np.asarray(sc["rotation"], np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    R = _quat_axes(q)
    order = np.argsort(np.asarray(sc["scale"], np.float64), axis=1)  # ascending
    V = np.take_along_axis(R, order[:, None, :], axis=2)            # columns: smallest .. largest
    kind = rng.integers(0, 3, n)
    lam = np.ones((n, 3))
    r_s = rng.uniform(0.05, 0.5, n)
    r_f = rng.uniform(0.05, 0.3, n)
    lam[kind == 0, 1] = r_s[kind == 0] ** 2
    lam[kind == 0, 2] = r_s[kind == 0] ** 2
    lam[kind == 2, 2] = r_f[kind == 2] ** 2
    S = np.einsum("nij,nj,nkj->nik", V, lam, V)
    S[kind == 1] = np.eye(3)
    pick = rng.uniform(0, 1, n) < frac
    out["material"] = np.where(pick, 2, np.asarray(sc["material"])).astype(np.int32)
    out["sggx"] = np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]],
                           1).astype(np.float32)
    for k in range(n):
        if not pick[k]:
            out["sggx"][k] = (1, 1, 1, 0, 0, 0)
    if base == "disney":
        out["material"] = np.where(pick, 3, out["material"]).astype(np.int32)
        out["roughness"] = np.where(pick, rng.uniform(0.05, 1.0, n), sc["roughness"]).astype(np.float32)
        out["metallic"] = rng.uniform(0, 1, n).astype(np.float32)
    elif base != "lambert":
        raise ValueError(base)
    return out


def render_settings(name: str) -> dict:
    return {"tiny_random": {"spp": 4, "max_depth": 4, "seed": 0},
            "needles": {"spp": 4, "max_depth": 6, "seed": 4},
            "mixed_100k": {"spp": 16, "max_depth": 8, "seed": 1},
            "room_5p5m": {"spp": 64, "max_depth": 12, "seed": 2}}[name]


def scene(name: str, **kw) -> dict:
    return {"tiny_random": tiny_random, "mixed_100k": mixed_100k, "room_5p5m": room_5p5m}[name](**kw)


# ---------------------------------------------------------------------------
# rays for per-ray parity tests
# ---------------------------------------------------------------------------
def probe_rays(sc: dict, n: int, seed: int = 0, aimed_frac: float = 0.7,
               finite_frac: float = 0.3) -> np.ndarray:
    """Rays [n, 8] = (o, w, t0, t1): origins uniform in the scene bounds
    (slightly enlarged), aimed_frac of them pointed at a random primitive's
    mean, the rest in uniform random directions; t0 = 0 and t1 = +inf except
    finite_frac of them ending at a random distance (some inside primitives)."""
    rng = _rng(seed)
    lo, hi = (np.asarray(b, np.float64) for b in sc["bounds"])
    ext = hi - lo
    o = rng.uniform(lo - 0.1 * ext, hi + 0.1 * ext, (n, 3))
    w = rng.normal(size=(n, 3))
    m = rng.uniform(0, 1, n) < aimed_frac
    tgt = sc["mean"][rng.integers(0, sc["mean"].shape[0], n)].astype(np.float64)
    w[m] = tgt[m] - o[m]
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    t0 = np.zeros(n)
    t1 = np.full(n, np.inf)
    f = rng.uniform(0, 1, n) < finite_frac
    dist = np.linalg.norm(tgt - o, axis=1)
    t1[f] = dist[f] * rng.uniform(0.2, 1.5, f.sum())
    rays = np.concatenate([o, w, t0[:, None], t1[:, None]], axis=1).astype(np.float32)
    return rays
