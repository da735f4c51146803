"""Seeded synthetic inputs: geometries of the benchmark workloads, random
ellipsoid phantoms and random projection data.

This module holds no arithmetic of the projector itself; it only describes
and draws inputs.  The tests pass its arrays to both the HIP path and the CPU
oracle.  Every generator takes an explicit seed (NumPy PCG64).
"""
import math

import numpy as np


def angles(n_views: int, arc_deg: float = 360.0) -> np.ndarray:
    """Equally spaced rotation angles lambda_v = v * arc / V (radians)."""
    return np.arange(n_views, dtype=np.float64) * (math.radians(arc_deg) / n_views)


def geometry(vol_dims, voxel_mm, det_cols, det_rows, pitch_mm, sid_mm, sdd_mm,
             n_views, arc_deg=360.0, vol_offset_mm=(0.0, 0.0, 0.0), principal_px=None):
    """Plain parameter dict of a circular cone-beam geometry (flat detector)."""
    if np.isscalar(voxel_mm):
        voxel_mm = (voxel_mm,) * 3
    if np.isscalar(pitch_mm):
        pitch_mm = (pitch_mm, pitch_mm)
    if np.isscalar(vol_dims):
        vol_dims = (vol_dims,) * 3
    return dict(vol_dims=tuple(int(v) for v in vol_dims),
                voxel_mm=tuple(float(v) for v in voxel_mm),
                vol_offset_mm=tuple(float(v) for v in vol_offset_mm),
                det_cols=int(det_cols), det_rows=int(det_rows),
                pitch_mm=tuple(float(v) for v in pitch_mm),
                principal_px=principal_px,
                sid_mm=float(sid_mm), sdd_mm=float(sdd_mm),
                angles_rad=angles(n_views, arc_deg))


# The five workloads (volume, detector, trajectory).
def config_small():
    """64^3 voxels of 1.0 mm, 96x96 pixels of 1.6 mm, SID 750 / SDD 1200,
    32 views over 360 degrees."""
    return geometry(64, 1.0, 96, 96, 1.6, 750.0, 1200.0, 32, 360.0)


def config_cone():
    """256^3 voxels of 0.5 mm, 512x384 pixels of 0.388 mm, SID 600 / SDD 900,
    360 views over 360 degrees (cone angle about 12 degrees)."""
    return geometry(256, 0.5, 512, 384, 0.388, 600.0, 900.0, 360, 360.0)


def config_carm():
    """512^3 voxels of 0.25 mm, 616x480 pixels of 0.616 mm, SID 749 / SDD 1198,
    248 views over 200 degrees (C-arm short scan)."""
    return geometry(512, 0.25, 616, 480, 0.616, 749.0, 1198.0, 248, 200.0)


def config_warmstart():
    """128^3 voxels of 1.0 mm, 256x256 pixels of 1.0 mm, SID 750 / SDD 1200,
    180 views over 360 degrees."""
    return geometry(128, 1.0, 256, 256, 1.0, 750.0, 1200.0, 180, 360.0)


def config_batch(seed: int = 41, n_problems: int = 16):
    """16 uneven problems: edge in {96,128,192,256,320} voxels of 0.5-1.0 mm,
    detectors 256x192 .. 512x384, 60-400 views over 360 or 200 degrees,
    SID 750 / SDD 1200; the pitch makes the volume fit the detector."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dets = [(256, 192), (320, 240), (384, 288), (448, 336), (512, 384)]
    out = []
    for _ in range(n_problems):
        edge = int(rng.choice([96, 128, 192, 256, 320]))
        vox = float(rng.uniform(0.5, 1.0))
        cols, rows = dets[int(rng.integers(0, len(dets)))]
        views = int(rng.integers(60, 401))
        arc = float(rng.choice([360.0, 200.0]))
        pitch = 1.05 * 1.6 * edge * vox * math.sqrt(2.0) / cols
        out.append(geometry(edge, vox, cols, rows, pitch, 750.0, 1200.0, views, arc))
    return out


def draw_ellipsoids(vol_dims, voxel_mm, n_ellipsoids, seed, semi_axes_mm=(3.0, 25.0),
                    mu_range=(0.001, 0.02)):
    """Random ellipsoids as an (n, 16) float64 array: centre (3), semi-axes (3),
    rotation matrix R row-major (9, body frame -> world), attenuation (1).

    Centres are uniform in a ball of radius 0.45 * (smallest volume edge),
    semi-axes uniform in semi_axes_mm, orientation uniform (random rotation
    from a normalised Gaussian quaternion), attenuation uniform in mu_range."""
    n1, n2, n3 = (vol_dims,) * 3 if np.isscalar(vol_dims) else vol_dims
    a = (voxel_mm,) * 3 if np.isscalar(voxel_mm) else voxel_mm
    rng = np.random.Generator(np.random.PCG64(seed))
    radius = 0.45 * min(n1 * a[0], n2 * a[1], n3 * a[2])
    out = np.zeros((n_ellipsoids, 16))
    for e in range(n_ellipsoids):
        while True:
            c = rng.uniform(-radius, radius, size=3)
            if np.dot(c, c) <= radius * radius:
                break
        sa = rng.uniform(semi_axes_mm[0], semi_axes_mm[1], size=3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                      [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                      [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
        mu = rng.uniform(mu_range[0], mu_range[1])
        out[e, 0:3], out[e, 3:6], out[e, 6:15], out[e, 15] = c, sa, R.ravel(), mu
    return out, rng


def ellipsoid_phantom(vol_dims, voxel_mm, n_ellipsoids, seed, semi_axes_mm=(3.0, 25.0),
                      mu_range=(0.001, 0.02), noise_frac=0.0, dtype=np.float32):
    """Sum of random ellipsoids (draw_ellipsoids), sampled at voxel centres: a
    voxel gets the sum of mu over the ellipsoids containing its centre.
    noise_frac > 0 adds U[0, noise_frac * max mu) per voxel.
    Returned layout: [n3][n2][n1] (x1 fastest)."""
    n1, n2, n3 = (vol_dims,) * 3 if np.isscalar(vol_dims) else vol_dims
    a = (voxel_mm,) * 3 if np.isscalar(voxel_mm) else voxel_mm
    ells, rng = draw_ellipsoids(vol_dims, voxel_mm, n_ellipsoids, seed, semi_axes_mm, mu_range)
    ax = [(np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * av for n, av in zip((n1, n2, n3), a)]
    vol = np.zeros((n3, n2, n1), dtype=np.float64)
    for e in ells:
        c, sa, R, mu = e[0:3], e[3:6], e[6:15].reshape(3, 3), e[15]
        rmax = sa.max()
        lo = [np.searchsorted(ax[d], c[d] - rmax) for d in range(3)]
        hi = [np.searchsorted(ax[d], c[d] + rmax, side="right") for d in range(3)]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        X = ax[0][lo[0]:hi[0]][None, None, :] - c[0]
        Y = ax[1][lo[1]:hi[1]][None, :, None] - c[1]
        Z = ax[2][lo[2]:hi[2]][:, None, None] - c[2]
        # coordinates in the ellipsoid frame: p' = R^T p
        px = R[0, 0] * X + R[1, 0] * Y + R[2, 0] * Z
        py = R[0, 1] * X + R[1, 1] * Y + R[2, 1] * Z
        pz = R[0, 2] * X + R[1, 2] * Y + R[2, 2] * Z
        inside = (px / sa[0]) ** 2 + (py / sa[1]) ** 2 + (pz / sa[2]) ** 2 <= 1.0
        vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += mu * inside
    if noise_frac > 0:
        vol += rng.uniform(0.0, noise_frac * vol.max(), size=vol.shape)
    return vol.astype(dtype)


def uniform_projections(shape, seed, dtype=np.float32):
    """Projection data drawn from U[0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(size=shape, dtype=np.float64).astype(dtype)


def uniform_volume(shape, seed, dtype=np.float32):
    """Volume data drawn from U[0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(size=shape, dtype=np.float64).astype(dtype)


def gaussian_noise(shape, sigma, seed, dtype=np.float32):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (sigma * rng.standard_normal(size=shape)).astype(dtype)


# ---------------------------------------------------------------- Philox noise
# Host definition of the counter-based Gaussian noise that the GPU generator
# adds (same counters and key), used to check it.  Philox4x32-10 as published
# by Salmon, Moraes, Dror and Shaw (SC 2011): ten rounds of two 32x32->64-bit
# multiplications with the key bumped by the Weyl constants between rounds.
_PH_M = (0xD2511F53, 0xCD9E8D57)
_PH_W = (0x9E3779B9, 0xBB67AE85)


def philox4x32_10(counters, key):
    """counters: (n, 4) integer array (uint32 values); key: (k0, k1).
    Returns the (n, 4) uint32 outputs."""
    c = [np.asarray(counters, dtype=np.uint64)[:, e].copy() for e in range(4)]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(_PH_M[0]) * c[0]
        p1 = np.uint64(_PH_M[1]) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k0), p1 & mask,
             (p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k1), p0 & mask]
        k0 = (k0 + _PH_W[0]) & 0xFFFFFFFF
        k1 = (k1 + _PH_W[1]) & 0xFFFFFFFF
    return np.stack(c, axis=1).astype(np.uint32)


def philox_gaussian(n: int, seed: int) -> np.ndarray:
    """Standard normal draws z[i], i < n: counter (i // 4, hi, 0, 0), key =
    (seed low, seed high); Box-Muller on output pairs (0,1) and (2,3) with
    u = (float32(x) + 0.5) * 2^-32 formed in float32, as the GPU forms them;
    the transcendental functions in float64."""
    nq = (n + 3) // 4
    q = np.arange(nq, dtype=np.uint64)
    ctr = np.zeros((nq, 4), dtype=np.uint64)
    ctr[:, 0] = q & np.uint64(0xFFFFFFFF)
    ctr[:, 1] = q >> np.uint64(32)
    out = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    scale = np.float32(2.3283064365386963e-10)
    u = (out.astype(np.float32) + np.float32(0.5)) * scale          # float32 arithmetic
    z = np.empty((nq, 4))
    for h in range(2):
        u1 = u[:, 2 * h].astype(np.float64)
        ang = (np.float32(6.283185307179586) * u[:, 2 * h + 1]).astype(np.float64)
        r = np.sqrt(-2.0 * np.log(u1))
        z[:, 2 * h] = r * np.cos(ang)
        z[:, 2 * h + 1] = r * np.sin(ang)
    return z.reshape(-1)[:n]


def matrix_geometry(vol_dims, voxel_mm, det_cols, det_rows, pitch_mm, sid_mm, sdd_mm, n_views, arc_deg=360.0,
                    seed=0, wobble=True, vol_offset_mm=(0.0, 0.0, 0.0)):
    """A general trajectory given as one camera matrix per view (world mm ->
    homogeneous pixel-index coordinates, x~ = P [x; 1]): a circular C-arm
    orbit with, per view and seeded, the source raised or lowered (+-2 mm),
    the source and detector distances jittered (+-1 %), the principal point
    shifted (+-3 px), the detector yawed about the vertical (+-1 degree,
    so chi1 still does not depend on x3) and the pixels slightly
    anisotropic; chi2 runs opposite to x3 (the paper's convention).
    P = K [R | -R s] with K = [[f/b1, 0, c1], [0, f/b2, c2], [0, 0, 1]]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if np.isscalar(voxel_mm):
        voxel_mm = (voxel_mm,) * 3
    if np.isscalar(pitch_mm):
        pitch_mm = (pitch_mm, pitch_mm)
    if np.isscalar(vol_dims):
        vol_dims = (vol_dims,) * 3
    lam = angles(n_views, arc_deg)
    P = np.zeros((n_views, 3, 4))
    for v in range(n_views):
        w = wobble
        D = sid_mm * (1.0 + (rng.uniform(-0.01, 0.01) if w else 0.0))
        f = sdd_mm * (1.0 + (rng.uniform(-0.01, 0.01) if w else 0.0))
        dz = rng.uniform(-2.0, 2.0) if w else 0.0
        yaw = math.radians(rng.uniform(-1.0, 1.0)) if w else 0.0
        c1 = (det_cols - 1) / 2.0 + (rng.uniform(-3.0, 3.0) if w else 0.0)
        c2 = (det_rows - 1) / 2.0 + (rng.uniform(-3.0, 3.0) if w else 0.0)
        b1 = pitch_mm[0] * (1.0 + (rng.uniform(-0.02, 0.02) if w else 0.0))
        b2 = pitch_mm[1]
        cl, sl = math.cos(lam[v]), math.sin(lam[v])
        s = np.array([D * cl, D * sl, dz])
        cy, sy = math.cos(yaw), math.sin(yaw)
        d = np.array([-cl * cy + sl * sy, -sl * cy - cl * sy, 0.0])
        e1 = np.array([-d[1], d[0], 0.0])
        R = np.array([e1, [0.0, 0.0, -1.0], d])
        K = np.array([[f / b1, 0.0, c1], [0.0, f / b2, c2], [0.0, 0.0, 1.0]])
        P[v, :, :3] = K @ R
        P[v, :, 3] = -(K @ R) @ s
    return dict(vol_dims=tuple(int(x) for x in vol_dims), voxel_mm=tuple(float(x) for x in voxel_mm),
                vol_offset_mm=tuple(float(x) for x in vol_offset_mm), det_cols=int(det_cols),
                det_rows=int(det_rows), matrices=P)


def circular_matrices(p):
    """The camera matrices of a circular geometry dict (see geometry):
    source (D cos l, D sin l, 0), e1 = (-sin l, cos l, 0), e2 = (0, 0, -1),
    d = (-cos l, -sin l, 0), K from f/b and the principal point."""
    M, N = p["det_cols"], p["det_rows"]
    pp = p.get("principal_px")
    c1, c2 = ((M - 1) / 2.0, (N - 1) / 2.0) if pp is None else pp
    b1, b2 = p["pitch_mm"]
    D, f = p["sid_mm"], p["sdd_mm"]
    K = np.array([[f / b1, 0.0, c1], [0.0, f / b2, c2], [0.0, 0.0, 1.0]])
    out = np.zeros((len(p["angles_rad"]), 3, 4))
    for v, l in enumerate(p["angles_rad"]):
        cl, sl = math.cos(l), math.sin(l)
        R = np.array([[-sl, cl, 0.0], [0.0, 0.0, -1.0], [-cl, -sl, 0.0]])
        s = np.array([D * cl, D * sl, 0.0])
        out[v, :, :3] = K @ R
        out[v, :, 3] = -(K @ R) @ s
    return out
