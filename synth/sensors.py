"""Seeded sensor descriptions (intrinsics, pose at the sweep start, motion) for the workloads.

A sensor description is a plain dict whose keys mirror the C struct `salf_sensor`:
  model               PINHOLE | FISHEYE_EQUIDISTANT | LIDAR_SPINNING
  width, height       camera pixels; LiDAR: width = azimuth steps per sweep, height = beams
  fx, fy, cx, cy      pinhole focal lengths and principal point (pixels); fisheye uses fx as f
  max_theta           fisheye half field of view (radians)
  elev_min, elev_max  LiDAR lowest / highest beam elevation (radians)
  az0                 LiDAR azimuth offset (radians)
  t0, dt_line         time of row 0 / column 0 and the time step per camera row / LiDAR column
  R0 (9, row-major), p0 (3)   sensor-to-world rotation and position at t0
  v (3), w (3)        constant linear (m/s) and angular (rad/s, world frame) velocity
  t_near, t_far       ray extent
Camera frame: x right, y down, z forward.  LiDAR frame: x forward, y left, z up.  World: z up.
Nothing here casts a ray.
"""
from __future__ import annotations

import math

import numpy as np

PINHOLE = 0
FISHEYE_EQUIDISTANT = 1
LIDAR_SPINNING = 2


def _base(model, width, height, R0, p0, t0, dt_line, v, w, t_near, t_far):
    return dict(model=int(model), width=int(width), height=int(height), fx=0.0, fy=0.0, cx=0.0, cy=0.0,
                max_theta=0.0, elev_min=0.0, elev_max=0.0, az0=0.0, t0=float(t0), dt_line=float(dt_line),
                R0=[float(x) for x in np.asarray(R0, np.float64).reshape(9)],
                p0=[float(x) for x in np.asarray(p0, np.float64).reshape(3)],
                v=[float(x) for x in np.asarray(v, np.float64).reshape(3)],
                w=[float(x) for x in np.asarray(w, np.float64).reshape(3)],
                t_near=float(t_near), t_far=float(t_far))


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """Camera-to-world rotation (columns = camera x right, y down, z forward in world)."""
    eye, target, up = (np.asarray(a, np.float64) for a in (eye, target, up))
    f = target - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    dn = np.cross(f, r)
    return np.stack([r, dn, f], axis=1)


def yaw_pitch_camera(yaw_deg, pitch_deg):
    """Camera looking along world heading `yaw` (about +z from +x) tilted by `pitch` (up > 0)."""
    y, p = math.radians(yaw_deg), math.radians(pitch_deg)
    f = np.array([math.cos(p) * math.cos(y), math.cos(p) * math.sin(y), math.sin(p)])
    return look_at(np.zeros(3), f)


def yaw_lidar(yaw_deg):
    y = math.radians(yaw_deg)
    c, s = math.cos(y), math.sin(y)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def pinhole(width, height, hfov_deg, R0, p0, t0=0.0, dt_line=0.0, v=(0, 0, 0), w=(0, 0, 0),
            t_near=0.0, t_far=math.inf):
    s = _base(PINHOLE, width, height, R0, p0, t0, dt_line, v, w, t_near, t_far)
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    s.update(fx=f, fy=f, cx=width / 2.0, cy=height / 2.0)
    return s


def fisheye_equidistant(width, height, fov_deg, R0, p0, t0=0.0, dt_line=0.0, v=(0, 0, 0), w=(0, 0, 0),
                        t_near=0.0, t_far=math.inf):
    """Equidistant fisheye r = f * theta whose full field of view `fov_deg` spans the image width."""
    s = _base(FISHEYE_EQUIDISTANT, width, height, R0, p0, t0, dt_line, v, w, t_near, t_far)
    th = math.radians(fov_deg) / 2.0
    f = (width / 2.0) / th
    s.update(fx=f, fy=f, cx=width / 2.0, cy=height / 2.0, max_theta=th)
    return s


def lidar_spinning(beams, steps, elev_min_deg, elev_max_deg, R0, p0, sweep_time, t0=0.0, v=(0, 0, 0),
                   w=(0, 0, 0), az0_deg=0.0, t_near=0.0, t_far=math.inf):
    s = _base(LIDAR_SPINNING, steps, beams, R0, p0, t0, sweep_time / steps, v, w, t_near, t_far)
    s.update(elev_min=math.radians(elev_min_deg), elev_max=math.radians(elev_max_deg),
             az0=math.radians(az0_deg))
    return s


# --- the workloads' sensors --------------------------------------------------------------------
def config0_camera():
    """64x48 pinhole, 60 deg horizontal FOV, 15 m from the tiny scene's centre."""
    a, e = math.radians(30.0), math.radians(20.0)
    eye = 15.0 * np.array([math.cos(e) * math.sin(a), -math.cos(e) * math.cos(a), math.sin(e)])
    return pinhole(64, 48, 60.0, look_at(eye, np.zeros(3)), eye)


def config1_camera(width=1920, height=1080):
    """Driving camera at 1.6 m height looking down the road (+x), pitched 5 deg down."""
    return pinhole(width, height, 60.0, yaw_pitch_camera(0.0, -5.0), (-95.0, 0.0, 1.6))


def config2_lidar(beams=64, steps=2048):
    """Spinning LiDAR: 64 beams in [-25, +15] deg, 2,048 columns over a 0.1 s sweep, moving at
    10 m/s along +x (rolling timestamps per column)."""
    return lidar_spinning(beams, steps, -25.0, 15.0, np.eye(3), (-60.0, 0.37, 1.85), 0.1, t0=0.0,
                          v=(10.0, 0.0, 0.0))


def random_rays(seed, n, lo, hi, inside_frac=0.25):
    """Seeded explicit rays: origins uniform in a box around the scene (a fraction inside it),
    directions uniform on the sphere.  float32 [n, 3] origins and unit directions."""
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    c, h = (lo + hi) / 2, (hi - lo) / 2
    o = c + rng.uniform(-1.6, 1.6, size=(n, 3)) * h
    k = int(n * inside_frac)
    o[:k] = c + rng.uniform(-1.0, 1.0, size=(k, 3)) * h
    d = rng.standard_normal((n, 3))
    # aim most outside rays roughly at the scene so they hit something
    tgt = c + rng.uniform(-0.8, 0.8, size=(n, 3)) * h
    aim = rng.random(n) < 0.7
    d[aim] = tgt[aim] - o[aim]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
