"""Sensor rays in float64: pinhole and equidistant-fisheye cameras and a spinning LiDAR,
all with an optional rolling shutter (the paper casts rays from sensor intrinsics and
extrinsics, Sec. 1, and simulates camera and LiDAR rolling shutter, Sec. 5.3).

Pose at time t under constant motion from the sweep start t0:
    p(t) = p0 + v (t - t0),   R(t) = Exp([w]x (t - t0)) R0   (w in the world frame).
Camera row r is exposed at t0 + r dt_line (row 0 first); LiDAR column j fires at
t0 + j dt_line with all its beams together.  dt_line = 0 is a global shutter.

pinhole   pixel (u, r): d_cam = ((u + 1/2 - cx) / fx, (r + 1/2 - cy) / fy, 1), normalized.
fisheye   equidistant r = f theta: x = (u + 1/2 - cx) / f, y = (r + 1/2 - cy) / f,
          theta = |(x, y)|, phi = atan2(y, x); d_cam = (sin theta cos phi, sin theta sin phi,
          cos theta); the ray is valid iff theta <= max_theta.
LiDAR     beam b, column j: elevation e_b = e_min + (e_max - e_min) b / (B - 1), azimuth
          a_j = az0 + 2 pi (j + 1/2) / J (counter-clockwise about +z from the sensor's +x);
          d_s = (cos e cos a, cos e sin a, sin e).
Camera frame x right, y down, z forward; rays are ordered row-major (index = r W + u).
LiDAR rays are ordered [beam, column] (index = b J + j).
"""
from __future__ import annotations

import math

import numpy as np

PINHOLE, FISHEYE_EQUIDISTANT, LIDAR_SPINNING = 0, 1, 2


def rodrigues(w, dt):
    """Exp([w]x dt): rotation by angle |w| dt about w / |w| (float64 3x3)."""
    w = np.asarray(w, np.float64)
    th = float(np.linalg.norm(w)) * dt
    if th == 0.0:
        return np.eye(3)
    k = w / np.linalg.norm(w)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(th) * K + (1.0 - math.cos(th)) * (K @ K)


def _pose(s, t):
    R0 = np.asarray(s["R0"], np.float64).reshape(3, 3)
    dt = t - s["t0"]
    return rodrigues(s["w"], dt) @ R0, np.asarray(s["p0"], np.float64) + np.asarray(s["v"], np.float64) * dt


def sensor_rays(s):
    """(o [n, 3], d [n, 3], t [n], valid [n]) of a sensor description, float64."""
    W, H = s["width"], s["height"]
    n = W * H
    o = np.zeros((n, 3))
    d = np.zeros((n, 3))
    t = np.zeros(n)
    valid = np.ones(n, bool)
    if s["model"] in (PINHOLE, FISHEYE_EQUIDISTANT):
        u = np.arange(W) + 0.5
        for r in range(H):
            tr = s["t0"] + r * s["dt_line"]
            R, p = _pose(s, tr)
            if s["model"] == PINHOLE:
                dc = np.stack([(u - s["cx"]) / s["fx"], np.full(W, (r + 0.5 - s["cy"]) / s["fy"]), np.ones(W)], 1)
                dc /= np.linalg.norm(dc, axis=1, keepdims=True)
                ok = np.ones(W, bool)
            else:
                x = (u - s["cx"]) / s["fx"]
                y = np.full(W, (r + 0.5 - s["cy"]) / s["fx"])
                th = np.hypot(x, y)
                ph = np.arctan2(y, x)
                dc = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
                ok = th <= s["max_theta"]
            sl = slice(r * W, (r + 1) * W)
            o[sl] = p
            d[sl] = dc @ R.T
            t[sl] = tr
            valid[sl] = ok
        d[~valid] = 0.0
    elif s["model"] == LIDAR_SPINNING:
        B, J = H, W
        e = np.array([s["elev_min"] + (s["elev_max"] - s["elev_min"]) * (b / (B - 1) if B > 1 else 0.0)
                      for b in range(B)])
        for j in range(J):
            tj = s["t0"] + j * s["dt_line"]
            R, p = _pose(s, tj)
            a = s["az0"] + 2.0 * math.pi * (j + 0.5) / J
            ds = np.stack([np.cos(e) * math.cos(a), np.cos(e) * math.sin(a), np.sin(e)], 1)
            idx = np.arange(B) * J + j
            o[idx] = p
            d[idx] = ds @ R.T
            t[idx] = tj
    else:
        raise ValueError(f"unknown sensor model {s['model']}")
    return o, d, t, valid
