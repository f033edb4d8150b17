"""Local field of one voxel at normalized local coordinates x in [-1, 1]^3 (float64).

Two parameterizations share the per-voxel buffers z_geo [N, 8], z_rgb [N, 3, 8], z_int [N, 8]:

corner mode   Each voxel stores raw logits at its 8 corners (corner c = bx + 2 by + 4 bz,
              b = 0 on an axis's low face).  Corner values are activated first
              (density: softplus, colour and intensity: sigmoid) and then trilinearly
              interpolated at x.  This is the workload's field; the paper leaves the choice
              of local field open beyond Eq. 1-2.

paper mode    Eq. 1: sigma = exp(W_sigma [x, 1]) with W_sigma = z_geo[v, 0:4].
              Eq. 2: c = sigmoid(W_c x + W_sh gamma(omega)) with, per colour channel ch,
              W_c row = z_rgb[v, ch, 0:3] and W_sh row = z_rgb[v, ch, 3:7];
              gamma(omega) = (C0, C1 wx, C1 wy, C1 wz) is the real spherical-harmonic basis of
              degree <= 1 (4 coefficients) at the view direction omega.
              Intensity (a LiDAR channel the paper does not define): sigmoid(z_int[v, 0:4] [x, 1]).

sdf mode      Surface parameterization (Eq. 5-6): the density of paper mode is replaced by a
              signed distance s = W_s [x, 1] with W_s = z_geo[v, 0:4], turned into density by
              sigma = a/2 + a/2 sign(s) (1 - exp(-|s| / b)); the voxel's a, b are stored as
              logarithms, a = exp(z_geo[v, 4]), b = exp(z_geo[v, 5]), so that they stay positive
              under any update (the paper does not say how they are kept positive).  Colour and
              intensity as in paper mode.
"""
from __future__ import annotations

import math

import numpy as np

SH_C0 = 0.5 / math.sqrt(math.pi)
SH_C1 = math.sqrt(3.0) / (2.0 * math.sqrt(math.pi))


def softplus(z):
    z = np.asarray(z, np.float64)
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    z = np.asarray(z, np.float64)
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def corner_weights(x):
    """Trilinear weights of the 8 corners at local coordinates x (float64 [3])."""
    x = np.asarray(x, np.float64)
    w = np.empty(8)
    for c in range(8):
        p = 1.0
        for a in range(3):
            b = (c >> a) & 1
            p *= (1.0 + (2 * b - 1) * x[a]) / 2.0
        w[c] = p
    return w


def corner_field(z_geo_v, z_rgb_v, z_int_v, x):
    """(sigma, rgb [3], intensity) of one voxel in corner mode."""
    w = corner_weights(x)
    sigma = float(w @ softplus(z_geo_v))
    rgb = sigmoid(z_rgb_v) @ w
    inten = float(w @ sigmoid(z_int_v)) if z_int_v is not None else 0.0
    return sigma, rgb, inten


def sh_basis(omega):
    omega = np.asarray(omega, np.float64)
    return np.array([SH_C0, SH_C1 * omega[0], SH_C1 * omega[1], SH_C1 * omega[2]])


def sdf_density(z_geo_v, x):
    """(sigma, s, a, b) of Eq. 5-6 at local coordinates x."""
    xh = np.append(np.asarray(x, np.float64), 1.0)
    z = np.asarray(z_geo_v, np.float64)
    s = float(z[:4] @ xh)
    a, b = math.exp(z[4]), math.exp(z[5])
    sigma = a / 2.0 + a / 2.0 * np.sign(s) * (1.0 - math.exp(-abs(s) / b))
    return float(sigma), s, a, b


def sdf_field(z_geo_v, z_rgb_v, z_int_v, x, omega):
    """(sigma, rgb [3], intensity) of one voxel in sdf mode (Eq. 5-6 density, Eq. 2 colour)."""
    sigma = sdf_density(z_geo_v, x)[0]
    _, rgb, inten = paper_field(z_geo_v, z_rgb_v, z_int_v, x, omega)
    return sigma, rgb, inten


def paper_field(z_geo_v, z_rgb_v, z_int_v, x, omega):
    """(sigma, rgb [3], intensity) of one voxel in the paper's parameterization (Eq. 1-2)."""
    xh = np.append(np.asarray(x, np.float64), 1.0)
    sigma = float(np.exp(np.asarray(z_geo_v[:4], np.float64) @ xh))
    zr = np.asarray(z_rgb_v, np.float64)
    rgb = sigmoid(zr[:, 0:3] @ xh[:3] + zr[:, 3:7] @ sh_basis(omega))
    inten = float(sigmoid(np.asarray(z_int_v[:4], np.float64) @ xh)) if z_int_v is not None else 0.0
    return sigma, rgb, inten
