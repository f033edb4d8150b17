"""Analytic gradient of the composited outputs w.r.t. the raw field parameters (float64).

Let the samples of a ray be j = 1..M in compositing order (the stop index M is held
fixed), with tau_j = sigma_j delta_j, T_1 = 1, T_{j+1} = T_j exp(-tau_j), w_j = T_j - T_{j+1}
and T_end = T_{M+1}.  The outputs are (Eq. 3 with Eq. 4 per sample)
    C = sum_j w_j c_j + T_end bg,   D = sum_j w_j t_j,   I = sum_j w_j i_j,   O = 1 - T_end.
Differentiating:
    dC/dc_j = w_j,  dI/di_j = w_j
    dC/dtau_j = T_{j+1} c_j - (sum_{k>j} w_k c_k + T_end bg)
    dD/dtau_j = T_{j+1} t_j - sum_{k>j} w_k t_k,   dI/dtau_j likewise,   dO/dtau_j = T_end
    dtau_j/dsigma_j = delta_j
and through the corner activations (softplus' = sigmoid, sigmoid' = s (1 - s)):
    dsigma_j/dz_geo[c] = W_c(x_j) sigmoid(z_geo[c]),   dc_j/dz_rgb[ch, c] = W_c(x_j) s (1 - s).
In the paper's field (Eq. 1-2), sigma = exp(a . x + b) and c = sigmoid(A x + B SH(omega)), so with
xh = (x, 1):
    dsigma_j/dz_geo[0:4] = sigma_j xh_j,
    dc_j[ch]/dz_rgb[ch, 0:3] = s (1 - s) x_j,   dc_j[ch]/dz_rgb[ch, 3:7] = s (1 - s) SH(omega),
    di_j/dz_int[0:4] = i_j (1 - i_j) xh_j,
and the remaining slots of each record are unused (zero gradient).  In the SDF variant (Eq. 5-6)
the density is sigma = a/2 + a/2 sign(s) (1 - exp(-|s|/b)) with s = z_geo[0:4] . xh,
a = exp(z_geo[4]), b = exp(z_geo[5]); with e = exp(-|s|/b):
    dsigma/dz_geo[0:4] = (a / (2 b)) e xh,   dsigma/dz_geo[4] = sigma,
    dsigma/dz_geo[5] = -(a / 2) (s / b) e,
and colour and intensity as in the paper's field.
The suffix sums are formed directly from their definition.
"""
from __future__ import annotations

import numpy as np

from .field import corner_weights, paper_field, sdf_density, sh_basis, sigmoid, softplus
from .hitspec import PreparedScene, hit_list
from .render import RenderOpts, _sample_points


def _ray_samples(ps: PreparedScene, o, d, opts: RenderOpts):
    sc = ps.scene
    ids, t_ins, t_outs = hit_list(ps, o, d, opts.t_near, opts.t_far)
    o64 = np.asarray(o, np.float32).astype(np.float64)
    d64 = np.asarray(d, np.float32).astype(np.float64)
    T = 1.0
    rec = []
    for v, ti, to in zip(ids, t_ins, t_outs):
        for tk, x, dk in _sample_points(ps, o64, d64, v, float(ti), float(to), opts.samples):
            if opts.field in ("paper", "sdf"):
                W = None
                sigma, rgb, inten = paper_field(sc.z_geo[v], sc.z_rgb[v], sc.z_int[v] if sc.z_int is not None
                                                else None, x, d64)
                if opts.field == "sdf":
                    sigma, s_sd, a_sd, b_sd = sdf_density(sc.z_geo[v], x)
            else:
                W = corner_weights(x)
                sigma = float(W @ softplus(sc.z_geo[v]))
                rgb = sigmoid(sc.z_rgb[v]) @ W
                inten = float(W @ sigmoid(sc.z_int[v])) if sc.z_int is not None else 0.0
            tau = sigma * dk
            Tn = T * np.exp(-tau)
            r = dict(v=v, W=W, x=x, sigma=sigma, rgb=rgb, inten=inten, tk=tk, dk=dk, T=T, Tn=Tn,
                     w=T - Tn, omega=d64)
            if opts.field == "sdf":
                r.update(s=s_sd, a=a_sd, b=b_sd)
            rec.append(r)
            T = Tn
        if T < opts.t_min:
            break
    return rec, T


def grad_rays(ps: PreparedScene, o, d, opts: RenderOpts, g_rgb, g_depth, g_opacity, g_int):
    """Gradient of L = sum_r (g_rgb[r] . C_r + g_depth[r] D_r + g_opacity[r] O_r + g_int[r] I_r)
    w.r.t. z_geo [N, 8], z_rgb [N, 3, 8] and z_int [N, 8] (float64)."""
    if opts.field not in ("corner", "paper", "sdf"):
        raise ValueError(f"unknown field {opts.field!r}")
    sc = ps.scene
    dg = np.zeros(sc.z_geo.shape)
    dr = np.zeros(sc.z_rgb.shape)
    di = np.zeros(sc.z_geo.shape)
    bg = np.asarray(opts.background, np.float64)
    for r in range(o.shape[0]):
        rec, T_end = _ray_samples(ps, o[r], d[r], opts)
        gC = np.asarray(g_rgb[r], np.float64)
        gD, gO, gI = float(g_depth[r]), float(g_opacity[r]), float(g_int[r])
        m = len(rec)
        sufC, sufD, sufI = T_end * bg, 0.0, 0.0     # sums over samples k > j (plus background)
        for j in range(m - 1, -1, -1):
            s = rec[j]
            v = s["v"]
            dtau = (gC @ (s["Tn"] * s["rgb"] - sufC) + gD * (s["Tn"] * s["tk"] - sufD)
                    + gI * (s["Tn"] * s["inten"] - sufI) + gO * T_end)
            dsig = dtau * s["dk"]
            if opts.field in ("paper", "sdf"):
                xh = np.append(s["x"], 1.0)
                if opts.field == "sdf":
                    e = np.exp(-abs(s["s"]) / s["b"])
                    dg[v, :4] += dsig * (s["a"] / (2.0 * s["b"])) * e * xh
                    dg[v, 4] += dsig * s["sigma"]
                    dg[v, 5] += dsig * (-(s["a"] / 2.0) * (s["s"] / s["b"]) * e)
                else:
                    dg[v, :4] += dsig * s["sigma"] * xh
                basis = np.concatenate([s["x"], sh_basis(s["omega"])])
                c = s["rgb"]
                dr[v, :, :7] += (gC * s["w"] * c * (1.0 - c))[:, None] * basis[None, :]
                if sc.z_int is not None:
                    di[v, :4] += gI * s["w"] * s["inten"] * (1.0 - s["inten"]) * xh
            else:
                dg[v] += dsig * s["W"] * sigmoid(sc.z_geo[v])
                sr = sigmoid(sc.z_rgb[v])
                dr[v] += (gC[:, None] * s["w"]) * s["W"][None, :] * sr * (1.0 - sr)
                if sc.z_int is not None:
                    si = sigmoid(sc.z_int[v])
                    di[v] += gI * s["w"] * s["W"] * si * (1.0 - si)
            sufC = sufC + s["w"] * s["rgb"]
            sufD = sufD + s["w"] * s["tk"]
            sufI = sufI + s["w"] * s["inten"]
    return dg, dr, di
