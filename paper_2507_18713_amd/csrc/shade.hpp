// Shading and compositing of one ray-voxel segment (Eq. 1-6 at S midpoint samples, Eq. 3-4 with FP32
// transmittance), shared by the ray-casting kernels and the splatting kernel so that a hit composites
// to the same bits in both.
#pragma once

#include "device.hpp"

namespace salf {

// Composited state of one ray.
struct Accum {
  float T, C[3], D, I;
  int32_t n;
};

// Density of the SDF variant (Eq. 6) at signed distance q: a/2 + a/2 sign(q) (1 - exp(-|q| / b)),
// with ha = a / 2 and ib = 1 / b.
__device__ __forceinline__ float sdf_sigma(float q, float ha, float ib) {
  const float m = ha * (1.0f - __expf(-fabsf(q) * ib));
  return q > 0.0f ? ha + m : (q < 0.0f ? ha - m : ha);
}

// Shade one voxel segment [t_in, t_out] and composite it into acc, from the voxel's parameter rows
// geo [8], rgb [3][8], intensity [8] (rows in device memory, or copies staged in LDS by the
// splatting kernel: the arithmetic is the same).  Returns false once the ray has become opaque
// enough to stop (T < t_min after the voxel).
template <int FIELD, bool RGB, bool INT>
__device__ __forceinline__ bool shade_rows(const SceneView& s, const RayFrame& f, const float sh[4], const Hit& h,
                                           int S, double rS, float t_min, Accum& acc, const float* geo_row,
                                           const float* rgb_row, const float* int_row,
                                           const double* seg = nullptr, int seg_stride = 0) {
  const float ti = h.t_in;
  float g[8], c[3][8], it[8];
  {
    const float4* gp = reinterpret_cast<const float4*>(geo_row);
    const float4 g0 = gp[0], g1 = gp[1];
    g[0] = g0.x; g[1] = g0.y; g[2] = g0.z; g[3] = g0.w; g[4] = g1.x; g[5] = g1.y; g[6] = g1.z; g[7] = g1.w;
  }
  // the paper field (and its SDF variant) evaluates affine forms of x; the corner fields
  // interpolate corner values
  constexpr bool kAffine = FIELD == SALF_FIELD_PAPER || FIELD == kFieldSdf;
  // the colour and intensity rows are read with the density row, so that their loads are in
  // flight during the samples (reading them after the samples, which the corner fields could,
  // holds fewer registers but waits on the loads: slower)
  if (RGB) {
    const float4* cp = reinterpret_cast<const float4*>(rgb_row);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float4 a = cp[2 * ch], b = cp[2 * ch + 1];
      c[ch][0] = a.x; c[ch][1] = a.y; c[ch][2] = a.z; c[ch][3] = a.w;
      c[ch][4] = b.x; c[ch][5] = b.y; c[ch][6] = b.z; c[ch][7] = b.w;
    }
  }
  if (INT) {
    const float4* ip = reinterpret_cast<const float4*>(int_row);
    const float4 a = ip[0], b = ip[1];
    it[0] = a.x; it[1] = a.y; it[2] = a.z; it[3] = a.w; it[4] = b.x; it[5] = b.y; it[6] = b.z; it[7] = b.w;
  }
  float shc[3] = {0.0f, 0.0f, 0.0f};  // view-dependent colour term (paper field)
  float sdf_ha = 0.0f, sdf_ib = 0.0f;  // SDF variant: a / 2 and 1 / b
  if (FIELD == kFieldSdf) {
    sdf_ha = 0.5f * __expf(g[4]);
    sdf_ib = __expf(-g[5]);
  }
  if (FIELD == SALF_FIELD_CORNER) {
#pragma unroll
    for (int i = 0; i < 8; ++i) g[i] = softplus_f(g[i]);
    if (RGB) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int i = 0; i < 8; ++i) c[ch][i] = sigmoid_f(c[ch][i]);
    }
    if (INT) {
#pragma unroll
      for (int i = 0; i < 8; ++i) it[i] = sigmoid_f(it[i]);
    }
  } else if (kAffine && RGB) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
      shc[ch] = fmaf(c[ch][3], sh[0], fmaf(c[ch][4], sh[1], fmaf(c[ch][5], sh[2], c[ch][6] * sh[3])));
  }

  float rel[3], stp[3], delta, sc;
  if (seg) segment_frame_of(seg, seg_stride, h, rS, rel, stp, delta, sc);
  else segment_frame(s, f, h, rS, rel, stp, delta, sc);

  if (!kAffine) {
    // Corner fields: colour and intensity are linear in the corner values, so the voxel's share
    // of the composite, sum_k w_k sum_c b_c(u_k) v_c, is sum_c v_c W_c with W_c = sum_k w_k
    // b_c(u_k): only the density is interpolated per sample, and each colour or intensity
    // channel takes one dot product per voxel.
    float W[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) W[i] = 0.0f;
    for (int k = 0; k < S; ++k) {
      const float fk = (float)k + 0.5f;
      float u[3], w[8];
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = sample_u(rel[a], stp[a], fk, sc);
      corner_weights(u, w);
      const float sigma = dot8(w, g);
      const float e = __expf(-sigma * delta);
      const float wgt = acc.T * (1.0f - e);
      if (RGB || INT) {
#pragma unroll
        for (int i = 0; i < 8; ++i) W[i] = fmaf(wgt, w[i], W[i]);
      }
      acc.D = fmaf(wgt, fmaf(fk, delta, ti), acc.D);
      acc.T *= e;
    }
    if (RGB) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) acc.C[ch] += dot8(W, c[ch]);
    }
    if (INT) acc.I += dot8(W, it);
    acc.n += 1;
    return !(acc.T < t_min);
  }

  // the paper field and its SDF variant: colour and intensity are sigmoids of affine forms, so
  // every sample evaluates them
  for (int k = 0; k < S; ++k) {
    const float fk = (float)k + 0.5f;
    float u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = sample_u(rel[a], stp[a], fk, sc);
    float sigma, col[3] = {0.0f, 0.0f, 0.0f}, inten = 0.0f;
    float x[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fmaf(2.0f, u[a], -1.0f);
    const float q = fmaf(g[0], x[0], fmaf(g[1], x[1], fmaf(g[2], x[2], g[3])));
    sigma = FIELD == kFieldSdf ? sdf_sigma(q, sdf_ha, sdf_ib) : __expf(q);
    if (RGB) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch)
        col[ch] = sigmoid_f(fmaf(c[ch][0], x[0], fmaf(c[ch][1], x[1], fmaf(c[ch][2], x[2], shc[ch]))));
    }
    if (INT) inten = sigmoid_f(fmaf(it[0], x[0], fmaf(it[1], x[1], fmaf(it[2], x[2], it[3]))));
    const float e = __expf(-sigma * delta);
    const float wgt = acc.T * (1.0f - e);
    if (RGB) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) acc.C[ch] = fmaf(wgt, col[ch], acc.C[ch]);
    }
    acc.D = fmaf(wgt, fmaf(fk, delta, ti), acc.D);
    if (INT) acc.I = fmaf(wgt, inten, acc.I);
    acc.T *= e;
  }
  acc.n += 1;
  return !(acc.T < t_min);
}

// Shade one voxel hit with its parameters read from the scene (activated copies for pre-activated
// corner scenes); coalescing across lanes comes from coherent rays.
template <int FIELD, bool RGB, bool INT>
__device__ __forceinline__ bool shade_voxel(const SceneView& s, const RayFrame& f, const float sh[4], const Hit& h,
                                            int S, double rS, float t_min, Accum& acc,
                                            const double* seg = nullptr, int seg_stride = 0) {
  const int64_t v = h.voxel;
  constexpr bool kAct = FIELD == kFieldCornerActivated;
  const float* geo = kAct ? s.act_geo : s.geo;
  const float* rgb = kAct ? s.act_rgb : s.rgb;
  const float* itn = kAct ? s.act_int : s.inten;
  return shade_rows<FIELD, RGB, INT>(s, f, sh, h, S, rS, t_min, acc, geo + v * 8, RGB ? rgb + v * 24 : nullptr,
                                     INT ? itn + v * 8 : nullptr, seg, seg_stride);
}

}  // namespace salf
