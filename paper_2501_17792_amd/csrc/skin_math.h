// Device math of the per-Gaussian stages: bone blending, linear blend
// skinning, EWA projection, SH colour and the opacity-aware footprint.
// Every function is written with explicit fmaf() and compiled with
// -ffp-contract=off so that a value computed in two kernels (for example the
// skinned mean in the skin kernel and again in the backward) has the same
// bits. The fused skinning + projection works in the camera frame and rounds
// differently from the separate stages (same mathematics).
#pragma once

#include "cs_internal.h"

namespace cs {

// M = sum_k w_k B[idx_k] for the 3x4 row-major bone matrices held in LDS.
__device__ __forceinline__ void blend_bones(const float* __restrict__ bones, uint32_t idx4, float4 w,
                                            float M[12]) {
  const float* b0 = bones + 12 * (idx4 & 0xffu);
  const float* b1 = bones + 12 * ((idx4 >> 8) & 0xffu);
  const float* b2 = bones + 12 * ((idx4 >> 16) & 0xffu);
  const float* b3 = bones + 12 * (idx4 >> 24);
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    float m = w.x * b0[e];
    m = fmaf(w.y, b1[e], m);
    m = fmaf(w.z, b2[e], m);
    m = fmaf(w.w, b3[e], m);
    M[e] = m;
  }
}

// Sigma' = L Sigma L^T for symmetric Sigma (xx xy xz yy yz zz); L row-major 3x3.
__device__ __forceinline__ void congruence(const float L[9], const float S[6], float out[6]) {
  const float s00 = S[0], s01 = S[1], s02 = S[2], s11 = S[3], s12 = S[4], s22 = S[5];
  float T[9];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float l0 = L[3 * r], l1 = L[3 * r + 1], l2 = L[3 * r + 2];
    T[3 * r + 0] = fmaf(l0, s00, fmaf(l1, s01, l2 * s02));
    T[3 * r + 1] = fmaf(l0, s01, fmaf(l1, s11, l2 * s12));
    T[3 * r + 2] = fmaf(l0, s02, fmaf(l1, s12, l2 * s22));
  }
  // rows r <= c of T L^T
  out[0] = fmaf(T[0], L[0], fmaf(T[1], L[1], T[2] * L[2]));
  out[1] = fmaf(T[0], L[3], fmaf(T[1], L[4], T[2] * L[5]));
  out[2] = fmaf(T[0], L[6], fmaf(T[1], L[7], T[2] * L[8]));
  out[3] = fmaf(T[3], L[3], fmaf(T[4], L[4], T[5] * L[5]));
  out[4] = fmaf(T[3], L[6], fmaf(T[4], L[7], T[5] * L[8]));
  out[5] = fmaf(T[6], L[6], fmaf(T[7], L[7], T[8] * L[8]));
}

// Posed mean, posed covariance and the 3x3 used for the colour direction of
// one template Gaussian under blended bone matrix M.
struct Posed {
  float mu[3];
  float cov[6];
  float L[9];
};

__device__ __forceinline__ void yaw_rotation(float yaw, float Ry[9]) {
  const float c = cosf(yaw), s = sinf(yaw);
  Ry[0] = c;    Ry[1] = 0.f; Ry[2] = s;
  Ry[3] = 0.f;  Ry[4] = 1.f; Ry[5] = 0.f;
  Ry[6] = -s;   Ry[7] = 0.f; Ry[8] = c;
}

__device__ __forceinline__ void skin_gaussian(const float* __restrict__ bones, float4 mean_idx,
                                              float4 w, float4 ca, float2 cb, int means_only,
                                              const float Ry[9], Posed& p) {
  float M[12];
  blend_bones(bones, __float_as_uint(mean_idx.w), w, M);
  const float x = mean_idx.x, y = mean_idx.y, z = mean_idx.z;
  p.mu[0] = fmaf(M[0], x, fmaf(M[1], y, fmaf(M[2], z, M[3])));
  p.mu[1] = fmaf(M[4], x, fmaf(M[5], y, fmaf(M[6], z, M[7])));
  p.mu[2] = fmaf(M[8], x, fmaf(M[9], y, fmaf(M[10], z, M[11])));
  if (means_only) {
#pragma unroll
    for (int e = 0; e < 9; ++e) p.L[e] = Ry[e];
  } else {
    p.L[0] = M[0]; p.L[1] = M[1]; p.L[2] = M[2];
    p.L[3] = M[4]; p.L[4] = M[5]; p.L[5] = M[6];
    p.L[6] = M[8]; p.L[7] = M[9]; p.L[8] = M[10];
  }
  const float S[6] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y};
  congruence(p.L, S, p.cov);
}

// Real orthonormal SH basis (no Condon-Shortley phase, polar axis +z) at a
// unit direction, evaluated against [(deg+1)^2][3] coefficients read from
// float4 planes (plane j holds flattened coefficients 4j..4j+3).
template <int DEG, class Planes>
__device__ __forceinline__ void sh_colour(Planes planes, int stride, float x, float y, float z, float rgb[3]) {
  constexpr int NB = (DEG + 1) * (DEG + 1);  // basis functions
  constexpr int N4 = (3 * NB + 3) / 4;       // float4 planes of the 3*NB coefficients
  float4 v[N4];
#pragma unroll
  for (int j = 0; j < N4; ++j) v[j] = planes[(size_t)j * stride];  // every plane in flight at once
  float Y[NB];
  Y[0] = 0.28209479177387814f;
  if constexpr (DEG >= 1) {
    Y[1] = 0.4886025119029199f * y;
    Y[2] = 0.4886025119029199f * z;
    Y[3] = 0.4886025119029199f * x;
  }
  if constexpr (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * (x * y);
    Y[5] = 1.0925484305920792f * (y * z);
    Y[6] = 0.31539156525252005f * fmaf(3.f, zz, -1.f);
    Y[7] = 1.0925484305920792f * (x * z);
    Y[8] = 0.5462742152960396f * (xx - yy);
    if constexpr (DEG >= 3) {
      Y[9] = 0.5900435899266435f * y * fmaf(3.f, xx, -yy);
      Y[10] = 2.890611442640554f * (x * y) * z;
      Y[11] = 0.4570457994644658f * y * fmaf(5.f, zz, -1.f);
      Y[12] = 0.3731763325901154f * z * fmaf(5.f, zz, -3.f);
      Y[13] = 0.4570457994644658f * x * fmaf(5.f, zz, -1.f);
      Y[14] = 1.445305721320277f * z * (xx - yy);
      Y[15] = 0.5900435899266435f * x * fmaf(-3.f, yy, xx);
    }
  }
  float acc[3] = {0.f, 0.f, 0.f};
  // coefficient q = 3k + c lives in plane q/4, lane q%4
#pragma unroll
  for (int j = 0; j < N4; ++j) {
    const float e[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int q = 4 * j + l;
      const int k = q / 3;
      if (k < NB) acc[q - 3 * k] = fmaf(e[l], Y[k], acc[q - 3 * k]);
    }
  }
  rgb[0] = fmaxf(0.f, 0.5f + acc[0]);
  rgb[1] = fmaxf(0.f, 0.5f + acc[1]);
  rgb[2] = fmaxf(0.f, 0.5f + acc[2]);
}

struct SplatRec {
  float4 r0, r1, r2;   // (u v rx ry) (A B C o) (r g b depth)
  uint32_t rect;
  uint32_t count;
};

// Screen-space tail shared by both projection forms: the opacity-aware
// footprint, the tile rect (tile sides are powers of two: 8, 16 or 32) and
// the colour along the unnormalised canonical-frame view direction (d0, d1,
// d2). a, b, c: the 2D covariance with the low-pass added; det = ac - b^2.
template <int DEG, class Planes>
__device__ __forceinline__ void finish_splat(float u, float v, float a, float b, float c, float det, float tz,
                                             float opacity, float d0, float d1, float d2, Planes sh_planes,
                                             int sh_stride, const CamDev& cam, SplatRec& out) {
  if (!(det > 0.f)) return;
  if (opacity < (1.f / 255.f)) return;
  // k = 2 ln(255 o) (1 + 1e-4); hardware log2 and sqrt (1 ulp each) sit far
  // inside the 1e-4 relative and 0.01 px margins of the box
  const float k = (2.f * 0.6931471805599453f) * __builtin_amdgcn_logf(fmaxf(255.f * opacity, 1.f)) * (1.f + 1e-4f);
  const float rx = __builtin_amdgcn_sqrtf(k * a) + 0.01f;
  const float ry = __builtin_amdgcn_sqrtf(k * c) + 0.01f;
  const float fx0 = floorf(u - rx), fx1 = floorf(u + rx);
  const float fy0 = floorf(v - ry), fy1 = floorf(v + ry);
  if (fx1 < 0.f || fx0 > (float)(cam.W - 1) || fy1 < 0.f || fy0 > (float)(cam.H - 1)) return;
  const int px0 = (int)fmaxf(fx0, 0.f), px1 = (int)fminf(fx1, (float)(cam.W - 1));
  const int py0 = (int)fmaxf(fy0, 0.f), py1 = (int)fminf(fy1, (float)(cam.H - 1));
  const int sx = __builtin_ctz((unsigned)cam.tw), sy = __builtin_ctz((unsigned)cam.th);
  const int x0 = px0 >> sx, x1 = px1 >> sx, y0 = py0 >> sy, y1 = py1 >> sy;
  const float inv = __builtin_amdgcn_rsqf(fmaf(d0, d0, fmaf(d1, d1, d2 * d2)));
  d0 *= inv; d1 *= inv; d2 *= inv;
  float rgb[3];
  sh_colour<DEG>(sh_planes, sh_stride, d0, d1, d2, rgb);
  out.r0 = make_float4(u, v, rx, ry);
  const float idet = __builtin_amdgcn_rcpf(det);  // det >= 0.09 (the 0.3 px^2 low-pass)
  out.r1 = make_float4(c * idet, -b * idet, a * idet, opacity);
  out.r2 = make_float4(rgb[0], rgb[1], rgb[2], tz);
  out.rect = (uint32_t)x0 | ((uint32_t)y0 << 8) | ((uint32_t)x1 << 16) | ((uint32_t)y1 << 24);
  out.count = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
}

// 2D covariance (a, b, c, low-pass added) of a Gaussian with 3D covariance S
// (xx xy xz yy yz zz) under the 2x3 map with rows T0, T1.
__device__ __forceinline__ void ewa_2d(const float T0[3], const float T1[3], const float S[6], float& a, float& b,
                                       float& c) {
  const float P00 = fmaf(T0[0], S[0], fmaf(T0[1], S[1], T0[2] * S[2]));
  const float P01 = fmaf(T0[0], S[1], fmaf(T0[1], S[3], T0[2] * S[4]));
  const float P02 = fmaf(T0[0], S[2], fmaf(T0[1], S[4], T0[2] * S[5]));
  const float P10 = fmaf(T1[0], S[0], fmaf(T1[1], S[1], T1[2] * S[2]));
  const float P11 = fmaf(T1[0], S[1], fmaf(T1[1], S[3], T1[2] * S[4]));
  const float P12 = fmaf(T1[0], S[2], fmaf(T1[1], S[4], T1[2] * S[5]));
  a = fmaf(P00, T0[0], fmaf(P01, T0[1], P02 * T0[2])) + 0.3f;
  b = fmaf(P00, T1[0], fmaf(P01, T1[1], P02 * T1[2]));
  c = fmaf(P10, T1[0], fmaf(P11, T1[1], P12 * T1[2])) + 0.3f;
}

// EWA projection + colour + footprint of one posed Gaussian (world-frame
// posed mean and covariance, as the separate skinning stage writes them).
// count = 0 means culled.
template <int DEG, class Planes>
__device__ __forceinline__ void project_gaussian(const Posed& p, float opacity, Planes sh_planes, int sh_stride,
                                                 const CamDev& cam, SplatRec& out) {
  out.count = 0u;
  out.rect = 0u;
  out.r0 = out.r1 = out.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
  const float dx = p.mu[0] - cam.eye[0], dy = p.mu[1] - cam.eye[1], dz = p.mu[2] - cam.eye[2];
  const float* R = cam.R;
  const float tx = fmaf(R[0], dx, fmaf(R[1], dy, R[2] * dz));
  const float ty = fmaf(R[3], dx, fmaf(R[4], dy, R[5] * dz));
  const float tz = fmaf(R[6], dx, fmaf(R[7], dy, R[8] * dz));
  if (!(tz > cam.near_plane)) return;
  // One hardware reciprocal (1 ulp) serves the perspective divide and the
  // Jacobian; tz > near > 0, so no special cases arise.
  const float itz = __builtin_amdgcn_rcpf(tz);
  const float xn = tx * itz, yn = ty * itz;
  if (fabsf(xn) > cam.lim_x || fabsf(yn) > cam.lim_y) return;
  const float u = fmaf(cam.fx, xn, cam.cx);
  const float v = fmaf(cam.fy, yn, cam.cy);
  const float j00 = cam.fx * itz, j11 = cam.fy * itz;
  const float j02 = -(cam.fx * xn) * itz, j12 = -(cam.fy * yn) * itz;
  float T0[3], T1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T0[k] = fmaf(j00, R[k], j02 * R[6 + k]);
    T1[k] = fmaf(j11, R[3 + k], j12 * R[6 + k]);
  }
  float a, b, c;
  ewa_2d(T0, T1, p.cov, a, b, c);
  const float det = a * c - b * b;
  // colour: view direction in the canonical frame, L^T (mu' - eye)
  const float* L = p.L;
  const float d0 = fmaf(L[0], dx, fmaf(L[3], dy, L[6] * dz));
  const float d1 = fmaf(L[1], dx, fmaf(L[4], dy, L[7] * dz));
  const float d2 = fmaf(L[2], dx, fmaf(L[5], dy, L[8] * dz));
  finish_splat<DEG>(u, v, a, b, c, det, tz, opacity, d0, d1, d2, sh_planes, sh_stride, cam, out);
}

// Skinning and projection in one step, in the camera frame. The bone
// matrices are given pre-rotated into the camera frame (Bc_j = R_c B_j), so
// the blended matrix is Mc = R_c M: the camera-space mean is
// t = Mc [mu; 1] - R_c eye (c0 = R_c eye), the EWA map J R_c L is J Lc with
// Lc = Mc[:, :3] (R_c R_y when only means are skinned: RcL), Sigma2D comes
// from the canonical covariance S directly (Sigma' = L S L^T is never
// formed), and the canonical-frame view direction L^T (mu' - eye) is Lc^T t
// (R_c is orthonormal). Same mathematics as skin_gaussian + project_gaussian,
// rounded differently.
template <int DEG, class Planes>
__device__ __forceinline__ void project_fused(const float* __restrict__ bones_cam, float4 mean_idx, float4 w,
                                              const float S[6], int means_only, const float RcL[9],
                                              const float c0[3], float opacity, Planes sh_planes,
                                              const CamDev& cam, SplatRec& out) {
  out.count = 0u;
  out.rect = 0u;
  out.r0 = out.r1 = out.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
  float M[12];
  blend_bones(bones_cam, __float_as_uint(mean_idx.w), w, M);
  const float x = mean_idx.x, y = mean_idx.y, z = mean_idx.z;
  const float tx = fmaf(M[0], x, fmaf(M[1], y, fmaf(M[2], z, M[3]))) - c0[0];
  const float ty = fmaf(M[4], x, fmaf(M[5], y, fmaf(M[6], z, M[7]))) - c0[1];
  const float tz = fmaf(M[8], x, fmaf(M[9], y, fmaf(M[10], z, M[11]))) - c0[2];
  if (!(tz > cam.near_plane)) return;
  const float itz = __builtin_amdgcn_rcpf(tz);
  const float xn = tx * itz, yn = ty * itz;
  if (fabsf(xn) > cam.lim_x || fabsf(yn) > cam.lim_y) return;
  const float u = fmaf(cam.fx, xn, cam.cx);
  const float v = fmaf(cam.fy, yn, cam.cy);
  const float j00 = cam.fx * itz, j11 = cam.fy * itz;
  const float j02 = -(cam.fx * xn) * itz, j12 = -(cam.fy * yn) * itz;
  float L[9];
  if (means_only) {
#pragma unroll
    for (int e = 0; e < 9; ++e) L[e] = RcL[e];
  } else {
    L[0] = M[0]; L[1] = M[1]; L[2] = M[2];
    L[3] = M[4]; L[4] = M[5]; L[5] = M[6];
    L[6] = M[8]; L[7] = M[9]; L[8] = M[10];
  }
  float T0[3], T1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T0[k] = fmaf(j00, L[k], j02 * L[6 + k]);
    T1[k] = fmaf(j11, L[3 + k], j12 * L[6 + k]);
  }
  float a, b, c;
  ewa_2d(T0, T1, S, a, b, c);
  const float det = a * c - b * b;
  const float d0 = fmaf(L[0], tx, fmaf(L[3], ty, L[6] * tz));
  const float d1 = fmaf(L[1], tx, fmaf(L[4], ty, L[7] * tz));
  const float d2 = fmaf(L[2], tx, fmaf(L[5], ty, L[8] * tz));
  finish_splat<DEG>(u, v, a, b, c, det, tz, opacity, d0, d1, d2, sh_planes, 1, cam, out);
}

}  // namespace cs
