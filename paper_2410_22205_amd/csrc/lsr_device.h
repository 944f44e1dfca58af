// Device-side building blocks of the narrow-band semi-Lagrangian solver
// (Preda & Semplice, arXiv:2410.22205): grid addressing, centred gradients,
// the cut-off, the Q1 and tensor WENO interpolants of Section 3.2 and the
// node update of Section 3.1.  Single precision throughout, except the
// distance field, which is built in double (lsr_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Unrolling of the foot-point loop and of the outer (x) WENO loop: fully
// unrolled, the 3D WENO update keeps all 256 stencil loads in flight and
// needs more registers than leave room for a second wave per SIMD.
#ifndef LSR_FOOT_UNROLL
#define LSR_FOOT_UNROLL 1
#endif
#ifndef LSR_WENO_X_UNROLL
#define LSR_WENO_X_UNROLL 2
#endif
#define LSR_PRAGMA(x) _Pragma(#x)
#define LSR_UNROLL(n) LSR_PRAGMA(unroll n)

namespace lsr {

// Four consecutive floats loaded with one 16-byte access at any 4-byte
// aligned address (global memory accepts dword-aligned multi-dword loads).
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

// Grid geometry as the kernels see it.  Band lists hold packed node
// coordinates: code = (i << (bits_j + bits_k)) | (j << bits_k) | k.
struct DevGrid {
  int n0, n1, n2;        // nodes per axis (n2 = 1 in 2D)
  uint32_t s0, s1;       // strides of axes 0 and 1 (axis 2 has stride 1)
  uint32_t N;            // total nodes
  int bits_j, bits_k;    // bit widths of j and k in a packed code
  float h, inv_h;
  double hd, lo0, lo1, lo2;
};

// Per-step constants of the update, derived on the host from the parameters.
struct StepConst {
  float gamma, beta, inv_gb3;  // band half width, cut-off radius, 1/(gamma-beta)^3
  float drift;                 // dt / h: drift in cells per unit C and |grad d|
  float diff2;                 // delta dt / (p h^2): squared diffusion reach in cells per unit C d
  float grad_thr;              // C dt^alpha of the fallback test
  float weno_e;                // h^4 (eps = h^2 with indicators scaled by h^2)
  float half_inv_h, inv_h;
};

__device__ __forceinline__ void decode(const DevGrid& g, uint32_t code, int& i, int& j, int& k) {
  k = (int)(code & ((1u << g.bits_k) - 1u));
  j = (int)((code >> g.bits_k) & ((1u << g.bits_j) - 1u));
  i = (int)(code >> (g.bits_j + g.bits_k));
}

__device__ __forceinline__ uint32_t encode(const DevGrid& g, int i, int j, int k) {
  return ((uint32_t)i << (g.bits_j + g.bits_k)) | ((uint32_t)j << g.bits_k) | (uint32_t)k;
}

__device__ __forceinline__ uint32_t lin(const DevGrid& g, int i, int j, int k) {
  return (uint32_t)i * g.s0 + (uint32_t)j * g.s1 + (uint32_t)k;
}

// Cut-off of eq. (cutoff).
__device__ __forceinline__ float cutoff(float phi, const StepConst& c) {
  float a = fabsf(phi);
  if (a <= c.beta) return 1.0f;
  if (a > c.gamma) return 0.0f;
  float t = a - c.gamma;
  return t * t * (2.0f * a + c.gamma - 3.0f * c.beta) * c.inv_gb3;
}

// Centred difference along one axis from the node value and its two
// neighbours; first-order one-sided on the domain boundary.
__device__ __forceinline__ float cdiff(float vm, float v, float vp, int idx, int n,
                                       const StepConst& c) {
  if (idx > 0 && idx < n - 1) return (vp - vm) * c.half_inv_h;
  if (idx == 0) return (vp - v) * c.inv_h;
  return (v - vm) * c.inv_h;
}

// Cell and local coordinate of a foot point given as node index + offset in
// cells, the point being moved onto the grid if it left it.
struct Loc {
  int i0;
  float t;
};

__device__ __forceinline__ Loc locate(int i, float off, int n) {
  float fl = floorf(off);
  Loc r;
  r.i0 = i + (int)fl;
  r.t = off - fl;
  if (r.i0 < 0) {
    r.i0 = 0;
    r.t = 0.0f;
  } else if (r.i0 >= n - 1) {
    r.i0 = n - 2;
    r.t = 1.0f;
  }
  return r;
}

__device__ __forceinline__ int clampi(int i, int n) { return i < 0 ? 0 : (i > n - 1 ? n - 1 : i); }

// Per-axis constants of the one-dimensional WENO interpolant at s = t.
struct WC {
  float t, ht, ht2, tr, cL, cR;
};

__device__ __forceinline__ WC wcoef(float t) {
  WC c;
  c.t = t;
  c.ht = 0.5f * t;
  c.ht2 = 0.5f * t * t;
  c.tr = c.ht2 - c.ht;
  c.cL = (2.0f - t) * (1.0f / 3.0f);
  c.cR = (1.0f + t) * (1.0f / 3.0f);
  return c;
}

// Third-order WENO on (v0, v1, v2, v3) = (v_{j-1}, v_j, v_{j+1}, v_{j+2}):
//   P_L = v_j + (t/2)(v_{j+1} - v_{j-1}) + (t^2/2) D_L,  D_L = v_{j-1} - 2v_j + v_{j+1}
//   P_R = v_j + t (v_{j+1} - v_j) + ((t^2 - t)/2) D_R,    D_R = v_j - 2v_{j+1} + v_{j+2}
// are the two quadratic interpolants, the indicators are D^2/h^2 and eps = h^2,
// so with s_k = D_k^2 + h^4 the weights are w_L = C_L s_R^2 / (C_L s_R^2 + C_R s_L^2)
// (the common factor h^4 of alpha_L and alpha_R cancels).
__device__ __forceinline__ float weno1(float v0, float v1, float v2, float v3, const WC& c,
                                       float e) {
  float dL = fmaf(-2.0f, v1, v0 + v2);
  float dR = fmaf(-2.0f, v2, v1 + v3);
  float pL = fmaf(c.ht2, dL, fmaf(c.ht, v2 - v0, v1));
  float pR = fmaf(c.tr, dR, fmaf(c.t, v2 - v1, v1));
  float sL = fmaf(dL, dL, e);
  float sR = fmaf(dR, dR, e);
  float aL = c.cL * (sR * sR);
  float aR = c.cR * (sL * sL);
  float w = aL * __builtin_amdgcn_rcpf(aL + aR);
  return fmaf(w, pL - pR, pR);
}

// Four values along the last axis at k0-1 .. k0+2 (indices clamped to the
// grid, i.e. the boundary node repeated) of the row starting at `row`.
__device__ __forceinline__ f4u row4(const float* __restrict__ A, uint32_t row, int k0, int n) {
  if (k0 >= 1 && k0 + 2 <= n - 1) return *(const f4u*)(A + row + (uint32_t)(k0 - 1));
  f4u r;
  r.x = A[row + clampi(k0 - 1, n)];
  r.y = A[row + clampi(k0, n)];
  r.z = A[row + clampi(k0 + 1, n)];
  r.w = A[row + clampi(k0 + 2, n)];
  return r;
}

// Tensor WENO (Section 3.2): one-dimensional WENO along the last axis
// first, then along the previous axes, x last.
__device__ __forceinline__ float interp_weno3(const float* __restrict__ A, const DevGrid& g,
                                              const Loc& lx, const Loc& ly, const Loc& lz,
                                              float e) {
  const WC cx = wcoef(lx.t), cy = wcoef(ly.t), cz = wcoef(lz.t);
  float wx[4];
LSR_UNROLL(LSR_WENO_X_UNROLL)
  for (int a = 0; a < 4; ++a) {
    const uint32_t ra = (uint32_t)clampi(lx.i0 - 1 + a, g.n0) * g.s0;
    float wy[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t row = ra + (uint32_t)clampi(ly.i0 - 1 + b, g.n1) * g.s1;
      f4u r = row4(A, row, lz.i0, g.n2);
      wy[b] = weno1(r.x, r.y, r.z, r.w, cz, e);
    }
    wx[a] = weno1(wy[0], wy[1], wy[2], wy[3], cy, e);
  }
  return weno1(wx[0], wx[1], wx[2], wx[3], cx, e);
}

__device__ __forceinline__ float interp_weno2(const float* __restrict__ A, const DevGrid& g,
                                              const Loc& lx, const Loc& ly, float e) {
  const WC cx = wcoef(lx.t), cy = wcoef(ly.t);
  float wx[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const uint32_t row = (uint32_t)clampi(lx.i0 - 1 + a, g.n0) * g.s0;
    f4u r = row4(A, row, ly.i0, g.n1);
    wx[a] = weno1(r.x, r.y, r.z, r.w, cy, e);
  }
  return weno1(wx[0], wx[1], wx[2], wx[3], cx, e);
}

// Multilinear interpolation, eq. (IQ1).
__device__ __forceinline__ float interp_q1_3(const float* __restrict__ A, const DevGrid& g,
                                             const Loc& lx, const Loc& ly, const Loc& lz) {
  const uint32_t r00 = (uint32_t)lx.i0 * g.s0 + (uint32_t)ly.i0 * g.s1 + (uint32_t)lz.i0;
  f2u a00 = *(const f2u*)(A + r00);
  f2u a01 = *(const f2u*)(A + r00 + g.s1);
  f2u a10 = *(const f2u*)(A + r00 + g.s0);
  f2u a11 = *(const f2u*)(A + r00 + g.s0 + g.s1);
  float tz = lz.t, ty = ly.t, tx = lx.t;
  float b00 = fmaf(tz, a00.y - a00.x, a00.x);
  float b01 = fmaf(tz, a01.y - a01.x, a01.x);
  float b10 = fmaf(tz, a10.y - a10.x, a10.x);
  float b11 = fmaf(tz, a11.y - a11.x, a11.x);
  float c0 = fmaf(ty, b01 - b00, b00);
  float c1 = fmaf(ty, b11 - b10, b10);
  return fmaf(tx, c1 - c0, c0);
}

__device__ __forceinline__ float interp_q1_2(const float* __restrict__ A, const DevGrid& g,
                                             const Loc& lx, const Loc& ly) {
  const uint32_t r0 = (uint32_t)lx.i0 * g.s0 + (uint32_t)ly.i0;
  f2u a0 = *(const f2u*)(A + r0);
  f2u a1 = *(const f2u*)(A + r0 + g.s0);
  float b0 = fmaf(ly.t, a0.y - a0.x, a0.x);
  float b1 = fmaf(ly.t, a1.y - a1.x, a1.x);
  return fmaf(lx.t, b1 - b0, b0);
}

enum { UPD_FALLBACK = 1, UPD_FRAME0 = 2 };


// New value of band node (i,j,k) from phi^n = A: eqs. (SL2d)/(SL3d) with
// C = c(phi^n_j) (p = 1), the fallback of eq. (SL:2) and the cut of eq. (cut).
// dp = (d_x, d_y, d_z, d) with the centred gradient of d precomputed.
// Foot points are carried as node index + offset in cells.
template <int DIM, int INTERP>
__device__ __forceinline__ float sl_update(const float* __restrict__ A, const DevGrid& g,
                                           const StepConst& c, int i, int j, int k, uint32_t idx,
                                           float v, float4 dp, int& flags) {
  float gx, gy, gz = 0.0f;
  float xm = i > 0 ? A[idx - g.s0] : v, xp = i < g.n0 - 1 ? A[idx + g.s0] : v;
  float ym = j > 0 ? A[idx - g.s1] : v, yp = j < g.n1 - 1 ? A[idx + g.s1] : v;
  gx = cdiff(xm, v, xp, i, g.n0, c);
  gy = cdiff(ym, v, yp, j, g.n1, c);
  float zm = v, zp = v;
  if (DIM == 3) {
    zm = k > 0 ? A[idx - 1] : v;
    zp = k < g.n2 - 1 ? A[idx + 1] : v;
    gz = cdiff(zm, v, zp, k, g.n2, c);
  }
  float nrm2 = gx * gx + gy * gy + gz * gz;
  float nrm = sqrtf(nrm2);
  float out;
  if (nrm < c.grad_thr) {
    float sum = 0.0f, cnt = 0.0f;
    if (i > 0) { sum += xm; cnt += 1.0f; }
    if (i < g.n0 - 1) { sum += xp; cnt += 1.0f; }
    if (j > 0) { sum += ym; cnt += 1.0f; }
    if (j < g.n1 - 1) { sum += yp; cnt += 1.0f; }
    if (DIM == 3) {
      if (k > 0) { sum += zm; cnt += 1.0f; }
      if (k < g.n2 - 1) { sum += zp; cnt += 1.0f; }
    }
    out = sum / cnt;
    flags |= UPD_FALLBACK;
  } else {
    const float C = cutoff(v, c);
    const float dd = dp.w;
    const float amp = sqrtf(C * dd * c.diff2);  // diffusion reach in cells
    const float cd = C * c.drift;
    const float bx = cd * dp.x, by = cd * dp.y;
    if (DIM == 2) {
      const float inv = 1.0f / nrm;
      const float sx = gy * inv * amp, sy = -gx * inv * amp;  // eq. (sigma2d), scaled
      float acc = 0.0f;
#pragma unroll
      for (int l = -1; l <= 1; l += 2) {
        Loc lx = locate(i, bx + sx * (float)l, g.n0);
        Loc ly = locate(j, by + sy * (float)l, g.n1);
        acc += INTERP == 0 ? interp_q1_2(A, g, lx, ly) : interp_weno2(A, g, lx, ly, c.weno_e);
      }
      out = 0.5f * acc;
    } else {
      const float bz = cd * dp.z;
      float n1x, n1y, n1z, n2x, n2y, n2z;
      const float s2 = gx * gx + gz * gz;
      if (s2 != 0.0f) {  // eq. (sigma3d)
        const float s = sqrtf(s2);
        const float is = 1.0f / s;
        const float isn = is / nrm;
        n1x = -gz * is; n1y = 0.0f; n1z = gx * is;
        n2x = -gx * gy * isn; n2y = s / nrm; n2z = -gy * gz * isn;
      } else {
        n1x = 1.0f; n1y = 0.0f; n1z = 0.0f;
        n2x = 0.0f; n2y = 0.0f; n2z = 1.0f;
        flags |= UPD_FRAME0;
      }
      n1x *= amp; n1y *= amp; n1z *= amp;
      n2x *= amp; n2y *= amp; n2z *= amp;
      float acc = 0.0f;
LSR_UNROLL(LSR_FOOT_UNROLL)
      for (int q = 0; q < 4; ++q) {
        const float f1 = (q & 2) ? 1.0f : -1.0f, f2 = (q & 1) ? 1.0f : -1.0f;
        Loc lx = locate(i, bx + f1 * n1x + f2 * n2x, g.n0);
        Loc ly = locate(j, by + f1 * n1y + f2 * n2y, g.n1);
        Loc lz = locate(k, bz + f1 * n1z + f2 * n2z, g.n2);
        acc += INTERP == 0 ? interp_q1_3(A, g, lx, ly, lz)
                           : interp_weno3(A, g, lx, ly, lz, c.weno_e);
      }
      out = 0.25f * acc;
    }
  }
  return fminf(fmaxf(out, -c.gamma), c.gamma);
}

}  // namespace lsr
