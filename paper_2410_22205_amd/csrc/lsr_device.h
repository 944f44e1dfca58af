// Device-side building blocks of the narrow-band semi-Lagrangian solver
// (Preda & Semplice, arXiv:2410.22205): grid addressing, centred gradients,
// the cut-off, the Q1 and tensor WENO interpolants of Section 3.2 and the
// node update of Section 3.1.  Templated on the real type T of the state
// (float or double); the distance field is always built in double.
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

// Consecutive values loaded with 16-byte accesses at any element-aligned
// address (global memory accepts dword-aligned multi-dword loads).
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef double d4u __attribute__((ext_vector_type(4), aligned(8)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

typedef float f4a __attribute__((ext_vector_type(4)));   // naturally aligned
typedef double d4a __attribute__((ext_vector_type(4)));

template <typename T> struct Vec;
template <> struct Vec<float> {
  typedef f4u v4;
  typedef f2u v2;
  typedef float4 pack;  // (d_x, d_y, d_z, d) as stored
  typedef f4a p4;       // the same, as the step kernel reads it
};
template <> struct Vec<double> {
  typedef d4u v4;
  typedef d2u v2;
  typedef double4 pack;
  typedef d4a p4;
};

// Pointers into device memory with the address space in the type.  Loads
// and stores through them compile to global-memory instructions even when the
// pointer itself was read from a table in memory (the batched kernels), where
// the compiler cannot infer the address space and would use flat ones.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
using gwptr = __attribute__((address_space(1))) T*;

// Grid geometry as the kernels see it.  Band lists hold packed node
// coordinates: code = (i << (bits_j + bits_k)) | (j << bits_k) | k.
struct DevGrid {
  int n0, n1, n2;        // nodes per axis (n2 = 1 in 2D)
  uint32_t s0, s1;       // strides of axes 0 and 1 (axis 2 has stride 1)
  uint32_t N;            // total nodes
  int bits_j, bits_k;    // bit widths of j and k in a packed code
  double hd, lo0, lo1, lo2;
};

// Per-step constants of the update, derived on the host from the parameters.
template <typename T>
struct StepConst {
  T gamma, beta, inv_gb3;  // band half width, cut-off radius, 1/(gamma-beta)^3
  T drift;                 // dt / h: drift in cells per unit C and |grad d|
  T diff2;                 // delta dt / (p h^2): squared diffusion reach in cells per unit C d
  T grad_thr;              // C dt^alpha of the fallback test
  T weno_e;                // h^4 (eps = h^2 with indicators scaled by h^2)
  T pm1;                   // p - 1: 0 or 1 (p = 1 or 2)
  T inv_E;                 // 1 / E_p(phi^n) when p = 2, reduced on the device per step
  T half_inv_h, inv_h;
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

// Sign words of phi: one bit per node, 1 where phi < 0, packed 32 to a word
// along rows of the last axis (3D: rows (i, j) along k; 2D: rows i along j),
// each row starting a new word; bits past a row's end are 0.
__host__ __device__ inline uint32_t sign_row_words(int n_last) { return ((uint32_t)n_last + 31u) / 32u; }

__device__ __forceinline__ void sign_word_of(const DevGrid& g, int i, int j, int k, uint32_t& w,
                                             uint32_t& bit) {
  if (g.n2 > 1) {
    w = ((uint32_t)i * (uint32_t)g.n1 + (uint32_t)j) * sign_row_words(g.n2) + (uint32_t)k / 32u;
    bit = 1u << (k & 31);
  } else {
    w = (uint32_t)i * sign_row_words(g.n1) + (uint32_t)j / 32u;
    bit = 1u << (j & 31);
  }
}

// The node's bit set to its new side (idempotent: repeating it changes nothing).
__device__ __forceinline__ void sign_set(uint32_t* sgn, uint32_t w, uint32_t bit, bool neg) {
  if (neg)
    atomicOr(sgn + w, bit);
  else
    atomicAnd(sgn + w, ~bit);
}

// Reciprocal: the hardware approximation in single precision (1 ulp); in
// double, the approximation refined by one Newton step.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Cut-off of eq. (cutoff).
template <typename T>
__device__ __forceinline__ T cutoff(T phi, const StepConst<T>& c) {
  T a = fabs(phi);
  if (a <= c.beta) return T(1);
  if (a > c.gamma) return T(0);
  T t = a - c.gamma;
  return t * t * (T(2) * a + c.gamma - T(3) * c.beta) * c.inv_gb3;
}

// Centred difference along one axis from the node value and its two
// neighbours; first-order one-sided on the domain boundary.
template <typename T>
__device__ __forceinline__ T cdiff(T vm, T v, T vp, int idx, int n, const StepConst<T>& c) {
  if (idx > 0 && idx < n - 1) return (vp - vm) * c.half_inv_h;
  if (idx == 0) return (vp - v) * c.inv_h;
  return (v - vm) * c.inv_h;
}

// Cell and local coordinate of a foot point given as node index + offset in
// cells, the point being moved onto the grid if it left it.
template <typename T>
struct Loc {
  int i0;
  T t;
};

template <typename T>
__device__ __forceinline__ Loc<T> locate(int i, T off, int n) {
  T fl = floor(off);
  Loc<T> r;
  r.i0 = i + (int)fl;
  r.t = off - fl;
  if (r.i0 < 0) {
    r.i0 = 0;
    r.t = T(0);
  } else if (r.i0 >= n - 1) {
    r.i0 = n - 2;
    r.t = T(1);
  }
  return r;
}

__device__ __forceinline__ int clampi(int i, int n) { return i < 0 ? 0 : (i > n - 1 ? n - 1 : i); }

// Per-axis constants of the one-dimensional WENO interpolant at s = t.
template <typename T>
struct WC {
  T t, ht, ht2, tr, cL, cR;
};

template <typename T>
__device__ __forceinline__ WC<T> wcoef(T t) {
  WC<T> c;
  c.t = t;
  c.ht = T(0.5) * t;
  c.ht2 = T(0.5) * t * t;
  c.tr = c.ht2 - c.ht;
  c.cL = (T(2) - t) * (T(1) / T(3));
  c.cR = (T(1) + t) * (T(1) / T(3));
  return c;
}

// Third-order WENO on (v0, v1, v2, v3) = (v_{j-1}, v_j, v_{j+1}, v_{j+2}):
//   P_L = v_j + (t/2)(v_{j+1} - v_{j-1}) + (t^2/2) D_L,  D_L = v_{j-1} - 2v_j + v_{j+1}
//   P_R = v_j + t (v_{j+1} - v_j) + ((t^2 - t)/2) D_R,    D_R = v_j - 2v_{j+1} + v_{j+2}
// are the two quadratic interpolants, the indicators are D^2/h^2 and eps = h^2,
// so with s_k = D_k^2 + h^4 the weights are w_L = C_L s_R^2 / (C_L s_R^2 + C_R s_L^2)
// (the common factor h^4 of alpha_L and alpha_R cancels).
template <typename T>
__device__ __forceinline__ T weno1(T v0, T v1, T v2, T v3, const WC<T>& c, T e) {
  T dL = fma(T(-2), v1, v0 + v2);
  T dR = fma(T(-2), v2, v1 + v3);
  T pL = fma(c.ht2, dL, fma(c.ht, v2 - v0, v1));
  T pR = fma(c.tr, dR, fma(c.t, v2 - v1, v1));
  T sL = fma(dL, dL, e);
  T sR = fma(dR, dR, e);
  T aL = c.cL * (sR * sR);
  T aR = c.cR * (sL * sL);
  T w = aL * rcp(aL + aR);
  return fma(w, pL - pR, pR);
}

// The m-th of (x, y, z, w), m in 0..3, by selects (no indexed register
// access).
template <typename T>
__device__ __forceinline__ T pick4(T x, T y, T z, T w, int m) {
  return m == 0 ? x : (m == 1 ? y : (m == 2 ? z : w));
}

// Four values along the last axis at k0-1 .. k0+2 (indices clamped to the
// grid, i.e. the boundary node repeated) of the row starting at `row`.  One
// four-wide load from a start clamped into the row (every axis has at least
// four nodes) serves every lane; lanes within one node of the row's ends
// then take the clamped indices from it.  The load is issued the same way on
// every lane, so the loads of consecutive rows stay in flight together.
template <typename T>
__device__ __forceinline__ typename Vec<T>::v4 row4(gptr<T> A, uint32_t row, int k0,
                                                   int n) {
  typedef typename Vec<T>::v4 V;
  const int kb = k0 - 1 < 0 ? 0 : (k0 - 1 > n - 4 ? n - 4 : k0 - 1);
  V r = *(gptr<V>)(A + row + (uint32_t)kb);
  if (kb != k0 - 1) {
    const T x = r.x, y = r.y, z = r.z, w = r.w;
    r.x = pick4<T>(x, y, z, w, clampi(k0 - 1, n) - kb);
    r.y = pick4<T>(x, y, z, w, clampi(k0, n) - kb);
    r.z = pick4<T>(x, y, z, w, clampi(k0 + 1, n) - kb);
    r.w = pick4<T>(x, y, z, w, clampi(k0 + 2, n) - kb);
  }
  return r;
}

// Tensor WENO (Section 3.2): one-dimensional WENO along the last axis
// first, then along the previous axes, x last.  R supplies the rows of four
// values along z (stencil indices clamped to the grid): from device memory or
// from a staged copy in LDS; the arithmetic is the same either way.
template <typename T, typename R>
__device__ __forceinline__ T interp_weno3(const R& rows, const Loc<T>& lx, const Loc<T>& ly,
                                          const Loc<T>& lz, T e) {
  const WC<T> cx = wcoef(lx.t), cy = wcoef(ly.t), cz = wcoef(lz.t);
  T wx[4];
  LSR_UNROLL(LSR_WENO_X_UNROLL)
  for (int a = 0; a < 4; ++a) {
    T wy[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      typename Vec<T>::v4 r = rows.w4(lx.i0 - 1 + a, ly.i0 - 1 + b, lz.i0);
      wy[b] = weno1(r.x, r.y, r.z, r.w, cz, e);
    }
    wx[a] = weno1(wy[0], wy[1], wy[2], wy[3], cy, e);
  }
  return weno1(wx[0], wx[1], wx[2], wx[3], cx, e);
}

template <typename T>
__device__ __forceinline__ T interp_weno2(gptr<T> A, const DevGrid& g,
                                          const Loc<T>& lx, const Loc<T>& ly, T e) {
  const WC<T> cx = wcoef(lx.t), cy = wcoef(ly.t);
  T wx[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const uint32_t row = (uint32_t)clampi(lx.i0 - 1 + a, g.n0) * g.s0;
    typename Vec<T>::v4 r = row4(A, row, ly.i0, g.n1);
    wx[a] = weno1(r.x, r.y, r.z, r.w, cy, e);
  }
  return weno1(wx[0], wx[1], wx[2], wx[3], cx, e);
}

// Multilinear interpolation, eq. (IQ1).
template <typename T, typename R>
__device__ __forceinline__ T interp_q1_3(const R& rows, const Loc<T>& lx, const Loc<T>& ly,
                                         const Loc<T>& lz) {
  typedef typename Vec<T>::v2 V2;
  V2 a00 = rows.w2(lx.i0, ly.i0, lz.i0);
  V2 a01 = rows.w2(lx.i0, ly.i0 + 1, lz.i0);
  V2 a10 = rows.w2(lx.i0 + 1, ly.i0, lz.i0);
  V2 a11 = rows.w2(lx.i0 + 1, ly.i0 + 1, lz.i0);
  T tz = lz.t, ty = ly.t, tx = lx.t;
  T b00 = fma(tz, a00.y - a00.x, a00.x);
  T b01 = fma(tz, a01.y - a01.x, a01.x);
  T b10 = fma(tz, a10.y - a10.x, a10.x);
  T b11 = fma(tz, a11.y - a11.x, a11.x);
  T c0 = fma(ty, b01 - b00, b00);
  T c1 = fma(ty, b11 - b10, b10);
  return fma(tx, c1 - c0, c0);
}

template <typename T>
__device__ __forceinline__ T interp_q1_2(gptr<T> A, const DevGrid& g,
                                         const Loc<T>& lx, const Loc<T>& ly) {
  typedef typename Vec<T>::v2 V2;
  const uint32_t r0 = (uint32_t)lx.i0 * g.s0 + (uint32_t)ly.i0;
  V2 a0 = *(gptr<V2>)(A + r0);
  V2 a1 = *(gptr<V2>)(A + r0 + g.s0);
  T b0 = fma(ly.t, a0.y - a0.x, a0.x);
  T b1 = fma(ly.t, a1.y - a1.x, a1.x);
  return fma(lx.t, b1 - b0, b0);
}

enum { UPD_FALLBACK = 1, UPD_FRAME0 = 2 };

// Rows of phi^n read from device memory (3D): four values along z at
// k0-1 .. k0+2 of row (ii, jj), or two at k0, k0+1; indices clamped.
template <typename T>
struct GlobalRows {
  gptr<T> A;
  int n0, n1, n2;
  uint32_t s0, s1;
  __device__ __forceinline__ typename Vec<T>::v4 w4(int ii, int jj, int k0) const {
    return row4(A, (uint32_t)clampi(ii, n0) * s0 + (uint32_t)clampi(jj, n1) * s1, k0, n2);
  }
  __device__ __forceinline__ typename Vec<T>::v2 w2(int ii, int jj, int k0) const {
    return *(gptr<typename Vec<T>::v2>)(A + (uint32_t)ii * s0 + (uint32_t)jj * s1 + (uint32_t)k0);
  }
};

// phi^n as the node update reads it, from device memory: neighbours of the
// node, and the interpolant at a located foot point.
template <int DIM, int INTERP, typename T>
struct GlobalSrc {
  gptr<T> A;
  const DevGrid& g;
  T e;
  // neighbour (di, dj, dk) of node idx if `inside` (on the grid), else the node
  __device__ __forceinline__ T nb(uint32_t idx, bool inside, int di, int dj, int dk) const {
    return A[inside ? idx + (uint32_t)(di * (int)g.s0 + dj * (int)g.s1 + dk) : idx];
  }
  __device__ __forceinline__ T foot3(const Loc<T>& lx, const Loc<T>& ly, const Loc<T>& lz) const {
    const GlobalRows<T> r{A, g.n0, g.n1, g.n2, g.s0, g.s1};
    return INTERP == 0 ? interp_q1_3(r, lx, ly, lz) : interp_weno3(r, lx, ly, lz, e);
  }
  __device__ __forceinline__ T foot2(const Loc<T>& lx, const Loc<T>& ly) const {
    return INTERP == 0 ? interp_q1_2(A, g, lx, ly) : interp_weno2(A, g, lx, ly, e);
  }
};

// New value of band node (i,j,k) from phi^n (read through S): eqs.
// (SL2d)/(SL3d) with C = c(phi^n_j) (p = 1), the fallback of eq. (SL:2) and
// the cut of eq. (cut).  dp = (d_x, d_y, d_z, d) with the centred gradient of
// d precomputed.  Foot points are carried as node index + offset in cells.
//
// LANES = 1: one lane interpolates all foot points of the node.  LANES = 2
// (2D) or 4 (3D): the node is handled by a group of LANES consecutive lanes,
// lane `sub` interpolating foot point `sub`, and the group sums its values
// with two cross-lane exchanges.  Both ways add the foot values as
// (v0 + v1) + (v2 + v3), so they give bitwise identical results.
template <int DIM, typename T, typename S>
__device__ __forceinline__ T foot_value(const S& src, const DevGrid& g, int i, int j, int k, int q,
                                        T bx, T by, T bz, T n1x, T n1y, T n1z, T n2x, T n2y,
                                        T n2z) {
  if (DIM == 2) {
    const T l = (q & 1) ? T(1) : T(-1);
    Loc<T> lx = locate(i, bx + n1x * l, g.n0);
    Loc<T> ly = locate(j, by + n1y * l, g.n1);
    return src.foot2(lx, ly);
  }
  const T f1 = (q & 2) ? T(1) : T(-1), f2 = (q & 1) ? T(1) : T(-1);
  Loc<T> lx = locate(i, bx + f1 * n1x + f2 * n2x, g.n0);
  Loc<T> ly = locate(j, by + f1 * n1y + f2 * n2y, g.n1);
  Loc<T> lz = locate(k, bz + f1 * n1z + f2 * n2z, g.n2);
  return src.foot3(lx, ly, lz);
}

template <int DIM, typename T, int LANES, typename S>
__device__ __forceinline__ T sl_update_src(const S& src, const DevGrid& g, const StepConst<T>& c,
                                           int i, int j, int k, uint32_t idx, T v,
                                           typename Vec<T>::p4 dp, int sub, int& flags) {
  constexpr int FP = DIM == 3 ? 4 : 2;  // foot points per node
  T gx, gy, gz = T(0);
  // neighbours off the grid read the node itself (the value v)
  T xm = src.nb(idx, i > 0, -1, 0, 0), xp = src.nb(idx, i < g.n0 - 1, 1, 0, 0);
  T ym = src.nb(idx, j > 0, 0, -1, 0), yp = src.nb(idx, j < g.n1 - 1, 0, 1, 0);
  T zm = v, zp = v;
  if (DIM == 3) {
    zm = src.nb(idx, k > 0, 0, 0, -1);
    zp = src.nb(idx, k < g.n2 - 1, 0, 0, 1);
  }
  gx = cdiff(xm, v, xp, i, g.n0, c);
  gy = cdiff(ym, v, yp, j, g.n1, c);
  if (DIM == 3) gz = cdiff(zm, v, zp, k, g.n2, c);
  T nrm = sqrt(gx * gx + gy * gy + gz * gz);
  T out;
  if (nrm < c.grad_thr) {
    T sum = T(0), cnt = T(0);
    if (i > 0) { sum += xm; cnt += T(1); }
    if (i < g.n0 - 1) { sum += xp; cnt += T(1); }
    if (j > 0) { sum += ym; cnt += T(1); }
    if (j < g.n1 - 1) { sum += yp; cnt += T(1); }
    if (DIM == 3) {
      if (k > 0) { sum += zm; cnt += T(1); }
      if (k < g.n2 - 1) { sum += zp; cnt += T(1); }
    }
    out = sum / cnt;
    flags |= UPD_FALLBACK;
  } else {
    // C = c(phi) [d / E_p]^(p - 1), eqs. (SL2d)/(SL3d), p = 1 or 2
    T C = cutoff(v, c);
    if (c.pm1 != T(0)) C *= dp.w * c.inv_E;
    const T amp = sqrt(C * dp.w * c.diff2);  // diffusion reach in cells
    const T cd = C * c.drift;
    const T bx = cd * dp.x, by = cd * dp.y, bz = DIM == 3 ? cd * dp.z : T(0);
    T n1x, n1y, n1z = T(0), n2x = T(0), n2y = T(0), n2z = T(0);
    if (DIM == 2) {
      const T inv = T(1) / nrm;
      n1x = gy * inv * amp;  // eq. (sigma2d), scaled
      n1y = -gx * inv * amp;
    } else {
      const T s2 = gx * gx + gz * gz;
      if (s2 != T(0)) {  // eq. (sigma3d)
        const T s = sqrt(s2);
        const T is = T(1) / s;
        const T isn = is / nrm;
        n1x = -gz * is; n1y = T(0); n1z = gx * is;
        n2x = -gx * gy * isn; n2y = s / nrm; n2z = -gy * gz * isn;
      } else {
        n1x = T(1); n1y = T(0); n1z = T(0);
        n2x = T(0); n2y = T(0); n2z = T(1);
        flags |= UPD_FRAME0;
      }
      n1x *= amp; n1y *= amp; n1z *= amp;
      n2x *= amp; n2y *= amp; n2z *= amp;
    }
    T acc;
    if (LANES == 1) {
      T prev = T(0), s01 = T(0), s23 = T(0);
      LSR_UNROLL(LSR_FOOT_UNROLL)
      for (int q = 0; q < FP; ++q) {
        const T vq = foot_value<DIM, T>(src, g, i, j, k, q, bx, by, bz, n1x, n1y, n1z, n2x, n2y,
                                        n2z);
        if (q & 1) {
          if (q == 1) s01 = prev + vq;
          else s23 = prev + vq;
        } else {
          prev = vq;
        }
      }
      acc = FP == 4 ? s01 + s23 : s01;
    } else {
      const T vq = foot_value<DIM, T>(src, g, i, j, k, sub, bx, by, bz, n1x, n1y, n1z, n2x, n2y,
                                      n2z);
      acc = vq + __shfl_xor(vq, 1, LANES);
      if (FP == 4) acc = acc + __shfl_xor(acc, 2, LANES);
    }
    out = acc * (T(1) / T(FP));
  }
  return fmin(fmax(out, -c.gamma), c.gamma);
}

// The update reading phi^n from device memory.
template <int DIM, int INTERP, typename T, int LANES>
__device__ __forceinline__ T sl_update(gptr<T> A, const DevGrid& g, const StepConst<T>& c, int i,
                                       int j, int k, uint32_t idx, T v, typename Vec<T>::p4 dp,
                                       int sub, int& flags) {
  const GlobalSrc<DIM, INTERP, T> src{A, g, c.weno_e};
  return sl_update_src<DIM, T, LANES>(src, g, c, i, j, k, idx, v, dp, sub, flags);
}

}  // namespace lsr
