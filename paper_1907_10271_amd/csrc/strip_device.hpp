// Device building blocks of the strip model (Section 3.1 of the paper):
// rotated ply stiffness at a Gauss point and the bilinear element operator
// with 2x2 Gauss quadrature, written for uniform rectangles.
#pragma once

#include "common.hpp"

namespace mlmc {

// rotated plane-stress stiffness at one Gauss point (global axes, engineering shear)
template <typename T>
struct QbT {
  T q11, q22, q12, q66, q16, q26;
};
using Qb = QbT<double>;

// sin and cos from their Taylor series (Horner in x^2): for |x| <= 1 the first
// omitted terms are below x^19/19! < 1e-17 and x^20/20! < 1e-18, so the result
// is within a few ulp.
// Loads and stores through the global address space.  Generic (flat) accesses
// also count against the LDS/scalar counter, so the wait for a lane shuffle or
// a work-group sum would also wait for every row prefetch still in flight.
#define MLMC_GLOBAL __attribute__((address_space(1)))
// clang vector types for the accesses (HIP's vector structs copy through a
// generic reference, which would turn the access back into a flat one)
template <typename V>
struct NativeOf;
template <>
struct NativeOf<double2> {
  typedef double type __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ double2 from(type n) { return make_double2(n.x, n.y); }
  static __device__ __forceinline__ type to(const double2 &v) { return type{v.x, v.y}; }
};
template <>
struct NativeOf<float2> {
  typedef float type __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ float2 from(type n) { return make_float2(n.x, n.y); }
  static __device__ __forceinline__ type to(const float2 &v) { return type{v.x, v.y}; }
};
template <>
struct NativeOf<float4> {
  typedef float type __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ float4 from(type n) { return make_float4(n.x, n.y, n.z, n.w); }
};
template <>
struct NativeOf<double> {
  typedef double type;
  static __device__ __forceinline__ double from(type n) { return n; }
  static __device__ __forceinline__ type to(double v) { return v; }
};
template <>
struct NativeOf<uint4> {
  typedef unsigned int type __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ uint4 from(type n) { return make_uint4(n.x, n.y, n.z, n.w); }
};
template <>
struct NativeOf<uint2> {
  typedef unsigned int type __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ uint2 from(type n) { return make_uint2(n.x, n.y); }
};
template <typename V>
__device__ __forceinline__ V gload(const void *p) {
  return NativeOf<V>::from(*(const MLMC_GLOBAL typename NativeOf<V>::type *)p);
}
template <typename V>
__device__ __forceinline__ void gstore(void *p, const V &v) {
  *(MLMC_GLOBAL typename NativeOf<V>::type *)p = NativeOf<V>::to(v);
}

__device__ __forceinline__ void sincos_poly(double x, double *s, double *c) {
  const double z = x * x;
  double ps = -1.0 / 355687428096000.0;  // -1/17!
  ps = fma(ps, z, 1.0 / 1307674368000.0);
  ps = fma(ps, z, -1.0 / 6227020800.0);
  ps = fma(ps, z, 1.0 / 39916800.0);
  ps = fma(ps, z, -1.0 / 362880.0);
  ps = fma(ps, z, 1.0 / 5040.0);
  ps = fma(ps, z, -1.0 / 120.0);
  ps = fma(ps, z, 1.0 / 6.0);
  *s = fma(-x * z, ps, x);               // x - x^3/3! + ...
  double pc = 1.0 / 6402373705728000.0;  // 1/18!
  pc = fma(pc, z, -1.0 / 20922789888000.0);
  pc = fma(pc, z, 1.0 / 87178291200.0);
  pc = fma(pc, z, -1.0 / 479001600.0);
  pc = fma(pc, z, 1.0 / 3628800.0);
  pc = fma(pc, z, -1.0 / 40320.0);
  pc = fma(pc, z, 1.0 / 720.0);
  pc = fma(pc, z, -1.0 / 24.0);
  pc = fma(pc, z, 0.5);
  *c = fma(-z, pc, 1.0);                 // 1 - x^2/2! + ...
}

// sin and cos of any angle: |x| <= 1 directly; otherwise Cody-Waite reduction
// by pi/2 (pi/2 split into three doubles, subtracted with FMA) to |r| <= pi/4
// and the quadrant's sign and swap.  Accurate while k pi/2 is well inside the
// double range of exact integers (|x| up to ~1e9); non-finite x gives NaN.
__device__ __forceinline__ void sincos_small(double x, double *s, double *c) {
  if (fabs(x) <= 1.0) {
    sincos_poly(x, s, c);
    return;
  }
  constexpr double TWO_OVER_PI = 0.6366197723675814;
  constexpr double P1 = 1.5707963267948966, P2 = 6.123233995736766e-17, P3 = -1.4973849048591698e-33;
  const double k = rint(x * TWO_OVER_PI);
  double r = fma(-k, P1, x);
  r = fma(-k, P2, r);
  r = fma(-k, P3, r);
  double sr, cr;
  sincos_poly(r, &sr, &cr);
  const long long qk = isfinite(k) ? (long long)fmod(k, 4.0) : 0;
  const int q = (int)(qk & 3);
  const double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// 1/d from the hardware reciprocal and Newton steps (two for FP64, one for
// FP32: each doubles the correct bits of the estimate)
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  return fma(fma(-d, r, 1.0), r, r);
}
__device__ __forceinline__ float rcp_nr(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return fmaf(fmaf(-d, r, 1.0f), r, r);
}

// Angles are kept by the solver as their tangent t = tan theta (clamped to
// +-1e150, so that t^2 stays finite; for every double angle |cos theta| is far
// above 1e-150; NaN stays NaN).  The rotation then needs no trigonometric series and no
// stored constants:
//   cos 2theta = (1 - t^2) / (1 + t^2),  sin 2theta = 2 t / (1 + t^2),
// with 1/(1 + t^2) from the hardware reciprocal and two Newton steps (each
// doubles the number of correct bits of the initial estimate).
__device__ __forceinline__ double angle_code(double th) {
  double s, c;
  sincos_small(th, &s, &c);
  const double t = s / c;
  return fabs(t) > 1e150 ? copysign(1e150, t) : t;  // a NaN angle stays NaN
}
__device__ __forceinline__ void cs_of_code(double t, double *s2, double *c2) {
  const double r = rcp_nr(fma(t, t, 1.0));
  *c2 = fma(-t, t, 1.0) * r;
  *s2 = (t + t) * r;
}
// (cos 2theta, sin 2theta) of an angle, through its code (every path of the
// library evaluates the rotation this way, so they agree bit for bit)
__device__ __forceinline__ void cs_of_angle(double th, double *s2, double *c2) { cs_of_code(angle_code(th), s2, c2); }

// Qbar from c2 = cos 2theta and s2 = sin 2theta (rotation invariants: the
// fibre axes are turned by +theta from x; entries are linear in cos 2theta,
// sin 2theta, cos 4theta, sin 4theta)
__device__ __forceinline__ Qb qbar_cs(const StripMat &m, double s2, double c2) {
  const double c4 = 2.0 * c2 * c2 - 1.0;
  const double s4 = 2.0 * s2 * c2;
  Qb q;
  q.q11 = m.U1 + m.U2 * c2 + m.U3 * c4;
  q.q22 = m.U1 - m.U2 * c2 + m.U3 * c4;
  q.q12 = m.U4 - m.U3 * c4;
  q.q66 = m.U5 - m.U3 * c4;
  const double h = 0.5 * m.U2 * s2;
  q.q16 = h + m.U3 * s4;
  q.q26 = h - m.U3 * s4;
  return q;
}

// Qbar(theta): the same from the angle itself
__device__ __forceinline__ Qb qbar_of(const StripMat &m, double th) {
  double s2, c2;
  cs_of_angle(th, &s2, &c2);
  const double c4 = 2.0 * c2 * c2 - 1.0;
  const double s4 = 2.0 * s2 * c2;
  Qb q;
  q.q11 = m.U1 + m.U2 * c2 + m.U3 * c4;
  q.q22 = m.U1 - m.U2 * c2 + m.U3 * c4;
  q.q12 = m.U4 - m.U3 * c4;
  q.q66 = m.U5 - m.U3 * c4;
  const double h = 0.5 * m.U2 * s2;
  q.q16 = h + m.U3 * s4;
  q.q26 = h - m.U3 * s4;
  return q;
}

// (cos 2theta, sin 2theta) at the four Gauss points of element e (index within
// the sample's data `ang`), read as stored pairs (cs != 0) or evaluated from
// the stored angle codes
__device__ __forceinline__ void elem_cs(const double *__restrict__ ang, int cs, size_t e, double2 out[4]) {
  if (cs) {
    const double2 *cp = reinterpret_cast<const double2 *>(ang) + 4 * e;
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = gload<double2>(cp + q);
  } else {
    const double2 a = gload<double2>(ang + 4 * e);
    const double2 b = gload<double2>(ang + 4 * e + 2);
    const double t[4] = {a.x, a.y, b.x, b.y};
#pragma unroll
    for (int q = 0; q < 4; ++q) cs_of_code(t[q], &out[q].y, &out[q].x);
  }
}

// Element forces f = sum_q w_q detJ B_q^T Qbar_q B_q d_e for one bilinear
// rectangle.  Nodes are numbered counter-clockwise from the lower-left
// corner; Gauss point q has xi index (q & 1) and eta index (q >> 1), low = -1/sqrt3.
//
// With edge differences du_b = u1 - u0, du_t = u2 - u3, du_l = u3 - u0,
// du_r = u2 - u1 the derivatives at the Gauss points are
//   du/dx = (P du_b + M du_t)/hx at eta = -g,  (M du_b + P du_t)/hx at eta = +g,
//   du/dy = (P du_l + M du_r)/hy at xi  = -g,  (M du_l + P du_r)/hy at xi  = +g,
// (P, M the interpolation weights of the Gauss abscissae), so every
// derivative is shared by two Gauss points; the transposed operator uses the
// same pairs.  Gauss points are processed one at a time so only one rotated
// stiffness is live.  QB(q) must yield the Qb of Gauss point q.
template <typename T, class QbAt>
__device__ __forceinline__ void elem_forces_q(const StripGeom &g, QbAt QB, const T u[4], const T v[4], T fu[4],
                                              T fv[4]) {
  const T pxi = (T)g.pxi, mxi = (T)g.mxi, pyi = (T)g.pyi, myi = (T)g.myi;
  const T pxw = (T)g.pxw, mxw = (T)g.mxw, pyw = (T)g.pyw, myw = (T)g.myw;
  const T dub = u[1] - u[0], dut = u[2] - u[3], dul = u[3] - u[0], dur = u[2] - u[1];
  const T dvb = v[1] - v[0], dvt = v[2] - v[3], dvl = v[3] - v[0], dvr = v[2] - v[1];
  const T ux[2] = {fma(pxi, dub, mxi * dut), fma(mxi, dub, pxi * dut)};
  const T vx[2] = {fma(pxi, dvb, mxi * dvt), fma(mxi, dvb, pxi * dvt)};
  const T uy[2] = {fma(pyi, dul, myi * dur), fma(myi, dul, pyi * dur)};
  const T vy[2] = {fma(pyi, dvl, myi * dvr), fma(myi, dvl, pyi * dvr)};
  // stress sums: sxx and txy paired by eta (x-derivative), syy and txy paired by xi
  T ax[2], ay[2], aty[2], atx[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = q & 1, b = q >> 1;
    const QbT<T> qb = QB(q);
    const T ex = ux[b], ey = vy[a], gm = uy[a] + vx[b];
    const T sxx = qb.q11 * ex + qb.q12 * ey + qb.q16 * gm;
    const T syy = qb.q12 * ex + qb.q22 * ey + qb.q26 * gm;
    const T txy = qb.q16 * ex + qb.q26 * ey + qb.q66 * gm;
    if (q == 0) {
      ax[0] = sxx; ay[0] = syy; aty[0] = txy; atx[0] = txy;
    } else if (q == 1) {
      ax[0] += sxx; ay[1] = syy; aty[1] = txy; atx[0] += txy;
    } else if (q == 2) {
      ax[1] = sxx; ay[0] += syy; aty[0] += txy; atx[1] = txy;
    } else {
      ax[1] += sxx; ay[1] += syy; aty[1] += txy; atx[1] += txy;
    }
  }
  // transposed derivative operators with the quadrature weight folded in
  const T gub = fma(pxw, ax[0], mxw * ax[1]), gut = fma(mxw, ax[0], pxw * ax[1]);
  const T gul = fma(pyw, aty[0], myw * aty[1]), gur = fma(myw, aty[0], pyw * aty[1]);
  const T gvl = fma(pyw, ay[0], myw * ay[1]), gvr = fma(myw, ay[0], pyw * ay[1]);
  const T gvb = fma(pxw, atx[0], mxw * atx[1]), gvt = fma(mxw, atx[0], pxw * atx[1]);
  fu[0] = -gub - gul;
  fu[1] = gub - gur;
  fu[2] = gut + gur;
  fu[3] = -gut + gul;
  fv[0] = -gvb - gvl;
  fv[1] = gvb - gvr;
  fv[2] = gvt + gvr;
  fv[3] = -gvt + gvl;
}

__device__ __forceinline__ void elem_forces(const StripGeom &g, const Qb q[4], const double u[4],
                                            const double v[4], double fu[4], double fv[4]) {
  elem_forces_q<double>(g, [&](int k) { return q[k]; }, u, v, fu, fv);
}

// FP32 rotated stiffness from a bfloat16 angle (mixed-precision inner operator)
__device__ __forceinline__ QbT<float> qbar_f32(const StripMat &m, float th) {
  float s2, c2;
  __sincosf(2.0f * th, &s2, &c2);
  const float c4 = 2.0f * c2 * c2 - 1.0f;
  const float s4 = 2.0f * s2 * c2;
  QbT<float> q;
  q.q11 = m.fU1 + m.fU2 * c2 + m.fU3 * c4;
  q.q22 = m.fU1 - m.fU2 * c2 + m.fU3 * c4;
  q.q12 = m.fU4 - m.fU3 * c4;
  q.q66 = m.fU5 - m.fU3 * c4;
  const float h = 0.5f * m.fU2 * s2;
  q.q16 = h + m.fU3 * s4;
  q.q26 = h - m.fU3 * s4;
  return q;
}

__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// largest compressive stress along the fibres at the four Gauss points:
// sigma_11 = cos^2 sxx + sin^2 syy + 2 sin cos txy, written with cos 2theta, sin 2theta
// cs[2q], cs[2q + 1] = cos 2theta, sin 2theta at Gauss point q
__device__ __forceinline__ double elem_max_fibre_compression(const StripGeom &g, const StripMat &m,
                                                             const double cs[8], const double u[4],
                                                             const double v[4]) {
  const double P = GP_P, M = GP_M;
  const double dub = u[1] - u[0], dut = u[2] - u[3], dul = u[3] - u[0], dur = u[2] - u[1];
  const double dvb = v[1] - v[0], dvt = v[2] - v[3], dvl = v[3] - v[0], dvr = v[2] - v[1];
  const double ux[2] = {(P * dub + M * dut) * g.ihx, (M * dub + P * dut) * g.ihx};
  const double vx[2] = {(P * dvb + M * dvt) * g.ihx, (M * dvb + P * dvt) * g.ihx};
  const double uy[2] = {(P * dul + M * dur) * g.ihy, (M * dul + P * dur) * g.ihy};
  const double vy[2] = {(P * dvl + M * dvr) * g.ihy, (M * dvl + P * dvr) * g.ihy};
  double best = -1.0 / 0.0;
  for (int q = 0; q < 4; ++q) {
    const int a = q & 1, b = q >> 1;
    double s2, c2;
    c2 = cs[2 * q];
    s2 = cs[2 * q + 1];
    const double c4 = 2.0 * c2 * c2 - 1.0, s4 = 2.0 * s2 * c2;
    const double q11 = m.U1 + m.U2 * c2 + m.U3 * c4, q22 = m.U1 - m.U2 * c2 + m.U3 * c4;
    const double q12 = m.U4 - m.U3 * c4, q66 = m.U5 - m.U3 * c4;
    const double q16 = 0.5 * m.U2 * s2 + m.U3 * s4, q26 = 0.5 * m.U2 * s2 - m.U3 * s4;
    const double ex = ux[b], ey = vy[a], gm = uy[a] + vx[b];
    const double sxx = q11 * ex + q12 * ey + q16 * gm;
    const double syy = q12 * ex + q22 * ey + q26 * gm;
    const double txy = q16 * ex + q26 * ey + q66 * gm;
    const double s11 = 0.5 * ((1.0 + c2) * sxx + (1.0 - c2) * syy) + s2 * txy;
    best = fmax(best, -s11);
  }
  return best;
}

// ---------------------------------------------------------------- reductions
// Fixed-order work-group sum (256 threads): butterfly within each wave of 64,
// then the four wave sums in order.  Every thread returns the total.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block of `waves` waves (blockDim = 64 * waves, waves <= 8): wave sums, then in order
__device__ __forceinline__ double block_sum_w(double v, double *red, int waves) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < waves; ++w) t += red[w];
  return t;
}

__device__ __forceinline__ double block_sum(double v, double *red4) { return block_sum_w(v, red4, 4); }

// sum of n values in fixed order: thread t adds entries t, t+256, ... then block_sum
__device__ __forceinline__ double block_sum_strided(const double *a, int n, double *red4) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += a[k];
  return block_sum(s, red4);
}

// sum in a fixed order for TILE_THREADS-wide blocks
__device__ __forceinline__ double tile_sum(double v, double *red) { return block_sum_w(v, red, TILE_WAVES); }

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double block_max(double v, double *red4) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red4[wid] = v;
  __syncthreads();
  return fmax(fmax(red4[0], red4[1]), fmax(red4[2], red4[3]));
}

}  // namespace mlmc
