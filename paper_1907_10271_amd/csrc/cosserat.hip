// Cosserat continuum model of Test Problem I (Section 3.1 of the paper) on the
// GPU: three unknowns (u, v, theta_3) per node of a uniform bilinear mesh,
// Cosserat strains eps_ij = du_i/dx_j + e_ij3 theta_3 and curvatures
// kappa_j = d theta_3 / dx_j, stresses from the fibre-frame matrices C (4 x 4
// on (11, 22, 12, 21)) and D (2 x 2) rotated by the local fibre angle
// (C* = T^-1 C T, D* = R^-1 D R, with T and R orthogonal), 2x2 Gauss
// quadrature (Eq. VarCosserat, Eq. matrixinplane).
//
// Every kernel works on 16 x 16 node tiles, one owned node per thread: the
// input vector is staged with a one-node halo in LDS, the 17 x 17 elements
// touching the tile compute their nodal forces into LDS, and each node sums
// its four elements' contributions in a fixed order.  The PCG iteration is
// two launches (operator pass with the fused search-direction update, and a
// pointwise vector pass), with per-tile partial sums reduced in a fixed order
// by every work-group that needs them, so a sample's result does not depend
// on the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.hpp"
#include "cosserat.hpp"
#include "kl_setup.hpp"
#include "strip_device.hpp"
#include "strip_kernels.hpp"

namespace mlmc {
namespace {

constexpr int CT = 16;               // node tile side: one owned node per thread
constexpr int CH = CT + 2;           // tile with a one-node halo
constexpr int CE = CT + 1;           // elements touching the owned nodes
constexpr int CTHREADS = CT * CT;    // 256
constexpr int CBLOCK = 32;           // PCG iterations between checks of the host
constexpr int MAXKL = 1024;          // largest number of KL terms

struct CosGeom {
  int nx, ny, nnx, nny, nnode, nelem;
  int tx, ty, ntiles;         // node tiles
  int qx0, qx1, qy0, qy1;     // elements of the QoI square [qx0, qx1) x [qy0, qy1)
  int nkl;                    // KL terms of this level
  double hx, hy, delta;       // u = delta on x = L
};

struct CosMat {
  double C11, C12, C22, Gp, Go;   // fibre frame: (11, 22) block, shear parallel / orthogonal to the fibres
  double D1, D2;                  // couple-stress moduli along / across the fibres
  double R, tau_y;                // failure criterion
};

// per-slot solver state of a level pool (device pointers, slot stride S)
struct CosSlots {
  double *x, *r, *p0, *p1, *Ap, *dinv;  // [S][3 nnode]
  double *cs;                           // [S][nelem][4][2] (cos 2phi, sin 2phi) per Gauss point
  double *part_pap;                     // [S][ntiles]
  double *part_rz, *part_rr;            // [2][S][ntiles]
  double *bb, *relres;                  // [S]
  int *iters, *status, *active;         // [S]
  int S, max_iter;
  double rtol2;
};

__device__ __forceinline__ bool cos_constrained(const CosGeom &g, int i, int j, int c) {
  if (c == 0) return i == 0 || i == g.nx;
  if (c == 1) return j == 0 || j == g.ny;
  return false;
}

// interpolation weights and scaled derivatives of the four element nodes
// (counter-clockwise from the lower-left) at Gauss point q of the order
// (-,-), (+,-), (-,+), (+,+)
struct GpShape {
  double N[4], dx[4], dy[4];
};

__device__ __forceinline__ GpShape gp_shape(const CosGeom &g, int q) {
  const double fx = (q & 1) ? GP_P : GP_M, fy = (q & 2) ? GP_P : GP_M;
  const double wx0 = 1.0 - fx, wx1 = fx, wy0 = 1.0 - fy, wy1 = fy;
  const double ihx = 1.0 / g.hx, ihy = 1.0 / g.hy;
  GpShape s;
  s.N[0] = wx0 * wy0;
  s.N[1] = wx1 * wy0;
  s.N[2] = wx1 * wy1;
  s.N[3] = wx0 * wy1;
  s.dx[0] = -wy0 * ihx;
  s.dx[1] = wy0 * ihx;
  s.dx[2] = wy1 * ihx;
  s.dx[3] = -wy1 * ihx;
  s.dy[0] = -wx0 * ihy;
  s.dy[1] = -wx1 * ihy;
  s.dy[2] = wx1 * ihy;
  s.dy[3] = wx0 * ihy;
  return s;
}

// stresses at one Gauss point: global (s11, s22, s12, s21), fibre-frame
// (t22, t12) and couple stresses (m1, m2)
struct GpStress {
  double s11, s22, s12, s21, t22, t12, m1, m2;
};

__device__ __forceinline__ GpStress gp_stress(const CosMat &m, const GpShape &sh, double c2, double s2,
                                              const double ue[4], const double ve[4], const double te[4]) {
  double e11 = 0.0, e22 = 0.0, uy = 0.0, vx = 0.0, th = 0.0, k1 = 0.0, k2 = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    e11 += sh.dx[a] * ue[a];
    e22 += sh.dy[a] * ve[a];
    uy += sh.dy[a] * ue[a];
    vx += sh.dx[a] * ve[a];
    th += sh.N[a] * te[a];
    k1 += sh.dx[a] * te[a];
    k2 += sh.dy[a] * te[a];
  }
  const double e12 = uy + th, e21 = vx - th;
  // cos^2, sin^2 and cos sin of the fibre angle
  const double cc = 0.5 * (1.0 + c2), ss = 0.5 * (1.0 - c2), sc = 0.5 * s2;
  // fibre-frame strains eps' = R eps R^T
  const double esum = e12 + e21, ed = sc * (e22 - e11);
  const double l11 = cc * e11 + ss * e22 + sc * esum;
  const double l22 = ss * e11 + cc * e22 - sc * esum;
  const double l12 = ed + cc * e12 - ss * e21;
  const double l21 = ed - ss * e12 + cc * e21;
  GpStress o;
  const double t11 = m.C11 * l11 + m.C12 * l22;
  o.t22 = m.C12 * l11 + m.C22 * l22;
  o.t12 = m.Gp * l12;
  const double t21 = m.Go * l21;
  // back to global axes, sigma = R^T sigma' R
  const double tsum = o.t12 + t21, td = sc * (t11 - o.t22);
  o.s11 = cc * t11 + ss * o.t22 - sc * tsum;
  o.s22 = ss * t11 + cc * o.t22 + sc * tsum;
  o.s12 = td + cc * o.t12 - ss * t21;
  o.s21 = td - ss * o.t12 + cc * t21;
  // couple stresses m = R^T D R kappa
  const double dm = sc * (m.D1 - m.D2);
  o.m1 = (cc * m.D1 + ss * m.D2) * k1 + dm * k2;
  o.m2 = dm * k1 + (ss * m.D1 + cc * m.D2) * k2;
  return o;
}

// nodal forces K_e d_e of one element (unknowns of its four nodes) for the
// (cos 2phi, sin 2phi) of its Gauss points
__device__ __forceinline__ void elem_forces(const CosGeom &g, const CosMat &m, const double cs[8], const double ue[4],
                                            const double ve[4], const double te[4], double fu[4], double fv[4],
                                            double ft[4]) {
  const double w = 0.25 * g.hx * g.hy;
#pragma unroll
  for (int a = 0; a < 4; ++a) fu[a] = fv[a] = ft[a] = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const GpShape sh = gp_shape(g, q);
    const GpStress st = gp_stress(m, sh, cs[2 * q], cs[2 * q + 1], ue, ve, te);
    const double sa = st.s12 - st.s21;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      fu[a] += w * (sh.dx[a] * st.s11 + sh.dy[a] * st.s12);
      fv[a] += w * (sh.dy[a] * st.s22 + sh.dx[a] * st.s21);
      ft[a] += w * (sh.N[a] * sa + sh.dx[a] * st.m1 + sh.dy[a] * st.m2);
    }
  }
}

__device__ __forceinline__ void load_cs(const double *cs_e, double cs[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 v = *reinterpret_cast<const double2 *>(cs_e + 2 * k);
    cs[2 * k] = v.x;
    cs[2 * k + 1] = v.y;
  }
}

// forces of the elements touching the tile with origin (i0, j0), from the
// halo node values xs, into fe[12][CE * CE] (zero for elements off the mesh)
__device__ void tile_forces(const CosGeom &g, const CosMat &m, const double *cs_s, int i0, int j0,
                            double (*xs)[CH * CH], double (*fe)[CE * CE]) {
  for (int k = threadIdx.x; k < CE * CE; k += CTHREADS) {
    const int le = k % CE, me = k / CE;
    const int ex = i0 - 1 + le, ey = j0 - 1 + me;
    double fu[4] = {0, 0, 0, 0}, fv[4] = {0, 0, 0, 0}, ft[4] = {0, 0, 0, 0};
    if (ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny) {
      const int h0 = me * CH + le;
      const int hn[4] = {h0, h0 + 1, h0 + CH + 1, h0 + CH};
      double ue[4], ve[4], te[4], cs[8];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        ue[a] = xs[0][hn[a]];
        ve[a] = xs[1][hn[a]];
        te[a] = xs[2][hn[a]];
      }
      load_cs(cs_s + 8 * ((size_t)ey * g.nx + ex), cs);
      elem_forces(g, m, cs, ue, ve, te, fu, fv, ft);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      fe[3 * a][k] = fu[a];
      fe[3 * a + 1][k] = fv[a];
      fe[3 * a + 2][k] = ft[a];
    }
  }
}

// sum at owned node (li, lj) of the forces of its four elements, in a fixed
// order: element below-left (its node 2), below-right (3), above-left (1),
// above-right (0)
__device__ __forceinline__ void gather(double (*fe)[CE * CE], int li, int lj, double y[3]) {
  const int bl = lj * CE + li, br = bl + 1, al = bl + CE, ar = al + 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) y[c] = fe[6 + c][bl] + fe[9 + c][br] + fe[3 + c][al] + fe[c][ar];
}

__device__ __forceinline__ void tile_origin(const CosGeom &g, int tile, int *i0, int *j0) {
  *i0 = (tile % g.tx) * CT;
  *j0 = (tile / g.tx) * CT;
}

// ------------------------------------------------------------------ kernels
// stand-alone operator: y = P K P x + (I - P) x, or K x (raw)
__global__ __launch_bounds__(CTHREADS) void k_cos_apply(CosGeom g, CosMat m, const double *cs, const double *x,
                                                        double *y, int raw) {
  __shared__ double xs[3][CH * CH];
  __shared__ double fe[12][CE * CE];
  const int s = blockIdx.y;
  int i0, j0;
  tile_origin(g, blockIdx.x, &i0, &j0);
  const size_t vb = (size_t)s * 3 * g.nnode;
  for (int k = threadIdx.x; k < CH * CH; k += CTHREADS) {
    const int i = i0 - 1 + k % CH, j = j0 - 1 + k / CH;
    double v[3] = {0.0, 0.0, 0.0};
    if (i >= 0 && i < g.nnx && j >= 0 && j < g.nny) {
      const size_t o = vb + 3 * ((size_t)j * g.nnx + i);
      for (int c = 0; c < 3; ++c) v[c] = (!raw && cos_constrained(g, i, j, c)) ? 0.0 : x[o + c];
    }
    for (int c = 0; c < 3; ++c) xs[c][k] = v[c];
  }
  __syncthreads();
  tile_forces(g, m, cs + (size_t)s * 8 * g.nelem, i0, j0, xs, fe);
  __syncthreads();
  const int li = threadIdx.x % CT, lj = threadIdx.x / CT, i = i0 + li, j = j0 + lj;
  if (i < g.nnx && j < g.nny) {
    double f[3];
    gather(fe, li, lj, f);
    const size_t o = vb + 3 * ((size_t)j * g.nnx + i);
    for (int c = 0; c < 3; ++c) y[o + c] = (!raw && cos_constrained(g, i, j, c)) ? x[o + c] : f[c];
  }
}

// set-up of each slot: b = -P K g (g: u = delta on x = L), the Jacobi
// diagonal, x = 0, r = b, and the partial sums of r.z and r.r (parity 1, as
// if written by the vector pass of iteration -1); optional copies of b and
// 1 / diag
__global__ __launch_bounds__(CTHREADS) void k_cos_setup(CosGeom g, CosMat m, CosSlots S, double *b_out,
                                                        double *dinv_out) {
  __shared__ double xs[3][CH * CH];
  __shared__ double fe[12][CE * CE];
  __shared__ double red[4];
  const int s = blockIdx.y, tile = blockIdx.x;
  int i0, j0;
  tile_origin(g, tile, &i0, &j0);
  const double *cs_s = S.cs + (size_t)s * 8 * g.nelem;
  // K g: the prescribed end-shortening as the input vector
  for (int k = threadIdx.x; k < CH * CH; k += CTHREADS) {
    const int i = i0 - 1 + k % CH, j = j0 - 1 + k / CH;
    const bool on = i == g.nx && j >= 0 && j < g.nny;
    xs[0][k] = on ? g.delta : 0.0;
    xs[1][k] = 0.0;
    xs[2][k] = 0.0;
  }
  __syncthreads();
  tile_forces(g, m, cs_s, i0, j0, xs, fe);
  __syncthreads();
  const int li = threadIdx.x % CT, lj = threadIdx.x / CT, i = i0 + li, j = j0 + lj;
  const bool mine = i < g.nnx && j < g.nny;
  double kg[3] = {0.0, 0.0, 0.0};
  if (mine) gather(fe, li, lj, kg);
  __syncthreads();
  // diagonal entries: each element's operator applied to its unit vectors
  for (int k = threadIdx.x; k < CE * CE; k += CTHREADS) {
    const int le = k % CE, me = k / CE;
    const int ex = i0 - 1 + le, ey = j0 - 1 + me;
    double dg[12];
    for (int t = 0; t < 12; ++t) dg[t] = 0.0;
    if (ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny) {
      double cs[8];
      load_cs(cs_s + 8 * ((size_t)ey * g.nx + ex), cs);
      for (int t = 0; t < 12; ++t) {
        double ue[4] = {0, 0, 0, 0}, ve[4] = {0, 0, 0, 0}, te[4] = {0, 0, 0, 0}, fu[4], fv[4], ft[4];
        const int a = t / 3, c = t % 3;
        if (c == 0) ue[a] = 1.0;
        else if (c == 1) ve[a] = 1.0;
        else te[a] = 1.0;
        elem_forces(g, m, cs, ue, ve, te, fu, fv, ft);
        dg[t] = c == 0 ? fu[a] : c == 1 ? fv[a] : ft[a];
      }
    }
    for (int t = 0; t < 12; ++t) fe[t][k] = dg[t];
  }
  __syncthreads();
  double prz = 0.0, prr = 0.0;
  if (mine) {
    double dg[3];
    gather(fe, li, lj, dg);
    const size_t o = (size_t)s * 3 * g.nnode + 3 * ((size_t)j * g.nnx + i);
    for (int c = 0; c < 3; ++c) {
      const bool con = cos_constrained(g, i, j, c);
      const double b = con ? 0.0 : -kg[c];
      const double di = 1.0 / (con ? 1.0 : dg[c]);
      S.x[o + c] = 0.0;
      S.r[o + c] = b;
      S.dinv[o + c] = di;
      if (b_out) b_out[o + c] = b;
      if (dinv_out) dinv_out[o + c] = di;
      prz += b * di * b;
      prr += b * b;
    }
  }
  prz = block_sum(prz, red);
  prr = block_sum(prr, red);
  if (threadIdx.x == 0) {
    const size_t pp = ((size_t)1 * S.S + s) * g.ntiles + tile;
    S.part_rz[pp] = prz;
    S.part_rr[pp] = prr;
    if (tile == 0) {
      S.active[s] = 1;
      S.status[s] = S_NOCONV;
      S.iters[s] = 0;
    }
  }
}

// operator pass of iteration `it`: stopping test on r_it, p_it = z_it +
// beta p_{it-1} (halo included, owned nodes stored), A p_it, partials of p.Ap
// K fixed-order work-group sums at once (256 threads): each value summed as by
// block_sum (butterfly within each wave, then the four wave sums in order),
// with one pair of barriers for all of them; red holds 4 K values
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double *red) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[4 * k + wid] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = red[4 * k];
    for (int w = 1; w < 4; ++w) t += red[4 * k + w];
    v[k] = t;
  }
}

// the tiles' partial sums of a sample (entries t, t + 256, ... per thread, then
// block_sums), K arrays at once
template <int K>
__device__ __forceinline__ void partial_sums(const double *const (&a)[K], int n, double (&v)[K], double *red) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int t = threadIdx.x; t < n; t += 256)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += a[k][t];
  block_sums<K>(v, red);
}

__global__ __launch_bounds__(CTHREADS) void k_cos_pass1(CosGeom g, CosMat m, CosSlots S, int it) {
  __shared__ double xs[3][CH * CH];
  __shared__ double fe[12][CE * CE];
  __shared__ double red[12];
  const int s = blockIdx.y, tile = blockIdx.x;
  if (__builtin_amdgcn_readfirstlane(S.active[s]) == 0) return;
  const int nt = g.ntiles;
  const double *pold = (it & 1) ? S.p0 : S.p1;
  double *pnew = (it & 1) ? S.p1 : S.p0;
  int i0, j0;
  tile_origin(g, tile, &i0, &j0);
  const size_t vb = (size_t)s * 3 * g.nnode;
  // the tile's r, dinv and p_old (tile and halo), requested before the
  // cross-tile sums so that both round trips overlap
  constexpr int NPT = (CH * CH + CTHREADS - 1) / CTHREADS;
  double dv[NPT][3], rv[NPT][3], pv[NPT][3];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int k = threadIdx.x + q * CTHREADS;
    const int i = i0 - 1 + k % CH, j = j0 - 1 + k / CH;
    const bool in = k < CH * CH && i >= 0 && i < g.nnx && j >= 0 && j < g.nny;
    const size_t o = in ? vb + 3 * ((size_t)j * g.nnx + i) : vb;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dv[q][c] = in ? S.dinv[o + c] : 0.0;
      rv[q][c] = in ? S.r[o + c] : 0.0;
      pv[q][c] = (in && it > 0) ? pold[o + c] : 0.0;
    }
  }
  const size_t cur = ((size_t)((it + 1) & 1) * S.S + s) * nt;   // partials of r_it
  const size_t prv = ((size_t)(it & 1) * S.S + s) * nt;         // partials of r_{it-1}
  const double *const parts[3] = {S.part_rz + cur, S.part_rr + cur, S.part_rz + (it > 0 ? prv : cur)};
  double sums[3];
  partial_sums<3>(parts, nt, sums, red);
  const double rz = sums[0], rr = sums[1];
  const double bb = it == 0 ? rr : S.bb[s];
  // stopping test (every work-group of the sample takes the same decision)
  const bool bad = !isfinite(rr) || !isfinite(rz);
  if (bad || !(rr > S.rtol2 * bb) || it >= S.max_iter) {
    if (tile == 0 && threadIdx.x == 0) {
      S.active[s] = 0;
      S.iters[s] = it;
      S.relres[s] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
      S.status[s] = bad ? S_NAN : (rr > S.rtol2 * bb ? S_NOCONV : S_OK);
      if (it == 0) S.bb[s] = bb;
    }
    return;
  }
  if (it == 0 && tile == 0 && threadIdx.x == 0) S.bb[s] = bb;
  const double beta = it > 0 ? rz / sums[2] : 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int k = threadIdx.x + q * CTHREADS;
    if (k >= CH * CH) break;
    const int i = i0 - 1 + k % CH, j = j0 - 1 + k / CH;
    double v[3] = {0.0, 0.0, 0.0};
    if (i >= 0 && i < g.nnx && j >= 0 && j < g.nny) {
      const size_t o = vb + 3 * ((size_t)j * g.nnx + i);
      for (int c = 0; c < 3; ++c) {
        v[c] = dv[q][c] * rv[q][c];
        if (it > 0) v[c] += beta * pv[q][c];
      }
      if (i >= i0 && i < i0 + CT && j >= j0 && j < j0 + CT)
        for (int c = 0; c < 3; ++c) pnew[o + c] = v[c];
    }
    for (int c = 0; c < 3; ++c) xs[c][k] = v[c];
  }
  __syncthreads();
  tile_forces(g, m, S.cs + (size_t)s * 8 * g.nelem, i0, j0, xs, fe);
  __syncthreads();
  const int li = threadIdx.x % CT, lj = threadIdx.x / CT, i = i0 + li, j = j0 + lj;
  double pap = 0.0;
  if (i < g.nnx && j < g.nny) {
    double f[3];
    gather(fe, li, lj, f);
    const size_t o = vb + 3 * ((size_t)j * g.nnx + i);
    for (int c = 0; c < 3; ++c) {
      const double y = cos_constrained(g, i, j, c) ? 0.0 : f[c];
      S.Ap[o + c] = y;
      pap += xs[c][(lj + 1) * CH + li + 1] * y;
    }
  }
  pap = block_sum(pap, red);
  if (threadIdx.x == 0) S.part_pap[(size_t)s * nt + tile] = pap;
}

// vector pass of iteration `it`: alpha = r.z / p.Ap, x += alpha p, r -= alpha
// A p, partials of r.z and r.r (parity it & 1)
__global__ __launch_bounds__(CTHREADS) void k_cos_pass2(CosGeom g, CosSlots S, int it) {
  __shared__ double red[12];
  const int s = blockIdx.y, tile = blockIdx.x;
  if (__builtin_amdgcn_readfirstlane(S.active[s]) == 0) return;
  const int nt = g.ntiles;
  const double *p = (it & 1) ? S.p1 : S.p0;
  int i0, j0;
  tile_origin(g, tile, &i0, &j0);
  const int li = threadIdx.x % CT, lj = threadIdx.x / CT, i = i0 + li, j = j0 + lj;
  const bool in = i < g.nnx && j < g.nny;
  const size_t o = (size_t)s * 3 * g.nnode + (in ? 3 * ((size_t)j * g.nnx + i) : 0);
  // the node's vectors, requested before the cross-tile sums
  double xv[3], pv[3], rv[3], av[3], dv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    xv[c] = in ? S.x[o + c] : 0.0;
    pv[c] = in ? p[o + c] : 0.0;
    rv[c] = in ? S.r[o + c] : 0.0;
    av[c] = in ? S.Ap[o + c] : 0.0;
    dv[c] = in ? S.dinv[o + c] : 0.0;
  }
  const double *const parts[2] = {S.part_rz + ((size_t)((it + 1) & 1) * S.S + s) * nt, S.part_pap + (size_t)s * nt};
  double sums[2];
  partial_sums<2>(parts, nt, sums, red);
  const double rz = sums[0], pap = sums[1];
  if (!(pap > 0.0)) {
    if (tile == 0 && threadIdx.x == 0) {
      S.active[s] = 0;
      S.iters[s] = it;
      S.status[s] = isfinite(pap) ? S_BREAKDOWN : S_NAN;
    }
    return;
  }
  const double alpha = rz / pap;
  double prz = 0.0, prr = 0.0;
  if (in) {
    for (int c = 0; c < 3; ++c) {
      S.x[o + c] = xv[c] + alpha * pv[c];
      const double r = rv[c] - alpha * av[c];
      S.r[o + c] = r;
      prz += r * dv[c] * r;
      prr += r * r;
    }
  }
  double pr2[2] = {prz, prr};
  block_sums<2>(pr2, red);
  prz = pr2[0];
  prr = pr2[1];
  if (threadIdx.x == 0) {
    const size_t pp = ((size_t)(it & 1) * S.S + s) * nt + tile;
    S.part_rz[pp] = prz;
    S.part_rr[pp] = prr;
  }
}

// strength quantity of interest (Eq. failureCriterion), one work-group per
// slot: f = tau_e / tau_y maximised over the Gauss points of the elements of
// the central square, Q = -(mean sigma_x over the square) / f*; written through
// out_idx (entries below coarse_base: fine results and info fields, the
// others coarse ones)
__global__ __launch_bounds__(256) void k_cos_qoi(CosGeom g, CosMat m, CosSlots S, int n, const int *out_idx,
                                                  double *q_fine, double *q_coarse, mlmc_info *info, int coarse_base,
                                                  double *d_out) {
  __shared__ double red[4];
  const int s = blockIdx.x;
  if (s >= n) return;
  const double *xs = S.x + (size_t)s * 3 * g.nnode;
  const double *cs_s = S.cs + (size_t)s * 8 * g.nelem;
  const int qw = g.qx1 - g.qx0, nq = qw * (g.qy1 - g.qy0);
  double fmaxv = 0.0, sx = 0.0;
  for (int k = threadIdx.x; k < nq; k += 256) {
    const int ex = g.qx0 + k % qw, ey = g.qy0 + k / qw;
    const int n0 = ey * g.nnx + ex;
    const int nodes[4] = {n0, n0 + 1, n0 + g.nnx + 1, n0 + g.nnx};
    double ue[4], ve[4], te[4], cs[8];
    for (int a = 0; a < 4; ++a) {
      const int i = nodes[a] % g.nnx;
      ue[a] = xs[3 * nodes[a]] + (i == g.nx ? g.delta : 0.0);
      ve[a] = xs[3 * nodes[a] + 1];
      te[a] = xs[3 * nodes[a] + 2];
    }
    load_cs(cs_s + 8 * ((size_t)ey * g.nx + ex), cs);
    for (int q = 0; q < 4; ++q) {
      const GpStress st = gp_stress(m, gp_shape(g, q), cs[2 * q], cs[2 * q + 1], ue, ve, te);
      const double t2 = st.t22 / m.R;
      fmaxv = fmax(fmaxv, sqrt(st.t12 * st.t12 + t2 * t2) / m.tau_y);
      sx += st.s11;
    }
  }
  fmaxv = block_max(fmaxv, red);
  sx = block_sum(sx, red);
  if (d_out) {
    for (int k = threadIdx.x; k < g.nnode; k += 256) {
      const size_t o = (size_t)s * 3 * g.nnode + 3 * (size_t)k;
      d_out[o] = xs[3 * k] + ((k % g.nnx) == g.nx ? g.delta : 0.0);
      d_out[o + 1] = xs[3 * k + 1];
      d_out[o + 2] = xs[3 * k + 2];
    }
  }
  if (threadIdx.x == 0) {
    // the Gauss weights are equal: mean over the square = mean over its Gauss points
    const double q = -(sx / (4.0 * nq)) / fmaxv;
    const int o = out_idx ? out_idx[s] : s;
    if (o < coarse_base) {
      q_fine[o] = q;
      if (info) {
        info[o].iters_f = S.iters[s];
        info[o].relres_f = S.relres[s];
        info[o].status_f = S.status[s];
      }
    } else {
      q_coarse[o - coarse_base] = q;
      info[o - coarse_base].iters_c = S.iters[s];
      info[o - coarse_base].relres_c = S.relres[s];
      info[o - coarse_base].status_c = S.status[s];
    }
  }
}

// KL synthesis (Eq. inftyKL with the level's nkl terms): the separable modes
// are products X_k(x) Y_k(y) tabulated at the Gauss-point coordinates,
// X [K][2 nx], Y [K][2 ny]; a_k = sqrt(mu_k) xi_k.  Writes the angles and/or
// their (cos 2phi, sin 2phi) pairs.
__global__ __launch_bounds__(256) void k_cos_synth(CosGeom g, const double *X, const double *Y,
                                                   const double *sqrt_mu, const double *xi, int ld_xi,
                                                   const int64_t *rows, int n, double *theta, double *cs) {
  __shared__ double a[MAXKL];
  const int s = blockIdx.y;
  if (s >= n) return;
  const int64_t row = rows ? rows[s] : s;
  for (int k = threadIdx.x; k < g.nkl; k += 256) a[k] = sqrt_mu[k] * xi[(size_t)row * ld_xi + k];
  __syncthreads();
  const int ngp = 4 * g.nelem;
  const int gp = blockIdx.x * 256 + threadIdx.x;
  if (gp >= ngp) return;
  const int e = gp >> 2, q = gp & 3;
  const int gx = 2 * (e % g.nx) + (q & 1), gy = 2 * (e / g.nx) + (q >> 1);
  const int sx = 2 * g.nx, sy = 2 * g.ny;
  double th = 0.0;
  for (int k = 0; k < g.nkl; ++k) th = fma(a[k] * X[(size_t)k * sx + gx], Y[(size_t)k * sy + gy], th);
  if (theta) theta[(size_t)s * ngp + gp] = th;
  if (cs) {
    double s2, c2;
    cs_of_angle(th, &s2, &c2);
    *reinterpret_cast<double2 *>(cs + (size_t)s * 2 * ngp + 2 * (size_t)gp) = make_double2(c2, s2);
  }
}

// ------------------------------------------------------------------ host
struct CosLevel {
  CosGeom g{};
  double *X = nullptr, *Y = nullptr;   // mode tables at the Gauss-point coordinates
  int cap = 0;
  size_t bytes = 0;
  CosSlots S{};
  int64_t *rows = nullptr;
  int *outidx = nullptr;
};

}  // namespace

struct CosCtx {
  int nlev = 0, K = 0;
  CosMat mat{};
  double rtol = 1e-10;
  int max_iter = 200000;
  double *d_sqrt_mu = nullptr;
  std::vector<CosLevel> lv;
  size_t budget = 0, used = 0;
  int *h_active = nullptr;
  int h_cap = 0;
};

namespace {

void free_slots(CosCtx *c, CosLevel &L) {
  void *bufs[] = {L.S.x, L.S.r, L.S.p0, L.S.p1, L.S.Ap, L.S.dinv, L.S.cs, L.S.part_pap, L.S.part_rz,
                  L.S.part_rr, L.S.bb, L.S.relres, L.S.iters, L.S.status, L.S.active, L.rows, L.outidx};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  c->used -= L.bytes;
  L.S = CosSlots{};
  L.rows = nullptr;
  L.outidx = nullptr;
  L.cap = 0;
  L.bytes = 0;
}

size_t slot_bytes(const CosGeom &g) {
  const size_t vec = (size_t)3 * g.nnode * sizeof(double);
  return 6 * vec + (size_t)8 * g.nelem * sizeof(double) + (size_t)5 * g.ntiles * sizeof(double) +
         2 * sizeof(double) + 3 * sizeof(int) + sizeof(int64_t) + sizeof(int);
}

template <typename T>
bool dal(T **p, size_t n) {
  return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T)) == hipSuccess;
}

int ensure_slots(CosCtx *c, std::string &err, int level, int n) {
  CosLevel &L = c->lv[level];
  if (L.cap >= n) return MLMC_OK;
  free_slots(c, L);
  const size_t need = slot_bytes(L.g) * (size_t)n;
  if (c->used + need > c->budget) {
    err = "cosserat level " + std::to_string(level) + ": " + std::to_string(n) + " slots exceed the memory budget";
    return MLMC_ENOMEM;
  }
  const size_t v = (size_t)3 * L.g.nnode * n, nt = (size_t)L.g.ntiles * n;
  CosSlots &S = L.S;
  bool ok = dal(&S.x, v) && dal(&S.r, v) && dal(&S.p0, v) && dal(&S.p1, v) && dal(&S.Ap, v) && dal(&S.dinv, v) &&
            dal(&S.cs, (size_t)8 * L.g.nelem * n) && dal(&S.part_pap, nt) && dal(&S.part_rz, 2 * nt) &&
            dal(&S.part_rr, 2 * nt) && dal(&S.bb, (size_t)n) && dal(&S.relres, (size_t)n) &&
            dal(&S.iters, (size_t)n) && dal(&S.status, (size_t)n) && dal(&S.active, (size_t)n) &&
            dal(&L.rows, (size_t)n) && dal(&L.outidx, (size_t)n);
  if (!ok) {
    free_slots(c, L);
    err = "cosserat workspace allocation failed";
    return MLMC_ENOMEM;
  }
  S.S = n;
  L.cap = n;
  L.bytes = need;
  c->used += need;
  if (c->h_cap < n) {
    if (c->h_active) (void)hipHostFree(c->h_active);
    c->h_active = nullptr;
    c->h_cap = 0;
    if (hipHostMalloc((void **)&c->h_active, sizeof(int) * n) != hipSuccess) {
      err = "pinned flag buffer allocation failed";
      return MLMC_ENOMEM;
    }
    c->h_cap = n;
  }
  return MLMC_OK;
}

// largest batch of a level that fits beside the other levels' slots
int max_slots(const CosCtx *c, int level) {
  const size_t other = c->used - c->lv[level].bytes;
  if (c->budget <= other) return 0;
  return (int)std::min<size_t>((c->budget - other) / slot_bytes(c->lv[level].g), 8192);
}

#define COSCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                \
      return MLMC_EHIP;                                                       \
    }                                                                         \
  } while (0)

// set-up and PCG to completion of slots 0..n-1 of a level whose angle pairs
// are staged
int run_solves(CosCtx *c, std::string &err, int level, int n, double rtol, hipStream_t st, double *b_out = nullptr,
               double *dinv_out = nullptr) {
  CosLevel &L = c->lv[level];
  CosSlots S = L.S;
  S.max_iter = c->max_iter;
  S.rtol2 = rtol * rtol;
  const dim3 grid(L.g.ntiles, n);
  hipLaunchKernelGGL(k_cos_setup, grid, dim3(CTHREADS), 0, st, L.g, c->mat, S, b_out, dinv_out);
  COSCHK(hipGetLastError());
  for (long it = 0;; it += CBLOCK) {
    for (int b = 0; b < CBLOCK; ++b) {
      hipLaunchKernelGGL(k_cos_pass1, grid, dim3(CTHREADS), 0, st, L.g, c->mat, S, (int)(it + b));
      hipLaunchKernelGGL(k_cos_pass2, grid, dim3(CTHREADS), 0, st, L.g, S, (int)(it + b));
    }
    COSCHK(hipGetLastError());
    COSCHK(hipMemcpyAsync(c->h_active, S.active, sizeof(int) * n, hipMemcpyDeviceToHost, st));
    COSCHK(hipStreamSynchronize(st));
    bool any = false;
    for (int k = 0; k < n; ++k) any |= c->h_active[k] != 0;
    if (!any) break;
    if (it > (long)c->max_iter + 2 * CBLOCK) {
      err = "cosserat PCG loop did not terminate";
      return MLMC_EHIP;
    }
  }
  return MLMC_OK;
}

CosSlots with_tol(const CosCtx *c, const CosLevel &L, double rtol) {
  CosSlots S = L.S;
  S.max_iter = c->max_iter;
  S.rtol2 = rtol * rtol;
  return S;
}

}  // namespace

CosCtx *cos_create(const Json &cfg, size_t budget, std::string &err) {
  CosCtx *c = new CosCtx();
  try {
    c->budget = budget;
    c->nlev = (int)cfg.number("n_levels");
    if (c->nlev < 1 || c->nlev > 8) throw std::runtime_error("n_levels out of range");
    const Json &f = cfg.at("fibre");
    const double vf = f.number("v_f"), Ef = f.number("E_f"), Em = f.number("E_m"), Gf = f.number("G_f"),
                 Gm = f.number("G_m"), d = f.number("d"), nu12 = f.number("nu12");
    if (!(vf > 0.0 && vf < 1.0) || !(Ef > 0 && Em > 0 && Gf > 0 && Gm > 0 && d > 0))
      throw std::runtime_error("fibre constants out of range");
    // rule-of-mixtures constants, the reduced orthotropic stiffness and the
    // two shear moduli (parallel: matrix dominated; orthogonal: fibre dominated)
    const double E1 = vf * Ef + (1.0 - vf) * Em, E2 = 1.0 / (vf / Ef + (1.0 - vf) / Em);
    const double nu21 = nu12 * E2 / E1, den = 1.0 - nu12 * nu21;
    c->mat.C11 = E1 / den;
    c->mat.C12 = nu12 * E2 / den;
    c->mat.C22 = E2 / den;
    c->mat.Gp = 1.0 / (vf / Gf + (1.0 - vf) / Gm);
    c->mat.Go = vf * Gf + (1.0 - vf) * Gm;
    c->mat.D1 = vf * Ef * d * d / 16.0;
    c->mat.D2 = (1.0 - vf) * Em * d * d / 16.0;
    c->mat.R = f.number("R");
    c->mat.tau_y = f.number("tau_c");
    c->rtol = cfg.number_or("rtol", 1e-10);
    c->max_iter = (int)cfg.number_or("max_iter", 200000);
    const Json &kl = cfg.at("kl");
    if (kl.string_or("type", "") != "exp_separable")
      throw std::runtime_error("the Cosserat workload needs the separable exponential covariance");
    c->K = (int)kl.number("n_modes");
    if (c->K < 1 || c->K > MAXKL) throw std::runtime_error("n_modes must be in 1..1024");
    std::vector<double> mpl = kl.numbers("modes_per_level");
    if (mpl.size() != 2) throw std::runtime_error("modes_per_level needs [base, step]");
    const double sr = kl.has("sigma_rad") ? kl.number("sigma_rad") : kl.number("sigma_deg") * M_PI / 180.0;
    const double Lx = cfg.number("Lx"), Ly = cfg.number("Ly");
    SeparableKL sk = separable_kl(Lx, Ly, sr * sr, kl.number("corr_x"), kl.number("corr_y"), c->K);
    std::vector<double> smu(c->K);
    for (int k = 0; k < c->K; ++k) smu[k] = std::sqrt(sk.mu[k]);
    if (!dal(&c->d_sqrt_mu, (size_t)c->K)) throw std::runtime_error("device allocation failed");
    (void)hipMemcpy(c->d_sqrt_mu, smu.data(), sizeof(double) * c->K, hipMemcpyHostToDevice);
    std::vector<double> reg = cfg.numbers("qoi_region");
    if (reg.size() != 4) throw std::runtime_error("qoi_region needs [x0, x1, y0, y1]");
    c->lv.resize(c->nlev);
    for (int l = 0; l < c->nlev; ++l) {
      CosGeom &g = c->lv[l].g;
      g.nx = (int)cfg.number("nx0") << l;
      g.ny = (int)cfg.number("ny0") << l;
      g.nnx = g.nx + 1;
      g.nny = g.ny + 1;
      g.nnode = g.nnx * g.nny;
      g.nelem = g.nx * g.ny;
      g.tx = (g.nnx + CT - 1) / CT;
      g.ty = (g.nny + CT - 1) / CT;
      g.ntiles = g.tx * g.ty;
      g.hx = Lx / g.nx;
      g.hy = Ly / g.ny;
      g.delta = cfg.number("delta");
      g.nkl = std::min(c->K, (int)std::lround(mpl[0] + mpl[1] * l));
      // elements whose centroid lies in the QoI square
      auto first = [](double lo, double h, int n) {
        int k = 0;
        while (k < n && (k + 0.5) * h < lo) ++k;
        return k;
      };
      g.qx0 = first(reg[0], g.hx, g.nx);
      g.qx1 = first(reg[1], g.hx, g.nx);
      while (g.qx1 < g.nx && (g.qx1 + 0.5) * g.hx <= reg[1]) ++g.qx1;
      g.qy0 = first(reg[2], g.hy, g.ny);
      g.qy1 = first(reg[3], g.hy, g.ny);
      while (g.qy1 < g.ny && (g.qy1 + 0.5) * g.hy <= reg[3]) ++g.qy1;
      if (g.qx1 <= g.qx0 || g.qy1 <= g.qy0) throw std::runtime_error("qoi_region holds no element centroid");
      // mode tables at the Gauss-point coordinates (centred)
      std::vector<double> X((size_t)g.nkl * 2 * g.nx), Y((size_t)g.nkl * 2 * g.ny);
      for (int k = 0; k < g.nkl; ++k) {
        for (int t = 0; t < 2 * g.nx; ++t) {
          const double x = g.hx * ((double)(t / 2) + ((t & 1) ? GP_P : GP_M));
          X[(size_t)k * 2 * g.nx + t] = sk.x.mode(sk.ix[k], x - sk.x.a);
        }
        for (int t = 0; t < 2 * g.ny; ++t) {
          const double y = g.hy * ((double)(t / 2) + ((t & 1) ? GP_P : GP_M));
          Y[(size_t)k * 2 * g.ny + t] = sk.y.mode(sk.iy[k], y - sk.y.a);
        }
      }
      if (!dal(&c->lv[l].X, X.size()) || !dal(&c->lv[l].Y, Y.size()))
        throw std::runtime_error("device allocation failed");
      (void)hipMemcpy(c->lv[l].X, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice);
      (void)hipMemcpy(c->lv[l].Y, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice);
    }
  } catch (const std::exception &e) {
    err = e.what();
    cos_destroy(c);
    return nullptr;
  }
  return c;
}

void cos_destroy(CosCtx *c) {
  if (!c) return;
  for (auto &L : c->lv) {
    free_slots(c, L);
    if (L.X) (void)hipFree(L.X);
    if (L.Y) (void)hipFree(L.Y);
  }
  if (c->d_sqrt_mu) (void)hipFree(c->d_sqrt_mu);
  if (c->h_active) (void)hipHostFree(c->h_active);
  delete c;
}

int cos_num_levels(const CosCtx *c) { return c->nlev; }

int cos_num_params(const CosCtx *c) { return c->K + 3; }

void cos_level_sizes(const CosCtx *c, int level, int64_t *nn, int64_t *nd, int64_t *ne) {
  const CosGeom &g = c->lv[level].g;
  *nn = g.nnode;
  *nd = 3 * (int64_t)g.nnode;
  *ne = g.nelem;
}

size_t cos_slot_bytes(const CosCtx *c, int level) { return slot_bytes(c->lv[level].g); }

int cos_reserve(CosCtx *c, std::string &err, int level, int n) {
  if (level < 0 || level >= c->nlev || n < 0) {
    err = "level out of range or n < 0";
    return MLMC_EINVAL;
  }
  if (n == 0) return MLMC_OK;
  if (n > max_slots(c, level)) {
    err = "cosserat level " + std::to_string(level) + ": " + std::to_string(n) + " slots exceed the memory budget";
    return MLMC_ENOMEM;
  }
  return ensure_slots(c, err, level, n);
}

int cos_sample_field(CosCtx *c, std::string &err, int level, int n, const double *xi, int ld_xi, double *theta,
                     hipStream_t st) {
  if (ld_xi < c->K + 3) {
    err = "ld_xi < n_modes + 3";
    return MLMC_EINVAL;
  }
  if (n == 0) return MLMC_OK;
  if (n > 65535) {
    err = "n > 65535";
    return MLMC_EINVAL;
  }
  const CosLevel &L = c->lv[level];
  hipLaunchKernelGGL(k_cos_synth, dim3((4 * L.g.nelem + 255) / 256, n), dim3(256), 0, st, L.g, L.X, L.Y,
                     c->d_sqrt_mu, xi, ld_xi, nullptr, n, theta, nullptr);
  COSCHK(hipGetLastError());
  return MLMC_OK;
}

int cos_apply(CosCtx *c, std::string &err, int level, int n, const double *theta, const double *x, double *y,
              int raw, hipStream_t st) {
  if (n == 0) return MLMC_OK;
  if (n > 65535 || n > max_slots(c, level)) {
    err = "batch too large";
    return MLMC_ENOMEM;
  }
  if (int rc = ensure_slots(c, err, level, n)) return rc;
  CosLevel &L = c->lv[level];
  launch_theta_cs(theta, L.S.cs, (size_t)n * 4 * L.g.nelem, st);
  hipLaunchKernelGGL(k_cos_apply, dim3(L.g.ntiles, n), dim3(CTHREADS), 0, st, L.g, c->mat, L.S.cs, x, y, raw);
  COSCHK(hipGetLastError());
  return MLMC_OK;
}

int cos_rhs_diag(CosCtx *c, std::string &err, int level, int n, const double *theta, double *b, double *dinv,
                 hipStream_t st) {
  if (n == 0) return MLMC_OK;
  if (n > 65535 || n > max_slots(c, level)) {
    err = "batch too large";
    return MLMC_ENOMEM;
  }
  if (int rc = ensure_slots(c, err, level, n)) return rc;
  CosLevel &L = c->lv[level];
  launch_theta_cs(theta, L.S.cs, (size_t)n * 4 * L.g.nelem, st);
  hipLaunchKernelGGL(k_cos_setup, dim3(L.g.ntiles, n), dim3(CTHREADS), 0, st, L.g, c->mat,
                     with_tol(c, L, c->rtol), b, dinv);
  COSCHK(hipGetLastError());
  return MLMC_OK;
}

int cos_solve_theta(CosCtx *c, std::string &err, int level, int n, const double *theta, double *q, double *d,
                    mlmc_info *info, double rtol, hipStream_t st) {
  if (n == 0) return MLMC_OK;
  if (n > 65535 || n > max_slots(c, level)) {
    err = "batch exceeds the memory budget";
    return MLMC_ENOMEM;
  }
  if (int rc = ensure_slots(c, err, level, n)) return rc;
  CosLevel &L = c->lv[level];
  if (info) launch_info_init(info, nullptr, n, st);
  launch_theta_cs(theta, L.S.cs, (size_t)n * 4 * L.g.nelem, st);
  const double rt = rtol > 0 ? rtol : c->rtol;
  if (int rc = run_solves(c, err, level, n, rt, st)) return rc;
  hipLaunchKernelGGL(k_cos_qoi, dim3(n), dim3(256), 0, st, L.g, c->mat, with_tol(c, L, rt), n, nullptr, q, nullptr,
                     info, 1 << 30, d);
  COSCHK(hipGetLastError());
  COSCHK(hipStreamSynchronize(st));
  return MLMC_OK;
}

int cos_solve_batch(CosCtx *c, std::string &err, int n_req, const mlmc_request *req, const double *xi,
                    int64_t n_rows, int ld_xi, double *q_fine, double *q_coarse, mlmc_info *info, double rtol,
                    hipStream_t st) {
  if (ld_xi < c->K + 3) {
    err = "ld_xi < n_modes + 3";
    return MLMC_EINVAL;
  }
  for (int i = 0; i < n_req; ++i) {
    if (req[i].level < 0 || req[i].level >= c->nlev) {
      err = "request " + std::to_string(i) + ": bad level";
      return MLMC_EINVAL;
    }
    if (req[i].sample < 0 || req[i].sample >= n_rows) {
      err = "request " + std::to_string(i) + ": sample row outside [0, n_rows)";
      return MLMC_EINVAL;
    }
  }
  const double rt = rtol > 0 ? rtol : c->rtol;
  launch_info_init(info, q_coarse, n_req, st);
  COSCHK(hipGetLastError());
  // per level: fine solves of its requests, coarse solves of coupled requests
  // one level up (output index n_req + i)
  std::vector<std::vector<int64_t>> rows(c->nlev);
  std::vector<std::vector<int>> outs(c->nlev);
  for (int i = 0; i < n_req; ++i) {
    rows[req[i].level].push_back(req[i].sample);
    outs[req[i].level].push_back(i);
  }
  for (int i = 0; i < n_req; ++i)
    if (req[i].coupled && req[i].level > 0) {
      rows[req[i].level - 1].push_back(req[i].sample);
      outs[req[i].level - 1].push_back(n_req + i);
    }
  for (int l = 0; l < c->nlev; ++l) {
    const int total = (int)rows[l].size();
    if (!total) continue;
    CosLevel &L = c->lv[l];
    const int cap = std::min({std::max(L.cap, std::min(total, max_slots(c, l))), total, 65535});
    if (cap < 1) {
      err = "cosserat level " + std::to_string(l) + ": no slot fits the memory budget";
      return MLMC_ENOMEM;
    }
    if (int rc = ensure_slots(c, err, l, cap)) return rc;
    for (int off = 0; off < total; off += cap) {
      const int n = std::min(cap, total - off);
      COSCHK(hipMemcpyAsync(L.rows, rows[l].data() + off, sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
      COSCHK(hipMemcpyAsync(L.outidx, outs[l].data() + off, sizeof(int) * n, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_cos_synth, dim3((4 * L.g.nelem + 255) / 256, n), dim3(256), 0, st, L.g, L.X, L.Y,
                         c->d_sqrt_mu, xi, ld_xi, L.rows, n, nullptr, L.S.cs);
      COSCHK(hipGetLastError());
      if (int rc = run_solves(c, err, l, n, rt, st)) return rc;
      hipLaunchKernelGGL(k_cos_qoi, dim3(n), dim3(256), 0, st, L.g, c->mat, with_tol(c, L, rt), n, L.outidx, q_fine,
                         q_coarse, info, n_req, nullptr);
      COSCHK(hipGetLastError());
      COSCHK(hipStreamSynchronize(st));   // the row and index buffers are reused
    }
  }
  return MLMC_OK;
}

}  // namespace mlmc
