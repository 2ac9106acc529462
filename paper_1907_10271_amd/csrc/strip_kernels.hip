// HIP kernels of the strip sample solve (Section 3.1 of the paper):
// KL synthesis of the angle field, Dirichlet lifting and Jacobi diagonal,
// the two fused passes of batched Jacobi-PCG, the fibre-stress QoI and the
// FP64 level sums (Section 2.3).
//
// Work decomposition: a work-group owns a TILE_X x TILE_Y block of nodes of
// one sample (blockIdx.x = tile, blockIdx.y = slot).  It recomputes the
// elements touching its nodes (one-element halo), stages their nodal forces
// in LDS and gathers each owned node's four element contributions in a fixed
// order, so every result is independent of the batch it runs in and
// bit-reproducible.  Dot products use fixed-order wave butterflies and a
// fixed-order sum over tiles.
#include "strip_kernels.hpp"

#include "strip_device.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>

namespace mlmc {

namespace {

struct TileCoord {
  int i0, j0;
};

__device__ __forceinline__ TileCoord tile_of(const StripGeom &g, int t) {
  return {(t % g.tiles_x) * TILE_X, (t / g.tiles_x) * TILE_Y};
}

__device__ __forceinline__ bool node_in(const StripGeom &g, int i, int j) {
  return i >= 0 && i < g.nnx && j >= 0 && j < g.nny;
}

__device__ __forceinline__ bool elem_in(const StripGeom &g, int ex, int ey) {
  return ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
}

// element phase shared by the operator kernels: nodal values are in LDS
// (halo layout), element forces go to eo[8][TILE_ELEMS]
__device__ __forceinline__ void tile_elements(const StripGeom &g, const StripMat &m, const double *theta_s,
                                              TileCoord tc, const double *nu, const double *nv,
                                              double (*eo)[TILE_ELEMS]) {
  for (int k = threadIdx.x; k < TILE_ELEMS; k += TILE_THREADS) {
    const int lex = k % ELEM_X, ley = k / ELEM_X;
    const int ex = tc.i0 - 1 + lex, ey = tc.j0 - 1 + ley;
    double fu[4] = {0.0, 0.0, 0.0, 0.0}, fv[4] = {0.0, 0.0, 0.0, 0.0};
    if (elem_in(g, ex, ey)) {
      const double *tp = theta_s + 4 * ((size_t)ey * g.nx + ex);
      const double2 t01 = *reinterpret_cast<const double2 *>(tp);
      const double2 t23 = *reinterpret_cast<const double2 *>(tp + 2);
      const double th[4] = {t01.x, t01.y, t23.x, t23.y};
      const int n0 = ley * HALO_X + lex;
      const double u[4] = {nu[n0], nu[n0 + 1], nu[n0 + HALO_X + 1], nu[n0 + HALO_X]};
      const double v[4] = {nv[n0], nv[n0 + 1], nv[n0 + HALO_X + 1], nv[n0 + HALO_X]};
      elem_forces_q<double>(g, [&](int q) { return qbar_of(m, th[q]); }, u, v, fu, fv);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      eo[c][k] = fu[c];
      eo[4 + c][k] = fv[c];
    }
  }
}

// sum of the four element contributions of owned node (li, lj), fixed order
__device__ __forceinline__ void gather_node(const double (*eo)[TILE_ELEMS], int li, int lj, int cu,
                                            double &yu, double &yv) {
  const int e = lj * ELEM_X + li;
  // element (i-1, j-1): node 2; (i, j-1): node 3; (i-1, j): node 1; (i, j): node 0
  yu = ((eo[cu + 2][e] + eo[cu + 3][e + 1]) + eo[cu + 1][e + ELEM_X]) + eo[cu + 0][e + ELEM_X + 1];
  yv = ((eo[cu + 6][e] + eo[cu + 7][e + 1]) + eo[cu + 5][e + ELEM_X]) + eo[cu + 4][e + ELEM_X + 1];
}

}  // namespace

// ---------------------------------------------------------------- KL synthesis
// theta[s][gp] = sum_k modes[gp][k] xi[row_s][k] + A sech^2((x_gp - x0)/w)
// (modes pre-multiplied by sqrt(mu_k)); one thread per Gauss point, a group of
// SYN_SAMPLES samples per block so the mode row is read once per group.
// Outputs (each optional): theta in FP64; theta rounded to bfloat16 or FP32;
// and (cos 2theta, sin 2theta) per Gauss point, which is what the solver's
// rotated stiffness needs, evaluated once per sample instead of every
// iteration.
constexpr int SYN_SAMPLES = 8;
constexpr int MAX_MODES = 32;

__global__ __launch_bounds__(256) void k_kl_synth(const double *__restrict__ modes, int K, StripGeom g,
                                                  const double *__restrict__ xi, int ld_xi,
                                                  const int64_t *__restrict__ rows, int n,
                                                  double *__restrict__ th64, void *__restrict__ thlo,
                                                  int lo_fp32, int ld_out, double *__restrict__ cs, int code) {
  const int ngp = 4 * g.nelem;
  const int gp = blockIdx.x * 256 + threadIdx.x;
  if (gp >= ngp) return;
  double mk[MAX_MODES];
#pragma unroll
  for (int k = 0; k < MAX_MODES; ++k) mk[k] = (k < K) ? modes[(size_t)gp * K + k] : 0.0;
  const int e = gp >> 2, q = gp & 3;
  const double x = g.hx * ((e % g.nx) + ((q & 1) ? GP_P : GP_M));
  const int s0 = blockIdx.y * SYN_SAMPLES;
  for (int si = 0; si < SYN_SAMPLES; ++si) {
    const int s = s0 + si;
    if (s >= n) break;
    const int64_t row = rows ? rows[s] : s;
    const double *xr = xi + (size_t)row * ld_xi;
    double th = 0.0;
#pragma unroll
    for (int k = 0; k < MAX_MODES; ++k)
      if (k < K) th = fma(mk[k], xr[k], th);
    const double A = xr[K];
    if (A != 0.0) {
      const double c = cosh((x - xr[K + 1]) / xr[K + 2]);
      th += A / (c * c);
    }
    if (th64) th64[(size_t)s * ld_out + gp] = code ? angle_code(th) : th;
    if (cs) {
      double s2, c2;
      cs_of_angle(th, &s2, &c2);
      *reinterpret_cast<double2 *>(cs + (size_t)s * 2 * ngp + 2 * (size_t)gp) = make_double2(c2, s2);
    }
    if (thlo) {
      // round to float, then (bfloat16 storage) to bfloat16 with round-to-nearest-even
      const float f = (float)th;
      if (lo_fp32) {
        ((float *)thlo)[(size_t)s * ld_out + gp] = f;
      } else {
        uint32_t b = __float_as_uint(f);
        b += 0x7FFFu + ((b >> 16) & 1u);
        ((uint16_t *)thlo)[(size_t)s * ld_out + gp] = (uint16_t)(b >> 16);
      }
    }
  }
}

// Nystrom interpolation of the Matern eigenfunctions at every Gauss point:
// modes[gp][k] = sum_j k(x_gp, x_j) coef[j][k], coef = w_j phi_k(x_j) / sqrt(mu_k)
__global__ __launch_bounds__(256) void k_modes_nystrom(const double *__restrict__ gx, const double *__restrict__ gy,
                                                       const double *__restrict__ coef, int ngrid, int K,
                                                       double var, double kappa, StripGeom g,
                                                       double *__restrict__ modes) {
  const int ngp = 4 * g.nelem;
  const int gp = blockIdx.x * 256 + threadIdx.x;
  if (gp >= ngp) return;
  const int e = gp >> 2, q = gp & 3;
  const double x = g.hx * ((e % g.nx) + ((q & 1) ? GP_P : GP_M));
  const double y = g.hy * ((e / g.nx) + ((q & 2) ? GP_P : GP_M));
  double acc[MAX_MODES];
#pragma unroll
  for (int k = 0; k < MAX_MODES; ++k) acc[k] = 0.0;
  for (int j = 0; j < ngrid; ++j) {
    const double dx = x - gx[j], dy = y - gy[j];
    const double z = kappa * sqrt(dx * dx + dy * dy);
    const double kv = var * (1.0 + z) * exp(-z);
    const double *c = coef + (size_t)j * K;
#pragma unroll
    for (int k = 0; k < MAX_MODES; ++k)
      if (k < K) acc[k] = fma(kv, c[k], acc[k]);
  }
  for (int k = 0; k < K; ++k) modes[(size_t)gp * K + k] = acc[k];
}

// ---------------------------------------------------------------- operator
// y = P K P x + (I - P) x  (or y = K x when raw): test/diagnostic entry point
__global__ __launch_bounds__(TILE_THREADS) void k_apply(StripGeom g, StripMat m, const double *__restrict__ theta,
                                                        const double *__restrict__ x, double *__restrict__ y,
                                                        int raw) {
  __shared__ double nu[TILE_NODES_H], nv[TILE_NODES_H];
  __shared__ double eo[8][TILE_ELEMS];
  const int s = blockIdx.y;
  const TileCoord tc = tile_of(g, blockIdx.x);
  const size_t vb = (size_t)s * 2 * g.nnode;
  for (int k = threadIdx.x; k < TILE_NODES_H; k += TILE_THREADS) {
    const int i = tc.i0 - 1 + k % HALO_X, j = tc.j0 - 1 + k / HALO_X;
    double a = 0.0, b = 0.0;
    if (node_in(g, i, j)) {
      const double2 xv = *reinterpret_cast<const double2 *>(x + vb + 2 * ((size_t)j * g.nnx + i));
      a = xv.x;
      b = xv.y;
      if (!raw) {
        if (i == 0) { a = 0.0; b = 0.0; }
        if (i == g.nx) a = 0.0;
      }
    }
    nu[k] = a;
    nv[k] = b;
  }
  __syncthreads();
  tile_elements(g, m, theta + (size_t)s * 4 * g.nelem, tc, nu, nv, eo);
  __syncthreads();
  const int li = threadIdx.x % TILE_X, lj = threadIdx.x / TILE_X;
  const int i = tc.i0 + li, j = tc.j0 + lj;
  if (threadIdx.x < TILE_NODES && i < g.nnx && j < g.nny) {
    double yu, yv;
    gather_node(eo, li, lj, 0, yu, yv);
    const size_t o = vb + 2 * ((size_t)j * g.nnx + i);
    if (!raw) {
      const double2 xv = *reinterpret_cast<const double2 *>(x + o);
      if (i == 0) { yu = xv.x; yv = xv.y; }
      if (i == g.nx) yu = xv.x;
    }
    *reinterpret_cast<double2 *>(y + o) = make_double2(yu, yv);
  }
}

// ---------------------------------------------------------------- PCG set-up
// b = -P K g and dg = diag(P K P + I - P); x = 0, z = dinv b (dinv = 1/dg);
// b and dinv also to b_out / dinv_out when given; slot marked active at
// iteration 0.
__global__ __launch_bounds__(TILE_THREADS) void k_setup(StripGeom g, StripMat m, PcgSlots S,
                                                        double *__restrict__ b_out, double *__restrict__ dinv_out) {
  __shared__ double eo[16][TILE_ELEMS];
  const int s = blockIdx.y, t = blockIdx.x;
  const TileCoord tc = tile_of(g, t);
  const double *ang_s = (const double *)S.theta + (size_t)s * (S.cs ? 8 : 4) * g.nelem;
  for (int k = threadIdx.x; k < TILE_ELEMS; k += TILE_THREADS) {
    const int lex = k % ELEM_X, ley = k / ELEM_X;
    const int ex = tc.i0 - 1 + lex, ey = tc.j0 - 1 + ley;
    double du[4] = {0, 0, 0, 0}, dv[4] = {0, 0, 0, 0}, gu[4] = {0, 0, 0, 0}, gv[4] = {0, 0, 0, 0};
    if (elem_in(g, ex, ey)) {
      double2 cp[4];
      elem_cs(ang_s, S.cs, (size_t)ey * g.nx + ex, cp);
      Qb q[4] = {qbar_cs(m, cp[0].y, cp[0].x), qbar_cs(m, cp[1].y, cp[1].x), qbar_cs(m, cp[2].y, cp[2].x),
                 qbar_cs(m, cp[3].y, cp[3].x)};
      // diagonal entries: the element operator applied to unit vectors
      for (int a = 0; a < 4; ++a) {
        double u[4] = {0, 0, 0, 0}, v[4] = {0, 0, 0, 0}, fu[4], fv[4];
        u[a] = 1.0;
        elem_forces(g, q, u, v, fu, fv);
        du[a] = fu[a];
        u[a] = 0.0;
        v[a] = 1.0;
        elem_forces(g, q, u, v, fu, fv);
        dv[a] = fv[a];
      }
      // K g on elements touching the loaded edge (nodes 1 and 2 at x = Lx)
      if (ex == g.nx - 1) {
        const double u[4] = {0.0, -g.delta, -g.delta, 0.0}, v[4] = {0, 0, 0, 0};
        elem_forces(g, q, u, v, gu, gv);
      }
    }
    for (int c = 0; c < 4; ++c) {
      eo[c][k] = du[c];
      eo[4 + c][k] = dv[c];
      eo[8 + c][k] = gu[c];
      eo[12 + c][k] = gv[c];
    }
  }
  __syncthreads();
  const int li = threadIdx.x % TILE_X, lj = threadIdx.x / TILE_X;
  const int i = tc.i0 + li, j = tc.j0 + lj;
  if (threadIdx.x < TILE_NODES && i < g.nnx && j < g.nny) {
    double diu, div, kgu, kgv;
    gather_node(eo, li, lj, 0, diu, div);
    gather_node(eo, li, lj, 8, kgu, kgv);
    double bu = -kgu, bv = -kgv, gu = diu, gv = div;
    if (i == 0) { bu = 0.0; bv = 0.0; gu = 1.0; gv = 1.0; }
    if (i == g.nx) { bu = 0.0; gu = 1.0; }
    const double du = 1.0 / gu, dv = 1.0 / gv;
    const size_t o = (size_t)s * 2 * g.nnode + 2 * ((size_t)j * g.nnx + i);
    *reinterpret_cast<double2 *>(S.dg + o) = make_double2(gu, gv);
    *reinterpret_cast<double2 *>(S.z + o) = make_double2(du * bu, dv * bv);
    *reinterpret_cast<double2 *>(S.x + o) = make_double2(0.0, 0.0);
    if (b_out) *reinterpret_cast<double2 *>(b_out + o) = make_double2(bu, bv);
    if (dinv_out) *reinterpret_cast<double2 *>(dinv_out + o) = make_double2(du, dv);
  }
  if (t == 0 && threadIdx.x == 0) {
    S.it_a[s] = 0;
    S.status[s] = S_OK;
    S.active[s] = 1;
    S.xs[S.S + s] = 0;
  }
}

// initial partial sums of r.z and r.r (r = dg z) per vector-pass chunk, into
// parity buffer 0
__global__ __launch_bounds__(256) void k_init_partials(StripGeom g, PcgSlots S) {
  __shared__ double red4[4];
  const int s = blockIdx.y, c = blockIdx.x;
  const size_t vb = (size_t)s * 2 * g.nnode;
  double prz = 0.0, prr = 0.0;
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int node = c * CHUNK + k * 256 + threadIdx.x;
    if (node < g.nnode) {
      const double2 zv = *reinterpret_cast<const double2 *>(S.z + vb + 2 * (size_t)node);
      const double2 gv = *reinterpret_cast<const double2 *>(S.dg + vb + 2 * (size_t)node);
      const double ru = gv.x * zv.x, rv = gv.y * zv.y;
      prz += ru * zv.x + rv * zv.y;
      prr += ru * ru + rv * rv;
    }
  }
  prz = block_sum(prz, red4);
  prr = block_sum(prr, red4);
  if (threadIdx.x == 0) {
    S.part_rz[(size_t)s * g.nchunks + c] = prz;
    S.part_rr[(size_t)s * g.nchunks + c] = prr;
  }
}

// blocks are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous range of logical blocks so tiles that share halo rows and columns
// (neighbours of the same sample) meet in the same L2
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

template <typename T>
struct PairOf;
template <>
struct PairOf<double> {
  using type = double2;
};
template <>
struct PairOf<float> {
  using type = float2;
};

template <typename T>
__device__ __forceinline__ typename PairOf<T>::type ld2(const T *p) {
  return gload<typename PairOf<T>::type>(p);
}
template <typename T>
__device__ __forceinline__ void st2(T *p, T a, T b) {
  typename PairOf<T>::type v;
  v.x = a;
  v.y = b;
  gstore(p, v);
}
// Streaming forms (NT): nontemporal accesses, which do not displace what the
// caches hold.  Used when a launch's working set is larger than the Infinity
// Cache, so that the angles and the node rows the operator pass has just read
// stay cached while the vectors stream past them.
template <bool NT, typename T>
__device__ __forceinline__ typename PairOf<T>::type ld2s(const T *p) {
  using V = typename PairOf<T>::type;
  if constexpr (NT) return NativeOf<V>::from(__builtin_nontemporal_load((const MLMC_GLOBAL typename NativeOf<V>::type *)p));
  else return gload<V>(p);
}
template <bool NT, typename T>
__device__ __forceinline__ void st2s(T *p, T a, T b) {
  using V = typename PairOf<T>::type;
  V v;
  v.x = a;
  v.y = b;
  if constexpr (NT) __builtin_nontemporal_store(NativeOf<V>::to(v), (MLMC_GLOBAL typename NativeOf<V>::type *)p);
  else gstore(p, v);
}

// z and p_old of node (i, jr).  The loads are issued for every lane, from the
// nearest node inside the mesh, with no branch: the wait for the current row
// then covers exactly the loads issued before it and leaves the next row's in
// flight.  Values of nodes outside the mesh or the window are never used
// (their elements are skipped and their nodes not owned).  p is formed where
// the row is used, not here, for the same reason.
template <typename T>
struct RowVals {
  T zu, zv, qu, qv;
  // p = z + beta p_old (p_old = 0 before the first iteration, wp false)
  __device__ __forceinline__ T pu(T beta, bool wp) const { return fma(beta, wp ? qu : T(0), zu); }
  __device__ __forceinline__ T pv(T beta, bool wp) const { return fma(beta, wp ? qv : T(0), zv); }
};

__device__ __forceinline__ int clampi(int v, int hi) { return min(max(v, 0), hi); }

template <typename T>
__device__ __forceinline__ RowVals<T> load_row(const StripGeom &g, const PcgState<T> &S, size_t vb, int ic, int jr) {
  const size_t o = vb + 2 * ((size_t)clampi(jr, g.nny - 1) * g.nnx + ic);
  const auto zv = ld2(S.z + o);
  const auto po = ld2(S.p + o);  // not written before the first iteration: not used there
  RowVals<T> v;
  v.zu = zv.x;
  v.zv = zv.y;
  v.qu = po.x;
  v.qv = po.y;
  return v;
}

// the four Gauss-point angles of element (ic, ey) and the rotated stiffness at
// one of them.  FP64: CSM = 1 reads stored (cos 2theta, sin 2theta) pairs
// (64 B per element), CSM = 0 reads the angle codes tan theta (32 B) and
// evaluates the pairs one Gauss point at a time; both give the same bits.  As for the rows, the
// loads are unconditional (ic is clamped by the caller, ey here) and the values
// of elements outside the mesh are never used.
template <typename T, int CSM = 0>
struct Angles;
template <>
struct Angles<double, 1> {
  double2 cs[4];
  __device__ __forceinline__ void load(const void *theta, size_t eb, const StripGeom &g, int ic, int ey, int = 0) {
    const double2 *cp = (const double2 *)theta + 4 * (eb + (size_t)clampi(ey, g.ny - 1) * g.nx + ic);
#pragma unroll
    for (int q = 0; q < 4; ++q) cs[q] = gload<double2>(cp + q);
  }
  __device__ __forceinline__ QbT<double> qb(const StripMat &m, int q) const { return qbar_cs(m, cs[q].y, cs[q].x); }
};
template <>
struct Angles<double, 0> {
  double t[4];
  __device__ __forceinline__ void load(const void *theta, size_t eb, const StripGeom &g, int ic, int ey, int = 0) {
    const double *tp = (const double *)theta + 4 * (eb + (size_t)clampi(ey, g.ny - 1) * g.nx + ic);
    const double2 a = gload<double2>(tp);
    const double2 b = gload<double2>(tp + 2);
    t[0] = a.x; t[1] = a.y; t[2] = b.x; t[3] = b.y;
  }
  __device__ __forceinline__ QbT<double> qb(const StripMat &m, int q) const {
    double s2, c2;
    cs_of_code(t[q], &s2, &c2);
    return qbar_cs(m, s2, c2);
  }
};
template <>
struct Angles<float, 0> {
  uint2 w;  // two bfloat16 angles per word, decoded at use
  __device__ __forceinline__ void load(const void *theta, size_t eb, const StripGeom &g, int ic, int ey, int = 0) {
    w = gload<uint2>((const uint16_t *)theta + 4 * (eb + (size_t)clampi(ey, g.ny - 1) * g.nx + ic));
  }
  __device__ __forceinline__ QbT<float> qb(const StripMat &m, int q) const {
    const uint32_t h = (q >> 1) ? w.y : w.x;
    return qbar_f32(m, __uint_as_float((q & 1) ? (h & 0xFFFF0000u) : (h << 16)));
  }
};
template <>
struct Angles<float, 1> {
  float4 t;  // FP32 angles
  __device__ __forceinline__ void load(const void *theta, size_t eb, const StripGeom &g, int ic, int ey, int = 0) {
    t = gload<float4>((const float *)theta + 4 * (eb + (size_t)clampi(ey, g.ny - 1) * g.nx + ic));
  }
  __device__ __forceinline__ QbT<float> qb(const StripMat &m, int q) const {
    return qbar_f32(m, q == 0 ? t.x : q == 1 ? t.y : q == 2 ? t.z : t.w);
  }
};

// ---------------------------------------------------------------- PCG pass 1
// Iteration `it` (all slots of a batch iterate in lock-step; par = it & 1).
// One wave per column-sweep tile: lane l holds node column i0 - 1 + l (lanes
// 1..TW own their column, lanes 0 and TW + 1 are halo) and the element whose
// lower-left node is that column.  The wave walks up the element rows; the
// right neighbour's nodal values and the left neighbour's element forces come
// from lane shuffles, the previous row's forces stay in registers, and every
// owned node's four contributions are summed in the fixed order
// ((e(i-1,j-1).f2 + e(i,j-1).f3) + e(i-1,j).f1) + e(i,j).f0.
// Per sample: convergence test on r.r, beta = rz_it / rz_{it-1},
// p = z + beta p_old (not stored: pass 2 recomputes it bit-identically, so
// neighbours read p_old in their halos), Ap = A p, partial p.Ap per tile.
// The next node row is loaded while the current row is computed.  Dot
// products are accumulated in FP64 for both precisions.  NT: Ap is stored
// with streaming stores.
template <typename T, int CSM, bool NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_pass1(const PcgGroup<T> *__restrict__ G, int ng, StripMat m, int it_off,
                                             int nblocks, const int *__restrict__ itb) {
  const int it = itb ? __builtin_amdgcn_readfirstlane(*itb) + it_off : it_off;
  const int lb = xcd_remap(blockIdx.x, nblocks);
  int gi = 0;
  for (int k = 1; k < ng; ++k)
    if (lb >= G[k].blk0) gi = k;
  gi = __builtin_amdgcn_readfirstlane(gi);
  const StripGeom g = G[gi].g;
  const PcgState<T> S = G[gi].S;
  const int lt = lb - G[gi].blk0;
  const int s = lt / g.sw_ntiles, t = lt - s * g.sw_ntiles;
  const int lane = threadIdx.x;
  const int par = it & 1;
  const size_t vb = (size_t)s * 2 * g.nnode;
  const size_t eb = (size_t)s * g.nelem;   // first element of the sample
  const int active = __builtin_amdgcn_readfirstlane(S.active[s]);
  const size_t pb = ((size_t)par * S.S + s) * g.nchunks;
  double prz = 0.0, prr = 0.0;
  for (int k = lane; k < g.nchunks; k += 64) {
    prz += S.part_rz[pb + k];
    prr += S.part_rr[pb + k];
  }
  const double rz_prev = (it > 0) ? S.rzs[(size_t)(par ^ 1) * S.S + s] : 1.0;
  const double bb_old = (it > 0) ? S.bb[s] : 0.0;
  const double rr_ref = (S.mixed && it > 0) ? S.rr_ref[s] : 0.0;
  const int tx = t % g.sw_ntx, ty = t / g.sw_ntx;
  const int i0 = tx * g.sw_tw, j0 = ty * g.sw_ty;
  const int i = i0 - 1 + lane;
  const bool elv = lane <= g.sw_tw && i >= 0 && i < g.nx;
  const bool own = lane >= 1 && lane <= g.sw_tw && i < g.nnx;
  const int row_end = (ty == g.sw_nty - 1) ? g.nny : j0 + g.sw_ty;  // the last tile takes the remainder
  const bool wp = it > 0;
  const int ic = clampi(i, g.nnx - 1), ice = clampi(i, g.nx - 1);  // nearest node / element column
  RowVals<T> lo = load_row(g, S, vb, ic, j0 - 1);
  RowVals<T> nhi = load_row(g, S, vb, ic, j0);
  const double rz = wave_sum(prz);
  if (!active) return;
  const double rr = wave_sum(prr);
  const double bb = (it == 0) ? rr : bb_old;
  const double tol2 = S.rtol2 * bb;
  int verdict = -1;
  bool upd = false;
  if (!isfinite(rr) || !isfinite(rz)) verdict = S_NAN;
  else if (it >= S.max_iter) verdict = S_NOCONV;
  // mixed: ask for an FP64 residual when the FP32 one has fallen by the update
  // factor, or is 10% below the stopping threshold (the margin keeps a slot
  // whose FP64 residual just failed the test from asking again at once)
  else if (S.mixed) upd = rr <= 0.81 * tol2 || (it > 0 && rr <= S.ru2 * rr_ref);
  else if (rr <= tol2) verdict = S_OK;
  if (t == 0 && lane == 0) {
    if (it == 0) {
      S.bb[s] = rr;
      if (S.mixed) S.rr_ref[s] = rr;
    }
    // a paused iteration keeps the last r.z so beta stays consistent with p
    S.rzs[(size_t)par * S.S + s] = (upd && it > 0) ? rz_prev : rz;
    S.relres[s] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    S.it_b[s] = it;
    if (verdict >= 0) {
      S.status[s] = verdict;
      S.active[s] = 0;
    }
    if (upd) {
      S.ru[s] = it + 1;
      S.active[s] = 0;
    }
    if (sizeof(T) == 4 && verdict < 0 && !upd) {  // FP32 inner solver: state for this vector pass
      S.xs[s] = S.xs[S.S + s];
      S.xa[s] = S.xa[S.S + s];
    }
  }
  if (verdict >= 0 || upd) return;
  const double beta_d = (it == 0) ? 0.0 : rz / rz_prev;
  const T beta = (T)beta_d;
  T plu = lo.pu(beta, wp), plv = lo.pv(beta, wp);
  T f2u = 0, f2v = 0, f3u = 0, f3v = 0;  // previous element row: f2 of the left lane, own f3
  T yu = 0, yv = 0;                      // A p of the last node row, stored one row late
  double part = 0.0;
  const int nk = row_end - j0;
  // the next element row's angle codes are loaded one row ahead (not the
  // pairs: they would cost the fourth wave per SIMD)
  constexpr bool ahead = CSM == 0 && sizeof(T) == 8;
  Angles<T, CSM> nth;
  if (ahead) nth.load(S.theta, eb, g, ice, j0 - 1);
  // One node row per step.  Memory operations are issued in a fixed order and
  // without branches around them: the store of the previous row, this row's
  // angles, the next row's values.  Each wait then covers exactly what it
  // needs; the last step, which prefetches nothing, is a separate copy.
  auto step = [&](const int k, auto prefetch) {
    const int ey = j0 - 1 + k;
    // everything issued by the previous step has arrived: its prefetch and the
    // store before it (vmcnt 0; expcnt and lgkmcnt not waited for)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    if (k >= 2 && own) st2s<NT>(S.Ap + vb + 2 * ((size_t)(ey - 1) * g.nnx + i), yu, yv);
    const RowVals<T> hi = nhi;
    Angles<T, CSM> th;
    if constexpr (ahead) th = nth;
    else th.load(S.theta, eb, g, ice, ey);
    // keep this row's angle loads ahead of the prefetch, so that waiting for
    // them does not wait for the next row
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (decltype(prefetch)::value) {
      nhi = load_row(g, S, vb, ic, ey + 2);
      if constexpr (ahead) nth.load(S.theta, eb, g, ice, ey + 1);
    }
    const T phu = hi.pu(beta, wp), phv = hi.pv(beta, wp);
    const T rlu = __shfl_down(plu, 1, 64), rlv = __shfl_down(plv, 1, 64);
    const T rhu = __shfl_down(phu, 1, 64), rhv = __shfl_down(phv, 1, 64);
    T fu[4] = {0, 0, 0, 0}, fv[4] = {0, 0, 0, 0};
    if (elv && ey >= 0 && ey < g.ny) {
      const T u[4] = {plu, rlu, rhu, phu};
      const T v[4] = {plv, rlv, rhv, phv};
      elem_forces_q<T>(g, [&](int q) { return th.qb(m, q); }, u, v, fu, fv);
    }
    const T f1lu = __shfl_up(fu[1], 1, 64), f1lv = __shfl_up(fv[1], 1, 64);
    if (k >= 1 && own) {
      yu = ((f2u + f3u) + f1lu) + fu[0];
      yv = ((f2v + f3v) + f1lv) + fv[0];
      if (i == 0) { yu = plu; yv = plv; }
      if (i == g.nx) yu = plu;
      part += (double)plu * (double)yu + (double)plv * (double)yv;
    }
    // close a block of SWEEP_RB node rows: one partial per (row block, column tile)
    if (k >= 1 && ((ey + 1) % SWEEP_RB == 0 || ey + 1 == row_end)) {
      const double ps = wave_sum(part);
      if (lane == 0) gstore(S.part_pap + (size_t)s * g.sw_npart + (ey / SWEEP_RB) * g.sw_ntx + tx, ps);
      part = 0.0;
    }
    f2u = __shfl_up(fu[2], 1, 64);
    f2v = __shfl_up(fv[2], 1, 64);
    f3u = fu[3];
    f3v = fv[3];
    plu = phu;
    plv = phv;
  };
  for (int k = 0; k < nk; ++k) step(k, std::true_type{});
  step(nk, std::false_type{});
  if (nk >= 1 && own) st2s<NT>(S.Ap + vb + 2 * ((size_t)(row_end - 1) * g.nnx + i), yu, yv);
}

// ---------------------------------------------------------------- PCG pass 2
// alpha = rz / p.Ap; p = z + beta p_old (bit-identical to pass 1); x += alpha p;
// r = dg z - alpha Ap; z = r / dg; store p, x, z; partial r.z and r.r per
// chunk of CHUNK consecutive nodes (all loads issued before the reduction of
// p.Ap).  x moves at every second pass only, by both steps in the order of one
// step at a time (the deferred step's p is this pass's p_old), so x is read
// and written half as often with the same bits.  NT: streaming loads of Ap,
// x and dg and streaming stores; z and p_old, which pass 1 has just read,
// are loaded as cached data.
template <typename T, bool NT>
__global__ __launch_bounds__(256) void k_pass2(const PcgGroup<T> *__restrict__ G, int ng, int it_off,
                                              const int *__restrict__ itb) {
  const int it = itb ? __builtin_amdgcn_readfirstlane(*itb) + it_off : it_off;
  constexpr int PER = CHUNK / 256;
  using P2 = typename PairOf<T>::type;
  __shared__ double red4[4];
  __shared__ int flag;
  int gi = 0;
  for (int k = 1; k < ng; ++k)
    if ((int)blockIdx.x >= G[k].cblk0) gi = k;
  gi = __builtin_amdgcn_readfirstlane(gi);
  const StripGeom g = G[gi].g;
  const PcgState<T> S = G[gi].S;
  const int lb = blockIdx.x - G[gi].cblk0;
  const int s = lb / g.nchunks, c = lb - s * g.nchunks;
  const int par = it & 1;
  if (threadIdx.x == 0) flag = S.active[s];
  double ppap = 0.0;
  for (int k = threadIdx.x; k < g.sw_npart; k += 256) ppap += S.part_pap[(size_t)s * g.sw_npart + k];
  const double rz = S.rzs[(size_t)par * S.S + s];
  const double rz_prev = (it > 0) ? S.rzs[(size_t)(par ^ 1) * S.S + s] : 1.0;
  // a step is pending: this pass moves x by both.  The FP64 solver never
  // pauses: it defers at even iterations and keeps that step's alpha in
  // xa[0][s], so the pattern is known without a load.  The FP32 inner
  // solver's reliable updates can shift it: there pass 1 copies the state.
  const bool xstep = (sizeof(T) == 8) ? (it & 1) != 0 : S.xs[s] != 0;
  const T alpha_prev = xstep ? (T)S.xa[s] : T(0);
  const size_t vb = (size_t)s * 2 * g.nnode;
  P2 pv[PER], av[PER], xv[PER], zv[PER], gv[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int node = c * CHUNK + k * 256 + threadIdx.x;
    pv[k].x = pv[k].y = av[k].x = av[k].y = xv[k].x = xv[k].y = zv[k].x = zv[k].y = T(0);
    gv[k].x = gv[k].y = T(1);
    if (node < g.nnode) {
      const size_t o = vb + 2 * (size_t)node;
      if (it > 0) pv[k] = ld2(S.p + o);
      av[k] = ld2s<NT>(S.Ap + o);
      if (xstep) xv[k] = ld2s<NT>(S.x + o);
      zv[k] = ld2(S.z + o);
      gv[k] = ld2s<NT>(S.dg + o);
    }
  }
  const double pap = block_sum(ppap, red4);  // publishes flag
  if (!flag) return;
  if (!(pap > 0.0) || !isfinite(pap)) {
    if (c == 0 && threadIdx.x == 0) {
      S.status[s] = isfinite(pap) ? S_BREAKDOWN : S_NAN;
      S.active[s] = 0;
    }
    return;
  }
  const T alpha = (T)(rz / pap);
  const T beta = (T)((it == 0) ? 0.0 : rz / rz_prev);
  double prz = 0.0, prr = 0.0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int node = c * CHUNK + k * 256 + threadIdx.x;
    if (node < g.nnode) {
      const size_t o = vb + 2 * (size_t)node;
      const T pnx = fma(beta, pv[k].x, zv[k].x);
      const T pny = fma(beta, pv[k].y, zv[k].y);
      const T rx = fma(-alpha, av[k].x, gv[k].x * zv[k].x), ry = fma(-alpha, av[k].y, gv[k].y * zv[k].y);
      const T znx = rx * rcp_nr(gv[k].x), zny = ry * rcp_nr(gv[k].y);
      st2s<NT>(S.p + o, pnx, pny);
      if (xstep) {
        const T xx = fma(alpha_prev, pv[k].x, xv[k].x), xy = fma(alpha_prev, pv[k].y, xv[k].y);
        st2s<NT>(S.x + o, fma(alpha, pnx, xx), fma(alpha, pny, xy));
      }
      st2s<NT>(S.z + o, znx, zny);
      const double drx = rx, dry = ry;
      prz += drx * (double)znx + dry * (double)zny;
      prr += drx * drx + dry * dry;
    }
  }
  prz = block_sum(prz, red4);
  prr = block_sum(prr, red4);
  if (threadIdx.x == 0) {
    const size_t pb = ((size_t)(par ^ 1) * S.S + s) * g.nchunks + c;
    S.part_rz[pb] = prz;
    S.part_rr[pb] = prr;
    if (c == 0) {
      S.it_a[s] = it + 1;
      S.xs[S.S + s] = xstep ? 0 : 1;
      if (sizeof(T) == 4) S.xa[S.S + s] = (double)alpha;
      else if (!xstep) S.xa[s] = (double)alpha;  // read by the next (odd) pass only
    }
  }
}

// x += alpha p for slots whose last completed vector pass left its step
// pending (FP64 solver, after the iterations)
__global__ __launch_bounds__(256) void k_x_flush(StripGeom g, PcgSlots S) {
  const int s = blockIdx.y, c = blockIdx.x;
  if (!S.xs[S.S + s]) return;
  const double alpha = S.xa[s];  // FP64: the deferred step's alpha
  const size_t vb = (size_t)s * 2 * g.nnode;
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int node = c * CHUNK + k * 256 + threadIdx.x;
    if (node < g.nnode) {
      const size_t o = vb + 2 * (size_t)node;
      const double2 pv = *reinterpret_cast<const double2 *>(S.p + o);
      double2 xv = *reinterpret_cast<const double2 *>(S.x + o);
      xv.x = fma(alpha, pv.x, xv.x);
      xv.y = fma(alpha, pv.y, xv.y);
      *reinterpret_cast<double2 *>(S.x + o) = xv;
    }
  }
}

// ---------------------------------------------------------------- mixed precision
// Reliable update of slot s (requested by pass 1 of iteration it): the FP64
// residual r = b - A (x64 + x32) with the FP64 angles (column sweep as in
// pass 1, node values = x), stored preconditioned (z64 = r / dg); partial
// ||r||^2 per sweep tile.
__global__ __launch_bounds__(64) void k_resid64(StripGeom g, StripMat m, PcgSlots D, PcgState<float> I, MixedState M,
                                                int it_off, int every, int nblocks, const int *__restrict__ itb) {
  const int it = itb ? __builtin_amdgcn_readfirstlane(*itb) + it_off : it_off;
  const int lt = xcd_remap(blockIdx.x, nblocks);
  const int s = lt / g.sw_ntiles, t = lt - s * g.sw_ntiles;
  const int lane = threadIdx.x;
  // slots that asked during the last `every` iterations (each is served once)
  const int ask = __builtin_amdgcn_readfirstlane(I.ru[s]);
  if (ask < it + 2 - every || ask > it + 1) return;
  const size_t vb = (size_t)s * 2 * g.nnode;
  const size_t eb = (size_t)s * g.nelem;   // first element of the sample
  const int tx = t % g.sw_ntx, ty = t / g.sw_ntx;
  const int i0 = tx * g.sw_tw, j0 = ty * g.sw_ty;
  const int i = i0 - 1 + lane;
  const bool colv = lane <= g.sw_tw + 1 && i >= 0 && i < g.nnx;
  const bool elv = lane <= g.sw_tw && i >= 0 && i < g.nx;
  const bool own = lane >= 1 && lane <= g.sw_tw && i < g.nnx;
  const int row_end = (ty == g.sw_nty - 1) ? g.nny : j0 + g.sw_ty;  // the last tile takes the remainder
  // x = x64 + x32, with the inner solver's pending step (if any) added to x32
  // as the next vector pass would add it
  const bool pend = I.xs[I.S + s] != 0;
  const float xa = (float)I.xa[I.S + s];
  if (t == 0 && lane == 0) {  // for the fold-in that follows (it must not read what it writes)
    I.xs[s] = pend ? 1 : 0;
    I.xa[s] = I.xa[I.S + s];
  }
  auto xrow = [&](int jr, double &a, double &b) {
    a = b = 0.0;
    if (colv && jr >= 0 && jr < g.nny) {
      const size_t o = vb + 2 * ((size_t)jr * g.nnx + i);
      const double2 v = *reinterpret_cast<const double2 *>(D.x + o);
      float2 d = *reinterpret_cast<const float2 *>(I.x + o);
      if (pend) {
        const float2 pp = *reinterpret_cast<const float2 *>(I.p + o);
        d.x = fmaf(xa, pp.x, d.x);
        d.y = fmaf(xa, pp.y, d.y);
      }
      a = v.x + (double)d.x;
      b = v.y + (double)d.y;
    }
  };
  double plu, plv, nhu, nhv;
  xrow(j0 - 1, plu, plv);
  xrow(j0, nhu, nhv);
  double f2u = 0, f2v = 0, f3u = 0, f3v = 0, part = 0.0;
  const int nk = row_end - j0;
  for (int k = 0; k <= nk; ++k) {
    const int ey = j0 - 1 + k;
    const double phu = nhu, phv = nhv;
    double2 csq[4];
    if (elv && ey >= 0 && ey < g.ny) {
      elem_cs((const double *)D.theta + (D.cs ? 8 : 4) * eb, D.cs, (size_t)ey * g.nx + i, csq);
    } else {
      for (int q = 0; q < 4; ++q) csq[q] = make_double2(1.0, 0.0);
    }
    if (k < nk) xrow(ey + 2, nhu, nhv);
    const double rlu = __shfl_down(plu, 1, 64), rlv = __shfl_down(plv, 1, 64);
    const double rhu = __shfl_down(phu, 1, 64), rhv = __shfl_down(phv, 1, 64);
    double fu[4] = {0, 0, 0, 0}, fv[4] = {0, 0, 0, 0};
    if (elv && ey >= 0 && ey < g.ny) {
      const double u[4] = {plu, rlu, rhu, phu};
      const double v[4] = {plv, rlv, rhv, phv};
      elem_forces_q<double>(g, [&](int q) { return qbar_cs(m, csq[q].y, csq[q].x); }, u, v, fu, fv);
    }
    const double f1lu = __shfl_up(fu[1], 1, 64), f1lv = __shfl_up(fv[1], 1, 64);
    if (k >= 1 && own) {
      double yu = ((f2u + f3u) + f1lu) + fu[0];
      double yv = ((f2v + f3v) + f1lv) + fv[0];
      if (i == 0) { yu = plu; yv = plv; }
      if (i == g.nx) yu = plu;
      const size_t o = vb + 2 * ((size_t)ey * g.nnx + i);
      const double2 bv = *reinterpret_cast<const double2 *>(M.b + o);
      const double2 gv = *reinterpret_cast<const double2 *>(D.dg + o);
      const double ru = bv.x - yu, rv = bv.y - yv;
      *reinterpret_cast<double2 *>(D.z + o) = make_double2(ru * rcp_nr(gv.x), rv * rcp_nr(gv.y));
      part += ru * ru + rv * rv;
    }
    if (k >= 1 && ((ey + 1) % SWEEP_RB == 0 || ey + 1 == row_end)) {
      const double ps = wave_sum(part);
      if (lane == 0) M.part_rr[(size_t)s * g.sw_npart + (ey / SWEEP_RB) * g.sw_ntx + tx] = ps;
      part = 0.0;
    }
    f2u = __shfl_up(fu[2], 1, 64);
    f2v = __shfl_up(fv[2], 1, 64);
    f3u = fu[3];
    f3v = fv[3];
    plu = phu;
    plv = phv;
  }
}

// Second half of a reliable update: x64 += x32 (with a pending inner step),
// x32 = 0, z32 = z64; the FP64
// stopping test ||r|| <= rtol ||b||; the inner partial sums for the next
// iteration (parity of it + 1) and the slot's restart.
__global__ __launch_bounds__(256) void k_ru_apply(StripGeom g, PcgSlots D, PcgState<float> I, MixedState M, int it_off,
                                                  int every, const int *__restrict__ itb) {
  const int it = itb ? __builtin_amdgcn_readfirstlane(*itb) + it_off : it_off;
  __shared__ double red4[4];
  __shared__ int flag;
  const int s = blockIdx.y, c = blockIdx.x;
  if (threadIdx.x == 0) {
    const int ask = I.ru[s];
    flag = ask >= it + 2 - every && ask <= it + 1;
  }
  double prr = 0.0, pbb = 0.0;
  for (int k = threadIdx.x; k < g.sw_npart; k += 256) prr += M.part_rr[(size_t)s * g.sw_npart + k];
  for (int k = threadIdx.x; k < g.nchunks; k += 256) pbb += M.part_bb[(size_t)s * g.nchunks + k];
  const double rr = block_sum(prr, red4);
  if (!flag) return;
  const double bb = block_sum(pbb, red4);
  const bool done = !(rr > M.rtol2 * bb);
  const size_t vb = (size_t)s * 2 * g.nnode;
  const bool pend = I.xs[s] != 0;  // pending inner step, as the residual kernel saw it
  const float xa = (float)I.xa[s];
  double prz = 0.0, pr2 = 0.0;
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int node = c * CHUNK + k * 256 + threadIdx.x;
    if (node < g.nnode) {
      const size_t o = vb + 2 * (size_t)node;
      float2 d = *reinterpret_cast<const float2 *>(I.x + o);
      if (pend) {
        const float2 pp = *reinterpret_cast<const float2 *>(I.p + o);
        d.x = fmaf(xa, pp.x, d.x);
        d.y = fmaf(xa, pp.y, d.y);
      }
      double2 x = *reinterpret_cast<const double2 *>(D.x + o);
      x.x += (double)d.x;
      x.y += (double)d.y;
      *reinterpret_cast<double2 *>(D.x + o) = x;
      *reinterpret_cast<float2 *>(I.x + o) = make_float2(0.0f, 0.0f);
      const double2 zv = *reinterpret_cast<const double2 *>(D.z + o);
      const float2 z32 = make_float2((float)zv.x, (float)zv.y);
      *reinterpret_cast<float2 *>(I.z + o) = z32;
      const float2 g32 = *reinterpret_cast<const float2 *>(I.dg + o);
      const double a = g32.x * z32.x, b = g32.y * z32.y;  // r as the inner vector pass forms it
      prz += a * (double)z32.x + b * (double)z32.y;
      pr2 += a * a + b * b;
    }
  }
  prz = block_sum(prz, red4);
  pr2 = block_sum(pr2, red4);
  if (threadIdx.x == 0) {
    const size_t pb = ((size_t)((it + 1) & 1) * I.S + s) * g.nchunks + c;
    I.part_rz[pb] = prz;
    I.part_rr[pb] = pr2;
    if (c == 0) {
      I.xs[I.S + s] = 0;  // the pending step is in x64 now
      M.relres[s] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
      M.updates[s] += 1;
      I.rr_ref[s] = rr;
      if (!isfinite(rr)) I.status[s] = S_NAN;
      else if (done) I.status[s] = S_OK;
      I.active[s] = (done || !isfinite(rr)) ? 0 : 1;
    }
  }
}

// start of a mixed-precision solve (after the FP64 set-up): FP32 copies of
// z = dinv b and dg, x32 = 0, initial inner partial sums; slot flags
__global__ __launch_bounds__(256) void k_mixed_start(StripGeom g, PcgSlots D, PcgState<float> I, MixedState M) {
  __shared__ double red4[4];
  const int s = blockIdx.y, c = blockIdx.x;
  const size_t vb = (size_t)s * 2 * g.nnode;
  double prz = 0.0, pr2 = 0.0;
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int node = c * CHUNK + k * 256 + threadIdx.x;
    if (node < g.nnode) {
      const size_t o = vb + 2 * (size_t)node;
      const double2 zv = *reinterpret_cast<const double2 *>(D.z + o);
      const double2 gv = *reinterpret_cast<const double2 *>(D.dg + o);
      const float2 g32 = make_float2((float)gv.x, (float)gv.y);
      const float2 z32 = make_float2((float)zv.x, (float)zv.y);
      *reinterpret_cast<float2 *>(I.dg + o) = g32;
      *reinterpret_cast<float2 *>(I.z + o) = z32;
      *reinterpret_cast<float2 *>(I.x + o) = make_float2(0.0f, 0.0f);
      const double a = g32.x * z32.x, b = g32.y * z32.y;  // r as the inner vector pass forms it
      prz += a * (double)z32.x + b * (double)z32.y;
      pr2 += a * a + b * b;
    }
  }
  prz = block_sum(prz, red4);
  pr2 = block_sum(pr2, red4);
  if (threadIdx.x == 0) {
    I.part_rz[(size_t)s * g.nchunks + c] = prz;
    I.part_rr[(size_t)s * g.nchunks + c] = pr2;
    if (c == 0) {
      I.active[s] = 1;
      I.status[s] = S_OK;
      I.ru[s] = 0;
      I.xs[I.S + s] = 0;
      M.updates[s] = 0;
      M.relres[s] = 1.0;
    }
  }
}

// x64 += x32 for slots that stopped without a final reliable update
__global__ __launch_bounds__(256) void k_mixed_flush(StripGeom g, PcgSlots D, PcgState<float> I) {
  const int s = blockIdx.y, c = blockIdx.x;
  const size_t vb = (size_t)s * 2 * g.nnode;
  const bool pend = I.xs[I.S + s] != 0;
  const float xa = (float)I.xa[I.S + s];
  for (int k = 0; k < CHUNK / 256; ++k) {
    const int node = c * CHUNK + k * 256 + threadIdx.x;
    if (node < g.nnode) {
      const size_t o = vb + 2 * (size_t)node;
      float2 d = *reinterpret_cast<const float2 *>(I.x + o);
      if (pend) {
        const float2 pp = *reinterpret_cast<const float2 *>(I.p + o);
        d.x = fmaf(xa, pp.x, d.x);
        d.y = fmaf(xa, pp.y, d.y);
      }
      double2 x = *reinterpret_cast<const double2 *>(D.x + o);
      x.x += (double)d.x;
      x.y += (double)d.y;
      *reinterpret_cast<double2 *>(D.x + o) = x;
      *reinterpret_cast<float2 *>(I.x + o) = make_float2(0.0f, 0.0f);
    }
  }
}

// ---------------------------------------------------------------- QoI
// partial max of -sigma_11 over the Gauss points of the QoI-region elements
// (256 elements per block); final per-slot max written through an index map
__global__ __launch_bounds__(256) void k_qoi_part(StripGeom g, StripMat m, const double *__restrict__ ang, int csm,
                                                  const double *__restrict__ x, int nparts,
                                                  double *__restrict__ part) {
  __shared__ double red4[4];
  const int s = blockIdx.y;
  const int qw = g.qx1 - g.qx0, qh = g.qy1 - g.qy0;
  const int k = blockIdx.x * 256 + threadIdx.x;
  double best = -1.0 / 0.0;
  if (k < qw * qh) {
    const int ex = g.qx0 + k % qw, ey = g.qy0 + k / qw;
    const double *xs = x + (size_t)s * 2 * g.nnode;
    const int n0 = ey * g.nnx + ex;
    const int nd[4] = {n0, n0 + 1, n0 + g.nnx + 1, n0 + g.nnx};
    double u[4], v[4];
    for (int a = 0; a < 4; ++a) {
      const double2 d = *reinterpret_cast<const double2 *>(xs + 2 * (size_t)nd[a]);
      u[a] = d.x;
      v[a] = d.y;
    }
    // prescribed values are not stored in x: u = -delta on the loaded edge
    if (ex + 1 == g.nx) { u[1] = -g.delta; u[2] = -g.delta; }
    double2 cp[4];
    elem_cs(ang + (size_t)s * (csm ? 8 : 4) * g.nelem, csm, (size_t)ey * g.nx + ex, cp);
    const double c[8] = {cp[0].x, cp[0].y, cp[1].x, cp[1].y, cp[2].x, cp[2].y, cp[3].x, cp[3].y};
    best = elem_max_fibre_compression(g, m, c, u, v);
  }
  best = block_max(best, red4);
  if (threadIdx.x == 0) part[(size_t)s * nparts + blockIdx.x] = best;
}

// out_idx[s] < coarse_base: fine result of request out_idx[s]; otherwise the
// coarse result of request out_idx[s] - coarse_base
__global__ void k_qoi_final(const double *__restrict__ part, int nparts, int n, const int *__restrict__ out_idx,
                            double *__restrict__ q_fine, double *__restrict__ q_coarse, PcgSlots S,
                            mlmc_info_dev *__restrict__ info, int coarse_base) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double best = -1.0 / 0.0;
  for (int k = 0; k < nparts; ++k) best = fmax(best, part[(size_t)s * nparts + k]);
  int o = out_idx ? out_idx[s] : s;
  const bool coarse = o >= coarse_base;
  if (coarse) o -= coarse_base;
  double *q = coarse ? q_coarse : q_fine;
  if (q) q[o] = best;
  if (info) {
    if (coarse) {
      info[o].iters_c = S.it_b[s];
      info[o].relres_c = S.relres[s];
      info[o].status_c = S.status[s];
    } else {
      info[o].iters_f = S.it_b[s];
      info[o].relres_f = S.relres[s];
      info[o].status_f = S.status[s];
    }
  }
}

// total displacement d = x + g (g = -delta on the loaded-edge u)
__global__ void k_total_disp(StripGeom g, const double *__restrict__ x, double *__restrict__ d, int n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)n * 2 * g.nnode;
  if (k >= tot) return;
  const size_t node = (k / 2) % g.nnode;
  const int i = (int)(node % g.nnx);
  double v = x[k];
  if ((k & 1) == 0 && i == g.nx) v = -g.delta;
  d[k] = v;
}

__global__ void k_info_init(mlmc_info_dev *info, double *q_coarse, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  info[k].iters_f = 0;
  info[k].iters_c = 0;
  info[k].relres_f = 0.0;
  info[k].relres_c = 0.0;
  info[k].status_f = S_SKIPPED;
  info[k].status_c = S_SKIPPED;
  if (q_coarse) q_coarse[k] = 0.0;
}

// ---------------------------------------------------------------- level sums
// Neumaier-compensated FP64 sums in a fixed order: thread t takes entries
// t, t+256, ...; the 256 (sum, compensation) pairs are combined by a fixed
// tree with error-free additions.
struct Comp {
  double s, c;
};
__device__ __forceinline__ void neu_add(Comp &a, double v) {
  const double t = a.s + v;
  if (fabs(a.s) >= fabs(v)) a.c += (a.s - t) + v;
  else a.c += (v - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ Comp comp_merge(Comp a, Comp b) {
  Comp r = a;
  neu_add(r, b.s);
  r.c += b.c;
  return r;
}

__global__ __launch_bounds__(256) void k_level_stats(const double *__restrict__ qf, const double *__restrict__ qc,
                                                     int n, double lambda_star, int indicator,
                                                     double *__restrict__ out) {
  __shared__ Comp sh[4][256];
  __shared__ long long cnt[2][256];
  Comp a[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  long long np = 0, nm = 0;
  for (int k = threadIdx.x; k < n; k += 256) {
    double f = qf[k], c = qc ? qc[k] : 0.0;
    if (indicator) {
      f = (f < lambda_star) ? 1.0 : 0.0;
      if (qc) c = (c < lambda_star) ? 1.0 : 0.0;
    }
    const double y = f - c;
    neu_add(a[0], y);
    neu_add(a[1], y * y);
    neu_add(a[2], f);
    neu_add(a[3], c);
    np += (y > 0.5);
    nm += (y < -0.5);
  }
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = a[c];
  cnt[0][threadIdx.x] = np;
  cnt[1][threadIdx.x] = nm;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = comp_merge(sh[c][threadIdx.x], sh[c][threadIdx.x + w]);
      cnt[0][threadIdx.x] += cnt[0][threadIdx.x + w];
      cnt[1][threadIdx.x] += cnt[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int c = 0; c < 4; ++c) {
      out[2 * c] = sh[c][0].s;
      out[2 * c + 1] = sh[c][0].c;
    }
    out[8] = (double)cnt[0][0];
    out[9] = (double)cnt[1][0];
  }
}

// ---------------------------------------------------------------- launchers
static inline dim3 tile_grid(const StripGeom &g, int n) { return dim3(g.ntiles, n); }

void launch_kl_synth(const double *modes, int K, const StripGeom &g, const double *xi, int ld_xi,
                     const int64_t *rows, int n, double *th64, void *thlo, int lo_fp32, int ld_out, double *cs,
                     int code, hipStream_t st) {
  if (n <= 0) return;
  dim3 grid((4 * g.nelem + 255) / 256, (n + SYN_SAMPLES - 1) / SYN_SAMPLES);
  hipLaunchKernelGGL(k_kl_synth, grid, dim3(256), 0, st, modes, K, g, xi, ld_xi, rows, n, th64, thlo, lo_fp32, ld_out,
                     cs, code);
}

// (cos 2theta, sin 2theta) per Gauss point from given angles
__global__ void k_theta_cs(const double *__restrict__ th, double *__restrict__ cs, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s2, c2;
  cs_of_angle(th[k], &s2, &c2);
  *reinterpret_cast<double2 *>(cs + 2 * k) = make_double2(c2, s2);
}

// angle codes (tan theta) per Gauss point from given angles
__global__ void k_theta_code(const double *__restrict__ th, double *__restrict__ t, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) t[k] = angle_code(th[k]);
}

void launch_theta_code(const double *theta, double *code, size_t n, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_theta_code, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta, code, n);
}

void launch_theta_cs(const double *theta, double *cs, size_t n, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_theta_cs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta, cs, n);
}

void launch_modes_nystrom(const double *gx, const double *gy, const double *coef, int ngrid, int K, double var,
                          double kappa, const StripGeom &g, double *modes, hipStream_t st) {
  dim3 grid((4 * g.nelem + 255) / 256);
  hipLaunchKernelGGL(k_modes_nystrom, grid, dim3(256), 0, st, gx, gy, coef, ngrid, K, var, kappa, g, modes);
}

void launch_apply(const StripGeom &g, const StripMat &m, const double *theta, const double *x, double *y, int raw,
                  int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_apply, tile_grid(g, n), dim3(TILE_THREADS), 0, st, g, m, theta, x, y, raw);
}

void launch_setup(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, double *b_out, double *dinv_out,
                  hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_setup, tile_grid(g, n), dim3(TILE_THREADS), 0, st, g, m, S, b_out, dinv_out);
  hipLaunchKernelGGL(k_init_partials, dim3(g.nchunks, n), dim3(256), 0, st, g, S);
}

template <typename T>
void launch_pcg_pass1(const PcgGroup<T> *groups, int ng, int nblocks, const StripMat &m, int it, int cs,
                      const int *itb, hipStream_t st, bool nt) {
  // cs: stored (cos 2theta, sin 2theta) pairs (FP64), FP32 angles (FP32 solver)
  void (*f)(const PcgGroup<T> *, int, StripMat, int, int, const int *) =
      cs ? (nt ? k_pass1<T, 1, true> : k_pass1<T, 1, false>) : (nt ? k_pass1<T, 0, true> : k_pass1<T, 0, false>);
  hipLaunchKernelGGL(f, dim3(nblocks), dim3(64), 0, st, groups, ng, m, it, nblocks, itb);
}

template <typename T>
int pass1_resident_waves(int cs) {
  static std::atomic<int> cached[2];
  std::atomic<int> &v = cached[cs ? 1 : 0];
  if (v.load() == 0) {
    int dev = 0, ncu = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const void *f = cs ? (const void *)k_pass1<T, 1, false> : (const void *)k_pass1<T, 0, false>;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64, 0);
    (void)hipGetLastError();
    v.store(std::max(1, per_cu) * std::max(1, ncu));
  }
  return v.load();
}

template <typename T>
void launch_pcg_pass2(const PcgGroup<T> *groups, int ng, int nblocks, int it, const int *itb, hipStream_t st,
                      bool nt) {
  void (*f)(const PcgGroup<T> *, int, int, const int *) = nt ? k_pass2<T, true> : k_pass2<T, false>;
  hipLaunchKernelGGL(f, dim3(nblocks), dim3(256), 0, st, groups, ng, it, itb);
}

template void launch_pcg_pass1<double>(const PcgGroup<double> *, int, int, const StripMat &, int, int, const int *,
                                       hipStream_t, bool);
template void launch_pcg_pass1<float>(const PcgGroup<float> *, int, int, const StripMat &, int, int, const int *,
                                      hipStream_t, bool);
template int pass1_resident_waves<double>(int);
template int pass1_resident_waves<float>(int);
template void launch_pcg_pass2<double>(const PcgGroup<double> *, int, int, int, const int *, hipStream_t, bool);
template void launch_pcg_pass2<float>(const PcgGroup<float> *, int, int, int, const int *, hipStream_t, bool);

void launch_resid64(const StripGeom &g, const StripMat &m, const PcgSlots &D, const PcgState<float> &I,
                    const MixedState &M, int n, int it, int every, const int *itb, hipStream_t st) {
  const int nb = g.sw_ntiles * n;
  hipLaunchKernelGGL(k_resid64, dim3(nb), dim3(64), 0, st, g, m, D, I, M, it, every, nb, itb);
}

void launch_ru_apply(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, const MixedState &M, int n,
                     int it, int every, const int *itb, hipStream_t st) {
  hipLaunchKernelGGL(k_ru_apply, dim3(g.nchunks, n), dim3(256), 0, st, g, D, I, M, it, every, itb);
}

// iteration base of graph-replayed blocks: set, and advance after a block
__global__ void k_set_int(int *p, int v) {
  if (threadIdx.x == 0) *p = v;
}
__global__ void k_add_int(int *p, int v) {
  if (threadIdx.x == 0) *p += v;
}

// zero `words` 16-byte words at p (a kernel, not a memset node, so callers
// may capture it in a graph)
__global__ __launch_bounds__(256) void k_zero16(uint4 *p, size_t words) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += stride) p[k] = make_uint4(0, 0, 0, 0);
}

void launch_zero16(void *p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 16;
  if (!words) return;
  const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero16, dim3(blocks), dim3(256), 0, st, (uint4 *)p, words);
}

void launch_set_int(int *p, int v, hipStream_t st) { hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, p, v); }
void launch_add_int(int *p, int v, hipStream_t st) { hipLaunchKernelGGL(k_add_int, dim3(1), dim3(64), 0, st, p, v); }

void launch_mixed_start(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, const MixedState &M, int n,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_mixed_start, dim3(g.nchunks, n), dim3(256), 0, st, g, D, I, M);
}

void launch_x_flush(const StripGeom &g, const PcgSlots &S, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_x_flush, dim3(g.nchunks, n), dim3(256), 0, st, g, S);
}

void launch_mixed_flush(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_mixed_flush, dim3(g.nchunks, n), dim3(256), 0, st, g, D, I);
}

int qoi_parts(const StripGeom &g) { return ((g.qx1 - g.qx0) * (g.qy1 - g.qy0) + 255) / 256; }

void launch_qoi(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, double *part, const int *out_idx,
                double *q_fine, double *q_coarse, mlmc_info_dev *info, int coarse_base, hipStream_t st) {
  if (n <= 0) return;
  const int np = qoi_parts(g);
  hipLaunchKernelGGL(k_qoi_part, dim3(np, n), dim3(256), 0, st, g, m, (const double *)S.theta, S.cs, S.x, np, part);
  hipLaunchKernelGGL(k_qoi_final, dim3((n + 127) / 128), dim3(128), 0, st, part, np, n, out_idx, q_fine, q_coarse,
                     S, info, coarse_base);
}

void launch_total_disp(const StripGeom &g, const double *x, double *d, int n, hipStream_t st) {
  const size_t tot = (size_t)n * 2 * g.nnode;
  if (!tot) return;
  hipLaunchKernelGGL(k_total_disp, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g, x, d, n);
}

__global__ void k_to_lo(const double *__restrict__ a, void *__restrict__ b, int lo_fp32, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float f = (float)a[k];
  if (lo_fp32) {
    ((float *)b)[k] = f;
  } else {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    ((uint16_t *)b)[k] = (uint16_t)(u >> 16);
  }
}

void launch_to_lo(const double *a, void *b, int lo_fp32, size_t n, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_to_lo, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, lo_fp32, n);
}

void launch_info_init(mlmc_info_dev *info, double *q_coarse, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_info_init, dim3((n + 255) / 256), dim3(256), 0, st, info, q_coarse, n);
}

void launch_level_stats(const double *qf, const double *qc, int n, double lambda_star, int indicator, double *out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_level_stats, dim3(1), dim3(256), 0, st, qf, qc, n, lambda_star, indicator, out);
}

}  // namespace mlmc
