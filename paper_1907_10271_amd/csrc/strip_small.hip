// Whole-solve kernel for the coarse strip levels (Section 3.1 operator,
// Jacobi-PCG as in the lock-step engine): after the lifting kernel has written
// b and the Jacobi diagonal, one work-group owns one sample for every PCG
// iteration, with the search direction p and the operator output Ap in LDS
// and x, r and the Jacobi diagonal in registers.
// Only the Gauss-point (cos 2theta, sin 2theta) pairs are read from memory each
// iteration (they stay in L2), so a coarse level costs FP64 arithmetic instead
// of HBM traffic and no launch or host round-trip per iteration.
//
// The element loop runs in four colour phases (element (ex, ey) has colour
// (ex & 1) + 2 (ey & 1)); elements of one colour share no node, so each phase
// adds its forces into Ap without conflicts and every node receives its four
// contributions in the same colour order.  Dot products are fixed-order
// work-group sums, so results do not depend on the batch.
#include "strip_small.hpp"

#include <algorithm>

#include "strip_device.hpp"

namespace mlmc {

namespace {

constexpr int SMALL_MAX_THREADS = 512;

__device__ __forceinline__ void elem_nodes(const StripGeom &g, int ex, int ey, int nd[4]) {
  const int n0 = ey * g.nnx + ex;
  nd[0] = n0;
  nd[1] = n0 + 1;
  nd[2] = n0 + g.nnx + 1;
  nd[3] = n0 + g.nnx;
}

// (cos 2theta, sin 2theta) at the element's four Gauss points
__device__ __forceinline__ void load_angles(const double *ang_s, int cs, const StripGeom &g, int ex, int ey,
                                            double2 a[4]) {
  elem_cs(ang_s, cs, (size_t)ey * g.nx + ex, a);
}

// MAXN: owned nodes per thread (node k belongs to thread k mod blockDim)
template <int MAXN>
__global__ __launch_bounds__(SMALL_MAX_THREADS) void k_small_solve(StripGeom g, StripMat m, PcgSlots S) {
  extern __shared__ double lds[];
  double *pl = lds;                     // [2 nnode] p
  double *al = lds + 2 * g.nnode;       // [2 nnode] A p
  double *red = lds + 4 * g.nnode;      // [8] work-group sums
  const int s = blockIdx.x, tid = threadIdx.x, nt = blockDim.x, waves = nt >> 6;
  const double *th_s = (const double *)S.theta + (size_t)s * (S.cs ? 8 : 4) * g.nelem;
  const int hx = g.nx / 2, ncol = hx * (g.ny / 2);  // elements per colour

  // set-up state from the lifting kernel: z = dinv b and dg; here r = dg z, dinv = 1/dg
  const double *rs = S.z + (size_t)s * 2 * g.nnode, *ds = S.dg + (size_t)s * 2 * g.nnode;
  double x[MAXN][2], r[MAXN][2], dinv[MAXN][2];
  double prz = 0.0, prr = 0.0;
#pragma unroll
  for (int j = 0; j < MAXN; ++j) {
    const int k = tid + j * nt;
    x[j][0] = x[j][1] = r[j][0] = r[j][1] = 0.0;
    dinv[j][0] = dinv[j][1] = 1.0;
    if (k < g.nnode) {
      const double2 zv = *reinterpret_cast<const double2 *>(rs + 2 * (size_t)k);
      const double2 gv = *reinterpret_cast<const double2 *>(ds + 2 * (size_t)k);
      const double2 bv = make_double2(gv.x * zv.x, gv.y * zv.y);
      const double2 dv = make_double2(1.0 / gv.x, 1.0 / gv.y);
      r[j][0] = bv.x;
      r[j][1] = bv.y;
      dinv[j][0] = dv.x;
      dinv[j][1] = dv.y;
      prz += bv.x * (dv.x * bv.x) + bv.y * (dv.y * bv.y);
      prr += bv.x * bv.x + bv.y * bv.y;
    }
  }
  double rz = block_sum_w(prz, red, waves);
  double rr = block_sum_w(prr, red, waves);
  const double bb = rr, tol2 = S.rtol2 * bb;

  // ---- PCG iterations
  double rz_prev = 1.0;
  int it = 0, status;
  for (;; ++it) {
    if (!isfinite(rr) || !isfinite(rz)) { status = S_NAN; break; }
    if (it >= S.max_iter) { status = S_NOCONV; break; }
    if (rr <= tol2) { status = S_OK; break; }
    const double beta = (it == 0) ? 0.0 : rz / rz_prev;
    // p = z + beta p on the owned nodes; clear A p
#pragma unroll
    for (int j = 0; j < MAXN; ++j) {
      const int k = tid + j * nt;
      if (k < g.nnode) {
        const double pu = (it == 0) ? 0.0 : pl[2 * k], pv = (it == 0) ? 0.0 : pl[2 * k + 1];
        pl[2 * k] = fma(beta, pu, dinv[j][0] * r[j][0]);
        pl[2 * k + 1] = fma(beta, pv, dinv[j][1] * r[j][1]);
        al[2 * k] = 0.0;
        al[2 * k + 1] = 0.0;
      }
    }
    __syncthreads();
    for (int c = 0; c < 4; ++c) {
      for (int q = tid; q < ncol; q += nt) {
        const int ex = 2 * (q % hx) + (c & 1), ey = 2 * (q / hx) + (c >> 1);
        double2 a[4];
        load_angles(th_s, S.cs, g, ex, ey, a);
        int nd[4];
        elem_nodes(g, ex, ey, nd);
        const double u[4] = {pl[2 * nd[0]], pl[2 * nd[1]], pl[2 * nd[2]], pl[2 * nd[3]]};
        const double v[4] = {pl[2 * nd[0] + 1], pl[2 * nd[1] + 1], pl[2 * nd[2] + 1], pl[2 * nd[3] + 1]};
        double fu[4], fv[4];
        elem_forces_q<double>(g, [&](int k) { return qbar_cs(m, a[k].y, a[k].x); }, u, v, fu, fv);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          al[2 * nd[k]] += fu[k];
          al[2 * nd[k] + 1] += fv[k];
        }
      }
      __syncthreads();
    }
    // p . A p with A p = p on the prescribed unknowns
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < MAXN; ++j) {
      const int k = tid + j * nt;
      if (k < g.nnode) {
        const int i = k % g.nnx;
        const double pu = pl[2 * k], pv = pl[2 * k + 1];
        double yu = al[2 * k], yv = al[2 * k + 1];
        if (i == 0) { yu = pu; yv = pv; }
        if (i == g.nx) yu = pu;
        part += pu * yu + pv * yv;
      }
    }
    const double pap = block_sum_w(part, red, waves);
    if (!(pap > 0.0) || !isfinite(pap)) {
      status = isfinite(pap) ? S_BREAKDOWN : S_NAN;
      break;
    }
    const double alpha = rz / pap;
    prz = 0.0;
    prr = 0.0;
#pragma unroll
    for (int j = 0; j < MAXN; ++j) {
      const int k = tid + j * nt;
      if (k < g.nnode) {
        const int i = k % g.nnx;
        const double pu = pl[2 * k], pv = pl[2 * k + 1];
        double yu = al[2 * k], yv = al[2 * k + 1];
        if (i == 0) { yu = pu; yv = pv; }
        if (i == g.nx) yu = pu;
        x[j][0] = fma(alpha, pu, x[j][0]);
        x[j][1] = fma(alpha, pv, x[j][1]);
        r[j][0] = fma(-alpha, yu, r[j][0]);
        r[j][1] = fma(-alpha, yv, r[j][1]);
        prz += r[j][0] * (dinv[j][0] * r[j][0]) + r[j][1] * (dinv[j][1] * r[j][1]);
        prr += r[j][0] * r[j][0] + r[j][1] * r[j][1];
      }
    }
    rz_prev = rz;
    rz = block_sum_w(prz, red, waves);
    rr = block_sum_w(prr, red, waves);
  }
  // final state
  double *xs = S.x + (size_t)s * 2 * g.nnode;
#pragma unroll
  for (int j = 0; j < MAXN; ++j) {
    const int k = tid + j * nt;
    if (k < g.nnode) *reinterpret_cast<double2 *>(xs + 2 * (size_t)k) = make_double2(x[j][0], x[j][1]);
  }
  if (tid == 0) {
    S.it_b[s] = it;
    S.relres[s] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    S.status[s] = status;
    S.active[s] = 0;
  }
}

}  // namespace

int small_threads(const StripGeom &g) {
  const int per_colour = (g.nx / 2) * (g.ny / 2);
  return std::min(SMALL_MAX_THREADS, std::max(64, (per_colour + 63) / 64 * 64));
}

size_t small_lds_bytes(const StripGeom &g) { return ((size_t)4 * g.nnode + 8) * sizeof(double); }

int small_nodes_per_thread(const StripGeom &g) {
  const int t = small_threads(g);
  return (g.nnode + t - 1) / t;
}

bool small_fits(const StripGeom &g, size_t lds_per_block) {
  if (g.nx < 2 || g.ny < 2 || (g.nx & 1) || (g.ny & 1)) return false;
  if (small_nodes_per_thread(g) > SMALL_MAXN) return false;
  return small_lds_bytes(g) <= lds_per_block;
}

void launch_small_solve(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, hipStream_t st) {
  if (n <= 0) return;
  const int t = small_threads(g);
  const size_t lds = small_lds_bytes(g);
  // allow dynamic LDS beyond the default limit (up to what the device offers)
  static const bool opted_in = [] {
    (void)hipFuncSetAttribute((const void *)k_small_solve<5>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_small_solve<SMALL_MAXN>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)opted_in;
  if (small_nodes_per_thread(g) <= 5)
    hipLaunchKernelGGL(k_small_solve<5>, dim3(n), dim3(t), lds, st, g, m, S);
  else
    hipLaunchKernelGGL(k_small_solve<SMALL_MAXN>, dim3(n), dim3(t), lds, st, g, m, S);
}

}  // namespace mlmc
