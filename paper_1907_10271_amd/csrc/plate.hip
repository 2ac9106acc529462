// Buckling of a laminated Reissner-Mindlin plate (Section 4.1 of the paper):
// classical laminate theory (Eq. CLTABD) for each sample's perturbed ply
// angles, bilinear Q4 elements with selective reduced integration (membrane,
// coupling and bending 2x2, transverse shear 1x1), the geometric stiffness of
// a unit compressive edge load, and the smallest positive lambda of
// K phi = lambda K_G phi (Eq. matrixeig), found as the largest mu of
// K_G x = mu K x by block LOBPCG.
//
// One work-group solves one sample from start to finish (a persistent launch
// per level batch): laminate, element matrices, lower band of K on the free
// unknowns, banded Cholesky factor (the LOBPCG preconditioner T = K^-1), then
// LOBPCG with block size 2 and a Rayleigh-Ritz step in FP64.  In the mixed
// form the factor and the triangular solves are FP32; the operators,
// residuals and the Rayleigh-Ritz step stay FP64.  Every reduction runs in a
// fixed order inside the work-group, so a sample's result does not depend on
// the batch.
#include "plate.hpp"
#include "strip_kernels.hpp"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

namespace mlmc {

constexpr int PT = 256;      // threads per work-group
constexpr int NB = 2;        // LOBPCG block size
constexpr int NS = 3 * NB;   // Rayleigh-Ritz basis size [X, W, P]
constexpr int MAXPLY = 32;
constexpr int MAXBW = 664;  // largest band half-width (128 x 128 mesh: 654)
// entries allocated past the last band of a workspace: a band solve's row
// loads reach up to 799 entries past a row's start, and a row holds at least
// 16 (bw = 5 (nx + 2) >= 15); what lies past the row's band is never used
constexpr size_t BAND_PAD = MAXBW + 128;
// bands narrower than this are factored and solved by one work-group per
// sample (k_buckle); wider ones always take the wide form
constexpr int ONE_MAXBW = 256;
constexpr int RING_ONE = 512, RING_WIDE = 1024;  // band-solve window rows (>= bw + 3 x 32)
static_assert(RING_ONE >= ONE_MAXBW + 96 && RING_WIDE >= MAXBW + 96, "band-solve windows");

struct PlateGeom {
  int nx, ny, nnx, nny, nn, nfull, nfree, bw;
  double hx, hy, a, b;
  // eigensolver settings carried with every level: half-waves along x of the
  // first start vector (0: the integer nearest to a / b), and the relative
  // shift of the lowest-mode check (0: no check)
  int start_p0;
  double cert_shift;
  const int *free_of_full;  // [nfull] free index or -1
  const int *full_of_free;  // [nfree]
};

struct PlateMat {
  double Q11, Q22, Q12, Q66;
  double shear_k_G_t;  // k G t
  double N0;
  int mitc4;      // transverse shear: 0 one-point rule, 1 MITC4 assumed strain
  int condensed;  // decoupled laminate (A, 0, D* = D - B^T A^-1 B)
  int nply;
  double t_ply;
  double layup[MAXPLY];
};

// per-sample scratch of a level batch (device pointers, sample stride given)
struct PlateWork {
  double *band;    // [S][nfree][bw+1] FP64 factor (FP64 solves)
  float *bandf;    // [S][nfree][bw+1] FP32 factor (mixed)
  double *vec;     // [S][NVEC][nfree]
  double *kel;     // [S][KEL] element matrices K_e, K_G,e (factorisation spread over work-groups)
  int *flag;       // [S] non-positive pivot met
  double *lam;     // [S] lambda of the last solve (lowest-mode check of the wide path)
  double *side;    // [S][2][KP][LDPW] the last two factored panels of the wide factorisation (as B)
  int nvec;
  size_t band_stride, vec_stride;
};

constexpr int KEL = 800;   // K_e (400) and K_G,e (400) of one sample

enum { V_X = 0, V_W = NB, V_P = 2 * NB, V_KX = 3 * NB, V_KW = 4 * NB, V_KP = 5 * NB, V_GX = 6 * NB, V_GW = 7 * NB,
       V_GP = 8 * NB, V_R = 9 * NB, V_T = 10 * NB, NVEC = 11 * NB };

// ---------------------------------------------------------------- small helpers
// sum over the NT threads of a work-group (red: NT / 64 doubles of LDS); the
// wave sums are added in wave order
template <int NT = PT>
__device__ double block_reduce(double v, double *red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double sum = red[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) sum += red[k];
  return sum;
}

// rotated ply stiffness (fibres at angle th from x), engineering shear
__device__ void qbar_ply(const PlateMat &m, double th, double q[6]) {
  double s, c;
  sincos(th, &s, &c);
  const double c2 = c * c, s2 = s * s, cs = c * s;
  // Qbar = T^T Q T with T the engineering-strain rotation to fibre axes
  q[0] = m.Q11 * c2 * c2 + 2.0 * (m.Q12 + 2.0 * m.Q66) * s2 * c2 + m.Q22 * s2 * s2;        // 11
  q[1] = (m.Q11 + m.Q22 - 4.0 * m.Q66) * s2 * c2 + m.Q12 * (s2 * s2 + c2 * c2);             // 12
  q[2] = m.Q11 * s2 * s2 + 2.0 * (m.Q12 + 2.0 * m.Q66) * s2 * c2 + m.Q22 * c2 * c2;        // 22
  q[3] = (m.Q11 - m.Q12 - 2.0 * m.Q66) * c2 * cs + (m.Q12 - m.Q22 + 2.0 * m.Q66) * s2 * cs; // 16
  q[4] = (m.Q11 - m.Q12 - 2.0 * m.Q66) * s2 * cs + (m.Q12 - m.Q22 + 2.0 * m.Q66) * c2 * cs; // 26
  q[5] = (m.Q11 + m.Q22 - 2.0 * m.Q12 - 2.0 * m.Q66) * s2 * c2 + m.Q66 * (s2 * s2 + c2 * c2);  // 66
}

// generalised strain vector of unknown (node a, component c) at a point with
// shape derivatives (dNx, dNy): (eps_x, eps_y, gamma_xy, kappa_x, kappa_y, kappa_xy)
__device__ void gen_strain(int c, double dNx, double dNy, double e[6]) {
  for (int k = 0; k < 6; ++k) e[k] = 0.0;
  if (c == 0) { e[0] = dNx; e[2] = dNy; }
  else if (c == 1) { e[1] = dNy; e[2] = dNx; }
  else if (c == 3) { e[3] = dNx; e[5] = dNy; }
  else if (c == 4) { e[4] = dNy; e[5] = dNx; }
}

// K_e and K_G,e of the uniform element of a sample (20 x 20, unknowns 5 a + c,
// nodes counter-clockwise from the lower-left corner); Dmb = [[A, B], [B, D]]
__device__ void element_matrices(const PlateGeom &g, const PlateMat &m, const double *Dmb /*6x6*/, double *Ke,
                                 double *KGe) {
  const double gq = 0.57735026918962576451;
  const double jx = 0.5 * g.hx, jy = 0.5 * g.hy, det = jx * jy;
  const double xa[4] = {-1, 1, 1, -1}, ya[4] = {-1, -1, 1, 1};
  for (int idx = threadIdx.x; idx < 400; idx += PT) {
    const int I = idx / 20, J = idx % 20;
    const int a = I / 5, c = I % 5, b2 = J / 5, d = J % 5;
    double kv = 0.0, kg = 0.0;
    for (int q = 0; q < 4; ++q) {
      const double xi = (q & 1) ? gq : -gq, eta = (q & 2) ? gq : -gq;
      const double dNxa = 0.25 * xa[a] * (1 + ya[a] * eta) / jx, dNya = 0.25 * ya[a] * (1 + xa[a] * xi) / jy;
      const double dNxb = 0.25 * xa[b2] * (1 + ya[b2] * eta) / jx, dNyb = 0.25 * ya[b2] * (1 + xa[b2] * xi) / jy;
      double ea[6], eb[6];
      gen_strain(c, dNxa, dNya, ea);
      gen_strain(d, dNxb, dNyb, eb);
      double s = 0.0;
      for (int r = 0; r < 6; ++r)
        for (int t = 0; t < 6; ++t) s += ea[r] * Dmb[6 * r + t] * eb[t];
      kv += det * s;
      if (c == 2 && d == 2) kg += det * m.N0 * dNxa * dNxb;
    }
    if (!m.mitc4) {
      // transverse shear at the centre (weight 4): gamma = (w_x - theta_x, w_y - theta_y)
      const double Na = 0.25, Nb = 0.25;
      const double dNxa = 0.25 * xa[a] / jx, dNya = 0.25 * ya[a] / jy;
      const double dNxb = 0.25 * xa[b2] / jx, dNyb = 0.25 * ya[b2] / jy;
      double sa[2] = {0, 0}, sb[2] = {0, 0};
      if (c == 2) { sa[0] = dNxa; sa[1] = dNya; }
      if (c == 3) sa[0] = -Na;
      if (c == 4) sa[1] = -Na;
      if (d == 2) { sb[0] = dNxb; sb[1] = dNyb; }
      if (d == 3) sb[0] = -Nb;
      if (d == 4) sb[1] = -Nb;
      kv += 4.0 * det * m.shear_k_G_t * (sa[0] * sb[0] + sa[1] * sb[1]);
    } else {
      // MITC4 assumed shear strain (Bathe and Dvorkin): gamma_x of unknown
      // (node, component) tied at the edge midpoints (0, -1), (0, 1) and
      // interpolated linearly in eta; gamma_y tied at (-1, 0), (1, 0) and
      // interpolated in xi; 2x2 Gauss points
      auto tie_x = [&](int n, int cc, double et) {  // gamma_x row at (0, et)
        const double N = 0.25 * (1 + ya[n] * et);
        return cc == 2 ? 0.25 * xa[n] * (1 + ya[n] * et) / jx : cc == 3 ? -N : 0.0;
      };
      auto tie_y = [&](int n, int cc, double xt) {  // gamma_y row at (xt, 0)
        const double N = 0.25 * (1 + xa[n] * xt);
        return cc == 2 ? 0.25 * ya[n] * (1 + xa[n] * xt) / jy : cc == 4 ? -N : 0.0;
      };
      const double xa0 = tie_x(a, c, -1), xa1 = tie_x(a, c, 1), ya0 = tie_y(a, c, -1), ya1 = tie_y(a, c, 1);
      const double xb0 = tie_x(b2, d, -1), xb1 = tie_x(b2, d, 1), yb0 = tie_y(b2, d, -1), yb1 = tie_y(b2, d, 1);
      double ks = 0.0;
      for (int q = 0; q < 4; ++q) {
        const double xi = (q & 1) ? gq : -gq, eta = (q & 2) ? gq : -gq;
        const double gxa = 0.5 * (1 - eta) * xa0 + 0.5 * (1 + eta) * xa1;
        const double gya = 0.5 * (1 - xi) * ya0 + 0.5 * (1 + xi) * ya1;
        const double gxb = 0.5 * (1 - eta) * xb0 + 0.5 * (1 + eta) * xb1;
        const double gyb = 0.5 * (1 - xi) * yb0 + 0.5 * (1 + xi) * yb1;
        ks += gxa * gxb + gya * gyb;
      }
      kv += det * m.shear_k_G_t * ks;
    }
    Ke[idx] = kv;
    KGe[idx] = kg;
  }
}

// y = P K P x on the free unknowns (element-by-element gather at every node),
// rows shared out over the NT threads of the work-group (pointer types as the
// caller names them: the call form below names their memory)
template <bool GEOM, int NT, typename KPtr, typename XPtr, typename YPtr, typename IPtr>
__device__ __forceinline__ void plate_apply_body(const PlateGeom &g, KPtr Ke, XPtr x, YPtr y, IPtr full_of_free,
                                                 IPtr free_of_full) {
  for (int r = threadIdx.x; r < g.nfree; r += NT) {
    const int full = full_of_free[r];
    const int node = full / 5, c = full % 5;
    double acc = 0.0;
    if (!GEOM || c == 2) {
      const int i = node % g.nnx, j = node / g.nnx;
      // elements around the node in a fixed order: (i-1,j-1), (i,j-1), (i-1,j), (i,j)
      for (int e = 0; e < 4; ++e) {
        const int ex = i - 1 + (e & 1), ey = j - 1 + (e >> 1);
        if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) continue;
        const int n0 = ey * g.nnx + ex;
        const int nodes[4] = {n0, n0 + 1, n0 + g.nnx + 1, n0 + g.nnx};
        const int a = (e == 0) ? 2 : (e == 1) ? 3 : (e == 2) ? 1 : 0;  // local index of the node
        const auto row = Ke + 20 * (5 * a + c);
        for (int b2 = 0; b2 < 4; ++b2)
          for (int d = (GEOM ? 2 : 0); d < (GEOM ? 3 : 5); ++d) {
            const int f = free_of_full[5 * nodes[b2] + d];
            if (f >= 0) acc += row[5 * b2 + d] * x[f];
          }
      }
    }
    y[r] = acc;
  }
}

// pointers as the gathers use them: every caller passes the element matrix as
// its work-group's LDS copy, the vectors and index maps live in global memory
// (named so, their loads are not generic: LDS waits do not wait for them)
using KLds = const __attribute__((address_space(3))) double *;
using XGlb = const __attribute__((address_space(1))) double *;
using YGlb = __attribute__((address_space(1))) double *;
using IGlb = const __attribute__((address_space(1))) int *;

template <bool GEOM, int NT = PT>
__device__ void plate_apply(const PlateGeom &g, const double *Ke, const double *x, double *y) {
  plate_apply_body<GEOM, NT>(g, (KLds)Ke, (XGlb)x, (YGlb)y, (IGlb)g.full_of_free, (IGlb)g.free_of_full);
}

// plate_apply as a call of its own, for work-groups of more than PT threads,
// whose register budget the inlined gathers would share with the
// eigensolver's state
template <bool GEOM, int NT>
__device__ __noinline__ void plate_apply_call(const PlateGeom &g, const double *Ke, const double *x, double *y) {
  plate_apply<GEOM, NT>(g, Ke, x, y);
}

// lower band of K on the free unknowns: band[r][d] = K[r][r - d], d = 0..bw
// (rows r0 .. r1 - 1, entries shared out over `nthreads` threads from thread t)
template <typename B>
__device__ void assemble_band(const PlateGeom &g, const double *Ke_, B *band, int r0, int r1, int t, int nthreads) {
  const int w = g.bw + 1;  // nfree w < 2^31 for every mesh the band form accepts
  const KLds Ke = (KLds)Ke_;  // every caller's element matrix is its work-group's LDS copy
  const IGlb full_of_free = (IGlb)g.full_of_free;
  for (int idx = r0 * w + t; idx < r1 * w; idx += nthreads) {
    const int r = idx / w, d = idx - r * w;
    double v = 0.0;
    const int cfree = r - d;
    if (cfree >= 0) {
      const int fr = full_of_free[r], fc = full_of_free[cfree];
      const int nr = fr / 5, cr = fr % 5, nc = fc / 5, cc = fc % 5;
      const int ir = nr % g.nnx, jr = nr / g.nnx, ic = nc % g.nnx, jc = nc / g.nnx;
      if (abs(ir - ic) <= 1 && abs(jr - jc) <= 1) {
        for (int e = 0; e < 4; ++e) {
          const int ex = ir - 1 + (e & 1), ey = jr - 1 + (e >> 1);
          if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) continue;
          if (ic < ex || ic > ex + 1 || jc < ey || jc > ey + 1) continue;
          const int a = (e == 0) ? 2 : (e == 1) ? 3 : (e == 2) ? 1 : 0;
          const int lx = ic - ex, ly = jc - ey;
          const int b2 = (ly == 0) ? lx : 3 - lx;
          v += Ke[20 * (5 * a + cr) + 5 * b2 + cc];
        }
      }
    }
    ((__attribute__((address_space(1))) B *)band)[idx] = (B)v;
  }
}

// A 4 x 4 tile of a trailing window (rows and columns R .. R + m - 1, tile at
// offsets r0, c0; only entries with column <= row exist).  All sixteen entries
// are loaded before the tile's product is formed, so their loads are in flight
// together and overlap it, instead of one load-subtract-store round trip per
// entry; entries outside the window read the window's first entry and are
// never stored.
template <typename B>
__device__ __forceinline__ void tile_load(const B *band, int w, int R, int m, int r0, int c0, B (&v)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int r = r0 + a, cc = c0 + c;
      const bool in = r < m && cc <= r;
      v[a][c] = band[(size_t)(R + (in ? r : 0)) * w + (in ? r - cc : 0)];
    }
}

template <typename B>
__device__ __forceinline__ void tile_store(B *band, int w, int R, int m, int r0, int c0, const B (&v)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int r = r0 + a, cc = c0 + c;
      if (r < m && cc <= r) band[(size_t)(R + r) * w + (r - cc)] = v[a][c];
    }
}

// Blocked right-looking banded Cholesky in place (band[r][d] = A[r][r - d]).
// On return band[k][0] = L_kk and band[k + d][d] = L_{k+d,k}.  A pass takes a
// panel of KP = 2 NBK columns in two sub-panels of NBK: the first is factored,
// its product subtracted from the second's columns, the second factored, and
// the trailing band window then updated by both (4 x 4 register tiles per
// thread: the first sub-panel's NBK-term sum subtracted, then the second's).
// Every entry receives the operations of the NBK-column form in the same
// order, so the factor is bit-identical to the wide form's (k_band_step), while
// the trailing window, which does not fit on chip and bounds the pass, is read
// and written once per 2 NBK columns.  A sub-panel's top NBK x NBK block is
// factored by one thread in registers and each row below by its own thread
// (forward substitution with the block's factor).  The panel's rows and the
// window's tiles are final once the previous pass's stores are done (a
// work-group barrier), so a pass requests all of them first: the tile entries
// arrive while the panel is factored.
constexpr int NBK = 8, KP = 2 * NBK;
constexpr int LDP = KP + ONE_MAXBW, LDPW = KP + MAXBW;  // LDS panels (column-major): one-work-group and wide form
constexpr int TQ = 1;  // trailing tiles per thread in flight (the first TQ issued with the panel's loads)
static_assert(KP + ONE_MAXBW <= 2 * PT, "panel rows: at most two per thread");

// factors the nbs x nbs block of P (column-major, LD rows) at rows and columns
// c0 .. c0 + nbs - 1 (one thread, unblocked order); false at a non-positive pivot
template <int LD, typename B>
__device__ __forceinline__ bool factor_top(B *P, int c0, int nbs) {
  B a[NBK][NBK];
#pragma unroll
  for (int i = 0; i < NBK; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) a[i][j] = (i < nbs) ? P[(c0 + j) * LD + c0 + i] : B(0);
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NBK; ++j) {
    if (j < nbs && ok) {
      if (!(a[j][j] > B(0))) {
        ok = false;
      } else {
        const B piv = sqrt(a[j][j]);
        a[j][j] = piv;
#pragma unroll
        for (int i = j + 1; i < NBK; ++i)
          if (i < nbs) a[i][j] = a[i][j] / piv;
#pragma unroll
        for (int jj = j + 1; jj < NBK; ++jj)
#pragma unroll
          for (int i = jj; i < NBK; ++i)
            if (i < nbs) a[i][jj] -= a[i][j] * a[jj][j];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NBK; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      if (i < nbs) P[(c0 + j) * LD + c0 + i] = a[i][j];
  return ok;
}

// rows i0 .. rows - 1 of sub-panel columns c0 .. c0 + nbs - 1: forward
// substitution with the factored top block, one thread per row (NT threads)
template <int LD, typename B, int NT = PT>
__device__ __forceinline__ void factor_rows(B *P, int c0, int nbs, int i0, int rows) {
  for (int i = i0 + threadIdx.x; i < rows; i += NT) {
    B x[NBK];
#pragma unroll
    for (int j = 0; j < NBK; ++j) x[j] = P[(c0 + j) * LD + i];
#pragma unroll
    for (int j = 0; j < NBK; ++j) {
      if (j < nbs) {
        x[j] = x[j] / P[(c0 + j) * LD + c0 + j];
#pragma unroll
        for (int jj = j + 1; jj < NBK; ++jj)
          if (jj < nbs) x[jj] -= x[j] * P[(c0 + j) * LD + c0 + jj];
      }
    }
#pragma unroll
    for (int j = 0; j < NBK; ++j)
      if (j < nbs) P[(c0 + j) * LD + i] = x[j];
  }
}

// sub-panel A's product subtracted from sub-panel B's columns (rows NBK on):
// the NBK-term sum of the NBK-column form's trailing update, one thread per row
template <int LD, typename B, int NT = PT>
__device__ __forceinline__ void update_b(B *P, int nb, int rows) {
  for (int i = NBK + threadIdx.x; i < rows; i += NT) {
    B x[NBK];
#pragma unroll
    for (int j = 0; j < NBK; ++j) x[j] = P[j * LD + i];
#pragma unroll
    for (int jb = NBK; jb < KP; ++jb) {
      if (jb < nb && jb <= i) {
        B acc = B(0);
#pragma unroll
        for (int j = 0; j < NBK; ++j) acc += x[j] * P[j * LD + jb];
        P[jb * LD + i] -= acc;
      }
    }
  }
}

template <typename B>
__device__ __forceinline__ bool band_cholesky(const PlateGeom &g, B *band, B *P /* LDS [KP * LDP] */) {
  const int w = g.bw + 1, n = g.nfree;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  auto tile_of = [](int tix, int &r0, int &c0) {
    int ti = (int)((sqrtf(8.0f * tix + 1.0f) - 1.0f) * 0.5f);  // corrected below
    while ((ti + 1) * (ti + 2) / 2 <= tix) ++ti;
    while (ti * (ti + 1) / 2 > tix) --ti;
    r0 = 4 * ti;
    c0 = 4 * (tix - ti * (ti + 1) / 2);
  };
  for (int k0 = 0; k0 < n; k0 += KP) {
    const int nbA = min(NBK, n - k0), nbB = max(0, min(NBK, n - k0 - NBK)), nb = nbA + nbB;
    const int rows = min(nb + g.bw, n - k0);      // panel rows k0 .. k0 + rows - 1
    const int R = k0 + nb, m = min(g.bw, n - R);  // trailing window rows/columns R .. R + m - 1
    const int mt = (m + 3) / 4, ntile = m > 0 ? mt * (mt + 1) / 2 : 0;
    __syncthreads();  // the previous pass's stores are done and P is free
    // ---- loads: the panel's rows (one thread per band row: a row's entries are
    // contiguous) and the first TQ of this thread's trailing tiles
    auto row_load = [&](int i, B (&pe)[KP]) {
      const B *row = band + (size_t)(k0 + i) * w;
#pragma unroll
      for (int j = 0; j < KP; ++j) pe[j] = row[min(max(i - j, 0), g.bw)];
    };
    auto row_stage = [&](int i, const B (&pe)[KP]) {
#pragma unroll
      for (int j = 0; j < KP; ++j) P[j * LDP + i] = (j < nb && i >= j && i - j <= g.bw) ? pe[j] : B(0);
    };
    B pe[KP];
    if ((int)threadIdx.x < rows) row_load(threadIdx.x, pe);
    B tv[TQ][4][4];
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int tix = threadIdx.x + q * PT;
      if (tix < ntile) {
        int r0, c0;
        tile_of(tix, r0, c0);
        tile_load(band, w, R, m, r0, c0, tv[q]);
      }
    }
    if ((int)threadIdx.x < rows) row_stage(threadIdx.x, pe);
    if ((int)threadIdx.x + PT < rows) {  // panels of more than PT rows
      row_load(threadIdx.x + PT, pe);
      row_stage(threadIdx.x + PT, pe);
    }
    __syncthreads();
    // ---- sub-panel A (columns 0 .. nbA - 1)
    if (threadIdx.x == 0 && !factor_top<LDP>(P, 0, nbA)) bad = 1;
    __syncthreads();
    if (bad) return false;
    factor_rows<LDP>(P, 0, nbA, nbA, rows);
    __syncthreads();
    if (nbB > 0) {
      update_b<LDP>(P, nb, rows);
      __syncthreads();
      // ---- sub-panel B (columns NBK .. nb - 1)
      if (threadIdx.x == 0 && !factor_top<LDP>(P, NBK, nbB)) bad = 1;
      __syncthreads();
      if (bad) return false;
      factor_rows<LDP>(P, NBK, nbB, nb, rows);
      __syncthreads();
    }
    for (int idx = threadIdx.x; idx < rows * KP; idx += PT) {
      const int i = idx / KP, j = idx % KP;
      if (j < nb && i >= j && i - j <= g.bw) band[(size_t)(k0 + i) * w + (i - j)] = P[j * LDP + i];
    }
    // ---- trailing update of the window by both sub-panels (all inside the band)
    auto tile_update = [&](int r0, int c0, B (&v)[4][4]) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int j0 = half * NBK, j1 = half ? nb : nbA;
        if (j0 >= j1) break;
        B acc[4][4];
        for (int a = 0; a < 4; ++a)
          for (int c = 0; c < 4; ++c) acc[a][c] = B(0);
        for (int j = j0; j < j1; ++j) {
          B pr[4], pc[4];
          for (int a = 0; a < 4; ++a) {
            const int ir = nb + r0 + a, ic = nb + c0 + a;
            pr[a] = (r0 + a < m) ? P[j * LDP + ir] : B(0);
            pc[a] = (c0 + a < m) ? P[j * LDP + ic] : B(0);
          }
          for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 4; ++c) acc[a][c] += pr[a] * pc[c];
        }
        for (int a = 0; a < 4; ++a)
          for (int c = 0; c < 4; ++c) v[a][c] -= acc[a][c];
      }
      tile_store(band, w, R, m, r0, c0, v);
    };
    // tiles in groups of TQ from tv; after each, the loads of the tile TQ further on
    for (int q = 0; (int)threadIdx.x + q * PT < ntile; q += TQ) {
#pragma unroll
      for (int u = 0; u < TQ; ++u) {
        const int tix = threadIdx.x + (q + u) * PT;
        if (tix < ntile) {
          int r0, c0;
          tile_of(tix, r0, c0);
          tile_update(r0, c0, tv[u]);
          const int tnx = tix + TQ * PT;
          if (tnx < ntile) {
            tile_of(tnx, r0, c0);
            tile_load(band, w, R, m, r0, c0, tv[u]);
          }
        }
      }
    }
  }
  __syncthreads();
  return true;
}

// value of lane `l` (uniform) to every lane
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// ---- diagonal-block inverses
// A band-solve step needs the inverse of one PS x PS diagonal block of L.
// After the factorisation each such block (rows and columns k0 .. k0 + PS - 1,
// k0 a multiple of PS) is replaced in the band by its inverse X, lower
// triangular with the same positions, so that a solve step applies a
// matrix-vector product instead of a chain of PS dependent substitutions.
// Only the solve reads these positions.
constexpr int PS = 32;
static_assert(NB * PS == 64, "one lane per right-hand side and row of a solve step");

// Inverts the diagonal blocks blk0 .. blk0 + nstage - 1 that exist, one per
// half-wave and without work-group barriers: the block is staged in Ls (nstage
// PS x PS entries of LDS), inverted in place column by column from the last
// (lane i forms X_ij = -X_jj sum_{j<k<=i} X_ik L_kj, the columns right of j
// already holding X and column j still holding L), and written back.
template <typename B>
__device__ void invert_blocks(B *band, int w, int n, int blk0, int nstage, B *Ls) {
  const int h = threadIdx.x / PS, i = threadIdx.x % PS;
  const int k0 = (blk0 + h) * PS;
  if (h >= nstage || k0 >= n) return;
  const int nb = min(PS, n - k0);
  B *L = Ls + h * PS * PS;
  for (int rr = 0; rr < nb; ++rr)  // row rr of the block, lane i its column i (contiguous in the band)
    if (i <= rr) L[rr * PS + i] = band[(size_t)(k0 + rr) * w + (rr - i)];
  for (int j = nb - 1; j >= 0; --j) {
    const B xjj = B(1) / L[j * PS + j];
    B acc = B(0);
    if (i > j && i < nb)
      for (int k = j + 1; k <= i; ++k) acc += L[i * PS + k] * L[k * PS + j];
    // every lane of the half-wave has read column j (one wave, in order)
    if (i > j && i < nb) L[i * PS + j] = -acc * xjj;
    if (i == j) L[j * PS + j] = xjj;
  }
  for (int rr = 0; rr < nb; ++rr)
    if (i <= rr) band[(size_t)(k0 + rr) * w + (rr - i)] = L[rr * PS + i];
}

// z = (L L^T)^-1 r for NB right-hand sides, in steps of PS rows, with the
// diagonal blocks of the band holding their inverses X, by a work-group of NT
// threads.  The solved rows a step needs (fewer than bw + 3 PS) live in an LDS
// window of RING rows.
// Forward step (rows k0 .. k0 + PS - 1): t_i = r_i - sum_c L_ic y_c over the
// band columns c < k0, each row's entries read by NT / PS lanes in contiguous
// runs (its band row is contiguous), the partial sums combined by lane shuffles;
// then y = X t, one wave (lane = right-hand side x row).  The band entries of
// the next step are requested as soon as this step's are used, so they arrive
// during its reductions and barriers.  Backward step: z = X^T t, then each
// thread subtracts L_jc z_j from its rows c < k0 of the window (one column c
// per thread: neighbouring threads read neighbouring band entries).
template <typename B, int RING, int MAXB, int NT = PT>
__device__ void band_solve(const PlateGeom &g, const B *band, const double *r, double *z, int ld, B *tmp) {
  static_assert((RING & (RING - 1)) == 0 && RING >= MAXB + 3 * PS, "window rows: a power of two >= bw + 3 PS");
  static_assert(NT % PS == 0 && (PS * PS) % NT == 0, "whole rows per step and whole X entries per thread");
  constexpr int LPR = NT / PS;  // forward lanes per row of a step
  // band entries per lane and chunk (a chunk covers LPR CH columns of a row):
  // one chunk for the widest band when LPR 32 columns cover it, else 32
  constexpr int CH = LPR * 32 >= MAXB ? (MAXB - 1) / LPR + 1 : 32;
  constexpr int MAXCHUNK = (MAXB + LPR * CH - 1) / (LPR * CH);  // chunks of the widest band (bw <= MAXB)
  constexpr int XE = PS * PS / NT;                              // entries of X per thread
  // furthest reach of a row load past its row's start (fi + 1 + fq + LPR u + LPR CH c)
  static_assert(PS + LPR * CH * MAXCHUNK - 1 - 16 <= (int)BAND_PAD, "row loads stay inside the padding");
  const int w = g.bw + 1, n = g.nfree, bw = g.bw;
  // At more than PT threads the solve is a call of its own, whose pointer
  // arguments the compiler cannot place: named as global memory, its loads
  // count only against the vector-memory counter, so the waits for LDS
  // accesses do not also wait for the band entries in flight.  In every form
  // the loads are issued unconditionally (addresses clamped into the band or
  // its padding, values masked where used), so each wait covers just the
  // loads before it.
  constexpr bool LONG = NT > PT;
  using BP = std::conditional_t<LONG, const __attribute__((address_space(1))) B *, const B *>;
  using RP = std::conditional_t<LONG, const __attribute__((address_space(1))) double *, const double *>;
  using ZP = std::conditional_t<LONG, __attribute__((address_space(1))) double *, double *>;
  using TP = std::conditional_t<LONG, __attribute__((address_space(1))) B *, B *>;
  const BP bandp = (BP)band;
  const RP rp = (RP)r;
  const ZP zp = (ZP)z;
  const TP tp = (TP)tmp;
  __shared__ B ring[NB * RING], Lb[PS * PS], tb[NB * PS];
  auto win = [&](int v, int row) -> B & { return ring[v * RING + (row & (RING - 1))]; };
  const int v2 = threadIdx.x / PS, i2 = threadIdx.x % PS;  // mat-vec lanes (wave 0)
  const int fi = threadIdx.x / LPR, fq = threadIdx.x % LPR; // forward: row fi of the step, part fq
  B e[XE];
  int xnb = 0;  // rows of the step whose X is in e
  auto x_load = [&](int k0) {  // X of the step at k0: Lb[i PS + j] = X_ij (j <= i < nb), identity past the end
    const int nb = min(PS, n - k0);
    xnb = nb;
#pragma unroll
    for (int u = 0; u < XE; ++u) {
      const int idx = threadIdx.x + u * NT, i = idx / PS, j = idx % PS;
      const int ii = min(i, nb - 1);
      e[u] = bandp[(size_t)(k0 + ii) * w + max(ii - j, 0)];  // masked in x_store
    }
  };
  auto x_store = [&]() {
#pragma unroll
    for (int u = 0; u < XE; ++u) {
      const int idx = threadIdx.x + u * NT, i = idx / PS, j = idx % PS;
      Lb[idx] = (i < xnb && j <= i) ? e[u] : B(i == j ? 1 : 0);
    }
  };
  // chunk c of row fi's band entries left of the step: column k0 + fi - d,
  // d = fi + 1 + fq + LPR u + LPR CH c (entries past the row's band are not
  // used)
  auto row_load = [&](int k0, int c, B (&l)[CH]) {
    const int nb = min(PS, n - k0), d0 = fi + 1 + fq + LPR * CH * c;
    // past the row's band the reads land in the next row or in the band
    // allocation's padding (BAND_PAD entries)
    const BP p = bandp + (size_t)(k0 + min(fi, nb - 1)) * w + d0;
#pragma unroll
    for (int u = 0; u < CH; ++u) l[u] = p[LPR * u];
  };
  auto row_dot = [&](int k0, int c, const B (&l)[CH], B (&acc)[NB]) {
    const int nb = min(PS, n - k0), d0 = fi + 1 + fq + LPR * CH * c;
    const int col0 = k0 + fi - d0;                            // column of u = 0
    const int lim = fi < nb ? min(bw - d0, col0) : -1;        // u is used while LPR u <= lim
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const bool ok = LPR * u <= lim;
      const int idx = (col0 - LPR * u) & (RING - 1);
      for (int v = 0; v < NB; ++v) acc[v] += ok ? l[u] * ring[v * RING + idx] : B(0);
      // under the smaller register budget of a larger work-group, keep the
      // window reads of a few entries in flight, not of the whole chunk
      if constexpr (NT > PT)
        if (u % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    }
  };
  const int nchunk = (bw + LPR * CH - 1) / (LPR * CH);
  // ---- forward: L y = r
  B l[CH];
  double rv[NB];
  row_load(0, 0, l);
  for (int v = 0; v < NB; ++v) rv[v] = rp[(size_t)v * ld + min(fi, n - 1)];  // used where fq = 0, fi < nb
  x_load(0);
  x_store();
  for (int k0 = 0; k0 < n; k0 += PS) {
    const int nb = min(PS, n - k0);
    const bool next = k0 + PS < n;
    B acc[NB];
    for (int v = 0; v < NB; ++v) acc[v] = B(0);
    row_dot(k0, 0, l, acc);
    for (int c = 1; c < min(nchunk, MAXCHUNK); ++c) {  // bands wider than 8 CH: further chunks loaded here
      B lc[CH];
      row_load(k0, c, lc);
      row_dot(k0, c, lc, acc);
    }
    double rc[NB];
    for (int v = 0; v < NB; ++v) rc[v] = rv[v];
    if (next) {
      // the next step's entries, in flight during this step's reductions and
      // barriers; X first, since its wait at the end of this step covers all
      // loads issued before it
      x_load(k0 + PS);
      for (int v = 0; v < NB; ++v) rv[v] = rp[(size_t)v * ld + min(k0 + PS + fi, n - 1)];
      row_load(k0 + PS, 0, l);
    }
    for (int v = 0; v < NB; ++v)
#pragma unroll
      for (int o = 1; o < LPR; o <<= 1) acc[v] += __shfl_xor(acc[v], o, LPR);
    if (fq == 0 && fi < nb)
      for (int v = 0; v < NB; ++v) tb[v * PS + fi] = (B)rc[v] - acc[v];
    __syncthreads();  // tb holds t, Lb holds X
    if (threadIdx.x < 64) {
      // four partial sums: four independent chains of LDS reads and FMAs
      B y4[4] = {B(0), B(0), B(0), B(0)};
      int j = 0;
      for (; j + 4 <= nb; j += 4)
#pragma unroll
        for (int q = 0; q < 4; ++q) y4[q] += Lb[i2 * PS + j + q] * tb[v2 * PS + j + q];
      for (; j < nb; ++j) y4[0] += Lb[i2 * PS + j] * tb[v2 * PS + j];
      const B y = (y4[0] + y4[1]) + (y4[2] + y4[3]);
      if (i2 < nb) {
        win(v2, k0 + i2) = y;
        tp[(size_t)v2 * n + k0 + i2] = y;
      }
    }
    __syncthreads();  // y of the step in the window; Lb free
    if (next) x_store();
  }
  // ---- backward: L^T z = y.  At the start of step k0 the window holds rows
  // k0 - PS - bw .. k0 + nb - 1 (y less the later steps' updates).  A step's
  // column entries and entering rows are requested at the end of the step
  // before, after the next X (whose wait covers the loads issued before it).
  const int last = ((n - 1) / PS) * PS;
  for (int i = max(0, last - PS - bw) + threadIdx.x; i < n; i += NT)
    for (int v = 0; v < NB; ++v) win(v, i) = tp[(size_t)v * n + i];
  x_load(last);
  x_store();
  // column c of step k0: L(k0 + j, c) = band[(k0 + j) w + k0 + j - c], for k0 + j - c <= bw
  // (entries outside the band are not loaded and not used)
  auto col_load = [&](int k0, int c, B (&lv)[PS]) {
    const int nb = min(PS, n - k0);
    // 32-bit byte offsets from the sample's band (fewer than 2^32 bytes for
    // bw <= MAXBW): one address register per entry in flight.  Rows past the
    // last read the last row; entries past the band land in the next row or in
    // the padding; neither is used.
    using CP = const __attribute__((address_space(1))) char *;
    const unsigned o = (unsigned)(k0 * w + (k0 - c)) * (unsigned)sizeof(B);  // L(k0 + j, c) at o + j (w + 1) B
    const unsigned step = (unsigned)(w + 1) * (unsigned)sizeof(B);
#pragma unroll
    for (int j = 0; j < PS; ++j) lv[j] = *(BP)((CP)bandp + (o + min(j, nb - 1) * step));
  };
  B l0[PS], yin[NB];
  // every thread loads (clamped column and row), used where in range
  col_load(last, max(last - 1 - (int)threadIdx.x, max(0, last - bw)), l0);
  for (int v = 0; v < NB; ++v)
    yin[v] = tp[(size_t)v * n + min(max(last - 2 * PS - bw + (int)threadIdx.x, 0), n - 1)];
  for (int k0 = last; k0 >= 0; k0 -= PS) {
    const int nb = min(PS, n - k0);
    const bool next = k0 > 0;
    const int lo = max(0, k0 - bw), c0 = k0 - 1 - threadIdx.x;
    const int ent = k0 - 2 * PS - bw + threadIdx.x;  // row entering the window (threads < PS)
    __syncthreads();  // rows k0 .. k0 + nb - 1 of the window are final, Lb holds X
    if (threadIdx.x < 64) {
      B y4[4] = {B(0), B(0), B(0), B(0)};
      int j = 0;
      for (; j + 4 <= nb; j += 4)
#pragma unroll
        for (int q = 0; q < 4; ++q) y4[q] += Lb[(j + q) * PS + i2] * win(v2, k0 + j + q);
      for (; j < nb; ++j) y4[0] += Lb[j * PS + i2] * win(v2, k0 + j);
      const B y = (y4[0] + y4[1]) + (y4[2] + y4[3]);
      if (i2 < nb) {
        win(v2, k0 + i2) = y;  // every lane has read the window rows (one wave)
        zp[(size_t)v2 * ld + k0 + i2] = (double)y;
      }
    }
    __syncthreads();
    if (next) x_load(k0 - PS);
    auto col_update = [&](int c, const B (&lv)[PS]) {
      B acc[NB];
      for (int v = 0; v < NB; ++v) acc[v] = B(0);
#pragma unroll
      for (int j = 0; j < PS; ++j) {
        if (j < nb) {
          const B lj = (k0 + j - c <= bw) ? lv[j] : B(0);
          for (int v = 0; v < NB; ++v) acc[v] += lj * win(v, k0 + j);
        }
        if constexpr (NT > PT)
          if (j % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
      for (int v = 0; v < NB; ++v) win(v, c) -= acc[v];
    };
    if (c0 >= lo) col_update(c0, l0);
    if constexpr (MAXB >= NT) {  // bands at least as wide as the work-group: further columns
      for (int c = c0 - NT; c >= lo; c -= NT) {
        B lv[PS];
        col_load(k0, c, lv);
        col_update(c, lv);
      }
    }
    if (threadIdx.x < PS && ent >= 0)
      for (int v = 0; v < NB; ++v) win(v, ent) = yin[v];
    if (next) {
      const int kn = k0 - PS, cn = kn - 1 - threadIdx.x, en = kn - 2 * PS - bw + threadIdx.x;
      col_load(kn, max(cn, max(0, kn - bw)), l0);  // clamped; used where cn is in range
      for (int v = 0; v < NB; ++v) yin[v] = tp[(size_t)v * n + min(max(en, 0), n - 1)];
      x_store();
    }
  }
  __syncthreads();
}

// The band solve as a call of its own: at more than PT threads a work-group's
// register budget is too small for the eigensolver's state and the solve's
// loads in flight together, and a call keeps the solve's registers its own
// (the caller's live state is saved once per call, not spilled inside the
// solve's steps).
template <typename B, int RING, int MAXB, int NT>
__device__ __noinline__ void band_solve_call(const PlateGeom &g, const B *band, const double *r, double *z, int ld,
                                             B *tmp) {
  band_solve<B, RING, MAXB, NT>(g, band, r, z, ld, tmp);
}

// symmetric eigen-decomposition of a small dense matrix (cyclic Jacobi), one thread
__device__ void jacobi_small(double *A, double *V, int m) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) V[i * m + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, nrm = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        nrm += A[i * m + j] * A[i * m + j];
        if (i != j) off += A[i * m + j] * A[i * m + j];
      }
    if (off <= 1e-30 * nrm) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * m + q];
        if (apq == 0.0) continue;
        const double tau = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
        for (int k = 0; k < m; ++k) {
          const double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = cs * akp - sn * akq;
          A[k * m + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = cs * apk - sn * aqk;
          A[q * m + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[k * m + p], vkq = V[k * m + q];
          V[k * m + p] = cs * vkp - sn * vkq;
          V[k * m + q] = sn * vkp + cs * vkq;
        }
      }
  }
}

// Rayleigh-Ritz on span(S) (m columns): largest NB eigenpairs of GA c = mu GB c.
// GB = R^T R (Cholesky), C = R^-T GA R^-1.  Returns the usable basis size
// (columns whose Cholesky pivot is too small are dropped: m_used <= m).  One
// thread; its small matrices live in LDS (wk: RR_WORK doubles, iwk: 2 NS
// ints), where indexed accesses cost an LDS round trip rather than the
// private-memory round trip of a thread-local array.
constexpr int RR_WORK = 4 * NS * NS + NS;
__device__ int rayleigh_ritz(const double *GA, const double *GB, int m, double *coef /*m x NB*/, double *mu,
                             double *wk, int *iwk) {
  double *R = wk, *Ri = wk + NS * NS, *C = wk + 2 * NS * NS, *V = wk + 3 * NS * NS, *rj = wk + 4 * NS * NS;
  int *keep = iwk, *order = iwk + NS, mk = 0;
  // pivoted-free Cholesky with column dropping (columns are ordered X, W, P)
  for (int j = 0; j < m; ++j) {
    // tentative column j against the kept ones
    for (int i = 0; i < mk; ++i) {
      double s = GB[keep[i] * m + j];
      for (int k = 0; k < i; ++k) s -= R[k * NS + i] * rj[k];
      rj[i] = s / R[i * NS + i];
    }
    double d = GB[j * m + j];
    for (int k = 0; k < mk; ++k) d -= rj[k] * rj[k];
    if (d > 1e-13 * GB[j * m + j] && d > 0.0) {
      for (int k = 0; k < mk; ++k) R[k * NS + mk] = rj[k];
      R[mk * NS + mk] = sqrt(d);
      for (int k = mk + 1; k < NS; ++k) R[k * NS + mk] = 0.0;
      keep[mk++] = j;
    }
  }
  // Ri = R^-1 (upper triangular)
  for (int i = 0; i < mk; ++i)
    for (int j = 0; j < mk; ++j) Ri[i * NS + j] = 0.0;
  for (int j = 0; j < mk; ++j) {
    Ri[j * NS + j] = 1.0 / R[j * NS + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[i * NS + k] * Ri[k * NS + j];
      Ri[i * NS + j] = -s / R[i * NS + i];
    }
  }
  // C = Ri^T GA_kept Ri
  for (int i = 0; i < mk; ++i)
    for (int j = 0; j < mk; ++j) {
      double s = 0.0;
      for (int k = 0; k <= i; ++k)
        for (int l = 0; l <= j; ++l) s += Ri[k * NS + i] * GA[keep[k] * m + keep[l]] * Ri[l * NS + j];
      C[i * mk + j] = s;
    }
  jacobi_small(C, V, mk);
  // sort eigenvalues descending
  for (int i = 0; i < mk; ++i) order[i] = i;
  for (int i = 0; i < mk; ++i)
    for (int j = i + 1; j < mk; ++j)
      if (C[order[j] * mk + order[j]] > C[order[i] * mk + order[i]]) {
        const int t = order[i];
        order[i] = order[j];
        order[j] = t;
      }
  for (int v = 0; v < NB; ++v) {
    const int e = order[min(v, mk - 1)];
    mu[v] = C[e * mk + e];
    for (int j = 0; j < m; ++j) coef[j * NB + v] = 0.0;
    for (int i = 0; i < mk; ++i) {
      double s = 0.0;
      for (int k = i; k < mk; ++k) s += Ri[i * NS + k] * V[k * mk + e];
      coef[keep[i] * NB + v] = s;
    }
  }
  return mk;
}

// ---------------------------------------------------------------- the solver
struct PlateJob {
  const double *offsets;  // [rows][nply]
  const int64_t *rows;    // [n]
  const int *out_idx;     // [n]
  double *lam;            // output (indexed by out_idx)
  mlmc_info *info;
  int coarse;
  int n;
};

// laminate matrix Dmb = [[A, B], [B, D]] (6 x 6, Eq. CLTABD) of one sample's
// ply offsets; for the decoupled model (Section 4.1) [[A, 0], [0, D*]] with
// D* = D - B^T A^-1 B.  One thread.
__device__ void laminate_dmb(const PlateMat &m, const double *off, double *Dmb) {
  double A[6] = {0, 0, 0, 0, 0, 0}, Bm[6] = {0, 0, 0, 0, 0, 0}, D[6] = {0, 0, 0, 0, 0, 0};
  const double z0 = -0.5 * m.nply * m.t_ply;
  for (int k = 0; k < m.nply; ++k) {
    double q[6];
    qbar_ply(m, m.layup[k] + off[k], q);
    const double za = z0 + k * m.t_ply, zb = za + m.t_ply;
    for (int t = 0; t < 6; ++t) {
      A[t] += q[t] * (zb - za);
      Bm[t] += q[t] * (zb * zb - za * za) * 0.5;
      D[t] += q[t] * (zb * zb * zb - za * za * za) / 3.0;
    }
  }
  // 3x3 blocks from (11, 12, 22, 16, 26, 66)
  auto full3 = [](const double *v, double *M3) {
    const double f[9] = {v[0], v[1], v[3], v[1], v[2], v[4], v[3], v[4], v[5]};
    for (int i = 0; i < 9; ++i) M3[i] = f[i];
  };
  double A3[9], B3[9], D3[9];
  full3(A, A3);
  full3(Bm, B3);
  full3(D, D3);
  if (m.condensed) {
    // A^-1 by cofactors (A symmetric positive definite), then D - B A^-1 B
    const double c00 = A3[4] * A3[8] - A3[5] * A3[7], c01 = A3[5] * A3[6] - A3[3] * A3[8],
                 c02 = A3[3] * A3[7] - A3[4] * A3[6];
    const double det = A3[0] * c00 + A3[1] * c01 + A3[2] * c02;
    const double Ai[9] = {c00 / det, (A3[2] * A3[7] - A3[1] * A3[8]) / det, (A3[1] * A3[5] - A3[2] * A3[4]) / det,
                          c01 / det, (A3[0] * A3[8] - A3[2] * A3[6]) / det, (A3[2] * A3[3] - A3[0] * A3[5]) / det,
                          c02 / det, (A3[1] * A3[6] - A3[0] * A3[7]) / det, (A3[0] * A3[4] - A3[1] * A3[3]) / det};
    double AiB[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) AiB[3 * i + j] = Ai[3 * i] * B3[j] + Ai[3 * i + 1] * B3[3 + j] + Ai[3 * i + 2] * B3[6 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        D3[3 * i + j] -= B3[i] * AiB[j] + B3[3 + i] * AiB[3 + j] + B3[6 + i] * AiB[6 + j];  // (B^T A^-1 B)_ij
    for (int i = 0; i < 9; ++i) B3[i] = 0.0;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Dmb[6 * i + j] = A3[3 * i + j];
      Dmb[6 * i + 3 + j] = B3[3 * i + j];
      Dmb[6 * (3 + i) + j] = B3[3 * j + i];
      Dmb[6 * (3 + i) + 3 + j] = D3[3 * i + j];
    }
}

// laminate (Eq. CLTABD) of sample s and its uniform element matrices
__device__ void sample_elements(const PlateGeom &g, const PlateMat &m, const PlateJob &J, int s, double *Dmb,
                                double *Ke, double *KGe) {
  if (threadIdx.x == 0) laminate_dmb(m, J.offsets + (size_t)J.rows[s] * m.nply, Dmb);
  __syncthreads();
  element_matrices(g, m, Dmb, Ke, KGe);
  __syncthreads();
}

// lambda, iteration count and status of sample s
__device__ void write_result(const PlateJob &J, int s, double lam, int it, double res, int st) {
  const int o = J.out_idx[s];
  J.lam[o] = lam;
  if (J.coarse) {
    J.info[o].iters_c = it;
    J.info[o].relres_c = res;
    J.info[o].status_c = st;
  } else {
    J.info[o].iters_f = it;
    J.info[o].relres_f = res;
    J.info[o].status_f = st;
  }
}

// result of one eigen-solve (the same in every thread of the work-group)
struct EigResult {
  double lam, res;
  int it, status;
};

// LOBPCG (block NB) for the largest mu of K_G x = mu K x with the factored
// band as preconditioner, by a work-group of NT threads; returns lambda = 1/mu
template <typename B, int RING, int MAXB, int NT = PT>
__device__ __forceinline__ EigResult lobpcg(const PlateGeom &g, const double *Ke, const double *KGe, const B *band, double *vec,
                            double tol, int max_iter) {
  __shared__ double red[NT / 64];
  __shared__ double gram[2 * NS * NS];
  __shared__ double coef[NS * NB], mu[NB], resn[NB];
  __shared__ double rr_wk[RR_WORK];
  __shared__ int rr_iwk[2 * NS];
  const int n = g.nfree;
  auto V = [&](int k) { return vec + (size_t)k * n; };
  // ---- initial block: smooth mode shapes w = sin(p pi x/a) sin(pi y/b), theta = grad w,
  // for p = p0, p0 + 1 half-waves along x, p0 the integer nearest to a/b (a long
  // panel buckles in about a/b half-waves; 1 for a square panel)
  const int p0 = g.start_p0 > 0 ? g.start_p0 : max(1, (int)lround(g.a / g.b));
  for (int r = threadIdx.x; r < n; r += NT) {
    const int full = g.full_of_free[r], node = full / 5, c = full % 5;
    const double x = (node % g.nnx) * g.hx, y = (node / g.nnx) * g.hy;
    for (int v = 0; v < NB; ++v) {
      const double px = M_PI * (p0 + v) / g.a, py = M_PI / g.b;
      double val = 0.0;
      if (c == 2) val = sin(px * x) * sin(py * y);
      if (c == 3) val = px * cos(px * x) * sin(py * y);
      if (c == 4) val = py * sin(px * x) * cos(py * y);
      V(V_X + v)[r] = val;
    }
  }
  __syncthreads();
  for (int v = 0; v < NB; ++v) {
    if constexpr (NT > PT) {
      plate_apply_call<false, NT>(g, Ke, V(V_X + v), V(V_KX + v));
      plate_apply_call<true, NT>(g, KGe, V(V_X + v), V(V_GX + v));
    } else {
      plate_apply<false, NT>(g, Ke, V(V_X + v), V(V_KX + v));
      plate_apply<true, NT>(g, KGe, V(V_X + v), V(V_GX + v));
    }
  }
  __syncthreads();
  int it = 0, have_p = 0;
  double mu0 = 0.0, res0 = 1.0;
  for (;; ++it) {
    // Rayleigh quotients of the current block and residuals R = G X - mu K X
    double acc[2 * NB];
    for (int v = 0; v < NB; ++v) {
      double a = 0.0, b = 0.0;
      for (int r = threadIdx.x; r < n; r += NT) {
        a += V(V_X + v)[r] * V(V_GX + v)[r];
        b += V(V_X + v)[r] * V(V_KX + v)[r];
      }
      acc[2 * v] = block_reduce<NT>(a, red);
      acc[2 * v + 1] = block_reduce<NT>(b, red);
    }
    double rq[NB];
    for (int v = 0; v < NB; ++v) rq[v] = acc[2 * v] / acc[2 * v + 1];
    for (int v = 0; v < NB; ++v) {
      double rn = 0.0, kn = 0.0;
      for (int r = threadIdx.x; r < n; r += NT) {
        const double rv = V(V_GX + v)[r] - rq[v] * V(V_KX + v)[r];
        V(V_R + v)[r] = rv;
        rn += rv * rv;
        kn += V(V_KX + v)[r] * V(V_KX + v)[r];
      }
      rn = block_reduce<NT>(rn, red);
      kn = block_reduce<NT>(kn, red);
      if (threadIdx.x == 0) resn[v] = sqrt(rn) / (fabs(rq[v]) * sqrt(kn));
    }
    __syncthreads();
    mu0 = rq[0];
    res0 = resn[0];
    if (!(res0 > tol) || it >= max_iter || !isfinite(res0)) break;
    // W = T R with T = K^-1 (banded Cholesky)
    if constexpr (NT > PT)
      band_solve_call<B, RING, MAXB, NT>(g, band, V(V_R), V(V_W), n, (B *)V(V_T));
    else
      band_solve<B, RING, MAXB, NT>(g, band, V(V_R), V(V_W), n, (B *)V(V_T));
    for (int v = 0; v < NB; ++v) {
      if constexpr (NT > PT) {
        plate_apply_call<false, NT>(g, Ke, V(V_W + v), V(V_KW + v));
        plate_apply_call<true, NT>(g, KGe, V(V_W + v), V(V_GW + v));
      } else {
        plate_apply<false, NT>(g, Ke, V(V_W + v), V(V_KW + v));
        plate_apply<true, NT>(g, KGe, V(V_W + v), V(V_GW + v));
      }
    }
    __syncthreads();
    // Gram matrices of S = [X, W, P]
    const int ms = have_p ? NS : 2 * NB;
    for (int i = 0; i < ms; ++i)
      for (int j = i; j < ms; ++j) {
        const int vi = (i < NB) ? V_X + i : (i < 2 * NB) ? V_W + i - NB : V_P + i - 2 * NB;
        const int vj = (j < NB) ? V_X + j : (j < 2 * NB) ? V_W + j - NB : V_P + j - 2 * NB;
        const int gj = vj + (V_GX - V_X), kj = vj + (V_KX - V_X);
        double a = 0.0, b = 0.0;
        for (int r = threadIdx.x; r < n; r += NT) {
          a += V(vi)[r] * V(gj)[r];
          b += V(vi)[r] * V(kj)[r];
        }
        a = block_reduce<NT>(a, red);
        b = block_reduce<NT>(b, red);
        if (threadIdx.x == 0) {
          gram[i * ms + j] = gram[j * ms + i] = a;
          gram[NS * NS + i * ms + j] = gram[NS * NS + j * ms + i] = b;
        }
      }
    __syncthreads();
    if (threadIdx.x == 0) (void)rayleigh_ritz(gram, gram + NS * NS, ms, coef, mu, rr_wk, rr_iwk);
    __syncthreads();
    // new X = S c, new P = [W, P] c_{W,P}; images follow by linear combination
    for (int r = threadIdx.x; r < n; r += NT) {
      for (int grp = 0; grp < 3; ++grp) {
        const int base = grp == 0 ? 0 : grp == 1 ? V_KX : V_GX;
        double xs[NS];
        for (int i = 0; i < ms; ++i) {
          const int vi = (i < NB) ? V_X + i : (i < 2 * NB) ? V_W + i - NB : V_P + i - 2 * NB;
          xs[i] = V(vi + base)[r];
        }
        for (int v = 0; v < NB; ++v) {
          double nx = 0.0, np = 0.0;
          for (int i = 0; i < ms; ++i) {
            nx += coef[i * NB + v] * xs[i];
            if (i >= NB) np += coef[i * NB + v] * xs[i];
          }
          V(V_X + v + base)[r] = nx;
          V(V_P + v + base)[r] = np;
        }
      }
    }
    have_p = 1;
    __syncthreads();
  }
  const bool good = isfinite(mu0) && mu0 > 0.0 && isfinite(res0);
  const int st = !isfinite(res0) ? S_NAN : !(mu0 > 0.0) ? S_BREAKDOWN : (res0 > tol) ? S_NOCONV : S_OK;
  return EigResult{good ? 1.0 / mu0 : NAN, res0, it, st};
}

// Lowest-mode check (Eq. matrixeig asks for the smallest lambda, and LOBPCG
// stops at any eigenpair with a small residual).  K is positive definite and
// K_G semi-definite on the free unknowns, so K - sigma K_G is positive
// definite exactly when sigma is below the smallest eigenvalue lambda_1.  With
// sigma = lambda (1 - cert_shift) a Cholesky factorisation of the band of
// K - sigma K_G that meets no non-positive pivot shows lambda < lambda_1 /
// (1 - cert_shift): no eigenvalue lies below the computed one by more than
// the shift.  The band is assembled from the element matrix Ke - sigma KGe
// (Ke is overwritten) and factored in FP64.
__device__ void shift_elements(const PlateGeom &g, double lam, double *Ke, const double *KGe) {
  const double sigma = lam * (1.0 - g.cert_shift);
  __syncthreads();
  for (int k = threadIdx.x; k < 400; k += PT) Ke[k] -= sigma * KGe[k];
  __syncthreads();
}

// one work-group per sample from start to finish: the band of K assembled and
// factored, its diagonal blocks inverted, LOBPCG, then (FP64) the band of
// K - sigma K_G assembled and factored for the lowest-mode check.  In the FP64
// form both factorisations go through one call of the factorisation, so its
// code (and register allocation) is the same for both.
template <typename B>
// two waves per SIMD (a few registers spill): batches of small panels need the
// occupancy more than the solve's wide loads need registers
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(2))) void k_buckle(PlateGeom g, PlateMat m,
                                                                                       PlateWork W, PlateJob J,
                                                                                       double tol, int max_iter) {
  __shared__ double Ke[400], KGe[400], Dmb[36];
  // panel of the factorisation: FP64 room also in the FP32 form, for the FP64
  // lowest-mode check
  __shared__ double panel_mem[KP * LDP];
  B *panel = (B *)panel_mem;
  const int s = blockIdx.x;
  if (s >= J.n) return;
  sample_elements(g, m, J, s, Dmb, Ke, KGe);
  B *band = sizeof(B) == 8 ? (B *)(W.band + (size_t)s * W.band_stride) : (B *)(W.bandf + (size_t)s * W.band_stride);
  double *band64 = W.band + (size_t)s * W.band_stride;  // the check's band (free once LOBPCG is done)
  auto solve = [&]() {
    // diagonal blocks of the factor to their inverses (staged in the panel's LDS), then LOBPCG
    constexpr int nstage = (int)(sizeof(panel_mem) / (PS * PS * sizeof(B)));
    for (int b0 = 0; b0 * PS < g.nfree; b0 += nstage) invert_blocks<B>(band, g.bw + 1, g.nfree, b0, nstage, panel);
    __syncthreads();
    return lobpcg<B, RING_ONE, ONE_MAXBW - 1>(g, Ke, KGe, band, W.vec + (size_t)s * W.vec_stride, tol, max_iter);
  };
  EigResult r{};
  if constexpr (sizeof(B) == 8) {
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        if (!(r.status == S_OK && g.cert_shift > 0.0)) break;
        shift_elements(g, r.lam, Ke, KGe);
      }
      assemble_band<double>(g, Ke, band64, 0, g.nfree, threadIdx.x, PT);
      __syncthreads();
      const bool ok = band_cholesky<double>(g, band64, panel_mem);
      if (pass == 0) {
        if (!ok) {
          if (threadIdx.x == 0) write_result(J, s, NAN, 0, 0.0, S_BREAKDOWN);
          return;
        }
        r = solve();
      } else if (!ok) {
        r.status = S_NOTLOWEST;
      }
    }
  } else {
    assemble_band<B>(g, Ke, band, 0, g.nfree, threadIdx.x, PT);
    __syncthreads();
    if (!band_cholesky<B>(g, band, panel)) {
      if (threadIdx.x == 0) write_result(J, s, NAN, 0, 0.0, S_BREAKDOWN);
      return;
    }
    r = solve();
    // the FP64 band is free (the FP32 factor lives in its own band)
    if (r.status == S_OK && g.cert_shift > 0.0) {
      shift_elements(g, r.lam, Ke, KGe);
      assemble_band<double>(g, Ke, band64, 0, g.nfree, threadIdx.x, PT);
      __syncthreads();
      if (!band_cholesky<double>(g, band64, panel_mem)) r.status = S_NOTLOWEST;
    }
  }
  if (threadIdx.x == 0) write_result(J, s, r.lam, r.it, r.res, r.status);
}

// ---------------------------------------------------------------- wide factorisation
// Levels with a wide band spread one sample's factorisation over several
// work-groups, one launch per panel of NBK columns (the launch order takes the
// place of a grid-wide barrier).  In the launch of panel k0 every work-group
// loads the previous panel's factor columns on the rows of its trailing
// window; work-group 0 subtracts their product from the panel's own columns,
// factors the panel in LDS and writes it back, while the other work-groups
// subtract it from the rest of the window.  Every band entry receives the same
// updates, in the same order and with the same arithmetic, as in the
// one-work-group factorisation, so the factor is bit-identical.

// laminate and element matrices of each sample into W.kel; clears the pivot flag
__global__ __launch_bounds__(PT) void k_plate_prep(PlateGeom g, PlateMat m, PlateWork W, PlateJob J) {
  __shared__ double Ke[400], KGe[400], Dmb[36];
  const int s = blockIdx.x;
  if (s >= J.n) return;
  sample_elements(g, m, J, s, Dmb, Ke, KGe);
  double *kel = W.kel + (size_t)s * KEL;
  for (int k = threadIdx.x; k < 400; k += PT) {
    kel[k] = Ke[k];
    kel[400 + k] = KGe[k];
  }
  if (threadIdx.x == 0) W.flag[s] = 0;
}

template <typename B>
__device__ __forceinline__ B *sample_band(const PlateWork &W, int s) {
  return sizeof(B) == 8 ? (B *)(W.band + (size_t)s * W.band_stride) : (B *)(W.bandf + (size_t)s * W.band_stride);
}

// copy of the factored panel at k0 (column-major, KP x LDPW, row i at k0 + i),
// one of two per sample by the parity of k0 / KP: the next panel launch reads
// the previous panel's columns from it in rows (neighbouring threads,
// neighbouring entries) instead of in the band's row-major layout
template <typename B>
__device__ __forceinline__ B *panel_copy(const PlateWork &W, int s, int k0) {
  return (B *)(W.side + ((size_t)s * 2 + (k0 / KP) % 2) * (KP * LDPW));
}

// band rows [blockIdx.x * rows_per_wg, ...) of sample blockIdx.y
template <typename B>
__global__ __launch_bounds__(PT) void k_plate_assemble(PlateGeom g, PlateWork W, int n, int rows_per_wg) {
  __shared__ double Ke[400];
  const int s = blockIdx.y;
  if (s >= n) return;
  for (int k = threadIdx.x; k < 400; k += PT) Ke[k] = W.kel[(size_t)s * KEL + k];
  __syncthreads();
  const int r0 = blockIdx.x * rows_per_wg, r1 = min(g.nfree, r0 + rows_per_wg);
  if (r0 < r1) assemble_band<B>(g, Ke, sample_band<B>(W, s), r0, r1, threadIdx.x, PT);
}

// one panel of the wide factorisation (launch k0 / KP of a sample's band), in
// work-groups of NTB threads; a row's and a tile's arithmetic is one thread's
// whatever NTB, so the factor does not depend on it
template <typename B, int NTB>
__global__ __launch_bounds__(NTB) void k_band_step(PlateGeom g, PlateWork W, int n, int k0) {
  // one LDS area, column-major (columns contiguous: the tiles' reads are free of
  // bank conflicts): work-group 0 stages this panel in it (KP x LDPW), the others
  // the previous panel's columns on the rows of its trailing window (KP x MAXBW)
  __shared__ B S[KP * LDPW];
  __shared__ B Lq[KP * KP];  // work-group 0: the previous panel's columns on this panel's rows
  __shared__ int bad;
  const int s = blockIdx.y, wg = blockIdx.x, nwg = gridDim.x;
  if (s >= n) return;
  if (__builtin_amdgcn_readfirstlane(W.flag[s])) return;
  const int w = g.bw + 1, nf = g.nfree;
  B *band = sample_band<B>(W, s);
  // trailing window of the previous panel (columns k0 - KP .. k0 - 1): rows and
  // columns k0 .. k0 + m - 1; its sub-panels A (first NBK columns) and B
  const int m = (k0 > 0) ? min(g.bw, nf - k0) : 0;
  const int pA = (k0 > 0) ? NBK : 0, pB = (k0 > 0) ? NBK : 0;  // previous panels are always whole
  if (wg == 0) {
    if (k0 >= nf) return;
    B *P = S;
    const int nbA = min(NBK, nf - k0), nbB = max(0, min(NBK, nf - k0 - NBK)), nb = nbA + nbB;
    const int rows = min(nb + g.bw, nf - k0);  // panel rows k0 .. k0 + rows - 1
    if (threadIdx.x == 0) bad = 0;
    const B *prev = panel_copy<B>(W, s, k0 + KP);  // the previous panel's copy (parity of k0 - KP)
    // the previous panel's columns on this panel's rows (the pc side of its update)
    for (int idx = threadIdx.x; idx < KP * KP; idx += NTB) {
      const int j = idx / KP, c = idx % KP;  // row k0 + j, previous column k0 - KP + c
      const bool in = k0 > 0 && j < nb && j + KP - c <= g.bw;
      Lq[c * KP + j] = in ? prev[c * LDPW + KP + j] : B(0);
    }
    // the panel's entries, KP lanes per row (a row's entries in the panel's
    // columns are contiguous in the band)
    for (int idx = threadIdx.x; idx < rows * KP; idx += NTB) {
      const int i = idx / KP, j = idx % KP;
      const B v = band[(size_t)(k0 + i) * w + min(max(i - j, 0), g.bw)];
      P[j * LDPW + i] = (j < nb && i >= j && i - j <= g.bw) ? v : B(0);
    }
    __syncthreads();
    // each row of the panel less the previous panel's two NBK-term sums
    // (sub-panel A first) where the row is inside that panel's window
    for (int i = threadIdx.x; i < rows; i += NTB) {
      if (i < m) {
        B x[KP];  // the row's entries in the previous panel's columns (zero outside the band)
#pragma unroll
        for (int c = 0; c < KP; ++c) x[c] = (i + KP - c <= g.bw) ? prev[c * LDPW + KP + i] : B(0);
        for (int j = 0; j < min(nb, i + 1); ++j) {
          B accA = B(0), accB = B(0);
#pragma unroll
          for (int c = 0; c < NBK; ++c) accA += x[c] * Lq[c * KP + j];
#pragma unroll
          for (int c = NBK; c < KP; ++c) accB += x[c] * Lq[c * KP + j];
          B v = P[j * LDPW + i];
          v -= accA;
          v -= accB;
          P[j * LDPW + i] = v;
        }
      }
    }
    __syncthreads();
    // the panel: sub-panel A, A's product on B's columns, sub-panel B
    if (threadIdx.x == 0 && !factor_top<LDPW>(P, 0, nbA)) bad = 1;
    __syncthreads();
    if (bad) {
      if (threadIdx.x == 0) W.flag[s] = 1;
      return;
    }
    factor_rows<LDPW, B, NTB>(P, 0, nbA, nbA, rows);
    __syncthreads();
    if (nbB > 0) {
      update_b<LDPW, B, NTB>(P, nb, rows);
      __syncthreads();
      if (threadIdx.x == 0 && !factor_top<LDPW>(P, NBK, nbB)) bad = 1;
      __syncthreads();
      if (bad) {
        if (threadIdx.x == 0) W.flag[s] = 1;
        return;
      }
      factor_rows<LDPW, B, NTB>(P, NBK, nbB, nb, rows);
      __syncthreads();
    }
    for (int idx = threadIdx.x; idx < rows * KP; idx += NTB) {
      const int i = idx / KP, j = idx % KP;
      if (j < nb && i >= j && i - j <= g.bw) band[(size_t)(k0 + i) * w + (i - j)] = P[j * LDPW + i];
    }
    // the factored panel's copy for the next launch (rows of a column contiguous)
    B *cur = panel_copy<B>(W, s, k0);
    for (int idx = threadIdx.x; idx < KP * rows; idx += NTB) {
      const int j = idx / rows, i = idx % rows;
      cur[j * LDPW + i] = P[j * LDPW + i];
    }
    return;
  }
  // ---- the other work-groups: the rest of the previous panel's trailing window
  // (4 x 4 tiles of column offset >= KP), its sums A then B as in the
  // one-work-group form
  if (m <= 0 || nwg < 2) return;
  B *Lp = S;
  {
    const B *prev = panel_copy<B>(W, s, k0 + KP);  // the previous panel's copy
    for (int idx = threadIdx.x; idx < KP * m; idx += NTB) {
      const int j = idx / m, r = idx % m;
      Lp[j * MAXBW + r] = (r + KP - j <= g.bw) ? prev[j * LDPW + KP + r] : B(0);
    }
  }
  __syncthreads();
  const int mt = (m + 3) / 4, ntile = mt * (mt + 1) / 2;
  for (int tix = (wg - 1) * NTB + threadIdx.x; tix < ntile; tix += (nwg - 1) * NTB) {
    int ti = (int)((sqrtf(8.0f * tix + 1.0f) - 1.0f) * 0.5f);  // corrected below
    while ((ti + 1) * (ti + 2) / 2 <= tix) ++ti;
    while (ti * (ti + 1) / 2 > tix) --ti;
    const int tj = tix - ti * (ti + 1) / 2;
    if (tj < KP / 4) continue;  // columns of panel k0: work-group 0
    const int r0 = 4 * ti, c0 = 4 * tj;
    B v[4][4];
    tile_load(band, w, k0, m, r0, c0, v);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int j0 = half * NBK, j1 = half ? pA + pB : pA;
      B acc[4][4];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) acc[a][c] = B(0);
      for (int j = j0; j < j1; ++j) {
        B pr[4], pc[4];
        for (int a = 0; a < 4; ++a) {
          pr[a] = (r0 + a < m) ? Lp[j * MAXBW + r0 + a] : B(0);
          pc[a] = (c0 + a < m) ? Lp[j * MAXBW + c0 + a] : B(0);
        }
        for (int a = 0; a < 4; ++a)
          for (int c = 0; c < 4; ++c) acc[a][c] += pr[a] * pc[c];
      }
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) v[a][c] -= acc[a][c];
    }
    tile_store(band, w, k0, m, r0, c0, v);
  }
}

// diagonal blocks of each sample's factor to their inverses: 8 blocks per
// work-group (one per half-wave), grid (blocks / 8, samples)
template <typename B>
__global__ __launch_bounds__(PT) void k_invert_blocks(PlateGeom g, PlateWork W, int n) {
  __shared__ B Ls[8 * PS * PS];
  const int s = blockIdx.y;
  if (s >= n) return;
  if (__builtin_amdgcn_readfirstlane(W.flag[s])) return;
  invert_blocks<B>(sample_band<B>(W, s), g.bw + 1, g.nfree, blockIdx.x * 8, 8, Ls);
}

// LOBPCG of each sample on its factored band (element matrices from W.kel),
// one work-group of NT threads per sample
template <typename B, int NT>
__global__ __launch_bounds__(NT) void k_plate_lobpcg(PlateGeom g, PlateWork W, PlateJob J, double tol, int max_iter) {
  __shared__ double Ke[400], KGe[400];
  const int s = blockIdx.x;
  if (s >= J.n) return;
  for (int k = threadIdx.x; k < 400; k += NT) {
    Ke[k] = W.kel[(size_t)s * KEL + k];
    KGe[k] = W.kel[(size_t)s * KEL + 400 + k];
  }
  __syncthreads();
  if (__builtin_amdgcn_readfirstlane(W.flag[s])) {
    if (threadIdx.x == 0) write_result(J, s, NAN, 0, 0.0, S_BREAKDOWN);
    return;
  }
  const EigResult r = lobpcg<B, RING_WIDE, MAXBW, NT>(g, Ke, KGe, sample_band<B>(W, s), W.vec + (size_t)s * W.vec_stride, tol,
                                            max_iter);
  if (threadIdx.x == 0) {
    write_result(J, s, r.lam, r.it, r.res, r.status);
    W.lam[s] = r.lam;
    // samples the lowest-mode check skips stay flagged (2); the check's
    // factorisation sets 1 at a non-positive pivot
    W.flag[s] = (r.status == S_OK && g.cert_shift > 0.0) ? 0 : 2;
  }
}

// wide lowest-mode check, step 1: band of K - sigma K_G, sigma = lambda (1 -
// cert_shift), into the FP64 band of each checked sample (rows as in
// k_plate_assemble); the panel launches of k_band_step<double> then factor it
__global__ __launch_bounds__(PT) void k_cert_assemble(PlateGeom g, PlateWork W, int n, int rows_per_wg) {
  __shared__ double Kc[400];
  const int s = blockIdx.y;
  if (s >= n || __builtin_amdgcn_readfirstlane(W.flag[s])) return;
  const double sigma = W.lam[s] * (1.0 - g.cert_shift);
  for (int k = threadIdx.x; k < 400; k += PT) Kc[k] = W.kel[(size_t)s * KEL + k] - sigma * W.kel[(size_t)s * KEL + 400 + k];
  __syncthreads();
  const int r0 = blockIdx.x * rows_per_wg, r1 = min(g.nfree, r0 + rows_per_wg);
  if (r0 < r1) assemble_band<double>(g, Kc, W.band + (size_t)s * W.band_stride, r0, r1, threadIdx.x, PT);
}

// wide lowest-mode check, step 3: a sample whose factorisation met a
// non-positive pivot has a lower eigenvalue
__global__ void k_cert_finish(PlateWork W, PlateJob J) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= J.n || W.flag[s] != 1) return;
  const int o = J.out_idx[s];
  if (J.coarse) J.info[o].status_c = S_NOTLOWEST;
  else J.info[o].status_f = S_NOTLOWEST;
}

// diagnostic: y = K x or K_G x on full-dof vectors (constrained unknowns: y = 0)
__global__ __launch_bounds__(PT) void k_plate_apply(PlateGeom g, PlateMat m, const double *offsets, int geom,
                                                    const double *x, double *y, double *xf, double *yf) {
  __shared__ double Ke[400], KGe[400], Dmb[36];
  const int s = blockIdx.x;
  if (threadIdx.x == 0) laminate_dmb(m, offsets + (size_t)s * m.nply, Dmb);
  __syncthreads();
  element_matrices(g, m, Dmb, Ke, KGe);
  __syncthreads();
  double *xs = xf + (size_t)s * g.nfree, *ys = yf + (size_t)s * g.nfree;
  for (int r = threadIdx.x; r < g.nfree; r += PT) xs[r] = x[(size_t)s * g.nfull + g.full_of_free[r]];
  __syncthreads();
  if (geom) plate_apply<true>(g, KGe, xs, ys);
  else plate_apply<false>(g, Ke, xs, ys);
  __syncthreads();
  for (int r = threadIdx.x; r < g.nfull; r += PT) {
    const int f = g.free_of_full[r];
    y[(size_t)s * g.nfull + r] = f >= 0 ? ys[f] : 0.0;
  }
}

// ====================================================================== host
struct PlateLevelH {
  PlateGeom g{};
  int *d_free_of_full = nullptr, *d_full_of_free = nullptr;
  // batch workspace
  int cap = 0;
  size_t bytes = 0;
  double *band = nullptr, *vec = nullptr, *kel = nullptr, *side = nullptr;
  float *bandf = nullptr;
  int64_t *rows = nullptr;
  int *outidx = nullptr, *flag = nullptr;
  double *lam = nullptr;
};

struct PlateCtx {
  int nlev = 0;
  PlateMat mat{};
  double tol = 1e-8;
  int max_iter = 500;
  std::vector<PlateLevelH> lv;
  double *d_xf = nullptr, *d_yf = nullptr;
  size_t xf_cap = 0;
  size_t budget = 0;               // bound on the batch workspaces of all levels
  int wide_min_bw = 200;  // factorise over several work-groups from this band width on (0: from ONE_MAXBW on)
  int wide_eig_threads = 1024;  // threads of the wide-band eigensolver's work-group (256 or 1024)
  int wide_factor_threads = 1024;  // threads of a panel launch's work-groups (256 or 1024)
  double wide_batch_per_bw = 1.5;  // narrower bands: batches of at most this times bw take the wide form
};

// the factorisation spread over work-groups: element matrices, band assembly
// (256 rows per work-group), one launch per panel, then LOBPCG per sample in
// one work-group of eig_nt threads
template <typename B, int NTB>
static void launch_band_steps(const PlateGeom &g, const PlateWork &W, int n, hipStream_t st) {
  // work-groups per sample: work-group 0 plus enough for the window's 4 x 4
  // tiles (one per thread), fewer when many samples share the launch
  const int mt = (g.bw + 3) / 4, ntile = mt * (mt + 1) / 2;
  const int need = 1 + (ntile + NTB - 1) / NTB;
  const int nwg = std::max(2, std::min(need, std::max(2, (2048 * PT / NTB) / std::max(n, 1))));
  for (int k0 = 0; k0 < g.nfree; k0 += KP)
    hipLaunchKernelGGL((k_band_step<B, NTB>), dim3(nwg, n), dim3(NTB), 0, st, g, W, n, k0);
}

template <typename B>
static void band_steps(const PlateGeom &g, const PlateWork &W, int n, int ntb, hipStream_t st) {
  if (ntb == 1024)
    launch_band_steps<B, 1024>(g, W, n, st);
  else
    launch_band_steps<B, PT>(g, W, n, st);
}

template <typename B>
static void launch_wide(const PlateGeom &g, const PlateMat &m, const PlateWork &W, const PlateJob &J, int n,
                        double tol, int max_iter, int eig_nt, int ntb, hipStream_t st) {
  hipLaunchKernelGGL(k_plate_prep, dim3(n), dim3(PT), 0, st, g, m, W, J);
  const int rows_per_wg = 256;
  hipLaunchKernelGGL(k_plate_assemble<B>, dim3((g.nfree + rows_per_wg - 1) / rows_per_wg, n), dim3(PT), 0, st, g, W,
                     n, rows_per_wg);
  band_steps<B>(g, W, n, ntb, st);
  const int nblk = (g.nfree + PS - 1) / PS;
  hipLaunchKernelGGL(k_invert_blocks<B>, dim3((nblk + 7) / 8, n), dim3(PT), 0, st, g, W, n);
  if (eig_nt == 1024)
    hipLaunchKernelGGL((k_plate_lobpcg<B, 1024>), dim3(n), dim3(1024), 0, st, g, W, J, tol, max_iter);
  else
    hipLaunchKernelGGL((k_plate_lobpcg<B, PT>), dim3(n), dim3(PT), 0, st, g, W, J, tol, max_iter);
  if (g.cert_shift > 0.0) {
    // lowest-mode check: FP64 factorisation of K - sigma K_G, spread as above
    hipLaunchKernelGGL(k_cert_assemble, dim3((g.nfree + rows_per_wg - 1) / rows_per_wg, n), dim3(PT), 0, st, g, W,
                       n, rows_per_wg);
    band_steps<double>(g, W, n, ntb, st);
    hipLaunchKernelGGL(k_cert_finish, dim3((n + 255) / 256), dim3(256), 0, st, W, J);
  }
}

static PlateGeom plate_geom(const Json &cfg, int level) {
  PlateGeom g{};
  g.nx = (int)cfg.number("nx0") << level;
  g.ny = (int)cfg.number("ny0") << level;
  g.nnx = g.nx + 1;
  g.nny = g.ny + 1;
  g.nn = g.nnx * g.nny;
  g.nfull = 5 * g.nn;
  g.a = cfg.number("a");
  g.b = cfg.number("b");
  g.hx = g.a / g.nx;
  g.hy = g.b / g.ny;
  return g;
}

// hard simply-supported edges: w = 0 on all edges, tangential rotation = 0,
// u = 0 on x = 0 and v = 0 on y = 0 (removes the in-plane rigid motions)
static bool constrained(const PlateGeom &g, int full) {
  const int node = full / 5, c = full % 5, i = node % g.nnx, j = node / g.nnx;
  const bool xe = (i == 0 || i == g.nx), ye = (j == 0 || j == g.ny);
  if (c == 2) return xe || ye;
  if (c == 4) return xe;
  if (c == 3) return ye;
  if (c == 0) return i == 0;
  if (c == 1) return j == 0;
  return false;
}

PlateCtx *plate_create(const Json &cfg, std::string &err) {
  PlateCtx *p = new PlateCtx();
  try {
    p->nlev = (int)cfg.number("n_levels");
    if (p->nlev < 1 || p->nlev > 8) throw std::runtime_error("n_levels out of range");
    const Json &mm = cfg.at("material");
    const double E1 = mm.number("E11"), E2 = mm.number("E22"), G = mm.number("G12"), nu12 = mm.number("nu12");
    const double nu21 = nu12 * E2 / E1, den = 1.0 - nu12 * nu21;
    p->mat.Q11 = E1 / den;
    p->mat.Q22 = E2 / den;
    p->mat.Q12 = nu12 * E2 / den;
    p->mat.Q66 = G;
    std::vector<double> lay = cfg.numbers("layup_deg");
    if (lay.empty() || (int)lay.size() > MAXPLY) throw std::runtime_error("layup_deg needs 1..32 plies");
    p->mat.nply = (int)lay.size();
    for (size_t k = 0; k < lay.size(); ++k) p->mat.layup[k] = lay[k] * M_PI / 180.0;
    p->mat.t_ply = cfg.number("ply_t");
    const double t = p->mat.t_ply * p->mat.nply;
    p->mat.shear_k_G_t = cfg.number_or("shear_k", 5.0 / 6.0) * G * t;
    p->mat.N0 = cfg.number_or("N0", 1.0);
    const std::string shear = cfg.string_or("shear", "sri");
    if (shear != "sri" && shear != "mitc4") throw std::runtime_error("shear must be sri or mitc4");
    p->mat.mitc4 = shear == "mitc4";
    p->mat.condensed = 0;
    if (cfg.has("condensed")) {
      if (cfg.at("condensed").type != Json::Bool) throw std::runtime_error("condensed must be true or false");
      p->mat.condensed = cfg.at("condensed").b;
    }
    p->tol = cfg.number_or("eig_tol", 1e-8);
    p->max_iter = (int)cfg.number_or("eig_max_iter", 500);
    // band width from which one sample's factorisation is spread over work-groups
    p->wide_min_bw = (int)cfg.number_or("wide_factor_min_bw", 200);
    // threads of the wide-band eigensolver's work-group: 1024 keeps a step's
    // band entries in flight at once; 256 is the one-work-group kernel's form
    p->wide_eig_threads = (int)cfg.number_or("wide_eig_threads", 1024);
    if (p->wide_eig_threads != 256 && p->wide_eig_threads != 1024)
      throw std::runtime_error("wide_eig_threads must be 256 or 1024");
    // threads of a panel launch's work-groups (the factor is the same either way)
    p->wide_factor_threads = (int)cfg.number_or("wide_factor_threads", 1024);
    if (p->wide_factor_threads != 256 && p->wide_factor_threads != 1024)
      throw std::runtime_error("wide_factor_threads must be 256 or 1024");
    // batches of bands narrower than that of at most wide_batch_per_bw * bw
    // samples leave the one-work-group kernel's slots mostly empty: they take
    // the wide factorisation with the one-work-group eigensolver's order of
    // sums (the same results to the bit); 0 keeps them in the one-work-group kernel
    p->wide_batch_per_bw = cfg.number_or("wide_batch_per_bw", 1.5);
    if (!(p->wide_batch_per_bw >= 0.0)) throw std::runtime_error("wide_batch_per_bw must be >= 0");
    // half-waves along x of the first LOBPCG start vector (0: nearest to a / b)
    const int start_p0 = (int)cfg.number_or("eig_start_p0", 0);
    if (start_p0 < 0 || start_p0 > 64) throw std::runtime_error("eig_start_p0 must be in 0..64");
    // relative shift of the lowest-mode check (0 turns it off)
    const double cert_shift = cfg.number_or("cert_shift", 1e-6);
    if (!(cert_shift >= 0.0 && cert_shift < 0.5)) throw std::runtime_error("cert_shift must be in [0, 0.5)");
    p->lv.resize(p->nlev);
    for (int l = 0; l < p->nlev; ++l) {
      PlateLevelH &L = p->lv[l];
      L.g = plate_geom(cfg, l);
      L.g.start_p0 = start_p0;
      L.g.cert_shift = cert_shift;
      std::vector<int> fof(L.g.nfull, -1), fo;
      for (int f = 0; f < L.g.nfull; ++f)
        if (!constrained(L.g, f)) {
          fof[f] = (int)fo.size();
          fo.push_back(f);
        }
      L.g.nfree = (int)fo.size();
      int bw = 0;
      for (int r = 0; r < L.g.nfree; ++r) {
        const int nr = fo[r] / 5, ir = nr % L.g.nnx, jr = nr / L.g.nnx;
        // furthest coupled free unknown below r: node (i-1, j-1), component 0
        for (int dj = -1; dj <= 0; ++dj)
          for (int di = -1; di <= 1; ++di) {
            const int ic = ir + di, jc = jr + dj;
            if (ic < 0 || ic >= L.g.nnx || jc < 0) continue;
            for (int c = 0; c < 5; ++c) {
              const int f = fof[5 * (jc * L.g.nnx + ic) + c];
              if (f >= 0 && f < r) bw = std::max(bw, r - f);
            }
          }
      }
      L.g.bw = bw;
      if (bw > MAXBW) throw std::runtime_error("plate band too wide (mesh finer than 128 x 128 per side)");
      if (hipMalloc(&L.d_free_of_full, sizeof(int) * L.g.nfull) != hipSuccess ||
          hipMalloc(&L.d_full_of_free, sizeof(int) * L.g.nfree) != hipSuccess)
        throw std::runtime_error("device allocation failed");
      (void)hipMemcpy(L.d_free_of_full, fof.data(), sizeof(int) * L.g.nfull, hipMemcpyHostToDevice);
      (void)hipMemcpy(L.d_full_of_free, fo.data(), sizeof(int) * L.g.nfree, hipMemcpyHostToDevice);
      L.g.free_of_full = L.d_free_of_full;
      L.g.full_of_free = L.d_full_of_free;
    }
  } catch (const std::exception &e) {
    err = e.what();
    plate_destroy(p);
    return nullptr;
  }
  return p;
}

static void free_work(PlateLevelH &L) {
  if (L.band) (void)hipFree(L.band);
  if (L.bandf) (void)hipFree(L.bandf);
  if (L.vec) (void)hipFree(L.vec);
  if (L.rows) (void)hipFree(L.rows);
  if (L.outidx) (void)hipFree(L.outidx);
  if (L.kel) (void)hipFree(L.kel);
  if (L.flag) (void)hipFree(L.flag);
  if (L.lam) (void)hipFree(L.lam);
  if (L.side) (void)hipFree(L.side);
  L.side = nullptr;
  L.lam = nullptr;
  L.kel = nullptr;
  L.flag = nullptr;
  L.band = L.vec = nullptr;
  L.bandf = nullptr;
  L.rows = nullptr;
  L.outidx = nullptr;
  L.cap = 0;
  L.bytes = 0;
}

// workspace of one in-flight sample: FP64 and FP32 band factors plus the
// LOBPCG vectors (both precisions share one allocation so that a level's
// workspace serves either)
static size_t work_bytes(const PlateLevelH &L) {
  const size_t bs = (size_t)L.g.nfree * (L.g.bw + 1);
  return bs * (sizeof(double) + sizeof(float)) + (size_t)NVEC * L.g.nfree * sizeof(double) + sizeof(int64_t) +
         2 * sizeof(int) + (KEL + 1) * sizeof(double) + 2 * (size_t)KP * LDPW * sizeof(double);
}

// grow the workspace of level l to at least n samples within the budget
static int ensure_work(PlateCtx *p, std::string &err, int l, int n) {
  PlateLevelH &L = p->lv[l];
  if (L.cap >= n) return MLMC_OK;
  size_t other = 0;
  for (int k = 0; k < p->nlev; ++k)
    if (k != l) other += p->lv[k].bytes;
  const size_t need = work_bytes(L) * (size_t)n;
  if (other + need > p->budget) {
    err = "plate level " + std::to_string(l) + ": " + std::to_string(n) + " samples exceed the memory budget";
    return MLMC_ENOMEM;
  }
  free_work(L);
  const size_t bs = (size_t)L.g.nfree * (L.g.bw + 1);
  if (hipMalloc(&L.band, (bs * n + BAND_PAD) * sizeof(double)) != hipSuccess ||
      hipMalloc(&L.bandf, (bs * n + BAND_PAD) * sizeof(float)) != hipSuccess ||
      hipMalloc(&L.vec, (size_t)NVEC * L.g.nfree * sizeof(double) * n) != hipSuccess ||
      hipMalloc(&L.rows, sizeof(int64_t) * n) != hipSuccess || hipMalloc(&L.outidx, sizeof(int) * n) != hipSuccess ||
      hipMalloc(&L.kel, sizeof(double) * KEL * n) != hipSuccess || hipMalloc(&L.flag, sizeof(int) * n) != hipSuccess ||
      hipMalloc(&L.lam, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&L.side, sizeof(double) * 2 * KP * LDPW * n) != hipSuccess) {
    free_work(L);
    err = "plate workspace allocation failed";
    return MLMC_ENOMEM;
  }
  L.cap = n;
  L.bytes = need;
  return MLMC_OK;
}

// largest batch of level l that fits beside the other levels' workspaces
static int max_work(const PlateCtx *p, int l) {
  size_t other = 0;
  for (int k = 0; k < p->nlev; ++k)
    if (k != l) other += p->lv[k].bytes;
  if (p->budget <= other) return 0;
  return (int)std::min<size_t>((p->budget - other) / work_bytes(p->lv[l]), 2048);
}

void plate_destroy(PlateCtx *p) {
  if (!p) return;
  for (auto &L : p->lv) {
    free_work(L);
    if (L.d_free_of_full) (void)hipFree(L.d_free_of_full);
    if (L.d_full_of_free) (void)hipFree(L.d_full_of_free);
  }
  if (p->d_xf) (void)hipFree(p->d_xf);
  if (p->d_yf) (void)hipFree(p->d_yf);
  delete p;
}

int plate_num_levels(const PlateCtx *p) { return p->nlev; }

void plate_level_sizes(const PlateCtx *p, int level, int64_t *nn, int64_t *nd, int64_t *ne) {
  const PlateGeom &g = p->lv[level].g;
  *nn = g.nn;
  *nd = g.nfull;
  *ne = (int64_t)g.nx * g.ny;
}

size_t plate_slot_bytes(const PlateCtx *p, int level, int /*precision*/) { return work_bytes(p->lv[level]); }

int plate_reserve(PlateCtx *p, std::string &err, int level, int n) {
  if (level < 0 || level >= p->nlev || n < 0) { err = "level out of range or n < 0"; return MLMC_EINVAL; }
  return ensure_work(p, err, level, n);
}

void plate_set_budget(PlateCtx *p, size_t bytes) { p->budget = bytes; }

int plate_buckle_batch(PlateCtx *p, std::string &err, int n_req, const mlmc_request *req, const double *offsets,
                       int64_t n_rows, double *lam_fine, double *lam_coarse, mlmc_info *info, int precision,
                       double tol, hipStream_t st) {
  if (n_req < 0) { err = "n_req < 0"; return MLMC_EINVAL; }
  if (n_req == 0) return MLMC_OK;
  if (!req || !offsets || !lam_fine || !lam_coarse || !info) { err = "null pointer"; return MLMC_EINVAL; }
  if (precision != MLMC_FP64 && precision != MLMC_MIXED) { err = "bad precision"; return MLMC_EINVAL; }
  for (int i = 0; i < n_req; ++i) {
    if (req[i].level < 0 || req[i].level >= p->nlev) { err = "request " + std::to_string(i) + ": bad level"; return MLMC_EINVAL; }
    if (req[i].sample < 0 || req[i].sample >= n_rows) {
      err = "request " + std::to_string(i) + ": sample row outside [0, n_rows)";
      return MLMC_EINVAL;
    }
  }
  const double tl = tol > 0 ? tol : p->tol;
  launch_info_init(info, lam_coarse, n_req, st);
  std::vector<std::vector<int64_t>> rows(2 * p->nlev);
  std::vector<std::vector<int>> outs(2 * p->nlev);
  for (int i = 0; i < n_req; ++i) {
    const int l = req[i].level;
    rows[2 * l].push_back(req[i].sample);
    outs[2 * l].push_back(i);
    if (req[i].coupled && l > 0) {
      rows[2 * (l - 1) + 1].push_back(req[i].sample);
      outs[2 * (l - 1) + 1].push_back(i);
    }
  }
  const bool mixed = precision == MLMC_MIXED;
  for (int l = 0; l < p->nlev; ++l) {
    PlateLevelH &L = p->lv[l];
    for (int coarse = 0; coarse < 2; ++coarse) {
      const auto &R = rows[2 * l + coarse];
      const auto &O = outs[2 * l + coarse];
      const int total = (int)R.size();
      if (!total) continue;
      // batch capacity: what is reserved, else what fits the budget (at most 2048)
      const int cap = std::max(L.cap, std::min(total, max_work(p, l)));
      if (cap < 1) {
        err = "plate level " + std::to_string(l) + ": no sample fits the memory budget";
        return MLMC_ENOMEM;
      }
      if (int rc = ensure_work(p, err, l, cap)) return rc;
      PlateWork Wk{};
      Wk.band = L.band;
      Wk.bandf = L.bandf;
      Wk.vec = L.vec;
      Wk.kel = L.kel;
      Wk.flag = L.flag;
      Wk.lam = L.lam;
      Wk.side = L.side;
      Wk.band_stride = (size_t)L.g.nfree * (L.g.bw + 1);
      Wk.vec_stride = (size_t)NVEC * L.g.nfree;
      for (int off = 0; off < total; off += cap) {
        const int n = std::min(cap, total - off);
        if (hipMemcpyAsync(L.rows, R.data() + off, sizeof(int64_t) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(L.outidx, O.data() + off, sizeof(int) * n, hipMemcpyHostToDevice, st) != hipSuccess) {
          err = "copy failed";
          return MLMC_EHIP;
        }
        PlateJob J{offsets, L.rows, L.outidx, coarse ? lam_coarse : lam_fine, info, coarse, n};
        const bool wide_band = L.g.bw >= ONE_MAXBW || (p->wide_min_bw > 0 && L.g.bw >= p->wide_min_bw);
        const bool small_batch = !wide_band && n <= p->wide_batch_per_bw * L.g.bw;
        if (wide_band || small_batch) {
          // a small batch of a narrower band keeps the one-work-group order of sums
          const int eig_nt = wide_band ? p->wide_eig_threads : PT;
          if (mixed)
            launch_wide<float>(L.g, p->mat, Wk, J, n, tl, p->max_iter, eig_nt, p->wide_factor_threads, st);
          else
            launch_wide<double>(L.g, p->mat, Wk, J, n, tl, p->max_iter, eig_nt, p->wide_factor_threads, st);
        } else if (mixed) {
          hipLaunchKernelGGL(k_buckle<float>, dim3(n), dim3(PT), 0, st, L.g, p->mat, Wk, J, tl, p->max_iter);
        } else {
          hipLaunchKernelGGL(k_buckle<double>, dim3(n), dim3(PT), 0, st, L.g, p->mat, Wk, J, tl, p->max_iter);
        }
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
          err = std::string("buckle kernel: ") + hipGetErrorString(e);
          return MLMC_EHIP;
        }
      }
    }
  }
  return MLMC_OK;
}

int plate_apply_diag(PlateCtx *p, std::string &err, int level, int n, const double *offsets, int geom,
                     const double *x, double *y, hipStream_t st) {
  if (level < 0 || level >= p->nlev || n < 0) { err = "level out of range or n < 0"; return MLMC_EINVAL; }
  if (n == 0) return MLMC_OK;
  PlateLevelH &L = p->lv[level];
  const size_t need = (size_t)n * L.g.nfree;
  if (p->xf_cap < need) {
    if (p->d_xf) (void)hipFree(p->d_xf);
    if (p->d_yf) (void)hipFree(p->d_yf);
    if (hipMalloc(&p->d_xf, need * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->d_yf, need * sizeof(double)) != hipSuccess) {
      err = "allocation failed";
      return MLMC_ENOMEM;
    }
    p->xf_cap = need;
  }
  hipLaunchKernelGGL(k_plate_apply, dim3(n), dim3(PT), 0, st, L.g, p->mat, offsets, geom, x, y, p->d_xf, p->d_yf);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) { err = hipGetErrorString(e); return MLMC_EHIP; }
  return MLMC_OK;
}

}  // namespace mlmc
