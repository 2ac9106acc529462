// C ABI of the MLMC sample-solve library: context, level hierarchy, device
// pools and the host loop around the HIP kernels.  The declarations and their
// contracts are in include/mlmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.hpp"
#include "cosserat.hpp"
#include "json.hpp"
#include "kl_setup.hpp"
#include "mlmc.h"
#include "plate.hpp"
#include "strip_kernels.hpp"
#include "strip_small.hpp"

using namespace mlmc;

namespace {

thread_local std::string g_create_error;

struct StripPool {
  int cap = 0;
  double *x = nullptr, *z = nullptr, *p = nullptr, *Ap = nullptr, *dg = nullptr, *theta = nullptr;
  double *part_pap = nullptr, *part_rz = nullptr, *part_rr = nullptr, *rzs = nullptr;
  double *tol2 = nullptr, *bb = nullptr, *relres = nullptr, *qpart = nullptr, *xa = nullptr;
  int *it_a = nullptr, *it_b = nullptr, *status = nullptr, *active = nullptr, *outidx = nullptr, *xs = nullptr;
  int64_t *rows = nullptr;
  size_t bytes = 0;
  // mixed precision (allocated on first use): FP64 rhs, FP32 or BF16 angles, FP32 inner solver
  bool has_mixed = false;
  double *b64 = nullptr, *m_part_rr = nullptr, *m_relres = nullptr, *f_rr_ref = nullptr;
  int *m_updates = nullptr, *f_ru = nullptr;
  void *theta16 = nullptr;  // inner-solver angles: bfloat16 or FP32
  float *fx = nullptr, *fz = nullptr, *fp = nullptr, *fAp = nullptr, *fdg = nullptr;
  double *f_pap = nullptr, *f_rz = nullptr, *f_rr = nullptr, *f_rzs = nullptr, *f_tol2 = nullptr, *f_bb = nullptr,
         *f_relres = nullptr, *f_xa = nullptr;
  int *f_it_a = nullptr, *f_it_b = nullptr, *f_status = nullptr, *f_active = nullptr, *f_xs = nullptr;
  size_t mixed_bytes = 0;
};

struct StripLevel {
  StripGeom g{};
  double *modes = nullptr;  // dev [4 nelem][K], sqrt(mu) folded in
  StripPool pool;
  bool small = false;       // solved by the one-work-group-per-sample kernel
  bool cs = false;          // FP64 angle data stored as (cos 2theta, sin 2theta) pairs
  int sweep_rows = 0;       // operator-pass tile height of this mesh (0: chosen per launch)
};

}  // namespace

struct mlmc_ctx {
  std::string err;
  Json cfg;
  int kind = 0;  // 0 strip, 1 plate, 2 Cosserat strip (Test Problem I)
  int nlev = 0;
  int K = 0;
  StripMat mat{};
  double rtol = 1e-10;
  int max_iter = 100000;
  double ru_factor = 0.1;   // reliable update when the FP32 residual fell by this factor
  // FP64 residual checks every ru_every iterations.  Slots ask rarely (about
  // every 350 inner iterations at the default factor), so most checks find
  // nothing to do and cost two launches per level group: on the four-level
  // benchmark 16 gives 493 ms per mixed step against 500 (8) and 514 (4), for
  // 1.4% more inner iterations
  int ru_every = 16;
  int theta_fp32 = 1;       // mixed: angles stored as FP32 (1) or bfloat16 (0)
  std::vector<StripLevel> lv;
  size_t budget = 0, used = 0;
  int *h_active = nullptr;
  int h_active_cap = 0;
  double *d_stats = nullptr, *h_stats = nullptr;
  PlateCtx *plate = nullptr;
  CosCtx *cos = nullptr;
  int device = 0;
  // diagnostics: event timing of the PCG passes
  bool prof = false;
  std::vector<hipEvent_t> ev;
  double prof_ms[4] = {0, 0, 0, 0}, prof_bytes[4] = {0, 0, 0, 0}, prof_dofs[4] = {0, 0, 0, 0};
  int64_t prof_launches[4] = {0, 0, 0, 0};
  std::vector<int> h_iters;
  // group descriptors of the lock-step launches (device copy + pinned staging)
  PcgGroup<double> *d_grp64 = nullptr, *h_grp64 = nullptr;
  PcgGroup<float> *d_grp32 = nullptr, *h_grp32 = nullptr;
  // graph replay of iteration blocks: capture stream, device iteration base,
  // and instantiated graphs keyed by the launch configuration they captured
  bool graphs = false;      // measured: no gain on MI355X (iterations are GPU-bound), so off by default
  int sweep_rows = 0;       // operator-pass tile height: 0 = chosen per launch, else 4, 8 or 16
  // lock-step launches whose vectors and angles exceed this many bytes use
  // streaming accesses for the vectors that pass through once (the default is
  // the size of MI355X's Infinity Cache)
  double streaming_min_bytes = 256.0 * 1048576.0;
  hipStream_t cap_stream = nullptr;
  // whole-solve levels of a batch run on side_stream, next to the lock-step
  // launches on the caller's stream (fork after the set-up, join before the end)
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int *d_itb = nullptr;
  // device address of this GPU's fixed scratch array (mlmc_strip_solve_theta_noalloc)
  void *scratch = nullptr;
  std::string scratch_err;
  struct CachedGraph {
    std::vector<char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<CachedGraph> gcache;
};

namespace {

int fail(mlmc_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, MLMC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

// tile height of the operator pass (a multiple of SWEEP_RB)
// tiles of `ty` node rows; a remainder of at most half a tile joins the last
// tile instead of making a row of near-empty tiles (a mesh of 2^k element rows
// has 2^k + 1 node rows)
void set_sweep_rows(StripGeom &g, int ty) {
  g.sw_ty = ty;
  const int full = g.nny / ty, rem = g.nny - full * ty;
  g.sw_nty = (full == 0) ? 1 : (rem <= ty / 2 ? full : full + 1);
  g.sw_ntiles = g.sw_ntx * g.sw_nty;
}

StripGeom make_geom(const Json &cfg, int level) {
  StripGeom g{};
  g.nx = (int)cfg.number("nx0") << level;
  g.ny = (int)cfg.number("ny0") << level;
  g.nnx = g.nx + 1;
  g.nny = g.ny + 1;
  g.nnode = g.nnx * g.nny;
  g.nelem = g.nx * g.ny;
  g.tiles_x = (g.nnx + TILE_X - 1) / TILE_X;
  g.tiles_y = (g.nny + TILE_Y - 1) / TILE_Y;
  g.ntiles = g.tiles_x * g.tiles_y;
  g.sw_ntx = (g.nnx + SWEEP_MAXW - 1) / SWEEP_MAXW;
  g.sw_tw = (g.nnx + g.sw_ntx - 1) / g.sw_ntx;
  set_sweep_rows(g, SWEEP_MAXTY);
  g.sw_npart = ((g.nny + SWEEP_RB - 1) / SWEEP_RB) * g.sw_ntx;
  g.nchunks = (g.nnode + CHUNK - 1) / CHUNK;
  g.Lx = cfg.number("Lx");
  g.Ly = cfg.number("Ly");
  g.hx = g.Lx / g.nx;
  g.hy = g.Ly / g.ny;
  g.ihx = 1.0 / g.hx;
  g.ihy = 1.0 / g.hy;
  g.wdet = 0.25 * g.hx * g.hy;
  g.pxi = GP_P * g.ihx;
  g.mxi = GP_M * g.ihx;
  g.pyi = GP_P * g.ihy;
  g.myi = GP_M * g.ihy;
  g.pxw = GP_P * g.ihx * g.wdet;
  g.mxw = GP_M * g.ihx * g.wdet;
  g.pyw = GP_P * g.ihy * g.wdet;
  g.myw = GP_M * g.ihy * g.wdet;
  g.delta = cfg.number("delta");
  std::vector<double> reg = cfg.numbers("qoi_region");
  if (reg.size() != 4) throw std::runtime_error("qoi_region needs 4 numbers");
  // elements whose centroid (e + 1/2) h lies in [lo, hi]
  g.qx0 = std::max(0, (int)std::ceil(reg[0] / g.hx - 0.5));
  g.qx1 = std::min(g.nx, (int)std::floor(reg[1] / g.hx - 0.5) + 1);
  g.qy0 = std::max(0, (int)std::ceil(reg[2] / g.hy - 0.5));
  g.qy1 = std::min(g.ny, (int)std::floor(reg[3] / g.hy - 0.5) + 1);
  if (g.qx1 <= g.qx0 || g.qy1 <= g.qy0) throw std::runtime_error("qoi_region holds no element centroid");
  return g;
}

StripMat make_material(const Json &cfg) {
  const Json &m = cfg.at("material");
  const double E1 = m.number("E11"), E2 = m.number("E22"), G = m.number("G12"), nu12 = m.number("nu12");
  const double nu21 = nu12 * E2 / E1, den = 1.0 - nu12 * nu21;
  StripMat s{};
  s.Q11 = E1 / den;
  s.Q22 = E2 / den;
  s.Q12 = nu12 * E2 / den;
  s.Q66 = G;
  s.U1 = (3 * s.Q11 + 3 * s.Q22 + 2 * s.Q12 + 4 * s.Q66) / 8;
  s.U2 = (s.Q11 - s.Q22) / 2;
  s.U3 = (s.Q11 + s.Q22 - 2 * s.Q12 - 4 * s.Q66) / 8;
  s.U4 = (s.Q11 + s.Q22 + 6 * s.Q12 - 4 * s.Q66) / 8;
  s.U5 = (s.Q11 + s.Q22 - 2 * s.Q12 + 4 * s.Q66) / 8;
  s.fU1 = (float)s.U1;
  s.fU2 = (float)s.U2;
  s.fU3 = (float)s.U3;
  s.fU4 = (float)s.U4;
  s.fU5 = (float)s.U5;
  return s;
}

size_t strip_mixed_slot_bytes(const StripGeom &g) {
  const size_t n2 = (size_t)2 * g.nnode;
  return n2 * sizeof(double)                               // b
         + (size_t)4 * g.nelem * sizeof(float)             // inner angles (BF16 or FP32)
         + 5 * n2 * sizeof(float)                          // FP32 x, z, p, Ap, dg
         + (size_t)(2 * g.sw_npart + 4 * g.nchunks) * sizeof(double) + 16 * sizeof(double);  // and scalars
}

size_t strip_slot_bytes(const StripGeom &g) {
  const size_t vec = (size_t)2 * g.nnode * sizeof(double);
  return 5 * vec                                      // x, z, p, Ap, dg
         + (size_t)8 * g.nelem * sizeof(double)       // (cos 2theta, sin 2theta) per Gauss point
         + (size_t)(g.sw_npart + 4 * g.nchunks) * sizeof(double)   // partials
         + (size_t)qoi_parts(g) * sizeof(double)      // QoI partial maxima
         + 8 * sizeof(double) + 8 * sizeof(int) + sizeof(int64_t);
}

void free_pool(mlmc_ctx *c, StripPool &p) {
  void *bufs[] = {p.x, p.z, p.p, p.Ap, p.dg, p.theta, p.part_pap, p.part_rz, p.part_rr, p.rzs, p.tol2, p.bb,
                  p.relres, p.qpart, p.xa, p.it_a, p.it_b, p.status, p.active, p.outidx, p.xs, p.rows,
                  p.b64, p.m_part_rr, p.m_relres, p.f_rr_ref, p.m_updates, p.f_ru,
                  p.theta16, p.fx, p.fz, p.fp, p.fAp, p.fdg, p.f_pap, p.f_rz, p.f_rr, p.f_rzs, p.f_tol2, p.f_bb,
                  p.f_relres, p.f_xa, p.f_it_a, p.f_it_b, p.f_status, p.f_active, p.f_xs};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  c->used -= p.bytes + p.mixed_bytes;
  p = StripPool{};
}

template <class T>
hipError_t dalloc(T **p, size_t n) {
  return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

int alloc_mixed(mlmc_ctx *c, int level);

// make sure the pool of `level` holds at least n slots (n <= max fitting) and,
// if `mixed`, the buffers of the mixed-precision solver
int ensure_pool(mlmc_ctx *c, int level, int n, bool mixed = false) {
  StripLevel &L = c->lv[level];
  if (L.pool.cap >= n) return mixed && !L.pool.has_mixed ? alloc_mixed(c, level) : MLMC_OK;
  const bool had_mixed = L.pool.has_mixed;
  free_pool(c, L.pool);
  const StripGeom &g = L.g;
  const size_t need = strip_slot_bytes(g) * (size_t)n;
  if (c->used + need > c->budget)
    return fail(c, MLMC_ENOMEM, "level " + std::to_string(level) + ": " + std::to_string(n) +
                                     " slots exceed the memory budget");
  StripPool &p = L.pool;
  const size_t vec = (size_t)2 * g.nnode * n;
  HIPCHK(c, dalloc(&p.x, vec));
  HIPCHK(c, dalloc(&p.z, vec));
  HIPCHK(c, dalloc(&p.p, vec));
  HIPCHK(c, dalloc(&p.Ap, vec));
  HIPCHK(c, dalloc(&p.dg, vec));
  HIPCHK(c, dalloc(&p.theta, (size_t)8 * g.nelem * n));
  HIPCHK(c, dalloc(&p.part_pap, (size_t)g.sw_npart * n));
  HIPCHK(c, dalloc(&p.part_rz, (size_t)2 * g.nchunks * n));
  HIPCHK(c, dalloc(&p.part_rr, (size_t)2 * g.nchunks * n));
  HIPCHK(c, dalloc(&p.rzs, (size_t)2 * n));
  HIPCHK(c, dalloc(&p.tol2, (size_t)n));
  HIPCHK(c, dalloc(&p.bb, (size_t)n));
  HIPCHK(c, dalloc(&p.relres, (size_t)n));
  HIPCHK(c, dalloc(&p.xa, (size_t)2 * n));
  HIPCHK(c, dalloc(&p.qpart, (size_t)qoi_parts(g) * n));
  HIPCHK(c, dalloc(&p.it_a, (size_t)n));
  HIPCHK(c, dalloc(&p.it_b, (size_t)n));
  HIPCHK(c, dalloc(&p.status, (size_t)n));
  HIPCHK(c, dalloc(&p.active, (size_t)n));
  HIPCHK(c, dalloc(&p.outidx, (size_t)n));
  HIPCHK(c, dalloc(&p.xs, (size_t)2 * n));
  HIPCHK(c, hipMemset(p.xs, 0, sizeof(int) * 2 * n));
  HIPCHK(c, dalloc(&p.rows, (size_t)n));
  HIPCHK(c, hipMemset(p.active, 0, sizeof(int) * n));
  p.cap = n;
  p.bytes = need;
  c->used += need;
  if (c->h_active_cap < n) {
    if (c->h_active) (void)hipHostFree(c->h_active);
    HIPCHK(c, hipHostMalloc((void **)&c->h_active, sizeof(int) * n));
    c->h_active_cap = n;
  }
  if (mixed || had_mixed) return alloc_mixed(c, level);
  return MLMC_OK;
}

int alloc_mixed(mlmc_ctx *c, int level) {
  StripLevel &L = c->lv[level];
  StripPool &p = L.pool;
  const StripGeom &g = L.g;
  const int n = p.cap;
  const size_t need = strip_mixed_slot_bytes(g) * (size_t)n;
  if (c->used + need > c->budget)
    return fail(c, MLMC_ENOMEM, "level " + std::to_string(level) + ": mixed-precision buffers exceed the budget");
  const size_t n2 = (size_t)2 * g.nnode * n;
  HIPCHK(c, dalloc(&p.b64, n2));
  HIPCHK(c, dalloc(&p.m_part_rr, (size_t)g.sw_npart * n));
  HIPCHK(c, dalloc(&p.m_relres, (size_t)n));
  HIPCHK(c, dalloc(&p.f_rr_ref, (size_t)n));
  HIPCHK(c, dalloc(&p.m_updates, (size_t)n));
  HIPCHK(c, dalloc(&p.f_ru, (size_t)n));
  HIPCHK(c, hipMalloc(&p.theta16, (size_t)4 * g.nelem * n * (c->theta_fp32 ? 4 : 2)));
  HIPCHK(c, dalloc(&p.fx, n2));
  HIPCHK(c, dalloc(&p.fz, n2));
  HIPCHK(c, dalloc(&p.fp, n2));
  HIPCHK(c, dalloc(&p.fAp, n2));
  HIPCHK(c, dalloc(&p.fdg, n2));
  HIPCHK(c, dalloc(&p.f_pap, (size_t)g.sw_npart * n));
  HIPCHK(c, dalloc(&p.f_rz, (size_t)2 * g.nchunks * n));
  HIPCHK(c, dalloc(&p.f_rr, (size_t)2 * g.nchunks * n));
  HIPCHK(c, dalloc(&p.f_rzs, (size_t)2 * n));
  HIPCHK(c, dalloc(&p.f_tol2, (size_t)n));
  HIPCHK(c, dalloc(&p.f_bb, (size_t)n));
  HIPCHK(c, dalloc(&p.f_relres, (size_t)n));
  HIPCHK(c, dalloc(&p.f_xa, (size_t)2 * n));
  HIPCHK(c, dalloc(&p.f_xs, (size_t)2 * n));
  HIPCHK(c, hipMemset(p.f_xs, 0, sizeof(int) * 2 * n));
  HIPCHK(c, dalloc(&p.f_it_a, (size_t)n));
  HIPCHK(c, dalloc(&p.f_it_b, (size_t)n));
  HIPCHK(c, dalloc(&p.f_status, (size_t)n));
  HIPCHK(c, dalloc(&p.f_active, (size_t)n));
  HIPCHK(c, hipMemset(p.f_active, 0, sizeof(int) * n));
  HIPCHK(c, hipMemset(p.f_ru, 0, sizeof(int) * n));
  p.has_mixed = true;
  p.mixed_bytes = need;
  c->used += need;
  return MLMC_OK;
}

PcgState<float> inner_of(mlmc_ctx *c, int level) {
  StripPool &p = c->lv[level].pool;
  PcgState<float> I{};
  I.x = p.fx;
  I.z = p.fz;
  I.p = p.fp;
  I.Ap = p.fAp;
  I.dg = p.fdg;
  I.theta = p.theta16;
  I.part_pap = p.f_pap;
  I.part_rz = p.f_rz;
  I.part_rr = p.f_rr;
  I.rzs = p.f_rzs;
  I.tol2 = p.f_tol2;
  I.bb = p.f_bb;
  I.relres = p.f_relres;
  I.it_a = p.f_it_a;
  I.it_b = p.f_it_b;
  I.status = p.f_status;
  I.active = p.f_active;
  I.xa = p.f_xa;
  I.xs = p.f_xs;
  I.S = p.cap;
  I.max_iter = c->max_iter;
  I.mixed = 1;
  I.theta_fp32 = c->theta_fp32;
  I.cs = c->theta_fp32;  // selects the FP32-angle form of the operator pass
  I.ru2 = c->ru_factor * c->ru_factor;
  I.rr_ref = p.f_rr_ref;
  I.ru = p.f_ru;
  return I;
}

MixedState mixed_of(mlmc_ctx *c, int level, double rtol) {
  StripPool &p = c->lv[level].pool;
  MixedState M{};
  M.b = p.b64;
  M.part_rr = p.m_part_rr;
  M.part_bb = p.part_rr;  // parity-0 partials of ||b||^2 written by the FP64 set-up
  M.relres = p.m_relres;
  M.updates = p.m_updates;
  M.rtol2 = rtol * rtol;
  return M;
}

// FP64 solver state of the level's pool; the angle data is the pool's
// (cos 2theta, sin 2theta) buffer
PcgSlots slots_of(mlmc_ctx *c, int level, double rtol) {
  StripPool &p = c->lv[level].pool;
  PcgSlots S{};
  S.x = p.x;
  S.z = p.z;
  S.p = p.p;
  S.Ap = p.Ap;
  S.dg = p.dg;
  S.theta = p.theta;
  S.cs = c->lv[level].cs ? 1 : 0;
  S.part_pap = p.part_pap;
  S.part_rz = p.part_rz;
  S.part_rr = p.part_rr;
  S.rzs = p.rzs;
  S.tol2 = p.tol2;
  S.bb = p.bb;
  S.relres = p.relres;
  S.xa = p.xa;
  S.xs = p.xs;
  S.it_a = p.it_a;
  S.it_b = p.it_b;
  S.status = p.status;
  S.active = p.active;
  S.S = p.cap;
  S.max_iter = c->max_iter;
  S.rtol2 = rtol * rtol;
  return S;
}

// caller angles [n][4 nelem] into the pool's angle data (as codes tan theta, or as pairs)
int stage_angles(mlmc_ctx *c, int level, const double *theta, int n, hipStream_t st) {
  StripLevel &L = c->lv[level];
  const size_t ngp = (size_t)n * 4 * L.g.nelem;
  if (L.cs) launch_theta_cs(theta, L.pool.theta, ngp, st);
  else launch_theta_code(theta, L.pool.theta, ngp, st);
  HIPCHK(c, hipGetLastError());
  return MLMC_OK;
}

// largest batch of `level` that fits next to the other pools
int max_slots(mlmc_ctx *c, int level, bool mixed = false) {
  const StripPool &p = c->lv[level].pool;
  const size_t per = strip_slot_bytes(c->lv[level].g) +
                     ((mixed || p.has_mixed) ? strip_mixed_slot_bytes(c->lv[level].g) : 0);
  const size_t other = c->used - p.bytes - p.mixed_bytes;
  if (c->budget <= other) return 0;
  return (int)std::min<size_t>((c->budget - other) / per, 8192);
}

// one level's batch in a lock-step solve
template <typename T>
struct IterGroup {
  int level;
  PcgState<T> S;     // the solver state that iterates (FP32 inner state in mixed mode)
  int n;
};

template <typename T>
PcgGroup<T> *dev_groups(mlmc_ctx *c);
template <>
PcgGroup<double> *dev_groups<double>(mlmc_ctx *c) { return c->d_grp64; }
template <>
PcgGroup<float> *dev_groups<float>(mlmc_ctx *c) { return c->d_grp32; }
template <typename T>
PcgGroup<T> *host_groups(mlmc_ctx *c);
template <>
PcgGroup<double> *host_groups<double>(mlmc_ctx *c) { return c->h_grp64; }
template <>
PcgGroup<float> *host_groups<float>(mlmc_ctx *c) { return c->h_grp32; }

int ensure_host_active(mlmc_ctx *c, int n) {
  if (c->h_active_cap >= n) return MLMC_OK;
  if (c->h_active) (void)hipHostFree(c->h_active);
  c->h_active = nullptr;
  c->h_active_cap = 0;
  HIPCHK(c, hipHostMalloc((void **)&c->h_active, sizeof(int) * n));
  c->h_active_cap = n;
  return MLMC_OK;
}

// Lock-step PCG iterations of up to MAX_GROUPS level batches in shared
// launches (one operator pass and one vector pass per iteration for all of
// them) until every slot is inactive.  The host checks the slot flags every
// `block` iterations and drops finished groups from the launch.  extra(k,
// alive, itb, stream) launches what runs after iteration k.  prof_k: profile
// counters (2 per precision).  Unless profiling, a block of iterations is
// captured once as a graph (keyed by its launch configuration and `sig`, the
// bytes of any arguments `extra` bakes in) and replayed.
template <typename T, class Extra>
int pcg_iterate(mlmc_ctx *c, const std::vector<IterGroup<T>> &grp, hipStream_t st, int prof_k, Extra extra,
                const std::vector<char> &sig = {}) {
  const int ng_all = (int)grp.size();
  if (ng_all == 0) return MLMC_OK;
  if (ng_all > MAX_GROUPS) return fail(c, MLMC_EINVAL, "too many level groups in one lock-step solve");
  const int block = 32;
  // profiling times one iteration per block, in the middle (the queue is
  // full there): iteration 16 of even blocks and 17 of odd ones, so both
  // variants of the vector pass (x moves at odd iterations) are sampled; it
  // counts the algorithmic bytes of exactly those launches
  auto timed_b = [&](long base) { return block / 2 + (int)((base / block) & 1); };
  std::vector<long> timed_its;
  if (c->prof && c->ev.size() < 3) {
    c->ev.resize(3);
    for (auto &e : c->ev) HIPCHK(c, hipEventCreate(&e));
  }
  int tot = 0;
  for (const auto &gr : grp) tot += gr.n;
  if (int rc = ensure_host_active(c, tot)) return rc;
  std::vector<char> alive(ng_all, 1);
  PcgGroup<T> *hg = host_groups<T>(c), *dg = dev_groups<T>(c);
  int ng = 0, nb2 = 0;
  int ngm[2] = {0, 0}, nb1m[2] = {0, 0};   // operator-pass groups and blocks per angle mode
  int nt = 0;                             // streaming accesses in both passes
  // compact the live groups into the descriptor array, groups with stored
  // angles first, then those with stored (cos, sin) pairs (each mode has its
  // own operator-pass kernel; the vector pass takes all groups).  The staging
  // buffer is only rewritten after the stream has been synchronised.
  auto upload = [&]() -> int {
    ng = nb2 = 0;
    for (int mode = 0; mode < 2; ++mode) {
      ngm[mode] = nb1m[mode] = 0;
      // tile height of this operator-pass launch: 8 element rows, or 4 when 8
      // leaves the device with fewer waves than it holds at once (small
      // batches, single requests).  Measured on the 4-level benchmark, 8
      // beats 16 and 4 at every lock-step level (16-row tiles leave a large,
      // partly filled last round of waves).  The sums do not depend on it.
      const long resident = pass1_resident_waves<T>(mode);
      int ty = 2 * SWEEP_RB;
      {
        long waves = 0;
        for (int k = 0; k < ng_all; ++k) {
          if (!alive[k] || (grp[k].S.cs != 0) != (mode == 1)) continue;
          StripGeom gg = c->lv[grp[k].level].g;
          set_sweep_rows(gg, ty);
          waves += (long)gg.sw_ntiles * grp[k].n;
        }
        if (waves < resident) ty = SWEEP_RB;
      }
      if (c->sweep_rows) ty = c->sweep_rows;
      for (int k = 0; k < ng_all; ++k) {
        if (!alive[k] || (grp[k].S.cs != 0) != (mode == 1)) continue;
        PcgGroup<T> &D = hg[ng++];
        D.g = c->lv[grp[k].level].g;
        // a height tuned for the mesh wins over the per-launch choice (the
        // sums, hence the results, do not depend on it)
        const int tyk = c->lv[grp[k].level].sweep_rows;
        set_sweep_rows(D.g, tyk ? tyk : ty);
        D.S = grp[k].S;
        D.n = grp[k].n;
        D.blk0 = nb1m[mode];
        D.cblk0 = nb2;
        nb1m[mode] += D.g.sw_ntiles * D.n;
        nb2 += D.g.nchunks * D.n;
        ngm[mode]++;
      }
    }
    // bytes one iteration touches: x, z, p, Ap, dg and the angles (FP64:
    // codes 32 B or pairs 64 B per element; FP32: bfloat16 8 B or FP32 16 B)
    double ws = 0;
    for (int k = 0; k < ng; ++k) {
      const double ab = sizeof(T) == 8 ? (hg[k].S.cs ? 64.0 : 32.0) : (hg[k].S.cs ? 16.0 : 8.0);
      ws += (double)hg[k].n * (10.0 * sizeof(T) * hg[k].g.nnode + ab * hg[k].g.nelem);
    }
    nt = ws > c->streaming_min_bytes;
    HIPCHK(c, hipMemcpyAsync(dg, hg, sizeof(PcgGroup<T>) * ng, hipMemcpyHostToDevice, st));
    return MLMC_OK;
  };
  if (int rc = upload()) return rc;
  // one block of iterations: kernel launches for iterations base + 0..block-1
  // (itb null: `base` is passed directly; otherwise it is read from *itb)
  auto launch_block = [&](int base, const int *itb, hipStream_t s, bool timed) -> int {
    for (int b = 0; b < block; ++b) {
      const int k = base + b;
      const bool ev = timed && b == timed_b(base);
      if (ev) HIPCHK(c, hipEventRecord(c->ev[0], s));
      if (ngm[0]) launch_pcg_pass1<T>(dg, ngm[0], nb1m[0], c->mat, k, 0, itb, s, nt);
      if (ngm[1]) launch_pcg_pass1<T>(dg + ngm[0], ngm[1], nb1m[1], c->mat, k, 1, itb, s, nt);
      if (ev) HIPCHK(c, hipEventRecord(c->ev[1], s));
      launch_pcg_pass2<T>(dg, ng, nb2, k, itb, s, nt);
      if (ev) HIPCHK(c, hipEventRecord(c->ev[2], s));
      extra(k, alive, itb, s);
    }
    return MLMC_OK;
  };
  // graph replay (not while profiling: the passes are then timed one by one)
  const bool use_graph = c->graphs && !c->prof;
  hipGraphExec_t exec = nullptr;
  auto prepare_graph = [&]() -> int {
    std::vector<char> key(sig.begin(), sig.end());
    auto put = [&](const void *p, size_t n) { key.insert(key.end(), (const char *)p, (const char *)p + n); };
    const int tsz = (int)sizeof(T);
    put(&tsz, sizeof tsz);
    put(ngm, sizeof ngm);
    put(nb1m, sizeof nb1m);
    put(&nb2, sizeof nb2);
    put(&nt, sizeof nt);
    for (char a : alive) key.push_back(a);
    for (auto &e : c->gcache)
      if (e.key == key) {
        exec = e.exec;
        return MLMC_OK;
      }
    mlmc_ctx::CachedGraph e;
    e.key = key;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch_block(0, c->d_itb, c->cap_stream, false);
    launch_add_int(c->d_itb, block, c->cap_stream);
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &e.graph);
    if (rc) return rc;
    HIPCHK(c, ec);
    HIPCHK(c, hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
    if (c->gcache.size() >= 16) {
      (void)hipGraphExecDestroy(c->gcache.front().exec);
      (void)hipGraphDestroy(c->gcache.front().graph);
      c->gcache.erase(c->gcache.begin());
    }
    c->gcache.push_back(e);
    exec = e.exec;
    return MLMC_OK;
  };
  if (use_graph) {
    launch_set_int(c->d_itb, 0, st);
    if (int rc = prepare_graph()) return rc;
  }
  for (long it = 0;; it += block) {
    if (use_graph) {
      HIPCHK(c, hipGraphLaunch(exec, st));
    } else {
      if (int rc = launch_block((int)it, nullptr, st, c->prof)) return rc;
    }
    HIPCHK(c, hipGetLastError());
    int off = 0;
    for (int g = 0; g < ng_all; ++g) {
      if (alive[g])
        HIPCHK(c, hipMemcpyAsync(c->h_active + off, grp[g].S.active, sizeof(int) * grp[g].n, hipMemcpyDeviceToHost,
                                 st));
      off += grp[g].n;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->prof) {
      float t1 = 0, t2 = 0;
      HIPCHK(c, hipEventElapsedTime(&t1, c->ev[0], c->ev[1]));
      HIPCHK(c, hipEventElapsedTime(&t2, c->ev[1], c->ev[2]));
      c->prof_ms[prof_k] += t1;
      c->prof_ms[prof_k + 1] += t2;
      c->prof_launches[prof_k] += 1;
      c->prof_launches[prof_k + 1] += 1;
      timed_its.push_back(it + timed_b(it));
    }
    bool changed = false, any = false;
    off = 0;
    for (int g = 0; g < ng_all; ++g) {
      if (alive[g]) {
        bool a = false;
        for (int k = 0; k < grp[g].n; ++k) a |= c->h_active[off + k] != 0;
        if (!a) {
          alive[g] = 0;
          changed = true;
        }
        any |= a;
      }
      off += grp[g].n;
    }
    if (!any) break;
    if (it > (long)c->max_iter + 4 * block) return fail(c, MLMC_EHIP, "PCG loop did not terminate");
    if (changed) {
      if (int rc = upload()) return rc;
      if (use_graph)
        if (int rc = prepare_graph()) return rc;
    }
  }
  if (c->prof) {
    for (const auto &gr : grp) {
      const StripGeom &g = c->lv[gr.level].g;
      c->h_iters.resize(gr.n);
      HIPCHK(c, hipMemcpyAsync(c->h_iters.data(), gr.S.it_b, sizeof(int) * gr.n, hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipStreamSynchronize(st));
      // a slot with final iteration count K is active in iterations 0..K-1
      const double w = sizeof(T);
      const double wt = (sizeof(T) == 8) ? (gr.S.cs ? 64.0 : 32.0) : (c->theta_fp32 ? 16.0 : 8.0);  // angle bytes/element
      for (long ti : timed_its) {
        double act = 0;
        for (int k = 0; k < gr.n; ++k) act += c->h_iters[k] > ti ? 1.0 : 0.0;
        c->prof_bytes[prof_k] += act * (3.0 * 2 * w * g.nnode + wt * g.nelem);  // z, p_old in; A p out
        // x, z, p_old, A p, dg in; x, z, p out, x every second pass (odd
        // iterations; in mixed mode a reliable update can shift the parity)
        const double vec = (ti & 1) ? 8.0 : 6.0;
        c->prof_bytes[prof_k + 1] += act * vec * 2 * w * g.nnode;
        c->prof_dofs[prof_k] += act * 2.0 * g.nnode;
        c->prof_dofs[prof_k + 1] += act * 2.0 * g.nnode;
      }
    }
  }
  return MLMC_OK;
}

// a level batch whose angles are ready in S.theta
struct SolveGroup {
  int level;
  PcgSlots S;
  int n;
};

// FP64: set-up + lock-step PCG to completion for the groups
// (after_setup, when given, runs once the set-up kernels are queued and before
// the iterations)
int run_pcg(mlmc_ctx *c, const std::vector<SolveGroup> &sg, hipStream_t st,
            const std::function<int()> &after_setup = {}) {
  std::vector<IterGroup<double>> ig;
  for (const auto &x : sg) {
    launch_setup(c->lv[x.level].g, c->mat, x.S, x.n, nullptr, nullptr, st);
    ig.push_back({x.level, x.S, x.n});
  }
  HIPCHK(c, hipGetLastError());
  if (after_setup)
    if (int rc = after_setup()) return rc;
  if (int rc = pcg_iterate<double>(c, ig, st, 0, [](int, const std::vector<char> &, const int *, hipStream_t) {}))
    return rc;
  for (const auto &x : sg) launch_x_flush(c->lv[x.level].g, x.S, x.n, st);
  HIPCHK(c, hipGetLastError());
  return MLMC_OK;
}

// coarse level: set-up + PCG to completion by one work-group per sample, FP64
int run_small(mlmc_ctx *c, int level, const PcgSlots &S, int n, hipStream_t st) {
  launch_setup(c->lv[level].g, c->mat, S, n, nullptr, nullptr, st);
  launch_small_solve(c->lv[level].g, c->mat, S, n, st);
  HIPCHK(c, hipGetLastError());
  return MLMC_OK;
}

// mixed precision: FP32 PCG (FP32 or BF16 angles) with reliable updates in FP64 (the
// residual b - A x recomputed with the FP64 angles whenever the FP32 residual
// fell by the update factor, and as the only stopping test); x accumulates in
// FP64.  On return the FP64 pool state of every group holds x.
int run_mixed(mlmc_ctx *c, const std::vector<SolveGroup> &sg, hipStream_t st,
              const std::function<int()> &after_setup = {}) {
  std::vector<IterGroup<float>> ig;
  std::vector<MixedState> ms;
  for (const auto &x : sg) {
    const StripGeom &g = c->lv[x.level].g;
    PcgState<float> I = inner_of(c, x.level);
    MixedState M = mixed_of(c, x.level, std::sqrt(x.S.rtol2));
    I.rtol2 = x.S.rtol2;
    launch_setup(g, c->mat, x.S, x.n, M.b, nullptr, st);
    launch_mixed_start(g, x.S, I, M, x.n, st);
    ig.push_back({x.level, I, x.n});
    ms.push_back(M);
  }
  HIPCHK(c, hipGetLastError());
  if (after_setup)
    if (int rc = after_setup()) return rc;
  const int every = c->ru_every;
  // the graph key covers the per-group arguments the reliable-update launches bake in
  std::vector<char> sig;
  auto put = [&](const void *p, size_t n) { sig.insert(sig.end(), (const char *)p, (const char *)p + n); };
  put(&every, sizeof every);
  for (size_t q = 0; q < sg.size(); ++q) {
    put(&sg[q].S, sizeof(PcgSlots));
    put(&ig[q].S, sizeof(PcgState<float>));
    put(&ms[q], sizeof(MixedState));
    put(&sg[q].n, sizeof(int));
  }
  int rc = pcg_iterate<float>(
      c, ig, st, 2,
      [&](int k, const std::vector<char> &alive, const int *itb, hipStream_t s) {
        if ((k + 1) % every != 0) return;
        for (size_t q = 0; q < sg.size(); ++q) {
          if (!alive[q]) continue;
          const StripGeom &g = c->lv[sg[q].level].g;
          launch_resid64(g, c->mat, sg[q].S, ig[q].S, ms[q], sg[q].n, k, every, itb, s);
          launch_ru_apply(g, sg[q].S, ig[q].S, ms[q], sg[q].n, k, every, itb, s);
        }
      },
      sig);
  if (rc) return rc;
  for (size_t q = 0; q < sg.size(); ++q) launch_mixed_flush(c->lv[sg[q].level].g, sg[q].S, ig[q].S, sg[q].n, st);
  HIPCHK(c, hipGetLastError());
  return MLMC_OK;
}

// slot reports of the last solve in the given precision (for the QoI kernel)
PcgSlots report_view(mlmc_ctx *c, int level, const PcgSlots &D, int precision) {
  if (precision != MLMC_MIXED) return D;
  StripPool &p = c->lv[level].pool;
  PcgSlots V = D;
  V.it_b = p.f_it_b;
  V.relres = p.m_relres;
  V.status = p.f_status;
  return V;
}

int build_strip(mlmc_ctx *c) {
  const Json &cfg = c->cfg;
  c->nlev = (int)cfg.number("n_levels");
  if (c->nlev < 1 || c->nlev > 12) throw std::runtime_error("n_levels out of range");
  c->mat = make_material(cfg);
  c->rtol = cfg.number_or("rtol", 1e-10);
  c->max_iter = (int)cfg.number_or("max_iter", 100000);
  if (cfg.has("mixed")) {
    const Json &mx = cfg.at("mixed");
    c->ru_factor = mx.number_or("update_factor", c->ru_factor);
    c->ru_every = (int)mx.number_or("update_every", c->ru_every);
    const std::string ts = mx.string_or("theta_storage", "fp32");
    if (ts != "bf16" && ts != "fp32") throw std::runtime_error("mixed.theta_storage must be bf16 or fp32");
    c->theta_fp32 = ts == "fp32";
  }
  if (c->ru_every < 1 || 32 % c->ru_every != 0)
    throw std::runtime_error("mixed.update_every must divide 32 (1, 2, 4, 8, 16 or 32)");
  if (!(c->ru_factor > 0.0 && c->ru_factor < 1.0)) throw std::runtime_error("mixed.update_factor must be in (0, 1)");
  const Json &kl = cfg.at("kl");
  c->K = (int)kl.number("n_modes");
  if (c->K < 1 || c->K > 32) throw std::runtime_error("n_modes must be in 1..32");
  const double s = kl.number("sigma_deg") * M_PI / 180.0, var = s * s;
  const std::string type = kl.string_or("type", "");
  c->lv.resize(c->nlev);
  for (int l = 0; l < c->nlev; ++l) c->lv[l].g = make_geom(cfg, l);
  // coarse levels whose PCG state fits one work-group's LDS are solved whole
  // by one work-group per sample ("small_solver": "auto" or "off"); the
  // choice depends on the level only, never on the batch
  if (cfg.has("graphs")) {
    if (cfg.at("graphs").type != Json::Bool) throw std::runtime_error("graphs must be true or false");
    c->graphs = cfg.at("graphs").b;
  }
  c->sweep_rows = (int)cfg.number_or("sweep_rows", 0);
  if (c->sweep_rows < 0 || c->sweep_rows > SWEEP_MAXTY || c->sweep_rows % SWEEP_RB != 0)
    throw std::runtime_error("sweep_rows must be 0 (automatic), 4, 8, 12 or 16");
  {
    const double mb = cfg.number_or("streaming_min_mb", 256.0);
    if (!(mb >= 0.0)) throw std::runtime_error("streaming_min_mb must be a number >= 0");
    c->streaming_min_bytes = mb * 1048576.0;
  }
  const std::string sm = cfg.string_or("small_solver", "auto");
  if (sm != "auto" && sm != "off") throw std::runtime_error("small_solver must be auto or off");
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
    throw std::runtime_error("hipDeviceGetAttribute failed");
  const int small_max_nodes = (int)cfg.number_or("small_max_nodes", 1 << 30);
  // FP64 angle data: stored angles (the solver evaluates cos/sin 2theta every
  // iteration) or stored (cos 2theta, sin 2theta) pairs (twice the bytes, no
  // trigonometry in the loop); both give bit-identical results.  Default: pairs
  // for the coarse levels solved whole per work-group (arithmetic-bound),
  // angles for the lock-step levels (bandwidth-bound).  "level_options" keyed
  // by mesh ("NXxNY") overrides engine and angle storage per level.
  const std::string as = cfg.string_or("angle_storage", "auto");
  if (as != "auto" && as != "cs" && as != "theta") throw std::runtime_error("angle_storage must be auto, cs or theta");
  for (int l = 0; l < c->nlev; ++l) {
    StripLevel &L = c->lv[l];
    const bool fits = L.g.nnode <= small_max_nodes && small_fits(L.g, (size_t)lds);
    L.small = sm == "auto" && fits;
    L.cs = as == "cs" || (as == "auto" && L.small);
    const std::string key = std::to_string(L.g.nx) + "x" + std::to_string(L.g.ny);
    if (cfg.has("level_options") && cfg.at("level_options").has(key)) {
      const Json &o = cfg.at("level_options").at(key);
      const std::string eng = o.string_or("engine", "");
      if (eng == "small") L.small = fits;
      else if (eng == "lockstep") L.small = false;
      else if (!eng.empty()) throw std::runtime_error("level_options engine must be small or lockstep");
      const std::string an = o.string_or("angles", "");
      if (an == "cs") L.cs = true;
      else if (an == "theta") L.cs = false;
      else if (!an.empty()) throw std::runtime_error("level_options angles must be cs or theta");
      const int sr = (int)o.number_or("sweep_rows", 0);
      if (sr < 0 || sr > SWEEP_MAXTY || sr % SWEEP_RB != 0)
        throw std::runtime_error("level_options sweep_rows must be 0 (per launch), 4, 8, 12 or 16");
      L.sweep_rows = sr;
    }
    if (sm == "off") L.small = false;   // an explicit "off" wins over per-level options
  }
  const int K = c->K;
  if (type == "exp_separable") {
    SeparableKL sk = separable_kl(cfg.number("Lx"), cfg.number("Ly"), var, kl.number("corr_x"),
                                  kl.number("corr_y"), K);
    for (int l = 0; l < c->nlev; ++l) {
      StripGeom &g = c->lv[l].g;
      const size_t ngp = (size_t)4 * g.nelem;
      std::vector<double> tab(ngp * K);
      for (size_t gp = 0; gp < ngp; ++gp) {
        const size_t e = gp / 4;
        const int q = (int)(gp % 4);
        const double x = g.hx * ((double)(e % g.nx) + ((q & 1) ? GP_P : GP_M));
        const double y = g.hy * ((double)(e / g.nx) + ((q & 2) ? GP_P : GP_M));
        for (int k = 0; k < K; ++k)
          tab[gp * K + k] = std::sqrt(sk.mu[k]) * sk.x.mode(sk.ix[k], x - sk.x.a) * sk.y.mode(sk.iy[k], y - sk.y.a);
      }
      HIPCHK(c, dalloc(&c->lv[l].modes, tab.size()));
      HIPCHK(c, hipMemcpy(c->lv[l].modes, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
      c->used += tab.size() * sizeof(double);
    }
  } else if (type == "matern32") {
    std::vector<double> nq = kl.numbers("nystrom");
    if (nq.size() != 2) throw std::runtime_error("nystrom needs [nqx, nqy]");
    const double len = kl.number("length");
    MaternKL mk = matern_kl(cfg.number("Lx"), cfg.number("Ly"), var, len, (int)nq[0], (int)nq[1], K);
    if (!(mk.max_residual < 1e-10)) throw std::runtime_error("Nystrom eigen-solve did not converge");
    std::vector<double> coef((size_t)mk.n * K);
    for (int j = 0; j < mk.n; ++j)
      for (int k = 0; k < K; ++k) coef[(size_t)j * K + k] = mk.wq[j] * mk.phi[(size_t)j * K + k] / std::sqrt(mk.mu[k]);
    double *dgx, *dgy, *dcoef;
    HIPCHK(c, dalloc(&dgx, mk.n));
    HIPCHK(c, dalloc(&dgy, mk.n));
    HIPCHK(c, dalloc(&dcoef, coef.size()));
    HIPCHK(c, hipMemcpy(dgx, mk.px.data(), mk.n * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(dgy, mk.py.data(), mk.n * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(dcoef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
    for (int l = 0; l < c->nlev; ++l) {
      StripGeom &g = c->lv[l].g;
      const size_t ngp = (size_t)4 * g.nelem;
      HIPCHK(c, dalloc(&c->lv[l].modes, ngp * K));
      c->used += ngp * K * sizeof(double);
      launch_modes_nystrom(dgx, dgy, dcoef, mk.n, K, var, std::sqrt(3.0) / len, g, c->lv[l].modes, nullptr);
      HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipDeviceSynchronize());
    (void)hipFree(dgx);
    (void)hipFree(dgy);
    (void)hipFree(dcoef);
  } else {
    throw std::runtime_error("unknown kl.type '" + type + "'");
  }
  return MLMC_OK;
}

bool bad_level(const mlmc_ctx *c, int level) { return level < 0 || level >= c->nlev; }

}  // namespace

// ---------------------------------------------------------------- fixed scratch
// Workspace of mlmc_strip_solve_theta_noalloc: one fixed array per GPU, part of
// the code object, so that entry point allocates nothing.  In host code the
// name `scratch` only stands for the symbol; the array's device address comes
// from hipGetSymbolAddress, once per device, at context creation.
static __device__ __align__(256) unsigned char scratch[MLMC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_addr;  // by device id

// look up (once per device) the current device's scratch address into c->scratch
int scratch_address(mlmc_ctx *c) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= c->device) g_scratch_addr.resize(c->device + 1, nullptr);
  if (!g_scratch_addr[c->device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, MLMC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[c->device] = p;
  }
  c->scratch = g_scratch_addr[c->device];
  return MLMC_OK;
}

// Lay the FP64 solver state of n slots of a strip level out from `base` in
// 256-byte aligned pieces (the same buffers a pool slot holds, angles as codes
// or pairs as the level stores them).  Returns the bytes used; with base ==
// nullptr it only sizes the layout.
size_t carve_slots(const mlmc_ctx *c, int level, int n, double rtol, unsigned char *base, PcgSlots *S,
                   double **qpart) {
  const StripLevel &L = c->lv[level];
  const StripGeom &g = L.g;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    void *p = base ? (void *)(base + off) : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const size_t vec = sizeof(double) * 2 * (size_t)g.nnode * n;
  *S = PcgSlots{};
  S->x = (double *)take(vec);
  S->z = (double *)take(vec);
  S->p = (double *)take(vec);
  S->Ap = (double *)take(vec);
  S->dg = (double *)take(vec);
  S->theta = take(sizeof(double) * (L.cs ? 8 : 4) * (size_t)g.nelem * n);
  S->cs = L.cs ? 1 : 0;
  S->part_pap = (double *)take(sizeof(double) * g.sw_npart * (size_t)n);
  S->part_rz = (double *)take(sizeof(double) * 2 * g.nchunks * (size_t)n);
  S->part_rr = (double *)take(sizeof(double) * 2 * g.nchunks * (size_t)n);
  S->rzs = (double *)take(sizeof(double) * 2 * (size_t)n);
  S->tol2 = (double *)take(sizeof(double) * n);
  S->bb = (double *)take(sizeof(double) * n);
  S->relres = (double *)take(sizeof(double) * n);
  S->xa = (double *)take(sizeof(double) * 2 * (size_t)n);
  S->xs = (int *)take(sizeof(int) * 2 * (size_t)n);
  S->it_a = (int *)take(sizeof(int) * n);
  S->it_b = (int *)take(sizeof(int) * n);
  S->status = (int *)take(sizeof(int) * n);
  S->active = (int *)take(sizeof(int) * n);
  *qpart = (double *)take(sizeof(double) * qoi_parts(g) * (size_t)n);
  S->S = n;
  S->max_iter = c->max_iter;
  S->rtol2 = rtol * rtol;
  return off;
}

// slots the pinned flag buffer holds from creation on (the no-alloc entry
// point never grows it)
constexpr int NOALLOC_MAX_SLOTS = 4096;

}  // namespace

// ====================================================================== C ABI
extern "C" {

int mlmc_create(const char *config_json, size_t mem_budget_bytes, mlmc_ctx **out) {
  if (!out) { g_create_error = "out is NULL"; return MLMC_EINVAL; }
  *out = nullptr;
  if (!config_json) { g_create_error = "config_json is NULL"; return MLMC_EINVAL; }
  mlmc_ctx *c = new mlmc_ctx();
  int rc = MLMC_OK;
  try {
    c->cfg = parse_json(config_json);
    const std::string kind = c->cfg.string_or("kind", "");
    if (hipGetDevice(&c->device) != hipSuccess) throw std::runtime_error("no HIP device");
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) throw std::runtime_error("hipMemGetInfo failed");
    c->budget = mem_budget_bytes ? mem_budget_bytes : (size_t)(0.9 * (double)fr);
    if (hipMalloc((void **)&c->d_stats, 16 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_stats, 16 * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&c->d_grp64, MAX_GROUPS * sizeof(PcgGroup<double>)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_grp64, MAX_GROUPS * sizeof(PcgGroup<double>)) != hipSuccess ||
        hipMalloc((void **)&c->d_grp32, MAX_GROUPS * sizeof(PcgGroup<float>)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_grp32, MAX_GROUPS * sizeof(PcgGroup<float>)) != hipSuccess ||
        hipMalloc((void **)&c->d_itb, sizeof(int)) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
      throw std::runtime_error("allocation of the stats buffers failed");
    // a failed look-up only disables the allocation-free entry point
    if (scratch_address(c) != MLMC_OK) c->scratch_err = c->err;
    if (hipHostMalloc((void **)&c->h_active, sizeof(int) * NOALLOC_MAX_SLOTS) != hipSuccess)
      throw std::runtime_error("allocation of the slot flag buffer failed");
    c->h_active_cap = NOALLOC_MAX_SLOTS;
    if (kind == "strip") {
      c->kind = 0;
      rc = build_strip(c);
    } else if (kind == "cosserat") {
      c->kind = 2;
      c->cos = cos_create(c->cfg, c->budget, c->err);
      if (!c->cos) rc = MLMC_EINVAL;
      else {
        c->nlev = cos_num_levels(c->cos);
        c->K = cos_num_params(c->cos) - 3;
      }
    } else if (kind == "plate") {
      c->kind = 1;
      c->plate = plate_create(c->cfg, c->err);
      if (!c->plate) {
        rc = MLMC_EINVAL;
      } else {
        c->nlev = plate_num_levels(c->plate);
        plate_set_budget(c->plate, c->budget);
      }
    } else {
      throw std::runtime_error("config 'kind' must be \"strip\", \"plate\" or \"cosserat\"");
    }
  } catch (const std::exception &e) {
    c->err = e.what();
    rc = MLMC_EINVAL;
  }
  if (rc != MLMC_OK) {
    g_create_error = c->err;
    mlmc_destroy(c);
    return rc;
  }
  *out = c;
  return MLMC_OK;
}

void mlmc_destroy(mlmc_ctx *c) {
  if (!c) return;
  for (auto &L : c->lv) {
    free_pool(c, L.pool);
    if (L.modes) (void)hipFree(L.modes);
  }
  if (c->h_active) (void)hipHostFree(c->h_active);
  if (c->d_stats) (void)hipFree(c->d_stats);
  if (c->h_stats) (void)hipHostFree(c->h_stats);
  if (c->d_grp64) (void)hipFree(c->d_grp64);
  if (c->h_grp64) (void)hipHostFree(c->h_grp64);
  if (c->d_grp32) (void)hipFree(c->d_grp32);
  if (c->h_grp32) (void)hipHostFree(c->h_grp32);
  for (auto &e : c->gcache) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
  }
  if (c->d_itb) (void)hipFree(c->d_itb);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->plate) plate_destroy(c->plate);
  if (c->cos) cos_destroy(c->cos);
  for (auto &e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

const char *mlmc_last_error(const mlmc_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int mlmc_num_levels(const mlmc_ctx *c) { return c ? c->nlev : MLMC_EINVAL; }

int mlmc_level_info(const mlmc_ctx *c, int level, int64_t *n_nodes, int64_t *n_dofs, int64_t *n_elem,
                    int64_t *n_gp) {
  if (!c) return MLMC_EINVAL;
  if (bad_level(c, level)) return fail(const_cast<mlmc_ctx *>(c), MLMC_EINVAL, "level out of range");
  int64_t nn, nd, ne, ng;
  if (c->kind == 0) {
    const StripGeom &g = c->lv[level].g;
    nn = g.nnode;
    nd = 2 * (int64_t)g.nnode;
    ne = g.nelem;
    ng = 4 * (int64_t)g.nelem;
  } else if (c->kind == 2) {
    cos_level_sizes(c->cos, level, &nn, &nd, &ne);
    ng = 4 * ne;
  } else {
    plate_level_sizes(c->plate, level, &nn, &nd, &ne);
    ng = 4 * ne;
  }
  if (n_nodes) *n_nodes = nn;
  if (n_dofs) *n_dofs = nd;
  if (n_elem) *n_elem = ne;
  if (n_gp) *n_gp = ng;
  return MLMC_OK;
}

int mlmc_footprint(const mlmc_ctx *c, int kind, int level, int precision, size_t *bytes) {
  if (!c || !bytes) return MLMC_EINVAL;
  mlmc_ctx *m = const_cast<mlmc_ctx *>(c);
  if (kind != c->kind) return fail(m, MLMC_ESTATE, "kind does not match the context's model");
  if (bad_level(c, level)) return fail(m, MLMC_EINVAL, "level out of range");
  if (precision != MLMC_FP64 && precision != MLMC_MIXED) return fail(m, MLMC_EINVAL, "bad precision");
  *bytes = (kind == 0) ? strip_slot_bytes(c->lv[level].g) +
                             (precision == MLMC_MIXED && !c->lv[level].small ? strip_mixed_slot_bytes(c->lv[level].g)
                                                                            : 0)
                       : (kind == 2) ? cos_slot_bytes(c->cos, level)
                                     : plate_slot_bytes(c->plate, level, precision);
  return MLMC_OK;
}

int mlmc_reserve(mlmc_ctx *c, int level, int n, int precision) {
  if (!c) return MLMC_EINVAL;
  if (bad_level(c, level) || n < 0) return fail(c, MLMC_EINVAL, "level out of range or n < 0");
  if (precision != MLMC_FP64 && precision != MLMC_MIXED) return fail(c, MLMC_EINVAL, "bad precision");
  if (n == 0) return MLMC_OK;
  if (c->kind == 1) return plate_reserve(c->plate, c->err, level, n);
  if (c->kind == 2) return cos_reserve(c->cos, c->err, level, n);
  const bool mixed = precision == MLMC_MIXED && !c->lv[level].small;
  if (n > max_slots(c, level, mixed))
    return fail(c, MLMC_ENOMEM, "level " + std::to_string(level) + ": " + std::to_string(n) +
                                    " slots exceed the memory budget");
  return ensure_pool(c, level, n, mixed);
}

int mlmc_sample_field(mlmc_ctx *c, int level, int n, const double *xi, int ld_xi, void *theta, int dtype,
                      void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind == 1) return fail(c, MLMC_ESTATE, "sample_field needs a strip or Cosserat context");
  if (bad_level(c, level)) return fail(c, MLMC_EINVAL, "level out of range");
  if (n < 0 || ld_xi < c->K + 3) return fail(c, MLMC_EINVAL, "n < 0 or ld_xi < n_modes + 3");
  if (dtype != 0 && dtype != 1) return fail(c, MLMC_EINVAL, "dtype must be 0 (FP64) or 1 (BF16)");
  if (c->kind == 2 && dtype != 0) return fail(c, MLMC_EINVAL, "the Cosserat model writes FP64 angles only");
  if (n == 0) return MLMC_OK;
  if (!xi || !theta) return fail(c, MLMC_EINVAL, "null pointer");
  if (c->kind == 2) return cos_sample_field(c->cos, c->err, level, n, xi, ld_xi, (double *)theta, (hipStream_t)stream);
  const StripGeom &g = c->lv[level].g;
  launch_kl_synth(c->lv[level].modes, c->K, g, xi, ld_xi, nullptr, n, dtype == 0 ? (double *)theta : nullptr,
                  dtype == 1 ? theta : nullptr, 0, 4 * g.nelem, nullptr, 0, (hipStream_t)stream);
  HIPCHK(c, hipGetLastError());
  return MLMC_OK;
}

int mlmc_strip_apply(mlmc_ctx *c, int level, int n, const double *theta, const double *x, double *y, int raw,
                     void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind == 1) return fail(c, MLMC_ESTATE, "strip_apply needs a strip or Cosserat context");
  if (bad_level(c, level) || n < 0) return fail(c, MLMC_EINVAL, "level out of range or n < 0");
  if (n == 0) return MLMC_OK;
  if (!theta || !x || !y) return fail(c, MLMC_EINVAL, "null pointer");
  if (n > 65535) return fail(c, MLMC_EINVAL, "n > 65535");
  if (c->kind == 2) return cos_apply(c->cos, c->err, level, n, theta, x, y, raw, (hipStream_t)stream);
  launch_apply(c->lv[level].g, c->mat, theta, x, y, raw, n, (hipStream_t)stream);
  HIPCHK(c, hipGetLastError());
  return MLMC_OK;
}

int mlmc_strip_rhs_diag(mlmc_ctx *c, int level, int n, const double *theta, double *b, double *dinv,
                        void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind == 1) return fail(c, MLMC_ESTATE, "needs a strip or Cosserat context");
  if (bad_level(c, level) || n < 0) return fail(c, MLMC_EINVAL, "level out of range or n < 0");
  if (n == 0) return MLMC_OK;
  if (!theta || !b || !dinv) return fail(c, MLMC_EINVAL, "null pointer");
  if (c->kind == 2) return cos_rhs_diag(c->cos, c->err, level, n, theta, b, dinv, (hipStream_t)stream);
  if (n > max_slots(c, level)) return fail(c, MLMC_ENOMEM, "batch exceeds the memory budget");
  int rc = ensure_pool(c, level, n);
  if (rc) return rc;
  if (int rc2 = stage_angles(c, level, theta, n, (hipStream_t)stream)) return rc2;
  PcgSlots S = slots_of(c, level, c->rtol);
  launch_setup(c->lv[level].g, c->mat, S, n, b, dinv, (hipStream_t)stream);
  HIPCHK(c, hipGetLastError());
  return MLMC_OK;
}

int mlmc_strip_solve_theta(mlmc_ctx *c, int level, int n, const double *theta, double *q, double *d,
                           mlmc_info *info, int precision, double rtol, void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind == 1) return fail(c, MLMC_ESTATE, "needs a strip or Cosserat context");
  if (bad_level(c, level) || n < 0) return fail(c, MLMC_EINVAL, "level out of range or n < 0");
  if (precision != MLMC_FP64 && precision != MLMC_MIXED) return fail(c, MLMC_EINVAL, "bad precision");
  if (n == 0) return MLMC_OK;
  if (!theta || !q) return fail(c, MLMC_EINVAL, "null pointer");
  if (c->kind == 2) {
    if (precision != MLMC_FP64) return fail(c, MLMC_EINVAL, "the Cosserat model is solved in FP64 only");
    return cos_solve_theta(c->cos, c->err, level, n, theta, q, d, info, rtol, (hipStream_t)stream);
  }
  const bool small = c->lv[level].small;
  const bool mixed = precision == MLMC_MIXED && !small;
  const int cap = max_slots(c, level, mixed);
  if (n > cap) return fail(c, MLMC_ENOMEM, "batch exceeds the memory budget");
  hipStream_t st = (hipStream_t)stream;
  int rc = ensure_pool(c, level, n, mixed);
  if (rc) return rc;
  if (info) launch_info_init(info, nullptr, n, st);
  if ((rc = stage_angles(c, level, theta, n, st))) return rc;
  PcgSlots S = slots_of(c, level, rtol > 0 ? rtol : c->rtol);
  if (small) {
    rc = run_small(c, level, S, n, st);
  } else if (mixed) {
    launch_to_lo(theta, c->lv[level].pool.theta16, c->theta_fp32, (size_t)n * 4 * c->lv[level].g.nelem, st);
    rc = run_mixed(c, {{level, S, n}}, st);
  } else {
    rc = run_pcg(c, {{level, S, n}}, st);
  }
  if (rc) return rc;
  launch_qoi(c->lv[level].g, c->mat, report_view(c, level, S, mixed ? MLMC_MIXED : MLMC_FP64), n,
             c->lv[level].pool.qpart, nullptr, q, nullptr, info, 1 << 30, st);
  if (d) launch_total_disp(c->lv[level].g, S.x, d, n, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  return MLMC_OK;
}

int mlmc_strip_solve_theta_noalloc(mlmc_ctx *c, int level, int n, const double *theta, double *q, mlmc_info *info,
                                   double rtol, void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind != 0) return fail(c, MLMC_ESTATE, "needs a strip context");
  if (bad_level(c, level) || n < 0) return fail(c, MLMC_EINVAL, "level out of range or n < 0");
  if (n == 0) return MLMC_OK;
  if (!theta || !q) return fail(c, MLMC_EINVAL, "null pointer");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (!c->scratch) return fail(c, MLMC_EHIP, "no scratch address on this device: " + c->scratch_err);
  if (dev != c->device) return fail(c, MLMC_ESTATE, "the context's device must be current");
  const double rt = rtol > 0 ? rtol : c->rtol;
  PcgSlots S{};
  double *qpart = nullptr;
  const size_t need = carve_slots(c, level, n, rt, nullptr, &S, &qpart);
  if (need > (size_t)MLMC_SCRATCH_BYTES || n > NOALLOC_MAX_SLOTS)
    return fail(c, MLMC_ENOMEM, "level " + std::to_string(level) + ": " + std::to_string(n) + " solves need " +
                                    std::to_string(need) + " bytes of scratch, more than the fixed " +
                                    std::to_string((size_t)MLMC_SCRATCH_BYTES) + " (or more than " +
                                    std::to_string(NOALLOC_MAX_SLOTS) + " solves)");
  carve_slots(c, level, n, rt, (unsigned char *)c->scratch, &S, &qpart);
  hipStream_t st = (hipStream_t)stream;
  StripLevel &L = c->lv[level];
  // the array keeps the last call's contents: flags, counters and pending-step
  // markers must start at zero
  launch_zero16(c->scratch, need, st);
  if (info) launch_info_init(info, nullptr, n, st);
  const size_t ngp = (size_t)n * 4 * L.g.nelem;
  double *ang = (double *)S.theta;
  if (L.cs) launch_theta_cs(theta, ang, ngp, st);
  else launch_theta_code(theta, ang, ngp, st);
  HIPCHK(c, hipGetLastError());
  // neither event timing nor graph capture (each would create runtime objects)
  const bool prof = c->prof, graphs = c->graphs;
  c->prof = false;
  c->graphs = false;
  const int rc = L.small ? run_small(c, level, S, n, st) : run_pcg(c, {{level, S, n}}, st);
  c->prof = prof;
  c->graphs = graphs;
  if (rc) return rc;
  launch_qoi(L.g, c->mat, S, n, qpart, nullptr, q, nullptr, info, 1 << 30, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(st));
  return MLMC_OK;
}

int mlmc_solve_batch(mlmc_ctx *c, int n_req, const mlmc_request *req, const double *xi, int64_t n_rows, int ld_xi,
                     double *q_fine, double *q_coarse, mlmc_info *info, int precision, double rtol, void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind == 1) return fail(c, MLMC_ESTATE, "solve_batch needs a strip or Cosserat context");
  if (n_req < 0) return fail(c, MLMC_EINVAL, "n_req < 0");
  if (n_req == 0) return MLMC_OK;
  if (!req || !xi || !q_fine || !q_coarse || !info) return fail(c, MLMC_EINVAL, "null pointer");
  if (ld_xi < c->K + 3) return fail(c, MLMC_EINVAL, "ld_xi < n_modes + 3");
  if (precision != MLMC_FP64 && precision != MLMC_MIXED) return fail(c, MLMC_EINVAL, "bad precision");
  if (c->kind == 2) {
    if (precision != MLMC_FP64) return fail(c, MLMC_EINVAL, "the Cosserat model is solved in FP64 only");
    return cos_solve_batch(c->cos, c->err, n_req, req, xi, n_rows, ld_xi, q_fine, q_coarse, info, rtol,
                           (hipStream_t)stream);
  }
  for (int i = 0; i < n_req; ++i) {
    if (bad_level(c, req[i].level)) return fail(c, MLMC_EINVAL, "request " + std::to_string(i) + ": bad level");
    if (req[i].sample < 0 || req[i].sample >= n_rows)
      return fail(c, MLMC_EINVAL, "request " + std::to_string(i) + ": sample row outside [0, n_rows)");
  }
  hipStream_t st = (hipStream_t)stream;
  const double rt = rtol > 0 ? rtol : c->rtol;
  launch_info_init(info, q_coarse, n_req, st);
  HIPCHK(c, hipGetLastError());
  // jobs per level: the fine solves of its requests and the coarse solves of
  // coupled requests one level up share the level's slots; output index i
  // stands for the fine result of request i, n_req + i for its coarse result
  std::vector<std::vector<int64_t>> rows(c->nlev);
  std::vector<std::vector<int>> outs(c->nlev);
  for (int i = 0; i < n_req; ++i) {
    const int l = req[i].level;
    rows[l].push_back(req[i].sample);
    outs[l].push_back(i);
  }
  for (int i = 0; i < n_req; ++i) {
    const int l = req[i].level;
    if (req[i].coupled && l > 0) {
      rows[l - 1].push_back(req[i].sample);
      outs[l - 1].push_back(n_req + i);
    }
  }
  // slots per level (coarse levels solved whole per work-group run in FP64 in either precision)
  std::vector<int> cap(c->nlev, 0), done(c->nlev, 0);
  for (int l = 0; l < c->nlev; ++l) {
    const int total = (int)rows[l].size();
    if (!total) continue;
    const bool mixed = precision == MLMC_MIXED && !c->lv[l].small;
    cap[l] = std::min(max_slots(c, l, mixed), total);
    if (cap[l] < 1) return fail(c, MLMC_ENOMEM, "level " + std::to_string(l) + ": no slot fits the budget");
    if (int rc = ensure_pool(c, l, cap[l], mixed)) return rc;
  }
  // rounds: every level with work left takes its next chunk; the coarse levels
  // run whole per work-group, the others share lock-step launches
  for (;;) {
    std::vector<int> lvls, cnt;
    for (int l = 0; l < c->nlev; ++l)
      if (done[l] < (int)rows[l].size()) lvls.push_back(l);
    if (lvls.empty()) break;
    std::vector<SolveGroup> lock;
    bool any_small = false;
    for (int l : lvls) {
      StripLevel &L = c->lv[l];
      const int n = std::min(cap[l], (int)rows[l].size() - done[l]);
      const bool mixed = precision == MLMC_MIXED && !L.small;
      HIPCHK(c, hipMemcpyAsync(L.pool.rows, rows[l].data() + done[l], sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
      HIPCHK(c, hipMemcpyAsync(L.pool.outidx, outs[l].data() + done[l], sizeof(int) * n, hipMemcpyHostToDevice, st));
      launch_kl_synth(L.modes, c->K, L.g, xi, ld_xi, L.pool.rows, n, L.cs ? nullptr : L.pool.theta,
                      mixed ? L.pool.theta16 : nullptr, c->theta_fp32, 4 * L.g.nelem, L.cs ? L.pool.theta : nullptr,
                      1, st);
      if (L.small) any_small = true;
      else lock.push_back({l, slots_of(c, l, rt), n});
      cnt.push_back(n);
    }
    // whole-solve levels (one work-group per sample, few waves per CU) run on
    // the side stream while the lock-step launches run on the caller's.  They
    // start after the lock-step set-up kernels: their work-groups live for a
    // whole solve, and the set-up's last work-groups would otherwise wait for
    // them to leave the CUs before the first iteration could start.
    hipStream_t side = lock.empty() ? st : c->side_stream;
    bool side_started = false;
    auto start_side = [&]() -> int {
      if (side_started) return MLMC_OK;
      side_started = true;
      if (any_small && side != st) {
        HIPCHK(c, hipEventRecord(c->ev_fork, st));
        HIPCHK(c, hipStreamWaitEvent(side, c->ev_fork, 0));
      }
      for (size_t k = 0; k < lvls.size(); ++k) {
        const int l = lvls[k];
        StripLevel &L = c->lv[l];
        if (!L.small) continue;
        PcgSlots S = slots_of(c, l, rt);
        if (int rc = run_small(c, l, S, cnt[k], side)) return rc;
        launch_qoi(L.g, c->mat, report_view(c, l, S, MLMC_FP64), cnt[k], L.pool.qpart, L.pool.outidx, q_fine,
                   q_coarse, info, n_req, side);
      }
      return MLMC_OK;
    };
    if (lock.empty())
      if (int rc = start_side()) return rc;
    for (size_t k0 = 0; k0 < lock.size(); k0 += MAX_GROUPS) {
      std::vector<SolveGroup> part(lock.begin() + k0, lock.begin() + std::min(lock.size(), k0 + MAX_GROUPS));
      const int rc = precision == MLMC_MIXED ? run_mixed(c, part, st, start_side) : run_pcg(c, part, st, start_side);
      if (rc) return rc;
    }
    for (size_t k = 0; k < lvls.size(); ++k) {
      const int l = lvls[k];
      StripLevel &L = c->lv[l];
      if (L.small) continue;
      const bool mixed = precision == MLMC_MIXED;
      PcgSlots S = slots_of(c, l, rt);
      launch_qoi(L.g, c->mat, report_view(c, l, S, mixed ? MLMC_MIXED : MLMC_FP64), cnt[k], L.pool.qpart,
                 L.pool.outidx, q_fine, q_coarse, info, n_req, st);
    }
    if (any_small && side != st) {
      HIPCHK(c, hipEventRecord(c->ev_join, side));
      HIPCHK(c, hipStreamWaitEvent(st, c->ev_join, 0));
    }
    for (size_t k = 0; k < lvls.size(); ++k) done[lvls[k]] += cnt[k];
    HIPCHK(c, hipGetLastError());
    // the row/index buffers are reused by the next round
    HIPCHK(c, hipStreamSynchronize(st));
  }
  return MLMC_OK;
}

int mlmc_buckle_batch(mlmc_ctx *c, int n_req, const mlmc_request *req, const double *ply_offsets, int64_t n_rows,
                      double *lam_fine, double *lam_coarse, mlmc_info *info, int precision, double tol,
                      void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind != 1) return fail(c, MLMC_ESTATE, "buckle_batch needs a plate context");
  return plate_buckle_batch(c->plate, c->err, n_req, req, ply_offsets, n_rows, lam_fine, lam_coarse, info,
                            precision, tol, (hipStream_t)stream);
}

int mlmc_level_stats(mlmc_ctx *c, int level, int n, const double *q_fine, const double *q_coarse,
                     double cost_per_sample, double lambda_star, mlmc_level_acc *acc, void *stream) {
  if (!c) return MLMC_EINVAL;
  if (bad_level(c, level) || n < 0) return fail(c, MLMC_EINVAL, "level out of range or n < 0");
  if (!acc) return fail(c, MLMC_EINVAL, "acc is NULL");
  if (n == 0) return MLMC_OK;
  if (!q_fine) return fail(c, MLMC_EINVAL, "q_fine is NULL");
  hipStream_t st = (hipStream_t)stream;
  const int ind = std::isnan(lambda_star) ? 0 : 1;
  launch_level_stats(q_fine, q_coarse, n, lambda_star, ind, c->d_stats, st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->h_stats, c->d_stats, 10 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  const double *o = c->h_stats;
  auto add = [](double &s, double &cp, double v, double vc) {
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v)) cp += (s - t) + v;
    else cp += (v - t) + s;
    s = t;
    cp += vc;
  };
  add(acc->sum_y, acc->comp_y, o[0], o[1]);
  add(acc->sum_y2, acc->comp_y2, o[2], o[3]);
  add(acc->sum_qf, acc->comp_qf, o[4], o[5]);
  add(acc->sum_qc, acc->comp_qc, o[6], o[7]);
  acc->n += n;
  acc->n_plus += (int64_t)o[8];
  acc->n_minus += (int64_t)o[9];
  acc->sum_cost += cost_per_sample * n;
  return MLMC_OK;
}

int mlmc_plate_apply(mlmc_ctx *c, int level, int n, const double *ply_offsets, int geometric, const double *x,
                     double *y, void *stream) {
  if (!c) return MLMC_EINVAL;
  if (c->kind != 1) return fail(c, MLMC_ESTATE, "plate_apply needs a plate context");
  if (n > 0 && (!ply_offsets || !x || !y)) return fail(c, MLMC_EINVAL, "null pointer");
  return plate_apply_diag(c->plate, c->err, level, n, ply_offsets, geometric, x, y, (hipStream_t)stream);
}

int mlmc_profile_enable(mlmc_ctx *c, int on) {
  if (!c) return MLMC_EINVAL;
  c->prof = on != 0;
  for (int k = 0; k < 4; ++k) {
    c->prof_ms[k] = 0;
    c->prof_bytes[k] = 0;
    c->prof_dofs[k] = 0;
    c->prof_launches[k] = 0;
  }
  return MLMC_OK;
}

int mlmc_profile_read(mlmc_ctx *c, int kernel, double *total_ms, int64_t *launches, double *alg_bytes) {
  if (!c) return MLMC_EINVAL;
  if (kernel < 0 || kernel > 7) return fail(c, MLMC_EINVAL, "kernel must be 0..7");
  const int k = kernel & 3;
  if (total_ms) *total_ms = c->prof_ms[k];
  if (launches) *launches = c->prof_launches[k];
  if (alg_bytes) *alg_bytes = kernel < 4 ? c->prof_bytes[k] : c->prof_dofs[k];
  return MLMC_OK;
}

}  // extern "C"
