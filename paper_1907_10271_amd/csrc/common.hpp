// Shared host/device definitions of the MLMC library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mlmc {

// node tile of the strip operator: owned nodes per work-group
constexpr int TILE_X = 32;
constexpr int TILE_Y = 8;
constexpr int TILE_NODES = TILE_X * TILE_Y;    // owned nodes per tile
constexpr int TILE_THREADS = 320;              // >= halo elements: one element per thread
constexpr int HALO_X = TILE_X + 2;             // nodes incl. one-node halo
constexpr int HALO_Y = TILE_Y + 2;
constexpr int ELEM_X = TILE_X + 1;             // elements touching the owned nodes
constexpr int ELEM_Y = TILE_Y + 1;
constexpr int TILE_NODES_H = HALO_X * HALO_Y;
constexpr int TILE_ELEMS = ELEM_X * ELEM_Y;
static_assert(TILE_ELEMS <= TILE_THREADS && TILE_NODES <= TILE_THREADS, "tile too large for the block");
constexpr int TILE_WAVES = TILE_THREADS / 64;

// column sweep: one wave owns up to SWEEP_MAXW node columns plus one halo
// column on each side and walks up the element rows
constexpr int SWEEP_MAXW = 62;
constexpr int SWEEP_MAXTY = 16;
// dot-product partials of the operator pass are kept per block of SWEEP_RB node
// rows (and column tile), so any tile height that is a multiple of SWEEP_RB
// gives the same sums: the height can follow the batch size
constexpr int SWEEP_RB = 4;
// vector pass: CHUNK consecutive nodes per 256-thread block
constexpr int CHUNK = 1024;

// 2x2 Gauss rule: the bilinear interpolation weights at +-1/sqrt(3) are
// (1 + 1/sqrt3)/2 and (1 - 1/sqrt3)/2
constexpr double GP_P = 0.78867513459481288225;
constexpr double GP_M = 0.21132486540518711775;

// geometry of one strip level (uniform rectangles hx x hy)
struct StripGeom {
  int nx, ny;        // elements per row / column
  int nnx, nny;      // nodes per row / column
  int nnode, nelem;
  int tiles_x, tiles_y, ntiles;    // 2-D LDS tiles (set-up and the stand-alone operator)
  int sw_tw, sw_ty, sw_ntx, sw_nty, sw_ntiles;  // column-sweep tiles of the PCG operator pass
  int sw_npart;                    // operator-pass partials per sample: row blocks x column tiles
  int nchunks;                     // contiguous node chunks of the PCG vector pass
  int qx0, qx1, qy0, qy1;  // QoI element index ranges [q*0, q*1)
  double hx, hy, ihx, ihy, wdet;  // wdet = Gauss weight x det J = hx hy / 4
  // interpolation weights with the 1/h of the derivative folded in (strain),
  // and with the quadrature weight as well (transposed operator)
  double pxi, mxi, pyi, myi, pxw, mxw, pyw, myw;
  double delta;                   // u = -delta on x = Lx
  double Lx, Ly;
};

// rotation invariants of the ply stiffness: Qbar(theta) is linear in
// cos 2theta, sin 2theta, cos 4theta, sin 4theta with these coefficients
struct StripMat {
  double U1, U2, U3, U4, U5;
  double Q11, Q22, Q12, Q66;
  float fU1, fU2, fU3, fU4, fU5;   // the same invariants rounded to FP32
};

// per-slot PCG state of a level pool (device pointers); T = double for the
// FP64 solver, float for the inner solver of the mixed-precision form
// The residual is kept preconditioned: z = dinv r with dinv = 1/dg, dg the
// Jacobi diagonal (1 on prescribed unknowns); r is recovered as dg z where it
// is needed.  The operator pass then reads one vector less per node.
template <typename T>
struct PcgState {
  T *x, *z, *p, *Ap, *dg;          // [S][2 nnode]; all slots iterate in lock-step
  const void *theta;               // [S][4 nelem]: double (FP64) or bfloat16 bits (float solver)
  double *part_pap;                // [S][sw_ntiles]
  double *part_rz, *part_rr;       // [2][S][nchunks]
  double *rzs;                     // [2][S]
  double *tol2, *bb, *relres;      // [S]
  int *it_a, *it_b, *status, *active;  // [S]
  int S;
  int max_iter;
  double rtol2;
  // reliable updates (inner solver of the mixed form only; unused when mixed == 0):
  // a slot whose FP32 residual fell by ru2 since its last FP64 residual, or
  // meets the stopping test, records ru[s] = it + 1 and pauses for one iteration
  int mixed;
  int theta_fp32;                  // float solver: angles stored as FP32 instead of bfloat16
  int cs;                          // FP64 solver: angle data holds (cos 2theta, sin 2theta) pairs
                                   // [nelem][4][2] (1) or the angles [nelem][4] (0)
  double ru2;
  double *rr_ref;                  // [S] ||r||^2 at the last FP64 residual
  int *ru;                         // [S]
  // x takes two steps at once, every second completed vector pass (the
  // deferred step's p is the next pass's p_old, already loaded there).
  // xs[1][s]: whether the last completed vector pass left its step pending
  // (set-up clears it).  FP32 inner solver: xa[1][s] is that step's alpha,
  // and xs[0] / xa[0] the same copied by the operator pass for the vector pass
  // of its iteration (so no launch reads what it writes).  FP64 solver: steps
  // are deferred at even iterations, whose alpha is xa[0][s].
  double *xa;                      // [2][S]
  int *xs;                         // [2][S]
};
using PcgSlots = PcgState<double>;

// one level's batch inside a lock-step launch that serves several levels at
// once (fine and coarse solves of coupled samples, uneven batch sizes): the
// launch's blocks are laid out group after group
constexpr int MAX_GROUPS = 4;
template <typename T>
struct PcgGroup {
  StripGeom g;
  PcgState<T> S;
  int n;        // slots of the group
  int blk0;     // first operator-pass block (sweep tiles x slots)
  int cblk0;    // first vector-pass block (chunks x slots)
};

// FP64 side of the mixed-precision solver
struct MixedState {
  double *b;                       // [S][2 nnode] right-hand side
  double *part_rr;                 // [S][sw_ntiles] partial ||b - A x||^2
  double *part_bb;                 // [S][nchunks] partial ||b||^2 (from the FP64 set-up)
  double *relres;                  // [S] last FP64 relative residual
  int *updates;                    // [S] FP64 residuals computed
  double rtol2;
};

enum SampleStatus { S_OK = 0, S_NOCONV = 1, S_NAN = 2, S_BREAKDOWN = 3, S_SKIPPED = 4, S_NOTLOWEST = 5 };

}  // namespace mlmc
