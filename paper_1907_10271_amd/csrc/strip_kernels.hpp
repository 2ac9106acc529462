// Launchers of the strip kernels (host side).
#pragma once

#include "common.hpp"
#include "mlmc.h"

namespace mlmc {

using mlmc_info_dev = ::mlmc_info;

// KL synthesis of n samples (parameter rows rows[s], or s); optional outputs:
// th64 [n][ld_out] FP64 angles (code != 0: their codes tan theta, the solver's
// storage), thlo [n][ld_out] bfloat16/FP32 angles, cs [n][4 nelem][2]
// (cos 2theta, sin 2theta)
void launch_kl_synth(const double *modes, int K, const StripGeom &g, const double *xi, int ld_xi,
                     const int64_t *rows, int n, double *th64, void *thlo, int lo_fp32, int ld_out, double *cs,
                     int code, hipStream_t st);
// (cos 2theta, sin 2theta) of n angles
void launch_theta_cs(const double *theta, double *cs, size_t n, hipStream_t st);
// angle codes tan theta of n angles
void launch_theta_code(const double *theta, double *code, size_t n, hipStream_t st);
void launch_modes_nystrom(const double *gx, const double *gy, const double *coef, int ngrid, int K, double var,
                          double kappa, const StripGeom &g, double *modes, hipStream_t st);
void launch_apply(const StripGeom &g, const StripMat &m, const double *theta, const double *x, double *y, int raw,
                  int n, hipStream_t st);
void launch_setup(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, double *b_out, double *dinv_out,
                  hipStream_t st);
// one lock-step PCG iteration over the groups of a device descriptor array
// (nblocks = sum of sweep tiles x slots, resp. chunks x slots)
// (cs: the groups' FP64 angle data holds (cos 2theta, sin 2theta) pairs, or,
// for the FP32 solver, FP32 angles instead of bfloat16 ones).
// The iteration index is `it`, or *itb + it when itb is not null (graph
// replay: the captured launches carry offsets, the base lives on the device).
// nt: streaming (nontemporal) accesses for the vectors that pass through
// once, for launches whose working set is larger than the Infinity Cache;
// the results do not depend on it.
template <typename T>
void launch_pcg_pass1(const PcgGroup<T> *groups, int ng, int nblocks, const StripMat &m, int it, int cs,
                      const int *itb, hipStream_t st, bool nt);
// operator-pass waves (one per work-group) the device keeps resident at once
template <typename T>
int pass1_resident_waves(int cs);
template <typename T>
void launch_pcg_pass2(const PcgGroup<T> *groups, int ng, int nblocks, int it, const int *itb, hipStream_t st,
                      bool nt);
void launch_resid64(const StripGeom &g, const StripMat &m, const PcgSlots &D, const PcgState<float> &I,
                    const MixedState &M, int n, int it, int every, const int *itb, hipStream_t st);
void launch_ru_apply(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, const MixedState &M, int n,
                     int it, int every, const int *itb, hipStream_t st);
// zero `bytes` (a multiple of 16) at a 16-byte aligned device address
void launch_zero16(void *p, size_t bytes, hipStream_t st);
// *p = v and *p += v by one thread (kernel nodes, so they can be captured)
void launch_set_int(int *p, int v, hipStream_t st);
void launch_add_int(int *p, int v, hipStream_t st);
void launch_mixed_start(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, const MixedState &M, int n,
                        hipStream_t st);
// after the FP64 iterations: add the pending step of slots 0..n-1 to x
void launch_x_flush(const StripGeom &g, const PcgSlots &S, int n, hipStream_t st);
void launch_mixed_flush(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, int n, hipStream_t st);
int qoi_parts(const StripGeom &g);
// QoI of n slots, written through out_idx: entries below coarse_base go to
// q_fine, the others (minus coarse_base) to q_coarse and the coarse info fields
void launch_qoi(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, double *part, const int *out_idx,
                double *q_fine, double *q_coarse, mlmc_info_dev *info, int coarse_base, hipStream_t st);
void launch_total_disp(const StripGeom &g, const double *x, double *d, int n, hipStream_t st);
void launch_to_lo(const double *a, void *b, int lo_fp32, size_t n, hipStream_t st);
void launch_info_init(mlmc_info_dev *info, double *q_coarse, int n, hipStream_t st);
void launch_level_stats(const double *qf, const double *qc, int n, double lambda_star, int indicator, double *out,
                        hipStream_t st);

}  // namespace mlmc
