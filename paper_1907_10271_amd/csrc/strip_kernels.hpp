// Launchers of the strip kernels (host side).
#pragma once

#include "common.hpp"
#include "mlmc.h"

namespace mlmc {

using mlmc_info_dev = ::mlmc_info;

void launch_kl_synth(const double *modes, int K, const StripGeom &g, const double *xi, int ld_xi,
                     const int64_t *rows, int n, double *th64, void *thlo, int lo_fp32, int ld_out, hipStream_t st);
void launch_modes_nystrom(const double *gx, const double *gy, const double *coef, int ngrid, int K, double var,
                          double kappa, const StripGeom &g, double *modes, hipStream_t st);
void launch_apply(const StripGeom &g, const StripMat &m, const double *theta, const double *x, double *y, int raw,
                  int n, hipStream_t st);
void launch_setup(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, double *b_out, double *dinv_out,
                  hipStream_t st);
template <typename T>
void launch_pcg_pass1(const StripGeom &g, const StripMat &m, const PcgState<T> &S, int n, int it, hipStream_t st);
template <typename T>
void launch_pcg_pass2(const StripGeom &g, const PcgState<T> &S, int n, int it, hipStream_t st);
void launch_resid64(const StripGeom &g, const StripMat &m, const PcgSlots &D, const PcgState<float> &I,
                    const MixedState &M, int n, int it, int every, hipStream_t st);
void launch_ru_apply(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, const MixedState &M, int n,
                     int it, int every, hipStream_t st);
void launch_mixed_start(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, const MixedState &M, int n,
                        hipStream_t st);
void launch_mixed_flush(const StripGeom &g, const PcgSlots &D, const PcgState<float> &I, int n, hipStream_t st);
int qoi_parts(const StripGeom &g);
void launch_qoi(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, double *part, const int *out_idx,
                double *q, mlmc_info_dev *info, int coarse, hipStream_t st);
void launch_total_disp(const StripGeom &g, const double *x, double *d, int n, hipStream_t st);
void launch_to_lo(const double *a, void *b, int lo_fp32, size_t n, hipStream_t st);
void launch_info_init(mlmc_info_dev *info, double *q_coarse, int n, hipStream_t st);
void launch_level_stats(const double *qf, const double *qc, int n, double lambda_star, int indicator, double *out,
                        hipStream_t st);

}  // namespace mlmc
