// Plate buckling part of the library (Section 4.1 of the paper): laminate
// set-up, the Reissner-Mindlin operators and the batched eigen-solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "json.hpp"
#include "mlmc.h"

namespace mlmc {

struct PlateCtx;

PlateCtx *plate_create(const Json &cfg, std::string &err);
void plate_destroy(PlateCtx *p);
int plate_num_levels(const PlateCtx *p);
void plate_level_sizes(const PlateCtx *p, int level, int64_t *n_nodes, int64_t *n_dofs, int64_t *n_elem);
size_t plate_slot_bytes(const PlateCtx *p, int level, int precision);
int plate_reserve(PlateCtx *p, std::string &err, int level, int n);
void plate_set_budget(PlateCtx *p, size_t bytes);
int plate_buckle_batch(PlateCtx *p, std::string &err, int n_req, const mlmc_request *req, const double *offsets,
                       int64_t n_rows, double *lam_fine, double *lam_coarse, mlmc_info *info, int precision, double tol,
                       hipStream_t st);

int plate_apply_diag(PlateCtx *p, std::string &err, int level, int n, const double *offsets, int geom,
                     const double *x, double *y, hipStream_t st);

}  // namespace mlmc
