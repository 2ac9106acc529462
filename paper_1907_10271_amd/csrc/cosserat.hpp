// Cosserat model of Test Problem I (Section 3.1 of the paper): host side of
// the batched sample solves (KL synthesis with the level's number of modes,
// matrix-free operator with three unknowns per node, lock-step Jacobi-PCG and
// the strength quantity of interest).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "json.hpp"
#include "mlmc.h"

namespace mlmc {

struct CosCtx;

CosCtx *cos_create(const Json &cfg, size_t budget, std::string &err);
void cos_destroy(CosCtx *c);
int cos_num_levels(const CosCtx *c);
int cos_num_params(const CosCtx *c);  // values per parameter row the calls read (modes + 3)
void cos_level_sizes(const CosCtx *c, int level, int64_t *n_nodes, int64_t *n_dofs, int64_t *n_elem);
size_t cos_slot_bytes(const CosCtx *c, int level);
int cos_reserve(CosCtx *c, std::string &err, int level, int n);
int cos_sample_field(CosCtx *c, std::string &err, int level, int n, const double *xi, int ld_xi, double *theta,
                     hipStream_t st);
int cos_apply(CosCtx *c, std::string &err, int level, int n, const double *theta, const double *x, double *y,
              int raw, hipStream_t st);
int cos_rhs_diag(CosCtx *c, std::string &err, int level, int n, const double *theta, double *b, double *dinv,
                 hipStream_t st);
int cos_solve_theta(CosCtx *c, std::string &err, int level, int n, const double *theta, double *q, double *d,
                    mlmc_info *info, double rtol, hipStream_t st);
int cos_solve_batch(CosCtx *c, std::string &err, int n_req, const mlmc_request *req, const double *xi,
                    int64_t n_rows, int ld_xi, double *q_fine, double *q_coarse, mlmc_info *info, double rtol,
                    hipStream_t st);

}  // namespace mlmc
