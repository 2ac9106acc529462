// Plate buckling (Section 4.1): placeholder until the batched eigen-solver lands.
#include "plate.hpp"

namespace mlmc {

struct PlateCtx {
  int nlev = 0;
  int nx0 = 0, ny0 = 0;
};

PlateCtx *plate_create(const Json &cfg, std::string &err) {
  PlateCtx *p = new PlateCtx();
  try {
    p->nlev = (int)cfg.number("n_levels");
    p->nx0 = (int)cfg.number("nx0");
    p->ny0 = (int)cfg.number("ny0");
  } catch (const std::exception &e) {
    err = e.what();
    delete p;
    return nullptr;
  }
  return p;
}

void plate_destroy(PlateCtx *p) { delete p; }
int plate_num_levels(const PlateCtx *p) { return p->nlev; }

void plate_level_sizes(const PlateCtx *p, int level, int64_t *nn, int64_t *nd, int64_t *ne) {
  const int64_t nx = (int64_t)p->nx0 << level, ny = (int64_t)p->ny0 << level;
  *nn = (nx + 1) * (ny + 1);
  *nd = 5 * *nn;
  *ne = nx * ny;
}

size_t plate_slot_bytes(const PlateCtx *p, int level, int) {
  int64_t nn, nd, ne;
  plate_level_sizes(p, level, &nn, &nd, &ne);
  return (size_t)nd * 8 * 16;
}

int plate_buckle_batch(PlateCtx *, std::string &err, int, const mlmc_request *, const double *, int64_t, double *, double *,
                       mlmc_info *, int, double, hipStream_t) {
  err = "plate buckling solver is not built";
  return MLMC_ESTATE;
}

}  // namespace mlmc
