// C ABI: multigrid context entry points.
#include "kernels.h"

using namespace mg;

static int notsup(const char *f) {
  set_error(std::string(f) + ": not built yet");
  return MG_ENOTSUP;
}

extern "C" int mg_setup(const mg_lattice_t *, const void *, double, const mg_params_t *, mg_ctx_t **,
                        hipStream_t) { return notsup("mg_setup"); }
extern "C" int mg_set_precond_prec(mg_ctx_t *, mg_prec_t) { return notsup("mg_set_precond_prec"); }
extern "C" int mg_set_timing(mg_ctx_t *, int) { return notsup("mg_set_timing"); }
extern "C" int mg_restrict(mg_ctx_t *, int, const void *, void *, int, hipStream_t) { return notsup("mg_restrict"); }
extern "C" int mg_prolong(mg_ctx_t *, int, const void *, void *, int, hipStream_t) { return notsup("mg_prolong"); }
extern "C" int coarse_apply(mg_ctx_t *, int, const void *, void *, int, int, hipStream_t) {
  return notsup("coarse_apply");
}
extern "C" int mg_solve(mg_ctx_t *, const void *, void *, int, double, mg_info_t *, hipStream_t) {
  return notsup("mg_solve");
}
extern "C" int mg_time_dslash(mg_ctx_t *, mg_prec_t, int, int, double *, hipStream_t) {
  return notsup("mg_time_dslash");
}
extern "C" int mg_time_coarse(mg_ctx_t *, int, mg_prec_t, int, int, double *, hipStream_t) {
  return notsup("mg_time_coarse");
}
extern "C" int mg_destroy(mg_ctx_t *) { return MG_OK; }
extern "C" int mg_export_maps(mg_ctx_t *, int, int32_t *, int32_t *, int32_t *, int32_t *) {
  return notsup("mg_export_maps");
}
extern "C" int mg_export_P(mg_ctx_t *, int, void *) { return notsup("mg_export_P"); }
extern "C" int mg_export_coarse_op(mg_ctx_t *, int, void *, void *) { return notsup("mg_export_coarse_op"); }
extern "C" int mg_export_nullvecs(mg_ctx_t *, int, void *) { return notsup("mg_export_nullvecs"); }
extern "C" int mg_level_info(mg_ctx_t *, int, int *, int *) { return notsup("mg_level_info"); }
