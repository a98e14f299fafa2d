// Declarations shared by the orchestration (mg.cpp) and the C entry points.
#pragma once

#include "solver.h"

namespace mg {

template <typename R> Work<R> &work(mg_ctx *c);
int ensure_scalars(mg_ctx *c, size_t part_count);
void clear_graphs(mg_ctx *c);
size_t np_coarse(const Level &L);
size_t part_need(mg_ctx *c, int nrhs);
int ensure_prec(mg_ctx *c, mg_prec_t prec, hipStream_t st);
template <typename R> int ensure_work(mg_ctx *c, int nrhs);
template <typename R>
int apply_A(mg_ctx *c, int l, const c_t<R> *in, c_t<R> *out, int nrhs, DslashMode mode, const c_t<R> *b,
            hipStream_t st);
template <typename R>
int transfer_restrict(mg_ctx *c, int l, const c_t<R> *fine, c_t<R> *coarse, int nrhs, hipStream_t st);
template <typename R>
int transfer_prolong(mg_ctx *c, int l, const c_t<R> *coarse, c_t<R> *fine, int nrhs, int accumulate,
                     hipStream_t st);
template <typename R> int vcycle(mg_ctx *c, int l, const c_t<R> *rin, c_t<R> *x, int nrhs, hipStream_t st);
int fgcr(mg_ctx *c, const double2 *b, double2 *x, int nrhs, double tol, int *iters, double *relres,
         hipStream_t st);
int setup(mg_ctx *c, const void *U, hipStream_t st);
int check_lattice(const mg_lattice_t *lat);

}  // namespace mg
