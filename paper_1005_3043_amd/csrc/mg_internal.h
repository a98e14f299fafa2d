// Declarations shared by the orchestration (mg.cpp) and the C entry points.
#pragma once

#include "solver.h"

namespace mg {

template <typename R> Work<R> &work(mg_ctx *c);
template <typename P> int coarse_variant(mg_ctx *c, int l, int nrhs, hipStream_t st);
int ensure_scalars(mg_ctx *c, size_t part_count);
void clear_graphs(mg_ctx *c);
size_t np_coarse(const Level &L);
size_t part_need(mg_ctx *c, int nrhs);
int ensure_prec(mg_ctx *c, mg_prec_t prec, hipStream_t st);
template <typename R> int ensure_work(mg_ctx *c, int nrhs);
// buffers of the fine-level MR by the q recursion for precision class prec
// (MG_F32 or MG_F16; no-op otherwise) and MR runs of `steps` steps (default:
// those of the cycle's smoother; no-op when it is not MR)
int ensure_mrq(mg_ctx *c, mg_prec_t prec, int nrhs, int steps = -1);
template <typename P>
int apply_A(mg_ctx *c, int l, const vec_t<P> *in, vec_t<P> *out, int nrhs, DslashMode mode, const vec_t<P> *b,
            hipStream_t st);
// fine stored as TR: vec_t<P>, or h16 on level 0 of the FP16 class
template <typename P, typename TR = vec_t<P>>
int transfer_restrict(mg_ctx *c, int l, const TR *fine, vec_t<P> *coarse, int nrhs, hipStream_t st);
template <typename P>
int transfer_prolong(mg_ctx *c, int l, const vec_t<P> *coarse, vec_t<P> *fine, int nrhs, int accumulate,
                     hipStream_t st);
template <typename P> int cgnr(mg_ctx *c, int l, const vec_t<P> *b, vec_t<P> *e, int nrhs, hipStream_t st);
template <typename P> int vcycle(mg_ctx *c, int l, const vec_t<P> *rin, vec_t<P> *x, int nrhs, hipStream_t st);
int ensure_fgcr(mg_ctx *c, int nrhs);
int fgcr(mg_ctx *c, const double2 *b, double2 *x, int nrhs, double tol, int *iters, double *relres,
         hipStream_t st);
int precondition_at(mg_ctx *c, mg_prec_t prec, const double2 *r, double2 *z, int nrhs, hipStream_t st);
int setup(mg_ctx *c, const void *U, hipStream_t st);
int check_lattice(const mg_lattice_t *lat);
template <typename P> const typename P::S *links_of_level(Level &L);
template <typename P> const typename P::S *cop_of_level(Level &L);
template <typename P> const void *cop_t_of_level(mg_ctx *c, Level &L, hipStream_t st);

}  // namespace mg
