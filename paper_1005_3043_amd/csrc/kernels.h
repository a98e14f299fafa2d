// Host-side launchers of the HIP kernels (one translation unit per kernel
// family).  Every launcher enqueues on `st` and returns the launch status.
#pragma once

#include "common.h"

namespace mg {

// ---- pack.hip: canonical complex128 [nvec][sites lex][ncomp] <-> internal
//      [nvec][ncomp][V] site-blocked planes of complex<T>.
template <typename T>
hipError_t pack_field(const Geom &g, const double2 *canon, c_t<T> *internal, int ncomp, int nvec,
                      hipStream_t st);
template <typename T>
hipError_t unpack_field(const Geom &g, const c_t<T> *internal, double2 *canon, int ncomp, int nvec,
                        hipStream_t st);

// ---- dslash.hip: fine Wilson operator on internal spinors (12 planes).
enum DslashMode { DS_PLAIN = 0, DS_RESID = 1, DS_MR = 2 };
// out = diag*in - 1/2 hop(in)              (DS_PLAIN)
// out = b - (diag*in - 1/2 hop(in))        (DS_RESID)
// out = D in; partials[blk] += (<out,in>, ||out||^2)  (DS_MR, 3 doubles / block)
template <typename R>
hipError_t dslash(const Geom &g, const c_t<R> *U, const c_t<R> *in, c_t<R> *out, const c_t<R> *b,
                  double diag, int nrhs, DslashMode mode, double *partials, hipStream_t st);
int dslash_blocks(const Geom &g);  // number of partial slots per RHS of DS_MR

// ---- blas.hip
template <typename R> hipError_t zero(c_t<R> *x, size_t n, hipStream_t st);
template <typename R> hipError_t copy(c_t<R> *y, const c_t<R> *x, size_t n, hipStream_t st);
template <typename Rd, typename Rs>
hipError_t convert(c_t<Rd> *y, const c_t<Rs> *x, size_t n, hipStream_t st);

}  // namespace mg
