// Multigrid context and the launchers of the solver's streaming kernels.
#pragma once

#include <vector>

#include "kernels.h"

namespace mg {

constexpr int RED_BLOCKS = 1024;  // fixed grid of generic reductions
constexpr int CG_NS = 8;          // CGNR scalars per right-hand side

// ---- solver_kernels.hip
template <typename R>
hipError_t mr_update(c_t<R> *x, c_t<R> *r, const c_t<R> *q, size_t n, int nrhs, const double *part, int np,
                     double omega, double2 *alpha, int first, hipStream_t st);
template <typename R> hipError_t norm2(const c_t<R> *a, size_t n, int nrhs, double *part, double *out, hipStream_t st);
// launches the per-block partials of ||a||^2 and returns their count per RHS
template <typename R> int norm2_partials(const c_t<R> *a, size_t n, int nrhs, double *part, hipStream_t st);
template <typename R>
hipError_t dot(const c_t<R> *a, const c_t<R> *b, size_t n, int nrhs, double *part, double2 *out, hipStream_t st);
hipError_t finish_sum1(const double *part, int np, int nrhs, double *out, hipStream_t st);
hipError_t cg_init_scalars(const double *part_z, int npz, const double *part_b, int npb, int nrhs, double *cg,
                           int *done, int *it, double tol, hipStream_t st);
hipError_t cg_alpha(const double *part, int np, int nrhs, double *cg, int *done, hipStream_t st);
template <typename R>
hipError_t cg_update(c_t<R> *e, const c_t<R> *p, c_t<R> *r, const c_t<R> *w, size_t n, int nrhs, double *cg,
                     int *done, int *it, int maxit, double *part, hipStream_t st);
hipError_t cg_beta(const double *part, int np, int nrhs, double *cg, int *done, hipStream_t st);
template <typename R>
hipError_t cg_p(c_t<R> *p, const c_t<R> *z, size_t n, int nrhs, const double *cg, const int *done, hipStream_t st);
hipError_t gcr_sub2(double2 *y, const double2 *x, double2 *v, const double2 *u, size_t n, int nrhs,
                    const double2 *sc, const int *skip, hipStream_t st);
hipError_t gcr_scale2(double2 *y, double2 *v, size_t n, int nrhs, const double *nrm2, const int *skip,
                      hipStream_t st);
hipError_t gcr_update(double2 *x, const double2 *z, double2 *r, const double2 *w, size_t n, int nrhs,
                      const double2 *sc, const int *skip, double *part, double *rr, hipStream_t st);
// v -= x
template <typename R> hipError_t sub_inplace(c_t<R> *v, const c_t<R> *x, size_t n, int nrhs, hipStream_t st);
// v *= 1 / sqrt(nrm2[rhs])
template <typename R> hipError_t scale_rsqrt(c_t<R> *v, size_t n, int nrhs, const double *nrm2, hipStream_t st);
// out = b - out
template <typename R> hipError_t resid_from(c_t<R> *out, const c_t<R> *b, size_t n, int nrhs, hipStream_t st);

// ---- pack.hip (site-major coarse vectors)
template <typename T>
hipError_t pack_aos(const Geom &g, const double2 *canon, c_t<T> *internal, int ncomp, int nvec, hipStream_t st);
template <typename T>
hipError_t unpack_aos(const Geom &g, const c_t<T> *internal, double2 *canon, int ncomp, int nvec, hipStream_t st);
// ---- maps (pack.hip)
hipError_t export_maps_k(const Geom &g, const Geom &gc, int32_t *f2c, int32_t *f2l, int32_t *face, int32_t *cnbr,
                         hipStream_t st);

// ---------------------------------------------------------------- buffers
template <typename T> struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  int alloc(size_t count) {
    if (p && n >= count) return MG_OK;
    release();
    if (count == 0) return MG_OK;
    hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      set_error(hip_error_string(e, "hipMalloc"));
      return e == hipErrorOutOfMemory ? MG_ENOMEM : MG_EHIP;
    }
    n = count;
    return MG_OK;
  }
  operator T *() const { return p; }
};

template <typename R> struct PrecBufs;
template <> struct PrecBufs<double> {
  static DevBuf<double2> &pick(DevBuf<double2> &a, DevBuf<float2> &) { return a; }
};
template <> struct PrecBufs<float> {
  static DevBuf<float2> &pick(DevBuf<double2> &, DevBuf<float2> &b) { return b; }
};

struct Level {
  Geom g;     // this level's lattice; tile = aggregate shape to the next level
  int n = 0;  // complex components per site (12 on the fine level)
  int nv = 0; // null vectors defining the next level (0 on the coarsest)
  DevBuf<double2> U64;  DevBuf<float2> U32;   // fine links [36][V]
  DevBuf<double2> L64;  DevBuf<float2> L32;   // coarse stencil [V][9][n][n]
  DevBuf<double2> P64;  DevBuf<float2> P32;   // prolongator to next level
  DevBuf<double2> NV;                         // relaxed candidates before QR
  size_t vsize() const { return (size_t)g.V * n; }  // complex entries per vector
};

template <typename R> struct Work {
  // per level: x, r, q (smoother / cycle), rin (cycle input)
  DevBuf<c_t<R>> x[MG_MAX_LEVELS], r[MG_MAX_LEVELS], q[MG_MAX_LEVELS], rin[MG_MAX_LEVELS];
  // coarsest CGNR
  DevBuf<c_t<R>> ce, cr, cz, cp, cw;
  int nrhs = 0;
};

struct EventTimer {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  ~EventTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  hipEvent_t next() {
    if (used == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
  double total_ms() {  // pairs (start, stop); call after synchronisation
    double t = 0.0;
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) t += ms;
    }
    return t;
  }
  int launches() const { return (int)(used / 2); }
  void reset() { used = 0; }
};

}  // namespace mg

struct mg_ctx {
  mg_lattice_t lat{};
  mg_params_t p{};
  double mass = 0.0;
  int nlev = 0;
  mg::Level lev[MG_MAX_LEVELS];
  mg_prec_t prec = MG_F64;
  int timing = 0;
  // scalars and partials
  mg::DevBuf<double> part, part2, dsc, cg;
  mg::DevBuf<double2> csc;
  mg::DevBuf<int> done, it;
  int *h_done = nullptr;   // pinned host mirrors
  double *h_rr = nullptr;
  int *h_it = nullptr;
  mg::Work<double> w64;
  mg::Work<float> w32;
  // outer solver (FP64, fine level)
  mg::DevBuf<double2> gx, gr, gb, gZ, gW, gtmp;
  mg::DevBuf<int> skip;
  int gcr_rhs = 0;
  // statistics
  long n_fine = 0, n_coarse = 0, n_cgnr = 0, n_vcyc = 0;
  mg::EventTimer tm_dslash, tm_coarse;
  double t_setup = 0.0;
};
