// Multigrid context and the launchers of the solver's streaming kernels.
#pragma once

#include <vector>

#include "kernels.h"

namespace mg {

constexpr int RED_BLOCKS = 1024;  // fixed grid of generic reductions
constexpr int CG_NS = 8;          // CGNR scalars per right-hand side
constexpr int GCR_CHUNK = 8;      // FGCR directions orthogonalised against per pass
// double2 scalars per right-hand side of the deferred-update FGCR (gcr.hip)
// with restart length m: g_ij (m x m), a, e, c (m each), f, and a flag (the
// fused step's fallback, see gcr2_step_residual)
__host__ __device__ constexpr size_t gcr_scalars_per_rhs(int m) { return (size_t)m * m + 3 * (size_t)m + 2; }

// ---- solver_kernels.hip
// x = (first ? 0 : x) + alpha r_in and, when upd_r, r_out = r_in - alpha q
// (r_out may be r_in), with alpha = omega <q,r>/<q,q> from the stencil's np
// partials per right-hand side
template <typename R>
hipError_t mr_update(c_t<R> *x, c_t<R> *r_out, const c_t<R> *r_in, const c_t<R> *q, size_t n, int nrhs,
                     const double *part, int np, double omega, double2 *alpha, int first, int upd_r,
                     hipStream_t st);
// the same on the fine level g with r and q in binary16 with a per-site
// scale (13 slots per site) and x in FP32
hipError_t mr_update_h(float2 *x, h16 *r_out, const h16 *r_in, const h16 *q, const Geom &g, int nrhs,
                       const double *part, int np, double omega, double2 *alpha, int first, int upd_r,
                       hipStream_t st);
// alpha[rhs] = omega <q,r>/<q,q> from the np MR partials per right-hand side
hipError_t fin_mr(const double *part, int np, int nrhs, double omega, double2 *alpha, hipStream_t st);
// MR by the q recursion on the fine level g (FP32 x; TR = float2 or h16
// residuals): after steps n of the stencil in DS_MR then DS_MRQ mode, which
// produced r_0 .. r_{n-1} (list r) and q_{n-1} (q) with a_k at
// alpha[k * MG_MAX_RHS + rhs],  x = (first ? 0 : x) + xs sum_k a_k r_k  and,
// when upd_r, r_out = r_{n-1} - a_{n-1} q_{n-1} (r_out may be r_0); xs = 1,
// or -1 to subtract the MR solution from x.
template <typename TR>
hipError_t mrq_combine(float2 *x, TR *r_out, const MrqList<TR> &rs, const TR *q, const Geom &g, int steps, int nrhs,
                       const double2 *alpha, int first, int upd_r, float xs, hipStream_t st);
template <typename R> hipError_t norm2(const c_t<R> *a, size_t n, int nrhs, double *part, double *out, hipStream_t st);
// launches the per-block partials of ||a||^2 and returns their count per RHS
template <typename R> int norm2_partials(const c_t<R> *a, size_t n, int nrhs, double *part, hipStream_t st);
template <typename R>
hipError_t dot(const c_t<R> *a, const c_t<R> *b, size_t n, int nrhs, double *part, double2 *out, hipStream_t st);
hipError_t finish_sum1(const double *part, int np, int nrhs, double *out, hipStream_t st);
hipError_t gcr_sub2(double2 *y, const double2 *x, double2 *v, const double2 *u, size_t n, int nrhs,
                    const double2 *sc, const int *skip, hipStream_t st);
hipError_t gcr_scale2(double2 *y, double2 *v, size_t n, int nrhs, const double *nrm2, const int *skip,
                      hipStream_t st);
// w_j -= sum_i <w_i, w_j> w_i and z_j -= (same) z_i over the ni <= 8 earlier
// directions W + i vs, Z + i vs (classical Gram-Schmidt, coefficients in
// sc[rhs * 8 + i]); nrm2[rhs] = ||w_j||^2 afterwards.
hipError_t gcr_cgs(const double2 *W, const double2 *Z, size_t vs, int ni, double2 *wj, double2 *zj, size_t n,
                   int nrhs, double2 *sc, const int *skip, double *part, double *nrm2, hipStream_t st);
hipError_t gcr_update(double2 *x, const double2 *z, double2 *r, const double2 *w, size_t n, int nrhs,
                      const double2 *sc, const int *skip, double *part, double *rr, hipStream_t st);
// ---- gcr.hip: flexible GCR with the solution update deferred to the end of
// each restart cycle.  Wh holds w_0 .. w_{m-1} (stride vs); w_j = D z_j on
// entry to gcr2_step, which orthogonalises it against w^_0 .. w^_{j-1} in
// place and derives a_j from the residual r_in; gcr2_residual moves r along
// w^_j (rr[rhs] = ||r||^2; r32 or r16, if not null, receives r in FP32 or in
// binary16 with per-site scales, n = 12 Vpad);
// gcr2_solution adds the cycle's update Z T^{-1} a to x, over the cnt[rhs]
// steps each right-hand side took (kmax = steps of the cycle).  gs: double2
// [MG_MAX_RHS][gcr_scalars_per_rhs(m)], nu: double [MG_MAX_RHS][m].
hipError_t gcr2_step(double2 *Wh, size_t vs, int j, int m, const double2 *r_in, size_t n, int nrhs,
                     double2 *gs, double *nu, int *cnt, const int *skip, double *part, hipStream_t st);
hipError_t gcr2_residual(double2 *r, const double2 *Wh, size_t vs, int j, int m, size_t n, int nrhs,
                         const double2 *gs, const int *skip, double *part, double *rr, float2 *r32, h16 *r16,
                         hipStream_t st);
// gcr2_step followed by gcr2_residual, with the orthogonalisation of w_j and
// the residual update in one pass over the vectors for 1 <= j <= GCR_CHUNK:
// a_j is taken before the pass from ||w^_j||^2 = ||w_j||^2 - sum_i
// |<w^_i, w_j>|^2 / ||w^_i||^2 (exact for the classical Gram-Schmidt step),
// unless that difference has cancelled to below 1e-4 ||w_j||^2; then the
// pass only orthogonalises and a second one updates r with a_j from the
// measured ||w^_j||^2 (per right-hand side).
// mode: 1 fused as described, 0 two passes always, 2 the fused pass with
// every right-hand side taking the second pass.
hipError_t gcr2_step_residual(double2 *Wh, size_t vs, int j, int m, double2 *r, size_t n, int nrhs, double2 *gs,
                              double *nu, int *cnt, const int *skip, double *part, double *rr, float2 *r32,
                              h16 *r16, int mode, hipStream_t st);
template <typename TZ>
hipError_t gcr2_solution(double2 *x, const TZ *Z, size_t vs, int kmax, int m, size_t n, int nrhs, double2 *gs,
                         double *nu, const int *cnt, hipStream_t st);
// Fused CGNR steps (no finisher kernels): scalars are re-derived from the
// per-block partials by every consuming workgroup in a fixed order.
hipError_t cg2_init(const double *part_b, int npb, int nrhs, double *cg, int *done, int *it, double tol,
                    hipStream_t st);
// returns the number of residual partials written per RHS
template <typename R>
int cg2_update(c_t<R> *e, const c_t<R> *p, c_t<R> *r, const c_t<R> *w, size_t n, int nrhs, const double *part_w,
               const double *part_z, int npc, int *done, double *part_r, hipStream_t st);
template <typename R>
hipError_t cg2_p(c_t<R> *p, const c_t<R> *z, size_t n, int nrhs, const double *part_znew, const double *part_zold,
                 int npc, const int *done, hipStream_t st);
// v -= x
template <typename R> hipError_t sub_inplace(c_t<R> *v, const c_t<R> *x, size_t n, int nrhs, hipStream_t st);
// v *= 1 / sqrt(nrm2[rhs])
template <typename R> hipError_t scale_rsqrt(c_t<R> *v, size_t n, int nrhs, const double *nrm2, hipStream_t st);
// out = b - out
template <typename R> hipError_t resid_from(c_t<R> *out, const c_t<R> *b, size_t n, int nrhs, hipStream_t st);

// ---- gmres.hip (GMRES(k) relaxation, k <= GM_KMAX)
constexpr int GM_KMAX = 8;
// v0 = b / ||b|| from nrm2 = ||b||^2; beta = ||b||
template <typename R>
hipError_t gm_start(c_t<R> *v0, const c_t<R> *b, size_t n, int nrhs, const double *nrm2, double *beta,
                    hipStream_t st);
// with V[j+1] = A v_j on entry: column j of H and v_{j+1} (basis stride vs)
template <typename R>
hipError_t gm_arnoldi_col(c_t<R> *V, size_t vs, int j, size_t n, int nrhs, double2 *H, double *part,
                          hipStream_t st);
hipError_t gm_lsq(const double2 *H, const double *beta, int k, int nrhs, double2 *y, hipStream_t st);
// x = (accumulate ? x : 0) + omega sum_{j<k} y_j v_j
template <typename R>
hipError_t gm_combine(c_t<R> *x, const c_t<R> *V, size_t vs, int k, size_t n, int nrhs, const double2 *y,
                      double omega, int accumulate, hipStream_t st);
// v += x
template <typename R> hipError_t add_inplace(c_t<R> *v, const c_t<R> *x, size_t n, int nrhs, hipStream_t st);

// ---- pack.hip (site-major coarse vectors)
template <typename T>
hipError_t pack_aos(const Geom &g, const double2 *canon, c_t<T> *internal, int ncomp, int nvec, hipStream_t st);
template <typename T>
hipError_t unpack_aos(const Geom &g, const c_t<T> *internal, double2 *canon, int ncomp, int nvec, hipStream_t st);
// ---- maps (pack.hip)
hipError_t export_maps_k(const Geom &g, const Geom &gc, int32_t *f2c, int32_t *f2l, int32_t *face, int32_t *cnbr,
                         hipStream_t st);

// ---------------------------------------------------------------- buffers
// Device allocations through the library's cache (pool.cpp): pool_alloc
// reuses a cached block of the same rounded size or calls hipMalloc;
// pool_free keeps the block for the next request (up to a per-device cap).
hipError_t pool_alloc(void **out, size_t bytes);
void pool_free(void *p, size_t bytes);

template <typename T> struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) pool_free(p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  // zero = false only for buffers whose every entry is written before it is
  // read (e.g. fine-level vectors of a lattice without padding sites, fully
  // overwritten by a kernel that covers every site).
  int alloc(size_t count, bool zero = true) {
    if (p && n >= count) return MG_OK;
    release();
    if (count == 0) return MG_OK;
    hipError_t e = pool_alloc((void **)&p, count * sizeof(T));
    // Zero-filled (padding entries stay zero), and the fill has completed
    // on return: the buffer is next used on streams that do not order
    // themselves after the default stream.
    if (e == hipSuccess && zero) e = hipMemsetAsync(p, 0, count * sizeof(T), nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
      if (p) pool_free(p, count * sizeof(T));
      p = nullptr;
      set_error(hip_error_string(e, "hipMalloc"));
      return e == hipErrorOutOfMemory ? MG_ENOMEM : MG_EHIP;
    }
    n = count;
    return MG_OK;
  }
  operator T *() const { return p; }
};

// Preconditioner precisions: R = arithmetic of vectors and accumulation,
// S = storage of the operators (links, prolongator, coarse stencil).
struct PF64 { using R = double; using S = double2; static constexpr int id = 0; };
struct PF32 { using R = float; using S = float2; static constexpr int id = 1; };
struct PF16 { using R = float; using S = chalf; static constexpr int id = 2; };
template <typename P> using vec_t = c_t<typename P::R>;
// Storage of the fine level's residual-type vectors inside a V-cycle (the
// cycle's input, the smoother's residual and the stencil's output q): the
// arithmetic type, except binary16 with a per-site scale in the FP16 class.
// The fine-level correction x is always vec_t.
template <typename P> struct FineRes { using T = vec_t<P>; };
template <> struct FineRes<PF16> { using T = h16; };
template <typename P> using fres_t = typename FineRes<P>::T;

struct Level {
  Geom g;            // this level's lattice; tile = aggregate shape to the next level
  bool fine = false; // fine level: tile-interleaved fields of Vpad sites
  int n = 0;         // complex components per site (12 on the fine level)
  int nv = 0;        // null vectors defining the next level (0 on the coarsest)
  int nl = 9;        // fine links stored with 9 (full) or 6 (two rows) entries
  DevBuf<double2> U64;   // fine links, full, FP64 [36 components]
  DevBuf<double2> U64c;  // fine links, two rows, FP64 [24 components] (nl = 6)
  DevBuf<float2> U32;    // fine links in FP32, nl entries per direction
  DevBuf<chalf> U16;     // fine links in FP16, nl entries per direction
  DevBuf<double2> L64;  DevBuf<float2> L32;  DevBuf<chalf> L16;  // coarse stencil [V][9][n][n]
  DevBuf<float2> L32t;  DevBuf<chalf> L16t;  // row-major copies [V][n][9n] (matrix-core variants 8 + KS)
  DevBuf<double2> P64;  DevBuf<float2> P32;  DevBuf<chalf> P16;  // prolongator to next level
  DevBuf<double2> NV;                         // relaxed candidates before QR
  // complex entries per vector
  size_t vsize() const { return (size_t)(fine ? g.Vpad : g.V) * n; }
  const double2 *links64() const { return nl == 6 ? U64c.p : U64.p; }
};

template <typename R> struct Work {
  // per level: x, r, q (smoother / cycle), rin (cycle input)
  DevBuf<c_t<R>> x[MG_MAX_LEVELS], r[MG_MAX_LEVELS], q[MG_MAX_LEVELS], rin[MG_MAX_LEVELS];
  // coarsest CGNR
  DevBuf<c_t<R>> ce, cr, cz, cp, cw, cp2, cr2;  // cp2, cr2: second p, r of the fused CGNR
  // GMRES relaxation basis per level; W-cycle residual and correction per level
  DevBuf<c_t<R>> gv[MG_MAX_LEVELS], w2r[MG_MAX_LEVELS], w2x[MG_MAX_LEVELS];
  // fine-level r, q and cycle input of the FP16 class (binary16, 13 slots
  // per site; allocated in the FP32 work set only)
  DevBuf<h16> hr, hq, hrin;
  int nrhs = 0;
  // fine-level MR by the q recursion (FP32 work set): second q and the
  // residuals r_1 .. r_{n-1}, FP32 ([0]) and binary16 ([1]) storage, for
  // mrq_nrhs[i] right-hand sides and mrq_steps[i] steps
  DevBuf<float2> q2, rk[MRQ_MAX - 1];
  DevBuf<h16> hq2, hrk[MRQ_MAX - 1];
  int mrq_nrhs[2] = {0, 0}, mrq_steps[2] = {0, 0};
};

// Device-side timing of one kernel class: (start, stop) event pairs recorded
// around launches; harvest() adds the elapsed times of the recorded pairs to
// the accumulators (after the work has completed).  A timer owned by a
// captured graph keeps its events (they are re-recorded by every replay).
struct EventTimer {
  std::vector<hipEvent_t> ev;
  std::vector<double> pair_sites;  // sites x right-hand sides of each pair
  std::vector<int> pair_launches;  // kernel launches covered by each pair
  size_t used = 0;
  double ms = 0.0, sites = 0.0;    // accumulated
  long launches = 0;
  EventTimer() = default;
  EventTimer(const EventTimer &) = delete;
  EventTimer &operator=(const EventTimer &) = delete;
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
  // accumulate the recorded pairs into dst (default: this timer)
  void harvest(EventTimer *dst = nullptr, bool keep = false) {
    if (!dst) dst = this;
    for (size_t i = 0; i + 1 < used; i += 2) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) continue;
      dst->ms += t;
      dst->launches += i / 2 < pair_launches.size() ? pair_launches[i / 2] : 1;
      if (i / 2 < pair_sites.size()) dst->sites += pair_sites[i / 2];
    }
    if (!keep) {
      used = 0;
      pair_sites.clear();
      pair_launches.clear();
    }
    (void)hipGetLastError();  // a failed elapsed-time query must not latch into later launches
  }
  void reset() {
    used = 0;
    pair_sites.clear();
    pair_launches.clear();
    ms = sites = 0.0;
    launches = 0;
  }
};

// A captured chunk of CGNR iterations for one (level, precision, nrhs).
struct ChunkGraph {
  int level = -1, prec = -1, nrhs = 0, variant = 0, fused = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~ChunkGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// One part of a V-cycle captured for replay: part 0 = smoothing, residual
// and restriction on every level down to the coarsest, part 1 = prolongation,
// residual and smoothing on every level back up (the coarsest solve between
// them stays host-driven).  Keyed by precision, right-hand sides and the
// cycle's input and output buffers.  state 0: the key was seen once and ran
// eagerly (which tuned its kernels and made the operator copies it needs);
// 1: captured; -1: capture failed, runs eagerly.  The host-side counts of
// one execution are kept so that replays add them.
struct VGraph {
  int prec = -1, nrhs = 0, part = 0;
  const void *rin = nullptr, *x = nullptr;
  int state = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  long dfine = 0, dcoarse = 0, ddisp = 0;
  ~VGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};
constexpr int VGRAPH_MAX = 48;

constexpr int CG_FUSE_MAXV = 1024;  // fused CGNR up to this many coarse sites (<= RED_BLOCKS)
constexpr int CG_CHUNK = 8;  // CGNR iterations per chunk (even: parity slots repeat)

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
  mg::DevBuf<double> cgp;  // CGNR partials: w, z[2], r, b
  // coarse-stencil variant per (level, precision class, nrhs): -1 = not yet
  // tuned; 0 = per right-hand side; 1, 2, 4 = matrix-core GEMM K split
  int cvar[MG_MAX_LEVELS][3][MG_MAX_RHS + 1];
  float cvar_us[MG_MAX_LEVELS][3][MG_MAX_RHS + 1];
  int cvar_force = -1;  // >= 0: use this variant wherever it can run
  // fine-level transfer kernel per (direction, precision, nrhs): 0 = vector
  // kernels, 1 = matrix-core GEMM; -1 = not tuned yet
  int tvar[2][3][MG_MAX_RHS + 1];
  float tvar_us[2][3][MG_MAX_RHS + 1][2];  // tuning times of both variants
  int tvar_force = -1;
  hipStream_t sti = nullptr;                  // library-owned stream of mg_solve
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_chunk[2] = {nullptr, nullptr};
  int use_graph = 1;
  mg::ChunkGraph *graphs[16] = {};            // captured CGNR chunks
  std::vector<mg::VGraph *> vgraphs;          // captured V-cycle parts
  int vgraph_on = 0;                          // set by the outer solver around its cycles
  mg::DevBuf<double2> csc;
  mg::DevBuf<int> done, it;
  // whole-solve cooperative CGNR (one RHS): barrier counter, give-up flag,
  // on/off, and per (level, precision class) whether the launch was refused
  mg::DevBuf<unsigned> cgp_bar;
  mg::DevBuf<int> cgp_fail;
  int cg_persist = 1;
  int gcr_fuse = 1;  // mg_set_gcr_fusion
  unsigned cgp_spin = 1u << 20;  // barrier polls before a wait gives up
  int cgp_off[MG_MAX_LEVELS][3] = {};
  int *h_done = nullptr;   // pinned host mirrors
  double *h_rr = nullptr;
  int *h_it = nullptr;
  mg::Work<double> w64;
  mg::Work<float> w32;
  // outer solver (FP64, fine level)
  mg::DevBuf<double2> gx, gr, gb, gZ, gW, gtmp;
  mg::DevBuf<float2> gZf, gr32;  // FP32 preconditioned vectors and preconditioner input (FP32/FP16 precond)
  mg::DevBuf<mg::h16> gr16;      // preconditioner input of the FP16 class
  mg::DevBuf<double2> gsc;       // deferred-update FGCR scalars
  mg::DevBuf<double> gnu;
  mg::DevBuf<int> gcnt;
  // GMRES relaxation scalars: Hessenberg matrices, least-squares
  // coefficients, ||b|| and column partials
  mg::DevBuf<double2> gmH, gmy;
  mg::DevBuf<double> gmb, gmp;
  mg::DevBuf<int> skip;
  int gcr_rhs = 0;
  // statistics
  long n_fine = 0, n_coarse = 0, n_coarse_disp = 0, n_cgnr = 0, n_vcyc = 0, n_cg_fallback = 0;
  // (fine, coarse) x (FP64, FP32, FP16 storage), whole-solve CGNR (FP32, FP16),
  // fine stencil of the MR q recursion (FP32, FP16)
  mg::EventTimer tm[MG_KERNEL_CLASSES];
  double t_setup = 0.0;
};
