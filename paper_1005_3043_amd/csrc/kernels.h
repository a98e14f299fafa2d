// Host-side launchers of the HIP kernels (one translation unit per kernel
// family).  Every launcher enqueues on `st` and returns the launch status.
#pragma once

#include "common.h"

namespace mg {

// ---- pack.hip: canonical complex128 [nvec][sites lex][ncomp] <-> internal
//      tile-interleaved fine fields (fidx), nvec fields of ncomp * Vpad entries.
template <typename T>
hipError_t pack_field(const Geom &g, const double2 *canon, c_t<T> *internal, int ncomp, int nvec,
                      hipStream_t st);
template <typename T>
hipError_t unpack_field(const Geom &g, const c_t<T> *internal, double2 *canon, int ncomp, int nvec,
                        hipStream_t st);
// canonical gauge field U[4][lex site][3][3] -> internal 36-component field
template <typename T> hipError_t pack_gauge(const Geom &g, const double2 *canon, c_t<T> *internal, hipStream_t st);

// ---- dslash.hip: fine Wilson operator on internal spinors (12 components).
// nl = 9: full links [36 components]; nl = 6: first two rows [24 components].
enum DslashMode { DS_PLAIN = 0, DS_RESID = 1, DS_MR = 2, DS_MRQ = 3 };
// out = diag*in - 1/2 hop(in)              (DS_PLAIN)
// out = b - (diag*in - 1/2 hop(in))        (DS_RESID)
// out = D in; partials[slot] = (<out,in>, ||out||^2)  (DS_MR, 3 doubles per slot,
//   dslash_partials(g, nrhs) slots per right-hand side)
// MR step by the q recursion (DS_MRQ, in = q_k, which is D r_k, TI = TO):
//   out = q_{k+1} = q_k - a D q_k, rout = r_{k+1} = rprev - a q_k with
//   a = alpha[rhs] (complex), partials as DS_MR of (q_{k+1}, r_{k+1});
//   R = float and TI = TO only (hipErrorInvalidValue otherwise).
template <typename TO> struct MrqArgs {
  const TO *rprev = nullptr;
  TO *rout = nullptr;
  const double2 *alpha = nullptr;
};
// R = arithmetic precision of vectors and accumulation, S = link storage
// (double2, float2 or chalf), TI / TO = storage of the input / output (and
// b) spinors: c_t<R>, or h16 (binary16 with a per-site scale, 13 slots per
// site) with R = float.  Instantiated: (double, double2, double2, double2),
// (float, float2, float2, float2), (float, chalf, float2, float2),
// (float, chalf, h16, h16), (float, chalf, float2, h16).
template <typename T> struct same_t { using type = T; };  // keeps b out of template argument deduction
template <typename R, typename S, typename TI = c_t<R>, typename TO = c_t<R>>
hipError_t dslash(const Geom &g, const S *U, int nl, const TI *in, TO *out, const typename same_t<TO>::type *b,
                  double diag, int nrhs, DslashMode mode, double *partials, hipStream_t st,
                  MrqArgs<typename same_t<TO>::type> mq = {});
// out = D in (DS_PLAIN) in FP64 arithmetic on FP32-stored input spinors
hipError_t dslash_in32(const Geom &g, const double2 *U, int nl, const float2 *in, double2 *out, double diag,
                       int nrhs, hipStream_t st);
// Uc = first two rows of every link of U (full FP64 links) in storage type S;
// blockmax[blk] = max |row2 - conj(row0 x row1)| (dslash_blocks(g) entries).
template <typename S>
hipError_t compress_links(const Geom &g, const double2 *U, S *Uc, double *blockmax, hipStream_t st);
int dslash_blocks(const Geom &g);  // 256-site workgroups of the single-RHS stencil
// number of DS_MR partial slots per right-hand side for a launch of nrhs
int dslash_partials(const Geom &g, int nrhs);

// ---- blas.hip
template <typename R> hipError_t zero(c_t<R> *x, size_t n, hipStream_t st);
template <typename R> hipError_t copy(c_t<R> *y, const c_t<R> *x, size_t n, hipStream_t st);
template <typename Rd, typename Rs>
hipError_t convert(c_t<Rd> *y, const c_t<Rs> *x, size_t n, hipStream_t st);
// operator storage: y[i] = x[i] rounded to storage type S (nearest even)
// x[i] = v + 0 i
template <typename R> hipError_t fill_const(c_t<R> *x, size_t n, R v, hipStream_t st);
template <typename S> hipError_t store_convert(S *y, const double2 *x, size_t n, hipStream_t st);
// diagonal shift X += delta I of a coarse stencil's slot-0 blocks
hipError_t shift_diag(double2 *L, uint32_t V, int n, double delta, hipStream_t st);
// Fine-level spinor fields (Vpad sites, nrhs of them back to back) between
// complex storage (12 entries per site, Cs / Cd = double2 or float2) and
// binary16 with a per-site scale (h16, 13 slots per site); copy_h16 copies
// h16 fields.
template <typename Cs> hipError_t to_h16(h16 *y, const Cs *x, uint32_t Vpad, int nrhs, hipStream_t st);
template <typename Cd> hipError_t from_h16(Cd *y, const h16 *x, uint32_t Vpad, int nrhs, hipStream_t st);
hipError_t copy_h16(h16 *y, const h16 *x, uint32_t Vpad, int nrhs, hipStream_t st);

}  // namespace mg

namespace mg {

// ---- coarse.hip: 9-point coarse stencil on site-major coarse vectors.
constexpr int COARSE_NMAX = 64;
int coarse_threads(int n, uint32_t V);
// workgroups per coarse site; partial-sum producers of the coarse stencil
// write V * coarse_split(n, V) entries (times pw) per right-hand side
int coarse_split(int n, uint32_t V);
// Optional CGNR convergence prologue of the coarse stencil: every workgroup
// sums the np_r residual partials of its right-hand side, reads the number of
// completed iterations it_in[rhs], tests ||r||^2 <= tol^2 ||b||^2 (cg scalars
// [3] = ||b||^2, [4] = tol^2) or it_in + 1 >= maxit, and returns when
// converged; workgroup 0 writes it_out[rhs] = it_in[rhs] + 1 and done[rhs].
// it_in and it_out are distinct slots (alternating by iteration parity) so
// no workgroup reads a value written by the same launch.
// With fused = 1 (the fused CGNR step below) the test runs before the p
// update of iteration it_in and checks the residual after it_in updates:
// nothing is tested at it_in = 0, a converged right-hand side records it_in
// iterations, otherwise it_out = it_in + 1; iterations stop at maxit.
struct CgCheck {
  const double *part_r = nullptr;
  int np_r = 0;
  const double *cg = nullptr;
  int *done = nullptr;
  const int *it_in = nullptr;
  int *it_out = nullptr;
  int maxit = 0;
  int fused = 0;
};
// Fused CGNR vector updates of the per-RHS coarse stencil: the stencil's
// input is formed while staging, in = a + sgn c b with the coefficient c =
// (sum num) / (sum den) over np partials per right-hand side, and the
// workgroup of site s also stores that combination at s:
//   kind 1 (w = A p):       p_new = z + beta p_old, beta = 0 when it0 = 0;
//   kind 2 (z = A^dag r):   r_new = r_old - alpha w, e += alpha p_new at s,
//                           ||r_new||^2 per workgroup into part_own; den <= 0
//                           marks the right-hand side done.
struct CgFuse {
  int kind = 0;
  const void *a = nullptr, *b = nullptr;
  void *own = nullptr;
  void *e = nullptr;
  const void *p = nullptr;
  const double *num = nullptr, *den = nullptr;
  int np = 0;
  double *part_own = nullptr;
  int *done_w = nullptr;
  const int *it0 = nullptr;
};
// Whole coarsest-level CGNR of one right-hand side in one cooperative
// launch (FP32 arithmetic): the state the chunked fused iteration starts from
// (e = 0, r[0] = b, p[1] = 0, z = A^dag b with its partials in pz[0], cg from
// cg2_init), the same two phases per iteration with a grid barrier between
// them, and on exit it[0] = it[1] = iterations, done[0] = 1.  bar (zero on
// entry, CGP_BAR_WORDS words) counts barrier arrivals; *fail is set when a
// barrier wait gave up.
// Returns an error without launching when the shape does not suit the
// kernel, and the cooperative launch's error when the grid cannot be
// co-resident; the caller then takes the chunked path.
constexpr int CGP_BAR_WORDS = 64 * 64;  // barrier counters: 64, one per 256-byte line
struct CgPersist {
  float2 *e = nullptr, *z = nullptr, *w = nullptr;
  float2 *p[2] = {nullptr, nullptr}, *r[2] = {nullptr, nullptr};
  double *pz[2] = {nullptr, nullptr}, *pw = nullptr, *pr = nullptr;
  const double *cg = nullptr;
  int *it = nullptr, *done = nullptr;
  int maxit = 0;
  unsigned *bar = nullptr;
  int *fail = nullptr;
  unsigned spin = 1u << 20;  // barrier polls before a wait gives up
};
template <typename S>
hipError_t cgnr_persistent(const Geom &g, int n, const S *L, const CgPersist &a, hipStream_t st);
// Reduction outputs and options of the coarse stencil.
//  part/pw: when part != nullptr each workgroup writes pw doubles at
//    part[(rhs * nwg + wg) * pw] (nwg = workgroups per right-hand side = V):
//    pw = 1: ||out||^2;  pw = 3: <out, in>, ||out||^2 (in = centre input).
//  done: a right-hand side with done[rhs] != 0 is skipped (may be nullptr).
//  chk: CGNR convergence prologue (see CgCheck).
//  variant: 0 = one workgroup per (site, right-hand side), FP vector FMA;
//    KS = 1, 2, 4 = one workgroup per site for all right-hand sides, a
//    complex GEMM on FP32 matrix cores with the K dimension split over KS
//    wavefront groups (FP32 arithmetic only); 8 + KS = the same GEMM reading
//    the row-major operator copy `lt` four columns per access (n % 4 == 0).
struct CoarseArgs {
  double *part = nullptr;
  int pw = 1;
  const int *done = nullptr;
  const CgCheck *chk = nullptr;
  const CgFuse *fuse = nullptr;  // per-RHS kernel (variant 0) only
  int variant = 0;
  const void *lt = nullptr;  // row-major operator copy (variants 8 + KS)
};
// Row-major copy of a coarse operator (Lt[site][row][9n] from the
// column-major FP64 stencil), for the matrix-core variants 8 + KS.
template <typename S> hipError_t transpose_convert(S *Lt, const double2 *L, uint32_t V, int n, hipStream_t st);
// out = D_c in (dagger: sigma3 D_c sigma3) for nrhs right-hand sides
// (site-major vectors [nrhs][V][n]).
template <typename R, typename S>
hipError_t coarse_apply_k(const Geom &g, int n, const S *L, const c_t<R> *in, c_t<R> *out, int nrhs, int dagger,
                          const CoarseArgs &a, hipStream_t st);
// Whether the matrix-core variant can run this shape (LDS and thread limits).
bool coarse_mma_ok(int n, int nrhs, int ks);

// ---- transfer.hip
// Fine level: P = nv null-vector fields in the fine layout [nv][12 * Vpad].
// g = geometry of the finer level (tile = aggregate), gc = geometry of the
// coarser level (its own site-blocked order).
// S = storage type of P (double2, float2 or chalf); vectors in c_t<R>; the
// fine vectors of the restriction may also be h16 (R = float, S = chalf).
template <typename R, typename S, typename TF = c_t<R>>
hipError_t restrict_fine(const Geom &g, const Geom &gc, int nv, const S *P, const TF *fine, c_t<R> *coarse,
                         int nrhs, hipStream_t st);
// fine (+)= P coarse  (accumulate != 0: add into fine)
template <typename R, typename S>
hipError_t prolong_fine(const Geom &g, const Geom &gc, int nv, const S *P, const c_t<R> *coarse, c_t<R> *fine,
                        int nrhs, int accumulate, hipStream_t st);
// Many right-hand sides on the FP32 matrix cores (transfer_mma.hip):
// one workgroup per aggregate for all nrhs <= 16; requires |B| % 4 == 0.
bool transfer_mma_ok(const Geom &g, int nv, int nrhs);
// TF = float2, or h16 with S = chalf
// The residuals r_0 .. r_{n-1} of an MR run by the q recursion (n <= MRQ_MAX).
constexpr int MRQ_MAX = 8;
template <typename TR> struct MrqList {
  const TR *r[MRQ_MAX];
};
// With q given, the restriction takes r = fine - a q per right-hand side
// (a = alpha[rhs]): the last residual of such a run formed on the fly.
template <typename S, typename TF>
hipError_t restrict_fine_mma(const Geom &g, const Geom &gc, int nv, const S *P, const TF *fine, float2 *coarse,
                             int nrhs, hipStream_t st, const TF *q = nullptr, const double2 *alpha = nullptr);
// With rs given (steps > 0), fine = P coarse + sum_k a_k r_k (a_k of
// right-hand side i at alpha[k MG_MAX_RHS + i]): the run's solution added to
// the prolongated correction without a pass of its own; accumulate ignored.
template <typename S, typename TR = float2>
hipError_t prolong_fine_mma(const Geom &g, const Geom &gc, int nv, const S *P, const float2 *coarse, float2 *fine,
                            int nrhs, int accumulate, hipStream_t st, const MrqList<TR> *rs = nullptr,
                            int steps = 0, const double2 *alpha = nullptr);
// Coarse level l -> l+1: P = nv vectors in coarse AoS layout [nv][V][n];
// requires block volume * n <= 2048.
template <typename R, typename S>
hipError_t restrict_coarse(const Geom &g, const Geom &gc, int n, int nv, const S *P, const c_t<R> *fine,
                           c_t<R> *coarse, int nrhs, hipStream_t st);
template <typename R, typename S>
hipError_t prolong_coarse(const Geom &g, const Geom &gc, int n, int nv, const S *P, const c_t<R> *coarse,
                          c_t<R> *fine, int nrhs, int accumulate, hipStream_t st);

// ---- ortho.hip: in-place block orthonormalisation (MGS applied twice) per
// (aggregate, chirality); rank-deficiency sets *flag = 1.
hipError_t ortho_fine(const Geom &g, int nv, double2 *V, int *flag, hipStream_t st);
hipError_t ortho_coarse(const Geom &g, int n, int nv, double2 *V, int *flag, hipStream_t st);

// ---- galerkin.hip: D_c = P^dag D P into L[Vc][9][n][n] (column-major blocks).
hipError_t galerkin_fine(const Geom &g, const Geom &gc, double mass, const double2 *U, int nv, const double2 *P,
                         double2 *Lc, hipStream_t st);
hipError_t galerkin_coarse(const Geom &g, const Geom &gc, int n, const double2 *L1, int nv, const double2 *P,
                           double2 *Lc, hipStream_t st);

}  // namespace mg
