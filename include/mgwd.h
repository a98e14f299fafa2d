/* mgwd.h - C ABI of the MI355X adaptive multigrid solver for the lattice
 * Wilson-Dirac system D(U) psi = b (Babich et al., "Adaptive multigrid
 * algorithm for the lattice Wilson-Dirac operator", 2010).
 *
 * Plain C: every argument is a plain pointer (host or device, as stated per
 * function), a size or a small struct.  No exception crosses this boundary;
 * every entry point returns an int status (MG_OK = 0, MG_NOT_CONVERGED = 1,
 * negative = error) and mg_last_error() gives a message for the calling
 * thread.
 *
 * Canonical layouts at the boundary (complex128 = two doubles re, im; C
 * order; x fastest; mu = 0,1,2,3 = x,y,z,t):
 *   gauge field   U[4][Lt][Lz][Ly][Lx][3][3]   row = colour at x,
 *                                               column = colour at x + mu
 *   fine spinor   psi[nrhs][Lt][Lz][Ly][Lx][4][3]
 *   coarse vector v[nrhs][Lct][Lcz][Lcy][Lcx][2*Nv]  component chi*Nv + k,
 *                 chi = coarse chirality (sigma_3 = diag(+1_Nv, -1_Nv))
 * Gamma matrices (chiral basis): gamma_k = [[0, -i s_k], [i s_k, 0]],
 * gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1); chirality 0 =
 * spins {0, 1}.  Time boundary antiperiodic when t_antiperiodic != 0: a hop
 * across it carries a factor -1.
 *
 * Ownership: the caller owns every buffer it passes; device buffers need to
 * stay valid only for the duration of the call (asynchronous calls: until
 * the work enqueued on the stream has run).  mg_setup copies U into its own
 * layout.  The context owns its prolongators, coarse operators, work
 * vectors and graphs; mg_destroy frees them.
 * Streams: work is enqueued on the hipStream_t argument (NULL = default
 * stream).  wilson_apply, mg_restrict, mg_prolong and coarse_apply are
 * asynchronous; mg_setup and mg_solve return after completion because their
 * convergence decisions are taken on the host.  mg_solve runs on a stream
 * owned by the context, ordered after prior work on the argument stream.
 */
#ifndef MGWD_H
#define MGWD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_OK 0
#define MG_NOT_CONVERGED 1
#define MG_EINVAL (-1)     /* null pointer, argument out of range          */
#define MG_ESHAPE (-2)     /* block does not divide L, Nv too large, level  */
#define MG_EHIP (-3)       /* HIP runtime error                             */
#define MG_ENOMEM (-4)     /* device allocation failed                      */
#define MG_ENONFINITE (-5) /* NaN/Inf in an input or a reduction            */
#define MG_ENOTSUP (-6)    /* precision or feature combination not built    */
#define MG_ERANK (-7)      /* rank-deficient aggregate in block QR          */

#define MG_MAX_LEVELS 3
#define MG_MAX_RHS 16
#define MG_KERNEL_CLASSES 10 /* kernel timing classes of mg_info_t */

typedef struct {
  int L[4];            /* Lx, Ly, Lz, Lt                                    */
  int t_antiperiodic;  /* 1: antiperiodic time boundary, 0: periodic       */
} mg_lattice_t;

typedef enum { MG_F64 = 0, MG_F32 = 1, MG_F16 = 2, MG_BF16 = 3 } mg_prec_t;

typedef struct mg_ctx mg_ctx_t;

typedef struct {
  int n_levels;                      /* 2 or 3 (fine + coarse levels)        */
  int block[MG_MAX_LEVELS - 1][4];   /* aggregate shape level l -> l+1       */
  int nv[MG_MAX_LEVELS - 1];         /* null vectors defining level l -> l+1 */
  int setup_rounds;                  /* relaxation rounds per vector (5)     */
  int setup_mr_steps;                /* MR steps per round (4)               */
  double omega;                      /* MR under-relaxation (0.9)            */
  int pre, post;                     /* MR smoothing steps (4, 4)            */
  double coarse_tol;                 /* coarsest CGNR relative tol (1e-3)    */
  int coarse_maxiter;                /* coarsest CGNR cap (1000)             */
  int gcr_restart;                   /* flexible GCR restart length (8)      */
  int max_iter;                      /* outer iteration cap                  */
  mg_prec_t precond_prec;            /* MG_F64, MG_F32 or MG_F16 (FP16-stored
                                        links, P and D_c; inside the cycle
                                        the fine level's input, smoother
                                        residual and stencil output stored
                                        as binary16 with per-site scales;
                                        FP32 arithmetic)                     */
  int max_rhs;                       /* largest nrhs passed to mg_solve      */
  int use_graph;                     /* 1: replay the coarsest-level CGNR
                                        iterations from captured hipGraphs  */
  /* Setup start vectors, DEVICE complex128, required:
   *   init_vectors[0]: [nv[0]][Lt][Lz][Ly][Lx][4][3]
   *   init_vectors[1]: [nv[1]][Lct][Lcz][Lcy][Lcx][2*nv[0]] (3 levels)    */
  const void *init_vectors[MG_MAX_LEVELS - 1];
  /* Setup stage two ("Numerical Results"), on every level l below the
   * coarsest, after its relaxation: the prototypes are refined in groups of
   * refine_group (0 = off; at most 16 and below nv[0]; a level with at most
   * refine_group prototypes is left as relaxed).  Each group is taken out, a
   * truncated two-level method from level l is built from the other
   * prototypes (block orthonormalisation and Galerkin operator as in stage
   * one, FP64), refine_iters iterations
   * (at most gcr_restart) of the MG-preconditioned flexible GCR are run on
   * A_l v = 0 from each prototype of the group (GCR in FP64, its cycles in
   * precond_prec), and the normalised iterates replace the group before
   * the next one is taken.                                                */
  int refine_group;
  int refine_iters;
  /* Relaxation and cycle ("Formulating an algorithm", "Numerical Results").
   * smoother MG_SMOOTH_MR: pre and post steps of MR (GMRES(1)) with
   * under-relaxation omega per step (on the fine level of the FP32 and
   * FP16 classes, smoothings of 2 to 8 steps run by the q recursion: the
   * same iterates in exact arithmetic, one fused update pass per
   * smoothing; the device memory for it, max(pre, post) fine vectors per
   * right-hand side, is taken at the first solve or cycle in that class;
   * the FP32 setup relaxation takes it the same way with setup_mr_steps).
   * MG_SMOOTH_GMRES: one GMRES(pre)
   * cycle before and one GMRES(post) cycle after the coarse correction
   * (pre, post <= 8; 0 = none), each from zero and scaled by omega; the
   * paper's V(0,4) is pre = 0, post = 4.  cycles: cycles of level l+1 per
   * correction of level l whenever l+1 is not the coarsest level (1 or 0:
   * V-cycle; 2: the paper's W-cycle, the second cycle applied to the
   * residual the first leaves and added; at most 4).                      */
  int smoother;
  int cycles;
  /* Arithmetic of setup stage one (the relaxation of the start vectors):
   * MG_F64 (0, default), or MG_F32 (FP32 copies of the level's operator and
   * vectors, batches of at most 12 vectors; the relaxed vectors are widened
   * to FP64 before the block orthonormalisation, which, like the Galerkin
   * construction, is always FP64).                                        */
  mg_prec_t setup_prec;
  /* Learned start vectors (the network of the ptc_* calls below, an
   * extension): learned_setup = 1 takes the level-0 start vectors from the
   * network instead of from init_vectors[0] directly: init_vectors[0] then
   * holds ONE noise field eta ([Lt][Lz][Ly][Lx][4][3], DEVICE complex128),
   * the starts are Y = net(eta) with the DEVICE complex64 weights
   * ptc_weights[0] = W1 [ptc_hidden][1][9][4][4] and ptc_weights[1] = W2
   * [nv[0]][ptc_hidden][9][4][4] (n_out = nv[0]) on the links U, and the
   * setup_rounds relaxation rounds start from Y (0 rounds: Y itself).
   * The links and the aggregate shape are those of mg_setup (block[0]).
   * learned_setup = 0 (default): plain start vectors.  Errors: MG_EINVAL
   * (missing weights, ptc_hidden outside [1, 64]).                        */
  int learned_setup;
  int ptc_hidden;
  const void *ptc_weights[2];
  /* Storage of the prolongator the FP32 preconditioner's transfers read
   * (restriction and prolongation on every level): MG_F16 takes the
   * binary16 copy of P (FP32 arithmetic, FP32 vectors), halving the bytes
   * of P that every cycle streams; any other value (MG_F64 = 0, the
   * default, or MG_F32): each preconditioner class reads P in its own
   * storage (FP32 in the FP32 class, binary16 in the FP16 class, FP64 in
   * the FP64 class).  Errors: MG_ENOTSUP for values outside MG_F64..MG_F16. */
  mg_prec_t transfer_prec;
} mg_params_t;

#define MG_SMOOTH_MR 0
#define MG_SMOOTH_GMRES 1

typedef struct {
  int iters[MG_MAX_RHS];        /* outer FGCR iterations per RHS             */
  double rel_resid[MG_MAX_RHS]; /* final true ||b - D x|| / ||b|| per RHS    */
  int n_fine_dslash;            /* fine D applications (per RHS summed)      */
  int n_coarse_apply;           /* coarse stencil applications, all levels   */
  int n_coarse_dispatch;        /* coarse stencil applications dispatched,
                                   including those that returned at once
                                   because their RHS had converged (those
                                   inside a whole-solve CGNR launch are
                                   applications, not dispatches)          */
  int n_cgnr_iters;             /* coarsest CGNR iterations, summed          */
  int n_vcycles;                /* preconditioner applications               */
  double t_setup_s, t_solve_s;  /* wall time of the last setup / solve       */
  /* Kernel timing (filled when mg_set_timing(ctx, 1) is on): summed device
   * time in ms, launch count and sites x right-hand sides processed, per
   * kernel class 2 p + k: p = 0 FP64, 1 FP32, 2 FP16-stored operators with
   * FP32 arithmetic; k = 0 fine stencil, 1 coarse stencil (all coarse
   * levels).  Launch counts include dispatches that returned early because
   * their right-hand side had converged.  Classes 6 and 7: the whole-solve
   * coarsest CGNR launches (mg_set_cgnr_persistent) with the FP32 and the
   * FP16-stored operator, one launch per coarsest solve, sites = coarse
   * sites x stencil applications inside the launches.  Classes 8 and 9:
   * the fine stencil launches of the MR steps taken by the q recursion
   * (each also reads the previous residual and writes the next one) in
   * the FP32 and FP16 classes; class 2 and 4 count the other fine-stencil
   * launches of those classes.                                            */
  double kernel_ms[MG_KERNEL_CLASSES];
  int kernel_launches[MG_KERNEL_CLASSES];
  double kernel_sites[MG_KERNEL_CLASSES];
  int n_cgnr_fallbacks;         /* whole-solve CGNR launches whose barrier
                                   wait gave up, so that the coarsest solve
                                   was done again by the chunks            */
} mg_info_t;

/* Fine Wilson operator out = D(U) in (Eq. 2) on nrhs canonical spinors.
 * U, in, out: DEVICE complex128 canonical layouts (in and out may not
 * alias).  prec selects the arithmetic of the stencil: MG_F64, MG_F32, or
 * MG_F16 (links and spinors stored in binary16, the spinors of each site
 * divided by the largest |Re|, |Im| of its 12 components, which is kept in
 * FP32; FP32 arithmetic; the input is rounded to FP32, then to binary16, so
 * every stored entry carries a relative rounding of up to 2^-11).  Inputs
 * and outputs stay complex128.  Stateless: converts to the library's
 * internal site-blocked SoA layout and back on every call.               */
int wilson_apply(const mg_lattice_t *lat, const void *U, double mass,
                 const void *in, void *out, int nrhs, mg_prec_t prec,
                 hipStream_t stream);

/* wilson_apply for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the same operator, arguments, layouts and kernels as wilson_apply, with
 * the internal layouts (links and nrhs input and output spinors, (36 +
 * 24 nrhs) x Vpad complex entries of the arithmetic precision, Vpad = V
 * rounded up to 64) in a library-owned device array of MG_NOALLOC_BYTES
 * that each GPU holds from its first call until the process ends.  This
 * call allocates nothing.  Lattices and nrhs that need more scratch than
 * MG_NOALLOC_BYTES are refused with MG_ENOMEM before any work is enqueued
 * (FP64 and one right-hand side: up to 131 072 sites, e.g. 16^3 x 32).
 * Every call on one GPU uses the same array: calls that overlap on a GPU
 * (from several streams or threads) race, and the caller must order them.
 * Asynchronous on `stream`.                                               */
#define MG_NOALLOC_BYTES (128u << 20)
int wilson_apply_noalloc(const mg_lattice_t *lat, const void *U, double mass,
                         const void *in, void *out, int nrhs, mg_prec_t prec,
                         hipStream_t stream);

/* Adaptive MG setup (paper: "Adaptive Multigrid", "Formulating an
 * algorithm", setup stage one in "Numerical Results"): relax the start
 * vectors on D x = 0 (setup_rounds x setup_mr_steps MR steps each,
 * normalising after each round), QR them per (aggregate, chirality) with a
 * positive real R diagonal to form P (P^dag P = I, Eq. 4), and build
 * D_c = P^dag D P as a 9-point stencil of 2Nv x 2Nv blocks; repeated on
 * D_c for 3 levels.  U: DEVICE complex128 canonical.  *ctx receives a new
 * context.  Returns MG_ESHAPE if a block does not divide the lattice or
 * Nv > 6 * block volume (fine) / Nv * block volume (coarse), MG_ERANK if an
 * aggregate is rank deficient.  Synchronous.                            */
int mg_setup(const mg_lattice_t *lat, const void *U, double mass,
             const mg_params_t *params, mg_ctx_t **ctx, hipStream_t stream);

/* Choose the preconditioner precision for later solves (MG_F64, MG_F32,
 * MG_F16); lower-precision copies of U, P and D_c are made on first use.  */
int mg_set_precond_prec(mg_ctx_t *ctx, mg_prec_t prec);

/* Reuse a setup at another mass ("Numerical Results": a setup made near the
 * critical mass serves heavier masses).  D(m') = D(m) + (m' - m), and P has
 * orthonormal columns per block (Eq. 4), so every Galerkin operator shifts
 * exactly: X(m') = X(m) + (m' - m) I, Y unchanged.  The null vectors and P
 * are kept.  Synchronous.  MG_EINVAL for a NULL ctx or non-finite mass.    */
int mg_set_mass(mg_ctx_t *ctx, double mass);

/* Turn per-kernel device timing on (1) or off (0) for later solves.       */
int mg_set_timing(mg_ctx_t *ctx, int on);

/* Restriction r_c = P^dag r from level `level` to level+1 (R = P^dag,
 * Eq. 8 with chirality kept: P^dag gamma_5 = sigma_3 P^dag).
 * level 0: fine canonical spinors in, coarse canonical vectors out;
 * level 1: coarse level-1 vectors in, level-2 vectors out.  DEVICE
 * complex128 buffers, nrhs vectors each.  Asynchronous.                  */
int mg_restrict(mg_ctx_t *ctx, int level, const void *fine, void *coarse,
                int nrhs, hipStream_t stream);

/* Prolongation e = P e_c from level+1 to level (layouts as mg_restrict).   */
int mg_prolong(mg_ctx_t *ctx, int level, const void *coarse, void *fine,
               int nrhs, hipStream_t stream);

/* Coarse operator of level `level` (1 or 2) applied to nrhs canonical
 * coarse vectors: out(x_c) = X(x_c) in(x_c) + sum_mu [Y_+mu(x_c)
 * in(x_c+mu) + Y_-mu(x_c) in(x_c-mu)], periodic on the coarse lattice.
 * dagger != 0 applies D_c^dag = sigma_3 D_c sigma_3.  FP64.  Async.       */
int coarse_apply(mg_ctx_t *ctx, int level, const void *in, void *out,
                 int nrhs, int dagger, hipStream_t stream);

/* The operator of level `level` as the preconditioner applies it: level 0
 * is the fine Wilson operator of Eq. 2 with the context's links (two-row
 * compressed when they are SU(3)), level >= 1 the Galerkin coarse operator
 * D_c = P^dag D P ("Formulating an algorithm").  prec selects the stored
 * copies: MG_F64; MG_F32 (FP32 operators and arithmetic); MG_F16 (operators
 * stored as binary16 complex, FP32 arithmetic), the mixed-precision scheme
 * of "Numerical Results".  in/out are canonical DEVICE complex128 arrays of
 * the level (layouts as mg_restrict), converted to and from the working
 * precision on the device.  Builds the low-precision copies on first use.
 * Async.  Errors: MG_EINVAL (NULL/aliased buffers, nrhs < 1), MG_ESHAPE
 * (level out of range), MG_ENOTSUP (prec).                                  */
int mg_apply_op(mg_ctx_t *ctx, int level, mg_prec_t prec, const void *in,
                void *out, int nrhs, hipStream_t stream);

/* One application of the multigrid preconditioner z = K(r) ("Formulating an
 * algorithm"; the cycle of Eq. 3 with smoothing): MR pre-smoothing (pre
 * steps), restriction, the next level's cycle (CGNR to coarse_tol on the
 * coarsest level), prolongation added to the smoothed iterate, MR
 * post-smoothing on the new residual (post steps), on every level below the
 * coarsest.  prec as mg_apply_op; with MG_F16 the cycle keeps the fine
 * level's input, smoother residual and stencil output in binary16 with
 * per-site scales (its correction x in FP32).  in/out: DEVICE complex128 canonical fine
 * spinors [nrhs][Lt][Lz][Ly][Lx][4][3], not aliased; 1 <= nrhs <= 16.
 * cgnr_iters (host, may be NULL) receives the coarsest-level CGNR
 * iterations of this call summed over the right-hand sides.  Ordered on
 * `stream`; synchronous.  Errors: MG_EINVAL, MG_ENOTSUP (prec).            */
int mg_vcycle(mg_ctx_t *ctx, mg_prec_t prec, const void *in, void *out,
              int nrhs, int *cgnr_iters, hipStream_t stream);

/* Restriction (direction 0: out = P^dag in, level -> level+1) or
 * prolongation (direction 1: out = P in, level+1 -> level, overwritten)
 * with the stored P of precision prec (Eq. 4, Eq. 8): MG_F64, MG_F32, or
 * MG_F16 (binary16-stored P, FP32 arithmetic), the copies the
 * preconditioner uses.  in/out: canonical DEVICE complex128 arrays of the
 * two levels (layouts as mg_restrict), not aliased.  Builds the
 * low-precision copies on first use.  Async.  Errors: MG_EINVAL, MG_ESHAPE
 * (level), MG_ENOTSUP (prec).                                              */
int mg_transfer(mg_ctx_t *ctx, int level, mg_prec_t prec, int direction,
                const void *in, void *out, int nrhs, hipStream_t stream);

/* Fine-level transfer kernel choice for FP32 arithmetic (MG_F32, MG_F16)
 * and 2..16 right-hand sides: vector kernels serving four right-hand sides
 * per workgroup (variant 0) or one complex GEMM per aggregate for all of
 * them on the FP32 matrix cores (variant 1; needs an aggregate volume
 * divisible by 4).  By default each direction is timed once per (lattice,
 * aggregate, Nv, precision, nrhs) on first use and the faster kept for the
 * process; mg_set_transfer_variant forces one (-1 restores tuning; variant
 * 1 falls back to 0 where it cannot run).  mg_transfer_variant reports the
 * choice for restriction and prolongation (-1: not tuned yet) and, when us
 * is not NULL, the tuning times in microseconds per application in us[4]
 * (restriction variant 0, 1, prolongation variant 0, 1; 0 if not timed).   */
int mg_set_transfer_variant(mg_ctx_t *ctx, int variant);
int mg_transfer_variant(mg_ctx_t *ctx, mg_prec_t prec, int nrhs,
                        int *restrict_variant, int *prolong_variant,
                        double *us);

/* Coarse-stencil kernel choice.  For FP32 arithmetic (MG_F32, MG_F16) the
 * coarse operator D_c ("Formulating an algorithm") can be applied either by
 * one workgroup per (site, right-hand side) (variant 0) or, for a batch of
 * right-hand sides, as one complex GEMM per coarse site on the FP32 matrix
 * cores with the K range split over 1, 2 or 4 wavefront groups (variants
 * 1, 2, 4), reading either the stencil itself or a row-major copy of it
 * made on first use (variants 9, 10, 12; four columns per access; needs
 * n = 2 Nv divisible by 4).  By default the library times the candidates once per
 * (operator size, coarse volume, nrhs, precision) on first use and keeps the
 * fastest for the process.  mg_set_coarse_variant forces a variant
 * (-1 restores tuning; a variant that cannot run a shape falls back to 0).
 * mg_coarse_variant reports the tuned choice (-1: not tuned yet) and its
 * time in microseconds (0 when forced or FP64).  MG_EINVAL on bad
 * arguments, MG_ESHAPE on a bad level, MG_ENOTSUP on prec.                */
int mg_set_coarse_variant(mg_ctx_t *ctx, int variant);
int mg_coarse_variant(mg_ctx_t *ctx, int level, mg_prec_t prec, int nrhs,
                      int *variant, double *us);

/* Coarsest-level CGNR of a single right-hand side (paper, "Numerical
 * Results": CG on the normal equations to 10^-3 on the coarsest grid) in
 * the FP32 and FP16-storage preconditioners: on (default), all iterations
 * run in one cooperative launch that keeps each coarse site's operator rows
 * in registers and joins its two stencil phases per iteration with grid
 * barriers; off, they run as chunks of captured per-iteration launches.
 * Both forms do the same arithmetic in the same order (same iterates, same
 * iteration counts).  Where the device cannot hold the whole coarse grid at
 * once (or the operator rows do not fit), the chunks run regardless.  A
 * barrier wait gives up after 2^20 polls (on >= 2: after `on` polls, to
 * exercise this path); the launch then leaves, and that coarsest solve is
 * done again from its right-hand side by the chunks, which that (level,
 * precision) keeps using until this function is called again.
 * MG_EINVAL on a NULL context or on < 0.                                   */
int mg_set_cgnr_persistent(mg_ctx_t *ctx, int on);

/* Outer flexible GCR ("Formulating an algorithm"): mode 1 (default) forms
 * the step length a_j = <w^_j, r> / ||w^_j||^2 before the orthogonalisation
 * of w_j, with ||w^_j||^2 = ||w_j||^2 - sum_i |<w^_i, w_j>|^2 / ||w^_i||^2
 * (exact for the classical Gram-Schmidt step), and updates the residual in
 * the same pass over the vectors; where that difference has cancelled below
 * 1e-4 ||w_j||^2 the pass only orthogonalises and a second pass updates the
 * residual with a_j from the measured ||w^_j||^2.  Mode 0: orthogonalisation
 * and residual update as two passes always; mode 2: the fused pass with
 * every step taking the second pass (exercises that path).  The iterates
 * agree to rounding.  MG_EINVAL on a NULL context or a mode outside 0..2. */
int mg_set_gcr_fusion(mg_ctx_t *ctx, int mode);

/* The coarsest-level solve of the cycle ("Numerical Results": CG on the
 * normal equations D_c^dag D_c e = D_c^dag b to ||b - D_c e|| <=
 * coarse_tol ||b||, at most coarse_maxiter iterations, D_c^dag = sigma_3 D_c
 * sigma_3) with the stored coarsest operator of precision prec (MG_F64,
 * MG_F32, MG_F16 as mg_apply_op), exactly as the V-cycle runs it: one
 * whole-solve launch for one right-hand side in FP32 arithmetic (see
 * mg_set_cgnr_persistent), chunks of captured iterations otherwise.
 * b, x: DEVICE complex128 canonical vectors of the coarsest level
 * [nrhs][Lct][Lcz][Lcy][Lcx][n], not aliased; 1 <= nrhs <= 16.  iters (HOST,
 * may be NULL) receives the CGNR iterations of each right-hand side (nrhs
 * ints).  Ordered on `stream`; synchronous.  Errors: MG_EINVAL (NULL or
 * aliased buffers, nrhs), MG_ENOTSUP (prec).                              */
int mg_coarse_solve(mg_ctx_t *ctx, mg_prec_t prec, const void *b, void *x, int nrhs, int *iters,
                    hipStream_t stream);

/* Solve D x = b for nrhs canonical spinors (DEVICE complex128) with
 * flexible GCR(gcr_restart) preconditioned by one MG V-cycle (MR pre/post
 * smoothing, CGNR on the coarsest level), to ||b - D x|| <= tol ||b|| per
 * RHS, restarting with the true residual.  x is overwritten (zero start).
 * info (HOST, may be NULL) receives iteration counts and timings.
 * Returns MG_NOT_CONVERGED when max_iter is reached (x = last iterate).
 * Synchronous.                                                           */
int mg_solve(mg_ctx_t *ctx, const void *b, void *x, int nrhs, double tol,
             mg_info_t *info, hipStream_t stream);

/* Device time of `reps` back-to-back fine-stencil launches on the
 * context's internal layouts (nrhs vectors, precision prec), measured with
 * HIP events on `stream`.  avg_ms (HOST) receives the mean per launch.    */
int mg_time_dslash(mg_ctx_t *ctx, mg_prec_t prec, int nrhs, int reps,
                   double *avg_ms, hipStream_t stream);

/* The same for the fine-stencil form of the MR step by the q recursion
 * (q' = q - a D q and r' = r - a q written, with the MR partial sums of
 * (q', r')) that the V-cycle of the FP32 and FP16 classes launches, with
 * a = 0.1 for every right-hand side.  prec: MG_F32 or MG_F16 (MG_ENOTSUP
 * otherwise).                                                             */
int mg_time_dslash_mrq(mg_ctx_t *ctx, mg_prec_t prec, int nrhs, int reps,
                       double *avg_ms, hipStream_t stream);

/* Device time of `reps` coarse-stencil launches of level `level`.        */
int mg_time_coarse(mg_ctx_t *ctx, int level, mg_prec_t prec, int nrhs,
                   int reps, double *avg_ms, hipStream_t stream);

/* Frees a context.  Its device buffers go back to the library's cache of
 * device allocations (per device, at most 60 % of the device's memory,
 * oldest blocks freed first), from which later contexts with the same
 * buffer sizes take them instead of allocating again: allocating the
 * buffers of a 32^3 x 64 context anew takes seconds.                      */
int mg_destroy(mg_ctx_t *ctx);

/* Frees every cached device allocation of the current device (see
 * mg_destroy); *released (may be NULL) receives the number of bytes.
 * Returns MG_OK, or MG_EHIP if no device is current.                      */
int mg_release_cached_memory(size_t *released);

/* Message describing the last error on the calling thread ("" if none).   */
const char *mg_last_error(void);

/* ---- Exports for parity checks (HOST output buffers) ------------------- */
/* Aggregate maps of level `level` (int32, canonical lexicographic order of
 * the level's sites): f2c[V] coarse site, f2l[V] index within the block
 * (o_x + b_x (o_y + b_y (o_z + b_z o_t))), cnbr[Vc][8] coarse neighbour in
 * slot 2 mu + dir (dir 0 = +mu, 1 = -mu), face[V] bit 2 mu + dir set when
 * that hop leaves the block.  Any pointer may be NULL.                    */
int mg_export_maps(mg_ctx_t *ctx, int level, int32_t *f2c, int32_t *f2l,
                   int32_t *cnbr, int32_t *face);

/* Prolongator of level `level` as complex128 [Vc][2][rows][Nv] with row =
 * l * h + j (h = 6 on the fine level: j = 3 s' + c for spin 2 chi + s';
 * h = Nv(level) on coarse levels).                                       */
int mg_export_P(mg_ctx_t *ctx, int level, void *P_host);

/* Coarse operator of level `level` (1 or 2): X[Vc][n][n] and Y[8][Vc][n][n]
 * complex128, coarse sites lexicographic, [row][col].                     */
int mg_export_coarse_op(mg_ctx_t *ctx, int level, void *X_host, void *Y_host);

/* Relaxed null vectors of level `level` before orthonormalisation, in the
 * canonical layout of that level (complex128, nv vectors).               */
int mg_export_nullvecs(mg_ctx_t *ctx, int level, void *V_host);

/* Geometry of level `level`: L (4 ints) and component count per site.   */
int mg_level_info(mg_ctx_t *ctx, int level, int *L_out, int *ncomp_out);

/* ---- Learned proposal of near-null vectors ---------------------------
 * A two-layer gauge-equivariant network of parallel-transport convolutions
 * maps a noise spinor eta and the links U to n_out candidate vectors that
 * replace the random start vectors of the setup relaxation ("Adaptive
 * Multigrid"; the network itself is an extension the paper does not
 * have).  Hops T_0 = 1 and, for k = 1 + 2 mu + dir, the parallel transport
 * of the hopping term of Eq. 2 (dir 0 from x + mu with U_mu(x), dir 1 from
 * x - mu with U_mu(x - mu)^dag, sign -1 across the antiperiodic time
 * boundary).  Layer: out_a = sum_{b,k} W_abk T_k in_b with W_abk a complex
 * 4x4 spin matrix; psi1 = layer(W1, eta) (1 -> n_hidden), Y = layer(W2,
 * psi1) (n_hidden -> n_out); no nonlinearity.
 *
 * Weights: DEVICE complex64, W1 [n_hidden][1][9][4][4], W2
 * [n_out][n_hidden][9][4][4] (row-major, [s][t] spin matrices).  Fields:
 * DEVICE complex128 canonical spinors.  FP32 arithmetic.
 *
 * ptc_create: block = aggregate shape of the subspace-fit loss (must divide
 *   the lattice).  Owns its buffers until ptc_destroy.
 * ptc_set_links: packs U (canonical complex128 links) for later calls.
 * ptc_set_targets: the nv target vectors of the loss (the null vectors of
 *   the plain setup), canonical complex128 [nv][sites][4][3].
 * ptc_forward: Y [n_out][sites][4][3] from eta [sites][4][3].
 * ptc_loss_grad: forward pass, loss L = sum over chirality-split
 *   aggregates of the least-squares residual of the targets in the span of
 *   Y, divided by sum ||V||^2 (host double), and the gradients
 *   gW = dL/dRe W + i dL/dIm W (device complex64, layouts of W).  Synchronous.
 *   MG_ERANK if Y is rank deficient on a block.
 * ptc_adam: one Adam step on n complex parameters (real and imaginary parts
 *   separately): m (complex64) and v (2n floats, interleaved re/im) are the
 *   moment buffers (zero before step 1), step counts from 1.  Async.
 * Errors: MG_EINVAL (NULL, ranges), MG_ESHAPE (block does not divide L).  */
typedef struct ptc_ctx ptc_ctx_t;
int ptc_create(const mg_lattice_t *lat, const int block[4], int n_hidden,
               int n_out, ptc_ctx_t **ctx);
int ptc_set_links(ptc_ctx_t *ctx, const void *U, hipStream_t stream);
int ptc_set_targets(ptc_ctx_t *ctx, const void *V, int nv, hipStream_t stream);
int ptc_forward(ptc_ctx_t *ctx, const void *W1, const void *W2, const void *eta,
                void *Y, hipStream_t stream);
int ptc_loss_grad(ptc_ctx_t *ctx, const void *W1, const void *W2,
                  const void *eta, double *loss, void *gW1, void *gW2,
                  hipStream_t stream);
int ptc_adam(void *W, const void *g, void *m, void *v, size_t n, int step,
             double lr, double b1, double b2, double eps, hipStream_t stream);
int ptc_destroy(ptc_ctx_t *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MGWD_H */
