// C ABI: multigrid context entry points (argument validation, layout
// conversion at the boundary, dispatch to the orchestration in mg.cpp).
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include <type_traits>

#include "mg_internal.h"

using namespace mg;

namespace {

int hip_rc(hipError_t e, const char *what) {
  if (e == hipSuccess) return MG_OK;
  set_error(hip_error_string(e, what));
  return MG_EHIP;
}
#define HIPK(expr) MG_TRY(hip_rc((expr), #expr))

int bad(int rc, const char *msg) {
  set_error(msg);
  return rc;
}

int check_params(const mg_lattice_t *lat, const mg_params_t *p) {
  if (p->n_levels < 2 || p->n_levels > MG_MAX_LEVELS) return bad(MG_EINVAL, "n_levels must be 2 or 3");
  int L[4] = {lat->L[0], lat->L[1], lat->L[2], lat->L[3]};
  int n = 12;
  for (int l = 0; l < p->n_levels - 1; ++l) {
    long vb = 1;
    for (int mu = 0; mu < 4; ++mu) {
      const int b = p->block[l][mu];
      if (b < 1 || L[mu] % b != 0) return bad(MG_ESHAPE, "aggregate shape does not divide the lattice");
      vb *= b;
      L[mu] /= b;
    }
    const int nv = p->nv[l];
    if (nv < 1 || 2 * nv > COARSE_NMAX) return bad(MG_ESHAPE, "Nv must be in [1, 32]");
    if (l == 0) {
      if (vb > 256) return bad(MG_ESHAPE, "fine aggregates larger than 256 sites are not supported");
      if (nv > 6 * vb) return bad(MG_ESHAPE, "Nv exceeds 6 x aggregate volume");
    } else {
      if (vb * n > 2048) return bad(MG_ESHAPE, "coarse aggregate volume x components exceeds 2048");
      if (nv > (n / 2) * vb) return bad(MG_ESHAPE, "Nv exceeds (n/2) x aggregate volume");
    }
    if (!p->init_vectors[l]) return bad(MG_EINVAL, "init_vectors missing for a level");
    n = 2 * nv;
  }
  if (p->setup_rounds < 0 || p->setup_mr_steps < 0 || p->pre < 0 || p->post < 0)
    return bad(MG_EINVAL, "negative step count");
  if (!std::isfinite(p->omega) || !(p->coarse_tol > 0) || p->coarse_maxiter < 1)
    return bad(MG_EINVAL, "bad omega / coarse tolerance / coarse iteration cap");
  if (p->gcr_restart < 1 || p->gcr_restart > 64 || p->max_iter < 1) return bad(MG_EINVAL, "bad GCR parameters");
  if (p->max_rhs < 1 || p->max_rhs > MG_MAX_RHS) return bad(MG_EINVAL, "max_rhs out of range");
  if (p->refine_group < 0 || p->refine_group > MG_MAX_RHS || (p->refine_group > 0 && p->refine_group >= p->nv[0]))
    return bad(MG_EINVAL, "refine_group must be 0 (off) or in [1, min(16, nv[0] - 1)]");
  if (p->refine_group > 0 && (p->refine_iters < 0 || p->refine_iters > p->gcr_restart))
    return bad(MG_EINVAL, "refine_iters must be in [0, gcr_restart]");
  if (p->smoother != MG_SMOOTH_MR && p->smoother != MG_SMOOTH_GMRES)
    return bad(MG_EINVAL, "smoother must be MG_SMOOTH_MR or MG_SMOOTH_GMRES");
  if (p->smoother == MG_SMOOTH_GMRES && (p->pre > GM_KMAX || p->post > GM_KMAX))
    return bad(MG_EINVAL, "GMRES relaxation: pre and post must be at most 8");
  if (p->cycles < 0 || p->cycles > 4) return bad(MG_EINVAL, "cycles must be in [0, 4]");
  if (p->precond_prec != MG_F64 && p->precond_prec != MG_F32 && p->precond_prec != MG_F16)
    return bad(MG_ENOTSUP, "precond_prec must be MG_F64, MG_F32 or MG_F16");
  if (p->setup_prec != MG_F64 && p->setup_prec != MG_F32)
    return bad(MG_ENOTSUP, "setup_prec must be MG_F64 or MG_F32");
  if (p->transfer_prec != MG_F64 && p->transfer_prec != MG_F32 && p->transfer_prec != MG_F16)
    return bad(MG_ENOTSUP, "transfer_prec must be MG_F64, MG_F32 or MG_F16");
  if (p->learned_setup != 0 && p->learned_setup != 1) return bad(MG_EINVAL, "learned_setup must be 0 or 1");
  if (p->learned_setup) {
    if (!p->ptc_weights[0] || !p->ptc_weights[1]) return bad(MG_EINVAL, "learned_setup: ptc_weights missing");
    if (p->ptc_hidden < 1 || p->ptc_hidden > 64) return bad(MG_EINVAL, "learned_setup: ptc_hidden must be in [1, 64]");
  }
  return MG_OK;
}

int check_ctx_level(mg_ctx_t *ctx, int level, int lo, int hi) {
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (level < lo || level > hi) return bad(MG_ESHAPE, "level out of range");
  return MG_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <typename T> struct AsyncBuf {
  T *p = nullptr;
  hipStream_t st;
  explicit AsyncBuf(hipStream_t s) : st(s) {}
  ~AsyncBuf() {
    if (p) (void)hipFreeAsync(p, st);
  }
  hipError_t alloc(size_t n) { return hipMallocAsync((void **)&p, n * sizeof(T), st); }
};

// canonical <-> internal for a vector of level l (FP64)
hipError_t pack_level(mg_ctx *c, int l, const void *canon, double2 *internal, int nvec, hipStream_t st) {
  const Level &L = c->lev[l];
  if (l == 0) return pack_field<double>(L.g, (const double2 *)canon, internal, 12, nvec, st);
  return pack_aos<double>(L.g, (const double2 *)canon, internal, L.n, nvec, st);
}
hipError_t unpack_level(mg_ctx *c, int l, const double2 *internal, void *canon, int nvec, hipStream_t st) {
  const Level &L = c->lev[l];
  if (l == 0) return unpack_field<double>(L.g, internal, (double2 *)canon, 12, nvec, st);
  return unpack_aos<double>(L.g, internal, (double2 *)canon, L.n, nvec, st);
}

}  // namespace

extern "C" int mg_setup(const mg_lattice_t *lat, const void *U, double mass, const mg_params_t *params,
                        mg_ctx_t **ctx, hipStream_t stream) {
  set_error("");
  MG_TRY(check_lattice(lat));
  if (!U || !params || !ctx) return bad(MG_EINVAL, "mg_setup: NULL argument");
  if (!std::isfinite(mass)) return bad(MG_ENONFINITE, "mg_setup: non-finite mass");
  MG_TRY(check_params(lat, params));
  mg_ctx *c = new (std::nothrow) mg_ctx();
  if (!c) return bad(MG_ENOMEM, "mg_setup: out of host memory");
  c->lat = *lat;
  c->p = *params;
  c->mass = mass;
  c->prec = params->precond_prec;
  c->use_graph = params->use_graph ? 1 : 0;
  std::memset(c->cvar, 0xff, sizeof(c->cvar));  // -1: not tuned
  std::memset(c->tvar, 0xff, sizeof(c->tvar));
  const double t0 = now_s();
  int rc = hip_rc(hipStreamCreateWithFlags(&c->sti, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  if (rc == MG_OK) rc = hip_rc(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming), "hipEventCreate");
  if (rc == MG_OK) rc = hip_rc(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming), "hipEventCreate");
  for (int i = 0; i < 2 && rc == MG_OK; ++i)
    rc = hip_rc(hipEventCreateWithFlags(&c->ev_chunk[i], hipEventDisableTiming), "hipEventCreate");
  // learned start vectors: the network's output replaces init_vectors[0]
  // for the relaxation (kept in Y until the setup has used it)
  AsyncBuf<double2> Y(stream);
  if (rc == MG_OK && params->learned_setup) {
    ptc_ctx_t *pc = nullptr;
    rc = ptc_create(lat, params->block[0], params->ptc_hidden, params->nv[0], &pc);
    if (rc == MG_OK) {
      uint64_t V = 1;
      for (int mu = 0; mu < 4; ++mu) V *= (uint64_t)lat->L[mu];
      rc = hip_rc(Y.alloc((size_t)12 * V * params->nv[0]), "hipMallocAsync");
      if (rc == MG_OK) rc = ptc_set_links(pc, U, stream);
      if (rc == MG_OK)
        rc = ptc_forward(pc, params->ptc_weights[0], params->ptc_weights[1], params->init_vectors[0], Y.p, stream);
      const int rd = ptc_destroy(pc);
      if (rc == MG_OK) rc = rd;
    }
    if (rc == MG_OK) c->p.init_vectors[0] = Y.p;
  }
  if (rc == MG_OK) rc = setup(c, U, stream);
  c->p.init_vectors[0] = params->init_vectors[0];
  if (rc == MG_OK) rc = ensure_prec(c, c->prec, stream);
  if (rc == MG_OK) rc = hip_rc(hipStreamSynchronize(stream), "mg_setup");
  if (rc != MG_OK) {
    mg_destroy(c);
    return rc;
  }
  c->t_setup = now_s() - t0;
  *ctx = c;
  return MG_OK;
}

extern "C" int mg_set_precond_prec(mg_ctx_t *ctx, mg_prec_t prec) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(ensure_prec(ctx, prec, nullptr));
  HIPK(hipStreamSynchronize(nullptr));
  ctx->prec = prec;
  return MG_OK;
}

extern "C" int mg_set_mass(mg_ctx_t *ctx, double mass) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (!std::isfinite(mass)) return bad(MG_EINVAL, "mg_set_mass: mass must be finite");
  const double delta = mass - ctx->mass;
  HIPK(hipStreamSynchronize(ctx->sti));
  for (int l = 1; l < ctx->nlev; ++l) {
    Level &L = ctx->lev[l];
    HIPK(shift_diag(L.L64, L.g.V, L.n, delta, nullptr));
    L.L32.release();  // low-precision copies are rebuilt from the shifted FP64 stencil
    L.L16.release();
    L.L32t.release();
    L.L16t.release();
  }
  clear_graphs(ctx);
  HIPK(hipStreamSynchronize(nullptr));
  ctx->mass = mass;
  if (ctx->prec != MG_F64) MG_TRY(ensure_prec(ctx, ctx->prec, nullptr));
  HIPK(hipStreamSynchronize(nullptr));
  return MG_OK;
}

extern "C" int mg_set_timing(mg_ctx_t *ctx, int on) {
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  ctx->timing = on ? 1 : 0;
  return MG_OK;
}

extern "C" int mg_set_cgnr_persistent(mg_ctx_t *ctx, int on) {
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (on < 0) return bad(MG_EINVAL, "mg_set_cgnr_persistent: on must be >= 0");
  ctx->cg_persist = on ? 1 : 0;
  ctx->cgp_spin = on >= 2 ? (unsigned)on : 1u << 20;
  for (auto &lv : ctx->cgp_off)
    for (int &o : lv) o = 0;
  return MG_OK;
}

extern "C" int mg_set_gcr_fusion(mg_ctx_t *ctx, int mode) {
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (mode < 0 || mode > 2) return bad(MG_EINVAL, "mg_set_gcr_fusion: mode must be 0, 1 or 2");
  ctx->gcr_fuse = mode;
  return MG_OK;
}

extern "C" int mg_set_coarse_variant(mg_ctx_t *ctx, int variant) {
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (variant != -1 && variant != 0 && variant != 1 && variant != 2 && variant != 4 && variant != 9 &&
      variant != 10 && variant != 12)
    return bad(MG_EINVAL, "mg_set_coarse_variant: variant must be -1, 0, 1, 2, 4, 9, 10 or 12");
  ctx->cvar_force = variant;
  clear_graphs(ctx);
  return MG_OK;
}

extern "C" int mg_coarse_variant(mg_ctx_t *ctx, int level, mg_prec_t prec, int nrhs, int *variant, double *us) {
  if (!ctx || !variant || !us) return bad(MG_EINVAL, "mg_coarse_variant: NULL argument");
  MG_TRY(check_ctx_level(ctx, level, 1, ctx->nlev - 1));
  if (nrhs < 1 || nrhs > MG_MAX_RHS) return bad(MG_EINVAL, "mg_coarse_variant: nrhs out of range");
  if (prec != MG_F64 && prec != MG_F32 && prec != MG_F16) return bad(MG_ENOTSUP, "mg_coarse_variant: prec");
  const int pi = prec == MG_F64 ? 0 : prec == MG_F32 ? 1 : 2;
  *variant = pi == 0 ? 0 : ctx->cvar[level][pi][nrhs];
  *us = pi == 0 ? 0.0 : (*variant >= 0 ? (double)ctx->cvar_us[level][pi][nrhs] : 0.0);
  return MG_OK;
}

extern "C" int mg_set_transfer_variant(mg_ctx_t *ctx, int variant) {
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (variant != -1 && variant != 0 && variant != 1)
    return bad(MG_EINVAL, "mg_set_transfer_variant: variant must be -1, 0 or 1");
  ctx->tvar_force = variant;
  clear_graphs(ctx);
  return MG_OK;
}

extern "C" int mg_transfer_variant(mg_ctx_t *ctx, mg_prec_t prec, int nrhs, int *restrict_variant,
                                   int *prolong_variant, double *us) {
  if (!ctx || !restrict_variant || !prolong_variant) return bad(MG_EINVAL, "mg_transfer_variant: NULL argument");
  if (nrhs < 1 || nrhs > MG_MAX_RHS) return bad(MG_EINVAL, "mg_transfer_variant: nrhs out of range");
  if (prec != MG_F64 && prec != MG_F32 && prec != MG_F16) return bad(MG_ENOTSUP, "mg_transfer_variant: prec");
  const int pi = prec == MG_F64 ? 0 : prec == MG_F32 ? 1 : 2;
  *restrict_variant = pi == 0 ? 0 : ctx->tvar[0][pi][nrhs];
  *prolong_variant = pi == 0 ? 0 : ctx->tvar[1][pi][nrhs];
  if (us) {
    for (int d = 0; d < 2; ++d)
      for (int v = 0; v < 2; ++v)
        us[2 * d + v] = (pi == 0 || ctx->tvar[d][pi][nrhs] < 0) ? 0.0 : (double)ctx->tvar_us[d][pi][nrhs][v];
  }
  return MG_OK;
}

extern "C" int mg_restrict(mg_ctx_t *ctx, int level, const void *fine, void *coarse, int nrhs, hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 2));
  if (!fine || !coarse || nrhs < 1) return bad(MG_EINVAL, "mg_restrict: bad buffers or nrhs");
  MG_TRY(ensure_scalars(ctx, part_need(ctx, 1)));
  AsyncBuf<double2> a(st), b(st);
  HIPK(a.alloc(ctx->lev[level].vsize() * nrhs));
  HIPK(b.alloc(ctx->lev[level + 1].vsize() * nrhs));
  HIPK(pack_level(ctx, level, fine, a.p, nrhs, st));
  MG_TRY(transfer_restrict<PF64>(ctx, level, a.p, b.p, nrhs, st));
  HIPK(unpack_level(ctx, level + 1, b.p, coarse, nrhs, st));
  return MG_OK;
}

extern "C" int mg_prolong(mg_ctx_t *ctx, int level, const void *coarse, void *fine, int nrhs, hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 2));
  if (!fine || !coarse || nrhs < 1) return bad(MG_EINVAL, "mg_prolong: bad buffers or nrhs");
  AsyncBuf<double2> a(st), b(st);
  HIPK(a.alloc(ctx->lev[level].vsize() * nrhs));
  HIPK(b.alloc(ctx->lev[level + 1].vsize() * nrhs));
  HIPK(pack_level(ctx, level + 1, coarse, b.p, nrhs, st));
  MG_TRY(transfer_prolong<PF64>(ctx, level, b.p, a.p, nrhs, 0, st));
  HIPK(unpack_level(ctx, level, a.p, fine, nrhs, st));
  return MG_OK;
}

extern "C" int coarse_apply(mg_ctx_t *ctx, int level, const void *in, void *out, int nrhs, int dagger,
                            hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(check_ctx_level(ctx, level, 1, ctx->nlev - 1));
  if (!in || !out || in == out || nrhs < 1) return bad(MG_EINVAL, "coarse_apply: bad buffers or nrhs");
  const Level &L = ctx->lev[level];
  AsyncBuf<double2> a(st), b(st);
  HIPK(a.alloc(L.vsize() * nrhs));
  HIPK(b.alloc(L.vsize() * nrhs));
  HIPK(pack_level(ctx, level, in, a.p, nrhs, st));
  HIPK((coarse_apply_k<double, double2>(L.g, L.n, L.L64, a.p, b.p, nrhs, dagger ? 1 : 0, CoarseArgs{}, st)));
  HIPK(unpack_level(ctx, level, b.p, out, nrhs, st));
  return MG_OK;
}

namespace {
template <typename P> int apply_op_t(mg_ctx *c, int level, const double2 *a, double2 *b, int nrhs, hipStream_t st) {
  using R = typename P::R;
  if constexpr (sizeof(R) == 8) {
    return apply_A<P>(c, level, a, b, nrhs, DS_PLAIN, nullptr, st);
  } else {
    const size_t n = c->lev[level].vsize() * nrhs;
    AsyncBuf<float2> x(st), y(st);
    HIPK(x.alloc(n));
    HIPK(y.alloc(n));
    HIPK((convert<float, double>(x.p, a, n, st)));
    MG_TRY(apply_A<P>(c, level, x.p, y.p, nrhs, DS_PLAIN, nullptr, st));
    HIPK((convert<double, float>(b, y.p, n, st)));
    return MG_OK;
  }
}
}  // namespace

namespace {
template <typename P>
int transfer_t(mg_ctx *c, int level, int dir, const double2 *a, double2 *b, int nrhs, hipStream_t st) {
  using R = typename P::R;
  if constexpr (sizeof(R) == 8) {
    if (dir == 0) return transfer_restrict<P>(c, level, a, b, nrhs, st);
    return transfer_prolong<P>(c, level, a, b, nrhs, 0, st);
  } else {
    const size_t nf = c->lev[level].vsize() * nrhs, nc = c->lev[level + 1].vsize() * nrhs;
    const size_t nin = dir == 0 ? nf : nc, nout = dir == 0 ? nc : nf;
    AsyncBuf<float2> x(st), y(st);
    HIPK(x.alloc(nin));
    HIPK(y.alloc(nout));
    HIPK((convert<float, double>(x.p, a, nin, st)));
    if (dir == 0) MG_TRY(transfer_restrict<P>(c, level, x.p, y.p, nrhs, st));
    else MG_TRY(transfer_prolong<P>(c, level, x.p, y.p, nrhs, 0, st));
    HIPK((convert<double, float>(b, y.p, nout, st)));
    return MG_OK;
  }
}
}  // namespace

extern "C" int mg_transfer(mg_ctx_t *ctx, int level, mg_prec_t prec, int direction, const void *in, void *out,
                           int nrhs, hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 2));
  if (!in || !out || in == out || nrhs < 1) return bad(MG_EINVAL, "mg_transfer: bad buffers or nrhs");
  if (direction != 0 && direction != 1) return bad(MG_EINVAL, "mg_transfer: direction must be 0 or 1");
  if (prec != MG_F64 && prec != MG_F32 && prec != MG_F16)
    return bad(MG_ENOTSUP, "mg_transfer: prec must be MG_F64, MG_F32 or MG_F16");
  MG_TRY(ensure_prec(ctx, prec, st));
  MG_TRY(ensure_scalars(ctx, part_need(ctx, 1)));
  const int lin = direction == 0 ? level : level + 1, lout = direction == 0 ? level + 1 : level;
  AsyncBuf<double2> a(st), b(st);
  HIPK(a.alloc(ctx->lev[lin].vsize() * nrhs));
  HIPK(b.alloc(ctx->lev[lout].vsize() * nrhs));
  HIPK(pack_level(ctx, lin, in, a.p, nrhs, st));
  int rc;
  if (prec == MG_F64) rc = transfer_t<PF64>(ctx, level, direction, a.p, b.p, nrhs, st);
  else if (prec == MG_F32) rc = transfer_t<PF32>(ctx, level, direction, a.p, b.p, nrhs, st);
  else rc = transfer_t<PF16>(ctx, level, direction, a.p, b.p, nrhs, st);
  MG_TRY(rc);
  HIPK(unpack_level(ctx, lout, b.p, out, nrhs, st));
  return MG_OK;
}

extern "C" int mg_apply_op(mg_ctx_t *ctx, int level, mg_prec_t prec, const void *in, void *out, int nrhs,
                           hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 1));
  if (!in || !out || in == out || nrhs < 1) return bad(MG_EINVAL, "mg_apply_op: bad buffers or nrhs");
  if (prec != MG_F64 && prec != MG_F32 && prec != MG_F16)
    return bad(MG_ENOTSUP, "mg_apply_op: prec must be MG_F64, MG_F32 or MG_F16");
  MG_TRY(ensure_prec(ctx, prec, st));
  const Level &L = ctx->lev[level];
  AsyncBuf<double2> a(st), b(st);
  HIPK(a.alloc(L.vsize() * nrhs));
  HIPK(b.alloc(L.vsize() * nrhs));
  HIPK(pack_level(ctx, level, in, a.p, nrhs, st));
  int rc;
  if (prec == MG_F64) rc = apply_op_t<PF64>(ctx, level, a.p, b.p, nrhs, st);
  else if (prec == MG_F32) rc = apply_op_t<PF32>(ctx, level, a.p, b.p, nrhs, st);
  else rc = apply_op_t<PF16>(ctx, level, a.p, b.p, nrhs, st);
  MG_TRY(rc);
  HIPK(unpack_level(ctx, level, b.p, out, nrhs, st));
  return MG_OK;
}

extern "C" int mg_solve(mg_ctx_t *ctx, const void *b, void *x, int nrhs, double tol, mg_info_t *info,
                        hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (!b || !x || b == x) return bad(MG_EINVAL, "mg_solve: bad buffers");
  if (nrhs < 1 || nrhs > ctx->p.max_rhs) return bad(MG_EINVAL, "mg_solve: nrhs out of range (max_rhs)");
  if (!(tol > 0.0)) return bad(MG_EINVAL, "mg_solve: tol must be positive");
  mg_ctx *c = ctx;
  MG_TRY(ensure_fgcr(c, nrhs));
  MG_TRY(ensure_prec(c, c->prec, st));
  if (c->prec == MG_F64) MG_TRY(ensure_work<double>(c, nrhs));
  else MG_TRY(ensure_work<float>(c, nrhs));
  MG_TRY(ensure_mrq(c, c->prec, nrhs));
  MG_TRY(ensure_scalars(c, part_need(c, nrhs)));
  c->n_fine = c->n_coarse = c->n_coarse_disp = c->n_cgnr = c->n_vcyc = c->n_cg_fallback = 0;
  for (auto &t : c->tm) t.reset();
  HIPK(hipStreamSynchronize(st));
  const double t0 = now_s();
  hipStream_t s2 = c->sti;
  HIPK(hipEventRecord(c->ev_in, st));
  HIPK(hipStreamWaitEvent(s2, c->ev_in, 0));
  HIPK(pack_field<double>(c->lev[0].g, (const double2 *)b, c->gb, 12, nrhs, s2));
  int iters[MG_MAX_RHS];
  double relres[MG_MAX_RHS];
  const int rc = fgcr(c, c->gb, c->gx, nrhs, tol, iters, relres, s2);
  if (rc < 0) {
    (void)hipStreamSynchronize(s2);
    return rc;
  }
  HIPK(unpack_field<double>(c->lev[0].g, c->gx, (double2 *)x, 12, nrhs, s2));
  HIPK(hipEventRecord(c->ev_out, s2));
  HIPK(hipStreamWaitEvent(st, c->ev_out, 0));
  HIPK(hipStreamSynchronize(s2));
  const double t1 = now_s();
  for (auto &t : c->tm) t.harvest();
  if (info) {
    std::memset(info, 0, sizeof(*info));
    for (int i = 0; i < nrhs; ++i) {
      info->iters[i] = iters[i];
      info->rel_resid[i] = relres[i];
    }
    info->n_fine_dslash = (int)c->n_fine;
    info->n_coarse_apply = (int)c->n_coarse;
    info->n_cgnr_iters = (int)c->n_cgnr;
    info->n_coarse_dispatch = (int)c->n_coarse_disp;
    info->n_vcycles = (int)c->n_vcyc;
    info->n_cgnr_fallbacks = (int)c->n_cg_fallback;
    info->t_setup_s = c->t_setup;
    info->t_solve_s = t1 - t0;
    if (c->timing) {
      for (int k = 0; k < MG_KERNEL_CLASSES; ++k) {
        info->kernel_ms[k] = c->tm[k].ms;
        info->kernel_launches[k] = (int)c->tm[k].launches;
        info->kernel_sites[k] = c->tm[k].sites;
      }
    }
  }
  return rc;
}

extern "C" int mg_vcycle(mg_ctx_t *ctx, mg_prec_t prec, const void *in, void *out, int nrhs, int *cgnr_iters,
                         hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (!in || !out || in == out) return bad(MG_EINVAL, "mg_vcycle: bad buffers");
  if (nrhs < 1 || nrhs > MG_MAX_RHS) return bad(MG_EINVAL, "mg_vcycle: nrhs out of range");
  if (prec != MG_F64 && prec != MG_F32 && prec != MG_F16)
    return bad(MG_ENOTSUP, "mg_vcycle: prec must be MG_F64, MG_F32 or MG_F16");
  mg_ctx *c = ctx;
  MG_TRY(ensure_prec(c, prec, st));
  if (prec == MG_F64) MG_TRY(ensure_work<double>(c, nrhs));
  else MG_TRY(ensure_work<float>(c, nrhs));
  MG_TRY(ensure_mrq(c, prec, nrhs));
  MG_TRY(ensure_scalars(c, part_need(c, nrhs)));
  const Level &L0 = c->lev[0];
  DevBuf<double2> a, b;
  MG_TRY(a.alloc(L0.vsize() * nrhs));
  MG_TRY(b.alloc(L0.vsize() * nrhs));
  c->n_cgnr = 0;
  // the cycle runs on the context's own stream (graph capture needs a
  // non-default stream), ordered after and before the caller's stream
  hipStream_t s2 = c->sti;
  HIPK(hipEventRecord(c->ev_in, st));
  HIPK(hipStreamWaitEvent(s2, c->ev_in, 0));
  HIPK(pack_field<double>(L0.g, (const double2 *)in, a, 12, nrhs, s2));
  const int rc = precondition_at(c, prec, a, b, nrhs, s2);
  if (rc < 0) {
    (void)hipStreamSynchronize(s2);
    return rc;
  }
  HIPK(unpack_field<double>(L0.g, b, (double2 *)out, 12, nrhs, s2));
  HIPK(hipStreamSynchronize(s2));
  if (cgnr_iters) *cgnr_iters = (int)c->n_cgnr;
  return MG_OK;
}

namespace {
template <typename P>
int coarse_solve_t(mg_ctx *c, const double2 *b, double2 *x, int nrhs, int *iters, hipStream_t st) {
  using R = typename P::R;
  const int l = c->nlev - 1;
  const size_t n = c->lev[l].vsize() * nrhs;
  const vec_t<P> *bb;
  vec_t<P> *xx;
  if constexpr (sizeof(R) == 8) {
    bb = b;
    xx = x;
  } else {
    Work<float> &w = c->w32;
    HIPK((convert<float, double>(w.rin[l], b, n, st)));
    bb = w.rin[l];
    xx = w.x[l];
  }
  MG_TRY(cgnr<P>(c, l, bb, xx, nrhs, st));
  // per right-hand side counts as the solve left them (both parity slots of
  // the chunks; the whole-solve launch writes both)
  for (int i = 0; i < nrhs && iters; ++i)
    iters[i] = std::max(c->h_it[i], c->h_it[(nrhs == 1 ? 1 : nrhs + i)]);
  if constexpr (sizeof(R) != 8) HIPK((convert<double, float>(x, xx, n, st)));
  return MG_OK;
}
}  // namespace

extern "C" int mg_coarse_solve(mg_ctx_t *ctx, mg_prec_t prec, const void *b, void *x, int nrhs, int *iters,
                               hipStream_t st) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  if (!b || !x || b == x) return bad(MG_EINVAL, "mg_coarse_solve: bad buffers");
  if (nrhs < 1 || nrhs > MG_MAX_RHS) return bad(MG_EINVAL, "mg_coarse_solve: nrhs out of range");
  if (prec != MG_F64 && prec != MG_F32 && prec != MG_F16)
    return bad(MG_ENOTSUP, "mg_coarse_solve: prec must be MG_F64, MG_F32 or MG_F16");
  mg_ctx *c = ctx;
  MG_TRY(ensure_prec(c, prec, st));
  if (prec == MG_F64) MG_TRY(ensure_work<double>(c, nrhs));
  else MG_TRY(ensure_work<float>(c, nrhs));
  MG_TRY(ensure_scalars(c, part_need(c, nrhs)));
  const int l = c->nlev - 1;
  DevBuf<double2> a, e;
  MG_TRY(a.alloc(c->lev[l].vsize() * nrhs));
  MG_TRY(e.alloc(c->lev[l].vsize() * nrhs));
  hipStream_t s2 = c->sti;
  HIPK(hipEventRecord(c->ev_in, st));
  HIPK(hipStreamWaitEvent(s2, c->ev_in, 0));
  HIPK(pack_level(c, l, b, a, nrhs, s2));
  int rc;
  if (prec == MG_F64) rc = coarse_solve_t<PF64>(c, a, e, nrhs, iters, s2);
  else if (prec == MG_F32) rc = coarse_solve_t<PF32>(c, a, e, nrhs, iters, s2);
  else rc = coarse_solve_t<PF16>(c, a, e, nrhs, iters, s2);
  if (rc < 0) {
    (void)hipStreamSynchronize(s2);
    return rc;
  }
  HIPK(unpack_level(c, l, e, x, nrhs, s2));
  HIPK(hipStreamSynchronize(s2));
  return MG_OK;
}

namespace {
template <typename P> int time_dslash_t(mg_ctx *c, int nrhs, int reps, hipEvent_t e0, hipEvent_t e1, hipStream_t st) {
  using R = typename P::R;
  using S = typename P::S;
  Level &L = c->lev[0];
  const size_t n = L.vsize() * nrhs;
  DevBuf<vec_t<P>> a, b;
  MG_TRY(a.alloc(n));
  MG_TRY(b.alloc(n));
  if constexpr (sizeof(R) == 8) HIPK(copy<double>(a, L.P64, std::min(n, L.P64.n), st));
  else HIPK((convert<float, double>(a, L.P64, std::min(n, L.P64.n), st)));
  const S *U = links_of_level<P>(L);
  if constexpr (std::is_same<fres_t<P>, h16>::value) {
    // the FP16 class applies the stencil to binary16 spinors inside the cycle
    const size_t nh = (size_t)13 * L.g.Vpad * nrhs;
    DevBuf<h16> ah, bh;
    MG_TRY(ah.alloc(nh));
    MG_TRY(bh.alloc(nh));
    HIPK(to_h16<float2>(ah, a, L.g.Vpad, nrhs, st));
    for (int i = 0; i < 2; ++i)
      HIPK((dslash<R, S, h16, h16>(L.g, U, L.nl, ah.p, bh.p, nullptr, 4.0 + c->mass, nrhs, DS_PLAIN, nullptr, st)));
    HIPK(hipEventRecord(e0, st));
    for (int i = 0; i < reps; ++i)
      HIPK((dslash<R, S, h16, h16>(L.g, U, L.nl, ah.p, bh.p, nullptr, 4.0 + c->mass, nrhs, DS_PLAIN, nullptr, st)));
    HIPK(hipEventRecord(e1, st));
    HIPK(hipEventSynchronize(e1));
    return MG_OK;
  }
  for (int i = 0; i < 2; ++i)
    HIPK((dslash<R, S>(L.g, U, L.nl, a.p, b.p, nullptr, 4.0 + c->mass, nrhs, DS_PLAIN, nullptr, st)));
  HIPK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i)
    HIPK((dslash<R, S>(L.g, U, L.nl, a.p, b.p, nullptr, 4.0 + c->mass, nrhs, DS_PLAIN, nullptr, st)));
  HIPK(hipEventRecord(e1, st));
  HIPK(hipEventSynchronize(e1));
  return MG_OK;
}
// The DS_MRQ stencil on the level-0 vectors of the FP32 or FP16 class:
// q' and r' alternate between two buffer pairs, a = 0.1 for every RHS.
template <typename P, typename T>
static int time_mrq_t(mg_ctx *c, int nrhs, int reps, hipEvent_t e0, hipEvent_t e1, hipStream_t st) {
  using R = typename P::R;
  using S = typename P::S;
  Level &L = c->lev[0];
  const size_t nv = L.vsize() * nrhs, nt = (size_t)site_slots<T>() * L.g.Vpad * nrhs;
  DevBuf<float2> a;
  DevBuf<T> q[2], r[2];
  DevBuf<double> part;
  DevBuf<double2> alpha;
  MG_TRY(a.alloc(nv));
  for (int i = 0; i < 2; ++i) {
    MG_TRY(q[i].alloc(nt));
    MG_TRY(r[i].alloc(nt));
  }
  MG_TRY(part.alloc((size_t)3 * dslash_partials(L.g, nrhs) * nrhs));
  MG_TRY(alpha.alloc(nrhs));
  HIPK((convert<float, double>(a, L.P64, std::min(nv, L.P64.n), st)));
  if constexpr (std::is_same<T, h16>::value) {
    HIPK(to_h16<float2>(q[0], a, L.g.Vpad, nrhs, st));
    HIPK(to_h16<float2>(r[0], a, L.g.Vpad, nrhs, st));
  } else {
    HIPK(copy<float>(q[0], a, nv, st));
    HIPK(copy<float>(r[0], a, nv, st));
  }
  HIPK(fill_const<double>(alpha, nrhs, 0.1, st));
  const S *U = links_of_level<P>(L);
  auto launch = [&](int i) {
    MrqArgs<T> mq;
    mq.rprev = r[i & 1];
    mq.rout = r[(i + 1) & 1];
    mq.alpha = alpha;
    return dslash<R, S, T, T>(L.g, U, L.nl, q[i & 1].p, q[(i + 1) & 1].p, nullptr, 4.0 + c->mass, nrhs, DS_MRQ,
                              part, st, mq);
  };
  for (int i = 0; i < 2; ++i) HIPK(launch(i));
  HIPK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) HIPK(launch(i));
  HIPK(hipEventRecord(e1, st));
  HIPK(hipEventSynchronize(e1));
  return MG_OK;
}

template <typename P>
int time_coarse_t(mg_ctx *c, int level, int nrhs, int reps, hipEvent_t e0, hipEvent_t e1, hipStream_t st) {
  using R = typename P::R;
  using S = typename P::S;
  Level &L = c->lev[level];
  const size_t n = L.vsize() * nrhs;
  DevBuf<vec_t<P>> a, b;
  MG_TRY(a.alloc(n));
  MG_TRY(b.alloc(n));
  const S *Lop = cop_of_level<P>(L);
  CoarseArgs ca;
  ca.variant = coarse_variant<P>(c, level, nrhs, st);
  if (ca.variant < 0) return ca.variant;
  if (ca.variant >= 8) ca.lt = cop_t_of_level<P>(c, L, st);
  for (int i = 0; i < 2; ++i) HIPK((coarse_apply_k<R, S>(L.g, L.n, Lop, a, b, nrhs, 0, ca, st)));
  HIPK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) HIPK((coarse_apply_k<R, S>(L.g, L.n, Lop, a, b, nrhs, 0, ca, st)));
  HIPK(hipEventRecord(e1, st));
  HIPK(hipEventSynchronize(e1));
  return MG_OK;
}
}  // namespace

extern "C" int mg_time_dslash(mg_ctx_t *ctx, mg_prec_t prec, int nrhs, int reps, double *avg_ms, hipStream_t st) {
  set_error("");
  if (!ctx || !avg_ms || nrhs < 1 || reps < 1) return bad(MG_EINVAL, "mg_time_dslash: bad arguments");
  MG_TRY(ensure_prec(ctx, prec, st));
  hipEvent_t e0, e1;
  HIPK(hipEventCreate(&e0));
  HIPK(hipEventCreate(&e1));
  int rc;
  if (prec == MG_F64) rc = time_dslash_t<PF64>(ctx, nrhs, reps, e0, e1, st);
  else if (prec == MG_F32) rc = time_dslash_t<PF32>(ctx, nrhs, reps, e0, e1, st);
  else rc = time_dslash_t<PF16>(ctx, nrhs, reps, e0, e1, st);
  float ms = 0.f;
  if (rc == MG_OK) rc = hip_rc(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return rc;
}

extern "C" int mg_time_dslash_mrq(mg_ctx_t *ctx, mg_prec_t prec, int nrhs, int reps, double *avg_ms,
                                  hipStream_t st) {
  set_error("");
  if (!ctx || !avg_ms || nrhs < 1 || reps < 1) return bad(MG_EINVAL, "mg_time_dslash_mrq: bad arguments");
  if (prec != MG_F32 && prec != MG_F16) return bad(MG_ENOTSUP, "mg_time_dslash_mrq: prec must be MG_F32 or MG_F16");
  MG_TRY(ensure_prec(ctx, prec, st));
  hipEvent_t e0, e1;
  HIPK(hipEventCreate(&e0));
  HIPK(hipEventCreate(&e1));
  int rc;
  if (prec == MG_F32) rc = time_mrq_t<PF32, float2>(ctx, nrhs, reps, e0, e1, st);
  else rc = time_mrq_t<PF16, h16>(ctx, nrhs, reps, e0, e1, st);
  float ms = 0.f;
  if (rc == MG_OK) rc = hip_rc(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return rc;
}

extern "C" int mg_time_coarse(mg_ctx_t *ctx, int level, mg_prec_t prec, int nrhs, int reps, double *avg_ms,
                              hipStream_t st) {
  set_error("");
  if (!ctx || !avg_ms || nrhs < 1 || reps < 1) return bad(MG_EINVAL, "mg_time_coarse: bad arguments");
  MG_TRY(check_ctx_level(ctx, level, 1, ctx->nlev - 1));
  MG_TRY(ensure_prec(ctx, prec, st));
  hipEvent_t e0, e1;
  HIPK(hipEventCreate(&e0));
  HIPK(hipEventCreate(&e1));
  int rc;
  if (prec == MG_F64) rc = time_coarse_t<PF64>(ctx, level, nrhs, reps, e0, e1, st);
  else if (prec == MG_F32) rc = time_coarse_t<PF32>(ctx, level, nrhs, reps, e0, e1, st);
  else rc = time_coarse_t<PF16>(ctx, level, nrhs, reps, e0, e1, st);
  float ms = 0.f;
  if (rc == MG_OK) rc = hip_rc(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return rc;
}

extern "C" int mg_destroy(mg_ctx_t *ctx) {
  if (!ctx) return MG_OK;
  (void)hipDeviceSynchronize();
  clear_graphs(ctx);
  if (ctx->sti) (void)hipStreamDestroy(ctx->sti);
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
  for (auto e : ctx->ev_chunk)
    if (e) (void)hipEventDestroy(e);
  if (ctx->h_done) (void)hipHostFree(ctx->h_done);
  if (ctx->h_rr) (void)hipHostFree(ctx->h_rr);
  if (ctx->h_it) (void)hipHostFree(ctx->h_it);
  delete ctx;
  return MG_OK;
}

extern "C" int mg_level_info(mg_ctx_t *ctx, int level, int *L_out, int *ncomp_out) {
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 1));
  if (L_out)
    for (int mu = 0; mu < 4; ++mu) L_out[mu] = ctx->lev[level].g.L[mu];
  if (ncomp_out) *ncomp_out = ctx->lev[level].n;
  return MG_OK;
}

extern "C" int mg_export_maps(mg_ctx_t *ctx, int level, int32_t *f2c, int32_t *f2l, int32_t *cnbr, int32_t *face) {
  set_error("");
  if (!ctx) return bad(MG_EINVAL, "ctx is NULL");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 2));
  const Geom &g = ctx->lev[level].g, &gc = ctx->lev[level + 1].g;
  DevBuf<int32_t> d;
  MG_TRY(d.alloc(3 * (size_t)g.V + 8 * (size_t)gc.V));
  int32_t *df2c = d.p, *df2l = d.p + g.V, *dface = d.p + 2 * (size_t)g.V, *dn = d.p + 3 * (size_t)g.V;
  HIPK(export_maps_k(g, gc, df2c, df2l, dface, dn, nullptr));
  HIPK(hipStreamSynchronize(nullptr));
  if (f2c) HIPK(hipMemcpy(f2c, df2c, sizeof(int32_t) * g.V, hipMemcpyDeviceToHost));
  if (f2l) HIPK(hipMemcpy(f2l, df2l, sizeof(int32_t) * g.V, hipMemcpyDeviceToHost));
  if (face) HIPK(hipMemcpy(face, dface, sizeof(int32_t) * g.V, hipMemcpyDeviceToHost));
  if (cnbr) HIPK(hipMemcpy(cnbr, dn, sizeof(int32_t) * 8 * gc.V, hipMemcpyDeviceToHost));
  return MG_OK;
}

extern "C" int mg_export_P(mg_ctx_t *ctx, int level, void *P_host) {
  set_error("");
  if (!ctx || !P_host) return bad(MG_EINVAL, "mg_export_P: NULL argument");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 2));
  const Level &L = ctx->lev[level];
  const size_t cnt = L.P64.n;
  std::vector<double2> h(cnt);
  HIPK(hipDeviceSynchronize());
  HIPK(hipMemcpy(h.data(), L.P64, cnt * sizeof(double2), hipMemcpyDeviceToHost));
  double2 *out = (double2 *)P_host;
  const int nv = L.nv, n = L.n, h2 = n / 2;
  const size_t V = L.g.V, vb = L.g.vb, rows = vb * h2;
  for (int k = 0; k < nv; ++k)
    for (size_t s = 0; s < V; ++s) {
      const size_t B = s / vb, l = s % vb;
      for (int c = 0; c < n; ++c) {
        const double2 v = (level == 0) ? h[(size_t)k * 12 * L.g.Vpad + fidx((uint32_t)s, c, 12)]
                                       : h[((size_t)k * V + s) * n + c];
        const int chi = c / h2, j = c % h2;
        out[((B * 2 + chi) * rows + l * h2 + j) * nv + k] = v;
      }
    }
  return MG_OK;
}

extern "C" int mg_export_coarse_op(mg_ctx_t *ctx, int level, void *X_host, void *Y_host) {
  set_error("");
  if (!ctx || !X_host || !Y_host) return bad(MG_EINVAL, "mg_export_coarse_op: NULL argument");
  MG_TRY(check_ctx_level(ctx, level, 1, ctx->nlev - 1));
  const Level &L = ctx->lev[level];
  const size_t cnt = L.L64.n;
  std::vector<double2> h(cnt);
  HIPK(hipDeviceSynchronize());
  HIPK(hipMemcpy(h.data(), L.L64, cnt * sizeof(double2), hipMemcpyDeviceToHost));
  const size_t V = L.g.V;
  const int n = L.n;
  double2 *X = (double2 *)X_host, *Y = (double2 *)Y_host;
  for (uint32_t s = 0; s < V; ++s) {
    const Coords k = decode(L.g, s);
    const size_t i = canon_index(L.g, k);
    for (int slot = 0; slot < 9; ++slot)
      for (int j = 0; j < n; ++j)
        for (int r = 0; r < n; ++r) {
          const double2 v = h[(((size_t)s * 9 + slot) * n + j) * n + r];
          if (slot == 0) X[(i * n + r) * n + j] = v;
          else Y[((((size_t)(slot - 1)) * V + i) * n + r) * n + j] = v;
        }
  }
  return MG_OK;
}

extern "C" int mg_export_nullvecs(mg_ctx_t *ctx, int level, void *V_host) {
  set_error("");
  if (!ctx || !V_host) return bad(MG_EINVAL, "mg_export_nullvecs: NULL argument");
  MG_TRY(check_ctx_level(ctx, level, 0, ctx->nlev - 2));
  const Level &L = ctx->lev[level];
  DevBuf<double2> d;
  MG_TRY(d.alloc(L.NV.n));
  HIPK(unpack_level(ctx, level, L.NV, d.p, L.nv, nullptr));
  HIPK(hipStreamSynchronize(nullptr));
  HIPK(hipMemcpy(V_host, d.p, L.NV.n * sizeof(double2), hipMemcpyDeviceToHost));
  return MG_OK;
}
