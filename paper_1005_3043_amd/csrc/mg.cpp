// Host orchestration of the adaptive multigrid solver: setup (null-vector
// relaxation, block orthonormalisation, Galerkin construction), the V-cycle
// preconditioner (MR smoothing, restriction, recursive coarse correction,
// prolongation, CGNR on the coarsest level) and flexible GCR.  Every step runs
// in the HIP kernels; the host only sequences launches on one stream and
// reads residual norms / convergence flags for its decisions.
#include <chrono>
#include <cmath>
#include <cstring>

#include "mg_internal.h"

namespace mg {

template <> Work<double> &work<double>(mg_ctx *c) { return c->w64; }
template <> Work<float> &work<float>(mg_ctx *c) { return c->w32; }

static int hip_rc(hipError_t e, const char *what) {
  if (e == hipSuccess) return MG_OK;
  set_error(hip_error_string(e, what));
  return MG_EHIP;
}
#define HIPK(expr) MG_TRY(hip_rc((expr), #expr))

int ensure_scalars(mg_ctx *c, size_t part_count) {
  MG_TRY(c->part.alloc(part_count));
  MG_TRY(c->part2.alloc(part_count));
  MG_TRY(c->dsc.alloc(16 * MG_MAX_RHS * 8));
  MG_TRY(c->csc.alloc(16 * MG_MAX_RHS * 8));
  MG_TRY(c->cg.alloc(CG_NS * MG_MAX_RHS * 8));
  MG_TRY(c->done.alloc(MG_MAX_RHS * 8));
  MG_TRY(c->it.alloc(MG_MAX_RHS * 8));
  if (!c->h_done) {
    if (hipHostMalloc((void **)&c->h_done, sizeof(int) * MG_MAX_RHS * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_rr, sizeof(double) * MG_MAX_RHS * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_it, sizeof(int) * MG_MAX_RHS * 8, hipHostMallocDefault) != hipSuccess) {
      set_error("hipHostMalloc failed");
      return MG_ENOMEM;
    }
  }
  return MG_OK;
}

// Partial-sum slots needed by a batch of nrhs vectors on every level.
size_t part_need(mg_ctx *c, int nrhs) {
  size_t m = (size_t)RED_BLOCKS * 2;
  m = std::max(m, (size_t)dslash_blocks(c->lev[0].g) * 3);
  for (int l = 1; l < c->nlev; ++l) m = std::max(m, (size_t)c->lev[l].g.V * 3);
  return m * (size_t)nrhs;
}

int ensure_prec(mg_ctx *c, mg_prec_t prec, hipStream_t st) {
  if (prec == MG_F64) return MG_OK;
  if (prec != MG_F32) {
    set_error("preconditioner precision must be MG_F64 or MG_F32");
    return MG_ENOTSUP;
  }
  Level &L0 = c->lev[0];
  if (!L0.U32.p) {
    MG_TRY(L0.U32.alloc(36 * (size_t)L0.g.V));
    HIPK((convert<float, double>(L0.U32, L0.U64, 36 * (size_t)L0.g.V, st)));
  }
  for (int l = 0; l < c->nlev; ++l) {
    Level &L = c->lev[l];
    if (L.nv > 0 && !L.P32.p) {
      MG_TRY(L.P32.alloc(L.P64.n));
      HIPK((convert<float, double>(L.P32, L.P64, L.P64.n, st)));
    }
    if (l > 0 && !L.L32.p) {
      MG_TRY(L.L32.alloc(L.L64.n));
      HIPK((convert<float, double>(L.L32, L.L64, L.L64.n, st)));
    }
  }
  return MG_OK;
}

template <typename R> int ensure_work(mg_ctx *c, int nrhs) {
  Work<R> &w = work<R>(c);
  if (w.nrhs >= nrhs) return MG_OK;
  for (int l = 0; l < c->nlev; ++l) {
    const size_t n = c->lev[l].vsize() * nrhs;
    MG_TRY(w.x[l].alloc(n));
    MG_TRY(w.r[l].alloc(n));
    MG_TRY(w.q[l].alloc(n));
    MG_TRY(w.rin[l].alloc(n));
  }
  const size_t n = c->lev[c->nlev - 1].vsize() * nrhs;
  MG_TRY(w.ce.alloc(n));
  MG_TRY(w.cr.alloc(n));
  MG_TRY(w.cz.alloc(n));
  MG_TRY(w.cp.alloc(n));
  MG_TRY(w.cw.alloc(n));
  MG_TRY(ensure_scalars(c, part_need(c, nrhs)));
  w.nrhs = nrhs;
  return MG_OK;
}
template int ensure_work<double>(mg_ctx *, int);
template int ensure_work<float>(mg_ctx *, int);

// ------------------------------------------------------------ operators
template <typename R> const c_t<R> *U_of(Level &L) { return PrecBufs<R>::pick(L.U64, L.U32).p; }
template <typename R> const c_t<R> *L_of(Level &L) { return PrecBufs<R>::pick(L.L64, L.L32).p; }
template <typename R> const c_t<R> *P_of(Level &L) { return PrecBufs<R>::pick(L.P64, L.P32).p; }

int np_mr(mg_ctx *c, int l) { return l == 0 ? dslash_blocks(c->lev[0].g) : (int)c->lev[l].g.V; }

struct TimerScope {
  EventTimer *t = nullptr;
  hipEvent_t e1 = nullptr;
  hipStream_t st;
  TimerScope(mg_ctx *c, EventTimer &tm, hipStream_t s) : st(s) {
    if (c->timing) {
      hipEvent_t e0 = tm.next();
      e1 = tm.next();
      if (e0 && e1) {
        (void)hipEventRecord(e0, st);
        t = &tm;
      }
    }
  }
  ~TimerScope() {
    if (t) (void)hipEventRecord(e1, st);
  }
};

// out = A_l in  (DS_MR: MR partials into c->part; DS_RESID: out = b - A_l in)
template <typename R>
int apply_A(mg_ctx *c, int l, const c_t<R> *in, c_t<R> *out, int nrhs, DslashMode mode, const c_t<R> *b,
            hipStream_t st) {
  Level &L = c->lev[l];
  if (l == 0) {
    TimerScope ts(c, c->tm_dslash, st);
    HIPK(dslash<R>(L.g, U_of<R>(L), in, out, b, 4.0 + c->mass, nrhs, mode, c->part, st));
    c->n_fine += nrhs;
  } else {
    {
      TimerScope ts(c, c->tm_coarse, st);
      HIPK(coarse_apply_k<R>(L.g, L.n, L_of<R>(L), in, out, nrhs, 0, mode == DS_MR ? c->part.p : nullptr, 3,
                             nullptr, st));
    }
    if (mode == DS_RESID) HIPK(resid_from<R>(out, b, L.vsize(), nrhs, st));
    c->n_coarse += nrhs;
  }
  return MG_OK;
}

template <typename R>
int coarse_dag_or_not(mg_ctx *c, int l, const c_t<R> *in, c_t<R> *out, int nrhs, int dagger, double *part,
                      const int *done, hipStream_t st) {
  Level &L = c->lev[l];
  TimerScope ts(c, c->tm_coarse, st);
  HIPK(coarse_apply_k<R>(L.g, L.n, L_of<R>(L), in, out, nrhs, dagger, part, 1, done, st));
  return MG_OK;
}

// MR smoothing of A_l x = r0 from x = 0 (accumulate: add into x): on return
// r holds the recursively updated residual.
template <typename R>
int mr(mg_ctx *c, int l, c_t<R> *x, c_t<R> *r, c_t<R> *q, int steps, bool accumulate, int nrhs, hipStream_t st) {
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  if (steps == 0 && !accumulate) HIPK(zero<R>(x, n * nrhs, st));
  for (int k = 0; k < steps; ++k) {
    MG_TRY(apply_A<R>(c, l, r, q, nrhs, DS_MR, nullptr, st));
    HIPK(mr_update<R>(x, r, q, n, nrhs, c->part, np_mr(c, l), c->p.omega, c->csc, (!accumulate && k == 0) ? 1 : 0,
                      st));
  }
  return MG_OK;
}

template <typename R>
int transfer_restrict(mg_ctx *c, int l, const c_t<R> *fine, c_t<R> *coarse, int nrhs, hipStream_t st) {
  Level &L = c->lev[l], &Lc = c->lev[l + 1];
  if (l == 0) HIPK(restrict_fine<R>(L.g, Lc.g, L.nv, P_of<R>(L), fine, coarse, nrhs, st));
  else HIPK(restrict_coarse<R>(L.g, Lc.g, L.n, L.nv, P_of<R>(L), fine, coarse, nrhs, st));
  return MG_OK;
}

template <typename R>
int transfer_prolong(mg_ctx *c, int l, const c_t<R> *coarse, c_t<R> *fine, int nrhs, int accumulate,
                     hipStream_t st) {
  Level &L = c->lev[l], &Lc = c->lev[l + 1];
  if (l == 0) HIPK(prolong_fine<R>(L.g, Lc.g, L.nv, P_of<R>(L), coarse, fine, nrhs, accumulate, st));
  else HIPK(prolong_coarse<R>(L.g, Lc.g, L.n, L.nv, P_of<R>(L), coarse, fine, nrhs, accumulate, st));
  return MG_OK;
}

// CGNR on A^dag A e = A^dag b (coarsest level), A^dag = sigma3 A sigma3,
// stopping at ||b - A e|| <= tol ||b|| (recursive residual).
template <typename R> int cgnr(mg_ctx *c, int l, const c_t<R> *b, c_t<R> *e, int nrhs, hipStream_t st) {
  Work<R> &w = work<R>(c);
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  const int V = (int)L.g.V;
  c_t<R> *r = w.cr, *z = w.cz, *p = w.cp, *ww = w.cw;
  HIPK(zero<R>(e, n * nrhs, st));
  HIPK(copy<R>(r, b, n * nrhs, st));
  const int npb = norm2_partials<R>(b, n, nrhs, c->part2, st);
  MG_TRY(coarse_dag_or_not<R>(c, l, r, z, nrhs, 1, c->part, nullptr, st));
  HIPK(cg_init_scalars(c->part, V, c->part2, npb, nrhs, c->cg, c->done, c->it, c->p.coarse_tol, st));
  HIPK(copy<R>(p, z, n * nrhs, st));
  const int maxit = c->p.coarse_maxiter;
  const int chunk = 8;
  for (int it0 = 0; it0 < maxit; it0 += chunk) {
    for (int k = 0; k < chunk; ++k) {
      MG_TRY(coarse_dag_or_not<R>(c, l, p, ww, nrhs, 0, c->part, c->done, st));
      HIPK(cg_alpha(c->part, V, nrhs, c->cg, c->done, st));
      HIPK(cg_update<R>(e, p, r, ww, n, nrhs, c->cg, c->done, c->it, maxit, c->part2, st));
      MG_TRY(coarse_dag_or_not<R>(c, l, r, z, nrhs, 1, c->part, c->done, st));
      HIPK(cg_beta(c->part, V, nrhs, c->cg, c->done, st));
      HIPK(cg_p<R>(p, z, n, nrhs, c->cg, c->done, st));
    }
    HIPK(hipMemcpyAsync(c->h_done, c->done, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    HIPK(hipStreamSynchronize(st));
    bool all = true;
    for (int i = 0; i < nrhs; ++i) all = all && c->h_done[i];
    if (all) break;
  }
  HIPK(hipMemcpyAsync(c->h_it, c->it, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
  HIPK(hipStreamSynchronize(st));
  for (int i = 0; i < nrhs; ++i) {
    c->n_cgnr += c->h_it[i];
    c->n_coarse += 1 + 2L * c->h_it[i];
  }
  return MG_OK;
}

// One V-cycle K_l(rin) -> x (levels l..coarsest).
template <typename R> int vcycle(mg_ctx *c, int l, const c_t<R> *rin, c_t<R> *x, int nrhs, hipStream_t st) {
  if (l == c->nlev - 1) return cgnr<R>(c, l, rin, x, nrhs, st);
  Work<R> &w = work<R>(c);
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  c_t<R> *r = w.r[l], *q = w.q[l];
  HIPK(copy<R>(r, rin, n * nrhs, st));
  MG_TRY(mr<R>(c, l, x, r, q, c->p.pre, false, nrhs, st));
  MG_TRY(transfer_restrict<R>(c, l, r, w.rin[l + 1], nrhs, st));
  MG_TRY(vcycle<R>(c, l + 1, w.rin[l + 1], w.x[l + 1], nrhs, st));
  MG_TRY(transfer_prolong<R>(c, l, w.x[l + 1], x, nrhs, 1, st));
  MG_TRY(apply_A<R>(c, l, x, r, nrhs, DS_RESID, rin, st));
  MG_TRY(mr<R>(c, l, x, r, q, c->p.post, true, nrhs, st));
  return MG_OK;
}

// z = K(r) in the context's preconditioner precision (FP64 in and out).
int precondition(mg_ctx *c, const double2 *r, double2 *z, int nrhs, hipStream_t st) {
  c->n_vcyc += nrhs;
  if (c->prec == MG_F64) return vcycle<double>(c, 0, r, z, nrhs, st);
  Work<float> &w = c->w32;
  const size_t n = c->lev[0].vsize() * nrhs;
  float2 *rin = w.rin[0], *x = w.x[0];
  HIPK((convert<float, double>(rin, r, n, st)));
  MG_TRY(vcycle<float>(c, 0, rin, x, nrhs, st));
  HIPK((convert<double, float>(z, x, n, st)));
  return MG_OK;
}

// ------------------------------------------------------------ FGCR
int fgcr(mg_ctx *c, const double2 *b, double2 *x, int nrhs, double tol, int *iters, double *relres,
         hipStream_t st) {
  Level &L0 = c->lev[0];
  const size_t n = L0.vsize();
  const size_t nn = n * nrhs;
  const int restart = c->p.gcr_restart;
  double2 *r = c->gr, *Z = c->gZ, *W = c->gW;
  double *rr = c->dsc;
  double2 *sc = c->csc;
  int *skip = c->skip;
  HIPK(zero<double>(x, nn, st));
  HIPK(copy<double>(r, b, nn, st));
  HIPK(norm2<double>(b, n, nrhs, c->part, rr, st));
  double nb2[MG_MAX_RHS];
  int hskip[MG_MAX_RHS];
  HIPK(hipMemcpyAsync(c->h_rr, rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  HIPK(hipStreamSynchronize(st));
  for (int i = 0; i < nrhs; ++i) {
    nb2[i] = c->h_rr[i];
    if (!std::isfinite(nb2[i])) {
      set_error("mg_solve: non-finite right-hand side");
      return MG_ENONFINITE;
    }
    hskip[i] = nb2[i] == 0.0 ? 1 : 0;
    iters[i] = 0;
    relres[i] = 0.0;
  }
  const double tol2 = tol * tol;
  HIPK(hipMemcpyAsync(skip, hskip, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
  int total = 0;
  bool all_conv = true;
  for (int i = 0; i < nrhs; ++i) all_conv = all_conv && hskip[i];
  while (!all_conv) {
    for (int j = 0; j < restart; ++j) {
      double2 *Zj = Z + (size_t)j * nn, *Wj = W + (size_t)j * nn;
      MG_TRY(precondition(c, r, Zj, nrhs, st));
      {
        TimerScope ts(c, c->tm_dslash, st);
        HIPK(dslash<double>(L0.g, L0.U64, Zj, Wj, nullptr, 4.0 + c->mass, nrhs, DS_PLAIN, nullptr, st));
      }
      c->n_fine += nrhs;
      for (int i = 0; i < j; ++i) {
        const double2 *Wi = W + (size_t)i * nn, *Zi = Z + (size_t)i * nn;
        HIPK(dot<double>(Wi, Wj, n, nrhs, c->part, sc, st));
        HIPK(gcr_sub2(Wj, Wi, Zj, Zi, n, nrhs, sc, skip, st));
      }
      HIPK(norm2<double>(Wj, n, nrhs, c->part, rr + MG_MAX_RHS, st));
      HIPK(gcr_scale2(Wj, Zj, n, nrhs, rr + MG_MAX_RHS, skip, st));
      HIPK(dot<double>(Wj, r, n, nrhs, c->part, sc, st));
      HIPK(gcr_update(x, Zj, r, Wj, n, nrhs, sc, skip, c->part, rr, st));
      HIPK(hipMemcpyAsync(c->h_rr, rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
      HIPK(hipStreamSynchronize(st));
      ++total;
      bool all = true, changed = false;
      for (int i = 0; i < nrhs; ++i) {
        if (hskip[i]) continue;
        iters[i]++;
        if (!std::isfinite(c->h_rr[i])) {
          set_error("mg_solve: non-finite residual");
          return MG_ENONFINITE;
        }
        if (c->h_rr[i] <= tol2 * nb2[i]) {
          hskip[i] = 1;
          changed = true;
        } else {
          all = false;
        }
      }
      if (changed && !all) HIPK(hipMemcpyAsync(skip, hskip, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
      if (all || total >= c->p.max_iter) break;
    }
    // true residual r = b - D x
    {
      TimerScope ts(c, c->tm_dslash, st);
      HIPK(dslash<double>(L0.g, L0.U64, x, r, b, 4.0 + c->mass, nrhs, DS_RESID, nullptr, st));
    }
    c->n_fine += nrhs;
    HIPK(norm2<double>(r, n, nrhs, c->part, rr, st));
    HIPK(hipMemcpyAsync(c->h_rr, rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    HIPK(hipStreamSynchronize(st));
    all_conv = true;
    for (int i = 0; i < nrhs; ++i) {
      relres[i] = nb2[i] > 0 ? std::sqrt(c->h_rr[i] / nb2[i]) : 0.0;
      if (nb2[i] == 0.0 || c->h_rr[i] <= tol2 * nb2[i]) {
        hskip[i] = 1;
      } else {
        hskip[i] = 0;
        all_conv = false;
      }
    }
    HIPK(hipMemcpyAsync(skip, hskip, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    if (!all_conv && total >= c->p.max_iter) return MG_NOT_CONVERGED;
  }
  return MG_OK;
}

// ------------------------------------------------------------ setup
// Null-vector relaxation: v <- v - MR(A, A v), v <- v / ||v||, `rounds` times,
// all nv vectors as one batch (FP64).
int relax(mg_ctx *c, int l, double2 *V, int nv, hipStream_t st) {
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  DevBuf<double2> x, r, q;
  MG_TRY(x.alloc(n * nv));
  MG_TRY(r.alloc(n * nv));
  MG_TRY(q.alloc(n * nv));
  for (int round = 0; round < c->p.setup_rounds; ++round) {
    MG_TRY(apply_A<double>(c, l, V, r, nv, DS_PLAIN, nullptr, st));
    MG_TRY(mr<double>(c, l, x, r, q, c->p.setup_mr_steps, false, nv, st));
    HIPK(sub_inplace<double>(V, x, n, nv, st));
    HIPK(norm2<double>(V, n, nv, c->part, c->dsc, st));
    HIPK(scale_rsqrt<double>(V, n, nv, c->dsc, st));
  }
  HIPK(hipStreamSynchronize(st));
  return MG_OK;
}

int setup(mg_ctx *c, const void *U, hipStream_t st) {
  const mg_params_t &p = c->p;
  const int anti = c->lat.t_antiperiodic ? 1 : 0;
  int L[4];
  for (int mu = 0; mu < 4; ++mu) L[mu] = c->lat.L[mu];
  const int one[4] = {1, 1, 1, 1};
  c->nlev = p.n_levels;
  for (int l = 0; l < c->nlev; ++l) {
    Level &Lv = c->lev[l];
    const int *tile = (l < c->nlev - 1) ? p.block[l] : one;
    Lv.g = make_geom(L, tile, l == 0 ? anti : 0);
    Lv.n = (l == 0) ? 12 : 2 * p.nv[l - 1];
    Lv.nv = (l < c->nlev - 1) ? p.nv[l] : 0;
    for (int mu = 0; mu < 4; ++mu) L[mu] = Lv.g.C[mu];
  }
  size_t pn = part_need(c, 1);
  for (int l = 0; l < c->nlev - 1; ++l) {
    const Level &Lv = c->lev[l];
    const size_t per = (l == 0) ? (size_t)dslash_blocks(Lv.g) * 3 : (size_t)Lv.g.V * 3;
    pn = std::max(pn, std::max(per, (size_t)RED_BLOCKS * 2) * Lv.nv);
  }
  MG_TRY(ensure_scalars(c, pn));
  Level &L0 = c->lev[0];
  MG_TRY(L0.U64.alloc(36 * (size_t)L0.g.V));
  HIPK(pack_field<double>(L0.g, (const double2 *)U, L0.U64, 9, 4, st));
  int *flag = c->done;  // reused as rank-deficiency flag during setup
  for (int l = 0; l < c->nlev - 1; ++l) {
    Level &Lv = c->lev[l], &Lc = c->lev[l + 1];
    const size_t nvs = Lv.vsize() * Lv.nv;
    MG_TRY(Lv.NV.alloc(nvs));
    MG_TRY(Lv.P64.alloc(nvs));
    if (l == 0) HIPK(pack_field<double>(Lv.g, (const double2 *)p.init_vectors[0], Lv.NV, 12, Lv.nv, st));
    else HIPK(pack_aos<double>(Lv.g, (const double2 *)p.init_vectors[l], Lv.NV, Lv.n, Lv.nv, st));
    MG_TRY(relax(c, l, Lv.NV, Lv.nv, st));
    HIPK(hipMemcpyAsync(Lv.P64, Lv.NV, nvs * sizeof(double2), hipMemcpyDeviceToDevice, st));
    HIPK(hipMemsetAsync(flag, 0, sizeof(int), st));
    if (l == 0) HIPK(ortho_fine(Lv.g, Lv.nv, Lv.P64, flag, st));
    else HIPK(ortho_coarse(Lv.g, Lv.n, Lv.nv, Lv.P64, flag, st));
    HIPK(hipMemcpyAsync(c->h_done, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPK(hipStreamSynchronize(st));
    if (c->h_done[0]) {
      set_error("mg_setup: rank-deficient aggregate in block orthonormalisation");
      return MG_ERANK;
    }
    MG_TRY(Lc.L64.alloc((size_t)Lc.g.V * 9 * Lc.n * Lc.n));
    if (l == 0) HIPK(galerkin_fine(Lv.g, Lc.g, c->mass, Lv.U64, Lv.nv, Lv.P64, Lc.L64, st));
    else HIPK(galerkin_coarse(Lv.g, Lc.g, Lv.n, Lv.L64, Lv.nv, Lv.P64, Lc.L64, st));
    HIPK(hipStreamSynchronize(st));
  }
  return MG_OK;
}

#define INST(R)                                                                                              \
  template int vcycle<R>(mg_ctx *, int, const c_t<R> *, c_t<R> *, int, hipStream_t);                         \
  template int apply_A<R>(mg_ctx *, int, const c_t<R> *, c_t<R> *, int, DslashMode, const c_t<R> *, hipStream_t); \
  template int transfer_restrict<R>(mg_ctx *, int, const c_t<R> *, c_t<R> *, int, hipStream_t);              \
  template int transfer_prolong<R>(mg_ctx *, int, const c_t<R> *, c_t<R> *, int, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace mg
