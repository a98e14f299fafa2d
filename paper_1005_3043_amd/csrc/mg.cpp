// Host orchestration of the adaptive multigrid solver: setup (null-vector
// relaxation, block orthonormalisation, Galerkin construction), the V-cycle
// preconditioner (MR smoothing, restriction, recursive coarse correction,
// prolongation, CGNR on the coarsest level) and flexible GCR.  Every step runs
// in the HIP kernels; the host only sequences launches on one stream and
// reads residual norms / convergence flags for its decisions.
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

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

// Partial sums written per RHS by one coarse-stencil launch of a level.
size_t np_coarse(const Level &L) { return (size_t)L.g.V * coarse_split(L.n, L.g.V); }

// Partial-sum slots needed by a batch of nrhs vectors on every level.
size_t part_need(mg_ctx *c, int nrhs) {
  size_t m = (size_t)RED_BLOCKS * (4 * GCR_CHUNK + 3);  // FGCR inner-product pass
  m = std::max(m, (size_t)dslash_partials(c->lev[0].g, nrhs) * 3);
  for (int l = 1; l < c->nlev; ++l) m = std::max(m, np_coarse(c->lev[l]) * 3);
  return m * (size_t)nrhs;
}

// Operator copies in storage type S (rounded to nearest even): links (two
// rows or full, as the FP64 set-up chose), prolongators, coarse stencils.
template <typename S>
static int make_copies(mg_ctx *c, DevBuf<S> &U, DevBuf<S> Level::*Pm, DevBuf<S> Level::*Lm, hipStream_t st) {
  Level &L0 = c->lev[0];
  if (!U.p) {
    MG_TRY(U.alloc(4 * (size_t)L0.nl * L0.g.Vpad));
    if (L0.nl == 6) HIPK(compress_links<S>(L0.g, L0.U64, U, c->part, st));
    else HIPK(store_convert<S>(U, L0.U64, 36 * (size_t)L0.g.Vpad, st));
  }
  for (int l = 0; l < c->nlev; ++l) {
    Level &L = c->lev[l];
    DevBuf<S> &P = L.*Pm, &Lc = L.*Lm;
    if (L.nv > 0 && !P.p) {
      MG_TRY(P.alloc(L.P64.n));
      HIPK(store_convert<S>(P, L.P64, L.P64.n, st));
    }
    if (l > 0 && !Lc.p) {
      MG_TRY(Lc.alloc(L.L64.n));
      HIPK(store_convert<S>(Lc, L.L64, L.L64.n, st));
    }
  }
  return MG_OK;
}

int ensure_prec(mg_ctx *c, mg_prec_t prec, hipStream_t st) {
  if (prec == MG_F64) return MG_OK;
  if (prec == MG_F32) {
    MG_TRY(make_copies<float2>(c, c->lev[0].U32, &Level::P32, &Level::L32, st));
    if (c->p.transfer_prec == MG_F16) {
      // the binary16 prolongators the FP32 class's transfers read
      for (int l = 0; l < c->nlev; ++l) {
        Level &L = c->lev[l];
        if (L.nv > 0 && !L.P16.p) {
          MG_TRY(L.P16.alloc(L.P64.n));
          HIPK(store_convert<chalf>(L.P16, L.P64, L.P64.n, st));
        }
      }
    }
    return MG_OK;
  }
  if (prec == MG_F16) return make_copies<chalf>(c, c->lev[0].U16, &Level::P16, &Level::L16, st);
  set_error("preconditioner precision must be MG_F64, MG_F32 or MG_F16");
  return MG_ENOTSUP;
}

void clear_graphs(mg_ctx *c) {
  for (auto &g : c->graphs) {
    delete g;
    g = nullptr;
  }
  for (VGraph *g : c->vgraphs) delete g;
  c->vgraphs.clear();
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
  if constexpr (sizeof(R) == 4) {
    const size_t nh = (size_t)13 * c->lev[0].g.Vpad * nrhs;
    MG_TRY(w.hr.alloc(nh));
    MG_TRY(w.hq.alloc(nh));
    MG_TRY(w.hrin.alloc(nh));
  }
  clear_graphs(c);
  const size_t n = c->lev[c->nlev - 1].vsize() * nrhs;
  MG_TRY(c->cgp.alloc(3 * np_coarse(c->lev[c->nlev - 1]) * MG_MAX_RHS + 2 * (size_t)RED_BLOCKS * MG_MAX_RHS));
  MG_TRY(w.ce.alloc(n));
  MG_TRY(w.cr.alloc(n));
  MG_TRY(w.cz.alloc(n));
  MG_TRY(w.cp.alloc(n));
  MG_TRY(w.cw.alloc(n));
  MG_TRY(w.cp2.alloc(n));
  MG_TRY(w.cr2.alloc(n));
  MG_TRY(ensure_scalars(c, part_need(c, nrhs)));
  if (c->p.smoother == MG_SMOOTH_GMRES) {
    const int K = std::max(c->p.pre, c->p.post);
    for (int l = 0; l < c->nlev - 1; ++l) MG_TRY(w.gv[l].alloc((size_t)(K + 1) * c->lev[l].vsize() * nrhs));
    MG_TRY(c->gmH.alloc((size_t)MG_MAX_RHS * (GM_KMAX + 1) * GM_KMAX));
    MG_TRY(c->gmy.alloc((size_t)MG_MAX_RHS * GM_KMAX));
    MG_TRY(c->gmb.alloc(2 * MG_MAX_RHS));
    MG_TRY(c->gmp.alloc((size_t)RED_BLOCKS * MG_MAX_RHS * 2 * (GM_KMAX + 1)));
  }
  if (c->p.cycles > 1) {
    for (int l = 1; l < c->nlev - 1; ++l) {
      MG_TRY(w.w2r[l].alloc(c->lev[l].vsize() * nrhs));
      MG_TRY(w.w2x[l].alloc(c->lev[l].vsize() * nrhs));
    }
  }
  w.nrhs = nrhs;
  return MG_OK;
}
template int ensure_work<double>(mg_ctx *, int);
template int ensure_work<float>(mg_ctx *, int);

// MR steps of the fine-level smoother taken by the q recursion (0: the
// smoother does not take it)
static int mrq_steps(const mg_ctx *c) {
  if (c->p.smoother != MG_SMOOTH_MR) return 0;
  const int n = std::max(c->p.pre, c->p.post);
  return (n >= 2 && n <= MRQ_MAX) ? n : 0;
}

int ensure_mrq(mg_ctx *c, mg_prec_t prec, int nrhs, int steps) {
  if (prec != MG_F32 && prec != MG_F16) return MG_OK;
  if (steps < 0) steps = mrq_steps(c);
  if (steps < 2 || steps > MRQ_MAX) return MG_OK;
  Work<float> &w = c->w32;
  const int i = prec == MG_F16 ? 1 : 0;
  if (w.mrq_nrhs[i] >= nrhs && w.mrq_steps[i] >= steps) return MG_OK;
  nrhs = std::max(nrhs, w.mrq_nrhs[i]);
  steps = std::max(steps, w.mrq_steps[i]);
  const size_t Vpad = c->lev[0].g.Vpad;
  // q_k and r_k are written at every site by the stencil before they are
  // read: only padding sites need the zero fill
  const bool pad = c->lev[0].g.Vpad != c->lev[0].g.V;
  if (i == 0) {
    MG_TRY(w.q2.alloc(12 * Vpad * nrhs, pad));
    for (int k = 0; k + 1 < steps; ++k) MG_TRY(w.rk[k].alloc(12 * Vpad * nrhs, pad));
  } else {
    MG_TRY(w.hq2.alloc(13 * Vpad * nrhs, pad));
    for (int k = 0; k + 1 < steps; ++k) MG_TRY(w.hrk[k].alloc(13 * Vpad * nrhs, pad));
  }
  w.mrq_nrhs[i] = nrhs;
  w.mrq_steps[i] = steps;
  clear_graphs(c);  // captured cycles took the other MR path
  return MG_OK;
}

// ------------------------------------------------------------ operators
template <typename P> const typename P::S *links_of(Level &L);
template <> const double2 *links_of<PF64>(Level &L) { return L.links64(); }
template <> const float2 *links_of<PF32>(Level &L) { return L.U32.p; }
template <> const chalf *links_of<PF16>(Level &L) { return L.U16.p; }
template <typename P> const typename P::S *cop_of(Level &L);
template <> const double2 *cop_of<PF64>(Level &L) { return L.L64.p; }
template <> const float2 *cop_of<PF32>(Level &L) { return L.L32.p; }
template <> const chalf *cop_of<PF16>(Level &L) { return L.L16.p; }
template <typename P> const typename P::S *P_of(Level &L);
template <> const double2 *P_of<PF64>(Level &L) { return L.P64.p; }
template <> const float2 *P_of<PF32>(Level &L) { return L.P32.p; }
template <> const chalf *P_of<PF16>(Level &L) { return L.P16.p; }

// Calls f with the prolongator the transfers of class P read on level L:
// P's own storage, or the binary16 copy in the FP32 class when transfer_prec
// is MG_F16.  f returns the same type for every storage.
template <typename P, typename F> static auto with_transfer_P(const mg_ctx *c, Level &L, F &&f) {
  if constexpr (std::is_same<P, PF32>::value) {
    if (c->p.transfer_prec == MG_F16) return f(P_of<PF16>(L));
  }
  return f(P_of<P>(L));
}
// identifies the transfers' P storage in the process-wide tuning cache
template <typename P> static int transfer_store_id(const mg_ctx *c) {
  return (std::is_same<P, PF32>::value && c->p.transfer_prec == MG_F16) ? 3 : P::id;
}
template <typename T> using stor_t = std::remove_cv_t<std::remove_pointer_t<T>>;

template <typename P> const typename P::S *links_of_level(Level &L) { return links_of<P>(L); }
template <typename P> const typename P::S *cop_of_level(Level &L) { return cop_of<P>(L); }

// Row-major copy of level l's operator for the matrix-core variants 8 + KS,
// made from the FP64 stencil on first use (nullptr in FP64 or on failure).
template <typename P> const void *cop_t_of(mg_ctx *, Level &, hipStream_t) { return nullptr; }
template <typename S> static const void *make_cop_t(DevBuf<S> &Lt, Level &L, hipStream_t st) {
  if (!Lt.p) {
    if (Lt.alloc(L.L64.n) != MG_OK) return nullptr;
    if (transpose_convert<S>(Lt.p, L.L64.p, L.g.V, L.n, st) != hipSuccess) {
      Lt.release();
      return nullptr;
    }
  }
  return Lt.p;
}
template <> const void *cop_t_of<PF32>(mg_ctx *, Level &L, hipStream_t st) { return make_cop_t(L.L32t, L, st); }
template <> const void *cop_t_of<PF16>(mg_ctx *, Level &L, hipStream_t st) { return make_cop_t(L.L16t, L, st); }
template const double2 *links_of_level<PF64>(Level &);
template const float2 *links_of_level<PF32>(Level &);
template const chalf *links_of_level<PF16>(Level &);
template const double2 *cop_of_level<PF64>(Level &);
template const float2 *cop_of_level<PF32>(Level &);
template const chalf *cop_of_level<PF16>(Level &);
template <typename P> const void *cop_t_of_level(mg_ctx *c, Level &L, hipStream_t st) {
  return cop_t_of<P>(c, L, st);
}
template const void *cop_t_of_level<PF64>(mg_ctx *, Level &, hipStream_t);
template const void *cop_t_of_level<PF32>(mg_ctx *, Level &, hipStream_t);
template const void *cop_t_of_level<PF16>(mg_ctx *, Level &, hipStream_t);

int np_mr(mg_ctx *c, int l, int nrhs) {
  return l == 0 ? dslash_partials(c->lev[0].g, nrhs) : (int)np_coarse(c->lev[l]);
}

// kernel-class index of the timers: 2 * precision id + (coarse ? 1 : 0)
template <typename P> constexpr int tclass(bool coarse) { return 2 * P::id + (coarse ? 1 : 0); }

// Records a (start, stop) event pair around the launches in its scope when
// timing is on.  With timing on the solver runs its launches eagerly (the
// runtime refuses event records inside a stream capture), so a scope never
// sits inside a capture; should one, it records nothing.
struct TimerScope {
  EventTimer *t = nullptr;
  hipEvent_t e1 = nullptr;
  hipStream_t st;
  TimerScope(mg_ctx *c, EventTimer &tm, hipStream_t s, double sites, bool sample = true, int nlaunch = 1) : st(s) {
    if (c->timing && sample) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
      hipEvent_t e0 = tm.next();
      e1 = tm.next();
      if (e0 && e1) {
        (void)hipEventRecord(e0, st);
        t = &tm;
        tm.pair_sites.push_back(sites);
        tm.pair_launches.push_back(nlaunch);
      }
    }
  }
  ~TimerScope() {
    if (t) (void)hipEventRecord(e1, st);
  }
};

// ------------------------------------------------------------ autotuner
// Coarse-stencil variant for (operator size, coarse volume, right-hand
// sides, precision): the per-RHS kernel (0) or the matrix-core GEMM with K
// split 1, 2 or 4.  Each candidate is timed on the level's own operator with
// its partial sums and final reduction, as the CGNR uses it; the fastest is
// kept for the process (shapes, not contexts, decide it).  Never called
// under stream capture.
namespace {
struct TuneKey {
  int n, prec, nrhs;
  uint32_t V;
  bool operator==(const TuneKey &o) const { return n == o.n && prec == o.prec && nrhs == o.nrhs && V == o.V; }
};
struct TuneVal {
  TuneKey k;
  int variant;
  float us;
};
std::mutex tune_mu;
std::vector<TuneVal> tune_cache;
}  // namespace

template <typename P> int coarse_variant(mg_ctx *c, int l, int nrhs, hipStream_t st) {
  using R = typename P::R;
  using S = typename P::S;
  if constexpr (sizeof(R) == 8) {
    return 0;
  } else {
    Level &L = c->lev[l];
    if (c->cvar_force >= 0)
      return (c->cvar_force == 0 || coarse_mma_ok(L.n, nrhs, c->cvar_force)) ? c->cvar_force : 0;
    if (nrhs > MG_MAX_RHS) return 0;  // the matrix-core variants take at most 16
    int &v = c->cvar[l][P::id][nrhs];
    if (v >= 0) return v;
    const TuneKey key{L.n, P::id, nrhs, L.g.V};
    {
      std::lock_guard<std::mutex> lk(tune_mu);
      for (const TuneVal &t : tune_cache)
        if (t.k == key) {
          v = t.variant;
          c->cvar_us[l][P::id][nrhs] = t.us;
          return v;
        }
    }
    const size_t nn = L.vsize() * nrhs;
    DevBuf<float2> a, b;
    MG_TRY(a.alloc(nn));
    MG_TRY(b.alloc(nn));
    MG_TRY(ensure_scalars(c, part_need(c, nrhs)));
    HIPK(fill_const<float>(a, nn, 1.0f, st));
    hipEvent_t e0, e1;
    HIPK(hipEventCreate(&e0));
    HIPK(hipEventCreate(&e1));
    int best = 0;
    float best_t = 1e30f;
    const int cands[7] = {0, 1, 2, 4, 9, 10, 12};
    int rc = MG_OK;
    for (int ci = 0; ci < 7 && rc == MG_OK; ++ci) {
      const int cv = cands[ci];
      if (cv > 0 && !coarse_mma_ok(L.n, nrhs, cv)) continue;
      CoarseArgs ca;
      ca.part = c->part;
      ca.pw = 1;
      ca.variant = cv;
      if (cv >= 8 && (ca.lt = cop_t_of<P>(c, L, st)) == nullptr) continue;
      const int reps = 8;
      for (int i = 0; i < 2 + reps && rc == MG_OK; ++i) {
        if (i == 2) rc = hip_rc(hipEventRecord(e0, st), "hipEventRecord");
        if (rc == MG_OK)
          rc = hip_rc((coarse_apply_k<R, S>(L.g, L.n, cop_of<P>(L), a.p, b.p, nrhs, 0, ca, st)), "coarse tune");
      }
      if (rc == MG_OK) rc = hip_rc(hipEventRecord(e1, st), "hipEventRecord");
      if (rc == MG_OK) rc = hip_rc(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      if (rc == MG_OK) rc = hip_rc(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      const float us = ms * 1e3f / reps;
      if (rc == MG_OK && us < best_t) {
        best_t = us;
        best = cv;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    MG_TRY(rc);
    v = best;
    c->cvar_us[l][P::id][nrhs] = best_t;
    std::lock_guard<std::mutex> lk(tune_mu);
    tune_cache.push_back(TuneVal{key, best, best_t});
    return v;
  }
}

namespace {
struct TKey {
  uint32_t V, vb;
  int nv, prec, nrhs, dir;
  bool operator==(const TKey &o) const {
    return V == o.V && vb == o.vb && nv == o.nv && prec == o.prec && nrhs == o.nrhs && dir == o.dir;
  }
};
struct TVal {
  TKey k;
  int variant;
  float us[2];
};
std::vector<TVal> ttune_cache;
}  // namespace

// Fine-level transfer kernel for (direction dir: 0 restriction, 1
// prolongation; nrhs): the vector kernels (0) or the matrix-core GEMM (1),
// timed once per shape on first use and kept for the process.
template <typename P> int transfer_variant(mg_ctx *c, int dir, int nrhs, hipStream_t st) {
  using R = typename P::R;
  if constexpr (sizeof(R) == 8) {
    return 0;
  } else {
    Level &L = c->lev[0], &Lc = c->lev[1];
    if (nrhs < 2 || nrhs > MG_MAX_RHS || !transfer_mma_ok(L.g, L.nv, nrhs)) return 0;
    if (c->tvar_force >= 0) return c->tvar_force > 0 ? 1 : 0;
    int &v = c->tvar[dir][P::id][nrhs];
    if (v >= 0) return v;
    const TKey key{L.g.V, L.g.vb, L.nv, transfer_store_id<P>(c), nrhs, dir};
    {
      std::lock_guard<std::mutex> lk(tune_mu);
      for (const TVal &t : ttune_cache)
        if (t.k == key) {
          v = t.variant;
          c->tvar_us[dir][P::id][nrhs][0] = t.us[0];
          c->tvar_us[dir][P::id][nrhs][1] = t.us[1];
          return v;
        }
    }
    DevBuf<float2> a, b;
    MG_TRY(a.alloc(L.vsize() * nrhs));
    MG_TRY(b.alloc(Lc.vsize() * nrhs));
    HIPK(fill_const<float>(a, L.vsize() * nrhs, 1.0f, st));
    HIPK(fill_const<float>(b, Lc.vsize() * nrhs, 1.0f, st));
    hipEvent_t e0, e1;
    HIPK(hipEventCreate(&e0));
    HIPK(hipEventCreate(&e1));
    int best = 0, rc = MG_OK;
    float best_t = 1e30f, t_us[2] = {0.f, 0.f};
    for (int cv = 0; cv < 2 && rc == MG_OK; ++cv) {
      const int reps = 6;
      for (int i = 0; i < 2 + reps && rc == MG_OK; ++i) {
        if (i == 2) rc = hip_rc(hipEventRecord(e0, st), "hipEventRecord");
        hipError_t e;
        e = with_transfer_P<P>(c, L, [&](auto Pp) -> hipError_t {
          using SS = stor_t<decltype(Pp)>;
          if (dir == 0)
            return cv ? restrict_fine_mma<SS, float2>(L.g, Lc.g, L.nv, Pp, a.p, b.p, nrhs, st)
                      : restrict_fine<R, SS, float2>(L.g, Lc.g, L.nv, Pp, a.p, b.p, nrhs, st);
          return cv ? prolong_fine_mma<SS>(L.g, Lc.g, L.nv, Pp, b.p, a.p, nrhs, 1, st)
                    : prolong_fine<R, SS>(L.g, Lc.g, L.nv, Pp, b.p, a.p, nrhs, 1, st);
        });
        if (rc == MG_OK) rc = hip_rc(e, "transfer tune");
      }
      if (rc == MG_OK) rc = hip_rc(hipEventRecord(e1, st), "hipEventRecord");
      if (rc == MG_OK) rc = hip_rc(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      if (rc == MG_OK) rc = hip_rc(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      const float us = ms * 1e3f / reps;
      t_us[cv] = us;
      if (rc == MG_OK && us < best_t) {
        best_t = us;
        best = cv;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    MG_TRY(rc);
    v = best;
    c->tvar_us[dir][P::id][nrhs][0] = t_us[0];
    c->tvar_us[dir][P::id][nrhs][1] = t_us[1];
    std::lock_guard<std::mutex> lk(tune_mu);
    ttune_cache.push_back(TVal{key, best, {t_us[0], t_us[1]}});
    return v;
  }
}

// out = D in on the fine level with the input stored as TI and the output
// (and b) as TO (DS_MR: MR partials into c->part; DS_RESID: out = b - D in).
template <typename P, typename TI, typename TO>
static int apply_fine(mg_ctx *c, const TI *in, TO *out, int nrhs, DslashMode mode, const TO *b, hipStream_t st,
                      MrqArgs<TO> mq = {}) {
  using R = typename P::R;
  using S = typename P::S;
  Level &L = c->lev[0];
  const int tc = mode == DS_MRQ ? (P::id == 2 ? 9 : 8) : tclass<P>(false);
  TimerScope ts(c, c->tm[tc], st, (double)L.g.V * nrhs);
  HIPK((dslash<R, S, TI, TO>(L.g, links_of<P>(L), L.nl, in, out, b, 4.0 + c->mass, nrhs, mode, c->part, st, mq)));
  c->n_fine += nrhs;
  return MG_OK;
}

// out = A_l in  (DS_MR: MR partials into c->part; DS_RESID: out = b - A_l in)
template <typename P>
int apply_A(mg_ctx *c, int l, const vec_t<P> *in, vec_t<P> *out, int nrhs, DslashMode mode, const vec_t<P> *b,
            hipStream_t st) {
  using R = typename P::R;
  using S = typename P::S;
  Level &L = c->lev[l];
  if (l == 0) {
    MG_TRY((apply_fine<P, vec_t<P>, vec_t<P>>(c, in, out, nrhs, mode, b, st)));
  } else {
    const int var = coarse_variant<P>(c, l, nrhs, st);
    if (var < 0) return var;
    CoarseArgs ca;
    if (mode == DS_MR) {
      ca.part = c->part;
      ca.pw = 3;
    }
    ca.variant = var;
    if (var >= 8) ca.lt = cop_t_of<P>(c, L, st);
    {
      TimerScope ts(c, c->tm[tclass<P>(true)], st, (double)L.g.V * nrhs);
      HIPK((coarse_apply_k<R, S>(L.g, L.n, cop_of<P>(L), in, out, nrhs, 0, ca, st)));
    }
    if (mode == DS_RESID) HIPK(resid_from<R>(out, b, L.vsize(), nrhs, st));
    c->n_coarse += nrhs;
    c->n_coarse_disp += nrhs;
  }
  return MG_OK;
}

// MR smoothing of A_l x = r0 from x = 0 (accumulate: add into x): on return
// r holds the recursively updated residual, unless keep_r = false (the
// caller does not use it; the last step then updates x only).  r0 is r on
// entry, or the separate vector r_in when given (read by the first step,
// which then writes r: no copy of the input).  TR = storage of r and q:
// vec_t<P>, or h16 on the fine level of the FP16 class.
//
// On the fine level of the FP32 and FP16 classes the steps take the q
// recursion when its buffers are there: with q_0 = A r_0, step k forms
// q_k = q_{k-1} - a_{k-1} A q_{k-1} and r_k = r_{k-1} - a_{k-1} q_{k-1} in
// the stencil's epilogue (q_k = A r_k in exact arithmetic), with a_k from
// the partials of (q_k, r_k); x = sum a_k r_k and the last residual update
// follow in one pass.  The same iterates as the update after each stencil,
// without the separate pass over x, r and q per step.
// The step lengths a_k of the fine-level runs sit at csc + MRQ_ABASE +
// k MG_MAX_RHS, apart from the coarse levels' (csc[0 .. nrhs)), so that a
// pre-smoothing whose combine is deferred to the transfers keeps them over
// the coarse-grid correction.
constexpr size_t MRQ_ABASE = 96 * MG_MAX_RHS;

// The residual list r_0 .. r_{steps-1} of a fine-level run from r0, and its
// last q (q_{steps-1}), in the q-recursion buffers (TR: their storage).
template <typename TR> static MrqList<TR> mrq_list(mg_ctx *c, const TR *r0, int steps) {
  MrqList<TR> rs{};
  rs.r[0] = r0;
  for (int k = 1; k < steps; ++k) {
    if constexpr (std::is_same<TR, h16>::value) rs.r[k] = c->w32.hrk[k - 1].p;
    else rs.r[k] = c->w32.rk[k - 1].p;
  }
  return rs;
}
template <typename TR> static TR *mrq_q(mg_ctx *c, TR *q, int k) {
  if ((k & 1) == 0) return q;
  if constexpr (std::is_same<TR, h16>::value) return c->w32.hq2.p;
  else return c->w32.q2.p;
}

// defer: stop after the steps (no combine pass): x and the last residual
// are formed later from the list by the transfers (smooth_pre).
template <typename P, typename TR>
static int mr_q(mg_ctx *c, vec_t<P> *x, TR *r, TR *q, int steps, bool accumulate, int nrhs, hipStream_t st,
                bool keep_r, const TR *r_in, float xs = 1.f, bool defer = false) {
  const int np = np_mr(c, 0, nrhs);
  const MrqList<TR> rs = mrq_list<TR>(c, r_in ? r_in : r, steps);
  double2 *al = c->csc + MRQ_ABASE;
  MG_TRY((apply_fine<P, TR, TR>(c, rs.r[0], q, nrhs, DS_MR, nullptr, st)));
  HIPK(fin_mr(c->part, np, nrhs, c->p.omega, al, st));
  for (int k = 1; k < steps; ++k) {
    MrqArgs<TR> mq;
    mq.rprev = rs.r[k - 1];
    mq.rout = const_cast<TR *>(rs.r[k]);
    mq.alpha = al + (size_t)(k - 1) * MG_MAX_RHS;
    MG_TRY((apply_fine<P, TR, TR>(c, mrq_q<TR>(c, q, k - 1), mrq_q<TR>(c, q, k), nrhs, DS_MRQ, nullptr, st, mq)));
    HIPK(fin_mr(c->part, np, nrhs, c->p.omega, al + (size_t)k * MG_MAX_RHS, st));
  }
  if (defer) return MG_OK;
  HIPK(mrq_combine<TR>(x, r, rs, mrq_q<TR>(c, q, steps - 1), c->lev[0].g, steps, nrhs, al, accumulate ? 0 : 1,
                       keep_r ? 1 : 0, xs, st));
  return MG_OK;
}

// Whether the fine-level MR of `steps` steps on nrhs vectors takes the q
// recursion (TR: storage of r and q).
template <typename TR> static bool mrq_ready(const mg_ctx *c, int l, int steps, int nrhs) {
  const int i = std::is_same<TR, h16>::value ? 1 : 0;
  const Work<float> &w = c->w32;
  return l == 0 && steps >= 2 && steps <= w.mrq_steps[i] && nrhs <= w.mrq_nrhs[i];
}

template <typename P, typename TR = vec_t<P>>
int mr(mg_ctx *c, int l, vec_t<P> *x, TR *r, TR *q, int steps, bool accumulate, int nrhs, hipStream_t st,
       bool keep_r = true, const TR *r_in = nullptr) {
  using R = typename P::R;
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  if constexpr (sizeof(R) == 4) {
    if (mrq_ready<TR>(c, l, steps, nrhs)) return mr_q<P, TR>(c, x, r, q, steps, accumulate, nrhs, st, keep_r, r_in);
  }
  if (steps == 0 && !accumulate) HIPK(zero<R>(x, n * nrhs, st));
  for (int k = 0; k < steps; ++k) {
    const TR *src = (k == 0 && r_in) ? r_in : r;
    const int upd_r = (keep_r || k + 1 < steps) ? 1 : 0;
    const int first = (!accumulate && k == 0) ? 1 : 0;
    if constexpr (std::is_same<TR, h16>::value) {
      MG_TRY((apply_fine<P, h16, h16>(c, src, q, nrhs, DS_MR, nullptr, st)));
      HIPK(mr_update_h(x, r, src, q, L.g, nrhs, c->part, np_mr(c, l, nrhs), c->p.omega, c->csc, first, upd_r, st));
    } else {
      MG_TRY(apply_A<P>(c, l, src, q, nrhs, DS_MR, nullptr, st));
      HIPK(mr_update<R>(x, r, src, q, n, nrhs, c->part, np_mr(c, l, nrhs), c->p.omega, c->csc, first, upd_r, st));
    }
  }
  return MG_OK;
}

// GMRES relaxation of A_l x = b: x (+)= omega y, y the GMRES(k) iterate
// from zero (one cycle), b unchanged.
template <typename P>
int gmres_smooth(mg_ctx *c, int l, vec_t<P> *x, const vec_t<P> *b, int k, bool accumulate, int nrhs,
                 hipStream_t st) {
  using R = typename P::R;
  Work<R> &w = work<R>(c);
  const size_t n = c->lev[l].vsize(), vs = n * nrhs;
  if (k == 0) {
    if (!accumulate) HIPK(zero<R>(x, vs, st));
    return MG_OK;
  }
  vec_t<P> *V = w.gv[l];
  double *nrm2 = c->gmb + MG_MAX_RHS, *beta = c->gmb;
  HIPK(norm2<R>(b, n, nrhs, c->gmp, nrm2, st));
  HIPK(gm_start<R>(V, b, n, nrhs, nrm2, beta, st));
  for (int j = 0; j < k; ++j) {
    MG_TRY(apply_A<P>(c, l, V + (size_t)j * vs, V + (size_t)(j + 1) * vs, nrhs, DS_PLAIN, nullptr, st));
    HIPK(gm_arnoldi_col<R>(V, vs, j, n, nrhs, c->gmH, c->gmp, st));
  }
  HIPK(gm_lsq(c->gmH, beta, k, nrhs, c->gmy, st));
  HIPK(gm_combine<R>(x, V, vs, k, n, nrhs, c->gmy, c->p.omega, accumulate ? 1 : 0, st));
  return MG_OK;
}

template <typename P, typename TR>
int transfer_restrict(mg_ctx *c, int l, const TR *fine, vec_t<P> *coarse, int nrhs, hipStream_t st) {
  using R = typename P::R;
  Level &L = c->lev[l], &Lc = c->lev[l + 1];
  if (l == 0) {
    const int tv = transfer_variant<P>(c, 0, nrhs, st);
    if (tv < 0) return tv;
    HIPK(with_transfer_P<P>(c, L, [&](auto Pp) -> hipError_t {
      using SS = stor_t<decltype(Pp)>;
      if constexpr (sizeof(R) == 4) {
        if (tv == 1) return restrict_fine_mma<SS, TR>(L.g, Lc.g, L.nv, Pp, fine, coarse, nrhs, st);
      }
      return restrict_fine<R, SS, TR>(L.g, Lc.g, L.nv, Pp, fine, coarse, nrhs, st);
    }));
  } else if constexpr (std::is_same<TR, vec_t<P>>::value) {
    HIPK(with_transfer_P<P>(c, L, [&](auto Pp) -> hipError_t {
      return restrict_coarse<R, stor_t<decltype(Pp)>>(L.g, Lc.g, L.n, L.nv, Pp, fine, coarse, nrhs, st);
    }));
  }
  return MG_OK;
}

template <typename P>
int transfer_prolong(mg_ctx *c, int l, const vec_t<P> *coarse, vec_t<P> *fine, int nrhs, int accumulate,
                     hipStream_t st) {
  using R = typename P::R;
  Level &L = c->lev[l], &Lc = c->lev[l + 1];
  if (l == 0) {
    const int tv = transfer_variant<P>(c, 1, nrhs, st);
    if (tv < 0) return tv;
    HIPK(with_transfer_P<P>(c, L, [&](auto Pp) -> hipError_t {
      using SS = stor_t<decltype(Pp)>;
      if constexpr (sizeof(R) == 4) {
        if (tv == 1) return prolong_fine_mma<SS>(L.g, Lc.g, L.nv, Pp, coarse, fine, nrhs, accumulate, st);
      }
      return prolong_fine<R, SS>(L.g, Lc.g, L.nv, Pp, coarse, fine, nrhs, accumulate, st);
    }));
  } else {
    HIPK(with_transfer_P<P>(c, L, [&](auto Pp) -> hipError_t {
      return prolong_coarse<R, stor_t<decltype(Pp)>>(L.g, Lc.g, L.n, L.nv, Pp, coarse, fine, nrhs, accumulate, st);
    }));
  }
  return MG_OK;
}

// CGNR on A^dag A e = A^dag b (coarsest level), A^dag = sigma3 A sigma3,
// stopping at ||b - A e|| <= tol ||b|| (recursive residual) or after
// coarse_maxiter iterations.  Four launches per iteration and no host round
// trip: w = A p (partials ||w||^2); update of e and r with alpha from the
// partials (partials ||r||^2); convergence test fused into z = A^dag r
// (partials ||z||^2); p = z + beta p.  Iterations run in chunks of CG_CHUNK
// (captured once into a hipGraph when enabled); the host reads the done flags
// of one chunk while the next is already queued, and kernels of converged
// right-hand sides return at once.
struct CgPtrs {
  double *pw, *pz[2], *pr, *pb;
};
static CgPtrs cg_ptrs(mg_ctx *c, int l, int nrhs) {
  const size_t stride = np_coarse(c->lev[l]) * nrhs;
  CgPtrs q;
  q.pw = c->cgp;
  q.pz[0] = c->cgp + stride;
  q.pz[1] = c->cgp + 2 * stride;
  q.pr = c->cgp + 3 * stride;
  q.pb = q.pr + (size_t)RED_BLOCKS * nrhs;
  return q;
}

template <typename P>
int cgnr_chunk(mg_ctx *c, int l, vec_t<P> *e, int nrhs, int var, bool fused, hipStream_t st, EventTimer &tm) {
  using R = typename P::R;
  using S = typename P::S;
  Work<R> &w = work<R>(c);
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  const double sites = (double)L.g.V * nrhs;
  c_t<R> *r = w.cr, *z = w.cz, *p = w.cp, *ww = w.cw;
  const S *Lop = cop_of<P>(L);
  const CgPtrs q = cg_ptrs(c, l, nrhs);
  const int npc = (int)np_coarse(L);
  if (fused) {
    // Two launches per iteration: w = A p with p = z + beta p_old formed
    // while staging (and the convergence test of the previous update), then
    // z = A^dag r with r = r_old - alpha w formed while staging (and e +=
    // alpha p).  p and r alternate between two buffers by iteration parity.
    c_t<R> *Pb[2] = {w.cp, w.cp2}, *Rb[2] = {w.cr, w.cr2};
    // the chunk is 2 CG_CHUNK consecutive stencil launches: one event pair
    // times them all
    TimerScope ts(c, tm, st, sites * 2 * CG_CHUNK, true, 2 * CG_CHUNK);
    for (int k = 0; k < CG_CHUNK; ++k) {
      CgCheck chk;
      chk.part_r = q.pr;
      chk.np_r = npc;
      chk.cg = c->cg;
      chk.done = c->done;
      chk.it_in = c->it + (size_t)(k & 1) * nrhs;
      chk.it_out = c->it + (size_t)((k + 1) & 1) * nrhs;
      chk.maxit = c->p.coarse_maxiter;
      chk.fused = 1;
      CgFuse f1;
      f1.kind = 1;
      f1.a = z;
      f1.b = Pb[(k + 1) & 1];
      f1.own = Pb[k & 1];
      f1.num = q.pz[k & 1];
      f1.den = q.pz[(k + 1) & 1];
      f1.np = npc;
      f1.it0 = chk.it_in;
      CoarseArgs ca;
      ca.part = q.pw;
      ca.done = c->done;
      ca.chk = &chk;
      ca.fuse = &f1;
      HIPK((coarse_apply_k<R, S>(L.g, L.n, Lop, z, ww, nrhs, 0, ca, st)));
      CgFuse f2;
      f2.kind = 2;
      f2.a = Rb[k & 1];
      f2.b = ww;
      f2.own = Rb[(k + 1) & 1];
      f2.e = e;
      f2.p = Pb[k & 1];
      f2.num = q.pz[k & 1];
      f2.den = q.pw;
      f2.np = npc;
      f2.part_own = q.pr;
      f2.done_w = c->done;
      CoarseArgs cb;
      cb.part = q.pz[(k + 1) & 1];
      cb.done = c->done;
      cb.fuse = &f2;
      HIPK((coarse_apply_k<R, S>(L.g, L.n, Lop, Rb[k & 1], z, nrhs, 1, cb, st)));
    }
    return MG_OK;
  }
  for (int k = 0; k < CG_CHUNK; ++k) {
    CoarseArgs ca;
    ca.part = q.pw;
    ca.done = c->done;
    ca.variant = var;
    if (var >= 8) ca.lt = cop_t_of<P>(c, L, st);
    {
      TimerScope ts(c, tm, st, sites, k == 0);
      HIPK((coarse_apply_k<R, S>(L.g, L.n, Lop, p, ww, nrhs, 0, ca, st)));
    }
    const int npr = cg2_update<R>(e, p, r, ww, n, nrhs, q.pw, q.pz[k & 1], npc, c->done, q.pr, st);
    HIPK(hipGetLastError());
    CgCheck chk;
    chk.part_r = q.pr;
    chk.np_r = npr;
    chk.cg = c->cg;
    chk.done = c->done;
    chk.it_in = c->it + (size_t)(k & 1) * nrhs;
    chk.it_out = c->it + (size_t)((k + 1) & 1) * nrhs;
    chk.maxit = c->p.coarse_maxiter;
    ca.part = q.pz[(k + 1) & 1];
    ca.chk = &chk;
    {
      TimerScope ts(c, tm, st, sites, k == 0);
      HIPK((coarse_apply_k<R, S>(L.g, L.n, Lop, r, z, nrhs, 1, ca, st)));
    }
    HIPK(cg2_p<R>(p, z, n, nrhs, q.pz[(k + 1) & 1], q.pz[k & 1], npc, c->done, st));
  }
  return MG_OK;
}

template <typename P>
ChunkGraph *chunk_graph(mg_ctx *c, int l, vec_t<P> *e, int nrhs, int var, bool fused, hipStream_t st) {
  const int prec = P::id;
  for (ChunkGraph *g : c->graphs)
    if (g && g->level == l && g->prec == prec && g->nrhs == nrhs && g->variant == var && g->fused == (int)fused)
      return g;
  ChunkGraph *g = new ChunkGraph();
  g->level = l;
  g->prec = prec;
  g->nrhs = nrhs;
  g->variant = var;
  g->fused = fused ? 1 : 0;
  EventTimer unused;
  bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) == hipSuccess;
  if (ok) {
    const int rc = cgnr_chunk<P>(c, l, e, nrhs, var, fused, st, unused);
    ok = hipStreamEndCapture(st, &g->graph) == hipSuccess && rc == MG_OK;
  }
  if (ok) ok = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    delete g;
    return nullptr;
  }
  for (auto &slot : c->graphs)
    if (!slot) {
      slot = g;
      return g;
    }
  delete c->graphs[0];
  c->graphs[0] = g;
  return g;
}

// The iterations of the fused CGNR of one right-hand side as one cooperative
// launch (FP32 arithmetic, same arithmetic and iteration count as the chunked
// path), from the state the chunks start from.  ran = false, and nothing is
// launched, when the shape or the device cannot take it; the caller then
// runs the chunks.
template <typename P>
int cgnr_whole(mg_ctx *c, int l, vec_t<P> *e, hipStream_t st, bool &ran, bool &retry) {
  ran = false;
  retry = false;
  using R = typename P::R;
  if constexpr (sizeof(R) == 8) {
    return MG_OK;
  } else {
    using S = typename P::S;
    const int pc = P::id;
    if (c->cgp_off[l][pc]) return MG_OK;
    Level &L = c->lev[l];
    Work<R> &w = work<R>(c);
    const CgPtrs q = cg_ptrs(c, l, 1);
    if (c->cgp_bar.n == 0) {
      MG_TRY(c->cgp_bar.alloc(CGP_BAR_WORDS));
      MG_TRY(c->cgp_fail.alloc(1));
    }
    HIPK(hipMemsetAsync(c->cgp_bar, 0, sizeof(unsigned) * CGP_BAR_WORDS, st));
    HIPK(hipMemsetAsync(c->cgp_fail, 0, sizeof(int), st));
    CgPersist a;
    a.e = e;
    a.z = w.cz;
    a.w = w.cw;
    a.p[0] = w.cp;
    a.p[1] = w.cp2;
    a.r[0] = w.cr;
    a.r[1] = w.cr2;
    a.pz[0] = q.pz[0];
    a.pz[1] = q.pz[1];
    a.pw = q.pw;
    a.pr = q.pr;
    a.cg = c->cg;
    a.it = c->it;
    a.done = c->done;
    a.maxit = c->p.coarse_maxiter;
    a.bar = c->cgp_bar;
    a.fail = c->cgp_fail;
    a.spin = c->cgp_spin;
    EventTimer &tw = c->tm[P::id == 2 ? 7 : 6];  // whole-solve CGNR classes
    const size_t npairs = tw.pair_launches.size();
    hipError_t err;
    {
      TimerScope ts(c, tw, st, (double)L.g.V * 2, true, 1);
      err = cgnr_persistent<S>(L.g, L.n, cop_of<P>(L), a, st);
    }
    if (err != hipSuccess) {
      // not launched: this shape or device takes the chunked path from now on
      (void)hipGetLastError();
      c->cgp_off[l][pc] = 1;
      if (tw.pair_launches.size() > npairs) {  // drop the unused event pair
        tw.pair_launches.pop_back();
        tw.pair_sites.pop_back();
        tw.used -= 2;
      }
      return MG_OK;
    }
    ran = true;
    HIPK(hipMemcpyAsync(c->h_it, c->it, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
    HIPK(hipMemcpyAsync(c->h_done, c->cgp_fail, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPK(hipStreamSynchronize(st));
    if (c->h_done[0]) {
      // a barrier wait gave up (the grid was not all resident at once, e.g.
      // beside other work on the device): this (level, precision) takes the
      // chunks from now on, and the caller solves again from b with them
      c->cgp_off[l][pc] = 1;
      c->n_cg_fallback += 1;
      ran = false;
      retry = true;
      return MG_OK;
    }
    const long it = std::max(c->h_it[0], c->h_it[1]);
    c->n_cgnr += it;
    // the initial application before the launch, then those inside it
    // (applications, not dispatches)
    c->n_coarse += 1 + 2L * it;
    c->n_coarse_disp += 1;
    if (tw.pair_launches.size() > npairs)  // the launch made 2 it stencil applications
      tw.pair_sites.back() = (double)L.g.V * (double)(2L * it);
    return MG_OK;
  }
}

template <typename P> int cgnr(mg_ctx *c, int l, const vec_t<P> *b, vec_t<P> *e, int nrhs, hipStream_t st) {
  using R = typename P::R;
  using S = typename P::S;
  Work<R> &w = work<R>(c);
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  const CgPtrs q = cg_ptrs(c, l, nrhs);
  EventTimer &tm = c->tm[tclass<P>(true)];
  const int var = coarse_variant<P>(c, l, nrhs, st);
  if (var < 0) return var;
  // Fused updates when the per-RHS stencil runs and every workgroup can sum
  // the V partials of the step lengths cheaply.
  const bool fused = var == 0 && L.g.V <= (uint32_t)CG_FUSE_MAXV;
  HIPK(zero<R>(e, n * nrhs, st));
  HIPK(copy<R>(w.cr, b, n * nrhs, st));
  if (fused) HIPK(zero<R>(w.cp2, n * nrhs, st));
  const int npb = norm2_partials<R>(b, n, nrhs, q.pb, st);
  HIPK(cg2_init(q.pb, npb, nrhs, c->cg, c->done, c->it, c->p.coarse_tol, st));
  {
    CoarseArgs ca;
    ca.part = q.pz[0];
    ca.done = c->done;
    ca.variant = var;
    if (var >= 8) ca.lt = cop_t_of<P>(c, L, st);
    TimerScope ts(c, tm, st, (double)L.g.V * nrhs);
    HIPK((coarse_apply_k<R, S>(L.g, L.n, cop_of<P>(L), w.cr, w.cz, nrhs, 1, ca, st)));
  }
  if (!fused) HIPK(copy<R>(w.cp, w.cz, n * nrhs, st));
  if (fused && nrhs == 1 && c->cg_persist) {
    bool ran = false, retry = false;
    MG_TRY(cgnr_whole<P>(c, l, e, st, ran, retry));
    if (ran) return MG_OK;
    if (retry) return cgnr<P>(c, l, b, e, nrhs, st);
  }
  // Captured chunks (not with timing on: event records cannot be captured)
  ChunkGraph *gph = (c->use_graph && !c->timing) ? chunk_graph<P>(c, l, e, nrhs, var, fused, st) : nullptr;
  const int nchunks = (c->p.coarse_maxiter + CG_CHUNK - 1) / CG_CHUNK;
  c->n_coarse_disp += nrhs;  // the initial application above
  int last = 0;
  for (int ch = 0; ch < nchunks; ++ch) {
    last = ch;
    if (gph) HIPK(hipGraphLaunch(gph->exec, st));
    else MG_TRY(cgnr_chunk<P>(c, l, e, nrhs, var, fused, st, tm));
    c->n_coarse_disp += 2L * CG_CHUNK * nrhs;
    int *hd = c->h_done + (size_t)(ch & 1) * MG_MAX_RHS;
    HIPK(hipMemcpyAsync(hd, c->done, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    HIPK(hipEventRecord(c->ev_chunk[ch & 1], st));
    const int look = ch - 1;  // one chunk stays queued ahead of the host's check
    if (look < 0) continue;
    HIPK(hipEventSynchronize(c->ev_chunk[look & 1]));
    const int *hl = c->h_done + (size_t)(look & 1) * MG_MAX_RHS;
    bool all = true;
    for (int i = 0; i < nrhs; ++i) all = all && hl[i];
    if (all) break;
  }
  HIPK(hipMemcpyAsync(c->h_it, c->it, sizeof(int) * 2 * nrhs, hipMemcpyDeviceToHost, st));
  HIPK(hipStreamSynchronize(st));
  for (int i = 0; i < nrhs; ++i) {
    const long it = std::max(c->h_it[i], c->h_it[nrhs + i]);
    c->n_cgnr += it;
    c->n_coarse += 1 + 2L * it;
  }
  return MG_OK;
}

// The smoother's residual and stencil-output buffers of level l, stored as
// TR (binary16 ones exist on the fine level of the FP16 class only).
template <typename P, typename TR> static void res_bufs(mg_ctx *c, int l, TR *&r, TR *&q) {
  if constexpr (std::is_same<TR, h16>::value) {
    r = c->w32.hr;
    q = c->w32.hq;
  } else {
    Work<typename P::R> &w = work<typename P::R>(c);
    r = w.r[l];
    q = w.q[l];
  }
}

// dst = src for residual-type vectors of level l.
template <typename P, typename TR>
static int copy_res(mg_ctx *c, int l, TR *dst, const TR *src, int nrhs, hipStream_t st) {
  if constexpr (std::is_same<TR, h16>::value) HIPK(copy_h16(dst, src, c->lev[0].g.Vpad, nrhs, st));
  else HIPK(copy<typename P::R>(dst, src, c->lev[l].vsize() * nrhs, st));
  return MG_OK;
}

// v as a vec_t<P> vector (binary16 fine vectors are expanded into the FP32
// work vector r of level 0, which the FP16 class does not use otherwise).
template <typename P, typename TR>
static const vec_t<P> *as_vec(mg_ctx *c, const TR *v, int nrhs, hipStream_t st, int &rc) {
  rc = MG_OK;
  if constexpr (std::is_same<TR, h16>::value) {
    float2 *o = c->w32.r[0];
    const hipError_t e = from_h16<float2>(o, v, c->lev[0].g.Vpad, nrhs, st);
    if (e != hipSuccess) rc = hip_rc(e, "from_h16");
    return o;
  } else {
    return v;
  }
}

// r = b - A_l x with r and b stored as TR.
template <typename P, typename TR>
static int resid(mg_ctx *c, int l, const vec_t<P> *x, TR *r, const TR *b, int nrhs, hipStream_t st) {
  if constexpr (std::is_same<TR, h16>::value) return apply_fine<P, vec_t<P>, h16>(c, x, r, nrhs, DS_RESID, b, st);
  else return apply_A<P>(c, l, x, r, nrhs, DS_RESID, b, st);
}

// Whether the pre-smoothing of level l leaves its combine pass to the
// transfers: on the fine level of the FP32 and FP16 classes with MR of two
// or more steps by the q recursion and the matrix-core restriction and
// prolongation chosen for nrhs.  The restriction then forms the last
// residual r_{n-1} - a_{n-1} q_{n-1} as it loads it, and the prolongation
// adds sum a_k r_k to P e_c as it stores x; x and the residual are not
// written in between (one pass over 4 + 2 vectors fewer, three more reads
// inside the transfers).  A pure function of the configuration and the
// tuned variants, so the two halves of a captured cycle agree.
template <typename P, typename TR> static int pre_fused(mg_ctx *c, int l, int nrhs, hipStream_t st, bool &on) {
  on = false;
  if constexpr (sizeof(typename P::R) == 4) {
    if (l != 0 || c->p.smoother == MG_SMOOTH_GMRES || !mrq_ready<TR>(c, 0, c->p.pre, nrhs)) return MG_OK;
    const int tr = transfer_variant<P>(c, 0, nrhs, st);
    if (tr < 0) return tr;
    const int tp = transfer_variant<P>(c, 1, nrhs, st);
    if (tp < 0) return tp;
    on = tr == 1 && tp == 1;
  }
  return MG_OK;
}

// The restriction of the residual smooth_pre left on level l (its deferred
// form when pre_fused).
template <typename P, typename TR>
static int restrict_pre(mg_ctx *c, int l, const TR *r, vec_t<P> *coarse, int nrhs, hipStream_t st) {
  if constexpr (sizeof(typename P::R) == 4) {
    bool fused;
    MG_TRY((pre_fused<P, TR>(c, l, nrhs, st, fused)));
    if (fused) {
      const int n = c->p.pre;
      Level &L = c->lev[0], &Lc = c->lev[1];
      TR *r0, *q0;
      res_bufs<P, TR>(c, 0, r0, q0);
      const MrqList<TR> rs = mrq_list<TR>(c, r0, n);
      HIPK(with_transfer_P<P>(c, L, [&](auto Pp) -> hipError_t {
        return restrict_fine_mma<stor_t<decltype(Pp)>, TR>(L.g, Lc.g, L.nv, Pp, rs.r[n - 1], coarse, nrhs, st,
                                                           mrq_q<TR>(c, q0, n - 1),
                                                           c->csc + MRQ_ABASE + (size_t)(n - 1) * MG_MAX_RHS);
      }));
      return MG_OK;
    }
  }
  return transfer_restrict<P, TR>(c, l, r, coarse, nrhs, st);
}

// Smoothing before the coarse correction on level l (x from zero, r the
// residual left for restriction).
template <typename P, typename TR>
static int smooth_pre(mg_ctx *c, int l, const TR *rin, vec_t<P> *x, int nrhs, hipStream_t st) {
  using R = typename P::R;
  const size_t n = c->lev[l].vsize();
  TR *r, *q;
  res_bufs<P, TR>(c, l, r, q);
  if (c->p.smoother != MG_SMOOTH_GMRES && c->p.pre > 0) {
    if constexpr (sizeof(R) == 4) {
      bool fused;
      MG_TRY((pre_fused<P, TR>(c, l, nrhs, st, fused)));
      if (fused) return mr_q<P, TR>(c, x, r, q, c->p.pre, false, nrhs, st, true, rin, 1.f, true);
    }
    MG_TRY((mr<P, TR>(c, l, x, r, q, c->p.pre, false, nrhs, st, true, rin)));
  } else if (c->p.smoother == MG_SMOOTH_GMRES && c->p.pre > 0) {
    int rc;
    const vec_t<P> *b = as_vec<P, TR>(c, rin, nrhs, st, rc);
    MG_TRY(rc);
    MG_TRY(gmres_smooth<P>(c, l, x, b, c->p.pre, false, nrhs, st));
    MG_TRY((resid<P, TR>(c, l, x, r, rin, nrhs, st)));
  } else {
    HIPK(zero<R>(x, n * nrhs, st));
    MG_TRY((copy_res<P, TR>(c, l, r, rin, nrhs, st)));
  }
  return MG_OK;
}

// After the coarse correction of level l: x += P e_c, the new residual, and
// the post-smoothing added into x.
template <typename P, typename TR>
static int smooth_post(mg_ctx *c, int l, const TR *rin, vec_t<P> *x, int nrhs, hipStream_t st) {
  using R = typename P::R;
  Work<R> &w = work<R>(c);
  TR *r, *q;
  res_bufs<P, TR>(c, l, r, q);
  bool fused = false;
  if constexpr (sizeof(R) == 4) MG_TRY((pre_fused<P, TR>(c, l, nrhs, st, fused)));
  if (fused) {
    if constexpr (sizeof(R) == 4) {
      // x = P e_c + sum a_k r_k of the deferred pre-smoothing
      Level &L = c->lev[0], &Lc = c->lev[1];
      const MrqList<TR> rs = mrq_list<TR>(c, rin, c->p.pre);
      HIPK(with_transfer_P<P>(c, L, [&](auto Pp) -> hipError_t {
        return prolong_fine_mma<stor_t<decltype(Pp)>, TR>(L.g, Lc.g, L.nv, Pp, w.x[1], x, nrhs, 0, st, &rs,
                                                          c->p.pre, c->csc + MRQ_ABASE);
      }));
    }
  } else {
    MG_TRY(transfer_prolong<P>(c, l, w.x[l + 1], x, nrhs, 1, st));
  }
  MG_TRY((resid<P, TR>(c, l, x, r, rin, nrhs, st)));
  if (c->p.smoother == MG_SMOOTH_GMRES) {
    int rc;
    const vec_t<P> *b = as_vec<P, TR>(c, r, nrhs, st, rc);
    MG_TRY(rc);
    MG_TRY(gmres_smooth<P>(c, l, x, b, c->p.post, true, nrhs, st));
  } else {
    MG_TRY((mr<P, TR>(c, l, x, r, q, c->p.post, true, nrhs, st, false)));
  }
  return MG_OK;
}

// The two fixed launch sequences of a V-cycle from level 0: part 0 runs
// smooth_pre and the restriction on every level down to the coarsest, part
// 1 smooth_post on every level back up.
template <typename P>
static int vcycle_part(mg_ctx *c, int part, const fres_t<P> *rin0, vec_t<P> *x0, int nrhs, hipStream_t st) {
  using R = typename P::R;
  using TR = fres_t<P>;
  Work<R> &w = work<R>(c);
  const int top = c->nlev - 2;
  if (part == 0) {
    TR *r0, *q0;
    res_bufs<P, TR>(c, 0, r0, q0);
    MG_TRY((smooth_pre<P, TR>(c, 0, rin0, x0, nrhs, st)));
    MG_TRY((restrict_pre<P, TR>(c, 0, r0, w.rin[1], nrhs, st)));
    for (int l = 1; l <= top; ++l) {
      MG_TRY((smooth_pre<P, vec_t<P>>(c, l, w.rin[l], w.x[l], nrhs, st)));
      MG_TRY((transfer_restrict<P, vec_t<P>>(c, l, w.r[l], w.rin[l + 1], nrhs, st)));
    }
  } else {
    for (int l = top; l >= 1; --l) MG_TRY((smooth_post<P, vec_t<P>>(c, l, w.rin[l], w.x[l], nrhs, st)));
    MG_TRY((smooth_post<P, TR>(c, 0, rin0, x0, nrhs, st)));
  }
  return MG_OK;
}

// Runs one part of the V-cycle from a captured graph: the first time a key
// is seen the part runs eagerly, the second time it is captured (and the
// graph launched), later it is replayed.
template <typename P>
static int vcycle_part_graphed(mg_ctx *c, int part, const fres_t<P> *rin0, vec_t<P> *x0, int nrhs,
                               hipStream_t st) {
  VGraph *g = nullptr;
  for (VGraph *v : c->vgraphs)
    if (v->prec == P::id && v->nrhs == nrhs && v->part == part && v->rin == rin0 && v->x == x0) {
      g = v;
      break;
    }
  if (!g) {
    if ((int)c->vgraphs.size() >= VGRAPH_MAX) clear_graphs(c);
    g = new VGraph();
    g->prec = P::id;
    g->nrhs = nrhs;
    g->part = part;
    g->rin = rin0;
    g->x = x0;
    c->vgraphs.push_back(g);
    return vcycle_part<P>(c, part, rin0, x0, nrhs, st);
  }
  if (g->state == 0) {
    const long f0 = c->n_fine, c0 = c->n_coarse, d0 = c->n_coarse_disp;
    bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) == hipSuccess;
    int rc = MG_OK;
    if (ok) {
      rc = vcycle_part<P>(c, part, rin0, x0, nrhs, st);
      ok = hipStreamEndCapture(st, &g->graph) == hipSuccess && rc == MG_OK;
    }
    if (ok) ok = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) == hipSuccess;
    // the capture launched nothing: its launches run below, by the graph or
    // eagerly, and are counted there
    g->dfine = c->n_fine - f0;
    g->dcoarse = c->n_coarse - c0;
    g->ddisp = c->n_coarse_disp - d0;
    c->n_fine = f0;
    c->n_coarse = c0;
    c->n_coarse_disp = d0;
    if (!ok) {
      // the part runs eagerly from now on (an error it meets there is reported)
      (void)hipGetLastError();
      if (g->graph) (void)hipGraphDestroy(g->graph);
      g->graph = nullptr;
      g->state = -1;
    } else {
      g->state = 1;
    }
  }
  if (g->state < 0) return vcycle_part<P>(c, part, rin0, x0, nrhs, st);
  HIPK(hipGraphLaunch(g->exec, st));
  c->n_fine += g->dfine;
  c->n_coarse += g->dcoarse;
  c->n_coarse_disp += g->ddisp;
  return MG_OK;
}

// One V-cycle K_l(rin) -> x (levels l..coarsest), rin stored as TR (fres_t
// on level 0, vec_t below).
template <typename P, typename TR>
static int vcycle_t(mg_ctx *c, int l, const TR *rin, vec_t<P> *x, int nrhs, hipStream_t st) {
  using R = typename P::R;
  if constexpr (std::is_same<TR, vec_t<P>>::value) {
    if (l == c->nlev - 1) return cgnr<P>(c, l, rin, x, nrhs, st);
  }
  Work<R> &w = work<R>(c);
  if constexpr (std::is_same<TR, fres_t<P>>::value) {
    if (l == 0 && c->vgraph_on && c->use_graph && !c->timing && c->p.cycles <= 1) {
      const int lc = c->nlev - 1;
      MG_TRY(vcycle_part_graphed<P>(c, 0, rin, x, nrhs, st));
      MG_TRY(cgnr<P>(c, lc, w.rin[lc], w.x[lc], nrhs, st));
      return vcycle_part_graphed<P>(c, 1, rin, x, nrhs, st);
    }
  }
  MG_TRY((smooth_pre<P, TR>(c, l, rin, x, nrhs, st)));
  const int m = l + 1;
  TR *r, *q;
  res_bufs<P, TR>(c, l, r, q);
  MG_TRY((restrict_pre<P, TR>(c, l, r, w.rin[m], nrhs, st)));
  MG_TRY((vcycle_t<P, vec_t<P>>(c, m, w.rin[m], w.x[m], nrhs, st)));
  if (m < c->nlev - 1) {
    // W-cycle: further cycles of level m on the residual the previous left
    for (int cyc = 1; cyc < c->p.cycles; ++cyc) {
      MG_TRY(apply_A<P>(c, m, w.x[m], w.w2r[m], nrhs, DS_RESID, w.rin[m], st));
      MG_TRY((vcycle_t<P, vec_t<P>>(c, m, w.w2r[m], w.w2x[m], nrhs, st)));
      HIPK(add_inplace<R>(w.x[m], w.w2x[m], c->lev[m].vsize(), nrhs, st));
    }
  }
  return smooth_post<P, TR>(c, l, rin, x, nrhs, st);
}

// One V-cycle from level 0 with the input in the class's fine storage.
template <typename P> static int vcycle_fine(mg_ctx *c, const fres_t<P> *rin, vec_t<P> *x, int nrhs, hipStream_t st) {
  return vcycle_t<P, fres_t<P>>(c, 0, rin, x, nrhs, st);
}

// One V-cycle K_l(rin) -> x (levels l..coarsest) with rin in the arithmetic
// type (on level 0 of the FP16 class it is first stored in binary16).
template <typename P> int vcycle(mg_ctx *c, int l, const vec_t<P> *rin, vec_t<P> *x, int nrhs, hipStream_t st) {
  if constexpr (std::is_same<fres_t<P>, h16>::value) {
    if (l == 0) {
      HIPK(to_h16<float2>(c->w32.hrin, rin, c->lev[0].g.Vpad, nrhs, st));
      return vcycle_fine<P>(c, c->w32.hrin, x, nrhs, st);
    }
  }
  return vcycle_t<P, vec_t<P>>(c, l, rin, x, nrhs, st);
}

// z = K(r) in the precision prec (FP64 in and out).
int precondition_at(mg_ctx *c, mg_prec_t prec, const double2 *r, double2 *z, int nrhs, hipStream_t st) {
  c->n_vcyc += nrhs;
  if (prec == MG_F64) return vcycle<PF64>(c, 0, r, z, nrhs, st);
  Work<float> &w = c->w32;
  const size_t n = c->lev[0].vsize() * nrhs;
  float2 *rin = w.rin[0], *x = w.x[0];
  if (prec == MG_F16) {
    HIPK(to_h16<double2>(w.hrin, r, c->lev[0].g.Vpad, nrhs, st));
    MG_TRY(vcycle_fine<PF16>(c, w.hrin, x, nrhs, st));
  } else {
    HIPK((convert<float, double>(rin, r, n, st)));
    MG_TRY(vcycle<PF32>(c, 0, rin, x, nrhs, st));
  }
  HIPK((convert<double, float>(z, x, n, st)));
  return MG_OK;
}

// z = K(r) in the context's preconditioner precision.
int precondition(mg_ctx *c, const double2 *r, double2 *z, int nrhs, hipStream_t st) {
  return precondition_at(c, c->prec, r, z, nrhs, st);
}

// ------------------------------------------------------------ FGCR
// Flexible GCR(m) in FP64 preconditioned by one V-cycle per step, with the
// solution update deferred to the end of each restart cycle (gcr.hip): the
// preconditioner writes z_j straight into Z in its own precision (FP64 for
// the FP64 preconditioner, FP32 otherwise), D z_j is taken in FP64, w_j is
// orthogonalised against the earlier directions by classical Gram-Schmidt
// (all inner products in one pass, one update pass), the residual moves
// along it, and x = x + Z c once per cycle.  Converged right-hand sides are
// frozen (skip flags); the host reads ||r||^2 once per step for the
// decision.  At the end of every cycle the true residual b - D x replaces
// the recursive one.
template <typename TZ>
static int fgcr_t(mg_ctx *c, const double2 *b, double2 *x, int nrhs, double tol, int *iters, double *relres,
                  TZ *Z, hipStream_t st) {
  Level &L0 = c->lev[0];
  const size_t n = L0.vsize();
  const size_t nn = n * nrhs;
  const int m = c->p.gcr_restart;
  constexpr bool f32z = sizeof(TZ) == 8;
  double2 *r = c->gr, *W = c->gW;
  // preconditioner input: FP32, or binary16 with per-site scales (FP16 class)
  const bool h16in = f32z && c->prec == MG_F16;
  float2 *r32 = f32z && !h16in ? c->gr32.p : nullptr;
  h16 *r16 = h16in ? c->gr16.p : nullptr;
  double *rr = c->dsc;
  int *skip = c->skip;
  // the cycles of the outer solver may run from captured V-cycle parts
  struct GraphGuard {
    mg_ctx *c;
    explicit GraphGuard(mg_ctx *cc) : c(cc) { c->vgraph_on = 1; }
    ~GraphGuard() { c->vgraph_on = 0; }
  } guard(c);
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
    HIPK(hipMemsetAsync(c->gcnt, 0, sizeof(int) * MG_MAX_RHS, st));
    if (r32) HIPK((convert<float, double>(r32, r, nn, st)));
    if (r16) HIPK(to_h16<double2>(r16, r, L0.g.Vpad, nrhs, st));
    int used = 0;
    for (int j = 0; j < m; ++j) {
      TZ *Zj = Z + (size_t)j * nn;
      double2 *Wj = W + (size_t)j * nn;
      // z_j = K(r_j), written in the preconditioner's precision
      c->n_vcyc += nrhs;
      if constexpr (f32z) {
        if (r16) MG_TRY(vcycle_fine<PF16>(c, r16, Zj, nrhs, st));
        else MG_TRY(vcycle<PF32>(c, 0, r32, Zj, nrhs, st));
      } else {
        MG_TRY(vcycle<PF64>(c, 0, r, Zj, nrhs, st));
      }
      {
        TimerScope ts(c, c->tm[0], st, (double)L0.g.V * nrhs);
        if constexpr (f32z)
          HIPK(dslash_in32(L0.g, L0.links64(), L0.nl, Zj, Wj, 4.0 + c->mass, nrhs, st));
        else
          HIPK((dslash<double, double2>(L0.g, L0.links64(), L0.nl, Zj, Wj, nullptr, 4.0 + c->mass, nrhs,
                                        DS_PLAIN, nullptr, st)));
      }
      c->n_fine += nrhs;
      HIPK(gcr2_step_residual(W, nn, j, m, r, n, nrhs, c->gsc, c->gnu, c->gcnt, skip, c->part, rr, r32, r16,
                              c->gcr_fuse, st));
      used = j + 1;
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
    // x += Z T^{-1} a over the steps of this cycle
    HIPK(gcr2_solution<TZ>(x, Z, nn, used, m, n, nrhs, c->gsc, c->gnu, c->gcnt, st));
    // true residual r = b - D x
    {
      TimerScope ts(c, c->tm[0], st, (double)L0.g.V * nrhs);
      HIPK((dslash<double, double2>(L0.g, L0.links64(), L0.nl, x, r, b, 4.0 + c->mass, nrhs, DS_RESID, nullptr,
                                    st)));
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

// Allocates the solver's outer buffers for nrhs right-hand sides.
int ensure_fgcr(mg_ctx *c, int nrhs) {
  const size_t n = c->lev[0].vsize() * nrhs;
  const int m = c->p.gcr_restart;
  MG_TRY(c->gx.alloc(n));
  MG_TRY(c->gr.alloc(n));
  MG_TRY(c->gb.alloc(n));
  // The directions w_j = D z_j and the preconditioned z_j are written at
  // every site before they are read; only padding sites (never written)
  // need the zero fill, which costs ~20 ms for the 58 GB of 12 right-hand
  // sides on 32^3 x 64.
  const bool pad = c->lev[0].g.Vpad != c->lev[0].g.V;
  MG_TRY(c->gW.alloc(n * m, pad));
  if (c->prec == MG_F64) {
    MG_TRY(c->gZ.alloc(n * m, pad));
  } else {
    MG_TRY(c->gZf.alloc(n * m, pad));
    if (c->prec == MG_F16) MG_TRY(c->gr16.alloc((size_t)13 * c->lev[0].g.Vpad * nrhs));
    else MG_TRY(c->gr32.alloc(n));
  }
  MG_TRY(c->gsc.alloc(MG_MAX_RHS * gcr_scalars_per_rhs(m)));
  MG_TRY(c->gnu.alloc((size_t)MG_MAX_RHS * m));
  MG_TRY(c->gcnt.alloc(MG_MAX_RHS));
  MG_TRY(c->skip.alloc(MG_MAX_RHS));
  return MG_OK;
}

int fgcr(mg_ctx *c, const double2 *b, double2 *x, int nrhs, double tol, int *iters, double *relres,
         hipStream_t st) {
  if (c->prec == MG_F64) return fgcr_t<double2>(c, b, x, nrhs, tol, iters, relres, c->gZ.p, st);
  return fgcr_t<float2>(c, b, x, nrhs, tol, iters, relres, c->gZf.p, st);
}

// ------------------------------------------------------------ setup
// The relaxation rounds of relax() in FP32 (setup_prec = MG_F32): FP32 copies of the level's
// operator (links of level 0, or the coarse stencil of a coarser level) and
// of the vectors, in batches of at most RELAX32_BATCH vectors so that the
// coarse levels take the matrix-core stencil; the relaxed vectors are
// widened back into V.
constexpr int RELAX32_BATCH = 12;
static int relax32(mg_ctx *c, int l, double2 *V, int nv, hipStream_t st) {
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  if (l == 0) {
    if (!L.U32.p) {
      MG_TRY(L.U32.alloc(4 * (size_t)L.nl * L.g.Vpad));
      if (L.nl == 6) HIPK(compress_links<float2>(L.g, L.U64, L.U32, c->part, st));
      else HIPK(store_convert<float2>(L.U32, L.U64, 36 * (size_t)L.g.Vpad, st));
    }
  } else if (!L.L32.p) {
    MG_TRY(L.L32.alloc(L.L64.n));
    HIPK(store_convert<float2>(L.L32, L.L64, L.L64.n, st));
  }
  const int B = std::min(nv, RELAX32_BATCH);
  if (l == 0) MG_TRY(ensure_mrq(c, MG_F32, B, c->p.setup_mr_steps));
  DevBuf<float2> v, x, r, q;
  MG_TRY(v.alloc(n * B));
  MG_TRY(x.alloc(n * B));
  MG_TRY(r.alloc(n * B));
  MG_TRY(q.alloc(n * B));
  const int steps = c->p.setup_mr_steps;
  for (int k0 = 0; k0 < nv; k0 += B) {
    const int nb = std::min(B, nv - k0);
    double2 *Vk = V + (size_t)k0 * n;
    HIPK((convert<float, double>(v, Vk, n * nb, st)));
    if (mrq_ready<float2>(c, l, steps, nb) && c->p.setup_rounds > 0) {
      // The combine pass of the q recursion subtracts the MR solution from v
      // in place, and the normalisation, which only scales the direction the
      // rounds produce (MR from zero is scale-covariant), is done once after
      // the last round.  The residual A v is recomputed every round: the
      // recursive one the MR steps leave (A v - A x) loses its relative
      // accuracy as the rounds shrink it (measured: 2.5e-4 instead of 7e-7
      // from the FP64 relaxation after five rounds).
      for (int round = 0; round < c->p.setup_rounds; ++round) {
        MG_TRY(apply_A<PF32>(c, l, v, r, nb, DS_PLAIN, nullptr, st));
        MG_TRY((mr_q<PF32, float2>(c, v, r.p, q.p, steps, true, nb, st, false, nullptr, -1.f)));
      }
      HIPK(norm2<float>(v, n, nb, c->part, c->dsc, st));
      HIPK(scale_rsqrt<float>(v, n, nb, c->dsc, st));
      HIPK((convert<double, float>(Vk, v, n * nb, st)));
      continue;
    }
    for (int round = 0; round < c->p.setup_rounds; ++round) {
      MG_TRY(apply_A<PF32>(c, l, v, r, nb, DS_PLAIN, nullptr, st));
      MG_TRY(mr<PF32>(c, l, x.p, r.p, q.p, c->p.setup_mr_steps, false, nb, st, false));
      HIPK(sub_inplace<float>(v, x, n, nb, st));
      HIPK(norm2<float>(v, n, nb, c->part, c->dsc, st));
      HIPK(scale_rsqrt<float>(v, n, nb, c->dsc, st));
    }
    HIPK((convert<double, float>(Vk, v, n * nb, st)));
  }
  HIPK(hipStreamSynchronize(st));
  return MG_OK;
}

// Null-vector relaxation: v <- v - MR(A, A v), v <- v / ||v||, `rounds` times,
// all nv vectors as one batch (FP64; FP32 in batches when setup_prec says so).
int relax(mg_ctx *c, int l, double2 *V, int nv, hipStream_t st) {
  Level &L = c->lev[l];
  const size_t n = L.vsize();
  if (c->p.setup_prec == MG_F32) return relax32(c, l, V, nv, st);
  DevBuf<double2> x, r, q;
  MG_TRY(x.alloc(n * nv));
  MG_TRY(r.alloc(n * nv));
  MG_TRY(q.alloc(n * nv));
  for (int round = 0; round < c->p.setup_rounds; ++round) {
    MG_TRY(apply_A<PF64>(c, l, V, r, nv, DS_PLAIN, nullptr, st));
    MG_TRY(mr<PF64>(c, l, x.p, r.p, q.p, c->p.setup_mr_steps, false, nv, st, false));
    HIPK(sub_inplace<double>(V, x, n, nv, st));
    HIPK(norm2<double>(V, n, nv, c->part, c->dsc, st));
    HIPK(scale_rsqrt<double>(V, n, nv, c->dsc, st));
  }
  HIPK(hipStreamSynchronize(st));
  return MG_OK;
}

// Drops the solver work buffers so that the next ensure_work allocates them
// afresh (zeroed) for the current level sizes.
template <typename R> void release_work(Work<R> &w) {
  for (int l = 0; l < MG_MAX_LEVELS; ++l) {
    w.x[l].release();
    w.r[l].release();
    w.q[l].release();
    w.rin[l].release();
    w.gv[l].release();
    w.w2r[l].release();
    w.w2x[l].release();
  }
  w.hr.release();
  w.hq.release();
  w.hrin.release();
  w.q2.release();
  w.hq2.release();
  for (int k = 0; k + 1 < MRQ_MAX; ++k) {
    w.rk[k].release();
    w.hrk[k].release();
  }
  w.mrq_nrhs[0] = w.mrq_nrhs[1] = 0;
  w.ce.release();
  w.cr.release();
  w.cz.release();
  w.cp.release();
  w.cw.release();
  w.cp2.release();
  w.cr2.release();
  w.nrhs = 0;
}

// Drops the low-precision copies of the level-0 prolongator and the level-1
// operator; the next ensure_prec rebuilds them from the FP64 data.
void drop_op_copies(mg_ctx *c, int l) {
  c->lev[l].P32.release();
  c->lev[l].P16.release();
  c->lev[l + 1].L32.release();
  c->lev[l + 1].L16.release();
  c->lev[l + 1].L32t.release();
  c->lev[l + 1].L16t.release();
}

// z = K_l(r): one cycle from level l in precision prec (FP64 in and out).
int cycle_from(mg_ctx *c, int l, mg_prec_t prec, const double2 *r, double2 *z, int nrhs, hipStream_t st) {
  if (prec == MG_F64) return vcycle<PF64>(c, l, r, z, nrhs, st);
  Work<float> &w = c->w32;
  const size_t n = c->lev[l].vsize() * nrhs;
  float2 *rin = w.rin[l], *x = w.x[l];
  if (prec == MG_F16 && l == 0) {
    HIPK(to_h16<double2>(w.hrin, r, c->lev[0].g.Vpad, nrhs, st));
    MG_TRY(vcycle_fine<PF16>(c, w.hrin, x, nrhs, st));
  } else {
    HIPK((convert<float, double>(rin, r, n, st)));
    if (prec == MG_F16) MG_TRY(vcycle<PF16>(c, l, rin, x, nrhs, st));
    else MG_TRY(vcycle<PF32>(c, l, rin, x, nrhs, st));
  }
  HIPK((convert<double, float>(z, x, n, st)));
  return MG_OK;
}

// Setup stage two ("Numerical Results") on the level-l prototypes in NV:
// groups of refine_group vectors are taken out in turn; the remaining
// prototypes define a truncated two-level method from level l (block
// orthonormalisation, Galerkin operator, the cycle of level l over the
// CGNR solve on the truncated level l+1); from each prototype v of the
// group, refine_iters steps of the flexible GCR preconditioned by that cycle
// are run on A_l v = 0 (residual -A_l v, no restart), and the normalised
// iterates replace the group.  The cycles run in the context's
// preconditioner precision (copies of the truncated P and operator made per
// group), the GCR steps in FP64.  Level sizes are shrunk while a group is
// out and restored afterwards; work buffers, captured graphs and tuned
// coarse variants made at the shrunk sizes are dropped.
int refine(mg_ctx *c, int l, hipStream_t st_in) {
  const int G0 = c->p.refine_group, iters = c->p.refine_iters;
  Level &Lv = c->lev[l], &Lc = c->lev[l + 1];
  const int nv = Lv.nv;
  if (G0 <= 0 || iters <= 0 || G0 >= nv) return MG_OK;
  // runs on the context's own stream (the coarsest-level CGNR captures
  // graphs, which the default stream does not allow), after st_in's work
  hipStream_t st = c->sti;
  HIPK(hipEventRecord(c->ev_in, st_in));
  HIPK(hipStreamWaitEvent(st, c->ev_in, 0));
  const int nlev = c->nlev, nc = Lc.n, nvc = Lc.nv;
  const mg_prec_t rp = c->prec;
  const size_t n = Lv.vsize();
  DevBuf<double2> X, R, Z, W;
  MG_TRY(X.alloc(n * G0));
  MG_TRY(R.alloc(n * G0));
  MG_TRY(Z.alloc(n * G0 * iters));
  MG_TRY(W.alloc(n * G0 * iters));
  MG_TRY(Lc.L64.alloc((size_t)Lc.g.V * 9 * nc * nc));
  double *rr = c->dsc;
  double2 *sc = c->csc;
  int *flag = c->done;
  int rc = MG_OK;
  for (int g0 = 0; g0 < nv && rc == MG_OK; g0 += G0) {
    const int G = std::min(G0, nv - g0), nk = nv - G;
    const size_t nn = n * G;
    // the kept prototypes, in order, as the truncated method's P
    if (g0 > 0) HIPK(hipMemcpyAsync(Lv.P64, Lv.NV, n * g0 * sizeof(double2), hipMemcpyDeviceToDevice, st));
    if (g0 + G < nv)
      HIPK(hipMemcpyAsync(Lv.P64 + n * g0, Lv.NV + n * (g0 + G), n * (nv - g0 - G) * sizeof(double2),
                          hipMemcpyDeviceToDevice, st));
    c->nlev = l + 2;
    Lv.nv = nk;
    Lc.n = 2 * nk;
    Lc.nv = 0;
    release_work(c->w64);
    release_work(c->w32);
    drop_op_copies(c, l);
    clear_graphs(c);
    std::memset(c->cvar, 0xff, sizeof(c->cvar));
    std::memset(c->tvar, 0xff, sizeof(c->tvar));
    HIPK(hipMemsetAsync(flag, 0, sizeof(int), st));
    if (l == 0) HIPK(ortho_fine(Lv.g, nk, Lv.P64, flag, st));
    else HIPK(ortho_coarse(Lv.g, Lv.n, nk, Lv.P64, flag, st));
    HIPK(hipMemcpyAsync(c->h_done, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPK(hipStreamSynchronize(st));
    if (c->h_done[0]) {
      set_error("mg_setup: rank-deficient aggregate in the refinement's block orthonormalisation");
      rc = MG_ERANK;
      break;
    }
    if (l == 0) HIPK(galerkin_fine(Lv.g, Lc.g, c->mass, Lv.U64, nk, Lv.P64, Lc.L64, st));
    else HIPK(galerkin_coarse(Lv.g, Lc.g, Lv.n, Lv.L64, nk, Lv.P64, Lc.L64, st));
    if ((rc = ensure_work<double>(c, G)) != MG_OK) break;
    if (rp != MG_F64) {
      if ((rc = ensure_prec(c, rp, st)) != MG_OK) break;
      if ((rc = ensure_work<float>(c, G)) != MG_OK) break;
      if ((rc = ensure_mrq(c, rp, G)) != MG_OK) break;
    }
    // x = v, r = -A v
    double2 *x = X, *r = R;
    HIPK(hipMemcpyAsync(x, Lv.NV + n * g0, nn * sizeof(double2), hipMemcpyDeviceToDevice, st));
    if ((rc = apply_A<PF64>(c, l, x, W, G, DS_PLAIN, nullptr, st)) != MG_OK) break;
    HIPK(zero<double>(r, nn, st));
    HIPK(sub_inplace<double>(r, W, n, G, st));
    for (int j = 0; j < iters && rc == MG_OK; ++j) {
      double2 *Zj = Z + (size_t)j * nn, *Wj = W + (size_t)j * nn;
      if ((rc = cycle_from(c, l, rp, r, Zj, G, st)) != MG_OK) break;
      if ((rc = apply_A<PF64>(c, l, Zj, Wj, G, DS_PLAIN, nullptr, st)) != MG_OK) break;
      for (int i = 0; i < j; ++i) {
        HIPK(dot<double>(W + (size_t)i * nn, Wj, n, G, c->part, sc, st));
        HIPK(gcr_sub2(Wj, W + (size_t)i * nn, Zj, Z + (size_t)i * nn, n, G, sc, nullptr, st));
      }
      HIPK(norm2<double>(Wj, n, G, c->part, rr + MG_MAX_RHS, st));
      HIPK(gcr_scale2(Wj, Zj, n, G, rr + MG_MAX_RHS, nullptr, st));
      HIPK(dot<double>(Wj, r, n, G, c->part, sc, st));
      HIPK(gcr_update(x, Zj, r, Wj, n, G, sc, nullptr, c->part, rr, st));
    }
    if (rc != MG_OK) break;
    HIPK(norm2<double>(x, n, G, c->part, rr, st));
    HIPK(scale_rsqrt<double>(x, n, G, rr, st));
    HIPK(hipMemcpyAsync(Lv.NV + n * g0, x, nn * sizeof(double2), hipMemcpyDeviceToDevice, st));
    HIPK(hipStreamSynchronize(st));
  }
  c->nlev = nlev;
  Lv.nv = nv;
  Lc.n = nc;
  Lc.nv = nvc;
  release_work(c->w64);
  release_work(c->w32);
  drop_op_copies(c, l);
  clear_graphs(c);
  std::memset(c->cvar, 0xff, sizeof(c->cvar));
  std::memset(c->tvar, 0xff, sizeof(c->tvar));
  return rc;
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
    Lv.fine = (l == 0);
    Lv.n = (l == 0) ? 12 : 2 * p.nv[l - 1];
    Lv.nv = (l < c->nlev - 1) ? p.nv[l] : 0;
    for (int mu = 0; mu < 4; ++mu) L[mu] = Lv.g.C[mu];
  }
  size_t pn = part_need(c, 1);
  for (int l = 0; l < c->nlev - 1; ++l) {
    const Level &Lv = c->lev[l];
    const size_t per = (l == 0) ? (size_t)dslash_partials(Lv.g, Lv.nv) * 3 : np_coarse(Lv) * 3;
    pn = std::max(pn, std::max(per, (size_t)RED_BLOCKS * 2) * Lv.nv);
  }
  MG_TRY(ensure_scalars(c, pn));
  Level &L0 = c->lev[0];
  MG_TRY(L0.U64.alloc(36 * (size_t)L0.g.Vpad));
  HIPK(pack_gauge<double>(L0.g, (const double2 *)U, L0.U64, st));
  // Compressed (two-row) links when every link is SU(3) to rounding.
  MG_TRY(L0.U64c.alloc(24 * (size_t)L0.g.Vpad));
  {
    const int nb = dslash_blocks(L0.g);
    HIPK(compress_links<double2>(L0.g, L0.U64, L0.U64c, c->part, st));
    std::vector<double> bm(nb);
    HIPK(hipMemcpyAsync(bm.data(), c->part, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    HIPK(hipStreamSynchronize(st));
    double dev = 0.0;
    for (double v : bm) dev = std::max(dev, v);
    if (!std::isfinite(dev)) {
      set_error("mg_setup: non-finite gauge field");
      return MG_ENONFINITE;
    }
    L0.nl = dev <= 1e-12 ? 6 : 9;
    if (L0.nl == 9) L0.U64c.release();
  }
  int *flag = c->done;  // reused as rank-deficiency flag during setup
  for (int l = 0; l < c->nlev - 1; ++l) {
    Level &Lv = c->lev[l], &Lc = c->lev[l + 1];
    const size_t nvs = Lv.vsize() * Lv.nv;
    MG_TRY(Lv.NV.alloc(nvs));
    MG_TRY(Lv.P64.alloc(nvs));
    if (l == 0) HIPK(pack_field<double>(Lv.g, (const double2 *)p.init_vectors[0], Lv.NV, 12, Lv.nv, st));
    else HIPK(pack_aos<double>(Lv.g, (const double2 *)p.init_vectors[l], Lv.NV, Lv.n, Lv.nv, st));
    MG_TRY(relax(c, l, Lv.NV, Lv.nv, st));
    MG_TRY(refine(c, l, st));
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

#define INST(P)                                                                                               \
  template int vcycle<P>(mg_ctx *, int, const vec_t<P> *, vec_t<P> *, int, hipStream_t);                        \
  template int apply_A<P>(mg_ctx *, int, const vec_t<P> *, vec_t<P> *, int, DslashMode, const vec_t<P> *,       \
                          hipStream_t);                                                                          \
  template int transfer_restrict<P>(mg_ctx *, int, const vec_t<P> *, vec_t<P> *, int, hipStream_t);             \
  template int transfer_prolong<P>(mg_ctx *, int, const vec_t<P> *, vec_t<P> *, int, int, hipStream_t);       \
  template int coarse_variant<P>(mg_ctx *, int, int, hipStream_t);                                              \
  template int cgnr<P>(mg_ctx *, int, const vec_t<P> *, vec_t<P> *, int, hipStream_t);
INST(PF64)
INST(PF32)
INST(PF16)
#undef INST

}  // namespace mg
