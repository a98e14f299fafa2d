// Coarse operator D_c = P^dag D P applied as a 9-point stencil of n x n
// complex blocks (n = 2 Nv):
//   out(x) = X(x) v(x) + sum_mu [ Y_{+mu}(x) v(x+mu) + Y_{-mu}(x) v(x-mu) ]
// and its adjoint D_c^dag = sigma_3 D_c sigma_3 (gamma_5-Hermiticity carried to
// the coarse grid by the chirality split, P^dag gamma_5 = sigma_3 P^dag).
//
// Storage: coarse vectors are site-major (AoS), v[site][n]; the operator is
// L[site][slot][j][i] with slot 0 = X, slot 1 + (2 mu + dir) = Y, each block
// stored column-major so that the n rows of one column are contiguous.
//
// RS workgroups per coarse site, each owning n / RS consecutive rows: the nine input vectors are staged in LDS; thread (i, g) owns RW
// consecutive rows (RW = 2 in FP32 so every load is 16 bytes) and a strided
// subset g, g+G, ... of the 9n (slot, column) pairs, so each group streams one
// contiguous column segment and the workgroup reads a contiguous window of the
// site's entries per step (coalesced, bandwidth-bound).  The first chunk of
// operator loads is issued before the input vectors are staged so the two
// memory phases overlap.  The G partial row sums are combined in LDS in a
// fixed order (deterministic).
//
// The matrix-core variant (k_coarse_mma) handles all right-hand sides of a
// site in one workgroup: out[:, 0:nrhs] = A [B_0 .. B_8], a complex GEMM with
// M = n rows, N = nrhs (padded to 16) and K = 9n, where A is the site's
// operator (loaded once for every right-hand side) and B the nine staged
// input blocks.  Each complex product is three real 16x16x4 FP32 MFMAs.
#include "solver.h"

namespace mg {

constexpr int CO_CHUNK = 8;   // operator loads in flight per thread
constexpr int CO_PARTS = 8;   // first-stage partial sums per row of the group reduction

// 16-byte (or 8-byte) load of RW consecutive operator entries in storage S.
template <typename S, int RW> struct OpVec;
template <> struct OpVec<double2, 1> {
  using V = double2;
  template <typename C> __device__ static void get(const V &v, C (&o)[1]) { o[0] = cvt<C>(v); }
};
template <> struct OpVec<float2, 2> {
  using V = float4;
  template <typename C> __device__ static void get(const V &v, C (&o)[2]) {
    o[0] = mk<C>(v.x, v.y);
    o[1] = mk<C>(v.z, v.w);
  }
};
template <> struct OpVec<chalf, 2> {
  using V = chalf2;
  template <typename C> __device__ static void get(const V &v, C (&o)[2]) {
    o[0] = cvt<C>(v.v[0]);
    o[1] = cvt<C>(v.v[1]);
  }
};
template <> struct OpVec<chalf, 4> {
  using V = chalf4;
  template <typename C> __device__ static void get(const V &v, C (&o)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = cvt<C>(v.v[q]);
  }
};

// Site read by stencil slot `slot` of coarse site s: slot 0 = s, slot
// 1 + 2 mu + dir = the neighbour in direction mu (dir 0 forward, 1 backward).
// The switch keeps every coordinate index a constant (no private arrays).
__device__ __forceinline__ uint32_t slot_site(const Geom &g, uint32_t s, int slot) {
  const Coords k = decode(g, s);
  switch (slot) {
    case 1: return nbr_fwd(g, s, k, 0);
    case 2: return nbr_bwd(g, s, k, 0);
    case 3: return nbr_fwd(g, s, k, 1);
    case 4: return nbr_bwd(g, s, k, 1);
    case 5: return nbr_fwd(g, s, k, 2);
    case 6: return nbr_bwd(g, s, k, 2);
    case 7: return nbr_fwd(g, s, k, 3);
    case 8: return nbr_bwd(g, s, k, 3);
    default: return s;
  }
}

// Sums of up to three partial arrays over the workgroup in one pass: out[0]
// = sum a[0..na), out[1] = sum b[0..nb), out[2] = sum c[0..nb) (NULL arrays
// give 0).  Fixed order; result in every thread.
__device__ __forceinline__ void block_allsum3(const double *__restrict__ a, int na, const double *__restrict__ b,
                                              const double *__restrict__ c, int nb, double (&out)[3],
                                              double *lds) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < na; i += blockDim.x) v[0] += a[i];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    v[1] += b[i];
    v[2] += c[i];
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < 3; ++q) v[q] = wave_sum(v[q]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) lds[w * 3 + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += lds[k * 3 + q];
    out[q] = t;
  }
  __syncthreads();
}

// Sum of np partials over the workgroup; result in every thread.
__device__ __forceinline__ double block_allsum_partials(const double *__restrict__ p, int np, double *lds) {
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) a += p[i];
  a = wave_sum(a);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = a;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < nw; ++q) t += lds[q];
  __syncthreads();
  return t;
}


// Workgroup i of a per-RHS launch -> (logical workgroup ws of its right-hand
// side, rhs).  Workgroups go round-robin to the 8 XCDs; when the per-RHS
// count is a multiple of 8, XCD x takes the contiguous workgroup range
// [x nbx / 8, (x + 1) nbx / 8) (neighbouring sites share L2) and runs the
// right-hand sides of one workgroup back to back, so that a site's operator
// blocks come from HBM once and from that XCD's L2 for the other RHS.
__device__ __forceinline__ void block_rhs_of(uint32_t i, uint32_t nbx, uint32_t nrhs, uint32_t &ws, int &rhs) {
  if ((nbx & 7u) == 0u) {
    const uint32_t t = i >> 3;
    ws = (i & 7u) * (nbx >> 3) + t / nrhs;
    rhs = (int)(t % nrhs);
  } else {
    ws = i / nrhs;
    rhs = (int)(i % nrhs);
  }
}

template <typename R, typename S, int RW>
__global__ __launch_bounds__(512) void k_coarse(Geom g, int n, const S *__restrict__ L,
                                                 const c_t<R> *__restrict__ in, c_t<R> *__restrict__ out,
                                                 int nrhs, int dagger, double *__restrict__ partials, int pw,
                                                 const int *__restrict__ done, CgCheck chk, CgFuse fz) {
  using C = c_t<R>;
  using VT = typename OpVec<S, RW>::V;
  __shared__ C vin[9 * COARSE_NMAX];
  __shared__ C red[512 * RW];
  __shared__ C red2[CO_PARTS * COARSE_NMAX];
  __shared__ double wred[8 * 4];
  const uint32_t nbx = gridDim.x / (uint32_t)nrhs;  // workgroups per right-hand side
  uint32_t ws;
  int rhs;
  block_rhs_of(blockIdx.x, nbx, (uint32_t)nrhs, ws, rhs);
  if (done != nullptr && done[rhs]) return;
  const int RS = (int)(nbx / g.V);
  const uint32_t s = ws / RS;
  const int nr = n / RS, r0 = (int)(ws - s * RS) * nr;
  const size_t rhs_off = (size_t)rhs * g.V * n;
  in += rhs_off;
  out += rhs_off;
  const int tid = threadIdx.x;
  const int npr = nr / RW;  // row units of this workgroup
  const int G = (int)blockDim.x / npr;
  const int ip = tid % npr, grp = tid / npr;
  const int nP = 9 * n;
  const int nu = n / RW;    // row units per column
  const VT *Ls = reinterpret_cast<const VT *>(L + (size_t)s * 9 * n * n + r0) + ip;
  // Issue the first chunk of operator loads before staging the input vectors
  // so that the two memory phases overlap.  Every load is issued
  // unconditionally (a lane without an entry of its own reads entry 0 and
  // never uses it): a load under a lane mask gets a basic block of its own,
  // where the compiler waits for it before the next one is issued.
  VT lv[CO_CHUNK];
  const bool on = grp < G;
#pragma unroll
  for (int q = 0; q < CO_CHUNK; ++q) {
    const int p = grp + q * G;
    lv[q] = Ls[(size_t)((on && p < nP) ? p : 0) * nu];
  }
  __shared__ uint32_t nbs[9];
  if (tid < 9) nbs[tid] = slot_site(g, s, tid);
  // Scalars of this launch, summed from per-workgroup partials in one pass
  // (one round trip): the CGNR convergence test on the residual of the
  // update just made, and the fused update's coefficient.
  const bool check = chk.part_r != nullptr;
  const bool first = fz.kind == 1 && fz.it0[rhs] == 0;
  const bool coef_on = fz.kind != 0 && !first;
  R coef = 0;
  if (check || coef_on) {
    const double *pa = check ? chk.part_r + (size_t)rhs * chk.np_r : nullptr;
    const double *pn = coef_on ? fz.num + (size_t)rhs * fz.np : nullptr;
    const double *pd = coef_on ? fz.den + (size_t)rhs * fz.np : nullptr;
    double sums[3];
    block_allsum3(pa, check ? chk.np_r : 0, pn, pd, coef_on ? fz.np : 0, sums, wred);
    if (check) {
      const double rr = sums[0];
      const double *cg = chk.cg + (size_t)rhs * CG_NS;
      const int iter = chk.it_in[rhs];
      bool conv;
      if (chk.fused) conv = (iter > 0 && !(rr > cg[4] * cg[3])) || iter >= chk.maxit;
      else conv = !(rr > cg[4] * cg[3]) || iter + 1 >= chk.maxit;
      if (ws == 0 && threadIdx.x == 0) {
        chk.it_out[rhs] = (chk.fused && conv) ? iter : iter + 1;
        if (conv) chk.done[rhs] = 1;
      }
      if (conv) return;
    }
    if (coef_on) {
      if (!(sums[2] > 0.0)) {
        if (fz.kind == 2) {
          if (ws == 0 && tid == 0) fz.done_w[rhs] = 1;
          return;
        }
      } else {
        coef = (R)(sums[1] / sums[2]);
      }
    }
  }
  __syncthreads();
  double own_sq = 0.0;
  if (fz.kind == 0) {
    for (int idx = tid; idx < nP; idx += blockDim.x) {
      const int slot = idx / n, j = idx - slot * n;
      C v = in[(size_t)nbs[slot] * n + j];
      if (dagger && j >= (n >> 1)) v = mk<C>(-v.x, -v.y);
      vin[idx] = v;
    }
  } else {
    const C *fa = reinterpret_cast<const C *>(fz.a) + rhs_off;
    const C *fb = reinterpret_cast<const C *>(fz.b) + rhs_off;
    const R sc = fz.kind == 1 ? coef : -coef;
    for (int idx = tid; idx < nP; idx += blockDim.x) {
      const int slot = idx / n, j = idx - slot * n;
      const size_t o = (size_t)nbs[slot] * n + j;
      C v = cfma(mk<C>(sc, 0), fb[o], fa[o]);
      if (slot == 0) {
        reinterpret_cast<C *>(fz.own)[rhs_off + o] = v;
        if (fz.kind == 2) {
          C *e = reinterpret_cast<C *>(fz.e) + rhs_off;
          const C *pp = reinterpret_cast<const C *>(fz.p) + rhs_off;
          e[o] = cfma(mk<C>(coef, 0), pp[o], e[o]);
          own_sq += (double)v.x * v.x + (double)v.y * v.y;
        }
      }
      if (dagger && j >= (n >> 1)) v = mk<C>(-v.x, -v.y);
      vin[idx] = v;
    }
  }
  __syncthreads();
  C acc[RW];
#pragma unroll
  for (int q = 0; q < RW; ++q) acc[q] = mk<C>(0, 0);
  for (int base = grp; on && base < nP; base += CO_CHUNK * G) {
    if (base != grp) {
#pragma unroll
      for (int q = 0; q < CO_CHUNK; ++q) {
        const int p = base + q * G;
        lv[q] = Ls[(size_t)(p < nP ? p : 0) * nu];
      }
    }
#pragma unroll
    for (int q = 0; q < CO_CHUNK; ++q) {
      const int p = base + q * G;
      if (p < nP) {
        const C x = vin[p];
        C o[RW];
        OpVec<S, RW>::get(lv[q], o);
#pragma unroll
        for (int t = 0; t < RW; ++t) acc[t] = cfma(o[t], x, acc[t]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RW; ++q) red[tid * RW + q] = acc[q];
  __syncthreads();
  // Sum of the G group partials of every row in two fixed-order stages:
  // CO_PARTS threads per row add every CO_PARTS-th group, then one thread
  // per row adds the CO_PARTS results (short dependent chains in LDS).
  if (tid < nr * CO_PARTS) {
    const int i = tid % nr, part = tid / nr;
    const int ipr = i / RW, sub = i % RW;
    C sum = mk<C>(0, 0);
    for (int q = part; q < G; q += CO_PARTS) sum = cadd(sum, red[(q * npr + ipr) * RW + sub]);
    red2[part * COARSE_NMAX + i] = sum;
  }
  __syncthreads();
  // partials (pw = 1): ||out||^2;  (pw = 3): <out, in>, ||out||^2 (in = centre)
  double t[3] = {0.0, 0.0, 0.0};
  if (tid < nr) {
    const int row = r0 + tid;
    C sum = red2[tid];
#pragma unroll
    for (int q = 1; q < CO_PARTS; ++q) sum = cadd(sum, red2[q * COARSE_NMAX + tid]);
    if (dagger && row >= (n >> 1)) sum = mk<C>(-sum.x, -sum.y);
    out[(size_t)s * n + row] = sum;
    const C c = vin[row];
    t[0] = (double)sum.x * c.x + (double)sum.y * c.y;
    t[1] = (double)sum.x * c.y - (double)sum.y * c.x;
    t[2] = (double)sum.x * sum.x + (double)sum.y * sum.y;
  }
  if (partials != nullptr || fz.kind == 2) {
    double v4[4] = {t[0], t[1], t[2], own_sq};
    block_sum<4>(v4, wred);
    if (tid == 0) {
      if (partials != nullptr) {
        double *p = partials + ((size_t)rhs * nbx + ws) * pw;
        if (pw == 1) {
          p[0] = v4[2];
        } else {
          p[0] = v4[0];
          p[1] = v4[1];
          p[2] = v4[2];
        }
      }
      if (fz.kind == 2) fz.part_own[(size_t)rhs * nbx + ws] = v4[3];
    }
  }
}

// ------------------------------------------------------------ persistent CGNR
// The whole coarsest-level CGNR of one right-hand side in one cooperative
// launch: the fused two-phase iteration of k_coarse (phase 1: p = z + beta
// p_old staged, w = A p; phase 2: r = r_old - alpha w staged, e += alpha p,
// z = A^dag r) with a grid-wide barrier after each phase instead of a kernel
// boundary.  Each workgroup (one coarse site) loads its operator rows once
// into registers and keeps them for every iteration; a kernel boundary would
// drop the L2 and fetch the operator again.  Every workgroup computes the
// same scalars from the same partials in the same order, so all of them take
// the same exit.  A barrier wait is bounded: a workgroup that gives up sets
// *fail and leaves, so the grid always drains.
constexpr int CGP_PMAX = 16;          // most operator entries per thread kept in registers

// Data exchanged between workgroups inside the launch (vectors and partial
// sums) is read and written as agent-scope relaxed atomics: the loads skip
// the XCD's non-coherent L2 and the stores write through it, so a barrier
// needs only each thread's stores acknowledged before its arrival, and no
// L2 write-back or invalidation (which cost about 80 us per barrier here).
__device__ __forceinline__ float2 cld(const float2 *p) {
  const unsigned long long v = __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<float2 *>(p)),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  float2 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}
__device__ __forceinline__ void cst(float2 *p, float2 v) {
  unsigned long long u;
  __builtin_memcpy(&u, &v, sizeof(u));
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double cldd(const double *p) {
  const unsigned long long v = __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<double *>(p)),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}
__device__ __forceinline__ void cstd(double *p, double v) {
  unsigned long long u;
  __builtin_memcpy(&u, &v, sizeof(u));
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums over partials written inside the launch, in block_allsum3's order
// (so each equals the chunked path's sum of the same array): out[0] over a,
// out[1] over b (when b != nullptr), n entries each.
__device__ __forceinline__ void cgp_allsum2(const double *__restrict__ a, const double *__restrict__ b, int n,
                                            double (&out)[2], double *lds) {
  double v[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    v[0] += cldd(a + i);
    if (b != nullptr) v[1] += cldd(b + i);
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < 2; ++q) v[q] = wave_sum(v[q]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) lds[w * 3 + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += lds[k * 3 + q];
    out[q] = t;
  }
  __syncthreads();
}

// Arrivals are spread over CGP_NC counters on separate 256-byte lines
// (workgroup i counts on i mod CGP_NC), so that no single address takes
// every workgroup's atomic; the first wavefront polls all of them at once.
//
// Why relaxed atomics order the exchange: every value another workgroup
// reads was stored with an agent-scope atomic store (written through to the
// agent's coherence point) and is read with an agent-scope atomic load
// (which bypasses the XCD's L2 and reads at that point).  s_waitcnt(0)
// holds each thread until its stores are acknowledged, i.e. performed at
// agent scope; the workgroup barrier then puts all of them before the one
// arrival increment.  A reader issues its data loads only after it has seen
// the count reach the target (the loop exit and the workgroup barrier order
// them after the poll).  So every data load is performed after every data
// store it depends on, at the same coherence point.  A release / acquire pair
// would give the same order with an L2 write-back and invalidate per barrier
// (about 80 us each here); with no data ever held in L2 they are not needed.
constexpr int CGP_NC = CGP_BAR_WORDS / 64;
__device__ __forceinline__ bool cgp_barrier(unsigned *bar, unsigned target, int *fail, unsigned spin_max,
                                            int *lds_ok) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores acknowledged
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_fetch_add(bar + (blockIdx.x % CGP_NC) * 64, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      unsigned v = lane < CGP_NC ? __hip_atomic_load(bar + lane * 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
      v = wave_sum(v);
      if (v >= target) break;
      if (++spins > spin_max) {
        ok = 0;
        if (lane == 0) __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) *lds_ok = ok;
  }
  __syncthreads();
  return *lds_ok != 0;
}

template <typename S, int RW, int PM>
__global__ __launch_bounds__(512, 4) void k_cgnr_persistent(Geom g, int n, const S *__restrict__ L, CgPersist a) {
  using C = float2;
  using VT = typename OpVec<S, RW>::V;
  __shared__ C vin[9 * COARSE_NMAX];
  __shared__ C red[512 * RW];
  __shared__ C red2[CO_PARTS * COARSE_NMAX];
  __shared__ double wred[8 * 4];
  __shared__ uint32_t nbs[9];
  __shared__ int bar_ok;
  const uint32_t s = blockIdx.x, nblk = gridDim.x;
  const int tid = threadIdx.x;
  const int npr = n / RW, G = (int)blockDim.x / npr;
  const int ip = tid % npr, grp = tid / npr;
  const int nP = 9 * n, half = n >> 1;
  const bool on = grp < G;
  const VT *Ls = reinterpret_cast<const VT *>(L + (size_t)s * 9 * n * n) + ip;
  VT lv[PM];
#pragma unroll
  for (int q = 0; q < PM; ++q) {
    const int p = grp + q * G;
    lv[q] = Ls[(size_t)((on && p < nP) ? p : 0) * n / RW];
  }
  if (tid < 9) nbs[tid] = slot_site(g, s, tid);
  __syncthreads();
  const double tol2b2 = a.cg[4] * a.cg[3];
  unsigned round = 0;
  double gam = 0.0;  // gamma_k = ||z_k||^2 of the current iteration
  int k = 0, final_it = 0;
  // a zero right-hand side was marked done before the launch (as the chunks
  // see it): no iteration, e stays zero
  const bool nothing = a.done[0] != 0;
  // rows of this workgroup times the staged vector, summed over the groups in
  // the fixed two-stage order of k_coarse; returns the row sum (tid < n)
  auto apply = [&]() -> C {
    C acc[RW];
#pragma unroll
    for (int t = 0; t < RW; ++t) acc[t] = make_float2(0.f, 0.f);
#pragma unroll
    for (int q = 0; q < PM; ++q) {
      const int p = grp + q * G;
      if (on && p < nP) {
        const C x = vin[p];
        C o[RW];
        OpVec<S, RW>::get(lv[q], o);
#pragma unroll
        for (int t = 0; t < RW; ++t) acc[t] = cfma(o[t], x, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < RW; ++t) red[tid * RW + t] = acc[t];
    __syncthreads();
    if (tid < n * CO_PARTS) {
      const int i = tid % n, part = tid / n;
      const int ipr = i / RW, sub = i % RW;
      C sum = make_float2(0.f, 0.f);
      for (int q = part; q < G; q += CO_PARTS) sum = cadd(sum, red[(q * npr + ipr) * RW + sub]);
      red2[part * COARSE_NMAX + i] = sum;
    }
    __syncthreads();
    C sum = make_float2(0.f, 0.f);
    if (tid < n) {
      sum = red2[tid];
#pragma unroll
      for (int q = 1; q < CO_PARTS; ++q) sum = cadd(sum, red2[q * COARSE_NMAX + tid]);
    }
    return sum;
  };
  for (; !nothing;) {
    // ---- phase 1: convergence test of the last update, p = z + beta p_old, w = A p
    float2 *pn = a.p[k & 1];
    const float2 *po = a.p[(k + 1) & 1];
    // ||r||^2 of the last update and gamma_k = ||z_k||^2; gamma_{k-1} is
    // the sum of the same array the previous phase 1 made (the chunked path
    // sums it again, to the same value)
    double sums[2] = {0.0, 0.0};
    if (k > 0) cgp_allsum2(a.pr, a.pz[k & 1], (int)nblk, sums, wred);
    if ((k > 0 && !(sums[0] > tol2b2)) || k >= a.maxit) {
      final_it = k;
      break;
    }
    const float beta = (k > 0 && gam > 0.0) ? (float)(sums[1] / gam) : 0.f;
    if (k > 0) gam = sums[1];
    for (int idx = tid; idx < nP; idx += blockDim.x) {
      const int slot = idx / n, j = idx - slot * n;
      const size_t o = (size_t)nbs[slot] * n + j;
      const C v = cfma(make_float2(beta, 0.f), cld(po + o), cld(a.z + o));
      if (slot == 0) cst(pn + o, v);
      vin[idx] = v;
    }
    __syncthreads();
    {
      const C wv = apply();
      double t2 = 0.0;
      if (tid < n) {
        cst(a.w + (size_t)s * n + tid, wv);
        t2 = (double)wv.x * wv.x + (double)wv.y * wv.y;
      }
      double v4[4] = {0.0, 0.0, t2, 0.0};
      block_sum<4>(v4, wred);
      if (tid == 0) cstd(a.pw + s, v4[2]);
    }
    if (!cgp_barrier(a.bar, ++round * nblk, a.fail, a.spin, &bar_ok)) {
      final_it = k;
      break;
    }
    // ---- phase 2: r = r_old - alpha w, e += alpha p, z = A^dag r
    const float2 *ro = a.r[k & 1];
    float2 *rn = a.r[(k + 1) & 1];
    // ||w||^2 (and gamma_0 at the first iteration)
    cgp_allsum2(a.pw, k == 0 ? a.pz[0] : nullptr, (int)nblk, sums, wred);
    if (k == 0) gam = sums[1];
    if (!(sums[0] > 0.0)) {
      final_it = k + 1;
      break;
    }
    const float alpha = (float)(gam / sums[0]);
    double own_sq = 0.0;
    for (int idx = tid; idx < nP; idx += blockDim.x) {
      const int slot = idx / n, j = idx - slot * n;
      const size_t o = (size_t)nbs[slot] * n + j;
      C v = cfma(make_float2(-alpha, 0.f), cld(a.w + o), cld(ro + o));
      if (slot == 0) {
        cst(rn + o, v);
        a.e[o] = cfma(make_float2(alpha, 0.f), cld(pn + o), a.e[o]);
        own_sq += (double)v.x * v.x + (double)v.y * v.y;
      }
      if (j >= half) v = make_float2(-v.x, -v.y);
      vin[idx] = v;
    }
    __syncthreads();
    {
      C zv = apply();
      double t2 = 0.0;
      if (tid < n) {
        if (tid >= half) zv = make_float2(-zv.x, -zv.y);
        cst(a.z + (size_t)s * n + tid, zv);
        t2 = (double)zv.x * zv.x + (double)zv.y * zv.y;
      }
      double v4[4] = {0.0, 0.0, t2, own_sq};
      block_sum<4>(v4, wred);
      if (tid == 0) {
        cstd(a.pz[(k + 1) & 1] + s, v4[2]);
        cstd(a.pr + s, v4[3]);
      }
    }
    ++k;
    if (!cgp_barrier(a.bar, ++round * nblk, a.fail, a.spin, &bar_ok)) {
      final_it = k;
      break;
    }
  }
  if (s == 0 && tid == 0) {
    a.it[0] = final_it;
    a.it[1] = final_it;
    a.done[0] = 1;
  }
}

template <typename S>
hipError_t cgnr_persistent(const Geom &g, int n, const S *L, const CgPersist &a, hipStream_t st) {
  const int rs = coarse_split(n, g.V);
  if (rs != 1 || n > COARSE_NMAX) return hipErrorInvalidValue;
  const int th = coarse_threads(n, g.V);
  const bool rw4 = sizeof(S) == 4 && n % 4 == 0;
  const int RW = sizeof(S) == 4 ? (rw4 ? 4 : 2) : 2;
  const int G = th / (n / RW);
  if ((9 * n + G - 1) / G > CGP_PMAX || th > 512 || 9 * n > 2 * th) return hipErrorInvalidValue;
  CgPersist args = a;
  Geom gg = g;
  const S *LL = L;
  int nn = n;
  void *kargs[] = {&gg, &nn, &LL, &args};
  // entries per thread decide the register array: 8 where they fit
  const bool p8 = (9 * n + G - 1) / G <= 8;
  const void *fn;
  if constexpr (sizeof(S) == 4) {
    if (rw4 && !p8) return hipErrorInvalidValue;  // 16 four-row entries would spill
    if (rw4) fn = reinterpret_cast<const void *>(&k_cgnr_persistent<S, 4, 8>);
    else fn = p8 ? reinterpret_cast<const void *>(&k_cgnr_persistent<S, 2, 8>)
                 : reinterpret_cast<const void *>(&k_cgnr_persistent<S, 2, 16>);
  } else {
    fn = p8 ? reinterpret_cast<const void *>(&k_cgnr_persistent<S, 2, 8>)
            : reinterpret_cast<const void *>(&k_cgnr_persistent<S, 2, 16>);
  }
  return hipLaunchCooperativeKernel(fn, dim3(g.V), dim3(th), kargs, 0, st);
}
template hipError_t cgnr_persistent<chalf>(const Geom &, int, const chalf *, const CgPersist &, hipStream_t);
template hipError_t cgnr_persistent<float2>(const Geom &, int, const float2 *, const CgPersist &, hipStream_t);

// ------------------------------------------------------------ matrix cores
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <typename S> __device__ __forceinline__ float2 op_f32(const S &v) { return cvt<float2>(v); }

// Four consecutive operator entries (16-byte aligned) as FP32 complex.
__device__ __forceinline__ void load4_op(const chalf *p, float2 (&o)[4]) {
  const chalf4 v = *reinterpret_cast<const chalf4 *>(p);
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = cvt<float2>(v.v[q]);
}
__device__ __forceinline__ void load4_op(const float2 *p, float2 (&o)[4]) {
  const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
  o[0] = make_float2(a.x, a.y);
  o[1] = make_float2(a.z, a.w);
  o[2] = make_float2(b.x, b.y);
  o[3] = make_float2(b.z, b.w);
}

constexpr int MMA_NR = 16;  // right-hand sides per GEMM tile (N of the MFMA)
constexpr int MMA_U = 8;    // operator k-steps per load batch

// Sums of nr partial vectors (np entries each) over the workgroup, all in one
// pass; results in every thread.
__device__ __forceinline__ void block_allsum_multi(const double *__restrict__ p, int np, int nr,
                                                   double (&out)[MMA_NR], double (*lds)[MMA_NR]) {
#pragma unroll
  for (int r = 0; r < MMA_NR; ++r) out[r] = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
#pragma unroll
    for (int r = 0; r < MMA_NR; ++r)
      if (r < nr) out[r] += p[(size_t)r * np + i];
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int r = 0; r < MMA_NR; ++r) out[r] = wave_sum(out[r]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int r = 0; r < MMA_NR; ++r) lds[w][r] = out[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < MMA_NR; ++r) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += lds[q][r];
    out[r] = t;
  }
  __syncthreads();
}

// One workgroup per coarse site, MT = ceil(n / 16) row tiles times KS groups
// of the K range: wavefront (mt, ks) accumulates rows 16 mt .. 16 mt + 15 of
// all right-hand sides over the k-steps ks, ks + KS, ... (4 of the 9n
// (slot, column) pairs per step).  MFMA lane layouts (16x16x4, FP32):
// A lane l = (row l % 16, k l / 16); B lane l = (k l / 16, column l % 16);
// C lane l = (rows 4 (l / 16) + 0..3, column l % 16).
template <typename S, int KS, bool RM>
__global__ __launch_bounds__(1024) void k_coarse_mma(Geom g, int n, const S *__restrict__ L,
                                                     const float2 *__restrict__ in, float2 *__restrict__ out,
                                                     int nrhs, int dagger, double *__restrict__ part, int pw,
                                                     const int *__restrict__ done, CgCheck chk) {
  extern __shared__ float2 bl[];  // staged inputs [9n][nrhs]; reused for the K-split reduction
  __shared__ double wred[16][MMA_NR];
  __shared__ double pr[4][64][3];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (done != nullptr) {
    bool all = true;
    for (int r = 0; r < nrhs; ++r) all = all && done[r] != 0;
    if (all) return;
  }
  if (chk.part_r != nullptr) {
    double rr[MMA_NR];
    block_allsum_multi(chk.part_r, chk.np_r, nrhs, rr, wred);
    bool allconv = true;
    for (int r = 0; r < nrhs; ++r) {
      if (chk.done[r]) continue;
      const double *cg = chk.cg + (size_t)r * CG_NS;
      const int iter = chk.it_in[r];
      const bool conv = !(rr[r] > cg[4] * cg[3]) || iter + 1 >= chk.maxit;
      if (blockIdx.x == 0 && tid == 0) {
        chk.it_out[r] = iter + 1;
        if (conv) chk.done[r] = 1;
      }
      allconv = allconv && conv;
    }
    if (allconv) return;
  }
  const uint32_t s = xcd_remap(blockIdx.x, gridDim.x);
  const int K = 9 * n, half = n >> 1;
  const int MT = (n + 15) >> 4;
  const int mt = wv % MT, ks = wv / MT;
  const int arow = mt * 16 + (lane & 15), kq = lane >> 4, col = lane & 15;
  const bool arow_ok = arow < n, col_ok = col < nrhs;
  const int colc = col_ok ? col : 0;
  // Operator loads are unconditional (indices clamped into the site's block,
  // out-of-range values zeroed afterwards) and double-buffered MMA_U k-steps
  // ahead, so every wavefront keeps MMA_U loads in flight; the first batch is
  // issued before the input staging.
  // Column-major operator (RM false): lane (row, kq) reads entry (row, k)
  // of each k-step, rows contiguous.  Row-major copy (RM true): lane (row,
  // kq) reads the four consecutive columns 16 b + 4 kq .. + 3 of its row in
  // one access for the four k-steps of block b (k-slot kq of step u takes
  // column 16 b + 4 kq + u; the sum over K does not depend on term order).
  const S *La = RM ? L + (size_t)s * K * n + (size_t)(arow_ok ? arow : 0) * K
                   : L + (size_t)s * K * n + (arow_ok ? arow : 0);
  const int KQ = (K + 3) >> 2;
  const int nq = RM ? 0 : (KQ - ks + KS - 1) / KS;  // k-steps of this wavefront
  const int KB = (K + 15) >> 4;
  const int nbk = RM ? (ks < KB ? (KB - ks + KS - 1) / KS : 0) : 0;  // k-blocks of this wavefront
  float2 abuf[2][MMA_U];
  auto load_batch = [&](float2 (&dst)[MMA_U], int q0) {
    if constexpr (RM) {
#pragma unroll
      for (int u = 0; u < MMA_U / 4; ++u) {
        const int k0 = min(16 * (ks + min(q0 + u, nbk - 1) * KS) + 4 * kq, K - 4);
        float2 o[4];
        load4_op(La + k0, o);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[4 * u + q] = o[q];
      }
    } else {
#pragma unroll
      for (int u = 0; u < MMA_U; ++u) {
        const int kk = min(4 * (ks + (q0 + u) * KS) + kq, K - 1);
        dst[u] = op_f32(La[(size_t)kk * n]);
      }
    }
  };
  if (RM ? nbk > 0 : true) load_batch(abuf[0], 0);
  __shared__ uint32_t nbs[9];
  if (tid < 9) nbs[tid] = slot_site(g, s, tid);
  __syncthreads();
  {
    // A thread stages 9 nrhs / (blockDim / n) entries (up to 36): SU of
    // them are loaded before any is stored, so that their round trips
    // overlap instead of one load, wait and store after another (the
    // 12-RHS level-1 stencil of 32^3 x 64: 0.400 -> 0.366 ms with SU = 8;
    // 0.373 with 4, 0.369 with 16).
    constexpr int SU = 8;
    const int jj = tid % n, tstep = (int)blockDim.x / n, nt = 9 * nrhs;
    const bool stager = tid < tstep * n;
    for (int t0 = tid / n; stager && t0 < nt; t0 += SU * tstep) {
      float2 v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int t = t0 + u * tstep;
        if (t < nt) v[u] = in[((size_t)(t % nrhs) * g.V + nbs[t / nrhs]) * n + jj];
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int t = t0 + u * tstep;
        if (t < nt) {
          const float2 w = (dagger && jj >= half) ? make_float2(-v[u].x, -v[u].y) : v[u];
          bl[((t / nrhs) * n + jj) * nrhs + (t % nrhs)] = w;
        }
      }
    }
  }
  __syncthreads();
  // Complex products with three real MFMAs each (Gauss): cre = sum a.x b.x,
  // c2 = sum a.y b.y, cim = sum (a.x + a.y)(b.x + b.y); then re = cre - c2
  // and im = cim - cre - c2.
  floatx4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f}, c2 = {0.f, 0.f, 0.f, 0.f};
  if constexpr (RM) {
    constexpr int BB = MMA_U / 4;  // k-blocks per load batch
    for (int b0 = 0; b0 < nbk; b0 += 2 * BB) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int bb = b0 + h * BB;
        if (bb >= nbk) break;
        if (bb + BB < nbk) load_batch(abuf[h ^ 1], bb + BB);
#pragma unroll
        for (int u = 0; u < BB; ++u) {
          const bool bok = bb + u < nbk;
          const int kbase = 16 * (ks + (bb + u) * KS) + 4 * kq;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int kk = kbase + q;
            const bool kok = bok && kk < K;
            const float2 a = (kok && arow_ok) ? abuf[h][4 * u + q] : make_float2(0.f, 0.f);
            const float2 bv = bl[min(kk, K - 1) * nrhs + colc];
            const float2 b = (kok && col_ok) ? bv : make_float2(0.f, 0.f);
            cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cre, 0, 0, 0);
            c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, c2, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, cim, 0, 0, 0);
          }
        }
      }
    }
  }
  for (int q0 = 0; q0 < nq; q0 += 2 * MMA_U) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int qb = q0 + h * MMA_U;
      if (qb >= nq) break;
      if (qb + MMA_U < nq) load_batch(abuf[h ^ 1], qb + MMA_U);
#pragma unroll
      for (int u = 0; u < MMA_U; ++u) {
        const int kk = 4 * (ks + (qb + u) * KS) + kq;
        const bool kok = qb + u < nq && kk < K;
        const float2 a = (kok && arow_ok) ? abuf[h][u] : make_float2(0.f, 0.f);
        const float2 bv = bl[min(kk, K - 1) * nrhs + colc];
        const float2 b = (kok && col_ok) ? bv : make_float2(0.f, 0.f);
        cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cre, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, c2, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, cim, 0, 0, 0);
      }
    }
  }
  cim = cim - cre - c2;
  cre = cre - c2;
  // centre inputs of this lane's output rows (for the <out, in> partial)
  float2 ctr[4];
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    const int row = mt * 16 + 4 * kq + r4;
    ctr[r4] = (row < n && col_ok) ? bl[row * nrhs + col] : make_float2(0.f, 0.f);
  }
  if (KS > 1) {
    __syncthreads();
    float *red = reinterpret_cast<float *>(bl);
    if (ks > 0) {
      float *d = red + (((size_t)(ks - 1) * MT + mt) * 64 + lane) * 8;
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        d[r4] = cre[r4];
        d[4 + r4] = cim[r4];
      }
    }
    __syncthreads();
    if (ks == 0) {
      for (int q = 1; q < KS; ++q) {
        const float *d = red + (((size_t)(q - 1) * MT + mt) * 64 + lane) * 8;
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          cre[r4] += d[r4];
          cim[r4] += d[4 + r4];
        }
      }
    }
  }
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  if (ks == 0) {
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      const int row = mt * 16 + 4 * kq + r4;
      if (row < n && col_ok) {
        float2 o = make_float2(cre[r4], cim[r4]);
        if (dagger && row >= half) o = make_float2(-o.x, -o.y);
        out[((size_t)col * g.V + s) * n + row] = o;
        const float2 c = ctr[r4];
        t0 += (double)o.x * c.x + (double)o.y * c.y;
        t1 += (double)o.x * c.y - (double)o.y * c.x;
        t2 += (double)o.x * o.x + (double)o.y * o.y;
      }
    }
  }
  if (part == nullptr) return;
  if (ks == 0) {
    pr[mt][lane][0] = t0;
    pr[mt][lane][1] = t1;
    pr[mt][lane][2] = t2;
  }
  __syncthreads();
  if (tid < nrhs) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int m = 0; m < MT; ++m)
      for (int g4 = 0; g4 < 4; ++g4) {
        a0 += pr[m][g4 * 16 + tid][0];
        a1 += pr[m][g4 * 16 + tid][1];
        a2 += pr[m][g4 * 16 + tid][2];
      }
    double *p = part + ((size_t)tid * gridDim.x + blockIdx.x) * pw;
    if (pw == 1) {
      p[0] = a2;
    } else {
      p[0] = a0;
      p[1] = a1;
      p[2] = a2;
    }
  }
}

static size_t mma_lds_bytes(int n, int nrhs, int ks) {
  const size_t b = (size_t)9 * n * nrhs * sizeof(float2);
  const size_t r = (size_t)(ks - 1) * ((n + 15) / 16) * 64 * 8 * sizeof(float);
  return b > r ? b : r;
}

bool coarse_mma_ok(int n, int nrhs, int variant) {
  const int ks = variant & 7;
  if (n > COARSE_NMAX || nrhs < 1 || nrhs > MMA_NR) return false;
  if (variant != ks && (variant != (ks | 8) || n % 4 != 0)) return false;  // row-major copy: 16-byte rows
  if (ks != 1 && ks != 2 && ks != 4) return false;
  if (((n + 15) / 16) * ks * 64 > 1024) return false;
  return mma_lds_bytes(n, nrhs, ks) <= 56 * 1024;  // + 8 KB static LDS
}

// Workgroups per coarse site.  Splitting a site's rows over several
// workgroups was measured slower at every coarse-lattice size here (it halves
// the contiguous column segments), so each site is one workgroup; the
// general form is kept for the row bookkeeping of the kernel.
int coarse_split(int, uint32_t) { return 1; }

// Threads per workgroup: G groups of the workgroup's rows (FP64 count), up to
// 512 threads (measured best against 256 and 1024) and at most 64 groups.
int coarse_threads(int n, uint32_t V) {
  const int nr = n / coarse_split(n, V);
  int G = 512 / nr;
  if (G > 64) G = 64;
  if (G < 1) G = 1;
  return (G * nr + 63) / 64 * 64;
}

template <typename R, typename S>
hipError_t coarse_apply_k(const Geom &g, int n, const S *L, const c_t<R> *in, c_t<R> *out, int nrhs, int dagger,
                          const CoarseArgs &a, hipStream_t st) {
  CgCheck c{};
  if (a.chk) c = *a.chk;
  if constexpr (sizeof(R) == 4) {
    if (a.variant > 0) {
      if (a.fuse && a.fuse->kind) return hipErrorInvalidValue;  // fusion is per-RHS kernel only
      const int ks = a.variant & 7;
      const bool rm = (a.variant & 8) != 0;
      if (!coarse_mma_ok(n, nrhs, a.variant)) return hipErrorInvalidValue;
      if (rm && a.lt == nullptr) return hipErrorInvalidValue;
      const S *Lk = rm ? static_cast<const S *>(a.lt) : L;
      const dim3 block(64 * ((n + 15) / 16) * ks);
      const size_t lds = mma_lds_bytes(n, nrhs, ks);
#define MG_MMA_LAUNCH(KSV, RMV)                                                                                 \
  hipLaunchKernelGGL((k_coarse_mma<S, KSV, RMV>), dim3(g.V), block, lds, st, g, n, Lk, in, out, nrhs, dagger, \
                     a.part, a.pw, a.done, c)
      if (ks == 1) {
        if (rm) MG_MMA_LAUNCH(1, true);
        else MG_MMA_LAUNCH(1, false);
      } else if (ks == 2) {
        if (rm) MG_MMA_LAUNCH(2, true);
        else MG_MMA_LAUNCH(2, false);
      } else {
        if (rm) MG_MMA_LAUNCH(4, true);
        else MG_MMA_LAUNCH(4, false);
      }
#undef MG_MMA_LAUNCH
      return hipGetLastError();
    }
  } else {
    if (a.variant > 0) return hipErrorInvalidValue;
  }
  const dim3 grid(g.V * coarse_split(n, g.V) * nrhs);
  dim3 block(coarse_threads(n, g.V));
  CgFuse f{};
  if (a.fuse) f = *a.fuse;
  if constexpr (sizeof(S) == 16) {
    hipLaunchKernelGGL((k_coarse<R, S, 1>), grid, block, 0, st, g, n, L, in, out, nrhs, dagger, a.part, a.pw, a.done,
                       c, f);
  } else if constexpr (sizeof(S) == 8) {
    hipLaunchKernelGGL((k_coarse<R, S, 2>), grid, block, 0, st, g, n, L, in, out, nrhs, dagger, a.part, a.pw, a.done,
                       c, f);
  } else {
    // half storage: four rows per 16-byte load when the rows of a workgroup
    // come in multiples of four, else two rows per 8-byte load
    if ((n / coarse_split(n, g.V)) % 4 == 0)
      hipLaunchKernelGGL((k_coarse<R, S, 4>), grid, block, 0, st, g, n, L, in, out, nrhs, dagger, a.part, a.pw, a.done,
                         c, f);
    else
      hipLaunchKernelGGL((k_coarse<R, S, 2>), grid, block, 0, st, g, n, L, in, out, nrhs, dagger, a.part, a.pw, a.done,
                         c, f);
  }
  return hipGetLastError();
}

template hipError_t coarse_apply_k<double, double2>(const Geom &, int, const double2 *, const double2 *, double2 *,
                                                    int, int, const CoarseArgs &, hipStream_t);
template hipError_t coarse_apply_k<float, float2>(const Geom &, int, const float2 *, const float2 *, float2 *, int,
                                                  int, const CoarseArgs &, hipStream_t);
template hipError_t coarse_apply_k<float, chalf>(const Geom &, int, const chalf *, const float2 *, float2 *, int,
                                                 int, const CoarseArgs &, hipStream_t);

}  // namespace mg
