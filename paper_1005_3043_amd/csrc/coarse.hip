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
#include "solver.h"

namespace mg {

constexpr int CO_CHUNK = 8;   // operator loads in flight per thread

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

template <typename R, typename S, int RW>
__global__ __launch_bounds__(512) void k_coarse(Geom g, int n, const S *__restrict__ L,
                                                 const c_t<R> *__restrict__ in, c_t<R> *__restrict__ out,
                                                 int dagger, double *__restrict__ partials, int pw,
                                                 const int *__restrict__ done, CgCheck chk) {
  using C = c_t<R>;
  using VT = typename OpVec<S, RW>::V;
  __shared__ C vin[9 * COARSE_NMAX];
  __shared__ C red[512 * RW];
  __shared__ double wred[8 * 3];
  const int rhs = blockIdx.y;
  if (done != nullptr && done[rhs]) return;
  if (chk.part_r != nullptr) {
    // CGNR convergence test on the residual of the update just made
    const double rr = block_allsum_partials(chk.part_r + (size_t)rhs * chk.np_r, chk.np_r, wred);
    const double *cg = chk.cg + (size_t)rhs * CG_NS;
    const int iter = chk.it_in[rhs];
    const bool conv = !(rr > cg[4] * cg[3]) || iter + 1 >= chk.maxit;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      chk.it_out[rhs] = iter + 1;
      if (conv) chk.done[rhs] = 1;
    }
    if (conv) return;
  }
  const uint32_t ws = xcd_remap(blockIdx.x, gridDim.x);
  const int RS = (int)(gridDim.x / g.V);
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
  // so that the two memory phases overlap.
  VT lv[CO_CHUNK];
  const bool on = grp < G;
#pragma unroll
  for (int q = 0; q < CO_CHUNK; ++q) {
    const int p = grp + q * G;
    lv[q] = (on && p < nP) ? Ls[(size_t)p * nu] : VT{};
  }
  const Coords k = decode(g, s);
  for (int idx = tid; idx < nP; idx += blockDim.x) {
    const int slot = idx / n, j = idx - slot * n;
    uint32_t site = s;
    if (slot > 0) {
      const int d = slot - 1, mu = d >> 1;
      site = (d & 1) ? nbr_bwd(g, s, k, mu) : nbr_fwd(g, s, k, mu);
    }
    C v = in[(size_t)site * n + j];
    if (dagger && j >= (n >> 1)) v = mk<C>(-v.x, -v.y);
    vin[idx] = v;
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
        lv[q] = p < nP ? Ls[(size_t)p * nu] : VT{};
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
  // partials (pw = 1): ||out||^2;  (pw = 3): <out, in>, ||out||^2 (in = centre)
  double t[3] = {0.0, 0.0, 0.0};
  if (tid < nr) {
    const int ipr = tid / RW, sub = tid % RW, row = r0 + tid;
    C sum = red[ipr * RW + sub];
    for (int q = 1; q < G; ++q) sum = cadd(sum, red[(q * npr + ipr) * RW + sub]);
    if (dagger && row >= (n >> 1)) sum = mk<C>(-sum.x, -sum.y);
    out[(size_t)s * n + row] = sum;
    const C c = vin[row];
    t[0] = (double)sum.x * c.x + (double)sum.y * c.y;
    t[1] = (double)sum.x * c.y - (double)sum.y * c.x;
    t[2] = (double)sum.x * sum.x + (double)sum.y * sum.y;
  }
  if (partials != nullptr) {
    block_sum<3>(t, wred);
    if (tid == 0) {
      double *p = partials + ((size_t)rhs * gridDim.x + blockIdx.x) * pw;
      if (pw == 1) {
        p[0] = t[2];
      } else {
        p[0] = t[0];
        p[1] = t[1];
        p[2] = t[2];
      }
    }
  }
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
                          double *partials, int pw, const int *done, hipStream_t st, const CgCheck *chk) {
  dim3 grid(g.V * coarse_split(n, g.V), nrhs);
  dim3 block(coarse_threads(n, g.V));
  CgCheck c{};
  if (chk) c = *chk;
  if constexpr (sizeof(S) == 16) {
    hipLaunchKernelGGL((k_coarse<R, S, 1>), grid, block, 0, st, g, n, L, in, out, dagger, partials, pw, done, c);
  } else if constexpr (sizeof(S) == 8) {
    hipLaunchKernelGGL((k_coarse<R, S, 2>), grid, block, 0, st, g, n, L, in, out, dagger, partials, pw, done, c);
  } else {
    // half storage: four rows per 16-byte load when the rows of a workgroup
    // come in multiples of four, else two rows per 8-byte load
    if ((n / coarse_split(n, g.V)) % 4 == 0)
      hipLaunchKernelGGL((k_coarse<R, S, 4>), grid, block, 0, st, g, n, L, in, out, dagger, partials, pw, done, c);
    else
      hipLaunchKernelGGL((k_coarse<R, S, 2>), grid, block, 0, st, g, n, L, in, out, dagger, partials, pw, done, c);
  }
  return hipGetLastError();
}

template hipError_t coarse_apply_k<double, double2>(const Geom &, int, const double2 *, const double2 *, double2 *,
                                                    int, int, double *, int, const int *, hipStream_t,
                                                    const CgCheck *);
template hipError_t coarse_apply_k<float, float2>(const Geom &, int, const float2 *, const float2 *, float2 *, int,
                                                  int, double *, int, const int *, hipStream_t, const CgCheck *);
template hipError_t coarse_apply_k<float, chalf>(const Geom &, int, const chalf *, const float2 *, float2 *, int,
                                                 int, double *, int, const int *, hipStream_t, const CgCheck *);

}  // namespace mg
