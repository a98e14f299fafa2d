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
// One workgroup per coarse site: the nine input vectors are staged in LDS;
// thread (i, g) owns row i and a strided subset g, g+G, ... of the 9n
// (slot, column) pairs, so each group of n threads streams one contiguous
// column and the whole workgroup reads a contiguous G*n-entry window of the
// site's 9 n^2 entries per step (coalesced, HBM-bound).  The G partial row
// sums are combined in LDS in a fixed order (deterministic).
#include "kernels.h"

namespace mg {

template <typename R>
__global__ __launch_bounds__(256) void k_coarse(Geom g, int n, const c_t<R> *__restrict__ L,
                                                const c_t<R> *__restrict__ in, c_t<R> *__restrict__ out,
                                                int dagger, double *__restrict__ partials, int pw,
                                                const int *__restrict__ done) {
  using C = c_t<R>;
  if (done != nullptr && done[blockIdx.y]) return;
  __shared__ C vin[9 * COARSE_NMAX];
  __shared__ C red[256];
  __shared__ double wred[4 * 3];
  const uint32_t s = xcd_remap(blockIdx.x, gridDim.x);
  const size_t rhs_off = (size_t)blockIdx.y * g.V * n;
  in += rhs_off;
  out += rhs_off;
  const Coords k = decode(g, s);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 9 * n; idx += blockDim.x) {
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
  const int G = blockDim.x / n;
  const int i = tid % n, grp = tid / n;
  C acc = mk<C>(0, 0);
  if (grp < G) {
    const C *Ls = L + (size_t)s * 9 * n * n + i;
    int p = grp;
#pragma unroll 4
    for (; p < 9 * n; p += G) acc = cfma(Ls[(size_t)p * n], vin[p], acc);
  }
  red[tid] = acc;
  __syncthreads();
  // partials (pw = 1): ||out||^2;  (pw = 3): <out, in>, ||out||^2 (in = centre)
  double t[3] = {0.0, 0.0, 0.0};
  if (tid < n) {
    C sum = red[tid];
    for (int q = 1; q < G; ++q) sum = cadd(sum, red[q * n + tid]);
    if (dagger && tid >= (n >> 1)) sum = mk<C>(-sum.x, -sum.y);
    out[(size_t)s * n + tid] = sum;
    const C c = vin[tid];
    t[0] = (double)sum.x * c.x + (double)sum.y * c.y;
    t[1] = (double)sum.x * c.y - (double)sum.y * c.x;
    t[2] = (double)sum.x * sum.x + (double)sum.y * sum.y;
  }
  if (partials != nullptr) {
    block_sum<3>(t, wred);
    if (tid == 0) {
      double *p = partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * pw;
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

int coarse_threads(int n) {
  int G = 256 / n;
  int t = G * n;
  return (t + 63) / 64 * 64;
}

template <typename R>
hipError_t coarse_apply_k(const Geom &g, int n, const c_t<R> *L, const c_t<R> *in, c_t<R> *out, int nrhs,
                          int dagger, double *partials, int pw, const int *done, hipStream_t st) {
  dim3 grid(g.V, nrhs);
  hipLaunchKernelGGL(k_coarse<R>, grid, dim3(coarse_threads(n)), 0, st, g, n, L, in, out, dagger, partials, pw,
                     done);
  return hipGetLastError();
}

template hipError_t coarse_apply_k<double>(const Geom &, int, const double2 *, const double2 *, double2 *, int,
                                           int, double *, int, const int *, hipStream_t);
template hipError_t coarse_apply_k<float>(const Geom &, int, const float2 *, const float2 *, float2 *, int, int,
                                          double *, int, const int *, hipStream_t);

}  // namespace mg
