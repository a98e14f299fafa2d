// Fine-level Wilson-Dirac operator, Eq. (2):
//   (D psi)(x) = (4+m) psi(x) - 1/2 sum_mu [ eta (1-gamma_mu) U_mu(x) psi(x+mu)
//                                          + eta (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// eta = -1 on hops across an antiperiodic time boundary.
//
// The spin projection (wilson_site.h) reduces each hop to a half spinor and
// two SU(3) mat-vecs: 1320 flops per site for all eight hops.
//
// One thread per site of the site-blocked, tile-interleaved layout (two
// right-hand sides per thread when there are several).  The loop over mu is
// rolled (wave-uniform): both hops of one direction issue their 42 (or 36
// with compressed links) loads together, then compute, which doubles the
// loads in flight per wave compared with one hop at a time.  Links are either stored in full (9
// complex) or as their first two rows (6 complex, NL = 6); the third row of an
// SU(3) matrix is the complex conjugate of the cross product of the first two,
// which trades 42 flops per link for a third less link traffic.
#include <type_traits>

#include "kernels.h"
#include "wilson_site.h"

namespace mg {

template <typename C> __host__ __device__ __forceinline__ void reconstruct_row2(C (&u)[9]) {
  // row 2 = conj(row0 x row1)
  const C a = csub(cmul(u[1], u[5]), cmul(u[2], u[4]));
  const C b = csub(cmul(u[2], u[3]), cmul(u[0], u[5]));
  const C c = csub(cmul(u[0], u[4]), cmul(u[1], u[3]));
  u[6] = mk<C>(a.x, -a.y);
  u[7] = mk<C>(b.x, -b.y);
  u[8] = mk<C>(c.x, -c.y);
}

template <int NL, typename C, typename S>
__device__ __forceinline__ void load_link_t(C (&u)[9], const S *__restrict__ U, int mu, uint32_t s) {
#pragma unroll
  for (int e = 0; e < NL; ++e) u[e] = cvt<C>(U[fidx(s, mu * NL + e, 4 * NL)]);
  if constexpr (NL == 6) reconstruct_row2(u);
}

// Full stencil at one site: res = D psi at s, ctr = psi(s).  The input
// spinors may be stored in a narrower type TI than the arithmetic type C.
template <int NL, typename C, typename S, typename TI>
__device__ __forceinline__ void dslash_site(C (&res)[12], C (&ctr)[12], const Geom &g, uint32_t s,
                                                     const S *__restrict__ U, const TI *__restrict__ in,
                                                     decltype(C::x) diag) {
  using R = decltype(C::x);
  const Coords k = decode(g, s);
  C acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = mk<C>(0, 0);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    C pf[12], pb[12], uf[9], ub[9];
    const uint32_t sf = nbr_fwd(g, s, k, mu), sb = nbr_bwd(g, s, k, mu);
    R ef = 1, eb = 1;
    if (mu == 3 && g.antiperiodic) {
      if (k.o[3] == g.b[3] - 1 && k.c[3] == g.C[3] - 1) ef = -1;
      if (k.o[3] == 0 && k.c[3] == 0) eb = -1;
    }
    load_site(pf, in, sf);
    load_site(pb, in, sb);
    load_link_t<NL>(uf, U, mu, s);
    load_link_t<NL>(ub, U, mu, sb);
    hop_dispatch<true>(mu, acc, pf, uf, ef);
    hop_dispatch<false>(mu, acc, pb, ub, eb);
  }
  load_site(ctr, in, s);
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    res[i].x = fma(diag, ctr[i].x, (R)-0.5 * acc[i].x);
    res[i].y = fma(diag, ctr[i].y, (R)-0.5 * acc[i].y);
  }
}

// The stencil at one site for K right-hand sides (input stride vs between
// them): each direction's two links are loaded once and applied to all K.
// Only the first kv are distinct; the spare slots repeat the last of them.
template <int K, int NL, typename C, typename S, typename TI>
__device__ __forceinline__ void dslash_site_k(C (&res)[K][12], C (&ctr)[K][12], const Geom &g, uint32_t s,
                                              const S *__restrict__ U, const TI *__restrict__ in, size_t vs, int kv,
                                              decltype(C::x) diag) {
  using R = decltype(C::x);
  const Coords kk = decode(g, s);
  C acc[K][12];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[k][i] = mk<C>(0, 0);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    const uint32_t sf = nbr_fwd(g, s, kk, mu), sb = nbr_bwd(g, s, kk, mu);
    R ef = 1, eb = 1;
    if (mu == 3 && g.antiperiodic) {
      if (kk.o[3] == g.b[3] - 1 && kk.c[3] == g.C[3] - 1) ef = -1;
      if (kk.o[3] == 0 && kk.c[3] == 0) eb = -1;
    }
    C u[9];
    load_link_t<NL>(u, U, mu, s);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      C p[12];
      load_site(p, in + (size_t)(k < kv ? k : kv - 1) * vs, sf);
      hop_dispatch<true>(mu, acc[k], p, u, ef);
    }
    load_link_t<NL>(u, U, mu, sb);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      C p[12];
      load_site(p, in + (size_t)(k < kv ? k : kv - 1) * vs, sb);
      hop_dispatch<false>(mu, acc[k], p, u, eb);
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    load_site(ctr[k], in + (size_t)(k < kv ? k : kv - 1) * vs, s);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      res[k][i].x = fma(diag, ctr[k][i].x, (R)-0.5 * acc[k][i].x);
      res[k][i].y = fma(diag, ctr[k][i].y, (R)-0.5 * acc[k][i].y);
    }
  }
}

// Block of `per` consecutive sites that workgroup bid of nblk visits.  The
// hardware deals workgroups to the eight XCDs round-robin; xcd_remap gives
// each XCD a contiguous range of the visiting order.  Where aggregates are
// whole blocks and the coarse z extent is divisible by 8, XCD k takes the
// aggregates of the z layers k C_z/8 .. (k+1) C_z/8 - 1 and walks them x
// fastest, then y, then t: the t neighbours of an aggregate are visited one
// x-y layer apart on the same XCD (L2), and the XCDs move through t in step,
// so the z neighbours another XCD needs are read at about the same time.
// (The aggregate-major order walks x, y, z, then t, with each XCD owning a
// t range; on 32^3 x 64 the visiting order above is 3-6 % faster, and
// walking 4x4-aggregate x-y quadrants in t or in z instead is 5-13 % slower.)
// Otherwise the order is the storage order.
__device__ __forceinline__ uint32_t visit_pos(uint32_t q, uint32_t nblk, const Geom &g, uint32_t per) {
  const uint32_t sub = g.vb / per;
  const uint32_t C0 = (uint32_t)g.C[0], C1 = (uint32_t)g.C[1], C2 = (uint32_t)g.C[2], C3 = (uint32_t)g.C[3];
  if ((nblk & 7u) == 0 && C2 % 8 == 0 && sub * per == g.vb && nblk == g.Vc * sub) {
    const uint32_t per_xcd = nblk >> 3, xcd = q / per_xcd, r0 = q - xcd * per_xcd;
    const uint32_t j = r0 % sub;
    uint32_t r = r0 / sub;
    const uint32_t cx = r % C0;
    r /= C0;
    const uint32_t cy = r % C1;
    r /= C1;
    const uint32_t ct = r % C3;
    const uint32_t cz = xcd * (C2 >> 3) + r / C3;
    return (cx + C0 * (cy + C1 * (cz + C2 * ct))) * sub + j;
  }
  return q;
}
__device__ __forceinline__ uint32_t visit_block(uint32_t bid, uint32_t nblk, const Geom &g, uint32_t per) {
  return visit_pos(xcd_remap(bid, nblk), nblk, g, per);
}

// 64-site tile (one wavefront) that wave w of workgroup bid (of nblk, with
// wpb waves each) visits.  With 4^4 aggregates a tile is the 4 x 4 x 4 cube
// at one time slice o_t of an aggregate; the tiles of XCD k are those of
// its z layers, walked x fastest, then y, then z, then the site time 4 c_t +
// o_t, so that a tile's time neighbours are one x-y layer of tiles away
// (1.6 MB of spinors and links for two FP32 right-hand sides on 32^3 x 64,
// against 6.3 MB for the layer of whole aggregates, more than an XCD's 4 MB
// L2): on 32^3 x 64 with 12 right-hand sides 2 % faster than visiting whole
// aggregates, 3-4 % fewer bytes fetched in FP32 and FP16.  Other shapes
// take visit_block's order, a wave per tile of each block.
__device__ __forceinline__ uint32_t visit_tile(uint32_t bid, uint32_t nblk, uint32_t w, uint32_t wpb,
                                               const Geom &g) {
  const uint32_t C0 = (uint32_t)g.C[0], C1 = (uint32_t)g.C[1], C2 = (uint32_t)g.C[2];
  const uint32_t ntile = nblk * wpb;
  if (g.vb == 256 && g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && (nblk & 7u) == 0 &&
      C2 % 8 == 0 && ntile == g.Vc * 4u) {
    const uint32_t q = xcd_remap(bid, nblk) * wpb + w;
    const uint32_t per_xcd = ntile >> 3, xcd = q / per_xcd;
    uint32_t r = q - xcd * per_xcd;
    const uint32_t cx = r % C0;
    r /= C0;
    const uint32_t cy = r % C1;
    r /= C1;
    const uint32_t nz = C2 >> 3, czl = r % nz, T = r / nz;
    const uint32_t cz = xcd * nz + czl, ct = T >> 2, ot = T & 3u;
    return (cx + C0 * (cy + C1 * (cz + C2 * ct))) * 4u + ot;
  }
  return visit_block(bid, nblk, g, 64 * wpb) * wpb + w;
}


// Minimum waves per SIMD requested from the register allocator (0 = none).
#ifndef MG_DSLASH_WAVES_F64
#define MG_DSLASH_WAVES_F64 0
#endif
#ifndef MG_DSLASH_WAVES_F32
#define MG_DSLASH_WAVES_F32 0
#endif
template <typename R> constexpr int dslash_waves() {
  return sizeof(R) == 8 ? MG_DSLASH_WAVES_F64 : MG_DSLASH_WAVES_F32;
}

// The MR step of the q recursion (DS_MRQ) at one site: res = D q_k and
// ctr = q_k on entry; q_{k+1} = q_k - a D q_k is written to qout and left in
// res, r_{k+1} = rprev - a q_k to rout and left in ctr (values as stored).
// rprev is read once by the launch: non-temporal loads keep L2 for the
// neighbour spinors and links (12-RHS FP32 3.37 -> 3.31 ms, FP16 class 2.41
// -> 2.33 ms on 32^3 x 64); likewise b of the residual form.
template <typename C, typename TO>
__device__ __forceinline__ void mrq_site(C (&res)[12], C (&ctr)[12], const TO *rprev, TO *qout, TO *rout,
                                         uint32_t s, double2 ad) {
  using R = decltype(C::x);
  const C ma = mk<C>((R)-ad.x, (R)-ad.y);
  C rp[12];
  load_site_nt(rp, rprev, s);
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const C t = res[i];
    res[i] = cfma(ma, t, ctr[i]);
    rp[i] = cfma(ma, ctr[i], rp[i]);
  }
  store_site<true>(qout, s, res);
  store_site<true>(rout, s, rp);
#pragma unroll
  for (int i = 0; i < 12; ++i) ctr[i] = rp[i];
}

// One site per thread, one right-hand side per grid row.  Input spinors
// are stored as TI, the output (and b of the residual mode) as TO: complex
// FP64 / FP32, or binary16 with a per-site scale (h16).
template <typename R, int MODE, int NL, typename S, typename TI, typename TO>
__global__ __launch_bounds__(256, dslash_waves<R>()) void k_dslash(Geom g, const S *__restrict__ U,
                                                const TI *__restrict__ in, TO *__restrict__ out,
                                                const TO *__restrict__ b, R diag,
                                                double *__restrict__ partials, MrqArgs<TO> mq) {
  using C = c_t<R>;
  in += (size_t)blockIdx.y * site_slots<TI>() * g.Vpad;
  const size_t off = (size_t)blockIdx.y * site_slots<TO>() * g.Vpad;
  out += off;
  const uint32_t s = visit_tile(blockIdx.x, gridDim.x, threadIdx.x >> 6, blockDim.x >> 6, g) * 64 + (threadIdx.x & 63);
  double red[3] = {0.0, 0.0, 0.0};
  if (s < g.V) {
    C res[12], ctr[12];
    dslash_site<NL, C>(res, ctr, g, s, U, in, diag);
    if constexpr (MODE == DS_RESID) {
      C bb[12];
      load_site_nt(bb, b + off, s);
#pragma unroll
      for (int i = 0; i < 12; ++i) res[i] = csub(bb[i], res[i]);
    }
    // the output is not read again by this launch: non-temporal stores leave
    // L2 to the neighbour spinors and links that are
    if constexpr (MODE == DS_MRQ) mrq_site(res, ctr, mq.rprev + off, out, mq.rout + off, s, mq.alpha[blockIdx.y]);
    else store_site<true>(out, s, res);
    if constexpr (MODE == DS_MR || MODE == DS_MRQ) {
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        // <q, r> = sum conj(q) r with q = D r (as stored), r = centre (DS_MRQ:
        // q_{k+1} and r_{k+1} as stored)
        red[0] += (double)res[i].x * ctr[i].x + (double)res[i].y * ctr[i].y;
        red[1] += (double)res[i].x * ctr[i].y - (double)res[i].y * ctr[i].x;
        red[2] += (double)res[i].x * res[i].x + (double)res[i].y * res[i].y;
      }
    }
  }
  if constexpr (MODE == DS_MR || MODE == DS_MRQ) {
    __shared__ double lds[16 * 3];
    block_sum<3>(red, lds);
    if (threadIdx.x == 0) {
      double *p = partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 3;
      p[0] = red[0];
      p[1] = red[1];
      p[2] = red[2];
    }
  }
}

// Several right-hand sides: K per thread (256-site workgroups), so that
// each direction's links are loaded once for all K; the workgroups of one
// group of K right-hand sides cover the lattice, grid.y = groups (K from
// mrhs_k below).  K = 2:
// on 32^3 x 64 with 12 right-hand sides, per right-hand side FP64 0.40 ms
// (one per thread: 0.47 ms), FP32 0.214 ms (0.231), FP16-stored links 0.195
// ms (0.198); K = 4 is slower in FP32 (0.248 ms: one wave per SIMD), and so
// is running the groups of one block back to back on an XCD (links from L2,
// but the spinor neighbours further apart: FP32 0.228 ms, more traffic).  A ragged last group repeats its last
// right-hand side in the spare slots and stores only the valid ones.
// Tile blocks per chunk of the right-hand-side-group order below (0: the
// groups one after another over the whole lattice).  On 32^3 x 64 with 12
// right-hand sides, 512 blocks (16 chunks, 25 MB of FP32 links each):
// FP32 2.52 -> 2.42 ms, FP16 class 1.74 -> 1.70 ms, FP64 4.77 -> 4.69 ms
// per launch, the MR q-recursion forms within 1 %; 128 and 2048 blocks
// gain less or lose.
#ifndef MG_DSLASH_CHUNK
#define MG_DSLASH_CHUNK 512
#endif
template <typename R, int MODE, int NL, typename S, int K, typename TI, typename TO>
__global__ __launch_bounds__(256, dslash_waves<R>()) void k_dslash_rb(Geom g, const S *__restrict__ U, const TI *__restrict__ in,
                                                   TO *__restrict__ out, const TO *__restrict__ b, R diag,
                                                   double *__restrict__ partials, int nrhs, MrqArgs<TO> mq) {
  using C = c_t<R>;
  // Right-hand-side groups in chunks of the lattice: the workgroups of the
  // launch (in dispatch order) take the groups of one chunk of RHS_CHUNK
  // tile blocks in turn before the next chunk, so that a chunk's links are
  // read again by the other groups while they are still in the last-level
  // cache.  The chunk is a multiple of 8 blocks: a workgroup's XCD (dispatch
  // order modulo 8) is the one its tile block belongs to.
  uint32_t bid = blockIdx.x;
  int grp = blockIdx.y;
  constexpr uint32_t CH = MG_DSLASH_CHUNK;
  if (CH > 0 && gridDim.x % CH == 0) {
    const uint32_t lin = blockIdx.y * gridDim.x + blockIdx.x, span = CH * gridDim.y;
    const uint32_t c = lin / span, rem = lin - c * span;
    grp = (int)(rem / CH);
    bid = c * CH + rem % CH;
  }
  const int r0 = grp * K;
  const uint32_t slot = bid, nslot = gridDim.x;
  const int kv = nrhs - r0 < K ? nrhs - r0 : K;
  const size_t vsi = (size_t)site_slots<TI>() * g.Vpad, vso = (size_t)site_slots<TO>() * g.Vpad;
  const uint32_t s = visit_tile(bid, gridDim.x, threadIdx.x >> 6, blockDim.x >> 6, g) * 64 + (threadIdx.x & 63);
  double red[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) red[k][0] = red[k][1] = red[k][2] = 0.0;
  if (s < g.V) {
    C res[K][12], ctr[K][12];
    dslash_site_k<K, NL, C>(res, ctr, g, s, U, in + (size_t)r0 * vsi, vsi, kv, diag);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k >= kv) break;
      const size_t off = (size_t)(r0 + k) * vso;
      if constexpr (MODE == DS_RESID) {
        C bb[12];
        load_site_nt(bb, b + off, s);
#pragma unroll
        for (int i = 0; i < 12; ++i) res[k][i] = csub(bb[i], res[k][i]);
      }
      if constexpr (MODE == DS_MRQ)
        mrq_site(res[k], ctr[k], mq.rprev + off, out + off, mq.rout + off, s, mq.alpha[r0 + k]);
      else
        store_site<true>(out + off, s, res[k]);
      if constexpr (MODE == DS_MR || MODE == DS_MRQ) {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          red[k][0] += (double)res[k][i].x * ctr[k][i].x + (double)res[k][i].y * ctr[k][i].y;
          red[k][1] += (double)res[k][i].x * ctr[k][i].y - (double)res[k][i].y * ctr[k][i].x;
          red[k][2] += (double)res[k][i].x * res[k][i].x + (double)res[k][i].y * res[k][i].y;
        }
      }
    }
  }
  if constexpr (MODE == DS_MR || MODE == DS_MRQ) {
    __shared__ double lds[4 * 3 * K];
    double v[3 * K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) v[3 * k + q] = red[k][q];
    block_sum<3 * K>(v, lds);
    if (threadIdx.x == 0) {
      for (int k = 0; k < kv; ++k) {
        double *p = partials + ((size_t)(r0 + k) * nslot + slot) * 3;
        p[0] = v[3 * k];
        p[1] = v[3 * k + 1];
        p[2] = v[3 * k + 2];
      }
    }
  }
}

// Right-hand sides per thread of the multi-RHS stencil: each link is loaded
// once per group.  Three for binary16 spinors (about 240 registers, two
// waves per SIMD as with two; the links are read four times per 12-RHS
// launch instead of six: 1.82 -> 1.72 ms plain, 2.55 -> 2.43 ms in the MR
// q-recursion form on 32^3 x 64) and for the outer method's FP64 operator on
// FP32-stored vectors (256 registers, no spill, one wave per SIMD: 7 % less
// time per step in that class), two otherwise (FP32 spinors: 2.51 against
// 2.58 ms with three, 3.40 against 3.38 ms; FP64 spinors spill with three).
template <typename R, typename TI> constexpr int mrhs_k() {
  return ((sizeof(R) == 4 && std::is_same<TI, h16>::value) || (sizeof(R) == 8 && std::is_same<TI, float2>::value))
             ? 3
             : 2;
}

int dslash_blocks(const Geom &g) { return div_up(g.V, 256); }
int dslash_partials(const Geom &g, int) { return dslash_blocks(g); }

template <typename R, int NL, typename S, typename TI, typename TO>
static hipError_t launch(const Geom &g, const S *U, const TI *in, TO *out, const TO *b, double diag, int nrhs,
                         DslashMode mode, double *partials, hipStream_t st, MrqArgs<TO> mq) {
  if (nrhs > 1) {
    constexpr int K = mrhs_k<R, TI>();
    dim3 grid(dslash_blocks(g), (nrhs + K - 1) / K);
    switch (mode) {
      case DS_PLAIN:
        hipLaunchKernelGGL((k_dslash_rb<R, DS_PLAIN, NL, S, K, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b,
                           (R)diag, partials, nrhs, mq);
        break;
      case DS_RESID:
        hipLaunchKernelGGL((k_dslash_rb<R, DS_RESID, NL, S, K, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b,
                           (R)diag, partials, nrhs, mq);
        break;
      case DS_MR:
        hipLaunchKernelGGL((k_dslash_rb<R, DS_MR, NL, S, K, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b,
                           (R)diag, partials, nrhs, mq);
        break;
      case DS_MRQ:
        if constexpr (std::is_same<TI, TO>::value && sizeof(R) == 4)
          hipLaunchKernelGGL((k_dslash_rb<R, DS_MRQ, NL, S, K, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b,
                             (R)diag, partials, nrhs, mq);
        else
          return hipErrorInvalidValue;
        break;
    }
    return hipGetLastError();
  }
  dim3 grid(dslash_blocks(g), nrhs);
  switch (mode) {
    case DS_PLAIN:
      hipLaunchKernelGGL((k_dslash<R, DS_PLAIN, NL, S, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b, (R)diag,
                         partials, mq);
      break;
    case DS_RESID:
      hipLaunchKernelGGL((k_dslash<R, DS_RESID, NL, S, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b, (R)diag,
                         partials, mq);
      break;
    case DS_MR:
      hipLaunchKernelGGL((k_dslash<R, DS_MR, NL, S, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b, (R)diag,
                         partials, mq);
      break;
    case DS_MRQ:
      if constexpr (std::is_same<TI, TO>::value && sizeof(R) == 4)
        hipLaunchKernelGGL((k_dslash<R, DS_MRQ, NL, S, TI, TO>), grid, dim3(256), 0, st, g, U, in, out, b, (R)diag,
                           partials, mq);
      else
        return hipErrorInvalidValue;
      break;
  }
  return hipGetLastError();
}

template <typename R, typename S, typename TI, typename TO>
hipError_t dslash(const Geom &g, const S *U, int nl, const TI *in, TO *out, const typename same_t<TO>::type *b,
                  double diag, int nrhs, DslashMode mode, double *partials, hipStream_t st,
                  MrqArgs<typename same_t<TO>::type> mq) {
  if (nl == 6) return launch<R, 6, S>(g, U, in, out, b, diag, nrhs, mode, partials, st, mq);
  return launch<R, 9, S>(g, U, in, out, b, diag, nrhs, mode, partials, st, mq);
}

// Plain stencil in FP64 arithmetic on FP32-stored input spinors (the
// flexible GCR applies D to the preconditioner's FP32 output this way).
hipError_t dslash_in32(const Geom &g, const double2 *U, int nl, const float2 *in, double2 *out, double diag,
                       int nrhs, hipStream_t st) {
  return dslash<double, double2, float2, double2>(g, U, nl, in, out, nullptr, diag, nrhs, DS_PLAIN, nullptr, st);
}

// ---------------------------------------------------------------- links
// Copy of the first two rows of every link (NL = 6 layout), and the largest
// deviation |row2 - conj(row0 x row1)| over all links (per-block maxima).
template <typename S>
__global__ __launch_bounds__(256) void k_compress_links(Geom g, const double2 *__restrict__ U,
                                                        S *__restrict__ Uc, double *__restrict__ blockmax) {
  __shared__ double lds[4];
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  double dev = 0.0;
  if (s < g.V) {
    for (int mu = 0; mu < 4; ++mu) {
      double2 u[9], w[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = U[fidx(s, mu * 9 + e, 36)];
#pragma unroll
      for (int e = 0; e < 9; ++e) w[e] = u[e];
      reconstruct_row2(w);
      for (int e = 6; e < 9; ++e) dev = fmax(dev, fabs(w[e].x - u[e].x) + fabs(w[e].y - u[e].y));
#pragma unroll
      for (int e = 0; e < 6; ++e) Uc[fidx(s, mu * 6 + e, 24)] = cvt<S>(u[e]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = lds[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, lds[w]);
    blockmax[blockIdx.x] = m;
  }
}

template <typename S>
hipError_t compress_links(const Geom &g, const double2 *U, S *Uc, double *blockmax, hipStream_t st) {
  hipLaunchKernelGGL(k_compress_links<S>, dim3(div_up(g.V, 256)), dim3(256), 0, st, g, U, Uc, blockmax);
  return hipGetLastError();
}

#define DSLASH_INST(R, S, TI, TO)                                                                      \
  template hipError_t dslash<R, S, TI, TO>(const Geom &, const S *, int, const TI *, TO *,                        \
                                           const typename same_t<TO>::type *, double, int, DslashMode, double *,   \
                                           hipStream_t, MrqArgs<typename same_t<TO>::type>);
DSLASH_INST(double, double2, double2, double2)
DSLASH_INST(float, float2, float2, float2)
DSLASH_INST(float, chalf, float2, float2)
DSLASH_INST(float, chalf, h16, h16)
DSLASH_INST(float, chalf, float2, h16)
#undef DSLASH_INST
template hipError_t compress_links<double2>(const Geom &, const double2 *, double2 *, double *, hipStream_t);
template hipError_t compress_links<float2>(const Geom &, const double2 *, float2 *, double *, hipStream_t);
template hipError_t compress_links<chalf>(const Geom &, const double2 *, chalf *, double *, hipStream_t);

}  // namespace mg
