// Launchers of the parallel-transport network kernels (ptc.hip).
#pragma once

#include "kernels.h"

namespace mg {

constexpr int PTC_HOPS = 9;      // T_0 and the eight hops
constexpr int PTC_MAX_OUT = 32;  // output channels (proposed vectors) at most
constexpr int PTC_WCHUNK = 16;   // site chunks of the weight-gradient reduction

// H[b * 9 + k] = T_k in[b] for cin channels (fields of 12 * Vpad entries).
hipError_t ptc_transport(const Geom &g, const float2 *U, const float2 *in, int cin, float2 *H, hipStream_t st);
// out[a] = sum_{b,k} W[a][b][k] H[b * 9 + k]  (W [cout][cin][9][4][4]).
hipError_t ptc_mix(const Geom &g, int cin, int cout, const float2 *W, const float2 *H, float2 *out, hipStream_t st);
// A[b * 9 + k] = sum_a W[a][b][k]^dag G[a].
hipError_t ptc_mix_adj(const Geom &g, int cin, int cout, const float2 *W, const float2 *G, float2 *A,
                       hipStream_t st);
// gin[b] = sum_k T_k^dag A[b * 9 + k].
hipError_t ptc_transport_adj(const Geom &g, const float2 *U, const float2 *A, int cin, float2 *gin, hipStream_t st);
// gW[a][b][k][s][t] = sum_{x,c} G_a(x)[s][c] conj(H_bk(x)[t][c]); part holds
// cout * cin * 9 * PTC_WCHUNK * 16 double2.
hipError_t ptc_wgrad(const Geom &g, int cin, int cout, const float2 *G, const float2 *H, double2 *part, float2 *gW,
                     hipStream_t st);
// Subspace fit per (aggregate, chirality): loss[0] = sum |V - Y C|^2 (not yet
// divided by Z), gY = -(2 / Z) E C^dag.  GR: 2 Vc ny (ny + nv) double2,
// C: 2 Vc ny nv double2, part: 2 Vc doubles; flag |= 1 on a singular block.
hipError_t ptc_fit(const Geom &g, int ny, int nv, const float2 *Y, const float2 *V, const double *Z, double2 *GR,
                   double2 *C, int *flag, float2 *gY, double *part, double *loss, hipStream_t st);
// out[0] = sum |x|^2 (part: 256 doubles).
hipError_t ptc_norm2(const float2 *x, size_t n, double *part, double *out, hipStream_t st);
hipError_t ptc_adam_k(float2 *W, const float2 *gW, float2 *m, float2 *v, size_t n, int step, double lr, double b1,
                      double b2, double eps, hipStream_t st);

}  // namespace mg
