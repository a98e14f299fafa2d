// C ABI of the learned null-vector proposal (parallel-transport network):
// context with packed FP32 links and work buffers, forward pass, fused
// forward + subspace-fit loss + backward pass, and the Adam step.
#include <cmath>
#include <new>

#include "mg_internal.h"
#include "ptc.h"

using namespace mg;

struct ptc_ctx {
  Geom g;
  int nh = 0, nout = 0, nt = 0;
  DevBuf<float2> U;          // links, 36 components
  DevBuf<float2> eta, psi1;  // input (1 channel), hidden (nh channels)
  DevBuf<float2> H1, H2;     // transports of the layer inputs: 9 and 9 nh fields
  DevBuf<float2> Y, gY, gpsi1, A2, A1, gin;
  DevBuf<float2> V;          // targets
  DevBuf<double> Z, loss, part, lpart;
  DevBuf<double2> wpart, GR, C;
  DevBuf<int> flag;
  DevBuf<float2> Wd;         // scratch for weights given as complex128
};

namespace {
int hipc(hipError_t e, const char *what) {
  if (e == hipSuccess) return MG_OK;
  set_error(hip_error_string(e, what));
  return MG_EHIP;
}
#define PK(expr) MG_TRY(hipc((expr), #expr))

int forward_impl(ptc_ctx *c, const float2 *W1, const float2 *W2, hipStream_t st) {
  const Geom &g = c->g;
  PK(ptc_transport(g, c->U, c->eta, 1, c->H1, st));
  PK(ptc_mix(g, 1, c->nh, W1, c->H1, c->psi1, st));
  PK(ptc_transport(g, c->U, c->psi1, c->nh, c->H2, st));
  PK(ptc_mix(g, c->nh, c->nout, W2, c->H2, c->Y, st));
  return MG_OK;
}
}  // namespace

extern "C" int ptc_create(const mg_lattice_t *lat, const int block[4], int n_hidden, int n_out, ptc_ctx_t **out) {
  set_error("");
  if (!out || !block) return (set_error("ptc_create: NULL argument"), MG_EINVAL);
  *out = nullptr;
  MG_TRY(check_lattice(lat));
  if (n_hidden < 1 || n_hidden > 64 || n_out < 1 || n_out > PTC_MAX_OUT)
    return (set_error("ptc_create: channel counts out of range"), MG_EINVAL);
  for (int mu = 0; mu < 4; ++mu)
    if (block[mu] < 1 || lat->L[mu] % block[mu] != 0)
      return (set_error("ptc_create: block must divide the lattice"), MG_ESHAPE);
  if ((long)block[0] * block[1] * block[2] * block[3] * 6 < n_out)
    return (set_error("ptc_create: blocks smaller than the number of outputs"), MG_ESHAPE);
  ptc_ctx *c = new (std::nothrow) ptc_ctx();
  if (!c) return (set_error("ptc_create: out of host memory"), MG_ENOMEM);
  c->g = make_geom(lat->L, block, lat->t_antiperiodic ? 1 : 0);
  c->nh = n_hidden;
  c->nout = n_out;
  const size_t F = (size_t)12 * c->g.Vpad;
  int rc = c->U.alloc(36 * (size_t)c->g.Vpad);
  if (rc == MG_OK) rc = c->eta.alloc(F);
  if (rc == MG_OK) rc = c->psi1.alloc(F * n_hidden);
  if (rc == MG_OK) rc = c->H1.alloc(F * PTC_HOPS);
  if (rc == MG_OK) rc = c->H2.alloc(F * PTC_HOPS * n_hidden);
  if (rc == MG_OK) rc = c->Y.alloc(F * n_out);
  if (rc == MG_OK) rc = c->Z.alloc(4);
  if (rc == MG_OK) rc = c->loss.alloc(4);
  if (rc == MG_OK) rc = c->part.alloc(256);
  if (rc == MG_OK) rc = c->flag.alloc(4);
  if (rc != MG_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return MG_OK;
}

extern "C" int ptc_set_links(ptc_ctx_t *c, const void *U, hipStream_t st) {
  set_error("");
  if (!c || !U) return (set_error("ptc_set_links: NULL argument"), MG_EINVAL);
  PK(pack_gauge<float>(c->g, (const double2 *)U, c->U, st));
  return MG_OK;
}

extern "C" int ptc_set_targets(ptc_ctx_t *c, const void *V, int nv, hipStream_t st) {
  set_error("");
  if (!c || !V) return (set_error("ptc_set_targets: NULL argument"), MG_EINVAL);
  if (nv < 1 || (long)c->nout * (c->nout + nv) > 2048)
    return (set_error("ptc_set_targets: nv out of range"), MG_EINVAL);
  const size_t F = (size_t)12 * c->g.Vpad;
  MG_TRY(c->V.alloc(F * nv));
  c->nt = nv;
  PK(pack_field<float>(c->g, (const double2 *)V, c->V, 12, nv, st));
  PK(ptc_norm2(c->V, F * nv, c->part, c->Z, st));
  return MG_OK;
}

extern "C" int ptc_forward(ptc_ctx_t *c, const void *W1, const void *W2, const void *eta, void *Y, hipStream_t st) {
  set_error("");
  if (!c || !W1 || !W2 || !eta || !Y) return (set_error("ptc_forward: NULL argument"), MG_EINVAL);
  PK(pack_field<float>(c->g, (const double2 *)eta, c->eta, 12, 1, st));
  MG_TRY(forward_impl(c, (const float2 *)W1, (const float2 *)W2, st));
  PK(unpack_field<float>(c->g, c->Y, (double2 *)Y, 12, c->nout, st));
  return MG_OK;
}

extern "C" int ptc_loss_grad(ptc_ctx_t *c, const void *W1, const void *W2, const void *eta, double *loss, void *gW1,
                             void *gW2, hipStream_t st) {
  set_error("");
  if (!c || !W1 || !W2 || !eta || !loss || !gW1 || !gW2)
    return (set_error("ptc_loss_grad: NULL argument"), MG_EINVAL);
  if (c->nt < 1) return (set_error("ptc_loss_grad: no targets set"), MG_EINVAL);
  const Geom &g = c->g;
  const size_t F = (size_t)12 * g.Vpad;
  const int nh = c->nh, no = c->nout, nt = c->nt;
  MG_TRY(c->gY.alloc(F * no));
  MG_TRY(c->gpsi1.alloc(F * nh));
  MG_TRY(c->A2.alloc(F * PTC_HOPS * nh));
  MG_TRY(c->A1.alloc(F * PTC_HOPS));
  MG_TRY(c->lpart.alloc(2 * (size_t)g.Vc));
  MG_TRY(c->GR.alloc(2 * (size_t)g.Vc * no * (no + nt)));
  MG_TRY(c->C.alloc(2 * (size_t)g.Vc * no * nt));
  MG_TRY(c->wpart.alloc((size_t)no * nh * PTC_HOPS * PTC_WCHUNK * 16));
  PK(pack_field<float>(g, (const double2 *)eta, c->eta, 12, 1, st));
  MG_TRY(forward_impl(c, (const float2 *)W1, (const float2 *)W2, st));
  PK(hipMemsetAsync(c->flag, 0, sizeof(int), st));
  PK(ptc_fit(g, no, nt, c->Y, c->V, c->Z, c->GR, c->C, c->flag, c->gY, c->lpart, c->loss, st));
  // layer 2: weight gradient from (gY, H2); gradient into psi1
  PK(ptc_wgrad(g, nh, no, c->gY, c->H2, c->wpart, (float2 *)gW2, st));
  PK(ptc_mix_adj(g, nh, no, (const float2 *)W2, c->gY, c->A2, st));
  PK(ptc_transport_adj(g, c->U, c->A2, nh, c->gpsi1, st));
  // layer 1: weight gradient from (gpsi1, H1)
  PK(ptc_wgrad(g, 1, nh, c->gpsi1, c->H1, c->wpart, (float2 *)gW1, st));
  double h[2];
  int bad = 0;
  PK(hipMemcpyAsync(h, c->loss, sizeof(double), hipMemcpyDeviceToHost, st));
  PK(hipMemcpyAsync(h + 1, c->Z, sizeof(double), hipMemcpyDeviceToHost, st));
  PK(hipMemcpyAsync(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  PK(hipStreamSynchronize(st));
  *loss = h[0] / h[1];
  if (bad) return (set_error("ptc_loss_grad: proposed vectors are rank deficient on a block"), MG_ERANK);
  if (!std::isfinite(*loss)) return (set_error("ptc_loss_grad: non-finite loss"), MG_ENONFINITE);
  return MG_OK;
}

extern "C" int ptc_adam(void *W, const void *g, void *m, void *v, size_t n, int step, double lr, double b1, double b2,
                        double eps, hipStream_t st) {
  set_error("");
  if (!W || !g || !m || !v || step < 1) return (set_error("ptc_adam: bad arguments"), MG_EINVAL);
  PK(ptc_adam_k((float2 *)W, (const float2 *)g, (float2 *)m, (float2 *)v, n, step, lr, b1, b2, eps, st));
  return MG_OK;
}

extern "C" int ptc_destroy(ptc_ctx_t *c) {
  delete c;
  return MG_OK;
}
