// Error reporting and geometry construction.
#include <cstdio>

#include "common.h"

namespace mg {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

std::string hip_error_string(hipError_t e, const char *what) {
  char buf[512];
  std::snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
  return std::string(buf);
}

Geom make_geom(const int L[4], const int b[4], int antiperiodic) {
  Geom g{};
  uint64_t V = 1, vb = 1, Vc = 1;
  for (int mu = 0; mu < 4; ++mu) {
    g.L[mu] = L[mu];
    g.b[mu] = b[mu];
    g.C[mu] = L[mu] / b[mu];
    V *= (uint64_t)L[mu];
    vb *= (uint64_t)b[mu];
    Vc *= (uint64_t)g.C[mu];
  }
  g.V = (uint32_t)V;
  g.Vpad = (uint32_t)((V + 63) / 64 * 64);
  g.vb = (uint32_t)vb;
  g.Vc = (uint32_t)Vc;
  g.Sl[0] = 1;
  g.Sb[0] = (int)vb;
  for (int mu = 1; mu < 4; ++mu) {
    g.Sl[mu] = g.Sl[mu - 1] * b[mu - 1];
    g.Sb[mu] = g.Sb[mu - 1] * g.C[mu - 1];
  }
  g.fvb = FastDiv(g.vb);
  for (int mu = 0; mu < 3; ++mu) {
    g.fb[mu] = FastDiv((uint32_t)b[mu]);
    g.fC[mu] = FastDiv((uint32_t)g.C[mu]);
  }
  g.antiperiodic = antiperiodic;
  return g;
}

}  // namespace mg
