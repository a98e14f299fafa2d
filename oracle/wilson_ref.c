/* Plain C Wilson-Dirac operator D(U) of Eq. (2), used by the oracle's
 * Arnoldi mass tuning as a faster matvec than the numpy version.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle; the GPU library shares
 * no code with it.  It is checked element by element against the numpy
 * oracle (oracle/wilson.py) in the CPU test-suite.
 *
 *   (D psi)(x) = (4+m) psi(x)
 *      - 1/2 sum_mu [ eta+ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                   + eta- (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * eta = -1 for hops that cross the time boundary when antiperiodic_t != 0.
 * Layouts (complex128 as interleaved re/im doubles, x fastest):
 *   U[mu][t][z][y][x][a][b], psi[t][z][y][x][s][c].
 * proj_minus / proj_plus: the 4x4 complex spin matrices (1 -/+ gamma_mu),
 * [mu][s][t], supplied by the caller so the gamma basis has one definition.
 */
#include <complex.h>
#include <stddef.h>

typedef double _Complex cplx;

void wilson_ref_apply(const int L[4], const cplx *U, const cplx *in, cplx *out,
                      double mass, int antiperiodic_t,
                      const cplx *proj_minus, const cplx *proj_plus)
{
  const long Lx = L[0], Ly = L[1], Lz = L[2], Lt = L[3];
  const long V = Lx * Ly * Lz * Lt;
  const long stride[4] = {1, Lx, Lx * Ly, Lx * Ly * Lz};
#pragma omp parallel for schedule(static)
  for (long i = 0; i < V; ++i) {
    long c[4] = {i % Lx, (i / Lx) % Ly, (i / (Lx * Ly)) % Lz, i / (Lx * Ly * Lz)};
    cplx acc[12];
    for (int k = 0; k < 12; ++k) acc[k] = (4.0 + mass) * in[i * 12 + k];
    for (int mu = 0; mu < 4; ++mu) {
      for (int dir = 0; dir < 2; ++dir) {
        long n = c[mu] + (dir == 0 ? 1 : -1);
        double eta = 1.0;
        if (n == L[mu]) { n = 0; if (mu == 3 && antiperiodic_t) eta = -1.0; }
        if (n < 0) { n = L[mu] - 1; if (mu == 3 && antiperiodic_t) eta = -1.0; }
        long j = i + (n - c[mu]) * stride[mu];
        /* link: forward U_mu(x); backward U_mu(x-mu)^dag */
        const cplx *Ul = U + ((long)mu * V + (dir == 0 ? i : j)) * 9;
        cplx t[12];
        for (int s = 0; s < 4; ++s)
          for (int a = 0; a < 3; ++a) {
            cplx v = 0;
            for (int b = 0; b < 3; ++b) {
              cplx u = (dir == 0) ? Ul[a * 3 + b] : conj(Ul[b * 3 + a]);
              v += u * in[j * 12 + s * 3 + b];
            }
            t[s * 3 + a] = v;
          }
        const cplx *G = (dir == 0 ? proj_minus : proj_plus) + mu * 16;
        for (int s = 0; s < 4; ++s)
          for (int a = 0; a < 3; ++a) {
            cplx v = 0;
            for (int r = 0; r < 4; ++r) v += G[s * 4 + r] * t[r * 3 + a];
            acc[s * 3 + a] -= 0.5 * eta * v;
          }
      }
    }
    for (int k = 0; k < 12; ++k) out[i * 12 + k] = acc[k];
  }
}
