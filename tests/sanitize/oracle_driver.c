/* Drives the CPU oracle through its entry points on small systems, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).  Exit 0 when every
 * call returns as expected; the sanitizers abort on any memory or undefined-behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "vmc_oracle.h"

int main(void) {
  enum { NP = 6, NE = 6, W = 3 };
  const double L = 6.2;
  double R[3 * NP], zeta[NP], C[NP * 3], ev[NP];
  for (int a = 0; a < NP; ++a) {
    for (int m = 0; m < 3; ++m) R[3 * a + m] = fmod(1.3 * a + 0.7 * m + 0.2, L);
    zeta[a] = 0.8 + 0.05 * a;
  }
  const int twists[4] = {0, 3, 6, 5};   /* the last one is the system's */
  for (int t = 0; t < 4; ++t)
    if (o_huckel_twist(NP, L, R, zeta, 3, twists[t], C, ev)) return 1;
  if (o_huckel(NP, L, R, zeta, 3, C, ev)) return 1;
  if (o_huckel_twist(NP, L, R, zeta, 3, 5, C, ev)) return 1;
  osys s = {NP, 3, 3, 3, L, OB_PERIODIC_GAUSS, OP_EWALD, 8.0 / L, 4, 1, 0.25, 0.5, 1.0, R, zeta, C, 1.5, 5};
  double x[W * 3 * NE];
  for (int i = 0; i < W * 3 * NE; ++i) x[i] = fmod(0.37 * i + 0.11, L);
  double bas[14], U, gU[3 * NE], lU[NE], dVdR[3 * NP], dVdx[3 * NE];
  const double r0[3] = {0.4, 5.9, 3.1};
  for (int a = 0; a < NP; ++a) o_basis(&s, a, r0, bas);
  o_jastrow(&s, x, &U, gU, lU);
  (void)o_potential(&s, x, dVdR, dVdx);
  double lnpsi, sgn, EL, dln[3 * NP], dEL[3 * NP];
  if (o_local(&s, x, &lnpsi, &sgn, &EL, dln, dEL)) return 2;
  double sums[W * (2 + 9 * NP)];
  int64_t nacc[W];
  if (o_vmc_run(&s, W, x, 1, 2, 1.0, 7u, 1u, 0u, sums, nacc, 1)) return 3;
  if (o_vmc_run_from(&s, 1, 2u, x, 1, 1, 1.0, 7u, 1u, 0u, sums, nacc, 1)) return 3;
  double E, sig, f[3 * NP], fw[W * 3 * NP], means[W * (1 + 9 * NP)], S[9 * NP * NP];
  if (o_reduce(W, 3 * NP, 2, sums, &E, &sig, f, fw, means)) return 4;
  o_build_S(W, 3 * NP, fw, f, S);
  double Rs[3 * NP], Rp[3 * NP], Sp[9 * NP * NP], I[9 * NP * NP] = {0};
  for (int i = 0; i < 3 * NP; ++i) { Rs[i] = Rp[i] = R[i]; I[i * 3 * NP + i] = 1.0; }
  for (int i = 0; i < 9 * NP * NP; ++i) Sp[i] = I[i];
  if (o_langevin(3 * NP, L, Rs, Rp, Sp, f, I, 0.01, 0.1, 0.2, 0u, 3u, 1u, 0u)) return 5;
  double Lc[9 * NP * NP], xi[3 * NP];
  if (o_cholesky(3 * NP, Sp, Lc)) return 7;
  o_normals(3u, 1u, 2u, 3 * NP, xi);
  double K[4] = {2.0, 0.3, 0.3, 1.0}, S2[4] = {1.0, 0.0, 0.0, 1.0}, R2[2] = {0.1, -0.2}, samp[2 * 5];
  if (o_langevin_harmonic_run(2, K, S2, 0.05, 0.1, 0.2, 0u, 4u, 10, R2, samp, 2)) return 8;
  const double xt[2] = {1.4, 0.1};
  double St[4];
  for (int k = 0; k < 4; ++k) o_toy_S(0.1, 2.0, 1.4, 1.0, k, xt, St);
  double Rt[2] = {1.4, 0.1}, Um, Us[50];
  for (int scheme = 0; scheme < 4; ++scheme)
    if (o_toy_run(0.1, 2.0, 1.4, 1.0, scheme == 1 ? 0 : 3, 0.01, 0.05, 0.2, scheme, 3u, 0u, 50, Rt, &Um, Us)) return 6;
  printf("oracle driver ok: E = %.6f\n", E);
  return 0;
}
