/*
 * Test infrastructure only: a standalone driver that runs the oracle's code
 * paths on small lattices, for a build with the address and undefined-
 * behaviour sanitizers (gcc -fsanitize=address,undefined).  It includes the
 * oracle source as one translation unit and exercises every step option
 * (conduction, convection in both heatings, the interpolated no-slip of f,
 * the conservative front update, a subcooled and more conductive solid, the
 * two periodic test modes), the outputs and the reference adjoint.  Exit
 * status 0 when every run finishes with finite results.
 */
#include <stdio.h>

#include "lbm_oracle.c"

static orc_params base(int n) {
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.n = n;
  p.ra = 1e5;
  p.pr = 1.0;
  p.ste = 1.0;
  p.t_h = 1.0;
  p.t_c = 0.0;
  p.t_m = 0.0;
  p.ma = 0.1;
  p.alpha_in = 0.1;
  p.s0 = 0.4 * n;
  p.heating = 0;
  p.flow = 1;
  p.ks_kl = 1.0;
  return p;
}

static int finite_all(const double *v, long long count) {
  for (long long i = 0; i < count; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

static int run(const char *name, orc_params p, int steps, int adjoint) {
  orc_sim *S = orc_create(&p);
  if (!S) {
    fprintf(stderr, "%s: allocation failed\n", name);
    return 1;
  }
  const int n = p.n;
  const long long nc = (long long)n * n * n, nn = (long long)n * n;
  int ok = 1;
  if (adjoint) {
    for (long long c = 0; c < nn; ++c) S->th[c] = 1.0 + 0.01 * (double)(c % 7);
    ok &= orc_record(S, steps) == 0;
    double *lf = calloc(Q19 * nc, sizeof(double)), *lg = calloc(Q7 * nc, sizeof(double));
    double *ls = malloc(sizeof(double) * nn), *lth = malloc(sizeof(double) * nn);
    for (long long c = 0; c < nn; ++c) ls[c] = 1.0 / (double)nc;
    ok &= orc_adjoint(S, lf, lg, ls, lth) == 0;
    ok &= finite_all(lth, nn) && finite_all(lf, Q19 * nc) && finite_all(lg, Q7 * nc);
    free(lf); free(lg); free(ls); free(lth);
    record_free();
  } else {
    orc_step(S, steps);
  }
  double *T = malloc(sizeof(double) * nc), *u = malloc(sizeof(double) * 3 * nc);
  double *rho = malloc(sizeof(double) * nc), *V = malloc(sizeof(double) * nn);
  double *nu = malloc(sizeof(double) * nn);
  orc_fields(S, T, u, u + nc, u + 2 * nc, rho);
  orc_front_velocity(S, V);
  orc_wall_nusselt(S, nu);
  double fl = orc_liquid_fraction(S), e = orc_energy(S);
  ok &= finite_all(T, nc) && finite_all(u, 3 * nc) && finite_all(rho, nc) && finite_all(V, nn) &&
        finite_all(nu, nn) && isfinite(fl) && isfinite(e);
  for (int x = 0; x < n; ++x)
    for (int q = 0; q < Q19; ++q) (void)orc_link_fraction19(S, x, n / 2, n / 3, q);
  for (int q = 0; q < Q7; ++q) (void)orc_link_fraction7(S, 1, n / 2, 1, q);
  printf("%-28s n=%d steps=%d f_l=%.6f %s\n", name, n, steps, fl, ok ? "ok" : "NOT FINITE");
  free(T); free(u); free(rho); free(V); free(nu);
  orc_destroy(S);
  return ok ? 0 : 1;
}

int main(void) {
  int bad = 0;
  orc_params p = base(9);
  p.flow = 0;
  p.seed_profile = 1;
  p.seed_lambda = 0.620063; /* Neumann constant at Ste = 1 */
  p.s0 = 1.0;
  bad |= run("conduction", p, 40, 0);
  p = base(10);
  bad |= run("convection hot y=0", p, 30, 0);
  p.heating = 1;
  bad |= run("convection hot z=0", p, 30, 0);
  p = base(8);
  p.f_wall = 1;
  bad |= run("interpolated no-slip", p, 20, 1);
  p = base(8);
  p.front_scheme = 1;
  bad |= run("conservative front", p, 20, 1);
  p = base(8);
  p.t_c = -0.3;
  p.ks_kl = 2.0;
  p.heating = 1;
  bad |= run("subcooled, kappa 2", p, 20, 1);
  p = base(7);
  bad |= run("adjoint, both walls", p, 15, 1);
  p = base(6);
  p.periodic = 1;
  bad |= run("periodic box", p, 10, 0);
  p = base(8);
  p.periodic = 2;
  p.ste = 0.0;
  p.body_fx = 1e-5;
  p.f_wall = 1;
  p.s0 = 5.3;
  bad |= run("channel", p, 20, 0);
  return bad;
}
