/* A plain C99 client of include/elwh.h: host-only entry points (no GPU is
 * touched).  Prints the plan of the 64^2 constant-medium square (rho = 1,
 * lambda = 2, mu = 1, omega = 10, all Dirichlet) and the discrete-filter
 * diagnostics for N_T = 63, then exits 0 if every call succeeded. */
#include <stdio.h>
#include <stdlib.h>

#include "elwh.h"

int main(void) {
    enum { N = 64, NN = (N + 1) * (N + 1) };
    static double rho[NN], lam[NN], mu[NN];
    for (int i = 0; i < NN; ++i) {
        rho[i] = 1.0;
        lam[i] = 2.0;
        mu[i] = 1.0;
    }
    elwh_grid g = {2, {N, N, 0}, {1.0, 1.0, 0.0}};
    int bc[6] = {ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET,
                 ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET, ELWH_BC_DIRICHLET};
    elwh_opts o;
    elwh_default_opts(&o);
    elwh_info info;
    elwh_status st = elwh_plan(&g, rho, lam, mu, 10.0, bc, &o, &info);
    if (st != ELWH_OK) {
        fprintf(stderr, "elwh_plan: %d %s\n", (int)st, elwh_last_error(NULL));
        return 1;
    }
    printf("nt %d dt %.17g c %.17g lambda_bound %.17g\n", info.nt, info.dt, info.c, info.lambda_bound);
    elwh_filter_diag d;
    st = elwh_filter_diagnostics(63, 1, 10.0, ELWH_SCHEME_CORRECTED, &d);
    if (st != ELWH_OK) {
        fprintf(stderr, "elwh_filter_diagnostics: %d %s\n", (int)st, elwh_last_error(NULL));
        return 1;
    }
    printf("gap %.17g beta_max %.17g\n", d.gap, d.beta_max);
    /* an argument error comes back as a status, with a message */
    st = elwh_plan(&g, rho, lam, mu, -1.0, bc, &o, &info);
    printf("bad omega -> %d (%s)\n", (int)st, elwh_last_error(NULL));
    return st == ELWH_ERR_ARG ? 0 : 1;
}
