/* The oracle under AddressSanitizer / UndefinedBehaviorSanitizer: formal solution (with both bottom
 * conditions and the diffusion slope), Lambda*, brute-force Lambda, OS steps, solves with and without
 * Ng, the 1D solver and the complex formal solution, on small grids.  Built with gcc by
 * tests/test_sanitizers.py together with oracle/oracle.c. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_formal_solution(int, int, int, int, int, const double *, const double *, double, const double *,
                        double *, double *, double *, int);
int orc_formal_solution_slope(int, int, int, int, int, const double *, const double *, double,
                              const double *, const double *, double *, double *, double *, int);
int orc_lstar(int, int, int, int, int, const double *, double *, int);
int orc_lambda_bruteforce(int, int, int, int, int, const double *, double *, int);
int orc_solve(int, int, int, int, int, const double *, const double *, const double *, double, int,
              const double *, double *, double, int, int, int *, double *, int);
int orc_solve_ng(int, int, int, int, int, const double *, const double *, const double *, double, int,
                 const double *, double *, double, int, int, int, int, int *, double *, int);
int orc_pp1d(int, int, const double *, const double *, double, double, double, double *);
int orc_fs_complex(int, int, int, int, int, const double *, const double *, const double *, const double *,
                   double, const double *, const double *, const double *, double *, double *, double *,
                   double *);
void orc_diffusion_slope(int, int, const double *, const double *, double *);

int main(void)
{
    const int nx = 5, ny = 4, nz = 3, nt = 4, np = 8, V = nx * ny * nz, nup = nt * np / 2;
    double *chi = malloc(sizeof(double) * V), *eps = malloc(sizeof(double) * V), *B = malloc(sizeof(double) * V);
    double *S = malloc(sizeof(double) * V), *J = malloc(sizeof(double) * V), *Ji = malloc(sizeof(double) * V);
    double *L = malloc(sizeof(double) * 27 * V), *Lam = malloc(sizeof(double) * V * V);
    double *Iem = malloc(sizeof(double) * nup * nx * ny), *Iemi = malloc(sizeof(double) * nup * nx * ny);
    double *chi_im = calloc(V, sizeof(double)), *slope = malloc(sizeof(double) * nx * ny);
    double *Ibar = malloc(sizeof(double) * nt * np * V);
    unsigned s = 12345u;
    for (int v = 0; v < V; ++v) {
        s = s * 1664525u + 1013904223u;
        chi[v] = 0.05 + 3.0 * (s >> 8) / 16777216.0;
        eps[v] = 0.1 + 0.5 * ((s >> 4) & 255) / 255.0;
        B[v] = 1.5 - 0.1 * (v / (nx * ny));
        S[v] = B[v];
    }
    int rc = 0, it = 0;
    double c = 0.0;
    rc |= orc_formal_solution(nx, ny, nz, nt, np, chi, S, 0.2, B, J, Iem, Ibar, 1);
    orc_diffusion_slope(nx, ny, chi, B, slope);
    rc |= orc_formal_solution_slope(nx, ny, nz, nt, np, chi, S, 0.2, B, slope, J, Iem, NULL, 1);
    rc |= orc_lstar(nx, ny, nz, nt, np, chi, L, 1);
    rc |= orc_lambda_bruteforce(nx, ny, nz, nt, np, chi, Lam, 1);
    for (int mode = 0; mode <= 2; ++mode) {
        for (int v = 0; v < V; ++v) J[v] = B[v];
        int r = orc_solve(nx, ny, nz, nt, np, chi, eps, B, 0.0, mode, L, J, 1e-10, 500, 4, &it, &c, 1);
        if (r < 0) rc |= 1;
        for (int v = 0; v < V; ++v) J[v] = B[v];
        r = orc_solve_ng(nx, ny, nz, nt, np, chi, eps, B, 0.0, mode, NULL, J, 1e-10, 500, 4, 3, 6, &it, &c, 1);
        if (r < 0) rc |= 1;
    }
    double dtau[3] = {2.0, 0.5, 0.1}, S1[3] = {1.0, 0.8, 0.5}, J1[3];
    rc |= orc_pp1d(3, 8, dtau, S1, 0.1, 1.2, 0.3, J1);
    chi_im[7] = 1e-30;
    rc |= orc_fs_complex(nx, ny, nz, nt, np, chi, chi_im, S, NULL, 0.2, B, slope, NULL, J, Ji, Iem, Iemi);
    printf("oracle driver %s: last solve %d steps, c = %.3e\n", rc ? "FAILED" : "ok", it, c);
    free(chi); free(eps); free(B); free(S); free(J); free(Ji); free(L); free(Lam); free(Iem); free(Iemi);
    free(chi_im); free(slope); free(Ibar);
    return rc ? 1 : 0;
}
