/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_sanitizers.py with gcc): quadratures, equilibria,
 * Landau frames and short runs on small grids with every boundary condition
 * and statistics.  Exits 0 after printing "ok"; any sanitizer report aborts
 * it.  Declarations of the oracle's entry points (rlbm_oracle.c). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_quad orc_quad;
typedef struct orc_sim orc_sim;
orc_quad* orc_quad_new(int Np, int K, int N, int rotate);
void orc_quad_free(orc_quad* q);
int orc_quad_nvel(const orc_quad* q);
int orc_quad_nbasis(const orc_quad* q);
void orc_quad_get(const orc_quad* q, double* p, double* theta, double* w, double* cth, double* sth);
void orc_quad_basis(const orc_quad* q, double* J, int* expo);
void orc_feq(const orc_quad* q, double n, double T, double ux, double uy, double* feq);
void orc_eq_coeffs(const orc_quad* q, double n, double T, double ux, double uy, double* a);
int orc_feq_qs(const orc_quad* q, double n, double T, double ux, double uy, int stat, double* feq);
void orc_moments(const orc_quad* q, const double* f, double* mom);
int orc_landau(const double* mom, double* out6);
int orc_qs_landau(const double* mom, int stat, double* out8);
orc_sim* orc_sim_new(const orc_quad* q, int nx, int ny, const double* n, const double* T, const double* ux,
                     const double* uy, double tau, double dt, int bcx, int bcy, int stat);
void orc_sim_free(orc_sim* s);
void orc_sim_step(orc_sim* s, int nsteps);
void orc_sim_stream(orc_sim* s, int nsteps);
long orc_sim_fields(const orc_sim* s, double* n, double* eps, double* ux, double* uy);
void orc_sim_moments(const orc_sim* s, double* mom);
void orc_sim_charges(const orc_sim* s, double* ch);
void orc_sim_get_f(const orc_sim* s, double* f);
void orc_sim_set_f(orc_sim* s, const double* f);
long orc_sim_nonphys(const orc_sim* s);

int main(void)
{
    const int sets[][3] = {{3, 5, 2}, {3, 32, 3}, {4, 16, 3}, {6, 40, 5}, {8, 30, 7}, {5, 20, 4}};
    long checks = 0;
    for (unsigned si = 0; si < sizeof(sets) / sizeof(sets[0]); ++si) {
        const int Np = sets[si][0], K = sets[si][1], N = sets[si][2];
        for (int rot = 0; rot < 2; ++rot) {
            orc_quad* q = orc_quad_new(Np, K, N, rot);
            if (!q) { printf("quadrature %d %d %d rejected\n", Np, K, N); return 1; }
            const int nv = orc_quad_nvel(q), nb = orc_quad_nbasis(q);
            double* buf = malloc(sizeof(double) * 5 * nv);
            orc_quad_get(q, buf, buf + nv, buf + 2 * nv, buf + 3 * nv, buf + 4 * nv);
            double* J = malloc(sizeof(double) * nb * nv);
            int* ex = malloc(sizeof(int) * 3 * nb);
            orc_quad_basis(q, J, ex);
            double* a = malloc(sizeof(double) * nb);
            double* f = malloc(sizeof(double) * nv);
            double mom[9], out[8];
            orc_eq_coeffs(q, 0.7, 1.1, 0.2, -0.1, a);
            orc_feq(q, 0.7, 1.1, 0.2, -0.1, f);
            orc_moments(q, f, mom);
            if (orc_landau(mom, out) || fabs(out[0] - 0.7) > 1e-12) { printf("landau\n"); return 1; }
            for (int stat = 1; stat <= 2; ++stat) {
                if (orc_feq_qs(q, 0.3, 1.0, 0.1, 0.05, stat, f)) { printf("feq_qs\n"); return 1; }
                orc_moments(q, f, mom);
                (void)orc_qs_landau(mom, stat, out);
            }
            free(buf); free(J); free(ex); free(a); free(f);
            /* short runs: every boundary condition pair (wall needs an even K) and statistics */
            const int nx = 9, ny = 5;
            double n[45], T[45], ux[45], uy[45];
            for (int i = 0; i < nx * ny; ++i) {
                n[i] = 0.3 + 0.05 * (i % 7);           /* n / T^2 < 0.75: below Bose-Einstein condensation */
                T[i] = 0.9 + 0.03 * (i % 5);
                ux[i] = 0.02 * ((i % 3) - 1);
                uy[i] = 0.01 * ((i % 4) - 1.5);
            }
            for (int bcx = 0; bcx <= 3; ++bcx)
                for (int bcy = 0; bcy <= 3; ++bcy)
                    for (int stat = 0; stat <= 2; ++stat) {
                        if ((bcx == 2 || bcy == 2) && (K % 2)) continue;
                        orc_sim* s = orc_sim_new(q, nx, ny, n, T, ux, uy, stat ? 4.0 : 2.5, 1.0, bcx, bcy, stat);
                        if (!s) {
                            printf("sim %d %d %d rejected\n", bcx, bcy, stat);
                            orc_quad_free(q);
                            return 1;
                        }
                        orc_sim_step(s, 3);
                        orc_sim_stream(s, 1);
                        double fn[45], fe[45], fx[45], fy[45], ch[4];
                        double* fm = malloc(sizeof(double) * 9 * nx * ny);
                        double* fp = malloc(sizeof(double) * nv * nx * ny);
                        (void)orc_sim_fields(s, fn, fe, fx, fy);
                        orc_sim_moments(s, fm);
                        orc_sim_charges(s, ch);
                        orc_sim_get_f(s, fp);
                        orc_sim_set_f(s, fp);
                        (void)orc_sim_nonphys(s);
                        free(fm); free(fp);
                        orc_sim_free(s);
                        ++checks;
                    }
            orc_quad_free(q);
        }
    }
    printf("ok: %ld runs\n", checks);
    return 0;
}
