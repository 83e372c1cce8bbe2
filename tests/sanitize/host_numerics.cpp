// Host-side numerics of the HIP library under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py with g++):
// quadrature and velocity tables, the zeta table, the per-shell equilibrium
// coefficients, the Landau frame and the Fermi-Dirac / Bose-Einstein frame,
// over the supported orders, shell counts, angle counts and random states.
// Exits 0 after printing "ok"; any sanitizer report aborts it.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2011_06856_amd/csrc/rlbm_internal.h"

static unsigned long long rng = 0x9e3779b97f4a7c15ULL;
static double uni()
{
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
    return (rng >> 11) * (1.0 / 9007199254740992.0);
}

int main()
{
    double ztab[RLBM_NZETA];
    build_zeta_table(ztab);
    long checks = 0;
    for (int N = 1; N <= RLBM_NMAX; ++N)
        for (int Np = (N + 4) / 2; Np <= N + 2; ++Np)
            for (int K : {2 * N + 1, 2 * N + 2, 24, 64})
                for (int rot = 0; rot < 2; ++rot) {
                    HostQuad q;
                    std::string err;
                    if (build_host_quad(q, Np, K, N, rot, err) != RLBM_OK) {
                        std::printf("rejected Np=%d K=%d N=%d: %s\n", Np, K, N, err.c_str());
                        return 1;
                    }
                    std::vector<VelRec<double>> vd;
                    build_vel_table(q, 0.75, vd);
                    for (int trial = 0; trial < 4; ++trial) {
                        const double n = 0.2 + uni(), T = 0.4 + uni(), ux = 0.6 * (uni() - 0.5),
                                     uy = 0.6 * (uni() - 0.5), U0 = std::sqrt(1.0 + ux * ux + uy * uy);
                        // f_eq from the per-shell coefficients, its moments,
                        // and the frame they give back
                        double mom[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                        for (int i = 0; i < q.Np; ++i) {
                            double c[RLBM_NT] = {};
                            shell_coeffs<RLBM_NMAX>(&q.G[(size_t)i * (RLBM_NMAX + 1) * (RLBM_NMAX + 1)], q.Pc.data(),
                                                    n, T, U0, ux, uy, [&](int m, double cm, double sm) {
                                                        if (m == 0) {
                                                            c[0] = cm;
                                                        } else {
                                                            c[2 * m - 1] = cm;
                                                            c[2 * m] = sm;
                                                        }
                                                    });
                            for (int j = 0; j < q.K; ++j) {
                                const VelRec<double>& R = vd[(size_t)i * q.K + j];
                                double f = 0.0;
                                for (int t = 0; t < RLBM_NT; ++t) f += c[t] * R.H[t];
                                for (int k = 0; k < 9; ++k) mom[k] += R.P[k] * f;
                            }
                        }
                        // (order 1 does not carry T^{mu nu}: its frame is only exercised)
                        const Frame fr = landau_frame(mom);
                        if (N >= 2 && (!fr.ok || std::fabs(fr.n - n) > 1e-9 * n || std::fabs(fr.T - T) > 1e-9 * T)) {
                            std::printf("frame mismatch Np=%d K=%d N=%d: n %.17g/%.17g T %.17g/%.17g\n", Np, K, N,
                                        fr.n, n, fr.T, T);
                            return 1;
                        }
                        ++checks;
                    }
                }
    // quantum statistics: the frame of (n, eps) and the factors of (n, T)
    for (int stat : {RLBM_STAT_FERMI, RLBM_STAT_BOSE})
        for (int trial = 0; trial < 200; ++trial) {
            const double n = 0.05 + 2.0 * uni(), T = 0.3 + 1.5 * uni();
            double phi[RLBM_NMAX + 1], phi2[RLBM_NMAX + 1], Tq = 0.0;
            if (stat == RLBM_STAT_BOSE && n / (T * T) >= 1.6) continue;   // above condensation
            if (qs_phi_of_nT(n, T, stat, RLBM_NMAX, ztab, phi)) {
                std::printf("no factors for stat %d n %g T %g\n", stat, n, T);
                return 1;
            }
            const double eps = 2.0 * n * T * phi[2];
            if (qs_frame(n, eps, stat, RLBM_NMAX, ztab, &Tq, phi2) || std::fabs(Tq - T) > 1e-8 * T) {
                std::printf("frame of stat %d: T %.17g against %.17g\n", stat, Tq, T);
                return 1;
            }
            ++checks;
        }
    std::printf("ok: %ld checks\n", checks);
    return 0;
}
