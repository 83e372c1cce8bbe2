// quadrature.cpp -- host tables of the product quadrature (Sec. 2.3) and of the
// closed-form equilibrium coefficients (Sec. 2.2), in FP64.
#include <algorithm>
#include <cmath>

#include "rlbm_internal.h"

namespace {

// Generalised Laguerre polynomial L_j^(alpha)(x) by its three-term recurrence.
double glaguerre(int j, double alpha, double x)
{
    double l0 = 1.0, l1 = 1.0 + alpha - x;
    if (j == 0) return l0;
    for (int k = 1; k < j; ++k) {
        const double l2 = ((2.0 * k + 1.0 + alpha - x) * l1 - (k + alpha) * l0) / (k + 1.0);
        l0 = l1;
        l1 = l2;
    }
    return l1;
}

double fact(int k)
{
    double r = 1.0;
    for (int i = 2; i <= k; ++i) r *= i;
    return r;
}

double dfact(int k)
{
    double r = 1.0;
    for (int i = k; i > 1; i -= 2) r *= i;
    return r;
}

double binom(int a, int b)
{
    if (b < 0 || b > a) return 0.0;
    return fact(a) / (fact(b) * fact(a - b));
}

// Gauss-Laguerre nodes by the Golub-Welsch route: eigenvalues of the
// symmetric Jacobi matrix (diagonal 2k+1, off-diagonal k) by cyclic Jacobi
// rotations, each refined by Newton steps on L_n.
std::vector<double> laguerre_nodes(int n)
{
    std::vector<double> A(n * n, 0.0);
    for (int k = 0; k < n; ++k) {
        A[k * n + k] = 2.0 * k + 1.0;
        if (k + 1 < n) A[k * n + k + 1] = A[(k + 1) * n + k] = k + 1.0;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
        if (off < 1e-60) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    std::vector<double> x(n);
    for (int k = 0; k < n; ++k) x[k] = A[k * n + k];
    std::sort(x.begin(), x.end());
    for (double& xi : x)
        for (int it = 0; it < 3; ++it) {
            const double ln = glaguerre(n, 0.0, xi), lm = glaguerre(n - 1, 0.0, xi);
            const double d = (n * ln - n * lm) / xi;  // x L_n' = n L_n - n L_{n-1}
            if (d == 0.0) break;
            xi -= ln / d;
        }
    return x;
}

}  // namespace

int build_host_quad(HostQuad& q, int Np, int K, int N, int rotate, std::string& err)
{
    if (Np < 1 || Np > 16) { err = "n_radial must be in [1, 16]"; return RLBM_EINVAL; }
    if (N < 1 || N > RLBM_NMAX) { err = "order must be in [1, 7]"; return RLBM_EINVAL; }
    if (K < 2 * N + 1) { err = "n_angle must be >= 2*order+1"; return RLBM_EINVAL; }
    if (2 * Np < N + 3) { err = "n_radial must be >= ceil((order+3)/2) for exact N^mu and T^munu"; return RLBM_EINVAL; }
    if ((long long)Np * K > 65536) { err = "too many velocities (max 65536)"; return RLBM_EINVAL; }
    q.Np = Np; q.K = K; q.N = N; q.rotate = rotate ? 1 : 0; q.nvel = Np * K;
    q.shell_p = laguerre_nodes(Np);
    q.shell_w.resize(Np);
    for (int i = 0; i < Np; ++i) {
        const double x = q.shell_p[i], l = glaguerre(Np + 1, 0.0, x);
        q.shell_w[i] = x / ((Np + 1.0) * (Np + 1.0) * l * l);   // Sec. 2.3 weight formula
    }
    const double two_pi = 2.0 * M_PI;
    q.p.resize(q.nvel); q.theta.resize(q.nvel); q.w.resize(q.nvel); q.cth.resize(q.nvel); q.sth.resize(q.nvel);
    for (int i = 0; i < Np; ++i)
        for (int j = 0; j < K; ++j) {
            const int v = i * K + j;
            const double th = (j + (q.rotate ? double(i) / Np : 0.0)) * two_pi / K;
            q.p[v] = q.shell_p[i];
            q.theta[v] = th;
            q.w[v] = q.shell_w[i] * two_pi / K;
            q.cth[v] = std::cos(th);
            q.sth[v] = std::sin(th);
        }

    // Orthonormal polar basis J_{m,j} = p^m L_j^(2m)(p) {cos, sin}(m th) / sqrt(h_mj),
    // h_mj = (j+2m)!/j! * (2 pi if m = 0 else pi), m + j <= N: (N+1)^2 functions
    // spanning the light-cone polynomials of degree <= N.  The coefficient
    // a_{mj} + i a'_{mj} = h_mj^{-1/2} sum_r l_r^{(j,2m)} M_{m+r,m}, with the
    // Laguerre power coefficients l_r = (-1)^r C(j+2m, j-r) / r! and
    // M_{k,m} = int f_eq p^k e^{i m th} = n T^{k-1} z^m P_{k,m}(U^0).  Summing
    // over j at the shell energy gives G[i][m][r].
    const int S1 = RLBM_NMAX + 1;
    q.G.assign((size_t)Np * S1 * S1, 0.0);
    for (int i = 0; i < Np; ++i) {
        const double pi_ = q.shell_p[i];
        for (int m = 0; m <= N; ++m)
            for (int r = 0; r + m <= N; ++r) {
                double g = 0.0;
                for (int j = r; j + m <= N; ++j) {
                    const double h = fact(j + 2 * m) / fact(j) * (m == 0 ? two_pi : M_PI);
                    const double lr = ((r & 1) ? -1.0 : 1.0) * binom(j + 2 * m, j - r) / fact(r);
                    g += std::pow(pi_, m) * glaguerre(j, 2.0 * m, pi_) * lr / h;
                }
                q.G[((size_t)i * S1 + m) * S1 + r] = g;
            }
    }
    // P_{k,m}(u) = sum_l (-1)^l (2k-2l-1)!! (k-m)! / ((k-m-2l)! l! 2^l) u^{k-m-2l},
    // stored for Horner in u^2 from the highest power: Pc[m][r][l] holds the
    // coefficient of u^{r-2l}.
    q.Pc.assign((size_t)S1 * S1 * RLBM_PC_L, 0.0);
    for (int m = 0; m <= RLBM_NMAX; ++m)
        for (int r = 0; r + m <= RLBM_NMAX; ++r) {
            const int k = m + r;
            for (int l = 0; 2 * l <= r; ++l)
                q.Pc[((size_t)m * S1 + r) * RLBM_PC_L + l] =
                    ((l & 1) ? -1.0 : 1.0) * dfact(2 * k - 2 * l - 1) * fact(r) / (fact(r - 2 * l) * fact(l) * std::pow(2.0, l));
        }
    return RLBM_OK;
}

void build_vel_table(const HostQuad& q, double dt, std::vector<VelRec<double>>& vd)
{
    vd.assign(q.nvel, VelRec<double>{});
    for (int v = 0; v < q.nvel; ++v) {
        VelRec<double>& R = vd[v];
        const double c = q.cth[v], s = q.sth[v], p = q.p[v];
        const double ax = dt * std::fabs(c), ay = dt * std::fabs(s);
        R.w00 = (1 - ax) * (1 - ay);
        R.w10 = ax * (1 - ay);
        R.w01 = (1 - ax) * ay;
        R.w11 = ax * ay;
        const double px = p * c, py = p * s;
        R.P[0] = p; R.P[1] = px; R.P[2] = py;
        R.P[3] = p * p; R.P[4] = p * px; R.P[5] = p * py;
        R.P[6] = px * px; R.P[7] = px * py; R.P[8] = py * py;
        R.cth = c; R.sth = s;
        R.sx = c >= 0 ? 1.0 : -1.0;
        R.sy = s >= 0 ? 1.0 : -1.0;
        for (int t = 0; t < RLBM_NT; ++t) R.H[t] = 0.0;
        R.H[0] = q.w[v];
        for (int m = 1; m <= q.N; ++m) {
            R.H[2 * m - 1] = q.w[v] * std::cos(m * q.theta[v]);
            R.H[2 * m] = q.w[v] * std::sin(m * q.theta[v]);
        }
    }
}

// Riemann zeta at integers for the radial integrals of the quantum
// statistics: n >= 2 by the sum to 63 plus the Euler-Maclaurin tail (four
// Bernoulli terms; error below 1e-21), zeta(0) = -1/2, and for m > 0
// zeta(-m) = 0 (m even) or (-1)^k 2 (2k-1)! zeta(2k) / (2 pi)^(2k) with
// m = 2k - 1 (the functional equation).
namespace {
double zeta_pos(int n)
{
    const int M = 64;
    double s = 0.0;
    for (int j = M - 1; j >= 1; --j) s += std::pow((double)j, -n);
    const double B[4] = {1.0 / 6.0, -1.0 / 30.0, 1.0 / 42.0, -1.0 / 30.0};   // B_2, B_4, B_6, B_8
    double tail = std::pow((double)M, 1 - n) / (n - 1) + 0.5 * std::pow((double)M, -n);
    double fact = 1.0, rise = 1.0;
    for (int k = 1; k <= 4; ++k) {
        fact *= (2.0 * k - 1.0) * (2.0 * k);                                  // (2k)!
        rise *= (k == 1) ? n : (double)(n + 2 * k - 3) * (n + 2 * k - 2);    // n (n+1) ... (n+2k-2)
        tail += B[k - 1] / fact * rise * std::pow((double)M, -n - 2 * k + 1);
    }
    return s + tail;
}
}  // namespace

void build_zeta_table(double* ztab)
{
    const double pi = 3.14159265358979323846;
    for (int n = -RLBM_ZMIN; n <= RLBM_ZMAX; ++n) {
        double z;
        if (n >= 2) {
            z = zeta_pos(n);
        } else if (n == 1) {
            z = 0.0;   // pole, never used
        } else if (n == 0) {
            z = -0.5;
        } else if ((-n) % 2 == 0) {
            z = 0.0;
        } else {
            const int k = (1 - n) / 2;
            double f = 1.0;
            for (int i = 2; i <= 2 * k - 1; ++i) f *= i;
            z = ((k & 1) ? -2.0 : 2.0) * f * zeta_pos(2 * k) / std::pow(2.0 * pi, 2 * k);
        }
        ztab[n + RLBM_ZMIN] = z;
    }
}
