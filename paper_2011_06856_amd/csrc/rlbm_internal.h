// rlbm_internal.h -- shared definitions of the HIP library (not installed).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/rlbm.h"

// Largest supported expansion order N and the stride of the harmonic tables.
#define RLBM_NMAX 7
#define RLBM_NT (2 * RLBM_NMAX + 1)

// Per-velocity constants of the fused kernel, read with wave-uniform indices
// (scalar loads).  32 entries of T:
//   w00 w10 w01 w11  bilinear weights of the cells (x,y) (x-sx,y) (x,y-sy)
//                    (x-sx,y-sy): (1-ax)(1-ay), ax(1-ay), (1-ax)ay, ax ay with
//                    ax = dt|cos|, ay = dt|sin| (Eq. interpolation)
//   P[9]             p, p c, p s, p^2, p^2 c, p^2 s, p^2 c^2, p^2 c s, p^2 s^2
//                    (Eq. discrete_sum_moments rows)
//   cth sth          direction n_v (collision frequency U^0 - U.n_v)
//   sx sy            upwind signs sgn(cos), sgn(sin) (sgn 0 = +1) as +-1
//   H[15]            w_v {1, cos th, sin th, cos 2th, sin 2th, ...}: the
//                    equilibrium is f_eq_v = sum_t coef_shell(v)[t] H[t]
template <typename T>
struct alignas(16) VelRec {
    T w00, w10, w01, w11;
    T P[9];
    T cth, sth;
    T sx, sy;
    T H[RLBM_NT];
};
static_assert(sizeof(VelRec<float>) == 32 * 4, "VelRec layout");

// Per-velocity records of the fused kernel, one per phase, read with
// wave-uniform scalar loads.  The tables are padded past nvel with null
// entries (zero weights, zero equilibrium row, last shell) so that every wave
// processes whole load batches without range checks; a null entry reads the
// last velocity's plane and writes the spare plane at the end of each buffer.
// The records hold only what the plane index v does not give (the plane
// offsets are v times the plane size, the upwind signs are those of P[1] and
// P[2]), so that the tables of a velocity set stay in the scalar cache.
//
// Streaming record (phase 1):
//   w[4]   bilinear weights of the cells (x,y) (x-sx,y) (x,y-sy) (x-sx,y-sy):
//          (1-ax)(1-ay), ax(1-ay), (1-ax)ay, ax ay, ax = dt|cos|, ay = dt|sin|
//   P[]    moment rows p, p c, p s, p^2, p^2 c, p^2 s, p^2 c^2, p^2 c s
//          (and p^2 s^2 in FP64; FP32 takes T^yy = T^00 - T^xx); the sign
//          bits of P[1] and P[2] are those of cos and sin (sx, sy; sgn 0 = +1)
template <typename T>
struct alignas(16) SRec {
    T w[4];
    T P[sizeof(T) == 8 ? 9 : 8];
};
static_assert(sizeof(SRec<float>) == 48 && sizeof(SRec<double>) == 112, "SRec layout");

// Collision record (phase 4):
//   H[2NM+1]  w_v {1, cos th, sin th, ..., cos NM th, sin NM th}: f_eq_v is
//             sum_t coef_shell[t] H[t] (zero above the expansion order)
//   cth sth   direction n_v (collision frequency U^0 - U.n_v)
//   shell     radial shell index i
template <typename T, int NM>
struct alignas(16) CRec {
    T H[2 * NM + 1];
    T cth, sth;
    int shell;
};

// Velocities per load batch and the padding of the velocity tables.
#define RLBM_LB 8
#define RLBM_VPAD (RLBM_LB * 16)

// Host-side quadrature and coefficient tables (FP64).
struct HostQuad {
    int Np = 0, K = 0, N = 0, nvel = 0, rotate = 1;
    std::vector<double> shell_p, shell_w;          // [Np]
    std::vector<double> p, theta, w, cth, sth;     // [nvel]
    // G[i][m][r]: equilibrium harmonic m of shell i is
    //   z^m sum_r G[i][m][r] n T^{m+r-1} P_{m+r,m}(U^0),  z = U^x + i U^y
    std::vector<double> G;                         // [Np][NMAX+1][NMAX+1]
    // Pc[m][r][l]: P_{m+r,m}(u) = sum_l Pc[m][r][l] u^{r-2l} (Horner from l = 0)
    std::vector<double> Pc;                        // [NMAX+1][NMAX+1][NMAX/2+1]
};

#define RLBM_PC_L (RLBM_NMAX / 2 + 1)

int build_host_quad(HostQuad& q, int Np, int K, int N, int rotate, std::string& err);
void build_vel_table(const HostQuad& q, double dt, std::vector<VelRec<double>>& vd);

// ---------------------------------------------------------------------------
// Device/host numerics shared by the kernels and the host debug entry points.
// ---------------------------------------------------------------------------

// Finite test usable on host and device.  (x - x == 0 is not: with FMA
// contraction x - x for x = a*b becomes fma(a, b, -x), the rounding error.)
__host__ __device__ inline bool finite_d(double x) { return __builtin_isfinite(x); }

struct Frame {
    double n, eps, U0, Ux, Uy, T;
    int ok;
};

// Landau frame of the nine moments m = (N0, Nx, Ny, T00, T0x, T0y, Txx, Txy,
// Tyy): eps = largest root of det(T^{mu nu} - lambda eta^{mu nu}) by Newton
// from the right (monotone on the concave branch beyond the largest root),
// then the boost beta from the two spatial rows of (T - eps eta) u = 0 with
// u_0 = 1, U = gamma (1, beta), n = U_mu N^mu, T = eps / (2n).
__host__ __device__ inline Frame landau_frame(const double* m)
{
    const double a = m[3], b = m[4], c = m[5], d = m[6], e = m[7], f = m[8];
    const double c2 = a - d - f;
    const double c1 = a * (d + f) - d * f + e * e - b * b - c * c;
    auto pv = [&](double l) {
        return (a - l) * ((d + l) * (f + l) - e * e) - b * (b * (f + l) - e * c) + c * (b * e - (d + l) * c);
    };
    auto dp = [&](double l) { return (-3.0 * l + 2.0 * c2) * l + c1; };
    double lam = a;
    if (!(pv(lam) <= 0.0 && dp(lam) < 0.0 && (-6.0 * lam + 2.0 * c2) < 0.0)) {
        const double g0 = a + fabs(b) + fabs(c);
        const double g1 = -d + fabs(b) + fabs(e);
        const double g2 = -f + fabs(c) + fabs(e);
        lam = fmax(g0, fmax(g1, g2));
    }
    for (int it = 0; it < 100; ++it) {
        const double step = pv(lam) / dp(lam);
        if (!(step > 0.0)) break;
        lam -= step;
        if (step <= 2.0e-16 * fabs(lam)) break;
    }
    Frame fr;
    const double eps = lam;
    const double A = d + eps, B = e, C = f + eps;
    const double det = A * C - B * B;
    const double bx = (b * C - B * c) / det;
    const double by = (A * c - B * b) / det;
    const double b2 = bx * bx + by * by;
    const double g = 1.0 / sqrt(1.0 - b2);
    fr.eps = eps;
    fr.U0 = g;
    fr.Ux = g * bx;
    fr.Uy = g * by;
    fr.n = g * (m[0] - bx * m[1] - by * m[2]);
    fr.T = eps / (2.0 * fr.n);
    fr.ok = (det > 0.0) && (b2 < 1.0) && (fr.n > 0.0) && (eps > 0.0) && finite_d(fr.n) && finite_d(fr.T) &&
            finite_d(fr.Ux) && finite_d(fr.Uy);
    return fr;
}

// Harmonic coefficients of the truncated equilibrium on one shell,
//   f_eq / w = sum_m C_m cos(m th) + S_m sin(m th),
// handed to emit(m, C_m, S_m) one harmonic at a time (few live registers).
// Gs = G[shell] ([NMAX+1][NMAX+1]), zero beyond the expansion order, so that
// harmonics above the order come out as zero.
template <int NM, typename PT, typename Emit>
__host__ __device__ inline void shell_coeffs(PT Gs, PT Pc, double n, double T, double U0, double Ux, double Uy,
                                             Emit emit, const double* phi = nullptr)
{
    const double u2 = U0 * U0;
    double zr = 1.0, zi = 0.0;   // (U^x + i U^y)^m
    double nTm = n / T;          // n T^{m-1}
#pragma unroll
    for (int m = 0; m <= NM; ++m) {
        double acc = 0.0, nTk = nTm;
#pragma unroll
        for (int r = 0; r + m <= NM; ++r) {
            // P_{m+r,m}(U^0) by Horner in (U^0)^2
            PT pc = Pc + (m * (RLBM_NMAX + 1) + r) * RLBM_PC_L;
            double pk = pc[0];
#pragma unroll
            for (int l = 1; 2 * l <= r; ++l) pk = pk * u2 + pc[l];
            if (r & 1) pk *= U0;
            // Fermi-Dirac / Bose-Einstein: the radial moment of power m + r
            // scaled by phi[m + r] (qs_frame below)
            acc += Gs[m * (RLBM_NMAX + 1) + r] * nTk * pk * (phi ? phi[m + r] : 1.0);
            nTk *= T;
        }
        emit(m, acc * zr, acc * zi);
        nTm *= T;
        const double nzr = zr * Ux - zi * Uy;
        zi = zr * Uy + zi * Ux;
        zr = nzr;
    }
}

// ---------------------------------------------------------------------------
// Fermi-Dirac and Bose-Einstein equilibria (Eq. feq_dist with epsilon = +1,
// -1): f_eq = (1/2pi) / (z^-1 exp(U.p/T) + epsilon).  As f_eq depends on p
// only through U.p/T, the moment of radial power k is the Maxwell-Juttner one
// at the same (n, T, U) times phi_k = G_k(z) / G_1(z), with the radial
// integrals G_k(z) = (1/k!) int_0^inf x^k / (z^-1 e^x + epsilon) dx, i.e.
// -Li_{k+1}(-z) (FD) and Li_{k+1}(z) (BE, z <= 1); n = T^2 G_1(z), eps =
// 2 n T phi_2.  ztab: zeta(n) for n = -RLBM_ZMIN .. RLBM_ZMAX (built by
// build_zeta_table; zeta(1) unused).
// ---------------------------------------------------------------------------
#define RLBM_ZMIN 40
#define RLBM_ZMAX 12
#define RLBM_NZETA (RLBM_ZMIN + RLBM_ZMAX + 1)
void build_zeta_table(double* ztab);   // quadrature.cpp

__host__ __device__ inline double ipow_d(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// sum_{j>=1} (-1)^(j+1) x^j / j^s for 0 <= x <= 1 (= -Li_s(-x)): the
// alternating-series acceleration of Cohen, Rodriguez Villegas and Zagier
// (algorithm 1), 28 terms (error below 5.8^-28 of the sum).
__host__ __device__ inline double qs_alt(int s, double x)
{
    constexpr int N = 28;
    const double e = 5.828427124746190;   // 3 + sqrt(8)
    double d = ipow_d(e, N);
    d = 0.5 * (d + 1.0 / d);
    double b = -1.0, c = -d, sum = 0.0, xp = 1.0;
    for (int k = 0; k < N; ++k) {
        c = b - c;
        xp *= x;
        sum += c * xp / ipow_d((double)(k + 1), s);
        b = (double)(k + N) * (double)(k - N) * b / ((k + 0.5) * (k + 1.0));
    }
    return sum / d;
}

// G_k(z) for statistics stat (RLBM_STAT_*), k >= 0.
template <typename ZT>
__host__ __device__ inline double qs_G(int k, double z, int stat, ZT ztab)
{
    const int s = k + 1;
    auto zeta = [&](int n) { return (double)ztab[n + RLBM_ZMIN]; };
    if (stat == RLBM_STAT_FERMI) {
        if (s == 1) return log1p(z);
        if (z <= 1.0) return qs_alt(s, z);
        // inversion: -Li_s(-z) = mu^s/s! + 2 sum_j eta(2j) mu^(s-2j)/(s-2j)! + (-1)^s Li_s(-1/z)
        const double mu = log(z);
        double f = 1.0, r;
        for (int i = 2; i <= s; ++i) f *= i;
        r = ipow_d(mu, s) / f;
        for (int j = 1; 2 * j <= s; ++j) {
            double g = 1.0;
            for (int i = 2; i <= s - 2 * j; ++i) g *= i;
            r += 2.0 * (1.0 - ipow_d(0.5, 2 * j - 1)) * zeta(2 * j) * ipow_d(mu, s - 2 * j) / g;
        }
        return r - ((s & 1) ? -1.0 : 1.0) * qs_alt(s, 1.0 / z);
    }
    if (stat == RLBM_STAT_BOSE) {
        if (s == 1) return -log1p(-z);
        if (z >= 1.0) return zeta(s);
        if (z <= 0.5) {
            double sum = 0.0, xp = 1.0;
            for (int j = 1; j <= 64; ++j) {
                xp *= z;
                sum += xp / ipow_d((double)j, s);
            }
            return sum;
        }
        // expansion in mu = ln z: sum_{j != s-1} zeta(s-j) mu^j/j! + mu^(s-1)/(s-1)! (H_{s-1} - ln(-mu))
        const double mu = log(z);
        double sum = 0.0, term = 1.0;
        for (int j = 0; j < 32 && s - j >= -RLBM_ZMIN; ++j) {
            if (j == s - 1) {
                double H = 0.0;
                for (int i = 1; i <= s - 1; ++i) H += 1.0 / i;
                sum += term * (H - log(-mu));
            } else {
                sum += zeta(s - j) * term;
            }
            term *= mu / (j + 1);
        }
        return sum;
    }
    return z;
}

// Safeguarded Newton in y = ln z for g(y) = target, g monotone with
// derivative dg(y); [lo, hi] brackets the root.  Returns 0 or 1 without a
// root in the bracket.
template <typename G, typename DG>
__host__ __device__ inline int qs_solve(G g, DG dg, double target, bool increasing, double lo, double hi, double y,
                                        double* out)
{
    const double glo = g(lo) - target, ghi = g(hi) - target;
    if (!(increasing ? (glo <= 0.0 && ghi >= 0.0) : (glo >= 0.0 && ghi <= 0.0))) return 1;
    y = fmin(fmax(y, lo), hi);
    for (int it = 0; it < 200; ++it) {
        const double v = g(y) - target;
        if (v == 0.0) break;
        if ((v < 0.0) == increasing) lo = y; else hi = y;
        const double d = dg(y);
        double yn = y - v / d;
        if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);   // Newton left the bracket: bisect
        if (fabs(yn - y) <= 1e-15 * fmax(1.0, fabs(y)) || hi - lo <= 1e-15 * fmax(1.0, fabs(y))) {
            y = yn;
            break;
        }
        y = yn;
    }
    *out = y;
    return 0;
}

// Temperature and moment factors phi[0..kmax] of a Landau frame (n, eps):
// z from 4 G_2^2 / G_1^3 = eps^2 / n^3 (decreasing in z), T = sqrt(n / G_1).
// Returns 0, or 1 without an equilibrium (FD below the degenerate limit,
// BE above condensation).
template <typename ZT>
__host__ __device__ inline int qs_frame(double n, double eps, int stat, int kmax, ZT ztab, double* T, double* phi)
{
    if (stat == RLBM_STAT_MJ) {
        *T = eps / (2.0 * n);
        for (int k = 0; k <= kmax; ++k) phi[k] = 1.0;
        return 0;
    }
    const double r = eps * eps / (n * n * n);
    auto h = [&](double y) {
        const double z = exp(y), g1 = qs_G(1, z, stat, ztab), g2 = qs_G(2, z, stat, ztab);
        return 4.0 * g2 * g2 / (g1 * g1 * g1);
    };
    auto dh = [&](double y) {   // z d/dz G_k = G_{k-1}
        const double z = exp(y), g0 = qs_G(0, z, stat, ztab), g1 = qs_G(1, z, stat, ztab),
                     g2 = qs_G(2, z, stat, ztab);
        return 4.0 * g2 * g2 / (g1 * g1 * g1) * (2.0 * g1 / g2 - 3.0 * g0 / g1);
    };
    double y;
    const double hi = stat == RLBM_STAT_BOSE ? 0.0 : 60.0;
    if (qs_solve(h, dh, r, false, -60.0, hi, fmin(log(4.0 / r), hi), &y)) return 1;
    const double z = exp(y), g1 = qs_G(1, z, stat, ztab);
    *T = sqrt(n / g1);
    for (int k = 0; k <= kmax; ++k) phi[k] = qs_G(k, z, stat, ztab) / g1;
    return !(finite_d(*T) && *T > 0.0);
}

// Moment factors phi[0..kmax] of the state (n, T): z from n = T^2 G_1(z).
// Returns 0, or 1 without an equilibrium (BE above condensation).
template <typename ZT>
__host__ __device__ inline int qs_phi_of_nT(double n, double T, int stat, int kmax, ZT ztab, double* phi)
{
    if (stat == RLBM_STAT_MJ) {
        for (int k = 0; k <= kmax; ++k) phi[k] = 1.0;
        return 0;
    }
    auto g = [&](double y) { return qs_G(1, exp(y), stat, ztab); };
    auto dg = [&](double y) { return qs_G(0, exp(y), stat, ztab); };
    const double target = n / (T * T);
    double y;
    const double hi = stat == RLBM_STAT_BOSE ? 0.0 : 60.0;
    if (qs_solve(g, dg, target, true, -60.0, hi, fmin(log(target), hi), &y)) return 1;
    const double z = exp(y), g1 = qs_G(1, z, stat, ztab);
    for (int k = 0; k <= kmax; ++k) phi[k] = qs_G(k, z, stat, ztab) / g1;
    return 0;
}

// Kernel launch parameters.
struct SCParams {
    const void* fin;
    void* fout;
    const void* srec;      // SRec<TC>[nvel + RLBM_VPAD]
    const void* crec;      // CRec<TC, NM>[nvel + RLBM_VPAD]
    const unsigned char* sgn;   // [nvel + RLBM_VPAD]: bit 0 cos < 0, bit 1 sin < 0 (upwind x + 1, y + 1),
                                // bit 2 the reversed velocity lies K/2 planes below (else above)
    const void* edges;     // initial populations of the edge cells (FIXED axes):
                           // [2][nvel][ny] (columns 0, nx-1) then [2][nvel][nx] (rows 0, ny-1)
    const double* G;       // [Np][NMAX+1][NMAX+1]
    const double* Pc;
    int nx, ny, nvel, K, Np, N;
    int bcx, bcy;
    int stat;              // RLBM_STAT_* of the equilibrium
    const double* ztab;    // zeta table of the quantum statistics
    long long S;
    double rate;           // dt / tau (0 for tau = inf)
    int* flag;
    int chunk;             // velocities per wave, a multiple of RLBM_LB
    int band;              // tile order: rows per band (tiles run column by column within a band)
};

// Velocity count from which RLBM_KERNEL_AUTO selects the push kernel.
#define RLBM_PUSH_MIN_NVEL 320

// Tile order of the tile kernel: rows per band.
#define RLBM_BAND_DEFAULT 1

// Work-group order of the push kernel: bands of 4 rows per group (a batch
// may choose another value).
#define RLBM_PUSH_BANDS 2

// One problem of a batch: its buffers, tables and step parameters, and the
// index of its first work item.
struct BatchDesc {
    void* f[2];
    SCParams P;            // srec, crec, G and the scalars (fin/fout unused)
    int item0, tiles;
};
static_assert(sizeof(BatchDesc) % 4 == 0, "BatchDesc is copied in 32-bit words");

// A simulation context (the opaque rlbm_ctx of the C ABI).
struct rlbm_ctx_s {
    HostQuad q;
    double zeta[RLBM_NZETA];             // zeta table of the quantum statistics (host)
    std::string err;
    int have_fields = 0;
    int dev = -1;                        // device of the workspace (rlbm_init_fields)
    int nx = 0, ny = 0, prec = RLBM_F64, bcx = 0, bcy = 0;
    long long S = 0;
    double tau = 0, dt = 1, rate = 0;
    int waves = 0;
    hipStream_t st = nullptr;
    char* ws = nullptr;
    bool ws_owned = false;
    size_t ws_bytes = 0;
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    double* d_fields = nullptr;
    double* d_partials = nullptr;
    void* d_edges = nullptr;             // SCParams::edges (in the workspace)
    int* d_flag = nullptr;
    void* d_srec = nullptr;              // SRec<TC>[nvel + RLBM_VPAD]
    void* d_crec = nullptr;              // CRec<TC, NM>[nvel + RLBM_VPAD]
    unsigned char* d_sgn = nullptr;      // upwind signs per table entry [nvel + RLBM_VPAD]
    VelRec<double>* d_veld = nullptr;    // FP64 table for init and fields [nvel]
    double* d_G = nullptr;
    double* d_Pc = nullptr;
    double* d_zeta = nullptr;            // zeta table (quantum statistics)
    int stat = RLBM_STAT_MJ;             // statistics of the next rlbm_init_fields
    int fstat = RLBM_STAT_MJ;            // statistics of the current fields
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    long long steps = 0;
    double* d_corr = nullptr;            // learned correction: w p^2 {cos, sin} 2th per velocity
    // push kernel (push.hip): segment-ordered velocity records, segments
    // (library-owned), double-buffered partial sums of the next step's
    // moments (in the workspace)
    int kern = 0;                        // RLBM_KERNEL_AUTO / _TILE / _PUSH
    void* d_prec = nullptr;
    void* d_paddr = nullptr;
    void* d_pseg = nullptr;
    void* pp[2] = {nullptr, nullptr};
    int pcur = 0;
    int pnrec = 0;                       // records in the push tables
    int pvalid = 0;                      // pp[pcur] holds the partial sums of f[cur]
    // deviation storage (deviation.hip, push.hip): per-shell equilibrium
    // coefficients paired with f[b] (in the workspace), the push kernel's
    // per-segment monomial sums Y of the equilibrium basis, and the
    // per-shell moment sums Z of the field output
    void* cf[2] = {nullptr, nullptr};
    void* d_pytab = nullptr;
    double* d_dz = nullptr;
};

inline int nmax_of(int N) { return N <= 3 ? 3 : (N <= 5 ? 5 : 7); }

// Deviation storage: g = f - F with the equilibrium F as coefficients.
inline bool is_dev(int prec) { return prec == RLBM_BF16DEV || prec == RLBM_F32DEV || prec == RLBM_F64DEV; }
inline bool valid_prec(int prec) { return prec >= RLBM_F64 && prec <= RLBM_F64DEV; }
// Bytes of one stored population (or deviation).
inline size_t store_size(int prec)
{
    return (prec == RLBM_F64 || prec == RLBM_F64DEV) ? 8 : (prec == RLBM_BF16DEV ? 2 : 4);
}
// Bytes of the arithmetic type (partial sums, equilibrium coefficients).
inline size_t arith_size(int prec) { return (prec == RLBM_F64 || prec == RLBM_F64DEV) ? 8 : 4; }
// Coefficient planes of the deviation storage: Np x (2 NMAX(N) + 1).
inline int dev_planes(int Np, int N) { return Np * (2 * nmax_of(N) + 1); }
SCParams make_params(rlbm_ctx c, int waves);   // capi.cpp

// A WALL or FIXED axis: upwind points outside the grid need the tile
// kernel's boundary loads.
inline bool special_bc(int bcx, int bcy) { return bcx >= RLBM_BC_WALL || bcy >= RLBM_BC_WALL; }
// A grid that needs the tile kernel's general instance (boundary loads,
// quantum statistics).
inline bool general_step(int bcx, int bcy, int stat) { return special_bc(bcx, bcy) || stat != RLBM_STAT_MJ; }

// Launchers (kernels.hip).
hipError_t launch_edges(int prec, const void* f, void* edges, int nx, int ny, int nvel, hipStream_t st);
hipError_t launch_init(int prec, int nmax, const double* fields, void* f, const VelRec<double>* vel, const double* G,
                       const double* Pc, int nx, int ny, int nvel, int K, int Np, int stat, const double* ztab,
                       hipStream_t st);
hipError_t launch_stream_collide(int prec, int nmax, int waves, const SCParams& p, hipStream_t st);
hipError_t launch_fields(int prec, const void* f, const VelRec<double>* vel, double* out, double* partials,
                         int* flag, int nx, int ny, int nvel, hipStream_t st);
hipError_t launch_landau_probe(const double* mom, double* out, int count, hipStream_t st);
// The fixed device scratch of rlbm_moments_device (kernels.hip): its
// address on a device is taken once (scratch_setup, device current) and
// read back by scratch_ptr (null if not set up); grids up to
// scratch_max_sites() sites.
int scratch_setup(int dev);
void* scratch_ptr(int dev);
long long scratch_max_sites();
hipError_t launch_fields_charges(int prec, const void* f, const VelRec<double>* vel, double* out, double* partials,
                                 double* charges, int* flag, int nx, int ny, int nvel, hipStream_t st);
// Persistent batch step: counters = 9 ints, 16 apart (8 range counters and
// the exit count), zero on entry and left at zero by the launch.
hipError_t launch_batch_step(int prec, int nmax, int waves, int grid, const BatchDesc* descs, int nprob,
                             int* counters, const int* bounds, int parity, const double* Pc, int max_np,
                             hipStream_t st);
hipError_t launch_batch_flat(int prec, int nmax, int waves, int items, const BatchDesc* descs, int nprob, int parity,
                             const double* Pc, int max_np, hipStream_t st);

// Deviation storage (deviation.hip).
int dev_setup(rlbm_ctx c, std::string& err);
hipError_t launch_dev_init(rlbm_ctx c, hipStream_t st);
hipError_t launch_dev_fields(rlbm_ctx c, double* out, double* partials, hipStream_t st);
// Sum of per-block partial charges into 4 device doubles (kernels.hip).
hipError_t launch_charges_sum(const double* partials, int nb, double* charges, hipStream_t st);

// Push kernel (push.hip).
void push_free(rlbm_ctx c);
int push_setup(rlbm_ctx c, std::string& err);
size_t push_partial_bytes(int prec, int nx, int ny);
hipError_t launch_push(rlbm_ctx c, bool init);
int push_prepare(rlbm_ctx c, std::string& err);
int push_batch_wgs(rlbm_ctx c);
// Descriptors of the push-kernel problems of a batch, with `bands` bands of
// 4 rows per work-group group (0: RLBM_PUSH_BANDS).  *d_descs is allocated
// here when null (cs.size() entries; free with hipFree), else overwritten.
int push_batch_descs(const std::vector<rlbm_ctx>& cs, int bands, void** d_descs, int* total_wgs);
hipError_t launch_push_batch(int prec, int nmax, const void* d_descs, int nprob, int total_wgs, int parity,
                             hipStream_t st);
// Copy the fields in d_fields (computed by launch_fields) and the charges to
// the host and report a sticky non-physical state (capi.cpp).
int fields_out(rlbm_ctx c, double* n, double* eps, double* ux, double* uy, double* charges);
// Kernel used by rlbm_step for this context (resolves RLBM_KERNEL_AUTO).
int resolve_kernel(rlbm_ctx c);
int batch_grid(int prec, int nmax, int waves, int max_np);
int default_waves(int prec, int nmax, int nvel);
int max_vpt(int prec, int nmax);
int fields_blocks(long long S);
