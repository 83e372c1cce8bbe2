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
#ifndef RLBM_LB
#define RLBM_LB 8
#endif
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
                                             Emit emit)
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
            acc += Gs[m * (RLBM_NMAX + 1) + r] * nTk * pk;
            nTk *= T;
        }
        emit(m, acc * zr, acc * zi);
        nTm *= T;
        const double nzr = zr * Ux - zi * Uy;
        zi = zr * Uy + zi * Ux;
        zr = nzr;
    }
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
    long long S;
    double rate;           // dt / tau (0 for tau = inf)
    int* flag;
    int chunk;             // velocities per wave, a multiple of RLBM_LB
    int band;              // tile order: rows per band (tiles run column by column within a band)
};

// Velocity count from which RLBM_KERNEL_AUTO selects the push kernel.
#ifndef RLBM_PUSH_MIN_NVEL
#define RLBM_PUSH_MIN_NVEL 320
#endif

#ifndef RLBM_BAND_DEFAULT
#define RLBM_BAND_DEFAULT 1
#endif

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
};

inline int nmax_of(int N) { return N <= 3 ? 3 : (N <= 5 ? 5 : 7); }
SCParams make_params(rlbm_ctx c, int waves);   // capi.cpp

// A WALL or FIXED axis: upwind points outside the grid need the tile
// kernel's boundary loads.
inline bool special_bc(int bcx, int bcy) { return bcx >= RLBM_BC_WALL || bcy >= RLBM_BC_WALL; }

// Launchers (kernels.hip).
hipError_t launch_edges(int prec, const void* f, void* edges, int nx, int ny, int nvel, hipStream_t st);
hipError_t launch_init(int prec, int nmax, const double* fields, void* f, const VelRec<double>* vel, const double* G,
                       const double* Pc, int nx, int ny, int nvel, int K, int Np, hipStream_t st);
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
hipError_t launch_batch_step(int prec, int nmax, int waves, int grid, const BatchDesc* descs, int nprob,
                             int* counters, const int* bounds, int parity, const double* Pc, int max_np,
                             hipStream_t st);
hipError_t launch_reset_counters(int* counters, hipStream_t st);
hipError_t launch_batch_flat(int prec, int nmax, int waves, int items, const BatchDesc* descs, int nprob, int parity,
                             const double* Pc, int max_np, hipStream_t st);

// Push kernel (push.hip).
void push_free(rlbm_ctx c);
int push_setup(rlbm_ctx c, std::string& err);
size_t push_partial_bytes(int prec, int nx, int ny);
hipError_t launch_push(rlbm_ctx c, bool init);
int push_prepare(rlbm_ctx c, std::string& err);
int push_batch_wgs(rlbm_ctx c);
int push_batch_descs(const std::vector<rlbm_ctx>& cs, void** d_descs, int* total_wgs);
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
