// push.hip -- the fused step for large velocity sets, with next-step moments
// pushed forward instead of gathered.
//
// The tile kernel (kernels.hip) needs all streamed values of a site before
// its collision, because the collision needs the site's moments (Eq.
// discrete_sum_moments) and these need every velocity.  With 1536 velocities
// one 64-site tile holds 393 KB of streamed values, most of a CU's register
// file, so the load phase of one tile cannot overlap the collision phase of
// another.  This kernel removes the dependency:
//
//   The moments that step t+1 will see at site y are a linear function of
//   the populations step t writes: f*_v(y) is the bilinear combination of
//   f_v at y, y - sx, y - sy, y - sx - sy (Eq. interpolation), so
//     M_k(y) = sum_v P_k(v) f*_v(y) = sum over sources s and corners c of
//              sum_{v with corner c at s} w_c(v) P_k(v) f_v(s).
//   While a wave writes f_v(s) it accumulates these per-source partial sums.
//   The x-displaced parts (targets s + sx) are moved to their target column
//   inside the wave by a cross-lane shuffle, so each site stores three row
//   slots (its contributions to rows y - 1, y, y + 1 at its own column) x 8
//   moments; the tile's first and last columns also store their x-displaced
//   parts in a small halo array (the parts that leave the tile, and the
//   images a clamped boundary needs).  The next step gathers its moments
//   from the three rows, with the stream's periodic or clamped index rules.
//
// A wave then owns 64 sites of one row and runs through all velocities once:
// stream, equilibrium, relaxation, store and partial sums, with no
// work-group barrier and no shared memory.  The velocities are grouped in
// segments of one shell and one quadrant; inside a segment the bilinear
// weights are ax = dt sx cos, ay = dt sy sin and the moment rows are p^a
// times {1, cos, sin, cos^2, cos sin}, so the 32 weighted moment sums of a
// segment follow from 9 angular monomial sums of f (9 FMAs per velocity).
//
// Deviation storage (DEV): a site stores g_v = f_v - F_v, with F the
// truncated equilibrium (Eq. mj-feq-expansion-truncated) its last collision
// produced, kept as per-shell harmonic coefficients C (F_v = sum_t C_t H_t(v),
// H_t = w_v {1, cos m th, sin m th}).  The streamed population is
//   f*_v(x) = sum_c w_c(v) g_v(x_c) + E_v(x),
//   E_v(x)  = sum_c w_c(v) F_v(x_c)   (corners x_c of Eq. interpolation).
// Inside a segment w_c are the bilinear monomials of ax = dt sx cos th and
// ay = dt sy sin th, so E_v / w_v is itself a harmonic series of order N + 2
// in th, whose coefficients follow from the four corners' C by the product
// rules of cos th, sin th and cos th sin th with the harmonics.  The
// collision then gives
//   g_new = f_new - F_new = (1 - omega_v) (f*_v - F_new,v),
// i.e. per velocity the bilinear sum of g plus one series of 2N + 5 terms
// (E - F_new, formed once per segment), and the stored deviation is rounded
// to the storage type (bfloat16: half the bytes of FP32).  The pushed partial
// sums hold the moments of the full f_new = g_new + F_new: the F part of a
// segment's monomial sums is sum_t C_t Y_t with per-segment tables Y.
#include <cstring>
#include <new>
#include <type_traits>

#include "rlbm_internal.h"

#ifdef __HIP_DEVICE_COMPILE__
#define PUSH_CONST_AS __attribute__((address_space(4)))
#else
#define PUSH_CONST_AS
#endif

namespace {

// Per-velocity records of the push kernel, in segment order, in two tables
// so that the loads of a whole batch can be addressed from a few scalar
// registers before any arithmetic:
// address record
//   roff     byte offset of the velocity's input plane
//   dx       byte shift to the upwind column, -sgn(cos th) * element size
//   sy       upwind row sign as +-1
struct alignas(16) PAddr {
    long long roff;
    int dx, sy;
};
// arithmetic record
//   w[4]     bilinear weights (1-ax)(1-ay), ax(1-ay), (1-ax)ay, ax ay
//   H[NH]    w_v {1, cos th, sin th, ..., cos m th, sin m th}: m up to NM
//            (NH = 2 NM + 1), or NM + 2 for deviation storage (NH = 2 NM + 5)
//   cth sth  direction (collision frequency U^0 - U.n_v)
//   mono[8]  c, s, c^2, c s, c^3, c^2 s, c^3 s, c^2 s^2 with c = cos th, s = sin th
//   woff     byte offset of the velocity's output plane (padding: the spare plane)
template <typename T, int NH>
struct alignas(16) PRec {
    T w[4];
    T H[NH];
    T cth, sth;
    T mono[8];
    long long woff;
};

// Harmonic entries of a record: the own-site equilibrium (order NM), or the
// deviation form's corner series (order NM + 2).
__host__ __device__ constexpr int push_nh(int NM, bool dev) { return 2 * NM + 1 + (dev ? 4 : 0); }

// Storage of the populations (plain) or deviations (DEV) and its conversion
// to the arithmetic type: FP64, FP32, or bfloat16 (the high half of the FP32
// pattern; rounding to nearest even).
template <typename T, typename ST>
__device__ __forceinline__ T st_to(ST s) { return (T)s; }
template <>
__device__ __forceinline__ float st_to<float, unsigned short>(unsigned short s)
{
    return __uint_as_float((unsigned)s << 16);
}
// Rounding to the storage type.  bfloat16 rounds stochastically: round to
// nearest would drop every per-step change of a deviation smaller than half
// a bfloat16 ulp, the same way each step (a bias that accumulates), while
// stochastic rounding rounds up with probability equal to the discarded
// fraction, so the stored value is exact in expectation.  r: 32 random bits.
template <typename ST, typename T>
__device__ __forceinline__ ST to_st(T v, unsigned r) { return (ST)v; }
template <>
__device__ __forceinline__ unsigned short to_st<unsigned short, float>(float v, unsigned r)
{
    // v_cvt_sr_bf16_f32 adds the high 16 bits of r to the 16 discarded bits
    // and truncates; the result is a bfloat16 pair (low half written here)
    // (the untouched high half is v's own: no extra register is cleared)
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned short,
                              __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(b2, v), v, r, false)[0]);
}

// 32-bit finaliser of MurmurHash3 (Appleby): a bijective mix of the bits.
__device__ __forceinline__ unsigned fmix32(unsigned h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// One segment: the velocities of shell i with upwind signs (sx, sy) of
// quadrant q, padded with null records to whole load batches.
struct PSeg {
    int begin, nbatch;
    double p;
};

struct PushParams {
    const PAddr* paddr;      // PAddr[]
    const void* prec;        // PRec<T, NH>[]
    const PSeg* seg;         // [4][Np]
    const void* ytab;        // deviation storage: [4][Np][push_ys(NM)] (T), Y[q][i][t * 9 + j] = sum over the
                             // segment's velocities of H_t mono_j, mono = (1, c, s, c^2, c s, c^3, c^2 s,
                             // c^3 s, c^2 s^2); null otherwise
    const double* G;
    const double* Pc;
    int nx, ny, Np, bcx, bcy, ntiles;
    int nrec;                // records in the tables (all segments)
    int sb;                  // bands of 4 rows taken column by column (work-group order)
    long long S;
    double rate, dt;
    int* flag;
};

// Work-group order of the push kernel: groups of P.sb bands of 4 rows are
// taken column by column, so that vertically adjacent work-groups (whose
// boundary rows are each other's upwind rows) run at the same time.

// Band (of 4 rows) and tile column of work-group b in that order.
__device__ __forceinline__ void push_wg_tile(int b, int ntx, int ny, int sb, int& band, int& col)
{
    const int nb = (ny + 3) >> 2;
    const int g = b / (sb * ntx);
    const int sbg = min(sb, nb - g * sb);   // bands in this group
    const int r = b - g * sb * ntx;
    band = g * sb + r % sbg;
    col = r / sbg;
}

// Scalar-cache prefetch distance of the push kernel, in load batches (0: off).
#define RLBM_PUSH_PREFETCH 2

constexpr int NMOM = 8;     // N^0 N^x N^y T^00 T^0x T^0y T^xx T^xy

// Quadrant q: upwind signs sx = +1 for q in {0, 1}, sy = +1 for q in {0, 3}.
__host__ __device__ constexpr int qsx(int q) { return q < 2 ? 1 : -1; }
__host__ __device__ constexpr int qsy(int q) { return (q == 0 || q == 3) ? 1 : -1; }

__device__ __forceinline__ int wrapi(int i, int n, int bc)
{
    if (bc == RLBM_BC_PERIODIC) {
        if (i < 0) i += n;
        if (i >= n) i -= n;
    } else {
        i = i < 0 ? 0 : (i >= n ? n - 1 : i);
    }
    return i;
}

__device__ __forceinline__ int xcd_remap_p(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, k = b & 7, j = b >> 3;
    return k * q + min(k, r) + j;
}

// Partial sums of a buffer (element type T):
//   R[d][k][S]   row slots: the contributions of the sources at (x, y) to the
//                moments k of the sites in row y + dy at column x, d = 0, 1, 2
//                for dy = 0, +1, -1 (the x-displaced parts already moved to
//                their target column inside the wave);
//   H[edge][dir][d][k][ny][ntx]   the x-displaced parts of the first (edge 0)
//                and last (edge 1) column of each tile, for sx = +1 (dir 0)
//                and sx = -1 (dir 1): the parts that leave the tile, and the
//                images a clamped boundary needs.
__host__ __device__ inline long long halo_off(long long S, int edge, int dir, int d, int k, int row, int tc, int ny,
                                              int ntx)
{
    return 3LL * NMOM * S + ((((long long)(edge * 2 + dir) * 3 + d) * NMOM + k) * ny + row) * ntx + tc;
}

// Corner series of the deviation form for one segment (upwind signs sx, sy):
// the harmonic coefficients De[0 .. 2 NM + 4] of
//   E(th) / w = A0 + al c A^x + be s A^y + al be c s A^xy,
// al = dt sx, be = dt sy, c = cos th, s = sin th, where A0 = C(x0), A^x =
// C(x1) - C(x0), A^y = C(x2) - C(x0), A^xy = C(x3) - C(x1) - C(x2) + C(x0) are
// the bilinear-monomial combinations of the corner coefficients (x1 the x
// upwind neighbour, x2 the y upwind one, x3 both).  Products with c, s and
// c s = sin(2 th) / 2 move a harmonic m to m +- 1 and m +- 2.  Index of
// cos m th: 2m - 1, of sin m th: 2m (m >= 1), constant: 0.
// AT: the arithmetic type (that of the step).
template <int NM, typename AT, typename LoadC>
__device__ __forceinline__ void corner_series(AT al, AT be, LoadC loadc, AT* De)
{
    constexpr int NT = 2 * NM + 1, NE = NT + 4;
#pragma unroll
    for (int t = 0; t < NE; ++t) De[t] = AT(0);
    auto ic = [](int k) { return k == 0 ? 0 : 2 * k - 1; };
    auto is = [](int k) { return 2 * k; };
    const AT hal = AT(0.5) * al, hbe = AT(0.5) * be, qab = AT(0.25) * al * be;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        AT c0, c1, c2, c3;
        loadc(t, c0, c1, c2, c3);
        const AT A0 = c0, Ax = c1 - c0, Ay = c2 - c0, Axy = (c3 - c1) - (c2 - c0);
        const AT h = hal * Ax, k = hbe * Ay, l = qab * Axy;
        if (t == 0) {
            De[0] += A0;
            De[ic(1)] += AT(2) * h;
            De[is(1)] += AT(2) * k;
            De[is(2)] += AT(2) * l;
        } else if (t & 1) {   // cos m th
            const int m = (t + 1) / 2;
            De[ic(m)] += A0;
            De[ic(m + 1)] += h;
            De[ic(m - 1)] += h;
            De[is(m + 1)] += k;
            if (m >= 2) De[is(m - 1)] -= k;
            De[is(m + 2)] += l;
            if (m >= 3) De[is(m - 2)] -= l;
            if (m == 1) De[is(1)] += l;
        } else {              // sin m th
            const int m = t / 2;
            De[is(m)] += A0;
            De[is(m + 1)] += h;
            if (m >= 2) De[is(m - 1)] += h;
            De[ic(m - 1)] += k;
            De[ic(m + 1)] -= k;
            De[ic(m + 2)] -= l;
            if (m >= 2) De[ic(m - 2)] += l;
            if (m == 1) De[ic(1)] += l;
        }
    }
}

// LDS entries per wave (arithmetic type): the halo accumulator, the row
// slots and, for deviation storage, the site's equilibrium coefficients of
// the current shell ([2 NM + 1][64]).
__host__ __device__ constexpr int push_acc_entries() { return 96 + 3 * NMOM * 64; }
__host__ __device__ constexpr int push_wlds(int NM, bool dev) { return push_acc_entries() + (dev ? (2 * NM + 1) * 64 : 0); }

// Entries per segment of the deviation form's Y table as staged in LDS (the
// 9 x (2 NM + 1) sums, padded to whole 16-byte rows).
__host__ __device__ constexpr int push_ys(int NM) { return ((2 * NM + 1) * 9 + 3) / 4 * 4; }

// One wave-tile: 64 sites of row ty starting at column 64 tx.  INIT computes
// only the partial sums of the current populations (no stream, no
// collision, no population store).  lh: this wave's LDS, the 96-entry halo
// accumulator [edge][dir][d][k] followed by the row slots [d][k][64] and,
// for deviation storage, the coefficients [2 NM + 1][64].
// ylds (DEV): the work-group's copy of the Y table, push_ys(NM) entries per
// segment.
// T is the arithmetic type, ST the storage type of the populations (plain)
// or of the deviations (DEV, with the per-shell equilibrium coefficients in
// cin / cout, [Np][2 NM + 1][S] of T).
template <typename T, typename ST, int NM, int LB, bool INIT, bool DEV>
__device__ __forceinline__ void push_tile(const ST* __restrict__ fin, ST* __restrict__ fout, const T* __restrict__ pin,
                                          T* __restrict__ pout, const T* __restrict__ cin, T* __restrict__ cout,
                                          const PushParams& P, int tile, T* __restrict__ lh, const T* ylds,
                                          bool live)
{
    constexpr int NT = 2 * NM + 1;
    constexpr int NH = push_nh(NM, DEV);
    constexpr int GS = (RLBM_NMAX + 1) * (RLBM_NMAX + 1);
    using CRec = const PUSH_CONST_AS PRec<T, NH>;
    using CAddr = const PUSH_CONST_AS PAddr;
    CAddr* const adr = (CAddr*)P.paddr;
    using CSeg = const PUSH_CONST_AS PSeg;
    using CDbl = const PUSH_CONST_AS double;
    CRec* const rec = (CRec*)P.prec;
    CSeg* const seg = (CSeg*)P.seg;
    CDbl* const Gtab = (CDbl*)P.G;
    CDbl* const Pc = (CDbl*)P.Pc;

    const int lane = threadIdx.x & 63;
    const int ntx = (P.nx + 63) >> 6;
    const int ty = tile / ntx;
    const int tx = tile - ty * ntx;
    const int x = tx * 64 + lane;
    const int last = min(63, P.nx - 1 - tx * 64);   // last column of the tile, as a lane
    const bool active = x < P.nx && live;
    const int xc = x < P.nx ? x : P.nx - 1;
    const bool interior = tx > 0 && (tx + 1) * 64 < P.nx && live;
    const long long S = P.S;
    const int xm = wrapi(xc - 1, P.nx, P.bcx), xp = wrapi(xc + 1, P.nx, P.bcx);
    const int ym = wrapi(ty - 1, P.ny, P.bcy), yp = wrapi(ty + 1, P.ny, P.bcy);
    const long long site = (long long)ty * P.nx + xc;
    const int rows[3] = {ty, ym, yp};   // source row of the slot d = 0 (dy 0), 1 (dy +1), 2 (dy -1)

    // 1. moments of the streamed populations, gathered from the partial sums
    //    pushed by the previous step: the three row slots at this column, and
    //    for the first / last column of the tile the halo parts of the
    //    upwind column outside it (FP64 sums)
    //    Collision factors: plain, omega = a0 - ax cos - ay sin; DEV,
    //    1 - omega = a0 + ax cos + ay sin.
    T a0 = DEV ? T(1) : T(0), ax = T(0), ay = T(0);
    double fn_ = 0, fT = 0, fU0 = 0, fUx = 0, fUy = 0;
    int ok = 0;
    unsigned srseed = 0;
    if (!INIT) {
        const int cl = wrapi(tx * 64 - 1, P.nx, P.bcx);            // column left of the tile
        const int cr = wrapi(tx * 64 + last + 1, P.nx, P.bcx);     // column right of the tile
        const int el = (cl & 63) == 0 ? 0 : 1, er = (cr & 63) == 0 ? 0 : 1;
        double mom[9];
#pragma unroll 1
        for (int k = 0; k < NMOM; ++k) {
            double s = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) s += (double)pin[(long long)(d * NMOM + k) * S + (long long)rows[d] * P.nx + xc];
            if (lane == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) s += (double)pin[halo_off(S, el, 0, d, k, rows[d], cl >> 6, P.ny, ntx)];
            }
            if (lane == last) {
#pragma unroll
                for (int d = 0; d < 3; ++d) s += (double)pin[halo_off(S, er, 1, d, k, rows[d], cr >> 6, P.ny, ntx)];
            }
            mom[k] = s;
        }
        mom[8] = mom[3] - mom[6];
        const Frame fr = landau_frame(mom);
        ok = fr.ok;
        if (!fr.ok && active) atomicOr(P.flag, 1);
        if (DEV) {
            a0 = fr.ok ? (T)(1.0 - P.rate * fr.U0) : T(1);
            ax = fr.ok ? (T)(P.rate * fr.Ux) : T(0);
            ay = fr.ok ? (T)(P.rate * fr.Uy) : T(0);
        } else {
            a0 = fr.ok ? (T)(P.rate * fr.U0) : T(0);
            ax = fr.ok ? (T)(P.rate * fr.Ux) : T(0);
            ay = fr.ok ? (T)(P.rate * fr.Uy) : T(0);
        }
        fn_ = fr.n; fT = fr.T; fU0 = fr.U0; fUx = fr.Ux; fUy = fr.Uy;
        // stochastic rounding (bfloat16 deviations): a random stream per site
        // and step drawn from the site index and the bits of its moments,
        // which change from step to step; deterministic in the stored state,
        // so that a resumed run or a replayed graph rounds alike
        if (DEV && sizeof(ST) == 2) {
            const unsigned long long b0 = __double_as_longlong(mom[0]), b3 = __double_as_longlong(mom[3]);
            srseed = fmix32((unsigned)site * 0x9e3779b9u ^ (unsigned)b0 ^ (unsigned)(b0 >> 32) ^
                            fmix32((unsigned)b3 ^ (unsigned)(b3 >> 32)));
        }
    }

    constexpr unsigned ES = sizeof(ST);
    const unsigned ocb = (unsigned)xc * ES;
    const unsigned omb = (unsigned)xm * ES;
    const unsigned opb = (unsigned)xp * ES;
    const long long rowb = (long long)ty * P.nx * ES;
    const long long dmb = (long long)ym * P.nx * ES - rowb;
    const long long dpb = (long long)yp * P.nx * ES - rowb;
    const char* const inb = reinterpret_cast<const char*>(fin) + rowb;
    char* const outb = reinterpret_cast<char*>(fout) + rowb;
    auto ld = [](const char* base, unsigned off) __attribute__((always_inline)) -> T {
        return st_to<T, ST>(*reinterpret_cast<const ST*>(base + off));
    };
    const T act = active ? T(1) : T(0);   // columns past the grid contribute nothing
    // value of lane (lane - sx), zero where that lane is outside the wave
    auto from_upwind = [&](T v, int sx) __attribute__((always_inline)) -> T {
        const int src = lane - sx;
        const T r = __shfl(v, src & 63, 64);
        return (src < 0 || src > 63) ? T(0) : r;
    };

    for (int j = lane; j < 96; j += 64) lh[j] = T(0);
    // row slots d = 0, 1, 2 (dy 0, +1, -1), touched once per segment: in
    // this wave's LDS after the halo accumulator, lane-contiguous
    T* const lrow = lh + 96;
    T* const lcc = lh + push_acc_entries();   // DEV: [2 NM + 1][64]
    auto R = [&](int d, int k) __attribute__((always_inline)) -> T& { return lrow[(d * NMOM + k) * 64 + lane]; };
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < NMOM; ++k) R(d, k) = T(0);
    const T dt = (T)P.dt;

    // 2. the velocities, shell by shell and, inside a shell, quadrant by
    //    quadrant; interior tiles (FAST) reach the x neighbour by a scalar
    //    shift of the plane offset and store without a lane mask
    auto run = [&](auto fast) __attribute__((always_inline)) {
        constexpr bool FAST = decltype(fast)::value;
        for (int i = 0; i < P.Np; ++i) {
            // plain: the new equilibrium's coefficients; DEV: the stored
            // (rounded) coefficients of the new equilibrium, or in INIT those
            // of the current state
            T cc[NT];
            if (!INIT) {
                // The frame as opaque values, once per shell.  Otherwise the
                // compiler hoists the shell-independent FP64 factors of the
                // coefficients (the polynomials in U^0) out of the shell loop
                // and holds them through every velocity batch: 50 to 100 more
                // VGPRs, which leaves the deviation forms, FP64 and order 7 at
                // 2 waves per SIMD.  The plain FP32 instances of orders 3 and 5
                // keep the hoisting (less FP64 work per site): at order 5 the
                // 158 VGPRs give 3 waves per SIMD, the measured optimum (a
                // fourth wave costs L2 reuse of the halo lines), and at order 3
                // both forms give 4.
                constexpr bool HOIST = !DEV && sizeof(T) == 4 && NM <= 5;
                double sn = fn_, sT = fT, sU0 = fU0, sUx = fUx, sUy = fUy;
                if (!HOIST) asm volatile("" : "+v"(sn), "+v"(sT), "+v"(sU0), "+v"(sUx), "+v"(sUy));
                shell_coeffs<NM>(Gtab + (size_t)i * GS, Pc, sn, sT, sU0, sUx, sUy,
                                 [&](int mm, double cm, double sm) __attribute__((always_inline)) {
                                     if (!ok) cm = sm = 0.0;
                                     if (mm == 0) {
                                         cc[0] = (T)cm;
                                     } else {
                                         cc[2 * mm - 1] = (T)cm;
                                         cc[2 * mm] = (T)sm;
                                     }
                                 });
                if (DEV && (FAST || active)) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) cout[(long long)(i * NT + t) * S + site] = cc[t];
                }
            } else if (DEV) {
#pragma unroll
                for (int t = 0; t < NT; ++t) cc[t] = cin[(long long)(i * NT + t) * S + site];
            }
            // DEV: the coefficients go to this wave's LDS, read back per
            // segment (few registers stay live across the quadrants)
            if (DEV) {
#pragma unroll
                for (int t = 0; t < NT; ++t) lcc[t * 64 + lane] = cc[t];
            }
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                const int sx = qsx(q), sy = qsy(q);
                const int dY = sy > 0 ? 1 : 2;   // row slot of the y-displaced parts
                CSeg& G = seg[q * P.Np + i];
                // DEV: the segment's series E - F_new (E from the corners' old
                // coefficients)
                T D[DEV ? NH : 1];
                if (DEV && !INIT) {
                    const int xs = sx > 0 ? xm : xp;
                    const int ys = sy > 0 ? ym : yp;
                    const long long s0 = site, s1 = (long long)ty * P.nx + xs, s2 = (long long)ys * P.nx + xc,
                                    s3 = (long long)ys * P.nx + xs;
                    corner_series<NM, T>(dt * (T)sx, dt * (T)sy,
                                         [&](int t, T& c0, T& c1, T& c2, T& c3) __attribute__((always_inline)) {
                                             const T* pl = cin + (long long)(i * NT + t) * S;
                                             c0 = pl[s0]; c1 = pl[s1]; c2 = pl[s2]; c3 = pl[s3];
                                         },
                                         D);
#pragma unroll
                    for (int t = 0; t < NT; ++t) D[t] -= lcc[t * 64 + lane];
                }
                // sum f, f c, f s, f c^2, f c s, f c^3, f c^2 s, f c^3 s,
                // f c^2 s^2 over the segment: each load batch's sums start from
                // zero in T and are carried into FP64 (compensated: T rounds
                // only within a batch)
                double Sm[9];
#pragma unroll
                for (int j = 0; j < 9; ++j) Sm[j] = 0.0;
                const int v0 = G.begin;
                const unsigned osb = sx > 0 ? omb : opb;   // to the upwind column (edge tiles)
                for (int kb = 0; kb < G.nbatch; ++kb) {
                    // the lanes' byte offsets, made opaque once per batch: each
                    // load and store is then addressed as a scalar base plus a
                    // 32-bit lane offset, with no 64-bit vector address
                    // arithmetic (hoisting base + offset out of the loop would
                    // keep the sums in vector registers)
                    unsigned oc = ocb, os = osb;
                    asm volatile("" : "+v"(oc), "+v"(os));
                    T Sb[9];
#pragma unroll
                    for (int j = 0; j < 9; ++j) Sb[j] = T(0);
                    // the records RLBM_PUSH_PREFETCH batches on (the table runs
                    // on across segments): one word of each scalar-cache line,
                    // taken in only at the end of this batch
                    unsigned pf = 0;
                    if (RLBM_PUSH_PREFETCH > 0) {
                        const int ahead = min(v0 + (kb + RLBM_PUSH_PREFETCH) * LB, P.nrec - LB);
                        using CWord = const PUSH_CONST_AS unsigned;
                        const PUSH_CONST_AS char* rb = (const PUSH_CONST_AS char*)(rec + ahead);
                        constexpr int RB = LB * (int)sizeof(PRec<T, NH>);
#pragma unroll
                        for (int o = 0; o < RB; o += 64) pf += *(CWord*)(rb + o);
                        pf += *(CWord*)(rb + RB - 4);
                        pf += *(CWord*)((const PUSH_CONST_AS char*)(adr + ahead));
                    }
                    // LB velocities' loads in flight, then their arithmetic
                    T raw[LB][4];
#pragma unroll
                    for (int b = 0; b < LB; ++b) {
                        CAddr& A = adr[v0 + kb * LB + b];
                        const char* p0 = inb + A.roff;
                        if (INIT) {
                            raw[b][0] = ld(p0, oc);
                        } else {
                            const char* p1 = p0 + (A.sy > 0 ? dmb : dpb);
                            if (FAST) {
                                raw[b][0] = ld(p0, oc); raw[b][1] = ld(p0 + A.dx, oc);
                                raw[b][2] = ld(p1, oc); raw[b][3] = ld(p1 + A.dx, oc);
                            } else {
                                raw[b][0] = ld(p0, oc); raw[b][1] = ld(p0, os);
                                raw[b][2] = ld(p1, oc); raw[b][3] = ld(p1, os);
                            }
                        }
                    }
#pragma unroll
                    for (int b = 0; b < LB; ++b) {
                        CRec& Rr = rec[v0 + kb * LB + b];
                        T fnew;
                        if (INIT) {
                            // padding records (zero equilibrium row) contribute
                            // nothing; real ones exactly their value, as in the step
                            fnew = Rr.H[0] != T(0) ? raw[b][0] : T(0);
                        } else if (DEV) {
                            const T gs = Rr.w[0] * raw[b][0] + Rr.w[1] * raw[b][1] + Rr.w[2] * raw[b][2] +
                                         Rr.w[3] * raw[b][3];
                            T dv = D[0] * Rr.H[0];
#pragma unroll
                            for (int t = 1; t < NH; ++t) dv += D[t] * Rr.H[t];
                            const T om1 = a0 + ax * Rr.cth + ay * Rr.sth;
                            // velocity v draws srseed + v phi (a Weyl sequence, phi
                            // the golden-ratio increment)
                            const unsigned rv = srseed + (unsigned)(v0 + kb * LB + b) * 0x9e3779b9u;
                            const ST gq = to_st<ST, T>(om1 * (gs + dv), rv);
                            fnew = st_to<T, ST>(gq);   // the stored value feeds the partial sums
                            ST* dst = reinterpret_cast<ST*>(outb + Rr.woff + oc);
                            if (FAST || active) __builtin_nontemporal_store(gq, dst);
                        } else {
                            const T f = Rr.w[0] * raw[b][0] + Rr.w[1] * raw[b][1] + Rr.w[2] * raw[b][2] +
                                        Rr.w[3] * raw[b][3];
                            T feq = cc[0] * Rr.H[0];
#pragma unroll
                            for (int t = 1; t < NT; ++t) feq += cc[t] * Rr.H[t];
                            const T om = a0 - ax * Rr.cth - ay * Rr.sth;
                            fnew = f + om * (feq - f);
                            // non-temporal: the next read of this plane is a step away
                            T* dst = reinterpret_cast<T*>(outb + Rr.woff + oc);
                            if (FAST || active) __builtin_nontemporal_store(fnew, dst);
                        }
                        // explicit FMAs: the step and the rebuild (INIT) must
                        // produce the same partial sums bit for bit
                        Sb[0] += fnew;
#pragma unroll
                        for (int j = 0; j < 8; ++j) Sb[1 + j] = fma(fnew, (T)Rr.mono[j], Sb[1 + j]);
                    }
#pragma unroll
                    for (int j = 0; j < 9; ++j) Sm[j] += (double)Sb[j];
                    if (RLBM_PUSH_PREFETCH > 0) asm volatile("" ::"s"(pf));
                }
                // DEV: add the monomial sums of the equilibrium part F of the
                // stored state, sum_t C_t Y_t (explicit FMAs, same order in
                // the step and the rebuild)
                if (DEV) {
                    // (2 NM + 1 terms in T, carried into the FP64 sums once)
                    const T* yq = ylds + (q * P.Np + i) * push_ys(NM);
                    T Sf[9];
#pragma unroll
                    for (int j = 0; j < 9; ++j) Sf[j] = T(0);
#pragma unroll 1
                    for (int t = 0; t < NT; ++t) {
                        const T c = lcc[t * 64 + lane];
#pragma unroll
                        for (int j = 0; j < 9; ++j) Sf[j] = fma(c, yq[t * 9 + j], Sf[j]);
                    }
#pragma unroll
                    for (int j = 0; j < 9; ++j) Sm[j] += (double)Sf[j];
                }
                // fold the monomial sums into the weighted moment sums of the
                // segment's four corners: with T_e = sum f e, the corner sums
                // of e are C0 = T_e - al T_ce - be T_se + ga T_cse (target
                // (x, y)), C1 = al T_ce - ga T_cse (x + sx, y), C2 = be T_se -
                // ga T_cse (x, y + sy), C3 = ga T_cse (x + sx, y + sy).  No
                // contraction here, so that both instantiations round alike.
                {
#pragma clang fp contract(off)
                // The fold runs in FP64 with the step's bilinear weights (dt in
                // T, as the tables hold it); each segment's corner parts are
                // rounded once to T as they enter the row slots.
                const double al = (double)(dt * (T)sx), be = (double)(dt * (T)sy), ga = al * be;
                const double S1 = Sm[0], Sc = Sm[1], Ss = Sm[2], Scc = Sm[3], Scs = Sm[4], Sccc = Sm[5],
                             Sccs = Sm[6], Scccs = Sm[7], Sccss = Sm[8];
                const double Sss = S1 - Scc, Scss = Sc - Sccc;
                // (T, Tc, Ts, Tcs) of e = 1, c, s, c^2, c s
                const double Te[5][4] = {{S1, Sc, Ss, Scs},
                                         {Sc, Scc, Scs, Sccs},
                                         {Ss, Scs, Sss, Scss},
                                         {Scc, Sccc, Sccs, Scccs},
                                         {Scs, Sccs, Scss, Sccss}};
                const double p = G.p, p2 = G.p * G.p;
                const double actd = (double)act;
                // moment k: angular factor e(k), radial factor p or p^2
                constexpr int EK[NMOM] = {0, 1, 2, 0, 1, 2, 3, 4};
                const int dir = sx > 0 ? 0 : 1;
#pragma unroll
                for (int k = 0; k < NMOM; ++k) {
                    const double* t4 = Te[EK[k]];
                    const double r = k < 3 ? p : p2;
                    const double d3 = actd * r * (ga * t4[3]);
                    const double d1 = actd * r * (al * t4[1]) - d3;
                    const double d2 = actd * r * (be * t4[2]) - d3;
                    const T c0 = (T)(actd * r * t4[0] - d1 - d2 - d3);
                    const T c1 = (T)d1, c2 = (T)d2, c3 = (T)d3;
                    // x-displaced parts move to their target column inside the
                    // wave; the tile's edge columns also keep them for the halo
                    R(0, k) += c0 + from_upwind(c1, sx);
                    R(dY, k) += c2 + from_upwind(c3, sx);
                    if (lane == 0) {
                        lh[((0 * 2 + dir) * 3 + 0) * NMOM + k] += c1;
                        lh[((0 * 2 + dir) * 3 + dY) * NMOM + k] += c3;
                    }
                    if (lane == last) {
                        lh[((1 * 2 + dir) * 3 + 0) * NMOM + k] += c1;
                        lh[((1 * 2 + dir) * 3 + dY) * NMOM + k] += c3;
                    }
                }
                }
            }
        }
    };
    if (interior)
        run(std::true_type{});
    else
        run(std::false_type{});

    // 3. partial sums for the next step: row slots of every column, halo
    //    parts of the tile's first and last columns
    if (interior || active) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int k = 0; k < NMOM; ++k) pout[(long long)(d * NMOM + k) * S + site] = R(d, k);
    }
    if (live && (lane == 0 || lane == last)) {
#pragma unroll 1
        for (int ed = 0; ed < 2; ++ed) {
            if ((ed == 0 && lane != 0) || (ed == 1 && lane != last)) continue;
            for (int dir = 0; dir < 2; ++dir)
                for (int d = 0; d < 3; ++d)
                    for (int k = 0; k < NMOM; ++k)
                        pout[halo_off(S, ed, dir, d, k, ty, tx, P.ny, ntx)] = lh[((ed * 2 + dir) * 3 + d) * NMOM + k];
        }
    }
}

// Minimum work-groups per execution unit, and the load batch of FP32.
#define RLBM_PUSH_WPE 1
#define RLBM_PUSH_LB_F32 8

template <typename T, typename ST, int NM, int LB, bool INIT, bool DEV>
__global__ __launch_bounds__(256, RLBM_PUSH_WPE) void k_push_step(const ST* __restrict__ fin, ST* __restrict__ fout,
                                                   const T* __restrict__ pin, T* __restrict__ pout,
                                                   const T* __restrict__ cin, T* __restrict__ cout, PushParams P)
{
    extern __shared__ __align__(16) unsigned char psmem[];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    // A work-group's 4 waves take the same 64 columns of 4 consecutive rows:
    // they run through the velocities side by side, so the upwind row one
    // wave reads is the row its neighbour reads at about the same time (L1/L2
    // reuse; one grid row of all velocities is far larger than the L2).
    const int ntx = (P.nx + 63) >> 6;
    const int b = xcd_remap_p(blockIdx.x, gridDim.x);
    int band, col;
    push_wg_tile(b, ntx, P.ny, P.sb, band, col);
    const int ty = band * 4 + wv;
    T* const ylds = reinterpret_cast<T*>(psmem) + 4 * push_wlds(NM, DEV);
    if (DEV) {
        // the work-group's copy of the Y table (read with broadcast LDS loads
        // in each segment's fold); the kernel's only barrier
        using CTab = const PUSH_CONST_AS T;
        const int n = 4 * P.Np * push_ys(NM);
        for (int j = threadIdx.x; j < n; j += 256) ylds[j] = ((CTab*)P.ytab)[j];
        __syncthreads();
    }
    if (ty >= P.ny) return;   // whole waves
    const bool live = true;
    const int tile = ty * ntx + col;
    T* lh = reinterpret_cast<T*>(psmem) + (size_t)wv * push_wlds(NM, DEV);
    push_tile<T, ST, NM, LB, INIT, DEV>(fin, fout, pin, pout, cin, cout, P, tile, lh, ylds, live);
}

// Batched form: the push-kernel problems of a batch advance together in one
// flat launch of 4-row work-groups; work-group g belongs to the problem
// whose range [wg0, wg0 + wgs) holds it.
struct PushDesc {
    void* f[2];
    void* pp[2];
    PushParams P;
    int wg0, wgs;
};

template <typename T, int NM, int LB>
__global__ __launch_bounds__(256, RLBM_PUSH_WPE) void k_push_batch(const PushDesc* __restrict__ descs, int nprob,
                                                                    int parity)
{
    extern __shared__ __align__(16) unsigned char psmem[];
    using CDesc = const PUSH_CONST_AS PushDesc;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int g = xcd_remap_p(blockIdx.x, gridDim.x);
    int p = 0;
    int step = 1;
    while (step * 2 <= nprob) step *= 2;
    for (; step > 0; step >>= 1)
        if (p + step < nprob && ((CDesc*)descs)[p + step].wg0 <= g) p += step;
    CDesc& D = ((CDesc*)descs)[p];
    const PushParams P = D.P;
    const int ntx = (P.nx + 63) >> 6;
    const int b = g - D.wg0;
    int band, col;
    push_wg_tile(b, ntx, P.ny, P.sb, band, col);
    const int ty = band * 4 + wv;
    if (ty >= P.ny) return;   // whole waves; the kernel has no barrier
    const int tile = ty * ntx + col;
    T* lh = reinterpret_cast<T*>(psmem) + (size_t)wv * push_wlds(NM, false);
    push_tile<T, T, NM, LB, false, false>(static_cast<const T*>(D.f[parity]), static_cast<T*>(D.f[parity ^ 1]),
                                          static_cast<const T*>(D.pp[parity]), static_cast<T*>(D.pp[parity ^ 1]),
                                          nullptr, nullptr, P, tile, lh, nullptr, true);
}

// Load batch per precision: FP64 holds half as many values per register.
template <typename T>
struct PushLB {
    static constexpr int value = sizeof(T) == 8 ? 4 : RLBM_PUSH_LB_F32;
};

template <typename T, typename ST, int NM, bool DEV>
hipError_t launch_push_t(bool init, const void* fin, void* fout, const void* pin, void* pout, const void* cin,
                         void* cout, const PushParams& P, hipStream_t st)
{
    constexpr int LB = PushLB<T>::value;
    const unsigned blocks = (unsigned)(((P.nx + 63) / 64) * ((P.ny + 3) / 4));
    // 4 waves x (halo + row slots), and the Y table of the deviation form
    const size_t lds = ((size_t)4 * push_wlds(NM, DEV) + (DEV ? (size_t)4 * P.Np * push_ys(NM) : 0)) * sizeof(T);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {   // beyond the default limit of dynamic LDS: opt in (set once per size)
        static size_t configured[2] = {0, 0};
        if (lds > configured[init]) {
            const void* fn = init ? reinterpret_cast<const void*>(&k_push_step<T, ST, NM, LB, true, DEV>)
                                  : reinterpret_cast<const void*>(&k_push_step<T, ST, NM, LB, false, DEV>);
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            configured[init] = lds;
        }
    }
    if (init)
        hipLaunchKernelGGL((k_push_step<T, ST, NM, LB, true, DEV>), dim3(blocks), dim3(256), lds, st,
                           (const ST*)fin, (ST*)fout, (const T*)pin, (T*)pout, (const T*)cin, (T*)cout, P);
    else
        hipLaunchKernelGGL((k_push_step<T, ST, NM, LB, false, DEV>), dim3(blocks), dim3(256), lds, st,
                           (const ST*)fin, (ST*)fout, (const T*)pin, (T*)pout, (const T*)cin, (T*)cout, P);
    return hipGetLastError();
}

template <typename T, int NM>
hipError_t launch_push_batch_t(const void* descs, int nprob, int wgs, int parity, hipStream_t st)
{
    constexpr int LB = PushLB<T>::value;
    const size_t lds = (size_t)4 * push_wlds(NM, false) * sizeof(T);
    hipLaunchKernelGGL((k_push_batch<T, NM, LB>), dim3((unsigned)wgs), dim3(256), lds, st,
                       static_cast<const PushDesc*>(descs), nprob, parity);
    return hipGetLastError();
}

// Tables of the push kernel: segment-ordered records (T arithmetic, ST
// storage), and for deviation storage the per-segment monomial sums Y of
// the equilibrium basis.
template <typename T, typename ST, int NM, bool DEV>
int upload_push_t(rlbm_ctx c, const std::vector<VelRec<double>>& vd, std::string& err)
{
    constexpr int LB = PushLB<T>::value;
    constexpr int NT = 2 * NM + 1;
    constexpr int NH = push_nh(NM, DEV);
    const int Np = c->q.Np, K = c->q.K, nv = c->q.nvel;
    const long long S = c->S, es = (long long)sizeof(ST);
    std::vector<PRec<T, NH>> recs;
    std::vector<PAddr> adrs;
    std::vector<PSeg> segs(4 * (size_t)Np);
    std::vector<T> ytab;
    if (DEV) ytab.assign((size_t)4 * Np * push_ys(NM), T(0));
    // padding records: zero weights and equilibrium row, a store to the
    // spare plane, loads from the plane of the record before them (cache
    // hits, no extra HBM reads)
    PRec<T, NH> null;
    std::memset(&null, 0, sizeof(null));
    null.woff = (long long)nv * S * es;
    for (int q = 0; q < 4; ++q)
        for (int i = 0; i < Np; ++i) {
            PSeg& G = segs[q * Np + i];
            G.begin = (int)recs.size();
            G.p = c->q.shell_p[i];
            int count = 0;
            double Y[NT][9] = {};
            for (int j = 0; j < K; ++j) {
                const int v = i * K + j;
                const VelRec<double>& R = vd[v];
                if ((int)R.sx != qsx(q) || (int)R.sy != qsy(q)) continue;
                PRec<T, NH> A;
                std::memset(&A, 0, sizeof(A));
                A.w[0] = (T)R.w00; A.w[1] = (T)R.w10; A.w[2] = (T)R.w01; A.w[3] = (T)R.w11;
                // harmonics w {1, cos m th, sin m th}: up to the expansion
                // order (the equilibrium), or two beyond it (the corner series)
                const int mtop = DEV ? c->q.N + 2 : c->q.N;
                double H[NH] = {};
                H[0] = c->q.w[v];
                for (int m = 1; 2 * m < NH && m <= mtop; ++m) {
                    H[2 * m - 1] = c->q.w[v] * std::cos(m * c->q.theta[v]);
                    H[2 * m] = c->q.w[v] * std::sin(m * c->q.theta[v]);
                }
                for (int t = 0; t < NH; ++t) A.H[t] = (T)H[t];
                const double cs = R.cth, sn = R.sth;
                A.cth = (T)cs; A.sth = (T)sn;
                const double mono[9] = {1.0, cs, sn, cs * cs, cs * sn, cs * cs * cs, cs * cs * sn, cs * cs * cs * sn,
                                        cs * cs * sn * sn};
                for (int t = 0; t < 8; ++t) A.mono[t] = (T)mono[t + 1];
                for (int t = 0; t < NT; ++t)
                    for (int k = 0; k < 9; ++k) Y[t][k] += R.H[t] * mono[k];
                A.woff = (long long)v * S * es;
                PAddr D;
                std::memset(&D, 0, sizeof(D));
                D.roff = (long long)v * S * es;
                D.dx = (R.sx > 0 ? -1 : 1) * (int)es;
                D.sy = R.sy > 0 ? 1 : -1;
                recs.push_back(A);
                adrs.push_back(D);
                ++count;
            }
            if (DEV)
                for (int t = 0; t < NT; ++t)
                    for (int k = 0; k < 9; ++k) ytab[(size_t)(q * Np + i) * push_ys(NM) + t * 9 + k] = (T)Y[t][k];
            while (count % LB) {
                PAddr nulla;
                std::memset(&nulla, 0, sizeof(nulla));
                if (!adrs.empty()) {
                    nulla = adrs.back();
                } else {
                    nulla.dx = -(int)es;
                    nulla.sy = 1;
                }
                recs.push_back(null);
                adrs.push_back(nulla);
                ++count;
            }
            G.nbatch = count / LB;
        }
    if ((long long)recs.size() > 4LL * nv + 4LL * Np * LB) {
        err = "push table size";
        return RLBM_EINVAL;
    }
    c->pnrec = (int)recs.size();
    hipError_t e;
    if ((e = hipMalloc(&c->d_prec, recs.size() * sizeof(PRec<T, NH>))) != hipSuccess) return RLBM_ENOMEM;
    if ((e = hipMalloc(&c->d_paddr, adrs.size() * sizeof(PAddr))) != hipSuccess) return RLBM_ENOMEM;
    if ((e = hipMemcpy(c->d_paddr, adrs.data(), adrs.size() * sizeof(PAddr), hipMemcpyHostToDevice)) != hipSuccess) {
        err = hipGetErrorString(e);
        return RLBM_EDEVICE;
    }
    if ((e = hipMalloc((void**)&c->d_pseg, segs.size() * sizeof(PSeg))) != hipSuccess) return RLBM_ENOMEM;
    if ((e = hipMemcpy(c->d_prec, recs.data(), recs.size() * sizeof(PRec<T, NH>), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_pseg, segs.data(), segs.size() * sizeof(PSeg), hipMemcpyHostToDevice)) != hipSuccess) {
        err = hipGetErrorString(e);
        return RLBM_EDEVICE;
    }
    if (DEV) {
        if ((e = hipMalloc(&c->d_pytab, ytab.size() * sizeof(T))) != hipSuccess) return RLBM_ENOMEM;
        if ((e = hipMemcpy(c->d_pytab, ytab.data(), ytab.size() * sizeof(T), hipMemcpyHostToDevice)) != hipSuccess) {
            err = hipGetErrorString(e);
            return RLBM_EDEVICE;
        }
    }
    return RLBM_OK;
}

}  // namespace

// Bytes of one partial-sum buffer of the push kernel: 3 row slots x 8
// moments per site, plus the halo of the tiles' first and last columns
// (2 edges x 2 directions x 3 rows x 8 moments per tile and row).
size_t push_partial_bytes(int prec, int nx, int ny)
{
    const size_t es = arith_size(prec);
    const size_t ntx = (size_t)(nx + 63) / 64;
    return ((size_t)3 * NMOM * nx * ny + (size_t)2 * 2 * 3 * NMOM * ny * ntx) * es;
}

// Drop the push kernel's tables (capi.cpp calls it when the grid or
// precision changes and at destroy).  The partial-sum buffers live in the
// context's workspace.
void push_free(rlbm_ctx c)
{
    if (c->d_prec) (void)hipFree(c->d_prec);
    if (c->d_paddr) (void)hipFree(c->d_paddr);
    if (c->d_pseg) (void)hipFree(c->d_pseg);
    if (c->d_pytab) (void)hipFree(c->d_pytab);
    c->d_prec = nullptr;
    c->d_paddr = nullptr;
    c->d_pseg = nullptr;
    c->d_pytab = nullptr;
    c->pvalid = 0;
}

namespace {
template <typename T, typename ST, bool DEV>
int push_setup_n(rlbm_ctx c, const std::vector<VelRec<double>>& vd, std::string& err)
{
    switch (nmax_of(c->q.N)) {
        case 3: return upload_push_t<T, ST, 3, DEV>(c, vd, err);
        case 5: return upload_push_t<T, ST, 5, DEV>(c, vd, err);
        default: return upload_push_t<T, ST, 7, DEV>(c, vd, err);
    }
}
}  // namespace

// Build the push tables for the context's grid and precision (at
// rlbm_init_fields, so that no step allocates).
int push_setup(rlbm_ctx c, std::string& err)
{
    push_free(c);
    std::vector<VelRec<double>> vd;
    build_vel_table(c->q, c->dt, vd);
    switch (c->prec) {
        case RLBM_F32: return push_setup_n<float, float, false>(c, vd, err);
        case RLBM_F64: return push_setup_n<double, double, false>(c, vd, err);
        case RLBM_BF16DEV: return push_setup_n<float, unsigned short, true>(c, vd, err);
        case RLBM_F32DEV: return push_setup_n<float, float, true>(c, vd, err);
        case RLBM_F64DEV: return push_setup_n<double, double, true>(c, vd, err);
    }
    err = "unknown precision";
    return RLBM_EINVAL;
}

// One launch of the push kernel: init = 1 recomputes the partial sums of
// the current populations into pp[pcur]; init = 0 advances one step
// (f[cur] -> f[cur^1], pp[pcur] -> pp[pcur^1]).
namespace {
PushParams make_push_params(rlbm_ctx c)
{
    PushParams P;
    P.paddr = static_cast<const PAddr*>(c->d_paddr);
    P.prec = c->d_prec;
    P.seg = static_cast<const PSeg*>(c->d_pseg);
    P.ytab = c->d_pytab;
    P.G = c->d_G;
    P.Pc = c->d_Pc;
    P.nx = c->nx; P.ny = c->ny; P.Np = c->q.Np; P.bcx = c->bcx; P.bcy = c->bcy;
    P.ntiles = ((c->nx + 63) / 64) * c->ny;
    P.nrec = c->pnrec;
    P.sb = RLBM_PUSH_BANDS;
    P.S = c->S;
    P.rate = c->rate;
    P.dt = c->dt;
    P.flag = c->d_flag;
    return P;
}
}  // namespace

namespace {
template <typename T, typename ST, bool DEV>
hipError_t launch_push_n(rlbm_ctx c, bool init, const PushParams& P)
{
    const void* fin = c->f[c->cur];
    void* fout = c->f[c->cur ^ 1];
    const void* pin = c->pp[c->pcur];
    void* pout = init ? c->pp[c->pcur] : c->pp[c->pcur ^ 1];
    const void* cin = DEV ? c->cf[c->cur] : nullptr;
    void* cout = DEV ? c->cf[c->cur ^ 1] : nullptr;
    switch (nmax_of(c->q.N)) {
        case 3: return launch_push_t<T, ST, 3, DEV>(init, fin, fout, pin, pout, cin, cout, P, c->st);
        case 5: return launch_push_t<T, ST, 5, DEV>(init, fin, fout, pin, pout, cin, cout, P, c->st);
        default: return launch_push_t<T, ST, 7, DEV>(init, fin, fout, pin, pout, cin, cout, P, c->st);
    }
}
}  // namespace

hipError_t launch_push(rlbm_ctx c, bool init)
{
    const PushParams P = make_push_params(c);
    switch (c->prec) {
        case RLBM_F32: return launch_push_n<float, float, false>(c, init, P);
        case RLBM_F64: return launch_push_n<double, double, false>(c, init, P);
        case RLBM_BF16DEV: return launch_push_n<float, unsigned short, true>(c, init, P);
        case RLBM_F32DEV: return launch_push_n<float, float, true>(c, init, P);
        case RLBM_F64DEV: return launch_push_n<double, double, true>(c, init, P);
    }
    return hipErrorInvalidValue;
}

// Batched form.  push_prepare: tables and buffers of a push-kernel problem,
// and its partial sums for the current populations (pcur = cur), issued on
// the context's stream.  push_batch_wgs: its work-groups per step.
// push_batch_descs: the device descriptors of a list of problems.
int push_prepare(rlbm_ctx c, std::string& err)
{
    if (!c->d_prec) {
        err = "push tables missing";
        return RLBM_ESTATE;
    }
    if (!c->pvalid) {
        c->pcur = c->cur;
        const hipError_t e = launch_push(c, true);
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return RLBM_EDEVICE;
        }
        c->pvalid = 1;
    }
    return RLBM_OK;
}

int push_batch_wgs(rlbm_ctx c) { return ((c->nx + 63) / 64) * ((c->ny + 3) / 4); }

int push_batch_descs(const std::vector<rlbm_ctx>& cs, int bands, void** d_descs, int* total_wgs)
{
    std::vector<PushDesc> d(cs.size());
    int wg = 0;
    for (size_t i = 0; i < cs.size(); ++i) {
        rlbm_ctx c = cs[i];
        d[i].f[0] = c->f[0];
        d[i].f[1] = c->f[1];
        d[i].pp[0] = c->pp[0];
        d[i].pp[1] = c->pp[1];
        d[i].P = make_push_params(c);
        if (bands > 0) d[i].P.sb = bands;
        d[i].wg0 = wg;
        d[i].wgs = push_batch_wgs(c);
        wg += d[i].wgs;
    }
    *total_wgs = wg;
    if (d.empty()) return RLBM_OK;
    if (!*d_descs && hipMalloc(d_descs, d.size() * sizeof(PushDesc)) != hipSuccess) {
        *d_descs = nullptr;
        return RLBM_ENOMEM;
    }
    if (hipMemcpy(*d_descs, d.data(), d.size() * sizeof(PushDesc), hipMemcpyHostToDevice) != hipSuccess)
        return RLBM_EDEVICE;
    return RLBM_OK;
}

// One step of all push-kernel problems of a batch (buffers of parity
// `parity` in, the other out).
hipError_t launch_push_batch(int prec, int nmax, const void* d_descs, int nprob, int total_wgs, int parity,
                             hipStream_t st)
{
    if (nprob < 1 || total_wgs < 1) return hipSuccess;
    if (prec == RLBM_F32) {
        if (nmax == 3) return launch_push_batch_t<float, 3>(d_descs, nprob, total_wgs, parity, st);
        if (nmax == 5) return launch_push_batch_t<float, 5>(d_descs, nprob, total_wgs, parity, st);
        return launch_push_batch_t<float, 7>(d_descs, nprob, total_wgs, parity, st);
    }
    if (nmax == 3) return launch_push_batch_t<double, 3>(d_descs, nprob, total_wgs, parity, st);
    if (nmax == 5) return launch_push_batch_t<double, 5>(d_descs, nprob, total_wgs, parity, st);
    return launch_push_batch_t<double, 7>(d_descs, nprob, total_wgs, parity, st);
}
