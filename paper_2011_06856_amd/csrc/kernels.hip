// kernels.hip -- gfx950 kernels of the relativistic lattice Boltzmann step.
//
// Layout: populations f[v][y][x] (structure of arrays), one plane per
// discrete velocity, so that 64 consecutive x sites of a wavefront read and
// write 64 consecutive elements of a plane.
//
// Fused stream-and-collide (Eq. discrete-rbe): a work-group owns a tile of 64
// consecutive sites of one row (lane = site) and splits the discrete
// velocities into contiguous chunks, one per wavefront.  Per step:
//   1. each wave pulls its velocities' bilinear upwind values (Eq.
//      interpolation) from the 2x2 upwind cell quad, keeps them in registers
//      and accumulates their moments (Eq. discrete_sum_moments);
//   2. the per-wave partial moments are reduced through LDS in FP64, and the
//      Landau frame (n, eps, U) is solved in FP64 per site;
//   3. the waves compute the truncated equilibrium's harmonic coefficients of
//      the shells (FP64, stored to LDS in the compute precision);
//   4. each wave rebuilds f_eq of its velocities from the coefficients,
//      relaxes (Eq. collision, relaxing sign) and stores to the other buffer.
// Velocities of a chunk beyond the register budget VPT are streamed twice
// (recomputed in step 4) instead of being held.
#include <mutex>
#include <type_traits>

#include "rlbm_internal.h"

// Constant address space for read-only tables in device code (the host pass
// of this file sees plain pointers).
#ifdef __HIP_DEVICE_COMPILE__
#define RLBM_CONST_AS __attribute__((address_space(4)))
#else
#define RLBM_CONST_AS
#endif

namespace {

// Work-groups are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8);
// renumber them so that each XCD owns one contiguous range of tiles, whose
// neighbouring rows then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, k = b & 7, j = b >> 3;
    return k * q + min(k, r) + j;
}

// Sum of one word of each 64-byte scalar-cache line of [p, p + BYTES): read
// to bring those lines into the scalar cache ahead of their use.
template <int BYTES>
__device__ __forceinline__ unsigned touch_lines(const RLBM_CONST_AS char* p)
{
    unsigned s = 0;
#pragma unroll
    for (int o = 0; o < BYTES; o += 64) s += *(const RLBM_CONST_AS unsigned*)(p + o);
    return s;
}

__device__ __forceinline__ int wrap_idx(int i, int n, int bc)
{
    if (bc == RLBM_BC_PERIODIC) {
        if (i < 0) i += n;
        if (i >= n) i -= n;
    } else {
        i = i < 0 ? 0 : (i >= n ? n - 1 : i);
    }
    return i;
}

// One work-group tile of the fused step (64 sites of one row, all
// velocities); smem is the work-group's dynamic LDS.  `tile` runs over bands
// of P.band rows, and within a band down each column of tiles before the
// next: consecutive tiles (those in flight together on one XCD) then form a
// block a few tiles wide and P.band tall, so that the upwind row a tile reads
// is read by its neighbour in the block at about the same time (L2 reuse even
// when one grid row of all velocities exceeds the L2).
template <typename TS, typename TC, int NM, int VPT, bool GEN = false>
__device__ __forceinline__ void sc_tile(const TS* __restrict__ fin, TS* __restrict__ fout,
                                        const SRec<TC>* srec_, const CRec<TC, NM>* crec_, const double* Gtab_,
                                        const double* Pc_, const SCParams& P, int tile, unsigned char* smem)
{
    constexpr int NT = 2 * NM + 1;
    constexpr int NMOM = sizeof(TC) == 8 ? 9 : 8;   // FP32: T^yy = T^00 - T^xx
    constexpr int GS = (RLBM_NMAX + 1) * (RLBM_NMAX + 1);
    constexpr int LB = RLBM_LB;
    // The tables are read through the constant address space: they are not
    // written during the kernel, so wave-uniform reads become scalar loads
    // even where the pointers themselves come from memory (batched form).
    using CSRec = const RLBM_CONST_AS SRec<TC>;
    using CCRec = const RLBM_CONST_AS CRec<TC, NM>;
    using CDbl = const RLBM_CONST_AS double;
    CSRec* const srec = (CSRec*)srec_;
    CCRec* const crec = (CCRec*)crec_;
    CDbl* const Gtab = (CDbl*)Gtab_;
    CDbl* const Pc = (CDbl*)Pc_;
    static_assert(VPT % LB == 0, "VPT must be a multiple of the load batch");
    static_assert(LB <= 8 && LB % 4 == 0, "a batch's upwind signs are read as one 8-byte word");
    const int NW = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double* part = reinterpret_cast<double*>(smem);    // [NW][NMOM][64]
    TC* coef = reinterpret_cast<TC*>(part + NW * NMOM * 64);   // [Np][NT][64]

    const int ntx = (P.nx + 63) >> 6;
    const int band = tile / (ntx * P.band);
    const int r = tile - band * ntx * P.band;
    const int bh = min(P.band, P.ny - band * P.band);
    const int tx = r / bh;
    const int ty = band * P.band + (r - tx * bh);
    const int x = tx * 64 + lane;
    const bool active = x < P.nx;
    const int xc = active ? x : P.nx - 1;
    // Interior tiles (all 64 columns and both x neighbours inside the grid)
    // reach the x neighbour by a scalar shift of the row base; edge tiles
    // select a wrapped or clamped column per lane.
    // WALL and FIXED axes: upwind points outside the grid take the boundary's
    // values (the rows next to such an edge are edge tiles too)
    const bool bxs = GEN && P.bcx >= RLBM_BC_WALL, bys = GEN && P.bcy >= RLBM_BC_WALL;
    const bool interior = tx > 0 && (tx + 1) * 64 < P.nx && !(bys && (ty == 0 || ty == P.ny - 1));
    constexpr unsigned ES = sizeof(TS);
    const unsigned ocb = (unsigned)xc * ES;
    const unsigned omb = (unsigned)wrap_idx(xc - 1, P.nx, P.bcx) * ES;
    const unsigned opb = (unsigned)wrap_idx(xc + 1, P.nx, P.bcx) * ES;
    const long long rowb = (long long)ty * P.nx * ES;
    const long long dmb = (long long)wrap_idx(ty - 1, P.ny, P.bcy) * P.nx * ES - rowb;
    const long long dpb = (long long)wrap_idx(ty + 1, P.ny, P.bcy) * P.nx * ES - rowb;
    const char* const inb = reinterpret_cast<const char*>(fin) + rowb;
    char* const outb = reinterpret_cast<char*>(fout) + rowb;
    const int v0 = w * P.chunk;
    const int nbatch = min(P.chunk, VPT) / LB;   // batches held in registers
    // plane offsets: velocity v reads its plane (a null entry the last
    // velocity's) and writes its plane (a null entry the spare one)
    const long long pbytes = P.S * (long long)ES;
    auto rplane = [&](int v) __attribute__((always_inline)) -> long long { return (long long)min(v, P.nvel - 1) * pbytes; };
    auto wplane = [&](int v) __attribute__((always_inline)) -> long long { return (long long)min(v, P.nvel) * pbytes; };
    // the held slots run through consecutive planes: running plane pointers
    const char* const rlast = inb + rplane(P.nvel);
    const char* rcur = inb + (long long)v0 * pbytes;
    auto rnext = [&](int v) __attribute__((always_inline)) -> const char* {
        const char* p = v < P.nvel ? rcur : rlast;
        rcur += pbytes;
        return p;
    };
    auto ld = [](const char* base, unsigned off) __attribute__((always_inline)) -> TC { return (TC)*reinterpret_cast<const TS*>(base + off); };
    // boundary values: the reversed velocity's plane (K/2 planes away) and
    // the initial populations of the edge cells
    const long long rev = (long long)(P.K / 2) * pbytes;
    const char* const edges = reinterpret_cast<const char*>(P.edges);
    auto edge_x = [&](int side, int v, int row) __attribute__((always_inline)) -> TC {
        return *reinterpret_cast<const TS*>(edges + (((long long)side * P.nvel + min(v, P.nvel - 1)) * P.ny + row) * ES);
    };
    auto edge_y = [&](int side, int v, int col) __attribute__((always_inline)) -> TC {
        return *reinterpret_cast<const TS*>(
            edges + ((2LL * P.nvel * P.ny) + ((long long)side * P.nvel + min(v, P.nvel - 1)) * P.nx + col) * ES);
    };
    // code: bit 0 upwind column x + 1, bit 1 upwind row y + 1, bit 2 the
    // reversed velocity K/2 planes below
    auto load4 = [&](auto fast, int v, unsigned code, const char* p0, TC* r) __attribute__((always_inline)) {
        const bool cneg = code & 1, sneg = code & 2;
        const char* p1 = p0 + (sneg ? dpb : dmb);
        if (decltype(fast)::value) {
            const int dx = cneg ? (int)ES : -(int)ES;
            r[0] = ld(p0, ocb); r[1] = ld(p0 + dx, ocb); r[2] = ld(p1, ocb); r[3] = ld(p1 + dx, ocb);
        } else {
            const unsigned osb = cneg ? opb : omb;
            r[0] = ld(p0, ocb); r[1] = ld(p0, osb); r[2] = ld(p1, ocb); r[3] = ld(p1, osb);
            if (GEN && (bxs || bys)) {
                const bool xo = bxs && (cneg ? xc + 1 >= P.nx : xc == 0);   // this lane's upwind column is outside
                const bool yo = bys && (sneg ? ty + 1 >= P.ny : ty == 0);   // the upwind row is outside
                if (xo || yo) {
                    const bool xw = xo && P.bcx == RLBM_BC_WALL, yw = yo && P.bcy == RLBM_BC_WALL;
                    TC back = TC(0);
                    if (xw || yw) back = ld(p0 + ((code & 4) ? -rev : rev), ocb);
                    const int sxi = cneg ? 1 : 0, syi = sneg ? 1 : 0;
                    const int ysrc = wrap_idx(sneg ? ty + 1 : ty - 1, P.ny, P.bcy);
                    if (xo) r[1] = xw ? back : edge_x(sxi, v, ty);
                    if (yo) r[2] = yw ? back : edge_y(syi, v, xc);
                    r[3] = (xw || yw) ? back : (xo ? edge_x(sxi, v, ysrc) : edge_y(syi, v, (int)(osb / ES)));
                }
            }
        }
    };
    auto bilin = [&](int v, const TC* r) __attribute__((always_inline)) -> TC {
        CSRec& R = srec[v];
        return R.w[0] * r[0] + R.w[1] * r[1] + R.w[2] * r[2] + R.w[3] * r[3];
    };

    // 1. stream and accumulate moments, LB velocities' loads in flight at once
    TC fs[VPT];
    TC m[NMOM];
    double md[NMOM];
#pragma unroll
    for (int j = 0; j < NMOM; ++j) {
        m[j] = TC(0);
        md[j] = 0.0;
    }
    auto phase1 = [&](auto fast) __attribute__((always_inline)) {
#pragma unroll
        for (int kb = 0; kb < VPT / LB; ++kb) {
            if (kb < nbatch) {
                TC raw[LB][4];
                // the batch's upwind signs in one scalar load (the streaming
                // records are needed only for the arithmetic that follows)
                const unsigned long long sg =
                    *(const RLBM_CONST_AS unsigned long long*)((const RLBM_CONST_AS unsigned char*)P.sgn + v0 + kb * LB);
#pragma unroll
                for (int b = 0; b < LB; ++b)
                    load4(fast, v0 + kb * LB + b, (unsigned)(sg >> (8 * b)) & 7u, rnext(v0 + kb * LB + b), raw[b]);
                // FP32: each batch's 8-term sums start from zero and are
                // carried into FP64 accumulators (FP32 rounds only within
                // a batch); FP64 accumulates directly
                TC mb[NMOM];
#pragma unroll
                for (int j = 0; j < NMOM; ++j) mb[j] = sizeof(TC) == 4 ? TC(0) : m[j];
#pragma unroll
                for (int b = 0; b < LB; ++b) {
                    const int v = v0 + kb * LB + b;
                    const TC f = bilin(v, raw[b]);
                    fs[kb * LB + b] = f;
                    CSRec& R = srec[v];
#pragma unroll
                    for (int j = 0; j < NMOM; ++j) mb[j] += R.P[j] * f;
                }
#pragma unroll
                for (int j = 0; j < NMOM; ++j) {
                    if constexpr (sizeof(TC) == 4)
                        md[j] += (double)mb[j];
                    else
                        m[j] = mb[j];
                }
            }
        }
        for (int v = v0 + VPT; v < v0 + P.chunk; ++v) {
            TC r[4];
            load4(fast, v, ((const RLBM_CONST_AS unsigned char*)P.sgn)[v], inb + rplane(v), r);
            const TC f = bilin(v, r);
            CSRec& R = srec[v];
#pragma unroll
            for (int j = 0; j < NMOM; ++j) m[j] += R.P[j] * f;
        }
    };
    if (interior)
        phase1(std::true_type{});
    else
        phase1(std::false_type{});

    // 2. cross-wave reduction in FP64 and Landau frame
#pragma unroll
    for (int j = 0; j < NMOM; ++j) part[(w * NMOM + j) * 64 + lane] = md[j] + (double)m[j];
    __syncthreads();
    double mom[9];
#pragma unroll
    for (int j = 0; j < NMOM; ++j) {
        double s = 0.0;
        for (int u = 0; u < NW; ++u) s += part[(u * NMOM + j) * 64 + lane];
        mom[j] = s;
    }
    if (NMOM == 8) mom[8] = mom[3] - mom[6];
    Frame fr = landau_frame(mom);
    // Fermi-Dirac / Bose-Einstein: temperature and moment factors of the
    // frame (no equilibrium of that statistics counts as non-physical)
    double phi[NM + 1];
    if (GEN && P.stat != RLBM_STAT_MJ && fr.ok) {
        double Tq = 0.0;
        if (qs_frame(fr.n, fr.eps, P.stat, NM, P.ztab, &Tq, phi)) fr.ok = 0;
        fr.T = Tq;
    }
    const double* phip = (GEN && P.stat != RLBM_STAT_MJ) ? phi : nullptr;
    if (!fr.ok && active) atomicOr(P.flag, 1);
    // a site without a physical frame is streamed without collision (its
    // frame may hold NaN, so the rates are zeroed rather than scaled)
    const TC a0 = fr.ok ? (TC)(P.rate * fr.U0) : TC(0);
    const TC ax = fr.ok ? (TC)(P.rate * fr.Ux) : TC(0);
    const TC ay = fr.ok ? (TC)(P.rate * fr.Uy) : TC(0);

    // 3. equilibrium coefficients per shell, shells dealt to waves
    for (int i = w; i < P.Np; i += NW) {
        TC* ci = coef + i * NT * 64 + lane;
        // the frame as opaque values: the shell-independent FP64 factors
        // are then not hoisted out of the shell loop and held (register
        // spills at order 7 otherwise)
        double sn = fr.n, sT = fr.T, sU0 = fr.U0, sUx = fr.Ux, sUy = fr.Uy;
        asm volatile("" : "+v"(sn), "+v"(sT), "+v"(sU0), "+v"(sUx), "+v"(sUy));
        shell_coeffs<NM>(Gtab + (size_t)i * GS, Pc, sn, sT, sU0, sUx, sUy,
                         [&](int mm, double cm, double sm) __attribute__((always_inline)) {
                             if (!fr.ok) cm = sm = 0.0;
                             if (mm == 0) {
                                 ci[0] = (TC)cm;
                             } else {
                                 ci[(2 * mm - 1) * 64] = (TC)cm;
                                 ci[(2 * mm) * 64] = (TC)sm;
                             }
                         },
                         phip);
    }
    __syncthreads();

    // 4. equilibrium, relaxation, store (null table entries write the spare plane)
    int shell = crec[v0].shell;
    TC cc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) cc[t] = coef[(shell * NT + t) * 64 + lane];
    char* wcur = outb + (long long)v0 * pbytes;
    char* const wspare = outb + wplane(P.nvel);
    auto wnext = [&](int v) __attribute__((always_inline)) -> char* {
        char* p = v < P.nvel ? wcur : wspare;
        wcur += pbytes;
        return p;
    };
    auto collide = [&](auto fast, int v, char* wbase, TC f) __attribute__((always_inline)) {
        CCRec& R = crec[v];
        if (R.shell != shell) {
            shell = R.shell;
#pragma unroll
            for (int t = 0; t < NT; ++t) cc[t] = coef[(shell * NT + t) * 64 + lane];
        }
        TC feq = cc[0] * R.H[0];
#pragma unroll
        for (int t = 1; t < NT; ++t) feq += cc[t] * R.H[t];
        const TC om_ = a0 - ax * R.cth - ay * R.sth;
        const TC fn = f + om_ * (feq - f);
        TS* dst = reinterpret_cast<TS*>(wbase + ocb);
        // non-temporal: the next read of this plane is a step away
        if (decltype(fast)::value || active) __builtin_nontemporal_store((TS)fn, dst);
    };
    auto phase4 = [&](auto fast) __attribute__((always_inline)) {
#pragma unroll
        for (int kb = 0; kb < VPT / LB; ++kb) {
            if (kb < nbatch) {
                // the next batch's collision records: one word of each
                // scalar-cache line now, taken in only after this batch (the
                // records of the work-group's velocities do not all stay
                // cached between the phases)
                const unsigned pf = touch_lines<LB * (int)sizeof(CRec<TC, NM>)>(
                    (const RLBM_CONST_AS char*)(crec + min(v0 + (kb + 1) * LB, P.nvel + RLBM_VPAD - LB)));
#pragma unroll
                for (int b = 0; b < LB; ++b) collide(fast, v0 + kb * LB + b, wnext(v0 + kb * LB + b), fs[kb * LB + b]);
                asm volatile("" ::"s"(pf));
            }
        }
        for (int v = v0 + VPT; v < v0 + P.chunk; ++v) {
            TC r[4];
            load4(fast, v, ((const RLBM_CONST_AS unsigned char*)P.sgn)[v], inb + rplane(v), r);
            collide(fast, v, outb + wplane(v), bilin(v, r));
        }
    };
    if (interior)
        phase4(std::true_type{});
    else
        phase4(std::false_type{});
}

// GEN: the general instance, with the boundary loads of WALL and FIXED axes
// and the Fermi-Dirac / Bose-Einstein equilibria (a separate instance, so
// that the others keep their register budget).
template <typename TS, typename TC, int NM, int VPT, bool GEN>
__global__ __launch_bounds__(1024) void k_stream_collide(const TS* __restrict__ fin, TS* __restrict__ fout,
                                                         const SRec<TC>* __restrict__ srec,
                                                         const CRec<TC, NM>* __restrict__ crec,
                                                         const double* __restrict__ Gtab,
                                                         const double* __restrict__ Pc, SCParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sc_tile<TS, TC, NM, VPT, GEN>(fin, fout, srec, crec, Gtab, Pc, P, xcd_remap(blockIdx.x, gridDim.x), smem);
}

// Batched form: many independent problems advance one step in one
// persistent launch.  The (problem, tile) items are split into 8 contiguous
// ranges, one per XCD; a work-group takes items from its own XCD's range
// through an atomic counter (neighbouring rows stay in that XCD's L2) and,
// once it is drained, from the other ranges in turn.  Every work-group leaves
// when all ranges are drained; the last one to leave (counted in
// counters[8 * 16]) sets the 9 counters back to zero for the next launch, so
// a step is this one launch.
template <typename TS, typename TC, int NM, int VPT>
__global__ __launch_bounds__(1024) void k_batch_step(const BatchDesc* __restrict__ descs, int nprob,
                                                     int* __restrict__ counters, const int* __restrict__ bounds,
                                                     int parity, const double* __restrict__ Pc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int item_sh;
    const int home = blockIdx.x & 7;
    for (int q = 0; q < 8; ++q) {
        const int part = (home + q) & 7;
        const int end = bounds[part + 1];
        for (;;) {
            if (threadIdx.x == 0) item_sh = bounds[part] + atomicAdd(&counters[part * 16], 1);
            __syncthreads();
            const int item = __builtin_amdgcn_readfirstlane(item_sh);
            __syncthreads();
            if (item >= end) break;
            int p = 0;   // problem owning the item: items of a problem are contiguous
            int step = 1;
            while (step * 2 <= nprob) step *= 2;
            for (; step > 0; step >>= 1)
                if (p + step < nprob && ((const RLBM_CONST_AS BatchDesc*)descs)[p + step].item0 <= item)
                    p += step;
            // the descriptors are read through the constant address space
            // (scalar loads): they are not written during the kernel
            using CDesc = const RLBM_CONST_AS BatchDesc;
            CDesc& D = ((CDesc*)descs)[p];
            const SCParams P = D.P;
            sc_tile<TS, TC, NM, VPT>(static_cast<const TS*>(D.f[parity]), static_cast<TS*>(D.f[parity ^ 1]),
                                     static_cast<const SRec<TC>*>(P.srec), static_cast<const CRec<TC, NM>*>(P.crec),
                                     P.G, Pc, P, item - D.item0, smem);
            __syncthreads();
        }
    }
    // Every atomic this work-group makes on the range counters has returned
    // before its exit is counted, so the last work-group out sees them all.
    if (threadIdx.x == 0 && atomicAdd(&counters[8 * 16], 1) == (int)gridDim.x - 1)
        for (int k = 0; k <= 8; ++k) atomicExch(&counters[k * 16], 0);
}

// Batched form, flat launch: one work-group per (problem, tile) item, no work
// queue; the hardware dispatcher balances the items.
template <typename TS, typename TC, int NM, int VPT>
__global__ __launch_bounds__(1024) void k_batch_flat(const BatchDesc* __restrict__ descs, int nprob, int parity,
                                                     const double* __restrict__ Pc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    using CDesc = const RLBM_CONST_AS BatchDesc;
    int p = 0;   // problem owning the item: items of a problem are contiguous
    int step = 1;
    while (step * 2 <= nprob) step *= 2;
    for (; step > 0; step >>= 1)
        if (p + step < nprob && ((CDesc*)descs)[p + step].item0 <= item) p += step;
    CDesc& D = ((CDesc*)descs)[p];
    const SCParams P = D.P;
    sc_tile<TS, TC, NM, VPT>(static_cast<const TS*>(D.f[parity]), static_cast<TS*>(D.f[parity ^ 1]),
                             static_cast<const SRec<TC>*>(P.srec), static_cast<const CRec<TC, NM>*>(P.crec), P.G, Pc,
                             P, item - D.item0, smem);
}

// Initial populations: the truncated equilibrium of given fields, one thread
// per site.  fields = [n | T | U^x | U^y], each S doubles.
template <typename TS, int NM>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ fields, TS* __restrict__ f,
                                              const VelRec<double>* __restrict__ vel, const double* __restrict__ G,
                                              const double* __restrict__ Pc, long long S, int K, int Np, int stat,
                                              const double* __restrict__ ztab)
{
    constexpr int NT = 2 * NM + 1;
    constexpr int GS = (RLBM_NMAX + 1) * (RLBM_NMAX + 1);
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double n = fields[s], T = fields[S + s], ux = fields[2 * S + s], uy = fields[3 * S + s];
    const double U0 = sqrt(1.0 + ux * ux + uy * uy);
    // quantum statistics: moment factors of (n, T) (the host has checked
    // that an equilibrium exists)
    double phi[NM + 1];
    if (stat != RLBM_STAT_MJ) (void)qs_phi_of_nT(n, T, stat, NM, ztab, phi);
    const double* phip = stat != RLBM_STAT_MJ ? phi : nullptr;
    for (int i = 0; i < Np; ++i) {
        double c[NT];
        shell_coeffs<NM>(G + (size_t)i * GS, Pc, n, T, U0, ux, uy, [&](int m, double cm, double sm) {
            if (m == 0) {
                c[0] = cm;
            } else {
                c[2 * m - 1] = cm;
                c[2 * m] = sm;
            }
        }, phip);
        for (int j = 0; j < K; ++j) {
            const int v = i * K + j;
            double fe = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) fe += c[t] * vel[v].H[t];
            f[(long long)v * S + s] = (TS)fe;
        }
    }
}

// Macroscopic fields of the stored populations (FP64 moments and Landau
// frame), one thread per site, plus per-block partial charges.
template <typename TS>
__global__ __launch_bounds__(256) void k_fields(const TS* __restrict__ f, const VelRec<double>* __restrict__ vel,
                                                double* __restrict__ out, double* __restrict__ partials,
                                                int* flag, long long S, int nvel)
{
    __shared__ double red[4][256];
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (s < S) {
        for (int v = 0; v < nvel; ++v) {
            const double fv = (double)f[(long long)v * S + s];
#pragma unroll
            for (int j = 0; j < 9; ++j) m[j] += vel[v].P[j] * fv;
        }
        const Frame fr = landau_frame(m);
        const double nan = __builtin_nan("");
        out[s] = fr.ok ? fr.n : nan;
        out[S + s] = fr.ok ? fr.eps : nan;
        out[2 * S + s] = fr.ok ? fr.Ux : nan;
        out[3 * S + s] = fr.ok ? fr.Uy : nan;
        if (!fr.ok) atomicOr(flag, 1);
    }
    red[0][threadIdx.x] = m[0];
    red[1][threadIdx.x] = m[3];
    red[2][threadIdx.x] = m[4];
    red[3][threadIdx.x] = m[5];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[(size_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

template <typename TS, typename TC, int NM, int VPT, bool GEN>
hipError_t launch_sc_b(int waves, const SCParams& p, hipStream_t st)
{
    constexpr int NT = 2 * NM + 1;
    constexpr int NMOM = sizeof(TC) == 8 ? 9 : 8;
    const size_t lds = (size_t)waves * NMOM * 64 * sizeof(double) + (size_t)p.Np * NT * 64 * sizeof(TC);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    static size_t configured = 0;
    if (lds > 64 * 1024 && lds > configured) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stream_collide<TS, TC, NM, VPT, GEN>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        configured = lds;
    }
    const long long tiles = (long long)((p.nx + 63) / 64) * p.ny;
    if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream_collide<TS, TC, NM, VPT, GEN>), dim3((unsigned)tiles), dim3(64 * waves), lds, st,
                       static_cast<const TS*>(p.fin), static_cast<TS*>(p.fout),
                       static_cast<const SRec<TC>*>(p.srec), static_cast<const CRec<TC, NM>*>(p.crec), p.G, p.Pc, p);
    return hipGetLastError();
}

template <typename TS, typename TC, int NM, int VPT>
hipError_t launch_sc_t(int waves, const SCParams& p, hipStream_t st)
{
    if (general_step(p.bcx, p.bcy, p.stat)) return launch_sc_b<TS, TC, NM, VPT, true>(waves, p, st);
    return launch_sc_b<TS, TC, NM, VPT, false>(waves, p, st);
}

// Held values per lane, by storage precision and order class: the register
// budget (128 VGPRs at 16 waves per work-group) is shared with the FP64
// coefficient evaluation, whose size grows with the order.
#define RLBM_VPT_F32_HI 48
#define RLBM_VPT_F32_LO 64
template <typename TC, int NM>
struct Vpt {
    static constexpr int value =
        sizeof(TC) == 8 ? (NM <= 3 ? 32 : 16) : (NM <= 3 ? RLBM_VPT_F32_LO : (NM <= 5 ? RLBM_VPT_F32_HI : 32));
};

// Values held per lane by the persistent batch kernel.
template <typename TC, int NM>
struct BVpt {
    static constexpr int value = Vpt<TC, NM>::value;
};

template <typename TS, typename TC>
hipError_t launch_sc_n(int nmax, int waves, const SCParams& p, hipStream_t st)
{
    switch (nmax) {
        case 3: return launch_sc_t<TS, TC, 3, Vpt<TC, 3>::value>(waves, p, st);
        case 5: return launch_sc_t<TS, TC, 5, Vpt<TC, 5>::value>(waves, p, st);
        case 7: return launch_sc_t<TS, TC, 7, Vpt<TC, 7>::value>(waves, p, st);
    }
    return hipErrorInvalidValue;
}

template <typename TS, typename TC, int NM, int VPT>
size_t batch_lds(int waves, int max_np)
{
    constexpr int NT = 2 * NM + 1;
    constexpr int NMOM = sizeof(TC) == 8 ? 9 : 8;
    return (size_t)waves * NMOM * 64 * sizeof(double) + (size_t)max_np * NT * 64 * sizeof(TC);
}

template <typename TS, typename TC, int NM, int VPT>
hipError_t launch_batch_t(int waves, int grid, const BatchDesc* descs, int nprob, int* counters, const int* bounds,
                          int parity, const double* Pc, int max_np, hipStream_t st)
{
    // the large-LDS attribute is set by batch_grid_t, before any graph capture
    const size_t lds = batch_lds<TS, TC, NM, VPT>(waves, max_np);
    if (lds > 160 * 1024 - 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_batch_step<TS, TC, NM, VPT>), dim3(grid), dim3(64 * waves), lds, st, descs, nprob,
                       counters, bounds, parity, Pc);
    return hipGetLastError();
}

template <typename TS, typename TC, int NM, int VPT>
hipError_t launch_batch_flat_t(int waves, int items, const BatchDesc* descs, int nprob, int parity,
                               const double* Pc, int max_np, hipStream_t st)
{
    const size_t lds = batch_lds<TS, TC, NM, VPT>(waves, max_np);
    if (lds > 160 * 1024 - 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_batch_flat<TS, TC, NM, VPT>), dim3(items), dim3(64 * waves), lds, st, descs, nprob, parity,
                       Pc);
    return hipGetLastError();
}

// Resident work-groups for a persistent launch: occupancy per CU times CUs.
template <typename TS, typename TC, int NM, int VPT>
int batch_grid_t(int waves, int max_np)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const size_t lds = batch_lds<TS, TC, NM, VPT>(waves, max_np);
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_step<TS, TC, NM, VPT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_flat<TS, TC, NM, VPT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_batch_step<TS, TC, NM, VPT>),
                                                     64 * waves, lds) != hipSuccess)
        return 0;
    return per * cus;
}

template <typename TS>
hipError_t launch_init_t(int nmax, const double* fields, void* f, const VelRec<double>* vel, const double* G,
                         const double* Pc, long long S, int K, int Np, int stat, const double* ztab, hipStream_t st)
{
    const unsigned blocks = (unsigned)((S + 255) / 256);
    switch (nmax) {
        case 3: hipLaunchKernelGGL((k_init<TS, 3>), dim3(blocks), dim3(256), 0, st, fields, (TS*)f, vel, G, Pc, S, K, Np, stat, ztab); break;
        case 5: hipLaunchKernelGGL((k_init<TS, 5>), dim3(blocks), dim3(256), 0, st, fields, (TS*)f, vel, G, Pc, S, K, Np, stat, ztab); break;
        case 7: hipLaunchKernelGGL((k_init<TS, 7>), dim3(blocks), dim3(256), 0, st, fields, (TS*)f, vel, G, Pc, S, K, Np, stat, ztab); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int max_vpt(int prec, int nmax)
{
    if (prec == RLBM_F64) return nmax <= 3 ? Vpt<double, 3>::value : (nmax <= 5 ? Vpt<double, 5>::value : Vpt<double, 7>::value);
    return nmax <= 3 ? Vpt<float, 3>::value : (nmax <= 5 ? Vpt<float, 5>::value : Vpt<float, 7>::value);
}

int default_waves(int prec, int nmax, int nvel)
{
    const int vpt = max_vpt(prec, nmax);
    int w = (nvel + vpt - 1) / vpt;
    return w < 1 ? 1 : (w > 16 ? 16 : w);
}

int fields_blocks(long long S) { return (int)((S + 255) / 256); }

hipError_t launch_batch_step(int prec, int nmax, int waves, int grid, const BatchDesc* descs, int nprob,
                             int* counters, const int* bounds, int parity, const double* Pc, int max_np,
                             hipStream_t st)
{
    if (waves < 1 || waves > 16 || grid < 1) return hipErrorInvalidValue;
#define RLBM_BATCH_CASE(TS, TC, NM)                                                                            \
    return launch_batch_t<TS, TC, NM, BVpt<TC, NM>::value>(waves, grid, descs, nprob, counters, bounds, parity, Pc, \
                                                           max_np, st)
    if (prec == RLBM_F32) {
        if (nmax == 3) RLBM_BATCH_CASE(float, float, 3);
        if (nmax == 5) RLBM_BATCH_CASE(float, float, 5);
        if (nmax == 7) RLBM_BATCH_CASE(float, float, 7);
    } else if (prec == RLBM_F64) {
        if (nmax == 3) RLBM_BATCH_CASE(double, double, 3);
        if (nmax == 5) RLBM_BATCH_CASE(double, double, 5);
        if (nmax == 7) RLBM_BATCH_CASE(double, double, 7);
    }
#undef RLBM_BATCH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_batch_flat(int prec, int nmax, int waves, int items, const BatchDesc* descs, int nprob, int parity,
                             const double* Pc, int max_np, hipStream_t st)
{
    if (waves < 1 || waves > 16 || items < 1) return hipErrorInvalidValue;
#define RLBM_BATCH_CASE(TS, TC, NM) \
    return launch_batch_flat_t<TS, TC, NM, BVpt<TC, NM>::value>(waves, items, descs, nprob, parity, Pc, max_np, st)
    if (prec == RLBM_F32) {
        if (nmax == 3) RLBM_BATCH_CASE(float, float, 3);
        if (nmax == 5) RLBM_BATCH_CASE(float, float, 5);
        if (nmax == 7) RLBM_BATCH_CASE(float, float, 7);
    } else if (prec == RLBM_F64) {
        if (nmax == 3) RLBM_BATCH_CASE(double, double, 3);
        if (nmax == 5) RLBM_BATCH_CASE(double, double, 5);
        if (nmax == 7) RLBM_BATCH_CASE(double, double, 7);
    }
#undef RLBM_BATCH_CASE
    return hipErrorInvalidValue;
}

int batch_grid(int prec, int nmax, int waves, int max_np)
{
#define RLBM_GRID_CASE(TS, TC, NM) return batch_grid_t<TS, TC, NM, BVpt<TC, NM>::value>(waves, max_np)
    if (prec == RLBM_F32) {
        if (nmax == 3) RLBM_GRID_CASE(float, float, 3);
        if (nmax == 5) RLBM_GRID_CASE(float, float, 5);
        if (nmax == 7) RLBM_GRID_CASE(float, float, 7);
    } else if (prec == RLBM_F64) {
        if (nmax == 3) RLBM_GRID_CASE(double, double, 3);
        if (nmax == 5) RLBM_GRID_CASE(double, double, 5);
        if (nmax == 7) RLBM_GRID_CASE(double, double, 7);
    }
#undef RLBM_GRID_CASE
    return 0;
}

namespace {
// Initial populations of the edge cells, for FIXED boundaries:
// E[side][v][y] = f[v][y][side ? nx-1 : 0], then E[side][v][x] = f[v][side ? ny-1 : 0][x].
template <typename TS>
__global__ __launch_bounds__(256) void k_edges(const TS* __restrict__ f, TS* __restrict__ E, int nx, int ny, int nvel)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nxe = 2LL * nvel * ny, total = nxe + 2LL * nvel * nx;
    if (i >= total) return;
    const long long S = (long long)nx * ny;
    if (i < nxe) {
        const int y = (int)(i % ny);
        const long long sv = i / ny;
        const int v = (int)(sv % nvel), side = (int)(sv / nvel);
        E[i] = f[(long long)v * S + (long long)y * nx + (side ? nx - 1 : 0)];
    } else {
        const long long j = i - nxe;
        const int x = (int)(j % nx);
        const long long sv = j / nx;
        const int v = (int)(sv % nvel), side = (int)(sv / nvel);
        E[i] = f[(long long)v * S + (long long)(side ? ny - 1 : 0) * nx + x];
    }
}
}  // namespace

hipError_t launch_edges(int prec, const void* f, void* edges, int nx, int ny, int nvel, hipStream_t st)
{
    const long long total = 2LL * nvel * (nx + ny);
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (prec == RLBM_F64)
        hipLaunchKernelGGL((k_edges<double>), dim3(blocks), dim3(256), 0, st, (const double*)f, (double*)edges, nx, ny, nvel);
    else if (prec == RLBM_F32)
        hipLaunchKernelGGL((k_edges<float>), dim3(blocks), dim3(256), 0, st, (const float*)f, (float*)edges, nx, ny, nvel);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_init(int prec, int nmax, const double* fields, void* f, const VelRec<double>* vel, const double* G,
                       const double* Pc, int nx, int ny, int nvel, int K, int Np, int stat, const double* ztab,
                       hipStream_t st)
{
    (void)nvel;
    const long long S = (long long)nx * ny;
    if (prec == RLBM_F64) return launch_init_t<double>(nmax, fields, f, vel, G, Pc, S, K, Np, stat, ztab, st);
    if (prec == RLBM_F32) return launch_init_t<float>(nmax, fields, f, vel, G, Pc, S, K, Np, stat, ztab, st);
    return hipErrorInvalidValue;
}

hipError_t launch_stream_collide(int prec, int nmax, int waves, const SCParams& p, hipStream_t st)
{
    if (waves < 1 || waves > 16) return hipErrorInvalidValue;
    if (prec == RLBM_F64) return launch_sc_n<double, double>(nmax, waves, p, st);
    if (prec == RLBM_F32) return launch_sc_n<float, float>(nmax, waves, p, st);
    return hipErrorInvalidValue;
}

hipError_t launch_fields(int prec, const void* f, const VelRec<double>* vel, double* out, double* partials, int* flag,
                         int nx, int ny, int nvel, hipStream_t st)
{
    const long long S = (long long)nx * ny;
    const unsigned blocks = (unsigned)fields_blocks(S);
    if (prec == RLBM_F64)
        hipLaunchKernelGGL((k_fields<double>), dim3(blocks), dim3(256), 0, st, (const double*)f, vel, out, partials, flag, S, nvel);
    else if (prec == RLBM_F32)
        hipLaunchKernelGGL((k_fields<float>), dim3(blocks), dim3(256), 0, st, (const float*)f, vel, out, partials, flag, S, nvel);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch of rlbm_moments_device: the per-block partial charges
// of k_fields live in this array instead of the context's workspace, so that
// the call needs no memory beyond its inputs and outputs.  Each device holds
// its own copy; its address is taken once per device (scratch_setup, called
// by rlbm_init_fields with the device current) and kept in scratch_addr.
// ---------------------------------------------------------------------------
namespace {
constexpr int SCRATCH_BLOCKS = 65536;   // partial-charge blocks: grids up to 65536 x 256 sites
constexpr int SCRATCH_DEVICES = 64;
static __device__ __align__(256) double scratch[SCRATCH_BLOCKS * 4];
void* scratch_addr[SCRATCH_DEVICES];
std::mutex scratch_mu;

// Sum of nb per-block partial charges [nb][4] into out[4], in FP64, one
// work-group of 256 threads: a fixed strided order, then a tree.
__global__ __launch_bounds__(256) void k_charges_sum(const double* __restrict__ partials, int nb,
                                                     double* __restrict__ out)
{
    __shared__ double red[4][256];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int k = 0; k < 4; ++k) a[k] += partials[(size_t)b * 4 + k];
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}
}  // namespace

long long scratch_max_sites() { return (long long)SCRATCH_BLOCKS * 256; }

int scratch_setup(int dev)
{
    if (dev < 0 || dev >= SCRATCH_DEVICES) return RLBM_EDEVICE;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_addr[dev]) return RLBM_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RLBM_EDEVICE;
    scratch_addr[dev] = p;
    return RLBM_OK;
}

void* scratch_ptr(int dev)
{
    if (dev < 0 || dev >= SCRATCH_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    return scratch_addr[dev];
}

// Fields of f into out (device [4][S], may be the context's own buffer) and
// the charges into charges (device [4] or null), with the partial charges in
// `partials` (the scratch array's device address); no allocation, no
// synchronisation.
hipError_t launch_fields_charges(int prec, const void* f, const VelRec<double>* vel, double* out, double* partials,
                                 double* charges, int* flag, int nx, int ny, int nvel, hipStream_t st)
{
    hipError_t e = launch_fields(prec, f, vel, out, partials, flag, nx, ny, nvel, st);
    if (e != hipSuccess || !charges) return e;
    hipLaunchKernelGGL(k_charges_sum, dim3(1), dim3(256), 0, st, partials, fields_blocks((long long)nx * ny), charges);
    return hipGetLastError();
}

hipError_t launch_charges_sum(const double* partials, int nb, double* charges, hipStream_t st)
{
    hipLaunchKernelGGL(k_charges_sum, dim3(1), dim3(256), 0, st, partials, nb, charges);
    return hipGetLastError();
}

namespace {
__global__ void k_landau_probe(const double* __restrict__ mom, double* __restrict__ out, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double m[9];
    for (int j = 0; j < 9; ++j) m[j] = mom[9 * i + j];
    const Frame fr = landau_frame(m);
    out[7 * i + 0] = fr.n;
    out[7 * i + 1] = fr.eps;
    out[7 * i + 2] = fr.Ux;
    out[7 * i + 3] = fr.Uy;
    out[7 * i + 4] = fr.T;
    out[7 * i + 5] = fr.U0;
    out[7 * i + 6] = fr.ok;
}
}  // namespace

hipError_t launch_landau_probe(const double* mom, double* out, int count, hipStream_t st)
{
    hipLaunchKernelGGL(k_landau_probe, dim3((count + 63) / 64), dim3(64), 0, st, mom, out, count);
    return hipGetLastError();
}
