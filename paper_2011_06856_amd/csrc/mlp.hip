// mlp.hip -- the learned correction: a small MLP that maps a 3x3 patch of
// coarse-angle macroscopic fields to a correction of the traceless stress,
// with hand-written forward, backward and Adam kernels and the in-loop
// application to the populations.
//
// Network: in_dim -> hidden (x n_hidden, GELU) -> out_dim.  Forward uses
// weights rounded to bfloat16 and accumulates in FP32; the FP32 master
// weights are what Adam updates.  Parameters are one flat FP32 vector
// [W1 (h x in), b1, W2 (h x h), b2, ..., Wout (out x h), bout], W row-major
// [out][in].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "rlbm_internal.h"

namespace {

__device__ inline unsigned short f2bf(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (unsigned short)(u >> 16);
}

__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ inline float ld_w(const float* p, long i) { return p[i]; }
__device__ inline float ld_w(const unsigned short* p, long i) { return bf2f(p[i]); }

// C[M][N] (+)= op(A) op(B), FP32 accumulate.  A is [M][K] (TA = false) or
// [K][M] (TA = true); B is [K][N] (TB = false) or [N][K] (TB = true), of
// element type TBt (float or bfloat16 bits).
// On the matrix cores: 64x64 output tile per 256-thread
// work-group, one 32x32 quadrant per wave, v_mfma_f32_32x32x2f32 (FP32
// operands, FP32 accumulate; bfloat16 weights are widened exactly), K in
// steps of 16 staged through LDS.  Operand layout of the instruction: lane l
// supplies A[l % 32][k0 + l / 32] and B[k0 + l / 32][l % 32]; accumulator
// register r of lane l is C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
typedef float floatx16 __attribute__((ext_vector_type(16)));

// Split K: work-group z of the grid's third dimension takes k in
// [z kslice, (z + 1) kslice) and writes its partial product to C + z M N
// (kslice a multiple of 16; one slice: the whole K, C itself).
template <bool TA, bool TB, typename TBt>
__global__ __launch_bounds__(256) void k_gemm_mfma(const float* __restrict__ A, const TBt* __restrict__ B,
                                                   float* __restrict__ C, int M, int N, int K, int accumulate,
                                                   int kslice)
{
    __shared__ float As[16][64 + 4];
    __shared__ float Bs[16][64 + 4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int kb = blockIdx.z * kslice, ke = min(K, kb + kslice);
    C += (long)blockIdx.z * M * N;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int k0 = kb; k0 < ke; k0 += 16) {
        for (int e = tid; e < 16 * 64; e += 256) {
            const int kk = e / 64, mm = e % 64;
            const int gm = m0 + mm, gk = k0 + kk;
            float va = 0.f;
            if (gm < M && gk < ke) va = TA ? A[(long)gk * M + gm] : A[(long)gm * K + gk];
            As[kk][mm] = va;
            const int gn = n0 + mm;
            float vb = 0.f;
            if (gn < N && gk < ke) vb = TB ? ld_w(B, (long)gn * K + gk) : ld_w(B, (long)gk * N + gn);
            Bs[kk][mm] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 2) {
            const float a = As[kk + (lane >> 5)][wm + (lane & 31)];
            const float b = Bs[kk + (lane >> 5)][wn + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int gm = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int gn = n0 + wn + (lane & 31);
        if (gm < M && gn < N) {
            float* c = C + (long)gm * N + gn;
            *c = accumulate ? *c + acc[r] : acc[r];
        }
    }
}

// C[i] (+)= sum over the S slices of P[z][i], in slice order (deterministic).
__global__ void k_sum_slices(const float* __restrict__ P, float* __restrict__ C, int S, long mn, int accumulate)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mn) return;
    float s = accumulate ? C[i] : 0.f;
    for (int z = 0; z < S; ++z) s += P[(long)z * mn + i];
    C[i] = s;
}

__device__ inline float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }

// Inference in one pass: a work-group takes 64 rows through every layer of
// a 64 -> 128^nh -> out network (out <= 32), the activations staying in LDS.
// Per layer the work-group stages W^T in LDS (bfloat16), and wave w forms
// output columns 32w..32w+31 of both 32-row blocks with
// v_mfma_f32_32x32x2f32, k in the same order as k_gemm_mfma, then adds the
// bias and applies GELU exactly as k_bias_act: the outputs equal those of
// the layer-by-layer path bit for bit.  The last layer (one 32-column block,
// padded with zero weights) is formed by waves 0 and 1.
struct FusedNet {
    int nl, out;          // layers (hidden + output), outputs
    int woff[9], boff[9]; // offsets of W_l ([dout][din]) and b_l
};

__global__ __launch_bounds__(256) void k_mlp_fused(const float* __restrict__ X, const unsigned short* __restrict__ pbf,
                                                   const float* __restrict__ p, float* __restrict__ Y, int B, FusedNet net)
{
    __shared__ float act[64 * 128];            // [row][col ^ (row & 31)]: conflict-free column reads
    __shared__ unsigned short Ws[128 * 128];   // W^T of the current layer, [k][n]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long r0 = (long)blockIdx.x * 64;
    auto A = [&](int row, int col) -> float& { return act[row * 128 + (col ^ (row & 31))]; };
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e >> 6, k = e & 63;
        A(r, k) = r0 + r < B ? X[(r0 + r) * 64 + k] : 0.f;
    }
    for (int l = 0; l < net.nl; ++l) {
        const bool last = l == net.nl - 1;
        const int din = l == 0 ? 64 : 128, dout = last ? net.out : 128, ncols = last ? 32 : 128;
        const unsigned short* W = pbf + net.woff[l];
        // stage W^T: thread -> column n, 8 consecutive k per read
        for (int e = tid; e < ncols * (din / 8); e += 256) {
            const int n = e % ncols, kc = (e / ncols) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j) Ws[(kc + j) * 128 + n] = n < dout ? W[(long)n * din + kc + j] : 0;
        }
        __syncthreads();
        floatx16 acc0, acc1;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0.f;
        const int cb = last ? 0 : w;
        if (!last) {
            for (int k0 = 0; k0 < din; k0 += 2) {
                const int k = k0 + (lane >> 5);
                const float b = bf2f(Ws[k * 128 + cb * 32 + (lane & 31)]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(A(lane & 31, k), b, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(A(32 + (lane & 31), k), b, acc1, 0, 0, 0);
            }
        } else if (w < 2) {
            for (int k0 = 0; k0 < din; k0 += 2) {
                const int k = k0 + (lane >> 5);
                const float b = bf2f(Ws[k * 128 + (lane & 31)]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(A(w * 32 + (lane & 31), k), b, acc0, 0, 0, 0);
            }
        }
        __syncthreads();   // every read of this layer's inputs and weights is done
        const float* bias = p + net.boff[l];
        if (!last) {
            const int col = cb * 32 + (lane & 31);
            const float bc = bias[col];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                A(row, col) = gelu(acc0[r] + bc);
                A(32 + row, col) = gelu(acc1[r] + bc);
            }
            __syncthreads();
        } else if (w < 2) {
            const int col = lane & 31;
            if (col < dout) {
                const float bc = bias[col];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const long row = r0 + w * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    if (row < B) Y[row * dout + col] = acc0[r] + bc;
                }
            }
        }
    }
}
__device__ inline float gelu_d(float x)
{
    return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

// Z[r][c] += b[c]; A = GELU(Z) (or A = Z for the output layer).
__global__ void k_bias_act(float* __restrict__ Z, float* __restrict__ A, const float* __restrict__ b, long rows,
                           int cols, int act)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const float z = Z[i] + b[i % cols];
    Z[i] = z;
    if (A) A[i] = act ? gelu(z) : z;
}

// dZ = dA * GELU'(Z), in place on dA.
__global__ void k_gelu_bwd(float* __restrict__ dA, const float* __restrict__ Z, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dA[i] *= gelu_d(Z[i]);
}

// Loss 0.5/B * sum (Y - T)^2 over rows and outputs: dY = (Y - T) / B and
// per-block partial sums of the squared error.
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY, long n,
                      float inv_b, double* __restrict__ partial)
{
    __shared__ double red[256];
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (i < n) {
        const float d = Y[i] - T[i];
        dY[i] = d * inv_b;
        e2 = (double)d * d;
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// db[c] = sum_r dZ[r][c]: one work-group per column block, fixed order.
__global__ void k_colsum(const float* __restrict__ dZ, float* __restrict__ db, long rows, int cols)
{
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (long r = threadIdx.x; r < rows; r += 256) s += dZ[r * cols + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = red[0];
}

// Adam on the FP32 master parameters, then the bfloat16 copy of the weights.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, unsigned short* __restrict__ pbf, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float v = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    p[i] = v;
    pbf[i] = f2bf(v);
}

__global__ void k_to_bf16(const float* __restrict__ p, unsigned short* __restrict__ pbf, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pbf[i] = f2bf(p[i]);
}

// Per-site macroscopic fields of the populations: n, eps, U^x, U^y and the
// lab-frame traceless stress pi^ij = T^ij - (eps + P) U^i U^j - P delta^ij,
// P = eps / 2 (FP64 moments and Landau frame).  stats[s][8].
template <typename TS>
__global__ __launch_bounds__(256) void k_site_stats(const TS* __restrict__ f, const VelRec<double>* __restrict__ vel,
                                                    float* __restrict__ stats, long long S, int nvel)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int v = 0; v < nvel; ++v) {
        const double fv = (double)f[(long long)v * S + s];
#pragma unroll
        for (int j = 0; j < 9; ++j) m[j] += vel[v].P[j] * fv;
    }
    const Frame fr = landau_frame(m);
    float* o = stats + s * 8;
    if (!fr.ok) {
        for (int k = 0; k < 8; ++k) o[k] = 0.f;
        return;
    }
    const double P = 0.5 * fr.eps, w = fr.eps + P;
    o[0] = (float)fr.n;
    o[1] = (float)fr.eps;
    o[2] = (float)fr.Ux;
    o[3] = (float)fr.Uy;
    o[4] = (float)(m[6] - w * fr.Ux * fr.Ux - P);
    o[5] = (float)(m[7] - w * fr.Ux * fr.Uy);
    o[6] = (float)(m[8] - w * fr.Uy * fr.Uy - P);
    o[7] = 0.f;
}

// Network input of site s: the 7 fields of its 3x3 neighbourhood (periodic),
// neighbour j = (dy+1)*3 + (dx+1), field k at column 7j + k, normalised by
// (x - mu_k) / sigma_k; column 63 is zero.
__global__ void k_patch(const float* __restrict__ stats, float* __restrict__ X, int nx, int ny,
                        const float* __restrict__ mu, const float* __restrict__ sig, float extra)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (long)nx * ny) return;
    const int y = (int)(s / nx), x = (int)(s - (long)y * nx);
    float* o = X + s * 64;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int yy = (y + dy + ny) % ny, xx = (x + dx + nx) % nx;
            const float* st = stats + ((long)yy * nx + xx) * 8;
            const int j = (dy + 1) * 3 + (dx + 1);
            for (int k = 0; k < 7; ++k) o[7 * j + k] = (st[k] - mu[k]) / sig[k];
        }
    o[63] = extra;
}

// Readout correction of the FP64 fields f = [n | eps | U^x | U^y] (each S):
// with the de-normalised outputs y, n (1 + y0), eps (1 + y1), U^x + y2,
// U^y + y3.
__global__ void k_readout(double* __restrict__ f, const float* __restrict__ Y, const float* __restrict__ omu,
                          const float* __restrict__ osig, long S)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double y[4];
    for (int k = 0; k < 4; ++k) y[k] = (double)(Y[s * 4 + k] * osig[k] + omu[k]);
    f[s] *= 1.0 + y[0];
    f[S + s] *= 1.0 + y[1];
    f[2 * S + s] += y[2];
    f[3 * S + s] += y[3];
}

// In-loop correction: the network output (de-normalised) is a traceless
// stress (dTxx, dTxy, dTyy); its m = 2 part is put into the populations
// through the orthonormal basis function p^2 {cos, sin}(2 th) / sqrt(24 pi),
// which leaves N^mu, T^00 and T^0i unchanged:
//   f_v += w_v p_v^2 [(dTxx - dTyy) cos 2th_v + 2 dTxy sin 2th_v] / (24 pi).
// With `cur` (site statistics, stride 8, pi at columns 4..6) the output is a
// target stress and the change is scale * (output - current pi): a relaxation
// toward the target instead of an increment.
template <typename TS>
__global__ void k_apply_corr(TS* __restrict__ f, const float* __restrict__ Y, const float* __restrict__ omu,
                             const float* __restrict__ osig, const float* __restrict__ cur,
                             const double* __restrict__ wc, const double* __restrict__ ws, long long S, int nvel,
                             float scale)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const float* y = Y + s * 3;
    double dxx = omu ? omu[0] + osig[0] * y[0] : y[0];
    double dxy = omu ? omu[1] + osig[1] * y[1] : y[1];
    double dyy = omu ? omu[2] + osig[2] * y[2] : y[2];
    if (cur) {
        dxx -= cur[s * 8 + 4];
        dxy -= cur[s * 8 + 5];
        dyy -= cur[s * 8 + 6];
    }
    const double a = scale * (dxx - dyy) / (24.0 * M_PI), b = scale * 2.0 * dxy / (24.0 * M_PI);
    for (int v = 0; v < nvel; ++v) {
        TS* p = f + (long long)v * S + s;
        *p = (TS)((double)*p + a * wc[v] + b * ws[v]);
    }
}

// Angular resampling between two angle sets on the same radial shells: per
// shell, the angular harmonics |m| <= M of the source are evaluated at the
// destination angles,
//   f_dst[i, j] = sum_j' R[i][j][j'] f_src[i, j'],
//   R[i][j][j'] = (1 / K_dst) (1 + 2 sum_{m=1..M} cos m (th_dst,ij - th_src,ij')),
// which keeps every moment of angular order <= M (N^mu and T^munu among them).
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_resample(const TS* __restrict__ src, TD* __restrict__ dst,
                                                  const double* __restrict__ R, long long S, int Ks, int Kd)
{
    const long long s = (long long)blockIdx.y * blockDim.x + threadIdx.x;
    const int vd = blockIdx.x, i = vd / Kd;
    if (s >= S) return;
    const double* r = R + (long long)vd * Ks;
    const TS* f = src + (long long)i * Ks * S + s;
    double acc = 0.0;
    for (int js = 0; js < Ks; ++js) acc += r[js] * (double)f[(long long)js * S];
    dst[(long long)vd * S + s] = (TD)acc;
}

inline unsigned nblk(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

struct rlbm_mlp_s {
    int in = 64, hid = 128, nh = 3, out = 3, maxb = 0;
    long np = 0;
    std::vector<long> woff, boff;   // offsets of W_l and b_l in the flat vector
    std::vector<int> din, dout;
    hipStream_t st = nullptr;
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    unsigned short* pbf = nullptr;
    float* Z = nullptr;   // pre-activations of the hidden layers [nh][maxb][hid]
    float* A = nullptr;   // activations [nh][maxb][hid]
    float* Y = nullptr;   // outputs [maxb][out]
    float* dY = nullptr;  // [maxb][max(hid, out)]
    float* dH = nullptr;  // [maxb][hid]
    float* X = nullptr;   // features [maxb][in]
    float* stats = nullptr;
    double* partial = nullptr;
    float* norm = nullptr;   // in_mu[7], in_sig[7], out_mu[out], out_sig[out] (out <= 8)
    float* gpart = nullptr;  // split-K partial weight gradients [MLP_SLICES][max dout x din]
    float extra = 0.f;       // input column 63 (a per-run input, e.g. log10 Kn)
    int adam_t = 0;
    std::string err;
};

namespace {

int mfail(rlbm_mlp m, int code, const std::string& msg)
{
    if (m) m->err = msg;
    return code;
}

template <bool TA, bool TB, typename TBt>
hipError_t gemm(hipStream_t st, const float* A, const TBt* B, float* C, int M, int N, int K, int acc)
{
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TBt>), grid, dim3(256), 0, st, A, B, C, M, N, K, acc, K);
    return hipGetLastError();
}

// The weight gradients (a few 64 x 64 output tiles, K = the batch's rows):
// K split into up to MLP_SLICES slices of at least 64 rows, so that the grid
// fills the chip, then the slices summed in order.
constexpr int MLP_SLICES = 64;

hipError_t gemm_wgrad(hipStream_t st, float* part, const float* A, const float* B, float* C, int M, int N, int K)
{
    const int S = std::max(1, std::min(MLP_SLICES, K / 64));
    if (S == 1) return gemm<true, false, float>(st, A, B, C, M, N, K, 0);
    const int kslice = ((K + S - 1) / S + 15) / 16 * 16;
    const int Su = (K + kslice - 1) / kslice;   // slices actually used
    dim3 grid((N + 63) / 64, (M + 63) / 64, Su);
    hipLaunchKernelGGL((k_gemm_mfma<true, false, float>), grid, dim3(256), 0, st, A, B, part, M, N, K, 0, kslice);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long mn = (long)M * N;
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, part, C, Su, mn, 0);
    return hipGetLastError();
}

// Forward for B rows of X; keeps Z and A of the hidden layers for backward.
// Inference: the one-pass kernel where the shape allows it (input 64,
// hidden 128, at most 32 outputs); it gives the same outputs as the
// layer-by-layer path, which training uses (it keeps every layer's
// pre-activations for the backward pass).
hipError_t infer(rlbm_mlp m, const float* X, int B, float* Y);

hipError_t forward(rlbm_mlp m, const float* X, int B, float* Y)
{
    const int L = m->nh + 1;
    const float* in = X;
    for (int l = 0; l < L; ++l) {
        const bool last = l == L - 1;
        float* Z = last ? Y : m->Z + (size_t)l * m->maxb * m->hid;
        float* Aout = last ? nullptr : m->A + (size_t)l * m->maxb * m->hid;
        hipError_t e = gemm<false, true, unsigned short>(m->st, in, m->pbf + m->woff[l], Z, B, m->dout[l], m->din[l], 0);
        if (e != hipSuccess) return e;
        const long n = (long)B * m->dout[l];
        hipLaunchKernelGGL(k_bias_act, dim3(nblk(n)), dim3(256), 0, m->st, Z, Aout, m->p + m->boff[l], (long)B,
                           m->dout[l], last ? 0 : 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        in = Aout;
    }
    return hipSuccess;
}

hipError_t infer(rlbm_mlp m, const float* X, int B, float* Y)
{
    if (m->in != 64 || m->hid != 128 || m->out > 32 || m->nh + 1 > 9) return forward(m, X, B, Y);
    FusedNet net;
    net.nl = m->nh + 1;
    net.out = m->out;
    for (int l = 0; l < net.nl; ++l) {
        net.woff[l] = (int)m->woff[l];
        net.boff[l] = (int)m->boff[l];
    }
    hipLaunchKernelGGL(k_mlp_fused, dim3((unsigned)((B + 63) / 64)), dim3(256), 0, m->st, X, m->pbf, m->p, Y, B, net);
    return hipGetLastError();
}

}  // namespace

// f_v += w_v p_v^2 [(dTxx - dTyy) cos 2th_v + 2 dTxy sin 2th_v] / (24 pi) * scale,
// with Y de-normalised by (omu, osig) when they are given.
int add_stress(rlbm_ctx c, const float* Y, const float* omu, const float* osig, const float* cur, float scale)
{
    c->pvalid = 0;   // the push kernel's partial sums no longer match the populations
    if (!c->d_corr) {
        std::vector<double> t(2 * (size_t)c->q.nvel);
        for (int v = 0; v < c->q.nvel; ++v) {
            const double wp2 = c->q.w[v] * c->q.p[v] * c->q.p[v];
            t[v] = wp2 * std::cos(2.0 * c->q.theta[v]);
            t[c->q.nvel + v] = wp2 * std::sin(2.0 * c->q.theta[v]);
        }
        if (hipMalloc((void**)&c->d_corr, t.size() * 8) != hipSuccess) return RLBM_ENOMEM;
        if (hipMemcpy(c->d_corr, t.data(), t.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return RLBM_EDEVICE;
    }
    const unsigned nb = nblk(c->S);
    if (c->prec == RLBM_F64)
        hipLaunchKernelGGL((k_apply_corr<double>), dim3(nb), dim3(256), 0, c->st, (double*)c->f[c->cur], Y, omu, osig, cur,
                           c->d_corr, c->d_corr + c->q.nvel, c->S, c->q.nvel, scale);
    else if (c->prec == RLBM_F32)
        hipLaunchKernelGGL((k_apply_corr<float>), dim3(nb), dim3(256), 0, c->st, (float*)c->f[c->cur], Y, omu, osig, cur,
                           c->d_corr, c->d_corr + c->q.nvel, c->S, c->q.nvel, scale);
    else
        return RLBM_EINVAL;
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EDEVICE;
}

extern "C" {

int rlbm_mlp_create(rlbm_mlp* out, int in_dim, int hidden, int n_hidden, int out_dim, int max_batch, void* hip_stream)
{
    if (!out || in_dim < 1 || hidden < 1 || n_hidden < 1 || n_hidden > 8 || out_dim < 1 || max_batch < 1)
        return RLBM_EINVAL;
    *out = nullptr;
    rlbm_mlp m = new (std::nothrow) rlbm_mlp_s();
    if (!m) return RLBM_ENOMEM;
    m->in = in_dim; m->hid = hidden; m->nh = n_hidden; m->out = out_dim; m->maxb = max_batch;
    m->st = static_cast<hipStream_t>(hip_stream);
    long off = 0;
    for (int l = 0; l <= n_hidden; ++l) {
        const int di = l == 0 ? in_dim : hidden, dd = l == n_hidden ? out_dim : hidden;
        m->din.push_back(di);
        m->dout.push_back(dd);
        m->woff.push_back(off);
        off += (long)di * dd;
        m->boff.push_back(off);
        off += dd;
    }
    m->np = off;
    const size_t act = (size_t)n_hidden * max_batch * hidden;
    const int wide = hidden > out_dim ? hidden : out_dim;
    hipError_t e = hipSuccess;
    auto al = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    al((void**)&m->p, m->np * 4);
    al((void**)&m->g, m->np * 4);
    al((void**)&m->m1, m->np * 4);
    al((void**)&m->m2, m->np * 4);
    al((void**)&m->pbf, m->np * 2);
    al((void**)&m->Z, act * 4);
    al((void**)&m->A, act * 4);
    al((void**)&m->Y, (size_t)max_batch * out_dim * 4);
    al((void**)&m->dY, (size_t)max_batch * wide * 4);
    al((void**)&m->dH, (size_t)max_batch * hidden * 4);
    al((void**)&m->X, (size_t)max_batch * in_dim * 4);
    al((void**)&m->stats, (size_t)max_batch * 8 * 4);
    al((void**)&m->partial, (size_t)nblk((long)max_batch * (out_dim > 1 ? out_dim : 1)) * 8);
    al((void**)&m->norm, 64 * 4);
    {
        size_t mn = 0;
        for (int l = 0; l <= n_hidden; ++l) mn = std::max(mn, (size_t)m->din[l] * m->dout[l]);
        al((void**)&m->gpart, MLP_SLICES * mn * 4);
    }
    if (e == hipSuccess) e = hipMemset(m->m1, 0, m->np * 4);
    if (e == hipSuccess) e = hipMemset(m->m2, 0, m->np * 4);
    if (e == hipSuccess) e = hipMemset(m->p, 0, m->np * 4);
    if (e == hipSuccess) e = hipMemset(m->pbf, 0, m->np * 2);
    if (e == hipSuccess) {
        float nrm[64];
        for (int k = 0; k < 64; ++k) nrm[k] = (k >= 7 && k < 14) || k >= 17 ? 1.f : 0.f;
        e = hipMemcpy(m->norm, nrm, sizeof(nrm), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        rlbm_mlp_destroy(m);
        return RLBM_ENOMEM;
    }
    *out = m;
    return RLBM_OK;
}

long rlbm_mlp_nparams(rlbm_mlp m) { return m ? m->np : RLBM_EINVAL; }

int rlbm_mlp_set_params(rlbm_mlp m, const float* host)
{
    if (!m || !host) return RLBM_EINVAL;
    hipError_t e = hipMemcpy(m->p, host, m->np * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_to_bf16, dim3(nblk(m->np)), dim3(256), 0, m->st, m->p, m->pbf, m->np);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemset(m->m1, 0, m->np * 4);
    if (e == hipSuccess) e = hipMemset(m->m2, 0, m->np * 4);
    if (e == hipSuccess) e = hipStreamSynchronize(m->st);
    m->adam_t = 0;
    return e == hipSuccess ? RLBM_OK : mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
}

int rlbm_mlp_get_params(rlbm_mlp m, float* host)
{
    if (!m || !host) return RLBM_EINVAL;
    hipError_t e = hipStreamSynchronize(m->st);
    if (e == hipSuccess) e = hipMemcpy(host, m->p, m->np * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? RLBM_OK : mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
}

int rlbm_mlp_get_grad(rlbm_mlp m, float* host)
{
    if (!m || !host) return RLBM_EINVAL;
    hipError_t e = hipStreamSynchronize(m->st);
    if (e == hipSuccess) e = hipMemcpy(host, m->g, m->np * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? RLBM_OK : mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
}

int rlbm_mlp_set_norm(rlbm_mlp m, const float* in_mu, const float* in_sig, const float* out_mu, const float* out_sig)
{
    if (!m || !in_mu || !in_sig || !out_mu || !out_sig) return RLBM_EINVAL;
    float nrm[64] = {};
    for (int k = 0; k < 7; ++k) {
        if (!(in_sig[k] > 0)) return mfail(m, RLBM_EINVAL, "input scales must be positive");
        nrm[k] = in_mu[k];
        nrm[7 + k] = in_sig[k];
    }
    for (int k = 0; k < m->out && k < 8; ++k) {
        nrm[14 + k] = out_mu[k];
        nrm[14 + m->out + k] = out_sig[k];
    }
    hipError_t e = hipMemcpy(m->norm, nrm, sizeof(nrm), hipMemcpyHostToDevice);
    return e == hipSuccess ? RLBM_OK : mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
}

int rlbm_mlp_forward(rlbm_mlp m, const float* dX, int B, float* dY)
{
    if (!m || !dX || !dY || B < 1 || B > m->maxb) return RLBM_EINVAL;
    hipError_t e = infer(m, dX, B, dY);
    return e == hipSuccess ? RLBM_OK : mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
}

// Gradient of loss = 0.5/B sum (y - t)^2 w.r.t. the parameters (the
// bfloat16-rounded weights are the ones differentiated), into the internal
// gradient buffer; *loss receives the loss.
int rlbm_mlp_grad(rlbm_mlp m, const float* dX, const float* dT, int B, double* loss)
{
    if (!m || !dX || !dT || B < 1 || B > m->maxb) return RLBM_EINVAL;
    hipError_t e = forward(m, dX, B, m->Y);
    if (e != hipSuccess) return mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
    const long no = (long)B * m->out;
    const unsigned nb = nblk(no);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, m->st, m->Y, dT, m->dY, no, 1.f / B, m->partial);
    const int L = m->nh + 1;
    float* dcur = m->dY;   // gradient w.r.t. the pre-activation of layer l
    for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
        const float* in = l == 0 ? dX : m->A + (size_t)(l - 1) * m->maxb * m->hid;
        // dW_l = dZ^T in ; db_l = column sums of dZ
        e = gemm_wgrad(m->st, m->gpart, dcur, in, m->g + m->woff[l], m->dout[l], m->din[l], B);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_colsum, dim3(m->dout[l]), dim3(256), 0, m->st, dcur, m->g + m->boff[l], (long)B,
                           m->dout[l]);
        if (l == 0) break;
        // dA_{l-1} = dZ W_l (bf16 weights), then through GELU
        float* dnext = dcur == m->dY ? m->dH : m->dY;
        e = gemm<false, false, unsigned short>(m->st, dcur, m->pbf + m->woff[l], dnext, B, m->din[l], m->dout[l], 0);
        if (e != hipSuccess) break;
        const long nh = (long)B * m->din[l];
        hipLaunchKernelGGL(k_gelu_bwd, dim3(nblk(nh)), dim3(256), 0, m->st, dnext,
                           m->Z + (size_t)(l - 1) * m->maxb * m->hid, nh);
        e = hipGetLastError();
        dcur = dnext;
    }
    if (e != hipSuccess) return mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
    std::vector<double> part(nb);
    e = hipMemcpyAsync(part.data(), m->partial, nb * 8, hipMemcpyDeviceToHost, m->st);
    if (e == hipSuccess) e = hipStreamSynchronize(m->st);
    if (e != hipSuccess) return mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
    double s = 0.0;
    for (double v : part) s += v;
    if (loss) *loss = 0.5 * s / B;
    return RLBM_OK;
}

int rlbm_mlp_adam_step(rlbm_mlp m, float lr, float b1, float b2, float eps)
{
    if (!m || !(lr > 0)) return RLBM_EINVAL;
    ++m->adam_t;
    const float c1 = 1.f - powf(b1, (float)m->adam_t), c2 = 1.f - powf(b2, (float)m->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(nblk(m->np)), dim3(256), 0, m->st, m->p, m->g, m->m1, m->m2, m->pbf, m->np, lr,
                       b1, b2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RLBM_OK : mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
}

// Per-site fields and traceless stress of a context's current populations:
// device array [S][8] = n, eps, U^x, U^y, pi^xx, pi^xy, pi^yy, 0.
int rlbm_site_stats(rlbm_ctx c, float* dstats)
{
    if (!c || !dstats || !c->have_fields) return RLBM_EINVAL;
    const unsigned nb = nblk(c->S);
    if (c->prec == RLBM_F64)
        hipLaunchKernelGGL((k_site_stats<double>), dim3(nb), dim3(256), 0, c->st, (const double*)c->f[c->cur],
                           c->d_veld, dstats, c->S, c->q.nvel);
    else if (c->prec == RLBM_F32)
        hipLaunchKernelGGL((k_site_stats<float>), dim3(nb), dim3(256), 0, c->st, (const float*)c->f[c->cur],
                           c->d_veld, dstats, c->S, c->q.nvel);
    else
        return RLBM_EINVAL;
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EDEVICE;
}

// Normalised network inputs of every site of a context: device [S][64].
int rlbm_mlp_features(rlbm_ctx c, rlbm_mlp m, float* dX)
{
    if (!c || !m || !dX || !c->have_fields) return RLBM_EINVAL;
    if (c->S > m->maxb || m->in != 64) return mfail(m, RLBM_EINVAL, "grid larger than the network batch");
    int rc = rlbm_site_stats(c, m->stats);
    if (rc != RLBM_OK) return rc;
    hipLaunchKernelGGL(k_patch, dim3(nblk(c->S)), dim3(256), 0, c->st, m->stats, dX, c->nx, c->ny, m->norm,
                       m->norm + 7, m->extra);
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EDEVICE;
}

// In-loop correction of a context: features, forward pass, and the change of
// the traceless stress put into the populations (scaled by `scale`).  The
// context and the network must share one stream.
int rlbm_mlp_correct(rlbm_ctx c, rlbm_mlp m, float scale, int relax)
{
    if (!c || !m || !c->have_fields) return RLBM_EINVAL;
    if (m->out != 3) return mfail(m, RLBM_EINVAL, "the correction needs three outputs");
    int rc = rlbm_mlp_features(c, m, m->X);
    if (rc != RLBM_OK) return rc;
    if ((rc = rlbm_mlp_forward(m, m->X, (int)c->S, m->Y)) != RLBM_OK) return rc;
    // w p^2 cos 2th and w p^2 sin 2th per velocity, from the FP64 table
    return add_stress(c, m->Y, m->norm + 14, m->norm + 17, relax ? m->stats : nullptr, scale);
}

// The per-run input that the features carry in column 63.
int rlbm_mlp_set_extra(rlbm_mlp m, float extra)
{
    if (!m) return RLBM_EINVAL;
    m->extra = extra;
    return RLBM_OK;
}

// Readout correction of a context's fields: features with column 63 =
// `extra`, forward pass, the fields of the current populations corrected by
// the de-normalised outputs (k_readout), copied to the host.
int rlbm_mlp_readout(rlbm_ctx c, rlbm_mlp m, float extra, double* n, double* eps, double* ux, double* uy)
{
    if (!c || !m || !c->have_fields) return RLBM_EINVAL;
    if (m->out != 4) return mfail(m, RLBM_EINVAL, "the readout correction needs four outputs");
    m->extra = extra;
    int rc = rlbm_mlp_features(c, m, m->X);
    if (rc != RLBM_OK) return rc;
    if ((rc = rlbm_mlp_forward(m, m->X, (int)c->S, m->Y)) != RLBM_OK) return rc;
    hipError_t e = launch_fields(c->prec, c->f[c->cur], c->d_veld, c->d_fields, c->d_partials, c->d_flag, c->nx, c->ny,
                                 c->q.nvel, c->st);
    if (e != hipSuccess) return mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
    hipLaunchKernelGGL(k_readout, dim3(nblk(c->S)), dim3(256), 0, c->st, c->d_fields, m->Y, m->norm + 14,
                       m->norm + 18, (long)c->S);
    if ((e = hipGetLastError()) != hipSuccess) return mfail(m, RLBM_EDEVICE, hipGetErrorString(e));
    return fields_out(c, n, eps, ux, uy, nullptr);
}

// Add a change of the traceless stress, device [S][3] = (dT^xx, dT^xy,
// dT^yy), times scale, to a context's populations through the m = 2 basis
// function (as rlbm_mlp_correct does with the network output).
int rlbm_add_stress(rlbm_ctx c, const float* dstress, float scale)
{
    if (!c || !dstress || !c->have_fields) return RLBM_EINVAL;
    return add_stress(c, dstress, nullptr, nullptr, nullptr, scale);
}

const char* rlbm_mlp_last_error(rlbm_mlp m) { return m ? m->err.c_str() : "null network"; }

// Resample the populations of src onto dst's angle set (same grid, same
// radial shells), keeping the angular harmonics that both sets resolve.
int rlbm_resample(rlbm_ctx src, rlbm_ctx dst)
{
    if (!src || !dst || !src->have_fields || !dst->have_fields) return RLBM_EINVAL;
    if (src->nx != dst->nx || src->ny != dst->ny || src->q.Np != dst->q.Np || src->q.rotate != dst->q.rotate)
        return RLBM_EINVAL;
    if ((src->prec != RLBM_F32 && src->prec != RLBM_F64) || (dst->prec != RLBM_F32 && dst->prec != RLBM_F64))
        return RLBM_EINVAL;
    const int Np = src->q.Np, Ks = src->q.K, Kd = dst->q.K, M = (std::min(Ks, Kd) - 1) / 2;
    dst->pvalid = 0;
    std::vector<double> R((size_t)Np * Kd * Ks);
    for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Kd; ++j)
            for (int k = 0; k < Ks; ++k) {
                const double d = dst->q.theta[i * Kd + j] - src->q.theta[i * Ks + k];
                double acc = 1.0;
                for (int m = 1; m <= M; ++m) acc += 2.0 * std::cos(m * d);
                R[((size_t)i * Kd + j) * Ks + k] = acc / Kd;
            }
    double* dR = nullptr;
    if (hipMalloc((void**)&dR, R.size() * 8) != hipSuccess) return RLBM_ENOMEM;
    int rc = RLBM_OK;
    if (hipStreamSynchronize(src->st) != hipSuccess ||
        hipMemcpy(dR, R.data(), R.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        rc = RLBM_EDEVICE;
    if (rc == RLBM_OK) {
        const dim3 grid((unsigned)(Np * Kd), nblk(src->S));
        const bool s64 = src->prec == RLBM_F64, d64 = dst->prec == RLBM_F64;
        void* fs = src->f[src->cur];
        void* fd = dst->f[dst->cur];
        if (s64 && d64)
            hipLaunchKernelGGL((k_resample<double, double>), grid, dim3(256), 0, dst->st, (const double*)fs, (double*)fd, dR, src->S, Ks, Kd);
        else if (s64)
            hipLaunchKernelGGL((k_resample<double, float>), grid, dim3(256), 0, dst->st, (const double*)fs, (float*)fd, dR, src->S, Ks, Kd);
        else if (d64)
            hipLaunchKernelGGL((k_resample<float, double>), grid, dim3(256), 0, dst->st, (const float*)fs, (double*)fd, dR, src->S, Ks, Kd);
        else
            hipLaunchKernelGGL((k_resample<float, float>), grid, dim3(256), 0, dst->st, (const float*)fs, (float*)fd, dR, src->S, Ks, Kd);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(dst->st) != hipSuccess) rc = RLBM_EDEVICE;
    }
    (void)hipFree(dR);
    return rc;
}

int rlbm_mlp_destroy(rlbm_mlp m)
{
    if (!m) return RLBM_EINVAL;
    if (m->st) (void)hipStreamSynchronize(m->st);
    void* ps[] = {m->p,  m->g,  m->m1,    m->m2,      m->pbf,  m->Z,   m->A,    m->Y,
                  m->dY, m->dH, m->X, m->stats, m->partial, m->norm, m->gpart};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    delete m;
    return RLBM_OK;
}

}  // extern "C"
