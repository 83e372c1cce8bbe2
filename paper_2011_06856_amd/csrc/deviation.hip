// deviation.hip -- initial state and field output of the deviation storage
// (RLBM_BF16DEV, RLBM_F32DEV, RLBM_F64DEV).
//
// A site holds g_v = f_v - F_v, the departure of its populations from the
// truncated equilibrium F of its last collision (Eq.
// mj-feq-expansion-truncated), and F itself as per-shell harmonic
// coefficients C[i][t] (F_v = sum_t C[shell(v)][t] H_t(v), H_t = w_v {1,
// cos m th, sin m th}), planes [Np][2 NM + 1][S] next to the deviations.  The
// step (push.hip) streams g and the coefficients together; here:
//   - the initial state: C of the given fields, g = 0 (f = F exactly);
//   - the fields: the moments (Eq. discrete_sum_moments) of f = g + F as
//     sum_v g_v P(v) + sum_{i,t} C[i][t] Z[i][t], Z[i][t] = sum over shell i of
//     H_t P, in FP64, then the Landau frame.
#include <cmath>
#include <cstring>
#include <vector>

#include "rlbm_internal.h"

namespace {

template <typename T, typename ST>
__device__ __forceinline__ double dev_load(const ST* p) { return (double)*p; }
template <>
__device__ __forceinline__ double dev_load<float, unsigned short>(const unsigned short* p)
{
    return (double)__uint_as_float((unsigned)*p << 16);
}

// Coefficients of the initial equilibrium, one thread per site.
template <typename CT, int NM>
__global__ __launch_bounds__(256) void k_dev_init(const double* __restrict__ fields, CT* __restrict__ cf,
                                                  const double* __restrict__ G, const double* __restrict__ Pc,
                                                  long long S, int Np)
{
    constexpr int NT = 2 * NM + 1;
    constexpr int GS = (RLBM_NMAX + 1) * (RLBM_NMAX + 1);
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double n = fields[s], T = fields[S + s], ux = fields[2 * S + s], uy = fields[3 * S + s];
    const double U0 = sqrt(1.0 + ux * ux + uy * uy);
    for (int i = 0; i < Np; ++i)
        shell_coeffs<NM>(G + (size_t)i * GS, Pc, n, T, U0, ux, uy, [&](int m, double cm, double sm) {
            if (m == 0) {
                cf[(long long)(i * NT) * S + s] = (CT)cm;
            } else {
                cf[(long long)(i * NT + 2 * m - 1) * S + s] = (CT)cm;
                cf[(long long)(i * NT + 2 * m) * S + s] = (CT)sm;
            }
        });
}

// Fields of the stored state (FP64 moments and Landau frame), one thread per
// site, plus per-block partial charges (as k_fields).
template <typename T, typename ST, int NM>
__global__ __launch_bounds__(256) void k_dev_fields(const ST* __restrict__ g, const T* __restrict__ cf,
                                                    const VelRec<double>* __restrict__ vel,
                                                    const double* __restrict__ Z, double* __restrict__ out,
                                                    double* __restrict__ partials, int* flag, long long S, int nvel,
                                                    int Np)
{
    constexpr int NT = 2 * NM + 1;
    __shared__ double red[4][256];
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (s < S) {
        for (int v = 0; v < nvel; ++v) {
            const double gv = dev_load<T, ST>(g + (long long)v * S + s);
#pragma unroll
            for (int j = 0; j < 9; ++j) m[j] += vel[v].P[j] * gv;
        }
        for (int i = 0; i < Np; ++i)
            for (int t = 0; t < NT; ++t) {
                const double c = (double)cf[(long long)(i * NT + t) * S + s];
#pragma unroll
                for (int j = 0; j < 9; ++j) m[j] += c * Z[(i * NT + t) * 9 + j];
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

template <typename CT>
hipError_t dev_init_t(rlbm_ctx c, hipStream_t st)
{
    const unsigned blocks = (unsigned)((c->S + 255) / 256);
    CT* cf = static_cast<CT*>(c->cf[c->cur]);
    switch (nmax_of(c->q.N)) {
        case 3: hipLaunchKernelGGL((k_dev_init<CT, 3>), dim3(blocks), dim3(256), 0, st, c->d_fields, cf, c->d_G, c->d_Pc, c->S, c->q.Np); break;
        case 5: hipLaunchKernelGGL((k_dev_init<CT, 5>), dim3(blocks), dim3(256), 0, st, c->d_fields, cf, c->d_G, c->d_Pc, c->S, c->q.Np); break;
        default: hipLaunchKernelGGL((k_dev_init<CT, 7>), dim3(blocks), dim3(256), 0, st, c->d_fields, cf, c->d_G, c->d_Pc, c->S, c->q.Np); break;
    }
    return hipGetLastError();
}

template <typename T, typename ST>
hipError_t dev_fields_t(rlbm_ctx c, double* out, double* partials, hipStream_t st)
{
    const unsigned blocks = (unsigned)fields_blocks(c->S);
    const ST* g = static_cast<const ST*>(c->f[c->cur]);
    const T* cf = static_cast<const T*>(c->cf[c->cur]);
    switch (nmax_of(c->q.N)) {
        case 3: hipLaunchKernelGGL((k_dev_fields<T, ST, 3>), dim3(blocks), dim3(256), 0, st, g, cf, c->d_veld, c->d_dz, out, partials, c->d_flag, c->S, c->q.nvel, c->q.Np); break;
        case 5: hipLaunchKernelGGL((k_dev_fields<T, ST, 5>), dim3(blocks), dim3(256), 0, st, g, cf, c->d_veld, c->d_dz, out, partials, c->d_flag, c->S, c->q.nvel, c->q.Np); break;
        default: hipLaunchKernelGGL((k_dev_fields<T, ST, 7>), dim3(blocks), dim3(256), 0, st, g, cf, c->d_veld, c->d_dz, out, partials, c->d_flag, c->S, c->q.nvel, c->q.Np); break;
    }
    return hipGetLastError();
}

}  // namespace

// Z[i][t][k] = sum over shell i of H_t(v) P_k(v) (FP64), uploaded at
// rlbm_init_fields.
int dev_setup(rlbm_ctx c, std::string& err)
{
    const int Np = c->q.Np, K = c->q.K, NT = 2 * nmax_of(c->q.N) + 1;
    std::vector<VelRec<double>> vd;
    build_vel_table(c->q, c->dt, vd);
    std::vector<double> Z((size_t)Np * NT * 9, 0.0);
    for (int i = 0; i < Np; ++i)
        for (int j = 0; j < K; ++j) {
            const VelRec<double>& R = vd[(size_t)i * K + j];
            for (int t = 0; t < NT; ++t)
                for (int k = 0; k < 9; ++k) Z[((size_t)i * NT + t) * 9 + k] += R.H[t] * R.P[k];
        }
    hipError_t e;
    if ((e = hipMalloc((void**)&c->d_dz, Z.size() * sizeof(double))) != hipSuccess) {
        err = "deviation table alloc";
        return RLBM_ENOMEM;
    }
    if ((e = hipMemcpy(c->d_dz, Z.data(), Z.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) {
        err = hipGetErrorString(e);
        return RLBM_EDEVICE;
    }
    return RLBM_OK;
}

// Initial deviation state of the fields in d_fields: coefficients into
// cf[cur], zero deviations in f[cur] (all planes, the spare one included).
hipError_t launch_dev_init(rlbm_ctx c, hipStream_t st)
{
    const size_t gbytes = (size_t)(c->q.nvel + 1) * c->S * store_size(c->prec);
    hipError_t e = hipMemsetAsync(c->f[c->cur], 0, gbytes, st);
    if (e != hipSuccess) return e;
    if ((e = hipMemsetAsync(c->f[c->cur ^ 1], 0, gbytes, st)) != hipSuccess) return e;
    return c->prec == RLBM_F64DEV ? dev_init_t<double>(c, st) : dev_init_t<float>(c, st);
}

// Fields and per-block partial charges of the current deviation state.
hipError_t launch_dev_fields(rlbm_ctx c, double* out, double* partials, hipStream_t st)
{
    switch (c->prec) {
        case RLBM_BF16DEV: return dev_fields_t<float, unsigned short>(c, out, partials, st);
        case RLBM_F32DEV: return dev_fields_t<float, float>(c, out, partials, st);
        case RLBM_F64DEV: return dev_fields_t<double, double>(c, out, partials, st);
    }
    return hipErrorInvalidValue;
}
