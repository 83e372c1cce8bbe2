// access_pattern.hip -- the memory ceiling of the tile kernel's access
// pattern, without its arithmetic.
//
// Populations f[v][y][x] (FP32, 1024 x 1024 sites, 256 planes, 1.07 GB per
// buffer), as in the circular-shock workload.  Kernels, each moving the
// buffer once in and once out (2 x 1.07 GB):
//   copy      a plain float4 copy with non-temporal stores;
//   stream4w  the tile kernel's tiles (64 sites of a row, 4 waves splitting
//             the velocities), each velocity read at the site row and the
//             upwind row and written back at once;
//   stream8w  the same with 8 waves;
//   hold4w    as stream4w, but every wave holds its 64 velocities' values in
//             registers until a work-group reduction, then writes them: the
//             tile kernel's two phases.
// Prints milliseconds per launch and GB/s counted as 2 x buffer bytes.
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops access_pattern.hip
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                                                  \
    do {                                                                                                       \
        hipError_t e_ = (x);                                                                                   \
        if (e_ != hipSuccess) {                                                                                \
            std::printf("hip error %s at line %d\n", hipGetErrorString(e_), __LINE__);                        \
            std::exit(1);                                                                                      \
        }                                                                                                      \
    } while (0)

constexpr int NX = 1024, NY = 1024, NV = 256;
constexpr long long S = (long long)NX * NY;
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void k_copy(const v4f* __restrict__ a, v4f* __restrict__ b, long long n4)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n4; i += st) __builtin_nontemporal_store(a[i], &b[i]);
}

// tiles dealt to the XCDs in contiguous ranges, as in the tile kernel
__device__ __forceinline__ int remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, k = b & 7, j = b >> 3;
    return k * q + min(k, r) + j;
}

template <int WAVES>
__global__ __launch_bounds__(512) void k_stream(const float* __restrict__ f, float* __restrict__ g)
{
    const int tile = remap(blockIdx.x, gridDim.x);
    const int ty = tile / (NX / 64), tx = tile % (NX / 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = tx * 64 + lane;
    const int ym = ty == 0 ? NY - 1 : ty - 1;
    constexpr int chunk = NV / WAVES;
    for (int v = w * chunk; v < (w + 1) * chunk; v += 16) {
        float a[16], b[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            a[k] = f[(v + k) * S + (long long)ty * NX + x];
            b[k] = f[(v + k) * S + (long long)ym * NX + x];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k)
            __builtin_nontemporal_store(a[k] + 0.5f * b[k], &g[(v + k) * S + (long long)ty * NX + x]);
    }
}

__global__ __launch_bounds__(256) void k_hold(const float* __restrict__ f, float* __restrict__ g)
{
    const int tile = remap(blockIdx.x, gridDim.x);
    const int ty = tile / (NX / 64), tx = tile % (NX / 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = tx * 64 + lane;
    const int ym = ty == 0 ? NY - 1 : ty - 1;
    const int v0 = w * 64;
    float h[64];
    float m = 0.f;
#pragma unroll
    for (int k0 = 0; k0 < 64; k0 += 8) {
        float a[8], b[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = f[(v0 + k0 + k) * S + (long long)ty * NX + x];
            b[k] = f[(v0 + k0 + k) * S + (long long)ym * NX + x];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            h[k0 + k] = a[k] + 0.5f * b[k];
            m += h[k0 + k];
        }
    }
    __shared__ float red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    const float s = red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 64; ++k)
        __builtin_nontemporal_store(h[k] * 0.999f + 1e-9f * s, &g[(v0 + k) * S + (long long)ty * NX + x]);
}

int main()
{
    float *f, *g;
    const size_t bytes = (size_t)NV * S * sizeof(float);
    CK(hipMalloc(&f, bytes));
    CK(hipMalloc(&g, bytes));
    CK(hipMemset(f, 0, bytes));
    CK(hipMemset(g, 0, bytes));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const int tiles = (NX / 64) * NY;
    const char* name[] = {"copy", "stream4w", "stream8w", "hold4w"};
    for (int t = 0; t < 4; ++t)
        for (int rep = 0; rep < 2; ++rep) {
            CK(hipEventRecord(e0));
            for (int it = 0; it < 10; ++it) {
                if (t == 0)
                    hipLaunchKernelGGL(k_copy, dim3(256 * 32), dim3(256), 0, 0, (const v4f*)f, (v4f*)g,
                                       (long long)(bytes / 16));
                if (t == 1) hipLaunchKernelGGL(k_stream<4>, dim3(tiles), dim3(256), 0, 0, f, g);
                if (t == 2) hipLaunchKernelGGL(k_stream<8>, dim3(tiles), dim3(512), 0, 0, f, g);
                if (t == 3) hipLaunchKernelGGL(k_hold, dim3(tiles), dim3(256), 0, 0, f, g);
            }
            CK(hipGetLastError());
            CK(hipEventRecord(e1));
            CK(hipEventSynchronize(e1));
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            std::printf("%-9s %.3f ms/launch  %.0f GB/s\n", name[t], ms / 10, 2.0 * bytes / (ms / 10 * 1e-3) / 1e9);
        }
    CK(hipFree(f));
    CK(hipFree(g));
    return 0;
}
