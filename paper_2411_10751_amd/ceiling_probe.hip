// Memory ceilings of the step's access pattern on one GPU (measurement tool,
// not part of the library).  The collision kernel reads Q structure-of-arrays
// planes at shifted positions (the pull of Eq. 4.4) and writes Q planes; this
// program times kernels with that access pattern and no arithmetic:
//   copy4      plain float4 copy of 1 GiB (the device's streaming rate);
//   planes     39-plane copy out[i][c] = in[i][c] (aligned sources);
//   pull       39-plane pull copy out[i][c] = in[i][c - shift_i] with the
//              D3Q39 shifts on a 256^3 grid, 4-byte elements;
//   pull16     the same with 2-byte elements (the 16-bit storage);
// each as the best of three timings of 20 launches.  The cells updated are
// those whose every source lies in the grid, so every access is in bounds.
//
// Built by `python -m paper_2411_10751_amd.build` (build_probe) into
// paper_2411_10751_amd/ceiling_probe; run it with no arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

namespace {

constexpr int Q = 39;
__constant__ int c_shift[Q];
typedef float vec4 __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                                            \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                         \
            exit(1);                                                                        \
        }                                                                                   \
    } while (0)

__global__ void __launch_bounds__(256) k_copy4(const vec4* __restrict__ in, vec4* __restrict__ out, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(in[i], &out[i]);
}

// SHIFTED = false: every plane read at the cell itself
template <class T, bool SHIFTED>
__global__ void __launch_bounds__(256) k_pull(const T* __restrict__ in, T* __restrict__ out, long long N,
                                              long long lo, long long ncells)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= ncells) return;
    const long long c = lo + t;
    T v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = in[i * N + c - (SHIFTED ? c_shift[i] : 0)];
#pragma unroll
    for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(v[i], &out[i * N + c]);
}

template <class F>
float best_ms(F&& launch)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    launch();  // warm-up
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        CHECK(hipEventRecord(a));
        for (int it = 0; it < 20; ++it) launch();
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, a, b));
        best = std::min(best, ms / 20);
    }
    CHECK(hipGetLastError());
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return best;
}

}  // namespace

int main()
{
    // D3Q39 velocities: rest; (+-1,0,0) and permutations; (+-1,+-1,+-1);
    // (+-2,0,0) and permutations; (+-2,+-2,0) and permutations; (+-3,0,0) and
    // permutations
    int cx[Q], cy[Q], cz[Q], k = 0;
    auto add = [&](int a, int b, int c) { cx[k] = a; cy[k] = b; cz[k] = c; ++k; };
    add(0, 0, 0);
    for (int s : {1, 2, 3}) {
        add(s, 0, 0); add(-s, 0, 0); add(0, s, 0); add(0, -s, 0); add(0, 0, s); add(0, 0, -s);
    }
    for (int a : {1, -1})
        for (int b : {1, -1})
            for (int c : {1, -1}) add(a, b, c);
    for (int a : {2, -2})
        for (int b : {2, -2}) { add(a, b, 0); add(a, 0, b); add(0, a, b); }
    if (k != Q) {
        fprintf(stderr, "velocity set has %d entries\n", k);
        return 1;
    }
    const long long n = 256, N = n * n * n;
    int shift[Q], maxs = 0;
    for (int i = 0; i < Q; ++i) {
        shift[i] = (int)((cz[i] * n + cy[i]) * n + cx[i]);
        maxs = std::max(maxs, std::abs(shift[i]));
    }
    CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_shift), shift, sizeof shift));
    // cells [lo, lo + ncells): every source c - shift_i lies in [0, N)
    const long long lo = ((maxs + 255) / 256) * 256;
    const long long ncells = ((N - 2 * lo) / 256) * 256;
    if (lo - maxs < 0 || lo + ncells - 1 + maxs >= N) {
        fprintf(stderr, "cell range out of bounds\n");
        return 1;
    }
    const dim3 grid((unsigned)(ncells / 256)), block(256);

    char* in = nullptr;
    char* out = nullptr;
    const size_t bytes = (size_t)Q * N * 4;
    CHECK(hipMalloc(&in, bytes));
    CHECK(hipMalloc(&out, bytes));
    CHECK(hipMemset(in, 0, bytes));

    const long long n4 = (1ll << 30) / 16;  // 1 GiB of float4
    const float t_copy = best_ms([&] {
        hipLaunchKernelGGL(k_copy4, dim3((unsigned)(n4 / 256)), block, 0, 0, (const vec4*)in, (vec4*)out, n4);
    });
    printf("copy4:  %.4f ms, %.3f TB/s (1 GiB read, 1 GiB written)\n", t_copy, 2.0 * (1 << 30) / (t_copy * 1e-3) / 1e12);

    const double cells = (double)ncells;
    const float t_planes = best_ms([&] {
        hipLaunchKernelGGL((k_pull<float, false>), grid, block, 0, 0, (const float*)in, (float*)out, N, lo, ncells);
    });
    printf("planes: %.4f ms, %.3f TB/s (39 aligned planes, 4 B, %.0f cells)\n", t_planes,
           2.0 * Q * 4 * cells / (t_planes * 1e-3) / 1e12, cells);
    const float t_pull = best_ms([&] {
        hipLaunchKernelGGL((k_pull<float, true>), grid, block, 0, 0, (const float*)in, (float*)out, N, lo, ncells);
    });
    printf("pull:   %.4f ms, %.3f TB/s (39 shifted planes, 4 B, %.0f cells)\n", t_pull,
           2.0 * Q * 4 * cells / (t_pull * 1e-3) / 1e12, cells);
    const float t_pull16 = best_ms([&] {
        hipLaunchKernelGGL((k_pull<unsigned short, true>), grid, block, 0, 0, (const unsigned short*)in,
                           (unsigned short*)out, N, lo, ncells);
    });
    printf("pull16: %.4f ms, %.3f TB/s (39 shifted planes, 2 B, %.0f cells)\n", t_pull16,
           2.0 * Q * 2 * cells / (t_pull16 * 1e-3) / 1e12, cells);
    CHECK(hipFree(in));
    CHECK(hipFree(out));
    return 0;
}
