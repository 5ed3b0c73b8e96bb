// Traversal probe: plain copies that move the elements of a complex64
// transform of n = 2^24 exactly as the library's passes do -- same tiles, same
// thread layout, in the XCD-contiguous tile order and in the spread orders
// the library uses at this length -- with no arithmetic and no LDS work, to
// measure what each pass's access pattern costs by itself.  One JSON object
// per line on stdout: {"probe": ..., "us": ..., ...}.
//
//   pass 1  (two-level 4096 x 4096): 2-column tiles, 512 threads, thread
//           (c = tid % 2, j = tid / 2) reads rows j + 256 r (r < 16) of
//           column c, writes the scratch slab S[j1/2][k2][j1%2]; run with
//           extra dynamic LDS so that 4, 3, 2 or 1 workgroups share a CU
//   pass 2  4-row tiles, 1024 threads, (c = tid % 4, j = tid / 4) reads
//           S[k1/2][k2][k1%2] for k1 = j + 256 r, writes X[k2 + 4096 k1]
//   A, B, C (three-level 256 x 256 x 256): 16-line tiles of 256 points,
//           256 threads, (c = tid % 16, j = tid / 16), elements j + 16 r;
//           element (line (lm, ld), i) at (lm << s0) + (ld << s1) + (i << s2)
//   pass 1 with 4- and 8-column tiles (512 threads), for comparison, and
//           with each thread owning whole rows of the 2-column tile
//   copy    a contiguous 16-byte-per-lane copy of the same bytes
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#include <vector>

#define CHECK(x)                                                                           \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) {                                                            \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            exit(1);                                                                       \
        }                                                                                  \
    } while (0)

namespace {
constexpr int L2N = 24, P = 4096, Q = 4096;
constexpr int64_t N = int64_t(1) << L2N;

// XCD-contiguous order: workgroup g runs tile (g % 8) * (G / 8) + i, i = g / 8.
// With a spread (log2s > 0) the XCD's range of G / 8 tiles is cut into groups
// of 2^log2g tiles laid out as 2^log2s rows, and i walks them column by
// column (the library's tile orders).
__host__ __device__ inline int tile_of(int g, int G, int log2g = 0, int log2s = 0) {
    const int per = G >> 3, i = g >> 3;
    if (!log2s) return (g & 7) * per + i;
    const int grp = i >> log2g, cols = per >> (log2g + log2s);
    return (g & 7) * per + ((((grp & ((1 << log2s) - 1)) * cols + (grp >> log2s)) << log2g) | (i & ((1 << log2g) - 1)));
}
// Whether tile_of(., G, log2g, log2s) is a permutation of 0 .. G-1.
bool order_is_permutation(int G, int log2g, int log2s) {
    if (G % 8 || ((G >> 3) % (1 << (log2g + log2s)))) return false;
    std::vector<char> seen(G, 0);
    for (int g = 0; g < G; ++g) {
        const int t = tile_of(g, G, log2g, log2s);
        if (t < 0 || t >= G || seen[t]++) return false;
    }
    return true;
}

__global__ __launch_bounds__(512) void pass1_copy(const float2 *__restrict__ x, float2 *__restrict__ s, int lg,
                                                  int ls) {
    extern __shared__ float reserve[]; // only sized to set the occupancy
    const int t = tile_of(blockIdx.x, gridDim.x, lg, ls), c = threadIdx.x & 1, j = threadIdx.x >> 1;
    const int j1 = 2 * t + c;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = x[int64_t(j1) + int64_t(P) * (j + 256 * r)];
#pragma unroll
    for (int r = 0; r < 16; ++r) s[int64_t(j1 >> 1) * 2 * Q + 2 * (j + 256 * r) + (j1 & 1)] = v[r];
    (void)reserve;
}

// Pass 1's traversal with tiles of T columns (T = 4, 8; 512 threads, thread
// (c = tid % T, j = tid / T) reads rows j + (512 / T) r): what wider tiles
// would cost to move, for comparison with the 2-column tiles above.
template <int T>
__global__ __launch_bounds__(512) void pass1_wide_copy(const float2 *__restrict__ x, float2 *__restrict__ s, int lg,
                                                       int ls) {
    constexpr int R = 512 / T, E = Q / R;
    const int t = tile_of(blockIdx.x, gridDim.x, lg, ls), c = threadIdx.x % T, j = threadIdx.x / T;
    const int j1 = T * t + c;
    float2 v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = x[int64_t(j1) + int64_t(P) * (j + R * r)];
#pragma unroll
    for (int r = 0; r < E; ++r) s[int64_t(t) * T * Q + int64_t(T) * (j + R * r) + c] = v[r];
}

// Pass 1's traversal with each thread owning whole rows of the 2-column tile
// (the row-lane pass 1): thread j loads both columns of rows j + (N / E) r,
// one 16-byte load per row, and stores each slab row as two 8-byte halves.
template <int E>
__global__ __launch_bounds__(Q / E) void pass1_rows_copy(const float2 *__restrict__ x, float2 *__restrict__ s, int lg,
                                                       int ls) {
    constexpr int R = Q / E;
    const int t = tile_of(blockIdx.x, gridDim.x, lg, ls), j = threadIdx.x;
    const float4 *col = reinterpret_cast<const float4 *>(x + 2 * int64_t(t));
    float4 v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = col[int64_t(P / 2) * (j + R * r)];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        float2 *d = s + (int64_t(t) * Q + (j + R * r)) * 2;
        d[0] = make_float2(v[r].x, v[r].y);
        __asm__ volatile("" ::: "memory"); // two 8-byte stores, as the pass does
        d[1] = make_float2(v[r].z, v[r].w);
    }
}

__global__ __launch_bounds__(1024) void pass2_copy(const float2 *__restrict__ s, float2 *__restrict__ x, int lg,
                                                   int ls) {
    const int t = tile_of(blockIdx.x, gridDim.x, lg, ls), c = threadIdx.x & 3, j = threadIdx.x >> 2;
    const int k2 = 4 * t + c;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int k1 = j + 256 * r;
        v[r] = s[int64_t(k1 >> 1) * 2 * Q + 2 * k2 + (k1 & 1)];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) x[int64_t(k2) + int64_t(Q) * (j + 256 * r)] = v[r];
}

__global__ __launch_bounds__(256) void axis_copy(const float2 *__restrict__ in, float2 *__restrict__ out, int i0, int i1,
                                                 int i2, int o0, int o1, int o2, int lg, int ls) {
    const int t = tile_of(blockIdx.x, gridDim.x, lg, ls), c = threadIdx.x & 15, j = threadIdx.x >> 4;
    const int line = 16 * t + c, lm = line & 255, ld = line >> 8;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = j + 16 * r;
        v[r] = in[(int64_t(lm) << i0) + (int64_t(ld) << i1) + (int64_t(i) << i2)];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = j + 16 * r;
        out[(int64_t(lm) << o0) + (int64_t(ld) << o1) + (int64_t(i) << o2)] = v[r];
    }
}

__global__ __launch_bounds__(256) void stream_copy(const float4 *__restrict__ in, float4 *__restrict__ out, int64_t n4) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += int64_t(gridDim.x) * blockDim.x)
        out[i] = in[i];
}
} // namespace

int main() {
    constexpr int SETS = 4, REPS = 20;
    std::vector<float2 *> a(SETS), b(SETS);
    for (int k = 0; k < SETS; ++k) {
        CHECK(hipMalloc(&a[k], N * sizeof(float2)));
        CHECK(hipMalloc(&b[k], N * sizeof(float2)));
        CHECK(hipMemset(a[k], 0, N * sizeof(float2)));
        CHECK(hipMemset(b[k], 0, N * sizeof(float2)));
    }
    CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(pass1_copy),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto time_us = [&](auto launch) {
        for (int i = 0; i < SETS; ++i) launch(i);
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0, 0));
        for (int i = 0; i < REPS; ++i) launch(i);
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipGetLastError());
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        return 1000.0 * ms / REPS;
    };
    printf("{\"probe\": \"copy\", \"what\": \"contiguous copy of 16 n bytes, 16 bytes per lane\", \"us\": %.1f}\n",
           time_us([&](int i) {
               hipLaunchKernelGGL(stream_copy, dim3(8192), dim3(256), 0, 0,
                                  reinterpret_cast<const float4 *>(a[i % SETS]),
                                  reinterpret_cast<float4 *>(b[i % SETS]), N / 2);
           }));
    fflush(stdout);
    // the spread orders the library uses at this length (g = 2^lg, s = 2^ls)
    constexpr int P1G = 1, P1S = 2, P2G = 0, P2S = 4, AG = 0, AS = 5, BG = 0, BS = 3;
    if (!order_is_permutation(P / 2, P1G, P1S) || !order_is_permutation(Q / 4, P2G, P2S) ||
        !order_is_permutation(int(N / 4096), AG, AS) || !order_is_permutation(int(N / 4096), BG, BS)) {
        fprintf(stderr, "tile order is not a permutation\n");
        return 1;
    }
    for (int kb : {0, 50, 76, 100}) {
        int per_cu = 0;
        CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(pass1_copy), 512,
                                                          size_t(kb) * 1024));
        printf("{\"probe\": \"pass 1\", \"workgroups_per_cu\": %d, \"us\": %.1f}\n", per_cu, time_us([&](int i) {
                   hipLaunchKernelGGL(pass1_copy, dim3(P / 2), dim3(512), size_t(kb) * 1024, 0, a[i % SETS],
                                      b[i % SETS], 0, 0);
               }));
        fflush(stdout);
    }
    for (int kb : {0, 76}) {
        int per_cu = 0;
        CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(pass1_copy), 512,
                                                          size_t(kb) * 1024));
        printf("{\"probe\": \"pass 1\", \"order\": \"g 2, s 4\", \"workgroups_per_cu\": %d, \"us\": %.1f}\n",
               per_cu, time_us([&](int i) {
                   hipLaunchKernelGGL(pass1_copy, dim3(P / 2), dim3(512), size_t(kb) * 1024, 0, a[i % SETS],
                                      b[i % SETS], P1G, P1S);
               }));
        fflush(stdout);
    }
    {
        struct Wide {
            int T, lg, ls;
        } wide[] = {{4, 0, 0}, {4, 0, 3}, {8, 0, 0}, {8, 1, 4}};
        for (const Wide &w : wide) {
            if (!order_is_permutation(P / w.T, w.lg, w.ls)) {
                fprintf(stderr, "tile order is not a permutation\n");
                return 1;
            }
            printf("{\"probe\": \"pass 1, %d-column tiles\", \"order\": \"g %d, s %d\", \"us\": %.1f}\n", w.T,
                   1 << w.lg, 1 << w.ls, time_us([&](int i) {
                       if (w.T == 4)
                           hipLaunchKernelGGL(pass1_wide_copy<4>, dim3(P / 4), dim3(512), 0, 0, a[i % SETS],
                                              b[i % SETS], w.lg, w.ls);
                       else
                           hipLaunchKernelGGL(pass1_wide_copy<8>, dim3(P / 8), dim3(512), 0, 0, a[i % SETS],
                                              b[i % SETS], w.lg, w.ls);
                   }));
            fflush(stdout);
        }
    }
    for (int ls : {0, 1}) {
        if (!order_is_permutation(P / 2, 0, ls)) {
            fprintf(stderr, "tile order is not a permutation\n");
            return 1;
        }
        printf("{\"probe\": \"pass 1, rows per thread, 8 rows (512 threads)\", \"order\": \"g 1, s %d\", "
               "\"us\": %.1f}\n",
               1 << ls, time_us([&](int i) {
                   hipLaunchKernelGGL(pass1_rows_copy<8>, dim3(P / 2), dim3(Q / 8), 0, 0, a[i % SETS], b[i % SETS], 0,
                                      ls);
               }));
        printf("{\"probe\": \"pass 1, rows per thread, 16 rows (256 threads)\", \"order\": \"g 1, s %d\", "
               "\"us\": %.1f}\n",
               1 << ls, time_us([&](int i) {
                   hipLaunchKernelGGL(pass1_rows_copy<16>, dim3(P / 2), dim3(Q / 16), 0, 0, a[i % SETS], b[i % SETS],
                                      0, ls);
               }));
        fflush(stdout);
    }
    printf("{\"probe\": \"pass 2\", \"us\": %.1f}\n", time_us([&](int i) {
               hipLaunchKernelGGL(pass2_copy, dim3(Q / 4), dim3(1024), 0, 0, a[i % SETS], b[i % SETS], 0, 0);
           }));
    printf("{\"probe\": \"pass 2\", \"order\": \"g 1, s 16\", \"us\": %.1f}\n", time_us([&](int i) {
               hipLaunchKernelGGL(pass2_copy, dim3(Q / 4), dim3(1024), 0, 0, a[i % SETS], b[i % SETS], P2G, P2S);
           }));
    fflush(stdout);
    struct Axis {
        const char *name;
        int in[3], out[3];
    } axes[] = {{"A", {0, 8, 16}, {0, 8, 16}}, {"B", {0, 16, 8}, {0, 16, 8}}, {"C", {16, 8, 0}, {0, 8, 16}}};
    for (const Axis &x : axes) {
        printf("{\"probe\": \"axis pass %s\", \"us\": %.1f}\n", x.name, time_us([&](int i) {
                   hipLaunchKernelGGL(axis_copy, dim3(int(N / 4096)), dim3(256), 0, 0, a[i % SETS], b[i % SETS],
                                      x.in[0], x.in[1], x.in[2], x.out[0], x.out[1], x.out[2], 0, 0);
               }));
        fflush(stdout);
    }
    for (int k = 0; k < 2; ++k) {
        const Axis &x = axes[k];
        const int lg = k ? BG : AG, ls = k ? BS : AS;
        printf("{\"probe\": \"axis pass %s\", \"order\": \"g 1, s %d\", \"us\": %.1f}\n", x.name, 1 << ls,
               time_us([&](int i) {
                   hipLaunchKernelGGL(axis_copy, dim3(int(N / 4096)), dim3(256), 0, 0, a[i % SETS], b[i % SETS],
                                      x.in[0], x.in[1], x.in[2], x.out[0], x.out[1], x.out[2], lg, ls);
               }));
        fflush(stdout);
    }
    for (int k = 0; k < SETS; ++k) {
        CHECK(hipFree(a[k]));
        CHECK(hipFree(b[k]));
    }
    return 0;
}
