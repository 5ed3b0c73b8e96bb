// libliftfft: plan, launch and C ABI of the dimension-lifted 1-D complex FFT
// for gfx950.  The ABI is declared (and documented) in include/liftfft.h.
//
// Kernels (all in this file, device code in fft_engine.hpp):
//   pass_kernel<K_SINGLE>  n <= 4096: one workgroup tile holds whole
//                          transforms; natural order in and out.
//   pass_kernel<K_PASS1>   block phase of the lift n = p*q (Section 4.2-4.7 of
//                          the paper, Fig. 4.8): for each j1 < p the q-point
//                          transform over j2 of x[j1 + p*j2]; then the
//                          inter-phase weight w_n^(-j1*k2) (the paper's
//                          weightcyclic factors, Section 4.5, Fig. 4.4) and a
//                          store into the tiled scratch array
//                          S[j1/T1][k2][j1%T1] (the block-to-cyclic
//                          redistribution, Fig. 5.3 / Fig. 5.9).
//   pass_kernel<K_PASS2>   cyclic phase (Section 4.6, Fig. 4.6): for each
//                          k2 < q the p-point transform over j1 of S, stored
//                          as X[k2 + q*k1] (natural order, the
//                          cyclic-to-centralized gather of Fig. 5.5).
//   twiddle_table_kernel   FP64 generation of the weight tables.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <array>
#include <new>
#include <utility>
#include <vector>

#include "fft_engine.hpp"
#include "liftfft.h"

using namespace liftfft;

namespace {

enum Kind { K_SINGLE = 0, K_PASS1 = 1, K_PASS2 = 2 };

constexpr int MAX_LOG2_LINE = 12;          // longest line one workgroup transforms
constexpr int64_t LDS_BUDGET = 160 * 1024; // bytes of LDS per workgroup on gfx950

struct PassArgs {
    const void *in;
    void *out;
    const void *tw;    // w_N^e, e < N (+1 root), N = this pass's line length
    const void *tw_hi; // pass 1: w_n^(a * 2^log2h), a < n / 2^log2h
    const void *tw_lo; // pass 1: w_n^b, b < 2^log2h
    int64_t lines;     // batch * lines per transform
    int64_t n;         // transform length
    int32_t log2p, log2q;
    int32_t log2T;  // lines per tile of this kernel
    int32_t log2T1; // lines per tile of pass 1 (scratch tile width)
    int32_t log2h;
    int32_t conj_in, conj_out;
    int32_t xcd_remap;
};

// Workgroup -> tile.  Workgroups are dispatched round-robin over the 8 XCDs;
// with the remap each XCD owns a contiguous range of tiles, so tiles that
// share cache lines (adjacent columns in pass 1, adjacent rows in pass 2) are
// in flight in the same L2 at the same time.
__device__ __forceinline__ int64_t tile_index(int remap) {
    const int64_t bid = blockIdx.x, G = gridDim.x;
    if (remap) return (bid & 7) * (G >> 3) + (bid >> 3); // G is a multiple of 8
    return bid;
}

// Largest workgroup: 1024 threads for complex64, 512 for complex128 (whose
// tiles keep up to 256 VGPRs per lane).
template <typename Real> constexpr int max_threads() { return sizeof(Real) == 4 ? 1024 : 512; }

// One launch of a pass: each workgroup transforms one tile of T consecutive
// lines.  All data accesses go through buffer descriptors covering exactly
// the tile's range.
template <typename Real, int N, int RMAX, int KIND>
__global__ __launch_bounds__(max_threads<Real>()) void pass_kernel(PassArgs a) {
    using C = typename Cx<Real>::T;
    constexpr uint32_t ES = sizeof(C);
    constexpr int E = vals_per_thread(N), TPL = N / E;
    constexpr int NST = sched_nstages(N, RMAX);
    constexpr int R0 = sched_radix(N, RMAX, 0), RL = sched_radix(N, RMAX, NST - 1);
    constexpr int PITCH = line_pitch(N);
    constexpr bool TILE = uses_tile(N, RMAX);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);

    const int log2T = a.log2T, T = 1 << log2T;
    const int tid = threadIdx.x, nthr = blockDim.x;
    int c, j; // line within the tile, position within the line
    if constexpr (KIND != K_SINGLE) {
        c = tid & (T - 1); // lanes sweep the lines first: adjacent columns / rows
        j = tid >> log2T;
    } else {
        j = tid & (TPL - 1); // lanes sweep one contiguous line first
        c = tid / TPL;
    }
    const int64_t line0 = tile_index(a.xcd_remap) << log2T; // workgroup-uniform
    const bool active = line0 + c < a.lines;
    C *twl = lds + (TILE ? T * PITCH : 0);
    C *ep = twl + (TILE ? tw_total(N, RMAX) : 0);
    const Real sin_ = a.conj_in ? Real(-1) : Real(1);
    const Real sout = a.conj_out ? Real(-1) : Real(1);
    const C *__restrict__ in = static_cast<const C *>(a.in);
    C *__restrict__ out = static_cast<C *>(a.out);
    const int64_t pmask = (int64_t(1) << a.log2p) - 1, qmask = (int64_t(1) << a.log2q) - 1;

    // 1. Data loads: a buffer descriptor over the tile's range, one 32-bit
    //    lane offset, and a uniform per-slot offset.
    C v[E];
    if (active) {
        if constexpr (KIND == K_SINGLE) {
            const int64_t nl = a.lines - line0 < T ? a.lines - line0 : T;
            const rsrc_t src = make_rsrc(in + line0 * N, uint32_t(nl * N) * ES);
            const uint32_t lane = (uint32_t(c) * N + uint32_t(j)) * ES;
#pragma unroll
            for (int s = 0; s < E; ++s)
                v[s] = scale_im(buf_load(in, src, lane, uint32_t(slot_off<N, R0>(s)) * ES), sin_);
        } else if constexpr (KIND == K_PASS1) {
            const int64_t b = line0 >> a.log2p, j10 = line0 & pmask;
            const rsrc_t src = make_rsrc(in + b * a.n + j10, uint32_t(a.n - j10) * ES);
            const uint32_t lane = (uint32_t(c) + (uint32_t(j) << a.log2p)) * ES;
#pragma unroll
            for (int s = 0; s < E; ++s)
                v[s] = scale_im(buf_load(in, src, lane, (uint32_t(slot_off<N, R0>(s)) << a.log2p) * ES),
                                sin_);
        } else {
            // Scratch layout S[j1/T1][k2][j1%T1]; the plan keeps T1 | TPL, so
            // j1 = j + off(s) with off(s) a multiple of T1.
            const int64_t b = line0 >> a.log2q, k20 = line0 & qmask;
            const int l2T1 = a.log2T1, T1 = 1 << l2T1;
            const rsrc_t src = make_rsrc(in + b * a.n + (k20 << l2T1), uint32_t(a.n - (k20 << l2T1)) * ES);
            const uint32_t lane = ((uint32_t(j >> l2T1) << (a.log2q + l2T1)) + uint32_t(j & (T1 - 1)) +
                                   (uint32_t(c) << l2T1)) * ES;
#pragma unroll
            for (int s = 0; s < E; ++s)
                v[s] = scale_im(buf_load(in, src, lane, (uint32_t(slot_off<N, R0>(s)) << a.log2q) * ES),
                                sin_);
        }
    } else {
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = mk<C>(Real(0), Real(0));
    }

    // 2. Weight tables into LDS (published by the first barrier of the stage
    //    loop, or the explicit one below when the schedule has one stage).
    if constexpr (TILE) fill_twiddles<C, N, RMAX>(twl, static_cast<const C *>(a.tw), tid, nthr);
    C A = mk<C>(Real(1), Real(0));
    if constexpr (KIND == K_PASS1) {
        // Inter-pass weight w_n^(-j1*k2) with k2 = j + off(s): w_n^(j1*j)
        // (per thread) times P[c][s] = w_n^(j1*off(s)) (per line, in LDS),
        // both from the two-level FP64-generated tables.
        const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
        const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
        const int lomask = (1 << a.log2h) - 1;
        const int j10 = int(line0 & pmask);
        const int xa = (j10 + c) * j;
        A = cmul(hi[xa >> a.log2h], lo[xa & lomask]);
        for (int i = tid; i < T * (E + 1); i += nthr) {
            const int cc = i / (E + 1), s = i - cc * (E + 1);
            if (s >= E) continue;
            const int off = (s / RL) * TPL + (s % RL) * (N / RL);
            const int x = (j10 + cc) * off;
            ep[i] = cmul(hi[x >> a.log2h], lo[x & lomask]);
        }
        if constexpr (!TILE) __syncthreads();
    }

    run_stages<C, N, RMAX>(v, lds + c * PITCH, twl, j);

    // 3. Stores.
    if (!active) return;
    if constexpr (KIND == K_SINGLE) {
        const int64_t nl = a.lines - line0 < T ? a.lines - line0 : T;
        const rsrc_t dst = make_rsrc(out + line0 * N, uint32_t(nl * N) * ES);
        const uint32_t lane = (uint32_t(c) * N + uint32_t(j)) * ES;
#pragma unroll
        for (int s = 0; s < E; ++s)
            buf_store(scale_im(v[s], sout), dst, lane, uint32_t(slot_off<N, RL>(s)) * ES);
    } else if constexpr (KIND == K_PASS1) {
        // Tile j1/T of the scratch array S[j1/T][k2][j1%T].
        const int64_t b = line0 >> a.log2p, j10 = line0 & pmask;
        const rsrc_t dst = make_rsrc(out + b * a.n + (j10 << a.log2q), uint32_t(T << a.log2q) * ES);
        const uint32_t lane = ((uint32_t(j) << log2T) + uint32_t(c)) * ES;
        const C *P = ep + c * (E + 1);
#pragma unroll
        for (int s = 0; s < E; ++s)
            buf_store(cmulc(v[s], cmul(A, P[s])), dst, lane, (uint32_t(slot_off<N, RL>(s)) << log2T) * ES);
    } else {
        const int64_t b = line0 >> a.log2q, k20 = line0 & qmask;
        const rsrc_t dst = make_rsrc(out + b * a.n + k20, uint32_t(a.n - k20) * ES);
        const uint32_t lane = (uint32_t(c) + (uint32_t(j) << a.log2q)) * ES;
#pragma unroll
        for (int s = 0; s < E; ++s)
            buf_store(scale_im(v[s], sout), dst, lane, (uint32_t(slot_off<N, RL>(s)) << a.log2q) * ES);
    }
}

// out[i] = w_N^(i*mult mod N) (the +1 root), each entry from its integer
// exponent in FP64 and rounded once to the element type.
template <typename Real>
__global__ void twiddle_table_kernel(typename Cx<Real>::T *out, int64_t count, int64_t mult,
                                     int log2N) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t N = uint64_t(1) << log2N;
    const uint64_t e = (uint64_t(i) * uint64_t(mult)) & (N - 1);
    double s, c;
    sincospi(2.0 * double(e) / double(N), &s, &c);
    typename Cx<Real>::T w;
    w.x = Real(c);
    w.y = Real(s);
    out[i] = w;
}

using KernelFn = void (*)(PassArgs);

template <typename Real, int KIND, int RMAX, int... L>
constexpr std::array<KernelFn, sizeof...(L)> kernel_row(std::integer_sequence<int, L...>) {
    return {{(L == 0 ? nullptr : &pass_kernel<Real, (1 << (L == 0 ? 1 : L)), RMAX, KIND>)...}};
}

template <typename Real, int KIND, int RMAX> KernelFn pick(int log2N) {
    static const auto row =
        kernel_row<Real, KIND, RMAX>(std::make_integer_sequence<int, MAX_LOG2_LINE + 1>{});
    if (log2N < 1 || log2N > MAX_LOG2_LINE) return nullptr;
    return row[log2N];
}

template <typename Real> KernelFn pick_real(int kind, int log2N, int rmax) {
    switch (kind * 100 + rmax) {
    case K_SINGLE * 100 + 16: return pick<Real, K_SINGLE, 16>(log2N);
    case K_SINGLE * 100 + 2: return pick<Real, K_SINGLE, 2>(log2N);
    case K_PASS1 * 100 + 16: return pick<Real, K_PASS1, 16>(log2N);
    case K_PASS1 * 100 + 2: return pick<Real, K_PASS1, 2>(log2N);
    case K_PASS2 * 100 + 16: return pick<Real, K_PASS2, 16>(log2N);
    case K_PASS2 * 100 + 2: return pick<Real, K_PASS2, 2>(log2N);
    default: return nullptr;
    }
}

KernelFn pick_kernel(int dtype, int kind, int log2N, int rmax) {
    return dtype == FFT_C64 ? pick_real<float>(kind, log2N, rmax)
                            : pick_real<double>(kind, log2N, rmax);
}

int ilog2_exact(int64_t v) {
    if (v < 1 || (v & (v - 1))) return -1;
    int t = 0;
    while ((int64_t(1) << t) < v) ++t;
    return t;
}

struct Launch {
    KernelFn fn = nullptr;
    int log2N = 0, log2T = 0;
    int64_t lines = 0, ntiles = 0, grid = 0;
    int threads = 0;
    size_t lds = 0;
    bool remap = false;
};

} // namespace

struct fft_plan {
    int64_t n = 0, batch = 0;
    int dtype = 0, passes = 0, log2n = 0, log2p = 0, log2q = 0, log2h = 0, radix = 16;
    int device = 0;
    size_t esize = 0;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    void *tables = nullptr;
    size_t table_bytes = 0;
    const void *tw1 = nullptr, *tw2 = nullptr, *tw_hi = nullptr, *tw_lo = nullptr;
    Launch k1, k2;
    // Benchmark timing: a ring of event triples (before pass 1, after pass 1,
    // after pass 2) recorded on the execute stream; drained on read.
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int ring_head = 0, ring_count = 0;
    double ms[2] = {0, 0};
    int64_t launches[2] = {0, 0};
};

namespace {

// Lines per tile: the smallest power of two T <= max_lines whose tile has at
// least `want_threads` threads and `min_T` lines, as long as it fits the
// thread and LDS limits; `cap` (0 = none) bounds T.
int choose_log2T(int log2N, int rmax, size_t esize, int64_t max_lines, int want_threads,
                 int min_T, int cap, bool epilogue) {
    const int64_t thread_cap = esize == 8 ? max_threads<float>() : max_threads<double>();
    const int N = 1 << log2N;
    const int64_t tpl = N / vals_per_thread(N);
    auto fits = [&](int64_t T) {
        return T <= max_lines && T * tpl <= thread_cap &&
               int64_t(lds_elems(N, rmax, int(T), epilogue)) * int64_t(esize) <= LDS_BUDGET &&
               (!cap || T <= cap);
    };
    int log2T = 0;
    for (;;) {
        const int64_t T = int64_t(1) << log2T;
        if (T * tpl >= want_threads && T >= min_T) break;
        if (!fits(2 * T)) break;
        ++log2T;
    }
    return log2T;
}

// Fill a launch description: tile shape, LDS and grid (one workgroup per
// tile).
bool fill_launch(Launch &L, int dtype, int kind, int log2N, int rmax, int log2T, int64_t lines) {
    const int N = 1 << log2N;
    const size_t esize = dtype == FFT_C64 ? 8 : 16;
    L.fn = pick_kernel(dtype, kind, log2N, rmax);
    if (!L.fn) return false;
    L.log2N = log2N;
    L.log2T = log2T;
    L.lines = lines;
    L.threads = (N / vals_per_thread(N)) << log2T;
    L.ntiles = (lines + (int64_t(1) << log2T) - 1) >> log2T;
    L.grid = L.ntiles;
    L.lds = size_t(lds_elems(N, rmax, 1 << log2T, kind == K_PASS1)) * esize;
    if (L.lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void *>(L.fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(L.lds)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    L.remap = (L.grid % 8 == 0) && L.grid >= 16;
    return L.grid <= INT32_MAX;
}

// Tile shape for a pass kernel: pass 1 aims at 512-thread tiles of at least
// two lines (two workgroups per CU), pass 2 at tiles of at least four lines
// (32-byte segments in the natural-order output), both capped by `cap`.
bool plan_pass(Launch &L, int dtype, int kind, int log2N, int rmax, int64_t lines_per_transform,
               int64_t lines, int cap) {
    const size_t esize = dtype == FFT_C64 ? 8 : 16;
    const bool p1 = kind == K_PASS1;
    const int l2T = choose_log2T(log2N, rmax, esize, lines_per_transform, 512, p1 ? 2 : 4, cap, p1);
    return fill_launch(L, dtype, kind, log2N, rmax, l2T, lines);
}

int gen_table(int dtype, void *dst, int64_t count, int64_t mult, int log2N) {
    const int threads = 256;
    const int64_t blocks = (count + threads - 1) / threads;
    if (dtype == FFT_C64)
        hipLaunchKernelGGL(twiddle_table_kernel<float>, dim3(unsigned(blocks)), dim3(threads), 0, 0,
                           static_cast<float2 *>(dst), count, mult, log2N);
    else
        hipLaunchKernelGGL(twiddle_table_kernel<double>, dim3(unsigned(blocks)), dim3(threads), 0,
                           0, static_cast<double2 *>(dst), count, mult, log2N);
    return hipGetLastError() == hipSuccess ? FFT_OK : FFT_E_HIP;
}

constexpr int TIMING_RING = 1024;

// Accumulate the durations recorded in ring slot `slot` (waits for them).
int drain_slot(fft_plan *p, int slot) {
    hipEvent_t *e = &p->ev[size_t(slot) * 3];
    const hipEvent_t last = p->passes == 1 ? e[1] : e[2];
    if (hipEventSynchronize(last) != hipSuccess) return FFT_E_HIP;
    float t = 0;
    if (hipEventElapsedTime(&t, e[0], e[1]) != hipSuccess) return FFT_E_HIP;
    p->ms[0] += t;
    p->launches[0] += 1;
    if (p->passes == 2) {
        if (hipEventElapsedTime(&t, e[1], e[2]) != hipSuccess) return FFT_E_HIP;
        p->ms[1] += t;
        p->launches[1] += 1;
    }
    return FFT_OK;
}

int drain_all(fft_plan *p) {
    int rc = FFT_OK;
    while (p->ring_count > 0) {
        const int slot = (p->ring_head - p->ring_count + TIMING_RING) % TIMING_RING;
        const int r = drain_slot(p, slot);
        if (r != FFT_OK) rc = r;
        --p->ring_count;
    }
    return rc;
}

void free_plan(fft_plan *p) {
    if (!p) return;
    for (auto &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    if (p->scratch) (void)hipFree(p->scratch);
    if (p->tables) (void)hipFree(p->tables);
    delete p;
}

int launch(const fft_plan *p, const Launch &L, const PassArgs &args, hipStream_t st) {
    if (L.grid <= 0) return FFT_OK;
    hipLaunchKernelGGL(L.fn, dim3(unsigned(L.grid)), dim3(unsigned(L.threads)), L.lds, st, args);
    (void)p;
    return hipGetLastError() == hipSuccess ? FFT_OK : FFT_E_HIP;
}

} // namespace

extern "C" {

int fft_abi_version(void) { return LIFTFFT_ABI_VERSION; }

const char *fft_strerror(int code) {
    switch (code) {
    case FFT_OK: return "success";
    case FFT_E_SIZE: return "invalid size: n must be a power of two >= 2, batch >= 1, no overflow";
    case FFT_E_DTYPE: return "unknown element type";
    case FFT_E_SIGN: return "sign must be -1 or +1";
    case FFT_E_NULL: return "required pointer is NULL";
    case FFT_E_ALIGN: return "buffer not aligned to its element size";
    case FFT_E_OOM: return "device allocation failed";
    case FFT_E_HIP: return "HIP runtime call or kernel launch failed";
    case FFT_E_UNSUPPORTED: return "valid request outside what this build supports";
    case FFT_E_ARG: return "invalid option";
    default: return "unknown status code";
    }
}

int fft_plan_create_ex(int64_t n, int64_t batch, int dtype, const fft_plan_opts *opts,
                       fft_plan **plan_out) {
    if (!plan_out) return FFT_E_NULL;
    *plan_out = nullptr;
    if (dtype != FFT_C64 && dtype != FFT_C128) return FFT_E_DTYPE;
    const int t = ilog2_exact(n);
    if (t < 1 || batch < 1) return FFT_E_SIZE;
    const size_t esize = dtype == FFT_C64 ? 8 : 16;
    if (batch > (INT64_MAX / 4) / n / int64_t(esize)) return FFT_E_SIZE;
    const int max_t = dtype == FFT_C64 ? FFT_MAX_LOG2N_C64 : FFT_MAX_LOG2N_C128;
    if (t > max_t) return FFT_E_UNSUPPORTED;

    fft_plan_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    for (int r : o.reserved)
        if (r) return FFT_E_ARG;
    int radix = o.radix ? o.radix : 16;
    if (radix != 2 && radix != 16) {
        if (radix == 4 || radix == 8) return FFT_E_UNSUPPORTED;
        return FFT_E_ARG;
    }
    if (o.log2_p < 0 || (o.log2_p && o.log2_p >= t)) return FFT_E_ARG;
    if (o.lines_per_block < 0 || (o.lines_per_block & (o.lines_per_block - 1))) return FFT_E_ARG;
    if (o.lines_per_block2 < 0 || (o.lines_per_block2 & (o.lines_per_block2 - 1))) return FFT_E_ARG;
    if (o.flags & ~int32_t(FFT_OPT_NO_XCD_REMAP)) return FFT_E_ARG;

    fft_plan *p = new (std::nothrow) fft_plan;
    if (!p) return FFT_E_OOM;
    p->n = n;
    p->batch = batch;
    p->dtype = dtype;
    p->log2n = t;
    p->radix = radix;
    p->esize = esize;
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        return FFT_E_HIP;
    }

    if (o.log2_p == 0 && t <= MAX_LOG2_LINE) {
        p->passes = 1;
        p->log2q = t;
        const int l2T = choose_log2T(t, radix, esize, batch, 256, 1, o.lines_per_block, false);
        if (!fill_launch(p->k1, dtype, K_SINGLE, t, radix, l2T, batch)) {
            free_plan(p);
            return FFT_E_UNSUPPORTED;
        }
    } else {
        p->passes = 2;
        p->log2q = o.log2_p ? t - o.log2_p : (t + 1) / 2;
        p->log2p = t - p->log2q;
        if (p->log2q > MAX_LOG2_LINE || p->log2p > MAX_LOG2_LINE) {
            free_plan(p);
            return FFT_E_UNSUPPORTED;
        }
        const int64_t P = int64_t(1) << p->log2p, Q = int64_t(1) << p->log2q;
        // Pass 2 reads the scratch tile layout of pass 1 with a separable
        // offset, which needs T1 | TPL2 (TPL2 = threads per pass-2 line).
        const int tpl2 = int(P / vals_per_thread(int(P)));
        const int cap1 = o.lines_per_block ? (o.lines_per_block < tpl2 ? o.lines_per_block : tpl2) : tpl2;
        if (!plan_pass(p->k1, dtype, K_PASS1, p->log2q, radix, P, P * batch, cap1) ||
            !plan_pass(p->k2, dtype, K_PASS2, p->log2p, radix, Q, Q * batch, o.lines_per_block2)) {
            free_plan(p);
            return FFT_E_UNSUPPORTED;
        }
    }
    if (o.flags & FFT_OPT_NO_XCD_REMAP) p->k1.remap = p->k2.remap = false;
    if (!p->k1.fn || (p->passes == 2 && !p->k2.fn)) {
        free_plan(p);
        return FFT_E_UNSUPPORTED;
    }

    // Device memory: scratch (two-pass only) and the weight tables.
    p->log2h = p->passes == 2 ? (t + 1) / 2 : 0;
    const int64_t n1 = int64_t(1) << p->log2q;                          // pass-1 line
    const int64_t n2 = p->passes == 2 ? (int64_t(1) << p->log2p) : 0;   // pass-2 line
    const int64_t nhi = p->passes == 2 ? (n >> p->log2h) : 0;
    const int64_t nlo = p->passes == 2 ? (int64_t(1) << p->log2h) : 0;
    const int64_t entries = n1 + n2 + nhi + nlo;
    p->table_bytes = size_t(entries) * esize;
    if (hipMalloc(&p->tables, p->table_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->tables = nullptr;
        free_plan(p);
        return FFT_E_OOM;
    }
    if (p->passes == 2) {
        p->scratch_bytes = size_t(n) * size_t(batch) * esize;
        if (hipMalloc(&p->scratch, p->scratch_bytes) != hipSuccess) {
            (void)hipGetLastError();
            p->scratch = nullptr;
            free_plan(p);
            return FFT_E_OOM;
        }
    }
    char *tb = static_cast<char *>(p->tables);
    p->tw1 = tb;
    int rc = gen_table(dtype, tb, n1, 1, p->log2q);
    if (p->passes == 2) {
        char *t2 = tb + n1 * esize, *th = t2 + n2 * esize, *tl = th + nhi * esize;
        p->tw2 = t2;
        p->tw_hi = th;
        p->tw_lo = tl;
        if (rc == FFT_OK) rc = gen_table(dtype, t2, n2, 1, p->log2p);
        if (rc == FFT_OK) rc = gen_table(dtype, th, nhi, nlo, t);
        if (rc == FFT_OK) rc = gen_table(dtype, tl, nlo, 1, t);
    }
    if (rc == FFT_OK && hipDeviceSynchronize() != hipSuccess) rc = FFT_E_HIP;
    if (rc != FFT_OK) {
        free_plan(p);
        return rc;
    }
    *plan_out = p;
    return FFT_OK;
}

int fft_plan_create(int64_t n, int64_t batch, int dtype, fft_plan **plan_out) {
    return fft_plan_create_ex(n, batch, dtype, nullptr, plan_out);
}

int fft_execute(const fft_plan *plan, const void *in, void *out, int sign, void *stream) {
    if (!plan || !in || !out) return FFT_E_NULL;
    if (sign != -1 && sign != 1) return FFT_E_SIGN;
    if ((reinterpret_cast<uintptr_t>(in) % plan->esize) ||
        (reinterpret_cast<uintptr_t>(out) % plan->esize))
        return FFT_E_ALIGN;
    {
        // Partial overlap of in and out is not allowed (exact aliasing is).
        const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
        const uintptr_t bytes = uintptr_t(plan->n) * uintptr_t(plan->batch) * plan->esize;
        if (a != b && a < b + bytes && b < a + bytes) return FFT_E_ARG;
    }
    fft_plan *p = const_cast<fft_plan *>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return FFT_E_HIP;
    if (cur != p->device && hipSetDevice(p->device) != hipSuccess) return FFT_E_HIP;

    const bool inv = sign > 0;
    PassArgs a;
    memset(&a, 0, sizeof(a));
    a.n = p->n;
    a.log2p = p->log2p;
    a.log2q = p->log2q;
    a.log2h = p->log2h;
    int rc = FFT_OK;
    hipEvent_t *ev = nullptr;
    if (p->timing) {
        if (p->ring_count == TIMING_RING) { // oldest slot still pending: drain it first
            const int slot = p->ring_head;
            rc = drain_slot(p, slot);
            --p->ring_count;
        }
        ev = &p->ev[size_t(p->ring_head) * 3];
        if (rc == FFT_OK) rc = hipEventRecord(ev[0], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
    }
    if (p->passes == 1) {
        a.in = in;
        a.out = out;
        a.tw = p->tw1;
        a.lines = p->k1.lines;
        a.log2T = a.log2T1 = p->k1.log2T;
        a.conj_in = a.conj_out = inv;
        a.xcd_remap = p->k1.remap;
        if (rc == FFT_OK) rc = launch(p, p->k1, a, st);
        if (rc == FFT_OK && ev) rc = hipEventRecord(ev[1], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
    } else {
        a.in = in;
        a.out = p->scratch;
        a.tw = p->tw1;
        a.tw_hi = p->tw_hi;
        a.tw_lo = p->tw_lo;
        a.lines = p->k1.lines;
        a.log2T = a.log2T1 = p->k1.log2T;
        a.conj_in = inv;
        a.conj_out = 0;
        a.xcd_remap = p->k1.remap;
        if (rc == FFT_OK) rc = launch(p, p->k1, a, st);
        if (rc == FFT_OK && ev) rc = hipEventRecord(ev[1], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
        a.in = p->scratch;
        a.out = out;
        a.tw = p->tw2;
        a.lines = p->k2.lines;
        a.log2T = p->k2.log2T;
        a.log2T1 = p->k1.log2T;
        a.conj_in = 0;
        a.conj_out = inv;
        a.xcd_remap = p->k2.remap;
        if (rc == FFT_OK) rc = launch(p, p->k2, a, st);
        if (rc == FFT_OK && ev) rc = hipEventRecord(ev[2], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
    }
    if (rc == FFT_OK && ev) {
        p->ring_head = (p->ring_head + 1) % TIMING_RING;
        ++p->ring_count;
    }
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
}

int fft_plan_destroy(fft_plan *plan) {
    free_plan(plan);
    return FFT_OK;
}

int fft_plan_get_info(const fft_plan *p, fft_plan_info *info) {
    if (!p || !info) return FFT_E_NULL;
    memset(info, 0, sizeof(*info));
    info->n = p->n;
    info->batch = p->batch;
    info->dtype = p->dtype;
    info->passes = p->passes;
    info->log2_p = p->log2p;
    info->log2_q = p->log2q;
    info->radix = p->radix;
    info->lines_per_block_pass1 = 1 << p->k1.log2T;
    info->lines_per_block_pass2 = p->passes == 2 ? (1 << p->k2.log2T) : 0;
    info->grid_pass1 = int32_t(p->k1.grid);
    info->grid_pass2 = p->passes == 2 ? int32_t(p->k2.grid) : 0;
    info->threads_pass1 = p->k1.threads;
    info->threads_pass2 = p->passes == 2 ? p->k2.threads : 0;
    info->lds_bytes_pass1 = int64_t(p->k1.lds);
    info->lds_bytes_pass2 = p->passes == 2 ? int64_t(p->k2.lds) : 0;
    info->scratch_bytes = int64_t(p->scratch_bytes);
    info->table_bytes = int64_t(p->table_bytes);
    return FFT_OK;
}

int fft_plan_set_timing(fft_plan *p, int enable) {
    if (!p) return FFT_E_NULL;
    if (enable && p->ev.empty()) {
        p->ev.assign(size_t(TIMING_RING) * 3, nullptr);
        for (auto &e : p->ev) {
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                e = nullptr;
                return FFT_E_HIP;
            }
        }
    }
    if (!enable && p->timing) {
        const int rc = drain_all(p);
        p->timing = false;
        return rc;
    }
    p->timing = enable != 0;
    return FFT_OK;
}

int fft_plan_read_timing(fft_plan *p, double ms_out[2], int64_t launches_out[2], int reset) {
    if (!p || !ms_out || !launches_out) return FFT_E_NULL;
    const int rc = p->ev.empty() ? FFT_OK : drain_all(p);
    for (int k = 0; k < 2; ++k) {
        ms_out[k] = p->ms[k];
        launches_out[k] = p->launches[k];
    }
    if (reset) {
        p->ms[0] = p->ms[1] = 0;
        p->launches[0] = p->launches[1] = 0;
    }
    return rc;
}

} // extern "C"
