// Device-side FFT engine for gfx950: complex helpers, DFT codelets, the radix
// schedule, the LDS layout and the workgroup-tile transform used by every
// pass kernel.
//
// A workgroup owns T "lines" (independent N-point transforms).  Each line is
// processed by TPL = N/E threads holding E = min(EMAX, N) complex values in
// registers (EMAX = 16 or 32).  The stage loop is the paper's stage loop (Section 2.1, Fig. 2.1:
// one butterfly stage per doubling of the column length) regrouped into
// radix-R stages, R <= 16: a radix-R stage is log2(R) radix-2 stages done at
// once in registers -- the same dimension lifting the paper applies between
// processors (Section 4.2), applied here between the register file and LDS.
// Stages are self-sorting (Stockham form), so no bit-reversal pass is needed:
// for stage s with radix R and Ns = product of the earlier radices, butterfly
// b < N/R reads elements b + r*(N/R), multiplies element r by
// w_{Ns*R}^(-r*(b mod Ns)), does an R-point DFT and writes element r to
// (b div Ns)*Ns*R + (b mod Ns) + r*Ns.  Data moves between stages through LDS.
//
// All transforms here use the exponent sign -1; sign +1 is obtained by
// conjugating on load and on store (F_+(x) = conj(F_-(conj x))).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace liftfft {

template <typename Real> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

template <typename C> __device__ __forceinline__ C mk(decltype(C::x) re, decltype(C::x) im) {
    C r;
    r.x = re;
    r.y = im;
    return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
// a * b
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(w): multiply by the sign -1 root when w holds the +1 root.
template <typename C> __device__ __forceinline__ C cmulc(C a, C w) {
    return mk<C>(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}
// a * (-i)
template <typename C> __device__ __forceinline__ C mul_mi(C a) { return mk<C>(a.y, -a.x); }
// Imaginary part times a uniform +1 or -1 (exact): conjugation on demand.
template <typename C> __device__ __forceinline__ C scale_im(C a, decltype(C::x) s) {
    return mk<C>(a.x, a.y * s);
}

// Multiply by w_16^(-e) (sign -1 root), e in 0..15, trivial cases folded.
template <int e, typename C> __device__ __forceinline__ C rot16(C a) {
    using R = decltype(C::x);
    constexpr R c1 = R(0.92387953251128675613); // cos(pi/8)
    constexpr R s1 = R(0.38268343236508977173); // sin(pi/8)
    constexpr R h = R(0.70710678118654752440);  // sqrt(1/2)
    constexpr int m = e & 15;
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return mul_mi(a);
    else if constexpr (m == 8) return mk<C>(-a.x, -a.y);
    else if constexpr (m == 12) return mk<C>(-a.y, a.x);
    else if constexpr (m == 2) return mk<C>((a.x + a.y) * h, (a.y - a.x) * h);
    else if constexpr (m == 6) return mk<C>((a.y - a.x) * h, -(a.x + a.y) * h);
    else if constexpr (m == 10) return mk<C>(-(a.x + a.y) * h, (a.x - a.y) * h);
    else if constexpr (m == 14) return mk<C>((a.x - a.y) * h, (a.x + a.y) * h);
    else {
        // w_16^(-m) = cos(2 pi m/16) - i sin(2 pi m/16)
        constexpr R cs[16] = {R(1), c1, h, s1, R(0), -s1, -h, -c1, R(-1), -c1, -h, -s1, R(0), s1, h, c1};
        constexpr R sn[16] = {R(0), s1, h, c1, R(1), c1, h, s1, R(0), -s1, -h, -c1, R(-1), -c1, -h, -s1};
        constexpr R wr = cs[m], wi = -sn[m];
        return mk<C>(a.x * wr - a.y * wi, a.x * wi + a.y * wr);
    }
}

// In-register R-point DFTs, sign -1, natural order in and out, on v[0..R).
template <typename C> __device__ __forceinline__ void dft2(C *v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename C> __device__ __forceinline__ void dft4(C &x0, C &x1, C &x2, C &x3) {
    C t0 = cadd(x0, x2), t1 = csub(x0, x2);
    C t2 = cadd(x1, x3), t3 = mul_mi(csub(x1, x3));
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3);
    x3 = csub(t1, t3);
}
template <typename C> __device__ __forceinline__ void dft4(C *v) { dft4(v[0], v[1], v[2], v[3]); }

template <typename C> __device__ __forceinline__ void dft8(C *v) {
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = rot16<2>(o1);
    o2 = rot16<4>(o2);
    o3 = rot16<6>(o3);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// 16 = 4 x 4: DFT4 over r1 for each r2 (element r2 + 4 r1), twiddle
// w_16^(-r2*k1), DFT4 over r2 for each k1; output k1 + 4 k2.
template <typename C> __device__ __forceinline__ void dft16(C *v) {
    C a[16];
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2) {
        C x0 = v[r2], x1 = v[r2 + 4], x2 = v[r2 + 8], x3 = v[r2 + 12];
        dft4(x0, x1, x2, x3);
        a[4 * r2 + 0] = x0;
        a[4 * r2 + 1] = x1;
        a[4 * r2 + 2] = x2;
        a[4 * r2 + 3] = x3;
    }
    a[5] = rot16<1>(a[5]);
    a[6] = rot16<2>(a[6]);
    a[7] = rot16<3>(a[7]);
    a[9] = rot16<2>(a[9]);
    a[10] = rot16<4>(a[10]);
    a[11] = rot16<6>(a[11]);
    a[13] = rot16<3>(a[13]);
    a[14] = rot16<6>(a[14]);
    a[15] = rot16<9>(a[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C x0 = a[k1], x1 = a[4 + k1], x2 = a[8 + k1], x3 = a[12 + k1];
        dft4(x0, x1, x2, x3);
        v[k1] = x0;
        v[k1 + 4] = x1;
        v[k1 + 8] = x2;
        v[k1 + 12] = x3;
    }
}

template <int R, typename C> __device__ __forceinline__ void dft(C *v) {
    if constexpr (R == 1) return;
    else if constexpr (R == 2) dft2(v);
    else if constexpr (R == 4) dft4(v);
    else if constexpr (R == 8) dft8(v);
    else dft16(v);
}

// ---------------------------------------------------------------------------
// Radix schedule and LDS layout.  Plain constexpr functions of (N, RMAX, ...)
// so the host computes the same sizes the kernels use.
//
// Schedule: as many RMAX stages as fit plus one smaller stage for the
// remainder, placed second so that the first and last stages (the ones that
// touch global memory) use the full radix.
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
__host__ __device__ constexpr int vals_per_thread(int N, int EMAX = 16) { return N < EMAX ? N : EMAX; }
__host__ __device__ constexpr int sched_logr(int N, int RMAX) { return ilog2c(RMAX < N ? RMAX : N); }
__host__ __device__ constexpr int sched_nstages(int N, int RMAX) {
    return ilog2c(N) / sched_logr(N, RMAX) + (ilog2c(N) % sched_logr(N, RMAX) ? 1 : 0);
}
__host__ __device__ constexpr int sched_radix(int N, int RMAX, int s) {
    return (ilog2c(N) % sched_logr(N, RMAX) && s == 1) ? (1 << (ilog2c(N) % sched_logr(N, RMAX)))
                                                        : (1 << sched_logr(N, RMAX));
}
__host__ __device__ constexpr int sched_ns(int N, int RMAX, int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= sched_radix(N, RMAX, i);
    return p;
}

// Tile: line c occupies [c*pitch, c*pitch + N + N/16) of the exchange array;
// element e sits at e + e/16 within its line (one spare slot per 16 elements
// spreads the strided Stockham writes over the banks).  The exchange array
// holds complex elements, or -- in the split form -- one real component at a
// time (half the LDS; each exchange then runs twice, real parts first).  The
// pitch is chosen on the host (exchange_pitch) so that the lines that share a
// wavefront start in different banks.
__host__ __device__ constexpr int padded_line(int N) { return N + N / 16; }
// Stage twiddles w_M^(r*k), M = Ns*R, k < Ns, r < R: with k = klo + 16*khi,
// w_M^(r*k) = LO[klo][r] * HI[khi][r], LO[klo][r] = w_M^(r*klo) (klo < 16),
// HI[khi][r] = w_{M/16}^(r*khi) (khi < Ns/16).  Rows padded to R+1 entries.
__host__ __device__ constexpr int tw_lo_rows(int N, int RMAX, int s) {
    return sched_ns(N, RMAX, s) < 16 ? sched_ns(N, RMAX, s) : 16;
}
__host__ __device__ constexpr int tw_hi_rows(int N, int RMAX, int s) {
    return sched_ns(N, RMAX, s) > 16 ? sched_ns(N, RMAX, s) / 16 : 0;
}
__host__ __device__ constexpr int tw_stage_size(int N, int RMAX, int s) {
    return (tw_lo_rows(N, RMAX, s) + tw_hi_rows(N, RMAX, s)) * (sched_radix(N, RMAX, s) + 1);
}
__host__ __device__ constexpr int tw_stage_off(int N, int RMAX, int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += tw_stage_size(N, RMAX, i);
    return o;
}
__host__ __device__ constexpr int tw_total(int N, int RMAX) {
    return tw_stage_off(N, RMAX, sched_nstages(N, RMAX));
}
__host__ __device__ constexpr bool uses_tile(int N, int RMAX) { return sched_nstages(N, RMAX) > 1; }

// Line pitch (in exchange elements of `esize` bytes) for a tile of T lines.
// LDS serves one 128-byte bank window per cycle; in the pass kernels the
// lanes of a wavefront sweep the T lines first, so line c is shifted by
// c * 128/T bytes within the window.  In the single-pass kernel
// (`lines_first` = false) the lanes sweep TPL positions of one line first,
// and consecutive lines are shifted by TPL elements.
inline int exchange_pitch(int N, int T, int TPL, int esize, bool lines_first) {
    const int window = 128 / esize; // exchange elements per bank window
    int target;
    if (lines_first) target = T >= window ? 1 : window / T;
    else target = TPL >= window ? 0 : TPL;
    int p = padded_line(N);
    while (p % window != target % window) ++p;
    return p;
}

// Byte offsets of the LDS regions of one workgroup: the exchange tile of T
// lines, the stage twiddle tables (16-byte aligned) and, in pass 1, two
// buffers of the inter-pass weight table of T x (E+1) entries (alternate
// tiles of a persistent workgroup use alternate buffers).
// `force` keeps the exchange tile for single-stage schedules (the
// matrix-core stages always pass through LDS).
__host__ __device__ constexpr int64_t lds_tile_bytes(int N, int RMAX, int T, int pitch, int lsize,
                                                     bool force = false) {
    return (uses_tile(N, RMAX) || force) ? ((int64_t(T) * pitch * lsize + 15) & ~int64_t(15)) : 0;
}
__host__ __device__ constexpr int64_t lds_ep_offset(int N, int RMAX, int T, int pitch, int lsize, int csize,
                                                    bool force = false) {
    return lds_tile_bytes(N, RMAX, T, pitch, lsize, force) +
           (uses_tile(N, RMAX) ? int64_t(tw_total(N, RMAX)) * csize : 0);
}
inline int64_t lds_bytes(int N, int RMAX, int T, int E, int pitch, int lsize, int csize, bool epilogue,
                         bool force = false) {
    return lds_ep_offset(N, RMAX, T, pitch, lsize, csize, force) +
           (epilogue ? 2 * int64_t(T) * (E + 1) * csize : 0);
}

template <int N> __device__ __forceinline__ constexpr int lpad(int e) { return e + (e >> 4); }

// ---------------------------------------------------------------------------
// Buffer-resource memory access.  Each pass addresses its global data through
// a buffer descriptor over exactly the bytes the workgroup may touch: one
// VGPR lane offset serves every slot (the per-slot stride is a scalar), and
// an access outside the range reads zero / is dropped instead of faulting.
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    // Word 3 = 0x00020000: raw (untyped) 32-bit data format on gfx9-class parts.
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), short(0), int(bytes),
                                             0x00020000);
}
// AUX is the instruction's cache-policy field (0: default; on gfx950 bit 1
// marks the access non-temporal, i.e. streamed past the caches' normal
// retention).
template <int AUX = 0>
__device__ __forceinline__ float2 buf_load(const float2 *, rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ double2 buf_load(const double2 *, rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
}
// 16 bytes at once: two adjacent complex64 elements.
__device__ __forceinline__ float4 buf_load_pair(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <int AUX = 0> __device__ __forceinline__ void buf_store(float2 v, rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, AUX);
}
// A 16-byte element is stored as two 8-byte stores.  Single 16-byte buffer
// stores of complex128 results gave, intermittently (about one transform in
// 200), an element whose first dword held another value; with two 8-byte
// stores no such element has been seen (repeat runs are checked bit for
// bit).  What caused it was not established.  (The empty asm statement
// keeps the two stores from being merged back.)
template <int AUX = 0> __device__ __forceinline__ void buf_store(double2 v, rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v.x), r, voff, soff, AUX);
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v.y), r, voff + 8, soff, AUX);
}
// Plain global store of one element (transforms addressed in 64 bits);
// complex128 as two 8-byte stores, as above.
__device__ __forceinline__ void global_store(float2 *p, float2 v) { *p = v; }
__device__ __forceinline__ void global_store(double2 *p, double2 v) {
    double *q = reinterpret_cast<double *>(p);
    q[0] = v.x;
    __asm__ volatile("" ::: "memory");
    q[1] = v.y;
}
// Element index held by register slot s on entry (first-stage layout) or on
// exit (last-stage layout) relative to the thread's j: slot i*R + r <->
// j + i*TPL + r*(N/R), TPL = N/E.
template <int N, int E, int R> __device__ __forceinline__ constexpr int slot_off(int s) {
    return (s / R) * (N / E) + (s % R) * (N / R);
}

// Source of entry i of the LDS stage tables (stages 1.. laid out back to
// back, rows of R+1 entries): the index e*(N/M) of w_M^e in the global table
// w_N^e (e < N, +1 root), or -1 for a row's padding slot.  LO rows hold
// w_M^(r*row), HI rows w_M^(16*r*(row-LO)).
template <int N, int RMAX, int STG = 1> __device__ __forceinline__ int tw_source(int i) {
    if constexpr (STG >= sched_nstages(N, RMAX)) {
        return -1;
    } else {
        constexpr int R = sched_radix(N, RMAX, STG), NS = sched_ns(N, RMAX, STG);
        constexpr int M = NS * R, ROW = R + 1, LO = tw_lo_rows(N, RMAX, STG);
        constexpr int SZ = tw_stage_size(N, RMAX, STG);
        if (i >= SZ) return tw_source<N, RMAX, STG + 1>(i - SZ);
        const int row = i / ROW, r = i - row * ROW;
        if (r >= R) return -1;
        return (row < LO ? r * row : 16 * r * (row - LO)) * (N / M);
    }
}

// Fill the stage twiddle tables in LDS from the global table.  Every thread
// of the workgroup takes part, from entry `first` on; a barrier must follow
// before the tables are read.
template <typename C, int N, int RMAX>
__device__ __forceinline__ void fill_twiddles(C *twl, const C *__restrict__ tw, int tid, int nthr, int first = 0) {
    for (int i = first + tid; i < tw_total(N, RMAX); i += nthr) {
        const int g = tw_source<N, RMAX>(i);
        if (g >= 0) twl[i] = tw[g];
    }
}

// Run the whole stage schedule on one thread's registers.
//   v      E values; on entry slot i*R0 + r = element j + i*TPL + r*(N/R0),
//          on exit slot i*RL + r = element j + i*TPL + r*(N/RL).
//   line   this thread's line in the LDS exchange array: complex elements,
//          or (SPLIT) one real component at a time
//   twl    the LDS twiddle tables
// The first LDS write happens without a barrier: the caller orders it after
// any earlier readers of the tile.
// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, then for every wave, without the memory fence of
// __syncthreads (which would also wait for outstanding global loads, among
// them direct-to-LDS loads still streaming the next tile).
__device__ __forceinline__ void lds_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <bool LDS_ONLY> __device__ __forceinline__ void tile_barrier() {
    if constexpr (LDS_ONLY) lds_barrier();
    else __syncthreads();
}

template <typename C, int N, int RMAX, int E, bool SPLIT, int STG = 0, bool LDS_ONLY = false>
__device__ __forceinline__ void run_stages(C *v, void *line_base, const C *twl, int j) {
    using Real = decltype(C::x);
    constexpr int TPL = N / E;
    constexpr int NST = sched_nstages(N, RMAX);
    constexpr int R = sched_radix(N, RMAX, STG);
    constexpr int NS = sched_ns(N, RMAX, STG);
    constexpr int NB = E / R;
    if constexpr (STG > 0 && NS > 1) {
        constexpr int ROW = R + 1, LO = tw_lo_rows(N, RMAX, STG);
        constexpr int OFF = tw_stage_off(N, RMAX, STG);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int k = (j + i * TPL) & (NS - 1);
            const C *lo = twl + OFF + (k & 15) * ROW;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w = lo[r];
                if constexpr (NS > 16) w = cmul(w, twl[OFF + (LO + (k >> 4)) * ROW + r]);
                v[i * R + r] = cmulc(v[i * R + r], w);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) dft<R>(&v[i * R]);
    if constexpr (STG + 1 < NST) {
        constexpr int R2 = sched_radix(N, RMAX, STG + 1), NB2 = E / R2;
        if constexpr (!SPLIT) {
            C *line = static_cast<C *>(line_base);
            if constexpr (STG > 0) tile_barrier<LDS_ONLY>(); // earlier readers of the tile are done
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = j + i * TPL;
                const int base = (b / NS) * NS * R + (b & (NS - 1));
#pragma unroll
                for (int r = 0; r < R; ++r) line[lpad<N>(base + r * NS)] = v[i * R + r];
            }
            tile_barrier<LDS_ONLY>();
#pragma unroll
            for (int i = 0; i < NB2; ++i) {
                const int b = j + i * TPL;
#pragma unroll
                for (int r = 0; r < R2; ++r) v[i * R2 + r] = line[lpad<N>(b + r * (N / R2))];
            }
        } else {
            // Real parts, then imaginary parts, through the same array.  The
            // second write reads only .y, which the first read left alone.
            Real *line = static_cast<Real *>(line_base);
#pragma unroll
            for (int part = 0; part < 2; ++part) {
                if (STG > 0 || part > 0) tile_barrier<LDS_ONLY>();
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const int b = j + i * TPL;
                    const int base = (b / NS) * NS * R + (b & (NS - 1));
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        line[lpad<N>(base + r * NS)] = part ? v[i * R + r].y : v[i * R + r].x;
                }
                tile_barrier<LDS_ONLY>();
#pragma unroll
                for (int i = 0; i < NB2; ++i) {
                    const int b = j + i * TPL;
#pragma unroll
                    for (int r = 0; r < R2; ++r) {
                        const Real x = line[lpad<N>(b + r * (N / R2))];
                        if (part) v[i * R2 + r].y = x;
                        else v[i * R2 + r].x = x;
                    }
                }
            }
        }
        run_stages<C, N, RMAX, E, SPLIT, STG + 1, LDS_ONLY>(v, line_base, twl, j);
    }
}

// The same schedule for NL lines per thread, split exchange only: thread j
// holds, for each line l, the values run_stages' thread j holds for one
// line (v[l], same slots), and line l's exchange array starts at
// lines + l * pitch.  Each exchange writes every line's part, then one
// barrier pair serves them all.
template <typename C, int N, int RMAX, int E, int NL, int STG = 0>
__device__ __forceinline__ void run_stages_lines(C (&v)[NL][E], decltype(C::x) *lines, int pitch, const C *twl,
                                                 int j) {
    using Real = decltype(C::x);
    constexpr int TPL = N / E;
    constexpr int NST = sched_nstages(N, RMAX);
    constexpr int R = sched_radix(N, RMAX, STG);
    constexpr int NS = sched_ns(N, RMAX, STG);
    constexpr int NB = E / R;
    if constexpr (STG > 0 && NS > 1) {
        constexpr int ROW = R + 1, LO = tw_lo_rows(N, RMAX, STG);
        constexpr int OFF = tw_stage_off(N, RMAX, STG);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int k = (j + i * TPL) & (NS - 1);
            const C *lo = twl + OFF + (k & 15) * ROW;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w = lo[r];
                if constexpr (NS > 16) w = cmul(w, twl[OFF + (LO + (k >> 4)) * ROW + r]);
#pragma unroll
                for (int l = 0; l < NL; ++l) v[l][i * R + r] = cmulc(v[l][i * R + r], w);
            }
        }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int i = 0; i < NB; ++i) dft<R>(&v[l][i * R]);
    if constexpr (STG + 1 < NST) {
        constexpr int R2 = sched_radix(N, RMAX, STG + 1), NB2 = E / R2;
        // Real parts, then imaginary parts (the second write reads only .y,
        // which the first read left alone).
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            if (STG > 0 || part > 0) __syncthreads(); // earlier readers of the arrays are done
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                Real *line = lines + l * pitch;
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const int b = j + i * TPL;
                    const int base = (b / NS) * NS * R + (b & (NS - 1));
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        line[lpad<N>(base + r * NS)] = part ? v[l][i * R + r].y : v[l][i * R + r].x;
                }
            }
            __syncthreads();
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const Real *line = lines + l * pitch;
#pragma unroll
                for (int i = 0; i < NB2; ++i) {
                    const int b = j + i * TPL;
#pragma unroll
                    for (int r = 0; r < R2; ++r) {
                        const Real x = line[lpad<N>(b + r * (N / R2))];
                        if (part) v[l][i * R2 + r].y = x;
                        else v[l][i * R2 + r].x = x;
                    }
                }
            }
        }
        run_stages_lines<C, N, RMAX, E, NL, STG + 1>(v, lines, pitch, twl, j);
    }
}

// ---------------------------------------------------------------------------
// Wavefront shuffles.  A 16 x 16 transpose across the 16 lanes of one DPP row
// (lanes 16k .. 16k+15): on entry lane j holds row j of a matrix M in
// v[0..16), on exit v[r] = M[r][j].  Four butterfly steps d = 1, 2, 4, 8; in
// step d, lanes j and j^d swap the eight entries whose register index
// differs from the lane index in bit d (lane j sends v[r | d] if bit d of j
// is clear, v[r] if it is set, and stores what it receives in the other
// slot).  Lane exchanges: DPP quad permutations for d = 1, 2, ds_swizzle
// (bit-mask mode, xor within 32 lanes) for d = 4, 8 -- no LDS storage and no
// barrier.
template <int D> __device__ __forceinline__ float xor_lanes(float x) {
    const int i = __builtin_bit_cast(int, x);
    if constexpr (D == 1) return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false));
    else if constexpr (D == 2) return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false));
    else if constexpr (D == 4) return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(i, 0x101F));
    else return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(i, 0x201F));
}
template <int D, typename C> __device__ __forceinline__ void transpose_step(C *v, int j) {
    const bool hi = (j & D) != 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        // the q-th register index with bit D clear, and its partner
        const int r = ((q & ~(D - 1)) << 1) | (q & (D - 1)), s = r | D;
        const C a = v[r], b = v[s];
        // selects on values (not on which register to write), so that the
        // array stays in registers
        const float sx = hi ? a.x : b.x, sy = hi ? a.y : b.y;
        const float rx = xor_lanes<D>(sx), ry = xor_lanes<D>(sy);
        v[r] = mk<C>(hi ? rx : a.x, hi ? ry : a.y);
        v[s] = mk<C>(hi ? b.x : rx, hi ? b.y : ry);
    }
}
template <typename C> __device__ __forceinline__ void transpose16_row(C *v, int j) {
    transpose_step<1>(v, j);
    transpose_step<2>(v, j);
    transpose_step<4>(v, j);
    transpose_step<8>(v, j);
}

// ---------------------------------------------------------------------------
// Precision forms on the matrix cores.  A radix-16 stage is, per group of 16
// butterflies, the product of the 16 x 16 DFT matrix with a 16 x 16 block of
// inputs.  With each complex input written as two real rows (row 2r its real
// part, row 2r + 1 its imaginary part) this is two real products Yr = Ar X,
// Yi = Ai X of a 16 x 32 matrix and the 32 x 16 block X -- one
// v_mfma_f32_16x16x32 each -- where Ar interleaves the columns Re F and
// -Im F, and Ai the columns Im F and Re F.
// FP16 / BF16 operands keep 11 / 8 significant bits, so both the DFT matrix
// and the inputs are split into a high and a low part, x = hi + lo, and the
// product is accumulated in FP32 as A_hi B_hi + A_hi B_lo + A_lo B_hi (the
// lo*lo term is below the FP32 rounding of the result).  FP16 inputs are
// scaled per butterfly by a power of two (exact) so that the largest of its
// 32 real parts lies in [2^14, 2^15): full use of the FP16 range, no
// overflow (|hi| < 65504); BF16 has the FP32 exponent range and is not
// scaled.
//
// Operand layout of v_mfma_f32_16x16x32 (checked on the device): lane l,
// element i holds A[l % 16][8(l/16) + i] and B[8(l/16) + i][l % 16]; the FP32
// result D[4(l/16) + i][l % 16] is element i of lane l.  The input block's
// rows and the matrix's rows are ordered so that lane row h = l/16 holds
// inputs h, h + 4, h + 8, h + 12 of butterfly l % 16 (row 8h + 2q + c of the
// block: component c of input h + 4q) and receives its outputs h, h + 4,
// h + 8, h + 12 (matrix row 4h + i computes output h + 4i): four 8-byte
// operand loads per lane, and the two rows of a 32-lane half address
// elements one input (or one output) stride apart.
enum { PREC_FP32 = 0, PREC_F16X2 = 1, PREC_BF16X2 = 2 };

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int PREC> struct MfmaOps;
template <> struct MfmaOps<PREC_F16X2> {
    using V = half8;
    using S = _Float16;
    static constexpr bool SCALE = true;
    __device__ static __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct MfmaOps<PREC_BF16X2> {
    using V = bf16x8;
    using S = __bf16;
    static constexpr bool SCALE = false;
    __device__ static __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// x = hi + lo in the operand type (lo rounds the remainder once more).
template <int PREC>
__device__ __forceinline__ void split_hilo(const float *x, typename MfmaOps<PREC>::V &hi, typename MfmaOps<PREC>::V &lo) {
    using V = typename MfmaOps<PREC>::V;
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    if constexpr (PREC == PREC_BF16X2) {
        // A BF16 value is the upper half of the FP32 value it stands for, so
        // the hi parts come back to FP32 by a shift or a mask of the packed
        // pair, not by converting each one again.
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const bf16x2 h = __builtin_convertvector((f32x2){x[i], x[i + 1]}, bf16x2);
            const uint32_t u = __builtin_bit_cast(uint32_t, h);
            const bf16x2 l = __builtin_convertvector(
                (f32x2){x[i] - __uint_as_float(u << 16), x[i + 1] - __uint_as_float(u & 0xffff0000u)}, bf16x2);
            hi[i] = h[0];
            hi[i + 1] = h[1];
            lo[i] = l[0];
            lo[i + 1] = l[1];
        }
    } else {
        // whole-vector conversions: two values per packed conversion, and the
        // remainders formed by mixed-precision FMAs from the FP16 hi parts
        typedef float f32x8 __attribute__((ext_vector_type(8)));
        f32x8 xv;
#pragma unroll
        for (int i = 0; i < 8; ++i) xv[i] = x[i];
        hi = __builtin_convertvector(xv, V);
        lo = __builtin_convertvector(xv - __builtin_convertvector(hi, f32x8), V);
    }
}

// This lane's share of the two DFT-matrix operands (forward sign), split
// into hi and lo parts: row m = l % 16, columns k = 8(l/16) + i.  The plan
// generates them once (dft_operand_table, FP64 angles rounded once to FP32,
// then split) and every workgroup loads its lanes' 64 bytes.
template <int PREC> struct DftOperands {
    using V = typename MfmaOps<PREC>::V;
    V rh, rl, ih, il;
    __device__ __forceinline__ DftOperands(int lane, const void *table) {
        const V *t = static_cast<const V *>(table) + 4 * lane;
        rh = t[0];
        rl = t[1];
        ih = t[2];
        il = t[3];
    }
};

// The operand table: entry 4*l + {0, 1, 2, 3} = lane l's {rh, rl, ih, il}.
// One wavefront of 64 threads.
template <int PREC> __global__ void dft_operand_table(typename MfmaOps<PREC>::V *out) {
    const int lane = threadIdx.x & 63;
    float ar[8], ai[8];
    const int m = lane & 15;
    // row m of the operand computes output o = m/4 + 4 (m mod 4); column
    // 8 (l/16) + i multiplies component i mod 2 of input l/16 + 4 (i/2)
    const int o = (m >> 2) + 4 * (m & 3);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = (lane >> 4) + 4 * (i >> 1), e = (o * r) & 15;
        double sn, cs;
        sincospi(double(e) / 8.0, &sn, &cs); // angle 2*pi*e/16
        // F[o][r] = cos - i sin;  Yr = sum cos Xr + sin Xi;  Yi = sum -sin Xr + cos Xi
        ar[i] = float((i & 1) == 0 ? cs : sn);
        ai[i] = float((i & 1) == 0 ? -sn : cs);
    }
    typename MfmaOps<PREC>::V rh, rl, ih, il;
    split_hilo<PREC>(ar, rh, rl);
    split_hilo<PREC>(ai, ih, il);
    out[4 * lane + 0] = rh;
    out[4 * lane + 1] = rl;
    out[4 * lane + 2] = ih;
    out[4 * lane + 3] = il;
}

// 4 x 4 transpose of 8-word blocks across the four 16-lane rows of a
// wavefront: lane (n, h) (row h = lane / 16) holds blocks x[0..3]; afterwards
// x[g] holds what was block h of lane (n, g).  Step one swaps blocks between
// the two 32-lane halves (v_permlane32_swap: rows 2, 3 of the first operand
// with rows 0, 1 of the second), step two between the rows of each half
// (v_permlane16_swap: odd rows of the first operand with even rows of the
// second).  The transpose is its own inverse.
__device__ __forceinline__ void row_transpose4(float (&x)[4][8]) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[d][f]), __float_as_uint(x[2 + d][f]),
                                                            false, false);
            x[d][f] = __uint_as_float(r[0]);
            x[2 + d][f] = __uint_as_float(r[1]);
        }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[2 * c][f]),
                                                            __float_as_uint(x[2 * c + 1][f]), false, false);
            x[2 * c][f] = __uint_as_float(r[0]);
            x[2 * c + 1][f] = __uint_as_float(r[1]);
        }
}

// One group of 16 radix-16 butterflies on the matrix cores: x is this lane's
// share of the input block (inputs h, h + 4, h + 8, h + 12 of butterfly
// l % 16, h = l/16, real and imaginary parts interleaved); on return yr[i],
// yi[i] hold output h + 4i of that butterfly, to be multiplied by
// `unscale`.
template <int PREC>
__device__ __forceinline__ void mfma_butterflies(float (&x)[8], const DftOperands<PREC> &F, f32x4 &yr, f32x4 &yi,
                                                 float &unscale) {
    using Ops = MfmaOps<PREC>;
    float scale = 1.f;
    unscale = 1.f;
    if constexpr (Ops::SCALE) {
        float mx = 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) mx = fmaxf(mx, fabsf(x[i]));
        // the butterfly's four lanes (n, n + 16, n + 32, n + 48): a swap of a
        // register with itself leaves both halves' values side by side
        const auto m32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(mx), __float_as_uint(mx), false, false);
        mx = fmaxf(__uint_as_float(m32[0]), __uint_as_float(m32[1]));
        const auto m16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(mx), __float_as_uint(mx), false, false);
        mx = fmaxf(__uint_as_float(m16[0]), __uint_as_float(m16[1]));
        if (mx > 0.f) {
            const int e = __builtin_amdgcn_frexp_expf(mx); // mx in [2^(e-1), 2^e)
            scale = __builtin_amdgcn_ldexpf(1.f, 15 - e);
            unscale = __builtin_amdgcn_ldexpf(1.f, e - 15);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] *= scale;
    }
    typename Ops::V bh, bl;
    split_hilo<PREC>(x, bh, bl);
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    yr = Ops::mma(F.rh, bh, z);
    yr = Ops::mma(F.rh, bl, yr);
    yr = Ops::mma(F.rl, bh, yr);
    yi = Ops::mma(F.ih, bh, z);
    yi = Ops::mma(F.ih, bl, yi);
    yi = Ops::mma(F.il, bh, yi);
}

// The whole radix-16 stage schedule of a tile on the matrix cores.  N is a
// power of 16 (every stage radix 16); each wave owns 64 butterflies per stage
// (four groups of 16).
//   v      on entry the thread's 16 inputs of stage 0 (slot r = element
//          j + r*N/16 of line c), on exit its 16 outputs in the same layout
//   tile   the LDS tile (complex elements, line pitch `pitch`); free on entry
//   twl    the stage twiddle tables (as for run_stages), written by the
//          caller and published by the first barrier here (as the caller's
//          weight table is) when there are two stages or more
// Thread t's (c, j) is (t mod T, t / T) when LINES_FIRST, else (t / (N/16),
// t mod N/16).  In the first and the last stage group g of a wave takes the
// butterflies of the wave's lanes 16g .. 16g + 15, so the operands of the
// first stage and the results of the last move between the thread layout and
// the matrix-core layout by a transpose across the wave's rows
// (row_transpose4), not through LDS; the stages in between take the tile's
// butterflies line by line.  Stage s writes output k of butterfly b to
// (b/NS)*NS*16 + b%NS + k*NS and applies there the twiddle the next stage
// would apply to that element.
template <int PREC, int N, bool LINES_FIRST>
__device__ __forceinline__ void mfma_stages(float2 *v, float2 *tile, int pitch, const float2 *twl, int log2T, int tid,
                                            const DftOperands<PREC> &F) {
    constexpr int TPL = N / 16, NST = sched_nstages(N, 16);
    static_assert(N >= 16 && ilog2c(N) % 4 == 0, "all stages radix 16");
    const int lane = tid & 63, wave = tid >> 6, hh = lane >> 4;
    // line and butterfly of group g in stage s
    auto butterfly = [&](int s, int g, int &cc, int &b) {
        const int t = 64 * wave + 16 * g + (lane & 15);
        if (s == 0 || s == NST - 1) {
            if constexpr (LINES_FIRST) {
                cc = t & ((1 << log2T) - 1);
                b = t >> log2T;
            } else {
                cc = t / TPL;
                b = t % TPL;
            }
        } else {
            cc = t / TPL;
            b = t % TPL;
        }
    };
    float x[4][8];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            x[h][2 * q] = v[h + 4 * q].x;
            x[h][2 * q + 1] = v[h + 4 * q].y;
        }
    row_transpose4(x);
#pragma unroll
    for (int s = 0; s < NST; ++s) {
        const int NS = 1 << (4 * s);
        if (s > 0) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                int cc, b;
                butterfly(s, g, cc, b);
                const float2 *ln = tile + cc * pitch;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float2 e = ln[lpad<N>(b + (hh + 4 * q) * TPL)];
                    x[g][2 * q] = e.x;
                    x[g][2 * q + 1] = e.y;
                }
            }
        }
        // The four groups' products, results in place of their operands
        // (still scaled when a twiddle follows: the twiddle takes `unscale`).
        float unscale[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            f32x4 yr, yi;
            mfma_butterflies<PREC>(x[g], F, yr, yi, unscale[g]);
            const float u = s + 1 < NST ? 1.f : unscale[g];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                x[g][2 * i] = yr[i] * u;
                x[g][2 * i + 1] = yi[i] * u;
            }
        }
        if (s + 1 < NST) {
            // Stage 0: the caller's LDS tables (twl, the weight table) are
            // published; later stages: every read of this stage precedes its
            // writes.
            __syncthreads();
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                int cc, b;
                butterfly(s, g, cc, b);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = hh + 4 * i, p = (b / NS) * NS * 16 + (b % NS) + k * NS;
                    // next stage's twiddle of element p: input r2 = p / TPL of
                    // butterfly b2 = p % TPL, exponent r2 * (b2 mod 16^(s+1))
                    const int NS2 = NS * 16, r2 = p / TPL, k2 = (p % TPL) & (NS2 - 1);
                    const int off = tw_stage_off(N, 16, s + 1);
                    float2 w = twl[off + (k2 & 15) * 17 + r2];
                    if (NS2 > 16) w = cmul(w, twl[off + (16 + (k2 >> 4)) * 17 + r2]);
                    w = mk<float2>(w.x * unscale[g], w.y * unscale[g]);
                    tile[cc * pitch + lpad<N>(p)] = cmulc(mk<float2>(x[g][2 * i], x[g][2 * i + 1]), w);
                }
            }
            __syncthreads(); // this stage's writes precede the next stage's reads
        }
    }
    row_transpose4(x);
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[h + 4 * q] = mk<float2>(x[h][2 * q], x[h][2 * q + 1]);
}

} // namespace liftfft
