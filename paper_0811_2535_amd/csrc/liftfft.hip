// libliftfft: plan, launch and C ABI of the dimension-lifted 1-D complex FFT
// for gfx950.  The ABI is declared (and documented) in include/liftfft.h.
//
// Kernels (all in this file, device code in fft_engine.hpp):
//   pass_kernel<K_SINGLE>  n up to one workgroup's line (2^14 complex64,
//                          2^13 complex128): a tile holds whole transforms;
//                          natural order in and out.
//   pass_kernel<K_PASS1>   block phase of the lift n = p*q (Section 4.2-4.7 of
//                          the paper, Fig. 4.8): for each j1 < p the q-point
//                          transform over j2 of x[j1 + p*j2]; then the
//                          inter-phase weight w_n^(-j1*k2) (the paper's
//                          weightcyclic factors, Section 4.5, Fig. 4.4) and a
//                          store into the slabs S[j1/W][k2][j1%W] of the
//                          scratch array (the block-to-cyclic
//                          redistribution, Fig. 5.3 / Fig. 5.9).
//   pass_kernel<K_PASS2>   cyclic phase (Section 4.6, Fig. 4.6): for each
//                          k2 < q the p-point transform over j1 of S, stored
//                          as X[k2 + q*k1] (natural order, the
//                          cyclic-to-centralized gather of Fig. 5.5).
//                          Variants of the pass kernels: values per thread,
//                          split exchange, persistent prefetch, register cap,
//                          and radix-16 stages on the matrix cores.
//   pass_kernel<K_AXIS>    one pass of the three-level lift n = n1*n2*n3
//                          (dimension lifting taken one level further,
//                          Section 1): transforms along one axis of x viewed
//                          as n3 x n2 x n1, each tile T adjacent lines of the
//                          contiguous axis, passes A and B with their
//                          inter-pass weights fused into the store;
//                          K_AXIS_WIDE is the same for transforms of 2^31
//                          bytes or more, addressed in 64 bits.
//   ragged_kernel          persistent pass 1 / pass 2 over the lifted length
//                          classes of a packed batch of uneven lengths.
//   twiddle_table_kernel   FP64 generation of the weight tables.
//   fill_pattern_kernel, compare_kernel   the autotuner's input and check.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "fft_engine.hpp"
#include "liftfft.h"
#include "paper_plan.hpp"

using namespace liftfft;

namespace {

enum Kind { K_SINGLE = 0, K_PASS1 = 1, K_PASS2 = 2, K_AXIS = 3, K_AXIS_WIDE = 4 };

constexpr int MAX_LOG2_LINE = 14; // longest line one workgroup transforms (complex64)
// Longest line per element type: 2^14 complex64 points (1024 threads of 16
// values, 139 KB of LDS for the complex exchange), 2^13 complex128 points
// (512 threads).  Two passes then reach 2^28 and 2^26.
constexpr int max_line(int dtype) { return dtype == 0 ? 14 : 13; }
template <typename Real> constexpr int max_line_of() { return sizeof(Real) == 4 ? 14 : 13; }
constexpr int64_t LDS_BUDGET = 160 * 1024; // bytes of LDS per workgroup on gfx950

struct PassArgs {
    const void *in;
    void *out;
    const void *tw;    // w_N^e, e < N (+1 root), N = this pass's line length
    const void *tw_hi; // weighted passes: w_n^(a * 2^log2h), a < n / 2^log2h
    const void *tw_lo; // weighted passes: w_n^b, b < 2^log2h
    int64_t lines;     // batch * lines per transform
    int64_t n;         // transform length
    int64_t ntiles;    // tiles of T lines
    int32_t log2p, log2q;
    int32_t log2T;  // lines per tile of this kernel
    int32_t log2T1; // scratch tile width W (lines of pass 1 per slab; divides pass 1's T)
    int32_t log2h;
    int32_t conj_in, conj_out;
    int32_t xcd_remap;
    // XCD-contiguous order with spread (0 = off): the tiles of an XCD's range
    // form groups of 2^tile_log2g adjacent tiles, and the groups that run at
    // the same time are 2^tile_log2s apart in the range instead of adjacent.
    int32_t tile_log2g, tile_log2s;
    int32_t pitch;  // exchange line pitch, in exchange elements
    const int64_t *offsets; // packed uneven batch: first element of each transform (else b*n)
    int64_t total;          // packed uneven batch: elements in the buffer
    const void *dft_ops;    // matrix-core forms: the DFT-matrix operand table
    // Axis passes of a three-level lift (K_AXIS, K_AXIS_WIDE).  Line l of a transform is
    // (lm, ld) = (l mod 2^ax_log2U, l div 2^ax_log2U); element i of the line
    // sits at (lm << ax_in[0]) + (ld << ax_in[1]) + (i << ax_in[2]) and
    // result k goes to the same form over ax_out.  ax_tw selects the fused
    // weight w_n^-(u (k0 + 2^ax_log2m k)): 0 none, 1 u = ld 2^ax_log2U and
    // k0 = 0, 2 u = lm and k0 = ld.
    int32_t ax_log2U, ax_log2L; // fast line axis; lines per transform
    int32_t ax_in[3], ax_out[3];
    int32_t ax_tw, ax_log2m;
};

// Workgroup g's k-th tile, or -1.  Workgroups are dispatched round-robin over
// the 8 XCDs; with the remap each XCD owns a contiguous range of tiles, so
// tiles that share cache lines (adjacent columns in pass 1, adjacent rows in
// pass 2) are in flight in the same L2 at the same time.  A persistent
// workgroup walks its XCD's range with stride (workgroups per XCD).
template <bool PERSIST> __device__ __forceinline__ int64_t tile_of(const PassArgs &a, int64_t k) {
    const int64_t g = blockIdx.x, G = gridDim.x;
    if constexpr (!PERSIST) {
        if (k) return -1;
        if (!a.xcd_remap) return g;
        const int64_t per = G >> 3, i = g >> 3; // G is a multiple of 8
        if (!a.tile_log2s) return (g & 7) * per + i;
        // per is a multiple of 2^(tile_log2g + tile_log2s): the range holds
        // 2^tile_log2s rows of `cols` groups, walked column by column
        const int gl = a.tile_log2g, sl = a.tile_log2s;
        const int64_t grp = i >> gl, cols = per >> (gl + sl);
        const int64_t loc = ((grp & ((1 << sl) - 1)) * cols + (grp >> sl)) << gl | (i & ((int64_t(1) << gl) - 1));
        return (g & 7) * per + loc;
    } else {
        if (a.xcd_remap) { // G and ntiles are multiples of 8
            const int64_t per = a.ntiles >> 3, loc = k * (G >> 3) + (g >> 3);
            return loc < per ? (g & 7) * per + loc : -1;
        }
        const int64_t t = k * G + g;
        return t < a.ntiles ? t : -1;
    }
}

// Largest workgroup: 1024 threads for complex64 with 16 values per thread;
// 512 (up to 256 VGPRs per lane) for complex128, for 32 values per thread
// and for persistent kernels, which hold the next tile in registers too.
// (With a 1024-thread bound the 32-value kernels were held to 128 VGPRs and
// spilled 130-180 bytes per lane.)
template <typename Real, int EMAX, bool PERSIST> constexpr int max_threads() {
    return sizeof(Real) == 4 && EMAX == 16 && !PERSIST ? 1024 : 512;
}
// Minimum waves per SIMD the register allocation must allow: 8 (64 VGPRs,
// two 1024-thread workgroups per CU) for the dense variants, else 1.
template <bool DENSE> constexpr int min_waves() { return DENSE ? 8 : 1; }

// Cache policies of the lifted passes' global accesses (the AUX field of the
// buffer instructions): pass-1 column loads, pass-1 scratch stores, pass-2
// scratch loads, pass-2 natural-order stores.
constexpr int CP_LOAD1 = 0, CP_STORE1 = 0, CP_LOAD2 = 0, CP_STORE2 = 0;

// The work of one workgroup on tiles of T lines of one kernel shape:
// loads, the pass-1 weights, the stage loop and the stores.  Shared by the
// pass kernels below and the ragged-batch kernel.  All data accesses go
// through buffer descriptors covering exactly the tile's range (for packed
// batches of uneven lengths, `a.offsets` gives each transform's first
// element and the single-pass descriptor covers the whole packed buffer).
//   EMAX   complex values per thread (16 or 32)
//   SPLIT  exchange real and imaginary parts in turn (half the LDS)
//   PREC   PREC_FP32: stages in FP32 on the vector units; PREC_F16X2 /
//          PREC_BF16X2: radix-16 stages on the matrix cores (mfma_stages)
struct NoOperands {
    __device__ __forceinline__ NoOperands(int, const void *) {}
};
template <typename Real, int N, int RMAX, int KIND, int EMAX, bool SPLIT, int PREC = PREC_FP32> struct Tile {
    using C = typename Cx<Real>::T;
    using L = typename std::conditional<SPLIT, Real, C>::type; // exchange element
    static constexpr uint32_t ES = sizeof(C);
    static constexpr int E = vals_per_thread(N, EMAX), TPL = N / E;
    static constexpr int NST = sched_nstages(N, RMAX);
    static constexpr int R0 = sched_radix(N, RMAX, 0), RL = sched_radix(N, RMAX, NST - 1);
    static constexpr bool TILE = uses_tile(N, RMAX);
    // Axis passes; the wide form addresses a transform of 2^31 bytes or more
    // through 64-bit global pointers instead of 32-bit buffer offsets.
    static constexpr bool AXIS = KIND == K_AXIS || KIND == K_AXIS_WIDE;
    static constexpr bool WIDE = KIND == K_AXIS_WIDE;

    const PassArgs &a;
    int log2T, T, tid, nthr, c, j;
    L *line;
    C *tile;
    typename std::conditional<PREC == PREC_FP32, NoOperands, DftOperands<PREC>>::type F;
    C *twl, *ep_base;
    Real sin_, sout;
    const C *__restrict__ in;
    C *__restrict__ out;
    int64_t pmask, qmask;

    __device__ __forceinline__ Tile(const PassArgs &args, unsigned char *smem)
        : a(args), F(int(threadIdx.x & 63), args.dft_ops) {
        log2T = a.log2T;
        T = 1 << log2T;
        tid = threadIdx.x;
        nthr = blockDim.x;
        if constexpr (KIND != K_SINGLE) {
            c = tid & (T - 1); // lanes sweep the lines first: adjacent columns / rows
            j = tid >> log2T;
        } else {
            j = tid & (TPL - 1); // lanes sweep one contiguous line first
            c = tid / TPL;
        }
        line = reinterpret_cast<L *>(smem) + c * a.pitch;
        tile = reinterpret_cast<C *>(smem);
        constexpr bool force = PREC != PREC_FP32;
        twl = reinterpret_cast<C *>(smem + lds_tile_bytes(N, RMAX, T, a.pitch, sizeof(L), force));
        ep_base = reinterpret_cast<C *>(smem + lds_ep_offset(N, RMAX, T, a.pitch, sizeof(L), sizeof(C), force));
        sin_ = a.conj_in ? Real(-1) : Real(1);
        sout = a.conj_out ? Real(-1) : Real(1);
        in = static_cast<const C *>(a.in);
        out = static_cast<C *>(a.out);
        pmask = (int64_t(1) << a.log2p) - 1;
        qmask = (int64_t(1) << a.log2q) - 1;
    }

    // First element of transform b.
    __device__ __forceinline__ int64_t base(int64_t b) const { return a.offsets ? a.offsets[b] : b * a.n; }

    // Single pass: descriptor and lane offset of this thread's line (the
    // tile's contiguous range, or the whole packed buffer).
    __device__ __forceinline__ void single_addr(int64_t line0, const C *buf, rsrc_t &r, uint32_t &lane) const {
        if (a.offsets) {
            r = make_rsrc(buf, uint32_t(a.total) * ES);
            lane = (uint32_t(a.offsets[line0 + c]) + uint32_t(j)) * ES;
        } else {
            const int64_t nl = a.lines - line0 < T ? a.lines - line0 : T;
            r = make_rsrc(buf + line0 * N, uint32_t(nl * N) * ES);
            lane = (uint32_t(c) * N + uint32_t(j)) * ES;
        }
    }

    // Axis passes: byte offset of this thread's element j of line c, within
    // its transform, for the stride triple `st` (fast line axis, slow line
    // axis, transform axis).  The plan keeps T | 2^ax_log2U, so the tile's
    // lines share one ld.
    __device__ __forceinline__ uint32_t axis_lane(int64_t line0, const int32_t *st) const {
        const uint32_t l = uint32_t(line0 & ((int64_t(1) << a.ax_log2L) - 1));
        const uint32_t lm = l & ((1u << a.ax_log2U) - 1), ld = l >> a.ax_log2U;
        return (((lm + uint32_t(c)) << st[0]) + (ld << st[1]) + (uint32_t(j) << st[2])) * ES;
    }
    // The same as an element offset in 64 bits (wide form).
    __device__ __forceinline__ int64_t axis_elem(int64_t line0, const int32_t *st) const {
        const int64_t l = line0 & ((int64_t(1) << a.ax_log2L) - 1);
        const int64_t lm = l & ((int64_t(1) << a.ax_log2U) - 1), ld = l >> a.ax_log2U;
        return ((lm + c) << st[0]) + (ld << st[1]) + (int64_t(j) << st[2]);
    }

    // Pass C of a three-level lift (contiguous rows, complex exchange, FP32
    // stages, one first-stage butterfly per thread): loaded row first.
    static constexpr bool ROWS_FIRST_KIND = KIND == K_AXIS && !SPLIT && PREC == PREC_FP32 && TILE && E == R0;
    __device__ __forceinline__ bool rows_first() const { return ROWS_FIRST_KIND && a.ax_in[2] == 0; }

    // Data loads of the tile starting at line0: a buffer descriptor, one
    // 32-bit lane offset, and a uniform per-slot offset.  Raw values: the
    // conjugation of sign +1 is applied by the caller, so that a prefetch is
    // not consumed (waited for) as soon as it is issued.
    __device__ __forceinline__ void load(int64_t line0, C *v) const {
        if (line0 + c >= a.lines) {
#pragma unroll
            for (int s = 0; s < E; ++s) v[s] = mk<C>(Real(0), Real(0));
            return;
        }
        if constexpr (KIND == K_SINGLE) {
            rsrc_t src;
            uint32_t lane;
            single_addr(line0, in, src, lane);
#pragma unroll
            for (int s = 0; s < E; ++s) v[s] = buf_load(in, src, lane, uint32_t(slot_off<N, E, R0>(s)) * ES);
        } else if constexpr (KIND == K_PASS1) {
            const int64_t b = line0 >> a.log2p, j10 = line0 & pmask;
            const rsrc_t src = make_rsrc(in + base(b) + j10, uint32_t(a.n - j10) * ES);
            const uint32_t lane = (uint32_t(c) + (uint32_t(j) << a.log2p)) * ES;
#pragma unroll
            for (int s = 0; s < E; ++s)
                v[s] = buf_load<CP_LOAD1>(in, src, lane, (uint32_t(slot_off<N, E, R0>(s)) << a.log2p) * ES);
        } else if constexpr (WIDE) {
            const C *src = in + base(line0 >> a.ax_log2L) + axis_elem(line0, a.ax_in);
#pragma unroll
            for (int s = 0; s < E; ++s) v[s] = src[int64_t(slot_off<N, E, R0>(s)) << a.ax_in[2]];
        } else if constexpr (KIND == K_AXIS) {
            const rsrc_t src = make_rsrc(in + base(line0 >> a.ax_log2L), uint32_t(a.n) * ES);
            if (rows_first()) {
                // Pass C's lines are contiguous rows: read them row first (a
                // wavefront instruction covers TPL consecutive elements of
                // each of 64/TPL lines instead of 64/T elements of each of T
                // lines).  Thread (cr, jr) = (tid / TPL, tid % TPL) holds the
                // inputs of the first stage's butterfly jr of line cr;
                // transform_store runs that stage in this layout and hands
                // the results to their line-first owners through the stage
                // exchange.
                const int cr = tid / TPL, jr = tid % TPL;
                const uint32_t l = uint32_t(line0 & ((int64_t(1) << a.ax_log2L) - 1));
                const uint32_t lm = l & ((1u << a.ax_log2U) - 1), ld = l >> a.ax_log2U;
                const uint32_t rlane = (((lm + uint32_t(cr)) << a.ax_in[0]) + (ld << a.ax_in[1]) + uint32_t(jr)) * ES;
#pragma unroll
                for (int s = 0; s < E; ++s) v[s] = buf_load(in, src, rlane, uint32_t(slot_off<N, E, R0>(s)) * ES);
                return;
            }
            const uint32_t lane = axis_lane(line0, a.ax_in);
#pragma unroll
            for (int s = 0; s < E; ++s)
                v[s] = buf_load(in, src, lane, (uint32_t(slot_off<N, E, R0>(s)) << a.ax_in[2]) * ES);
        } else {
            // Scratch layout S[j1/T1][k2][j1%T1]; the plan keeps T1 | TPL, so
            // j1 = j + off(s) with off(s) a multiple of T1.
            const int64_t b = line0 >> a.log2q, k20 = line0 & qmask;
            const int l2T1 = a.log2T1, T1 = 1 << l2T1;
            const rsrc_t src = make_rsrc(in + base(b) + (k20 << l2T1), uint32_t(a.n - (k20 << l2T1)) * ES);
            const uint32_t lane =
                ((uint32_t(j >> l2T1) << (a.log2q + l2T1)) + uint32_t(j & (T1 - 1)) + (uint32_t(c) << l2T1)) * ES;
#pragma unroll
            for (int s = 0; s < E; ++s)
                v[s] = buf_load<CP_LOAD2>(in, src, lane, (uint32_t(slot_off<N, E, R0>(s)) << a.log2q) * ES);
        }
    }

    __device__ __forceinline__ void conj_in(C *v) const {
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = scale_im(v[s], sin_);
    }

    // Stage weight tables into LDS (published by the first barrier of the
    // stage loop).
    __device__ __forceinline__ void fill_tw() const {
        if constexpr (TILE) fill_twiddles<C, N, RMAX>(twl, static_cast<const C *>(a.tw), tid, nthr);
    }

    // Weights fused into the store of pass 1 and of the weighted axis passes:
    // the factor of element (c, k = j + off(s)) is w_n^-(u(c) (k0 + m k)),
    // split as A = w_n^(u(c) (k0 + m j)) (per thread) times P[c][s] =
    // w_n^(u(c) m off(s)) (per line and slot, in the LDS buffer `ep`), each
    // from the two-level FP64-generated tables.  Pass 1: u = j1 (the column),
    // k0 = 0, m = 1.  Axis passes: as selected by ax_tw.  Exponents are
    // reduced mod n (a power of two) by unsigned wrap-around.  The LDS table
    // is published by the first barrier of the stage loop (or the explicit
    // one in transform_store when the schedule has one stage).
    static constexpr bool WEIGHTED = KIND == K_PASS1 || AXIS;
    __device__ __forceinline__ int weight_exponent(int j10, int cc, int s) const {
        return (j10 + cc) * ((s / RL) * TPL + (s % RL) * (N / RL));
    }
    struct WeightTerms {
        uint32_t u0, du, k0; // u(c) = u0 + du * c
    };
    __device__ __forceinline__ bool weighted() const { return KIND == K_PASS1 || (AXIS && a.ax_tw); }
    __device__ __forceinline__ WeightTerms weight_terms(int64_t line0) const {
        if constexpr (AXIS) {
            const uint32_t l = uint32_t(line0 & ((int64_t(1) << a.ax_log2L) - 1));
            const uint32_t lm = l & ((1u << a.ax_log2U) - 1), ld = l >> a.ax_log2U;
            return a.ax_tw == 2 ? WeightTerms{lm, 1u, ld} : WeightTerms{ld << a.ax_log2U, 0u, 0u};
        } else {
            return WeightTerms{uint32_t(line0 & pmask), 1u, 0u};
        }
    }
    __device__ __forceinline__ uint32_t exponent_A(const WeightTerms &w) const {
        const uint32_t m = AXIS ? uint32_t(a.ax_log2m) : 0u;
        return ((w.u0 + w.du * uint32_t(c)) * (w.k0 + (uint32_t(j) << m))) & uint32_t(a.n - 1);
    }
    __device__ __forceinline__ uint32_t exponent_P(const WeightTerms &w, int cc, int s) const {
        const uint32_t m = AXIS ? uint32_t(a.ax_log2m) : 0u;
        return ((w.u0 + w.du * uint32_t(cc)) * (uint32_t(slot_off<N, E, RL>(s)) << m)) & uint32_t(a.n - 1);
    }

    // Table entries of one tile (stage twiddles, weights), loaded into
    // registers before the tile's data and written to LDS after the data
    // loads are issued: global loads complete in order, so a table entry
    // loaded after the data (and consumed at once) would add its latency to
    // the data's.  The loads are unconditional (unused slots read entry 0)
    // so that the compiler's count of loads in flight stays exact.  Each
    // thread stages at most two entries of each table; the rest, if any, are
    // copied directly.
    struct TableRegs {
        C tw0, tw1, ahi, alo, ehi0, elo0, ehi1, elo1; // scalars: kept in registers
    };
    __device__ __forceinline__ int tw_slot(int k) const {
        const int i = tid + k * nthr;
        return i < tw_total(N, RMAX) ? tw_source<N, RMAX>(i) : -1;
    }
    __device__ __forceinline__ bool ep_slot(int k, int &cc, int &s) const {
        const int i = tid + k * nthr;
        cc = i / (E + 1);
        s = i - cc * (E + 1);
        return i < T * (E + 1) && s < E;
    }
    __device__ __forceinline__ void fetch_tables(int64_t line0, TableRegs &r) const {
        if constexpr (TILE) {
            const C *__restrict__ tw = static_cast<const C *>(a.tw);
            const int g0 = tw_slot(0), g1 = tw_slot(1);
            r.tw0 = tw[g0 < 0 ? 0 : g0];
            r.tw1 = tw[g1 < 0 ? 0 : g1];
        }
        if constexpr (WEIGHTED) {
            const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
            const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
            const uint32_t lomask = (1u << a.log2h) - 1;
            const WeightTerms w = weight_terms(line0);
            const uint32_t xa = exponent_A(w);
            r.ahi = hi[xa >> a.log2h];
            r.alo = lo[xa & lomask];
            int cc, s;
            const uint32_t x0 = ep_slot(0, cc, s) ? exponent_P(w, cc, s) : 0u;
            const uint32_t x1 = ep_slot(1, cc, s) ? exponent_P(w, cc, s) : 0u;
            r.ehi0 = hi[x0 >> a.log2h];
            r.elo0 = lo[x0 & lomask];
            r.ehi1 = hi[x1 >> a.log2h];
            r.elo1 = lo[x1 & lomask];
        }
    }
    // The same tables without staging, in the order the data arrives (for
    // kernels without registers to spare: complex128 tiles and the uneven-
    // batch kernel); returns A.
    __device__ __forceinline__ C direct_tables(int64_t line0, C *ep) const {
        if constexpr (TILE) fill_twiddles<C, N, RMAX>(twl, static_cast<const C *>(a.tw), tid, nthr);
        C A = mk<C>(Real(1), Real(0));
        if constexpr (WEIGHTED) {
            if (weighted()) {
                const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
                const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
                const uint32_t lomask = (1u << a.log2h) - 1;
                const WeightTerms w = weight_terms(line0);
                const uint32_t xa = exponent_A(w);
                A = cmul(hi[xa >> a.log2h], lo[xa & lomask]);
                for (int i = tid; i < T * (E + 1); i += nthr) {
                    const int c2 = i / (E + 1), s2 = i - c2 * (E + 1);
                    if (s2 >= E) continue;
                    const uint32_t x = exponent_P(w, c2, s2);
                    ep[i] = cmul(hi[x >> a.log2h], lo[x & lomask]);
                }
            }
        }
        return A;
    }
    // Write the staged entries (and any remaining ones) to LDS; returns A.
    __device__ __forceinline__ C publish_tables(int64_t line0, const TableRegs &r, C *ep) const {
        if constexpr (TILE) {
            const int g0 = tw_slot(0), g1 = tw_slot(1);
            if (g0 >= 0) twl[tid] = r.tw0;
            if (g1 >= 0) twl[tid + nthr] = r.tw1;
            if (2 * nthr < tw_total(N, RMAX))
                fill_twiddles<C, N, RMAX>(twl, static_cast<const C *>(a.tw), tid, nthr, 2 * nthr);
        }
        C A = mk<C>(Real(1), Real(0));
        if constexpr (WEIGHTED) {
            if (weighted()) {
                int cc, s;
                if (ep_slot(0, cc, s)) ep[tid] = cmul(r.ehi0, r.elo0);
                if (ep_slot(1, cc, s)) ep[tid + nthr] = cmul(r.ehi1, r.elo1);
                if (2 * nthr < T * (E + 1)) {
                    const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
                    const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
                    const uint32_t lomask = (1u << a.log2h) - 1;
                    const WeightTerms w = weight_terms(line0);
                    for (int i = tid + 2 * nthr; i < T * (E + 1); i += nthr) {
                        const int c2 = i / (E + 1), s2 = i - c2 * (E + 1);
                        if (s2 >= E) continue;
                        const uint32_t x = exponent_P(w, c2, s2);
                        ep[i] = cmul(hi[x >> a.log2h], lo[x & lomask]);
                    }
                }
                A = cmul(r.ahi, r.alo);
            }
        }
        return A;
    }

    // Transform the tile held in v and store it; `ep` and `A` are this
    // tile's pass-1 weights.
    __device__ __forceinline__ void transform_store(int64_t line0, C *v, const C *ep, C A) const {
        const bool active = line0 + c < a.lines;
        if constexpr ((KIND == K_PASS1 || AXIS) && !TILE) __syncthreads();

        if constexpr (ROWS_FIRST_KIND) {
            if (rows_first()) {
                // First stage (no twiddles) on the row-first layout of load():
                // butterfly jr of line cr writes output r to element 16 jr + r
                // of its line, then every thread reads its line-first inputs
                // of stage 1 and the stage loop continues from there.  Every
                // thread reaches the barrier: axis tiles are whole.
                const int cr = tid / TPL, jr = tid % TPL;
                dft<R0>(v);
                C *wl = tile + cr * a.pitch;
#pragma unroll
                for (int r = 0; r < R0; ++r) wl[lpad<N>(jr * R0 + r)] = v[r];
                __syncthreads();
                constexpr int R1 = sched_radix(N, RMAX, 1), NB1 = E / R1;
                const C *ln = tile + c * a.pitch;
#pragma unroll
                for (int i = 0; i < NB1; ++i) {
                    const int b = j + i * TPL;
#pragma unroll
                    for (int r = 0; r < R1; ++r) v[i * R1 + r] = ln[lpad<N>(b + r * (N / R1))];
                }
                run_stages<C, N, RMAX, E, SPLIT, 1>(v, line, twl, j);
            } else {
                run_stages<C, N, RMAX, E, SPLIT>(v, line, twl, j);
            }
        } else if constexpr (PREC == PREC_FP32) {
            run_stages<C, N, RMAX, E, SPLIT>(v, line, twl, j);
        } else {
            mfma_stages<PREC, N, KIND != K_SINGLE>(v, tile, a.pitch, twl, log2T, tid, F);
        }

        if (!active) return;
        if constexpr (KIND == K_SINGLE) {
            rsrc_t dst;
            uint32_t lane;
            single_addr(line0, out, dst, lane);
#pragma unroll
            for (int s = 0; s < E; ++s)
                buf_store(scale_im(v[s], sout), dst, lane, uint32_t(slot_off<N, E, RL>(s)) * ES);
        } else if constexpr (KIND == K_PASS1) {
            // Slabs of the scratch array S[j1/W][k2][j1%W], W = 2^log2T1: the
            // tile spans T/W whole slabs (W <= T) or T columns of one slab.
            const int64_t b = line0 >> a.log2p, j10 = line0 & pmask;
            const int lW = a.log2T1;
            rsrc_t dst;
            uint32_t lane;
            if (lW <= log2T) {
                dst = make_rsrc(out + base(b) + (j10 << a.log2q), uint32_t(T << a.log2q) * ES);
                lane = ((uint32_t(c >> lW) << (a.log2q + lW)) + (uint32_t(j) << lW) + uint32_t(c & ((1 << lW) - 1))) *
                       ES;
            } else {
                dst = make_rsrc(out + base(b) + ((j10 >> lW) << (a.log2q + lW)), uint32_t(1u << (a.log2q + lW)) * ES);
                lane = (uint32_t(j10 & ((1 << lW) - 1)) + uint32_t(c) + (uint32_t(j) << lW)) * ES;
            }
            const C *P = ep + c * (E + 1);
#pragma unroll
            for (int s = 0; s < E; ++s)
                buf_store<CP_STORE1>(cmulc(v[s], cmul(A, P[s])), dst, lane, (uint32_t(slot_off<N, E, RL>(s)) << lW) * ES);
        } else if constexpr (WIDE) {
            C *dst = out + base(line0 >> a.ax_log2L) + axis_elem(line0, a.ax_out);
            if (a.ax_tw) {
                const C *P = ep + c * (E + 1);
#pragma unroll
                for (int s = 0; s < E; ++s)
                    global_store(dst + (int64_t(slot_off<N, E, RL>(s)) << a.ax_out[2]), cmulc(v[s], cmul(A, P[s])));
            } else {
#pragma unroll
                for (int s = 0; s < E; ++s)
                    global_store(dst + (int64_t(slot_off<N, E, RL>(s)) << a.ax_out[2]), scale_im(v[s], sout));
            }
        } else if constexpr (KIND == K_AXIS) {
            const rsrc_t dst = make_rsrc(out + base(line0 >> a.ax_log2L), uint32_t(a.n) * ES);
            const uint32_t lane = axis_lane(line0, a.ax_out);
            if (a.ax_tw) {
                const C *P = ep + c * (E + 1);
#pragma unroll
                for (int s = 0; s < E; ++s)
                    buf_store(cmulc(v[s], cmul(A, P[s])), dst, lane,
                              (uint32_t(slot_off<N, E, RL>(s)) << a.ax_out[2]) * ES);
            } else {
#pragma unroll
                for (int s = 0; s < E; ++s)
                    buf_store(scale_im(v[s], sout), dst, lane, (uint32_t(slot_off<N, E, RL>(s)) << a.ax_out[2]) * ES);
            }
        } else {
            const int64_t b = line0 >> a.log2q, k20 = line0 & qmask;
            const rsrc_t dst = make_rsrc(out + base(b) + k20, uint32_t(a.n - k20) * ES);
            const uint32_t lane = (uint32_t(c) + (uint32_t(j) << a.log2q)) * ES;
#pragma unroll
            for (int s = 0; s < E; ++s)
                buf_store<CP_STORE2>(scale_im(v[s], sout), dst, lane, (uint32_t(slot_off<N, E, RL>(s)) << a.log2q) * ES);
        }
    }

    // One tile, start to finish (the caller orders it after any earlier
    // readers of the LDS).
    // STAGE: table entries staged in registers ahead of the data (complex64
    // pass kernels with 16 values per thread); else loaded after it (kernels
    // whose staged entries would be spilled to scratch memory: complex128
    // tiles, 32 values per thread, the 64-VGPR cap, the uneven-batch kernel).
    template <bool STAGE> __device__ __forceinline__ void run_one(int64_t t) const {
        C v[E];
        C A;
        if constexpr (STAGE) {
            TableRegs r;
            fetch_tables(t << log2T, r);
            load(t << log2T, v);
            A = publish_tables(t << log2T, r, ep_base);
            conj_in(v);
        } else {
            load(t << log2T, v);
            conj_in(v);
            A = direct_tables(t << log2T, ep_base);
        }
        transform_store(t << log2T, v, ep_base, A);
    }
};

// One launch of a pass.  Each workgroup transforms one tile, or (PERSIST) a
// sequence of tiles with the loads of the next tile issued before the current
// one is transformed.
//   DENSE  registers capped at 64 VGPRs so that two 1024-thread
//          workgroups share a CU
template <typename Real, int N, int RMAX, int KIND, int EMAX, bool SPLIT, bool PERSIST, bool DENSE,
          int PREC = PREC_FP32>
__global__ __launch_bounds__((max_threads<Real, EMAX, PERSIST>()), (min_waves<DENSE>())) void pass_kernel(
    PassArgs a) {
    using W = Tile<Real, N, RMAX, KIND, EMAX, SPLIT, PREC>;
    using C = typename W::C;
    constexpr int E = W::E, TPL = W::TPL, RL = W::RL;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const W w(a, smem_raw);

    int64_t t = tile_of<PERSIST>(a, 0);
    if (t < 0) return; // workgroup-uniform
    if constexpr (!PERSIST) {
        // 32 values per thread and the 64-VGPR cap leave no registers to stage tables in
        w.template run_one<sizeof(Real) == 4 && EMAX == 16 && !DENSE>(t);
    } else {
        const int log2T = w.log2T, T = w.T, tid = w.tid, nthr = w.nthr;
        C v[E];
        w.load(t << log2T, v);
#pragma unroll
        for (int s = 0; s < E; ++s) {
            v[s] = scale_im(v[s], w.sin_);
            // Materialise the first tile here: without this the conjugation
            // is merged into the loop below, and the wait for the first
            // tile's loads then also waits for every later prefetch.
            __asm__ volatile("" : "+v"(v[s].x), "+v"(v[s].y));
        }
        w.fill_tw();
        // The next tile's data and pass-1 weight inputs are loaded before this
        // tile is transformed and consumed only after its stores are issued:
        // loads complete in order, so any earlier use would also wait for them.
        // Each thread fetches at most EPT entries of the weight table.
        constexpr int EPT = 2;
        static_assert(KIND != K_PASS1 || E * (E + 1) <= EPT * N, "weight entries per thread");
        struct WeightLoads {
            C ahi, alo, ehi[EPT], elo[EPT];
        } wl;
        auto fetch_weights = [&](int64_t line0) {
            if constexpr (KIND == K_PASS1) {
                const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
                const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
                const int lomask = (1 << a.log2h) - 1;
                const int j10 = int(line0 & w.pmask);
                const int xa = (j10 + w.c) * w.j;
                wl.ahi = hi[xa >> a.log2h];
                wl.alo = lo[xa & lomask];
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const int i = tid + e * nthr, cc = i / (E + 1), s = i - cc * (E + 1);
                    if (i < T * (E + 1) && s < E) {
                        const int x = w.weight_exponent(j10, cc, s);
                        wl.ehi[e] = hi[x >> a.log2h];
                        wl.elo[e] = lo[x & lomask];
                    }
                }
            }
        };
        auto publish_weights = [&](C *ep) -> C {
            if constexpr (KIND != K_PASS1) {
                return mk<C>(Real(1), Real(0));
            } else {
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const int i = tid + e * nthr, s = i % (E + 1);
                    if (i < T * (E + 1) && s < E) ep[i] = cmul(wl.ehi[e], wl.elo[e]);
                }
                return cmul(wl.ahi, wl.alo);
            }
        };
        (void)TPL;
        (void)RL;
        C nxt[E];
        fetch_weights(t << log2T);
        C A = publish_weights(w.ep_base);
        for (int64_t k = 0;; ++k) {
            const int64_t tn = tile_of<PERSIST>(a, k + 1);
            if (tn >= 0) { // in flight while this tile is transformed
                fetch_weights(tn << log2T);
                w.load(tn << log2T, nxt);
            }
            if (k > 0) __syncthreads(); // the previous tile's LDS readers are done
            w.transform_store(t << log2T, v, w.ep_base + (k & 1) * T * (E + 1), A);
            if (tn < 0) break;
#pragma unroll
            for (int s = 0; s < E; ++s) v[s] = scale_im(nxt[s], w.sin_);
            // Buffer (k+1)&1 was last read by the stores of tile k-1, which
            // precede this tile's barriers.
            A = publish_weights(w.ep_base + ((k + 1) & 1) * T * (E + 1));
            t = tn;
        }
    }
}

// ---------------------------------------------------------------------------
// Axis pass of a three-level lift with 256-point lines (complex64) whose
// stage exchange is done by wavefront shuffles instead of the LDS tile.  A
// workgroup of 256 threads takes 16 adjacent lines; thread (c, j) = (tid >> 4,
// tid & 15) holds elements j + 16 r (r < 16) of line c, so each line's 16
// threads are one 16-lane DPP row.  Stage 0 is butterfly j's 16-point DFT;
// element 16 j' + r of its output is input r' = j' of stage 1's butterfly r,
// which a 16 x 16 transpose within the row (transpose16_row) delivers; stage
// 1 (twiddles w_256^(-r j), 16-point DFT) leaves output k = j + 16 r in v[r].
// LDS holds only the stage twiddles and the per-line weight factors.  The
// same loads, weights and stores as the LDS-tile axis kernel, with lanes
// sweeping a line's elements first instead of the lines first.
constexpr int SHUF_N = 256, SHUF_T = 16, SHUF_THREADS = 256;

__global__ __launch_bounds__(SHUF_THREADS) void axis_shuffle_kernel(PassArgs a) {
    using C = float2;
    constexpr uint32_t ES = sizeof(C);
    __shared__ C twl[SHUF_N];         // w_256^e, e < 256 (+1 root)
    __shared__ C ep[SHUF_T * 16];     // P[c][r] = w_n^(u(c) m 16 r)
    const int64_t t = tile_of<false>(a, 0);
    if (t < 0) return;
    const int tid = threadIdx.x, c = tid >> 4, j = tid & 15;
    const int64_t line0 = t * SHUF_T;
    const int64_t b = line0 >> a.ax_log2L;
    const uint32_t l = uint32_t(line0 & ((int64_t(1) << a.ax_log2L) - 1));
    const uint32_t lm = l & ((1u << a.ax_log2U) - 1), ld = l >> a.ax_log2U;
    const C *in = static_cast<const C *>(a.in) + b * a.n;
    C *out = static_cast<C *>(a.out) + b * a.n;
    const rsrc_t src = make_rsrc(in, uint32_t(a.n) * ES), dst = make_rsrc(out, uint32_t(a.n) * ES);
    auto lane_off = [&](const int32_t *st) {
        return (((lm + uint32_t(c)) << st[0]) + (ld << st[1]) + (uint32_t(j) << st[2])) * ES;
    };
    // Table entries first (loads complete in order), then the data.
    const C *__restrict__ tw = static_cast<const C *>(a.tw);
    const C tw_own = tw[tid];
    const bool weighted = a.ax_tw != 0;
    uint32_t u0 = 0, du = 0, k0 = 0;
    if (a.ax_tw == 2) {
        u0 = lm;
        du = 1;
        k0 = ld;
    } else if (a.ax_tw == 1) {
        u0 = ld << a.ax_log2U;
    }
    const uint32_t m = uint32_t(a.ax_log2m), nmask = uint32_t(a.n - 1), lomask = (1u << a.log2h) - 1;
    const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
    const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
    // A = w_n^(u(c) (k0 + m j)) for this thread; P entry (cp, rp) = (tid >> 4, tid & 15).
    const uint32_t xa = weighted ? ((u0 + du * uint32_t(c)) * (k0 + (uint32_t(j) << m))) & nmask : 0u;
    const uint32_t xp = weighted ? ((u0 + du * uint32_t(c)) * (uint32_t(16 * j) << m)) & nmask : 0u;
    const C ahi = hi[xa >> a.log2h], alo = lo[xa & lomask], phi = hi[xp >> a.log2h], plo = lo[xp & lomask];
    C v[16];
    const uint32_t li = lane_off(a.ax_in);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = buf_load(in, src, li, (uint32_t(16 * r) << a.ax_in[2]) * ES);
    twl[tid] = tw_own;
    ep[tid] = cmul(phi, plo); // entry (c, r = j)
    const C A = cmul(ahi, alo);
    const float sin_ = a.conj_in ? -1.f : 1.f, sout = a.conj_out ? -1.f : 1.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = scale_im(v[r], sin_);
    dft16(v);
    transpose16_row(v, j);
    __syncthreads(); // twl and ep published
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmulc(v[r], twl[r * j]);
    dft16(v);
    const uint32_t lo_off = lane_off(a.ax_out);
    if (weighted) {
        const C *P = ep + c * 16;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            buf_store(cmulc(v[r], cmul(A, P[r])), dst, lo_off, (uint32_t(16 * r) << a.ax_out[2]) * ES);
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            buf_store(scale_im(v[r], sout), dst, lo_off, (uint32_t(16 * r) << a.ax_out[2]) * ES);
    }
}

// ---------------------------------------------------------------------------
// Pass 1 of the two-level lift with the next tile staged in LDS by direct
// global-to-LDS loads (gfx950 global_load_lds_dwordx4), for complex64 columns
// of 4096 points, 2 columns per tile.  One persistent workgroup per CU walks
// its tiles; while tile k is transformed in registers (its stage exchange in
// the LDS buffer it arrived in), tile k+1 streams into the other buffer
// without occupying registers.  Row r of a staged tile is the 16-byte pair of
// the tile's two columns at row r.  Barriers inside the loop wait for LDS
// only (lds_barrier): a workgroup barrier with a memory fence would also wait
// for the staged loads in flight.  One wait for vector memory per tile, after
// the transform and before the stores: it covers the next tile's staged
// loads and the previous tile's stores, both issued a whole transform
// earlier.  The next tile's weight inputs are loaded just before that wait
// (a register load waited for later would also wait for what was issued
// after it), and the transform's base is computed, not loaded.
constexpr int DMA_N = 4096, DMA_T = 2, DMA_THREADS = 512, DMA_E = 16, DMA_TPL = DMA_N / DMA_E;
constexpr int DMA_ROWS_PER_OP = 64, DMA_WAVES = DMA_THREADS / 64;
constexpr int DMA_OPS = DMA_N / (DMA_ROWS_PER_OP * DMA_WAVES); // per wave per tile
constexpr int DMA_EP = DMA_T * (DMA_E + 1);

// Wait for every vector memory operation of this wave (the staged tile's
// direct-to-LDS loads among them).
__device__ __forceinline__ void wait_vmem() { __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__global__ __launch_bounds__(DMA_THREADS, 1) void pass1_dma_kernel(PassArgs a) {
    using C = float2;
    constexpr uint32_t ES = sizeof(C);
    __shared__ float4 buf0[DMA_N], buf1[DMA_N];
    __shared__ C twl[tw_total(DMA_N, 16)];
    __shared__ C ep[2][DMA_EP];
    const int tid = threadIdx.x, c = tid & (DMA_T - 1), j = tid >> 1;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const C *__restrict__ in = static_cast<const C *>(a.in);
    C *__restrict__ out = static_cast<C *>(a.out);
    const int64_t pmask = (int64_t(1) << a.log2p) - 1;
    const int64_t P = int64_t(1) << a.log2p;
    const float sin_ = a.conj_in ? -1.f : 1.f;
    const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
    const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
    const uint32_t lomask = (1u << a.log2h) - 1, nmask = uint32_t(a.n - 1);
    // Stage `t`'s rows into `dst`: wave w's op i covers rows (8i + w)*64 + lane.
    auto stage = [&](int64_t t, float4 *dst) {
        const int64_t line0 = t * DMA_T, b = line0 >> a.log2p, j10 = line0 & pmask;
        const C *col = in + b * a.n + j10; // single-length plans only (no packed offsets)
#pragma unroll
        for (int i = 0; i < DMA_OPS; ++i) {
            const int row0 = (i * DMA_WAVES + wave) * DMA_ROWS_PER_OP;
            __builtin_amdgcn_global_load_lds(col + int64_t(row0 + lane) * P, dst + row0, 16, 0, 0);
        }
    };
    // Weight inputs of tile `t`: this thread's base entry w^(j1 * j) and, for
    // the first DMA_EP threads, the per-row factors w^(j1 * 256 s) (last slot
    // of each column unused).
    const int ei = tid < DMA_EP ? tid : 0;
    const int ec = ei / (DMA_E + 1), es = ei - ec * (DMA_E + 1);
    const bool ep_writer = tid < DMA_EP && es < DMA_E;
    C ahi, alo, phi, plo;
    auto load_weights = [&](int64_t t) {
        const int64_t j10 = (t * DMA_T) & pmask;
        const uint32_t xa = (uint32_t(j10 + c) * uint32_t(j)) & nmask;
        const uint32_t xp = es < DMA_E ? (uint32_t(j10 + ec) * uint32_t(es * DMA_TPL)) & nmask : 0u;
        ahi = hi[xa >> a.log2h];
        alo = lo[xa & lomask];
        phi = hi[xp >> a.log2h];
        plo = lo[xp & lomask];
    };
    int64_t t = tile_of<true>(a, 0);
    if (t < 0) return; // workgroup-uniform
    stage(t, buf0);
    fill_twiddles<C, DMA_N, 16>(twl, static_cast<const C *>(a.tw), tid, DMA_THREADS);
    load_weights(t);
    wait_vmem();
    lds_barrier(); // the first staged tile and twl are in LDS
    C A = cmul(ahi, alo);
    if (ep_writer) ep[0][tid] = cmul(phi, plo);
    for (int64_t k = 0;; ++k) {
        float4 *cur = (k & 1) ? buf1 : buf0, *nxt = (k & 1) ? buf0 : buf1;
        const int64_t line0 = t * DMA_T, b = line0 >> a.log2p, j10 = line0 & pmask;
        C v[DMA_E];
        const float2 *rows = reinterpret_cast<const float2 *>(cur);
#pragma unroll
        for (int s = 0; s < DMA_E; ++s) v[s] = scale_im(rows[2 * (j + s * DMA_TPL) + c], sin_);
        // Every wave has read `cur` (it becomes this tile's exchange array) and
        // finished the previous tile (its exchange array `nxt` is free); this
        // tile's ep entries are published.
        lds_barrier();
        const int64_t tn = tile_of<true>(a, k + 1);
        if (tn >= 0) stage(tn, nxt);
        float *xline = reinterpret_cast<float *>(cur) + c * a.pitch;
        run_stages<C, DMA_N, 16, DMA_E, true, 0, true>(v, xline, twl, j);
        if (tn >= 0) load_weights(tn);
        wait_vmem();
        lds_barrier(); // the next tile is staged (every wave's part)
        C An = cmul(ahi, alo);
        // Keep the weight products ahead of the stores: a use of the loaded
        // weights placed among the stores would wait for the stores before it.
        __asm__ volatile("" : "+v"(An.x), "+v"(An.y));
        if (tn >= 0 && ep_writer) ep[(k + 1) & 1][tid] = cmul(phi, plo);
        // Store into the scratch slabs S[j1/2][k2][j1%2] (slab width 2 = T).
        const rsrc_t dst = make_rsrc(out + b * a.n + (j10 << a.log2q), uint32_t(DMA_T << a.log2q) * ES);
        const uint32_t lane_off = ((uint32_t(j) << 1) + uint32_t(c)) * ES;
        const C *Pc = ep[k & 1] + c * (DMA_E + 1);
#pragma unroll
        for (int s = 0; s < DMA_E; ++s)
            buf_store(cmulc(v[s], cmul(A, Pc[s])), dst, lane_off, (uint32_t(s * DMA_TPL) << 1) * ES);
        if (tn < 0) break;
        A = An;
        t = tn;
    }
}

// ---------------------------------------------------------------------------
// Pass 1 over 4096-point complex64 columns, two columns per tile, with each
// thread owning whole rows of the tile: with E values per column, thread j
// (N / E threads) loads the two columns' elements of rows j + (N / E) s
// (s < E), one 16-byte load per row, and runs butterfly j of both columns
// through a radix-E stage schedule (run_stages_lines: one split-exchange
// array per column, one barrier pair per exchange for both).  A wavefront
// load instruction then covers 64 rows of the tile, where the generic pass 1
// (two threads per row, one per column) covers 32; the tile, the weights and
// the scratch layout are the same (slabs S[j1/2][k2][j1%2]), and each row of
// a slab is stored as two 8-byte halves.  E = 16: 256 threads, radix 16;
// E = 8: 512 threads, radix 8 (four stages, the same data registers per
// thread as the generic kernel).  Selected by FFT_OPT_ROW_LANES only: at
// n = 2^24 both forms measured slower than the generic pass 1 (the 16-row
// form holds 168 VGPRs, three 256-thread workgroups per CU; the 8-row form
// stores its rows as 8-byte halves, a slower traversal).
constexpr int ROWS_N = 4096, ROWS_T = 2;
template <int E> constexpr int rows_threads() { return ROWS_N / E; }

template <int E>
__global__ __launch_bounds__(rows_threads<E>()) void pass1_rows_kernel(PassArgs a) {
    using C = float2;
    constexpr uint32_t ES = sizeof(C);
    constexpr int N = ROWS_N, T = ROWS_T, TPL = N / E, NTHR = TPL, RMAX = E;
    constexpr int TW = tw_total(N, RMAX), TW_PER = (TW + NTHR - 1) / NTHR, EP = T * (E + 1);
    static_assert(EP <= NTHR, "one weight factor per thread");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int64_t t = tile_of<false>(a, 0);
    if (t < 0) return; // workgroup-uniform
    float *xch = reinterpret_cast<float *>(smem_raw);
    C *twl = reinterpret_cast<C *>(smem_raw + lds_tile_bytes(N, RMAX, T, a.pitch, sizeof(float)));
    C *ep = reinterpret_cast<C *>(smem_raw + lds_ep_offset(N, RMAX, T, a.pitch, sizeof(float), sizeof(C)));
    const int tid = threadIdx.x, j = tid;
    const C *__restrict__ in = static_cast<const C *>(a.in);
    C *__restrict__ out = static_cast<C *>(a.out);
    const C *__restrict__ tw = static_cast<const C *>(a.tw);
    const C *__restrict__ hi = static_cast<const C *>(a.tw_hi);
    const C *__restrict__ lo = static_cast<const C *>(a.tw_lo);
    const int64_t pmask = (int64_t(1) << a.log2p) - 1;
    const int64_t line0 = t * T, b = line0 >> a.log2p, j10 = line0 & pmask;
    const int64_t tb = a.offsets ? a.offsets[b] : b * a.n; // first element of transform b
    const uint32_t lomask = (1u << a.log2h) - 1, nmask = uint32_t(a.n - 1);

    // Table entries first (global loads complete in order, so an entry
    // loaded after the data would wait for it): stage twiddles, this
    // thread's weights w_n^(j1 j) of both columns, and one per-slot factor
    // w_n^(j1 TPL s) (thread c (E + 1) + s; the last slot of each column is
    // padding).  Unused slots read entry 0.
    C twr[TW_PER];
#pragma unroll
    for (int k = 0; k < TW_PER; ++k) {
        const int i = tid + k * NTHR, g = i < TW ? tw_source<N, RMAX>(i) : -1;
        twr[k] = tw[g < 0 ? 0 : g];
    }
    C ahi[T], alo[T];
#pragma unroll
    for (int c = 0; c < T; ++c) {
        const uint32_t xa = (uint32_t(j10 + c) * uint32_t(j)) & nmask;
        ahi[c] = hi[xa >> a.log2h];
        alo[c] = lo[xa & lomask];
    }
    const int ec = tid / (E + 1), es = tid - ec * (E + 1);
    const bool ep_writer = tid < EP && es < E;
    const uint32_t xp = ep_writer ? (uint32_t(j10 + ec) * uint32_t(es * TPL)) & nmask : 0u;
    const C phi = hi[xp >> a.log2h], plo = lo[xp & lomask];

    // Data: row k = j + TPL s of the tile holds columns j10 and j10 + 1 at
    // element (j10 + k p) of the transform.
    C v[T][E];
    {
        const rsrc_t src = make_rsrc(in + tb + j10, uint32_t(a.n - j10) * ES);
        const uint32_t lane = (uint32_t(j) << a.log2p) * ES;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const float4 q = buf_load_pair(src, lane, (uint32_t(s * TPL) << a.log2p) * ES);
            v[0][s] = mk<C>(q.x, q.y);
            v[1][s] = mk<C>(q.z, q.w);
        }
    }
#pragma unroll
    for (int k = 0; k < TW_PER; ++k) {
        const int i = tid + k * NTHR;
        if (i < TW && tw_source<N, RMAX>(i) >= 0) twl[i] = twr[k];
    }
    if (ep_writer) ep[tid] = cmul(phi, plo); // published by the stage loop's first barrier
    C A[T];
#pragma unroll
    for (int c = 0; c < T; ++c) A[c] = cmul(ahi[c], alo[c]);
    const float sin_ = a.conj_in ? -1.f : 1.f;
#pragma unroll
    for (int c = 0; c < T; ++c)
#pragma unroll
        for (int s = 0; s < E; ++s) v[c][s] = scale_im(v[c][s], sin_);

    run_stages_lines<C, N, RMAX, E, T>(v, xch, a.pitch, twl, j);

    // Output k2 = j + TPL s of column c, times w_n^-(j1 k2), to slab
    // S[j1/2][k2][c]: the two halves of one 16-byte slab row.
    const rsrc_t dst = make_rsrc(out + tb + (j10 << a.log2q), uint32_t(T << a.log2q) * ES);
    const uint32_t lane = (uint32_t(j) << 1) * ES;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const uint32_t off = (uint32_t(s * TPL) << 1) * ES;
        buf_store(cmulc(v[0][s], cmul(A[0], ep[s])), dst, lane, off);
        __asm__ volatile("" ::: "memory"); // two 8-byte stores, not one 16-byte store
        buf_store(cmulc(v[1][s], cmul(A[1], ep[E + 1 + s])), dst, lane, off + ES);
    }
}

// ---------------------------------------------------------------------------
// Packed batches of uneven power-of-two lengths.  The plan groups the
// transforms into classes of equal length.  Lengths up to 2^12 run through
// the single-pass kernel, one launch per class, with `a.offsets` listing
// each transform's first element.  The lifted lengths share two persistent
// launches (pass 1 of every lifted class, then pass 2 of every lifted
// class): workgroups walk a work list of tiles ordered by class, longest
// lines first, with the same XCD-contiguous mapping as the pass kernels.
// The lifted classes use 512-thread tiles, 16 values per thread, radix 16
// and the split exchange.
struct RaggedClass {
    PassArgs a;          // in, out and the conjugation are set per launch
    int32_t kind, log2N; // kernel shape of the class
    int64_t item_begin;  // first work item (tile) of the class in its launch
};

constexpr int RAGGED_THREADS = 512;
constexpr int RAGGED_P1_MIN = 7, RAGGED_P2_MIN = 6; // shortest lift lines (t >= 13)
constexpr int RAGGED_LMAX = 12;                     // longest lift line (t <= 24)
constexpr int RAGGED_MAX_T = 24;

template <typename Real, int KIND, int L>
__device__ __forceinline__ void ragged_tile(const PassArgs &a, int64_t t, unsigned char *smem) {
    constexpr int LMIN = KIND == K_PASS1 ? RAGGED_P1_MIN : RAGGED_P2_MIN;
    if constexpr (L >= LMIN && L <= RAGGED_LMAX) {
        const Tile<Real, (1 << L), 16, KIND, 16, true> w(a, smem);
        w.template run_one<false>(t);
    }
}

template <typename Real, int KIND, int... L>
__device__ __forceinline__ void ragged_dispatch(int log2N, const PassArgs &a, int64_t t, unsigned char *smem,
                                                std::integer_sequence<int, L...>) {
    (void)((log2N == L ? (ragged_tile<Real, KIND, L>(a, t, smem), 0) : 0) + ...);
}

// Register budget: 128 VGPRs for complex64 (two 512-thread workgroups per
// CU at least), 256 for complex128.
template <typename Real> constexpr int ragged_min_waves() { return sizeof(Real) == 4 ? 4 : 2; }

// A workgroup-uniform record read from memory, word by word through
// readfirstlane, so that its fields live in scalar registers.
template <typename T> __device__ __forceinline__ T uniform_copy(const T *src) {
    static_assert(sizeof(T) % 4 == 0, "word-sized record");
    T r;
    const int *w = reinterpret_cast<const int *>(src);
    int *d = reinterpret_cast<int *>(&r);
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(w[i]);
    return r;
}

template <typename Real>
__global__ __launch_bounds__(RAGGED_THREADS, (ragged_min_waves<Real>())) void ragged_kernel(const RaggedClass *__restrict__ cls, int ncls,
                                                                int64_t items, const void *in, void *out, int inv) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int64_t G = gridDim.x, g = blockIdx.x;
    const int64_t rank = (G & 7) == 0 ? (g & 7) * (G >> 3) + (g >> 3) : g;
    for (int64_t it0 = 0; it0 < items; it0 += G) { // the exit test is workgroup-uniform
        const int64_t it = it0 + rank;
        if (it >= items) break;
        int k = 0;
        while (k + 1 < ncls && __builtin_amdgcn_readfirstlane(int(cls[k + 1].item_begin <= it))) ++k;
        const RaggedClass rc = uniform_copy(&cls[k]);
        PassArgs a = rc.a;
        const int kind = rc.kind, log2N = rc.log2N;
        if (kind == K_PASS1) a.in = in;   // pass 2 reads the scratch array
        if (kind == K_PASS2) a.out = out; // pass 1 writes it
        a.conj_in = kind == K_PASS1 ? inv : 0;
        a.conj_out = kind == K_PASS2 ? inv : 0;
        const int64_t t = it - rc.item_begin;
        __syncthreads(); // the previous tile's LDS readers are done
        constexpr auto seq = std::make_integer_sequence<int, RAGGED_LMAX + 1>{};
        if (kind == K_PASS1) ragged_dispatch<Real, K_PASS1>(log2N, a, t, smem_raw, seq);
        else ragged_dispatch<Real, K_PASS2>(log2N, a, t, smem_raw, seq);
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

// Debug mode: fill `words` 32-bit words with a quiet NaN (grid-stride).
__global__ void canary_fill_kernel(uint32_t *__restrict__ p, int64_t words) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0x7fc00000u;
}

// Tuner helpers.  A deterministic input pattern in [-1, 1) (an integer
// hash of the index), and per-block maxima of |a - b| and |b| for comparing
// two outputs (finished on the host).
template <typename Real>
__global__ void fill_pattern_kernel(typename Cx<Real>::T *x, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint32_t h = uint32_t(i) * 2654435761u ^ uint32_t(i >> 32);
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    typename Cx<Real>::T v;
    v.x = Real(int32_t(h & 0xffff) - 32768) / Real(32768);
    v.y = Real(int32_t(h >> 16) - 32768) / Real(32768);
    x[i] = v;
}

constexpr int CMP_THREADS = 256;

template <typename Real>
__global__ __launch_bounds__(CMP_THREADS) void compare_kernel(const typename Cx<Real>::T *a,
                                                              const typename Cx<Real>::T *b, int64_t count,
                                                              double *partial) {
    __shared__ double sd[CMP_THREADS], sb[CMP_THREADS];
    double md = 0, mb = 0;
    for (int64_t i = int64_t(blockIdx.x) * CMP_THREADS + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * CMP_THREADS) {
        const double dx = double(a[i].x) - double(b[i].x), dy = double(a[i].y) - double(b[i].y);
        const double d = fmax(fabs(dx), fabs(dy)), m = fmax(fabs(double(b[i].x)), fabs(double(b[i].y)));
        md = isnan(d) ? INFINITY : fmax(md, d);
        mb = fmax(mb, m);
    }
    sd[threadIdx.x] = md;
    sb[threadIdx.x] = mb;
    __syncthreads();
    for (int w = CMP_THREADS / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + w]);
            sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sd[0];
        partial[2 * blockIdx.x + 1] = sb[0];
    }
}

using KernelFn = void (*)(PassArgs);

// Kernel variant of the pass kernels.
struct Variant {
    int emax = 16;        // complex values per thread
    bool split = false;   // real/imaginary exchange in turn
    bool persist = false; // persistent workgroups with next-tile prefetch
    bool dense = false;   // 64-VGPR cap (two 1024-thread workgroups per CU)
    int prec = 0;         // PREC_*: radix-16 stages on the matrix cores when nonzero
    bool shuffle = false; // axis passes: stage exchange by wavefront shuffles
    bool lds_prefetch = false; // pass 1: persistent, next tile staged in LDS by direct loads
    bool rows = false;         // pass 1: each thread owns whole rows of a 2-column tile
    bool is_default() const {
        return emax == 16 && !split && !persist && !dense && !prec && !shuffle && !lds_prefetch && !rows;
    }
    int code() const {
        return (emax == 32 ? 1 : 0) | (split ? 2 : 0) | (persist ? 4 : 0) | (dense ? 8 : 0) | (prec << 4) |
               (shuffle ? 64 : 0) | (lds_prefetch ? 128 : 0) | (rows ? 256 : 0);
    }
};

template <typename Real, int KIND, int RMAX, int VAR, int LMIN, int LMAX, int L>
constexpr KernelFn kernel_entry() {
    if constexpr (L < LMIN || L < 1 || L > LMAX || L > max_line_of<Real>()) return nullptr;
    else
        return &pass_kernel<Real, (1 << L), RMAX, KIND, (VAR & 1) ? 32 : 16, (VAR & 2) != 0, (VAR & 4) != 0,
                            (VAR & 8) != 0>;
}

template <typename Real, int KIND, int RMAX, int VAR, int LMIN, int LMAX, int... L>
constexpr std::array<KernelFn, sizeof...(L)> kernel_row(std::integer_sequence<int, L...>) {
    return {{kernel_entry<Real, KIND, RMAX, VAR, LMIN, LMAX, L>()...}};
}

template <typename Real, int KIND, int RMAX, int VAR = 0, int LMIN = 1, int LMAX = MAX_LOG2_LINE>
KernelFn pick(int log2N) {
    static const auto row =
        kernel_row<Real, KIND, RMAX, VAR, LMIN, LMAX>(std::make_integer_sequence<int, MAX_LOG2_LINE + 1>{});
    if (log2N < 1 || log2N > MAX_LOG2_LINE) return nullptr;
    return row[log2N];
}

// Axis passes of the three-level lift: radix 16, lines of 2^5..2^11 (every
// pass has at least two stages, so its weight table is published by a stage
// barrier).
constexpr int AXIS_LMIN = 5, AXIS_LMAX = 11;
// Wide axis passes: transforms of 2^31 bytes or more (2^29 complex64 and
// 2^28 complex128 elements on), whose three factors are at least 2^9.
constexpr int AXIS_WIDE_LMIN = 9;

template <typename Real> KernelFn pick_default(int kind, int log2N, int rmax) {
    switch (kind * 100 + rmax) {
    case K_SINGLE * 100 + 16: return pick<Real, K_SINGLE, 16>(log2N);
    case K_SINGLE * 100 + 2: return pick<Real, K_SINGLE, 2>(log2N);
    case K_PASS1 * 100 + 16: return pick<Real, K_PASS1, 16>(log2N);
    case K_PASS1 * 100 + 2: return pick<Real, K_PASS1, 2>(log2N);
    case K_PASS2 * 100 + 16: return pick<Real, K_PASS2, 16>(log2N);
    case K_PASS2 * 100 + 2: return pick<Real, K_PASS2, 2>(log2N);
    case K_AXIS * 100 + 16: return pick<Real, K_AXIS, 16, 0, AXIS_LMIN, AXIS_LMAX>(log2N);
    case K_AXIS_WIDE * 100 + 16: return pick<Real, K_AXIS_WIDE, 16, 0, AXIS_WIDE_LMIN, AXIS_LMAX>(log2N);
    default: return nullptr;
    }
}

// The other variants exist for complex64 pass kernels with radix 16 and lines
// of 2^10..2^12 (the lifts of the largest transforms); the split exchange,
// the default at these lengths, also for lines of 2^13 and 2^14.
constexpr int VARIANT_LMIN = 10, VARIANT_LMAX = 12;

template <int KIND> KernelFn pick_variant(int log2N, const Variant &v) {
    switch (v.code()) {
    case 1: return pick<float, KIND, 16, 1, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    case 2: return pick<float, KIND, 16, 2, VARIANT_LMIN, MAX_LOG2_LINE>(log2N);
    case 3: return pick<float, KIND, 16, 3, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    case 4: return pick<float, KIND, 16, 4, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    case 5: return pick<float, KIND, 16, 5, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    case 6: return pick<float, KIND, 16, 6, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    case 7: return pick<float, KIND, 16, 7, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    case 8: return pick<float, KIND, 16, 8, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    case 10: return pick<float, KIND, 16, 10, VARIANT_LMIN, VARIANT_LMAX>(log2N);
    default: return nullptr; // dense variants exist with 16 values per thread, one tile each
    }
}

// Matrix-core kernels: complex64, lines of 16, 256 or 4096 points (every
// stage radix 16), 16 values per thread, complex exchange, one tile each.
template <int KIND, int PREC> KernelFn pick_mfma(int log2N) {
    switch (log2N) {
    case 4: return &pass_kernel<float, 16, 16, KIND, 16, false, false, false, PREC>;
    case 8: return &pass_kernel<float, 256, 16, KIND, 16, false, false, false, PREC>;
    case 12: return &pass_kernel<float, 4096, 16, KIND, 16, false, false, false, PREC>;
    default: return nullptr;
    }
}
template <int PREC> KernelFn pick_mfma_kind(int kind, int log2N) {
    if (kind == K_AXIS) // three-level passes over 256-point lines (n = 2^24 = 256^3)
        return log2N == 8 ? &pass_kernel<float, 256, 16, K_AXIS, 16, false, false, false, PREC> : nullptr;
    if (kind == K_AXIS_WIDE) return nullptr;
    return kind == K_SINGLE ? pick_mfma<K_SINGLE, PREC>(log2N)
           : kind == K_PASS1 ? pick_mfma<K_PASS1, PREC>(log2N)
                             : pick_mfma<K_PASS2, PREC>(log2N);
}

KernelFn pick_kernel(int dtype, int kind, int log2N, int rmax, const Variant &v) {
    if (v.prec) {
        if (dtype != FFT_C64 || rmax != 16 || v.emax != 16 || v.split || v.persist || v.dense) return nullptr;
        return v.prec == PREC_F16X2 ? pick_mfma_kind<PREC_F16X2>(kind, log2N)
                                    : pick_mfma_kind<PREC_BF16X2>(kind, log2N);
    }
    if (kind == K_AXIS_WIDE && !v.is_default()) return nullptr;
    if (v.lds_prefetch) { // complex64 pass 1 over 4096-point columns, 2 per tile, split exchange
        if (kind != K_PASS1 || dtype != FFT_C64 || rmax != 16 || log2N != 12 || v.code() != (128 | 2))
            return nullptr;
        return &pass1_dma_kernel;
    }
    if (v.rows) { // complex64 pass 1 over 4096-point columns, 2 per tile, rows per thread, split exchange
        if (kind != K_PASS1 || dtype != FFT_C64 || rmax != 16 || log2N != 12 || (v.code() & ~1) != (256 | 2))
            return nullptr;
        return v.emax == 32 ? &pass1_rows_kernel<16> : &pass1_rows_kernel<8>;
    }
    if (v.shuffle) { // complex64 axis passes over 256-point lines
        if (kind != K_AXIS || dtype != FFT_C64 || rmax != 16 || log2N != 8 || v.code() != 64) return nullptr;
        return &axis_shuffle_kernel;
    }
    if (kind == K_AXIS && !v.is_default()) { // the split exchange (complex64) only
        if (dtype != FFT_C64 || rmax != 16 || v.code() != 2) return nullptr;
        return pick<float, K_AXIS, 16, 2, AXIS_LMIN, AXIS_LMAX>(log2N);
    }
    if (v.is_default())
        return dtype == FFT_C64 ? pick_default<float>(kind, log2N, rmax)
                                : pick_default<double>(kind, log2N, rmax);
    if (dtype != FFT_C64 || rmax != 16) return nullptr;
    if (kind == K_PASS1) return pick_variant<K_PASS1>(log2N, v);
    if (kind == K_PASS2) return pick_variant<K_PASS2>(log2N, v);
    return nullptr;
}

int thread_cap(size_t esize, const Variant &v) {
    return esize == 8 && !v.persist && v.emax == 16 ? max_threads<float, 16, false>() : 512;
}

int ilog2_exact(int64_t v) {
    if (v < 1 || (v & (v - 1))) return -1;
    int t = 0;
    while ((int64_t(1) << t) < v) ++t;
    return t;
}

struct Launch {
    KernelFn fn = nullptr;
    Variant var;
    int kind = 0, rmax = 16;
    int log2N = 0, log2T = 0;
    int64_t lines = 0, ntiles = 0, grid = 0;
    int threads = 0;
    int pitch = 0;
    size_t lds = 0;
    bool remap = false;
    int spread_log2g = 0, spread_log2s = 0; // tile order within an XCD's range (remapped, not persistent)
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
    Launch k1, k2, k3; // k3: third pass of a three-level lift
    Launch k1_plain;   // pass 1 for inputs the LDS-staged or row-lane pass 1 cannot load (not 16-byte aligned)
    int log2n1 = 0, log2n2 = 0, log2n3 = 0; // three-level lift n = n1 n2 n3 (n1 contiguous)
    const void *tw3 = nullptr;
    Variant base1, base2, base3; // the variants chosen at creation (precision FP32)
    int log2W = 0;        // scratch slab width (two-pass plans)
    bool no_remap = false;
    bool kernel_defaults = false; // created without kernel-variant, tile-width or radix options
    bool tile_order_set = false;  // tile orders given by the caller (FFT_OPT_TILE_ORDER)
    int32_t tile_order = 0;      // their encoding, one byte per pass
    int precision = 0;
    void *dft_ops = nullptr; // matrix-core forms: DFT-matrix operand table (4 KB per form)
    int dft_ops_prec = 0;    // the form whose operands dft_ops holds
    int64_t total = 0; // elements in the input (and output) buffer
    // Packed batch of uneven lengths: two persistent launches over classes
    // of equal length, replayed as one captured graph per (in, out, sign).
    struct RaggedLaunch {
        int nclass = 0;
        int64_t items = 0, grid = 0;
        size_t lds = 0;
        const void *cls = nullptr; // device array of classes
    };
    bool ragged = false;
    int length_classes = 0;
    // Packed uneven batch, one plan per length class (the default form of
    // fft_plan_create_many): each class is a single-length plan over its
    // transforms' offsets, with its tables and scratch inside this plan's.
    // Classes run on up to four streams -- the execute stream and three of
    // the plan's own -- forked from and joined back into the execute
    // stream, or replayed as one captured graph with those branches.
    struct ClassRun {
        fft_plan *sub;
        int lane; // 0: the execute stream; k > 0: aux[k - 1]
    };
    std::vector<ClassRun> runs;
    static constexpr int AUX = 3;
    hipStream_t aux[AUX] = {nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[AUX] = {nullptr, nullptr, nullptr};
    int lanes = 1;
    const int64_t *offsets = nullptr; // a class plan: first element of each of its transforms
    int64_t packed_total = 0;         // a class plan: elements in the packed buffer
    // The paper's partitioned radix-2 plan (fft_plan_create_paper).
    bool paper = false;
    liftfft_paper::PaperPlan pp;
    RaggedLaunch ra, rb;
    struct SingleClass {
        Launch L;
        PassArgs a; // in, out and the conjugation are set per execute
    };
    std::vector<SingleClass> singles;
    void *meta = nullptr; // device: classes and transform offsets
    size_t meta_bytes = 0;
    bool use_graph = false;
    bool canary = false; // FFT_OPT_DEBUG_CANARY
    // Execute-time bookkeeping (mutable: fft_execute takes a const plan, whose
    // transform it only reads): the graph cache of uneven batches and the
    // timing event ring.
    mutable hipStream_t cap = nullptr; // private stream for graph capture
    struct GraphEntry {
        const void *in;
        void *out;
        int sign;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    mutable std::vector<GraphEntry> graphs;
    // Benchmark timing: a ring of event quadruples (before the first pass,
    // after each pass) recorded on the execute stream; drained on read.
    bool timing = false;
    std::vector<hipEvent_t> ev;
    mutable int ring_head = 0, ring_count = 0;
    mutable double ms[3] = {0, 0, 0};
    mutable int64_t launches[3] = {0, 0, 0};
};

namespace {

// Exchange pitch and LDS bytes of a tile of 2^log2T lines.
struct TileShape {
    int pitch = 0;
    int64_t lds = 0;
};
TileShape tile_shape(int log2N, int rmax, size_t esize, int log2T, const Variant &v, int kind) {
    const int N = 1 << log2N, E = vals_per_thread(N, v.emax), T = 1 << log2T;
    const int lsize = int(v.split ? esize / 2 : esize);
    TileShape ts;
    ts.pitch = exchange_pitch(N, T, N / E, lsize, kind != K_SINGLE);
    ts.lds = lds_bytes(N, rmax, T, E, ts.pitch, lsize, int(esize), kind == K_PASS1 || kind >= K_AXIS, v.prec != 0);
    return ts;
}

// Lines per tile: the smallest power of two T <= max_lines whose tile has at
// least `want_threads` threads and `min_T` lines, as long as it fits the
// thread and LDS limits and `cap` (0 = none).
int choose_log2T(int log2N, int rmax, size_t esize, int64_t max_lines, int want_threads, int min_T,
                 int cap, int kind, const Variant &v) {
    const int N = 1 << log2N;
    const int64_t tpl = N / vals_per_thread(N, v.emax);
    const int64_t tcap = thread_cap(esize, v);
    auto fits = [&](int l2T) {
        const int64_t T = int64_t(1) << l2T;
        return T <= max_lines && T * tpl <= tcap &&
               tile_shape(log2N, rmax, esize, l2T, v, kind).lds <= LDS_BUDGET && (!cap || T <= cap);
    };
    int log2T = 0;
    for (;;) {
        const int64_t T = int64_t(1) << log2T;
        if (T * tpl >= want_threads && T >= min_T) break;
        if (!fits(log2T + 1)) break;
        ++log2T;
    }
    return log2T;
}

// Fill a launch description: kernel, tile shape, LDS and grid (one
// workgroup per tile, or for persistent kernels as many as are resident at
// once).
bool fill_launch(Launch &L, int dtype, int kind, int log2N, int rmax, int log2T, int64_t lines,
                 const Variant &v, int device) {
    const int N = 1 << log2N;
    const size_t esize = dtype == FFT_C64 ? 8 : 16;
    L.fn = pick_kernel(dtype, kind, log2N, rmax, v);
    if (!L.fn) return false;
    L.var = v;
    L.log2N = log2N;
    L.log2T = log2T;
    L.lines = lines;
    L.threads = (N / vals_per_thread(N, v.emax)) << log2T;
    if (v.rows) { // fixed shape: 2 columns, E rows per thread (E = 16 for 32 values, else 8)
        if ((int64_t(1) << log2T) != ROWS_T) return false;
        L.threads = v.emax == 32 ? rows_threads<16>() : rows_threads<8>();
    }
    if (L.threads > thread_cap(esize, v)) return false;
    if (v.prec && L.threads % 64) return false; // waves own 64 butterflies per stage
    L.kind = kind;
    L.rmax = rmax;
    // Axis tiles must be whole: pass C's row-first load has two barriers that
    // every thread of the workgroup reaches, so no tile may be partial.
    if ((kind == K_AXIS || kind == K_AXIS_WIDE) && (lines & ((int64_t(1) << log2T) - 1))) return false;
    L.ntiles = (lines + (int64_t(1) << log2T) - 1) >> log2T;
    TileShape ts = tile_shape(log2N, rmax, esize, log2T, v, kind);
    if (v.rows) { // radix-E stages over E values of each of the 2 columns, split exchange
        const int Ec = v.emax / 2;
        ts.pitch = exchange_pitch(N, ROWS_T, N / Ec, int(esize / 2), true);
        ts.lds = lds_bytes(N, Ec, ROWS_T, Ec, ts.pitch, int(esize / 2), int(esize), true);
    }
    if (ts.lds > LDS_BUDGET) return false;
    L.pitch = ts.pitch;
    L.lds = size_t(ts.lds);
    if (v.shuffle) { // fixed shape: 16 lines of 256 points, tables in static LDS
        if ((int64_t(1) << log2T) != SHUF_T || L.threads != SHUF_THREADS) return false;
        L.lds = 0;
    }
    if (v.lds_prefetch) { // fixed shape: 2 columns of 4096 points, static LDS
        if ((int64_t(1) << log2T) != DMA_T || L.threads != DMA_THREADS) return false;
        L.lds = 0;
    }
    if (L.lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void *>(L.fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(L.lds)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (!v.persist && !v.lds_prefetch) {
        L.grid = L.ntiles;
        L.remap = (L.grid % 8 == 0) && L.grid >= 16;
    } else {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(L.fn),
                                                         L.threads, L.lds) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        if (per_cu < 1) return false;
        const int64_t resident = int64_t(per_cu) * cus;
        L.grid = L.ntiles < resident ? L.ntiles : resident;
        L.remap = L.ntiles % 8 == 0 && L.grid >= 16;
        if (L.remap) L.grid &= ~int64_t(7);
    }
    return L.grid <= INT32_MAX;
}

// Tile shape for a pass kernel: `want_T` lines if nonzero (the launch then
// fails if it does not fit), else pass 1 aims at 512-thread tiles of at least
// two lines and pass 2 at tiles of at least four lines (32-byte segments in
// the natural-order output), pass 1 within `cap1`.
bool plan_pass(Launch &L, int dtype, int kind, int log2N, int rmax, int64_t lines_per_transform,
               int64_t lines, int want_T, int cap1, const Variant &v, int device) {
    const size_t esize = dtype == FFT_C64 ? 8 : 16;
    int l2T;
    if (want_T) {
        l2T = ilog2_exact(want_T);
        if (want_T > lines_per_transform || (cap1 && want_T > cap1)) return false;
    } else if (kind >= K_AXIS) { // rows of at least 128 contiguous bytes, 256 threads
        l2T = choose_log2T(log2N, rmax, esize, lines_per_transform, 256, int(128 / esize), 0, kind, v);
        if ((int64_t(1) << l2T) * int64_t(esize) < 128) return false;
    } else {
        const bool p1 = kind == K_PASS1;
        l2T = choose_log2T(log2N, rmax, esize, lines_per_transform, 512, p1 ? 2 : 4, p1 ? cap1 : 0, kind, v);
    }
    return fill_launch(L, dtype, kind, log2N, rmax, l2T, lines, v, device);
}

int gen_table(int dtype, void *dst, int64_t count, int64_t mult, int log2N, hipStream_t st = nullptr) {
    const int threads = 256;
    const int64_t blocks = (count + threads - 1) / threads;
    if (dtype == FFT_C64)
        hipLaunchKernelGGL(twiddle_table_kernel<float>, dim3(unsigned(blocks)), dim3(threads), 0, st,
                           static_cast<float2 *>(dst), count, mult, log2N);
    else
        hipLaunchKernelGGL(twiddle_table_kernel<double>, dim3(unsigned(blocks)), dim3(threads), 0,
                           st, static_cast<double2 *>(dst), count, mult, log2N);
    return hipGetLastError() == hipSuccess ? FFT_OK : FFT_E_HIP;
}

// Whether a plan without level or two-level options lifts to three
// levels: from n = 2^24 on (both element types), where the three-level lift
// measured faster on MI355X (2^24 complex64: 175 us against 197 us; 2^26:
// 704 against 1199; 2^28: 3.35 ms against 6.65 ms); below that the two
// passes of the two-level lift are at least as fast.
bool default_three_level(int t, int dtype, int radix, const Variant &v) {
    (void)dtype;
    return t >= 24 && radix == 16 && v.is_default();
}

// Workgroup order of a single-length plan's launches (fill_launch sets the
// XCD-contiguous remap wherever the grid allows it).  Up to 2^24 passes B and
// C of the three-level lift run in the hardware workgroup order (measured at
// 2^24: 160 us against 166 us with every pass remapped; at 2^22 48.1 against
// 49.0); from 2^26 on remapping every pass is at least as fast.  Applied
// after plan creation and after every change of the plan's kernels.
// Tile order byte b of a launch (0x80 hardware order, else (log2 g << 4) |
// log2 s): false if the launch cannot take it.  A spread needs the
// XCD-contiguous order, one tile per workgroup and XCD ranges of whole g x s
// blocks.
bool set_tile_order(Launch &L, int b) {
    L.spread_log2g = L.spread_log2s = 0;
    const bool one_tile = !L.var.persist && !L.var.lds_prefetch;
    if (b == 0x80) {
        L.remap = false;
        return true;
    }
    if (one_tile) L.remap = L.grid % 8 == 0 && L.grid >= 16;
    const int log2g = b >> 4, log2s = b & 15;
    if (!log2s) return true;
    if (!one_tile || !L.remap || (L.grid >> 3) % (int64_t(1) << (log2g + log2s))) return false;
    L.spread_log2g = log2g;
    L.spread_log2s = log2s;
    return true;
}

int tile_order_byte(const Launch &L) {
    return L.remap ? (L.spread_log2g << 4) | L.spread_log2s : 0x80;
}

// Tile orders measured fastest on MI355X for the library's default plans of
// these complex64 shapes (the tile-order search of the benchmark: each pass
// in turn over the hardware order and spreads of g 1, s 2..32 and g 2, s 4
// and 8, medians of per-pass HIP events over four rotating buffer sets; kept
// where two searches agreed and the whole transform gained 3% or more).
// n = 2^24: two-level 4096 x 4096 pass 1 107 -> 92 us, pass 2 83 -> 76 us;
// three-level 256^3 pass A 61 -> 56 us, pass B 56 -> 46 us.  2^23 (4096 x
// 2048) pass 2 39 -> 35 us; 2^25 pass A 136 -> 125 us, pass C 111 -> 107
// us; 16 transforms of 2^20, pass 1 80 -> 61 us; 4096 transforms of 2^12
// in one pass 68 -> 65 us.  Every other plan keeps the plain order (at 256
// transforms of 2^20, for one, no spread won).
struct KnownOrder {
    int passes, log2n, log2p;
    int64_t batch;
    int32_t order;
};
constexpr KnownOrder known_orders[] = {
    {2, 24, 12, 1, 0x0412},   // pass 1 g 2, s 4; pass 2 g 1, s 16
    {3, 24, 0, 1, 0x800305},  // A g 1, s 32; B g 1, s 8; C hardware order
    {2, 23, 11, 1, 0x0112},   // pass 1 g 2, s 4; pass 2 g 1, s 2
    {3, 25, 0, 1, 0x800005},  // A g 1, s 32; B plain; C hardware order
    {2, 20, 10, 16, 0x8003},  // pass 1 g 1, s 8; pass 2 hardware order
    {1, 12, 0, 4096, 0x80},   // hardware order
};

// Workgroup order of each launch of a single-length plan: the caller's tile
// orders if given; else the orders measured for the plan's shape
// (known_orders, FP32 plans with the default kernels only); else the plain
// orders (XCD-contiguous, and the hardware order for passes B and C of a
// three-level lift up to 2^24).  Applied after plan creation and after every
// change of the plan's kernels (which keeps the grids); FFT_E_UNSUPPORTED if
// a given order does not fit its launch.
int apply_remap_policy(fft_plan *p) {
    Launch *L[3] = {&p->k1, &p->k2, &p->k3};
    for (Launch *x : {&p->k1, &p->k2, &p->k3, &p->k1_plain}) x->spread_log2g = x->spread_log2s = 0;
    if (p->tile_order_set) {
        for (int k = 0; k < p->passes; ++k) {
            const int b = (p->tile_order >> (8 * k)) & 0xff;
            if (p->no_remap) L[k]->remap = false; // with FFT_OPT_NO_XCD_REMAP only s = 1 is accepted
            else if (!set_tile_order(*L[k], b)) return FFT_E_UNSUPPORTED;
        }
        return FFT_OK;
    }
    if (p->passes == 3 && p->log2n <= 24) p->k2.remap = p->k3.remap = false;
    if (p->no_remap) {
        p->k1.remap = p->k2.remap = p->k3.remap = false;
        return FFT_OK;
    }
    if (!p->kernel_defaults || p->dtype != FFT_C64 || p->precision) return FFT_OK;
    for (const KnownOrder &e : known_orders) {
        if (e.passes != p->passes || e.log2n != p->log2n || e.log2p != p->log2p || e.batch != p->batch) continue;
        Launch trial[3] = {p->k1, p->k2, p->k3};
        bool ok = true;
        for (int k = 0; k < p->passes && ok; ++k) ok = set_tile_order(trial[k], (e.order >> (8 * k)) & 0xff);
        if (ok) {
            p->k1 = trial[0];
            p->k2 = trial[1];
            p->k3 = trial[2];
        }
        break;
    }
    return FFT_OK;
}

constexpr int TIMING_RING = 1024, RING_EVENTS = 4;

// Accumulate the durations recorded in ring slot `slot` (waits for them).
int drain_slot(const fft_plan *p, int slot) {
    const hipEvent_t *e = &p->ev[size_t(slot) * RING_EVENTS];
    if (hipEventSynchronize(e[p->passes]) != hipSuccess) return FFT_E_HIP;
    for (int k = 0; k < p->passes; ++k) {
        float t = 0;
        if (hipEventElapsedTime(&t, e[k], e[k + 1]) != hipSuccess) return FFT_E_HIP;
        p->ms[k] += t;
        p->launches[k] += 1;
    }
    return FFT_OK;
}

int drain_all(const fft_plan *p) {
    int rc = FFT_OK;
    while (p->ring_count > 0) {
        const int slot = (p->ring_head - p->ring_count + TIMING_RING) % TIMING_RING;
        const int r = drain_slot(p, slot);
        if (r != FFT_OK) rc = r;
        --p->ring_count;
    }
    return rc;
}

int launch(const fft_plan *p, const Launch &L, const PassArgs &args, hipStream_t st) {
    if (L.grid <= 0) return FFT_OK;
    PassArgs a = args;
    a.tile_log2g = L.spread_log2g;
    a.tile_log2s = a.xcd_remap && !L.var.persist && !L.var.lds_prefetch ? L.spread_log2s : 0;
    hipLaunchKernelGGL(L.fn, dim3(unsigned(L.grid)), dim3(unsigned(L.threads)), L.lds, st, a);
    (void)p;
    return hipGetLastError() == hipSuccess ? FFT_OK : FFT_E_HIP;
}

void free_plan(fft_plan *p) {
    if (!p) return;
    for (auto &r : p->runs) { // class plans: their device memory is this plan's
        r.sub->tables = r.sub->scratch = nullptr;
        free_plan(r.sub);
    }
    for (int k = 0; k < fft_plan::AUX; ++k) {
        if (p->aux[k]) (void)hipStreamDestroy(p->aux[k]);
        if (p->join_ev[k]) (void)hipEventDestroy(p->join_ev[k]);
    }
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    for (auto &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &g : p->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->scratch) (void)hipFree(p->scratch);
    if (p->tables) (void)hipFree(p->tables);
    if (p->meta) (void)hipFree(p->meta);
    if (p->dft_ops) (void)hipFree(p->dft_ops);
    delete p;
}

int launch_ragged(const fft_plan *p, const fft_plan::RaggedLaunch &R, const void *in, void *out, int inv,
                  hipStream_t st) {
    if (R.items <= 0) return FFT_OK;
    const RaggedClass *cls = static_cast<const RaggedClass *>(R.cls);
    if (p->dtype == FFT_C64)
        hipLaunchKernelGGL(ragged_kernel<float>, dim3(unsigned(R.grid)), dim3(RAGGED_THREADS), R.lds, st, cls,
                           R.nclass, R.items, in, out, inv);
    else
        hipLaunchKernelGGL(ragged_kernel<double>, dim3(unsigned(R.grid)), dim3(RAGGED_THREADS), R.lds, st, cls,
                           R.nclass, R.items, in, out, inv);
    return hipGetLastError() == hipSuccess ? FFT_OK : FFT_E_HIP;
}

// Every launch of a packed uneven batch in order: pass 1 of the lifted
// classes, the single-pass classes, then (after `ev_mid`, if given) pass 2
// of the lifted classes.
int ragged_sequence(const fft_plan *p, const void *in, void *out, int inv, hipStream_t st, hipEvent_t ev_mid) {
    int rc = launch_ragged(p, p->ra, in, out, inv, st);
    for (const auto &sc : p->singles) {
        if (rc != FFT_OK) break;
        PassArgs a = sc.a;
        a.in = in;
        a.out = out;
        a.conj_in = a.conj_out = inv;
        rc = launch(p, sc.L, a, st);
    }
    if (rc == FFT_OK && ev_mid) rc = hipEventRecord(ev_mid, st) == hipSuccess ? FFT_OK : FFT_E_HIP;
    if (rc == FFT_OK) rc = launch_ragged(p, p->rb, in, out, inv, st);
    return rc;
}

constexpr size_t MAX_GRAPHS = 16; // captured graphs kept per plan

// The two launches of a packed uneven batch, as one graph launch when
// possible: a graph is captured on the plan's private stream the first time
// an (in, out, sign) triple is seen and replayed afterwards.  When the
// caller's stream is itself being captured, or the cache is full, the
// kernels are launched directly.  `ev` (optional) brackets the work.
int launch_plan(const fft_plan *p, const void *in, void *out, int sign, hipStream_t st);

// Every class plan of a packed batch: forked from st onto the plan's
// streams (classes of the same lane run in order) and joined back into st.
int launch_classes(const fft_plan *p, const void *in, void *out, int sign, hipStream_t st) {
    const hipStream_t lane[1 + fft_plan::AUX] = {st, p->aux[0], p->aux[1], p->aux[2]};
    if (p->lanes > 1) {
        if (hipEventRecord(p->fork_ev, st) != hipSuccess) return FFT_E_HIP;
        for (int k = 1; k < p->lanes; ++k)
            if (hipStreamWaitEvent(lane[k], p->fork_ev, 0) != hipSuccess) return FFT_E_HIP;
    }
    int rc = FFT_OK;
    for (const auto &r : p->runs) {
        rc = launch_plan(r.sub, in, out, sign, lane[r.lane]);
        if (rc != FFT_OK) break;
    }
    for (int k = 1; k < p->lanes; ++k) // joined even after a failed launch
        if (hipEventRecord(p->join_ev[k - 1], lane[k]) != hipSuccess ||
            hipStreamWaitEvent(st, p->join_ev[k - 1], 0) != hipSuccess)
            return FFT_E_HIP;
    return rc;
}

// The work of a packed batch on stream st: the class plans, or the two
// persistent launches and the single-pass classes (ev_mid, if given, is
// recorded between the persistent passes).
int packed_sequence(const fft_plan *p, const void *in, void *out, int sign, hipStream_t st, hipEvent_t ev_mid) {
    if (!p->runs.empty()) {
        const int rc = launch_classes(p, in, out, sign, st);
        if (rc == FFT_OK && ev_mid) return hipEventRecord(ev_mid, st) == hipSuccess ? FFT_OK : FFT_E_HIP;
        return rc;
    }
    return ragged_sequence(p, in, out, sign > 0, st, ev_mid);
}

int execute_ragged(const fft_plan *p, const void *in, void *out, int sign, hipStream_t st, const hipEvent_t *ev) {
    bool graph = p->use_graph;
    if (graph) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
            (void)hipGetLastError();
            graph = false;
        } else if (cs != hipStreamCaptureStatusNone) {
            graph = false;
        }
    }
    if (graph) {
        const fft_plan::GraphEntry *hit = nullptr;
        for (const auto &g : p->graphs)
            if (g.in == in && g.out == out && g.sign == sign) hit = &g;
        if (!hit && p->graphs.size() < MAX_GRAPHS) {
            if (!p->cap && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                p->cap = nullptr;
            }
            if (p->cap && hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                const int rc = packed_sequence(p, in, out, sign, p->cap, nullptr);
                hipGraph_t g = nullptr;
                const bool ended = hipStreamEndCapture(p->cap, &g) == hipSuccess;
                hipGraphExec_t e = nullptr;
                if (rc == FFT_OK && ended && g && hipGraphInstantiate(&e, g, nullptr, nullptr, 0) == hipSuccess) {
                    p->graphs.push_back({in, out, sign, g, e});
                    hit = &p->graphs.back();
                } else {
                    (void)hipGetLastError();
                    if (g) (void)hipGraphDestroy(g);
                }
            } else {
                (void)hipGetLastError();
            }
        }
        if (hit) {
            if (ev && hipEventRecord(ev[0], st) != hipSuccess) return FFT_E_HIP;
            if (hipGraphLaunch(hit->exec, st) != hipSuccess) return FFT_E_HIP;
            if (ev && (hipEventRecord(ev[1], st) != hipSuccess || hipEventRecord(ev[2], st) != hipSuccess))
                return FFT_E_HIP;
            return FFT_OK;
        }
    }
    if (ev && hipEventRecord(ev[0], st) != hipSuccess) return FFT_E_HIP;
    int rc = packed_sequence(p, in, out, sign, st, ev ? ev[1] : nullptr);
    if (rc == FFT_OK && ev) rc = hipEventRecord(ev[2], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
    return rc;
}


// Weight-table entries of a single-length plan: one w_N table per pass (N
// its line length) and, for lifted plans, the two-level w_n table (n/2^h
// high and 2^h low entries).
int64_t table_entries(const fft_plan *p) {
    const bool lifted = p->passes >= 2;
    const int64_t n1 = int64_t(1) << p->k1.log2N;
    const int64_t n2 = lifted ? (int64_t(1) << p->k2.log2N) : 0;
    const int64_t n3 = p->passes == 3 ? (int64_t(1) << p->k3.log2N) : 0;
    const int64_t nhi = lifted ? (p->n >> p->log2h) : 0;
    const int64_t nlo = lifted ? (int64_t(1) << p->log2h) : 0;
    return n1 + n2 + n3 + nhi + nlo;
}

// Point the plan's table pointers into p->tables and (if `generate`) fill
// the tables on stream st (FP64 kernel, each entry from its integer
// exponent).
int fill_tables(fft_plan *p, hipStream_t st, bool generate = true) {
    const bool lifted = p->passes >= 2;
    const size_t esize = p->esize;
    const int t = p->log2n;
    const int64_t n1 = int64_t(1) << p->k1.log2N;
    const int64_t n2 = lifted ? (int64_t(1) << p->k2.log2N) : 0;
    const int64_t n3 = p->passes == 3 ? (int64_t(1) << p->k3.log2N) : 0;
    const int64_t nhi = lifted ? (p->n >> p->log2h) : 0;
    const int64_t nlo = lifted ? (int64_t(1) << p->log2h) : 0;
    char *tb = static_cast<char *>(p->tables);
    p->tw1 = tb;
    char *t2 = tb + n1 * esize, *t3 = t2 + n2 * esize, *th = t3 + n3 * esize, *tl = th + nhi * esize;
    if (lifted) {
        p->tw2 = t2;
        p->tw3 = t3;
        p->tw_hi = th;
        p->tw_lo = tl;
    }
    if (!generate) return FFT_OK;
    int rc = gen_table(p->dtype, tb, n1, 1, p->k1.log2N, st);
    if (lifted) {
        if (rc == FFT_OK) rc = gen_table(p->dtype, t2, n2, 1, p->k2.log2N, st);
        if (rc == FFT_OK && n3) rc = gen_table(p->dtype, t3, n3, 1, p->k3.log2N, st);
        if (rc == FFT_OK) rc = gen_table(p->dtype, th, nhi, nlo, t, st);
        if (rc == FFT_OK) rc = gen_table(p->dtype, tl, nlo, 1, t, st);
    }
    return rc;
}

// Validate a single-length request and choose its lift, its launches and
// the sizes of its device memory (scratch array and weight tables) without
// touching device memory.  p is a freshly constructed plan; on an error the
// caller releases it.
int shape_plan(fft_plan *p, int64_t n, int64_t batch, int dtype, const fft_plan_opts *opts) {
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
    int radix = o.radix ? o.radix : 16;
    if (radix != 2 && radix != 16) {
        if (radix == 4 || radix == 8) return FFT_E_UNSUPPORTED;
        return FFT_E_ARG;
    }
    if (o.log2_p < 0 || (o.log2_p && o.log2_p >= t)) return FFT_E_ARG;
    if (o.lines_per_block < 0 || (o.lines_per_block & (o.lines_per_block - 1))) return FFT_E_ARG;
    if (o.lines_per_block2 < 0 || (o.lines_per_block2 & (o.lines_per_block2 - 1))) return FFT_E_ARG;
    constexpr int32_t known_flags = FFT_OPT_NO_XCD_REMAP | FFT_OPT_SPLIT_EXCHANGE | FFT_OPT_FULL_EXCHANGE |
                                    FFT_OPT_PERSISTENT | FFT_OPT_ONE_TILE | FFT_OPT_DENSE |
                                    FFT_OPT_TWO_LEVEL | FFT_OPT_THREE_LEVEL | FFT_OPT_SHUFFLE_EXCHANGE |
                                    FFT_OPT_LDS_PREFETCH | FFT_OPT_DEBUG_CANARY | FFT_OPT_TILE_ORDER |
                                    FFT_OPT_ROW_LANES;
    // the staged pass 1 is a two-level variant of its own
    if ((o.flags & FFT_OPT_LDS_PREFETCH) &&
        (!(o.flags & FFT_OPT_TWO_LEVEL) || (o.flags & (FFT_OPT_SPLIT_EXCHANGE | FFT_OPT_FULL_EXCHANGE |
                                                         FFT_OPT_PERSISTENT | FFT_OPT_DENSE)) ||
         o.values_per_thread || o.scratch_width || (o.lines_per_block && o.lines_per_block != 2)))
        return FFT_E_ARG;
    // so is the row-lane pass 1
    if ((o.flags & FFT_OPT_ROW_LANES) &&
        (!(o.flags & FFT_OPT_TWO_LEVEL) || (o.flags & (FFT_OPT_SPLIT_EXCHANGE | FFT_OPT_FULL_EXCHANGE |
                                                         FFT_OPT_PERSISTENT | FFT_OPT_DENSE | FFT_OPT_LDS_PREFETCH)) ||
         o.scratch_width || (o.lines_per_block && o.lines_per_block != 2)))
        return FFT_E_ARG;
    // the shuffle exchange exists for three-level plans only, as the only variant
    if ((o.flags & FFT_OPT_SHUFFLE_EXCHANGE) &&
        (!(o.flags & FFT_OPT_THREE_LEVEL) || (o.flags & (FFT_OPT_SPLIT_EXCHANGE | FFT_OPT_FULL_EXCHANGE |
                                                           FFT_OPT_PERSISTENT | FFT_OPT_DENSE)) ||
         o.values_per_thread))
        return FFT_E_ARG;
    if (o.flags & ~known_flags) return FFT_E_ARG;
    if ((o.flags & FFT_OPT_TWO_LEVEL) && (o.flags & FFT_OPT_THREE_LEVEL)) return FFT_E_ARG;
    if ((o.flags & FFT_OPT_THREE_LEVEL) && (o.log2_p || o.lines_per_block2 || o.values_per_thread2 ||
                                             o.scratch_width))
        return FFT_E_ARG; // two-level options
    if ((o.flags & FFT_OPT_SPLIT_EXCHANGE) && (o.flags & FFT_OPT_FULL_EXCHANGE)) return FFT_E_ARG;
    if ((o.flags & FFT_OPT_PERSISTENT) && (o.flags & FFT_OPT_ONE_TILE)) return FFT_E_ARG;
    if (o.values_per_thread != 0 && o.values_per_thread != 16 && o.values_per_thread != 32)
        return FFT_E_ARG;
    if (o.values_per_thread2 != 0 && o.values_per_thread2 != 16 && o.values_per_thread2 != 32)
        return FFT_E_ARG;
    if (o.scratch_width < 0 || (o.scratch_width & (o.scratch_width - 1))) return FFT_E_ARG;
    if (o.flags & FFT_OPT_TILE_ORDER) {
        if (o.tile_order & int32_t(0xff000000)) return FFT_E_ARG;
        for (int k = 0; k < 3; ++k) {
            const int b = (o.tile_order >> (8 * k)) & 0xff;
            if ((b & 0x80) && b != 0x80) return FFT_E_ARG;
            if ((o.flags & FFT_OPT_NO_XCD_REMAP) && b != 0 && b != 0x80 && (b & 15)) return FFT_E_ARG;
        }
    } else if (o.tile_order) {
        return FFT_E_ARG;
    }
    // Pass-kernel variant: the defaults unless the options ask for another.
    Variant var;
    // (with FFT_OPT_ROW_LANES values_per_thread sets the row-lane pass 1 alone)
    if (o.values_per_thread && !(o.flags & FFT_OPT_ROW_LANES)) var.emax = o.values_per_thread;
    if (o.flags & FFT_OPT_SPLIT_EXCHANGE) var.split = true;
    if (o.flags & FFT_OPT_PERSISTENT) var.persist = true;
    if (o.flags & FFT_OPT_DENSE) var.dense = true;
    if (o.flags & FFT_OPT_SHUFFLE_EXCHANGE) var.shuffle = true;
    Variant var2 = var;
    if (o.values_per_thread2) var2.emax = o.values_per_thread2;
    const bool forced = !var.is_default() || !var2.is_default();
    p->n = n;
    p->batch = batch;
    p->total = n * batch;
    p->dtype = dtype;
    p->log2n = t;
    p->radix = radix;
    p->esize = esize;
    p->canary = (o.flags & FFT_OPT_DEBUG_CANARY) != 0;
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        return FFT_E_HIP;
    }

    const int mline = max_line(dtype);
    const bool three = (o.flags & FFT_OPT_THREE_LEVEL) ||
                       (!(o.flags & FFT_OPT_TWO_LEVEL) && !o.log2_p && !o.lines_per_block && !o.lines_per_block2 &&
                        !o.scratch_width && !o.values_per_thread2 && default_three_level(t, dtype, radix, var));
    if (three) {
        // n = n1 n2 n3: n1 the contiguous rows of the last pass, n3 the
        // slowest axis (first pass); near-equal factors, n3 >= n1 >= n2.
        p->passes = 3;
        p->log2n3 = (t + 2) / 3;
        p->log2n1 = (t - p->log2n3 + 1) / 2;
        p->log2n2 = t - p->log2n3 - p->log2n1;
        const int l1 = p->log2n1, l2 = p->log2n2, l3 = p->log2n3;
        if (radix != 16 || l2 < AXIS_LMIN || l3 > AXIS_LMAX) {
            return FFT_E_UNSUPPORTED;
        }
        const int want = o.lines_per_block;
        const int kind = n * int64_t(esize) > (int64_t(1) << 31) ? K_AXIS_WIDE : K_AXIS;
        // The shuffle exchange applies to the passes over 256-point lines;
        // the others keep the default kernel.
        auto axis_var = [&](int l2N) {
            Variant v = var;
            if (v.shuffle && (l2N != 8 || dtype != FFT_C64 || kind != K_AXIS)) v.shuffle = false;
            return v;
        };
        if (var.shuffle && ((l1 != 8 && l2 != 8 && l3 != 8) || dtype != FFT_C64 || kind != K_AXIS))
            return FFT_E_UNSUPPORTED;
        if (!plan_pass(p->k1, dtype, kind, l3, radix, int64_t(1) << l1, batch << (l1 + l2), want, 0, axis_var(l3),
                       p->device) ||
            !plan_pass(p->k2, dtype, kind, l2, radix, int64_t(1) << l1, batch << (l1 + l3), want, 0, axis_var(l2),
                       p->device) ||
            !plan_pass(p->k3, dtype, kind, l1, radix, int64_t(1) << l3, batch << (l2 + l3), want, 0, axis_var(l1),
                       p->device)) {
            return FFT_E_UNSUPPORTED;
        }
    } else if (o.log2_p == 0 && t <= mline) {
        p->passes = 1;
        p->log2q = t;
        if (forced) { // the other variants are pass kernels only
            return FFT_E_UNSUPPORTED;
        }
        const int l2T = o.lines_per_block ? ilog2_exact(o.lines_per_block)
                                          : choose_log2T(t, radix, esize, batch, 256, 1, 0, K_SINGLE, var);
        if (!fill_launch(p->k1, dtype, K_SINGLE, t, radix, l2T, batch, var, p->device)) {
            return FFT_E_UNSUPPORTED;
        }
    } else {
        p->passes = 2;
        p->log2q = o.log2_p ? t - o.log2_p : (t + 1) / 2;
        p->log2p = t - p->log2q;
        if (p->log2q > mline || p->log2p > mline) {
            return FFT_E_UNSUPPORTED;
        }
        const int64_t P = int64_t(1) << p->log2p, Q = int64_t(1) << p->log2q;
        // Pass 2 reads the scratch tile layout of pass 1 with a separable
        // offset, which needs T1 | TPL2 (TPL2 = threads per pass-2 line).
        // Default variant per pass: complex64 radix-16 lines of 2^10..2^12 use
        // the split exchange (measured faster at n = 2^24: the halved tile
        // lets more tiles share a CU; see the design notes).
        auto pass_variant = [&](int log2N, const Variant &base) {
            Variant v = base;
            if (!forced && !(o.flags & FFT_OPT_FULL_EXCHANGE) && dtype == FFT_C64 && radix == 16 &&
                log2N >= VARIANT_LMIN)
                v.split = true;
            return v;
        };
        const Variant v1 = pass_variant(p->log2q, var), v2 = pass_variant(p->log2p, var2);
        const int tpl2 = int(P / vals_per_thread(int(P), v2.emax));
        // Scratch slab width W: pass 1's tile width unless given; pass 2
        // reads W-wide slabs with a separable offset, so W | TPL2.
        if (o.scratch_width > tpl2) {
            return FFT_E_UNSUPPORTED;
        }
        if (!plan_pass(p->k1, dtype, K_PASS1, p->log2q, radix, P, P * batch, o.lines_per_block,
                       o.scratch_width ? 0 : tpl2, v1, p->device) ||
            !plan_pass(p->k2, dtype, K_PASS2, p->log2p, radix, Q, Q * batch, o.lines_per_block2, 0, v2,
                       p->device)) {
            return FFT_E_UNSUPPORTED;
        }
        p->log2W = o.scratch_width ? ilog2_exact(o.scratch_width) : p->k1.log2T;
        if (o.flags & FFT_OPT_LDS_PREFETCH) {
            // Pass 1 with the next tile staged in LDS: 4096-point complex64
            // columns, 2 per tile, slabs of width 2.  The plain pass-1 launch
            // stays for inputs not 16-byte aligned.
            Variant vd;
            vd.split = true;
            vd.lds_prefetch = true;
            p->k1_plain = p->k1;
            if (dtype != FFT_C64 || radix != 16 || p->log2q != 12 || p->log2W != 1 || p->k1.log2T != 1 ||
                !fill_launch(p->k1, dtype, K_PASS1, 12, 16, 1, P * batch, vd, p->device))
                return FFT_E_UNSUPPORTED;
        }
        if (o.flags & FFT_OPT_ROW_LANES) {
            // Pass 1 with whole rows per thread: 4096-point complex64
            // columns, 2 per tile, slabs of width 2.
            Variant vr;
            vr.split = true;
            vr.rows = true;
            vr.emax = o.values_per_thread ? o.values_per_thread : 16;
            p->k1_plain = p->k1; // for inputs not 16-byte aligned
            if (dtype != FFT_C64 || radix != 16 || p->log2q != 12 || p->log2W != 1 || p->k1.log2T != 1 ||
                !fill_launch(p->k1, dtype, K_PASS1, 12, 16, 1, P * batch, vr, p->device))
                return FFT_E_UNSUPPORTED;
        }
    }
    p->no_remap = (o.flags & FFT_OPT_NO_XCD_REMAP) != 0;
    p->kernel_defaults = !forced && radix == 16 && !o.lines_per_block && !o.lines_per_block2 &&
                         !o.scratch_width &&
                         !(o.flags & (FFT_OPT_SPLIT_EXCHANGE | FFT_OPT_FULL_EXCHANGE | FFT_OPT_LDS_PREFETCH |
                                      FFT_OPT_ROW_LANES));
    p->tile_order_set = (o.flags & FFT_OPT_TILE_ORDER) != 0;
    p->tile_order = o.tile_order;
    if (p->tile_order_set && (o.tile_order >> (8 * p->passes))) return FFT_E_ARG; // bytes beyond the passes
    if (const int orc = apply_remap_policy(p)) return orc;
    p->base1 = p->k1.var;
    p->base2 = p->k2.var;
    p->base3 = p->k3.var;
    if (!p->k1.fn || (p->passes >= 2 && !p->k2.fn) || (p->passes == 3 && !p->k3.fn)) {
        return FFT_E_UNSUPPORTED;
    }

    // Device memory: scratch (lifted plans only) and the weight tables: one
    // w_N table per pass (N its line length) and the two-level w_n table.
    const bool lifted = p->passes >= 2;
    p->log2h = lifted ? (t + 1) / 2 : 0;
    p->table_bytes = size_t(table_entries(p)) * esize;
    p->scratch_bytes = lifted ? size_t(n) * size_t(batch) * esize : 0;
    return FFT_OK;
}

// Scratch of the allocation-free entry point fft_execute_static: the
// inter-pass array (up to STATIC_SCRATCH_BYTES) followed by the weight
// tables (up to STATIC_TABLE_BYTES).  Each GPU the library runs on holds its
// own copy until the process ends; every call on that GPU shares it.  In host
// code the array's name is only a stand-in: kernels get the device address
// that hipGetSymbolAddress returns for the current device (StaticDevice).
constexpr size_t STATIC_SCRATCH_BYTES = size_t(32) << 20;
constexpr size_t STATIC_TABLE_BYTES = size_t(256) << 10;
__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES + STATIC_TABLE_BYTES];

// Per device: the address of `scratch` there, and which transform's tables
// the array holds (the last call's, in host order).
struct StaticDevice {
    bool ready = false;
    unsigned char *ptr = nullptr;
    int64_t table_n = 0;
    int table_dtype = -1;
};
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex static_mutex;
StaticDevice static_devices[STATIC_MAX_DEVICES];

// Class plans of a packed batch (p: its lengths grouped by log2 length in
// by_t as packed offsets; total elements, dtype, device set).  Each class is
// shaped like fft_plan_create(2^t, count) -- or, with `tune`, like the
// fastest configuration fft_plan_create_tuned finds for that shape -- and
// addresses its transforms through a device list of offsets; the tables of
// all classes share one allocation and the lifted classes one scratch array
// with the packed layout.  Classes are dealt to four lanes (streams) by
// decreasing size.
int build_class_plans(fft_plan *p, const std::vector<std::vector<int64_t>> &by_t, bool tune) {
    const int dtype = p->dtype;
    struct Spec {
        int t;
        size_t first; // index of its first offset
        int64_t count;
    };
    std::vector<Spec> specs;
    std::vector<int64_t> offsets;
    for (int t = int(by_t.size()) - 1; t >= 1; --t) { // longest first
        if (by_t[t].empty()) continue;
        specs.push_back({t, offsets.size(), int64_t(by_t[t].size())});
        offsets.insert(offsets.end(), by_t[t].begin(), by_t[t].end());
    }
    p->length_classes = int(specs.size());
    size_t table_bytes = 0;
    bool lifted = false;
    p->passes = 1;
    for (const Spec &sp : specs) {
        fft_plan *sub = new (std::nothrow) fft_plan;
        if (!sub) return FFT_E_OOM;
        p->runs.push_back({sub, 0});
        fft_plan_opts o;
        memset(&o, 0, sizeof(o));
        if (tune) {
            fft_plan *tp = nullptr;
            fft_tune_result res;
            const int rc = fft_plan_create_tuned(int64_t(1) << sp.t, sp.count, dtype, 16, &tp, &res);
            if (rc != FFT_OK) return rc;
            fft_plan_destroy(tp);
            o = res.opts;
        }
        const int rc = shape_plan(sub, int64_t(1) << sp.t, sp.count, dtype, &o);
        if (rc != FFT_OK) return rc;
        table_bytes += (sub->table_bytes + 255) & ~size_t(255);
        lifted = lifted || sub->passes >= 2;
    }
    p->passes = lifted ? 2 : 1; // timing: the whole batch, then an empty second interval
    p->table_bytes = table_bytes;
    if (hipMalloc(&p->tables, p->table_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->tables = nullptr;
        return FFT_E_OOM;
    }
    if (lifted) {
        p->scratch_bytes = size_t(p->total) * p->esize;
        if (hipMalloc(&p->scratch, p->scratch_bytes) != hipSuccess) {
            (void)hipGetLastError();
            p->scratch = nullptr;
            return FFT_E_OOM;
        }
    }
    p->meta_bytes = offsets.size() * sizeof(int64_t);
    if (hipMalloc(&p->meta, p->meta_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->meta = nullptr;
        return FFT_E_OOM;
    }
    if (hipMemcpy(p->meta, offsets.data(), p->meta_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return FFT_E_HIP;
    }
    const int64_t *dev_offsets = static_cast<const int64_t *>(p->meta);
    char *tb = static_cast<char *>(p->tables);
    // Lanes: classes by decreasing bytes, each to the lane with the least
    // work so far (lane 0 is the execute stream).
    std::vector<size_t> order(specs.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    auto bytes = [&](size_t k) {
        return (int64_t(1) << specs[k].t) * specs[k].count * int64_t(p->runs[k].sub->passes);
    };
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return bytes(a) > bytes(b); });
    const int lanes = int(specs.size()) < 1 + fft_plan::AUX ? int(specs.size()) : 1 + fft_plan::AUX;
    std::vector<int64_t> load(lanes, 0);
    for (size_t k : order) {
        int best = 0;
        for (int l = 1; l < lanes; ++l)
            if (load[l] < load[best]) best = l;
        p->runs[k].lane = best;
        load[best] += bytes(k);
    }
    int rc = FFT_OK;
    for (size_t k = 0; k < specs.size() && rc == FFT_OK; ++k) {
        fft_plan *sub = p->runs[k].sub;
        sub->tables = tb;
        tb += (sub->table_bytes + 255) & ~size_t(255);
        sub->scratch = sub->passes >= 2 ? p->scratch : nullptr;
        sub->offsets = dev_offsets + specs[k].first;
        sub->packed_total = p->total;
        rc = fill_tables(sub, nullptr);
    }
    // Run in the order of the work list (longest lengths first), so that in
    // each lane the large classes start first.
    std::stable_sort(p->runs.begin(), p->runs.end(), [](const fft_plan::ClassRun &a, const fft_plan::ClassRun &b) {
        return a.sub->n > b.sub->n;
    });
    if (rc == FFT_OK && hipDeviceSynchronize() != hipSuccess) rc = FFT_E_HIP;
    if (rc != FFT_OK) return rc;
    p->lanes = lanes;
    if (lanes > 1) {
        if (hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            p->fork_ev = nullptr;
            return FFT_E_HIP;
        }
        for (int k = 0; k + 1 < lanes; ++k) {
            if (hipStreamCreateWithFlags(&p->aux[k], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&p->join_ev[k], hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return FFT_E_HIP;
            }
        }
    }
    return FFT_OK;
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
    case FFT_E_UNSUPPORTED: return "valid request outside what the library supports";
    case FFT_E_ARG: return "invalid option";
    case FFT_E_CAPACITY: return "request exceeds the fixed scratch of fft_execute_static";
    default: return "unknown status code";
    }
}

int fft_plan_create_ex(int64_t n, int64_t batch, int dtype, const fft_plan_opts *opts,
                       fft_plan **plan_out) {
    if (!plan_out) return FFT_E_NULL;
    *plan_out = nullptr;
    fft_plan *p = new (std::nothrow) fft_plan;
    if (!p) return FFT_E_OOM;
    int rc = shape_plan(p, n, batch, dtype, opts);
    if (rc != FFT_OK) {
        free_plan(p);
        return rc;
    }
    if (hipMalloc(&p->tables, p->table_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->tables = nullptr;
        free_plan(p);
        return FFT_E_OOM;
    }
    if (p->scratch_bytes && hipMalloc(&p->scratch, p->scratch_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->scratch = nullptr;
        free_plan(p);
        return FFT_E_OOM;
    }
    rc = fill_tables(p, nullptr);
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

int fft_plan_create_paper(int64_t n, int64_t batch, int dtype, int32_t log2_m, int32_t breakpoint,
                          fft_plan **plan_out) {
    if (!plan_out) return FFT_E_NULL;
    *plan_out = nullptr;
    if (dtype != FFT_C64 && dtype != FFT_C128) return FFT_E_DTYPE;
    const int t = ilog2_exact(n);
    if (t < 1 || batch < 1) return FFT_E_SIZE;
    const size_t esize = dtype == FFT_C64 ? 8 : 16;
    if (batch > (INT64_MAX / 4) / n / int64_t(esize)) return FFT_E_SIZE;
    // m processors with psize = n/m >= m elements each; breakpoints
    // log2 m + 1 <= bp <= log2 psize + 1 (Section 4.8).
    if (log2_m < 0 || 2 * log2_m > t) return FFT_E_ARG;
    if (breakpoint < log2_m + 1 || breakpoint > t - log2_m + 1) return FFT_E_ARG;
    if (t > liftfft_paper::MAX_LOG2N || (batch << log2_m) > INT32_MAX) return FFT_E_UNSUPPORTED;

    fft_plan *p = new (std::nothrow) fft_plan;
    if (!p) return FFT_E_OOM;
    p->n = n;
    p->batch = batch;
    p->total = n * batch;
    p->dtype = dtype;
    p->log2n = t;
    p->radix = 2;
    p->esize = esize;
    p->passes = 2;
    p->paper = true;
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        return FFT_E_HIP;
    }
    p->pp.dtype = dtype;
    p->pp.log2n = t;
    p->pp.log2m = log2_m;
    p->pp.bp = breakpoint;
    p->pp.batch = batch;
    if (liftfft_paper::shape(p->pp) != int(hipSuccess)) {
        (void)hipGetLastError();
        free_plan(p);
        return FFT_E_HIP;
    }
    // Weights w_n^e, e < n/2, each from its integer exponent in FP64 (the
    // paper computes every weight directly, Section 3.5).
    const int64_t half = n / 2;
    p->table_bytes = size_t(half) * esize;
    p->scratch_bytes = size_t(n) * size_t(batch) * esize;
    if (hipMalloc(&p->tables, p->table_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->tables = nullptr;
        free_plan(p);
        return FFT_E_OOM;
    }
    if (hipMalloc(&p->scratch, p->scratch_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->scratch = nullptr;
        free_plan(p);
        return FFT_E_OOM;
    }
    p->pp.w = p->tables;
    int rc = gen_table(dtype, p->tables, half, 1, t);
    if (rc == FFT_OK && hipDeviceSynchronize() != hipSuccess) rc = FFT_E_HIP;
    if (rc != FFT_OK) {
        free_plan(p);
        return rc;
    }
    *plan_out = p;
    return FFT_OK;
}

int fft_plan_create_many(const int64_t *lengths, int64_t count, int dtype, uint32_t flags,
                         fft_plan **plan_out) {
    if (!plan_out) return FFT_E_NULL;
    *plan_out = nullptr;
    if (!lengths) return FFT_E_NULL;
    if (dtype != FFT_C64 && dtype != FFT_C128) return FFT_E_DTYPE;
    if (count < 1) return FFT_E_SIZE;
    if (flags & ~uint32_t(FFT_OPT_GRAPH | FFT_OPT_PERSISTENT | FFT_OPT_AUTOTUNE)) return FFT_E_ARG;
    if ((flags & FFT_OPT_PERSISTENT) && (flags & FFT_OPT_AUTOTUNE)) return FFT_E_ARG;
    const size_t esize = dtype == FFT_C64 ? 8 : 16;
    const int max_t = RAGGED_MAX_T, mline = max_line(dtype);
    // Lengths, packed offsets and the classes of equal length.
    std::vector<std::vector<int64_t>> by_t(max_t + 1);
    int64_t total = 0;
    bool unsupported = false;
    for (int64_t i = 0; i < count; ++i) {
        const int t = ilog2_exact(lengths[i]);
        if (t < 1) return FFT_E_SIZE;
        if (t > max_t) {
            unsupported = true;
            continue;
        }
        by_t[t].push_back(total);
        total += lengths[i];
        if (total > (int64_t(1) << 40)) return FFT_E_SIZE;
    }
    if (unsupported) return FFT_E_UNSUPPORTED;
    // Single-pass tiles address the packed buffer through one 32-bit
    // buffer descriptor.
    if (uint64_t(total) * esize > uint64_t(UINT32_MAX)) return FFT_E_UNSUPPORTED;

    fft_plan *p = new (std::nothrow) fft_plan;
    if (!p) return FFT_E_OOM;
    p->ragged = true;
    p->n = total;
    p->batch = count;
    p->total = total;
    p->dtype = dtype;
    p->esize = esize;
    p->radix = 16;
    p->use_graph = (flags & FFT_OPT_GRAPH) != 0;
    auto fail = [&](int rc) {
        free_plan(p);
        return rc;
    };
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FFT_E_HIP);
    }
    if (!(flags & FFT_OPT_PERSISTENT)) {
        const int rc = build_class_plans(p, by_t, (flags & FFT_OPT_AUTOTUNE) != 0);
        if (rc != FFT_OK) return fail(rc);
        *plan_out = p;
        return FFT_OK;
    }

    // Twiddle tables: w_N^e for each line length used, and the two-level
    // inter-pass tables of each lifted length.
    const int lsize = int(esize / 2), csize = int(esize);
    struct ClassSpec {
        int kind, log2N, t, log2T, log2W, pitch;
        int64_t lines, tiles, count;
        int64_t lds;
        size_t off_index; // first entry of the class's offsets
    };
    std::vector<ClassSpec> A, B;
    std::vector<int64_t> offsets;
    bool used_line[MAX_LOG2_LINE + 1] = {};
    bool two_pass = false;
    auto tile_lines = [](int log2N) {
        const int N = 1 << log2N;
        return RAGGED_THREADS / (N / vals_per_thread(N));
    };
    auto spec = [&](int kind, int log2N, int t, int64_t lines, int log2W, size_t off_index, int64_t cnt) {
        ClassSpec c;
        const int N = 1 << log2N, T = tile_lines(log2N), E = vals_per_thread(N);
        c.kind = kind;
        c.log2N = log2N;
        c.t = t;
        c.log2T = ilog2_exact(T);
        c.log2W = kind == K_SINGLE ? c.log2T : log2W;
        c.pitch = exchange_pitch(N, T, N / E, lsize, kind != K_SINGLE);
        c.lines = lines;
        c.tiles = (lines + T - 1) / T;
        c.count = cnt;
        c.lds = lds_bytes(N, 16, T, E, c.pitch, lsize, csize, kind == K_PASS1);
        c.off_index = off_index;
        used_line[log2N] = true;
        return c;
    };
    struct SingleSpec {
        int t;
        int64_t count;
        size_t off_index;
    };
    std::vector<SingleSpec> single_specs;
    int classes = 0;
    for (int t = max_t; t >= 1; --t) { // longest lines first
        if (by_t[t].empty()) continue;
        ++classes;
        const size_t oi = offsets.size();
        offsets.insert(offsets.end(), by_t[t].begin(), by_t[t].end());
        const int64_t cnt = int64_t(by_t[t].size());
        if (t <= mline) {
            single_specs.push_back({t, cnt, oi});
            used_line[t] = true;
        } else {
            two_pass = true;
            const int lq = (t + 1) / 2, lp = t - lq;
            // Scratch slabs W = min(T1, TPL2) wide: pass 2 reads them with a
            // separable offset.
            const int T1 = tile_lines(lq), tpl2 = (1 << lp) / vals_per_thread(1 << lp);
            const int lW = ilog2_exact(T1 < tpl2 ? T1 : tpl2);
            A.push_back(spec(K_PASS1, lq, t, cnt << lp, lW, oi, cnt));
            B.push_back(spec(K_PASS2, lp, t, cnt << lq, lW, oi, cnt));
        }
    }
    p->length_classes = classes;
    p->passes = two_pass ? 2 : 1;

    // Device memory: tables, scratch (two-pass classes), classes + offsets.
    std::vector<int64_t> tab_off(MAX_LOG2_LINE + 1, -1);
    std::vector<int64_t> hi_off(max_t + 1, -1), lo_off(max_t + 1, -1);
    int64_t entries = 0;
    for (int L = 1; L <= MAX_LOG2_LINE; ++L)
        if (used_line[L]) {
            tab_off[L] = entries;
            entries += int64_t(1) << L;
        }
    for (int t = mline + 1; t <= max_t; ++t)
        if (!by_t[t].empty()) {
            const int h = (t + 1) / 2;
            hi_off[t] = entries;
            entries += int64_t(1) << (t - h);
            lo_off[t] = entries;
            entries += int64_t(1) << h;
        }
    p->table_bytes = size_t(entries) * esize;
    if (hipMalloc(&p->tables, p->table_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->tables = nullptr;
        return fail(FFT_E_OOM);
    }
    if (two_pass) {
        p->scratch_bytes = size_t(total) * esize;
        if (hipMalloc(&p->scratch, p->scratch_bytes) != hipSuccess) {
            (void)hipGetLastError();
            p->scratch = nullptr;
            return fail(FFT_E_OOM);
        }
    }
    const size_t ncls = A.size() + B.size();
    p->meta_bytes = ncls * sizeof(RaggedClass) + offsets.size() * sizeof(int64_t);
    if (hipMalloc(&p->meta, p->meta_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->meta = nullptr;
        return fail(FFT_E_OOM);
    }
    char *tb = static_cast<char *>(p->tables);
    int rc = FFT_OK;
    for (int L = 1; L <= MAX_LOG2_LINE && rc == FFT_OK; ++L)
        if (tab_off[L] >= 0) rc = gen_table(dtype, tb + tab_off[L] * esize, int64_t(1) << L, 1, L);
    for (int t = mline + 1; t <= max_t && rc == FFT_OK; ++t)
        if (hi_off[t] >= 0) {
            const int h = (t + 1) / 2;
            rc = gen_table(dtype, tb + hi_off[t] * esize, int64_t(1) << (t - h), int64_t(1) << h, t);
            if (rc == FFT_OK) rc = gen_table(dtype, tb + lo_off[t] * esize, int64_t(1) << h, 1, t);
        }
    if (rc != FFT_OK) return fail(rc);

    // Class records.
    char *meta = static_cast<char *>(p->meta);
    const int64_t *dev_offsets = reinterpret_cast<const int64_t *>(meta + ncls * sizeof(RaggedClass));
    std::vector<RaggedClass> recs(ncls);
    auto fill = [&](const ClassSpec &c, RaggedClass &r, int64_t item_begin) {
        memset(&r, 0, sizeof(r));
        r.kind = c.kind;
        r.log2N = c.log2N;
        r.item_begin = item_begin;
        PassArgs &a = r.a;
        a.tw = tb + tab_off[c.log2N] * esize;
        a.lines = c.lines;
        a.ntiles = c.tiles;
        a.log2T = c.log2T;
        a.log2T1 = c.log2W;
        a.pitch = c.pitch;
        a.offsets = dev_offsets + c.off_index;
        a.total = total;
        if (c.kind == K_SINGLE) {
            a.n = int64_t(1) << c.t;
        } else {
            const int lq = (c.t + 1) / 2;
            a.n = int64_t(1) << c.t;
            a.log2q = lq;
            a.log2p = c.t - lq;
            a.log2h = lq;
            a.tw_hi = tb + hi_off[c.t] * esize;
            a.tw_lo = tb + lo_off[c.t] * esize;
            if (c.kind == K_PASS1) a.out = p->scratch;
            else a.in = p->scratch;
        }
    };
    auto build_launch = [&](std::vector<ClassSpec> &cs, size_t first, fft_plan::RaggedLaunch &R) -> int {
        R.nclass = int(cs.size());
        R.cls = meta + first * sizeof(RaggedClass);
        int64_t items = 0, lds = 0;
        for (size_t k = 0; k < cs.size(); ++k) {
            fill(cs[k], recs[first + k], items);
            items += cs[k].tiles;
            if (cs[k].lds > lds) lds = cs[k].lds;
        }
        R.items = items;
        R.lds = size_t(lds);
        if (items == 0) return FFT_OK;
        if (lds > LDS_BUDGET) return FFT_E_UNSUPPORTED;
        const void *fn = dtype == FFT_C64 ? reinterpret_cast<const void *>(&ragged_kernel<float>)
                                          : reinterpret_cast<const void *>(&ragged_kernel<double>);
        int per_cu = 0, cus = 0;
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(LDS_BUDGET)) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, RAGGED_THREADS, R.lds) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
            (void)hipGetLastError();
            return FFT_E_HIP;
        }
        if (per_cu < 1) return FFT_E_UNSUPPORTED;
        const int64_t resident = int64_t(per_cu) * cus;
        R.grid = items < resident ? items : resident;
        if (R.grid >= 8) R.grid &= ~int64_t(7);
        return FFT_OK;
    };
    rc = build_launch(A, 0, p->ra);
    if (rc == FFT_OK) rc = build_launch(B, A.size(), p->rb);
    if (rc != FFT_OK) return fail(rc);
    // Single-pass classes: the tuned single-pass kernel, one launch each.
    for (const SingleSpec &ss : single_specs) {
        fft_plan::SingleClass sc;
        const Variant v;
        const int l2T = choose_log2T(ss.t, 16, esize, ss.count, 256, 1, 0, K_SINGLE, v);
        if (!fill_launch(sc.L, dtype, K_SINGLE, ss.t, 16, l2T, ss.count, v, p->device)) return fail(FFT_E_UNSUPPORTED);
        memset(&sc.a, 0, sizeof(sc.a));
        sc.a.tw = tb + tab_off[ss.t] * esize;
        sc.a.lines = ss.count;
        sc.a.n = int64_t(1) << ss.t;
        sc.a.ntiles = sc.L.ntiles;
        sc.a.log2T = sc.a.log2T1 = sc.L.log2T;
        sc.a.pitch = sc.L.pitch;
        sc.a.xcd_remap = sc.L.remap;
        sc.a.offsets = dev_offsets + ss.off_index;
        sc.a.total = total;
        p->singles.push_back(sc);
    }
    if (hipMemcpy(meta, recs.data(), ncls * sizeof(RaggedClass), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(meta + ncls * sizeof(RaggedClass), offsets.data(), offsets.size() * sizeof(int64_t),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return fail(FFT_E_HIP);
    }
    *plan_out = p;
    return FFT_OK;
}

} // extern "C"

namespace {

// Enqueue every launch of plan p on stream st (arguments already checked,
// p's device current).
// Debug mode: quiet NaNs over `bytes` bytes at `dst` (stream order).
int canary_fill(void *dst, size_t bytes, hipStream_t st) {
    const int64_t words = int64_t(bytes / 4);
    if (words <= 0) return FFT_OK;
    const int64_t blocks = (words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096;
    hipLaunchKernelGGL(canary_fill_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, static_cast<uint32_t *>(dst),
                       words);
    return hipGetLastError() == hipSuccess ? FFT_OK : FFT_E_HIP;
}

int launch_plan(const fft_plan *p, const void *in, void *out, int sign, hipStream_t st) {
    const bool inv = sign > 0;
    const size_t out_bytes = size_t(p->total) * p->esize;
    PassArgs a;
    memset(&a, 0, sizeof(a));
    a.n = p->n;
    a.log2p = p->log2p;
    a.log2q = p->log2q;
    a.log2h = p->log2h;
    a.dft_ops = p->dft_ops;
    a.offsets = p->offsets;
    a.total = p->packed_total;
    int rc = FFT_OK;
    const hipEvent_t *ev = nullptr;
    if (p->timing) {
        if (p->ring_count == TIMING_RING) { // oldest slot still pending: drain it first
            const int slot = p->ring_head;
            rc = drain_slot(p, slot);
            --p->ring_count;
        }
        ev = &p->ev[size_t(p->ring_head) * RING_EVENTS];
        if (rc == FFT_OK && !p->ragged) rc = hipEventRecord(ev[0], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
    }
    if (p->ragged) {
        if (rc == FFT_OK) rc = execute_ragged(p, in, out, sign, st, ev);
    } else if (p->paper) {
        for (int phase = 0; phase < 2 && rc == FFT_OK; ++phase) {
            rc = liftfft_paper::launch(p->pp, phase, in, out, p->scratch, sign, st) == int(hipSuccess) ? FFT_OK
                                                                                                      : FFT_E_HIP;
            if (rc == FFT_OK && ev) rc = hipEventRecord(ev[phase + 1], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
        }
    } else if (p->passes == 1) {
        if (rc == FFT_OK && p->canary && out != in) rc = canary_fill(out, out_bytes, st);
        a.in = in;
        a.out = out;
        a.tw = p->tw1;
        a.lines = p->k1.lines;
        a.ntiles = p->k1.ntiles;
        a.pitch = p->k1.pitch;
        a.log2T = a.log2T1 = p->k1.log2T;
        a.conj_in = a.conj_out = inv;
        a.xcd_remap = p->k1.remap;
        if (rc == FFT_OK) rc = launch(p, p->k1, a, st);
        if (rc == FFT_OK && ev) rc = hipEventRecord(ev[1], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
    } else if (p->passes == 3) {
        // x -> out (slowest axis, weights w_(n2 n3)), out -> scratch (middle
        // axis, weights w_n), scratch -> out (contiguous rows, natural order).
        const int l1 = p->log2n1, l2 = p->log2n2, l3 = p->log2n3;
        const void *src[3] = {in, out, p->scratch};
        void *dst[3] = {out, p->scratch, out};
        const void *tw[3] = {p->tw1, p->tw2, p->tw3};
        const Launch *K[3] = {&p->k1, &p->k2, &p->k3};
        const int32_t U[3] = {l1, l1, l3}, Lt[3] = {l1 + l2, l1 + l3, l2 + l3};
        const int32_t ins[3][3] = {{0, l1, l1 + l2}, {0, l1 + l2, l1}, {l1 + l2, l1, 0}};
        const int32_t outs[3][3] = {{0, l1, l1 + l2}, {0, l1 + l2, l1}, {0, l3, l2 + l3}};
        a.tw_hi = p->tw_hi;
        a.tw_lo = p->tw_lo;
        if (rc == FFT_OK && p->canary) {
            rc = canary_fill(p->scratch, p->scratch_bytes, st);
            if (rc == FFT_OK && out != in) rc = canary_fill(out, out_bytes, st);
        }
        for (int k = 0; k < 3 && rc == FFT_OK; ++k) {
            // pass C rewrites `out`, which pass B has finished reading
            if (k == 2 && p->canary) rc = canary_fill(out, out_bytes, st);
            if (rc != FFT_OK) break;
            a.in = src[k];
            a.out = dst[k];
            a.tw = tw[k];
            a.lines = K[k]->lines;
            a.ntiles = K[k]->ntiles;
            a.pitch = K[k]->pitch;
            a.log2T = a.log2T1 = K[k]->log2T;
            a.conj_in = k == 0 ? inv : 0;
            a.conj_out = k == 2 ? inv : 0;
            a.xcd_remap = K[k]->remap;
            a.ax_log2U = U[k];
            a.ax_log2L = Lt[k];
            for (int d = 0; d < 3; ++d) {
                a.ax_in[d] = ins[k][d];
                a.ax_out[d] = outs[k][d];
            }
            a.ax_tw = k == 2 ? 0 : k + 1;
            a.ax_log2m = k == 1 ? l3 : 0;
            rc = launch(p, *K[k], a, st);
            if (rc == FFT_OK && ev) rc = hipEventRecord(ev[k + 1], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
        }
    } else {
        // The LDS-staged and the row-lane pass 1 load 16-byte row pairs:
        // other inputs take the plain pass-1 kernel.
        const Launch &K1 = (p->k1.var.lds_prefetch || p->k1.var.rows) && (reinterpret_cast<uintptr_t>(in) & 15)
                               ? p->k1_plain
                               : p->k1;
        if (rc == FFT_OK && p->canary) rc = canary_fill(p->scratch, p->scratch_bytes, st);
        a.in = in;
        a.out = p->scratch;
        a.tw = p->tw1;
        a.tw_hi = p->tw_hi;
        a.tw_lo = p->tw_lo;
        a.lines = K1.lines;
        a.ntiles = K1.ntiles;
        a.pitch = K1.pitch;
        a.log2T = K1.log2T;
        a.log2T1 = p->log2W;
        a.conj_in = inv;
        a.conj_out = 0;
        a.xcd_remap = K1.remap;
        if (rc == FFT_OK) rc = launch(p, K1, a, st);
        if (rc == FFT_OK && ev) rc = hipEventRecord(ev[1], st) == hipSuccess ? FFT_OK : FFT_E_HIP;
        // pass 1 has read the input: `out` (possibly the input) is free
        if (rc == FFT_OK && p->canary) rc = canary_fill(out, out_bytes, st);
        a.in = p->scratch;
        a.out = out;
        a.tw = p->tw2;
        a.lines = p->k2.lines;
        a.ntiles = p->k2.ntiles;
        a.pitch = p->k2.pitch;
        a.log2T = p->k2.log2T;
        a.log2T1 = p->log2W;
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
    return rc;
}

// Checks shared by the execute entry points: pointers, sign, alignment and
// overlap of the n*batch-element buffers.
int check_execute(const void *in, void *out, int sign, size_t esize, int64_t total) {
    if (!in || !out) return FFT_E_NULL;
    if (sign != -1 && sign != 1) return FFT_E_SIGN;
    if ((reinterpret_cast<uintptr_t>(in) % esize) || (reinterpret_cast<uintptr_t>(out) % esize))
        return FFT_E_ALIGN;
    // Partial overlap of in and out is not allowed (exact aliasing is).
    const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
    const uintptr_t bytes = uintptr_t(total) * esize;
    if (a != b && a < b + bytes && b < a + bytes) return FFT_E_ARG;
    return FFT_OK;
}

} // namespace

extern "C" {

int fft_execute(const fft_plan *plan, const void *in, void *out, int sign, void *stream) {
    if (!plan) return FFT_E_NULL;
    const int chk = check_execute(in, out, sign, plan->esize, plan->total);
    if (chk != FFT_OK) return chk;
    const fft_plan *p = plan;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return FFT_E_HIP;
    if (cur != p->device && hipSetDevice(p->device) != hipSuccess) return FFT_E_HIP;
    const int rc = launch_plan(p, in, out, sign, st);
    if (cur != p->device) (void)hipSetDevice(cur);
    return rc;
}

int fft_execute_static(int64_t n, int64_t batch, int dtype, const void *in, void *out, int sign, void *stream) {
    // The plan lives on the stack and owns no device memory: its scratch
    // array and tables point into this device's `scratch`.
    fft_plan p;
    int rc = shape_plan(&p, n, batch, dtype, nullptr);
    if (rc != FFT_OK) return rc;
    if (p.scratch_bytes > STATIC_SCRATCH_BYTES || p.table_bytes > STATIC_TABLE_BYTES) return FFT_E_CAPACITY;
    rc = check_execute(in, out, sign, p.esize, p.total);
    if (rc != FFT_OK) return rc;
    if (p.device < 0 || p.device >= STATIC_MAX_DEVICES) return FFT_E_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> g(static_mutex);
    StaticDevice &d = static_devices[p.device];
    if (!d.ready) { // once per device, with that device current (shape_plan took the current one)
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return FFT_E_HIP;
        }
        d.ptr = static_cast<unsigned char *>(ptr);
        d.ready = true;
    }
    p.scratch = p.scratch_bytes ? d.ptr : nullptr;
    p.tables = d.ptr + STATIC_SCRATCH_BYTES;
    const bool regenerate = d.table_n != n || d.table_dtype != dtype;
    rc = fill_tables(&p, st, regenerate);
    if (rc == FFT_OK && regenerate) {
        d.table_n = n;
        d.table_dtype = dtype;
    } else if (rc != FFT_OK) {
        d.table_n = 0; // contents unknown: regenerate next time
        d.table_dtype = -1;
    }
    if (rc == FFT_OK) rc = launch_plan(&p, in, out, sign, st);
    p.scratch = p.tables = nullptr;
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
    info->variant_pass1 = p->k1.var.code();
    info->variant_pass2 = p->passes == 2 ? p->k2.var.code() : 0;
    info->precision = p->precision;
    info->levels = p->ragged ? 0 : p->passes;
    if (!p->ragged && !p->paper) {
        const Launch *L[3] = {&p->k1, &p->k2, &p->k3};
        for (int k = 0; k < p->passes && k < 3; ++k) info->tile_order |= tile_order_byte(*L[k]) << (8 * k);
    }
    if (p->paper) {
        info->log2_p = p->pp.log2m;
        info->log2_q = p->log2n - p->pp.log2m;
        info->paper_breakpoint = p->pp.bp;
        info->lines_per_block_pass1 = info->lines_per_block_pass2 = 1;
        info->grid_pass1 = info->grid_pass2 = int32_t(p->batch << p->pp.log2m);
        info->threads_pass1 = info->threads_pass2 = p->pp.threads;
        info->lds_bytes_pass1 = info->lds_bytes_pass2 = int64_t(p->pp.lds_bytes);
        info->variant_pass1 = info->variant_pass2 = 0;
    }
    if (p->passes == 3 && !p->ragged) {
        info->log2_p = info->log2_q = 0;
        info->log2_n1 = p->log2n1;
        info->log2_n2 = p->log2n2;
        info->log2_n3 = p->log2n3;
        info->lines_per_block_pass2 = 1 << p->k2.log2T;
        info->grid_pass2 = int32_t(p->k2.grid);
        info->threads_pass2 = p->k2.threads;
        info->lds_bytes_pass2 = int64_t(p->k2.lds);
        info->variant_pass2 = p->k2.var.code();
        info->lines_per_block_pass3 = 1 << p->k3.log2T;
        info->grid_pass3 = int32_t(p->k3.grid);
        info->threads_pass3 = p->k3.threads;
        info->lds_bytes_pass3 = int64_t(p->k3.lds);
    }
    if (p->ragged && !p->runs.empty()) {
        info->lines_per_block_pass1 = info->lines_per_block_pass2 = 0;
        info->grid_pass1 = info->grid_pass2 = 0;
        info->threads_pass1 = info->threads_pass2 = 0;
        info->lds_bytes_pass1 = info->lds_bytes_pass2 = 0;
        info->variant_pass1 = info->variant_pass2 = 0;
        info->length_classes = p->length_classes;
        info->graph_launch = p->use_graph ? 1 : 0;
        info->streams = p->lanes;
    } else if (p->ragged) {
        info->lines_per_block_pass1 = info->lines_per_block_pass2 = 0;
        info->grid_pass1 = int32_t(p->ra.grid);
        info->grid_pass2 = int32_t(p->rb.grid);
        info->threads_pass1 = p->ra.items ? RAGGED_THREADS : 0;
        info->threads_pass2 = p->rb.items ? RAGGED_THREADS : 0;
        info->lds_bytes_pass1 = int64_t(p->ra.lds);
        info->lds_bytes_pass2 = int64_t(p->rb.lds);
        info->variant_pass1 = info->variant_pass2 = 2;
        info->length_classes = p->length_classes;
        info->graph_launch = p->use_graph ? 1 : 0;
    }
    return FFT_OK;
}

int fft_plan_set_precision(fft_plan *p, int mode) {
    if (!p) return FFT_E_NULL;
    if (mode != FFT_PREC_FP32 && mode != FFT_PREC_F16X2 && mode != FFT_PREC_BF16X2) return FFT_E_ARG;
    if (p->ragged || p->paper) return mode == FFT_PREC_FP32 ? FFT_OK : FFT_E_UNSUPPORTED;
    Launch n1 = p->k1, n2 = p->k2, n3 = p->k3;
    auto redo = [&](Launch &L, const Variant &base) {
        Variant v = base;
        if (mode != FFT_PREC_FP32) {
            v.split = false; // the matrix-core stages exchange complex elements
            v.rows = false;  // and run in the generic tile layout
            v.prec = mode;
        }
        return fill_launch(L, p->dtype, L.kind, L.log2N, L.rmax, L.log2T, L.lines, v, p->device);
    };
    if (!redo(n1, p->base1) || (p->passes >= 2 && !redo(n2, p->base2)) || (p->passes == 3 && !redo(n3, p->base3)))
        return FFT_E_UNSUPPORTED;
    if (mode != FFT_PREC_FP32 && p->dft_ops_prec != mode) {
        // The 16 x 16 DFT matrix in this form's operand layout, hi and lo
        // parts, generated once from FP64 angles.
        constexpr size_t OPS_BYTES = 64 * 4 * 16;
        if (!p->dft_ops && hipMalloc(&p->dft_ops, OPS_BYTES) != hipSuccess) {
            (void)hipGetLastError();
            p->dft_ops = nullptr;
            return FFT_E_OOM;
        }
        if (mode == FFT_PREC_F16X2)
            hipLaunchKernelGGL(dft_operand_table<PREC_F16X2>, dim3(1), dim3(64), 0, 0,
                               static_cast<MfmaOps<PREC_F16X2>::V *>(p->dft_ops));
        else
            hipLaunchKernelGGL(dft_operand_table<PREC_BF16X2>, dim3(1), dim3(64), 0, 0,
                               static_cast<MfmaOps<PREC_BF16X2>::V *>(p->dft_ops));
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            p->dft_ops_prec = 0;
            return FFT_E_HIP;
        }
        p->dft_ops_prec = mode;
    }
    p->k1 = n1;
    p->k2 = n2;
    p->k3 = n3;
    p->precision = mode;
    // the same grids as the kernels replaced, which took these orders (the
    // measured default orders are the FP32 kernels' only)
    (void)apply_remap_policy(p);
    return FFT_OK;
}

int fft_plan_set_timing(fft_plan *p, int enable) {
    if (!p) return FFT_E_NULL;
    if (enable && p->ev.empty()) {
        p->ev.assign(size_t(TIMING_RING) * RING_EVENTS, nullptr);
        // Timing-only events: without the system-scope fence a record does not
        // write back and invalidate the caches between the passes it brackets.
        for (auto &e : p->ev) {
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
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

int fft_plan_read_timing(fft_plan *p, double ms_out[3], int64_t launches_out[3], int reset) {
    if (!p || !ms_out || !launches_out) return FFT_E_NULL;
    const int rc = p->ev.empty() ? FFT_OK : drain_all(p);
    for (int k = 0; k < 3; ++k) {
        ms_out[k] = p->ms[k];
        launches_out[k] = p->launches[k];
        if (reset) {
            p->ms[k] = 0;
            p->launches[k] = 0;
        }
    }
    return rc;
}


} // extern "C"

namespace {

// Options of the best configuration found so far per (n, batch, dtype,
// device), so that a second tuned plan of the same shape is created directly.
struct TuneKey {
    int64_t n, batch;
    int dtype, device;
    bool operator<(const TuneKey &o) const {
        return n != o.n ? n < o.n : batch != o.batch ? batch < o.batch : dtype != o.dtype ? dtype < o.dtype
                                                                                           : device < o.device;
    }
};
std::mutex tune_mutex;
std::map<TuneKey, fft_tune_result> tune_cache;

// Tuning outcomes kept across processes when the environment variable
// LIFTFFT_TUNE_CACHE names a file: one JSON object per line, keyed by the
// device's architecture name, n, batch and dtype (the last line of a key
// wins), holding the chosen options and the tuner's timings.
std::string device_arch(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    return std::string(prop.gcnArchName);
}

// The value after "key": on one line of the cache file.
const char *json_value(const char *line, const char *key) {
    char pat[64];
    snprintf(pat, sizeof pat, "\"%s\":", key);
    const char *v = strstr(line, pat);
    if (!v) return nullptr;
    v += strlen(pat);
    while (*v == ' ') ++v;
    return v;
}
bool json_int(const char *line, const char *key, int64_t &out) {
    const char *v = json_value(line, key);
    if (!v) return false;
    char *end = nullptr;
    const long long x = strtoll(v, &end, 10);
    if (end == v) return false;
    out = x;
    return true;
}
bool json_double(const char *line, const char *key, double &out) {
    const char *v = json_value(line, key);
    if (!v) return false;
    char *end = nullptr;
    const double x = strtod(v, &end);
    if (end == v) return false;
    out = x;
    return true;
}
bool json_string(const char *line, const char *key, std::string &out) {
    const char *v = json_value(line, key);
    if (!v || *v != '"') return false;
    const char *e = strchr(v + 1, '"');
    if (!e) return false;
    out.assign(v + 1, e);
    return true;
}

bool tune_file_lookup(const std::string &arch, int64_t n, int64_t batch, int dtype, fft_tune_result &out) {
    const char *path = getenv("LIFTFFT_TUNE_CACHE");
    if (!path || !*path || arch.empty()) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[2048];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        std::string a;
        int64_t ln = 0, lb = 0, ld = 0;
        if (!json_string(line, "arch", a) || a != arch || !json_int(line, "n", ln) || ln != n ||
            !json_int(line, "batch", lb) || lb != batch || !json_int(line, "dtype", ld) || ld != dtype)
            continue;
        int64_t v[10];
        double ms = 0, msd = 0;
        const char *keys[10] = {"log2_p",     "radix", "lines_per_block",    "lines_per_block2", "flags",
                                "values_per_thread", "values_per_thread2", "scratch_width", "candidates", "rejected"};
        bool ok = json_double(line, "ms", ms) && json_double(line, "ms_default", msd);
        for (int k = 0; k < 10 && ok; ++k) ok = json_int(line, keys[k], v[k]);
        if (!ok) continue;
        fft_tune_result r;
        memset(&r, 0, sizeof r);
        r.opts.log2_p = int32_t(v[0]);
        r.opts.radix = int32_t(v[1]);
        r.opts.lines_per_block = int32_t(v[2]);
        r.opts.lines_per_block2 = int32_t(v[3]);
        r.opts.flags = int32_t(v[4]);
        r.opts.values_per_thread = int32_t(v[5]);
        r.opts.values_per_thread2 = int32_t(v[6]);
        r.opts.scratch_width = int32_t(v[7]);
        int64_t order = 0; // absent from lines written before tile orders were tuned
        if (json_int(line, "tile_order", order)) r.opts.tile_order = int32_t(order);
        r.candidates = int32_t(v[8]);
        r.rejected = int32_t(v[9]);
        r.ms = ms;
        r.ms_default = msd;
        out = r;
        found = true;
    }
    fclose(f);
    return found;
}

void tune_file_append(const std::string &arch, int64_t n, int64_t batch, int dtype, const fft_tune_result &r) {
    const char *path = getenv("LIFTFFT_TUNE_CACHE");
    if (!path || !*path || arch.empty()) return;
    char line[1024];
    const int len = snprintf(line, sizeof line,
                             "{\"arch\": \"%s\", \"n\": %lld, \"batch\": %lld, \"dtype\": %d, \"log2_p\": %d, "
                             "\"radix\": %d, \"lines_per_block\": %d, \"lines_per_block2\": %d, \"flags\": %d, "
                             "\"values_per_thread\": %d, \"values_per_thread2\": %d, \"scratch_width\": %d, "
                             "\"tile_order\": %d, \"ms\": %.6g, \"ms_default\": %.6g, \"candidates\": %d, "
                             "\"rejected\": %d}\n",
                             arch.c_str(), (long long)n, (long long)batch, dtype, r.opts.log2_p, r.opts.radix,
                             r.opts.lines_per_block, r.opts.lines_per_block2, r.opts.flags, r.opts.values_per_thread,
                             r.opts.values_per_thread2, r.opts.scratch_width, r.opts.tile_order, r.ms, r.ms_default,
                             r.candidates, r.rejected);
    if (len <= 0 || len >= int(sizeof line)) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fputs(line, f); // one write of a whole line: concurrent appends do not interleave
    fclose(f);
}

// Candidate configurations, most promising first: the default; the other
// splits n = p*q near the square one and the single/two-pass threshold;
// radix 2; then, for the default split, the kernel variants and tile widths.
std::vector<fft_plan_opts> tune_candidates(int t, int dtype) {
    std::vector<fft_plan_opts> c;
    // Every candidate after the library default names its lift explicitly.
    auto add = [&](int log2_p, int radix, int lpb, int lpb2, int flags, int vpt) {
        fft_plan_opts o;
        memset(&o, 0, sizeof(o));
        o.log2_p = log2_p;
        o.radix = radix;
        o.lines_per_block = lpb;
        o.lines_per_block2 = lpb2;
        o.flags = c.empty() || (flags & FFT_OPT_THREE_LEVEL) ? flags : flags | FFT_OPT_TWO_LEVEL;
        o.values_per_thread = vpt;
        c.push_back(o);
    };
    add(0, 0, 0, 0, 0, 0);
    if (t >= 15) // three-level lifts: tile widths 16 and 32, complex or split exchange
        for (int lpb : {16, 32})
            for (int f : {0, int(FFT_OPT_SPLIT_EXCHANGE)})
                if (dtype == FFT_C64 || !f) add(0, 0, lpb, 0, FFT_OPT_THREE_LEVEL | f, 0);
    add(0, 0, 0, 0, 0, 0); // the two-level default
    const int lq = (t + 1) / 2, lp = t - lq;
    for (int d : {1, -1, 2}) { // splits p = 2^(lp + d); q = 2^(t - lp - d)
        const int l2p = lp + d;
        if (l2p >= 1 && l2p < t && l2p <= max_line(dtype) && t - l2p <= max_line(dtype)) add(l2p, 0, 0, 0, 0, 0);
    }
    if (t <= max_line(dtype) && lp >= 1) add(lp, 0, 0, 0, 0, 0); // two passes below the threshold
    add(0, 2, 0, 0, 0, 0);
    if (t >= 2) {
        const int variants[][2] = {{FFT_OPT_FULL_EXCHANGE, 16}, {FFT_OPT_SPLIT_EXCHANGE, 16},
                                   {FFT_OPT_SPLIT_EXCHANGE, 32}, {0, 32},
                                   {FFT_OPT_PERSISTENT, 16}, {FFT_OPT_SPLIT_EXCHANGE | FFT_OPT_DENSE, 16}};
        const int tiles[][2] = {{0, 0}, {2, 4}, {1, 4}, {4, 4}, {2, 8}, {4, 8}, {8, 8}, {2, 2}};
        for (const auto &tl : tiles)
            for (const auto &v : variants) {
                if (dtype != FFT_C64 && (v[0] != FFT_OPT_FULL_EXCHANGE || v[1] != 16)) continue;
                add(0, 0, tl[0], tl[1], v[0], v[1] == 16 && !(v[0] & (FFT_OPT_PERSISTENT | FFT_OPT_DENSE)) ? 0 : v[1]);
            }
    }
    return c;
}

// Buffer sets the tuner rotates between executes, so that no candidate reads
// an input still resident in the 256 MB last-level cache from its previous
// execute (as a workload over distinct buffers would not); one set once a
// buffer is at least 512 MB, which the cache cannot hold anyway.
constexpr int TUNE_SETS = 3;
constexpr size_t TUNE_ROTATE_BELOW = size_t(512) << 20;

struct TuneBench {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *x[TUNE_SETS] = {}, *y[TUNE_SETS] = {}, *ref = nullptr;
    int sets = 1;
    int last = 0; // set whose output the last execute wrote
    double *partial = nullptr;
    int64_t count = 0;
    int dtype = 0;
    ~TuneBench() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (int k = 0; k < TUNE_SETS; ++k) {
            if (x[k]) (void)hipFree(x[k]);
            if (y[k]) (void)hipFree(y[k]);
        }
        if (ref) (void)hipFree(ref);
        if (partial) (void)hipFree(partial);
        if (st) (void)hipStreamDestroy(st);
    }
};
constexpr int CMP_BLOCKS = 1024;

// Milliseconds per forward execute of `plan` (negative on failure), each
// execute on the next buffer set.
double tune_time(const fft_plan *plan, TuneBench &b) {
    int k = 0;
    auto exec = [&]() {
        b.last = k;
        const int rc = fft_execute(plan, b.x[k], b.y[k], -1, b.st);
        k = (k + 1) % b.sets;
        return rc;
    };
    for (int w = 0; w < 2 * b.sets; ++w)
        if (exec() != FFT_OK) return -1;
    if (hipEventRecord(b.e0, b.st) != hipSuccess || exec() != FFT_OK ||
        hipEventRecord(b.e1, b.st) != hipSuccess || hipEventSynchronize(b.e1) != hipSuccess)
        return -1;
    float one = 0;
    if (hipEventElapsedTime(&one, b.e0, b.e1) != hipSuccess) return -1;
    int reps = one > 0 ? int(2.0 / one) : 50; // about 2 ms of timed work
    reps = reps < 3 ? 3 : reps > 50 ? 50 : reps;
    if (hipEventRecord(b.e0, b.st) != hipSuccess) return -1;
    for (int r = 0; r < reps; ++r)
        if (exec() != FFT_OK) return -1;
    float ms = 0;
    if (hipEventRecord(b.e1, b.st) != hipSuccess || hipEventSynchronize(b.e1) != hipSuccess ||
        hipEventElapsedTime(&ms, b.e0, b.e1) != hipSuccess)
        return -1;
    return double(ms) / reps;
}

// Largest |y - ref| relative to the largest |ref| (after tune_time left the
// candidate's output in y[last]; every input set holds the same pattern).
double tune_diff(TuneBench &b) {
    const void *y = b.y[b.last];
    if (b.dtype == FFT_C64)
        hipLaunchKernelGGL(compare_kernel<float>, dim3(CMP_BLOCKS), dim3(CMP_THREADS), 0, b.st,
                           static_cast<const float2 *>(y), static_cast<const float2 *>(b.ref), b.count, b.partial);
    else
        hipLaunchKernelGGL(compare_kernel<double>, dim3(CMP_BLOCKS), dim3(CMP_THREADS), 0, b.st,
                           static_cast<const double2 *>(y), static_cast<const double2 *>(b.ref), b.count,
                           b.partial);
    std::vector<double> h(2 * CMP_BLOCKS);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h.data(), b.partial, h.size() * sizeof(double), hipMemcpyDeviceToHost, b.st) != hipSuccess ||
        hipStreamSynchronize(b.st) != hipSuccess)
        return INFINITY;
    double md = 0, mb = 0;
    for (int i = 0; i < CMP_BLOCKS; ++i) {
        md = md > h[2 * i] ? md : h[2 * i];
        mb = mb > h[2 * i + 1] ? mb : h[2 * i + 1];
    }
    return mb > 0 ? md / mb : md;
}

} // namespace

extern "C" {

int fft_plan_create_tuned(int64_t n, int64_t batch, int dtype, int32_t max_candidates, fft_plan **plan_out,
                          fft_tune_result *result) {
    if (!plan_out) return FFT_E_NULL;
    *plan_out = nullptr;
    if (max_candidates < 0) return FFT_E_ARG;
    // The default plan validates the arguments and is the reference output.
    fft_plan *best = nullptr;
    int rc = fft_plan_create(n, batch, dtype, &best);
    if (rc != FFT_OK) return rc;
    const TuneKey key{n, batch, dtype, best->device};
    const std::string arch = device_arch(best->device);
    {
        std::lock_guard<std::mutex> g(tune_mutex);
        auto it = tune_cache.find(key);
        fft_tune_result stored;
        if (it == tune_cache.end() && tune_file_lookup(arch, n, batch, dtype, stored))
            it = tune_cache.emplace(key, stored).first;
        if (it != tune_cache.end()) {
            fft_plan *p = nullptr;
            rc = fft_plan_create_ex(n, batch, dtype, &it->second.opts, &p);
            if (rc == FFT_OK) {
                fft_plan_destroy(best);
                if (result) *result = it->second;
                *plan_out = p;
                return FFT_OK;
            }
            tune_cache.erase(it); // a stored configuration this build cannot create: tune again
        }
    }
    TuneBench b;
    b.dtype = dtype;
    b.count = n * batch;
    const size_t bytes = size_t(b.count) * best->esize;
    if (hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b.e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&b.e1, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipGetLastError();
        fft_plan_destroy(best);
        return FFT_E_HIP;
    }
    b.sets = bytes < TUNE_ROTATE_BELOW ? TUNE_SETS : 1;
    bool ok = hipMalloc(&b.ref, bytes) == hipSuccess &&
              hipMalloc(&b.partial, 2 * CMP_BLOCKS * sizeof(double)) == hipSuccess;
    for (int k = 0; ok && k < b.sets; ++k)
        ok = hipMalloc(&b.x[k], bytes) == hipSuccess && hipMalloc(&b.y[k], bytes) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        fft_plan_destroy(best);
        return FFT_E_OOM;
    }
    const int64_t fb = (b.count + 255) / 256;
    for (int k = 0; k < b.sets; ++k) {
        if (dtype == FFT_C64)
            hipLaunchKernelGGL(fill_pattern_kernel<float>, dim3(unsigned(fb)), dim3(256), 0, b.st,
                               static_cast<float2 *>(b.x[k]), b.count);
        else
            hipLaunchKernelGGL(fill_pattern_kernel<double>, dim3(unsigned(fb)), dim3(256), 0, b.st,
                               static_cast<double2 *>(b.x[k]), b.count);
    }
    if (hipGetLastError() != hipSuccess || fft_execute(best, b.x[0], b.ref, -1, b.st) != FFT_OK ||
        hipStreamSynchronize(b.st) != hipSuccess) {
        (void)hipGetLastError();
        fft_plan_destroy(best);
        return FFT_E_HIP;
    }
    double best_ms = tune_time(best, b);
    if (best_ms < 0) {
        fft_plan_destroy(best);
        return FFT_E_HIP;
    }
    fft_tune_result res;
    memset(&res, 0, sizeof(res));
    res.ms_default = best_ms;
    res.candidates = 1;
    const double tol = dtype == FFT_C64 ? 1e-4 : 1e-10;
    const int limit = max_candidates ? max_candidates : 48;
    const std::vector<fft_plan_opts> cands = tune_candidates(ilog2_exact(n), dtype);
    for (size_t i = 1; i < cands.size() && res.candidates < limit; ++i) {
        fft_plan *p = nullptr;
        if (fft_plan_create_ex(n, batch, dtype, &cands[i], &p) != FFT_OK) continue;
        const double ms = tune_time(p, b);
        ++res.candidates;
        if (ms < 0 || !(tune_diff(b) <= tol)) { // a configuration that disagrees is never chosen
            ++res.rejected;
            fft_plan_destroy(p);
            continue;
        }
        if (ms < best_ms) {
            fft_plan_destroy(best);
            best = p;
            best_ms = ms;
            res.opts = cands[i];
        } else {
            fft_plan_destroy(p);
        }
    }
    // Second stage: the tile order of each pass of the chosen configuration
    // in turn, the other passes keeping the orders in effect.
    fft_plan_info bi;
    if (fft_plan_get_info(best, &bi) == FFT_OK && bi.levels >= 1) {
        int32_t cur = bi.tile_order;
        for (int k = 0; k < bi.levels; ++k) {
            for (int log2s = 1; log2s <= 5; ++log2s) {
                const int32_t order = (cur & ~(0xff << (8 * k))) | (log2s << (8 * k));
                if (order == cur) continue;
                fft_plan_opts o = res.opts;
                o.flags |= FFT_OPT_TILE_ORDER;
                o.tile_order = order;
                fft_plan *p = nullptr;
                if (fft_plan_create_ex(n, batch, dtype, &o, &p) != FFT_OK) continue;
                const double ms = tune_time(p, b);
                ++res.candidates;
                if (ms < 0 || !(tune_diff(b) <= tol)) {
                    ++res.rejected;
                    fft_plan_destroy(p);
                    continue;
                }
                if (ms < best_ms) {
                    fft_plan_destroy(best);
                    best = p;
                    best_ms = ms;
                    res.opts = o;
                    cur = order;
                } else {
                    fft_plan_destroy(p);
                }
            }
        }
    }
    (void)hipStreamSynchronize(b.st);
    res.ms = best_ms;
    {
        std::lock_guard<std::mutex> g(tune_mutex);
        tune_cache[key] = res;
        tune_file_append(arch, n, batch, dtype, res);
    }
    if (result) *result = res;
    *plan_out = best;
    return FFT_OK;
}

} // extern "C"
