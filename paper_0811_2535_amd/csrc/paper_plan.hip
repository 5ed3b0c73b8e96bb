// The paper's partitioned radix-2 plan (Sections 4.2-4.8, Fig. 4.9) as two
// HIP kernels for gfx950: the block phase and the cyclic phase, one
// workgroup per (transform, processor).  This is the plan as the paper states
// it -- bit-reversed input, the in-place radix-2 stage loop of Fig. 2.1 / 3.9
// split at a breakpoint, the block-to-cyclic redistribution between the
// phases and only the needed weights in the cyclic phase -- kept for fidelity
// and for exploring breakpoints; the fast path of the library is the
// self-sorting lift in liftfft.hip.
//
// A processor's private copy (the paper's xblock / xcyclic) is held in LDS
// when psize elements fit a workgroup's LDS, else in global memory (the
// block phase in its own block of the scratch array, the cyclic phase at its
// own positions p, p + m, ... of the output), ordered between stages by the
// workgroup barrier.
#include "paper_plan.hpp"

namespace liftfft_paper {
namespace {

template <typename Real> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

struct Args {
    const void *in;
    void *out;
    void *scratch;
    const void *w; // w_n^e, e < n/2 (+1 root)
    int log2n, log2m, bp;
    int wsign; // +1: the paper's weights; -1: their conjugates (sign -1 transform)
};

// The butterfly of Section 3.5 on one pair (upper u, lower v) with weight w:
// c = w * v; u <- u + c; v <- u - c.
template <typename C> __device__ __forceinline__ void butterfly(C &u, C &v, C w) {
    C c;
    c.x = v.x * w.x - v.y * w.y;
    c.y = v.x * w.y + v.y * w.x;
    C a = u;
    u.x = a.x + c.x;
    u.y = a.y + c.y;
    v.x = a.x - c.x;
    v.y = a.y - c.y;
}

// w_L^(sign * e') for L = 2^q, read as w_n^(e' * n/L) from the table.
template <typename C> __device__ __forceinline__ C weight(const C *w, uint32_t e, int shift, int wsign) {
    C v = w[e << shift];
    v.y = wsign > 0 ? v.y : -v.y;
    return v;
}

// Block phase.  Processor p of transform b gathers its psize contiguous
// elements of the bit-reversed input, P_n x, and runs stages q = 1 .. bp-1:
// stage q views the private copy as columns of L = 2^q contiguous elements
// and applies B_L to each (butterfly pairs (i, i + L/2) within a column,
// weight w_L^row for the pair's row < L/2).  The result goes to the
// processor's block of the scratch array.
template <typename Real, bool LDS>
__global__ __launch_bounds__(1024) void block_phase(Args a) {
    using C = typename Cplx<Real>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.log2n, lm = a.log2m;
    const int64_t n = int64_t(1) << t;
    const int lps = t - lm;
    const uint32_t psize = 1u << lps;
    const int64_t b = int64_t(blockIdx.x) >> lm;
    const uint32_t p = blockIdx.x & ((1u << lm) - 1);
    const C *x = static_cast<const C *>(a.in) + b * n;
    C *y = static_cast<C *>(a.scratch) + b * n + int64_t(p) * psize;
    C *priv = LDS ? reinterpret_cast<C *>(smem) : y;
    const C *w = static_cast<const C *>(a.w);
    for (uint32_t i = threadIdx.x; i < psize; i += blockDim.x) {
        const uint32_t g = p * psize + i; // position in P_n x
        priv[i] = x[__brev(g) >> (32 - t)];
    }
    __syncthreads();
    for (int q = 1; q < a.bp; ++q) {
        const uint32_t h = 1u << (q - 1);
        for (uint32_t k = threadIdx.x; k < psize / 2; k += blockDim.x) {
            const uint32_t col = k >> (q - 1), row = k & (h - 1);
            const uint32_t i0 = (col << q) + row, i1 = i0 + h;
            C u = priv[i0], v = priv[i1];
            butterfly(u, v, weight(w, row, t - q, a.wsign));
            priv[i0] = u;
            priv[i1] = v;
        }
        __syncthreads();
    }
    if constexpr (LDS)
        for (uint32_t i = threadIdx.x; i < psize; i += blockDim.x) y[i] = priv[i];
}

// Cyclic phase.  Processor p owns the elements whose index is p mod m:
// private element i is element m*i + p of the scratch array (the
// redistribution).  Stage q = bp .. t views the private copy as columns of
// L/m elements; the butterfly partner of private row r' is r' + L/(2m) and
// its weight is w_L^(m*r' + p), the weightcyclic factor.  The result is
// stored back at the same positions of the output, which then holds the
// transform in natural order.
template <typename Real, bool LDS>
__global__ __launch_bounds__(1024) void cyclic_phase(Args a) {
    using C = typename Cplx<Real>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.log2n, lm = a.log2m;
    const int64_t n = int64_t(1) << t;
    const int lps = t - lm;
    const uint32_t psize = 1u << lps;
    const int64_t b = int64_t(blockIdx.x) >> lm;
    const uint32_t p = blockIdx.x & ((1u << lm) - 1);
    const C *y = static_cast<const C *>(a.scratch) + b * n + p;
    C *o = static_cast<C *>(a.out) + b * n + p;
    C *lds = reinterpret_cast<C *>(smem);
    const C *w = static_cast<const C *>(a.w);
    auto at = [&](uint32_t i) -> C & {
        if constexpr (LDS) return lds[i];
        else return o[int64_t(i) << lm];
    };
    for (uint32_t i = threadIdx.x; i < psize; i += blockDim.x) at(i) = y[int64_t(i) << lm];
    __syncthreads();
    for (int q = a.bp; q <= t; ++q) {
        const int lh = q - 1 - lm; // log2 of L/(2m)
        const uint32_t h = 1u << lh;
        for (uint32_t k = threadIdx.x; k < psize / 2; k += blockDim.x) {
            const uint32_t col = k >> lh, r = k & (h - 1);
            const uint32_t i0 = (col << (lh + 1)) + r, i1 = i0 + h;
            C u = at(i0), v = at(i1);
            butterfly(u, v, weight(w, (r << lm) + p, t - q, a.wsign));
            at(i0) = u;
            at(i1) = v;
        }
        __syncthreads();
    }
    if constexpr (LDS)
        for (uint32_t i = threadIdx.x; i < psize; i += blockDim.x) o[int64_t(i) << lm] = lds[i];
}

template <typename Real> const void *block_fn(bool lds) {
    return lds ? reinterpret_cast<const void *>(&block_phase<Real, true>)
               : reinterpret_cast<const void *>(&block_phase<Real, false>);
}
template <typename Real> const void *cyclic_fn(bool lds) {
    return lds ? reinterpret_cast<const void *>(&cyclic_phase<Real, true>)
               : reinterpret_cast<const void *>(&cyclic_phase<Real, false>);
}

} // namespace

int shape(PaperPlan &pp) {
    const int64_t psize = int64_t(1) << (pp.log2n - pp.log2m);
    const int64_t esize = pp.dtype == 0 ? 8 : 16;
    int64_t thr = psize / 2;
    thr = thr < 64 ? 64 : thr > 1024 ? 1024 : thr;
    pp.threads = int(thr);
    pp.lds = psize * esize <= LDS_LIMIT;
    pp.lds_bytes = pp.lds ? size_t(psize * esize) : 0;
    if (pp.lds_bytes > 65536) {
        const void *f[2] = {pp.dtype == 0 ? block_fn<float>(true) : block_fn<double>(true),
                            pp.dtype == 0 ? cyclic_fn<float>(true) : cyclic_fn<double>(true)};
        for (const void *fn : f) {
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(pp.lds_bytes));
            if (e != hipSuccess) return int(e);
        }
    }
    return int(hipSuccess);
}

int launch(const PaperPlan &pp, int phase, const void *in, void *out, void *scratch, int sign, hipStream_t st) {
    Args a;
    a.in = in;
    a.out = out;
    a.scratch = scratch;
    a.w = pp.w;
    a.log2n = pp.log2n;
    a.log2m = pp.log2m;
    a.bp = pp.bp;
    a.wsign = sign > 0 ? 1 : -1;
    const dim3 grid(unsigned(pp.batch << pp.log2m)), block(unsigned(pp.threads));
    const void *fn = phase == 0 ? (pp.dtype == 0 ? block_fn<float>(pp.lds) : block_fn<double>(pp.lds))
                                : (pp.dtype == 0 ? cyclic_fn<float>(pp.lds) : cyclic_fn<double>(pp.lds));
    void *args[] = {&a};
    return int(hipLaunchKernel(fn, grid, block, args, pp.lds_bytes, st));
}

} // namespace liftfft_paper
