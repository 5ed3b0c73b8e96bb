// Device-side FFT engine for gfx950: complex helpers, DFT codelets and the
// workgroup-tile transform used by every pass kernel.
//
// A workgroup owns T "lines" (independent N-point transforms) at once.  Each
// line is processed by TPL = N/E threads holding E = min(16, N) complex values
// in registers.  The stage loop is the paper's stage loop (Section 2.1,
// Fig. 2.1: one butterfly stage per doubling of the column length) regrouped
// into radix-R stages, R <= 16: each radix-R stage is R-1 radix-2 stages done
// at once in registers, i.e. the same dimension lifting the paper applies
// between processors (Section 4.2), applied here between the register file
// and LDS.  Stages are self-sorting (Stockham form), so no bit-reversal pass
// is needed: for stage s with radix R and Ns = product of the earlier radices,
// butterfly b < N/R reads elements b + r*(N/R), multiplies element r by
// w_{Ns*R}^(r*(b mod Ns)), does an R-point DFT and writes element r to
// (b div Ns)*Ns*R + (b mod Ns) + r*Ns.  Data moves between stages through LDS.
//
// All transforms here use the exponent sign -1; sign +1 is obtained by
// conjugating on load and on store (F_+(x) = conj(F_-(conj x))), which the
// pass kernels do with a runtime flag.
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
// a * conj(w): multiply by the sign -1 twiddle when w holds the +1 root.
template <typename C> __device__ __forceinline__ C cmulc(C a, C w) {
    return mk<C>(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}
// a * (-i)
template <typename C> __device__ __forceinline__ C mul_mi(C a) { return mk<C>(a.y, -a.x); }
template <typename C> __device__ __forceinline__ C conj_if(C a, bool c) {
    return c ? mk<C>(a.x, -a.y) : a;
}

// Multiply by w_16^(-e) (sign -1 root), e in 0..15, with the trivial cases
// folded at compile time.
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
    // a[4*r2 + k1] *= w_16^(-r2*k1)
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

// Radix schedule for an N-point line with largest radix RMAX: as many RMAX
// stages as fit, plus one smaller stage for the remainder, placed second so
// that the first and last stages (the ones touching global memory) use RMAX.
template <int N, int RMAX> struct Sched {
    static constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
    static constexpr int LOGN = ilog2(N);
    static constexpr int LOGR = ilog2(RMAX < N ? RMAX : N);
    static constexpr int FULL = LOGN / LOGR;
    static constexpr int REM = LOGN % LOGR;
    static constexpr int NSTAGES = FULL + (REM ? 1 : 0);
    static constexpr int radix(int s) {
        return (REM && s == 1) ? (1 << REM) : (1 << LOGR);
    }
    static constexpr int ns(int s) { // product of the radices before stage s
        int p = 1;
        for (int i = 0; i < s; ++i) p *= radix(i);
        return p;
    }
    static constexpr int E = N < 16 ? N : 16;   // values per thread
    static constexpr int TPL = N / E;           // threads per line
    static_assert(N >= 2 && (N & (N - 1)) == 0, "N must be a power of two >= 2");
    static_assert(E % (1 << LOGR) == 0, "radix must divide the values per thread");
};

// LDS addressing.  LINE_MINOR (pass kernels, lanes sweep the T lines first):
// element e of line c lives at pad(e)*T + c.  Otherwise (single-pass
// kernel, lanes sweep one line first): c*PITCH + pad(e).  pad() inserts one
// slot every 16 elements to spread the strided Stockham writes over banks.
__device__ __forceinline__ int pad16(int e) { return e + (e >> 4); }

template <int N, bool LINE_MINOR> struct LdsMap {
    __device__ __forceinline__ static int at(int c, int e, int T) {
        if constexpr (LINE_MINOR) return pad16(e) * T + c;
        else return c * (N + (N >> 4)) + pad16(e);
    }
    static constexpr int elems_per_line() { return N + (N >> 4); }
};

// Run the whole stage schedule on one thread's registers.  On entry v[] holds
// the stage-0 inputs: slot i*R0 + r = element j + i*TPL + r*(N/R0).  On exit
// v[] holds the outputs: slot i*RL + r = element j + i*TPL + r*(N/RL), where
// RL is the last stage's radix.  `tw` is the table w_N^e, e < N (+1 root).
template <typename C, int N, int RMAX, bool LINE_MINOR, int STG = 0>
__device__ __forceinline__ void run_stages(C *v, C *lds, int c, int j, int T,
                                           const C *__restrict__ tw) {
    using S = Sched<N, RMAX>;
    using M = LdsMap<N, LINE_MINOR>;
    constexpr int E = S::E, TPL = S::TPL;
    constexpr int R = S::radix(STG);
    constexpr int NS = S::ns(STG);
    constexpr int NB = E / R;
    if constexpr (STG > 0) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int b = j + i * TPL;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i * R + r] = lds[M::at(c, b + r * (N / R), T)];
        }
        if constexpr (NS > 1) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = j + i * TPL;
                const int k = b & (NS - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const C w = tw[r * k * (N / (NS * R))];
                    v[i * R + r] = cmulc(v[i * R + r], w);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) dft<R>(&v[i * R]);
    if constexpr (STG + 1 < S::NSTAGES) {
        if constexpr (STG > 0) __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int b = j + i * TPL;
            const int base = (b / NS) * NS * R + (b & (NS - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) lds[M::at(c, base + r * NS, T)] = v[i * R + r];
        }
        __syncthreads();
        run_stages<C, N, RMAX, LINE_MINOR, STG + 1>(v, lds, c, j, T, tw);
    }
}

// Element index held by register slot s on entry (first stage layout) or on
// exit (last stage layout): slot i*R + r <-> j + i*TPL + r*(N/R).
template <int N, int R, int E> __device__ __forceinline__ constexpr int slot_elem_off(int s) {
    return (s / R) * (N / E) + (s % R) * (N / R);
}

} // namespace liftfft
