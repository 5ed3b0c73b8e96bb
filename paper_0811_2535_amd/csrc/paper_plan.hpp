// The paper's own partitioned plan (Sections 4.2-4.8, Fig. 4.9) on the GPU:
// interface between the plan code in liftfft.hip and the kernels in
// paper_plan.hip.
//
// m = 2^log2m workgroups play the paper's m processors.  After the
// bit-reversal permutation P_n (applied as a gather on load), processor p
// owns the psize = n/m contiguous elements [p*psize, (p+1)*psize) and runs
// the radix-2 stages 1 .. bp-1 on its private copy (the block phase); the
// data is redistributed so that processor p owns the elements whose index is
// p mod m, and stages bp .. t run on that private copy with only the weights
// it needs, w_L^(m*r' + p) (the cyclic phase, the weightcyclic factors of
// Section 4.5).  Valid breakpoints: log2 m + 1 <= bp <= log2 psize + 1
// (Section 4.8).  The kernel boundary between the phases is the paper's
// SYNCHRONIZE; the redistribution is the cyclic phase's strided gather from
// the scratch array the block phase wrote.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace liftfft_paper {

struct PaperPlan {
    int dtype = 0;        // 0 complex64, 1 complex128
    int log2n = 0, log2m = 0, bp = 0;
    int64_t batch = 0;
    int threads = 0;      // per workgroup
    bool lds = false;     // private copies in LDS (else in global memory)
    size_t lds_bytes = 0;
    const void *w = nullptr; // w_n^e, e < n/2 (+1 root), FP64-generated
};

// Longest transform the plan takes, and the largest private copy kept in LDS.
constexpr int MAX_LOG2N = 20;
constexpr int64_t LDS_LIMIT = 160 * 1024;

// Fill the launch shape of a plan whose dtype, log2n, log2m, bp and batch are
// set (the arguments are checked by the caller).  Returns a hipError_t value.
int shape(PaperPlan &pp);

// Launch one phase: 0 = block phase (in -> scratch), 1 = cyclic phase
// (scratch -> out).  sign -1 uses the conjugated weights.  Returns a
// hipError_t value.
int launch(const PaperPlan &pp, int phase, const void *in, void *out, void *scratch, int sign, hipStream_t st);

} // namespace liftfft_paper
