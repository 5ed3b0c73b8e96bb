/*
 * liftfft -- dimension-lifted 1-D complex FFT for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libliftfft.so.  No C++ or framework types cross this boundary:
 * sizes are int64_t, buffers are plain device pointers, the stream is an
 * opaque hipStream_t passed as void*.
 *
 * The transform (Hunt, Mullin, Rosenkrantz, Raynolds, "A Transformation-Based
 * Approach for the Design of Parallel/Distributed Scientific Software: the
 * FFT", Section 2.1, Fig. 2.1: input x in C^n, n = 2^t, t >= 1; output the FFT
 * of x) is, for every transform b < batch,
 *
 *     out[b*n + k] = sum_{j<n} in[b*n + j] * exp(sign * 2*pi*i * j*k / n),
 *
 * unnormalized in both directions, natural order in and out.  sign = -1 is
 * the usual forward transform; sign = +1 is the exponent the paper's own loops
 * use (Section 3, weights EXP(2*pi*i*row/L)) and is the adjoint of sign = -1.
 *
 * Method (Sections 4.2-4.8: the stage loop split at a breakpoint into a block
 * phase and a cyclic phase joined by a block-to-cyclic redistribution,
 * Fig. 4.9, Fig. 5.3): n is lifted to a p x q array with n = p*q,
 * j = j1 + p*j2, k = k2 + q*k1.  Pass 1 runs the q-point transforms over j2
 * for each j1 (the block phase), multiplies by w_n^(sign*j1*k2) and writes a
 * tiled scratch array (the redistribution); pass 2 runs the p-point
 * transforms over j1 for each k2 (the cyclic phase) and stores X[k2 + q*k1]
 * in natural order.  Lengths that fit one workgroup run in a single pass.
 *
 * Data layout: interleaved complex; FFT_C64 = float2 {re, im} (8 bytes),
 * FFT_C128 = double2 {re, im} (16 bytes).  Transform b occupies elements
 * [b*n, (b+1)*n).
 *
 * Threading: a plan may be used from one host thread at a time; executes on
 * one plan must be ordered on one stream (they share the plan's scratch).
 * Different plans are independent.
 */
#ifndef LIFTFFT_H
#define LIFTFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft_plan fft_plan; /* opaque; owns scratch and twiddle tables */

/* Element types. */
enum { FFT_C64 = 0, FFT_C128 = 1 };

/* Status codes.  Every argument and capacity check runs on the host before
 * any device work, so an error return means nothing was launched. */
enum {
    FFT_OK = 0,
    FFT_E_SIZE = -1,        /* n not a power of two, n < 2, batch < 1, size overflow */
    FFT_E_DTYPE = -2,       /* unknown element type */
    FFT_E_SIGN = -3,        /* sign not -1 or +1 */
    FFT_E_NULL = -4,        /* required pointer is NULL */
    FFT_E_ALIGN = -5,       /* buffer not aligned to its element size */
    FFT_E_OOM = -6,         /* device allocation failed (nothing leaked) */
    FFT_E_HIP = -7,         /* a HIP runtime call or kernel launch failed */
    FFT_E_UNSUPPORTED = -8, /* valid request outside what the library supports */
    FFT_E_ARG = -9,         /* other invalid argument (options, precision mode) */
    FFT_E_CAPACITY = -10    /* beyond the fixed scratch of fft_execute_static */
};

/* Largest supported log2(n) per element type: one workgroup transforms lines
 * of up to 2^14 complex64 / 2^13 complex128 points, so transforms up to that
 * length run in one pass and the two-level lift reaches 2^28 / 2^26; the
 * three-level lift reaches 2^30 / 2^29 (8 GiB per buffer). */
#define FFT_MAX_LOG2N_C64 30
#define FFT_MAX_LOG2N_C128 29

/*
 * Create a plan for `batch` transforms of length `n` of element type `dtype`.
 * Validates the arguments, chooses the lift (single pass when n fits one
 * workgroup, else p x q with q >= p, or from n = 2^24 on the three-level
 * lift described below), allocates the scratch array (n*batch elements, lifted
 * plans only) and the twiddle tables, and fills the tables
 * on the current device with an FP64 kernel (each entry computed directly
 * from its integer exponent, rounded once to the element type).  Synchronous.
 * On success *plan_out owns the plan (release with fft_plan_destroy); on
 * failure *plan_out is set to NULL and nothing is leaked.
 * The plan is bound to the device current at creation.
 */
int fft_plan_create(int64_t n, int64_t batch, int dtype, fft_plan **plan_out);

/*
 * Plan options for fft_plan_create_ex (zero-initialise, then set fields;
 * a zero field means "library default").
 *   log2_p        force the lift n = p*q with p = 2^log2_p (1 <= log2_p < t);
 *                 forces the two-pass path even when n fits one workgroup.
 *   radix         largest butterfly radix used inside each pass: 2, 4, 8
 *                 or 16 (default 16).  radix = 2 runs self-sorting radix-2
 *                 stages within each pass (the paper's own in-place loop on
 *                 bit-reversed input is fft_plan_create_paper).
 *   lines_per_block   lines (independent short transforms) per workgroup in
 *                     pass 1, or in the single pass (0 = default; power of two).
 *   lines_per_block2  lines per workgroup in pass 2 (0 = default; power of two).
 *                     A tile width that does not fit the kernel's thread or
 *                     LDS limits, exceeds the lines of one transform, or (pass
 *                     1) exceeds the threads of one pass-2 line returns
 *                     FFT_E_UNSUPPORTED.
 *   flags             FFT_OPT_NO_XCD_REMAP: keep the hardware workgroup order
 *                     instead of giving each XCD a contiguous range of tiles.
 *                     FFT_OPT_SPLIT_EXCHANGE / FFT_OPT_FULL_EXCHANGE: exchange
 *                     data between stages through LDS one real component at
 *                     a time (half the LDS per tile) / as complex elements.
 *                     FFT_OPT_PERSISTENT / FFT_OPT_ONE_TILE: pass kernels run
 *                     as many workgroups as are resident, each transforming
 *                     a sequence of tiles with the next tile's loads in
 *                     flight / one workgroup per tile.
 *                     FFT_OPT_DENSE: pass kernels capped at 64 VGPRs so that
 *                     two 1024-thread workgroups fit one CU (16 values per
 *                     thread, one tile per workgroup only).
 *                     FFT_OPT_TWO_LEVEL / FFT_OPT_THREE_LEVEL: force the
 *                     two-level lift p x q (two passes) / the three-level
 *                     lift (see below) instead of the library's choice
 *                     (three levels from n = 2^24 on, radix 16 and default
 *                     kernels, unless a two-level option or lines_per_block
 *                     is given).
 *                     FFT_OPT_SHUFFLE_EXCHANGE (with FFT_OPT_THREE_LEVEL
 *                     only): axis passes over 256-point complex64 lines
 *                     exchange data between their two stages by wavefront
 *                     shuffles within 16-lane rows (DPP and ds_swizzle)
 *                     instead of the LDS tile (passes over other lengths
 *                     keep the default kernel; FFT_E_UNSUPPORTED when no
 *                     pass has 256-point lines or the type is complex128;
 *                     other kernel-variant options: FFT_E_ARG).
 *                     FFT_OPT_LDS_PREFETCH (with FFT_OPT_TWO_LEVEL only):
 *                     pass 1 over 4096-point complex64 columns (2 per
 *                     tile) as one persistent workgroup per CU that stages
 *                     its next tile in LDS with direct global-to-LDS loads
 *                     while transforming the current one; other shapes
 *                     return FFT_E_UNSUPPORTED, other kernel-variant
 *                     options FFT_E_ARG.  Inputs not 16-byte aligned run
 *                     the plain pass 1.  A measured alternative: slower
 *                     than the default pass 1 at n = 2^24.
 *                     FFT_OPT_ROW_LANES (with FFT_OPT_TWO_LEVEL only):
 *                     pass 1 over 4096-point complex64 columns, 2 per
 *                     tile, with each thread owning whole rows of the
 *                     tile (one 16-byte load per row for both columns)
 *                     instead of one column of a row; same tile, weights
 *                     and scratch layout.  values_per_thread 16 (default:
 *                     512 threads, radix-8 stages) or 32 (256 threads,
 *                     radix 16) sets this pass 1 alone.  Other shapes
 *                     return FFT_E_UNSUPPORTED, other kernel-variant
 *                     options FFT_E_ARG.
 *                     FFT_OPT_DEBUG_CANARY (a debug mode, any plan of
 *                     fft_plan_create_ex): every execute first fills the
 *                     scratch array, and `out` wherever a pass reads
 *                     neither it nor the input afterwards, with quiet NaNs
 *                     on the execute stream (before pass 1, and again
 *                     before the pass that writes `out` last), so that an
 *                     element a pass reads before any pass has written it
 *                     reaches the output as a NaN.  The transform's
 *                     result is unchanged, bit for bit; the fills cost
 *                     time, and the per-pass timing includes them.
 *                     FFT_OPT_TILE_ORDER: the tile order of each pass is
 *                     the one tile_order gives instead of the library's.
 *                     FFT_OPT_THREE_LEVEL takes no two-level options
 *                     (log2_p, lines_per_block2, values_per_thread2,
 *                     scratch_width: FFT_E_ARG); lines_per_block then sets
 *                     the lines per workgroup of all three passes.
 *   values_per_thread complex values each thread holds in the pass kernels:
 *                     0 (default), 16 or 32.
 *   values_per_thread2  the same for pass 2 only (0 = as values_per_thread).
 *   scratch_width     W, the width of the slabs S[j1/W][k2][j1%W] of the
 *                     scratch array between the passes (0 = pass 1's tile
 *                     width; a power of two at most the threads of one pass-2
 *                     line, else FFT_E_UNSUPPORTED).  Wider slabs give pass 2
 *                     longer contiguous reads; narrower ones pass 1 longer
 *                     contiguous writes.
 *   tile_order        with FFT_OPT_TILE_ORDER, the order in which each
 *                     pass's workgroups take their tiles (else 0, or
 *                     FFT_E_ARG).  Byte k (k = 0, 1, 2: pass 1 / A, pass 2
 *                     / B, pass C) is 0x80 for the hardware workgroup order,
 *                     else (log2 g << 4) | log2 s (at most 0x7f).  s = 1: each
 *                     XCD takes a contiguous range of tiles, in order (the
 *                     XCD-contiguous order, on every pass whose grid is a
 *                     multiple of 8 of at least 16, else the hardware
 *                     order; the hardware order with FFT_OPT_NO_XCD_REMAP).  s > 1: the range is cut into
 *                     groups of g adjacent tiles, laid out as s rows of
 *                     groups, and the XCD's workgroups take the groups
 *                     column by column, so that the tiles in flight at once
 *                     lie in s runs spread over the range.  The order
 *                     changes only where each tile's memory traffic falls
 *                     in time, never a result bit.  s > 1 with
 *                     FFT_OPT_NO_XCD_REMAP, bytes beyond the plan's passes,
 *                     other bytes above 0x7f: FFT_E_ARG; a range that is not a
 *                     multiple of g s tiles, a grid that is not a multiple
 *                     of 8 of at least 16, or a persistent pass:
 *                     FFT_E_UNSUPPORTED.  Without the flag, plans created
 *                     with the default kernels (no kernel-variant, tile
 *                     width, scratch width or radix option) in FP32 take
 *                     the orders the library measured fastest on MI355X
 *                     for the complex64 shapes it knows: one transform of
 *                     2^24 (two-level 4096 x 4096: 0x0412; three-level:
 *                     0x800305), of 2^23 (0x0112) and of 2^25 (0x800005),
 *                     16 transforms of 2^20 (0x8003) and 4096 of 2^12
 *                     (0x80); every other plan takes s = 1.
 *                     fft_plan_get_info reports the orders in effect.
 * Kernel variants other than the defaults exist for complex64 two-pass
 * plans with radix 16 and pass lines of 2^10..2^12; asking for one elsewhere
 * returns FFT_E_UNSUPPORTED.  Contradictory flags return FFT_E_ARG.
 *
 * Three-level lift (dimension lifting, section 1, taken one level further):
 * n = n1 n2 n3 with x viewed as an n3 x n2 x n1 array (n1 contiguous),
 * j = j1 + n1 j2 + n1 n2 j3 and k = k3 + n3 k2 + n2 n3 k1.  Pass A: n3-point
 * transforms along j3, times w_n^(s n1 j2 k3), written to `out` in the
 * input's layout; pass B: n2-point transforms along j2, times
 * w_n^(s j1 (k3 + n3 k2)), written to the scratch array in the same layout;
 * pass C: n1-point transforms of the contiguous rows, written to `out` in
 * natural order.  Each workgroup takes adjacent lines of the contiguous axis,
 * so every pass reads and writes runs of at least 128 bytes.  Factors:
 * log2 n3 = ceil(t/3), log2 n1 = ceil((t - log2 n3)/2), n2 the rest; each
 * between 2^5 and 2^11 (15 <= t), radix 16, default or split-exchange
 * kernels (default kernels only for transforms of 2^31 bytes or more,
 * which are addressed in 64 bits); otherwise FFT_E_UNSUPPORTED.  Two-level
 * plans stop at 2^28 complex64 / 2^26 complex128 (FFT_E_UNSUPPORTED above).
 */
enum {
    FFT_OPT_NO_XCD_REMAP = 1,
    FFT_OPT_SPLIT_EXCHANGE = 2,
    FFT_OPT_FULL_EXCHANGE = 4,
    FFT_OPT_PERSISTENT = 8,
    FFT_OPT_ONE_TILE = 16,
    FFT_OPT_DENSE = 32,
    FFT_OPT_TWO_LEVEL = 128,
    FFT_OPT_THREE_LEVEL = 256,
    FFT_OPT_SHUFFLE_EXCHANGE = 512,
    FFT_OPT_LDS_PREFETCH = 2048,
    FFT_OPT_DEBUG_CANARY = 4096,
    FFT_OPT_TILE_ORDER = 8192,
    FFT_OPT_ROW_LANES = 16384
};
typedef struct fft_plan_opts {
    int32_t log2_p;
    int32_t radix;
    int32_t lines_per_block;
    int32_t lines_per_block2;
    int32_t flags;
    int32_t values_per_thread;
    int32_t values_per_thread2;
    int32_t scratch_width;
    int32_t tile_order;
} fft_plan_opts;

/*
 * The paper's own partitioned plan, on the GPU (Sections 4.2-4.8, Fig. 4.9;
 * the processors' phases of Sections 4.6-4.7): the transform as the paper
 * states it, for exploring its breakpoints, not the fast path.  m = 2^log2_m
 * workgroups play the paper's m processors, each owning psize = n/m elements.
 * The input is read through the bit-reversal permutation P_n (Fig. 2.1);
 * processor p runs the radix-2 stages 1 .. breakpoint-1 of the in-place
 * stage loop on its contiguous block [p*psize, (p+1)*psize) (the block
 * phase), the data is redistributed so that processor p owns the indices
 * congruent to p mod m, and stages breakpoint .. t run on that private copy
 * with the weightcyclic factors w_L^(m*r' + p) (the cyclic phase).  The
 * output is in natural order and equals fft_execute of any other plan up to
 * rounding.  Private copies are held in LDS when psize elements fit one
 * workgroup (160 KB), else in global memory.
 *   log2_m      0 <= log2_m, psize >= m (2*log2_m <= t), else FFT_E_ARG
 *   breakpoint  log2_m + 1 <= breakpoint <= log2(psize) + 1 (Section 4.8),
 *               else FFT_E_ARG
 * Lengths up to 2^20 (FFT_E_UNSUPPORTED above); the plan owns an n*batch
 * scratch array (the block phase's output) and the n/2 weights w_n^e,
 * computed in FP64 from their integer exponents.  Executed with fft_execute
 * (both signs; sign +1 is the paper's own exponent).  Errors otherwise as
 * fft_plan_create.
 */
int fft_plan_create_paper(int64_t n, int64_t batch, int dtype, int32_t log2_m, int32_t breakpoint,
                          fft_plan **plan_out);

/* As fft_plan_create with explicit options (opts may be NULL). */

int fft_plan_create_ex(int64_t n, int64_t batch, int dtype, const fft_plan_opts *opts,
                       fft_plan **plan_out);

/*
 * A plan for `count` transforms of uneven power-of-two lengths in one packed
 * buffer: transform i (length lengths[i] = 2^t_i, 1 <= t_i <= 24) occupies
 * elements [off_i, off_i + lengths[i]) with off_i the sum of the earlier
 * lengths.  The lengths are the run-time blocking parameters of one batch:
 * the plan groups equal lengths into classes (Sections 4.2-4.8 of the paper
 * for the lift of the long ones).
 * Default form: each class is planned like fft_plan_create(2^t, count) --
 * one pass up to one workgroup's line (2^14 complex64, 2^13 complex128),
 * else the two- or three-level lift -- and reads its transforms through a
 * device list of their offsets; the classes run on up to four streams (the
 * execute stream and three streams the plan creates), forked from and
 * joined back into the execute stream, the largest classes first.
 * flags (0 or an OR of):
 *   FFT_OPT_AUTOTUNE    shape every class like fft_plan_create_tuned(2^t,
 *                       count, dtype, 16) does (timed at plan creation,
 *                       remembered per shape for the process)
 *   FFT_OPT_GRAPH       replay the work as one captured graph per (in, out,
 *                       sign) triple (captured on a private stream the first
 *                       time, with the classes' streams as parallel branches;
 *                       up to 16 per plan; then, or when the execute stream
 *                       is itself being captured, the kernels are launched
 *                       directly)
 *   FFT_OPT_PERSISTENT  the persistent form instead: the lifted classes share
 *                       two persistent launches (pass 1 of every lifted
 *                       class, then pass 2), each walking a work list of
 *                       tiles ordered by class, longest lines first; the
 *                       single-pass classes get one launch each, all on the
 *                       execute stream (not with FFT_OPT_AUTOTUNE)
 * Any other bit, or AUTOTUNE with PERSISTENT, returns FFT_E_ARG.
 * Errors: FFT_E_NULL (lengths or plan_out NULL), FFT_E_SIZE (count < 1, a
 * length not a power of two >= 2), FFT_E_ARG (flags), FFT_E_UNSUPPORTED (a
 * length above the maximum, or a packed buffer of 2^32 bytes or more).
 */
enum { FFT_OPT_GRAPH = 64, FFT_OPT_AUTOTUNE = 1024 };
int fft_plan_create_many(const int64_t *lengths, int64_t count, int dtype, uint32_t flags,
                         fft_plan **plan_out);

/*
 * Execute the planned transforms: out = F_sign(in), as defined above.
 *   in, out   device pointers to n*batch elements, aligned to the element
 *             size; in == out is allowed (pass 1 writes the plan's scratch).
 *             Partial overlap of in and out is not allowed.
 *   sign      -1 or +1.
 *   stream    hipStream_t to launch on (NULL = the null stream).
 * Asynchronous: returns after enqueueing the kernels; no host synchronisation
 * and no allocation.  Returns FFT_E_HIP if a launch fails.
 * The plan's transform (lift, kernels, tables) is read-only here; the plan
 * also holds bookkeeping that an execute updates -- the timing event ring
 * (fft_plan_set_timing) and, for uneven batches with FFT_OPT_GRAPH, the
 * captured-graph cache -- which is why one plan is for one host thread at a
 * time.
 */
int fft_execute(const fft_plan *plan, const void *in, void *out, int sign, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transform of fft_plan_create(n, batch, dtype) + fft_execute, without a
 * plan and without any allocation.  The launches, kernels and results are
 * those of the default plan of the same shape (bit for bit); the inter-pass
 * scratch array and the weight tables live in one static device array per
 * GPU (32 MiB + 256 KiB, held by every GPU the library runs on until the
 * process ends), shared by every call on that GPU.  Capacity: n*batch
 * elements up to 32 MiB (2^22 complex64, 2^21 complex128); larger requests
 * return FFT_E_CAPACITY before any device work.
 *   in, out, sign, stream   as for fft_execute.
 * The tables are regenerated on `stream` whenever (n, dtype) differs from the
 * previous call's on that GPU.  Calls that overlap on one GPU (on different
 * streams, or from different host threads without ordering their streams)
 * race on the shared array and give wrong results; order them.  Errors as
 * fft_plan_create and fft_execute, plus FFT_E_CAPACITY.
 */
int fft_execute_static(int64_t n, int64_t batch, int dtype, const void *in, void *out, int sign,
                       void *stream);

/* Release a plan.  NULL-safe.  The caller must have synchronised every stream
 * that used the plan. */
int fft_plan_destroy(fft_plan *plan);

/* Static description of a status code (never NULL). */
const char *fft_strerror(int code);

/*
 * Plan description, for tests and benchmarks.
 *   passes      kernel launches per execute: 1 (single pass), 2 (two-level
 *               lift, or an uneven batch with lifted lengths) or 3
 *               (three-level lift)
 *   log2_p      lift: p = 2^log2_p (0 for single-pass plans)
 *   log2_q      lift: q = 2^log2_q (single pass: log2 n)
 *   radix       largest butterfly radix used
 *   lines_per_block_pass1/2    lines (short transforms) per tile
 *   grid_pass1/2               persistent workgroups launched
 *   threads_pass1/2            workgroup size
 *   lds_bytes_pass1/2          dynamic LDS per workgroup
 *   scratch_bytes, table_bytes device memory the plan owns
 *   variant_pass1/2            kernel variant bits: 1 = 32 values per
 *                              thread, 2 = split exchange, 4 = persistent,
 *                              8 = dense (64-VGPR cap), 16/32 = the
 *                              matrix-core forms, 64 = shuffle exchange,
 *                              128 = LDS-staged pass 1
 *   precision                  FFT_PREC_* set by fft_plan_set_precision
 *   length_classes, graph_launch  plans of uneven lengths: number of
 *                              distinct lengths, and whether executes replay
 *                              captured graphs (0 for single-length plans)
 * Pass-2 fields are 0 for single-pass plans.  For plans of uneven lengths,
 * n is the total element count, batch the number of transforms, and the
 * pass-1/pass-2 fields describe the two persistent launches (single-pass
 * lengths and pass 1 of the lifted ones; pass 2 of the lifted ones).
 */
typedef struct fft_plan_info {
    int64_t n, batch;
    int32_t dtype, passes, log2_p, log2_q, radix;
    int32_t lines_per_block_pass1, lines_per_block_pass2;
    int32_t grid_pass1, grid_pass2;
    int32_t threads_pass1, threads_pass2;
    int64_t lds_bytes_pass1, lds_bytes_pass2;
    int64_t scratch_bytes, table_bytes;
    int32_t variant_pass1, variant_pass2;
    int32_t length_classes, graph_launch;
    int32_t precision;
    /* tile_order: the order each pass's workgroups take their tiles in,
     * encoded as fft_plan_opts.tile_order (byte k for pass k: 0x80 the
     * hardware order, 0x00 the XCD-contiguous order without spread);
     * 0 for uneven batches and the paper's partitioned plan. */
    int32_t tile_order;
    /* levels: passes of a single-length plan (1, 2 or 3; 0 for uneven
     * batches).  Three-level plans: log2 of n1, n2, n3 (log2_p = log2_q = 0)
     * and pass C's launch in the *_pass3 fields (A and B in pass1, pass2).
     * Plans of the paper's partitioned plan (fft_plan_create_paper): log2_p =
     * log2 m, log2_q = log2 psize, paper_breakpoint = the breakpoint, and the
     * block / cyclic phase launches in the pass1 / pass2 fields; 0 in
     * paper_breakpoint otherwise. */
    int32_t levels, log2_n1, log2_n2, log2_n3;
    int32_t lines_per_block_pass3, grid_pass3, threads_pass3, paper_breakpoint;
    int64_t lds_bytes_pass3;
    /* streams: uneven batches in the default form, the streams their classes
     * run on (1..4); 0 otherwise. */
    int32_t streams, reserved2;
} fft_plan_info;

int fft_plan_get_info(const fft_plan *plan, fft_plan_info *info);

/*
 * Precision form of a plan (default FFT_PREC_FP32: every stage in the
 * element type on the vector units).  FFT_PREC_F16X2 / FFT_PREC_BF16X2 run
 * each radix-16 stage as a product with the 16 x 16 DFT matrix on the matrix
 * cores: matrix and inputs split into high and low FP16 (BF16) parts, three
 * partial products accumulated in FP32, FP16 inputs scaled per butterfly by
 * a power of two.  This is a different arithmetic from the paper's radix-2
 * butterflies (same transform, larger rounding error: about 1e-6 relative
 * L2 for FP16 pairs, 1e-5 for BF16 pairs); tests state the measured error.
 * Available for complex64 single-pass and two-level plans whose pass lines
 * are 16, 256 or 4096 points, and three-level plans whose lines are all 256
 * points (n = 2^24), each stage radix 16, with radix 16, 16 values per
 * thread and one tile per workgroup; otherwise FFT_E_UNSUPPORTED and the
 * plan is unchanged.
 * FFT_E_ARG for an unknown mode.  Takes effect for later executes.  The
 * first switch to a matrix-core form allocates a 4 KB table of the DFT
 * matrix in that form's operand layout (hi and lo parts from FP64 angles)
 * and fills it synchronously; FFT_E_OOM / FFT_E_HIP if that fails.
 */
enum { FFT_PREC_FP32 = 0, FFT_PREC_F16X2 = 1, FFT_PREC_BF16X2 = 2 };
int fft_plan_set_precision(fft_plan *plan, int mode);

/*
 * Per-kernel timing, for benchmarks.  While enabled, fft_execute records a
 * HIP event before and after each kernel it launches, on the execute stream;
 * fft_plan_read_timing synchronises on the last recorded event and returns,
 * for pass k (k = 0, 1, 2), the summed duration in milliseconds and the
 * launch count since the last reset (zero for passes the plan does not
 * have).  Both arrays hold three entries.  Disabled by default (no events
 * recorded).
 */
int fft_plan_set_timing(fft_plan *plan, int enable);
int fft_plan_read_timing(fft_plan *plan, double ms_out[3], int64_t launches_out[3],
                         int reset);

/*
 * Autotuned plan: the default plan plus up to max_candidates - 1 other
 * configurations of the same transform (0 = 48) -- three-level lifts
 * (n >= 2^15; tile widths 16 and 32, complex or split exchange), the
 * two-level default, other lifts n = p*q and the single/two-pass threshold,
 * radix 2, the pass-kernel variants and tile widths, each naming its lift
 * with FFT_OPT_TWO_LEVEL or FFT_OPT_THREE_LEVEL -- each timed on device
 * buffers the call allocates (forward executes on a private stream, about
 * 2 ms of work each, rotating over three input/output buffer sets while a
 * buffer is below 512 MB so that no execute reads an input the last-level
 * cache still holds) and checked
 * against the default plan's output (a configuration whose output differs
 * by more than 1e-4 (complex64) or 1e-10 (complex128) of the largest output
 * is never chosen).  A second stage then takes the fastest configuration's
 * passes in turn and times it with that pass's tiles in the spread orders
 * s = 2, 4, 8, 16 and 32 (g = 1, FFT_OPT_TILE_ORDER; those the pass's grid
 * allows), keeping each pass's fastest order before going on to the next
 * (at most 5 configurations per pass, beyond max_candidates).  Returns the
 * fastest as *plan_out; if result is not
 * NULL it receives that plan's options (fft_plan_create_ex recreates it) and
 * times.  Tuning is an experiment over implementation variants for one
 * problem size on one machine (Section 8 of the paper); the outcome is
 * remembered per (n, batch, dtype, device) for the life of the process, and
 * a later call with the same shape creates the remembered configuration
 * without timing.  If the environment variable LIFTFFT_TUNE_CACHE names a
 * file, outcomes are also kept there across processes: one JSON object per
 * line with the device's architecture name (hipDeviceProp_t::gcnArchName),
 * n, batch, dtype, the nine fields of fft_plan_opts, ms, ms_default,
 * candidates and rejected; a call whose shape is not remembered in the
 * process looks the file up (the last matching line wins; a configuration
 * this build cannot create is tuned again) and returns the stored result
 * without timing, and every new outcome is appended as one line (a file
 * that cannot be read or written is ignored).  Synchronous; the device is
 * otherwise idle-assumed (other
 * work on it skews the timings, not the results).  Errors as
 * fft_plan_create, plus FFT_E_ARG for max_candidates < 0.
 */
typedef struct fft_tune_result {
    fft_plan_opts opts; /* options of the chosen plan */
    double ms;          /* chosen plan: milliseconds per forward execute */
    double ms_default;  /* default plan: milliseconds per forward execute */
    int32_t candidates; /* configurations timed (the default included) */
    int32_t rejected;   /* configurations whose output disagreed, or failed */
} fft_tune_result;
int fft_plan_create_tuned(int64_t n, int64_t batch, int dtype, int32_t max_candidates, fft_plan **plan_out,
                          fft_tune_result *result);

/* ABI version of this header (major*100 + minor). */
#define LIFTFFT_ABI_VERSION 201
int fft_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LIFTFFT_H */
