/*
 * tnamp.h - C ABI of the MI355X tensor-network amplitude engine.
 *
 * The library executes contraction plans for circuit amplitudes
 * a(x) = <x|C|0^n>.  A plan is the paper's separator-hierarchy contraction
 * order (proof of Theorem 1; Algorithm 1 and the supplemental section on the
 * numerical implementation) over the circuit's tensor network (section on
 * classical simulation of quantum circuits: gates as tensors, the initial
 * |0> and the projection onto |x> absorbed into them), with index slicing.
 * Every pairwise step of the plan multiplies entries over the union of both
 * operands' indices and sums the shared indices (Eq. (3)); on the device it
 * runs as an index permutation followed by a batched complex GEMM.
 *
 * Conventions
 *  - Bitstrings are uint64 words; bit q is the output value x_q of qubit q
 *    (plans have at most 64 qubits).
 *  - Results are complex128, written as 2*nb doubles: re, im per bitstring,
 *    in the order of the input words.
 *  - Slices are summed in float64 in ascending slice order; within a slice
 *    the arithmetic is float32 (complex64 storage), or split 16-bit products
 *    with float32 accumulation, as selected by `precision`.  The reduction
 *    order of every step is fixed by the plan, so a result does not depend on
 *    batch size, chunking or other work on the device.
 *  - All calls return TN_OK (0), TN_PENDING (1) or a negative error code;
 *    tn_last_error() gives a thread-local message for the last error.
 *  - Host pointers are owned by the caller and only read (or, for outputs,
 *    written) during the call.  Device memory, plans and streams created by
 *    the library are owned by the library.
 */
#ifndef TNAMP_H
#define TNAMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TN_OK 0
#define TN_PENDING 1
#define TN_EINVAL (-1)      /* bad argument or malformed plan blob          */
#define TN_ENOMEM (-2)      /* request can never fit in the arena            */
#define TN_EBUSY (-3)       /* plan still referenced by pending requests     */
#define TN_EDEVICE (-4)     /* HIP error; the context is poisoned            */
#define TN_ECANCELLED (-5)  /* request was cancelled                         */
#define TN_ENOTFOUND (-6)   /* unknown ticket                                */

/* precision modes */
#define TN_FP32_4M 0        /* complex64 operands, 4 real products, FP32 MFMA   */
#define TN_FP32_3M 1        /* complex64 operands, 3 real products on FP32 MFMA:
                               Ar Br, Ai Bi, (Ar+Ai)(Br+Bi); steps whose output
                               has at most 16 entries use the 4M dot kernel */
#define TN_SPLIT_BF16 2     /* x = hi + lo in bf16, hi*hi + hi*lo + lo*hi, FP32 acc */
#define TN_SPLIT_FP16 3     /* x = hi + lo in fp16 after a power-of-two scale per
                               row of A and column of B (largest |re|, |im|
                               scaled into [2^14, 2^15)), hi*hi + hi*lo + lo*hi,
                               FP32 acc, both scales undone exactly in the
                               epilogue; the scales depend only on that row's
                               (column's) own entries, so a result does not
                               depend on the chunk or co-scheduled requests */
#define TN_BF16_1TERM 4     /* operands rounded once to bf16, one product per
                               complex product, FP32 accumulation: the plain
                               rounding reference point for the split mode */

typedef struct tn_ctx tn_ctx;
typedef struct tn_plan tn_plan;

typedef struct tn_plan_info_t {
    int32_t n_qubits;
    int32_t n_leaves;
    int32_t n_steps;
    int32_t n_sliced;                 /* log2 of the number of slices            */
    int32_t max_rank;                 /* widest intermediate, labels (batch excl.) */
    int32_t reserved;
    double flops_per_slice_per_b;     /* algorithmic real flops, 8 per complex MAC */
    double flops_total_per_b;         /* over all slices: each step once per value
                                         of the sliced labels it depends on     */
    uint64_t peak_bytes_fixed;        /* workspace independent of the batch size */
    uint64_t peak_bytes_per_b;        /* plus this much per bitstring in a chunk */
} tn_plan_info_t;

typedef struct tn_req_stats {
    int64_t t_arrive_ns;              /* tn_submit                      */
    int64_t t_admit_ns;               /* memory granted                 */
    int64_t t_start_ns;               /* first kernel enqueued          */
    int64_t t_end_ns;                 /* results on the host            */
    int32_t batch;                    /* bitstrings in the device batch */
    int32_t plan_id;
} tn_req_stats;

/*
 * tn_ctx_create: one context per device.
 *   device     HIP device ordinal.
 *   arena      device pointer to caller-owned memory (e.g. a torch uint8
 *              tensor) or NULL to let the library allocate `arena_bytes`.
 *   arena_bytes size of the arena; every plan's workspace comes from it.
 * Errors: TN_EINVAL (bad device / size), TN_EDEVICE (allocation failed).
 */
int tn_ctx_create(int device, void* arena, size_t arena_bytes, tn_ctx** out);

/* Tear down: waits for pending work, frees library allocations. */
int tn_ctx_destroy(tn_ctx* ctx);

/*
 * tn_plan_load: copy and validate a TNP1 blob (written by the plan builder),
 * convert leaves from complex128 to complex64 (round to nearest even) and
 * upload them.  The plan stays resident until unloaded.
 * A blob with header flag bit 0 set is a projector plan: the network of C
 * and its complex conjugate for the quantity <0|C^dag (x)_q P_q C|0> (the
 * problem statement around Theorem 2), with P_q = |x_q><x_q| on qubits that
 * carry output labels (two per qubit, one in each layer) and P_q = 1 on the
 * others (no output label; their bitstring bits must be 0).  Contracting it
 * returns that value for each bitstring in place of an amplitude.
 * Errors: TN_EINVAL (malformed blob: bad magic/version, truncated, label out
 * of range, dimension other than 2, operand used twice, step orders that do
 * not form a batched GEMM), TN_EDEVICE.
 */
int tn_plan_load(tn_ctx* ctx, const void* blob, size_t nbytes, tn_plan** out);

/* Parse and validate a blob on the host only (no device needed). */
int tn_plan_validate(const void* blob, size_t nbytes, tn_plan_info_t* info);

int tn_plan_info(const tn_plan* plan, tn_plan_info_t* out);

/* TN_EBUSY while requests on the plan are pending; TN_EINVAL for a plan that
 * this context did not load or that was already unloaded.  tn_ctx_destroy
 * unloads the plans still loaded. */
int tn_plan_unload(tn_ctx* ctx, tn_plan* plan);

/*
 * tn_contract_amplitudes: blocking.  bits[nb] -> out_re_im[2*nb]: the
 * amplitudes <x|C|0>, or for a projector plan <0|C^dag (x)_q P_q C|0>.
 *   precision   one of the TN_* precision modes.
 *   hip_stream  a hipStream_t to run on, or NULL for the context's stream.
 * The batch is processed in chunks sized to the arena.
 * Errors: TN_EINVAL (nb <= 0, a bit set at position >= n_qubits, bad mode),
 * TN_ENOMEM (one bitstring does not fit), TN_EDEVICE.
 */
int tn_contract_amplitudes(tn_ctx* ctx, const tn_plan* plan, const uint64_t* bits,
                           int32_t nb, int32_t precision, void* hip_stream,
                           double* out_re_im);

/*
 * tn_submit / tn_poll / tn_cancel: the serving loop.  tn_submit copies
 * `bits` and returns at once with a ticket; a scheduler thread admits
 * requests as arena memory and execution slots free up (admission by the
 * plan's peak bytes at the request's batch), merges queued requests on the
 * same plan and precision into one device batch, and runs admitted batches
 * concurrently on separate streams.  tn_poll returns TN_PENDING until the
 * request is done, then TN_OK with the amplitudes (and stats if st != NULL);
 * a ticket can be polled to completion once.
 * Errors: TN_ENOMEM at submit when one bitstring of the plan cannot fit the
 * arena at all; TN_ECANCELLED from tn_poll after tn_cancel.
 */
int tn_submit(tn_ctx* ctx, const tn_plan* plan, const uint64_t* bits, int32_t nb,
              int32_t precision, uint64_t* ticket);
int tn_poll(tn_ctx* ctx, uint64_t ticket, double* out_re_im, tn_req_stats* st);
int tn_cancel(tn_ctx* ctx, uint64_t ticket);

/* Serving configuration: number of concurrent slots (streams), max merged
 * batch.  Call before the first tn_submit. */
int tn_server_config(tn_ctx* ctx, int32_t n_slots, int32_t max_batch);

/* Heavy batches: a merged batch whose algorithmic work (the plan's flops
 * per bitstring, summed over slices, times its bitstrings) is at least
 * `heavy_flops` runs only while fewer than `max_heavy` other heavy batches
 * run; lighter batches use the remaining slots meanwhile.  Defaults 1e14 and
 * 1.  May be called at any time; TN_EINVAL for a negative threshold or
 * max_heavy < 1. */
int tn_server_set_heavy(tn_ctx* ctx, double heavy_flops, int32_t max_heavy);

/* Stop the scheduler and slot threads (pending work finishes first);
 * tn_ctx_destroy calls it. */
int tn_server_stop(tn_ctx* ctx);

/* Per-context counters of the last tn_contract_amplitudes call (debug):
 * kernel time is not measured here; these are host-side counts. */
typedef struct tn_exec_stats {
    int64_t kernels_gemm;
    int64_t kernels_permute;
    int64_t kernels_gather;
    int64_t steps_executed;
    int64_t steps_reused;
    int32_t chunk;                    /* bitstrings per device chunk */
    int32_t n_chunks;
    int32_t slice_block;              /* slices computed together per pass */
    int32_t graph_replays;            /* chunks run by replaying a captured HIP graph */
    double algorithmic_flops;         /* sum over executed steps     */
    double permute_bytes;             /* 16 bytes per permuted element */
    /* per kernel class (0 dot-product GEMM for tiny outputs, 1 MFMA GEMM
     * 64x64 tile, 2 MFMA GEMM 128x128 tile (128x64 for FP32 3M), 3 MFMA GEMM
     * for skinny products (a 128x16 tile; FP32 3M: 128x32, or 64x32, 32x32 and
     * 32x128 for at most 64 or 32 rows), 4 permute, 5 leaf gather, 6 MFMA GEMM
     * one wave per 32x32 block for products of at most 4096 outputs per batch
     * entry): launches, summed
     * device time from HIP events
     * recorded around each launch on the executing stream (only when
     * profiling is on), algorithmic flops (GEMM: 8 per complex multiply-add)
     * and algorithmic bytes (GEMM: operands read once and C written once;
     * permute: 16 per element; gather: 8 per written element) */
    int64_t launches[7];
    double time_ms[7];
    double flops[7];
    double bytes[7];
} tn_exec_stats;

/* Turn per-launch event timing of tn_contract_amplitudes on (1) or off (0).
 * While it is on, chunks are launched kernel by kernel (no graph replay). */
int tn_ctx_set_profiling(tn_ctx* ctx, int32_t on);

/* HIP graphs for repeated calls (default on).  The kernels of one chunk
 * (accumulator reset, every gather, permute and GEMM of every pass, slice
 * sums and final scale) depend only on the plan, the chunk size, the slice
 * block, the precision and the workspace address; the bitstrings are read
 * from device memory that each call refills before the launch.  The second
 * time such a chunk runs it is captured into a graph, and later runs replay
 * it with one launch.  Graphs of a plan are destroyed when it is unloaded;
 * at most 256 are kept per context.  Results are bitwise the same either
 * way. */
int tn_ctx_set_graphs(tn_ctx* ctx, int32_t on);

/* Slices computed together per pass of the slice loop, as log2 (-1 =
 * automatic: the largest block that fits the workspace).  Tensors that depend
 * on the low slice bits then hold one copy per slice of the block, and the
 * slices of a block run as one batched (or folded) GEMM per step; every
 * slice's arithmetic is unchanged, so results do not depend on the block. */
int tn_ctx_set_slice_block(tn_ctx* ctx, int32_t log2_block);
int tn_last_exec_stats(tn_ctx* ctx, tn_exec_stats* out);

/*
 * Kernel entry points on caller-owned device memory (complex64 interleaved),
 * for kernel tests and per-kernel measurement.  They enqueue on `hip_stream`
 * (NULL = the default stream) and do not synchronise.
 *
 * tn_kernel_cgemm: for ob < nb, ib < nbatch:
 *   C[ob*sCb + ib*sCi + m*N + n] = sum_k A(m,k) * B(k,n)
 *   A(m,k) = A[ob*sAb + ib*sAi + (transA ? k*M + m : m*K + k)]
 *   B(k,n) = B[ob*sBb + ib*sBi + (transB ? n*K + k : k*N + n)]
 *   strides in complex elements; sAb or sBb may be 0 (broadcast); M, N, K
 *   powers of two.  precision TN_FP32_4M, TN_FP32_3M, TN_SPLIT_BF16,
 *   TN_SPLIT_FP16 or TN_BF16_1TERM.  `scratch`: device memory for split-K
 *   partial sums and, for TN_SPLIT_FP16, the row and column maxima (see
 *   tn_kernel_cgemm_scratch_bytes).  Returns TN_EINVAL for bad sizes or too
 *   little scratch, TN_EDEVICE on a launch error.
 * tn_kernel_permute: bit permutation of the element index:
 *   dst[b*2^rank + sum_p bit_{perm[p]}(i) << p] = src[b*2^rank + i]
 *   (destination bit p takes source bit perm[p]); rank <= 40, perm must be a
 *   permutation of 0..rank-1 (TN_EINVAL otherwise).
 */
int tn_kernel_cgemm(const void* A, const void* B, void* C, int32_t M, int32_t N, int32_t K,
                    int32_t transA, int32_t transB, int32_t nbatch, int32_t nb,
                    int64_t sAb, int64_t sBb, int64_t sCb, int64_t sAi, int64_t sBi,
                    int64_t sCi, int32_t precision, void* scratch, size_t scratch_bytes,
                    void* hip_stream);
/* Device scratch tn_kernel_cgemm needs for this shape in any precision mode
 * (split-K partials, 256-byte aligned, then 4 bytes per row of A and column
 * of B for TN_SPLIT_FP16); a call with less than its mode needs returns
 * TN_EINVAL. */
size_t tn_kernel_cgemm_scratch_bytes(int32_t M, int32_t N, int32_t K, int32_t nbatch, int32_t nb);
/* How tn_kernel_cgemm (and every plan step of this shape) sums over k, host
 * only: *kind is the kernel class (0: K-parallel dot product for M*N <= 16,
 * summed in float64; 1, 2, 3: MFMA tiles of 64x64, 128x128, 128x16 class;
 * 6: one wave per 32x32 block for M*N <= 4096, K <= 256 and one K range
 * in the FP32 modes (the split modes take the 128x16 tile there); every MFMA class
 * accumulates each output element in FP32 over its K range); *splits is the
 * number of K ranges of K/splits consecutive k (split-K), whose partial sums
 * are added in float64 in range order.  The summation order fixes the
 * rounding error of a step: the accumulation of one element rounds K/splits
 * times.  TN_EINVAL unless M, N, K are powers of two and nbatch >= 1. */
int tn_kernel_cgemm_shape(int32_t M, int32_t N, int32_t K, int32_t nbatch, int32_t* kind,
                          int32_t* splits);
/* tn_kernel_cgemm without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * tn_kernel_cgemm (bitwise); the split-K partials and split fp16 maxima live
 * in a device array of the library, one per GPU, of
 * tn_kernel_cgemm_noalloc_max_scratch() bytes (32 MiB), reserved when the
 * library is loaded on that GPU and held until the process ends.  A shape
 * whose scratch (tn_kernel_cgemm_scratch_bytes) exceeds it returns TN_EINVAL
 * before any device work.  Runs on the current device; no call allocates
 * (no hipMalloc, no allocating library routine).  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (concurrent
 * streams or threads) race; calls ordered on one stream do not.  TN_EDEVICE
 * if the array's address cannot be found. */
int tn_kernel_cgemm_noalloc(const void* A, const void* B, void* C, int32_t M, int32_t N,
                            int32_t K, int32_t transA, int32_t transB, int32_t nbatch,
                            int32_t nb, int64_t sAb, int64_t sBb, int64_t sCb, int64_t sAi,
                            int64_t sBi, int64_t sCi, int32_t precision, void* hip_stream);
size_t tn_kernel_cgemm_noalloc_max_scratch(void);
int tn_kernel_permute(const void* src, void* dst, int32_t rank, const int32_t* perm,
                      int32_t nb, void* hip_stream);

const char* tn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TNAMP_H */
