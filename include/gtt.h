/*
 * gtt.h -- C ABI of libgtt.so, the MI355X (gfx950) fast generalized tensor
 * transform (GTT).
 *
 * The transform (Shukla & Vedula, §2.6, Def. 2.4) is
 *
 *     y = G_N x,   G_N = W kron W kron ... kron W   (n factors),  N = b^n,
 *
 * with entries G_N(p, q) = prod_{j<n} W[p_j][q_j] (§2.6, product formula
 * after Def. 2.4), where p = sum_j p_j b^j is the base-b expansion of an index
 * (digit 0 least significant, §2.1) and W[r][c] is row r, column c of the
 * b x b base matrix (0-based, §2.1).  The fast algorithm (§3, Alg. 1) applies
 * W along one base-b digit at a time; this library fuses several such digit
 * passes per trip through HBM.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Layout: an instance is N contiguous elements, index i = sum_j i_j b^j,
 *    i_0 fastest.  A uniform batch is `batch` instances back to back.
 *  - W: row-major b x b matrix in the *compute* dtype of the plan:
 *      GTT_F64 -> double, GTT_F32/GTT_BF16/GTT_F16 -> float,
 *      GTT_C64 -> complex float (re, im interleaved), GTT_C128 -> complex
 *      double, GTT_I32 -> int32 (arithmetic mod 2^32, two's complement).
 *  - Complex data is interleaved (re, im), as in torch.complex64/complex128.
 *  - Pointers named x, y, W, gy, gx, gW, saved and ws are DEVICE pointers
 *    owned by the caller; the library never frees them.  Forward / inverse
 *    / backward allocate no device memory (a ragged plan's work list is
 *    uploaded by gtt_plan; see there).
 *  - All device work is enqueued on `stream` (a hipStream_t; NULL is the
 *    null stream).  Calls return as soon as the work is enqueued.
 *  - Argument checks run on the host, before any HIP call, and report a
 *    status code; nothing throws across this ABI.  A failed kernel launch is
 *    reported as GTT_ERR_HIP.
 *  - Aliasing: x == y (and gy == gx) is allowed (in place); any other
 *    partial overlap of buffers is undefined behaviour.
 *  - Alignment: every data pointer must be 16-byte aligned
 *    (GTT_ERR_ALIGNMENT otherwise).
 *  - A plan is immutable after creation and may be used concurrently from
 *    several host threads on different streams, provided each call has its
 *    own workspace.
 *  - Determinism: for a fixed plan and inputs y, gx and gW are bitwise
 *    reproducible (all reductions run in a fixed order).
 */
#ifndef GTT_H
#define GTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gtt_status {
    GTT_OK = 0,
    GTT_ERR_INVALID_VALUE = 1, /* null pointer, bad flag, count < 1, ... */
    GTT_ERR_SHAPE = 2,         /* b < 2, n < 0, b^n overflows int64, batch < 1 */
    GTT_ERR_DTYPE = 3,         /* unknown dtype */
    GTT_ERR_ALIGNMENT = 4,     /* a data pointer is not 16-byte aligned */
    GTT_ERR_WORKSPACE = 5,     /* ws_bytes smaller than the call needs */
    GTT_ERR_UNSUPPORTED = 6,   /* valid request the library does not implement */
    GTT_ERR_HIP = 7,           /* a HIP runtime call or kernel launch failed */
    GTT_ERR_INTERNAL = 8,
    GTT_ERR_TIMEOUT = 9        /* a persistent ragged launch gave up waiting at a
                                  grid barrier (reported by gtt_plan_check) */
} gtt_status;

typedef enum gtt_dtype {
    GTT_F64 = 0,
    GTT_F32 = 1,
    GTT_C128 = 2,
    GTT_C64 = 3,
    GTT_BF16 = 4,
    GTT_F16 = 5,
    GTT_I32 = 6
} gtt_dtype;

/* Plan flags (bit set). */
#define GTT_FLAG_FP32_INTERMEDIATE 0x1u /* bf16/f16 uniform plans: convert
                                           the operands to float32 inside the
                                           workspace, run every digit group in
                                           float32 and round to the storage
                                           dtype once, at the end (saved
                                           activations are then float32).
                                           No effect on the other dtypes;
                                           GTT_ERR_UNSUPPORTED for ragged and
                                           mixed-radix plans, and from
                                           gtt_filter / gtt_compress */
#define GTT_FLAG_NO_TUNE 0x2u           /* ignore the tuning table; use the
                                           built-in heuristics */
#define GTT_FLAG_PERSISTENT 0x4u        /* ragged batch: run every digit group
                                           of every instance in ONE persistent
                                           launch, grid barrier between digit
                                           groups (default: one launch per
                                           digit-group phase and tile class,
                                           with class-specialised kernels) */
#define GTT_FLAG_PER_INSTANCE 0x8u      /* ragged batch: one launch per digit
                                           group per instance (the plain path) */

typedef struct gtt_plan_s* gtt_plan_t;

/*
 * gtt_plan -- build an execution plan.
 *
 * Uniform batch (count == 1): instance radix b[0] and digit count n[0] apply to
 * `batch` contiguous instances; x_off and w_idx must be NULL.
 *
 * Ragged batch (count > 1, `batch` must be 1): instance t has radix b[t] and
 * n[t] digits (N_t = b[t]^n[t]) and starts at element offset x_off[t] of the
 * data buffers (x_off == NULL: instances packed back to back in order).
 * Instance t uses base matrix number w_idx[t] of the W table; the table holds
 * its matrices back to back in index order, matrix w being b_w x b_w where
 * b_w is the radix of the instances that use it (they must agree and every
 * index 0..max must be used).  w_idx == NULL means one matrix per distinct
 * radix, in ascending order of radix.  gW of a ragged plan has the layout of
 * the W table.
 *
 * n == 0 is allowed (N = 1, the identity; base case of §2.2).
 * Errors: GTT_ERR_SHAPE (b < 2, n < 0, b^n overflows, batch < 1),
 * GTT_ERR_DTYPE, GTT_ERR_INVALID_VALUE (out == NULL, count < 1, bad
 * w_idx / x_off), GTT_ERR_UNSUPPORTED (GTT_FLAG_FP32_INTERMEDIATE with
 * count > 1).  On error *out is set to NULL.
 * The plan holds host memory and, for ragged batches, a device work list
 * (one descriptor per instance and digit group, one entry per tile) and the
 * grid-barrier words.  gtt_plan builds the list and uploads it, synchronously,
 * to the device current at that time; calls on the plan must run with that
 * device current (GTT_ERR_INVALID_VALUE otherwise), and every forward /
 * inverse call, the first included, allocates nothing and can be captured
 * into a graph.  (Only when no device is visible to the process at plan
 * time is the upload deferred to the plan's first forward / inverse call.)
 * gtt_plan_destroy frees the list.  Without GTT_FLAG_PERSISTENT a ragged call
 * launches, in order on the caller's stream, one kernel per phase and tile
 * class.  With GTT_FLAG_PERSISTENT a call launches a one-thread reset of the
 * barrier words and then ONE kernel whose grid (occupancy x compute units)
 * waits at a grid barrier between digit groups; the wait is bounded (see
 * gtt_plan_barrier_limit) and a failed wait is reported by gtt_plan_check.
 * Calls with GTT_FLAG_PERSISTENT share the plan's barrier words: do not run
 * one such plan on two streams at once.
 */
gtt_status gtt_plan(gtt_plan_t* out, int32_t count, const int32_t* b, const int32_t* n,
                    int64_t batch, const int64_t* x_off, const int32_t* w_idx,
                    gtt_dtype dtype, uint32_t flags);

/*
 * gtt_plan_mixed -- plan for the heterogeneous transform
 *     G = W_0 kron W_1 kron ... kron W_{m-1},   N = prod_k b_k
 * (§2.6, remark on distinct tensor factors), factor W_k being b_k x b_k
 * (radices[k] = b_k).  As in the Kronecker product, the leftmost factor W_0
 * acts on the most significant mixed-radix digit: factor k acts on the digit
 * whose place value is b_{k+1} b_{k+2} ... b_{m-1}.  W is passed to forward /
 * inverse as the matrices W_0, W_1, ..., W_{m-1} back to back (compute
 * dtype, row-major).  `batch` contiguous instances of N elements.
 * gtt_backward returns gW in the same layout (the gradient of every factor);
 * gtt_filter returns GTT_ERR_UNSUPPORTED for mixed plans.
 */
gtt_status gtt_plan_mixed(gtt_plan_t* out, int32_t m, const int32_t* radices, int64_t batch,
                          gtt_dtype dtype, uint32_t flags);

/*
 * gtt_workspace_size -- bytes of device workspace a call needs.
 *   fwd   : forward and inverse (currently 0 unless the FP32-intermediate
 *           flag is set);
 *   bwd   : backward in the worst case (`saved` NULL, so the activations
 *           between digit groups are recomputed, and gx NULL or equal to
 *           gy, so the gradient between groups needs its own buffer); when
 *           `saved` is passed, *bwd - *saved bytes suffice;
 *   saved : size of the optional `saved` buffer of forward/backward (the
 *           activations at the boundaries between digit groups).
 * Any output pointer may be NULL.
 */
gtt_status gtt_workspace_size(gtt_plan_t p, size_t* fwd, size_t* bwd, size_t* saved);

/*
 * gtt_forward -- y = G_N x for every instance (Def. 2.4; fast algorithm §3).
 * If `saved` is non-NULL it receives the activations between digit groups
 * (size from gtt_workspace_size), for a later gtt_backward.
 */
gtt_status gtt_forward(gtt_plan_t p, const void* W, const void* x, void* y, void* saved,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * gtt_inverse -- x = G_N^dagger y = (W^H)^{kron n} y, the inverse transform
 * used by the paper's applications (§4.1, §4.3).  It is the inverse of
 * gtt_forward only when W is unitary; for GTT_I32 W^H is W^T (for the
 * unnormalised +-1 Hadamard, inverse(forward(x)) = 2^n x exactly).
 */
gtt_status gtt_inverse(gtt_plan_t p, const void* W, const void* y, void* x,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * gtt_backward -- gradients of a real loss L through y = G_N x, in the
 * convention dL/dRe + i dL/dIm (PyTorch's), given gy = dL/dy:
 *     gx = G_N^H gy;
 *     gW = sum over digits s, instances and fibres of digit s of c_s a_s^H,
 * where a_s is the input of the pass on digit s and c_s the gradient at its
 * output (for real dtypes ^H is ^T).  gW is overwritten (compute dtype; b x b
 * for uniform plans, the W table's layout for ragged plans, the factors
 * W_0 .. W_{m-1} back to back for mixed plans), never accumulated; it is
 * summed in FP64 (complex FP64 for complex data) and rounded once.  gx or gW
 * may be NULL to skip them (not both).  `saved` (nullable) is the buffer
 * filled by gtt_forward for the same x and W; without it the activations are
 * recomputed in the workspace.  Floating dtypes and radices up to 32 (every
 * factor of a mixed plan); GTT_ERR_UNSUPPORTED for GTT_I32 and larger radices.
 */
gtt_status gtt_backward(gtt_plan_t p, const void* W, const void* x, const void* saved,
                        const void* gy, void* gx, void* gW, void* ws, size_t ws_bytes,
                        void* stream);

/*
 * gtt_backward_noalloc -- gtt_backward for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same gradients, bit for bit, with no `ws`
 * argument.  The workspace is a device array of GTT_NOALLOC_SCRATCH_BYTES
 * inside the library, one per GPU, held until the process ends; the call
 * allocates nothing (its first call on a device looks up that array's
 * address).  GTT_ERR_WORKSPACE, before any HIP call, when the call needs more
 * than that: pass `saved` (else the activations between digit groups are
 * recomputed in the scratch) and a gx that is not gy (else the cotangent
 * between digit groups is kept there) to need only the gradient partial sums.
 * Every call on one GPU shares its array: calls that overlap on one GPU (on
 * different streams or host threads) race and must be serialised by the
 * caller.
 */
#define GTT_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
gtt_status gtt_backward_noalloc(gtt_plan_t p, const void* W, const void* x, const void* saved,
                                const void* gy, void* gx, void* gW, void* stream);

/*
 * gtt_filter -- classical natural-order filter (§4.3, Alg. 3 without the
 * ancilla): coefficients X = G_N x are split at natural index `cutoff`
 * (k < cutoff -> low, k >= cutoff -> high) and each part is mapped back with
 * G_N^dagger.  low or high may be NULL.  Uniform plans, floating dtypes.
 * Needs gtt_workspace_size's fwd bytes plus N*batch elements of the storage
 * dtype (the coefficients) in `ws`.
 */
gtt_status gtt_filter(gtt_plan_t p, const void* W, const void* x, int64_t cutoff,
                      void* low, void* high, void* ws, size_t ws_bytes, void* stream);

/*
 * gtt_compress -- classical state-transmission protocol (§4.1.1): the
 * coefficients X = G_N x of every instance, the k of largest magnitude
 * (|X|^2 in the compute precision; ties broken towards the lower index),
 * written as idx[t][j] (int64, ascending) and val[t][j] (storage dtype),
 * t < batch, j < k; if recon != NULL also recon = G_N^dagger applied to the
 * vector that keeps only those k coefficients (the receiver's
 * reconstruction).  1 <= k <= N.  Uniform plans.  Needs
 * gtt_compress_workspace_size bytes in `ws` (the coefficients, and for few
 * large instances the selection's state, histograms and per-chunk counts);
 * GTT_ERR_WORKSPACE when ws_bytes is smaller.
 */
gtt_status gtt_compress(gtt_plan_t p, const void* W, const void* x, int64_t k, int64_t* idx, void* val,
                        void* recon, void* ws, size_t ws_bytes, void* stream);

/*
 * gtt_compress_workspace_size -- bytes of `ws` gtt_compress needs for this
 * plan (independent of k).  GTT_ERR_UNSUPPORTED for plans gtt_compress
 * refuses.
 */
gtt_status gtt_compress_workspace_size(gtt_plan_t p, size_t* bytes);

/*
 * gtt_plan_check -- waits for the work enqueued on `stream`, then reports
 * whether a persistent ragged launch of this plan gave up waiting at a grid
 * barrier since the last check (GTT_ERR_TIMEOUT; its outputs are incomplete)
 * and clears that record.  GTT_OK for plans without persistent launches.
 * Synchronous; not for use inside a graph capture.
 */
gtt_status gtt_plan_check(gtt_plan_t p, void* stream);

/*
 * gtt_plan_barrier_limit -- polls (each followed by a short sleep) that a
 * work-group of a persistent ragged launch makes at a grid barrier before it
 * gives up (default 2^24, several seconds).  A work-group that gives up
 * raises the launch's failure word; every work-group leaves the kernel at its
 * next barrier, and gtt_plan_check reports GTT_ERR_TIMEOUT.
 * GTT_ERR_INVALID_VALUE for plans that are not ragged.
 */
gtt_status gtt_plan_barrier_limit(gtt_plan_t p, uint32_t polls);

/*
 * Frees the plan and its device memory (the ragged work list, timing
 * events).  NULL is accepted.  It calls hipFree: not while a stream capture
 * is running in the process in global capture mode (the capture would be
 * invalidated); the Python binding defers the destruction of a plan collected
 * during a capture until the capture has ended.
 */
gtt_status gtt_plan_destroy(gtt_plan_t p);

/* Static, human-readable name of a status code. */
const char* gtt_status_string(gtt_status s);

/*
 * gtt_plan_describe -- writes a NUL-terminated JSON description of the plan
 * (digit groups, tile shapes, launch sizes) into buf (truncated to len).
 */
gtt_status gtt_plan_describe(gtt_plan_t p, char* buf, size_t len);

/*
 * gtt_plan_timing -- instrumentation: when enable != 0, every kernel launch
 * made through this plan is bracketed by HIP events recorded on the call's
 * stream.  gtt_plan_timing_read waits for the recorded events and writes a
 * JSON object {name: {launches, total_ms, avg_ms, bytes_per_launch}} (one
 * entry per kernel kind and digit group; bytes_per_launch is the algorithmic
 * HBM traffic of one launch: 2 E s for a forward/inverse pass, 3 E s for a
 * backward group), then forgets the recorded launches.  Timing mutates the
 * plan: do not time a plan used concurrently by several threads.
 */
gtt_status gtt_plan_timing(gtt_plan_t p, int32_t enable);
gtt_status gtt_plan_timing_read(gtt_plan_t p, char* buf, size_t len);

/*
 * gtt_plan_timing_filter -- instrumentation: with timing enabled, bracket
 * only the launches whose name (as gtt_plan_timing_read reports it) starts
 * with `prefix`; the other launches record no events and cost nothing.
 * NULL or "" times every launch again.  The string is copied.
 */
gtt_status gtt_plan_timing_filter(gtt_plan_t p, const char* prefix);

/*
 * gtt_set_tuning -- override the launch heuristics for plans created after
 * this call, for radix b, digit count n (0: every n without an entry of its
 * own) and storage dtype (used by the autotuner; uniform plans and each
 * instance of a ragged plan look up their own (b, n)):
 *   lds_budget_bytes : LDS bytes of one forward tile (0 = default),
 *   min_row_bytes    : least contiguous bytes per tile row for strided digit
 *                      groups (0 = default),
 *   max_group_digits : most digits fused into one HBM round trip (0 = no
 *                      limit beyond the tile size),
 *   bwd_lds_bytes    : LDS bytes of one work-group of the general backward
 *                      (tiles and checkpoint slots; 0 = default search).
 * All four values 0 removes the entry for (b, n, dtype) (the radix-wide
 * entry or the defaults apply again).  Process-wide; not thread-safe against
 * concurrent gtt_plan calls.
 */
gtt_status gtt_set_tuning(int32_t b, int32_t n, gtt_dtype dtype, int32_t lds_budget_bytes, int32_t min_row_bytes,
                          int32_t max_group_digits, int32_t bwd_lds_bytes);

/*
 * gtt_selftest -- host-only checks of the index arithmetic (fast division by
 * constants, digit grouping); touches no GPU.  Returns GTT_OK on success.
 */
gtt_status gtt_selftest(void);

#ifdef __cplusplus
}
#endif

#endif /* GTT_H */
