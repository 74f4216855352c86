/*
 * sttsm.h -- C ABI of libsttsm.so: symmetric tensor times same matrix on
 * MI355X (gfx950), with tensors in Blocked Compact Symmetric Storage.
 *
 * Method: Schatz, Low, van de Geijn, Kolda, "Exploiting Symmetry in Tensors
 * for High Performance: Multiplication with Symmetric Tensors"
 * (arXiv:1301.7744).
 *
 * General rules
 *  - Every function that returns `int` returns an sttsm_status.  Nothing
 *    aborts or throws across this boundary; sttsm_last_error() gives a
 *    message for the calling thread.
 *  - Arguments are validated on the host before anything is launched.
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *    Launches are asynchronous on it; a device fault surfaces as
 *    STTSM_EHIP from a later call or from the caller's own synchronisation.
 *  - The caller owns every buffer passed in (device memory unless stated).
 *    The library owns only its plan cache (host and device index tables,
 *    built once per shape and kept until the process ends) and the serving
 *    bookkeeping.
 *  - Dense tensors are in dimensional order (App. A): element
 *    (i_0, ..., i_{m-1}) of an extent-n tensor is at sum_k i_k n^k.  For a
 *    symmetric tensor this is also the row-major layout of shape (n,)*m.
 *  - BCSS (§3.3, §4.3, §5.3): blocks of b^m entries; only blocks with sorted
 *    block index s_0 <= ... <= s_{m-1} are stored, in colex order
 *    (rank(s) = sum_k binom(s_k + k, k + 1); at b = 1, m = 2 this is the
 *    packing order 0 1 3 / 2 4 / 5 of §3.3).  Each block is stored whole, in
 *    dimensional order, padded with zeros when b does not divide n.
 *  - Reentrant: sttsm and bcss_* may be called from several threads.
 */
#ifndef STTSM_H
#define STTSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STTSM_OK = 0,
    STTSM_EINVAL = -1,    /* bad argument; nothing was launched               */
    STTSM_ENOMEM = -2,    /* host/device allocation failed, or too big to fit */
    STTSM_EHIP = -3,      /* a HIP runtime call failed                       */
    STTSM_EAGAIN = -4,    /* serving: result not ready yet                    */
    STTSM_ENOTFOUND = -5  /* serving: unknown or already fetched ticket      */
} sttsm_status;

typedef enum { STTSM_F32 = 0, STTSM_BF16 = 1, STTSM_F64 = 2 } sttsm_dtype;

/*
 * Precision forms of the block contractions.
 *  FP32                 FP32 operands, temporaries and accumulation
 *                       (v_mfma_f32_32x32x2_f32).  A, X: F32.
 *  BF16                 A, X and the temporaries T^(k) rounded to bf16
 *                       (nearest, ties to even), FP32 MFMA accumulation,
 *                       temporaries stored bf16, C in FP32.  A, X: F32 or
 *                       BF16 (same dtype for both).
 *  BF16X3_FIRST_FP32    first contraction A -> T^(m-1) as three bf16
 *                       products hi*hi + hi*lo + lo*hi of the split
 *                       a = hi + lo (hi = bf16(a), lo = bf16(a - hi));
 *                       later contractions FP32.  A, X: F32.
 *  BF16X3_FIRST_BF16    split first contraction, T^(m-1) stored bf16, later
 *                       contractions as in BF16.  A, X: F32.
 * C is always F32.
 */
typedef enum {
    STTSM_PREC_FP32 = 0,
    STTSM_PREC_BF16 = 1,
    STTSM_PREC_BF16X3_FIRST_FP32 = 2,
    STTSM_PREC_BF16X3_FIRST_BF16 = 3
} sttsm_prec;

/* Shape of a symmetric tensor: order m (1..8), extent n (>= 1), block size
 * b (>= 1), element type. */
typedef struct {
    int32_t m;
    int64_t n;
    int32_t b;
    int32_t dtype; /* sttsm_dtype */
} bcss_layout;

/* binom(nbar + m - 1, m), the number of stored blocks (Table 1); -1 when
 * m < 1, nbar < 1 or the count overflows int64. */
int64_t bcss_num_blocks(int32_t m, int64_t nbar);

/* Entries of the BCSS array, b^m * bcss_num_blocks(m, ceil(n/b)) (padded);
 * -1 on a bad layout. */
int64_t bcss_num_elems(const bcss_layout *L);

/* Dense -> BCSS (§5.3).  Copies each sorted block of the dense tensor into its
 * compact slot, bit for bit; entries beyond n are written as zero.  Only the
 * sorted blocks of `dense` are read, so a non-symmetric input is packed
 * without complaint (its other blocks are ignored).
 * dense: n^m elements of L->dtype on the device; bcss: bcss_num_elems(L). */
int bcss_pack(const bcss_layout *L, const void *dense, void *bcss, void *stream);

/* BCSS -> dense.  Every dense block t is read from stored block sort(t) with
 * its modes permuted by the stable argsort of t (App. B's meta-data tensor);
 * padding is dropped.  Same buffer sizes as bcss_pack. */
int bcss_unpack(const bcss_layout *L, const void *bcss, void *dense, void *stream);

/*
 * In-place symmetrisation of a BCSS tensor, the post-processing step the end
 * of §5.4 suggests for the rounding-level asymmetry inside blocks whose
 * block indices repeat (sttsm computes each entry of such a block on its
 * own).  Every entry of such a block becomes the average of its orbit under
 * the block's stabiliser, the permutations of modes that carry equal block
 * indices; afterwards mirrored entries are bitwise equal.  Blocks with
 * distinct block indices are not touched.  The result equals packing the
 * average of the dense tensor over all m! mode permutations.  Averages are
 * summed in fp32 (f64 for F64 tensors) in a fixed order; bf16 results are
 * rounded to nearest even.  Needs ceil(n/b)^m <= 2^24 (else ENOMEM).
 */
int bcss_symmetrize(const bcss_layout *L, void *bcss, void *stream);

/* Fills a BCSS tensor with a symmetric pseudo-random tensor, for tests and
 * benchmarks that cannot afford a dense original: the entry with sorted
 * index s_0 <= ... <= s_{m-1} is lo + (hi - lo) u, u = (h >> 40) 2^-24,
 * h = f(...f(f(seed) ^ s_0)...) ^ s_{m-1}) with f the SplitMix64 finaliser
 * (Steele, Lea, Flood 2014), rounded to L->dtype (nearest, ties to even);
 * padding entries are zero.  Asynchronous on `stream`. */
int bcss_fill_hashed(const bcss_layout *L, uint64_t seed, double lo, double hi, void *bcss, void *stream);

/* Symmetry-aware flop count of sttsm (Table 2, BCSS computation row, at the
 * padded sizes nbar*bA and pbar*bC); -1 on bad layouts. */
int64_t sttsm_flops(const bcss_layout *A, const bcss_layout *C);

/* Bytes of device workspace sttsm needs for these shapes and precision
 * (padded X panels and every temporary T^(m-1) .. T^(1)); 0 on bad input. */
size_t sttsm_workspace_bytes(const bcss_layout *A, const bcss_layout *C, int32_t prec);

/*
 * C := [A; X, ..., X]  (§2.5), evaluated algorithm-by-blocks (§5.4, Figure 6)
 * with the partial symmetry of the temporaries exploited (§6, Theorem 1):
 *   T^(m-1) = A x_{m-1} X,  T^(k) = T^(k+1) x_k X,  C = T^(1) x_0 X,
 * forming for each sorted tuple of C-block indices only the output blocks
 * whose leading (symmetric) block indices are sorted.
 *
 * A      : BCSS of layout *A (A->n = n, A->b = bA), device.
 * X      : p x n matrix on the device, entry (j, i) at X[j*rs_x + i*cs_x],
 *          dtype A->dtype.  p = C->n.
 * C      : BCSS of layout *C (C->b = bC, C->m = A->m, dtype F32), device;
 *          fully overwritten (padding entries come out exactly zero).
 * ws     : device workspace of at least sttsm_workspace_bytes(A, C, prec)
 *          bytes, 256-byte aligned.  Its contents on return are the padded X
 *          panels and the temporaries (see sttsm_workspace_temp).
 * Entries of C inside blocks with repeated indices are computed one by one
 * and may differ from their mirrored entries by rounding (§5.4).
 */
int sttsm(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
          const bcss_layout *C, void *C_dev, int32_t prec, void *ws, size_t ws_bytes, void *stream);

/*
 * sttsm for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * operation, arguments, layouts and precision forms as sttsm, and the same
 * kernels (bit-identical results), but no workspace argument: the X panels
 * and temporaries, and the plan's index tables, live in one static device
 * array of STTSM_NOALLOC_SCRATCH_BYTES (96 MiB; m = 3, n = p = 256, b = 16
 * needs 68.5 MiB in the split form, the largest) that every GPU the library
 * runs on holds until the process ends.
 *
 * The call allocates no device memory: the plan is built once per shape in
 * host memory and cached; each call copies its index tables into the array
 * on `stream` (hipMemcpyAsync) and launches the levels there.
 * Errors: STTSM_EINVAL when the problem needs more scratch than the array
 * holds (the message gives both sizes), plus those of sttsm.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * there; a call never reads a byte of it that the call has not written.
 * Calls that overlap in time on one GPU (other streams or host threads)
 * race on the array: order them on one stream.
 */
#define STTSM_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
int sttsm_noalloc(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
                  const bcss_layout *C, void *C_dev, int32_t prec, void *stream);

/*
 * "All modes but one" (the related operation §2.5 names next to sttsm): the
 * tensor A x_1 X x_2 X ... x_{m-1} X, which multiplies every mode but mode 0
 * and is symmetric in modes 1..m-1.  It is the temporary T^(1) of the sttsm
 * chain (the chain stops before the last level), written to T instead of the
 * workspace, in the layout sttsm_workspace_temp describes for k = 1:
 * [J][s][block], J over sorted (m-1)-tuples of C-block indices (colex),
 * s over the nbar A-block indices of mode 0, blocks of bA * bC^(m-1) entries
 * in dimensional order (mode 0 of extent bA fastest).  Its dtype is the
 * temporaries' dtype of `prec` (F32 for FP32 and BF16X3_FIRST_FP32, BF16
 * otherwise).  Arguments as for sttsm; C describes the output modes (its
 * n = p and b = bC); needs m >= 2 (EINVAL otherwise).  The workspace size is
 * sttsm_workspace_bytes(A, C, prec).
 */
int sttsm_all_but_one(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
                      const bcss_layout *C, void *T_dev, int32_t prec, void *ws, size_t ws_bytes, void *stream);
/* Entries of T for sttsm_all_but_one (padded); -1 on bad arguments or m < 2. */
int64_t sttsm_all_but_one_elems(const bcss_layout *A, const bcss_layout *C, int32_t prec);

/*
 * The rank-update form of sttsm (the second algorithmic variant of §8, which
 * the paper states for m = 2: with A split by rows A_i and X by columns X_i,
 * C = X A X^T = sum_i X_i (A_i X^T)).  For order m the product Y = A x_1 X
 * ... x_{m-1} X (the "all modes but one" tensor, symmetric in modes
 * 1..m-1) has block rows Y_i = A_i x_1 X ... x_{m-1} X, and
 * C = sum over the A-block indices i of Y_i x_0 X_{:,i}: a rank-bA update of
 * C per block row.  The block rows are taken `rows` at a time: a pass forms
 * its rows of Y in a buffer that holds one pass, then adds their update to C.
 * Levels above Y run as in sttsm.  Result: the same C as sttsm, with the
 * last contraction's sum split into passes (the first pass stores, each
 * later one adds, in increasing i; the result is the same on every call).
 * With rows >= nbar it is one pass and equals sttsm's result bit for bit when
 * sttsm runs the generic kernels (environment STTSM_GENERIC_KERNELS=1).
 *
 * Arguments as for sttsm, plus rows >= 1 (EINVAL otherwise); needs m >= 2
 * (EINVAL otherwise).  Every level runs on the generic staging kernel.
 * ws    : at least sttsm_rank_update_workspace_bytes(A, C, prec, rows)
 *         bytes, 256-byte aligned: the X panels, the temporaries
 *         T^(m-1) .. T^(2) and one pass of Y (in place of all of T^(1)).
 * Asynchronous on `stream`; C is fully overwritten.
 */
int sttsm_rank_update(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
                      const bcss_layout *C, void *C_dev, int32_t prec, int32_t rows, void *ws, size_t ws_bytes,
                      void *stream);
/* Workspace bytes of sttsm_rank_update; 0 on bad arguments (m < 2, rows < 1). */
size_t sttsm_rank_update_workspace_bytes(const bcss_layout *A, const bcss_layout *C, int32_t prec, int32_t rows);

/*
 * Batched vector products, the case of §2.5 where the matrix of sttsm is a
 * single vector (as in the CP decomposition): for V vectors x_v,
 *   y_v = A x_v^(m-1),  y_v[i] = sum_{i_2..i_m} a_{i i_2..i_m} x_v[i_2]...x_v[i_m],
 *   s_v = A x_v^m = x_v . y_v.
 * A   : BCSS, F32 or BF16, m >= 2, device.
 * x   : V rows of n entries, row v at x + v*rs_x (A's dtype), device.
 * y   : V rows of n fp32 entries, row v at y + v*rs_y, device, overwritten.
 * s   : V fp32 entries, device, or NULL.
 * ws  : device workspace of sttsm_vectors_workspace_bytes(A, V) bytes.
 * Each stored block is read for every distinct block index it holds; the
 * sums run in a fixed order (results are reproducible bit for bit); fp32
 * accumulation.
 */
int sttsm_vectors(const bcss_layout *A, const void *A_dev, const void *x_dev, int64_t V, int64_t rs_x, float *y_dev,
                  int64_t rs_y, float *s_dev, void *ws, size_t ws_bytes, void *stream);
/* Workspace bytes for sttsm_vectors; 0 on bad arguments. */
size_t sttsm_vectors_workspace_bytes(const bcss_layout *A, int64_t V);
/* Multiply-add count x 2 of sttsm_vectors (every term once: per vector,
 * b^m for each stored block and distinct block index in it); -1 on bad
 * arguments. */
int64_t sttsm_vectors_flops(const bcss_layout *A, int64_t V);

/*
 * Where sttsm leaves temporary T^(k) (1 <= k <= m-1) inside the workspace.
 * T^(k) has extent n in modes 0..k-1 (symmetric, Theorem 1) and p in modes
 * k..m-1.  It is stored as [J][s][block]: J runs over sorted tuples
 * (jbar_k <= ... <= jbar_{m-1}) of C-block indices in colex order
 * (*num_jtuples of them), s over sorted tuples (ibar_0 <= ... <= ibar_{k-1})
 * of A-block indices in colex order (*num_prefixes), and each block holds
 * bA^k * bC^(m-k) entries in dimensional order.  *dtype is sttsm_dtype.
 */
int sttsm_workspace_temp(const bcss_layout *A, const bcss_layout *C, int32_t prec, int32_t k,
                         size_t *byte_offset, int32_t *dtype, int64_t *num_jtuples,
                         int64_t *num_prefixes, int64_t *block_elems);

/*
 * Inspection of the plan sttsm runs for these shapes (host only, launches
 * nothing): for loop level `level` (0 forms T^(m-1), m-1 forms C) the number
 * of row groups (sorted C-block tuple of the level x unique output prefix of
 * the symmetric modes, Figure 6 with §6.3), of workgroup tasks, and the flops
 * the level performs (its term of Table 2).  tile (5 entries, may be NULL):
 * the level's kernel (0 generic, 1 FP32 block-copy, 2 bf16 block-copy, 3 bf16
 * block-copy with the X panel resident in LDS, 4 bf16 for m = 2 with 64 x 64
 * blocks, tiles of four row groups), its
 * tile rows and columns, K chunk and prefetch depth.  Any output may be NULL.
 */
int sttsm_plan_info(const bcss_layout *A, const bcss_layout *C, int32_t prec, int32_t level,
                    int64_t *groups, int64_t *tasks, int64_t *flops, int32_t *tile);

/*
 * Per-level timing for measurement tools.  While enabled, sttsm records a
 * pair of HIP events on its stream around each level's kernel launch (up to
 * max_launches launches; later ones are counted as dropped).  The events are
 * created here, not in sttsm.  sttsm_profile_read waits for the recorded
 * events, writes the summed milliseconds and launch count per level
 * (level_ms[d], level_launches[d], d < max_levels) and starts a new
 * recording.  Not meant for concurrent sttsm calls from several threads.
 */
int sttsm_profile_enable(int32_t max_launches);
int sttsm_profile_read(double *level_ms, int64_t *level_launches, int32_t max_levels, int64_t *dropped);
int sttsm_profile_disable(void);

/* ------------------------------------------------------------------ serving
 *
 * A server runs a continuous-batching loop over sttsm requests of mixed
 * order and size.  Each request's state (its BCSS A, X, C, temporaries and
 * index tables) lives in a caller-provided device arena whose size is the
 * HBM budget; a request is admitted (first come, first served) once its
 * footprint fits in the free arena and fewer than max_inflight requests
 * are active.  Work proceeds in rounds: one round stages the inputs of newly
 * admitted requests and then runs the next level (T^(m-1), ..., C) of every
 * active request in grouped persistent launches, where all workgroups draw
 * tiles of all requests from one shared task queue (the algorithm-by-blocks
 * unit of work, scheduled across requests as the paper's future-work
 * section suggests for block scheduling).  Requests that arrive while a
 * round runs join at the next round, so their work overlaps with that of
 * requests already on the GPU.  Each tile is computed whole (no split
 * reductions), so a request's C is bit-identical alone and in any mix.
 * A server owns one worker thread and one HIP stream of default priority.
 */
typedef struct sttsm_server sttsm_server;

typedef struct {
    bcss_layout A;        /* order, n, bA, dtype of A (C has the same order) */
    bcss_layout C;        /* p = C.n, bC = C.b, dtype F32                     */
    const void *A_bcss;   /* A in BCSS; must stay valid until admitted         */
    const void *X;        /* p x n, dtype A.dtype; (j, i) at X[j*rs_x+i*cs_x]  */
    int64_t rs_x, cs_x;
    int32_t prec;         /* sttsm_prec                                        */
    int32_t src_is_host;  /* 1: A_bcss and X are host pointers, else device    */
} sttsm_request;

enum { STTSM_QUEUED = 0, STTSM_ADMITTED = 1, STTSM_RUNNING = 2, STTSM_DONE = 3, STTSM_FAILED = 4 };

/* arena: device memory of arena_bytes (256-byte aligned) owned by the caller
 * and used by the server until sttsm_server_destroy returns.  EINVAL for a
 * null arena, zero size or max_inflight < 1. */
int sttsm_server_create(void *arena, size_t arena_bytes, int32_t max_inflight, sttsm_server **out);

/* Bytes of arena a request occupies while active (its C stays until fetched). */
size_t sttsm_request_footprint(const sttsm_request *req);

/* Queues a request; never waits for the GPU.  EINVAL for a bad request,
 * ENOMEM when its footprint exceeds the whole arena (it could never run).
 * The server copies A_bcss and X on its own stream some time after the call
 * returns and does not wait for work the caller queued elsewhere: their
 * values must be final (the producing stream synchronised) before the call,
 * and they must stay valid until the request is fetched. */
int sttsm_submit(sttsm_server *s, const sttsm_request *req, uint64_t *ticket);

/* *state <- STTSM_QUEUED .. STTSM_FAILED; ENOTFOUND for an unknown ticket. */
int sttsm_poll(sttsm_server *s, uint64_t ticket, int32_t *state);

/* Waits up to timeout_us (< 0: no limit) for the request to finish;
 * EAGAIN on time-out, ENOTFOUND for an unknown ticket. */
int sttsm_wait(sttsm_server *s, uint64_t ticket, int64_t timeout_us, int32_t *state);

/* Copies a finished request's C (bcss_num_elems(C) floats) to C_dst and
 * forgets the ticket; returns once the copy is complete (it runs on a
 * stream of the server's own, without waiting for queued rounds), and only
 * then gives C's arena region back.  EAGAIN if not finished, ENOTFOUND if
 * unknown or already fetched, EHIP if the request failed (the ticket is
 * forgotten). */
int sttsm_fetch(sttsm_server *s, uint64_t ticket, void *C_dst, int32_t dst_is_host);

/* Latency (submit -> done) percentiles and throughput of the requests
 * completed so far; zeros when none.  Also the number of rounds run and of
 * grouped launches made. */
int sttsm_server_stats(sttsm_server *s, double *p50_us, double *p99_us, double *req_per_s,
                       int64_t *completed, int64_t *rounds, int64_t *launches);

/* Stops the loop after the running round; unfinished requests fail.
 * Joins the worker and releases everything the server allocated. */
int sttsm_server_destroy(sttsm_server *s);

/* Message for the last failed call on this thread ("" if none). */
const char *sttsm_last_error(void);

/* Library version string. */
const char *sttsm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STTSM_H */
