/*
 * exsum.h -- C ABI of libexsum: multidimensional included and excluded sums
 * on AMD Instinct MI355X (gfx950).
 *
 * Paper: H. Xu, S. Fraser, C. E. Leiserson, "Multidimensional Included and
 * Excluded Sums", SIAM ACDA 2021 (arXiv 2106.00124).
 *
 * Problem (Sec. 2, Definition "Included and Excluded Sums"): given a
 * d-dimensional tensor A over a monoid (S, op, e) and a box size k, produce
 * for every coordinate x
 *     included sum  Inc(x) = op over A[x_0 : x_0+k_0, ..., x_{d-1} : x_{d-1}+k_{d-1}]
 *     excluded sum  Exc(x) = op over every element of A outside that box
 * (coordinates past the end of the tensor contribute e; Sec. 1 and the colon
 * notation of Sec. 2).  Both are the "strong" problems: no inverse of op is
 * used, so max and min work as well as +.  Included sums follow the bidirectional
 * box-sum (BDBS) algorithm (Sec. 3); excluded sums follow the box-complement
 * algorithm (Secs. 4-5: Theorem "Recursive Box-complement", Corollary
 * "Excluded-sum Components").
 *
 * Conventions shared by every call:
 *   - Coordinates are 0-based.  Tensors are dense and row-major (C order):
 *     dims[0] is the paper's dimension 1 (largest stride) and dims[d-1] is
 *     contiguous.  Outputs have the input's shape and element type (Sec. 2:
 *     the output is a tensor over the same monoid).
 *   - Element types and operators: + on f32, f64, i32, i64 (integer + wraps
 *     modulo 2^32 / 2^64, so it is associative and commutative); max and min
 *     on all four (the problem is stated over any commutative monoid, Sec. 2).
 *     Identity e: 0 for +, -inf / +inf for float max / min, the type's
 *     minimum / maximum for integer max / min (the value of an excluded sum
 *     whose complement is empty).
 *   - Preconditions: 1 <= d <= EXS_MAX_RANK; dims[i] >= 1; 1 <= box[i] <= dims[i]
 *     (Sec. 1 requires k_i <= n_i); the product of dims fits in int64.
 *   - Pointers named *_dev are device pointers (hipMalloc / PyTorch CUDA
 *     tensors); the caller owns every buffer.  The library never allocates or
 *     frees caller memory; plain calls take their scratch as a workspace
 *     argument.
 *   - Streams are passed as void* and must be a hipStream_t (NULL = the null
 *     stream).  Calls enqueue work and return without synchronising; results
 *     are valid once the stream has completed.
 *   - Every call returns an exs_status; nothing throws or exits across the
 *     ABI.  exs_last_error() returns a thread-local message for the last
 *     failing call on the calling thread.
 */
#ifndef EXSUM_H
#define EXSUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXS_MAX_RANK 8

typedef enum {
    EXS_OK = 0,
    EXS_EINVAL = 1,        /* bad argument (shape, box, null pointer, aliasing) */
    EXS_EUNSUPPORTED = 2,  /* valid request this build does not implement */
    EXS_ENOMEM = 3,        /* workspace too small, or a host allocation failed */
    EXS_EDEVICE = 4,       /* a HIP call failed (message in exs_last_error) */
    EXS_EAGAIN = 5,        /* resource temporarily unavailable */
    EXS_ENOTREADY = 6,     /* asynchronous result not complete yet */
    EXS_ENOTFOUND = 7      /* unknown ticket / handle */
} exs_status;

/* EXS_VALIDX: a struct element of 8 bytes, { float value; int32_t index; }
 * (value first, 8-byte aligned), under the operators EXS_MAX ("argmax": the
 * largest value, and among equal values the lowest index) and EXS_MIN
 * ("argmin": the smallest value, the lowest index among equal values).  Both
 * are max / min of a total order, hence commutative monoids (Sec. 2 states
 * the problem over a monoid); identity (-inf, INT32_MAX) for EXS_MAX and
 * (+inf, INT32_MAX) for EXS_MIN.  The index field is whatever the caller
 * stores (typically the flat position); it only breaks ties.  EXS_SUM and
 * EXS_WEAK return EXS_EUNSUPPORTED; the batched form does not take it. */
typedef enum { EXS_F32 = 0, EXS_F64 = 1, EXS_I32 = 2, EXS_I64 = 3, EXS_VALIDX = 4 } exs_dtype;
typedef enum { EXS_SUM = 0, EXS_MAX = 1, EXS_MIN = 2 } exs_op;

/* mode bit-mask */
#define EXS_INCLUDED 1u
#define EXS_EXCLUDED 2u
/* With EXS_EXCLUDED and op EXS_SUM only: compute the excluded sums as the
 * "weak" excluded sums total - included (the BDBSC route that Sec. 1 of the
 * paper contrasts with the strong, inverse-free box-complement; its Sec. 6
 * measures both).  Exact for the integer types (wrapping); for floating point
 * the total is accumulated in FP64 and the subtraction is done in the element
 * type, so cells whose excluded sum nearly cancels lose relative accuracy.
 * With op EXS_MAX or EXS_MIN: EXS_EUNSUPPORTED (no inverse).  Not accepted by
 * exs_batch_create (EXS_EUNSUPPORTED). */
#define EXS_WEAK 4u

/* One included/excluded-sums problem on one tensor.
 *   d            rank, 1..EXS_MAX_RANK
 *   dtype, op    element type and operator (see above)
 *   mode         EXS_INCLUDED, EXS_EXCLUDED or both, optionally | EXS_WEAK
 *   dims[0..d)   tensor side lengths n_i
 *   box[0..d)    box side lengths k_i
 *   in_dev       input tensor, prod(dims) elements
 *   inc_out_dev  included sums (same shape), required iff mode has EXS_INCLUDED
 *   exc_out_dev  excluded sums (same shape), required iff mode has EXS_EXCLUDED
 * Outputs must not overlap the input or each other. */
typedef struct exs_job {
    int32_t d;
    int32_t dtype;
    int32_t op;
    uint32_t mode;
    int64_t dims[EXS_MAX_RANK];
    int64_t box[EXS_MAX_RANK];
    const void *in_dev;
    void *inc_out_dev;
    void *exc_out_dev;
} exs_job;

/* ---------------------------------------------------------------------- */
/* Plain single-tensor call                                                 */
/* ---------------------------------------------------------------------- */

/* Bytes of device workspace exs_run needs for this job (0 is possible).
 * Validates the job's shape/box/dtype/op/mode; pointers are not inspected. */
exs_status exs_workspace_size(const exs_job *job, size_t *bytes);

/* Included and/or excluded sums of job->in_dev (Secs. 3-5).  ws_dev must be
 * at least exs_workspace_size() bytes of device memory, 256-byte aligned,
 * owned by the caller and not used by other work until the stream reaches
 * this call's end.  Enqueued on `stream`; no host synchronisation. */
exs_status exs_run(const exs_job *job, void *ws_dev, size_t ws_bytes, void *stream);

/* Allocation-free variant of exs_run, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same computation and kernels as
 * exs_run, with the workspace taken from a static device array of
 * EXS_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends.  The caller passes only the job (inputs and
 * outputs, as for exs_run) and the stream.  Makes no hipMalloc, hipFree or
 * other allocating call (per-kernel timing is not recorded for it); the first
 * call on a device looks up that device's array.  A job whose
 * exs_workspace_size exceeds EXS_NOALLOC_SCRATCH_BYTES returns EXS_ENOMEM
 * before anything is enqueued.  Every call on one GPU uses that GPU's one
 * array: calls whose work overlaps on the device (on different streams, or
 * from different threads without ordering) race and corrupt each other;
 * calls ordered on one stream are safe.  No workspace contents carry over
 * from one call to the next. */
#define EXS_NOALLOC_SCRATCH_BYTES (64ll << 20)
exs_status exs_run_noalloc(const exs_job *job, void *stream);

/* Human-readable name of a status, and the calling thread's last error. */
const char *exs_status_str(exs_status s);
const char *exs_last_error(void);

/* Library version string and the device architecture it was built for. */
const char *exs_version(void);

/* Per-kernel timing (measurement support).  While enabled, every kernel the
 * library enqueues is bracketed by a pair of HIP events recorded on the
 * stream it is launched on.  exs_timing_read synchronises those events and
 * returns, per kernel name, the number of launches and their summed duration
 * in milliseconds (at most `max` entries, names NUL-terminated in 64-byte
 * slots of `names`), then clears the record.  Host-side bookkeeping only;
 * not thread-safe against concurrent exs_run calls. */
exs_status exs_timing_enable(int32_t on);
exs_status exs_timing_read(int32_t max, char *names, int64_t *launches, double *total_ms,
                           int32_t *count);

/* An artificially expensive operator (measurement support, after the
 * experiment of Sec. 6, "Excluded Sums With Different Operators", which slows
 * its operator down with a recursive Fibonacci computation of tunable size to
 * see how the algorithms scale with the cost of op).  While cost > 0, f32 +
 * in exs_run and exs_run_noalloc (strong included/excluded sums; not EXS_WEAK)
 * runs through an operator that performs `cost` dependent 32-bit integer
 * multiply-add steps in every application before returning a + b: results
 * are unchanged, only slower.  cost = 0 restores the plain operator.
 * Process-wide; set it only while no other call of the library runs.
 * EXS_EINVAL for cost outside 0..2^20, EXS_EDEVICE if the device constant
 * cannot be written. */
exs_status exs_set_op_cost(int32_t cost);
/* Apply that operator `reps` times to each of the n f32 elements at data_dev
 * (data[i] <- data[i] + ... + data[i], reps terms, one thread per element),
 * enqueued on `stream`: the time of one application per element at the
 * parallelism of the library's kernels, to divide the time per element by. */
exs_status exs_op_probe(void *data_dev, int64_t n, int32_t reps, void *stream);

/* ---------------------------------------------------------------------- */
/* Corners algorithm: the paper's comparison system for strong excluded sums */
/* ---------------------------------------------------------------------- */

/* Strong excluded sums of a 2-D tensor by the corners algorithm (Sec. 1,
 * "Corners Algorithm for Strong Excluded Sums"; App. A, "Analysis of Corners
 * Algorithm"), kept beside exs_run to compare the two methods on the same
 * device.  The complement of each box is cut into four disjoint regions,
 * each holding one corner of the box and reaching the tensor's edges; each
 * region's reduction is one entry of a full-tensor table (prefix or suffix
 * along axis 0 of a prefix or suffix along axis 1), so no inverse is needed.
 * Results equal exs_run's excluded output: bit-exact for integer + (wrapping),
 * max and min; for f32/f64 + the same sums in another order.
 *
 * The job is as for exs_run with d == 2, mode == EXS_EXCLUDED, dtype EXS_F32,
 * EXS_F64, EXS_I32 or EXS_I64 and any op; in_dev and exc_out_dev are
 * C-contiguous n0 x n1 device tensors (caller-owned; exc_out_dev must not
 * overlap in_dev).  The workspace (exs_corners_workspace_size: four n0 x n1
 * tables plus six ceil(n0/64) x n1 arrays, 256-byte aligned, caller-owned)
 * must not overlap either tensor.  Enqueued on `stream` without host
 * synchronisation.  Errors: EXS_EINVAL for a malformed job or workspace,
 * EXS_EUNSUPPORTED for d != 2 or (value, index) pairs, EXS_ENOMEM for a
 * workspace smaller than needed, EXS_EDEVICE if a launch fails. */
exs_status exs_corners_workspace_size(const exs_job *job, size_t *bytes);
exs_status exs_run_corners(const exs_job *job, void *ws_dev, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* Input generation on the device (workload support, not part of the method) */
/* ---------------------------------------------------------------------- */

/* Fill `count` elements at out_dev with the counter-based generator: element
 * i is derived from output i of a SplitMix64 stream started at `seed`
 * (Steele, Lea, Flood 2014).  kind 0: f32 "normalish" (sum of four 16-bit
 * uniforms, centred and scaled to unit variance); kind 1: uniform integer in
 * [lo, hi] for EXS_I32 / EXS_I64; kind 2: f32 with random sign and magnitude
 * 2^e * (1 + m/2^23), e uniform in [-10, 9].  Bit-identical to the host twin
 * in paper_2106_00124_amd/workloads.py. */
exs_status exs_fill(void *out_dev, int64_t count, int32_t dtype, int32_t kind,
                    uint64_t seed, int64_t lo, int64_t hi, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched form: many tensors of uneven shapes, ranks, boxes, dtypes and    */
/* operators computed by one hipGraph launch of persistent work-list kernels */
/* ---------------------------------------------------------------------- */

typedef struct exs_batch exs_batch;

/* Plan a batch of n jobs (copied; the job pointers are bound at create time
 * and must stay valid for every launch).  tune_cache: path of the JSON
 * autotune cache to read and update, or NULL for built-in tile choices; a
 * file at that path that does not parse as such a cache is ignored and left
 * as it is (the batch is then tuned and the result not stored).
 * The call may time candidate tile shapes on the device (autotuning), which
 * synchronises the device and writes the outputs of the jobs. */
exs_status exs_batch_create(const exs_job *jobs, int32_t n, const char *tune_cache,
                            exs_batch **out);
/* Device workspace the batch needs. */
exs_status exs_batch_workspace_size(const exs_batch *b, size_t *bytes);
/* Enqueue the whole batch on `stream` as one graph launch (the graph is
 * captured on the first call for this workspace and replayed afterwards). */
exs_status exs_batch_launch(exs_batch *b, void *ws_dev, size_t ws_bytes, void *stream);
/* The same work as individual kernel launches (no graph), for comparison. */
exs_status exs_batch_launch_eager(exs_batch *b, void *ws_dev, size_t ws_bytes, void *stream);
/* Number of kernel nodes in the captured graph and work items in the lists. */
exs_status exs_batch_info(const exs_batch *b, int32_t *graph_nodes, int64_t *work_items);
void exs_batch_destroy(exs_batch *b);

/* ---------------------------------------------------------------------- */
/* Serving form: continuous batching of excluded-sum requests               */
/* ---------------------------------------------------------------------- */

typedef struct exs_server exs_server;

/* A server owns a device arena of hbm_budget bytes (allocated here, freed by
 * destroy) from which it carves each request's output and workspace, and up
 * to max_inflight HIP streams.  A dispatcher thread admits requests in
 * arrival order while their bytes fit the free budget and a stream slot is
 * free; admitted work overlaps on the device. */
exs_status exs_server_create(size_t hbm_budget, int32_t max_inflight, exs_server **out);
/* Queue a request.  job->in_dev (caller-owned) must stay valid and
 * unchanged until the ticket completes; job->mode selects outputs; output
 * pointers in the job are ignored (the server allocates them in its arena).
 * `stream` (a hipStream_t, NULL = the null stream) is the stream on which the
 * caller wrote job->in_dev: an event is recorded on it here and the request's
 * work waits for that event, so the input may still be in production when
 * submit is called.  Never blocks; fails only for an invalid job (EXS_EINVAL),
 * one larger than the whole budget (EXS_ENOMEM) or a failed event record
 * (EXS_EDEVICE).  A request that does not fit the free arena waits in the
 * queue, and so do the requests behind it.  The work computes what exs_run
 * computes for the same job. */
exs_status exs_server_submit(exs_server *s, const exs_job *job, void *stream, uint64_t *ticket);
/* The same, but the server builds the input tensor itself inside its arena
 * (exs_fill with fill_kind/seed/lo/hi, enqueued on the request's stream just
 * before its work), so request tensors are produced and kept on the device.
 * job->in_dev is ignored; fill kind 1 needs an integer dtype, kinds 0 and 2
 * need EXS_F32 (EXS_EINVAL otherwise). */
exs_status exs_server_submit_generated(exs_server *s, const exs_job *job, int32_t fill_kind,
                                       uint64_t seed, int64_t lo, int64_t hi, uint64_t *ticket);
/* EXS_OK and the device pointers of the outputs (row-major, the job's dims
 * and dtype; NULL for an output not requested) once the request completed,
 * EXS_ENOTREADY before, EXS_EDEVICE if its launch failed, EXS_ENOTFOUND for
 * an unknown or released ticket.  Pointers stay valid until release. */
exs_status exs_server_poll(exs_server *s, uint64_t ticket, const void **inc_dev,
                           const void **exc_dev, double *latency_ms);
/* Device pointer of a completed request's input (its generated tensor for
 * exs_server_submit_generated); valid until release. */
exs_status exs_server_input(exs_server *s, uint64_t ticket, const void **in_dev);
/* Block until every submitted request has completed.  EXS_EAGAIN when no
 * request runs and the queue head cannot fit because completed requests
 * still hold the arena (release them, then drain again). */
exs_status exs_server_drain(exs_server *s);
/* Forget a completed (or failed) request's ticket and return its memory to
 * the arena once `stream` (a hipStream_t, NULL = the null stream) has reached
 * this call: work the caller enqueued there that reads the outputs (a copy,
 * say) finishes before another request can reuse the range.  An event is
 * recorded on `stream`; the range is free again when it completes.
 * EXS_ENOTREADY while the request is queued or running. */
exs_status exs_server_release(exs_server *s, uint64_t ticket, void *stream);
/* Latency percentiles (submit -> completion event) and throughput over the
 * completed requests so far; queue depth and peak in-flight bytes. */
exs_status exs_server_stats(exs_server *s, double *p50_ms, double *p99_ms,
                            double *req_per_s, double *gelem_per_s,
                            int64_t *completed, int64_t *max_queue,
                            int64_t *peak_bytes);
void exs_server_destroy(exs_server *s);

#ifdef __cplusplus
}
#endif

#endif /* EXSUM_H */
