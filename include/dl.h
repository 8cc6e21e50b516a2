/*
 * dl.h -- C ABI of the MI355X (gfx950) library for linear-algebraic Datalog
 * evaluation (T. Sato, "A Linear Algebraic Approach to Datalog Evaluation").
 *
 * The library computes least Herbrand models of linear, binary-predicate
 * Datalog programs as fixpoints of thresholded dense N x N matrix products:
 *   - transitive closure   R = min1(R1 + R1 R)           (Sec. 3, program DB1)
 *     and its repeated-squaring form R = min1(R1 + R R)  (Sec. 8)
 *   - same generation      S = min1(I + R1 S R1^T)       (Sec. 7.2)
 *   - the purely linear form of Sec. 4, Proposition 1:
 *     X = (I - eps R1)^-1 eps R1, thresholded at > 0      (Theorem 1)
 *   - the epsilon forms of Sec. 6: tail-recursive X = eps (C + B X) and
 *     two-sided X = eps (Q + B X C) equations, the same-generation one
 *   - whole programs, layered by strongly connected components (Sec. 5),
 *     with stratified negation (Sec. 8)
 * around them: several closures per call (dl_tc_batch), continuous batching
 * of many small requests (dl_batch_*), and tile autotuners for the product
 * step (dl_tune*) and for the grouped serving step (dl_batch_tune).
 *
 * Matrix conventions (all entry points):
 *   - Every matrix is n x n, row-major, 0-based: element (i, j) at p[i*ld + j],
 *     ld >= n.  (R)_ij = 1 iff r(e_i, e_j) holds: row = first argument
 *     (adjacency encoding, Sec. 2).
 *   - Relation inputs are uint8 bytes; 0 is false and any nonzero byte is
 *     true.  Model outputs are exactly 0 or 1.
 *   - All matrix pointers are DEVICE pointers owned by the caller.  The
 *     library never frees or retains them past the call.  Inputs are read
 *     only; an output must not overlap an input.
 *   - min1(x) = 1 if x >= 1 else x (Sec. 2).  On the non-negative integer
 *     counts these products produce it is the test x != 0.
 *   - `iters` (host pointer) receives the number of applications of the
 *     update starting from the empty relation R^(0) = 0, including the first
 *     application that changes nothing.  For the plain series this is D + 1,
 *     D the longest shortest path; for repeated squaring 2 + ceil(log2 D)
 *     (1 when R1 is empty).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it; calls that report `iters` block until it is known.
 *
 * Errors: every call returns a dl_status.  DL_EINVAL for bad arguments
 * (n < 0, NULL pointer with n > 0, ld < n, overlapping input/output, eps out
 * of range, unknown enum); DL_ENOMEM when the workspace needed exceeds the
 * context's budget or hipMalloc fails; DL_EHIP for a HIP runtime error;
 * DL_ENOCONV if the step cap is hit (impossible for valid inputs);
 * DL_EUNSUPPORTED for a method/precision pair that is not built.  After an
 * error, dl_last_error() returns a message for the calling thread.  No C++
 * exception crosses this interface.  n == 0 is valid and returns at once
 * with iters = 1 (the empty model).
 *
 * Threading: a context may be used by one thread at a time; use one
 * context per thread (or per stream) for concurrency.  A program uses its
 * context's scratch, so calls on the program count as calls on the context.
 */
#ifndef DL_H_
#define DL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DL_OK = 0,
  DL_EINVAL = 1,
  DL_ENOMEM = 2,
  DL_EHIP = 3,
  DL_ENOCONV = 4,
  DL_EUNSUPPORTED = 5,
  DL_EAGAIN = 6 /* batch: no free request slot or pool memory; fetch finished requests and retry */
} dl_status;

/* How the closure fixpoint is iterated. */
typedef enum {
  DL_TC_PLAIN = 0,  /* R^(k+1) = min1(R1 + R1 R^(k))         (Sec. 3, "Iteration", Sec. 7.1) */
  DL_TC_SQUARE = 1  /* R^(k+1) = min1(R1 + R^(k) R^(k))      (non-linear program, Sec. 8)    */
} dl_tc_method;

/* Arithmetic of the products.  Operands are exactly 0/1 in every format, so
 * all are exact: int8 with int32 accumulation, and fp32/bf16/fp8(e4m3)/
 * fp4(e2m1, two elements per byte) with fp32 accumulation while counts stay
 * below 2^24 (n <= 65536 keeps every count below that). */
typedef enum { DL_I8 = 0, DL_F32 = 1, DL_BF16 = 2, DL_FP8 = 3, DL_FP4 = 4 } dl_prec;

typedef struct dl_ctx dl_ctx;

/* Create a context on HIP device `device`.  workspace_budget_bytes caps the
 * device memory the context may allocate for its internal buffers (0 = no
 * cap).  Workspace is allocated lazily by the first call that needs it and
 * reused by later calls. */
int dl_create(dl_ctx** ctx, int device, size_t workspace_budget_bytes);
int dl_destroy(dl_ctx* ctx);

/* Transitive closure of R1 = A (Sec. 3, Theorem 1 gives the same model).
 *   n      number of constants
 *   A      device uint8 [n x lda], nonzero = r1(e_i, e_j)
 *   R      device uint8 [n x ldr], receives the 0/1 least model of r2 (it
 *          may also hold intermediate iterates while the call runs)
 *   method dl_tc_method, prec dl_prec
 *   iters  host int32, see above. */
int dl_tc(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr,
          int method, int prec, int32_t* iters, void* stream);

/* As dl_tc, but stops after at most max_steps applications (max_steps >= 0)
 * and reports the per-step model sizes.  R receives the last iterate
 * computed, R^(min(max_steps, iters)).  ones (host int64, length
 * max_steps + 1, or NULL) receives ones[k] = number of true entries of
 * R^(k) for k = 0 .. *steps.  *steps = number of iterates computed;
 * *converged = 1 if the fixpoint was confirmed within max_steps. */
int dl_tc_steps(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr,
                int method, int prec, int32_t max_steps, int64_t* ones, int32_t* steps,
                int32_t* converged, void* stream);

/* Transitive closure of `count` relations of one size (Sec. 3, as dl_tc):
 * A[g] and R[g] (g < count) are device uint8 matrices [n x lda] and
 * [n x ldr], passed as host arrays of `count` device pointers; iters[g]
 * (host int32) receives each fixpoint's iteration count.  The fixpoints run
 * two at a time on `stream`, so the host's counter read-back of one overlaps
 * the products of the other; the device workspace is twice that of dl_tc
 * (one at a time if the budget allows only one).  Results are identical to
 * `count` dl_tc calls.  No R[g] may overlap any A[h] or another R[h]
 * (DL_EINVAL); count = 0 does nothing. */
int dl_tc_batch(dl_ctx* ctx, int32_t count, int64_t n, const uint8_t* const* A, int64_t lda,
                uint8_t* const* R, int64_t ldr, int method, int prec, int32_t* iters, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dl_tc with
 * method DL_TC_PLAIN for n <= 512 constants, any dl_prec, run by the same
 * one-launch kernel (tile configuration 5), with every device buffer it
 * needs (two iterates, counters, read-back words: 2.2 MB at most) in a
 * static device array that each GPU holds from the first call on it until
 * the process ends.  Allocates nothing and takes no context.  The current device is the
 * one used.  Calls on one GPU share that array: calls that overlap on one
 * GPU (other threads, other streams) race and must not be made.  Arguments
 * and results as dl_tc; n above the limit is DL_EINVAL; blocks until iters
 * is known. */
int dl_tc_noalloc(int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr, int prec,
                  int32_t* iters, void* stream);

/* Same generation (Sec. 7.2): least S with S = min1(I + P S P^T), where P is
 * the r1 relation (device uint8 [n x ldp]) and I encodes diag(x, x) for
 * every constant.  Each step runs two products, T = min1(P S) and
 * S' = min1(I + T P^T); thresholding the intermediate keeps the zero
 * pattern of P S P^T.  prec: any dl_prec.  S' is symmetric: with int8 on the
 * large tiles (n rounded up to 256 at least 4096 by the size rule, or tile
 * configuration 0) only its upper-triangle tiles are computed and then
 * mirrored, and the context's workspace also holds that product's partial
 * tiles (27 MB at n = 4096). */
int dl_sg(dl_ctx* ctx, int64_t n, const uint8_t* P, int64_t ldp, uint8_t* S, int64_t lds,
          int prec, int32_t* iters, void* stream);

/* Step-capped variant of dl_sg; arguments as in dl_tc_steps. */
int dl_sg_steps(dl_ctx* ctx, int64_t n, const uint8_t* P, int64_t ldp, uint8_t* S, int64_t lds,
                int prec, int32_t max_steps, int64_t* ones, int32_t* steps, int32_t* converged,
                void* stream);

/* Linear epsilon form (Sec. 4, Proposition 1 and Theorem 1): solves
 * (I - eps A) X = eps A in fp64 by block Gauss-Jordan elimination without
 * pivoting (diagonal panels inverted, the rows and the trailing matrix
 * updated by fp64 matrix products), then writes R = [X > 0].  Without
 * pivoting, every update adds terms of one sign, so R is exact up to fp64
 * underflow.  Device workspace: (n rounded up to 128)^2 * 16 bytes plus
 * 512 x (2 n) doubles of panel scratch.
 *   eps  must satisfy 0 < eps <= 1 / (1 + ||A||_inf), ||A||_inf = max row
 *        sum of the 0/1 matrix (Lemma 1); otherwise DL_EINVAL.
 *   X    optional device double [n x ldx] receiving the real solution
 *        (NULL to skip).
 *   iters is set to 0: the solve is direct, no fixpoint iteration.
 *   underflow (host int32, may be NULL) receives 1 when an entry of R may
 *        be a false negative from fp64 underflow, else 0.  A true entry is
 *        at least eps^L for a shortest path of length L (footnote to
 *        Lemma 2), and along that path the entries of X shrink by at most a
 *        factor eps per edge, so a true entry below the smallest normal
 *        double (DBL_MIN) implies one in [DBL_MIN, DBL_MIN / eps), computed
 *        accurately.  The flag is set when the smallest positive entry of X
 *        is below 2 DBL_MIN / eps; 0 guarantees R is the least model.  The
 *        flag is set for some inputs whose R is still exact (it is
 *        conservative), never missed for one whose R is not. */
int dl_solve_eps(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, double eps, uint8_t* R,
                 int64_t ldr, double* X, int64_t ldx, int32_t* iters, int32_t* underflow, void* stream);

/* Same-generation epsilon form (Sec. 7.2): solves X = eps (I + P X P^T), a
 * discrete Sylvester (Stein) equation (Sec. 6.3), in fp64 by Smith's
 * doubling (X += A X A^T, A = A A, from X = eps I and A = sqrt(eps) P) until
 * a doubling adds no positive entry (and, when X is requested, changes no
 * fp64 value), then writes S = [X > 0], the same-generation model
 * (Theorem 2).
 *   eps  must satisfy 0 < eps <= 1 / (1 + ||P||_inf^2), the bound the paper
 *        derives from ||P kron P||_inf (Sec. 6.3, Sec. 7.2); else DL_EINVAL.
 *   X    optional device double [n x ldx] for the real solution (NULL to skip).
 *   doublings  host int32: number of doublings run (the last one confirms).
 * Device workspace: 5 (n rounded up to 128)^2 * 8 bytes. */
int dl_sg_eps(dl_ctx* ctx, int64_t n, const uint8_t* P, int64_t ldp, double eps, uint8_t* S, int64_t lds,
              double* X, int64_t ldx, int32_t* doublings, void* stream);

/* Tail-recursive equation X = eps (C + B X) (Sec. 6.1, the equation of the
 * tail recursive class with the lower-layer part already summed into C):
 * solves (I - eps B) X = eps C in fp64 by the same block elimination as
 * dl_solve_eps and writes R = [X > 0].  B = C = A is dl_solve_eps.
 *   B, C  device uint8 [n x ldb], [n x ldc], nonzero = true.
 *   eps   0 < eps <= 1 / (1 + ||B||_inf) (the theorem on layered evaluation
 *         asks eps (C + B 1) <= 1 entrywise); else DL_EINVAL.
 *   X     optional device double [n x ldx] (NULL to skip).
 * Device workspace as dl_solve_eps. */
int dl_solve_linear(dl_ctx* ctx, int64_t n, const uint8_t* B, int64_t ldb, const uint8_t* C, int64_t ldc,
                    double eps, uint8_t* R, int64_t ldr, double* X, int64_t ldx, void* stream);

/* Two-sided equation X = eps (Q + B X C) (Sec. 6.3, a discrete Sylvester /
 * Stein equation; the transposed class of Sec. 6.2 reduces to it), solved in
 * fp64 by Smith's doubling: X_0 = eps Q, B_0 = sqrt(eps) B, C_0 = sqrt(eps) C,
 * X += B X C, B = B B, C = C C, until a doubling adds no positive entry (and,
 * when X is requested, changes no fp64 value); writes R = [X > 0].  Every
 * term is non-negative, so the zero pattern is exact up to fp64 underflow.
 *   eps  0 < eps <= 1 / (1 + ||C||_1 ||B||_inf), the bound the paper derives
 *        from ||C^T kron B||_inf (Sec. 6.3); else DL_EINVAL.
 *   X    optional device double [n x ldx] (NULL to skip).
 *   doublings  host int32: doublings run (the last one confirms).
 * Device workspace: 6 (n rounded up to 128)^2 * 8 bytes. */
int dl_solve_two_sided(dl_ctx* ctx, int64_t n, const uint8_t* Q, int64_t ldq, const uint8_t* B, int64_t ldb,
                       const uint8_t* C, int64_t ldc, double eps, uint8_t* R, int64_t ldr, double* X, int64_t ldx,
                       int32_t* doublings, void* stream);

/* Largest eps that Lemma 1 allows for A: 1 / (1 + max row sum).  Computed on
 * the device; host double out. */
int dl_eps_bound(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, double* eps_max,
                 void* stream);

/* Kernel timing.  When enabled, the library brackets launches of its
 * product kernels with HIP events on the call's stream and accumulates, per
 * kernel class, the number of timed launches that did work and their total
 * duration.  The fixpoint calls (dl_tc, dl_tc_batch, dl_sg) time the first
 * product of each chunk of steps they enqueue, so that the other launches
 * run back to back (an event pair between two launches adds about 10 us);
 * layered programs time every product.  Classes: 0 = boolean product step
 * (all precisions), 1 = fp64 trailing update of the epsilon solve, 2 = all
 * other kernels. */
int dl_set_timing(dl_ctx* ctx, int enable);
int dl_kernel_stats(dl_ctx* ctx, int kernel_class, int64_t* launches, double* total_ms,
                    int reset);

/* Measured matrix-core peak of this device: every compute unit runs chains of
 * independent MFMAs on register operands for a few milliseconds; *ops_per_s
 * receives the rate in operations per second (2 M N K per instruction).
 * kind: 0 int8 (32x32x32, the faster int8 shape), 1 fp32 16x16x4, 2 bf16
 * 16x16x32, 3 fp8 e4m3 and 4 fp4 e2m1 16x16x128, 5 fp64 16x16x4.  A reference for the kernels' rates
 * beside the datasheet figures.  Two data-path kinds report bytes per second
 * instead: 6 LDS reads (ds_read_b128, 1 KB per wave and instruction, no bank
 * conflicts, 16 waves per compute unit), 7 global-to-LDS fills
 * (global_load_lds_dwordx4 from a 1 MB L2-resident buffer, eight
 * instructions in flight per wave; uses 1 MB of the context's workspace).
 * Kind 8 is kind 5 with the accumulators in AGPRs instead of architectural
 * VGPRs (the library's fp64 kernels use VGPRs: on gfx950 the AGPR form runs
 * the fp64 MFMA at about 60% of the VGPR form's rate). */
int dl_measure_peak(dl_ctx* ctx, int kind, double* ops_per_s, void* stream);

/* Tile autotuner for the product step shared by every fixpoint (Sec. 3's
 * thresholded products).  Tile configurations:
 *   0  256 x 256 tile, 16 waves of 64 x 64, operands loaded straight to LDS
 *   1  128 x 128 tile, 4 waves of 64 x 64, register-staged loads
 *   2  64 x 64 tile, 4 waves of 32 x 32, register-staged loads
 *   3  (DL_I8 only) configuration 0 on the 32 x 32 x 32 int8 MFMA
 *   4  32 x 32 tile, 4 waves of 16 x 16, the whole K extent of its rows in
 *      LDS (operand rows of at most 2 KB: Np <= 2048 / element bytes)
 *   5  (the plain series only, Np <= 512) the whole fixpoint in one launch:
 *      one resident workgroup per 32 x 32 tile of the iterate, the constant
 *      right operand A + I held in LDS for every step, the workgroups of a
 *      tile row waiting only for each other between steps, the stop decided
 *      in the kernel from the model sizes (at most one step past the
 *      confirming one, whose iterate equals the model), R written by the
 *      kernel; for every other use of the product step it means the size
 *      rule.  The plain series uses it where it applies unless dl_tune_set
 *      chose another configuration for that size.  A wait that exceeds two
 *      seconds ends the launch with DL_EHIP.
 * Without an entry the library picks by size: 5 for the plain series when
 * Np <= 512 and its rows fit; otherwise 4 when Np = 256, or DL_F32 at
 * Np = 512; else 0 when (Np/256)^2 >= 256 tiles, 1 when (Np/128)^2 >= 128,
 * else 2 (Np = dl_padded_size).
 * dl_tune times squaring-step launches of every configuration on a
 * pseudo-random 0/1 relation of size n in precision prec (five interleaved
 * rounds of about 4 ms per configuration, median per configuration; on
 * `stream`, blocking), records the fastest for (prec, Np) in the context
 * (the size rule's choice when it is within 5% of the fastest) and
 * returns it in *cfg and its time per launch in *ms; cand_ms (host, five
 * doubles) receives every configuration's time, -1 for configurations that
 * do not apply (any of the three may be NULL).
 * Entries apply to dl_tc*, dl_sg* and programs on this context.
 * dl_tune_set records cfg for (prec, Np) without timing (cfg = -1 removes
 * the entry); a cfg that does not apply to (prec, n) is DL_EINVAL.  dl_tune_get copies up to cap
 * entries (precision, padded size, cfg, ms; ms = 0 for set entries) into the
 * host arrays (any may be NULL) and sets *count to the number of entries. */
int dl_tune(dl_ctx* ctx, int prec, int64_t n, int32_t* cfg, double* ms, double* cand_ms, void* stream);
int dl_tune_set(dl_ctx* ctx, int prec, int64_t n, int32_t cfg);
int dl_tune_get(dl_ctx* ctx, int32_t* prec, int64_t* np, int32_t* cfg, double* ms, int32_t cap,
                int32_t* count);

/* Padded size Np the library uses for n in this mode (multiple of its tile);
 * lets callers size budgets.  kind: 0 = closure, 1 = same generation,
 * 2 = epsilon solve. */
int64_t dl_padded_size(int64_t n, int kind, int prec);

/* ---------------------------------------------------------------- batching
 * Many independent fixpoints over uneven n, resident in one device pool and
 * advanced together: every dl_batch_step is one round of grouped launches
 * (64 x 64 output tiles for requests with n <= 256, 128 x 128 up to 1024,
 * 256 x 256 above) that moves each unfinished request forward by one product (a
 * closure request by one
 * repeated-squaring step R' = min1(A + R R), Sec. 8; a same-generation
 * request by one of the two products T = min1(P S), S' = min1(I + T P^T),
 * Sec. 7.2), followed by one read-back of the per-request model sizes.
 * Requests may be submitted between any two steps (continuous batching).
 * Arithmetic is int8 with int32 accumulation; results are identical to
 * dl_tc(DL_TC_SQUARE) / dl_sg on the same relation.  All calls on one batch
 * must use the same stream and one thread at a time. */
typedef struct dl_batch dl_batch;

/* pool_bytes of device memory hold the admitted requests (a request of n
 * constants takes 4 Np^2 bytes, closure and same generation alike,
 * Np = n rounded up to 64 for n <= 256, to 128 up to 1024, else to 256); max_active (<= 4096)
 * bounds the requests admitted and not yet fetched. */
int dl_batch_create(dl_ctx* ctx, int device, size_t pool_bytes, int max_active, dl_batch** batch);
int dl_batch_destroy(dl_batch* batch);

/* Admit a request: kind 0 = transitive closure, 1 = same generation; A is a
 * device uint8 [n x lda] relation (1 <= n <= 16384), copied into the pool
 * (the caller may reuse A after the stream reaches this point).  tag is an
 * opaque caller value returned by dl_batch_poll.  *slot receives the
 * request's slot.  DL_EAGAIN when no slot or pool memory is free. */
int dl_batch_submit(dl_batch* batch, int kind, int64_t n, const uint8_t* A, int64_t lda, int64_t tag,
                    int32_t* slot, void* stream);

/* Admit a request given as an edge list: edges is a device int32 array of m
 * pairs (i, j), row-major [m x 2], meaning r(e_i, e_j); pairs outside
 * [0, n) are skipped and repeated pairs count once.  The call only reserves
 * the slot and pool memory (no device work, `stream` is unused): the next
 * dl_batch_step builds the relations of every request admitted this way
 * since the previous round directly in their pool buffers, with one clear
 * and one scatter launch for all of them on the step's stream, ahead of
 * their first product.  edges must therefore stay valid and unchanged until
 * that dl_batch_step has returned.  Otherwise as dl_batch_submit. */
int dl_batch_submit_edges(dl_batch* batch, int kind, int64_t n, const int32_t* edges, int64_t m, int64_t tag,
                          int32_t* slot, void* stream);

/* Many dl_batch_submit_edges calls in one: request i has kind kinds[i], n
 * constants ns[i], the device edge list edges[i] of ms[i] pairs and tag
 * tags[i] (host arrays of `count` entries; edges[i] may be NULL when
 * ms[i] = 0).  Requests are admitted in order until one does not fit (in
 * slots or pool memory): *admitted (host) receives how many were, slots[i]
 * (host int32[count]) the slot of request i < *admitted.  A request that
 * does not fit is not an error (DL_OK, *admitted < count); an invalid
 * request is DL_EINVAL, with *admitted counting the requests before it.
 * The edge lists follow the rules of dl_batch_submit_edges. */
int dl_batch_submit_edges_n(dl_batch* batch, int32_t count, const int32_t* kinds, const int64_t* ns,
                            const int32_t* const* edges, const int64_t* ms, const int64_t* tags, int32_t* slots,
                            int32_t* admitted, void* stream);

/* One round (blocks until its model sizes are read back).  *active receives
 * the number of requests still running, *finished the number that finished
 * in this round.  With one round of look-ahead, the call enqueues the next
 * round and then waits for the round the previous call enqueued, so *finished
 * counts the requests found finished in that older round and the host work
 * between calls overlaps the device's products; every result is the same. */
int dl_batch_step(dl_batch* batch, int32_t* active, int32_t* finished, void* stream);

/* Rounds of look-ahead of dl_batch_step: 0 (the default: each call runs and
 * reads back one round) or 1 (each call enqueues one round and reads back
 * the previous one; a request that finishes in a round still has its next
 * product enqueued, which the device skips once it sees from that round's
 * counters that the request finished, and pool memory freed by dl_batch_fetch
 * returns to the pool after the round in flight completes).  Setting 0 while a round is
 * in flight is DL_EINVAL: call dl_batch_step until *active is 0 first. */
int dl_batch_set_lookahead(dl_batch* batch, int32_t rounds);

/* Up to cap finished requests since the last poll: their tags, slots and
 * iteration counts (the dl_tc / dl_sg convention). */
int dl_batch_poll(dl_batch* batch, int64_t* tags, int32_t* slots, int32_t* iters, int32_t cap,
                  int32_t* count);

/* Write the 0/1 model of a finished request into R (device uint8 [n x ldr];
 * NULL to discard), report its number of true entries in *ones (may be
 * NULL), and free the slot and its pool memory.  A request may be fetched
 * before it is polled; dl_batch_poll then no longer reports it. */
int dl_batch_fetch(dl_batch* batch, int32_t slot, uint8_t* R, int64_t ldr, int64_t* ones, void* stream);

/* dl_batch_fetch without the models for `count` finished requests: ones[i]
 * (host int64[count], may be NULL) receives the number of true entries of
 * slots[i]'s model, and every slot and its pool memory is freed.  A slot
 * that is not a finished request is DL_EINVAL; the slots before it have
 * been freed. */
int dl_batch_release_n(dl_batch* batch, int32_t count, const int32_t* slots, int64_t* ones);

/* Tile autotuner of the grouped step (the output tile size of each request's
 * products).  For each size n of `sizes` (host int64 array of k ascending
 * sizes; NULL / k = 0 for 96, 128, 192, 256, 384, 512, 768, 1024, 1536,
 * 2048) it times grouped squaring launches over the same pseudo-random
 * requests of n constants (1 to 256 of them, about eight 2048-sized
 * products of work) at each tile size 64, 128 and 256 (three interleaved
 * rounds, median), and records the fastest -- the built-in choice when it
 * is within 5% -- in the batch's tile table: a request of n constants then
 * takes the choice of the smallest tabled size >= n (the built-in rule above
 * the largest).  tiles (host int32[k]) and ms (host double[3 k]: time per
 * request-product for tiles 64, 128, 256) may be NULL.  Temporary device
 * memory of up to a few hundred MB is allocated outside the pool and freed;
 * the call blocks on `stream` and leaves admitted requests untouched (their
 * tile was fixed at admission).
 * dl_batch_set_tiles sets the table directly (sizes ascending, tiles 64, 128
 * or 256; k = 0 restores the built-in rule: 64 up to n = 256, 128 up to
 * 1024, else 256). */
int dl_batch_tune(dl_batch* batch, const int64_t* sizes, int32_t k, int32_t* tiles, double* ms, void* stream);
int dl_batch_set_tiles(dl_batch* batch, const int64_t* sizes, const int32_t* tiles, int32_t k);

/* Occupancy: running requests, used slots, free pool bytes. */
int dl_batch_info(dl_batch* batch, int32_t* active, int32_t* used_slots, size_t* pool_free_bytes);

/* ---------------------------------------------------------------- programs
 * Layered evaluation of a linear binary Datalog program (Sec. 5, Sec. 6,
 * stratified negation as in Sec. 8).  Syntax, one clause per '.':
 *     head(X,Y) :- atom, atom, ... .      atom = [not] pred(V,W)
 * Names of predicates start lower case, variables upper case; '%' starts a
 * comment; "\+" may replace "not".  Every body must be a chain of atoms from
 * the head's first variable to its second (each other variable in exactly two
 * atoms); an atom may name its variables in either order (the converse
 * relation).  eq is the built-in equality over the n constants.  Predicates
 * that head no clause are given relations, bound with dl_program_bind.
 * dl_program_create splits the predicates into strongly connected components
 * of the dependency graph (Tarjan's algorithm) and orders them as layers; it
 * returns DL_EUNSUPPORTED for a body that is not a chain, two atoms of the
 * head's layer in one body (not linear) or a negated atom of the head's layer
 * (not stratified), and DL_EINVAL for a syntax error.  Each layer is the
 * system R_h = min1(A_h + sum P R_j^o S) of its heads (R^o = R or R^T).
 * dl_program_run evaluates the layers in order on the device:
 *   DL_EVAL_ITERATION  every recursive layer by the Boolean series from 0
 *                      (int8 matrix products, Jacobi order, first repeat);
 *   DL_EVAL_MATRIX     tail-recursive layers as one stacked fp64 linear
 *                      system, a single two-sided or transposed clause as a
 *                      Stein equation (fp64 doubling), other layers by the
 *                      series; fp64 results are thresholded at > 0.
 * Both give the least (perfect) model, the epsilon forms up to fp64
 * underflow of long derivations.  A program handle is used by one thread at
 * a time; its results stay on the device until the next run or destroy. */
typedef struct dl_program dl_program;
typedef enum { DL_EVAL_ITERATION = 0, DL_EVAL_MATRIX = 1 } dl_eval_method;
typedef enum {
  DL_FORM_NONRECURSIVE = 0,
  DL_FORM_RIGHT_TAIL = 1, /* every recursive atom ends its chain: R = A + sum P R_j */
  DL_FORM_LEFT_TAIL = 2,  /* every recursive atom starts its chain: R = A + sum R_j S */
  DL_FORM_TWO_SIDED = 3,  /* one head, one clause P R^o S */
  DL_FORM_GENERAL = 4
} dl_layer_form;

int dl_program_create(dl_ctx* ctx, const char* text, dl_program** prog);
int dl_program_destroy(dl_program* prog);
/* Number of predicates (given, defined and eq) and of layers. */
int dl_program_counts(dl_program* prog, int32_t* n_predicates, int32_t* n_layers);
/* Predicate `index`: its name (owned by the program), kind (0 given,
 * 1 defined, 2 eq) and layer (-1 unless defined). */
int dl_program_predicate(dl_program* prog, int32_t index, const char** name, int32_t* kind,
                         int32_t* layer);
/* Binds a given relation to device uint8 [n x ldm] (nonzero = true).  The
 * pointer is read by the next dl_program_run; every relation has the same n. */
int dl_program_bind(dl_program* prog, const char* name, int64_t n, const uint8_t* M, int64_t ldm);
/* Evaluates every layer (blocks until done).  Device memory: two int8
 * (n rounded up to 256)^2 matrices per predicate plus per-layer temporaries
 * and the fp64 workspace of the epsilon forms. */
int dl_program_run(dl_program* prog, int method, void* stream);
/* Layer `layer` of the last run: its heads (predicate indices, up to cap),
 * form (dl_layer_form), the method used and its count: iterations of the
 * series (including the confirming one), doublings, or 0 for a linear solve. */
int dl_program_layer(dl_program* prog, int32_t layer, int32_t* n_heads, int32_t* heads, int32_t cap,
                     int32_t* form, int32_t* method_used, int32_t* iters);
/* Writes the model of a defined predicate into device uint8 [n x ldo] and
 * its number of true entries into *ones (may be NULL). */
int dl_program_fetch(dl_program* prog, const char* name, uint8_t* out, int64_t ldo, int64_t* ones,
                     void* stream);

const char* dl_status_str(int status);
const char* dl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DL_H_ */
