/*
 * mwntt.h -- C ABI of the multi-word modular NTT / BLAS library for MI355X (gfx950).
 *
 * Operations (arXiv 2509.12494, "Towards Closing the Performance Gap for
 * Cryptographic Kernels Between CPUs and Specialized Hardware"):
 *   - modular add / sub / mul over Z_q (Background, modular arithmetic,
 *     Eq. saddmod, Eq. ssubmod, Eq. barrett);
 *   - point-wise polynomial operations as BLAS: vector add, vector sub,
 *     point-wise vector multiply and axpy y = a*x + y (Background, polynomial
 *     operations);
 *   - the number theoretic transform of Eq. (ntt), in its negacyclic form over
 *     Z_q[X]/(X^N + 1), and its inverse (Background, polynomial multiplication
 *     using NTT).
 * Moduli are "double-word" (two 64-bit words, q < 2^124, the largest width the
 * paper's Barrett reduction allows for 128-bit arithmetic), single-word
 * (q < 2^60, the same rule for one 64-bit word) or four-word (q < 2^252: the
 * larger bit-widths the paper names as the next step, Discussion).
 *
 * Data layout.  A residue is `limbs` little-endian uint64_t words (word 0 is
 * the least significant; the paper's notation [x0, x1] lists the high word
 * first, which is notation only).  A vector of n residues is n*limbs words,
 * element-major ([n][limbs]); a batch of polynomials is [batch][N][limbs].
 * All device pointers must be aligned to 8*limbs bytes.
 *
 * Values.  Every input residue must be canonical, 0 <= x < q (the paper's
 * assumption for Eq. saddmod / ssubmod); results for non-canonical inputs are
 * unspecified, and in validate mode (mw_set_validate) they are reported as
 * MW_ENONCANON.  Every output is canonical.
 *
 * Moduli.  `q` points to `limbs` host words.  limbs == 1: 2 <= bitlen(q) <= 60
 * (q >= 3); limbs == 2: 61 <= bitlen(q) <= 124; limbs == 4:
 * 125 <= bitlen(q) <= 252.  Every operation takes every odd q of its class
 * (Barrett's reduction, Eq. barrett, holds for general moduli; the library
 * runs it on q scaled by a power of two to the top of the class).  Other limb
 * counts are MW_EINVAL.  Primality is the caller's responsibility (an NTT plan
 * checks that its root has order exactly 2N).
 *
 * Streams and errors.  `stream` is a hipStream_t (NULL = the null stream).
 * Argument errors return a negative status synchronously and enqueue nothing.
 * Kernels run asynchronously on the stream; a launch failure is reported as
 * MW_EDEVICE.  Functions never synchronize the device unless stated.
 *
 * Ownership.  The caller allocates and frees every data buffer.  A plan owns
 * its device tables and scratch and frees them in ntt_plan_destroy.
 */
#ifndef MWNTT_H
#define MWNTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mw_status {
  MW_OK = 0,
  MW_EINVAL = -1,    /* null pointer, zero/oversized length, bad flag */
  MW_EMODULUS = -2,  /* modulus width/parity/congruence not supported */
  MW_ESIZE = -3,     /* transform length outside 2^1 .. 2^17 */
  MW_ENOMEM = -4,    /* device or host allocation failed */
  MW_EDEVICE = -5,   /* HIP runtime error (launch failure, no device) */
  MW_EROOT = -6,     /* supplied root is not a primitive 2N-th root */
  MW_EBUSY = -7,     /* serving: the request has not completed yet */
  MW_ENONCANON = -8  /* validate mode: an input residue was >= q */
};

/* Returns a static string describing a status code. */
const char* mw_status_str(int status);

/* ------------------------------------------------------------------------ */
/* Validate mode (input canonicality, the paper's precondition 0 <= x < q    */
/* of Eq. saddmod / ssubmod).  While it is on, every entry point that reads  */
/* caller residues (the BLAS calls, ntt_forward / ntt_inverse /             */
/* ntt_forward_pass, ntt_batch_run, and the serving runtime's requests)     */
/* first enqueues a check kernel over those inputs on the same stream; a     */
/* residue >= q sets a library-wide error word held in pinned host memory.  */
/* The violation is reported, and the word cleared, by mw_check (which      */
/* synchronizes the stream first) or by the first entry point called after  */
/* the check kernel has completed: that call returns MW_ENONCANON and       */
/* enqueues nothing.  The work whose inputs failed still runs (its output   */
/* is unspecified).  Off by default; the environment variable               */
/* MWNTT_VALIDATE=1 turns it on when the library loads.  Costs one extra    */
/* read of every input.                                                      */
/* ------------------------------------------------------------------------ */
/* on != 0 enables validation, 0 disables it (a pending error is kept).
 * MW_ENOMEM if the pinned error word cannot be allocated. */
int mw_set_validate(int on);
/* 1 if validation is on, else 0. */
int mw_get_validate(void);
/* Synchronizes `stream`, then returns MW_ENONCANON (and clears the word) if
 * a check kernel found a non-canonical input since the last report, MW_EDEVICE
 * if the synchronization failed, else MW_OK. */
int mw_check(void* stream);

/* ------------------------------------------------------------------------ */
/* Element-wise modular BLAS (Background, polynomial operations as BLAS).    */
/* c[i] = (a[i] + b[i]) mod q, etc., for 0 <= i < n.  n == 0 is a no-op;   */
/* n > 2^40 is MW_EINVAL.                                                    */
/* Outputs may alias inputs exactly (c == a or c == b); partial overlap is   */
/* undefined.                                                                */
/* ------------------------------------------------------------------------ */
int vec_addmod(void* d_c, const void* d_a, const void* d_b, size_t n,
               const uint64_t* q, uint32_t limbs, void* stream);
int vec_submod(void* d_c, const void* d_a, const void* d_b, size_t n,
               const uint64_t* q, uint32_t limbs, void* stream);
/* Point-wise product reduced with Barrett's method (Eq. barrett). */
int vec_mulmod(void* d_c, const void* d_a, const void* d_b, size_t n,
               const uint64_t* q, uint32_t limbs, void* stream);
/* Product kernel of vec_mulmod for one width (limbs 1, 2 or 4): karatsuba = 1
 * forms the full product of the Barrett reduction by one level of Karatsuba
 * (Eq. mulk; three half-size products and the carry corrections), 0 by the
 * schoolbook columns (Eq. muls).  Results are identical; the default per width
 * is the measured faster one.  Process-wide, applies to later calls. */
int vec_mulmod_set_product(uint32_t limbs, uint32_t karatsuba);
int vec_mulmod_get_product(uint32_t limbs, uint32_t* karatsuba);
/* y[i] = (alpha * x[i] + y[i]) mod q; alpha is `limbs` host words, < q. */
int vec_axpymod(void* d_y, const uint64_t* alpha, const void* d_x, size_t n,
                const uint64_t* q, uint32_t limbs, void* stream);

/* ------------------------------------------------------------------------ */
/* Negacyclic NTT over Z_q[X]/(X^N + 1), N = 2^log2n, 1 <= log2n <= 17.     */
/*   forward: A[k] = sum_j a[j] psi^(j(2k+1)) mod q   (natural order)        */
/*   inverse: a[j] = N^-1 psi^-j sum_k A[k] psi^(-2jk) mod q                 */
/* i.e. Eq. (ntt) on the psi-twisted input with omega_N = psi^2.  psi is a   */
/* primitive 2N-th root of unity: the caller's, or by default the smallest   */
/* one in [1, q).  q must satisfy q = 1 (mod 2N).                            */
/* ------------------------------------------------------------------------ */
typedef struct ntt_plan_s* ntt_plan_t;

/* ntt_forward writes its output in bit-reversed order (A[bitrev(i)] at i).  */
#define NTT_BITREV_OUT 0x1u
/* ntt_inverse reads its input in bit-reversed order.                        */
#define NTT_BITREV_IN 0x2u
/* Arithmetic variants of the butterfly, for the GPU analog of the paper's MQX
 * ablation (Evaluation, sensitivity to the MQX components; Table tab:mqx):
 * NTT_ARITH_MULHI forms every 32x32 product from v_mul_lo_u32 and
 * v_mul_hi_u32 instead of the widening multiply-add v_mad_u64_u32;
 * NTT_ARITH_CMPCARRY recovers every carry and borrow by a compare and a select
 * instead of the hardware carry-out / carry-in; both together remove both.
 * Results are identical to the native arithmetic.  Only for two-word moduli
 * and N = 2^16 (MW_EINVAL otherwise); such a plan runs one fixed two-pass
 * shape (N1 = N2 = 2^8), rejects ntt_plan_set_split / set_tiles, and is
 * accepted by the plain entry points only (not by the batched executor or
 * the serving runtime). */
#define NTT_ARITH_MULHI 0x10u
#define NTT_ARITH_CMPCARRY 0x20u

/* Creates a plan on the current HIP device: builds the twiddle tables
 * (psi^bitrev(i) and psi^-bitrev(i) with their Shoup companions) on the host
 * and copies them to device memory, and allocates a scratch buffer for the
 * two-pass transforms (256 polynomials, within 64 .. 256 MiB; larger batches
 * run in chunks of that many).  psi may be NULL (canonical root) or point to `limbs`
 * host words.  flags: 0 or a combination of NTT_BITREV_OUT / NTT_BITREV_IN.
 * Argument, modulus and root errors are reported before any device call.
 * Synchronous (for four-word moduli the host tables take about 1 s at
 * N = 2^17, mostly the bitwise long divisions of the Shoup companions). */
int ntt_plan(ntt_plan_t* plan, uint32_t log2n, const uint64_t* q, uint32_t limbs,
             const uint64_t* psi, uint32_t flags);
/* Frees the plan's device memory (synchronizes the device first). */
int ntt_plan_destroy(ntt_plan_t plan);
/* The root psi the plan uses (limbs words written to psi_out). */
int ntt_plan_root(ntt_plan_t plan, uint64_t* psi_out);

/* Decomposition of the transform (used by the autotuner and by tests):
 * log_n1 == 0 runs each transform in one workgroup (N <= 2^12 for two-word
 * moduli, N <= 2^13 for one-word, N <= 2^11 for four-word moduli); otherwise
 * two passes over device
 * memory with N1 = 2^log_n1 rows and N2 = N / N1 columns, 3 <= log2(N1),
 * log2(N2) <= 9.  By default a plan holds two measured configurations, one
 * for calls with little work (a single transform spread over as many CUs as
 * possible) and one for large batches, and picks per call; setting a split
 * or a tile shape replaces both for every later call.  get_* report the
 * large-batch configuration unless one was set.  Results never depend on the
 * configuration.  Not thread-safe with concurrent transforms on the plan. */
int ntt_plan_set_split(ntt_plan_t plan, uint32_t log_n1);
int ntt_plan_get_split(ntt_plan_t plan, uint32_t* log_n1);
/* The configuration a call with `batch` transforms runs: *large = 1 for the
 * large-batch one (0 for the single-transform one, or when a split or shape
 * was set), *log_n1 its split. */
int ntt_plan_config_for(ntt_plan_t plan, uint32_t batch, uint32_t* large, uint32_t* log_n1);

/* Tile shape of one pass (pass 0: single-workgroup transform, 1: column pass,
 * 2: row pass): 2^log_p points per lane (1 <= log_p <= 4; <= 2 for four-word
 * moduli) and `lines`
 * sub-transforms per workgroup (a power of two; columns per column tile, rows
 * per row tile, transforms per single-workgroup tile).  Rejected (MW_EINVAL)
 * when the pass is not part of the plan's current split or the workgroup would
 * exceed its thread or LDS limits.  ntt_plan_set_split resets the shapes to
 * their defaults.  Results do not depend on the shape. */
int ntt_plan_set_tiles(ntt_plan_t plan, uint32_t pass, uint32_t log_p, uint32_t lines);
int ntt_plan_get_tiles(ntt_plan_t plan, uint32_t pass, uint32_t* log_p, uint32_t* lines);

/* Transforms `batch` polynomials [batch][N][limbs].  d_out == d_in is
 * allowed.  Calls on one plan must not overlap in time on different streams
 * (they share the plan's scratch buffer); plans are independent. */
int ntt_forward(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream);
int ntt_inverse(ntt_plan_t plan, void* d_out, const void* d_in, uint32_t batch, void* stream);

/* One pass of a two-pass forward transform, for callers that schedule the
 * passes themselves (or time them separately): pass 1 runs the first log N1
 * stages (column tiles) from d_in into the plan's scratch, pass 2 the
 * remaining stages (row tiles) from the scratch into d_out, in the order the
 * plan's flags give.  Running pass 1 then pass 2 with the same batch equals
 * ntt_forward.  MW_EINVAL if the plan's configuration for this batch is a
 * single-workgroup transform; MW_ESIZE if the batch exceeds the scratch. */
int ntt_forward_pass(ntt_plan_t plan, uint32_t pass, void* d_out, const void* d_in, uint32_t batch, void* stream);

/* Allocation-free transform, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): ntt_forward (inverse == 0) or ntt_inverse (inverse == 1) with
 * the same arguments and results, except that the two-pass intermediate lives
 * in a static 64 MiB device array that the library holds on each device it
 * runs on until the process ends, instead of the plan's scratch.  The call
 * allocates nothing and needs no plan scratch; the array's device address is
 * looked up on the first call on each device.  MW_ESIZE if a two-pass call's
 * intermediate (batch * N * limbs * 8 bytes) exceeds 64 MiB, e.g. more than
 * 32 two-word transforms of 2^16 points (single-workgroup sizes have no
 * limit).  Calls that overlap in time on one device share the array and race;
 * serialize them (one stream, or events).  Not covered by validate mode. */
int ntt_transform_noalloc(ntt_plan_t plan, uint32_t inverse, void* d_out, const void* d_in, uint32_t batch,
                          void* stream);

/* ------------------------------------------------------------------------ */
/* Batched executor: many jobs -- forward or inverse transforms, or fused     */
/* negacyclic products c = INTT(NTT(a) * NTT(b)) (Background, polynomial     */
/* multiplication using NTT; the schoolbook product reduced mod X^N + 1) --  */
/* of any mix of lengths (2^6 .. 2^17) and modulus widths, run as one       */
/* kernel launch per phase (two for transforms, three when a product is      */
/* present), each launch covering every job; four-word jobs' tiles take a   */
/* second launch in each phase (a kernel of their own).                      */
/* ------------------------------------------------------------------------ */
typedef struct ntt_batch_s* ntt_batch_t;

enum ntt_job_op { NTT_JOB_FORWARD = 0, NTT_JOB_INVERSE = 1, NTT_JOB_POLYMUL = 2 };

/* One job.  plan gives q, N, width, root and the order flags (NTT_BITREV_OUT
 * applies to forward outputs, NTT_BITREV_IN to inverse inputs; products take
 * and return natural order).  in / in2 / out are device buffers of N
 * residues; in2 is used by NTT_JOB_POLYMUL only (b; in is a).  out may alias
 * in or in2. */
typedef struct {
  ntt_plan_t plan;
  uint32_t op;
  const void* in;
  const void* in2;
  void* out;
} ntt_job;

/* Builds the device job list, tile list and scratch (N residues per
 * transform, 2N per product).  Synchronous.  The plans must outlive the
 * batch, and the job buffers must stay allocated at the same addresses for
 * every run. */
int ntt_batch_create(ntt_batch_t* batch, const ntt_job* jobs, uint32_t count);
/* Runs every job: 2 or 3 kernel launches on `stream` (twice that with
 * four-word jobs in the batch), no allocation and no
 * memset, so a run can be captured in a hipGraph and replayed.  Runs of one
 * batch must not overlap in time (they share the batch's scratch). */
int ntt_batch_run(ntt_batch_t batch, void* stream);
/* Tiles in the batch and launches per run (either pointer may be NULL). */
int ntt_batch_info(ntt_batch_t batch, uint32_t* tiles, uint32_t* launches);
/* Synchronizes the device; MW_EDEVICE if a previous launch failed. */
int ntt_batch_check(ntt_batch_t batch);
/* Frees the batch (synchronizes the device first). */
int ntt_batch_destroy(ntt_batch_t batch);

/* ------------------------------------------------------------------------ */
/* Serving runtime: continuous batching of NTT / BLAS requests.              */
/*                                                                           */
/* Requests are queued in arrival order.  A scheduler thread admits the     */
/* oldest requests whose device memory (output + scratch) fits in the       */
/* remaining HBM budget, forms a batch of up to max_batch of them and        */
/* launches it on one of max_inflight streams (transform and product        */
/* requests through the batched executor, BLAS requests as their own        */
/* kernels), while earlier batches are still running: requests that arrive */
/* during a batch join the next one as soon as a stream and memory are      */
/* free, and batches overlap on the device.  Completion is detected from    */
/* stream events; latency is completion minus submission.  Admission is     */
/* first-in first-out: a request that does not fit blocks the ones behind   */
/* it until memory is released.  With `resident` set, one- and two-word    */
/* requests run in a device-resident loop instead (mw_server_config).      */
/* ------------------------------------------------------------------------ */
typedef struct mw_server_s* mw_server_t;

typedef struct {
  size_t hbm_budget;      /* bytes of device memory for outputs and scratch */
  uint32_t max_inflight;  /* batches on the device at once (streams), >= 1 */
  uint32_t max_batch;     /* requests per batch, 1 .. 256 */
  uint32_t dry_run;       /* 1: scheduler only, no device memory or work; every
                             request completes after a modelled time and has no
                             output (for testing admission and queueing) */
  uint32_t spin_us;       /* 0: the scheduler thread sleeps whenever it has
                             nothing to do (woken by submissions, polling
                             running batches every few microseconds); n > 0:
                             it keeps polling without sleeping for n
                             microseconds after its last action, 0 .. 100000
                             (lower latency for one busy host core) */
  uint32_t resident;      /* 1: transform, product and BLAS requests of one-
                             and two-word moduli (BLAS: n <= 2^22)
                             run in a device-resident loop instead of kernel
                             launches: one persistent kernel (launched with
                             the first such request, leaving after 20 ms
                             without work, relaunched on demand) takes them
                             from a ring in mapped host memory and signals
                             completion there; the other requests, and all of
                             them in validate mode, keep the slot path.
                             The loop holds one of the device's hardware
                             queues while it runs: a kernel the caller
                             launches on a stream that shares that queue
                             starts only when the loop ends (20 ms after its
                             last request, or at mw_server_destroy).
                             0: every request takes the slot path.  Ignored in
                             a dry run. */
  uint32_t resident_max_tiles; /* with resident: only requests of at most
                             this many tiles (workgroup tasks: a BLAS tile is
                             1024 residues, a transform's tiles are the
                             batched executor's) go to the loop, the others
                             keep the slot path; 0 = every request the loop
                             can take (4096 tiles).  A slot batch whose
                             stream shares the loop's hardware queue waits
                             until the loop yields (after 0.5 ms) */
  uint32_t resident_wait_us; /* with resident: how long a tile waits for the
                             earlier phases of its request before giving up;
                             a request with a tile that gave up completes as
                             failed (mw_server_result: MW_EDEVICE).  0 = 2 s */
} mw_server_config;

enum mw_request_op {
  MW_REQ_NTT_FORWARD = 0, MW_REQ_NTT_INVERSE = 1, MW_REQ_POLYMUL = 2,
  MW_REQ_VEC_ADDMOD = 3, MW_REQ_VEC_SUBMOD = 4, MW_REQ_VEC_MULMOD = 5, MW_REQ_VEC_AXPYMOD = 6
};

/* One request.  Transform and product requests take q, N and the width from
 * `plan` (N >= 2^6); BLAS requests take q, limbs (1, 2 or 4; the first
 * `limbs` words of q and alpha are used), n (and alpha for axpy:
 * out = alpha*in + in2).  `in` / `in2` are device buffers owned by the
 * caller that must stay valid until the request completes; in2 is b for
 * products and BLAS, NULL otherwise. */
typedef struct {
  uint32_t op;
  ntt_plan_t plan;
  uint64_t q[4];
  uint32_t limbs;
  uint64_t alpha[4];
  uint64_t n;
  const void* in;
  const void* in2;
} mw_request;

typedef struct {
  uint64_t submitted, completed, batches, max_batch_seen;
  uint64_t queue_peak;          /* most requests waiting for admission at once */
  uint64_t inflight_peak;       /* most batches on the device at once */
  size_t pool_peak;             /* most budget bytes in use at once */
  uint64_t resident_requests;   /* requests run by the device-resident loop */
  uint64_t resident_launches;   /* launches of that loop */
  uint64_t resident_yields;     /* times the loop was asked to yield to a slot
                                   batch that waited behind it */
} mw_server_stats;

/* Creates the server on the current device (allocates the budget as one
 * pool, the streams and per-stream descriptor buffers; starts the scheduler
 * thread). */
int mw_server_create(mw_server_t* server, const mw_server_config* config);
/* Queues a request; returns its ticket.  MW_ENOMEM if the request alone can
 * never fit the budget.  Thread-safe. */
int mw_server_submit(mw_server_t server, const mw_request* request, uint64_t* ticket);
/* Result of a request: with wait != 0 blocks until it completes.  On MW_OK
 * *d_out (may be NULL) is the device buffer holding the output (owned by the
 * server until mw_server_release) and *latency_us (may be NULL) the
 * submission-to-completion time.  MW_EBUSY if not complete and wait == 0,
 * MW_EINVAL for an unknown ticket. */
int mw_server_result(mw_server_t server, uint64_t ticket, int wait, void** d_out, double* latency_us);
/* Returns a completed request's output memory to the pool. */
int mw_server_release(mw_server_t server, uint64_t ticket);
/* Blocks until every queued request has completed. */
int mw_server_drain(mw_server_t server);
int mw_server_get_stats(mw_server_t server, mw_server_stats* stats);
/* Open-loop replay: submits reqs[i] at arrival_us[i] microseconds after the
 * call starts (a driver thread), releases each result as soon as it
 * completes, and writes latency_us[i] = completion - scheduled arrival.
 * *makespan_us = time from the start to the last completion. */
int mw_server_replay(mw_server_t server, const mw_request* reqs, const double* arrival_us, uint32_t count,
                     double* latency_us, double* makespan_us);
/* Stops the scheduler (after draining) and frees everything. */
int mw_server_destroy(mw_server_t server);

/* ------------------------------------------------------------------------ */
/* Host-only helpers (no device needed): the plan's own arithmetic, exposed */
/* for inspection.                                                           */
/* ------------------------------------------------------------------------ */
/* Smallest primitive 2N-th root of unity modulo q (N = 2^log2n). */
int mw_canonical_root(const uint64_t* q, uint32_t limbs, uint32_t log2n, uint64_t* psi_out);
/* Shoup companion floor(w * 2^(64*limbs) / q) of a constant w < q. */
int mw_shoup_companion(const uint64_t* w, const uint64_t* q, uint32_t limbs, uint64_t* out);
/* Barrett constant of the normalised modulus, floor(2^(2T) / q') with
 * q' = q * 2^(T - bitlen(q)) and T = 60, 124, 252 for limbs 1, 2, 4 (T + 1
 * bits, limbs words). */
int mw_barrett_mu(const uint64_t* q, uint32_t limbs, uint64_t* out);
/* Asynchronous copy of `bytes` between any two HIP-visible buffers on
 * `stream` (used to read server-owned outputs). */
int mw_copy(void* dst, const void* src, size_t bytes, void* stream);
/* Library version string. */
const char* mw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MWNTT_H */
