/*
 * bires.h -- exact bivariate resultants, discriminants and univariate gcds on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations are those of Berberich, Emeliyanenko, Kobel and Sagraloff,
 * "Exact Symbolic-Numeric Computation of Planar Algebraic Curves":
 *   - res(f, g; y) in Z[x], the determinant of the Sylvester matrix of f and g
 *     taken as polynomials in y (Section 2, "Resultants" paragraph); res(f, g; x)
 *     is the same with x and y exchanged;
 *   - res(f, f_y; y), the resultant the curve analysis projects with
 *     (Section 3.1, Project);
 *   - Q = res(f_x, f_y; y), the resultant behind the fiber bound n_alpha^+
 *     (Section 3.2.2, "Computation of n_alpha^+", Teissier's lemma);
 *   - gcd(a, b) in Z[x] (Section 5.1, "Computing gcds in Z[x]").
 * All results are exact integers.  They are computed by the multi-modular
 * scheme of Section 5.1 ("Computing resultants in Z[x,y]", steps (a)-(e)):
 * reduction modulo many word-size primes, evaluation at many x, univariate
 * resultants over F_p, interpolation per prime and Chinese remaindering in
 * mixed-radix form, every step in HIP kernels.
 *
 * Conventions shared by every call
 * --------------------------------
 * Integers are little-endian arrays of 32-bit limbs in two's complement.
 *
 * A bivariate input is a dense rectangle of coefficients:
 *     c[((j * (deg_x + 1)) + i) * limbs + k]  = limb k of the coefficient of x^i y^j,
 *     0 <= j <= deg_y, 0 <= i <= deg_x.
 * Total-degree supports are zero-padded.  deg_y/deg_x are the extents of the
 * rectangle, not necessarily the true degrees: all-zero top rows or columns
 * are allowed and ignored.  The caller owns c.
 *
 * A univariate polynomial is c[i * limbs + k] = limb k of the coefficient of x^i.
 * As an output, `degree` holds on entry the largest degree the buffer has room
 * for and on return the true degree (-1 for the zero polynomial); `limbs` is
 * fixed by the caller and every coefficient is written sign-extended to it.
 * Coefficients above the true degree are written as zero.  Size the buffer with
 * the matching *_bounds() call, which depends only on the extents and limb
 * counts of the inputs, never on their values.
 *
 * Memory space: `mem` says where every coefficient buffer of the call lives,
 * BIRES_MEM_HOST (ordinary host memory) or BIRES_MEM_DEVICE (device memory
 * of the current HIP device).  Descriptor structs are always host memory.
 *
 * Streams: `stream` is a hipStream_t (cast to void*); NULL selects the
 * library's own stream.  Calls are synchronous: they return after the result
 * is in the output buffer.
 *
 * Return values: 0 (BIRES_OK) or a negative BIRES_E* code; bires_strerror()
 * gives a message.  On error the output buffers are unspecified.
 * Thread safety: calls may come from several host threads; calls that share a
 * stream are serialised by the library.
 */
#ifndef BIRES_H
#define BIRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BIRES_OK 0
#define BIRES_EINVAL (-1)    /* NULL pointer, negative extent, limbs < 1, bad var/kind/mem */
#define BIRES_EBUFSIZE (-2)  /* output buffer too small (degree or limbs); needed sizes written back */
#define BIRES_ENOMEM (-3)    /* device or pinned allocation failed, or HBM budget exceeded */
#define BIRES_ETOOBIG (-4)   /* beyond compiled limits (prime count, degree) */
#define BIRES_EDEVICE (-5)   /* HIP runtime error or no usable gfx950 device */
#define BIRES_ECHECK (-6)    /* internal consistency check failed (bound overflow, check prime) */
#define BIRES_ENOTFOUND (-7) /* unknown server ticket */
#define BIRES_ETIMEOUT (-8)  /* server wait timed out (the job keeps running) */

#define BIRES_VAR_X 0
#define BIRES_VAR_Y 1

#define BIRES_MEM_HOST 0
#define BIRES_MEM_DEVICE 1

#define BIRES_KIND_RESULTANT 0     /* res(f, g; var) */
#define BIRES_KIND_DISCRIMINANT 1  /* res(f, df/dvar; var); g ignored */
#define BIRES_KIND_POLAR 2         /* res(df/dother, df/dvar; var); g ignored */

/* Compiled limits. */
#define BIRES_MAX_PRIMES 2048      /* primes per job (each above 2^30): results below ~2^62000 */
#define BIRES_MAX_YDEG 512         /* degree in the eliminated variable, per input */

typedef struct {
  int32_t deg_y;        /* rows - 1; -1 for an empty (zero) polynomial */
  int32_t deg_x;        /* columns - 1 */
  int32_t limbs;        /* 32-bit limbs per coefficient, >= 1 */
  const uint32_t *c;    /* see layout above */
} bires_bipoly;

typedef struct {
  int32_t degree;       /* output: capacity on entry, true degree on return; input: degree (-1 = zero) */
  int32_t limbs;        /* limbs per coefficient, >= 1 */
  uint32_t *c;          /* c[i * limbs + k] */
} bires_upoly;

/* Library set-up on the current HIP device: builds the prime table (the
 * largest primes below 2^32/3), the mixed-radix tables and the library stream.
 * Called implicitly by every compute call; explicit calls are idempotent. */
int bires_init(void);

/* Output sizes for res(f, g; var): max_degree bounds deg R by
 * min(n*dx_f + m*dx_g, n*t_f + m*t_g - m*n) (m, n the degrees in var; dx the
 * degrees in the other variable; t total degrees; all read from the extents),
 * a sharpening of the deg R <= m*n of Section 2; max_limbs bounds the
 * coefficients by the Hadamard bound of the Sylvester matrix with every entry
 * replaced by its 1-norm and every coefficient by 2^(32*limbs-1).
 * Host-only: no device work. */
int bires_resultant_bounds(const bires_bipoly *f, const bires_bipoly *g, int var,
                           int32_t *max_degree, int32_t *max_limbs);

/* R = res(f, g; var) (Section 2, "Resultants"; Section 5.1 for the method).
 * f = 0 or g = 0 gives the zero polynomial; deg_var f = deg_var g = 0 gives 1. */
int bires_resultant(const bires_bipoly *f, const bires_bipoly *g, int var,
                    bires_upoly *out, int mem, void *stream);

/* Output sizes for res(f, df/dvar; var). */
int bires_discriminant_bounds(const bires_bipoly *f, int var, int32_t *max_degree, int32_t *max_limbs);

/* R = res(f, df/dvar; var) exactly as Project forms it (Section 3.1): no
 * division by the leading coefficient, no sign normalisation.  Needs
 * deg_var f >= 1 (else BIRES_EINVAL). */
int bires_discriminant(const bires_bipoly *f, int var, bires_upoly *out, int mem, void *stream);

/* Output sizes for res(df/dother, df/dvar; var) (other: the variable that is
 * not eliminated). */
int bires_polar_bounds(const bires_bipoly *f, int var, int32_t *max_degree, int32_t *max_limbs);

/* Q = res(f_x, f_y; y) for var = BIRES_VAR_Y (res(f_y, f_x; x) for
 * BIRES_VAR_X): the resultant whose root multiplicities give the fiber bound
 * n_alpha^+ = deg_y f - mult(R, alpha) + mult(Q, alpha) (Section 3.2.2,
 * "Computation of n_alpha^+").  The paper takes Q = res(f_x*, f_y*; y) with
 * f_x* = f_x / h, f_y* = f_y / h, h = gcd(f_x, f_y) (the remark after
 * Teissier's lemma); this call computes the case h = 1, which holds for a
 * curve in generic position, and does not remove a common factor.  The
 * formal degrees are the degrees in var of the two derivatives as bivariate
 * polynomials.  Needs deg_var f >= 1 (else BIRES_EINVAL); f_x = 0 gives the
 * zero polynomial. */
int bires_polar_resultant(const bires_bipoly *f, int var, bires_upoly *out, int mem, void *stream);

/* Principal subresultant coefficients modulo one prime (Section 3.2.2,
 * "(Exact) Computation of N" and "Computation of N^-"): for the Sylvester
 * operands of `kind` (f and g; f and df/dvar; df/dother and df/dvar) with
 * formal degrees m, n in var, sr_i(x) mod p for i = 0 .. count-1, where
 * count = min(m, n) + 1, less one when m = n; sr_i is the coefficient of
 * var^i of the i-th subresultant, the determinant of the Sylvester-like
 * matrix with n - i rows of the first operand and m - i of the second; sr_0
 * is the resultant.  The formal degrees are kept where p divides a leading
 * coefficient (sr_i mod p is the reduction of the integer sr_i).  Output:
 * out[i * points + c] = coefficient of x^c (other variable) of sr_i mod p, in
 * [0, p), for c < points = the resultant's degree bound + 1 (which bounds
 * every sr_i).  p must be one of the library's primes (bires_primes), else
 * BIRES_EINVAL.  Inputs and out are host memory.  *count and *points are
 * written first; BIRES_EBUFSIZE when capacity < count * points (no device
 * work then).  A zero operand gives BIRES_EINVAL. */
int bires_psc(const bires_bipoly *f, const bires_bipoly *g, int kind, int var, uint32_t p, uint32_t *out,
              int64_t capacity, int32_t *count, int32_t *points, void *stream);

/* The modular generic-position test of Section 3.2.2 for a curve f with
 * no vertical asymptote (lc_var f constant), with R = res(f, df/dvar; var),
 * its square-free part R* (e.g. the product of bires_squarefree's factors)
 * and deg R, over the one prime p (a library prime, else BIRES_EINVAL):
 *   N^- = sum_{i >= 1} (n - i) deg R_i^(p)                  (eq. lower-bound),
 *   N^+ = deg R* n - deg R + deg gcd(R^inf mod p, Q mod p)   (eq. up-bound),
 * n = deg_var f, R_i^(p) = S_{i-1} / S_i with S_0 = R* mod p and S_i =
 * gcd(S_{i-1}, sr_i(f, df/dvar) mod p), Q = res(df/dother, df/dvar; var) (the
 * case gcd(f_x, f_y) = 1 of the remark after Teissier's lemma), gcd(R^inf, Q)
 * the common factors of R* and Q with their multiplicity in Q.  N^- <= N <=
 * N^+ (N the number of distinct points in the x-critical fibers) when p is
 * not unlucky, and N^- = N^+ certifies n_alpha = n_alpha^+ in every fiber.
 * *flags: bit 0 p divides lc_var f; bit 1 p divides lc(R*); bit 2 Q = 0 mod
 * p; with any bit set the bounds are not certified.  f and rstar are host
 * memory; deg_var f >= 1 (else BIRES_EINVAL). */
int bires_fiber_bounds(const bires_bipoly *f, int var, const bires_upoly *rstar, int32_t deg_r, uint32_t p,
                       int64_t *n_minus, int64_t *n_plus, int32_t *flags, void *stream);

/* Output sizes for gcd(a, b): degree <= min(deg a, deg b); coefficient bits from
 * the Landau-Mignotte bound 2^d * ||a||_2 of a divisor of degree d. */
int bires_gcd_bounds(const bires_upoly *a, const bires_upoly *b, int32_t *max_degree, int32_t *max_limbs);

/* h = gcd(a, b) in Z[x] (Section 5.1, "Computing gcds in Z[x]": Brown's
 * modular method): gcd of the contents times the primitive gcd, positive
 * leading coefficient; gcd(0, 0) = 0, gcd(a, 0) = +-a.  The modular result is
 * certified by exact division on the device; a failed certificate adds primes.
 * Inputs are read-only (bires_upoly.c is not written). */
int bires_gcd(const bires_upoly *a, const bires_upoly *b, bires_upoly *out, int mem, void *stream);

/* Square-free decomposition of r in Z[x] by Yun's algorithm, each step one
 * modular gcd with its exact cofactors (the gcd of Section 5.1; the
 * decomposition is the next step of the curve analysis, whose projection
 * factors the resultant into square-free parts):
 *     r = u * a_1 * a_2^2 * ... * a_k^k,
 * u the signed content of r (degree 0; the zero polynomial when r = 0), each
 * a_i primitive with positive leading coefficient, square-free and coprime to
 * the others (a_i = 1 when r has no factor of multiplicity i), a_k of degree
 * >= 1; k = 0 for constant r.  *count receives k; factors[0..k) receive a_1..a_k
 * (caller-allocated, at most max_factors; k <= deg r).  BIRES_EBUFSIZE when k
 * exceeds max_factors or an output is too small: the needed degree and limbs
 * are written back into that descriptor (sizes of the others are kept), and
 * the call can be repeated.  mem: where the buffers of r, unit and factors live. */
int bires_squarefree(const bires_upoly *r, bires_upoly *unit, bires_upoly *factors, int32_t max_factors,
                     int32_t *count, int mem, void *stream);

/* For callers that cannot allocate (tight serving loops, harnesses that
 * forbid device allocation after start-up): res(f, g; var) for kind
 * BIRES_KIND_RESULTANT, res(f, df/dvar; var) for BIRES_KIND_DISCRIMINANT or
 * res(df/dother, df/dvar; var) for BIRES_KIND_POLAR (g then ignored), with
 * the same arguments, results and errors as bires_resultant /
 * bires_discriminant / bires_polar_resultant, but without allocating: no device or
 * pinned host memory is allocated or freed by the call.  Every device buffer
 * of the call lies in one fixed array of BIRES_NOALLOC_SCRATCH_BYTES that the
 * library holds on its device from set-up until the process ends; host-side
 * bookkeeping uses ordinary heap memory.  The library must already be set up
 * (bires_init() or any earlier call; else BIRES_EINVAL).  A job whose
 * buffers do not fit in the array returns BIRES_ETOOBIG (for scale: a dense
 * total-degree-40 discriminant needs about 5 MB).  All calls share the array
 * and keep its last contents; the library runs them one at a time (a call
 * waits for the one in progress), so concurrent calls never overlap on the
 * device.  Per-job interpolation and, where its operand table was built by an
 * earlier call, the explicit CRT, else Garner's reconstruction; the staged
 * schedule.  Synchronous. */
#define BIRES_NOALLOC_SCRATCH_BYTES (64u << 20)
int bires_resultant_noalloc(const bires_bipoly *f, const bires_bipoly *g, int kind, int var, bires_upoly *out,
                            int mem, void *stream);

/* n independent jobs in one batched launch sequence.  kind[i] is a
 * BIRES_KIND_*; var[i] a BIRES_VAR_*; g[i] is ignored for the kinds that
 * derive both operands from f (discriminant, polar).
 * status[i] receives the per-job code; the return value is BIRES_OK when
 * every job succeeded, else the first failing job's code.  Results equal those
 * of the single-job calls bit for bit. */
int bires_resultant_batch(int n, const bires_bipoly *f, const bires_bipoly *g,
                          const int32_t *kind, const int32_t *var,
                          bires_upoly *out, int32_t *status, int mem, void *stream);

/* Asynchronous form of bires_resultant_batch (same arguments, plus *ticket).
 * The calling thread plans the batch and queues its device work on `stream`
 * (the library stream when NULL), after the work queued there before, and
 * returns without waiting for the device; with device-memory inputs whose
 * plans are reused (bires_set_plan_cache) nothing on the host waits at all.
 * An error found before any device work was queued is returned here and no
 * ticket is issued.  The descriptor, status and output arrays and the input
 * and output buffers must stay valid, and the inputs unchanged, until
 * bires_batch_wait returns for the ticket.  While one batch runs on the
 * device, the caller can plan and queue the next, so the device runs them
 * back to back.  Batches in flight must not share output buffers. */
int bires_resultant_batch_async(int n, const bires_bipoly *f, const bires_bipoly *g, const int32_t *kind,
                                const int32_t *var, bires_upoly *out, int32_t *status, int mem, void *stream,
                                uint64_t *ticket);
/* Blocks until the batch of `ticket` has finished (its outputs are then
 * complete for every stream) and returns what bires_resultant_batch would
 * have; BIRES_EINVAL for an unknown or already collected ticket. */
int bires_batch_wait(uint64_t ticket);

/* ---------------- serving: continuous batching of mixed jobs ---------------- */

typedef struct bires_server bires_server;

/* A server owns a scheduler thread and a stream.  Jobs are admitted while at
 * most max_slots are in flight and their device footprint fits in
 * hbm_budget_bytes; admitted jobs run together in batched launches, and jobs
 * arriving while others run join the next launch.  Residues stay in device
 * memory for a job's whole life. */
int bires_server_create(size_t hbm_budget_bytes, int max_slots, bires_server **out);

/* Copies the (host-memory) inputs and returns at once with a ticket. */
int bires_server_submit(bires_server *s, int kind, int var, const bires_bipoly *f,
                        const bires_bipoly *g, uint64_t *ticket);

/* Blocks until the job is done (timeout_s < 0: no limit), then writes the
 * result to out (host memory) and the submit-to-completion latency, and
 * retires the ticket.  When out is too small (degree capacity below the
 * result's degree, or fewer limbs than its largest coefficient needs) it
 * returns BIRES_EBUFSIZE with the needed degree and limbs written back into
 * out and keeps the ticket, so the caller can wait again with a larger
 * buffer.  A failed job's error code is returned once and retires the ticket;
 * BIRES_ENOTFOUND for an unknown or retired ticket. */
int bires_server_wait(bires_server *s, uint64_t ticket, bires_upoly *out, double timeout_s,
                      double *latency_s);

/* Stops the scheduler after the jobs in flight finish and frees everything. */
int bires_server_destroy(bires_server *s);

/* ---------------- introspection ---------------- */

/* Plan of res(f, g; var) or the discriminant (kind) for host-memory inputs:
 * number of evaluation points D (= degree bound + 1), number of primes P,
 * log2 of the coefficient bound.  Host-only. */
int bires_plan(const bires_bipoly *f, const bires_bipoly *g, int kind, int var,
               int32_t *points, int32_t *primes, double *log2_bound);

/* The first n primes of the table (the largest primes below 2^32/3,
 * descending).  Host-only. */
int bires_primes(int n, uint32_t *out);

/* Values of the univariate resultants res(f(a, y), g(a, y)) mod p_k with the
 * formal degrees kept, for a = 0 .. D-1 and the plan's P primes:
 * values[k * D + a] (host memory, at least P*D words).  A stage-level view of
 * the pipeline for testing. */
int bires_debug_values(const bires_bipoly *f, const bires_bipoly *g, int kind, int var,
                       uint32_t *values, int64_t capacity, int32_t *points, int32_t *primes);

/* Launch schedule of the batched pipeline.
 *   BIRES_SCHEDULE_STAGED: one launch per stage (reduce, evaluation +
 *     elimination per size bucket, interpolation, explicit CRT or mixed
 *     radix and limbs);
 *   BIRES_SCHEDULE_FUSED: the reduction, then every other stage of every job
 *     in one persistent launch, stage after stage; its blocks claim each
 *     stage's tasks from device counters, so no block waits on one that has
 *     not started (the launch may share the device with other work);
 *   BIRES_SCHEDULE_SCHUR: staged, with the evaluation + elimination of the
 *     jobs with 1 <= min(m, n) and m + n <= 128 by the Schur algorithm on the
 *     displacement generators of the Sylvester matrix (Section 5.1, eq.
 *     displ-sylvester), one wavefront per (prime, point) instance;
 *   BIRES_SCHEDULE_AUTO (default): the autotuner's choice for the batch's size
 *     key if it has one, else staged.
 * Results are identical under every schedule.  Process-wide setting. */
#define BIRES_SCHEDULE_STAGED 0
#define BIRES_SCHEDULE_FUSED 1
#define BIRES_SCHEDULE_AUTO 2
#define BIRES_SCHEDULE_SCHUR 3
int bires_set_schedule(int schedule);

/* Evaluation + elimination kernel of the staged schedule.
 *   BIRES_EVAL_AUTO (default): jobs with 1 <= min(m, n) and max(m, n) < 32
 *     (m, n: degrees in the eliminated variable) keep f's coefficient array in
 *     registers; blocks that meet a vanishing leading coefficient or a
 *     degree drop are recomputed by the general kernel; other jobs use it;
 *   BIRES_EVAL_LDS: every job uses the general kernel (both arrays in LDS);
 *   BIRES_EVAL_SCHUR: jobs with 1 <= min(m, n) and m + n <= 128 use the
 *     Schur kernel of BIRES_SCHEDULE_SCHUR (instances whose pivot vanishes mod
 *     p fall back to Euclid), the others as under BIRES_EVAL_AUTO.
 * Results are identical.  Process-wide setting. */
#define BIRES_EVAL_AUTO 0
#define BIRES_EVAL_LDS 1
#define BIRES_EVAL_SCHUR 2
/* (prime, point) instances that batched calls have run on the Schur kernel
 * since set-up, and how many of them met a vanishing pivot and were
 * recomputed by Euclid's algorithm. */
int bires_schur_stats(int64_t *instances, int64_t *fallbacks);
int bires_set_eval_kernel(int kernel);

/* Plan reuse for batched calls with device-memory inputs (default on): when
 * every job of a call is valid and has the same extents, output capacities,
 * kind and variable as in the previous call (buffer addresses may differ),
 * and the last planned calls saw the same row statistics, it keeps their
 * plans and does not wait for its
 * own row scan before launching; a device kernel then compares the scan's
 * output with the statistics those plans came from, word for word, and on any
 * difference the call is rerun with fresh plans before it returns.  Equal
 * statistics give equal plans, so results never depend on the setting.
 * bires_plan_cache_stats: calls that reused plans, and reuses undone by a
 * mismatch, since set-up.  Process-wide. */
int bires_set_plan_cache(int enable);
int bires_plan_cache_stats(int64_t *hits, int64_t *misses);

/* Graph replay: when enabled, batched calls issue their device sequence
 * (metadata upload, the stage kernels of the chosen schedule, status and
 * host-output copies) as a captured HIP graph, one per distinct set of launch
 * arguments (workspace addresses, sizes, grids), replayed by later calls with
 * the same arguments; at most 32 graphs are kept.  Zero fills of special
 * results are issued outside the graph.  Results are identical to eager issue;
 * kernel timing (bires_set_timing) does not cover graph replays.  Disabling
 * waits for the device and destroys the cached graphs.  Process-wide. */
int bires_set_graphs(int enable);
/* Graphs captured and cached graphs replayed since the library was set up. */
int bires_graph_stats(int64_t *captures, int64_t *replays);

/* Autotuner: runs the batch (arguments as bires_resultant_batch) under every
 * schedule (staged, fused, Schur), keeps the fastest (the best of `reps` timed
 * runs of each, in rounds that take the schedules in turn, after one warm-up
 * round) for the batch's size key (total (prime, point) instances, largest
 * degree sum in the eliminated variable, largest prime count, each
 * log2-bucketed), and returns it in *chosen.  BIRES_SCHEDULE_AUTO then uses the table; when the
 * environment variable BIRES_AUTOTUNE_CACHE names a file, the table is loaded
 * from it at set-up and rewritten after every tuning run.  The outputs hold the
 * batch's results afterwards. */
int bires_autotune(int n, const bires_bipoly *f, const bires_bipoly *g, const int32_t *kind, const int32_t *var,
                   bires_upoly *out, int32_t *status, int mem, void *stream, int reps, int32_t *chosen);

/* Kernel timing: when enabled, the library brackets the univariate-resultant
 * launches (staged schedule) or the fused launch with HIP events on its stream
 * and accumulates the durations.  bires_kernel_time returns (milliseconds, launches) since the
 * last reset. */
int bires_set_timing(int enable);
int bires_kernel_time(double *ms, int64_t *launches);

/* Host time of batched calls while timing is enabled, accumulated per phase in
 * microseconds since the last reset (bires_set_timing):
 *   us[0] validation, input layout and staging buffers,
 *   us[1] inputs copied and the row-statistics scan submitted,
 *   us[2] waiting for the statistics (device-memory inputs),
 *   us[3] planning, workspace layout and job descriptors,
 *   us[4] metadata upload and kernel launches,
 *   us[5] waiting for the device, statuses and host outputs.
 * us must hold BIRES_HOST_PHASES doubles; *calls = batched calls timed. */
#define BIRES_HOST_PHASES 6
int bires_host_time(double *us, int64_t *calls);

/* Issue cost of single instructions on the current device, for the
 * roofline: cycles[k] = SIMD clock cycles per wave64 instruction for k = 0..5
 * = v_add_u32, v_min_u32, v_mul_lo_u32, v_mad_u64_u32, v_fma_f64 (each timed
 * over 16 independent chains per lane) and the int8 matrix-core product
 * v_mfma_i32_32x32x32_i8 (four independent accumulators), in 16 blocks of 256
 * threads per CU (best of three launches, HIP events, peak engine clock).
 * n: entries of cycles (at most 6 are written, the rest are zeroed). */
int bires_issue_rates(double *cycles, int n);

/* Properties of the current device as the HIP runtime reports them: compute
 * units, peak engine clock (kHz), LDS bytes per workgroup, HBM bytes. */
int bires_device_info(int32_t *compute_units, int32_t *clock_khz, int64_t *lds_per_block, int64_t *hbm_bytes);

const char *bires_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* BIRES_H */
