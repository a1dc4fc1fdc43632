/*
 * phiks.h -- C ABI of the MI355X (gfx950) library for actions of phi-functions of
 * Kronecker sums.
 *
 * The operation (Caliari, Cassini, Zivcovich, "A mu-mode approach for exponential
 * integrators: actions of phi-functions of Kronecker sums", arXiv 2210.07667):
 *
 *   K = A_d (+) ... (+) A_1 = sum_mu I_d x .. x I_{mu+1} x A_mu x I_{mu-1} x .. x I_1
 *   (eq. kronsum, Section 1), A_mu dense n_mu x n_mu, and
 *   phi_l(X) = int_0^1 theta^(l-1)/(l-1)! exp((1-theta) X) dtheta, phi_0 = exp
 *   (eq. phifunctions).
 *
 * Two tasks (Section 3):
 *   same vector   (eq. diffphi, eq. scaldiffphi): phi_l(2^-j tau K) v, l = 0..p,
 *                 j = 0..n_scales-1;
 *   combination   (eq. lincomb, eq. scallincomb): exp(c_j tau K) v_0 +
 *                 sum_{l=1}^p c_j^l phi_l(c_j tau K) v_l, c_j = 2^-j.
 * K is never formed: every exponential of K is a Tucker operator (chain of mu-mode
 * products, Section 2, eq. tucker) with small exponentials of the B_mu = tau A_mu,
 * inside a Gauss-Lobatto quadrature of the phi integral plus a scaling-and-squaring
 * recurrence (eqs. integrandsimul/simul, integrandcomb/comb).  The scaling s and the
 * number q of quadrature points are chosen from a remainder bound (Section 3.3).
 *
 * Vector layout (Lemma 1, Section 2): a vector of length N = n_1 * ... * n_d is
 * vec(V), stacked by columns: index i_1 runs fastest.  As a row-major array that is
 * the shape (n_d, ..., n_1).  All vectors are float64 in device memory.
 *
 * Conventions for every entry point:
 *   - return PHIKS_OK (0) or a negative status; nothing throws across the ABI;
 *   - every argument is validated before any device work is enqueued;
 *   - device work is enqueued on the given HIP stream (NULL = the null stream) and
 *     is stream-ordered; no entry point synchronises the stream except where noted;
 *   - inputs and outputs are caller-owned device buffers; outputs must not alias
 *     inputs; the library never frees them.
 */
#ifndef PHIKS_H
#define PHIKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct phiks_plan_s* phiks_plan_t;

enum {
  PHIKS_OK = 0,
  PHIKS_EINVAL = -1,      /* invalid argument (shape, count, pointer, task, ...) */
  PHIKS_ENOPLAN = -2,     /* no (s, q) with s <= s_max meets the tolerance */
  PHIKS_ENOMEM = -3,      /* device or host allocation failed */
  PHIKS_EDEVICE = -4,     /* a HIP call failed; phiks_last_error() has the text */
  PHIKS_EWORKSPACE = -5,  /* workspace pointer NULL or ws_bytes too small */
  PHIKS_ENONFINITE = -6,  /* non-finite matrix entry, tau or tolerance */
  PHIKS_ETIMEDOUT = -7    /* a served request's deadline passed before it finished */
};

enum { PHIKS_SAME_VECTOR = 0, PHIKS_LINCOMB = 1 };
/* Arithmetic of the mu-mode products.  PHIKS_FP32: FP32 MFMA products of FP32 copies
 * of the small exponentials, FP32 intermediates between the modes of a Tucker
 * operator.  PHIKS_BF16X3: as PHIKS_FP32, but each product of two FP32 operands is
 * formed from their bfloat16 splits x = hi + lo as hi*hi + hi*lo + lo*hi on BF16 MFMA
 * with FP32 accumulation (each term a*b within 3 * 2^-16 |a b|).  In both, the
 * small exponentials themselves, the quadrature sums, the squaring recurrence and
 * every output stay FP64. */
enum { PHIKS_FP64 = 0, PHIKS_FP32 = 1, PHIKS_BF16X3 = 2 };

#define PHIKS_MAX_D 8      /* largest number of modes d */
#define PHIKS_MAX_P 8      /* largest phi index p */
#define PHIKS_MAX_N 1024   /* largest mode size n_mu */

/*
 * phiks_plan -- choose (s, q) and build the small exponentials.
 *
 * Section 3.3: for s = max(0, n_scales-1), max(0, n_scales-1)+1, ... (up to s_max) take
 * the smallest q in [q_min, q_max] whose quadrature remainder bound (estimate
 * CPestimate over the rectangle Xi = Xi_1 + ... + Xi_d containing the numerical range
 * of tau K, Xi_mu the rectangle of tau A_mu) satisfies
 *   same vector:  b_{q,l}(s) ||v||_2 <= tol 2^(l s),                       l = 1..p
 *   combination:  sum_{k<=l} b_{q,l-k+1}(s) ||v_{p+1-k}||_2 / 2^((l-k+1)s) <= tol
 * and stop before the first s whose Tucker count (eq. Tpsv: q + s p + n_scales;
 * eq. Tlcp: q p + s p + n_scales) is strictly larger than the previous one.
 * q_min, q_max, s_max and the rectangle's kind are the planner options
 * (phiks_planner_options; defaults 3, 12, 64 and the Bendixson rectangle).
 * Then, on the device, the scaling-and-squaring exponentials (degree-24 Taylor)
 * exp((1 - theta_i) tau A_mu / 2^s) for every Gauss-Lobatto node theta_i < 1 and
 * exp(tau A_mu / 2^j) for j = s..0 (by squaring, Section 3.1) are computed.
 *
 *   d         number of modes, 1 <= d <= PHIKS_MAX_D
 *   n         host array of d sizes; n[0] = n_1 is the fastest index;
 *             1 <= n[mu] <= PHIKS_MAX_N
 *   A         host array of d host pointers; A[mu] is A_{mu+1}, row-major
 *             n[mu] x n[mu] float64 (A[i*n + j] multiplies u_j in row i); copied
 *   tau       time step, finite and > 0
 *   p         highest phi index, 0 <= p <= PHIKS_MAX_P (p = 0: exponential only)
 *   n_scales  number of scales 2^-j, j = 0..n_scales-1, 1 <= n_scales <= 16
 *   tol       absolute tolerance delta > 0 (relative when vnorms == NULL)
 *   task      PHIKS_SAME_VECTOR or PHIKS_LINCOMB
 *   vnorms    host array of 2-norms (same vector: 1 value ||v||; combination: p+1
 *             values ||v_0||..||v_p||), or NULL for all norms = 1
 *   precision PHIKS_FP64, PHIKS_FP32 or PHIKS_BF16X3 (see above)
 *   hip_stream stream for the device work (hipStream_t), may be NULL
 *   out       receives the plan; owned by the caller, release with
 *             phiks_plan_destroy.  Its device buffers live on the current device.
 *
 * Errors: EINVAL, ENONFINITE, ENOPLAN (before any device work), ENOMEM, EDEVICE.
 * The plan's matrices are ready in stream order; the call does not synchronise.
 */
int phiks_plan(int d, const int64_t* n, const double* const* A, double tau, int p,
               int n_scales, double tol, int task, const double* vnorms, int precision,
               void* hip_stream, phiks_plan_t* out);

/*
 * phiks_plan_complex -- as phiks_plan for complex A_mu and a complex step tau (the
 * paper admits both; the validation operators of Section 4.1 are complex).  A[mu]
 * is an n[mu] x n[mu] complex matrix, row-major, each entry two float64 (re, im);
 * tau = tau_re + i tau_im, nonzero.  Arithmetic FP64.  With such a plan every vector
 * of phiks_apply / phiks_combine (v, out) holds N complex values as 2N float64
 * (re, im interleaved), in the same index order, and the workspace is doubled.
 * Internally each complex matrix is used in its real form (2 x 2 blocks [[Re, -Im],
 * [Im, Re]]); the quadrature and squaring coefficients are real.
 */
int phiks_plan_complex(int d, const int64_t* n, const double* const* A, double tau_re,
                       double tau_im, int p, int n_scales, double tol, int task,
                       const double* vnorms, void* hip_stream, phiks_plan_t* out);

/*
 * phiks_apply -- same vector (eqs. integrandsimul and simul, multi-scale outputs
 * of eq. scaldiffphi).  Requires a plan made with PHIKS_SAME_VECTOR.
 *
 *   v     device, N float64
 *   out   device, n_scales * (p+1) * N float64;
 *         out[(j*(p+1) + l)*N + k] = (phi_l(2^-j tau K) v)[k], l = 0 is exp
 *   ws    device workspace of at least phiks_workspace_size() bytes
 * Errors: EINVAL (wrong task, NULL pointers), EWORKSPACE, EDEVICE.
 */
int phiks_apply(phiks_plan_t plan, const double* v, double* out, void* ws,
                size_t ws_bytes, void* hip_stream);

/*
 * phiks_apply_noalloc -- phiks_apply for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  No workspace argument: the workspace is a fixed device array of
 * PHIKS_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device, placed there
 * when the library is loaded and held until the process ends.  The call allocates
 * nothing (no hipMalloc / hipFree, no allocating library routine).
 *
 *   plan, v, out, hip_stream  as phiks_apply; results are those of phiks_apply
 * The scratch of the plan's device is used.  Every call on one device shares it and
 * it keeps the last call's contents (nothing in it needs to start at zero): calls
 * that overlap on one device (other streams, other threads) race, and the caller
 * must order them.
 * Errors: EINVAL (wrong task, NULL pointers), EWORKSPACE (phiks_workspace_size of
 * the plan exceeds PHIKS_NOALLOC_SCRATCH_BYTES; checked before any device work),
 * EDEVICE.
 */
#define PHIKS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int phiks_apply_noalloc(phiks_plan_t plan, const double* v, double* out, void* hip_stream);

/*
 * phiks_combine -- linear combination (eqs. integrandcomb and comb, eq. scallincomb).
 * Requires a plan made with PHIKS_LINCOMB.
 *
 *   v     host array of p+1 device pointers v_0..v_p (N float64 each); any entry
 *         may be NULL for a zero vector (v_0 == NULL skips the exponential term)
 *   out   device, n_scales * N float64;
 *         out[j*N + k] = (exp(c_j tau K) v_0 + sum_l c_j^l phi_l(c_j tau K) v_l)[k]
 *   ws    device workspace of at least phiks_workspace_size() bytes
 * Errors: EINVAL, EWORKSPACE, EDEVICE.
 */
int phiks_combine(phiks_plan_t plan, const double* const* v, double* out, void* ws,
                  size_t ws_bytes, void* hip_stream);

/*
 * phiks_tucker -- the Tucker operator of Section 2 (eq. tucker, Lemma 1):
 *   out = vec(V x_1 L_1 x_2 ... x_d L_d) = (L_d x ... x L_1) v
 * with no plan: d mu-mode products on the device.
 *
 *   d, n      as for phiks_plan
 *   L         host array of d device pointers; L[mu] row-major n[mu] x n[mu] float64
 *   v, out    device, N float64 each (out must not alias v)
 *   ws        device workspace of at least 2 * N * sizeof(double) bytes (d >= 2)
 * Errors: EINVAL, EWORKSPACE, EDEVICE.
 */
int phiks_tucker(int d, const int64_t* n, const double* const* L, const double* v,
                 double* out, void* ws, size_t ws_bytes, void* hip_stream);

/* Workspace bytes needed by phiks_apply / phiks_combine for this plan. */
int phiks_workspace_size(phiks_plan_t plan, size_t* bytes);

/*
 * Plan summary: scaling s, quadrature points q, the paper's Tucker count
 * (eq. Tpsv / eq. Tlcp) and the count actually executed (the node theta_q = 1 and,
 * for combinations with v_0 == NULL, the exponential terms need none).
 */
int phiks_plan_info(phiks_plan_t plan, int* s, int* q, int* tucker_paper,
                    int* tucker_exec);

/*
 * phiks_plan_matrix -- copy one of the plan's small exponentials (Section 3.1) into a
 * caller buffer, for inspection:
 *   kind PHIKS_MATRIX_NODE,  0 <= index < q-1 (p > 0):
 *        exp((1 - theta_{index+1}) tau A_mu / 2^s), theta_1 = 0 < ... < theta_q = 1
 *        the Gauss-Lobatto nodes on [0, 1];
 *   kind PHIKS_MATRIX_LEVEL, 0 <= index <= s:  exp(tau A_mu / 2^index).
 *   mu    0-based mode (the matrix of A_{mu+1})
 *   dst   device, n[mu]^2 float64, row-major (complex plans: the real form, 2n x 2n,
 *         2 x 2 blocks [[Re, -Im], [Im, Re]], 4 n[mu]^2 float64)
 * Stream-ordered device-to-device copy.  Errors: EINVAL, EDEVICE.
 */
enum { PHIKS_MATRIX_NODE = 0, PHIKS_MATRIX_LEVEL = 1 };
int phiks_plan_matrix(phiks_plan_t plan, int mu, int kind, int index, double* dst,
                      void* hip_stream);

/*
 * Release a plan.  Stream-ordered: its device memory is freed (hipFreeAsync) and its
 * host staging buffers are released after all work already enqueued on the stream the
 * plan was made with; the call itself does not wait.  Work using the plan that was
 * enqueued on other streams must be ordered before that point by the caller (e.g. an
 * event), and the plan's stream must still exist.  NULL is a no-op.
 */
void phiks_plan_destroy(phiks_plan_t plan);

/*
 * Kernel timing for measurement: while enabled, every mu-mode product kernel launch
 * is bracketed by HIP events recorded on the launch stream.  phiks_kernel_timing_read
 * waits for the recorded launches, returns the summed kernel time (ms), the number
 * of launches and their algorithmic flops (2 * rows * cols * contraction length per
 * product), and clears the record.  Kernels of one stream never overlap, so a launch
 * whose start stamp precedes the end of the previous timed launch on its stream is
 * counted from that end (an upper bound on its duration).
 */
int phiks_kernel_timing(int enable);
int phiks_kernel_timing_read(double* total_ms, int64_t* launches, double* flops);

/*
 * Batches of independent problems (same-vector task, eqs. integrandsimul / simul with
 * the outputs of eq. scaldiffphi): many small problems of different shapes whose
 * separate calls would each be too small to fill the GPU.
 *
 * phiks_batch_plan -- plan `count` problems at once.  Problem i has d[i] modes of
 * sizes n[i][0..d[i]-1], host matrices A[i][mu] (row-major, copied) and step tau[i];
 * p, n_scales, tol and precision are shared.  vnorms: host array of count values
 * ||v_i||_2, or NULL (norms 1).  Each problem gets exactly the (s, q) phiks_plan would
 * choose for it; the small exponentials of all problems are built in one device pass.
 * precision: PHIKS_FP64, or PHIKS_FP32 (FP32-MFMA mu-mode products; every product of a
 * problem then runs in the tile and kernel its single FP32 call gives it, so the
 * outputs are bitwise that call's).  Errors as phiks_plan; a failing problem is named in
 * phiks_last_error().
 *
 * phiks_batch_apply -- v: host array of count device pointers (N_i doubles each);
 * out: host array of count device pointers, out[i] laid out as phiks_apply's out for
 * problem i.  ws: device workspace of phiks_batch_workspace_size bytes, 16-byte
 * aligned.  Every out[i] is bitwise what phiks_apply returns for problem i alone.
 * Stream-ordered; calls on one batch must not overlap (they share its launch tables,
 * and a call waits on the host until the previous call's table upload has run).
 * The launches depend only on the batch and the pointers (v, out, ws): the second
 * call with one pointer set captures them into a HIP graph, and later calls with the
 * same set replay it (one graph launch, no host scheduling).  A call with other
 * pointers, or with kernel timing on, runs eagerly and drops the graph; dropping it
 * waits on the host until the graph's last launch has finished.
 */
typedef struct phiks_batch_s* phiks_batch_t;

int phiks_batch_plan(int count, const int* d, const int64_t* const* n,
                     const double* const* const* A, const double* tau, int p, int n_scales,
                     double tol, const double* vnorms, int precision, void* hip_stream,
                     phiks_batch_t* out);
int phiks_batch_apply(phiks_batch_t batch, const double* const* v, double* const* out,
                      void* ws, size_t ws_bytes, void* hip_stream);
int phiks_batch_workspace_size(phiks_batch_t batch, size_t* bytes);
/* (s, q, T# of eq. Tpsv, Tucker operators executed) of problem i. */
int phiks_batch_info(phiks_batch_t batch, int i, int* s, int* q, int* tucker_paper,
                     int* tucker_exec);
/* Stream-ordered release, as phiks_plan_destroy. */
void phiks_batch_destroy(phiks_batch_t batch);

/*
 * phiks_batch_tuning -- the rules that pick the tile class of the batched path's grouped
 * FP64 products (host only).  params[0..4]: the side from which 64 x 64 tiles are used
 * (1..128), and 0/1 switches for the skinny 32 x 128 / 128 x 32 classes, 128 x 64 tiles for
 * mode-1 plain stores, for plain stores of modes > 1, and for the squaring epilogue (each
 * with M >= 128, N >= 64).  set = 0 reads them into params; set = 1 replaces them (a
 * batch's captured graph is then rebuilt on its next calls) and reads them back.  The
 * built-in values are those tune_batch.py recorded for the batched workload.  Every
 * choice gives bitwise the same results (one k order in every FP64 kernel and tile).
 * PHIKS_EINVAL for out-of-range values.
 */
int phiks_batch_tuning(int set, int* params);

/*
 * phiks_batch_dryrun -- host only (no device, nothing launched): builds the launch
 * schedule phiks_batch_apply would issue for `count` problems of shapes d[i], n[i][..]
 * with plans (s[i], q[i]) and the given p, n_scales (FP64), and its fork plan over
 * fork_streams capture streams, on synthetic device addresses (each buffer a region
 * followed by a gap), and checks them: every operand range of every launch-table item
 * inside one buffer of its own problem, tile counts and first-tile offsets consistent,
 * every mu-mode product of every problem scheduled once (d (1 + s + n_scales) of them
 * for p > 0, d n_scales for p = 0), and the fork plan's events recorded before they are
 * waited for, indices in range, each launch issued once in step order.  Writes the
 * launch count, the table bytes and the number of failed checks (the first described
 * by phiks_last_error()).  PHIKS_EINVAL for invalid shapes or plans.
 */
int phiks_batch_dryrun(int count, const int* d, const int64_t* const* n, const int* s,
                       const int* q, int p, int n_scales, int fork_streams, int64_t* launches,
                       int64_t* table_bytes, int64_t* violations);

/*
 * Serving: phi-action requests (same vector, eq. scaldiffphi) submitted one at a time
 * and run by step-level continuous batching.
 *
 * Requests are routed by size to `lanes` lanes (phiks_server_lane), each with its own
 * stream.  In a lane, requests are admitted in arrival order as soon as a workspace
 * slot of the arena is free for them (a slot per request, allocated on admission,
 * released on completion) and fewer than max_active of the lane's requests run; the
 * lane then issues ticks, each one step of every running request (an FP64 mu-mode
 * product or node-sum pass, grouped across the requests into shared launches; for
 * FP32 / BF16x3 requests one Tucker operator).  A request submitted while others run
 * joins its lane at the next tick, and the lanes' work overlaps on the device.  Every
 * result is bitwise what phiks_plan (tolerance relative, vnorms = NULL) + phiks_apply
 * return for that request alone.
 *
 * phiks_server_create -- hbm_budget: device bytes for cached plans plus the workspace
 * arena; workspace_bytes: the arena (a request whose workspace, computed for the
 * largest q, exceeds it is refused with PHIKS_EWORKSPACE); max_active: most requests
 * running per lane; lanes: 1..PHIKS_SERVER_MAX_LANES.  Creates the lanes' streams and
 * a worker and a completion thread per lane.
 *
 * phiks_server_register -- copies the host matrices A_1..A_d (as phiks_plan) once and
 * returns an operator id for submit.  Operators stay registered until destroy.
 *
 * phiks_server_submit -- one request on a registered operator: tau, p, n_scales, tol
 * as phiks_plan (tolerance relative: norms taken as 1), precision PHIKS_FP64 /
 * PHIKS_FP32 / PHIKS_BF16X3, timeout_s (seconds from submission, >= 0; 0 = no
 * deadline), v (device, N doubles) and out (device, n_scales*(p+1)*N doubles, laid out
 * as phiks_apply's out).  v and out must stay valid until phiks_server_wait returns for
 * the ticket.  Validation errors are returned here, before anything is queued.  A
 * request still queued at its deadline completes with PHIKS_ETIMEDOUT without running
 * (out untouched); one running at its deadline is issued no further step and completes
 * with PHIKS_ETIMEDOUT once its steps already issued are done (out then holds partial
 * results).  Plans are cached on (operator, tau, p, n_scales, tol,
 * precision); least recently used plans that no running request holds are evicted when
 * the cache would exceed hbm_budget - workspace_bytes.
 *
 * phiks_server_wait -- blocks until the request is done, returns its status (the
 * result is then in out), its latency in seconds (submission to completion) and its
 * completion time on the phiks_server_clock() clock (either pointer may be NULL); the
 * ticket is then released.
 *
 * phiks_server_destroy -- runs everything still queued, waits for it, frees.
 */
#define PHIKS_SERVER_MAX_LANES 4
typedef struct phiks_server_s* phiks_server_t;
typedef struct {
  int64_t completed;     /* requests finished (any status) */
  int64_t ticks;         /* ticks issued (all lanes) */
  int64_t cache_hits;
  int64_t cache_misses;
  int64_t evictions;
  int64_t cache_bytes;   /* device bytes of the cached plans */
  int64_t cached_plans;
  int64_t timed_out;     /* requests completed with PHIKS_ETIMEDOUT */
} phiks_server_stats_t;

int phiks_server_create(size_t hbm_budget, size_t workspace_bytes, int max_active, int lanes,
                        phiks_server_t* out);
int phiks_server_register(phiks_server_t server, int d, const int64_t* n,
                          const double* const* A, int64_t* op_id);
int phiks_server_submit(phiks_server_t server, int64_t op_id, double tau, int p, int n_scales,
                        double tol, int precision, double timeout_s, const double* v,
                        double* out, int64_t* ticket);
int phiks_server_wait(phiks_server_t server, int64_t ticket, double* latency_s, double* done_s);
int phiks_server_stats(phiks_server_t server, phiks_server_stats_t* out);
void phiks_server_destroy(phiks_server_t server);
/* Seconds on the monotonic clock of the server's time stamps. */
double phiks_server_clock(void);

/*
 * The server's policy, host only (no device work; for tests without a GPU).
 *
 * phiks_server_lane -- the lane of a request of n_values values among `lanes`: lane 0
 * up to 2^18 values, then one lane per factor 8 (capped at lanes - 1).  Returns the
 * lane, or PHIKS_EINVAL for n_values < 1 or lanes < 1.
 *
 * phiks_server_select_evictions -- plans to evict before a new plan of new_bytes
 * joins a cache holding cache_bytes with room for capacity bytes; entry i holds
 * bytes[i], is held by refs[i] admitted requests and was last used at tick
 * last_use[i].  Unreferenced entries, least recently used first, until the new plan
 * fits; none beyond the unreferenced ones (the cache then runs over its budget).
 * Writes the chosen indices, in eviction order, to victims (room for count) and their
 * number to nvictims.  PHIKS_EINVAL for a negative count or a NULL array that count
 * requires, else PHIKS_OK.
 */
int phiks_server_lane(int64_t n_values, int lanes);
int phiks_server_select_evictions(int count, const size_t* bytes, const int* refs,
                                  const uint64_t* last_use, size_t cache_bytes, size_t new_bytes,
                                  size_t capacity, int* victims, int* nvictims);

/*
 * Elementwise device vector operations for time integrators built on the phi-actions
 * (the nonlinear terms and stage combinations of the exponential integrators of
 * Section 4): out[k] for k < n, with y[k] read as 0 when y is NULL.
 *   PHIKS_VOP_AXPBY     a x + b y
 *   PHIKS_VOP_RATIONAL  a / (1 + (b x)^2) + y
 *   PHIKS_VOP_CUBIC     a (x - x^3) + b y
 *   PHIKS_VOP_BRUSS_U   a + x^2 y       (Brusselator reaction of u, x = u, y = v; b unused)
 *   PHIKS_VOP_BRUSS_V   a x - x^2 y     (Brusselator reaction of v, x = u, y = v; b unused)
 * x, y, out: device arrays of n doubles; out may alias x or y.  Stream-ordered.
 */
enum { PHIKS_VOP_AXPBY = 0, PHIKS_VOP_RATIONAL = 1, PHIKS_VOP_CUBIC = 2, PHIKS_VOP_BRUSS_U = 3,
       PHIKS_VOP_BRUSS_V = 4 };
int phiks_vector_op(int op, int64_t n, double a, const double* x, double b, const double* y,
                    double* out, void* hip_stream);

/*
 * Device-memory plumbing for callers without their own allocator (the Python
 * binding and the tests use these, so that one HIP runtime -- the one this library
 * was built against -- serves the whole process).  Copies are synchronous.
 */
int phiks_device_count(int* count);            /* 0 when no GPU is visible */
int phiks_device_alloc(size_t bytes, void** ptr);
int phiks_device_free(void* ptr);
int phiks_memcpy_htod(void* dst, const void* src, size_t bytes);
int phiks_memcpy_dtoh(void* dst, const void* src, size_t bytes);
int phiks_memcpy_dtod(void* dst, const void* src, size_t bytes, void* hip_stream); /* async */
int phiks_device_synchronize(void);

/*
 * Stream plumbing for the same callers (one HIP runtime for the process).  Streams
 * are created non-blocking at the default priority on the current device.
 * phiks_stream_order: work enqueued on `then` after this call waits for all work
 * enqueued on `first` before it (an event recorded on `first`, waited on by `then`;
 * neither stream is synchronised with the host).  NULL is the null stream.
 */
int phiks_stream_create(void** stream);
int phiks_stream_destroy(void* stream);        /* NULL: no-op */
int phiks_stream_order(void* first, void* then);
int phiks_stream_synchronize(void* stream);

/* Static text for a status code. */
const char* phiks_status_string(int status);

/* Text of the last failure on the calling thread ("" if none). */
const char* phiks_last_error(void);

/*
 * Host-only helpers (no device work; usable without a GPU).  They expose the
 * planning steps of Section 3.3 for inspection and testing.
 */

/* The (s, q, T#) that phiks_plan would choose; arguments as for phiks_plan. */
int phiks_plan_params(int d, const int64_t* n, const double* const* A, double tau,
                      int p, int n_scales, double tol, int task, const double* vnorms,
                      int* s, int* q, int* tucker_paper);
/* The (s, q, T#) that phiks_plan_complex would choose. */
int phiks_plan_params_complex(int d, const int64_t* n, const double* const* A, double tau_re,
                              double tau_im, int p, int n_scales, double tol, int task,
                              const double* vnorms, int* s, int* q, int* tucker_paper);

/* Gauss-Lobatto-Legendre rule on [0,1] with q points, 2 <= q <= 12:
 * theta[0] = 0 < ... < theta[q-1] = 1 and weights w (host arrays of q doubles). */
int phiks_gll(int q, double* theta, double* w);

/* Bendixson rectangle of the n x n row-major host matrix B: re_lo, re_hi, im_lo,
 * im_hi (xi[0..3]) of [lambda(H)] x i[lambda(S)], H = (B+B^T)/2, S = (B-B^T)/(2i). */
int phiks_rectangle(int64_t n, const double* B, double* xi);

/* Planner options (Section 3.3: q is searched over 3..12 and s upward from n_scales - 1
 * until the Tucker count grows; the rectangle covering the numerical range of each A_mu
 * is to be built from its Hermitian and skew-Hermitian parts, with no construction
 * fixed).  Two readings of that rectangle:
 *   PHIKS_RECT_BENDIXSON      [lambda_min(H), lambda_max(H)] x i[lambda_min(G),
 *                             lambda_max(G)], H = (B+B^*)/2, G = (B-B^*)/(2i): the
 *                             tightest axis-aligned box around W(B) (default);
 *   PHIKS_RECT_NORM_CENTERED  the box centred at sigma = tr(B)/n (the shift of the
 *                             remark in Section 3.1) with half-widths
 *                             ||H - Re(sigma) I||_2 and ||G - Im(sigma) I||_2; it
 *                             contains the Bendixson box. */
enum { PHIKS_RECT_BENDIXSON = 0, PHIKS_RECT_NORM_CENTERED = 1 };

typedef struct phiks_planner_options_s {
  int q_min;  /* smallest q tried, >= 3 */
  int q_max;  /* largest q tried, q_min <= q_max <= 12 */
  int s_max;  /* largest s tried, 0..64; no feasible s <= s_max gives PHIKS_ENOPLAN */
  int rect;   /* PHIKS_RECT_BENDIXSON or PHIKS_RECT_NORM_CENTERED */
} phiks_planner_options_t;

/* phiks_planner_options -- reads and/or replaces the process-wide planner options that
 * every later plan uses (phiks_plan, phiks_plan_complex, phiks_plan_params*,
 * phiks_batch_plan, the server's plans; existing plans keep their (s, q)).
 *   set  host struct, or NULL to leave the options unchanged.
 *   get  host struct receiving the options in force before this call, or NULL.
 * Defaults: q 3..12, s_max 64, Bendixson.  At the first plan or options call the
 * environment variables PHIKS_QMIN, PHIKS_QMAX, PHIKS_SMAX (integers) and
 * PHIKS_PLAN_RECT (bendixson | normcentered) override them; a malformed or out-of-range
 * setting keeps the defaults and makes every plan, and this call with set == NULL,
 * return PHIKS_EINVAL until a valid `set` replaces it.  Returns PHIKS_EINVAL (nothing
 * changed) for an invalid `set`.  Thread-safe; the server's plan cache does not reuse
 * plans made under earlier options. */
int phiks_planner_options(const phiks_planner_options_t* set, phiks_planner_options_t* get);

/* The rectangle of kind `rect` (PHIKS_RECT_*) of the n x n row-major host matrix B:
 * re_lo, re_hi, im_lo, im_hi in xi[0..3]. */
int phiks_range_rectangle(int64_t n, const double* B, int rect, double* xi);

/* Remainder bound of estimate (CPestimate) at one point w = w_re + i w_im of the
 * numerical range: |R_q(f_l(., w))| for l = 1..p written to err[0..p-1], computed
 * as the contour integral over an ellipse with foci 0 and 1 of the kernel k_q
 * (Section 3.3), without the factor (1 + sqrt 2). */
int phiks_remainder(int q, int p, double w_re, double w_im, double* err);

#ifdef __cplusplus
}
#endif

#endif /* PHIKS_H */
