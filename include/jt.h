/*
 * jt.h -- C ABI of the MI355X fast multi-dimensional Jacobi transform.
 *
 * The library applies the uniform forward and inverse Jacobi polynomial
 * transform on tensor-product Gauss-Jacobi grids in 1, 2 or 3 dimensions, by
 * the method of Bremer, Pang and Yang, "Fast algorithms for the
 * multi-dimensional Jacobi polynomial transform" (arXiv:1901.07275):
 *
 *   * 1D (Section 3.1, eqs. (35)-(39)): the orthogonal n x n matrix W J with
 *     (W J)_{jk} = sqrt(w_j) Ptilde_k(t_j) = sqrt(omega_j) phat_k(x_j), where
 *     x_j = cos t_j are the Gauss-Jacobi nodes for (1-x)^a (1+x)^b ordered by
 *     ascending t, omega_j the Gauss-Jacobi weights and phat_k the
 *     orthonormal Jacobi polynomials.  It is applied as the direct block of
 *     degrees < 27 plus r diagonally scaled inverse FFTs (eq. (50)); the
 *     inverse is the transpose (eq. (51)).
 *   * dD (Sections 3.2-3.3, eqs. (54), (55), (59), (60)): the Kronecker
 *     product of the per-axis matrices, applied axis by axis.
 *
 * Conventions shared by every entry point
 *   - Tensors are contiguous, row-major, shape (n[0], ..., n[d-1]).  Axis i
 *     uses the parameters (n[i], a[i], b[i]).  Element [k0, k1, ...] of a
 *     coefficient tensor multiplies phat_{k0} (x) phat_{k1} (x) ...; element
 *     [j0, j1, ...] of a value tensor is the weighted value at the node tuple
 *     (t_{j0}, t_{j1}, ...).
 *   - forward: g = (W0 J0 (x) W1 J1 (x) ...) alpha.
 *     inverse: alpha = (W0 J0 (x) W1 J1 (x) ...)^T g.  Both are orthogonal.
 *   - Device buffers are owned by the caller.  The library never allocates
 *     device memory; it allocates host memory only inside jt_plan*.
 *   - Every call returns a jt_status; no exception crosses the ABI.  On error
 *     jt_last_error() returns a message for the calling thread.  Kernel
 *     launch failures are reported as JT_EDEVICE; faults during execution
 *     surface at the caller's next synchronisation on the stream.
 *   - A plan is immutable after jt_plan_bind; a bound plan may be used from
 *     several streams at once (kernels only read the bound factors).
 */
#ifndef JT_H
#define JT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jt_plan_s *jt_plan_t;

typedef enum {
    JT_OK = 0,
    JT_EINVAL = 1,         /* invalid argument */
    JT_ENOMEM = 2,         /* host allocation failed, or a device buffer is too small */
    JT_EDEVICE = 3,        /* HIP runtime or kernel-launch error */
    JT_ENOTCONV = 4,       /* node search or randomized SVD did not converge */
    JT_EUNSUPPORTED = 5,   /* size/precision combination not built */
    JT_ESTATE = 6          /* plan not bound to device memory */
} jt_status;

typedef enum { JT_F64 = 0, JT_F32 = 1 } jt_dtype;

typedef enum {
    JT_PREC_FP64 = 0,      /* fp64 factors, twiddles, FFTs and accumulation */
    JT_PREC_FP32_BULK = 1  /* fp32 factors, twiddles and FFTs; fp64 rank-sum accumulation.
                              Phases and bins are always fixed on the host in fp64/long double. */
} jt_prec;

typedef enum { JT_FORWARD = 0, JT_INVERSE = 1 } jt_direction;

/* Optional planning knobs; jt_plan() uses the defaults listed here. */
typedef struct {
    int nu0;          /* width of the direct (low-degree) block; default 27 (Section 3.1);
                         at most 64 (JT_EINVAL above) */
    int dense_below;  /* n below this (and at most 1024) keeps the whole matrix: the dense
                         matrix-core pass, no FFT terms; default 64 */
    int oversample;   /* q of Algorithm 2.1; default 2 */
    int iterations;   /* repetitions of steps 2-3 of Algorithm 2.1; default 2 (Section 2.1) */
    uint64_t seed;    /* 0: derived from (n, a, b, tol), so plans are reproducible */
    int kind;         /* 0 or 1: the transform of the modified Jacobi functions of the first
                         kind Ptilde_k; 2: of the second kind Qtilde_k (Section 1; Section 3:
                         "the transform for Qtilde is similar"), read as
                         Qtilde_k(t) = sqrt(sin t / w(x)) q_k(x) / pi with q_k the finite
                         Hilbert transform of w phat_k, i.e. the imaginary part of W B of
                         eq. (45) before the DFT phase.  A second-kind plan has only the
                         forward transform (its matrix is not orthogonal) */
    int planner;      /* how the host finds the nodes, the weights and the sampled columns of
                         Algorithm 2.1: 0 = automatic (phase functions from 1024 points on
                         where they apply), 1 = the three-term recurrence throughout (exact
                         evaluation, O(n^2)), 2 = the nonoscillatory phase and amplitude
                         functions of Section 2.2 wherever they apply: uniform plans with
                         |a|, |b| < 1/2 and tol >= 1e-8.  They are tabulated on the paper's
                         piecewise Chebyshev grid by the third-order ODE for N = M^2 (eq.
                         (phase:Neq)) and spectral integration of psi' = W / N, and read by
                         barycentric interpolation (eq. (cheby:bary)); the nodes solve
                         psi = pi/2 (mod pi) and the weights are pi / psi'.  Sampled rows
                         and the direct block always come from the recurrence */
} jt_plan_options;

/* Per-axis facts about a plan. */
typedef struct {
    int n;            /* points and degrees on this axis */
    int L;            /* FFT length: smallest power of two >= max(n, 64) */
    int nu0;          /* direct-block width */
    int rank;         /* r: number of FFTs per line (eq. (50)) */
    int max_per_bin;  /* most nodes sharing one DFT bin [t_j L / 2 pi] */
    int rsvd_rounds;  /* rank-growth rounds Algorithm 2.1 needed */
    double rel_err;   /* measured ||W B - sum_l u_l v_l^T||_F / ||W B||_F */
    double fro;       /* ||W B||_F */
    int planner;      /* 1: recurrence throughout; 2: phase functions gave the nodes, weights
                         and sampled columns (jt_plan_options.planner) */
} jt_axis_info;

/*
 * Build a plan on the host (fp64 / long double).  For each axis: Gauss-Jacobi
 * nodes and weights (eq. (2), eq. (9)), DFT bins (eq. (45)), the direct block,
 * and the rank-r factors of the weighted low-rank matrix W B (eq. (45)) by
 * Algorithm 2.1 (randomized sampling, pivoted QR/LQ, middle matrix, SVD), with
 * the rank grown until the relative Frobenius error is at most tol.
 *   d    : 1, 2 or 3
 *   n    : d sizes, 1 <= n[i] <= 16384
 *   a, b : d Jacobi parameters each, in (-1, 1) (the paper's analysis covers
 *          (-1/2, 1/2); its experiments also use (-1, 1))
 *   tol  : low-rank relative tolerance, in [1e-14, 1e-2]
 *   out  : receives the plan handle (owned by the caller; free with jt_plan_destroy)
 * Errors: JT_EINVAL (bad argument), JT_ENOMEM, JT_ENOTCONV.
 */
jt_status jt_plan(int d, const int *n, const double *a, const double *b, double tol, jt_plan_t *out);

/* As jt_plan, with explicit options (opt may be NULL for the defaults). */
jt_status jt_plan_ex(int d, const int *n, const double *a, const double *b, double tol,
                     const jt_plan_options *opt, jt_plan_t *out);

/*
 * Plan the nonuniform forward transform at given points (Section 3.1, the
 * remark on nonuniform transforms after eq. (39) and after eq. (51); Sections
 * 3.2-3.3 for 2D and 3D): along axis i, f_j = sum_k alpha_k Ptilde_k(t_{i,j})
 * with the modified Jacobi functions Ptilde_k(t) = sqrt(w(cos t) sin t)
 * phat_k(cos t) (Section 1) and no quadrature weights, computed like the
 * uniform transform (direct block of low degrees plus r scaled FFTs, eq.
 * (50)) with the DFT bins [t_j L / 2 pi] of the given points.
 *   d, n, a, b, tol, opt : as jt_plan_ex; axis i has n[i] points and n[i]
 *                          coefficients (the square transform of the paper)
 *   t    : the points of every axis concatenated (sum of n[i] values, host
 *          fp64), each axis' points non-decreasing and inside (0, pi)
 * Only jt_forward (and jt_apply_axis / batch items in the forward direction)
 * accept such a plan: its inverse is an ill-conditioned solve, not the
 * transpose, and the transpose calls return JT_EUNSUPPORTED.  jt_plan_nodes
 * returns the points, their cosines and omega = 0.
 * Errors: JT_EINVAL (bad argument, points outside (0, pi) or decreasing),
 * JT_ENOMEM, JT_ENOTCONV.
 */
jt_status jt_plan_points(int d, const int *n, const double *t, const double *a, const double *b, double tol,
                         const jt_plan_options *opt, jt_plan_t *out);

/* Release a plan (host memory only; the caller still owns the bound device buffer).
 * NULL is accepted. */
jt_status jt_plan_destroy(jt_plan_t plan);

/* Number of axes of the plan. */
jt_status jt_plan_dims(jt_plan_t plan, int *d);

/* Per-axis facts (axis in [0, d)). */
jt_status jt_plan_info(jt_plan_t plan, int axis, jt_axis_info *info);

/* Copy the axis' nodes t_j (ascending), x_j = cos t_j and Gauss-Jacobi weights
 * omega_j into caller host arrays of length n.  Any pointer may be NULL.
 * The nodes are the n zeros of the degree-n Jacobi polynomial for the weight
 * (1-x)^a (1+x)^b and omega_j the weights of the n-point Gauss-Jacobi rule
 * (Section 2, eq. (2); Section 3.1, eq. (35)), in the order of ascending
 * t_j = arccos x_j; the trigonometric weights of eq. (9) are
 * w_j = omega_j / ((1-x_j)^a (1+x_j)^b sin t_j).
 * Errors: JT_EINVAL (null plan or axis out of range). */
jt_status jt_plan_nodes(jt_plan_t plan, int axis, double *t, double *x, double *omega);

/* Copy the axis' factors to caller host arrays (any pointer may be NULL):
 *   bins : n int32, m_j = [t_j L / 2 pi] in [0, L/2] (eq. (45), eq. (47))
 *   wv   : nu0 * n fp64, wv[k*n + j] = sqrt(omega_j) phat_k(x_j) (direct block)
 *   u    : rank * n complex fp64 (re, im interleaved), u[l*n + j] = (W U S^1/2)_{j,l}
 *   v    : rank * (n - nu0) complex fp64, v[l*(n-nu0) + c] = (S^1/2 V)_{l,c},
 *          column c standing for degree nu0 + c (eq. (49)). */
jt_status jt_plan_factors(jt_plan_t plan, int axis, int32_t *bins, double *wv, double *u, double *v);

/* Exact entries of W B (eq. (45), weights folded in) at (row j, degree k),
 * nu0 <= k < n, computed on the host in long double; out holds count complex
 * values (re, im interleaved).  For diagnostics. */
jt_status jt_plan_entries(jt_plan_t plan, int axis, int count, const int *rows, const int *degrees,
                          double *out);

/* Bytes of device memory the bound factors need. */
jt_status jt_plan_device_bytes(jt_plan_t plan, size_t *bytes);

/* Copy the packed factors into the caller's device buffer dev_buf (at least
 * jt_plan_device_bytes bytes, 256-byte aligned) with one copy enqueued on
 * `stream` (a hipStream_t; NULL = default stream), then wait for that stream
 * (the copy reads the plan's host image), so the call returns with the
 * stream drained.  The plan keeps the pointer; the buffer must stay
 * allocated and unmodified while the plan is used.
 * Errors: JT_EINVAL, JT_ENOMEM (buffer too small), JT_EDEVICE. */
jt_status jt_plan_bind(jt_plan_t plan, void *dev_buf, size_t bytes, void *stream);

/* Copy the packed factor image (jt_plan_device_bytes bytes) into caller host
 * memory, for callers that move it to the device themselves or want to check
 * a bound copy.  Errors: JT_EINVAL, JT_ENOMEM (buffer too small). */
jt_status jt_plan_pack(jt_plan_t plan, void *host_dst, size_t bytes);

/* Device workspace a transform needs beyond its input and output: always 0
 * (every axis pass works in place on the output buffer). */
jt_status jt_workspace_bytes(jt_plan_t plan, jt_prec prec, size_t *bytes);

/*
 * Forward transform g = (W0 J0 (x) ... ) alpha on device buffers: the
 * uniform forward Jacobi transform of Section 3.1 (eqs. (35)-(39): g_j =
 * sqrt(w_j) sum_k alpha_k Ptilde_k(t_j), the values of the expansion at the
 * Gauss-Jacobi nodes weighted by the square roots of the quadrature weights),
 * computed per line as eq. (50), and along every axis for d = 2, 3
 * (Section 3.2, eq. (54); Section 3.3, eq. (59)).
 *   alpha_dev : input, prod n[i] elements of dtype `in`
 *   g_dev     : output, prod n[i] elements of dtype `out`; may equal alpha_dev
 *               only when in == out
 *   prec      : arithmetic of the FFT bulk (jt_prec)
 *   stream    : hipStream_t to launch on (NULL = default stream)
 * One kernel launch per axis (axes d-1, ..., 0), no host synchronisation.
 * With d > 1 the intermediate results live in g_dev, in dtype `out`.
 * Errors: JT_EINVAL, JT_ESTATE (not bound), JT_EUNSUPPORTED, JT_EDEVICE.
 */
jt_status jt_forward(jt_plan_t plan, const void *alpha_dev, jt_dtype in, void *g_dev, jt_dtype out,
                     jt_prec prec, void *stream);

/* Inverse transform alpha = (W0 J0 (x) ... )^T g on device buffers: the
 * transpose of the forward map, which is its inverse because W J is
 * orthogonal (Section 3.1: eq. (51) per line; Section 3.2, eq. (55);
 * Section 3.3, eq. (60)).  Same argument rules and errors as jt_forward. */
jt_status jt_inverse(jt_plan_t plan, const void *g_dev, jt_dtype in, void *alpha_dev, jt_dtype out,
                     jt_prec prec, void *stream);

/* One axis pass only: applies W_i J_i (JT_FORWARD) or its transpose
 * (JT_INVERSE) along axis `axis` of the full tensor.  in_dev and out_dev may be
 * the same buffer (in place) when in == out.  Same errors as jt_forward. */
jt_status jt_apply_axis(jt_plan_t plan, int axis, jt_direction dir, const void *in_dev, jt_dtype in,
                        void *out_dev, jt_dtype out, jt_prec prec, void *stream);

/* ----------------------------------------------------------------------
 * Many plans at once.  Builds `count` plans on the host, one host thread per
 * plan (the plans of a batch of independent transforms, Section 3 applied to
 * each item).
 *   dims   : count entries in {1, 2, 3}
 *   n, a, b: the items' axis parameters concatenated (sum of dims entries);
 *            item i uses entries s_i .. s_i + dims[i] - 1, s_i = dims[0] + ... + dims[i-1]
 *   tol    : as jt_plan (one tolerance for the whole batch)
 *   opt    : NULL, or count option structs (one per item)
 *   plans  : receives count handles (each freed with jt_plan_destroy)
 * On error no handle is returned (all are freed) and jt_last_error names the item.
 */
jt_status jt_plan_many(int count, const int *dims, const int *n, const double *a, const double *b,
                       double tol, const jt_plan_options *opt, jt_plan_t *plans);

/* ----------------------------------------------------------------------
 * Batched form: many independent transforms (uneven n, d, (a, b); forward or
 * inverse) in ONE persistent kernel launch that takes work units from a
 * device queue.  Every axis pass of every item is cut into units of a few
 * lines; a block takes the next unit from an atomic head counter; a unit of
 * an item's later pass waits (bounded, on a device counter) for that item's
 * previous pass.  The unit table lives in a caller-owned device buffer.
 */
typedef struct jt_batch_s *jt_batch_t;

typedef struct {
    int max_split;     /* largest rank split S (groups sharing a line set); 0 = 16 */
    int min_units;     /* raise S until a pass has at least this many units; 0 = 1 */
    int grid;          /* persistent blocks; 0 = one per compute unit */
} jt_batch_options;

typedef struct {
    int units;         /* work units in the queue */
    int passes;        /* axis passes (sum of item dims) */
    int grid;          /* blocks of the persistent launch */
    int threads;       /* threads per block (1024 for fp32, 512 for fp64) */
    size_t lds_bytes;  /* dynamic LDS per block */
    double cost;       /* estimated work (arbitrary units) of the whole queue */
} jt_batch_info;

/*
 * Describe a batch.  Item i applies plans[i] in direction dirs[i] to the
 * tensor at byte offset in_off[i] of the run's input buffer, writing byte
 * offset out_off[i] of the output buffer (the two may coincide when in == out).
 * All items share the dtypes and the precision.  The plans must outlive the
 * batch and be bound (jt_plan_bind) before jt_batch_bind.  opt may be NULL.
 * Errors: JT_EINVAL, JT_EUNSUPPORTED (fp64 with n > 8192), JT_ENOMEM.
 */
jt_status jt_batch_create(int count, const jt_plan_t *plans, const int *dirs, const uint64_t *in_off,
                          const uint64_t *out_off, jt_dtype in, jt_dtype out, jt_prec prec,
                          const jt_batch_options *opt, jt_batch_t *batch);
jt_status jt_batch_destroy(jt_batch_t batch);
jt_status jt_batch_info_get(jt_batch_t batch, jt_batch_info *info);
/* Host copy of the unit table in queue order: 7 int32 per unit
 * (pass, first line, lines, split S, pass waited for or -1, units waited for,
 * passes run whole: > 0 for a small multi-axis item done inside one block,
 * whose row then covers passes pass .. pass + npass - 1 and every line),
 * and of the pass table: 4 int32 per pass (item, axis, lines, units).
 * Either pointer may be NULL. */
jt_status jt_batch_tables(jt_batch_t batch, int32_t *units, int32_t *passes);
/* Device bytes the batch needs (unit table, pass table, counters). */
jt_status jt_batch_device_bytes(jt_batch_t batch, size_t *bytes);
/* Copy the tables into dev_buf (256-byte aligned, >= jt_batch_device_bytes);
 * synchronises `stream`.  Errors: JT_ESTATE (a plan is not bound), JT_ENOMEM, JT_EDEVICE. */
jt_status jt_batch_bind(jt_batch_t batch, void *dev_buf, size_t bytes, void *stream);
/* Run every item: one counter-clearing kernel and the persistent kernel on
 * `stream`, no host synchronisation.  Runs of one batch must not overlap. */
jt_status jt_batch_run(jt_batch_t batch, const void *in_base, void *out_base, void *stream);
/* As jt_batch_run, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the run's counters (queue head, error word, done-units per pass) live in an
 * array the library keeps in each device's memory (256 KiB, 65536 words, held
 * until the process ends) instead of the batch's bound buffer, and the call
 * allocates nothing.  The batch must still be bound (its unit and pass
 * tables stay in the bound buffer).  The run's error word is copied to the
 * batch's own slot afterwards, so jt_batch_errors reads it as usual.  Every
 * call on one device shares that array: calls (and jt_batch_run_static runs
 * of different batches) must not overlap on one device; they race.
 * Errors: JT_EINVAL (more than 65534 axis passes, null argument, in-place
 * with unequal dtypes), JT_ESTATE (not bound), JT_EDEVICE. */
jt_status jt_batch_run_static(jt_batch_t batch, const void *in_base, void *out_base, void *stream);
/* Capture jt_batch_run(in_base, out_base) into a HIP graph held by the batch
 * (replaces an earlier capture); jt_batch_replay launches it on `stream`. */
jt_status jt_batch_capture(jt_batch_t batch, const void *in_base, void *out_base);
jt_status jt_batch_replay(jt_batch_t batch, void *stream);
/* Error word of the last run (synchronises `stream`): bit 0 = a unit's wait
 * for its previous pass timed out, bit 1 = unsupported length. 0 = clean. */
jt_status jt_batch_errors(jt_batch_t batch, void *stream, uint32_t *flags);

/* ----------------------------------------------------------------------
 * Serving form: a request loop with continuous batching.  Requests carry
 * host input and output buffers (pinned memory lets the copies overlap).  A
 * scheduler thread admits them in arrival order while the device arena has
 * room for their input and output (HBM-footprint admission), copies them in,
 * and launches every admitted request whose axis plans are resident as one
 * persistent batch launch; requests arriving meanwhile go into the next
 * launch as memory frees up.  Axis plans are cached in the arena keyed by
 * (n, a, b, tol), built on host threads on a miss and evicted least recently
 * used.  A request's result does not depend on the other requests it runs
 * with.  The arena is caller-owned device memory the server sub-allocates.
 */
typedef struct jt_server_s *jt_server_t;

typedef struct {
    double tol;              /* low-rank tolerance of every plan; 0 = 1e-7 */
    int prec;                /* jt_prec; default JT_PREC_FP64 (0): pass JT_PREC_FP32_BULK for the fp32 form */
    int in_dtype, out_dtype; /* jt_dtype of request data; default JT_F64 (0) */
    int max_batch;           /* most requests per launch; 0 = 256 */
    int max_inflight;        /* launches in flight; 0 = 2 */
    int plan_threads;        /* host planning threads; 0 = hardware threads (at most 16) */
    jt_batch_options batch;  /* unit shaping of each launch */
    int dense_below;         /* axes shorter than this (at most 1024) use the dense matrix-core
                                pass; 0 = 64 */
    int dense_below_1d;      /* the same for 1D requests, whose passes have a single line (the
                                crossover is lower there); 0 = dense_below */
} jt_server_options;

typedef struct {
    int state;               /* 0 queued, 1 admitted, 2 running, 3 done, 4 failed */
    int cold;                /* one of its axis plans was built for it (cache miss) */
    double t_submit, t_admit, t_launch, t_done;  /* jt_clock() seconds */
    double plan_seconds;     /* host planning time of its missed plans */
    int status;              /* jt_status of a failed request */
} jt_request_info;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t plan_hits, plan_misses, plans_cached, plans_evicted;
    uint64_t launches;
    double coeffs;           /* coefficients of completed requests */
    size_t arena_bytes, arena_used, arena_peak;
    int queued, admitted, running;
} jt_server_stats;

/* Monotonic clock (seconds) the server stamps requests with. */
double jt_clock(void);
/* dev_arena: caller-owned device memory, 256-byte aligned, kept until destroy.
 * Errors: JT_EINVAL, JT_EDEVICE. */
jt_status jt_server_create(void *dev_arena, size_t bytes, const jt_server_options *opt, jt_server_t *server);
/* Queue one transform of a d-dimensional row-major tensor.  host_in and
 * host_out must stay valid until the request is done.  Errors: JT_EINVAL,
 * JT_ENOMEM (input and output alone exceed the arena), JT_EUNSUPPORTED. */
jt_status jt_server_submit(jt_server_t server, int d, const int *n, const double *a, const double *b,
                           jt_direction dir, const void *host_in, void *host_out, uint64_t *ticket);
/* State and timestamps of a request (non-blocking). */
jt_status jt_server_poll(jt_server_t server, uint64_t ticket, jt_request_info *info);
/* Block until the request is done or failed, return its info and forget the ticket. */
jt_status jt_server_wait(jt_server_t server, uint64_t ticket, jt_request_info *info);
jt_status jt_server_stats_get(jt_server_t server, jt_server_stats *stats);
/* Finish running launches, fail queued requests, release host resources. */
jt_status jt_server_destroy(jt_server_t server);

/* Message describing the last error on the calling thread ("" if none). */
const char *jt_last_error(void);

/* ABI version of this header (major * 100 + minor). */
int jt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JT_H */
