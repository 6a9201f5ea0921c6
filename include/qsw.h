/*
 * qsw.h - C ABI of libqsw: L-QSW (locally interacting quantum stochastic
 * walk) propagation on one AMD MI355X (gfx950) GPU.
 *
 * The library builds the vectorised Lindblad superoperator L of a walk on a
 * graph (Section 2.5.1 eq. qsw, vectorised by eq. vec_mappings) as a
 * complex128 CSR matrix in device memory, and evaluates
 *     rho(t_k) = unvec( exp(t_k L) vec(rho0) ),  t_k = t0 + k dt,
 * by the truncated-Taylor method with scaling and early termination that the
 * paper adopts (Section 3.1: Al-Mohy and Higham's single-time algorithm,
 * `step`, and time-series algorithm, `series`), without balancing or shift.
 *
 * Conventions
 *   - Graphs: CSR of the N x N adjacency G with G[i][j] = weight of the arc
 *     from source vertex j to target vertex i (row = target, column =
 *     source), weights > 0, no diagonal (simple graphs, Section 2.1).
 *   - Density matrices are complex128 (interleaved re, im doubles), N x N,
 *     ROW-MAJOR: element (a, b) at index a*N + b.  The superoperator acts on
 *     this row-major vec.  (The paper stacks columns; the two orders differ
 *     by a fixed permutation and give the same rho.)
 *   - Every pointer documented "device" must be memory of the device that
 *     was current when the handle was built; "host" pointers are ordinary
 *     CPU memory.  Host arrays are only read during the call.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  All device
 *     work of a call is enqueued on it; calls return before it completes
 *     unless stated otherwise.  Caller-owned device buffers must stay alive
 *     until the stream has finished the call's work.
 *   - Errors are returned as qsw_status_t; nothing aborts or throws across
 *     the ABI.  Argument and graph checks are synchronous.  Device faults and
 *     non-finite values surface through qsw_last_stats.
 */
#ifndef QSW_H
#define QSW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsw_superop_s *qsw_superop_t;

typedef enum {
    QSW_OK = 0,
    QSW_ERR_ARG = 1,        /* bad argument (null pointer, omega outside [0,1], sizes) */
    QSW_ERR_GRAPH = 2,      /* malformed graph CSR (self-loop, w <= 0, unsorted, duplicate, out of range) */
    QSW_ERR_OOM = 3,        /* device allocation failed */
    QSW_ERR_DEVICE = 4,     /* HIP runtime error (launch, copy, no device) */
    QSW_ERR_NONFINITE = 5,  /* a norm or value was NaN or infinite */
    QSW_ERR_STATE = 6,      /* handle used on another device, or workspace too small */
    QSW_ERR_SIZE = 7,       /* N*N does not fit the 32-bit column index (N > 46340) */
    QSW_ERR_SCRATCH = 8     /* qsw_propagate_noalloc: the call needs more than its static scratch */
} qsw_status_t;

/* Build flags (bitwise OR). */
enum {
    QSW_H_LAPLACIAN = 0,    /* H = transition matrix of G^u (eq. generator_matrix on the
                               undirected companion, Section 2.5.1): the weighted Laplacian for gamma = 1 */
    QSW_H_ADJACENCY = 1,    /* H = G^u itself (the paper's three-vertex example passes H = GU) */
    QSW_R_TRANSITION = 0,   /* L_k = sqrt(gamma G_ij)|i><j| for every arc (eq. lindblad) */
    QSW_R_COLNORM = 2,      /* L_k = sqrt(G_ij / OutDeg(j))|i><j| (column-normalised rates) */
    QSW_DEPHASING = 4       /* also the diagonal L_k = sqrt(|M_jj|)|j><j| that eq. qsw sums over */
};

/* Precision of qsw_propagate (qsw_superop_set_precision) and of the
 * tolerance used for theta_m and the stopping test. */
enum {
    QSW_PREC_DOUBLE = 0,  /* complex128 throughout, u = 2^-53 */
    QSW_PREC_SINGLE = 1,  /* complex64 operator values, complex128 vectors, u = 2^-24 */
    QSW_PREC_FP32 = 2     /* complex64 values, vectors and products with two-float
                             accumulation, u = 2^-24 and Taylor degree at most 20 */
};

typedef struct {
    int32_t N;           /* graph order */
    int64_t n;           /* superoperator dimension N*N */
    int64_t nnz;         /* stored entries of L (explicit zeros kept: pattern independent of omega) */
    double omega;
    double norm1;        /* ||L||_1, exact (max column sum) */
    double d[10];        /* d[p] = estimate of ||L^p||_1^(1/p), p = 2..9 (d[0] = d[1] = norm1) */
    int64_t d_index[10]; /* column e_j whose image attains the estimate of ||L^p||_1, or -1 when
                            the estimate came from the first (non-unit) probe block */
    int32_t d_probe[10]; /* for d_index == -1: which probe column (0 = all-ones/n, 1 = +-1/n) */
    int32_t norm_products; /* sparse products spent on the estimates */
    double build_ms;     /* host wall time of the build call, including device sync */
    int32_t split;       /* 1: the product kernels read phase-split values (every
                            off-diagonal entry real or imaginary: one real coefficient
                            per entry, its phase in the column index, the complex
                            diagonal per row); 0: complex values */
    int64_t stream_entries; /* entries the product kernels read per row (without the shared ones) */
    int64_t shared_entries; /* entries stored once per 64-row block for all its rows (same offset
                               from the row and same value; phase-split values only; padded) */
    int64_t distinct_entries; /* per-row entries in the copies the blocks read: blocks whose
                                 stored rows are word for word equal (columns as offsets from
                                 the row) read one copy */
    int32_t engine;      /* product kernel of complex128 qsw_propagate calls: traversal (0
                            plain, 100 rho-row staged in LDS, 200 staged with XCD column
                            bands, 300 staged with wide position groups, taken for
                            operators with long rows) + 10 for phase-split values; 3: the
                            CSR stream engine; 4..64: the CSR vector engine with that many
                            lanes per row */
} qsw_info_t;

typedef struct {
    int32_t branch;      /* 0: one single-time application per interval (q <= s);
                            1: time-series blocks with stored powers (q > s) */
    int32_t m;           /* Taylor degree used for each interval (branch 0) or block (branch 1) */
    int32_t s;           /* scaling steps per interval (branch 0) or for the whole span (branch 1) */
    int32_t m0, s0;      /* parameters of the exp(t0 L) start, 0/1 when t0 = 0 */
    int64_t launched;    /* sparse-product kernels enqueued */
    int64_t products;    /* sparse products actually computed (early termination skips the rest) */
    int32_t nonfinite;   /* 1 if any norm in the run was NaN or infinite */
    double ms;           /* device time of the last propagate call (events on its stream) */
    double bytes;        /* algorithmic HBM bytes of the computed products: per product
                            E e + 16 s + 8 (n+1) + D n + (64 or 80) n for branch 0 or 1 (branch
                            1 adds the accumulation pass, except with one grid point per block,
                            which runs in the fused term kernel), with e = stream_entries and s =
                            shared_entries of qsw_info_t, and (E, D) = (20, 0) / (12, 0) for
                            complex double / single values and (12, 16) / (8, 8) for
                            phase-split double / single values (D: the diagonal per row) */
    int32_t prec;        /* QSW_PREC_* the call ran with */
    double trace_dev;    /* QSW_PREC_FP32: largest |Tr rho_k - Tr rho0| of the output points
                            before their trace renormalisation (0 for the other precisions) */
} qsw_stats_t;

/* ---------------------------------------------------------------- build */

/*
 * Build the L-QSW superoperator of a graph (Section 2.5.1; H from G^u,
 * L_k from the CTRW transition matrix of G, eq. generator_matrix and eq.
 * lindblad), assemble it in device CSR (int64 row_ptr, int32 columns,
 * complex128 values; each row in structural order: the H rho entries by
 * ascending c (column c N + b of row a N + b), the diagonal, the rho H
 * entries by ascending c (column a N + c), then the population-transfer
 * entries (column j (N + 1)); no column repeats), compute ||L||_1 exactly and estimate
 * ||L^p||_1, p = 2..9 (the 1-norm series the paper computes at construction,
 * Section 4 footnote).
 *
 *   N, row_ptr[N+1], col_idx[nnz], w[nnz]: host CSR of G (see Conventions).
 *   omega in [0, 1]; gamma > 0 (system-wide transition rate).
 *   flags: QSW_H_*, QSW_R_*, QSW_DEPHASING.
 *   *out receives a handle owning the device CSR; free with qsw_superop_destroy.
 * Synchronises `hip_stream` before returning.
 */
qsw_status_t qsw_superop_build(int32_t N, const int64_t *row_ptr, const int32_t *col_idx,
                               const double *w, double omega, double gamma, uint32_t flags,
                               void *hip_stream, qsw_superop_t *out);

/*
 * qsw_superop_build on the augmented digraph of Section 2.5.1 (eq.
 * dimer_aug, eq. qsw_ss): n_sources source vertices (numbered N .. N +
 * n_sources - 1, source k feeding graph vertex source_vertex[k] at rate
 * source_rate[k]) and n_sinks sink vertices (numbered after them, sink k
 * draining graph vertex sink_vertex[k] at rate sink_rate[k]).  The channels
 * act outside omega; H and the omega-scaled rates come from G as for
 * qsw_superop_build and are zero on the added vertices.  rho0 and the
 * outputs are (N + n_sources + n_sinks)^2.  Synchronises `hip_stream`.
 */
qsw_status_t qsw_superop_build_channels(int32_t N, const int64_t *row_ptr, const int32_t *col_idx,
                                        const double *w, double omega, double gamma,
                                        uint32_t flags, int32_t n_sources,
                                        const int32_t *source_vertex, const double *source_rate,
                                        int32_t n_sinks, const int32_t *sink_vertex,
                                        const double *sink_rate, void *hip_stream,
                                        qsw_superop_t *out);

/*
 * Build from explicit operators, as the paper's LQSW(omega, H, M_L) does
 * (Section 4): H is a Hermitian N x N host CSR (complex128 values,
 * interleaved; it may hold a diagonal; its pattern must be symmetric), M_L
 * the condensed Lindblad matrix (eq. condensed_lindblads) as a real host CSR:
 * each entry (i, j) is one L_k = M_L[i][j] |i><j| (rates |M_L[i][j]|^2;
 * diagonal entries are dephasing channels).  Columns sorted, no duplicates.
 * flags: 0.  Synchronises `hip_stream`.
 */
qsw_status_t qsw_superop_build_ops(int32_t N,
                                   const int64_t *h_row_ptr, const int32_t *h_col,
                                   const double *h_val,
                                   const int64_t *l_row_ptr, const int32_t *l_col,
                                   const double *l_val,
                                   double omega, uint32_t flags, void *hip_stream,
                                   qsw_superop_t *out);

/*
 * qsw_superop_build_ops with absorption and emission channels (Section 2.5.1,
 * eq. qsw_ss): M_free is a second real coefficient matrix (host CSR, same
 * rules as M_L) whose L_k = M_free[i][j] |i><j| enter with rate
 * |M_free[i][j]|^2 OUTSIDE the factor omega, e.g. sources (arcs from a source
 * vertex into the graph, rate Gamma) and sinks (arcs from the graph into a
 * sink vertex, rate Theta) of the augmented digraph.  The order N counts the
 * source and sink vertices.  M_free may be NULL (then this is
 * qsw_superop_build_ops).  flags: 0.  Synchronises `hip_stream`.
 */
qsw_status_t qsw_superop_build_open(int32_t N, const int64_t *h_row_ptr, const int32_t *h_col,
                                    const double *h_val, const int64_t *l_row_ptr,
                                    const int32_t *l_col, const double *l_val,
                                    const int64_t *f_row_ptr, const int32_t *f_col,
                                    const double *f_val, double omega, uint32_t flags,
                                    void *hip_stream, qsw_superop_t *out);

/*
 * A walk with explicit Lindblad operators (Section 2.5.2, eq. L_global, and
 * the non-moralising form eq. nm_gqsw):
 *     L rho = -i(1-omega)[H, rho] + omega ( i[H_rot, rho] + sum_k D[L_k] rho ),
 *     D[L] rho = L rho L^dag - 1/2 {L^dag L, rho}.
 * H and H_rot: Hermitian complex host CSR (H_rot may be NULL); L_k: n_ops
 * complex host CSRs (arrays of their row_ptr / col / interleaved val).  The
 * G-QSW is n_ops = 1, L_1 = G.  Assembled on the host (Kronecker terms; the
 * superoperator's density grows as the square of the L_k's), then handled
 * exactly as the other builds.  Synchronises `hip_stream`.
 */
qsw_status_t qsw_superop_build_general(int32_t N, const int64_t *h_row_ptr, const int32_t *h_col,
                                       const double *h_val, int32_t n_ops,
                                       const int64_t *const *l_row_ptr,
                                       const int32_t *const *l_col, const double *const *l_val,
                                       const int64_t *r_row_ptr, const int32_t *r_col,
                                       const double *r_val, double omega, void *hip_stream,
                                       qsw_superop_t *out);

/*
 * The non-moralising G-QSW of a digraph (Section 2.5.2, graph demoralisation
 * and eq. nm_gqsw), built on the expanded vertex set: vertex v keeps
 * d_v = max(1, number of arcs into v) copies (qsw_demoralised_order),
 * numbered consecutively; copies of joined vertices are linked with weight
 * G_vw / sqrt(d_v d_w); H_D is the transition matrix of the linked G^u, the
 * single L_D takes copy u of parent w of v to copy k of v with coefficient
 * exp(2 pi i k m / d_v) G_vw / sqrt(d_v d_w) (m: rank of w among v's
 * parents), and H_rot links consecutive copies of a vertex (+i forward, -i
 * back, cyclic for d_v > 2).  Graph CSR as for qsw_superop_build.  rho0 and
 * outputs live on the expanded set (qsw_demoralised_state /
 * _populations map to and from it).  Synchronises `hip_stream`.
 */
qsw_status_t qsw_superop_build_demoralised(int32_t N, const int64_t *row_ptr,
                                           const int32_t *col_idx, const double *w, double omega,
                                           double gamma, void *hip_stream, qsw_superop_t *out);

/* Host only: order of the expanded vertex set, copies[v] = d_v (copies may
 * be NULL); -1 for a malformed graph or an order beyond int32. */
int32_t qsw_demoralised_order(int32_t N, const int64_t *row_ptr, const int32_t *col_idx,
                              int32_t *copies);

/* Host only: rho (N x N complex128, interleaved) -> V rho V^dag on the
 * expanded set, V|v> = d_v^(-1/2) sum_k |v^k> (trace and positivity kept). */
qsw_status_t qsw_demoralised_state(int32_t N, const int32_t *copies, const double *rho,
                                   double *rho_d);

/* Host only: p(v) = sum over the copies of v (eq. nm_rho_map), for `count`
 * population vectors of the expanded set (count x M doubles -> count x N). */
qsw_status_t qsw_demoralised_populations(int32_t N, const int32_t *copies, const double *pops_d,
                                         int32_t count, double *pops);

/*
 * Rebuild the handle's superoperator for another omega (the paper's
 * set_omega), from the operators it was built from; the handle keeps its
 * identity and precision, and the result is the same as a fresh build at
 * that omega.  Waits for work in flight on the device.
 */
qsw_status_t qsw_superop_set_omega(qsw_superop_t h, double omega, void *hip_stream);

void qsw_superop_destroy(qsw_superop_t h);

qsw_status_t qsw_superop_info(qsw_superop_t h, qsw_info_t *info);

/*
 * Precision of later qsw_propagate calls on this handle (default
 * QSW_PREC_DOUBLE).
 *   QSW_PREC_SINGLE: the product kernels read a single-precision copy of the
 *     superoperator values (each real and imaginary part rounded to nearest;
 *     made here, 8 bytes per entry of device memory for complex values, 4 per
 *     entry and 8 per row for phase-split values, kept until QSW_PREC_DOUBLE
 *     is set or the handle is destroyed), theta_m and the stopping test use
 *     u = 2^-24 (Al-Mohy and Higham's single-precision choice), and vectors,
 *     products, sums and norms stay complex128 / double.  rho(t) then carries
 *     a backward error of at most about 2 u ||L||_1 per unit time (value
 *     rounding plus truncation) instead of u = 2^-53.
 *   QSW_PREC_FP32: the same single-precision values, and the vectors and
 *     products in single precision too: each Taylor term is a complex64
 *     vector (the row sums in float, scaled in double and rounded once), the
 *     accumulator is an unevaluated pair hi + lo of complex64 vectors updated
 *     by two-sum (about twice the float significand, so adding the terms
 *     loses nothing beyond their own rounding), and the norms, the stopping
 *     test and (m, s) stay in double with u = 2^-24.  The Taylor degree is at
 *     most 20 (p <= 5 in the alpha_p rule): the terms of one scaling step then
 *     grow to at most about e^theta_20 = 35 times the step's input before they
 *     cancel, which bounds the single-precision rounding they carry.  Every
 *     interval is one single-time application (no time-series reuse).  Each
 *     output point is checked in double: its trace is summed from hi + lo and,
 *     when it is within 2^-10 relative of Tr rho0, the point (and the state
 *     carried on) is scaled to Tr rho0, which the exact evolution keeps
 *     (every Lindblad generator preserves the trace); the largest deviation
 *     before scaling is qsw_stats_t.trace_dev.  Outputs are complex128
 *     (hi + lo); out[0] = rho0 exactly when t0 = 0.  Workspace: 48 bytes per
 *     element of vec(rho) instead of 64.
 *   ||L||_1, the d_p and the parameter choice always come from the complex128
 *   values; qsw_apply and qsw_superop_copy_csr always use them.
 * Returns QSW_ERR_STATE when the handle runs a product engine other than the
 * default one (the copy exists for its layout only), QSW_ERR_OOM when the copy
 * does not fit.  Synchronous; changes the workspace size a plan needs.
 */
qsw_status_t qsw_superop_set_precision(qsw_superop_t h, int32_t prec);

/*
 * Launch pacing of later qsw_propagate calls on this handle (default 0: off).
 * The single-time branch launches up to m Taylor terms per scaling step and
 * the terms after the one that passes the stopping test (Al-Mohy and
 * Higham's two-term test) exit at once; each such launch still costs a few
 * microseconds.  With lookahead > 0 every term launch posts to a pinned host
 * word that its predecessor has ended and whether the step passed the test
 * after it, and qsw_propagate keeps at most `lookahead` term launches beyond
 * the last one known to have ended (2 or more keeps the device busy),
 * enqueuing no further terms of a step once it has passed the test.  The
 * results are the same.  qsw_propagate then returns only when its last
 * launches are enqueued (it waits on the device meanwhile), and paced calls
 * on one handle are serialised.  Allocates 256 bytes of pinned host memory
 * on first use.  QSW_ERR_ARG for lookahead outside 0..4096.
 */
qsw_status_t qsw_superop_set_pacing(qsw_superop_t h, int32_t lookahead);

/* Launch configuration of the product kernels, as chosen by qsw_superop_autotune. */
typedef struct {
    int32_t staged;          /* 1: the rho-row is staged in LDS for the rho H gathers;
                                2: staged, and each XCD takes one band of columns of rho
                                (N = 512, 1024 or 2048); 3: staged, with wider groups of
                                positions at fewer waves per SIMD (double values) */
    int32_t grid;            /* workgroups per product launch */
    double us_per_product;   /* measured time of one product in that configuration */
    int32_t from_cache;      /* 1: taken from an earlier tuning of the same key */
} qsw_tuning_t;

/*
 * Time the product kernel on this handle for each launch configuration
 * (rho-row staging off, on where N*16 bytes fit, with XCD column bands
 * where N allows, and staged with wide position groups for double values;
 * grid of 1, 2, 4 and 8 times the resident workgroups),
 * keep the fastest for later qsw_propagate /
 * qsw_apply calls and remember it for the key (N, entries per row, precision)
 * in the process, so that later handles with the same key take it without
 * timing.  No configuration changes any sum's order: results are bitwise
 * the same whichever is chosen.  Allocates two vectors of n complex128 for
 * the timing; synchronises `hip_stream`.
 */
qsw_status_t qsw_superop_autotune(qsw_superop_t h, void *hip_stream, qsw_tuning_t *out);

/* Copy the device CSR to caller host buffers (row_ptr[n+1], col[nnz],
 * val[2*nnz] doubles), rows in the structural order described at
 * qsw_superop_build (rows of qsw_superop_build_general are sorted by
 * column).  Any pointer may be NULL to skip it.  Synchronous. */
qsw_status_t qsw_superop_copy_csr(qsw_superop_t h, int64_t *row_ptr, int32_t *col,
                                  double *val);

/* ------------------------------------------------------------ propagate */

/* Device workspace (bytes) that qsw_propagate needs for these arguments. */
size_t qsw_propagate_workspace_bytes(qsw_superop_t h, double t0, double dt, int32_t n_steps);

/*
 * out[k] = rho(t0 + k dt) = unvec(exp((t0 + k dt) L) vec(rho0)), k = 0..n_steps
 * (the paper's `series(t1 = t0, tq = t0 + n_steps dt, steps = n_steps)`;
 * n_steps = 1, t0 = 0 is its `step(dt)`).
 *
 *   rho0: device, N*N complex128, row-major; read only.
 *   out:  device, (n_steps+1) * N*N complex128; out[0] = exp(t0 L) rho0.
 *         Must not overlap rho0.
 *   workspace: device, >= qsw_propagate_workspace_bytes(...) bytes, 256-byte
 *         aligned; its contents on entry are ignored.
 *   n_steps >= 0; dt and t0 finite.
 * Enqueues everything on `hip_stream` and returns; no device memory is
 * allocated.  Concurrent calls on one handle need distinct workspaces and
 * outputs; qsw_last_stats then reports whichever call finished last.
 */
qsw_status_t qsw_propagate(qsw_superop_t h, const void *rho0, double t0, double dt,
                           int32_t n_steps, void *out, void *workspace, size_t ws_bytes,
                           void *hip_stream);

/*
 * qsw_propagate for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that forbid allocation, harnesses without
 * hipMalloc): the same computation, kernels and results, with the workspace
 * taken from a static device array of QSW_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends.  It calls
 * no allocating routine; the caller still passes rho0 and out (as for
 * qsw_propagate).  QSW_ERR_SCRATCH when qsw_propagate_workspace_bytes(h, t0,
 * dt, n_steps) exceeds QSW_NOALLOC_SCRATCH_BYTES (e.g. the time-series branch
 * on a large operator, which stores m powers).  Every call on a device
 * shares that device's scratch (its contents are those of the last call;
 * each call sets up what it needs itself): calls that overlap on one device,
 * from several threads or streams, race and must be serialised by the
 * caller.
 */
#define QSW_NOALLOC_SCRATCH_BYTES (80u << 20)
qsw_status_t qsw_propagate_noalloc(qsw_superop_t h, const void *rho0, double t0, double dt,
                                   int32_t n_steps, void *out, void *hip_stream);

/* Statistics of the last qsw_propagate on this handle (waits for it). */
qsw_status_t qsw_last_stats(qsw_superop_t h, qsw_stats_t *st);

/* -------------------------------------------------------- batched walks */

/*
 * A walk: one superoperator, n0 <= 4 initial density matrices propagated
 * together (each exactly as qsw_propagate would propagate it alone: same
 * parameters, same terms, same stopping decisions, bitwise the same result),
 * and its own time grid t0 + k dt, k = 0..n_steps.  Many walks advance
 * together in one engine, so small operators share launches and each
 * operator's values are read once per product for all n0 right-hand sides.
 *
 *   op:    built handle, on the engine's device; its precision applies
 *          (QSW_PREC_DOUBLE, QSW_PREC_SINGLE, or QSW_PREC_FP32: single-precision
 *          products with hi + lo accumulation and the FP64 trace check at every
 *          point, exactly as qsw_propagate runs them).  It must stay alive until
 *          the walk has finished; walks of every precision share one engine.
 *   rho0:  device, n0 consecutive N*N complex128 row-major matrices.
 *   out:   device, (n_steps+1) x n0 x N*N complex128 (point-major), or NULL.
 *   pops:  device, (n_steps+1) x n0 x N doubles (Re rho_aa), or NULL.
 */
typedef struct {
    qsw_superop_t op;
    int32_t n0;
    const void *rho0;
    double t0, dt;
    int32_t n_steps;
    void *out;
    void *pops;
} qsw_walk_t;

typedef struct qsw_engine_s *qsw_engine_t;

typedef struct {
    int64_t cycles;      /* control + work launch pairs so far */
    int64_t products;    /* sparse products of the finished walks */
    int32_t live;        /* walks admitted and not finished */
    int32_t nonfinite;   /* 1 once any norm was NaN or infinite */
    double ms;           /* device time of the last qsw_engine_run */
    double bytes;        /* algorithmic bytes of the finished walks' products: per product
                            each stored entry's column and value, the block-shared entries,
                            row data, the diagonal per row, and 64 bytes per element and
                            right-hand side (x, the term, the accumulator read and written) */
    int64_t graphs;      /* chunk graphs captured (a walk finishing or joining changes them) */
    int64_t graph_launches; /* chunk graphs launched (one per chunk of cycles) */
    int32_t rounds;      /* launch shape in use: work-launch grid of `rounds` x the
                            resident workgroups (at most one wave per block) */
    int32_t staged;      /*   and rho-row staging in LDS on (1) or off (0) */
    double trace_dev;    /* walks with single-precision products (QSW_PREC_FP32): largest
                            |Tr rho_k - Tr rho0| of their checked points before scaling, over
                            the finished walks and their right-hand sides */
} qsw_engine_stats_t;

/* Device bytes one walk takes in an engine with `rhs` (1, 2 or 4)
 * right-hand sides: six work vectors of n*rhs complex128 (complex64 with
 * single-precision products), plus m stored powers in the time-series
 * branch.  0 for a bad walk. */
size_t qsw_walk_bytes(const qsw_walk_t *walk, int32_t rhs);

/* Bytes the engine's own tables take at the start of its arena.  The engine
 * also keeps a map of the running walks' 64-row blocks: about
 * arena_bytes / (384 rhs) + 8 (max_walks + 1) bytes after the tables. */
size_t qsw_engine_table_bytes(int32_t max_walks);

/*
 * An engine over a caller-owned device arena (256-byte aligned, at least
 * qsw_engine_table_bytes(max_walks)); it allocates no device memory.  The
 * rest of the arena holds the walks' vectors.  All work goes to hip_stream.
 */
qsw_status_t qsw_engine_create(int32_t max_walks, int32_t rhs, void *arena, size_t arena_bytes,
                               void *hip_stream, qsw_engine_t *out);

/* Admit a walk: QSW_OK and a ticket, or QSW_ERR_OOM when no slot or not
 * enough free arena is available now (admission control: try again after
 * walks have finished).  Synchronises the engine's stream. */
qsw_status_t qsw_engine_submit(qsw_engine_t e, const qsw_walk_t *walk, int64_t *ticket);

/* Run up to max_cycles cycles, or until every admitted walk has finished;
 * *live receives the number still running.  Synchronous. */
qsw_status_t qsw_engine_run(qsw_engine_t e, int32_t max_cycles, int32_t *live);

/* Tickets of walks finished since the last poll (their outputs are complete
 * and their arena space is free again). */
qsw_status_t qsw_engine_poll(qsw_engine_t e, int64_t *tickets, int32_t capacity, int32_t *count);

qsw_status_t qsw_engine_stats(qsw_engine_t e, qsw_engine_stats_t *st);

void qsw_engine_destroy(qsw_engine_t e);

/* Workspace for qsw_batch_propagate: tables plus every walk's bytes. */
size_t qsw_batch_workspace_bytes(const qsw_walk_t *walks, int32_t count, int32_t rhs);

/* All walks to completion in one engine on `workspace` (synchronous; no
 * device allocation). */
qsw_status_t qsw_batch_propagate(const qsw_walk_t *walks, int32_t count, int32_t rhs,
                                 void *workspace, size_t ws_bytes, void *hip_stream,
                                 qsw_engine_stats_t *stats);

/* ------------------------------------------------ continuous batching */

typedef struct qsw_server_s *qsw_server_t;

typedef struct {
    int64_t submitted, completed;
    int64_t cache_hits, cache_misses, evictions;
    int64_t cycles, products;
    int64_t cache_bytes;     /* device bytes of the cached operators */
    double build_ms;         /* builder-thread time spent building operators */
} qsw_server_stats_t;

/*
 * A server for walks that arrive one at a time (one density matrix each),
 * all running in one batch engine (qsw_engine_*) over an arena of
 * arena_bytes that the server allocates now.  Operators are cached on the
 * device under cache_bytes, keyed by (N, graph CSR, omega, gamma, flags);
 * unused ones are evicted least recently used first.  The walks' work goes
 * to hip_stream; operator builds run on a stream of the server's own that
 * does not wait for the legacy default stream.  A walk whose graph order is
 * at least QSW_SERVER_DIRECT_N (environment, read here; default 384, 0: off)
 * fills the device on its own: it runs through qsw_propagate (launch pacing
 * 2) in a direct lane, on a runner thread and stream of the server's own,
 * one such walk at a time in arrival order, beside the engine; the lane's
 * workspace and the output series of a populations-only walk are device
 * buffers the server allocates and keeps (growing them as needed).
 */
qsw_status_t qsw_server_create(size_t arena_bytes, size_t cache_bytes, int32_t max_walks,
                               void *hip_stream, qsw_server_t *out);

/*
 * Queue a walk: the graph and options as for qsw_superop_build (host CSR,
 * copied during the call), rho0 (device, N*N complex128), the grid t0 + k dt,
 * k = 0..n_steps, and device outputs out ((n_steps+1) x N*N complex128)
 * and/or pops ((n_steps+1) x N doubles), either may be NULL.  rho0 and the
 * outputs must stay alive until the walk is reported done.  An operator not
 * in the cache is built by the server's builder thread on its own stream
 * (so walks on the device keep advancing), once the cache budget has room
 * for it: before the build its size counts as an upper bound from the graph,
 * afterwards as the handle's size.  The walk joins the engine as soon as its
 * operator is ready and its work vectors fit; walks with ready operators are
 * admitted in arrival order.  QSW_ERR_OOM when the vectors could not fit
 * even in an empty arena (reported here for a cached operator, else by the
 * qsw_server_step that sees the build finish, which also completes the
 * request).
 */
qsw_status_t qsw_server_submit(qsw_server_t s, int32_t N, const int64_t *row_ptr,
                               const int32_t *col_idx, const double *w, double omega,
                               double gamma, uint32_t flags, const void *rho0, double t0,
                               double dt, int32_t n_steps, void *out, void *pops,
                               int64_t *request);

/* Take finished operator builds, run up to max_cycles engine cycles (when
 * nothing runs and walks wait for builds, first wait up to 5 ms for one),
 * collect finished walks and admit waiting ones; reports how many run and
 * wait.  Synchronous.  A failed build finishes its requests (they are
 * polled as done, with no output) and its status is returned here. */
qsw_status_t qsw_server_step(qsw_server_t s, int32_t max_cycles, int32_t *running,
                             int32_t *pending);

/* Requests finished since the last poll, with their latency from submit to
 * the step that saw them finish (latency_ms may be NULL). */
qsw_status_t qsw_server_poll(qsw_server_t s, int64_t *requests, double *latency_ms,
                             int32_t capacity, int32_t *count);

qsw_status_t qsw_server_stats(qsw_server_t s, qsw_server_stats_t *st);

void qsw_server_destroy(qsw_server_t s);

/* ------------------------------------------------------------- helpers */

/* y = L x (device complex128 vectors of length n).  Enqueued on the stream. */
qsw_status_t qsw_apply(qsw_superop_t h, const void *x, void *y, void *hip_stream);

/* pops[k*N + a] = Re rho_k[a][a] for k < count (the paper's
 * gather_populations).  rho: device count*N*N complex128; pops: device
 * count*N doubles.  Enqueued on the stream. */
qsw_status_t qsw_populations(qsw_superop_t h, const void *rho, int32_t count, void *pops,
                             void *hip_stream);

/* ------------------------------------------- host-only (no GPU needed) */

/* theta_m (1 <= m <= 55) of the truncated-Taylor backward-error bound,
 * computed by the library from its definition; prec = QSW_PREC_*.
 * Returns a negative value for a bad argument. */
double qsw_theta(int32_t m, int32_t prec);

/*
 * Taylor degree m and scaling s for exp(t L) from ||L||_1 and d[p], p = 2..9
 * (d may be NULL: the 1-norm alone is used), n0 right-hand sides, tolerance
 * prec.  The rule is Al-Mohy and Higham's (cited in Section 3.1): the 1-norm
 * choice when ||tL||_1 is small, else the minimum of m * ceil(alpha_p / theta_m)
 * over 2 <= p <= p_max, p(p-1)-1 <= m <= m_max, alpha_p = t max(d_p, d_{p+1});
 * smallest m on ties; t||L||_1 = 0 gives m = 0, s = 1.  (m_max, p_max) =
 * (55, 8), or (20, 5) for QSW_PREC_FP32, whose theta_m are the single ones.
 * prec | QSW_PARAMS_KNOWN_NORMS: the alpha_p rule whenever d is given, also
 * for small ||tL||_1 (their switch to the 1-norm rule only saves the products
 * of estimating the d_p).  qsw_propagate chooses this way: a handle's d_p are
 * estimated once, at construction.
 */
#define QSW_PARAMS_KNOWN_NORMS 16
qsw_status_t qsw_select_params(double norm1, const double *d, double t, int32_t n0,
                               int32_t prec, int32_t *m, int32_t *s);

const char *qsw_status_str(qsw_status_t s);

/* Library version string. */
const char *qsw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QSW_H */
