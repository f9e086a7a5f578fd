/*
 * gst.h -- C ABI of the MI355X gate-set-tomography likelihood library.
 *
 * The library evaluates, for a gate set of Pauli-transfer matrices and a list
 * of gate sequences (thesis Sec. 6.3.1, Eqs. GSTBornRuleVectorized and
 * GSTFullFiducialsGerms):
 *
 *   p[s][m] = e_m^T G[s_L] ... G[s_1] rho          outcome probabilities
 *   F       = - sum_{s,m: N[s][m] > 0} N[s][m] log p[s][m]
 *                                                   negative multinomial log-likelihood
 *                                                   of the outcome counts (the data-only
 *                                                   multinomial constant is dropped and
 *                                                   0 log 0 := 0)
 *   dF/dtheta                                       gradient with respect to every entry of
 *                                                   rho, of each e_m and of each G_k
 *
 * These are the three quantities of the black-box problem of Sec. 6.3.1: a state
 * (INIT), gates (buttons), a measurement (MEAS) and the counts of each outcome.
 *
 * Numbers and layouts (all IEEE binary64 unless stated):
 *   n_qubits n in 1..3, d = 2^n, D = d*d = 4^n.
 *   Pauli index i = sum_q a_q 4^(n-1-q), a in {I:0, X:1, Y:2, Z:3}, qubit 0 the
 *     leftmost tensor factor (Eq. paulibasis); basis normalized by 1/sqrt(d).
 *   rho[D]; effects[M][D], row m = e_m; gates[K][D][D] row-major,
 *     gates[k][i][j] = Tr(P_i G_k(P_j))/d (Eq. paulitransfermatrix).
 *   Sequences in CSR form: offsets[S+1] (int64, offsets[0] = 0, non-decreasing),
 *     gate_idx[offsets[S]] (uint8, time order: gate_idx[offsets[s]] acts first;
 *     Sec. 2.2.2: the matrix product is the reverse of time order). Empty
 *     sequences are allowed.
 *   counts[S][M] int32 >= 0; probs[S][M]; dLoss/dp weights w[S][M].
 *   Gradient layout: [rho (D) | effects (M*D) | gates (K*D*D)], D + M*D + K*D*D
 *     doubles (1616 for two qubits with M = 4, K = 6, the count of Sec. 6.3.1).
 *
 * Memory and ownership: unless a name ends in _host, every pointer is a DEVICE
 * pointer on the context's device, owned by the caller; inputs must stay valid
 * and unmodified until the stream reaches the call, outputs are written in
 * stream order.  The library owns contexts, requests and their workspaces.
 *
 * Streams and errors: calls are enqueued on the stream given to gst_create and
 * return immediately.  Argument errors detectable on the host are returned at
 * once (negative gst_status) and nothing is enqueued.  Data-dependent errors
 * (a gate index >= K, a probability <= 0 where the count is > 0) are recorded
 * on the device and reported by gst_sync.  For GST_ENONPOS the objective is
 * written as +inf and the gradient output is left untouched.
 *
 * Probabilities are computed with one fused multiply-add per term, in ascending
 * column order from zero, exactly like the plain definition of the product;
 * objective and gradient are sums whose order differs from a sequential loop.
 * Results do not depend on what else runs on the device.
 *
 * Thread safety: a context must not be used by two host threads at once.
 */
#ifndef GST_H_
#define GST_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gst_status {
  GST_OK = 0,
  GST_EINVAL = -1,   /* bad shape, null pointer, unsupported size */
  GST_EINDEX = -2,   /* a gate index >= n_gates */
  GST_ENONPOS = -3,  /* p <= 0 where N > 0: objective = +inf */
  GST_ENOMEM = -4,   /* device allocation failed */
  GST_EDEVICE = -5,  /* HIP runtime error */
  GST_EBUSY = -6     /* admission refused (footprint or slots) */
} gst_status;

typedef struct gst_ctx gst_ctx;  /* opaque; one device, one stream */
typedef struct gst_req gst_req;  /* opaque resident request */

/* Gate set theta = (rho, effects, gates).  Device pointers. */
typedef struct gst_gateset {
  int n_qubits;          /* 1..3 */
  int n_gates;           /* K, 1..gst_max_gates(n_qubits) */
  int n_outcomes;        /* M, 1..D */
  const double* rho;     /* [D] */
  const double* effects; /* [M][D] */
  const double* gates;   /* [K][D][D] row-major */
} gst_gateset;

/* Sequence list.  Device pointers (host pointers for gst_req_create_host). */
typedef struct gst_seqlist {
  int64_t n_seq;            /* S >= 0 */
  const int64_t* offsets;   /* [S+1] */
  const uint8_t* gate_idx;  /* [offsets[S]] */
  int64_t max_len;          /* max_s (offsets[s+1]-offsets[s]) if known, else -1 */
} gst_seqlist;

/* Data-dependent diagnostics collected since the previous gst_sync. */
typedef struct gst_diag {
  int64_t n_bad_index;  /* gate indices >= K that were seen */
  int64_t n_nonpos;     /* entries with p <= 0 and N > 0 */
} gst_diag;

/* Largest K supported for a qubit count: 8 for one and two qubits (the
   on-chip gradient tiles of the tile kernels), 5 for three (the gate set of
   the per-sequence kernel fills the 160 KB of LDS of a CU); 0 for other qubit
   counts.  Every call given more gates returns GST_EINVAL. */
int gst_max_gates(int n_qubits);

/* Create a context on device `device_ordinal` that enqueues work on
   `hip_stream` (a hipStream_t; NULL = the default stream). */
int gst_create(gst_ctx** out, int device_ordinal, void* hip_stream);
int gst_destroy(gst_ctx* ctx);

/* Wait for all work enqueued by this context and report data-dependent
   errors since the previous call (GST_EINDEX before GST_ENONPOS).  `diag`
   may be NULL.  Resets the counters. */
int gst_sync(gst_ctx* ctx, gst_diag* diag);

/* Probabilities only: probs[S][M]. */
int gst_probs(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs, double* probs);

/* Objective (objective[0]), optionally probabilities and the gradient.
   probs and grad may be NULL; objective must not be NULL. */
int gst_loglik(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs,
               const int32_t* counts, double* probs, double* objective, double* grad);

/* Vector-Jacobian product: grad = sum_{s,m} w[s][m] dp[s][m]/dtheta (the
   backward of probs for automatic differentiation). */
int gst_vjp(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs, const double* w,
            double* grad);

/*
 * gst_loglik_noalloc: gst_loglik for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, outputs and kernels as gst_loglik; the
 * kernels' scratch (partial sums, checkpoints) lives in a static device array
 * of 128 MiB that each GPU running the library holds until the process ends,
 * and the call allocates nothing.  One or two qubits; seqs->max_len must be
 * given (>= 0), so that nothing is read back.  GST_EINVAL for three qubits, an
 * unknown max_len, or a list whose scratch exceeds the array (the message
 * names the bytes needed: about 8 (w P + 16 w (ceil(max_len / 8) + 1) 16)
 * with w = ceil(S / 16) workgroups, at most 2048, and P = 1 + D + M D + K D^2).
 * All calls on one GPU share the array: calls that overlap on one GPU (on
 * different streams) race, so keep them on one stream.
 */
int gst_loglik_noalloc(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs,
                       const int32_t* counts, double* probs, double* objective, double* grad);

/*
 * Resident requests: the sequence list and the counts are copied to the
 * device once, the prefix-sharing plan (a trie of the sequences, thesis Eq.
 * GSTFullFiducialsGerms: every distinct prefix is evaluated once) is built
 * once, and each evaluation only supplies a new gate set, as in the
 * iterations of a maximum-likelihood fit.
 *
 * gst_req_create_host: offsets, gate_idx and counts are HOST pointers; they
 * are copied before the call returns.  counts may be NULL (probs/vjp only).
 */
int gst_req_create_host(gst_ctx* ctx, int n_qubits, int n_gates, int n_outcomes,
                        const gst_seqlist* seqs_host, const int32_t* counts_host,
                        gst_req** out);
/* gst_req_create: the same with DEVICE pointers (offsets, gate_idx, counts on
   the context's device, as for gst_loglik).  The call waits for the context's
   stream, reads the list (and counts) back to build the plan on the host, and
   returns with its own copies; the caller's buffers may be reused at once.
   Argument errors as for gst_req_create_host, including GST_EINDEX for a gate
   index >= n_gates (reported at creation, not through gst_sync). */
int gst_req_create(gst_ctx* ctx, int n_qubits, int n_gates, int n_outcomes, const gst_seqlist* seqs,
                   const int32_t* counts, gst_req** out);
/* Device bytes held by the request (plan, copies of the inputs, workspace). */
int gst_req_footprint(const gst_req* req, size_t* bytes);
/* Evaluate at gate set `theta`; same outputs and conventions as gst_loglik. */
int gst_req_eval(gst_req* req, const gst_gateset* theta, double* probs, double* objective,
                 double* grad);
/* Probabilities only, with the request's resident sequence list. */
int gst_req_probs(gst_req* req, const gst_gateset* theta, double* probs);
/* vjp with the request's resident sequence list. */
int gst_req_vjp(gst_req* req, const gst_gateset* theta, const double* w, double* grad);
int gst_req_destroy(gst_req* req);
/* Sharing-plan statistics of a request (diagnostics): info[0..n) receives
   {plan used (0/1), total steps of the plain evaluation, trie nodes, trunks,
    trunk steps, item steps, levels, injection slots, chain mat-vecs of
    the trunks (jumps counted once), longest trunk chain, trunks with jumps,
    fill tasks, grouped-chain plan used (three qubits: 0/1), its tiles, its
    chains, its state rows}; n <= 16. */
int gst_req_plan_info(const gst_req* req, int64_t* info, int n);

/*
 * Batches: several resident requests evaluated together, as the continuous
 * batching of a fit service needs.  Requests without a sharing plan are cut
 * into tiles of 16 to 128 sequences (sorted by length; the cut depends on the
 * request alone) that one persistent launch takes from a work queue; every
 * tile writes its own partial sums and each request's tiles are added in
 * tile order, so each result is identical whether the request is evaluated
 * alone or in any batch.  The one- and two-qubit sharing plans of a batch run
 * together, one launch per plan kernel and level for all of them; each keeps
 * the partition of its partial sums (per item chunk, per trunk) of its
 * standalone evaluation, so its results too are identical alone and in any
 * batch.  The three-qubit grouped-chain plans likewise run as one launch per
 * kernel and level for all of them, each on its standalone grid; three-qubit
 * lists without a plan run their own launch sequences after these.
 *
 * gst_batch_create fixes the requests (each at most once: GST_EINVAL
 * otherwise), the gate sets (device pointers whose
 * contents may change between runs) and the output pointers; any of probs,
 * objectives, grads may be NULL or hold NULL entries (an objective is needed
 * for a gradient).  capture_graph != 0 records the batched launch sequence
 * into a HIP graph once (the sequences of three-qubit lists without a plan are
 * enqueued eagerly after it); gst_batch_run then replays it on the context
 * stream (eagerly instead while kernel timing is enabled).
 * gst_batch_nonpos synchronizes and returns, per request, the number of
 * p <= 0 entries with positive counts in the last run (objective +inf).
 */
typedef struct gst_batch gst_batch;
int gst_batch_create(gst_ctx* ctx, int n, gst_req* const* reqs, const gst_gateset* thetas,
                     double* const* probs, double* const* objectives, double* const* grads,
                     int capture_graph, gst_batch** out);
int gst_batch_run(gst_batch* batch);
int gst_batch_nonpos(gst_batch* batch, int64_t* counts);
int gst_batch_destroy(gst_batch* batch);

/*
 * Tile policy (the knob of the autotuner): sequences per tile and workgroups
 * per CU of the tile kernels for gate sets of `n_qubits` qubits, for the
 * requests created afterwards on this context (a request keeps the tile cut
 * it was created with, so its results stay the same alone and in any
 * batch).  seqs_per_tile is rounded up to the kernel's granularity (64 for
 * one qubit with at most four gates, else 16; any value for three qubits);
 * 0 restores the default.  blocks_per_cu = 0 uses as many as fit.
 */
int gst_tune_set(gst_ctx* ctx, int n_qubits, int seqs_per_tile, int blocks_per_cu);

/*
 * Germ-power jumps of the sharing plan, for requests created afterwards on
 * this context.  Germ-power sequences (thesis Eq. GSTFullFiducialsGerms) put
 * long runs of one repeated germ on a trunk.  With reps > 0 the trunk chain
 * applies such a run `reps` repetitions at a time with the matrix power of
 * the germ (built per evaluation in LDS by repeated squaring), and independent
 * fill tasks compute the states and adjoints inside each jump; this shortens
 * the sequential chain several times over.  The states after a jump carry the
 * rounding of the matrix products, so probabilities agree with the plain
 * evaluation to rounding (a few 1e-13 relative on the germ-power lists)
 * instead of bit for bit.  reps = 0 turns jumps off (bit-identical
 * probabilities); otherwise a power of two from 2 to 16.  Default 8.
 */
int gst_set_plan_jump(gst_ctx* ctx, int reps);

/*
 * Predictions of repeated gate applications (thesis Eq. GSTPrediction):
 *   probs[(p * n_gates + s) * (r_max + 1) + r][m] = <<E_m| (G_{gates[s]})^r G_prep(p) |rho>>
 * for r = 0 .. r_max, every preparation word p (host CSR: prep_offsets[n_prep + 1],
 * prep_gates in time order, at most 64 gates each, gate indices < n_gates of theta)
 * and every gate index gates[s] (host array of n_gates).  One or two qubits; theta
 * and probs are device pointers, probs holds n_prep * n_gates * (r_max + 1) * M
 * doubles.  The powers run in blocks of 32 repetitions: a chain steps from block to
 * block with (G_s)^32 (built per call by repeated squaring) and every block then
 * takes single steps, so the probabilities for r < 32 equal the plain evaluation of
 * the word bit for bit and later ones agree to rounding.  The host arrays are read
 * before the call returns (copied into pinned staging memory); the evaluation is
 * stream-ordered on the context's stream and the call does not wait for it.  The
 * context's workspace holds the block-start states until the next call.  GST_EINVAL for
 * three qubits, a word longer than 64 gates, a gate index out of range,
 * r_max outside 0 .. 2^24 or more than 2^24 (preparation, gate) pairs.
 */
int gst_predict(gst_ctx* ctx, const gst_gateset* theta, int n_prep, const int64_t* prep_offsets,
                const uint8_t* prep_gates, int n_gates, const int32_t* gates, int r_max, double* probs);

/*
 * Statistical (total variation) distance of Eq. statisticaldistance for n rows of
 * m probabilities: out[i] = 1/2 sum_j |p[i*m + j] - q[i*m + j]| (j ascending).
 * Device pointers; stream-ordered.
 */
int gst_tv_distance(gst_ctx* ctx, const double* p, const double* q, int64_t n, int m, double* out);

/*
 * Parameterizations of the gate set: the estimation modes of the fit (thesis
 * Sec. 6.3.2: fully unconstrained, trace-preserving, completely positive and
 * trace-preserving).  A parameter vector theta (device, doubles) maps to the full
 * parameterization (rho [D], effects [M][D], gates [K][D][D], the layout of
 * gst_gateset), and the gradient with respect to the full parameters
 * ([rho | effects | gates], the layout of gst_loglik's grad) maps back to theta.
 *
 *   GST_PARAM_FULL: theta is the full parameter vector itself.
 *   GST_PARAM_TP:   row 0 of every gate is e_0 (trace preservation), rho[0] = 1/sqrt(d)
 *                   (unit trace), effect M-1 = vec(1) - sum of the others (complete).
 *                   theta = [rho[1..D-1] | effects 0..M-2 | rows 1..D-1 of each gate].
 *   GST_PARAM_CPTP: G_k = exp(L_k) targets_k (Eq. GateDecompositionLindbladCorrespondence),
 *                   L_k the transfer matrix of -i[H, .] + sum_jk C_jk (P_j . P_k - {P_k P_j, .}/2),
 *                   H = sum_{k>=1} h_k P_k / 2 (Eq. GateDecompositionHamiltonian), C = T T^dagger
 *                   (Eq. masterequation's form with a positive semidefinite coefficient
 *                   matrix, so every gate is CPTP); rho = A A^dagger / tr(A A^dagger); effects as TP.
 *                   theta = [A (D) | effects 0..M-2 | per gate: h (D-1), T ((D-1)^2)], A and T
 *                   as their real diagonals followed by the entries below the diagonal in
 *                   row-major order as (real, imaginary) pairs; P_j in the order of the basis.
 *                   One and two qubits; `targets` = the fixed gates G0 [K][D][D] (device).
 *
 * gst_param_count: the length of theta.  gst_param_forward writes rho, effects
 * and gates (device); gst_param_backward writes grad_theta (device, the length of
 * theta) from grad_full.  Stream-ordered; TP maps are exact (bit-identical
 * copies and differences), CPTP gates use a degree-16 Taylor polynomial with
 * scaling and squaring (and its block form for the adjoint of the derivative).
 * GST_EINVAL for an unknown mode, sizes out of range, CPTP with three qubits or
 * without targets, NULL pointers.
 */
enum { GST_PARAM_FULL = 0, GST_PARAM_TP = 1, GST_PARAM_CPTP = 2 };
int gst_param_count(int mode, int n_qubits, int n_outcomes, int n_gates, int64_t* count);
int gst_param_forward(gst_ctx* ctx, int mode, int n_qubits, int n_outcomes, int n_gates, const double* theta,
                      const double* targets, double* rho, double* effects, double* gates);
int gst_param_backward(gst_ctx* ctx, int mode, int n_qubits, int n_outcomes, int n_gates, const double* theta,
                       const double* targets, const double* grad_full, double* grad_theta);

/*
 * The fit (thesis Sec. 6.3.1).  The gate set is determined only up to the GST
 * gauge (E -> E X^-1, G -> X G X^-1, rho -> X rho).
 *
 * gst_lgst: linear-inversion estimates from a host sequence list with counts.
 * The list must hold, for every preparation fiducial F_j and measurement
 * fiducial F_i (host CSR word lists, time order, each containing the empty
 * word), the words F_j F_i and F_j G_k F_i for every gate k.  AB[J + M i][j] and
 * B_k[J + M i][j] are their outcome frequencies; with AB = U S V^T truncated to
 * rank D (each singular pair signed so that the largest-magnitude entry of its V
 * column is positive) and Ahat = U^T AB V: G_k = Ahat^-1 U^T B_k V,
 * rho = Ahat^-1 U^T AB[:, empty], E_J = AB[J + M empty, :] V (host outputs).
 * GST_EINVAL if a word is missing, a fiducial list lacks the empty word, or AB
 * has rank below D.
 *
 * gst_gauge_optimize: minimizes sum_k ||X G_k X^-1 - T_k||_F^2 + w (||X rho - rho_T||^2
 * + sum_m ||X^-T e_m - e_T,m||^2) over X (L-BFGS until the largest gradient
 * entry is <= gtol) from the least-squares solution of the same relations
 * multiplied through by X (X G_k = T_k X, X rho = rho_T, X^T e_T,m = e_m: linear in
 * X), and applies X to rho, effects and gates in place (one or two qubits: the
 * linear start solves D^2 normal equations)
 * (host arrays); optional outputs: X (row-major D x D) and the objective.
 *
 * gst_mlgst: iterative MLGST on the GPU.  For each stage (resident requests of
 * this context, same sizes, usually lists of growing length) it minimizes the
 * negative log-likelihood per shot (F / sum of the stage's counts) over theta
 * in the TP or CPTP parameterization (gst_param_*) with limited-memory BFGS
 * (two-loop recursion with opt->memory pairs; strong Wolfe line search with
 * c1 = 1e-4, c2 = 0.9: the step doubles from 1 until it brackets an acceptable
 * one, then the bracket is bisected; a step with some p <= 0 where N > 0
 * counts as too long),
 * starting from the previous stage's result.  theta: host array of
 * gst_param_count entries, in/out.  reports (optional): one per stage.
 * A stage whose start gives some p <= 0 where N > 0 starts instead from it moved
 * inward by the smallest delta in 2^-10, 2^-9, ..., 1/2 that makes the
 * likelihood finite: TP (an estimate need not be completely positive) with
 * every gate depolarized (rows 1.. of the transfer matrices times 1 - delta);
 * CPTP (gates and state are physical, the effects only complete) with the free
 * effects mixed with the uniform POVM: e_m <- (1 - delta) e_m + delta vec(1)/M.
 * GST_ENONPOS if a stage still starts where some p <= 0 with N > 0 (no direction
 * of descent is defined there); theta then holds that start.
 * Errors pending on the context before the call are returned (gst_sync) and
 * the fit does not start; the data-error counters are clear afterwards.
 */
typedef struct gst_fit_options {
  int max_iter;  /* iterations per stage, >= 1 */
  double gtol;   /* stop when max |dF/dtheta| / sum N <= gtol */
  int memory;    /* correction pairs, 1..100 */
} gst_fit_options;
typedef struct gst_fit_report {
  int iterations;
  int evaluations;
  int status;        /* 0 tolerance met, 1 iteration limit, 2 the line search found no decrease */
  double objective;  /* F at the stage's result */
  double grad_max;   /* max |dF/dtheta| / sum N there */
  double shrink;     /* delta applied to the stage's start (0 = none) */
} gst_fit_report;
int gst_lgst(int n_qubits, int n_outcomes, int n_gates, int64_t n_seq, const int64_t* offsets, const uint8_t* gate_idx,
             const int32_t* counts, int n_prep, const int64_t* prep_offsets, const uint8_t* prep_gates, int n_meas,
             const int64_t* meas_offsets, const uint8_t* meas_gates, double* rho, double* effects, double* gates);
int gst_gauge_optimize(int n_qubits, int n_outcomes, int n_gates, double* rho, double* effects, double* gates,
                       const double* target_rho, const double* target_effects, const double* target_gates,
                       double spam_weight, double gtol, double* gauge, double* objective);
int gst_mlgst(gst_ctx* ctx, int n_stages, gst_req* const* stages, int mode, const double* targets, double* theta,
              const gst_fit_options* opt, gst_fit_report* reports);

/*
 * Post-fit metrics of estimates (host arrays).
 *
 * gst_avg_gate_fidelity: for each gate k, the average gate fidelity (thesis Eq.
 * gatemetricsaveragegatefidelity) of the transfer matrix gates[k] against the
 * unitary channel with transfer matrix targets[k]: (Tr(T^T R) + N R[0][0]) /
 * (N (N + 1)), N = 2^n (for R of rho -> M rho M^dagger the closed form Eq.
 * gatemetricsaveragegatefidelityEvaluation).
 *
 * gst_diamond_unitary: diamond distance of the channels of the dim x dim
 * unitaries U and V (row-major, interleaved real and imaginary parts), App. H
 * Eq. appdiamondunitaryResult: 1 if the origin lies in the convex hull of the
 * eigenvalues of U^dagger V, else half their largest distance.
 *
 * gst_hamiltonian_decomposition: App. J for the transfer matrix G: h (D entries,
 * h[0] = 0) of the projection of the real principal logarithm of G onto the
 * transfer matrices of -i[H, .], H = sum_k h_k P_k / 2 (Eq.
 * GateDecompositionHamiltonianProjection); angle = |h| (Eq. GSTHamiltonianAngle,
 * the axis is h / |h|); gamma = ||G - exp(L^H)||_F (Eq.
 * GateDecompositionHamiltonianProjectionError).  GST_EINVAL where G has no real
 * principal logarithm (an eigenvalue on the closed negative real axis, e.g. the
 * ideal CZ).  angle and gamma may be NULL.
 */
int gst_avg_gate_fidelity(int n_qubits, int n_gates, const double* gates, const double* targets, double* f_avg);
int gst_diamond_unitary(int dim, const double* U, const double* V, double* dist);
int gst_hamiltonian_decomposition(int n_qubits, const double* G, double* h, double* angle, double* gamma);
/*
 * gst_hamiltonian_decomposition_target: App. J's other route, which also covers
 * gates without a real principal logarithm (the ideal CZ and CNOT, whose
 * transfer matrices have eigenvalues -1): h (D entries, h[0] = 0) minimizing
 * gamma(h) = ||G - exp(L^H(h))||_F (Eq. GateDecompositionHamiltonianProjectionError)
 * by L-BFGS, starting from the Hamiltonian of the intended target unitary U
 * (dim x dim, dim = 2^n, row-major, interleaved real and imaginary parts):
 * H_U = i log U with each eigenvalue's argument in (-pi, pi].  angle = |h|,
 * gamma at the result (both may be NULL).  One or two qubits; GST_EINVAL
 * otherwise or if the target's eigen-decomposition fails.
 */
int gst_hamiltonian_decomposition_target(int n_qubits, const double* G, const double* U, double* h, double* angle,
                                         double* gamma);

/*
 * Kernel timing (diagnostics).  While enabled, every kernel the context
 * enqueues is launched with a pair of HIP events on the context's stream that
 * the runtime stamps with the kernel's own start and end (no marker is queued
 * between kernels).  A family's time is the sum over its kernels, and a
 * kernel also counts for the families enclosing it ("batch").
 * gst_profile_read synchronizes the stream and returns, for the kernel family
 * `kernel` ("leaf", "reduce", "trunk_fwd", "trunk_bwd", "inject",
 * "grad_gemm", "fill", "tiles_2q", "tiles_1q", "tiles_reduce",
 * "chain_3q", "gemm_3q", "reduce_3q", "predict_chain", "predict_fill",
 * "tv_distance", "param_fwd", "param_bwd", or "batch" for a whole
 * gst_batch_run), the summed
 * elapsed milliseconds and the number of kernels since profiling was
 * enabled; the counters are not reset by reading.
 */
int gst_profile_enable(gst_ctx* ctx, int enable);
/* Restrict the events to one kernel family (NULL = all families): a timed
   region can then carry the events of the kernel it reports on and no
   others. */
int gst_profile_only(gst_ctx* ctx, const char* kernel);
int gst_profile_read(gst_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);

/* Message of the last failing call on this host thread ("" if none). */
const char* gst_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GST_H_ */
