/*
 * qaoa.h — C ABI of the MI355X (gfx950) QAOA statevector library (libqaoa.so).
 *
 * The library evaluates the p-round QAOA state of Eq. (1) of Golden et al., "JuliQAOA:
 * Fast, Flexible QAOA Simulation" (SC-W 2023):
 *
 *   |beta, gamma> = e^{-i beta_p H_M} e^{-i gamma_p H_C} ... e^{-i beta_1 H_M} e^{-i gamma_1 H_C} |psi0>
 *
 * with H_C |x> = C(x) |x> (Sec. 1), the objective <beta,gamma| H_C |beta,gamma> (Sec. 1) and
 * its gradient in (beta, gamma) (Sec. 2.3 and Sec. 4). The calls follow the paper's problem
 * statement (a cost function tabulated over the feasible states, an initial state, a mixer,
 * 2p angles; Sec. 1 and Sec. 2.1) and its simulate/expectation calls (Sec. 3).
 *
 * Conventions shared by every call:
 *  - Basis index x = sum_i x_i 2^i: vertex i of the graph is bit i of x. For a Hamming-weight
 *    constrained problem the feasible states are the weight-k integers in increasing order
 *    (the order in which Gosper's hack walks them, Sec. 2.4) and amplitudes are stored in that
 *    order.
 *  - Angles are FP64, laid out [beta_1 .. beta_p, gamma_1 .. gamma_p] (first code listing,
 *    Sec. 3). Gradients use the same layout. Batched angles are [n_sets][2p], row major.
 *  - <C> is returned as E / Nrm with E = sum_x |psi(x)|^2 C(x) and Nrm = sum_x |psi(x)|^2
 *    (Nrm is 1 in exact arithmetic; dividing removes rounding drift of the norm). The
 *    gradient is returned divided by the same Nrm. Callers maximise <C>; to minimise, negate
 *    (Sec. 3, angle-finding paragraph).
 *  - Pointers named host_* / out_* are host memory owned by the caller. Pointers named d_*
 *    are device memory on the context's device, owned by the caller. Handles own their own
 *    device buffers (the cost table, the mixer eigenbasis, state and scratch vectors), which
 *    are allocated when the handle or the first evaluation needs them and reused afterwards
 *    (pre-allocated, reused memory: Sec. 2.2).
 *  - Streams: every call takes a hipStream_t passed as void* (NULL = the null stream). Work is
 *    enqueued on that stream; calls with host outputs synchronise that stream before return.
 *  - Calls that share a context must not overlap in time (same stream, or host-serialised):
 *    the context's scratch vectors are reused by every evaluation.
 *  - Errors: every call returns a status (0 = QAOA_OK, negative = error). On error outputs
 *    are undefined and qaoa_last_error() returns a thread-local message. No C++ exception
 *    crosses this interface.
 */
#ifndef QAOA_H
#define QAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define QAOA_OK 0
#define QAOA_ERR_INVALID_ARG (-1)   /* an argument is out of range, NULL, or inconsistent */
#define QAOA_ERR_OUT_OF_MEMORY (-2) /* a device or host allocation failed                */
#define QAOA_ERR_HIP (-3)           /* a HIP runtime call or kernel launch failed        */
#define QAOA_ERR_UNSUPPORTED (-4)   /* valid request this build does not implement        */

/* Arithmetic of the state vector. QAOA_FP32: complex64 amplitudes, FP32 arithmetic, FP64
 * accumulation of every sum (<C>, norm, gradient). QAOA_FP64: complex128 throughout. */
#define QAOA_FP32 0
#define QAOA_FP64 1

typedef struct qaoa_ctx qaoa_ctx;         /* one HIP device + reusable scratch         */
typedef struct qaoa_problem qaoa_problem; /* cost diagonal C(x) over the feasible set   */
typedef struct qaoa_mixer qaoa_mixer;     /* H_M: transverse field, eigenbasis mixers (clique, ring, matrix), Grover, X products */

/* Create a context on HIP device `hip_device` (>= 0). *out receives the handle.
 * INVALID_ARG for a bad device index or out == NULL; HIP on runtime failure.
 * Read once here from the environment (both optional, for tests and memory-limited runs):
 * QAOA_GRAD_CHECKPOINT = "0" never keep the forward passes' outputs for the gradient's
 * reverse sweep (undo the state in place), "1" always keep them; unset: keep them when they
 * fit in half the free device memory. QAOA_XPROD_TILES = "0" runs X-product and per-qubit
 * mixers on separate Walsh-Hadamard and diagonal kernels instead of the tile passes.
 * QAOA_AUTOTUNE = "1" turns the plan tuner on (qaoa_ctx_set_autotune). */
int qaoa_ctx_create(int hip_device, qaoa_ctx **out);

/* Plan tuner of the tile-pass evaluations (every problem above the whole-state size: the
 * transverse-field mixer and the X-product mixers). A plan fixes choices that leave the
 * result exact up to rounding: the reverse sweep reading the forward passes' outputs or
 * undoing the state in place, the tile cover (narrow 64-byte runs where they save a tile;
 * which strided tile takes the narrowest runs, also the odd bit of two evenly split strided
 * tiles), which tile rotates the low qubits, the tile order of the first
 * round, which strided tile takes the round boundaries (three tiles), the XCD-aware
 * workgroup order, and, on narrow covers of the transverse-field mixer, the state layout in
 * device memory (natural, or the top ten index bits XOR-folded into ten middle ones; never
 * visible to the caller: an evaluation with a caller's initial state or final-state output
 * runs the natural layout; the layout changes no arithmetic, so its results are identical
 * bit for bit). Off (enable = 0, the default): a fixed rule.
 * On: the first evaluation of each (n, precision, gradient or not, mixer, whether the
 * checkpoints fit in memory) times the alternatives one at a time on the caller's stream
 * (min(p, 4) layers per trial, by the summed kernel durations; a change is kept when it is
 * at least 2 % faster) and keeps the fastest. Every later evaluation of that key, single or
 * batched, any number of angle sets, uses the choice; a batched call itself does not tune
 * (an instance whose key has no choice yet follows the fixed rule). Different
 * plans round differently (FP32: within the 1e-5 bound), so a run that must repeat another
 * bit for bit saves the plans (qaoa_plans_save) and loads them (qaoa_plans_load).
 * INVALID_ARG for ctx == NULL. */
int qaoa_ctx_set_autotune(qaoa_ctx *ctx, int enable);

/* The context's chosen plans as text, one line per key:
 *   "n precision grad mixer ckpt_fits : narrow narrow_top lowbits down xcd ckpt swap swz"
 * after a header line "qaoa-plans 3" (files with the header "qaoa-plans 1" and no swap field
 * still load, with swap 0; files with "qaoa-plans 1" or "qaoa-plans 2" and no swz field load
 * with swz 1, the fixed rule's layout). buf may be NULL; *needed (if not NULL) receives the
 * length including the terminating NUL; at most len bytes are written (always terminated
 * when len > 0). INVALID_ARG for ctx == NULL. */
int qaoa_plans_text(const qaoa_ctx *ctx, char *buf, size_t len, size_t *needed);

/* Write the plans to a file (qaoa_plans_text's format; written to path.tmp and renamed), or
 * add the plans of such a file to the context (a line for a key already present replaces
 * it). INVALID_ARG for NULL arguments or a malformed file; HIP is not involved. */
int qaoa_plans_save(const qaoa_ctx *ctx, const char *path);
int qaoa_plans_load(qaoa_ctx *ctx, const char *path);

/* Destroy a context and free its scratch. Problems and mixers created on it must be
 * destroyed first: while any is alive the call returns QAOA_ERR_INVALID_ARG and destroys
 * nothing. NULL is accepted (no-op). */
int qaoa_ctx_destroy(qaoa_ctx *ctx);

/* Step (a): tabulate the MaxCut cost diagonal on the device (Sec. 2.1, pre-computation):
 *   C(x) = sum_{e < n_edges} w[e] * [bit u[e] of x != bit v[e] of x]
 * for every feasible x: all 2^n strings (hamming_k < 0) or the weight-k strings in
 * increasing order (0 <= hamming_k <= n). u, v, w are host arrays of n_edges int32
 * (w == NULL: unit weights). Requires 1 <= n <= 32 (hamming_k >= 0: C(n,k) <= 2^26),
 * 0 <= u, v < n, u != v, w >= 0 and sum of w <= 65535 (the table is stored as uint8 when
 * every value is <= 255, else uint16). The table is computed exactly (integers).
 * *out owns the device table. The call synchronises `stream`. */
int qaoa_cost_table(qaoa_ctx *ctx, int n, int n_edges, const int32_t *u, const int32_t *v,
                    const int32_t *w, int hamming_k, qaoa_problem **out, void *stream);

/* Step (a) for any objective (Sec. 2.1 pre-computation; Sec. 3 hands the objective over as a
 * list of values, one per feasible state): C(x) = host_values[i] for the i-th feasible state
 * in the basis order above (x = i over all 2^n strings for hamming_k < 0, the i-th weight-k
 * integer for 0 <= hamming_k <= n). host_values: len finite doubles, len = feasible-set size,
 * caller-owned, read during the call only. At most 1024 distinct values (the phase is applied
 * through a table of e^{-i gamma c} over the distinct values c; QAOA_ERR_UNSUPPORTED beyond
 * that); the device table stores each state's index among the distinct values in increasing
 * order (uint8 for up to 256 of them, else uint16). Tables with C(~x) != C(x) are supported
 * (the transverse-field path then also keeps the reversed table). *out owns the device
 * table. Synchronises `stream`. */
int qaoa_problem_from_values(qaoa_ctx *ctx, int n, int hamming_k, const double *host_values, size_t len,
                             qaoa_problem **out, void *stream);

/* Copy the table back as int64 into host_dst (len must equal the feasible-set size), in the
 * basis order above: the cost values of a graph problem (qaoa_cost_table), the value indices
 * of a qaoa_problem_from_values problem. For exact comparisons; synchronises `stream`. */
int qaoa_problem_copy_table(const qaoa_problem *prob, int64_t *host_dst, size_t len, void *stream);

/* Copy C(x) as doubles into host_dst (len = feasible-set size, basis order above), for either
 * kind of problem. Synchronises `stream`. */
int qaoa_problem_copy_values(const qaoa_problem *prob, double *host_dst, size_t len, void *stream);

/* Problem metadata: qubits n, hamming_k (-1 = unconstrained), feasible-set size, largest
 * table entry (a graph problem's largest C value; for a qaoa_problem_from_values problem the
 * number of distinct values minus one). Any output pointer may be NULL. */
int qaoa_problem_info(const qaoa_problem *prob, int *n, int *hamming_k, int64_t *size,
                      int64_t *max_value);

/* Free a problem (NULL accepted). */
int qaoa_problem_destroy(qaoa_problem *prob);

/* Transverse-field mixer H_M = sum_q X_q on n qubits (Sec. 2.1; the factorisation of
 * Eq. (2): e^{-i b H_M} is a product of single-qubit rotations). 1 <= n <= 32. */
int qaoa_mixer_x(qaoa_ctx *ctx, int n, qaoa_mixer **out);

/* Clique mixer H_M = sum_{i<j} X_i X_j + Y_i Y_j restricted to Hamming weight k (Sec. 2.1):
 * its matrix on the weight-k strings has entry 2 between strings that differ by moving one
 * 1-bit, else 0. The eigendecomposition H_M = V D V^T is computed once here in FP64 on the
 * device (V is real orthogonal, so V^{-1} = V^T) and kept by the handle. Requires
 * 2 <= n <= 20, 1 <= k <= n-1 and C(n,k) <= 16384. Synchronises `stream`. */
int qaoa_mixer_clique(qaoa_ctx *ctx, int n, int k, qaoa_mixer **out, void *stream);

/* Ring mixer H_M = sum_i X_i X_{i+1} + Y_i Y_{i+1} (Sec. 2.1; i + 1 taken mod n, so the ring
 * closes for n >= 3) restricted to Hamming weight k: entry 2 between strings that differ by
 * swapping the bits of one ring edge. Applied like the clique mixer (FP64 eigendecomposition
 * once, V kept by the handle); same limits. Synchronises `stream`. */
int qaoa_mixer_ring(qaoa_ctx *ctx, int n, int k, qaoa_mixer **out, void *stream);

/* Mixer given as a matrix (Sec. 2.1: any mixer can be handed over as a matrix, and its
 * eigendecomposition is computed and stored): host_matrix is an N x N real symmetric matrix
 * (row i, column j at host_matrix[i * N + j]; symmetric to 1e-12 of its largest entry, else
 * INVALID_ARG) over the feasible states in the basis order above, N = 2^n for hamming_k < 0
 * or C(n, hamming_k) otherwise, N <= 16384, read during the call only. Applied like the clique
 * mixer. Synchronises `stream`. */
int qaoa_mixer_matrix(qaoa_ctx *ctx, int n, int hamming_k, const double *host_matrix, qaoa_mixer **out,
                      void *stream);

/* Mixers built from products of Pauli X (Sec. 2.1, Eq. (2): a Hadamard on every qubit turns
 * f(X) into the diagonal f(Z)), for unconstrained problems, n <= 32. Every layer runs as the
 * cost phase, a Walsh-Hadamard transform, the diagonal e^{-i beta d(y)} and the transform again,
 * in FP32 or FP64 like the other mixers; the gradient comes from the same reverse sweep.
 *
 * qaoa_mixer_x_orders: H_M = sum over k in orders[0..n_orders) of the sum over all k-subsets S
 * of prod_{i in S} X_i (orders distinct, in [1, n]; {1} is the transverse field). The diagonal
 * depends on the Hamming weight w of y only: d = sum_k K_k(w), K_k the Krawtchouk polynomial. */
int qaoa_mixer_x_orders(qaoa_ctx *ctx, int n, const int *orders, int n_orders, qaoa_mixer **out);

/* H_M = sum_t coefs[t] prod_{i: bit i of masks[t] set} X_i, 1 <= n_terms <= 10 (masks nonzero,
 * below 2^n; coefs finite). d(y) = sum_t coefs[t] (-1)^{popcount(y & masks[t])}. */
int qaoa_mixer_x_terms(qaoa_ctx *ctx, int n, const uint64_t *masks, const double *coefs, int n_terms,
                       qaoa_mixer **out);

/* Multi-angle mixer (Sec. 3: several mixers per layer, each with its own angle): layer k applies
 * prod_q e^{-i beta_{k,q} X_q}. With this mixer an angle set holds p (n + 1) entries,
 * [beta_{1,0..n-1}, ..., beta_{p,0..n-1}, gamma_1..gamma_p], and the gradient has the same
 * layout; qaoa_expect, qaoa_expect_grad, qaoa_state and the batched and paired calls accept it
 * (all mixers of one batched or paired call must take the same number of angles). */
int qaoa_mixer_x_multiangle(qaoa_ctx *ctx, int n, qaoa_mixer **out);

/* Mixer metadata: qubits, hamming_k (-1: all states), angles per layer of an angle set (2, or
 * n + 1 for the multi-angle mixer). Any output pointer may be NULL. */
int qaoa_mixer_info(const qaoa_mixer *mix, int *n, int *hamming_k, int *angles_per_layer);

/* Stored eigendecomposition of a clique, ring or matrix mixer (Sec. 2.1: the decomposition
 * is computed once and stored for re-use): copies the FP64 eigenvectors (column j, the j-th
 * eigenvector, at host_V[j * N .. j * N + N)) and eigenvalues host_D[0..N) to the host. N must
 * equal the mixer's state count. QAOA_ERR_UNSUPPORTED for the transverse-field and Grover
 * mixers. Synchronises `stream`. */
int qaoa_mixer_eigen(const qaoa_mixer *mix, double *host_V, double *host_D, size_t N, void *stream);

/* A mixer from a stored eigendecomposition H_M = V diag(D) V^T (the layout of qaoa_mixer_eigen)
 * over the feasible states of (n, hamming_k), N <= 16384: no eigensolver runs. V must be real
 * orthogonal; the call checks that entries are finite and columns have unit length (to 1e-9),
 * not full orthogonality. Applied like the clique mixer. Synchronises `stream`. */
int qaoa_mixer_from_eigen(qaoa_ctx *ctx, int n, int hamming_k, const double *host_V, const double *host_D,
                          qaoa_mixer **out, void *stream);

/* Grover mixer H_M = |psi0><psi0| (Sec. 2.4), psi0 the equal superposition over the feasible
 * states of an n-qubit problem (all 2^n for hamming_k < 0, else the weight-k states; the mixer
 * keeps the Hamming weight). 1 <= n <= 62. Evaluations with it use fair sampling (Sec. 2.4):
 * states of equal cost keep equal amplitudes, so the rounds run on the problem's distinct cost
 * values weighted by their degeneracies (counted once per problem, on first use), in FP64 for
 * either precision argument; at most 2048 distinct values (table indices for a tabulated
 * problem). Only the default initial state (d_psi0 == NULL). qaoa_state expands the result
 * over a tabulated problem's states. */
int qaoa_mixer_grover(qaoa_ctx *ctx, int n, int hamming_k, qaoa_mixer **out);

/* Degeneracies of the MaxCut cost without a table (Sec. 2.4: for the Grover mixer only the
 * distinct values and how many states take each are stored, counted in parallel over the
 * states): all 2^n strings (hamming_k < 0, 1 <= n <= 40; consecutive states in Gray-code order)
 * or the weight-k strings (Gosper's order, n <= 32). Edges as qaoa_cost_table, total
 * weight <= 16383. *out is a problem with no table: it serves qaoa_mixer_grover evaluations
 * (batched included) and qaoa_problem_degeneracies; other mixers, qaoa_state and the table
 * copies return QAOA_ERR_UNSUPPORTED. Synchronises `stream`. */
int qaoa_cost_degeneracies(qaoa_ctx *ctx, int n, int n_edges, const int32_t *u, const int32_t *v,
                           const int32_t *w, int hamming_k, qaoa_problem **out, void *stream);

/* Distinct cost values (increasing) that at least one feasible state takes, with their
 * degeneracies: values[i], counts[i] for i < *count (host arrays of cap entries, either may
 * be NULL to query *count only; INVALID_ARG when cap is too small). Counts a tabulated
 * problem's table on first use. */
int qaoa_problem_degeneracies(const qaoa_problem *prob, double *values, int64_t *counts, size_t cap,
                              size_t *count, void *stream);

/* Free a mixer (NULL accepted). */
int qaoa_mixer_destroy(qaoa_mixer *mix);

/* <C> for one angle set: evolve Eq. (1) with p >= 1 rounds and reduce step (d).
 * angles: host double[2p], finite. d_psi0: device initial state (complex64 for QAOA_FP32,
 * complex128 for QAOA_FP64, feasible-set order, need not be normalised) or NULL for the
 * default start, the uniform superposition over the feasible set (Sec. 3). The mixer must
 * act on the problem's space (same n; clique mixers need the same hamming_k).
 * *out_expect receives E / Nrm. Synchronises `stream`. */
int qaoa_expect(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *angles,
                const void *d_psi0, int precision, double *out_expect, void *stream);

/* <C> and d<C>/d(beta, gamma) for one angle set (gradient: Sec. 2.3 and Sec. 4). The
 * gradient is formed by a reverse sweep that undoes each layer (inverse mixer and inverse
 * phase applied to the state and to the adjoint vector), so no per-layer states are kept.
 * out_grad: host double[2p], layout of `angles`. Other arguments as qaoa_expect. */
int qaoa_expect_grad(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *angles,
                     const void *d_psi0, int precision, double *out_expect, double *out_grad,
                     void *stream);

/* Final state psi_p of Eq. (1) (Sec. 3: the simulate result holds the state vector), written
 * to d_out (device, caller-owned, feasible-set length, complex64 or complex128 by
 * `precision`), not renormalised. Other arguments as qaoa_expect. */
int qaoa_state(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *angles,
               const void *d_psi0, int precision, void *d_out, void *stream);

/* Batched <C>: every problem probs[i] (with mixer mixers[i]) at every angle set
 * angles[s][0..2p), s < n_sets, default initial state (the repeated evaluations of the
 * angle-finding loops, Sec. 2.3 and Sec. 3). out_expect: host double [n_probs][n_sets].
 * Every (problem, set) pair whose state fits one workgroup (n <= 13 for QAOA_FP32, n <= 12
 * for QAOA_FP64, transverse-field mixer) runs in one launch, one workgroup per pair; each
 * larger problem runs as one sequence of tile passes (or eigenbasis products) that covers
 * all n_sets angle sets per launch. Problems may differ in n and in mixer. A call repeats bit
 * for bit; its results equal single evaluations' bit for bit except in the QAOA_FP32 form of
 * the eigenbasis mixers when a product needs more than one round of the GPU's workgroups
 * (about 320 sets at C(16,8) states): such products split part of their sums along K over
 * two XCDs and round differently, within the same error bound. */
int qaoa_expect_batched(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers,
                        int n_probs, int n_sets, int p, const double *angles, int precision,
                        double *out_expect, void *stream);

/* Batched <C> and gradient; out_grad: host double [n_probs][n_sets][2p]. */
int qaoa_expect_grad_batched(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers,
                             int n_probs, int n_sets, int p, const double *angles, int precision,
                             double *out_expect, double *out_grad, void *stream);

/* <C> of n_pairs independent evaluations: pair i is problem probs[i] with mixer mixers[i] at
 * angles[i][0..2p) (the many instances of an angle-finding study, each at its own point).
 * probs and mixers are arrays of n_pairs handles (repeats allowed, one context); out_expect:
 * host double [n_pairs]. Whole-state transverse-field pairs and Grover-mixer pairs each run
 * as one launch over all pairs; the other pairs run grouped by (problem, mixer). */
int qaoa_expect_pairs(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_pairs, int p,
                      const double *angles, int precision, double *out_expect, void *stream);

/* As qaoa_expect_pairs, with the gradient; out_grad: host double [n_pairs][2p]. */
int qaoa_expect_grad_pairs(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_pairs, int p,
                           const double *angles, int precision, double *out_expect, double *out_grad,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): qaoa_expect_grad_pairs restricted to pairs whose
 * state fits one workgroup (transverse-field mixer, n <= 13 for QAOA_FP32, n <= 12 for
 * QAOA_FP64), with the same arguments, kernels and results. The items, angle sets and result
 * rows of a call live in a 4 MiB device array that the library holds per GPU from load to
 * process end; the call makes no device allocation (the problems' tables were built when
 * they were created). A call needs 56 n_pairs + 8 n_pairs (4p + 1) bytes plus alignment:
 * beyond 4 MiB it returns QAOA_ERR_INVALID_ARG; other pairs give QAOA_ERR_UNSUPPORTED.
 * Every call on one GPU shares that array (and a host staging array): calls that overlap in
 * time, on any stream or thread, race. Synchronises `stream`. */
int qaoa_expect_grad_pairs_noalloc(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_pairs,
                                   int p, const double *angles, int precision, double *out_expect, double *out_grad,
                                   void *stream);

/* ---------------------------------------------------------------- angle finding (Sec. 2.3)
 *
 * Host-side outer loop over the paired evaluation: every objective value and gradient comes
 * from qaoa_expect_grad_pairs, with all restarts (or basinhopping chains) of a step, of every
 * instance being solved, as its pairs, so one launch advances all of them. The objective is <C> (maximised by
 * default, Sec. 3; minimised with maximize = 0). The optimiser state lives in host memory. */
typedef struct qaoa_angle_opts {
  int maximize;          /* 1: maximise <C> (default); 0: minimise                          */
  int precision;         /* QAOA_FP32 (default) or QAOA_FP64 evaluations                    */
  int max_iter;          /* BFGS: accepted steps per local minimisation (default 100)       */
  double gtol;           /* BFGS: stop once max_i |d<C>/d angle_i| <= gtol max(1, |<C>|) (1e-5) */
  int n_chains;          /* basinhopping chains run side by side (default 8), <= 65535     */
  int n_hops;            /* basinhopping steps per chain after the first minimisation (10)  */
  double step;           /* hop: each angle moves by a uniform draw in [-step, step] (0.5)  */
  double temperature;    /* Metropolis temperature in units of <C> (1.0); 0: improvements only */
  uint64_t seed;         /* counter-based random draws (SplitMix64), keyed by round, chain, hop */
  int max_sets_per_call; /* angle sets per batched call; 0: automatic (see qaoa_minimize)    */
} qaoa_angle_opts;

/* Fill *opts with the defaults above. */
void qaoa_angle_opts_default(qaoa_angle_opts *opts);

/* Local minimisation from n_starts points at once (Sec. 2.3: BFGS to the closest local
 * optimum): BFGS in inverse-Hessian form, started from the identity and rescaled after the
 * first step, with a backtracking line search that accepts on sufficient decrease or on the
 * approximate Wolfe conditions (a slope test that still works where single-precision
 * rounding hides the change of <C>); a trial step moves no angle by more than one radian. angles: host double [n_starts][2p], in:
 * starting points, out: the optima found; out_values: host double [n_starts], <C> there;
 * out_iters (NULL allowed): accepted steps taken. Starts are batched max_sets_per_call at a
 * time (automatic: as many as keep 2 x sets x states x 16 bytes under 4 GiB). Stops on
 * gtol, max_iter, or a line search that finds no acceptable step in 20 halvings. */
int qaoa_minimize(const qaoa_problem *prob, const qaoa_mixer *mix, int p, int n_starts, double *angles,
                  double *out_values, int *out_iters, const qaoa_angle_opts *opts, void *stream);

/* Basinhopping (Sec. 2.3 and Sec. 3) from one point x0 (host double [2p]): n_chains chains
 * each minimise from x0, then take n_hops steps of perturb, minimise, Metropolis accept. The
 * chains run independently (each starts its next hop when its minimisation ends) and every
 * optimiser step evaluates the pending points of all chains as one batch. out_angles (host [2p]) and out_value
 * receive the best optimum seen by any chain (ties: earliest step, then lowest chain). */
int qaoa_basinhopping(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *x0,
                      const qaoa_angle_opts *opts, double *out_angles, double *out_value, void *stream);

/* Iterative angle finding (Sec. 2.3 and Sec. 3): round 1 runs basinhopping from uniform
 * random angles in [0, 2 pi); round r > 1 seeds chain 0 with the round r-1 optimum padded by
 * a zero layer (the same state, so the optimum never gets worse with r) and the other chains
 * with its linear interpolation to r layers (endpoints kept). out_angles: host double
 * [p_max][2 p_max], row r-1 holds round r's 2r angles (beta_1..beta_r, gamma_1..gamma_r),
 * the rest zero; out_values: host double [p_max]. checkpoint_path (NULL: none): a text file
 * that receives each round's result as it completes (written to path.tmp, then renamed); if
 * it exists, its rounds are loaded and the search resumes after the last one. A file made
 * for another problem shape or objective sense is refused (QAOA_ERR_INVALID_ARG). Rounds
 * draw their random numbers from (seed, round) only, so a resumed run gives the same results
 * as an uninterrupted one. */
int qaoa_find_angles(const qaoa_problem *prob, const qaoa_mixer *mix, int p_max, const qaoa_angle_opts *opts,
                     const char *checkpoint_path, double *out_angles, double *out_values, void *stream);

/* qaoa_find_angles for n_inst instances at once (the studies of Sec. 2.3 run many instances,
 * e.g. 50 graphs to p = 10): every optimiser step of every instance shares one paired
 * evaluation. Instance i uses probs[i], mixers[i] and checkpoint_paths[i] (checkpoint_paths
 * may be NULL, or hold NULL entries); it gets the same result as a qaoa_find_angles call of
 * its own. Instances may resume from different rounds. out_angles: host double
 * [n_inst][p_max][2 p_max]; out_values: host double [n_inst][p_max]. */
int qaoa_find_angles_multi(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_inst,
                           int p_max, const qaoa_angle_opts *opts, const char *const *checkpoint_paths,
                           double *out_angles, double *out_values, void *stream);

/* Random local-minima search (the listing of Sec. 3): n_restarts starts uniform in
 * [0, 2 pi)^{2p}, all minimised as one batch; out_angles (host [2p]) and out_value receive
 * the best (ties: lowest restart index). out_all_values (NULL allowed): host [n_restarts]. */
int qaoa_find_angles_random(const qaoa_problem *prob, const qaoa_mixer *mix, int p, int n_restarts,
                            const qaoa_angle_opts *opts, double *out_angles, double *out_value,
                            double *out_all_values, void *stream);

/* Kernel timing (a tracing aid). While enabled, every kernel launch an evaluation on this
 * context makes is bracketed by two HIP events recorded on the call's stream; after the
 * call's final synchronisation the elapsed times are added to per-class totals together
 * with the launch's algorithmic bytes (each vector read and written once, plus the cost
 * table when the kernel reads it). Classes: QAOA_KC_FWD_PASS (tile pass over one vector),
 * QAOA_KC_REV_PASS (tile pass over the state and the adjoint vector), QAOA_KC_SMALL
 * (whole-state kernel), QAOA_KC_DENSE (constrained-mixer products), QAOA_KC_OTHER
 * (lookup tables, reductions), QAOA_KC_GROVER and QAOA_KC_COUNT_STATES (Grover mixer; the
 * flops total of the latter counts states).
 * enable: 1 on, 0 off; enabling clears the totals. */
#define QAOA_KC_FWD_PASS 0
#define QAOA_KC_REV_PASS 1
#define QAOA_KC_SMALL 2
#define QAOA_KC_DENSE 3
#define QAOA_KC_OTHER 4
#define QAOA_KC_GROVER 5       /* Grover-mixer rounds on the cost classes */
#define QAOA_KC_COUNT_STATES 6 /* table-free degeneracy counting */
#define QAOA_KC_XMIX 7         /* X-product mixers: Walsh-Hadamard passes and diagonals */
#define QAOA_KC_COUNT 8
int qaoa_profile_enable(qaoa_ctx *ctx, int enable);

/* Totals of class `kernel_class` since the last enable: launches, summed milliseconds,
 * summed algorithmic bytes and summed algorithmic flops. Any output may be NULL. */
int qaoa_profile_read(const qaoa_ctx *ctx, int kernel_class, int64_t *launches, double *ms,
                      double *bytes, double *flops);

/* Measurement aid, not a step of the method: copies `bytes` from device buffer d_src to
 * device buffer d_dst (both caller-owned, on the context's device, 16-byte aligned, not
 * overlapping; bytes a multiple of 16, else INVALID_ARG) with the library's plain streaming
 * kernel (each byte read once and written once: one 16-byte non-temporal load and store per
 * thread). Its rate is the HBM roof a streaming kernel reaches on the device, and the
 * calibration of the traffic counters.
 * Enqueued on `stream`; does not synchronise. */
int qaoa_stream_copy(qaoa_ctx *ctx, const void *d_src, void *d_dst, size_t bytes, void *stream);

/* Static text for a status code. */
const char *qaoa_status_string(int status);

/* Thread-local detail of the last error on the calling thread ("" if none). */
const char *qaoa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QAOA_H */
