/*
 * tsat.h -- C-ABI of the MI355X (gfx950) gradient-guided SAT hot path.
 *
 * Method: TurboSAT (Dai, Yu, Krishnamani, Khailany; arXiv 2511.07737).
 * A CNF with V variables and C clauses is the binary Problem Matrix
 * P in {0,1}^{C x 2V}; N candidate assignments are the columns of the
 * Assignment Matrix A in {0,1}^{2V x N} (complete assignments: the negated
 * literal is the complement); R = P A counts the true literals of every
 * (clause, candidate) pair (Sec. III-A, Eq. 1).  Candidates are held as
 * real logits theta in R^{V x N}; each iteration binarizes them after the
 * per-variable normalization (Eq. 5, Eq. 2), evaluates R, the SmoothMin loss
 * (Eq. 3, Eq. 4), back-propagates with the straight-through estimator and
 * takes an AdamW step with the step-decay/restart schedule (Sec. IV-A).
 *
 * Conventions for every entry point:
 *  - Return value: TSAT_OK (0) or a negative TSAT_E_* code.  No call aborts
 *    the process.  On error, outputs are left untouched and
 *    tsat_last_error() describes the failure (thread-local string, valid
 *    until the next call on the same thread).
 *  - Host pointers are owned by the caller and only read/written during the
 *    call.  Device pointers (the *_dev calls) are owned by the caller (e.g.
 *    torch tensors) and must stay valid until the work on the given stream
 *    completes.  The solver owns all of its internal device memory.
 *  - Arrays named [A][B] are row-major with B contiguous.  Candidate c of a
 *    bit-packed row is bit (c % 64) of 64-bit word (c / 64); rows have
 *    W = ceil(N / 64) words and pad bits are ignored on input, 0 on output.
 *  - A solver is not internally synchronized: one host thread at a time.
 */
#ifndef TSAT_H
#define TSAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSAT_OK 0
#define TSAT_E_ARG (-1)     /* invalid argument, size or range */
#define TSAT_E_PARSE (-2)   /* malformed DIMACS input */
#define TSAT_E_OOM (-3)     /* host or device allocation failed */
#define TSAT_E_HIP (-4)     /* HIP runtime error (no device, launch failure) */
#define TSAT_E_STATE (-5)   /* call out of order (e.g. step before init) */
#define TSAT_E_NUMERIC (-6) /* a logit or optimizer moment became NaN/Inf */

#define TSAT_MODE_NONE 0 /* b = B(theta) */
#define TSAT_MODE_MEAN 1 /* b = B(theta / mean_row(theta)), Eq. 5 then Eq. 2 */

#define TSAT_MAX_WIDTH 32 /* widest clause (after de-duplication) */
#define TSAT_MAX_STEP_N 1024 /* candidates per batch for the gradient step */
#define TSAT_NOALLOC_SCRATCH_BYTES (4u << 20) /* fixed device scratch of tsat_fwd_dev_noalloc, per GPU */

typedef struct tsat_solver tsat_solver;

/* Hyper-parameters.  Defaults (tsat_default_params): the paper's AdamW
 * schedule (Sec. IV-A: lr 1e-1, x0.1 every 30 iterations, reset every 360,
 * floor 1e-15), PyTorch's AdamW defaults for the constants the paper leaves
 * open, SmoothMin tau = 1, Eq. 5 normalization on, convergence at 99% of the
 * clauses (Sec. IV-B). */
typedef struct {
    double tau;           /* SmoothMin temperature, Eq. 4 (>= 0) */
    double lr0;           /* initial / restart learning rate */
    double lr_decay;      /* factor applied every decay_every iterations */
    double lr_min;        /* floor of the learning rate */
    double beta1, beta2;  /* AdamW moment decays */
    double eps;           /* AdamW epsilon */
    double weight_decay;  /* AdamW decoupled weight decay */
    double converge_frac; /* convergence: best candidate satisfies > frac * C */
    int32_t decay_every;  /* iterations per decay (> 0) */
    int32_t restart_every;/* iterations per learning-rate restart (> 0) */
    int32_t norm_mode;    /* TSAT_MODE_MEAN or TSAT_MODE_NONE */
    int32_t k_partial;    /* partial-assignment size; <= 0: max(20, ceil(V/1e4)) */
    int32_t mix;          /* 1: assignment mixing at every learning-rate restart (iterations t > 0 with
                             t mod restart_every = 0; the paragraph of Sec. IV-A the published text
                             leaves out, with its equation): after the iteration's forward pass each
                             candidate i other than the best one i* (most satisfied clauses, lower
                             index on ties) becomes (theta_i + theta_i*) / 2 per variable, and the
                             optimizer is reset (m = v = 0, bias corrections counted from the next
                             iteration); the iteration takes no gradient step.  0 (default): off */
    int32_t reserved;
} tsat_params;

typedef struct {
    int32_t device;     /* HIP device ordinal */
    int32_t reserved;
    void* stream;       /* hipStream_t to run on; NULL: the solver creates one */
    tsat_params params; /* defaults for tsat_step(params = NULL) */
} tsat_config;

typedef struct {
    int64_t steps_done;           /* AdamW updates performed by this call */
    int64_t first_sat_step;       /* first iteration whose binarized batch held a
                                     satisfying candidate; -1 if none (since init) */
    int64_t first_converged_step; /* first iteration with best > converge_frac*C; -1 */
    int64_t best_sat_count;       /* satisfied clauses of the best candidate, last forward */
    int64_t next_step;            /* 0-based index of the next iteration */
    double loss;                  /* Eq. 3 at the last forward pass */
    int32_t best_candidate;       /* most satisfied clauses, lowest index on ties */
    int32_t sat_candidate;        /* first satisfying candidate, -1 if none */
    int32_t nonfinite;            /* 1 if a value became NaN/Inf */
    int32_t reserved;
} tsat_report;

/* Per-instance results of a batch (tsat_get_instance_status). */
typedef struct {
    int64_t first_sat_step;       /* first iteration with a satisfying candidate, -1 if none */
    int64_t first_converged_step; /* first iteration with best > converge_frac*C, -1 if none */
    int64_t best_sat_count;       /* satisfied clauses of the best candidate, last forward */
    int64_t num_clauses;
    double loss;                  /* Eq. 3 of this instance at the last forward pass */
    uint64_t start_ticks;         /* device real-time counter at the first forward pass */
    uint64_t sat_ticks;           /* device real-time counter when first satisfied (0 if never) */
    uint64_t conv_ticks;          /* device real-time counter when first converged (0 if never) */
    int32_t best_candidate;
    int32_t sat_candidate;        /* -1 if none */
    int32_t frozen;               /* 1: frozen by the stop mode of tsat_step */
    int32_t num_vars;
} tsat_instance_status;

typedef struct {
    int32_t num_vars;
    int32_t max_width;        /* widest clause after de-duplication */
    int64_t num_clauses;      /* including empty clauses */
    int64_t num_lits;         /* literal occurrences after de-duplication */
    int64_t num_empty;        /* empty clauses (no candidate can satisfy the CNF) */
    int64_t num_dup_removed;  /* repeated literals removed */
    int64_t num_tautologies;  /* clauses holding both v and -v (kept) */
    int64_t width_count[TSAT_MAX_WIDTH + 1]; /* clauses per width 0..32 */
} tsat_cnf_info;

/* ---------------------------------------------------------------- misc --- */

/* Description of the last error on this thread ("" if none). */
const char* tsat_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t tsat_version(void);

/* Fill *p with the defaults listed above.  E_ARG if p is NULL. */
int32_t tsat_default_params(tsat_params* p);

/* ------------------------------------------------ host-only CNF helpers --- */

/* Validate a DIMACS literal stream and describe the clause store it yields
 * (Sec. III-A: one P row per clause, one column per literal).  lits holds
 * num_lits signed 1-based literals, each clause terminated by 0.  Repeated
 * literals inside a clause are removed; tautologies and empty clauses are
 * kept.  No GPU is used.  E_ARG: |lit| > num_vars, num_vars < 1, a clause
 * wider than TSAT_MAX_WIDTH after de-duplication, or an unterminated final
 * clause.  OOM on allocation failure. */
int32_t tsat_cnf_info_of(int32_t num_vars, int64_t num_lits, const int32_t* lits, tsat_cnf_info* out);

/* Parse a DIMACS CNF file ("c" comment lines, one "p cnf V C" header, then
 * clauses as 0-terminated integers).  Two-call pattern: with lits == NULL,
 * *num_lits receives the stream length (literals plus terminators) and
 * *num_vars the declared V; with lits != NULL and cap >= that length the
 * stream is written.  E_PARSE: missing/duplicate header, non-integer token,
 * literal out of range, clause count differing from the header.
 * E_ARG: NULL outputs or cap too small. */
int32_t tsat_dimacs_read(const char* path, int32_t* num_vars, int64_t* num_lits, int32_t* lits, int64_t cap);

/* ------------------------------------------------------------- lifecycle --- */

/* Create a solver on cfg->device (cfg NULL: device 0, own stream, default
 * params).  E_HIP if the device is absent or the runtime fails. */
int32_t tsat_create(const tsat_config* cfg, tsat_solver** out);

/* Release the solver and all its device memory.  NULL-safe. */
void tsat_destroy(tsat_solver* s);

/* Load a CNF (Sec. III-A; the sparse clause store of Sec. IV-A).  lits as in
 * tsat_cnf_info_of; the input is copied.  Builds the width-bucketed clause
 * store (forward pass) and the per-variable occurrence store (backward
 * pass) on the device.  Replaces any previous CNF and batch.  E_ARG as in
 * tsat_cnf_info_of; OOM; HIP. */
int32_t tsat_load_cnf(tsat_solver* s, int32_t num_vars, int64_t num_lits, const int32_t* lits);

/* tsat_dimacs_read + tsat_load_cnf. */
int32_t tsat_load_dimacs(tsat_solver* s, const char* path);

/* Load a batch of independent instances of uneven size, solved together
 * (one launch per kernel covers all of them).  Instance j is the DIMACS
 * stream lits[lit_offsets[j] .. lit_offsets[j+1]) over variables
 * 1..num_vars[j]; lit_offsets has n_inst + 1 entries, lit_offsets[0] = 0.
 * Every instance gets the same number of candidates N (tsat_init_batch);
 * theta of the batch is [sum_j V_j][N] with instance j's rows starting at
 * sum_{i<j} V_i.  Histograms, SmoothMin, the loss, SAT detection and (with
 * stop_on_sat) freezing are per instance; the learning-rate schedule is
 * shared.  E_ARG as in tsat_load_cnf, per instance. */
int32_t tsat_load_cnf_batch(tsat_solver* s, int32_t n_inst, const int32_t* num_vars, const int64_t* lit_offsets,
                            const int32_t* lits);

/* Instances loaded (1 after tsat_load_cnf), 0 before any load. */
int32_t tsat_num_instances(const tsat_solver* s);

/* Variables of the loaded CNF (sum over the instances of a batch). */
int32_t tsat_num_vars(const tsat_solver* s);

/* Start a batch of N candidates (Sec. IV-A).  init_logits: host [V][N]
 * float logits, or NULL for theta ~ N(0,1) drawn on the device from `seed`
 * (Philox4x32-10 + Box-Muller).  AdamW moments and the iteration index are
 * reset to 0, the binarized batch is computed.  E_STATE before a CNF is
 * loaded; E_ARG for N < 1 or N > TSAT_MAX_STEP_N (the check-only call
 * tsat_check_bits has no such limit). */
int32_t tsat_init_batch(tsat_solver* s, int32_t N, uint64_t seed, const float* init_logits);

/* --------------------------------------------------------------- solving --- */

/* Run up to max_steps iterations (Sec. III-B, IV-A), each: forward R = P A
 * on the current bits -> SmoothMin/loss -> straight-through adjoint ->
 * Eq. 5 backward -> AdamW with lr(t) -> re-binarize.  Iteration t whose
 * forward finds a satisfying candidate is recorded in first_sat_step, the
 * first whose best candidate satisfies more than converge_frac*C clauses in
 * first_converged_step.  stop_on_sat: 0 runs all max_steps; 1 freezes an
 * instance without updating at its first satisfying candidate (its bits
 * hold the witness); 2 freezes it at the first of that and convergence (the
 * hand-off to CDCL of Sec. IV-B; its bits are the converged candidates);
 * with 1 or 2 the run stops once every instance is frozen.
 * params NULL: the solver's defaults.  Blocks until the work is done and
 * fills *report (may be NULL); for a batch, loss and best_sat_count are
 * summed over the instances, first_sat_step is the earliest one, the
 * candidate fields are those of instance 0.  E_STATE before
 * tsat_init_batch; E_ARG for max_steps < 0 or invalid params; E_NUMERIC if
 * a value became non-finite (the report is still filled). */
int32_t tsat_step(tsat_solver* s, int32_t max_steps, const tsat_params* params, int32_t stop_on_sat,
                  tsat_report* report);

/* Note on norm_mode: the binarized batch is always that of the
 * normalization mode of the last call that used it; a call whose params
 * carry another mode re-binarizes theta with that mode first. */

/* Replay iterations through a captured HIP graph (two iterations, one per
 * bit-buffer parity, captured on first use and re-captured when the
 * arguments change).  Not combined with tsat_set_timing.  Default off. */
int32_t tsat_set_graph(tsat_solver* s, int32_t enable);

/* Per-instance results for instances [first, first + count). */
int32_t tsat_get_instance_status(tsat_solver* s, int32_t first, int32_t count, tsat_instance_status* out);

/* Frequency in Hz of the device real-time counter behind start_ticks,
 * sat_ticks and conv_ticks. */
int32_t tsat_device_clock_hz(tsat_solver* s, double* hz);

/* Exact check of the current binarized batch (Sec. III-A, Satisfiability
 * Matrix): sat_counts[n_inst][N] = clauses with >= 1 true literal,
 * is_sat[n_inst][N] = 1 iff every clause of that instance has one.  Either
 * output may be NULL.  E_STATE before init. */
int32_t tsat_check(tsat_solver* s, int64_t* sat_counts, uint8_t* is_sat);

/* Stateless exact check of caller bits: packed is host [V][ceil(N/64)]
 * uint64 (bit c%64 of word c/64 = value of the variable in candidate c).
 * Any N >= 1 that fits in device memory.  Does not touch the batch.
 * Outputs [n_inst][N].  E_STATE before a CNF is loaded; E_ARG for N < 1 or
 * NULL packed. */
int32_t tsat_check_bits(tsat_solver* s, const uint64_t* packed, int32_t N, int64_t* sat_counts,
                        uint8_t* is_sat);

/* Current binarized values of candidate `cand`: vals[V] in {0,1}.
 * E_ARG if cand is outside [0, N). */
int32_t tsat_get_assignment(tsat_solver* s, int32_t cand, uint8_t* vals);

/* First satisfying assignment found since init (vals[V]) and its candidate
 * index in *cand.  E_STATE if none has been found or more than one instance
 * is loaded. */
int32_t tsat_get_witness(tsat_solver* s, uint8_t* vals, int32_t* cand);

/* Same for instance inst of a batch: vals[V_inst] over its own variables. */
int32_t tsat_get_witness_instance(tsat_solver* s, int32_t inst, uint8_t* vals, int32_t* cand);

/* Handoff buffer for CPU CDCL refinement (Sec. IV-B).  Candidates are taken
 * in order of satisfied clauses (descending; ties: lower index); for each of
 * the first max_cands, the k variables with the smallest |dL/dtheta| at the
 * current state (ties: lower variable index; variables that occur in no
 * clause are skipped) are written as signed DIMACS literals of the
 * candidate's current values, most confident first.  k <= 0 uses
 * params.k_partial, whose default is max(20, ceil(V/1e4)).  Slots beyond
 * the number of eligible variables hold 0.  Outputs: cand_ids[max_cands],
 * lits[max_cands][k], sat_counts[max_cands] (may be NULL).  E_ARG for
 * max_cands outside [1, N] or k > 4096; E_STATE before init or with more
 * than one instance loaded. */
int32_t tsat_extract_partial(tsat_solver* s, int32_t max_cands, int32_t k, int32_t* cand_ids, int32_t* lits,
                             int64_t* sat_counts);

/* ------------------------------------------------------- state and hooks --- */

/* Number of candidates of the current batch (0 before init). */
int32_t tsat_num_candidates(const tsat_solver* s);

/* Widest clause of the loaded CNF (histogram bins are max_width + 1). */
int32_t tsat_max_width(const tsat_solver* s);

/* Replace theta (host [V][N]) keeping m, v and the iteration index; the bits
 * are recomputed.  E_STATE before init. */
int32_t tsat_set_logits(tsat_solver* s, const float* theta);

/* Copy theta to host [V][N]. */
int32_t tsat_get_logits(tsat_solver* s, float* theta);

/* Replace the whole optimizer state: theta, m, v (host [V][N]) and the
 * 0-based iteration index t; bits are recomputed, the SAT bookkeeping reset.
 * m or v NULL: zeros. */
int32_t tsat_set_state(tsat_solver* s, const float* theta, const float* m, const float* v, int64_t t);

/* Copy the optimizer state out; any pointer may be NULL. */
int32_t tsat_get_state(tsat_solver* s, float* theta, float* m, float* v, int64_t* t);

/* Iteration at which the AdamW moments last started from zero: 0 after
 * tsat_init_batch / tsat_set_state, t + 1 after a mixing iteration t
 * (params.mix).  The update of iteration t uses the bias-correction count
 * t - origin + 1.  Get and set it to checkpoint and resume a run with
 * mixing (set it after tsat_set_state; E_ARG if origin > the next
 * iteration index or < 0). */
int32_t tsat_get_adam_origin(tsat_solver* s, int64_t* origin);
int32_t tsat_set_adam_origin(tsat_solver* s, int64_t origin);

/* Current binarized batch, host [V][ceil(N/64)] uint64. */
int32_t tsat_get_bits(tsat_solver* s, uint64_t* packed);

/* Forward-only evaluation of the current bits (no update, no SAT
 * bookkeeping): hist[n_inst][N][max_width+1] uint32 = #{c : R_ci = r}
 * (Eq. 1), S[n_inst][N] (Eq. 4, FP64), *loss (Eq. 3, summed over the
 * instances).  Any output may be NULL. */
int32_t tsat_eval(tsat_solver* s, const tsat_params* params, uint32_t* hist, double* S, double* loss);

/* Gradients at the current state without updating: U[V][N] = dL/d(theta_norm)
 * through the straight-through estimator (Sec. III-B), g[V][N] = dL/dtheta
 * after the Eq. 5 backward.  Either output may be NULL. */
int32_t tsat_get_grad(tsat_solver* s, const tsat_params* params, float* U, float* g);

/* -------------------------------------------------- device-pointer API --- */
/* For framework integration (e.g. a torch.autograd.Function).  All pointers
 * are device memory owned by the caller; work is enqueued on `stream`
 * (hipStream_t; NULL = the null/default stream, which is what torch reports
 * for its default stream) and the call returns without waiting.  The solver keeps scratch space sized for the largest N seen;
 * calls on one solver must not overlap in time on different streams.
 * Forward and backward need a single-instance solver (E_STATE otherwise). */

/* Pack a float assignment (device [V][N], value > 0.5 means True) into bits
 * (device [V][ceil(N/64)] uint64). */
int32_t tsat_pack_dev(tsat_solver* s, const float* assign, int32_t N, uint64_t* bits, void* stream);

/* Forward of the differentiable layer: R = P A for the candidates in bits
 * (device [V][ceil(N/64)]), then SmoothMin per candidate (Eq. 4).  Outputs:
 * S[N] float (may be NULL), hist[N][max_width+1] uint32 (may be NULL). */
int32_t tsat_fwd_dev(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, float* S, uint32_t* hist,
                     void* stream);

/* Backward of the layer: given dS[N] = dLoss/dS_i, writes U[V][N] =
 * dLoss/dA for the positive literal rows with the straight-through
 * estimator (Sec. III-B), i.e. sum over clauses of P^T dLoss/dR with +1
 * for x_v and -1 for not-x_v.  N <= TSAT_MAX_STEP_N. */
int32_t tsat_bwd_dev(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, const float* dS, float* U,
                     void* stream);

/* The same backward by the clause-major design the library does not use for
 * its step: one thread per (clause, 32 candidates) computes R and adds the
 * dL/dR table entry into every literal's row of U with FP32 atomics (the
 * first literal of each clause into an LDS tile of the block, flushed with
 * atomics at the end).  U is zeroed first.  Kept as the measured comparison
 * point of the variable-major gather; the order of the atomic additions is
 * not fixed, so results may differ from run to run in the last bits (each
 * U entry within (degree + 1) * 2^-24 of the sum of its terms' magnitudes).
 * Single-instance solvers, N <= 256; E_ARG / E_STATE as tsat_bwd_dev. */
int32_t tsat_bwd_scatter_dev(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, const float* dS, float* U,
                             void* stream);

/* The differentiable path of Fig. 3 on caller logits theta (device [V][N]
 * float, the real-valued assignment matrix; N <= TSAT_MAX_STEP_N), for a
 * single-instance solver; mode is TSAT_MODE_MEAN (Eq. 5 normalization
 * before Eq. 2) or TSAT_MODE_NONE.  Same stream and scratch rules as above.
 * E_ARG for NULL required pointers, N or mode out of range, tau < 0;
 * E_STATE before a CNF is loaded or with more than one instance. */

/* Eq. 5 then Eq. 2 (Sec. IV-A, Sec. III-B): mu_v = (1/N) sum_i theta_vi
 * (FP64; |mu| < 1e-12 is clamped to +-1e-12, 0 to +1e-12) and
 * b_vi = B(theta_vi / mu_v) = [theta_vi mu_v > 0] (mean mode) or
 * [theta_vi > 0] (none).  Outputs, any may be NULL but not all: bits device
 * [V][ceil(N/64)] uint64 (the literal x_v; not x_v is the complement),
 * assign device [V][N] float (b as 0.0 / 1.0), mu device [V] double (the
 * unclamped means; 1.0 in none mode). */
int32_t tsat_binarize_dev(tsat_solver* s, const float* theta, int32_t N, int32_t mode, uint64_t* bits, float* assign,
                          double* mu, void* stream);

/* Backward of Eq. 5 (the straight-through estimator passes the gradient
 * through Eq. 2 unchanged, Sec. III-B): given dA = dLoss/d(theta/mu)
 * (device [V][N]), writes g = dLoss/dtheta (device [V][N]):
 * g_vi = dA_vi / mu_v - (sum_k dA_vk theta_vk) / (N mu_v^2) in mean mode
 * (the second term is dropped where the mean is clamped), g = dA in none
 * mode.  The row means are recomputed from theta as tsat_binarize_dev forms
 * them. */
int32_t tsat_norm_backward_dev(tsat_solver* s, const float* theta, const float* dA, int32_t N, int32_t mode, float* g,
                               void* stream);

/* Loss of the logits: Eq. 5 -> Eq. 2 -> R = P A (Eq. 1) -> SmoothMin with
 * temperature tau (Eq. 4) -> loss = -sum_i S_i (Eq. 3).  Outputs: loss
 * (device float scalar, required; the sum is formed in FP64), S device [N]
 * float and bits device [V][ceil(N/64)] (both may be NULL). */
int32_t tsat_loss_dev(tsat_solver* s, const float* theta, int32_t N, float tau, int32_t mode, float* loss, float* S,
                      uint64_t* bits, void* stream);

/* Gradient of that loss times the upstream scalar dloss (device float,
 * NULL = 1): g = dloss * dLoss/dtheta (device [V][N], required), through
 * the transpose product with the straight-through estimator and the Eq. 5
 * backward in one pass over the variables; U (device [V][N], may be NULL)
 * receives dloss * dLoss/d(theta/mu). */
int32_t tsat_loss_backward_dev(tsat_solver* s, const float* theta, int32_t N, float tau, int32_t mode,
                               const float* dloss, float* g, float* U, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward of tsat_fwd_dev with the same arguments, outputs and results
 * (bitwise), but it allocates nothing.  The literal rows are read straight
 * from `bits` (a negated literal is the complement of its variable's row),
 * and the histogram accumulator and the forward work units live in one
 * fixed device array of TSAT_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends and shared by every call on that GPU: calls that overlap in
 * time on one GPU (any solver, any stream) race and must be ordered by the
 * caller.  Each call clears what it needs.  1 <= N <= TSAT_MAX_STEP_N;
 * E_ARG when the accumulator ((64 ceil(N/64)) x (max width + 1) x 4 bytes)
 * plus the work units (24 bytes per unit, about C / 8000 units per width
 * bucket at N = 256) exceed the array; E_STATE as tsat_fwd_dev. */
int32_t tsat_fwd_dev_noalloc(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, float* S, uint32_t* hist,
                             void* stream);

/* --------------------------------------------------- learned proposal --- */
/*
 * A per-variable network proposes P(x_v = true) for every variable of the
 * loaded CNF; the batch then starts from draws of that proposal instead of
 * the N(0,1) logits of Sec. IV-A.  The network, its features and the
 * proposal start are this library's extension, not part of the paper.
 *
 * Features (16 per variable, FP32), over the non-tautological clauses:
 *   [0] log(1+pos_v)  [1] log(1+neg_v)  [2] (pos_v-neg_v)/max(1,deg_v)
 *   [3] mean width of the clauses of v / 4 (0 if deg_v = 0)
 *   [4+4(r-1) .. 7+4(r-1)] = h_r[v], r = 1..3, where
 *   h_0[v] = ((pos-neg)/max(1,deg), (pos-neg)/sqrt(max(1,deg)),
 *             log(1+pos)-log(1+neg), 1) and h_r[v] = (1/max(1,Z_v)) * sum
 *   over clauses c of v and co-literals l' of c on another variable u of
 *   sgn(l_v) sgn(l') h_{r-1}[u]; Z_v counts those (c, l') pairs.
 * Network: a1 = bf16(X) bf16(W1) + b1, h1 = bf16(relu(a1)),
 *   a2 = h1 bf16(W2) + b2, logit = relu(a2) bf16(w3) + b3; bf16() rounds to
 *   nearest-even; products accumulate in FP32.  Parameters are one FP32
 *   vector of TSAT_MLP_NUM_PARAMS values: W1 [16][128], b1 [128],
 *   W2 [128][128], b2 [128], w3 [128], b3 [1] (W[in][out]).
 */
#define TSAT_MLP_FEATURES 16
#define TSAT_MLP_HIDDEN 128
#define TSAT_MLP_NUM_PARAMS 18817

typedef struct tsat_mlp tsat_mlp;

/* Features of the loaded CNF (all instances of a batch) into host X[V][16]. */
int32_t tsat_get_features(tsat_solver* s, float* X);

/* Same, into caller-owned device memory X[V][16] on `stream` (NULL: the
 * null stream).  The call returns after enqueueing. */
int32_t tsat_features_dev(tsat_solver* s, float* X, void* stream);

/* Network handle on `device` with the given host parameters (required).
 * Adam state starts at zero, step count 0.  E_HIP without a device. */
int32_t tsat_mlp_create(int32_t device, const float* params, tsat_mlp** out);

/* NULL-safe. */
void tsat_mlp_destroy(tsat_mlp* m);

/* Replace the parameters (host [TSAT_MLP_NUM_PARAMS]); resets Adam state
 * and the step count. */
int32_t tsat_mlp_set_params(tsat_mlp* m, const float* params);

/* Copy the parameters to host memory. */
int32_t tsat_mlp_get_params(tsat_mlp* m, float* params);

/* Host copies of the gradient and loss of the last train step (either
 * pointer may be NULL).  E_STATE before the first train step. */
int32_t tsat_mlp_get_grad(tsat_mlp* m, float* grad, float* loss);

/* Adam steps taken since creation or the last set_params. */
int64_t tsat_mlp_step_count(const tsat_mlp* m);

/* Forward of B rows of device X[B][16] (16-byte aligned): logits[B] and/or
 * probs[B] = sigmoid(logit) (device, either may be NULL, not both), on
 * `stream` (NULL: the null stream).  Returns after enqueueing. */
int32_t tsat_mlp_forward_dev(tsat_mlp* m, const float* X, int64_t B, float* logits, float* probs, void* stream);

/* One training step on B >= 1 device rows X[B][16], labels y[B] in {0,1}
 * and optional weights w[B] (NULL: 1): the gradient of the weighted mean
 * binary cross-entropy with logits, taken with the rounded tensors held
 * fixed (the gradient of a master weight is that of its rounded copy; the
 * relu of layer 1 passes where h1 > 0), summed in a fixed order; then, if
 * lr > 0, one Adam step (beta 0.9/0.999, eps 1e-8, bias-corrected, 1-based
 * step count).  lr <= 0 computes the gradient only.  Calls on one handle
 * share its scratch: issue them in order on one stream.  Returns after
 * enqueueing; tsat_mlp_get_grad synchronizes. */
int32_t tsat_mlp_train_step_dev(tsat_mlp* m, const float* X, const float* y, const float* w, int64_t B, float lr,
                                void* stream);

/* Run the features and the network over the loaded CNF and keep
 * p_v = sigmoid(logit_v) in the solver (optionally copied to host p[V]).
 * The network must live on the solver's device. */
int32_t tsat_propose(tsat_solver* s, tsat_mlp* m, float* p);

/* Start a batch of N candidates from a proposal: p_true host [V] in [0,1]
 * (values outside are clamped, NaN counts as 0), or NULL for the one kept by
 * tsat_propose.  Candidate i of variable v draws b_vi = 1 with probability
 * p_v and theta_vi = +|z_vi| if b_vi = 1, -|z_vi| otherwise, with z_vi the
 * same N(0,1) draw tsat_init_batch(seed) makes (Philox4x32-10, counter
 * (e mod 2^32, e div 2^32, 0x5A17, 0) for e = v N + i, key = seed; the
 * Bernoulli draw compares the third output word with floor(p_v 2^32)).
 * In mean mode (the solver's norm_mode) the negative entries of a row are
 * scaled by min(1, 0.5 sum_{b=1}|z| / sum_{b=0}|z|) so that Eq. 5 followed
 * by Eq. 2 reproduces b, and a row without b = 1 gets it at i = v mod N.
 * Optimizer state and step count start at zero as in tsat_init_batch. */
int32_t tsat_init_from_proposal(tsat_solver* s, int32_t N, uint64_t seed, const float* p_true);

/* ------------------------------------------------------- launch shapes --- */

/* Launch shapes of the step kernels.  They change how work is split over
 * the GPU, never the arithmetic: results are identical under every shape. */
typedef struct {
    int32_t fwd_target_blocks; /* forward histogram: work units per launch to aim for (clause tile size
                                  follows from it); default 1024 */
    int32_t var_blocks_per_cu; /* fused update: persistent blocks per CU, 0 = 4 x occupancy */
    int32_t pure_group;        /* uniform-width stores: occurrence records per load group, 1, 2 or 4 */
    int32_t clause_planes;     /* uniform widths 2, 3 and N <= 256: 1 = the forward stores R of every
                                  clause in binary and the update gathers it (one record per
                                  occurrence), 0 = the update gathers the other literals' rows */
    int32_t window_gather;     /* with clause planes: 1 = the update loads the planes of 64 consecutive
                                  occurrence records per vector load and transposes their bits across
                                  the wavefront (up to 32 candidates: two variables per wavefront),
                                  0 = record by record through the scalar cache; default 1.  A store
                                  with a variable in 2^16 or more clauses of one sign always takes
                                  the record-by-record gather */
    double fwd_ms;             /* tsat_autotune output: forward time per iteration of the choice */
    double var_ms;             /* tsat_autotune output: fused update time per iteration of the choice */
} tsat_launch_config;

/* Current launch shapes (fwd_ms/var_ms zero). */
int32_t tsat_get_launch_config(tsat_solver* s, tsat_launch_config* out);

/* Set launch shapes (fwd_ms/var_ms ignored); drops a captured graph.
 * E_ARG outside the documented ranges.  The environment variables
 * TSAT_FWD_TARGET_BLOCKS, TSAT_VAR_BLOCKS_PER_CU, TSAT_PURE_GROUP,
 * TSAT_CLAUSE_PLANES and TSAT_WINDOW_GATHER set the initial values of a new
 * solver. */
int32_t tsat_set_launch_config(tsat_solver* s, const tsat_launch_config* cfg);

/* Autotuner: times candidate shapes on real iterations of the current batch
 * (`iters` in [1, 64] iterations per candidate, per-kernel HIP-event timing):
 * first the forward work-unit target (256, 512, ..., 32768), then the fused
 * update's blocks per CU (auto, 8, 16, ..., 1024) with, for uniform-width stores, the
 * clause-plane gather on (by windows and record by record) and off and,
 * without it, the record group (1, 2, 4), compared on forward + update
 * time; keeps the fastest and returns it in *best
 * (may be NULL) with the measured times.  The iterations advance the batch
 * (p as in tsat_step, no early stop); *iters_used (may be NULL) receives
 * their number.  Callers that want a fresh start re-initialize the batch. */
int32_t tsat_autotune(tsat_solver* s, int32_t iters, const tsat_params* p, tsat_launch_config* best,
                      int32_t* iters_used);

/* ------------------------------------------------------------ profiling --- */

/* Enable (1) or disable (0) per-kernel HIP-event timing inside tsat_step.
 * While enabled, events are recorded on the solver's stream around each
 * kernel of each iteration. */
int32_t tsat_set_timing(tsat_solver* s, int32_t enable);

/* Average device time in milliseconds per launch of each kernel over the
 * timed iterations of the last tsat_step: ms[0] forward histogram (all width
 * buckets), ms[1] SmoothMin/table, ms[2] fused adjoint/update/pack;
 * *iters = iterations averaged.  E_STATE if nothing was timed. */
int32_t tsat_get_timing(tsat_solver* s, double* ms, int32_t* iters);

/* Reference point for hardware byte counters: allocates two device buffers
 * of `bytes` bytes (a multiple of 16, at least 16) on the solver's device,
 * runs one plain coalesced copy kernel over them (bytes read + bytes
 * written), frees them and returns its device time in *ms (may be NULL).
 * E_OOM if the buffers cannot be allocated. */
int32_t tsat_copy_calibrate(tsat_solver* s, int64_t bytes, double* ms);

/* Independent literal rows (Sec. III-B writes the real-valued assignment
 * as 2V x N, one row per literal; the incomplete-assignment passage of
 * Sec. III-A): with enable = 1 the next tsat_init_batch holds 2V logit
 * rows, row 2v for x_v and row 2v + 1 for not-x_v, each normalized (Eq. 5)
 * and binarized (Eq. 2) on its own, so a candidate may set both literals of
 * a variable (either satisfies its clauses: a "don't care") or neither.
 * R counts a clause's literals whose own row is 1; the adjoint of a
 * literal row is the sum of dL/dR over the clauses holding that literal
 * (+1 through the straight-through estimator), followed by the Eq. 5
 * backward and AdamW of that row.  Every host array of the batch is then
 * [2V][N] (init_logits, logits, state, U and g) and tsat_get_bits returns
 * all 2V literal rows ([2V][ceil(N/64)]).  Single-instance solvers with
 * clauses at most 15 wide, N <= 256, and the clause planes and window gather
 * on (E_ARG otherwise, at this call or at tsat_init_batch); the proposal
 * start, the hand-off buffer, tsat_get_assignment and witnesses need
 * complete assignments (E_STATE).  Calling it drops the current batch;
 * enable = 0 returns to one row per variable.  E_STATE before a CNF is
 * loaded. */
int32_t tsat_set_literal_rows(tsat_solver* s, int32_t enable);

/* Bandwidth references for the roofline: allocates arrays of `bytes` each
 * (a positive multiple of 16384), runs one untimed and then `reps` (1..1000)
 * timed launches of a streaming kernel over them and returns the average
 * device time per launch in *ms (may be NULL).  kind 0: copy of one array
 * into another (bytes read + bytes written), 16-byte non-temporal accesses,
 * four loads in flight per thread; kind 1: three arrays read and written in
 * place (3 bytes read + 3 bytes written), same accesses; kind 2: as kind 1
 * with the update kernels' pattern (rows of 256 floats, one 4-byte load per
 * lane and array element).  E_ARG for sizes or kinds out of range, E_OOM if
 * the arrays cannot be allocated; the arrays are freed before returning. */
int32_t tsat_stream_calibrate(tsat_solver* s, int64_t bytes, int32_t kind, int32_t reps, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* TSAT_H */
