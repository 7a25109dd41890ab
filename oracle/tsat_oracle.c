/*
 * tsat_oracle.c -- plain, slow, FP64 reference of the gradient-guided SAT step
 * (TurboSAT, arXiv 2511.07737).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark are the only code allowed to load this
 * library.  The GPU path never calls it and shares no code with it.
 *
 * Every function is written as the definition it follows, with no blocking,
 * fusion or reordering beyond what that definition states.  Section names
 * refer to the paper:
 *   - Sec. III-A "Binary Matrix Encoding": Problem Matrix P (one row per
 *     clause, one column per literal), Assignment Matrix A (complete
 *     assignments only: the negated literal is the complement), Result Matrix
 *     R = PA (Eq. 1) = number of true literals per (clause, candidate), and
 *     the Satisfiability Matrix (column minimum of R; nonzero iff the
 *     candidate satisfies every clause).
 *   - Sec. III-B "Differentiable Solving": binarization B(x) = clip(sign(x),0,1)
 *     (Eq. 2), loss L = -sum_i S_i (Eq. 3), SmoothMin (Eq. 4), straight-through
 *     estimator (identity gradient through B).
 *   - Sec. IV-A "Gradient-based Optimization on GPU": N(0,1) initialization,
 *     AdamW with lr 1e-1, x0.1 every 30 iterations, reset every 360
 *     iterations, per-variable normalization by the row mean (Eq. 5) in front
 *     of B.
 *   - Sec. IV-B "CDCL-based Refinement on CPU": convergence at >99% satisfied
 *     clauses, the k = max(20, 0.01% of V) most confident variables (smallest
 *     final |gradient|), candidates dispatched by satisfied-clause count.
 *
 * Readings where the paper is silent or ambiguous (each also listed in the
 * design notes of the repository):
 *   R1  A_real is held as V x N logits theta; literal x_v takes B(theta_norm),
 *       literal not-x_v takes 1 - B(theta_norm) (complete assignments).
 *   R2  Eq. 5 is applied per variable over the N candidates; the mean mu is
 *       clamped to +-1e-12 when |mu| < 1e-12 (sign kept, mu = 0 -> +1e-12).
 *       In the clamped region the clamp is locally constant, so the backward
 *       pass drops the d(mu)/d(theta) term there.
 *   R3  B(0) = 0 (non-positive maps to 0), so b = [theta/mu > 0], evaluated
 *       as a sign test.
 *   R4  SmoothMin temperature tau is a parameter (default 1).  It is
 *       evaluated with the exponent shifted by the column minimum, which is
 *       the same value as Eq. 4.  A CNF with no clauses gives S_i = 0.
 *   R5  Duplicate literals inside a clause are removed; tautologies are kept.
 *   R6  AdamW follows PyTorch's documented decoupled form (the paper uses
 *       PyTorch 2.2 and states no beta/eps/weight decay; defaults 0.9, 0.999,
 *       1e-8, 1e-2).  The bias-correction step count starts at 1 and is not
 *       reset by the learning-rate restart.
 *   R7  lr(t) = max(lr_min, lr0 * decay^floor((t mod restart)/every)), t the
 *       0-based iteration index.
 *   R8  Partial extraction ranks variables by |g| where g is the gradient of
 *       the loss with respect to theta; variables that occur in no clause are
 *       skipped; ties go to the lower variable index.
 *
 * The learned proposal is not part of the paper; its definitions are this
 * library's own and are written out here as plainly as the paper's:
 *   R9  Per-variable features (orc_features) ignore tautological clauses.
 *   R10 The random streams are Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *       SC'11) with counter (e mod 2^32, e div 2^32, 0x5A17, 0) for element
 *       e = v*N + i and key (seed mod 2^32, seed div 2^32); the N(0,1) draw is
 *       Box-Muller on the first two output words, the Bernoulli draw compares
 *       the third word with floor(p * 2^32).
 *   R12 Assignment mixing (the paragraph of Sec. IV-A that the source leaves
 *       commented out, with its equation): it happens at the learning-rate
 *       restarts, i.e. iterations t > 0 with t mod 360 = 0, after that
 *       iteration's forward pass; the best candidate i* has the most
 *       satisfied clauses (lower index on ties); every other candidate's
 *       real-valued row entries become the average of its own and i*'s;
 *       "resetting the optimizer" is read as a fresh AdamW: m = v = 0 and
 *       the bias-correction count restarts at 1 with the next update.  The
 *       mixing iteration takes no gradient step of its own.  Off unless
 *       params.mix is set (the published method does not mix).
 *   R13 Independent literal rows (A_real in R^{2V x N}, Sec. III-B, with the
 *       incomplete-assignment passage of Sec. III-A that the source leaves
 *       commented out): each literal has its own row of logits, Eq. 5 and
 *       Eq. 2 apply per literal row, R counts the literals whose own row is
 *       1 (a variable with both rows 1 is a "don't care" that satisfies
 *       every clause holding either literal; both rows 0 satisfy nothing),
 *       and the straight-through gradient of a literal row is the sum of
 *       dL/dR over the clauses holding that literal.
 *   R11 Initialisation from a proposal p_v (orc_init_proposal): b ~ Bern(p_v),
 *       theta = +|z| where b = 1 and -|z| where b = 0 (z the N(0,1) draw of
 *       the random initialisation).  In mean mode a row's negative entries are
 *       scaled by min(1, 0.5 * (sum of its positive magnitudes) / (sum of its
 *       negative magnitudes)) so that the row mean stays positive and Eq. 5
 *       followed by Eq. 2 returns exactly b; a row with no b = 1 gets b = 1 at
 *       candidate v mod N first (mean mode cannot represent an all-false row).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_OOM (-3)

/* ------------------------------------------------------------------------ */
/* CNF container (oracle-private)                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t V;       /* number of variables */
    int64_t C;       /* number of clauses */
    int64_t L;       /* number of literal occurrences after de-duplication */
    int32_t K;       /* maximum clause width */
    int64_t *off;    /* [C+1] */
    int32_t *lit;    /* [L] signed 1-based literals */
} ocnf;

/* Parse a DIMACS literal stream (each clause terminated by 0) into clauses,
 * removing repeated literals inside a clause (reading R5). */
int orc_cnf_new(int32_t V, int64_t n, const int32_t *stream, void **out)
{
    if (!out || V < 0 || n < 0 || (n > 0 && !stream)) return ORC_E_ARG;
    *out = NULL;
    int64_t C = 0;
    for (int64_t j = 0; j < n; ++j) {
        int32_t x = stream[j];
        if (x == 0) { ++C; continue; }
        int64_t a = x < 0 ? -(int64_t)x : x;
        if (a > V) return ORC_E_ARG;
    }
    if (n > 0 && stream[n - 1] != 0) return ORC_E_ARG; /* unterminated clause */
    ocnf *f = (ocnf *)calloc(1, sizeof(ocnf));
    if (!f) return ORC_E_OOM;
    f->V = V;
    f->C = C;
    f->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C + 1));
    f->lit = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!f->off || !f->lit) { free(f->off); free(f->lit); free(f); return ORC_E_OOM; }
    int64_t c = 0, L = 0, start = 0;
    f->off[0] = 0;
    f->K = 0;
    for (int64_t j = 0; j < n; ++j) {
        int32_t x = stream[j];
        if (x == 0) {
            ++c;
            f->off[c] = L;
            int32_t w = (int32_t)(L - start);
            if (w > f->K) f->K = w;
            start = L;
            continue;
        }
        int dup = 0;
        for (int64_t q = start; q < L; ++q)
            if (f->lit[q] == x) { dup = 1; break; }
        if (!dup) f->lit[L++] = x;
    }
    f->L = L;
    *out = f;
    return ORC_OK;
}

void orc_cnf_free(void *h)
{
    ocnf *f = (ocnf *)h;
    if (!f) return;
    free(f->off);
    free(f->lit);
    free(f);
}

int64_t orc_cnf_num_clauses(const void *h) { return ((const ocnf *)h)->C; }
int64_t orc_cnf_num_lits(const void *h) { return ((const ocnf *)h)->L; }
int32_t orc_cnf_max_width(const void *h) { return ((const ocnf *)h)->K; }
int32_t orc_cnf_num_vars(const void *h) { return ((const ocnf *)h)->V; }

int orc_cnf_get(const void *h, int64_t *off, int32_t *lit)
{
    const ocnf *f = (const ocnf *)h;
    if (!f) return ORC_E_ARG;
    if (off) memcpy(off, f->off, sizeof(int64_t) * (size_t)(f->C + 1));
    if (lit) memcpy(lit, f->lit, sizeof(int32_t) * (size_t)f->L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. 5 + Eq. 2: per-variable normalization, then binarization              */
/* ------------------------------------------------------------------------ */

#define ORC_MU_EPS 1e-12

/* mode 1 ("mean"): b = B(theta / mu_v) with mu_v the mean of row v (reading
 * R2, R3).  mode 0 ("none"): b = B(theta).  mu_out receives the clamped mean
 * (mode 0: 1). */
int orc_binarize(int32_t V, int32_t N, const double *theta, int32_t mode,
                 uint8_t *b, double *mu_out)
{
    if (V < 0 || N <= 0 || !theta || !b) return ORC_E_ARG;
    for (int32_t v = 0; v < V; ++v) {
        const double *row = theta + (int64_t)v * N;
        double mu = 1.0;
        if (mode == 1) {
            double s = 0.0;
            for (int32_t i = 0; i < N; ++i) s += row[i];
            mu = s / (double)N;
            if (fabs(mu) < ORC_MU_EPS) mu = (mu >= 0.0) ? ORC_MU_EPS : -ORC_MU_EPS;
        }
        if (mu_out) mu_out[v] = mu;
        for (int32_t i = 0; i < N; ++i) {
            double a = (mode == 1) ? row[i] / mu : row[i];
            /* B(x) = clip(sign(x), 0, 1): 1 for x > 0, 0 otherwise */
            b[(int64_t)v * N + i] = (a > 0.0) ? 1 : 0;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1: R = P A, and the exact check                                       */
/* ------------------------------------------------------------------------ */

/* Value of literal x (signed, 1-based) for candidate i: A[x_v] = b,
 * A[not x_v] = 1 - b (complete assignments, Sec. III-A). */
static inline int lit_value(const uint8_t *b, int32_t N, int32_t x, int32_t i)
{
    int32_t v = (x > 0 ? x : -x) - 1;
    int bv = b[(int64_t)v * N + i];
    return x > 0 ? bv : 1 - bv;
}

/* R[c][i] = number of true literals of clause c under candidate i. */
int orc_result_matrix(const void *h, int32_t N, const uint8_t *b, int32_t *R)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || N <= 0 || !b || !R) return ORC_E_ARG;
    for (int64_t c = 0; c < f->C; ++c)
        for (int32_t i = 0; i < N; ++i) {
            int32_t r = 0;
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) r += lit_value(b, N, f->lit[q], i);
            R[c * N + i] = r;
        }
    return ORC_OK;
}

/* H[i][r] = #{c : R[c][i] = r}, r = 0..K. */
int orc_histogram(const void *h, int32_t N, const uint8_t *b, int64_t *H)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || N <= 0 || !b || !H) return ORC_E_ARG;
    int32_t K = f->K;
    memset(H, 0, sizeof(int64_t) * (size_t)N * (size_t)(K + 1));
    for (int64_t c = 0; c < f->C; ++c)
        for (int32_t i = 0; i < N; ++i) {
            int32_t r = 0;
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) r += lit_value(b, N, f->lit[q], i);
            H[(int64_t)i * (K + 1) + r] += 1;
        }
    return ORC_OK;
}

/* Satisfiability Matrix (Sec. III-A): candidate i satisfies the CNF iff the
 * column minimum of R is nonzero.  sat_count[i] = number of clauses with at
 * least one true literal. */
int orc_check(const void *h, int32_t N, const uint8_t *b, int64_t *sat_count, uint8_t *is_sat)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || N <= 0 || !b) return ORC_E_ARG;
    for (int32_t i = 0; i < N; ++i) {
        int64_t sat = 0;
        int32_t colmin = INT32_MAX;
        for (int64_t c = 0; c < f->C; ++c) {
            int32_t r = 0;
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) r += lit_value(b, N, f->lit[q], i);
            if (r > 0) ++sat;
            if (r < colmin) colmin = r;
        }
        if (sat_count) sat_count[i] = sat;
        if (is_sat) is_sat[i] = (f->C == 0 || colmin > 0) ? 1 : 0;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. 3 + Eq. 4: SmoothMin and the loss; dL/dR as a table over r            */
/* ------------------------------------------------------------------------ */

/* S_i = sum_c R_ci e^{-tau R_ci} / sum_c e^{-tau R_ci}, evaluated from the
 * histogram H (R takes values 0..K) with the exponent shifted by r0 = min R
 * (reading R4).  The derivative of S_i with respect to one entry R_ci = r is
 * (w_r / D)(1 - tau (r - S_i)) with w_r = e^{-tau (r - r0)}, D = sum H w.
 * table[i][r] = dS[i] * dS_i/dR_ci, i.e. dL/dR_ci for upstream gradient dS
 * (dS == NULL means the loss of Eq. 3, dS_i = -1). */
int orc_smoothmin(int32_t N, int32_t K, const int64_t *H, double tau, const double *dS,
                  double *S, double *table, double *loss)
{
    if (N <= 0 || K < 0 || !H) return ORC_E_ARG;
    double total = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        const int64_t *h = H + (int64_t)i * (K + 1);
        int32_t r0 = -1;
        for (int32_t r = 0; r <= K; ++r)
            if (h[r] > 0) { r0 = r; break; }
        double Si = 0.0, D = 0.0, num = 0.0;
        if (r0 >= 0) {
            for (int32_t r = 0; r <= K; ++r) {
                double w = exp(-tau * (double)(r - r0));
                D += (double)h[r] * w;
                num += (double)r * (double)h[r] * w;
            }
            Si = num / D;
        }
        if (S) S[i] = Si;
        total += Si;
        if (table) {
            double up = dS ? dS[i] : -1.0;
            for (int32_t r = 0; r <= K; ++r) {
                double t = 0.0;
                if (r0 >= 0) {
                    double w = exp(-tau * (double)(r - r0));
                    t = up * (w / D) * (1.0 - tau * ((double)r - Si));
                }
                table[(int64_t)i * (K + 1) + r] = t;
            }
        }
    }
    if (loss) *loss = -total;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Backward: dL/dA = P^T dL/dR, then the straight-through estimator          */
/* ------------------------------------------------------------------------ */

/* U[v][i] = dL/d(theta_norm)_vi.  Every clause c and literal l in c adds
 * dL/dR_ci to dL/dA[l][i] (the transpose product); A[x_v] = B(.) passes it
 * with +1 and A[not x_v] = 1 - B(.) with -1 (straight-through estimator). */
int orc_adjoint(const void *h, int32_t N, const uint8_t *b, int32_t K, const double *table, double *U)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || N <= 0 || !b || !table || !U || K < f->K) return ORC_E_ARG;
    memset(U, 0, sizeof(double) * (size_t)f->V * (size_t)N);
    for (int64_t c = 0; c < f->C; ++c)
        for (int32_t i = 0; i < N; ++i) {
            int32_t r = 0;
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) r += lit_value(b, N, f->lit[q], i);
            double dR = table[(int64_t)i * (K + 1) + r];
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) {
                int32_t x = f->lit[q];
                int32_t v = (x > 0 ? x : -x) - 1;
                U[(int64_t)v * N + i] += (x > 0) ? dR : -dR;
            }
        }
    return ORC_OK;
}

/* Backward of Eq. 5.  theta_norm_vi = theta_vi / mu_v, mu_v = mean_k theta_vk:
 *   d theta_norm_vi / d theta_vk = delta_ik / mu_v - theta_vi / (N mu_v^2)
 * so g_vk = U_vk / mu_v - (sum_i U_vi theta_vi) / (N mu_v^2).
 * In the clamped region (reading R2) only the first term remains.
 * mode 0: g = U. */
int orc_norm_backward(int32_t V, int32_t N, const double *theta, int32_t mode, const double *U, double *g)
{
    if (V < 0 || N <= 0 || !theta || !U || !g) return ORC_E_ARG;
    for (int32_t v = 0; v < V; ++v) {
        const double *th = theta + (int64_t)v * N;
        const double *u = U + (int64_t)v * N;
        double *gv = g + (int64_t)v * N;
        if (mode != 1) {
            for (int32_t i = 0; i < N; ++i) gv[i] = u[i];
            continue;
        }
        double s = 0.0;
        for (int32_t i = 0; i < N; ++i) s += th[i];
        double mu = s / (double)N;
        int clamped = fabs(mu) < ORC_MU_EPS;
        if (clamped) mu = (mu >= 0.0) ? ORC_MU_EPS : -ORC_MU_EPS;
        double ut = 0.0;
        for (int32_t i = 0; i < N; ++i) ut += u[i] * th[i];
        for (int32_t k = 0; k < N; ++k)
            gv[k] = clamped ? u[k] / mu : u[k] / mu - ut / ((double)N * mu * mu);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Optimizer (Sec. IV-A) -- readings R6, R7                                 */
/* ------------------------------------------------------------------------ */

double orc_lr(int64_t t, double lr0, double decay, int32_t every, int32_t restart, double lr_min)
{
    int64_t phase = (restart > 0) ? (t % restart) : t;
    int64_t e = (every > 0) ? phase / every : 0;
    double lr = lr0 * pow(decay, (double)e);
    return lr > lr_min ? lr : lr_min;
}

/* One AdamW step over n parameters, t = 1-based step count:
 *   theta <- theta (1 - lr wd)
 *   m <- b1 m + (1 - b1) g ;  v <- b2 v + (1 - b2) g^2
 *   theta <- theta - (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps) */
void orc_adamw(int64_t n, double *theta, double *m, double *v, const double *g, double lr,
               double b1, double b2, double eps, double wd, int64_t t)
{
    double bc1 = 1.0 - pow(b1, (double)t);
    double bc2 = 1.0 - pow(b2, (double)t);
    for (int64_t j = 0; j < n; ++j) {
        theta[j] *= 1.0 - lr * wd;
        m[j] = b1 * m[j] + (1.0 - b1) * g[j];
        v[j] = b2 * v[j] + (1.0 - b2) * g[j] * g[j];
        double denom = sqrt(v[j]) / sqrt(bc2) + eps;
        theta[j] -= (lr / bc1) * m[j] / denom;
    }
}

/* ------------------------------------------------------------------------ */
/* One iteration of the method, in the order of Sec. III-B and IV-A          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double tau, lr0, decay, lr_min, beta1, beta2, eps, weight_decay;
    int32_t every, restart, mode, mix;
} orc_params;

/* ------------------------------------------------------------------------ */
/* Assignment mixing at a learning-rate restart (Sec. IV-A, the paragraph    */
/* left commented out in the source, and its equation) -- reading R12        */
/* ------------------------------------------------------------------------ */

/* The best candidate: most satisfied clauses, i.e. fewest clauses with
 * R = 0 (H[i][0]), the lower index on ties. */
int32_t orc_best_candidate(int32_t N, int32_t K, const int64_t *H)
{
    int32_t best = 0;
    for (int32_t i = 1; i < N; ++i)
        if (H[(int64_t)i * (K + 1)] < H[(int64_t)best * (K + 1)]) best = i;
    return best;
}

/* Every candidate column i other than istar becomes the average of itself
 * and column istar, row by row: theta[v][i] <- (theta[v][i] + theta[v][istar]) / 2. */
int orc_mix(int32_t rows, int32_t N, double *theta, int32_t istar)
{
    if (rows < 0 || N <= 0 || !theta || istar < 0 || istar >= N) return ORC_E_ARG;
    for (int32_t v = 0; v < rows; ++v) {
        double *row = theta + (int64_t)v * N;
        double best = row[istar];
        for (int32_t i = 0; i < N; ++i)
            if (i != istar) row[i] = 0.5 * (row[i] + best);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Independent literal rows (Sec. III-B: A_real has 2V rows; the            */
/* incomplete-assignment passage of Sec. III-A left commented out in the    */
/* source) -- reading R13                                                    */
/* ------------------------------------------------------------------------ */

/* Row of literal x (signed, 1-based) in a [2V][N] literal-row matrix:
 * x_v is row 2(v-1), not-x_v row 2(v-1)+1. */
static inline int64_t lit_row(int32_t x) { return x > 0 ? 2 * (int64_t)(x - 1) : 2 * (int64_t)(-x - 1) + 1; }

/* H[i][r] = #{c : R[c][i] = r} with R_ci = sum over the literals l of c of
 * bl[row(l)][i]: a literal counts when its own row holds 1, whatever the
 * row of its complement holds (both 1: either literal satisfies its
 * clauses; both 0: neither does). */
int orc_lit_histogram(const void *h, int32_t N, const uint8_t *bl, int64_t *H)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || N <= 0 || !bl || !H) return ORC_E_ARG;
    int32_t K = f->K;
    memset(H, 0, sizeof(int64_t) * (size_t)N * (size_t)(K + 1));
    for (int64_t c = 0; c < f->C; ++c)
        for (int32_t i = 0; i < N; ++i) {
            int32_t r = 0;
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) r += bl[lit_row(f->lit[q]) * N + i];
            H[(int64_t)i * (K + 1) + r] += 1;
        }
    return ORC_OK;
}

/* U2[l][i] = dL/dA[l][i] = sum over the clauses c holding literal l of
 * dL/dR_ci (the transpose product); with independent rows the
 * straight-through estimator passes it to the literal's own row with +1. */
int orc_lit_adjoint(const void *h, int32_t N, const uint8_t *bl, int32_t K, const double *table, double *U2)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || N <= 0 || !bl || !table || !U2 || K < f->K) return ORC_E_ARG;
    memset(U2, 0, sizeof(double) * (size_t)f->V * 2 * (size_t)N);
    for (int64_t c = 0; c < f->C; ++c)
        for (int32_t i = 0; i < N; ++i) {
            int32_t r = 0;
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) r += bl[lit_row(f->lit[q]) * N + i];
            double dR = table[(int64_t)i * (K + 1) + r];
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) U2[lit_row(f->lit[q]) * N + i] += dR;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One iteration of the method, in the order of Sec. III-B and IV-A          */
/* ------------------------------------------------------------------------ */

/* Given theta, m, v (updated in place) and the 0-based iteration index t:
 * binarize -> R -> SmoothMin/loss -> dL/dR -> P^T + STE -> Eq. 5 backward
 * -> AdamW with lr(t).  rows_per_var = 1: theta is V x N, one row per
 * variable (complete assignments, reading R1); 2: theta is 2V x N, one row
 * per literal (reading R13).  t_reset: the iteration at which the optimizer
 * state last started from zero (0 for a fresh batch); the bias-correction
 * count of the update is t - t_reset + 1.
 * With p->mix, an iteration t > 0 with t mod restart = 0 does not take a
 * gradient step: after the forward pass it mixes the candidates into the
 * best one (orc_best_candidate, orc_mix) and resets the optimizer (m = v =
 * 0; the next update is the first of a fresh AdamW, so the caller passes
 * t_reset = t + 1 from then on); *mixed_out (may be NULL) receives the best
 * candidate, else -1.  Optional outputs (any may be NULL): the bits used by
 * the forward pass, H, S, loss, U and g (zero at a mixing iteration). */
int orc_step_ex(const void *h, int32_t N, const orc_params *p, int32_t rows_per_var, int64_t t, int64_t t_reset,
                double *theta, double *m, double *v, uint8_t *b_out, int64_t *H_out, double *S_out,
                double *loss_out, double *U_out, double *g_out, int32_t *mixed_out)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || !p || N <= 0 || !theta || !m || !v || (rows_per_var != 1 && rows_per_var != 2) || t_reset > t)
        return ORC_E_ARG;
    int32_t K = f->K;
    int32_t rows = rows_per_var * f->V;
    int64_t RN = (int64_t)rows * N;
    uint8_t *b = (uint8_t *)malloc((size_t)(RN > 0 ? RN : 1));
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * (size_t)(K + 1));
    double *S = (double *)malloc(sizeof(double) * (size_t)N);
    double *table = (double *)malloc(sizeof(double) * (size_t)N * (size_t)(K + 1));
    double *U = (double *)calloc((size_t)(RN > 0 ? RN : 1), sizeof(double));
    double *g = (double *)calloc((size_t)(RN > 0 ? RN : 1), sizeof(double));
    int rc = ORC_E_OOM;
    if (!b || !H || !S || !table || !U || !g) goto done;
    double loss = 0.0;
    rc = orc_binarize(rows, N, theta, p->mode, b, NULL);
    if (!rc) rc = rows_per_var == 1 ? orc_histogram(h, N, b, H) : orc_lit_histogram(h, N, b, H);
    if (!rc) rc = orc_smoothmin(N, K, H, p->tau, NULL, S, table, &loss);
    if (rc) goto done;
    const int mixing = p->mix && t > 0 && p->restart > 0 && t % p->restart == 0;
    if (!mixing) {
        rc = rows_per_var == 1 ? orc_adjoint(h, N, b, K, table, U) : orc_lit_adjoint(h, N, b, K, table, U);
        if (!rc) rc = orc_norm_backward(rows, N, theta, p->mode, U, g);
        if (rc) goto done;
    }
    if (b_out) memcpy(b_out, b, (size_t)RN);
    if (H_out) memcpy(H_out, H, sizeof(int64_t) * (size_t)N * (size_t)(K + 1));
    if (S_out) memcpy(S_out, S, sizeof(double) * (size_t)N);
    if (loss_out) *loss_out = loss;
    if (U_out) memcpy(U_out, U, sizeof(double) * (size_t)RN);
    if (g_out) memcpy(g_out, g, sizeof(double) * (size_t)RN);
    if (mixing) {
        int32_t istar = orc_best_candidate(N, K, H);
        rc = orc_mix(rows, N, theta, istar);
        for (int64_t j = 0; j < RN; ++j) m[j] = v[j] = 0.0;
        if (mixed_out) *mixed_out = istar;
    } else {
        orc_adamw(RN, theta, m, v, g, orc_lr(t, p->lr0, p->decay, p->every, p->restart, p->lr_min),
                  p->beta1, p->beta2, p->eps, p->weight_decay, t - t_reset + 1);
        if (mixed_out) *mixed_out = -1;
    }
done:
    free(b); free(H); free(S); free(table); free(U); free(g);
    return rc;
}

/* The iteration of orc_step_ex for complete assignments from a fresh
 * optimizer (t_reset = 0). */
int orc_step(const void *h, int32_t N, const orc_params *p, int64_t t, double *theta, double *m,
             double *v, uint8_t *b_out, int64_t *H_out, double *S_out, double *loss_out,
             double *U_out, double *g_out)
{
    return orc_step_ex(h, N, p, 1, t, 0, theta, m, v, b_out, H_out, S_out, loss_out, U_out, g_out, NULL);
}

/* ------------------------------------------------------------------------ */
/* Relaxed objective (for finite-difference pins of the gradient)            */
/* ------------------------------------------------------------------------ */

/* For a real-valued assignment x (V x N, x_vi in [0,1], not-x_v = 1 - x_v),
 * R~_ci = sum_{l in c} value(l), S~_i = SmoothMin over the column (Eq. 4
 * written directly, no histogram).  Returns S~ for candidate i only. */
double orc_relaxed_S(const void *h, int32_t N, const double *x, int32_t i, double tau)
{
    const ocnf *f = (const ocnf *)h;
    if (f->C == 0) return 0.0;
    double rmin = INFINITY;
    for (int64_t c = 0; c < f->C; ++c) {
        double r = 0.0;
        for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) {
            int32_t l = f->lit[q];
            int32_t v = (l > 0 ? l : -l) - 1;
            double xv = x[(int64_t)v * N + i];
            r += (l > 0) ? xv : 1.0 - xv;
        }
        if (r < rmin) rmin = r;
    }
    double num = 0.0, den = 0.0;
    for (int64_t c = 0; c < f->C; ++c) {
        double r = 0.0;
        for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) {
            int32_t l = f->lit[q];
            int32_t v = (l > 0 ? l : -l) - 1;
            double xv = x[(int64_t)v * N + i];
            r += (l > 0) ? xv : 1.0 - xv;
        }
        double w = exp(-tau * (r - rmin));
        num += r * w;
        den += w;
    }
    return num / den;
}

/* Central difference (S~_i(x + h e_vi) - S~_i(x - h e_vi)) / (2h) of the
 * relaxed SmoothMin of candidate i, evaluated without cancelling the large
 * column sums: with num = sum_c R~ w and den = sum_c w over all clauses
 * (w = e^{-tau (R~ - m)}, m a fixed shift), only clauses containing v change,
 * and S+ - S- = [num (dd- - dd+) + den (dn+ - dn-) + dn+ dd- - dn- dd+]
 *              / [(den + dd+)(den + dd-)]. */
double orc_relaxed_fd(const void *h, int32_t N, const double *x, int32_t v, int32_t i, double step, double tau)
{
    const ocnf *f = (const ocnf *)h;
    if (f->C == 0) return 0.0;
    double m = INFINITY;
    for (int64_t c = 0; c < f->C; ++c) {
        double r = 0.0;
        for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) {
            int32_t l = f->lit[q];
            int32_t u = (l > 0 ? l : -l) - 1;
            double xu = x[(int64_t)u * N + i];
            r += (l > 0) ? xu : 1.0 - xu;
        }
        if (r < m) m = r;
    }
    m -= step; /* keep every shifted exponent non-positive */
    double num = 0.0, den = 0.0, dnp = 0.0, ddp = 0.0, dnm = 0.0, ddm = 0.0;
    for (int64_t c = 0; c < f->C; ++c) {
        double r = 0.0, dr = 0.0;
        for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) {
            int32_t l = f->lit[q];
            int32_t u = (l > 0 ? l : -l) - 1;
            double xu = x[(int64_t)u * N + i];
            r += (l > 0) ? xu : 1.0 - xu;
            if (u == v) dr += (l > 0) ? step : -step;
        }
        double w = exp(-tau * (r - m));
        num += r * w;
        den += w;
        if (dr != 0.0) {
            double wp = exp(-tau * (r + dr - m)), wm = exp(-tau * (r - dr - m));
            dnp += (r + dr) * wp - r * w;
            ddp += wp - w;
            dnm += (r - dr) * wm - r * w;
            ddm += wm - w;
        }
    }
    double diff = (num * (ddm - ddp) + den * (dnp - dnm) + dnp * ddm - dnm * ddp) / ((den + ddp) * (den + ddm));
    return diff / (2.0 * step);
}

/* Relaxed loss L~(x) = -sum_i S~_i (Eq. 3). */
double orc_relaxed_loss(const void *h, int32_t N, const double *x, double tau)
{
    double s = 0.0;
    for (int32_t i = 0; i < N; ++i) s += orc_relaxed_S(h, N, x, i, tau);
    return -s;
}

/* ------------------------------------------------------------------------ */
/* Handoff (Sec. IV-B): confident partial assignments, candidate priority   */
/* ------------------------------------------------------------------------ */

/* Candidates ordered by satisfied-clause count (descending, ties: lower
 * index).  For each of the first max_cands candidates: the k variables that
 * occur in some clause and have the smallest |g_vi| (ties: lower v), in that
 * order, as signed DIMACS literals of the candidate's bits b (+(v+1) for
 * True, -(v+1) for False).  Slots beyond the number of eligible variables
 * are 0.  Outputs: cand_ids[max_cands], lits[max_cands][k],
 * sat_out[max_cands]. */
int orc_extract_partial(const void *h, int32_t N, const double *g, const uint8_t *b,
                        const int64_t *sat_count, int32_t max_cands, int32_t k,
                        int32_t *cand_ids, int32_t *lits, int64_t *sat_out)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || N <= 0 || !g || !b || !sat_count || max_cands <= 0 || max_cands > N || k <= 0)
        return ORC_E_ARG;
    int32_t V = f->V;
    uint8_t *occurs = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    uint8_t *taken = (uint8_t *)malloc((size_t)(V > 0 ? V : 1));
    if (!occurs || !order || !taken) { free(occurs); free(order); free(taken); return ORC_E_OOM; }
    for (int64_t q = 0; q < f->L; ++q) occurs[(f->lit[q] > 0 ? f->lit[q] : -f->lit[q]) - 1] = 1;
    /* selection sort of candidates: plain and obviously correct */
    for (int32_t i = 0; i < N; ++i) order[i] = i;
    for (int32_t a = 0; a < N; ++a) {
        int32_t best = a;
        for (int32_t j = a + 1; j < N; ++j) {
            int64_t sj = sat_count[order[j]], sb = sat_count[order[best]];
            if (sj > sb || (sj == sb && order[j] < order[best])) best = j;
        }
        int32_t tmp = order[a]; order[a] = order[best]; order[best] = tmp;
    }
    for (int32_t a = 0; a < max_cands; ++a) {
        int32_t i = order[a];
        cand_ids[a] = i;
        if (sat_out) sat_out[a] = sat_count[i];
        memset(taken, 0, (size_t)(V > 0 ? V : 1));
        for (int32_t s = 0; s < k; ++s) {
            int32_t pick = -1;
            double pm = 0.0;
            for (int32_t v = 0; v < V; ++v) {
                if (!occurs[v] || taken[v]) continue;
                double mag = fabs(g[(int64_t)v * N + i]);
                if (pick < 0 || mag < pm) { pick = v; pm = mag; }
            }
            if (pick < 0) { lits[(int64_t)a * k + s] = 0; continue; }
            taken[pick] = 1;
            lits[(int64_t)a * k + s] = b[(int64_t)pick * N + i] ? (pick + 1) : -(pick + 1);
        }
    }
    free(occurs); free(order); free(taken);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Learned proposal: per-variable features (reading R9)                      */
/* ------------------------------------------------------------------------ */

#define ORC_NF 16

static int clause_is_tautology(const ocnf *f, int64_t c)
{
    for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q)
        for (int64_t r = q + 1; r < f->off[c + 1]; ++r)
            if (f->lit[q] == -f->lit[r]) return 1;
    return 0;
}

/* X[v][16] = [log(1+pos_v), log(1+neg_v), (pos_v-neg_v)/max(1,deg_v),
 *             (mean width of the clauses of v)/4 (0 when deg_v = 0),
 *             h1[v][0..3], h2[v][0..3], h3[v][0..3]]
 * with pos_v / neg_v the number of non-tautological clauses holding +v / -v,
 * deg_v = pos_v + neg_v, and the signed neighbour aggregation
 *   h0[v] = [(pos-neg)/max(1,deg), (pos-neg)/sqrt(max(1,deg)),
 *            log(1+pos)-log(1+neg), 1]
 *   h_r[v][ch] = (1/max(1,Z_v)) * sum over non-tautological clauses c, over the
 *                literal l of c on v and every literal l' of c on another
 *                variable u, of sgn(l) sgn(l') h_{r-1}[u][ch],
 *   Z_v = number of such (c, l') pairs. */
int orc_features(const void *h, double *X)
{
    const ocnf *f = (const ocnf *)h;
    if (!f || !X) return ORC_E_ARG;
    const int32_t V = f->V;
    double *pos = (double *)calloc((size_t)(V > 0 ? V : 1), sizeof(double));
    double *neg = (double *)calloc((size_t)(V > 0 ? V : 1), sizeof(double));
    double *wsum = (double *)calloc((size_t)(V > 0 ? V : 1), sizeof(double));
    double *Z = (double *)calloc((size_t)(V > 0 ? V : 1), sizeof(double));
    double *hp = (double *)calloc((size_t)(V > 0 ? V : 1) * 4, sizeof(double));
    double *hn = (double *)calloc((size_t)(V > 0 ? V : 1) * 4, sizeof(double));
    uint8_t *taut = (uint8_t *)calloc((size_t)(f->C > 0 ? f->C : 1), 1);
    if (!pos || !neg || !wsum || !Z || !hp || !hn || !taut) {
        free(pos); free(neg); free(wsum); free(Z); free(hp); free(hn); free(taut);
        return ORC_E_OOM;
    }
    for (int64_t c = 0; c < f->C; ++c) {
        taut[c] = (uint8_t)clause_is_tautology(f, c);
        if (taut[c]) continue;
        int64_t k = f->off[c + 1] - f->off[c];
        for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) {
            int32_t l = f->lit[q];
            int32_t v = (l > 0 ? l : -l) - 1;
            if (l > 0) pos[v] += 1.0; else neg[v] += 1.0;
            wsum[v] += (double)k;
            Z[v] += (double)(k - 1);
        }
    }
    for (int32_t v = 0; v < V; ++v) {
        double deg = pos[v] + neg[v];
        double *x = X + (int64_t)v * ORC_NF;
        x[0] = log(1.0 + pos[v]);
        x[1] = log(1.0 + neg[v]);
        x[2] = (pos[v] - neg[v]) / (deg > 1.0 ? deg : 1.0);
        x[3] = deg > 0.0 ? wsum[v] / deg / 4.0 : 0.0;
        hp[4 * v + 0] = x[2];
        hp[4 * v + 1] = (pos[v] - neg[v]) / sqrt(deg > 1.0 ? deg : 1.0);
        hp[4 * v + 2] = x[0] - x[1];
        hp[4 * v + 3] = 1.0;
    }
    for (int r = 1; r <= 3; ++r) {
        memset(hn, 0, sizeof(double) * 4 * (size_t)V);
        for (int64_t c = 0; c < f->C; ++c) {
            if (taut[c]) continue;
            for (int64_t q = f->off[c]; q < f->off[c + 1]; ++q) {
                int32_t l = f->lit[q];
                int32_t v = (l > 0 ? l : -l) - 1;
                for (int64_t e = f->off[c]; e < f->off[c + 1]; ++e) {
                    int32_t l2 = f->lit[e];
                    int32_t u = (l2 > 0 ? l2 : -l2) - 1;
                    if (u == v) continue;
                    double sg = ((l > 0) == (l2 > 0)) ? 1.0 : -1.0;
                    for (int ch = 0; ch < 4; ++ch) hn[4 * v + ch] += sg * hp[4 * u + ch];
                }
            }
        }
        for (int32_t v = 0; v < V; ++v) {
            double z = Z[v] > 1.0 ? Z[v] : 1.0;
            for (int ch = 0; ch < 4; ++ch) {
                hn[4 * v + ch] /= z;
                X[(int64_t)v * ORC_NF + 4 * r + ch] = hn[4 * v + ch];
            }
        }
        double *t = hp; hp = hn; hn = t;
    }
    free(pos); free(neg); free(wsum); free(Z); free(hp); free(hn); free(taut);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Random streams and initialisation (readings R10, R11)                     */
/* ------------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds: each round multiplies words 0 and 2 by the two
 * published constants, swaps the high/low halves across the pairs and xors in
 * the key, which is bumped by the two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, int64_t e, uint32_t w[4])
{
    uint32_t ctr[4] = {(uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0x5A17u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

/* N(0,1) by Box-Muller on two uniforms in (0,1), rounded to FP32. */
static float box_muller(const uint32_t w[4])
{
    double u1 = ((double)w[0] + 0.5) / 4294967296.0;
    double u2 = ((double)w[1] + 0.5) / 4294967296.0;
    return (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2));
}

/* Random initialisation theta[v][i] ~ N(0,1) (Sec. IV-A), FP32. */
int orc_init_normal(int32_t V, int32_t N, uint64_t seed, float *theta)
{
    if (V < 0 || N <= 0 || !theta) return ORC_E_ARG;
    for (int64_t e = 0; e < (int64_t)V * N; ++e) {
        uint32_t w[4];
        draw(seed, e, w);
        theta[e] = box_muller(w);
    }
    return ORC_OK;
}

/* Initialisation from a proposal p[v] = P(x_v = true) (reading R11). */
int orc_init_proposal(int32_t V, int32_t N, uint64_t seed, const float *p, int32_t mode, float *theta)
{
    if (V < 0 || N <= 0 || !theta || (V > 0 && !p)) return ORC_E_ARG;
    uint8_t *b = (uint8_t *)malloc((size_t)N);
    float *a = (float *)malloc(sizeof(float) * (size_t)N);
    if (!b || !a) { free(b); free(a); return ORC_E_OOM; }
    for (int32_t v = 0; v < V; ++v) {
        double pv = p[v];
        if (!(pv >= 0.0)) pv = 0.0; /* NaN and negatives */
        if (pv > 1.0) pv = 1.0;
        double thr = floor(pv * 4294967296.0);
        int any = 0;
        for (int32_t i = 0; i < N; ++i) {
            uint32_t w[4];
            draw(seed, (int64_t)v * N + i, w);
            a[i] = fabsf(box_muller(w));
            b[i] = ((double)w[2] < thr) ? 1 : 0;
            any |= b[i];
        }
        double rho = 1.0;
        if (mode == 1) {
            if (!any) b[v % N] = 1;
            double sp = 0.0, sn = 0.0;
            for (int32_t i = 0; i < N; ++i) {
                if (b[i]) sp += a[i]; else sn += a[i];
            }
            if (sn > 0.0 && 0.5 * sp / sn < 1.0) rho = 0.5 * sp / sn;
        }
        for (int32_t i = 0; i < N; ++i)
            theta[(int64_t)v * N + i] = b[i] ? a[i] : (float)(-rho * (double)a[i]);
    }
    free(b); free(a);
    return ORC_OK;
}
