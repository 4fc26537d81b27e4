/*
 * sisso_oracle.c -- plain, slow, FP64 reference of the SISSO hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP path (different language, different algorithms where the method
 * allows: enumeration by nested loops instead of closed-form index inversion,
 * two-pass statistics instead of shifted one-pass sums, Gaussian elimination
 * instead of incremental Cholesky).
 *
 * What it computes, step by step, in the paper's order (Sec. 2):
 *   1. Feature expansion (Sec. 2.1, eq. feature-exp): phi_l built from
 *      phi_{l-1} by applying unary and binary operators.  phi_l contains all
 *      lower levels (worked example of Sec. 2.1).  Pairs are unordered and
 *      never a feature with itself (the example has no x1+x1); a binary pair
 *      needs one operand that is new at the previous level (the example's
 *      count of 14, which excludes regenerated x1+x2 and x1*x2).
 *   2. SIS (Sec. 2.2, eq. sis-weight and sis-method): weight of a feature =
 *      correlation of the standardised feature with the target / residual;
 *      keep the k largest |w|.
 *   3. SO (Sec. 2.3, eq. residual and subspace-expansion): exhaustive least
 *      squares over every t-subset of S_t, residual of the best model feeds
 *      the next SIS; S_{t+1} = S_t u SIS(r_t*).
 *
 * Readings where the paper is silent (the same readings the HIP path takes):
 *   - canonical numbering: P_0 = base features; level l appends, first, for
 *     each operand a new at level l-1 (ascending) each unary op (list order);
 *     then for each unordered pair (i < j) with j new at level l-1, ordered by
 *     (j, i), each binary slot.  Slots: ADD, SUB, MUL give op(P[j], P[i]);
 *     DIV gives P[j]/P[i] then P[i]/P[j].
 *   - one-sided next-level slice (used at rung 3, rect = 1): after the last
 *     pool level L, for each u new at level L: each unary op of u; then for
 *     each u new at level L, each v in P_{L-1}, each binary slot: op(u, v)
 *     (DIV: u/v, v/u).
 *   - the whole next level (rect = 2): level L + 1 numbered as every TRI
 *     level, without stored tables (its ids are decoded by searching the pair
 *     counts), so that a rung-3 space of 10^13 features can be sliced.
 *   - validity: a feature is invalid if an operand is invalid, a domain is
 *     violated (sqrt of a negative, log of a non-positive, division by zero,
 *     1/0), a value is non-finite or exceeds 1e15 in magnitude, the feature
 *     is near-constant (sd <= 1e-6 |mean| or sd == 0), or it is a sum or
 *     difference that cancels (sd <= 1e-5 x the larger root-mean-square of
 *     its two operands): such a feature is an identity that is zero or
 *     constant in exact arithmetic and carries only rounding noise.
 *   - score = |Pearson correlation| (standardised features; the variance
 *     convention cancels).  Ties ordered by (score desc, id asc).
 *   - duplicates: classes = connected components of 1 - |corr| <= 1e-9 over
 *     the screened list plus the previous subspace; representative = min id,
 *     class score = max member score; classes touching the previous subspace
 *     are dropped.
 *   - per-sample weights (optional; Sec. 2.4's whitening for noise with a
 *     known diagonal covariance, w_s = 1 / sigma_s^2, the intercept whitened
 *     with the features): every mean, variance and covariance is the
 *     weighted one (sum_s w_s (.)), so the score is the weighted |corr| and
 *     SO is weighted least squares; unit weights give the plain method.
 *   - SO fits y (not the residual) with an intercept that is not counted in
 *     the t terms; eq. residual is read with an inverse (normal equations);
 *     a tuple is rank deficient when a Gaussian-elimination pivot of the unit-
 *     diagonal (correlation-scaled) normal matrix is <= 1e-10; the best tuple
 *     is the lexicographically smallest id tuple whose SSE is within
 *     1e-12 * S_yy of the minimum.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_DIV = 3, OP_SQ = 4, OP_CUBE = 5,
       OP_SQRT = 6, OP_INV = 7, OP_EXP = 8, OP_NEXP = 9, OP_LOG = 10, OP_SIN = 11 };

#define OR_MAX_LEVELS 4
#define VALUE_CAP 1e15
#define CONST_REL 1e-6
#define CANCEL_REL 1e-5
#define DUP_TOL 1e-9
#define PIVOT_TOL 1e-10
#define TIE_REL 1e-12

typedef struct {
    int d, n_unary, n_binary, levels, rect;
    int unary[16], binary[8];
    int n_slots, slot_op[16], slot_rev[16];
    int64_t p[OR_MAX_LEVELS + 1];   /* p[l] = |P_l| */
    int64_t pool_count;             /* |P_levels| */
    int64_t rect_unary, rect_binary;
    int64_t total;
    int32_t *op;                    /* per pool id: op (-1 for base) */
    int64_t *left, *right;          /* per pool id: operand ids (-1 if none) */
    int n_dim;                      /* base dimensions of the units (0: no units) */
    double *units;                  /* d x n_dim exponents of the base features */
} or_space;

static int is_binary(int op) { return op >= OP_ADD && op <= OP_DIV; }

void or_space_free(or_space *s)
{
    if (!s) return;
    free(s->op); free(s->left); free(s->right); free(s->units); free(s);
}

/* Build the pool tables by enumerating the levels with nested loops. */
or_space *or_space_new(int d, const int *unary, int n_unary, const int *binary, int n_binary,
                       int levels, int rect)
{
    if (d < 1 || levels < 0 || levels > OR_MAX_LEVELS || n_unary < 0 || n_unary > 16 ||
        n_binary < 0 || n_binary > 8 || (rect && levels < 1) || rect < 0 || rect > 2)
        return NULL;
    or_space *s = (or_space *)calloc(1, sizeof(or_space));
    s->d = d; s->n_unary = n_unary; s->n_binary = n_binary; s->levels = levels; s->rect = rect;
    for (int i = 0; i < n_unary; i++) s->unary[i] = unary[i];
    for (int i = 0; i < n_binary; i++) s->binary[i] = binary[i];
    s->n_slots = 0;
    for (int i = 0; i < n_binary; i++) {
        s->slot_op[s->n_slots] = binary[i]; s->slot_rev[s->n_slots] = 0; s->n_slots++;
        if (binary[i] == OP_DIV) { s->slot_op[s->n_slots] = OP_DIV; s->slot_rev[s->n_slots] = 1; s->n_slots++; }
    }
    /* sizes first */
    int64_t p_prev2 = 0, p_prev = d;
    s->p[0] = d;
    for (int l = 1; l <= levels; l++) {
        int64_t nnew = p_prev - p_prev2;
        int64_t pairs = 0;
        for (int64_t j = p_prev2; j < p_prev; j++) pairs += j;  /* i in [0, j) */
        int64_t size = (int64_t)n_unary * nnew + (int64_t)s->n_slots * pairs;
        s->p[l] = p_prev + size;
        p_prev2 = p_prev; p_prev = s->p[l];
    }
    s->pool_count = s->p[levels];
    if (s->pool_count > ((int64_t)1 << 28)) { free(s); return NULL; }
    s->op = (int32_t *)malloc(sizeof(int32_t) * s->pool_count);
    s->left = (int64_t *)malloc(sizeof(int64_t) * s->pool_count);
    s->right = (int64_t *)malloc(sizeof(int64_t) * s->pool_count);
    for (int64_t i = 0; i < d; i++) { s->op[i] = -1; s->left[i] = -1; s->right[i] = -1; }
    int64_t pos = d;
    for (int l = 1; l <= levels; l++) {
        int64_t lo = (l >= 2) ? s->p[l - 2] : 0, hi = s->p[l - 1];
        for (int64_t a = lo; a < hi; a++)
            for (int o = 0; o < n_unary; o++) {
                s->op[pos] = unary[o]; s->left[pos] = a; s->right[pos] = -1; pos++;
            }
        for (int64_t j = lo; j < hi; j++)
            for (int64_t i = 0; i < j; i++)
                for (int sl = 0; sl < s->n_slots; sl++) {
                    s->op[pos] = s->slot_op[sl];
                    if (s->slot_rev[sl]) { s->left[pos] = i; s->right[pos] = j; }
                    else { s->left[pos] = j; s->right[pos] = i; }
                    pos++;
                }
    }
    s->total = s->pool_count;
    if (rect) {
        int64_t nlast = s->p[levels] - s->p[levels - 1];
        s->rect_unary = (int64_t)n_unary * nlast;
        if (rect == 1) {
            s->rect_binary = (int64_t)s->n_slots * nlast * s->p[levels - 1];
        } else {                       /* pairs i < j with j new at level L */
            int64_t pairs = 0;
            for (int64_t j = s->p[levels - 1]; j < s->p[levels]; j++) pairs += j;
            s->rect_binary = (int64_t)s->n_slots * pairs;
        }
        s->total += s->rect_unary + s->rect_binary;
    }
    return s;
}

int64_t or_space_total(const or_space *s) { return s->total; }
int64_t or_space_pool(const or_space *s, int level) { return (level >= 0 && level <= s->levels) ? s->p[level] : -1; }

/* Structure of feature `id`: op and operand ids (-1 if absent). */
int or_decode(const or_space *s, int64_t id, int32_t *op, int64_t *left, int64_t *right)
{
    if (id < 0 || id >= s->total) return -1;
    if (id < s->pool_count) { *op = s->op[id]; *left = s->left[id]; *right = s->right[id]; return 0; }
    int64_t loc = id - s->pool_count;
    int64_t lo = s->p[s->levels - 1];
    if (loc < s->rect_unary) {
        *op = s->unary[loc % s->n_unary];
        *left = lo + loc / s->n_unary; *right = -1;
        return 0;
    }
    loc -= s->rect_unary;
    int sl = (int)(loc % s->n_slots);
    int64_t pair = loc / s->n_slots;
    int64_t u, v;
    if (s->rect == 1) {
        u = lo + pair / lo; v = pair % lo;       /* v in P_{L-1} = [0, lo) */
    } else {
        /* pairs (j, i), i < j, j from lo upwards: j is the largest index whose
           first pair number (the pairs of all smaller j) is <= pair; found by
           bisection on that count */
        int64_t a = lo, b = s->p[s->levels] - 1;
        while (a < b) {
            int64_t m = a + (b - a + 1) / 2;
            int64_t first = (m * (m - 1) - lo * (lo - 1)) / 2;
            if (first <= pair) a = m; else b = m - 1;
        }
        u = a; v = pair - (a * (a - 1) - lo * (lo - 1)) / 2;
    }
    *op = s->slot_op[sl];
    if (s->slot_rev[sl]) { *left = v; *right = u; } else { *left = u; *right = v; }
    return 0;
}

/* ---------------------------------------------------------------- values */

/* Returns 1 if valid.  Checks finiteness, magnitude cap and near-constancy. */
static int check_values(const double *f, int n)
{
    double mean = 0.0;
    for (int s = 0; s < n; s++) {
        if (!isfinite(f[s]) || fabs(f[s]) > VALUE_CAP) return 0;
        mean += f[s];
    }
    mean /= n;
    double ss = 0.0;
    for (int s = 0; s < n; s++) ss += (f[s] - mean) * (f[s] - mean);
    double sd = sqrt(ss / n);
    if (sd == 0.0 || sd <= CONST_REL * fabs(mean)) return 0;
    return 1;
}

/* Apply op to operand values; returns 0 on a domain violation. */
static int apply_op(int op, const double *a, const double *b, double *out, int n)
{
    for (int s = 0; s < n; s++) {
        double x = a[s], y = b ? b[s] : 0.0, r;
        switch (op) {
        case OP_ADD: r = x + y; break;
        case OP_SUB: r = x - y; break;
        case OP_MUL: r = x * y; break;
        case OP_DIV: if (y == 0.0) return 0; r = x / y; break;
        case OP_SQ: r = x * x; break;
        case OP_CUBE: r = x * x * x; break;
        case OP_SQRT: if (x < 0.0) return 0; r = sqrt(x); break;
        case OP_INV: if (x == 0.0) return 0; r = 1.0 / x; break;
        case OP_EXP: r = exp(x); break;
        case OP_NEXP: r = exp(-x); break;
        case OP_LOG: if (x <= 0.0) return 0; r = log(x); break;
        case OP_SIN: r = sin(x); break;
        default: return 0;
        }
        out[s] = r;
    }
    return 1;
}

/* Evaluate feature `id` on the n samples of X (column-major, leading dim
 * ldx).  Returns 1 if valid, 0 if invalid (out is then unspecified). */
static double rms(const double *f, int n)
{
    double a = 0.0;
    for (int s = 0; s < n; s++) a += f[s] * f[s];
    return sqrt(a / n);
}

static double sd_of(const double *f, int n)
{
    double m = 0.0, ss = 0.0;
    for (int s = 0; s < n; s++) m += f[s];
    m /= n;
    for (int s = 0; s < n; s++) ss += (f[s] - m) * (f[s] - m);
    return sqrt(ss / n);
}

/* Dimensional analysis (Sec. 2.1; the dimensionality option of Sec. 3.3):
 * units are vectors of exponents over base dimensions.  A sum or difference
 * needs equal units; a product adds them, a quotient subtracts them; x^2,
 * x^3, sqrt(x), 1/x scale them by 2, 3, 1/2, -1; exp, exp(-x), ln and sin
 * need a dimensionless argument and give a dimensionless result.  Returns 0
 * for a feature that breaks a rule (not physical), else its units in u. */
int or_space_set_units(or_space *s, const double *units, int n_dim)
{
    if (!s || n_dim < 0 || n_dim > 16 || (n_dim > 0 && !units)) return 1;
    free(s->units);
    s->units = NULL;
    s->n_dim = n_dim;
    if (n_dim > 0) {
        s->units = (double *)malloc(sizeof(double) * s->d * n_dim);
        memcpy(s->units, units, sizeof(double) * s->d * n_dim);
    }
    return 0;
}

static int unit_rec(const or_space *s, int64_t id, double *u)
{
    int32_t op; int64_t l, r;
    if (or_decode(s, id, &op, &l, &r)) return 0;
    const int k = s->n_dim;
    if (op < 0) {
        for (int q = 0; q < k; q++) u[q] = s->units[(size_t)id * k + q];
        return 1;
    }
    double a[16], b[16];
    if (!unit_rec(s, l, a)) return 0;
    if (is_binary(op) && !unit_rec(s, r, b)) return 0;
    int dimless = 1;
    for (int q = 0; q < k; q++) if (a[q] != 0.0) dimless = 0;
    for (int q = 0; q < k; q++) {
        switch (op) {
        case OP_ADD: case OP_SUB: if (a[q] != b[q]) return 0; u[q] = a[q]; break;
        case OP_MUL: u[q] = a[q] + b[q]; break;
        case OP_DIV: u[q] = a[q] - b[q]; break;
        case OP_SQ: u[q] = 2.0 * a[q]; break;
        case OP_CUBE: u[q] = 3.0 * a[q]; break;
        case OP_SQRT: u[q] = 0.5 * a[q]; break;
        case OP_INV: u[q] = -a[q]; break;
        default: if (!dimless) return 0; u[q] = 0.0; break;   /* exp, exp(-x), ln, sin */
        }
    }
    return 1;
}

/* Units of feature `id` (n_dim values) and whether it is physical. */
int or_units(const or_space *s, int64_t id, double *u)
{
    if (!s->units) return 1;
    return unit_rec(s, id, u);
}

static int eval_rec(const or_space *s, const double *X, int n, int ldx, int64_t id, double *out)
{
    int32_t op; int64_t l, r;
    if (or_decode(s, id, &op, &l, &r)) return 0;
    if (s->units) {
        double u[16];
        if (!unit_rec(s, id, u)) return 0;
    }
    if (op < 0) {
        memcpy(out, X + (size_t)id * ldx, sizeof(double) * n);
        return check_values(out, n);
    }
    double *a = (double *)malloc(sizeof(double) * n);
    double *b = is_binary(op) ? (double *)malloc(sizeof(double) * n) : NULL;
    int ok = eval_rec(s, X, n, ldx, l, a);
    if (ok && b) ok = eval_rec(s, X, n, ldx, r, b);
    if (ok) ok = apply_op(op, a, b, out, n);
    if (ok) ok = check_values(out, n);
    if (ok && (op == OP_ADD || op == OP_SUB)) {
        const double ra = rms(a, n), rb = rms(b, n);
        if (sd_of(out, n) <= CANCEL_REL * (ra > rb ? ra : rb)) ok = 0;
    }
    free(a); free(b);
    return ok;
}

int or_eval(const or_space *s, const double *X, int n, int ldx, int64_t id, double *out)
{
    return eval_rec(s, X, n, ldx, id, out);
}

/* Evaluate a list of ids; valid[i] = 1/0; invalid columns are filled with NaN. */
void or_eval_many(const or_space *s, const double *X, int n, int ldx, const int64_t *ids,
                  int64_t count, double *out, int ldo, int32_t *valid)
{
    for (int64_t i = 0; i < count; i++) {
        double *o = out + (size_t)i * ldo;
        valid[i] = eval_rec(s, X, n, ldx, ids[i], o);
        if (!valid[i]) for (int t = 0; t < n; t++) o[t] = NAN;
    }
}

/* |Pearson correlation| by the two-pass definition, with sample weights w
 * (NULL: all 1): weighted means, then weighted sums of squares and products. */
double or_abs_corr_w(const double *f, const double *r, const double *w, int n)
{
    double mf = 0.0, mr = 0.0, sw = 0.0;
    for (int s = 0; s < n; s++) {
        double ws = w ? w[s] : 1.0;
        mf += ws * f[s]; mr += ws * r[s]; sw += ws;
    }
    mf /= sw; mr /= sw;
    double sff = 0.0, srr = 0.0, sfr = 0.0;
    for (int s = 0; s < n; s++) {
        double ws = w ? w[s] : 1.0;
        double a = f[s] - mf, b = r[s] - mr;
        sff += ws * a * a; srr += ws * b * b; sfr += ws * a * b;
    }
    if (sff <= 0.0 || srr <= 0.0) return NAN;
    return fabs(sfr) / sqrt(sff * srr);
}

double or_abs_corr(const double *f, const double *r, int n) { return or_abs_corr_w(f, r, NULL, n); }

/* Scores for every id in [begin, end): NaN for invalid features. */
void or_score_range_w(const or_space *s, const double *X, int n, int ldx, const double *r, const double *w,
                      int64_t begin, int64_t end, double *scores)
{
    double *f = (double *)malloc(sizeof(double) * n);
    for (int64_t id = begin; id < end; id++) {
        if (eval_rec(s, X, n, ldx, id, f)) scores[id - begin] = or_abs_corr_w(f, r, w, n);
        else scores[id - begin] = NAN;
    }
    free(f);
}

void or_score_range(const or_space *s, const double *X, int n, int ldx, const double *r,
                    int64_t begin, int64_t end, double *scores)
{
    or_score_range_w(s, X, n, ldx, r, NULL, begin, end, scores);
}

/* ------------------------------------------------------------------ SIS */

static int better(double sa, int64_t ia, double sb, int64_t ib)
{
    return sa > sb || (sa == sb && ia < ib);
}

static int in_sorted(const int64_t *arr, int64_t n, int64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) { int64_t m = (lo + hi) / 2; if (arr[m] < key) lo = m + 1; else hi = m; }
    return lo < n && arr[lo] == key;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Best `keep` valid features over [begin, end) by (score desc, id asc),
 * skipping excluded ids.  Returns the number kept (<= keep), sorted. */
int64_t or_sis_w(const or_space *s, const double *X, int n, int ldx, const double *r, const double *w,
                 int64_t begin, int64_t end, const int64_t *exclude, int64_t n_exclude,
                 int64_t keep, int64_t *out_ids, double *out_scores)
{
    int64_t *ex = (int64_t *)malloc(sizeof(int64_t) * (n_exclude > 0 ? n_exclude : 1));
    if (n_exclude > 0) memcpy(ex, exclude, sizeof(int64_t) * n_exclude);
    qsort(ex, n_exclude, sizeof(int64_t), cmp_i64);
    double *f = (double *)malloc(sizeof(double) * n);
    int64_t cnt = 0, worst = -1;
    for (int64_t id = begin; id < end; id++) {
        if (n_exclude > 0 && in_sorted(ex, n_exclude, id)) continue;
        if (!eval_rec(s, X, n, ldx, id, f)) continue;
        double sc = or_abs_corr_w(f, r, w, n);
        if (isnan(sc)) continue;
        if (cnt < keep) {
            out_ids[cnt] = id; out_scores[cnt] = sc; cnt++;
            if (cnt == keep) {
                worst = 0;
                for (int64_t q = 1; q < cnt; q++)
                    if (better(out_scores[worst], out_ids[worst], out_scores[q], out_ids[q])) worst = q;
            }
        } else if (keep > 0 && better(sc, id, out_scores[worst], out_ids[worst])) {
            out_ids[worst] = id; out_scores[worst] = sc;
            worst = 0;
            for (int64_t q = 1; q < cnt; q++)
                if (better(out_scores[worst], out_ids[worst], out_scores[q], out_ids[q])) worst = q;
        }
    }
    /* sort the kept list (insertion sort; the list is small) */
    for (int64_t a = 1; a < cnt; a++) {
        int64_t ki = out_ids[a]; double ks = out_scores[a]; int64_t b = a - 1;
        while (b >= 0 && better(ks, ki, out_scores[b], out_ids[b])) {
            out_ids[b + 1] = out_ids[b]; out_scores[b + 1] = out_scores[b]; b--;
        }
        out_ids[b + 1] = ki; out_scores[b + 1] = ks;
    }
    free(f); free(ex);
    return cnt;
}

int64_t or_sis(const or_space *s, const double *X, int n, int ldx, const double *r,
               int64_t begin, int64_t end, const int64_t *exclude, int64_t n_exclude,
               int64_t keep, int64_t *out_ids, double *out_scores)
{
    return or_sis_w(s, X, n, ldx, r, NULL, begin, end, exclude, n_exclude, keep, out_ids, out_scores);
}

/* ---------------------------------------------------------------- dedup */

static int64_t uf_find(int64_t *par, int64_t a)
{
    while (par[a] != a) { par[a] = par[par[a]]; a = par[a]; }
    return a;
}

/* Duplicate classes over m columns F (n x m, leading dim ldf): connected
 * components of 1 - |corr| <= 1e-9.  comp[i] = smallest column index of
 * the component of column i. */
void or_dup_components_w(const double *F, int n, int ldf, int64_t m, const double *w, int64_t *comp)
{
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int64_t i = 0; i < m; i++) par[i] = i;
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = i + 1; j < m; j++) {
            double c = or_abs_corr_w(F + (size_t)i * ldf, F + (size_t)j * ldf, w, n);
            if (1.0 - c <= DUP_TOL) {
                int64_t a = uf_find(par, i), b = uf_find(par, j);
                if (a != b) { if (a < b) par[b] = a; else par[a] = b; }
            }
        }
    for (int64_t i = 0; i < m; i++) comp[i] = uf_find(par, i);
    free(par);
}

void or_dup_components(const double *F, int n, int ldf, int64_t m, int64_t *comp)
{
    or_dup_components_w(F, n, ldf, m, NULL, comp);
}

/* New subspace members from a screened list.
 *   list: ids/scores (count), prev: previous subspace ids (n_prev).
 * Writes up to k representatives (ids, class scores) in rank order and
 * returns how many.  *n_classes gets the number of surviving classes. */
int64_t or_dedup_w(const or_space *s, const double *X, int n, int ldx, const double *w,
                   const int64_t *list_ids, const double *list_scores, int64_t count,
                   const int64_t *prev, int64_t n_prev, int64_t k,
                   int64_t *out_ids, double *out_scores, int64_t *n_classes)
{
    int64_t m = count + n_prev;
    double *F = (double *)malloc(sizeof(double) * (size_t)n * (m > 0 ? m : 1));
    int32_t *valid = (int32_t *)malloc(sizeof(int32_t) * (m > 0 ? m : 1));
    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int64_t i = 0; i < n_prev; i++) ids[i] = prev[i];
    for (int64_t i = 0; i < count; i++) ids[n_prev + i] = list_ids[i];
    or_eval_many(s, X, n, ldx, ids, m, F, n, valid);
    int64_t *comp = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    or_dup_components_w(F, n, n, m, w, comp);
    /* per component: excluded?, representative id, class score */
    int64_t *rep = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    double *csc = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    char *excl = (char *)calloc(m > 0 ? m : 1, 1);
    for (int64_t i = 0; i < m; i++) { rep[i] = INT64_MAX; csc[i] = -1.0; }
    for (int64_t i = 0; i < m; i++) {
        int64_t c = comp[i];
        if (i < n_prev) { excl[c] = 1; continue; }
        if (ids[i] < rep[c]) rep[c] = ids[i];
        double sc = list_scores[i - n_prev];
        if (sc > csc[c]) csc[c] = sc;
    }
    /* collect surviving classes */
    int64_t nc = 0;
    int64_t *cls = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int64_t c = 0; c < m; c++)
        if (comp[c] == c && !excl[c] && rep[c] != INT64_MAX) cls[nc++] = c;
    /* rank by (score desc, rep asc): insertion sort */
    for (int64_t a = 1; a < nc; a++) {
        int64_t key = cls[a], b = a - 1;
        while (b >= 0 && better(csc[key], rep[key], csc[cls[b]], rep[cls[b]])) { cls[b + 1] = cls[b]; b--; }
        cls[b + 1] = key;
    }
    int64_t take = nc < k ? nc : k;
    for (int64_t i = 0; i < take; i++) { out_ids[i] = rep[cls[i]]; out_scores[i] = csc[cls[i]]; }
    *n_classes = nc;
    free(F); free(valid); free(ids); free(comp); free(rep); free(csc); free(excl); free(cls);
    return take;
}

int64_t or_dedup(const or_space *s, const double *X, int n, int ldx,
                 const int64_t *list_ids, const double *list_scores, int64_t count,
                 const int64_t *prev, int64_t n_prev, int64_t k,
                 int64_t *out_ids, double *out_scores, int64_t *n_classes)
{
    return or_dedup_w(s, X, n, ldx, NULL, list_ids, list_scores, count, prev, n_prev, k, out_ids, out_scores,
                      n_classes);
}

/* ------------------------------------------------------------------- SO */

/* Solve the D x D system A x = b (row-major, in place) by Gaussian
 * elimination with partial pivoting.  Returns 0 if a pivot is <= tol. */
static int gauss_solve(double *A, double *b, int D, double tol)
{
    for (int c = 0; c < D; c++) {
        int piv = c;
        for (int r = c + 1; r < D; r++) if (fabs(A[r * D + c]) > fabs(A[piv * D + c])) piv = r;
        if (fabs(A[piv * D + c]) <= tol) return 0;
        if (piv != c) {
            for (int q = 0; q < D; q++) { double t = A[c * D + q]; A[c * D + q] = A[piv * D + q]; A[piv * D + q] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < D; r++) {
            double fct = A[r * D + c] / A[c * D + c];
            for (int q = c; q < D; q++) A[r * D + q] -= fct * A[c * D + q];
            b[r] -= fct * b[c];
        }
    }
    for (int c = D - 1; c >= 0; c--) {
        double acc = b[c];
        for (int q = c + 1; q < D; q++) acc -= A[c * D + q] * b[q];
        b[c] = acc / A[c * D + c];
    }
    return 1;
}

/* SSE of the least-squares fit of centred y on the centred columns listed in
 * tup, from the centred Gram G (m x m) and b = F~' y~.  Works on the unit-
 * diagonal scaled system.  Returns -1 if rank deficient. */
static double tuple_sse(const double *G, const double *bv, int64_t m, const int64_t *tup, int D,
                        double syy, double *coef_scaled)
{
    double A[64], rhs[8], sc[8];
    for (int a = 0; a < D; a++) {
        double g = G[tup[a] * m + tup[a]];
        if (g <= 0.0) return -1.0;
        sc[a] = sqrt(g);
    }
    for (int a = 0; a < D; a++) {
        for (int c = 0; c < D; c++) A[a * D + c] = G[tup[a] * m + tup[c]] / (sc[a] * sc[c]);
        rhs[a] = bv[tup[a]] / sc[a];
    }
    double rhs0[8];
    for (int a = 0; a < D; a++) rhs0[a] = rhs[a];
    if (!gauss_solve(A, rhs, D, PIVOT_TOL)) return -1.0;
    double fit = 0.0;
    for (int a = 0; a < D; a++) fit += rhs0[a] * rhs[a];
    if (coef_scaled) for (int a = 0; a < D; a++) coef_scaled[a] = rhs[a] / sc[a];
    double sse = syy - fit;
    return sse > 0.0 ? sse : 0.0;
}

static int next_comb(int64_t *t, int D, int64_t m)
{
    int i = D - 1;
    while (i >= 0 && t[i] == m - D + i) i--;
    if (i < 0) return 0;
    t[i]++;
    for (int j = i + 1; j < D; j++) t[j] = t[j - 1] + 1;
    return 1;
}

/* Exhaustive l0 search over all D-subsets of the m columns of F (n x m,
 * leading dim ldf), whose column order must be ascending in feature id so
 * that lexicographic position order equals lexicographic id order.
 * Outputs: best tuple (positions), its SSE, the runner-up SSE (best SSE over
 * the other tuples), coefficients (intercept first), and counts.
 * Returns 0 on success, 1 if every tuple is rank deficient. */
int or_l0_w(const double *F, int n, int ldf, int64_t m, const double *y, const double *w, int D,
            int64_t *best, double *best_sse, double *runner_up, double *coef,
            int64_t *n_tuples, int64_t *n_singular)
{
    if (D < 1 || D > 8 || m < D) return 2;
    double ym = 0.0, sw = 0.0;
    for (int s = 0; s < n; s++) { double ws = w ? w[s] : 1.0; ym += ws * y[s]; sw += ws; }
    ym /= sw;
    double *mu = (double *)malloc(sizeof(double) * m);
    for (int64_t i = 0; i < m; i++) {
        double a = 0.0;
        for (int s = 0; s < n; s++) a += (w ? w[s] : 1.0) * F[(size_t)i * ldf + s];
        mu[i] = a / sw;
    }
    double syy = 0.0;
    for (int s = 0; s < n; s++) syy += (w ? w[s] : 1.0) * (y[s] - ym) * (y[s] - ym);
    double *G = (double *)malloc(sizeof(double) * m * m);
    double *bv = (double *)malloc(sizeof(double) * m);
    for (int64_t i = 0; i < m; i++) {
        double bb = 0.0;
        for (int s = 0; s < n; s++) bb += (w ? w[s] : 1.0) * (F[(size_t)i * ldf + s] - mu[i]) * (y[s] - ym);
        bv[i] = bb;
        for (int64_t j = 0; j <= i; j++) {
            double g = 0.0;
            for (int s = 0; s < n; s++)
                g += (w ? w[s] : 1.0) * (F[(size_t)i * ldf + s] - mu[i]) * (F[(size_t)j * ldf + s] - mu[j]);
            G[i * m + j] = g; G[j * m + i] = g;
        }
    }
    /* pass 1: minimum SSE (and the second smallest) */
    int64_t t[8];
    double min1 = INFINITY, min2 = INFINITY;
    int64_t cnt = 0, sing = 0;
    for (int a = 0; a < D; a++) t[a] = a;
    do {
        double e = tuple_sse(G, bv, m, t, D, syy, NULL);
        cnt++;
        if (e < 0.0) { sing++; continue; }
        if (e < min1) { min2 = min1; min1 = e; } else if (e < min2) min2 = e;
    } while (next_comb(t, D, m));
    *n_tuples = cnt; *n_singular = sing;
    if (!isfinite(min1)) { free(mu); free(G); free(bv); return 1; }
    /* pass 2: lexicographically first tuple within the tie band */
    double band = min1 + TIE_REL * syy;
    for (int a = 0; a < D; a++) t[a] = a;
    do {
        double e = tuple_sse(G, bv, m, t, D, syy, NULL);
        if (e >= 0.0 && e <= band) break;
    } while (next_comb(t, D, m));
    double cs[8];
    double e = tuple_sse(G, bv, m, t, D, syy, cs);
    for (int a = 0; a < D; a++) best[a] = t[a];
    *best_sse = e;
    *runner_up = (e == min1) ? min2 : min1;
    double icpt = ym;
    for (int a = 0; a < D; a++) { coef[1 + a] = cs[a]; icpt -= cs[a] * mu[t[a]]; }
    coef[0] = icpt;
    free(mu); free(G); free(bv);
    return 0;
}

int or_l0(const double *F, int n, int ldf, int64_t m, const double *y, int D,
          int64_t *best, double *best_sse, double *runner_up, double *coef,
          int64_t *n_tuples, int64_t *n_singular)
{
    return or_l0_w(F, n, ldf, m, y, NULL, D, best, best_sse, runner_up, coef, n_tuples, n_singular);
}

/* --------------------------------------------------------------- driver */

/* Residual of a fitted model: r = y - (c0 + sum c_a F[:, tup[a]]). */
void or_residual(const double *F, int n, int ldf, const int64_t *tup, int D, const double *coef,
                 const double *y, double *r)
{
    for (int s = 0; s < n; s++) {
        double yh = coef[0];
        for (int a = 0; a < D; a++) yh += coef[1 + a] * F[(size_t)tup[a] * ldf + s];
        r[s] = y[s] - yh;
    }
}

typedef struct {
    int64_t n_list;          /* length of the screened list before dedup */
    int64_t list_ids[4096];
    double list_scores[4096];
    int64_t n_sub;           /* |S_t| */
    int64_t sub_ids[1024];   /* S_t in order (previous members first) */
    int64_t best_ids[8];     /* best tuple, ascending ids */
    double coef[9];          /* intercept first */
    double sse, runner_up, rmse, r2;
    int64_t n_tuples, n_singular;
    int status;
} or_step;

/* Full SISSO loop for t = 1..dmax (oracle).  keep0 = initial screened-list
 * size (k + slack); the slack doubles while duplicate removal leaves fewer
 * than k classes and the space is not exhausted.  Writes one or_step per t.
 * Returns the number of completed steps. */
int or_fit_w(const or_space *s, const double *X, int n, int ldx, const double *y, const double *w, int k,
             int dmax, int64_t keep0, or_step *steps)
{
    double *r = (double *)malloc(sizeof(double) * n);
    memcpy(r, y, sizeof(double) * n);
    int64_t sub[1024]; int64_t nsub = 0;
    int done = 0;
    for (int t = 1; t <= dmax; t++) {
        or_step *st = &steps[t - 1];
        memset(st, 0, sizeof(*st));
        int64_t keep = keep0;
        int64_t newids[1024]; double newsc[1024]; int64_t nnew = 0, ncls = 0, cnt = 0;
        int64_t *lids = NULL; double *lsc = NULL;
        for (;;) {
            lids = (int64_t *)realloc(lids, sizeof(int64_t) * keep);
            lsc = (double *)realloc(lsc, sizeof(double) * keep);
            cnt = or_sis_w(s, X, n, ldx, r, w, 0, s->total, sub, nsub, keep, lids, lsc);
            nnew = or_dedup_w(s, X, n, ldx, w, lids, lsc, cnt, sub, nsub, k, newids, newsc, &ncls);
            if (nnew >= k || cnt < keep || keep >= 4096) break;
            keep *= 2;
            if (keep > 4096) keep = 4096;
        }
        st->n_list = cnt < 4096 ? cnt : 4096;
        for (int64_t i = 0; i < st->n_list; i++) { st->list_ids[i] = lids[i]; st->list_scores[i] = lsc[i]; }
        free(lids); free(lsc);
        for (int64_t i = 0; i < nnew && nsub < 1024; i++) sub[nsub++] = newids[i];
        st->n_sub = nsub;
        for (int64_t i = 0; i < nsub; i++) st->sub_ids[i] = sub[i];
        if (nsub < t) { st->status = 3; break; }
        /* SO over S_t sorted by id */
        int64_t sorted[1024];
        memcpy(sorted, sub, sizeof(int64_t) * nsub);
        qsort(sorted, nsub, sizeof(int64_t), cmp_i64);
        double *F = (double *)malloc(sizeof(double) * (size_t)n * nsub);
        int32_t *valid = (int32_t *)malloc(sizeof(int32_t) * nsub);
        or_eval_many(s, X, n, ldx, sorted, nsub, F, n, valid);
        int64_t bt[8];
        int rc = or_l0_w(F, n, n, nsub, y, w, t, bt, &st->sse, &st->runner_up, st->coef,
                         &st->n_tuples, &st->n_singular);
        if (rc) { st->status = 4; free(F); free(valid); break; }
        for (int a = 0; a < t; a++) st->best_ids[a] = sorted[bt[a]];
        or_residual(F, n, n, bt, t, st->coef, y, r);
        double ss = 0.0, ym = 0.0, syy = 0.0, sw = 0.0;
        for (int q = 0; q < n; q++) {
            double wq = w ? w[q] : 1.0;
            ss += wq * r[q] * r[q]; ym += wq * y[q]; sw += wq;
        }
        ym /= sw;
        for (int q = 0; q < n; q++) syy += (w ? w[q] : 1.0) * (y[q] - ym) * (y[q] - ym);
        st->rmse = sqrt(ss / sw);
        st->r2 = 1.0 - st->sse / syy;
        free(F); free(valid);
        done = t;
    }
    free(r);
    return done;
}

int or_fit(const or_space *s, const double *X, int n, int ldx, const double *y, int k, int dmax,
           int64_t keep0, or_step *steps)
{
    return or_fit_w(s, X, n, ldx, y, NULL, k, dmax, keep0, steps);
}

int or_step_size(void) { return (int)sizeof(or_step); }
