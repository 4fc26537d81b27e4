/*
 * sisso.h -- C ABI of the SISSO hot path on MI355X (gfx950).
 *
 * The library implements the data-parallel core of SISSO (sure independence
 * screening + sparsifying operator), following Sec. 2 of "TorchSISSO"
 * (arXiv 2410.01752):
 *
 *   feature expansion   Sec. 2.1, eq. feature-exp  -> sisso_materialize_pools,
 *                                                     sisso_materialize_ids
 *   SIS screening       Sec. 2.2, eq. sis-weight,
 *                       eq. sis-method              -> sisso_prepare_residual,
 *                                                     sisso_expand_score,
 *                                                     sisso_topk
 *   subspace update     Sec. 2.3, eq. subspace-expansion
 *                       (duplicate features, Sec. 2.1 remark that some
 *                       combinations are not unique) -> sisso_subspace_update
 *   SO (l0 search)      Sec. 2.3, eq. residual      -> sisso_l0_search
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless marked [host].  Device
 *     arrays are column-major: element (s, j) of an n x m matrix with leading
 *     dimension ld is at base[j*ld + s]; ld >= n.
 *   - The caller owns every buffer, the workspace and the stream.  The
 *     library allocates no device memory inside these calls and keeps no
 *     pointer after the call's work on `stream` completes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue asynchronous work and return without synchronising;
 *     outputs are valid once the stream passes the call.
 *   - Every call validates its arguments on the host before enqueueing
 *     anything and returns a status; it never aborts, throws or prints.
 *     A launch failure reported by the HIP runtime returns SISSO_E_DEVICE.
 *   - Feature ids are canonical 64-bit integers (numbering below).  Scores are
 *     |Pearson correlation| in [0, 1].  Invalid features never appear in a
 *     screened list.
 *
 * Canonical feature numbering (the "space").  P_0 = the d base features,
 * ids 0..d-1.  Level l (1 <= l <= levels) appends N_l to the pool,
 * P_l = P_{l-1} ++ N_l, with N_{l-1} = ids [p_{l-2}, p_{l-1}) (p_{-1} = 0):
 *   1. for each a in N_{l-1} ascending, for each unary op in list order: op(a);
 *   2. for each unordered pair i < j with j in N_{l-1}, ordered by (j, i),
 *      for each binary slot: ADD, SUB, MUL give op(P[j], P[i]); DIV gives
 *      P[j] / P[i], then P[i] / P[j].
 * Pairs are never a feature with itself and need an operand new at the
 * previous level, which reproduces the paper's worked example of Sec. 2.1
 * (|phi_1| = 4, |phi_2| = 14 for d = 2 and {I, +, x}).  If `rect` is 1, the
 * SIS space adds the one-sided slice of the next level: for each u in N_L,
 * each unary op(u); then for each u in N_L, each v in P_{L-1}, each binary
 * slot: op(u, v) (DIV: u/v then v/u).  If `rect` is 2, it adds the whole next
 * level N_{L+1} of eq. feature-exp, numbered as every level above (unary
 * block, then pairs v < u with u in N_L ordered by (u, v)) but not stored:
 * its features are generated in registers like the slice's.
 *
 * Validity: a feature is invalid if an operand is invalid, a domain is
 * violated (sqrt of a negative, log of a non-positive, division by zero,
 * 1/0), a value is non-finite or exceeds 1e15 in magnitude, it is
 * near-constant (population sd <= 1e-6 |mean|, or sd == 0), or it is a sum
 * or difference that cancels (sd <= 1e-5 x the larger root-mean-square of
 * its operands: an identity that is zero or constant in exact arithmetic).
 */
#ifndef SISSO_H
#define SISSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SISSO_OK = 0,
    SISSO_E_NULL = 1,        /* a required pointer is NULL                       */
    SISSO_E_SHAPE = 2,       /* n, ld, m, d or another size is out of range       */
    SISSO_E_RANGE = 3,       /* an id, a range or k is outside the space         */
    SISSO_E_WORKSPACE = 4,   /* the workspace is smaller than its size query     */
    SISSO_E_UNSUPPORTED = 5, /* a valid request the library does not implement */
    SISSO_E_DEVICE = 6,      /* the HIP runtime reported an error                */
    SISSO_E_NUMERIC = 7      /* e.g. a constant residual (nothing to screen)     */
} sisso_status;

/* Operator codes.  Binary: 0..3, unary: 4..11 (exp(-x) is NEXP). */
typedef enum {
    SISSO_ADD = 0, SISSO_SUB = 1, SISSO_MUL = 2, SISSO_DIV = 3,
    SISSO_SQ = 4, SISSO_CUBE = 5, SISSO_SQRT = 6, SISSO_INV = 7,
    SISSO_EXP = 8, SISSO_NEXP = 9, SISSO_LOG = 10, SISSO_SIN = 11
} sisso_op;

#define SISSO_MAX_UNARY 8
#define SISSO_MAX_BINARY 4
#define SISSO_MAX_LEVELS 2
#define SISSO_MAX_N 65536          /* samples per problem                    */
#define SISSO_MAX_KEEP 2048        /* screened-list length per call          */
#define SISSO_MAX_BAND 7168        /* BF16 candidates rescored exactly       */
#define SISSO_MAX_SUBSPACE 1024    /* |S_t|                                  */
#define SISSO_MAX_D 3              /* terms per SO model                     */
#define SISSO_MAX_BATCH 4096       /* problems per batched call              */
#define SISSO_UNIT_DIMS 8          /* base dimensions of feature units        */
#define SISSO_UNIT_SCALE 16        /* unit exponents are stored times this    */

/* Feature space description (host struct).  Fill d, levels, rect and the
 * operator lists, then call sisso_space_init, which validates them and fills
 * the derived counts.  Paper: Sec. 2.1, eq. feature-exp and the count bound
 * that follows it. */
typedef struct {
    int32_t d;                         /* base features, >= 1                  */
    int32_t levels;                    /* full levels stored as pools, 1..2    */
    int32_t rect;                      /* 1: add the one-sided next-level slice;
                                          2: add the whole next level (generated) */
    int32_t n_unary, n_binary;
    int32_t unary[SISSO_MAX_UNARY];    /* sisso_op codes 4..11, distinct       */
    int32_t binary[SISSO_MAX_BINARY];  /* sisso_op codes 0..3, distinct        */
    /* filled by sisso_space_init: */
    int32_t n_slots;                   /* binary slots per pair (DIV counts 2) */
    int32_t slot_op[2 * SISSO_MAX_BINARY], slot_rev[2 * SISSO_MAX_BINARY];
    int64_t pool[SISSO_MAX_LEVELS + 1];/* pool[l] = |P_l|                      */
    int64_t rect_unary, rect_binary;   /* sizes of the slice's two blocks      */
    int64_t total;                     /* size of the SIS space                */
} sisso_space;

/* Per pool column statistics written by sisso_materialize_pools (device,
 * one record per column).  All values are taken from the FP64 column. */
typedef struct {
    float mean;      /* mean                                                   */
    float sd;        /* population standard deviation                          */
    float mean_rcp;  /* mean of 1/f (inf if the column has a zero)             */
    float maxabs;    /* max |f|                                                */
    float minabs;    /* min |f| (0 => the column has a zero)                    */
    float minval;    /* min f                                                  */
    float valid;     /* 1 = valid feature, 0 = invalid                         */
    float rms;       /* root-mean-square sqrt(mean f^2)                        */
} sisso_colstat;

/* Validate a space and fill its derived fields [host].  Errors:
 * SISSO_E_NULL, SISSO_E_SHAPE (d < 1, levels outside 1..2, rect outside
 * 0..2, operator lists too long or with wrong or repeated codes),
 * SISSO_E_RANGE (total size overflows 2^62). */
sisso_status sisso_space_init(sisso_space *space);

/* Structure of feature `id` [host]: op code (-1 for a base feature) and
 * operand ids (-1 when absent; for unary ops *right = -1).  Errors:
 * SISSO_E_NULL, SISSO_E_RANGE (id outside [0, total)). */
sisso_status sisso_decode(const sisso_space *space, int64_t id, int32_t *op, int64_t *left,
                          int64_t *right);

/* Evaluate the pool columns P_levels (ids [0, pool[levels])) in FP64 from X
 * and store them rounded to FP32 with their statistics (Sec. 2.1,
 * eq. feature-exp; step "operand pools" of the path).
 *   X        n x d FP64, leading dim ldx >= n.
 *   pool32   n x pool[levels] FP32 output, leading dim ld32 >= n, ld32 % 4 == 0.
 *   pool1_64 n x pool[1] FP64 output (level-1 values, kept for FP64
 *            re-evaluation by sisso_materialize_ids), leading dim ld64 >= n.
 *   stats    pool[levels] records output.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE (n < 2, n > SISSO_MAX_N, bad ld). */
sisso_status sisso_materialize_pools(const sisso_space *space, const double *X, int32_t n,
                                     int32_t ldx, float *pool32, int64_t ld32, double *pool1_64,
                                     int64_t ld64, sisso_colstat *stats, void *stream);

/* Evaluate arbitrary features (any id of the space) in FP64 (Sec. 2.1).
 *   pool1_64, stats  the FP64 level-1 pool and the column statistics written
 *                    by sisso_materialize_pools (operand values and validity).
 *   ids              count ids (device); ids outside [0, total) give invalid
 *                    columns, so a screened list padded with sentinels is fine.
 *   out              n x count FP64 output (leading dim ldo); invalid columns
 *                    are filled with NaN.  valid: count int32 flags (1/0).
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE. */
sisso_status sisso_materialize_ids(const sisso_space *space, int32_t n, const double *pool1_64,
                                   int64_t ld64, const sisso_colstat *stats, const int64_t *ids,
                                   int32_t count, double *out, int32_t ldo, int32_t *valid,
                                   void *stream);

/* As sisso_materialize_ids, for a caller that stored only the pool levels
 * 1..stored_levels (stats covers ids [0, pool[stored_levels])): features of
 * higher TRI levels are evaluated from their operands like slice features.
 * Used by batched problems, which store P_{levels-1}.  Errors: as
 * sisso_materialize_ids; SISSO_E_SHAPE for stored_levels outside
 * 1..levels. */
sisso_status sisso_materialize_ids_stored(const sisso_space *space, int32_t stored_levels, int32_t n,
                                          const double *pool1_64, int64_t ld64, const sisso_colstat *stats,
                                          const int64_t *ids, int32_t count, double *out, int32_t ldo,
                                          int32_t *valid, void *stream);

/* Dimensional analysis (Sec. 2.1, last paragraph; the dimensionality option
 * of Sec. 3.3).  The units of a feature are its exponents over up to
 * SISSO_UNIT_DIMS base dimensions, stored as int16 times SISSO_UNIT_SCALE
 * (exact through four nested square roots); a feature that breaks a rule
 * carries INT16_MIN as its first exponent.  The rules (a reading of the
 * paper, which names the first): a sum or difference needs operands of
 * equal units and keeps them; a product adds the exponents, a quotient
 * subtracts them; x^2, x^3, sqrt(x), 1/x scale them by 2, 3, 1/2, -1; exp,
 * exp(-x), ln and sin need a dimensionless operand and are dimensionless.
 * A feature that breaks a rule is not generated: sisso_pool_units computes
 * the units of every pool column from those of the base features and clears
 * `valid` in the stats of the columns that break a rule (so they are neither
 * scored nor combined further), and with sisso_score_args.units set the
 * screening kernels apply the same rules to the slice candidates they form.
 *   base_units  device, d rows of SISSO_UNIT_DIMS int16 (base features).
 *   units       device output, |P_levels| rows of SISSO_UNIT_DIMS int16.
 *   stats       device in/out, as sisso_materialize_pools wrote them.
 * Exponents whose magnitude would exceed 2^14 are reported as breaking a
 * rule.  Errors: SISSO_E_NULL, SISSO_E_SHAPE. */
sisso_status sisso_pool_units(const sisso_space *space, const int16_t *base_units, int16_t *units,
                              sisso_colstat *stats, void *stream);

/* Residual record used by the screening kernels (device, 4 doubles). */
typedef struct {
    double sum_r32;   /* sum of the FP32 centred residual values            */
    double s_rr;      /* sum of squares about their mean                    */
    double mean_r;    /* mean of the FP64 residual before centring          */
    double n;         /* number of samples                                  */
} sisso_resid_info;

/* Centre a FP64 residual (or the target y) and round it to FP32 for
 * screening (Sec. 2.2: SIS of the target at t = 1, of the best residual
 * r_t* afterwards, eq. subspace-expansion).
 *   r      n FP64 input.  r32: n FP32 output (padded samples untouched).
 *   info   one sisso_resid_info output.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE. */
sisso_status sisso_prepare_residual(const double *r, int32_t n, float *r32,
                                    sisso_resid_info *info, void *stream);

/* Weighted form of sisso_prepare_residual for a pass under sample weights
 * (Sec. 2.4: whitening by W = Sigma^(-1/2) when the noise covariance Sigma is
 * diagonal and known; w_s = 1 / sigma_s^2).  The model keeps its intercept,
 * so the whitened problem is weighted least squares and the screening score
 * of a candidate is its weighted |Pearson correlation| with the residual.
 *   r, w   n FP64 inputs (device); every w_s must be finite and > 0.
 *   r32    n FP32 output: wn_s (r_s - mu), with wn = w n / sum(w) (weights
 *          scaled to mean 1) and mu the weighted mean of r.
 *   w32    n FP32 output: wn (the screening kernels read it from
 *          sisso_score_args.w32).  Both buffers are read as float4 by the
 *          kernels: allocate n rounded up to a multiple of 4 floats.
 *   info   record: sum_r32 = sum of r32, s_rr = sum wn (r - mu)^2, mean_r = mu,
 *          n = n.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE.  Weights that are not positive and
 * finite give a record with s_rr = NaN, and every score of the pass is then
 * -1 (no candidate is admitted). */
sisso_status sisso_prepare_residual_weighted(const double *r, const double *w, int32_t n, float *r32, float *w32,
                                             sisso_resid_info *info, void *stream);

/* Screening precision. */
typedef enum { SISSO_FP32 = 0, SISSO_BF16 = 1 } sisso_precision;

/* Arguments of one screening pass. */
typedef struct {
    int32_t n;                    /* samples                                     */
    const float *pool32;          /* pool columns (sisso_materialize_pools)      */
    int64_t ld32;
    const sisso_colstat *stats;   /* their statistics                            */
    const float *r32;             /* centred FP32 residual (sisso_prepare_residual) */
    const sisso_resid_info *info; /* its record                                  */
    const int64_t *exclude;       /* sorted ascending ids never admitted, or NULL */
    int32_t n_exclude;
    int32_t keep;                 /* list length K', 1..SISSO_MAX_KEEP           */
    int32_t precision;            /* SISSO_FP32 (SISSO_BF16: see below)          */
    int32_t grid;                 /* persistent blocks of the binary block's
                                     kernels, 0 = default (the stored-column pass
                                     takes col_grid)                             */
    int32_t tile;                 /* tile-shape variant, 0 = default             */
    int32_t list_base;            /* first list slot this call writes: 0 starts a
                                     new pass (resets the workspace); > 0 appends
                                     to the lists of earlier calls of the pass   */
    const float *w32;             /* NULL, or the sample weights of a weighted
                                     pass (sisso_prepare_residual_weighted; r32
                                     and info must come from the same call):
                                     scores are weighted |corr| (Sec. 2.4).
                                     FP32 precision only                        */
    const int16_t *units;         /* NULL, or the pool columns' units from
                                     sisso_pool_units: slice candidates that
                                     break dimensional analysis are invalid.
                                     FP32 and 16-bit screening forms only       */
    int32_t col_grid;             /* blocks of the stored-column pass, 0 =
                                     default (2048), at most 16384              */
} sisso_score_args;

/* Workspace of a screening pass: per-block candidate lists plus a header.
 * The size depends on keep and on the launch shape of the call. */
size_t sisso_score_workspace_size(const sisso_space *space, const sisso_score_args *args);

/* Reset a workspace header (fill kernel on `stream`).  sisso_expand_score
 * with list_base == 0 does this itself. */
sisso_status sisso_score_reset(void *ws, size_t ws_bytes, void *stream);

/* Number of per-block lists one sisso_expand_score call over
 * [cand_begin, cand_end) writes [host]; a pass split into several calls over
 * disjoint ranges sets each call's list_base to the sum of the earlier calls'
 * counts.  Returns -1 on invalid arguments. */
int32_t sisso_expand_score_lists(const sisso_space *space, const sisso_score_args *args,
                                 int64_t cand_begin, int64_t cand_end);

/* Score every feature with id in [cand_begin, cand_end) against the residual
 * and keep, per block, the best `keep` valid ones (score desc, id asc),
 * admitting only candidates not in `exclude` (Sec. 2.2, eq. sis-weight and
 * eq. sis-method).  Pool columns are scored from their stored FP32 values;
 * the slice features op(u, v) are generated in registers from the stored
 * operand columns and never written to memory.  Several calls may feed one
 * workspace (e.g. disjoint ranges); sisso_topk then merges them.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE, SISSO_E_RANGE (empty or outside
 * [0, total) range, keep outside 1..SISSO_MAX_KEEP), SISSO_E_WORKSPACE (also
 * when list_base plus this call's lists exceeds the workspace's capacity),
 * SISSO_E_UNSUPPORTED (precision other than SISSO_FP32 in this entry point). */
sisso_status sisso_expand_score(const sisso_space *space, const sisso_score_args *args,
                                int64_t cand_begin, int64_t cand_end, void *ws, size_t ws_bytes,
                                void *stream);

/* 16-bit screening of the one-sided slice's binary block (Sec. 2.2's
 * screening carried out on matrix cores, an addition to the paper's method;
 * the entry points keep the name bf16 of their first form).  With centred
 * operands the sums of every form op(u, v) are contractions over the samples;
 * twelve GEMMs per tile of (u, v) pairs run on FP16 MFMA (operands scaled by
 * powers of two near their inverse RMS) with FP32 accumulation and give
 * approximate scores.  A candidate whose approximate variance is too
 * ill-conditioned for 16-bit operands (below 1e-2 of the magnitude of the
 * terms it is formed from) is scored exactly instead.  The best `band`
 * candidates by approximate score, and the exactly scored ones, are then
 * rescored with the FP32 path's arithmetic and written as per-block lists
 * into `ws` (list_base as in sisso_expand_score), so sisso_topk returns FP32
 * scores.  A list of flagged candidates that overflows its capacity is
 * reported by sisso_topk_status (3).
 *   ops       u-side column constants from sisso_prepare_bf16 (size from
 *             sisso_bf16_operands_size; residual-independent, once per problem).
 *   bws       per-call workspace (size from sisso_bf16_workspace_size).
 *   band      candidates rescored, keep <= band <= SISSO_MAX_BAND: the
 *             band best approximate scores of the slice (score desc, id asc;
 *             every block keeps its best band and the grid shares the running
 *             bound, so the band does not depend on the grid).  A band wider
 *             than keep is the margin that absorbs 16-bit ranking errors near
 *             the cutoff.
 * [cand_begin, cand_end) must lie in the binary block of the slice.  The
 * recall of the band against the FP32 screening is measured by the tests.
 * Errors: as sisso_expand_score; SISSO_E_UNSUPPORTED without a one-sided
 * slice (rect 1). */
size_t sisso_bf16_operands_size(const sisso_space *space, int32_t n);
sisso_status sisso_prepare_bf16(const sisso_space *space, const sisso_score_args *args, void *ops,
                                size_t ops_bytes, void *stream);
size_t sisso_bf16_workspace_size(const sisso_space *space, const sisso_score_args *args, int32_t band);
int32_t sisso_expand_score_bf16_lists(const sisso_space *space, const sisso_score_args *args,
                                      int32_t band);
/* The three steps of sisso_expand_score_bf16, for callers that time or
 * overlap them: the residual-dependent operands (v-side column sums, the u
 * side's residual sums and the v-side staging image that the moments screens
 * of sisso_bf16_screen_moments copy), the MFMA screen into the band lists of
 * `bws`, and the band top-k plus exact FP32 rescore into `ws`. */
sisso_status sisso_bf16_residual(const sisso_space *space, const sisso_score_args *args, int32_t band,
                                 void *bws, size_t bws_bytes, void *stream);
sisso_status sisso_bf16_screen(const sisso_space *space, const sisso_score_args *args, const void *ops,
                               size_t ops_bytes, int32_t band, int64_t cand_begin, int64_t cand_end,
                               void *bws, size_t bws_bytes, void *stream);
sisso_status sisso_bf16_rescore(const sisso_space *space, const sisso_score_args *args, int32_t band,
                                void *bws, size_t bws_bytes, void *ws, size_t ws_bytes, void *stream);
sisso_status sisso_expand_score_bf16(const sisso_space *space, const sisso_score_args *args,
                                     const void *ops, size_t ops_bytes, int32_t band,
                                     int64_t cand_begin, int64_t cand_end, void *bws, size_t bws_bytes,
                                     void *ws, size_t ws_bytes, void *stream);

/* Residual-independent moments of the 16-bit screen.  The weights of
 * Sec. 2.2 take the columns of the feature matrix standardised (zero mean,
 * unit variance); that standardisation depends on the features alone, not on
 * the residual, so the SIS passes of one fit (one per SO dimension) share it.
 * Likewise, of the twelve GEMMs of the 16-bit screen, nine give per-pair sums
 * that do not involve the residual.  A screen in mode SISSO_MOMENTS_WRITE
 * first runs those nine and stores, for every (u, v) pair of the tiles it
 * covers, six FP32 values (sum h and the variance of u v, u/v and v/u), the
 * candidates the conditioning test flags, and the u side's FP16 operands;
 * then, like a screen in mode SISSO_MOMENTS_READ, it runs only the three
 * residual GEMMs, stores their per-pair results, and scores every pair from
 * them and the stored moments.  The approximate scores of these screens
 * equal, bit for bit, those of a plain screen of the same residual, so the
 * band, the rescore and the result are the same.
 *   moments        device buffer of sisso_bf16_moments_size(space, n) bytes,
 *                  owned by the caller: 24 bytes per pair of the padded
 *                  64 x 64 tiles (about 69 GB for 2.65M x 1030 operand
 *                  pairs), the flagged candidates, 8 bytes per sample of each
 *                  newest-level operand (its FP16 operands, about 42 GB at
 *                  n = 2000), 12 bytes per pair of scratch for a pass's
 *                  residual GEMMs (about 35 GB), and 12 bytes per sample of
 *                  each previous-level operand.
 *   mode           SISSO_MOMENTS_NONE (moments unused, may be NULL: the same
 *                  as sisso_bf16_screen), SISSO_MOMENTS_WRITE or
 *                  SISSO_MOMENTS_READ.
 * The moments screens size their own grids (args->grid applies to the plain
 * form).  Over a large range the scores are taken in two steps: the best
 * candidate of every 32 x 32 pair sub-tile of every eighth 64-column u tile
 * gives a bound tau (their band-th best score, a lower bound of the range's
 * band-th best), then every candidate scoring at least tau is appended to the
 * workspace; if more reach tau than the workspace holds, the range is scored
 * again with per-block band lists (same band, more time).  The environment
 * variable SISSO_BF16_BOUND_STEP (1 .. 1024, read at each call) replaces the
 * sampling step 8.
 * A READ screen requires an earlier WRITE screen over the same pools, the same
 * operands (`ops`) and a candidate range covering its own, into the same
 * buffer; any residual, keep, band or exclusion list may differ.  The library
 * does not track this: reading moments that were never written gives wrong
 * scores, not an error.
 * Errors: as sisso_bf16_screen; SISSO_E_RANGE (unknown mode), SISSO_E_NULL
 * (moments NULL in mode WRITE or READ), SISSO_E_WORKSPACE (moments_bytes
 * smaller than the size query). */
typedef enum { SISSO_MOMENTS_NONE = 0, SISSO_MOMENTS_WRITE = 1, SISSO_MOMENTS_READ = 2 } sisso_moments_mode;
size_t sisso_bf16_moments_size(const sisso_space *space, int32_t n);
sisso_status sisso_bf16_screen_moments(const sisso_space *space, const sisso_score_args *args,
                                       const void *ops, size_t ops_bytes, int32_t band,
                                       int64_t cand_begin, int64_t cand_end, void *moments,
                                       size_t moments_bytes, int32_t mode, void *bws, size_t bws_bytes,
                                       void *stream);
/* The moments work of a WRITE screen in two steps, for callers that time or
 * overlap them: sisso_bf16_moments_images writes both sides' FP16 operand
 * images into `moments` (residual-independent), sisso_bf16_moments_pass then
 * runs the nine residual-independent GEMMs and stores the moments and the
 * flagged candidates.  images, pass, then a READ screen of the same call
 * arguments equal a WRITE screen, bit for bit.  Both need the call's
 * sisso_bf16_residual step first (they read the v-side column sums in `bws`).
 * Arguments and errors as sisso_bf16_screen_moments (no mode). */
sisso_status sisso_bf16_moments_images(const sisso_space *space, const sisso_score_args *args,
                                       const void *ops, size_t ops_bytes, int32_t band,
                                       int64_t cand_begin, int64_t cand_end, void *moments,
                                       size_t moments_bytes, void *bws, size_t bws_bytes, void *stream);
sisso_status sisso_bf16_moments_pass(const sisso_space *space, const sisso_score_args *args,
                                     const void *ops, size_t ops_bytes, int32_t band,
                                     int64_t cand_begin, int64_t cand_end, void *moments,
                                     size_t moments_bytes, void *bws, size_t bws_bytes, void *stream);

/* Merge the workspace's per-block lists into the global best k (score desc,
 * id asc) (Sec. 2.2, eq. sis-method).  The merge takes no exclusion list:
 * the ids of S_{t-1} are excluded when candidates enter the per-block lists
 * (sisso_score_args.exclude), so that an excluded feature never occupies a
 * list slot that a screened candidate needs; filtering them at the merge
 * would need lists longer by |S_{t-1}|.  out_ids / out_scores: k entries;
 * out_count: number written (< k when fewer valid features exist).
 * Deterministic: identical for any grid or tile choice.  The entries above the
 * k-th score and those tied with it are gathered in a buffer of 8192; the BF16
 * band (k <= SISSO_MAX_BAND = 8192 - 1024) thus leaves room for 1024 ties at
 * its cutoff.
 * Errors: SISSO_E_NULL, SISSO_E_RANGE (k < 1 or k larger than the keep the
 * workspace was filled with). */
sisso_status sisso_topk(const void *ws, size_t ws_bytes, int32_t k, int64_t *out_ids,
                        float *out_scores, int32_t *out_count, void *stream);

/* Threshold alternative of Sec. 2.2: instead of the best k, every screened
 * candidate whose score is at least tau (0 <= tau <= 1), by (score desc, id
 * asc), at most max_out of them (1..SISSO_MAX_BAND): out_ids / out_scores
 * (device, max_out entries), *out_count (device) the number returned.  The
 * per-block lists of the screening pass hold K' entries each, so the list is
 * complete only if no block filled its list with candidates at or above tau:
 * sisso_topk_status reports 4 when one did (screen again with a larger K'), 5
 * when more than max_out candidates reach tau (the best max_out are
 * returned).  A workspace filled by the BF16 form holds the rescored band
 * only: its threshold list is complete for the candidates the band reached.
 * Errors: SISSO_E_NULL, SISSO_E_RANGE (max_out or tau), SISSO_E_WORKSPACE. */
sisso_status sisso_select_threshold(const void *ws, size_t ws_bytes, float tau, int32_t max_out,
                                    int64_t *out_ids, float *out_scores, int32_t *out_count, void *stream);

/* Outcome of the last sisso_topk on a workspace, copied on `stream` into
 * *out_status (device int32): 0 = exact result; 1 = more entries tie at the
 * k-th score than the gather buffer holds behind the entries above it (every
 * entry above the cutoff is still returned, and every returned score is
 * correct, but the tied entries returned need not be those of smallest id);
 * 2 = k was larger than the keep the workspace was filled with (nothing
 * returned); 3 = a BF16-form screen into this workspace could not keep every
 * candidate it had to score exactly (the band may lack some); 4, 5: see
 * sisso_select_threshold.  A caller that needs the (score desc, id asc) order exactly
 * checks it once the stream has passed the call.
 * Errors: SISSO_E_NULL, SISSO_E_WORKSPACE. */
sisso_status sisso_topk_status(const void *ws, size_t ws_bytes, int32_t *out_status, void *stream);

/* ---------------------------------------------------------------- batches
 * Many independent problems over one space: cross-validation folds and
 * bootstrap resamples of a dataset, or several datasets (Sec. 3 evaluates
 * by cross-validation; Sec. 4 runs independent fits side by side).  The
 * space must be TRI with levels == 2 (rect == 0).  Each problem stores only
 * P_1 (sisso_materialize_pools with a copy of the space whose levels is 1);
 * the level-2 features are evaluated in registers from P_1 by the screening
 * kernel.  The problem table is a DEVICE array of n_problems records. */
typedef struct {
    int32_t n;                     /* samples, 2..SISSO_MAX_N                     */
    int32_t keep;                  /* list length K' of this problem, 1..keep_max */
    int64_t ld32;                  /* leading dim of pool32 and r32: >= n, % 4 == 0 */
    const float *pool32;           /* P_1: pool[1] FP32 columns                   */
    const sisso_colstat *stats;    /* their statistics                            */
    const double *r64;             /* FP64 residual (n), read by prepare          */
    float *r32;                    /* centred FP32 residual, written by prepare   */
    sisso_resid_info *info;        /* its record, written by prepare              */
    const int64_t *exclude;        /* sorted ascending ids never admitted, or NULL */
    int32_t n_exclude;
    int32_t reserved;              /* 0                                           */
} sisso_problem;

/* sisso_prepare_residual for every problem of a table (one launch).  Entries
 * with n outside 2..SISSO_MAX_N or a NULL r64/r32/info are skipped.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE (n_problems outside 1..SISSO_MAX_BATCH). */
sisso_status sisso_prepare_residual_batched(const sisso_problem *problems, int32_t n_problems, void *stream);

/* Workspace of a batched screening pass (0 for an unsupported space or
 * out-of-range sizes), and the work items per problem (-1 if unsupported). */
size_t sisso_batch_workspace_size(const sisso_space *space, int32_t n_problems, int32_t keep_max);
int32_t sisso_batch_items(const sisso_space *space);

/* Screen every problem of the table against its prepared residual in one
 * persistent launch (Sec. 2.2, eq. sis-weight and eq. sis-method).  Work
 * items (problem, 32 x 32 pair tile) and (problem, 64 stored columns) are
 * taken from an atomic counter, largest n first; each keeps its best K'_p
 * (score desc, id asc) not in the problem's exclude list.  grid: persistent
 * blocks, 0 = as many as fit on the device at once.  The scores are those of
 * the single-problem FP32 kernels.  An entry with an invalid field (n, keep,
 * ld32, a NULL pointer) is skipped and reported by sisso_topk_batched.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE (n_problems, keep_max, grid),
 * SISSO_E_UNSUPPORTED (space not TRI level 2), SISSO_E_WORKSPACE. */
sisso_status sisso_expand_score_batched(const sisso_space *space, const sisso_problem *problems,
                                        int32_t n_problems, int32_t keep_max, int32_t grid, void *ws,
                                        size_t ws_bytes, void *stream);

/* Per-problem merge of a batched screening workspace (one block per problem):
 * row p of out_ids / out_scores (stride keep_max, the value of the screening
 * call) receives problem p's best keep_p (score desc, id asc); out_count[p]
 * the number written; out_status[p] (nullable) 0, SISSO_E_SHAPE for a skipped
 * entry, or SISSO_E_RANGE if more than 4096 candidates tie at the cut.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE. */
sisso_status sisso_topk_batched(const sisso_problem *problems, int32_t n_problems, const void *ws,
                                size_t ws_bytes, int64_t *out_ids, float *out_scores, int32_t *out_count,
                                int32_t *out_status, void *stream);

/* ---------------------------------------------------------- learned proposal
 * A two-layer network (144 inputs, 256 ReLU units, one output) ranks the
 * candidates op(u, v) of the one-sided slice's binary block so that only the
 * top fraction is scored exactly (an addition to the screening of Sec. 2.2,
 * which scores every candidate).  Input of candidate (u, v, form):
 * [enc(u) | enc(v) | onehot(form) | 0], form 0..4 = u+v, u-v, u*v, u/v, v/u.
 * enc(x) (SISSO_ENC values per pool column) holds one-hot classes of x's
 * operator and of its operands and statistics of x against the residual:
 *   [0,14) [14,28) [28,42): class of x's operator, left and right operand
 *           (0 base feature, 1 + op code, 13 none);
 *   42 corr(x,r), 43 |corr(x,r)|, 44 corr(1/x,r), 45 corr(log|x|,r),
 *   46 corr(x^2,r), 47 |corr(1/x,r)|, 48 |corr(log|x|,r)|,
 *   49 clip(log10(sd/|mean|),-4,4)/4, 50 clip(skewness,-10,10)/10,
 *   51 clip(log10|mean|,-6,6)/6, 52 clip(log10 sd,-6,6)/6, 53 [min > 0],
 *   54 [x has a zero], 55 1, [56,64) 0; undefined or non-finite values 0.
 * Parameters: one FP32 array of SISSO_MLP_PARAMS values, W1 (256 x 144,
 * row-major) | b1 (256) | w2 (256) | b2 (1).  The products with W1 use BF16
 * operands (inputs and W1 rounded to nearest even) on matrix cores with FP32
 * accumulation. */
#define SISSO_ENC 64
#define SISSO_MLP_IN 144
#define SISSO_MLP_HIDDEN 256
#define SISSO_MLP_PARAMS (256 * 144 + 256 + 256 + 1)
#define SISSO_MLP_TABLES (5 * 256 + 256 + 1)

int32_t sisso_mlp_param_count(void);
int32_t sisso_mlp_table_count(void);

/* Encodings of pool columns [c_begin, c_end) against the prepared residual of
 * args (n, pool32, ld32, stats, r32, info): enc receives (c_end - c_begin)
 * rows of SISSO_ENC FP32 values.  Errors: SISSO_E_NULL, SISSO_E_SHAPE,
 * SISSO_E_RANGE (columns outside the stored pool). */
sisso_status sisso_encode_operands(const sisso_space *space, const sisso_score_args *args, int64_t c_begin,
                                   int64_t c_end, float *enc, void *stream);

/* Network inputs (count x SISSO_MLP_IN, FP32 row-major) of slice binary ids,
 * from an encoding table of every stored column (row c = column c); an id
 * outside the binary block gives a zero row.  Errors: SISSO_E_NULL,
 * SISSO_E_UNSUPPORTED (no slice), SISSO_E_SHAPE. */
sisso_status sisso_candidate_inputs(const sisso_space *space, const float *enc, const int64_t *ids, int32_t count,
                                    float *X, void *stream);

/* Exact FP32 scores of slice binary ids (the screening kernels' arithmetic;
 * -1 for an invalid candidate or an id outside the block).  Used to label
 * training examples.  Errors: as sisso_candidate_inputs. */
sisso_status sisso_score_ids(const sisso_space *space, const sisso_score_args *args, const int64_t *ids,
                             int32_t count, float *out_scores, void *stream);

/* Forward pass on a batch X (batch x SISSO_MLP_IN): Z (batch x 256) = X W1^T
 * + b1 (pre-activations), s (batch) = w2 . relu(Z) + b2. */
sisso_status sisso_mlp_forward(const float *params, const float *X, int32_t batch, float *Z, float *s,
                               void *stream);

/* Backward pass of the weighted loss sum_i w_i (s_i - t_i)^2 / sum_i w_i for
 * the forward results Z, s: grads (SISSO_MLP_PARAMS, layout of params) and
 * *loss (device, nullable).  ws: sisso_mlp_workspace_size(batch) bytes.
 * The rounding of X and W1 to BF16 is passed through unchanged. */
size_t sisso_mlp_workspace_size(int32_t batch);
sisso_status sisso_mlp_backward(const float *params, const float *X, const float *Z, const float *s,
                                const float *t, const float *w, int32_t batch, float *grads, float *loss, void *ws,
                                size_t ws_bytes, void *stream);

/* Training target of the network for count screening scores (|corr| in
 * [0, 1]): out[i] = atanh(min(|scores[i]|, 1 - 1e-6)), the Fisher z-transform,
 * which spreads the top of the score range the proposal has to rank.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE (count < 1). */
sisso_status sisso_mlp_target(const float *scores, int32_t count, float *out, void *stream);

/* Adam update of count parameters with bias-corrected moments m, v (step >= 1
 * is the update's number).  Errors: SISSO_E_NULL, SISSO_E_SHAPE. */
sisso_status sisso_adam_step(float *params, const float *grads, float *m, float *v, int64_t count, int32_t step,
                             float lr, float beta1, float beta2, float eps, void *stream);

/* First-layer parts for factorised scoring: out (rows x 256) = enc W1[:, side
 * block]^T, side 0 = the u block (columns 0..63), 1 = the v block (64..127). */
sisso_status sisso_mlp_parts(const float *params, const float *enc, int64_t rows, int32_t side, float *out,
                             void *stream);
/* Tables of the factorised score (SISSO_MLP_TABLES floats): per form the
 * BF16-rounded W1 column 128 + form plus b1, then w2, then b2. */
sisso_status sisso_mlp_tables(const float *params, float *tables, void *stream);

/* Network scores of slice binary ids from the parts (Au: rows per u - pool[L-1]
 * of N_L, Bv: rows per v of P_{L-1}); -inf outside the block.  Same value as
 * the pruned screening kernel computes. */
sisso_status sisso_mlp_score_ids(const sisso_space *space, const float *Au, const float *Bv, const float *tables,
                                 const int64_t *ids, int32_t count, float *out, void *stream);

/* *out_value (device) = the q-th largest of x[0..count) (NaN lowest). */
sisso_status sisso_select_kth(const float *x, int32_t count, int32_t q, float *out_value, void *stream);

/* Reliability of the proposal on a residual: given exact scores and network
 * scores of the same uniform id sample, out[0] (device int32) receives the
 * number of sample ids with exact score >= *exact_thr (e.g. the sample's 64th
 * best, from sisso_select_kth) and out[1] how many of them have a network
 * score >= *net_thr (the pruning threshold): out[1] / out[0] estimates the
 * recall of the pruned screening for the top of the distribution. */
sisso_status sisso_count_pass(const float *exact, const float *net, int32_t count, const float *exact_thr,
                              const float *net_thr, int32_t *out, void *stream);

/* Pruned screening of the slice's binary block over [cand_begin, cand_end):
 * candidates whose network score is >= *tau (device) are scored exactly and
 * enter the per-block lists of ws as in sisso_expand_score (list_base, grid
 * and keep of args; sisso_topk merges).  *kept (device, nullable) is
 * increased by the number of candidates scored exactly.  Exact scores are
 * bit-identical to those of sisso_expand_score.  Errors: as
 * sisso_expand_score; SISSO_E_UNSUPPORTED without a one-sided slice (rect 1). */
int32_t sisso_expand_score_pruned_lists(const sisso_space *space, const sisso_score_args *args, int64_t cand_begin,
                                        int64_t cand_end);
sisso_status sisso_expand_score_pruned(const sisso_space *space, const sisso_score_args *args, const float *Au,
                                       const float *Bv, const float *tables, const float *tau, int64_t cand_begin,
                                       int64_t cand_end, void *ws, size_t ws_bytes, unsigned long long *kept,
                                       void *stream);

/* Subspace update (Sec. 2.3, eq. subspace-expansion, with the duplicate
 * rule for non-unique features of Sec. 2.1).  Inputs: the screened list
 * (count ids, FP64 columns cand (n x count, ldc) with validity), the current
 * subspace (m_prev FP64 columns sub (n x m_prev, leading dim lds) and their
 * ids sub_ids), and the FP64 residual r the list was screened against.
 * Duplicate classes are the connected components of 1 - |corr| <= 1e-9 over
 * list + subspace; classes touching the subspace are dropped; each remaining
 * class is represented by its smallest id and scored by the largest FP64
 * |corr| of its members; the best k classes (score desc, id asc) are
 * appended to the subspace (ids to sub_ids[m_prev..], columns to sub).
 * *n_new (device int32) receives the number appended (<= k) and *n_classes
 * the number of surviving classes.  Any number of duplicate pairs is handled
 * (the components are formed by union-find as the pairs are found).
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE (m_prev + k > SISSO_MAX_SUBSPACE,
 * count > SISSO_MAX_KEEP). */
size_t sisso_subspace_workspace_size(int32_t n, int32_t count, int32_t m_prev);
sisso_status sisso_subspace_update(const double *cand, int32_t ldc, const int64_t *cand_ids,
                                   const int32_t *cand_valid, const int32_t *count_dev,
                                   int32_t count_max, const double *r, int32_t n, double *sub,
                                   int32_t lds, int64_t *sub_ids, int32_t m_prev, int32_t k,
                                   int32_t *n_new, int32_t *n_classes, void *ws, size_t ws_bytes,
                                   void *stream);

/* sisso_subspace_update under sample weights w (device, n FP64, positive;
 * NULL: the unweighted call): every correlation (the FP64 re-score of the
 * list and the duplicate test) is the weighted one (Sec. 2.4 whitening with a
 * diagonal covariance, intercept whitened).  A non-finite weight makes every
 * column invalid. */
sisso_status sisso_subspace_update_weighted(const double *cand, int32_t ldc, const int64_t *cand_ids,
                                            const int32_t *cand_valid, const int32_t *count_dev,
                                            int32_t count_max, const double *r, const double *w, int32_t n,
                                            double *sub, int32_t lds, int64_t *sub_ids, int32_t m_prev, int32_t k,
                                            int32_t *n_new, int32_t *n_classes, void *ws, size_t ws_bytes,
                                            void *stream);

/* Outcome of a finished SO search from its stats record [host]: `stats` is
 * a host copy of the 4 doubles out_stats received.  SISSO_OK when a model was
 * found; SISSO_E_NUMERIC when every tuple was singular (no model exists: the
 * call wrote tuple -1, SSE +inf and the residual y); SISSO_E_NULL. */
sisso_status sisso_l0_outcome(const double *stats);

/* SO: exhaustive l0 search (Sec. 2.3, eq. residual read with an inverse;
 * all C(m, D) models, best by residual norm).  F: n x m FP64 columns (ld)
 * whose order must be ascending in feature id (ties are broken towards the
 * lexicographically smallest position tuple among models whose SSE is within
 * 1e-12 * S_yy of the minimum).  The intercept is fitted and not counted in
 * D.  Columns are centred and scaled, their FP64 correlation Gram is formed
 * on the device, and every tuple is solved by an incremental Cholesky
 * factorisation; tuples with a pivot <= singular_tol are skipped.
 * Outputs (device): out_tuple D int32 positions (ascending), out_sse[0],
 * out_coef D + 1 doubles (intercept first), out_resid n doubles (y - fit),
 * out_stats 4 doubles (rmse, r2, tuples evaluated, tuples skipped).
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE (D outside 1..SISSO_MAX_D, m < D,
 * m > SISSO_MAX_SUBSPACE), SISSO_E_WORKSPACE.  If every tuple is singular
 * the stats record tuples skipped == tuples evaluated and out_sse = +inf;
 * the search runs asynchronously, so this outcome is read from the stats
 * record by sisso_l0_outcome (SISSO_E_NUMERIC). */
size_t sisso_l0_workspace_size(int32_t m, int32_t n, int32_t D);
sisso_status sisso_l0_search(const double *F, int32_t m, int32_t ld, int32_t n, const double *y,
                             int32_t D, double singular_tol, int32_t *out_tuple, double *out_sse,
                             double *out_coef, double *out_resid, double *out_stats, void *ws,
                             size_t ws_bytes, void *stream);

/* sisso_l0_search under sample weights w (device, n FP64, positive; NULL:
 * the unweighted call): weighted least squares, i.e. least squares on the
 * whitened problem W y, W [1, F] with W = diag(sqrt(w)) (Sec. 2.4 with a
 * diagonal noise covariance, w_s = 1 / sigma_s^2).  out_sse is
 * sum w_s e_s^2, out_resid the plain residual y - fit, out_stats[0] the
 * weighted RMSE sqrt(sum w e^2 / sum w) and out_stats[1] the weighted R^2.
 * Workspace and errors as sisso_l0_search. */
sisso_status sisso_l0_search_weighted(const double *F, int32_t m, int32_t ld, int32_t n, const double *y,
                                      const double *w, int32_t D, double singular_tol, int32_t *out_tuple,
                                      double *out_sse, double *out_coef, double *out_resid, double *out_stats,
                                      void *ws, size_t ws_bytes, void *stream);

/* sisso_l0_search for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same search with its workspace in a fixed device array of
 * the library (sisso_l0_scratch_capacity() bytes, 32 MiB, held on every
 * device the library runs on until the process ends) instead of a `ws`
 * argument.  Arguments and outputs as sisso_l0_search.  The call allocates
 * nothing.  Every call on one device shares that device's array: calls that
 * overlap on one device (concurrent streams, threads) race and must be
 * serialised by the caller; each call re-initialises what it reads.
 * Errors: as sisso_l0_search; SISSO_E_WORKSPACE when the search needs more
 * than the array holds (sisso_l0_workspace_size(m, n, D) > capacity: e.g.
 * m = 600 columns hold n <= 4400 samples, m = 1024 hold n <= 2000);
 * SISSO_E_DEVICE if the array's device address cannot be obtained. */
size_t sisso_l0_scratch_capacity(void);
sisso_status sisso_l0_search_noalloc(const double *F, int32_t m, int32_t ld, int32_t n, const double *y,
                                     int32_t D, double singular_tol, int32_t *out_tuple, double *out_sse,
                                     double *out_coef, double *out_resid, double *out_stats, void *stream);

/* ------------------------------------------------- batched subspace steps
 * The per-problem steps between screening and SO for a table of problems in
 * a fixed number of launches (the records are DEVICE arrays; every field has
 * the meaning of the single-problem argument of the same name).  Each entry's
 * results equal those of the single-problem call.  out_status (device,
 * nullable, n_problems int32) receives 0, or SISSO_E_SHAPE for an entry that
 * was skipped (a NULL pointer or a size outside its range or the bounds).
 *
 * sisso_materialize_ids_stored per entry; count <= count_max [host]. */
typedef struct {
    int32_t n, count;
    const double *pool1_64;
    int64_t ld64;
    const sisso_colstat *stats;
    const int64_t *ids;
    double *out;
    int32_t ldo, reserved;
    int32_t *valid;
} sisso_eval_problem;

sisso_status sisso_materialize_ids_batched(const sisso_space *space, int32_t stored_levels,
                                           const sisso_eval_problem *problems, int32_t n_problems,
                                           int32_t count_max, int32_t *out_status, void *stream);

/* sisso_subspace_update per entry; m_prev + count_max <= nodes_max and
 * k <= k_max [host] (nodes_max <= SISSO_MAX_SUBSPACE + SISSO_MAX_KEEP; the
 * duplicate-class step's LDS, 24 B per node, must fit the device). */
typedef struct {
    const double *cand;
    int32_t ldc, count_max;
    const int64_t *cand_ids;
    const int32_t *cand_valid;
    const int32_t *count_dev;
    const double *r;
    int32_t n, lds;
    double *sub;
    int64_t *sub_ids;
    int32_t m_prev, k;
    int32_t *n_new, *n_classes;
    void *ws;               /* sisso_subspace_workspace_size(n, count_max, m_prev) */
    int64_t ws_bytes;
} sisso_subspace_problem;

sisso_status sisso_subspace_update_batched(const sisso_subspace_problem *problems, int32_t n_problems,
                                           int32_t nodes_max, int32_t k_max, int32_t *out_status, void *stream);

/* sisso_sort_subspace per entry; m <= m_max [host]. */
typedef struct {
    const double *src;
    int32_t lds, m;
    const int64_t *ids;
    int32_t n, ldd;
    double *dst;
    int64_t *ids_sorted;
    int32_t *perm;
} sisso_sort_problem;

sisso_status sisso_sort_subspace_batched(const sisso_sort_problem *problems, int32_t n_problems, int32_t m_max,
                                         int32_t *out_status, void *stream);

/* sisso_l0_search for many independent problems (cross-validation folds,
 * bootstrap resamples: Sec. 3 and 4 run such fits side by side) in seven
 * launches in all.  The table is a DEVICE array of n_problems records; every
 * field has the meaning of the sisso_l0_search argument of the same name,
 * ws has at least sisso_l0_workspace_size(m, n, D) bytes (ws_bytes), and all
 * problems share D and singular_tol.  m_max and n_max [host] bound m and n
 * of every entry and size the launch.  out_status (device, nullable,
 * n_problems int32) receives 0, or SISSO_E_SHAPE for an entry that was
 * skipped (a NULL pointer, m outside D..m_max, n outside 2..n_max, ld < n,
 * or a short workspace).  Each problem's results equal those of
 * sisso_l0_search on it.  Errors: SISSO_E_NULL, SISSO_E_SHAPE (n_problems
 * outside 1..SISSO_MAX_BATCH, D outside 1..SISSO_MAX_D, m_max outside
 * D..SISSO_MAX_SUBSPACE, n_max outside 2..SISSO_MAX_N), SISSO_E_RANGE
 * (singular_tol). */
typedef struct {
    const double *F;       /* n x m subspace columns, ascending ids        */
    int32_t m, ld, n, reserved;
    const double *y;       /* n                                            */
    int32_t *out_tuple;    /* D (0-based columns of F)                     */
    double *out_sse;       /* 1                                            */
    double *out_coef;      /* D + 1, intercept first                       */
    double *out_resid;     /* n                                            */
    double *out_stats;     /* 4: RMSE, R^2, tuples evaluated, skipped      */
    void *ws;              /* workspace of this problem                    */
    int64_t ws_bytes;
} sisso_l0_problem;

sisso_status sisso_l0_search_batched(const sisso_l0_problem *problems, int32_t n_problems, int32_t D,
                                     int32_t m_max, int32_t n_max, double singular_tol, int32_t *out_status,
                                     void *stream);

/* Gather columns: dst[:, i] = src[:, perm[i]] for i < m (FP64), with ids.
 * Used to put a subspace in ascending id order before sisso_l0_search.
 * perm_out (device, m int32) receives the permutation that sorts ids. */
sisso_status sisso_sort_subspace(const double *src, int32_t lds, const int64_t *ids, int32_t m,
                                 int32_t n, double *dst, int32_t ldd, int64_t *ids_sorted,
                                 int32_t *perm_out, void *stream);

/* ------------------------------------------------------- pre-screening
 * Ranking of the base features before expansion, for problems with many
 * primary features (Sec. 3.1, eq. mi-exact, and the initial screening option
 * of Sec. 3.3 with its methods "mi" and "spearman").
 *   SISSO_PRESCREEN_MI        mutual information of eq. mi-exact estimated by
 *                             Gaussian kernel densities: x and y standardised
 *                             (population sd), bandwidths h_k = (4 / (k + 2))^
 *                             (1 / (k + 4)) n^(-1 / (k + 4)) (k = 1 for each
 *                             marginal, k = 2 for the joint product kernel),
 *                             the integral replaced by the mean over the n
 *                             observations of log(p(x, y) / (p(x) p(y))) with
 *                             every density the kernel average over all n
 *                             observations; 0 for a constant column.
 *   SISSO_PRESCREEN_SPEARMAN  |Pearson correlation| of the ranks (ties share
 *                             their average rank); 0 for a constant column.
 * sisso_prescreen_scores: X n x d FP64 (leading dim ldx), y n FP64, out d
 * FP64 scores (device); ws of sisso_prescreen_workspace_size(n, d) bytes.
 * Errors: SISSO_E_NULL, SISSO_E_SHAPE (n < 2, d < 1, ldx < n), SISSO_E_RANGE
 * (unknown method), SISSO_E_UNSUPPORTED (Spearman with n > 4096),
 * SISSO_E_WORKSPACE.
 * sisso_prescreen_select: the indices of the best ceil(quantile d) features by
 * (score desc, index asc) into out_idx (device, that many int32), their number
 * into *out_count (device).  Errors: SISSO_E_NULL, SISSO_E_SHAPE (d outside
 * 1..8192), SISSO_E_RANGE (quantile outside (0, 1]). */
typedef enum { SISSO_PRESCREEN_MI = 0, SISSO_PRESCREEN_SPEARMAN = 1 } sisso_prescreen_method;
size_t sisso_prescreen_workspace_size(int32_t n, int32_t d);
sisso_status sisso_prescreen_scores(const double *X, int32_t n, int32_t ldx, int32_t d, const double *y,
                                    int32_t method, double *out, void *ws, size_t ws_bytes, void *stream);
sisso_status sisso_prescreen_select(const double *scores, int32_t d, double quantile, int32_t *out_idx,
                                    int32_t *out_count, void *stream);

/* Human-readable name of a status. */
const char *sisso_status_string(sisso_status status);

/* Library version string. */
const char *sisso_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SISSO_H */
