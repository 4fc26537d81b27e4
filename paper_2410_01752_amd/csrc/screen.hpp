// screen.hpp -- pieces shared by the screening kernels (FP32 and BF16):
// workspace layout, the score formula and the per-form arithmetic of the
// one-sided rung-3 slice.  The exact FP32 rescore of a BF16 band uses the
// same functions as the plain FP32 kernel, so its scores are bit-identical.
#pragma once

#include "common.hpp"

namespace sisso {

constexpr int kSC = 32;            // samples per LDS chunk of the FP32 slice kernel

// Result slot of each of the five binary forms (ADD, SUB, MUL, u/v, v/u) in
// the pair's slot list, or -1 if the op is not in the operator set.
struct FormSlots {
    int slot[5];
};

inline FormSlots form_slots(const sisso_space *space)
{
    FormSlots fs;
    for (int k = 0; k < 5; ++k) fs.slot[k] = -1;
    for (int sl = 0; sl < space->n_slots; ++sl) {
        const int op = space->slot_op[sl], rev = space->slot_rev[sl];
        fs.slot[op == SISSO_DIV ? (rev ? 4 : 3) : op] = sl;
    }
    return fs;
}

// ------------------------------------------------------------- workspace

constexpr int kHistBins = 4096;
constexpr int kFinalCap = 8192;
static_assert(SISSO_MAX_BAND + 1024 <= kFinalCap, "a BF16 band leaves room for 1024 ties at its cutoff");

struct WsHeader {
    unsigned gthr;          // grid-wide admission bound (float bits)
    int keep;               // list length
    int n_lists;            // lists written by the last sisso_expand_score
    int status;             // 0 ok; 1 = tie overflow in sisso_topk
    unsigned prefix;        // radix select state
    int need;
    int total;              // entries considered by the select
    int n_gt, n_eq;         // gather counters
    int lists_cap;          // list slots the workspace was laid out for
    int scr_status;         // 0 ok; 3 = a 16-bit screen could not keep every flagged candidate
    int thr_count;          // threshold selection: entries at or above the threshold
    unsigned long long app; // entries appended by a 16-bit scorer in append mode
    int redo;               // 1: the append overflowed and the pass is scored again in lists
    int pad;
    unsigned hist[kHistBins];
};

struct WsView {
    WsHeader *h;
    float *sc;              // n_lists x keep
    int64_t *id;
    float *fin_sc;          // kFinalCap gather buffer
    int64_t *fin_id;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline size_t ws_bytes_for(int lists, int keep)
{
    size_t b = align256(sizeof(WsHeader));
    b += align256((size_t)lists * keep * sizeof(float));
    b += align256((size_t)lists * keep * sizeof(int64_t));
    b += align256((size_t)kFinalCap * sizeof(float));
    b += align256((size_t)kFinalCap * sizeof(int64_t));
    return b;
}

__host__ __device__ inline WsView ws_view(void *ws, int lists, int keep)
{
    char *p = (char *)ws;
    WsView v;
    v.h = (WsHeader *)p;
    p += align256(sizeof(WsHeader));
    v.sc = (float *)p;
    p += align256((size_t)lists * keep * sizeof(float));
    v.id = (int64_t *)p;
    p += align256((size_t)lists * keep * sizeof(int64_t));
    v.fin_sc = (float *)p;
    p += align256((size_t)kFinalCap * sizeof(float));
    v.fin_id = (int64_t *)p;
    return v;
}

__device__ __forceinline__ WsView ws_view_dev(void *ws)
{
    const WsHeader *h = (const WsHeader *)ws;
    return ws_view(ws, h->lists_cap, h->keep);
}

// Scores of a candidate from its shifted sums.  Returns -1 when the FP32
// statistics show a non-positive or near-constant variance.
__device__ __forceinline__ float score_from_sums(double A, double B, double C, double shift, double n,
                                                 double R1, double Srr)
{
    const double var = B - A * (A / n);
    if (!(var > 0.0)) return -1.0f;
    const double mean = shift + A / n;
    if (!(sqrt(var / n) > kConstRel * fabs(mean))) return -1.0f;
    const double cov = C - A * (R1 / n);
    double s = fabs(cov) / sqrt(var * Srr);
    if (!(s <= 1.0)) s = (s > 1.0) ? 1.0 : -1.0;   // rounding above 1, or NaN
    return (float)s;
}


// The five binary forms of a pair (u, v): ADD, SUB, MUL, u/v, v/u.  Inputs are
// the raw value x, the mean-shifted value x - mean(x) and the reciprocal of each
// operand, and the shifts of the multiplicative forms; the result is the form's
// value minus its shift.
__device__ __forceinline__ float binary_form(int k, float ur, float us, float uq, float vr, float vs, float vq,
                                             float cm, float c3, float c4)
{
    switch (k) {
    case 0: return us + vs;
    case 1: return us - vs;
    case 2: return fmaf(ur, vr, -cm);
    case 3: return fmaf(ur, vq, -c3);
    default: return fmaf(vr, uq, -c4);
    }
}

// Validity, magnitude and cancellation rules of form k of a pair, and its
// score from the shifted sums.  cu, cv: the operands' FP32 columns (read only
// when the magnitude bound does not clear the 1e15 cap).
__device__ inline float form_score(int k, float fA, double dB, double dC, double shift, const float *cu,
                                   const float *cv, int n, float umx, float umn, float urm, float vmx, float vmn,
                                   float vrm, double nd, double R1, double Srr)
{
    const bool dom = k < 3 ? true : (k == 3 ? vmn > 0.f : umn > 0.f);
    if (!dom) return -1.0f;
    const float bnd = k < 2 ? umx + vmx : (k == 2 ? umx * vmx : (k == 3 ? umx / vmn : vmx / umn));
    if (!(bnd <= kCapSafe)) {
        // exact per-sample magnitude check (rare)
        for (int t = 0; t < n; ++t) {
            const float x = cu[t], y = cv[t];
            const float f = k == 0 ? x + y : k == 1 ? x - y : k == 2 ? x * y
                          : k == 3 ? x * __builtin_amdgcn_rcpf(y) : y * __builtin_amdgcn_rcpf(x);
            if (!(fabsf(f) <= 1e15f)) return -1.0f;
        }
    }
    float sc = score_from_sums((double)fA, dB, dC, shift, nd, R1, Srr);
    if (k < 2 && sc >= 0.0f) {
        // a sum or difference that cancels to rounding noise
        const double var = dB - (double)fA * ((double)fA / nd);
        const double scale = fmax((double)urm, (double)vrm);
        if (!(sqrt(fmax(var, 0.0) / nd) > kCancelRel * scale)) sc = -1.0f;
    }
    return sc;
}

// Score of one stored pool column against the residual (one wave; every lane
// returns the score, -1 if the column is invalid).  Lane l accumulates the
// samples l*4 + 256 j in FP32; the wave sum is taken in FP64.  The single-
// problem and batched screening kernels use this same sequence of operations.
// WT: A and B are weighted by the sample weights w32 (Sec. 2.4 whitening with
// a diagonal covariance; the residual of such a pass carries its weights).
template <bool WT>
__device__ inline float score_stored_column_t(const float *col, const float *r32, const float *w32, int n,
                                              float mean, bool valid, double nd, double R1, double Srr)
{
    const int lane = threadIdx.x & 63;
    float a0 = 0.f, b0 = 0.f, c0 = 0.f;
    for (int t = lane * 4; t < n; t += 256) {
        const float4 fv = *reinterpret_cast<const float4 *>(col + t);
        const float4 rv = *reinterpret_cast<const float4 *>(r32 + t);
        float4 wv = make_float4(1.f, 1.f, 1.f, 1.f);
        if (WT) wv = *reinterpret_cast<const float4 *>(w32 + t);
        const float fa[4] = {fv.x, fv.y, fv.z, fv.w};
        const float ra[4] = {rv.x, rv.y, rv.z, rv.w};
        const float wa[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (t + e < n) {
                const float g = fa[e] - mean;
                const float wg = WT ? wa[e] * g : g;
                a0 += wg;
                b0 = fmaf(wg, g, b0);
                c0 = fmaf(g, ra[e], c0);
            }
    }
    const double A = wave_sum_dpp((double)a0), B = wave_sum_dpp((double)b0), C = wave_sum_dpp((double)c0);
    return valid ? score_from_sums(A, B, C, (double)mean, nd, R1, Srr) : -1.0f;
}

__device__ inline float score_stored_column(const float *col, const float *r32, int n, float mean, bool valid,
                                            double nd, double R1, double Srr)
{
    return score_stored_column_t<false>(col, r32, nullptr, n, mean, valid, nd, R1, Srr);
}

int score_lists_capacity(const sisso_space *s, const sisso_score_args *a);

// Header bookkeeping of one screening call writing lists_this_call lists from
// slot `base` on: base 0 starts a pass (reset), base > 0 appends.
bool ws_begin_call(void *ws, int keep, int base, int lists_this_call, int lists_cap, hipStream_t st);
sisso_status topk_launch(void *ws, int k, int64_t *out_ids, float *out_scores, int32_t *out_count,
                         hipStream_t st, bool allow_above_keep);

}  // namespace sisso
