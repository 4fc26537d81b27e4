// common.hpp -- shared helpers of the SISSO HIP library (gfx950).
//
// Canonical numbering decode (host and device), operator application in
// FP64 and FP32, wave reductions, and the per-block top-K' list kept in LDS
// by the screening kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sisso.h"

#define SISSO_HD __host__ __device__ __forceinline__

namespace sisso {

constexpr double kValueCap = 1e15;     // |f| above this makes a feature invalid
constexpr double kConstRel = 1e-6;     // sd <= kConstRel |mean| -> near-constant
constexpr double kCancelRel = 1e-5;    // a +/- b with sd <= kCancelRel max rms -> cancels
constexpr double kDupTol = 1e-9;       // 1 - |corr| <= kDupTol -> duplicates
constexpr double kTieRel = 1e-12;      // SO tie band, relative to S_yy
// A candidate whose magnitude bound (from operand max/min |f|) stays below
// this needs no per-sample cap check.
constexpr float kCapSafe = 0.999e15f;

// ------------------------------------------------------------ numbering

SISSO_HD int64_t choose2(int64_t j) { return j * (j - 1) / 2; }

// Unordered pair (i < j) with index Q = C(j, 2) + i.
SISSO_HD void pair_from_index(int64_t Q, int64_t *j, int64_t *i)
{
    double x = 0.5 * (1.0 + sqrt(1.0 + 8.0 * (double)Q));
    int64_t jj = (int64_t)x;
    while (jj > 1 && choose2(jj) > Q) --jj;
    while (choose2(jj + 1) <= Q) ++jj;
    *j = jj;
    *i = Q - choose2(jj);
}

// Decode a canonical id into (op, left, right); op = -1 for base features.
SISSO_HD int decode_id(const sisso_space &s, int64_t id, int *op, int64_t *l, int64_t *r)
{
    if (id < 0 || id >= s.total) return -1;
    if (id < s.d) { *op = -1; *l = -1; *r = -1; return 0; }
    const int L = s.levels;
    if (id < s.pool[L]) {
        int lev = 1;
        while (id >= s.pool[lev]) ++lev;
        const int64_t lo = lev >= 2 ? s.pool[lev - 2] : 0, hi = s.pool[lev - 1];
        int64_t loc = id - hi;
        const int64_t nu = (int64_t)s.n_unary * (hi - lo);
        if (loc < nu) {
            *op = s.unary[loc % s.n_unary];
            *l = lo + loc / s.n_unary;
            *r = -1;
            return 0;
        }
        loc -= nu;
        const int64_t pair = loc / s.n_slots;
        const int slot = (int)(loc % s.n_slots);
        int64_t j, i;
        pair_from_index(pair + choose2(lo), &j, &i);
        *op = s.slot_op[slot];
        if (s.slot_rev[slot]) { *l = i; *r = j; } else { *l = j; *r = i; }
        return 0;
    }
    const int64_t lo = s.pool[L - 1];
    int64_t loc = id - s.pool[L];
    if (loc < s.rect_unary) {
        *op = s.unary[loc % s.n_unary];
        *l = lo + loc / s.n_unary;
        *r = -1;
        return 0;
    }
    loc -= s.rect_unary;
    const int64_t pair = loc / s.n_slots;
    const int slot = (int)(loc % s.n_slots);
    int64_t u, v;
    if (s.rect == 1) {
        u = lo + pair / lo; v = pair % lo;            // v in P_{L-1}
    } else {
        pair_from_index(pair + choose2(lo), &u, &v);  // the next TRI level: v < u
    }
    *op = s.slot_op[slot];
    if (s.slot_rev[slot]) { *l = v; *r = u; } else { *l = u; *r = v; }
    return 0;
}

// ------------------------------------------------------------ operators

SISSO_HD bool is_binary(int op) { return op >= SISSO_ADD && op <= SISSO_DIV; }

// FP64 operator; sets ok = false on a domain violation.
__device__ __forceinline__ double apply64(int op, double a, double b, bool &ok)
{
    switch (op) {
    case SISSO_ADD: return a + b;
    case SISSO_SUB: return a - b;
    case SISSO_MUL: return a * b;
    case SISSO_DIV: if (b == 0.0) ok = false; return a / b;
    case SISSO_SQ: return a * a;
    case SISSO_CUBE: return a * a * a;
    case SISSO_SQRT: if (a < 0.0) ok = false; return sqrt(a);
    case SISSO_INV: if (a == 0.0) ok = false; return 1.0 / a;
    case SISSO_EXP: return exp(a);
    case SISSO_NEXP: return exp(-a);
    case SISSO_LOG: if (a <= 0.0) ok = false; return log(a);
    case SISSO_SIN: return sin(a);
    default: ok = false; return 0.0;
    }
}

// FP32 unary operator as the screening kernels evaluate it.
__device__ __forceinline__ float unary32(int op, float a)
{
    switch (op) {
    case SISSO_SQ: return a * a;
    case SISSO_CUBE: return a * a * a;
    case SISSO_SQRT: return __builtin_amdgcn_sqrtf(a);
    case SISSO_INV: return __builtin_amdgcn_rcpf(a);
    case SISSO_EXP: return expf(a);
    case SISSO_NEXP: return expf(-a);
    case SISSO_LOG: return logf(a);
    case SISSO_SIN: return sinf(a);
    default: return 0.0f;
    }
}

// ----------------------------------------------------------------- units

// One column's units (SISSO_UNIT_DIMS int16 exponents times SISSO_UNIT_SCALE)
// as one 16-byte word; kUnitNone as the first exponent marks a feature that
// breaks dimensional analysis.
static_assert(SISSO_UNIT_DIMS * sizeof(int16_t) == sizeof(uint4), "units of a column are one 16-byte word");
constexpr int kUnitNone = -32768;
__device__ __forceinline__ uint4 unit_of(const int16_t *units, int64_t c)
{
    return reinterpret_cast<const uint4 *>(units)[c];
}
__device__ __forceinline__ bool unit_eq(uint4 a, uint4 b)   // branch-free
{
    return ((a.x ^ b.x) | (a.y ^ b.y) | (a.z ^ b.z) | (a.w ^ b.w)) == 0u;
}
__device__ __forceinline__ bool unit_dimless(uint4 a) { return (a.x | a.y | a.z | a.w) == 0u; }
// exp, exp(-x), ln and sin take a dimensionless argument
__device__ __forceinline__ bool unary_needs_dimless(int op)
{
    return op == SISSO_EXP || op == SISSO_NEXP || op == SISSO_LOG || op == SISSO_SIN;
}

// Domain check and magnitude bound of a unary op applied to a column with
// the given statistics.  Returns false if the domain is violated; *bound
// receives an upper bound of |op(f)| (or +inf when no cheap bound exists).
__device__ __forceinline__ bool unary_domain_bound(int op, const sisso_colstat &st, float *bound)
{
    const float mx = st.maxabs, mn = st.minabs;
    switch (op) {
    case SISSO_SQ: *bound = mx * mx; return true;
    case SISSO_CUBE: *bound = mx * mx * mx; return true;
    case SISSO_SQRT: *bound = sqrtf(mx); return st.minval >= 0.0f;
    case SISSO_INV: *bound = mn > 0.0f ? 1.0f / mn : INFINITY; return mn > 0.0f;
    case SISSO_EXP: *bound = expf(mx); return true;
    case SISSO_NEXP: *bound = expf(mx); return true;
    case SISSO_LOG: *bound = fmaxf(fabsf(logf(fmaxf(mn, 1e-38f))), fabsf(logf(mx))); return st.minval > 0.0f;
    case SISSO_SIN: *bound = 1.0f; return true;
    default: *bound = INFINITY; return false;
    }
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_or(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// Wave reductions through DPP lane moves (no LDS crossbar): quad
// permutations, half-row and row mirrors, then the row broadcasts of lanes 15
// and 31, after which lane 63 holds the result, read back as a wave-uniform
// value.  All 64 lanes must be active; the order of the additions is fixed, so
// the result is deterministic (it may differ from wave_sum in the last bits).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move(int v)
{
    // rows outside ROWS receive 0
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v)
{
    int2 h;
    __builtin_memcpy(&h, &v, 8);
    h.x = dpp_move<CTRL, ROWS>(h.x);
    h.y = dpp_move<CTRL, ROWS>(h.y);
    double r;
    __builtin_memcpy(&r, &h, 8);
    return r;
}
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_move<0xB1, 0xF>(v);     // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E, 0xF>(v);     // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141, 0xF>(v);    // row_half_mirror: sums of 8 lanes
    v += dpp_move<0x140, 0xF>(v);    // row_mirror: sums of 16-lane rows
    v += dpp_move<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    int2 h;
    __builtin_memcpy(&h, &v, 8);
    h.x = __builtin_amdgcn_readlane(h.x, 63);
    h.y = __builtin_amdgcn_readlane(h.y, 63);
    double r;
    __builtin_memcpy(&r, &h, 8);
    return r;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(dpp_move<CTRL, ROWS>(__float_as_int(v)));
}
// rows outside a broadcast's ROWS take 0, which never reaches lane 63
__device__ __forceinline__ float wave_max_dpp(float v)
{
    v = fmaxf(v, dpp_move<0xB1, 0xF>(v));
    v = fmaxf(v, dpp_move<0x4E, 0xF>(v));
    v = fmaxf(v, dpp_move<0x141, 0xF>(v));
    v = fmaxf(v, dpp_move<0x140, 0xF>(v));
    v = fmaxf(v, dpp_move<0x142, 0xA>(v));
    v = fmaxf(v, dpp_move<0x143, 0xC>(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_min_dpp(float v)
{
    v = fminf(v, dpp_move<0xB1, 0xF>(v));
    v = fminf(v, dpp_move<0x4E, 0xF>(v));
    v = fminf(v, dpp_move<0x141, 0xF>(v));
    v = fminf(v, dpp_move<0x140, 0xF>(v));
    v = fminf(v, dpp_move<0x142, 0xA>(v));
    v = fminf(v, dpp_move<0x143, 0xC>(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ int wave_or_dpp(int v)
{
    v |= dpp_move<0xB1, 0xF>(v);
    v |= dpp_move<0x4E, 0xF>(v);
    v |= dpp_move<0x141, 0xF>(v);
    v |= dpp_move<0x140, 0xF>(v);
    v |= dpp_move<0x142, 0xA>(v);
    v |= dpp_move<0x143, 0xC>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

// Block-wide sum of one double per thread; result broadcast to all threads.
// `red` must hold blockDim.x / 64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// ------------------------------------------------------- ordering of keys

// (score desc, id asc): true if a ranks before b.
SISSO_HD bool ranks_before(float sa, int64_t ia, float sb, int64_t ib)
{
    return sa > sb || (sa == sb && ia < ib);
}

// Bitonic sort of `cap` (power of two) keys in LDS into rank order.
__device__ inline void bitonic_sort_keys(float *sc, int64_t *id, int cap)
{
    for (int size = 2; size <= cap; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (cap >> 1); t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const bool j_first = ranks_before(sc[j], id[j], sc[i], id[i]);
                if (j_first == up) {
                    float ts = sc[i]; sc[i] = sc[j]; sc[j] = ts;
                    int64_t ti = id[i]; id[i] = id[j]; id[j] = ti;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ bool in_sorted_ids(const int64_t *arr, int n, int64_t key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (arr[m] < key) lo = m + 1; else hi = m;
    }
    return lo < n && arr[lo] == key;
}

// ---------------------------------------------------- per-block top-K' list
//
// The list holds up to `cap` entries (cap a power of two, >= keep +
// blockDim).  Entries [0, cnt) are live.  `thr` is the block's admission
// threshold: the keep-th best score once the list has been merged full.
// Together with the grid-wide bound `gthr` (atomic max over the blocks'
// thresholds, a true lower bound of the global keep-th score) it rejects
// candidates that cannot be in the global top-K'.  Equal scores are
// admitted, so ties are resolved by id at the merges.

struct BlockList {
    float *sc;
    int64_t *id;
    int *cnt;
    float *thr;
    int cap, keep;
};

__device__ __forceinline__ float load_gthr(const unsigned *g)
{
    return __uint_as_float(__hip_atomic_load(g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ inline void list_init(BlockList &L)
{
    if (threadIdx.x == 0) { *L.cnt = 0; *L.thr = 0.0f; }
    __syncthreads();
}

// Sort, truncate to keep and raise the thresholds.  Block-uniform call.
__device__ inline void list_merge(BlockList &L, unsigned *gthr)
{
    const int c = *L.cnt;
    for (int i = threadIdx.x; i < L.cap; i += blockDim.x)
        if (i >= c) { L.sc[i] = -1.0f; L.id[i] = INT64_MAX; }
    __syncthreads();
    bitonic_sort_keys(L.sc, L.id, L.cap);
    if (threadIdx.x == 0) {
        const int nc = c < L.keep ? c : L.keep;
        *L.cnt = nc;
        if (nc == L.keep) {
            *L.thr = L.sc[L.keep - 1];
            atomicMax(gthr, __float_as_uint(L.sc[L.keep - 1]));
        }
    }
    __syncthreads();
}

// Every thread offers NC candidates (score < 0 = none).  Block-uniform call.
template <int NC>
__device__ inline void list_offer(BlockList &L, const float (&sc)[NC], const int64_t (&id)[NC],
                                  unsigned *gthr, const int64_t *excl, int n_excl)
{
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        __syncthreads();
        const int c = *L.cnt;
        __syncthreads();
        if (c + (int)blockDim.x > L.cap) list_merge(L, gthr);
        const float t = fmaxf(*L.thr, load_gthr(gthr));
        if (sc[q] >= 0.0f && sc[q] >= t) {
            if (n_excl == 0 || !in_sorted_ids(excl, n_excl, id[q])) {
                const int slot = atomicAdd(L.cnt, 1);
                L.sc[slot] = sc[q];
                L.id[slot] = id[q];
            }
        }
    }
}

// Final merge and write of the block's list to its workspace slot.
__device__ inline void list_flush(BlockList &L, unsigned *gthr, float *out_sc, int64_t *out_id)
{
    __syncthreads();
    list_merge(L, gthr);
    const int c = *L.cnt;
    for (int i = threadIdx.x; i < L.keep; i += blockDim.x) {
        out_sc[i] = i < c ? L.sc[i] : -1.0f;
        out_id[i] = i < c ? L.id[i] : INT64_MAX;
    }
}

// Allow a kernel more than the default 64 KB of dynamic LDS (gfx950 has 160 KB).
template <typename K>
inline bool allow_dynamic_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return true;
    if (bytes > 160 * 1024) return false;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

SISSO_HD int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace sisso
