// score.hip -- SIS screening: |Pearson correlation| of every candidate with
// the residual and a deterministic grid-wide top-K' (Sec. 2.2, eq. sis-weight
// and eq. sis-method).
//
// Per candidate f and centred FP32 residual r the kernels accumulate, with a
// per-candidate shift c (the candidate's value at sample 0),
//     A = sum (f - c),   B = sum (f - c)^2,   C = sum (f - c) r
// and score = |C - A R1/n| / sqrt((B - A^2/n) S_rr), where R1 = sum r and
// S_rr = sum (r - R1/n)^2 come from sisso_prepare_residual.  Partial sums run
// in FP32 over short sample chunks and are carried in FP64.
//
// Two kernels cover the space:
//   k_score_columns  stored pool columns (one wave per column; bound by the
//                    VALU work of the unary children),
//                    plus the one-sided slice's unary block on the newest
//                    pool level, evaluated while the column streams by;
//   k_score_rect     the slice's binary block op(u, v): a block owns a tile of
//                    newest-level operands u and sweeps every v tile of the
//                    previous pool, staging sample chunks of both through LDS
//                    and evaluating all binary slots in registers.  Slice
//                    candidates are never written to memory.
// Every block keeps its best K' candidates (score desc, id asc) in LDS and
// writes them to its list slot of the workspace; sisso_topk merges the lists.
#include "tiles.hpp"

namespace sisso {

__global__ void k_ws_reset(WsHeader *h, int keep, int n_lists, int lists_cap)
{
    if (threadIdx.x == 0) {
        h->gthr = 0u;
        h->keep = keep;
        h->n_lists = n_lists;
        h->lists_cap = lists_cap;
        h->status = 0;
        h->scr_status = 0;
    }
}

__global__ void k_ws_append(WsHeader *h, int n_lists)
{
    if (threadIdx.x == 0) h->n_lists = n_lists;
}

// ------------------------------------------------------ pool columns kernel

template <int NU, bool WT>
__global__ void __launch_bounds__(256, 3) k_score_columns(
    sisso_space s, int n, const float *__restrict__ pool32, int64_t ld32,
    const sisso_colstat *__restrict__ stats, const float *__restrict__ r32,
    const sisso_resid_info *__restrict__ info, const int64_t *__restrict__ excl, int n_excl,
    int64_t c_lo, int64_t c_hi, int64_t id_begin, int64_t id_end, int list_base, void *ws,
    int lists_total, int keep, int cap, const float *__restrict__ w32, const int16_t *__restrict__ units)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    WsView W = ws_view(ws, lists_total, keep);
    float *lsc = (float *)smem;
    int64_t *lid = (int64_t *)(smem + cap * sizeof(float));
    __shared__ int lcnt;
    __shared__ float lthr;
    constexpr int PER = 1 + NU;
    __shared__ float st_sc[kColWaves * kColBatch * PER];
    __shared__ int64_t st_id[kColWaves * kColBatch * PER];
    BlockList L{lsc, lid, &lcnt, &lthr, cap, keep};
    list_init(L);

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int Lv = s.levels;
    const int64_t newlo = s.pool[Lv - 1], pL = s.pool[Lv];
    const bool rect = s.rect != 0;
    const int nu = rect ? s.n_unary : 0;
    int uop[NU > 0 ? NU : 1];
#pragma unroll
    for (int o = 0; o < (NU > 0 ? NU : 1); ++o) uop[o] = (o < nu) ? s.unary[o] : 0;
    const double nd = (double)n, R1 = info->sum_r32, Srr = info->s_rr;
    const int per_batch = kColWaves * kColBatch;
    const int64_t ncols = c_hi - c_lo;
    constexpr int NC = (kColWaves * kColBatch * PER + 255) / 256;

    // n <= 256 kColRegs: the residual stays in registers and each column is
    // loaded whole before it is scored (three waves per SIMD overlap one
    // wave's loads with the others' arithmetic)
    const bool regs = n <= 256 * kColRegs;
    float4 rv[kColRegs], wv[kColRegs], cur[kColRegs];
    auto load_col = [&](int64_t c, float4 (&dst)[kColRegs]) {
        const float *col = pool32 + (size_t)c * ld32;
#pragma unroll
        for (int k = 0; k < kColRegs; ++k) {
            const int t = lane * 4 + 256 * k;
            dst[k] = t < n ? *reinterpret_cast<const float4 *>(col + t) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (regs) {
#pragma unroll
        for (int k = 0; k < kColRegs; ++k) {
            const int t = lane * 4 + 256 * k;
            rv[k] = t < n ? *reinterpret_cast<const float4 *>(r32 + t) : make_float4(0.f, 0.f, 0.f, 0.f);
            wv[k] = make_float4(1.f, 1.f, 1.f, 1.f);
            if (WT && t < n) wv[k] = *reinterpret_cast<const float4 *>(w32 + t);
        }
    }

    for (int64_t b0 = (int64_t)blockIdx.x * per_batch; b0 < ncols; b0 += (int64_t)gridDim.x * per_batch) {
        const int64_t cw = c_lo + b0 + w * kColBatch;     // this wave's first column
        for (int j = 0; j < kColBatch; ++j) {
            const int slot_base = (w * kColBatch + j) * PER;
            const int64_t c = cw + j;
            float scs[PER];
#pragma unroll
            for (int o = 0; o < PER; ++o) scs[o] = -1.0f;
            if (regs && c < c_hi) load_col(c, cur);
            if (c < c_hi) {
                const sisso_colstat st = stats[c];
                if (regs)
                    score_column_regs<NU, kColRegs, WT>(cur, rv, wv, st, n, nd, R1, Srr, uop, nu,
                                                        NU > 0 && rect && c >= newlo, scs);
                else
                    score_column<NU, WT>(pool32 + (size_t)c * ld32, st, r32, n, nd, R1, Srr, uop, nu,
                                         NU > 0 && rect && c >= newlo, scs, w32);
                if (!(c >= id_begin && c < id_end)) scs[0] = -1.0f;
                // dimensional analysis: exp, exp(-x), ln, sin of a dimensionless column only
                const bool dimless = !units || unit_dimless(unit_of(units, c));
#pragma unroll
                for (int o = 0; o < NU; ++o) {
                    const int64_t uid = pL + (c - newlo) * nu + o;
                    if (!(uid >= id_begin && uid < id_end) || (!dimless && o < nu && unary_needs_dimless(uop[o])))
                        scs[1 + o] = -1.0f;
                }
            }
            if (lane == 0) {
#pragma unroll
                for (int o = 0; o < PER; ++o) {
                    st_sc[slot_base + o] = scs[o];
                    st_id[slot_base + o] = o == 0 ? c : pL + (c - newlo) * nu + (o - 1);
                }
            }
        }
        __syncthreads();
        float osc[NC];
        int64_t oid[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int e = threadIdx.x + q * 256;
            osc[q] = e < kColWaves * kColBatch * PER ? st_sc[e] : -1.0f;
            oid[q] = e < kColWaves * kColBatch * PER ? st_id[e] : INT64_MAX;
        }
        list_offer<NC>(L, osc, oid, &W.h->gthr, excl, n_excl);
        __syncthreads();
    }
    const int list = list_base + blockIdx.x;
    list_flush(L, &W.h->gthr, W.sc + (size_t)list * keep, W.id + (size_t)list * keep);
}

// --------------------------------------------------------- binary slice

template <int RU, int RV, bool WT>
__global__ void __launch_bounds__(256) k_score_rect(
    sisso_space s, FormSlots fs, int n, const float *__restrict__ pool32, int64_t ld32,
    const sisso_colstat *__restrict__ stats, const float *__restrict__ r32,
    const sisso_resid_info *__restrict__ info, const int64_t *__restrict__ excl, int n_excl,
    int64_t ut_lo, int64_t ut_hi, int64_t id_begin, int64_t id_end, int list_base, void *ws,
    int lists_total, int keep, int cap, const float *__restrict__ w32, const int16_t *__restrict__ units)
{
    using Cfg = RectCfg<RU, RV>;
    constexpr int TU = Cfg::TU, TV = Cfg::TV;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *buf0 = (float *)smem;
    float *buf1 = buf0 + Cfg::BUF;
    float *lsc = buf1 + Cfg::BUF;
    int64_t *lid = (int64_t *)(lsc + cap);
    __shared__ int lcnt;
    __shared__ float lthr;
    WsView W = ws_view(ws, lists_total, keep);
    BlockList L{lsc, lid, &lcnt, &lthr, cap, keep};
    list_init(L);

    // one-sided slice (rect 1): v in P_{L-1}; whole next TRI level (rect 2):
    // v < u over P_L, the u tile's v range ending at its last u
    const int Lv = s.levels;
    const bool tri = s.rect == 2;
    const int64_t ulo = s.pool[Lv - 1], uhi = s.pool[Lv];
    const int64_t vcount = tri ? uhi : ulo;
    const PairIds ids{s.pool[Lv] + s.rect_unary, ulo, ulo, s.n_slots, tri};
    const double nd = (double)n, R1 = info->sum_r32, Srr = info->s_rr;

    for (int64_t ut = ut_lo + blockIdx.x; ut < ut_hi; ut += gridDim.x) {
        const int64_t u0 = ulo + ut * TU;
        USide<RU, RV> U;
        load_uside<RU, RV>(U, stats, ids, u0, uhi);
        const int64_t vlim = tri ? (u0 + TU < uhi ? u0 + TU : uhi) : vcount;
        const int64_t nvt = (vlim + TV - 1) / TV;
        for (int64_t vt = 0; vt < nvt; ++vt) {
            float osc[RU * RV * 5];
            int64_t oid[RU * RV * 5];
            score_pair_tile<RU, RV, WT>(pool32, ld32, stats, r32, n, nd, R1, Srr, fs, ids, u0, U, vt * TV,
                                        vcount, id_begin, id_end, buf0, buf1, osc, oid, w32, units);
            list_offer<RU * RV * 5>(L, osc, oid, &W.h->gthr, excl, n_excl);
        }
    }
    const int list = list_base + blockIdx.x;
    list_flush(L, &W.h->gthr, W.sc + (size_t)list * keep, W.id + (size_t)list * keep);
}

// ----------------------------------------------------------------- top-k

__device__ __forceinline__ bool considered(float sc, unsigned g)
{
    return sc >= 0.0f && __float_as_uint(sc) >= g;
}

__global__ void k_tk_init(WsHeader *h, int k)
{
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) h->hist[i] = 0u;
    if (threadIdx.x == 0) {
        h->prefix = 0u; h->need = k; h->total = 0; h->n_gt = 0; h->n_eq = 0; h->status = 0;
    }
}

// pass 0: bits [31:20]; pass 1: bits [19:8] under prefix; pass 2: bits [7:0].
__global__ void __launch_bounds__(256) k_tk_hist(void *ws, int pass)
{
    __shared__ unsigned hist[kHistBins];
    WsView W = ws_view_dev(ws);
    const int keep = W.h->keep;
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const unsigned g = W.h->gthr, pre = W.h->prefix;
    const int64_t M = (int64_t)W.h->n_lists * keep;
    unsigned cnt = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M; e += (int64_t)gridDim.x * blockDim.x) {
        const float sc = W.sc[e];
        if (!considered(sc, g)) continue;
        const unsigned u = __float_as_uint(sc);
        unsigned bin;
        if (pass == 0) { bin = u >> 20; cnt++; }
        else if (pass == 1) { if ((u >> 20) != (pre >> 20)) continue; bin = (u >> 8) & 0xFFFu; }
        else { if ((u >> 8) != (pre >> 8)) continue; bin = u & 0xFFu; }
        atomicAdd(&hist[bin], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x)
        if (hist[i]) atomicAdd(&W.h->hist[i], hist[i]);
    if (pass == 0 && cnt) atomicAdd(&W.h->total, (int)cnt);
}

__global__ void k_tk_select(WsHeader *h, int pass)
{
    // the histogram into LDS (coalesced), a single-thread scan from the top
    // bin there; then clear the histogram
    __shared__ unsigned hs[kHistBins];
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) hs[i] = h->hist[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int bins = pass == 2 ? 256 : kHistBins;
        const int shift = pass == 0 ? 20 : (pass == 1 ? 8 : 0);
        int need = h->need;
        if (pass == 0 && h->total <= need) {
            h->need = -1;       // take everything that is considered
        } else if (need > 0) {
            int b = bins - 1;
            for (; b > 0; --b) {
                const int c = (int)hs[b];
                if (c >= need) break;
                need -= c;
            }
            h->prefix |= ((unsigned)b) << shift;
            h->need = need;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) h->hist[i] = 0u;
}

__global__ void __launch_bounds__(256) k_tk_gather(void *ws, int k)
{
    WsView W = ws_view_dev(ws);
    const int keep = W.h->keep;
    const unsigned g = W.h->gthr, sstar = W.h->prefix;
    const bool all = W.h->need < 0;
    // after the select passes exactly k - need entries lie above the cutoff:
    // the front of the buffer holds them, ties may use the slots behind them
    const int front = all ? kFinalCap : k - W.h->need;
    const int64_t M = (int64_t)W.h->n_lists * keep;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M; e += (int64_t)gridDim.x * blockDim.x) {
        const float sc = W.sc[e];
        if (!considered(sc, g)) continue;
        // Entries above the k-th score (k - need < k of them) fill the gather
        // buffer from the front, entries equal to it from the back down to the
        // front's end: only ties at the cutoff can exceed the buffer, and only
        // tied entries are lost then (reported as status 1).
        const unsigned u = __float_as_uint(sc);
        if (all || u > sstar) {
            const int slot = atomicAdd(&W.h->n_gt, 1);
            if (slot < kFinalCap) { W.fin_sc[slot] = sc; W.fin_id[slot] = W.id[e]; }
        } else if (u == sstar) {
            const int slot = kFinalCap - 1 - atomicAdd(&W.h->n_eq, 1);
            if (slot >= front) { W.fin_sc[slot] = sc; W.fin_id[slot] = W.id[e]; }
        }
    }
}

__global__ void __launch_bounds__(1024) k_tk_final(void *ws, int k, int allow_above_keep,
                                                   int64_t *__restrict__ out_ids, float *__restrict__ out_sc,
                                                   int32_t *out_count)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    WsView W = ws_view_dev(ws);
    if (k > kFinalCap || (!allow_above_keep && k > W.h->keep)) {
        // k larger than the list length the workspace was filled with
        for (int i = threadIdx.x; i < k; i += blockDim.x) { out_ids[i] = INT64_MAX; out_sc[i] = -1.0f; }
        if (threadIdx.x == 0) { *out_count = 0; W.h->status = 2; }
        return;
    }
    // front: the entries above the cutoff; back: the ties at it (as many as fit)
    const int m_gt = W.h->n_gt < kFinalCap ? W.h->n_gt : kFinalCap;
    const int room = kFinalCap - m_gt;
    const int m_eq = W.h->n_eq < room ? W.h->n_eq : room;
    const int m = m_gt + m_eq;
    const int cap = next_pow2(m > 1 ? m : 2);
    float *sc = (float *)smem;
    int64_t *id = (int64_t *)(smem + kFinalCap * sizeof(float));
    for (int i = threadIdx.x; i < cap; i += blockDim.x) {
        const int src = i < m_gt ? i : kFinalCap - 1 - (i - m_gt);
        sc[i] = i < m ? W.fin_sc[src] : -1.0f;
        id[i] = i < m ? W.fin_id[src] : INT64_MAX;
    }
    __syncthreads();
    bitonic_sort_keys(sc, id, cap);
    const int take = m < k ? m : k;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        out_ids[i] = i < take ? id[i] : INT64_MAX;
        out_sc[i] = i < take ? sc[i] : -1.0f;
    }
    if (threadIdx.x == 0) {
        *out_count = take;
        if (W.h->n_gt + W.h->n_eq > kFinalCap) W.h->status = 1;
    }
}

}  // namespace sisso

// ------------------------------------------------------------------ C ABI

using namespace sisso;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kColGrid = 2048, kMaxColGrid = 16384;
constexpr int kMaxRectGrid = 1024;

struct Plan {
    int64_t c_lo = 0, c_hi = 0;       // columns for k_score_columns
    int64_t ut_lo = 0, ut_hi = 0;     // u tiles for k_score_rect
    int g_cols = 0, g_rect = 0;
    int ru = 2, rv = 2;
};

int rect_tu(int ru) { return 16 * ru; }

// The stored-column pass has its own launch shape (col_grid); the grid
// argument tunes the binary block's kernels only.
int max_col_grid(const sisso_score_args *a) { return a->col_grid > 0 ? a->col_grid : kColGrid; }
int max_rect_grid(const sisso_score_args *a) { return a->grid > 0 ? a->grid : kMaxRectGrid; }

void tile_shape(const sisso_score_args *a, int *ru, int *rv)
{
    switch (a->tile) {
    case 1: *ru = 2; *rv = 1; break;
    case 2: *ru = 1; *rv = 2; break;
    default: *ru = 2; *rv = 2; break;
    }
}

Plan make_plan(const sisso_space *s, const sisso_score_args *a, int64_t begin, int64_t end)
{
    Plan p;
    tile_shape(a, &p.ru, &p.rv);
    const int L = s->levels;
    const int64_t pL = s->pool[L], newlo = s->pool[L - 1];
    // pool columns in range
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    if (begin < pL) { lo = begin; hi = end < pL ? end : pL; }
    // unary slice ids -> their N_L columns
    if (s->rect && s->n_unary > 0) {
        const int64_t ub = pL, ue = pL + s->rect_unary;
        const int64_t b = begin > ub ? begin : ub, e = end < ue ? end : ue;
        if (b < e) {
            const int64_t cl = newlo + (b - pL) / s->n_unary;
            const int64_t ch = newlo + (e - 1 - pL) / s->n_unary + 1;
            lo = lo < cl ? lo : cl;
            hi = hi > ch ? hi : ch;
        }
    }
    if (lo < hi) {
        p.c_lo = lo; p.c_hi = hi;
        const int64_t batches = (hi - lo + kColWaves * kColBatch - 1) / (kColWaves * kColBatch);
        p.g_cols = (int)(batches < max_col_grid(a) ? batches : max_col_grid(a));
    }
    if (s->rect) {
        const int64_t bb = pL + s->rect_unary, be = s->total;
        const int64_t b = begin > bb ? begin : bb, e = end < be ? end : be;
        if (b < e) {
            int64_t ul, uh;                  // u range (from the first u of N_L) of the ids
            if (s->rect == 1) {
                const int64_t per_u = newlo * s->n_slots;
                ul = (b - bb) / per_u;
                uh = (e - 1 - bb) / per_u + 1;
            } else {
                int64_t jb, je, ib, ie;
                pair_from_index((b - bb) / s->n_slots + choose2(newlo), &jb, &ib);
                pair_from_index((e - 1 - bb) / s->n_slots + choose2(newlo), &je, &ie);
                ul = jb - newlo;
                uh = je - newlo + 1;
            }
            const int tu = rect_tu(p.ru);
            p.ut_lo = ul / tu;
            p.ut_hi = (uh + tu - 1) / tu;
            const int64_t tiles = p.ut_hi - p.ut_lo;
            p.g_rect = (int)(tiles < max_rect_grid(a) ? tiles : max_rect_grid(a));
        }
    }
    return p;
}

int lists_capacity(const sisso_space *s, const sisso_score_args *a)
{
    const Plan p = make_plan(s, a, 0, s->total);
    // the binary block's lists come from k_score_rect, or from the exact rescore
    // of a BF16 band (at most kFinalCap / 256 lists)
    return p.g_cols + (p.g_rect > kFinalCap / 256 ? p.g_rect : kFinalCap / 256);
}

int list_cap(int keep) { return next_pow2(keep + 256); }

size_t rect_smem(int ru, int rv, int cap)
{
    int buf = 0;
    if (ru == 2 && rv == 2) buf = RectCfg<2, 2>::BUF;
    else if (ru == 2 && rv == 1) buf = RectCfg<2, 1>::BUF;
    else buf = RectCfg<1, 2>::BUF;
    return (size_t)2 * buf * sizeof(float) + (size_t)cap * (sizeof(float) + sizeof(int64_t));
}

}  // namespace

namespace sisso {
int score_lists_capacity(const sisso_space *s, const sisso_score_args *a) { return lists_capacity(s, a); }

bool ws_begin_call(void *ws, int keep, int base, int lists_this_call, int lists_cap, hipStream_t st)
{
    if (base == 0)
        hipLaunchKernelGGL(k_ws_reset, dim3(1), dim3(64), 0, st, (WsHeader *)ws, keep, lists_this_call, lists_cap);
    else
        hipLaunchKernelGGL(k_ws_append, dim3(1), dim3(64), 0, st, (WsHeader *)ws, base + lists_this_call);
    return hipGetLastError() == hipSuccess;
}
}  // namespace sisso

extern "C" size_t sisso_score_workspace_size(const sisso_space *space, const sisso_score_args *args)
{
    if (!space || !args || args->keep < 1 || args->keep > SISSO_MAX_KEEP || space->total <= 0 ||
        args->col_grid < 0 || args->col_grid > kMaxColGrid)
        return 0;
    return ws_bytes_for(lists_capacity(space, args), args->keep);
}

extern "C" int32_t sisso_expand_score_lists(const sisso_space *space, const sisso_score_args *args,
                                            int64_t cand_begin, int64_t cand_end)
{
    if (!space || !args || space->total <= 0 || cand_begin < 0 || cand_end > space->total ||
        cand_begin >= cand_end || args->tile < 0 || args->tile > 2 || args->grid < 0 ||
        args->col_grid < 0 || args->col_grid > kMaxColGrid)
        return -1;
    const Plan p = make_plan(space, args, cand_begin, cand_end);
    return p.g_cols + p.g_rect;
}

extern "C" sisso_status sisso_score_reset(void *ws, size_t ws_bytes, void *stream)
{
    if (!ws) return SISSO_E_NULL;
    if (ws_bytes < sizeof(WsHeader)) return SISSO_E_WORKSPACE;
    hipLaunchKernelGGL(k_ws_reset, dim3(1), dim3(64), 0, as_stream(stream), (WsHeader *)ws, 1, 0, 0);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_expand_score(const sisso_space *space, const sisso_score_args *args,
                                           int64_t cand_begin, int64_t cand_end, void *ws,
                                           size_t ws_bytes, void *stream)
{
    if (!space || !args || !ws || !args->pool32 || !args->stats || !args->r32 || !args->info)
        return SISSO_E_NULL;
    if (args->n_exclude > 0 && !args->exclude) return SISSO_E_NULL;
    if (space->total <= 0 || space->levels < 1 || space->levels > SISSO_MAX_LEVELS) return SISSO_E_SHAPE;
    if (args->n < 2 || args->n > SISSO_MAX_N || args->ld32 < args->n || (args->ld32 % 4) != 0 ||
        args->n_exclude < 0)
        return SISSO_E_SHAPE;
    if (args->keep < 1 || args->keep > SISSO_MAX_KEEP) return SISSO_E_RANGE;
    if (cand_begin < 0 || cand_end > space->total || cand_begin >= cand_end) return SISSO_E_RANGE;
    if (args->precision != SISSO_FP32) return SISSO_E_UNSUPPORTED;
    if (args->tile < 0 || args->tile > 2 || args->grid < 0 || args->col_grid < 0 || args->col_grid > kMaxColGrid)
        return SISSO_E_RANGE;
    const int lists = lists_capacity(space, args);
    if (ws_bytes < ws_bytes_for(lists, args->keep)) return SISSO_E_WORKSPACE;
    if (space->rect && space->pool[space->levels - 1] < 1) return SISSO_E_SHAPE;

    const Plan p = make_plan(space, args, cand_begin, cand_end);
    if (args->list_base < 0 || args->list_base + p.g_cols + p.g_rect > lists) return SISSO_E_WORKSPACE;
    const bool weighted = args->w32 != nullptr;
    hipStream_t st = as_stream(stream);
    const int keep = args->keep, cap = list_cap(keep);
    const int base = args->list_base;
    if (base == 0)
        hipLaunchKernelGGL(k_ws_reset, dim3(1), dim3(64), 0, st, (WsHeader *)ws, keep, p.g_cols + p.g_rect, lists);
    else
        hipLaunchKernelGGL(k_ws_append, dim3(1), dim3(64), 0, st, (WsHeader *)ws, base + p.g_cols + p.g_rect);
    if (hipGetLastError() != hipSuccess) return SISSO_E_DEVICE;
    const size_t lsmem = (size_t)cap * (sizeof(float) + sizeof(int64_t));
    if (p.g_cols > 0) {
        const int nu = space->rect ? space->n_unary : 0;
        auto launch_cols = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(p.g_cols), dim3(256), lsmem, st, *space, args->n, args->pool32, args->ld32,
                               args->stats, args->r32, args->info, args->exclude, args->n_exclude, p.c_lo, p.c_hi,
                               cand_begin, cand_end, base, ws, lists, keep, cap, args->w32, args->units);
        };
        if (!weighted) {
            if (nu == 0) launch_cols(k_score_columns<0, false>);
            else if (nu <= 3) launch_cols(k_score_columns<3, false>);
            else launch_cols(k_score_columns<8, false>);
        } else {
            if (nu == 0) launch_cols(k_score_columns<0, true>);
            else if (nu <= 3) launch_cols(k_score_columns<3, true>);
            else launch_cols(k_score_columns<8, true>);
        }
        if (hipGetLastError() != hipSuccess) return SISSO_E_DEVICE;
    }
    if (p.g_rect > 0) {
        const FormSlots fs = form_slots(space);
        const size_t smem = rect_smem(p.ru, p.rv, cap);
        auto launch = [&](auto kern) -> sisso_status {
            if (!allow_dynamic_lds(kern, smem)) return SISSO_E_UNSUPPORTED;
            hipLaunchKernelGGL(kern, dim3(p.g_rect), dim3(256), smem, st, *space, fs, args->n, args->pool32,
                               args->ld32, args->stats, args->r32, args->info, args->exclude, args->n_exclude,
                               p.ut_lo, p.ut_hi, cand_begin, cand_end, base + p.g_cols, ws, lists, keep, cap,
                               args->w32, args->units);
            return SISSO_OK;
        };
        sisso_status rs;
        if (!weighted) {
            if (p.ru == 2 && p.rv == 2) rs = launch(k_score_rect<2, 2, false>);
            else if (p.ru == 2 && p.rv == 1) rs = launch(k_score_rect<2, 1, false>);
            else rs = launch(k_score_rect<1, 2, false>);
        } else {
            if (p.ru == 2 && p.rv == 2) rs = launch(k_score_rect<2, 2, true>);
            else if (p.ru == 2 && p.rv == 1) rs = launch(k_score_rect<2, 1, true>);
            else rs = launch(k_score_rect<1, 2, true>);
        }
        if (rs != SISSO_OK) return rs;
        if (hipGetLastError() != hipSuccess) return SISSO_E_DEVICE;
    }
    return SISSO_OK;
}

namespace sisso {
// Top-k merge of a screening workspace.  With allow_above_keep, k may exceed the
// per-block list length (up to the gather buffer): the result is then the best k
// of the union of the lists, which is what a screening band needs.
sisso_status topk_launch(void *ws, int k, int64_t *out_ids, float *out_scores, int32_t *out_count,
                         hipStream_t st, bool allow_above_keep)
{
    WsHeader *h = (WsHeader *)ws;
    hipLaunchKernelGGL(k_tk_init, dim3(1), dim3(256), 0, st, h, k);
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_tk_hist, dim3(512), dim3(256), 0, st, ws, pass);
        hipLaunchKernelGGL(k_tk_select, dim3(1), dim3(256), 0, st, h, pass);
    }
    hipLaunchKernelGGL(k_tk_gather, dim3(512), dim3(256), 0, st, ws, k);
    const size_t smem = (size_t)kFinalCap * (sizeof(float) + sizeof(int64_t));
    if (!allow_dynamic_lds(k_tk_final, smem)) return SISSO_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_tk_final, dim3(1), dim3(1024), smem, st, ws, k, allow_above_keep ? 1 : 0, out_ids,
                       out_scores, out_count);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
}  // namespace sisso

extern "C" sisso_status sisso_topk(const void *ws_c, size_t ws_bytes, int32_t k, int64_t *out_ids,
                                   float *out_scores, int32_t *out_count, void *stream)
{
    void *ws = const_cast<void *>(ws_c);
    if (!ws || !out_ids || !out_scores || !out_count) return SISSO_E_NULL;
    if (k < 1 || k > SISSO_MAX_KEEP) return SISSO_E_RANGE;
    if (ws_bytes < ws_bytes_for(0, 1)) return SISSO_E_WORKSPACE;
    return topk_launch(ws, k, out_ids, out_scores, out_count, as_stream(stream), false);
}

namespace sisso {
// Threshold selection (Sec. 2.2's alternative to a fixed k): count the list
// entries at or above tau, then keep that prefix of the merged list.
__global__ void k_thr_reset(WsHeader *h)
{
    if (threadIdx.x == 0) h->thr_count = 0;
}

__global__ void __launch_bounds__(256) k_thr_count(void *ws, float tau)
{
    WsView W = ws_view_dev(ws);
    const int64_t M = (int64_t)W.h->n_lists * W.h->keep;
    int c = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M; e += (int64_t)gridDim.x * blockDim.x) {
        const float sc = W.sc[e];
        c += (sc >= 0.0f && sc >= tau) ? 1 : 0;
    }
    c = (int)wave_sum_dpp((double)c);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&W.h->thr_count, c);
}

// *out_count = the merged entries at or above tau; status 4 when a block's
// list was full with its last entry at or above tau (it may have dropped
// candidates that reach tau), 5 when more than max_out candidates reach it.
__global__ void k_thr_final(WsHeader *h, float tau, int max_out, int32_t *out_count)
{
    if (threadIdx.x == 0) {
        const int c = h->thr_count;
        const int take = *out_count;
        *out_count = c < take ? c : take;
        if (h->status == 0) {
            if (__uint_as_float(h->gthr) >= tau && h->gthr != 0u) h->status = 4;
            else if (c > max_out) h->status = 5;
        }
    }
}

__global__ void k_tk_status(const WsHeader *h, int32_t *out)
{
    if (threadIdx.x == 0) *out = h->status != 0 ? h->status : h->scr_status;
}
}  // namespace sisso

extern "C" sisso_status sisso_select_threshold(const void *ws_c, size_t ws_bytes, float tau, int32_t max_out,
                                               int64_t *out_ids, float *out_scores, int32_t *out_count,
                                               void *stream)
{
    void *ws = const_cast<void *>(ws_c);
    if (!ws || !out_ids || !out_scores || !out_count) return SISSO_E_NULL;
    if (max_out < 1 || max_out > SISSO_MAX_BAND || !(tau >= 0.0f) || tau > 1.0f) return SISSO_E_RANGE;
    if (ws_bytes < ws_bytes_for(0, 1)) return SISSO_E_WORKSPACE;
    hipStream_t st = as_stream(stream);
    const sisso_status rs = topk_launch(ws, max_out, out_ids, out_scores, out_count, st, true);
    if (rs != SISSO_OK) return rs;
    hipLaunchKernelGGL(k_thr_reset, dim3(1), dim3(64), 0, st, (WsHeader *)ws);
    hipLaunchKernelGGL(k_thr_count, dim3(512), dim3(256), 0, st, ws, tau);
    hipLaunchKernelGGL(k_thr_final, dim3(1), dim3(64), 0, st, (WsHeader *)ws, tau, max_out, out_count);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_topk_status(const void *ws, size_t ws_bytes, int32_t *out_status, void *stream)
{
    if (!ws || !out_status) return SISSO_E_NULL;
    if (ws_bytes < ws_bytes_for(0, 1)) return SISSO_E_WORKSPACE;
    hipLaunchKernelGGL(k_tk_status, dim3(1), dim3(64), 0, as_stream(stream), (const WsHeader *)ws, out_status);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
