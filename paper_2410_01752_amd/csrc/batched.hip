// batched.hip -- SIS for many independent problems over one feature space in
// one persistent launch: cross-validation folds and bootstrap resamples of a
// dataset, or several datasets (Sec. 3's cross-validated evaluation; the
// outlook of Sec. 4, where independent fits are run on GPUs side by side).
//
// Every problem stores its pool P_{L-1} (FP32 columns + statistics); its SIS
// space is the TRI space of level L.  The last level N_L is never stored: its
// unary block is evaluated while the operand column streams by, and its
// binary block (pairs v < u, u new at level L-1) is evaluated in registers per
// 32 x 32 pair tile from LDS-staged operand chunks.  Both use the single-
// problem kernels' arithmetic (tiles.hpp).
//
// Work items are (problem, pair tile) and (problem, batch of 64 stored
// columns).  Items are ordered by problem size n (largest first, so the short
// problems fill the tail), pair tiles before column batches; persistent
// blocks take the next item from an atomic counter.  Each item keeps its best
// K'_p candidates (score desc, id asc) in LDS and writes them to its own list
// slot; a per-problem grid-wide bound (atomicMax on the K'-th score of every
// full list) lets later items skip what cannot enter the problem's top K'_p.
// sisso_topk_batched then merges each problem's lists with one block per
// problem (radix select on the score bits, then a bitonic sort).
#include "tiles.hpp"

namespace sisso {

constexpr int kBatchTU = 32, kBatchTV = 32;          // pair tile (RectCfg<2, 2>)
constexpr int kBatchCols = kColWaves * kColBatch;    // stored columns per item
constexpr int kBatchFinalCap = 4096;                 // merge buffer per problem
static_assert(kBatchFinalCap % 1024 == 0 && SISSO_MAX_KEEP < kBatchFinalCap,
              "the per-problem merge moves kBatchFinalCap / 1024 entries per thread, and the entries above the cutoff (fewer than keep) must fit");
constexpr int kMaxBatch = SISSO_MAX_BATCH;

struct BatchHeader {
    int next_item;          // work counter of the persistent launch
    int n_items;
    int n_problems;
    int keep_max;           // list slot stride
    int items_per_problem;
    int pair_items;         // of which pair tiles (first in a problem's range)
    int pad[2];
};

struct BatchView {
    BatchHeader *h;
    unsigned *gthr;         // per problem: admission bound (float bits)
    int *order;             // rank -> problem (n descending, index ascending)
    int *rank;              // problem -> rank
    int *pstatus;           // per problem: 0 or SISSO_E_SHAPE
    float *sc;              // n_items x keep_max
    int64_t *id;
};

__host__ __device__ inline size_t batch_ws_bytes(int problems, int64_t items, int keep_max)
{
    size_t b = align256(sizeof(BatchHeader));
    b += 4 * align256((size_t)problems * sizeof(int));
    b += align256((size_t)items * keep_max * sizeof(float));
    b += align256((size_t)items * keep_max * sizeof(int64_t));
    return b;
}

__host__ __device__ inline BatchView batch_view(void *ws, int problems, int64_t items, int keep_max)
{
    char *p = (char *)ws;
    BatchView v;
    v.h = (BatchHeader *)p;
    p += align256(sizeof(BatchHeader));
    v.gthr = (unsigned *)p;
    p += align256((size_t)problems * sizeof(int));
    v.order = (int *)p;
    p += align256((size_t)problems * sizeof(int));
    v.rank = (int *)p;
    p += align256((size_t)problems * sizeof(int));
    v.pstatus = (int *)p;
    p += align256((size_t)problems * sizeof(int));
    v.sc = (float *)p;
    p += align256((size_t)items * keep_max * sizeof(float));
    v.id = (int64_t *)p;
    return v;
}

__device__ inline BatchView batch_view_dev(void *ws)
{
    const BatchHeader *h = (const BatchHeader *)ws;
    return batch_view(ws, h->n_problems, h->n_items, h->keep_max);
}

// Pair tiles of the last TRI level: u tiles over N_{L-1} = [lo, hi), and for
// each the v tiles covering [0, min(u0 + TU, hi) - 1).
struct TriTiles {
    int64_t lo, hi;
    __host__ __device__ int64_t n_ut() const { return (hi - lo + kBatchTU - 1) / kBatchTU; }
    __host__ __device__ int64_t vlim(int64_t ut) const
    {
        const int64_t u0 = lo + ut * kBatchTU;
        const int64_t ue = u0 + kBatchTU < hi ? u0 + kBatchTU : hi;
        return ue - 1;
    }
    __host__ __device__ int64_t n_vt(int64_t ut) const { return (vlim(ut) + kBatchTV - 1) / kBatchTV; }
    __host__ __device__ int64_t count() const
    {
        int64_t c = 0;
        for (int64_t ut = 0; ut < n_ut(); ++ut) c += n_vt(ut);
        return c;
    }
};

__device__ inline bool problem_ok(const sisso_problem &P, int keep_max)
{
    return P.n >= 2 && P.n <= SISSO_MAX_N && P.keep >= 1 && P.keep <= keep_max && P.ld32 >= P.n &&
           (P.ld32 % 4) == 0 && P.pool32 && P.stats && P.r32 && P.info && (P.n_exclude == 0 || P.exclude) &&
           P.n_exclude >= 0;
}

// Header, per-problem bounds and the size order of the problems (one block).
__global__ void __launch_bounds__(256) k_batch_reset(void *ws, const sisso_problem *__restrict__ probs,
                                                     int problems, int items_per_problem, int pair_items,
                                                     int keep_max)
{
    BatchView W = batch_view(ws, problems, (int64_t)problems * items_per_problem, keep_max);
    if (threadIdx.x == 0) {
        W.h->next_item = 0;
        W.h->n_items = problems * items_per_problem;
        W.h->n_problems = problems;
        W.h->keep_max = keep_max;
        W.h->items_per_problem = items_per_problem;
        W.h->pair_items = pair_items;
    }
    for (int p = threadIdx.x; p < problems; p += blockDim.x) {
        const int np = probs[p].n;
        int r = 0;
        for (int q = 0; q < problems; ++q) {
            const int nq = probs[q].n;
            r += (nq > np || (nq == np && q < p)) ? 1 : 0;
        }
        W.order[r] = p;
        W.rank[p] = r;
        W.gthr[p] = 0u;
        W.pstatus[p] = problem_ok(probs[p], keep_max) ? 0 : (int)SISSO_E_SHAPE;
    }
}

template <int NU>
__global__ void __launch_bounds__(256) k_score_batch(sisso_space s, FormSlots fs,
                                                     const sisso_problem *__restrict__ probs, void *ws, int cap)
{
    using Cfg = RectCfg<2, 2>;
    constexpr int PER = 1 + NU;
    constexpr int NC = (kBatchCols * PER + 255) / 256;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *buf0 = (float *)smem;
    float *buf1 = buf0 + Cfg::BUF;
    float *lsc = buf1 + Cfg::BUF;
    int64_t *lid = (int64_t *)(lsc + cap);
    __shared__ int lcnt, s_item;
    __shared__ float lthr;
    __shared__ int64_t s_ut, s_vt;
    __shared__ float st_sc[kBatchCols * PER];
    __shared__ int64_t st_id[kBatchCols * PER];

    BatchView W = batch_view_dev(ws);
    const int I = W.h->items_per_problem, n_items = W.h->n_items, keep_max = W.h->keep_max;
    const int pair_items = W.h->pair_items;
    const int L = s.levels;
    const TriTiles tt{s.pool[L - 2], s.pool[L - 1]};
    const int64_t lo = tt.lo, hi = tt.hi;
    const int nu = s.n_unary;
    const PairIds ids{hi + (int64_t)nu * (hi - lo), lo, 0, s.n_slots, true};
    int uop[NU > 0 ? NU : 1];
#pragma unroll
    for (int o = 0; o < (NU > 0 ? NU : 1); ++o) uop[o] = (o < nu) ? s.unary[o] : 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const int it = atomicAdd(&W.h->next_item, 1);
            s_item = it;
            if (it < n_items) {
                const int local = it % I;
                if (local < pair_items) {
                    int64_t rem = local, ut = 0;
                    for (;; ++ut) {
                        const int64_t c = tt.n_vt(ut);
                        if (rem < c) break;
                        rem -= c;
                    }
                    s_ut = ut;
                    s_vt = rem;
                }
            }
        }
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        const int q = it / I, local = it % I;
        const int p = W.order[q];
        if (W.pstatus[p] != 0) continue;
        const sisso_problem P = probs[p];
        const int n = P.n;
        const double nd = (double)n, R1 = P.info->sum_r32, Srr = P.info->s_rr;
        BlockList Lst{lsc, lid, &lcnt, &lthr, cap, P.keep};
        list_init(Lst);
        unsigned *gthr = W.gthr + p;
        if (local < pair_items) {
            const int64_t ut = s_ut, vt = s_vt;
            const int64_t u0 = lo + ut * kBatchTU;
            USide<2, 2> U;
            load_uside<2, 2>(U, P.stats, ids, u0, hi);
            float osc[20];
            int64_t oid[20];
            score_pair_tile<2, 2>(P.pool32, P.ld32, P.stats, P.r32, n, nd, R1, Srr, fs, ids, u0, U,
                                  vt * kBatchTV, tt.vlim(ut), 0, s.total, buf0, buf1, osc, oid);
            list_offer<20>(Lst, osc, oid, gthr, P.exclude, P.n_exclude);
        } else {
            const int64_t c0 = (int64_t)(local - pair_items) * kBatchCols;
            for (int j = 0; j < kColBatch; ++j) {
                const int slot_base = (w * kColBatch + j) * PER;
                const int64_t c = c0 + w * kColBatch + j;
                float scs[PER];
#pragma unroll
                for (int o = 0; o < PER; ++o) scs[o] = -1.0f;
                if (c < hi)
                    score_column<NU>(P.pool32 + (size_t)c * P.ld32, P.stats[c], P.r32, n, nd, R1, Srr, uop, nu,
                                     NU > 0 && c >= lo, scs);
                if (lane == 0) {
#pragma unroll
                    for (int o = 0; o < PER; ++o) {
                        st_sc[slot_base + o] = scs[o];
                        st_id[slot_base + o] = o == 0 ? c : hi + (c - lo) * nu + (o - 1);
                    }
                }
            }
            __syncthreads();
            float osc[NC];
            int64_t oid[NC];
#pragma unroll
            for (int e = 0; e < NC; ++e) {
                const int x = threadIdx.x + e * 256;
                osc[e] = x < kBatchCols * PER ? st_sc[x] : -1.0f;
                oid[e] = x < kBatchCols * PER ? st_id[x] : INT64_MAX;
            }
            list_offer<NC>(Lst, osc, oid, gthr, P.exclude, P.n_exclude);
        }
        list_flush(Lst, gthr, W.sc + (size_t)it * keep_max, W.id + (size_t)it * keep_max);
    }
}

// Per-problem merge: one block of 1024 threads per problem.
__global__ void __launch_bounds__(1024) k_topk_batch(const sisso_problem *__restrict__ probs, void *ws,
                                                     int64_t *__restrict__ out_ids, float *__restrict__ out_sc,
                                                     int32_t *__restrict__ out_count, int32_t *__restrict__ out_status)
{
    __shared__ unsigned hist[kHistBins];
    __shared__ unsigned s_prefix;
    __shared__ int s_need, s_total, s_gt, s_eq;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *fsc = (float *)smem;
    int64_t *fid = (int64_t *)(smem + kBatchFinalCap * sizeof(float));

    BatchView W = batch_view_dev(ws);
    const int p = blockIdx.x;
    const int keep_max = W.h->keep_max, I = W.h->items_per_problem;
    int64_t *oi = out_ids + (size_t)p * keep_max;
    float *os = out_sc + (size_t)p * keep_max;
    if (p >= W.h->n_problems) {
        // more problems than the screening call covered
        for (int i = threadIdx.x; i < keep_max; i += blockDim.x) { oi[i] = INT64_MAX; os[i] = -1.0f; }
        if (threadIdx.x == 0) {
            out_count[p] = 0;
            if (out_status) out_status[p] = (int)SISSO_E_SHAPE;
        }
        return;
    }
    if (W.pstatus[p] != 0) {
        for (int i = threadIdx.x; i < keep_max; i += blockDim.x) { oi[i] = INT64_MAX; os[i] = -1.0f; }
        if (threadIdx.x == 0) {
            out_count[p] = 0;
            if (out_status) out_status[p] = W.pstatus[p];
        }
        return;
    }
    const int keep = probs[p].keep;
    const unsigned g = W.gthr[p];
    const int64_t first = (int64_t)W.rank[p] * I;
    const int64_t M = (int64_t)I * keep;
    auto entry = [&](int64_t e) -> size_t { return (size_t)(first + e / keep) * keep_max + (size_t)(e % keep); };
    auto considered = [&](float sc) { return sc >= 0.0f && __float_as_uint(sc) >= g; };

    if (threadIdx.x == 0) { s_prefix = 0u; s_need = keep; s_total = 0; s_gt = 0; s_eq = 0; }
    bool all = false;
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
        const unsigned pre = s_prefix;
        int cnt = 0;
        for (int64_t e = threadIdx.x; e < M; e += blockDim.x) {
            const float sc = W.sc[entry(e)];
            if (!considered(sc)) continue;
            const unsigned u = __float_as_uint(sc);
            unsigned bin;
            if (pass == 0) { bin = u >> 20; ++cnt; }
            else if (pass == 1) { if ((u >> 20) != (pre >> 20)) continue; bin = (u >> 8) & 0xFFFu; }
            else { if ((u >> 8) != (pre >> 8)) continue; bin = u & 0xFFu; }
            atomicAdd(&hist[bin], 1u);
        }
        if (pass == 0 && cnt) atomicAdd(&s_total, cnt);
        __syncthreads();
        if (pass == 0 && s_total <= keep) { all = true; break; }
        if (threadIdx.x == 0) {
            const int bins = pass == 2 ? 256 : kHistBins;
            const int shift = pass == 0 ? 20 : (pass == 1 ? 8 : 0);
            int need = s_need, b = bins - 1;
            for (; b > 0; --b) {
                const int c = (int)hist[b];
                if (c >= need) break;
                need -= c;
            }
            s_prefix |= ((unsigned)b) << shift;
            s_need = need;
        }
        __syncthreads();
    }
    const unsigned sstar = s_prefix;
    // Entries above the keep-th score (keep - need < keep of them) fill the
    // buffer from the front, entries equal to it from the back down to the
    // front's end: only ties at the cutoff can exceed the buffer, and only
    // tied entries are lost then.
    const int front = all ? kBatchFinalCap : keep - s_need;
    for (int64_t e = threadIdx.x; e < M; e += blockDim.x) {
        const size_t x = entry(e);
        const float sc = W.sc[x];
        if (!considered(sc)) continue;
        const unsigned u = __float_as_uint(sc);
        if (all || u > sstar) {
            const int slot = atomicAdd(&s_gt, 1);
            if (slot < kBatchFinalCap) { fsc[slot] = sc; fid[slot] = W.id[x]; }
        } else if (u == sstar) {
            const int slot = kBatchFinalCap - 1 - atomicAdd(&s_eq, 1);
            if (slot >= front) { fsc[slot] = sc; fid[slot] = W.id[x]; }
        }
    }
    __syncthreads();
    const int n_gt = s_gt, n_eq = s_eq;
    const int m_gt = n_gt < kBatchFinalCap ? n_gt : kBatchFinalCap;
    const int room = kBatchFinalCap - m_gt;
    const int m_eq = n_eq < room ? n_eq : room;
    const int m = m_gt + m_eq;
    // Move the ties behind the front entries.  The two ranges may overlap, so
    // every thread reads its entries before any thread writes (1024 threads x
    // kTiePer entries cover the buffer).
    constexpr int kTiePer = kBatchFinalCap / 1024;
    float tsc[kTiePer];
    int64_t tid[kTiePer];
#pragma unroll
    for (int j = 0; j < kTiePer; ++j) {
        const int i = threadIdx.x + 1024 * j;
        if (i < m_eq) { tsc[j] = fsc[kBatchFinalCap - 1 - i]; tid[j] = fid[kBatchFinalCap - 1 - i]; }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTiePer; ++j) {
        const int i = threadIdx.x + 1024 * j;
        if (i < m_eq) { fsc[m_gt + i] = tsc[j]; fid[m_gt + i] = tid[j]; }
    }
    const int cap = next_pow2(m > 1 ? m : 2);
    for (int i = threadIdx.x; i < cap; i += blockDim.x)
        if (i >= m) { fsc[i] = -1.0f; fid[i] = INT64_MAX; }
    __syncthreads();
    bitonic_sort_keys(fsc, fid, cap);
    const int take = m < keep ? m : keep;
    for (int i = threadIdx.x; i < keep_max; i += blockDim.x) {
        oi[i] = i < take ? fid[i] : INT64_MAX;
        os[i] = i < take ? fsc[i] : -1.0f;
    }
    if (threadIdx.x == 0) {
        out_count[p] = take;
        if (out_status) out_status[p] = n_gt + n_eq > kBatchFinalCap ? (int)SISSO_E_RANGE : 0;
    }
}

}  // namespace sisso

// ------------------------------------------------------------------ C ABI

using namespace sisso;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

bool batch_space_ok(const sisso_space *s)
{
    return s && s->total > 0 && s->levels == 2 && !s->rect;
}

struct BatchPlan {
    int pair_items = 0, col_items = 0, items_per_problem = 0;
};

BatchPlan batch_plan(const sisso_space *s)
{
    BatchPlan b;
    const TriTiles tt{s->pool[s->levels - 2], s->pool[s->levels - 1]};
    b.pair_items = (int)tt.count();
    b.col_items = (int)((s->pool[s->levels - 1] + kBatchCols - 1) / kBatchCols);
    b.items_per_problem = b.pair_items + b.col_items;
    return b;
}

int batch_list_cap(int keep_max) { return next_pow2(keep_max + 256); }

size_t batch_smem(int cap)
{
    return (size_t)2 * RectCfg<2, 2>::BUF * sizeof(float) + (size_t)cap * (sizeof(float) + sizeof(int64_t));
}

template <typename K>
int resident_grid(K kernel, size_t smem)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(kernel), 256, smem) !=
            hipSuccess || per <= 0)
        per = 1;
    return cus * per;
}

}  // namespace

extern "C" size_t sisso_batch_workspace_size(const sisso_space *space, int32_t n_problems, int32_t keep_max)
{
    if (!batch_space_ok(space) || n_problems < 1 || n_problems > kMaxBatch || keep_max < 1 ||
        keep_max > SISSO_MAX_KEEP)
        return 0;
    const BatchPlan b = batch_plan(space);
    return batch_ws_bytes(n_problems, (int64_t)n_problems * b.items_per_problem, keep_max);
}

extern "C" int32_t sisso_batch_items(const sisso_space *space)
{
    if (!batch_space_ok(space)) return -1;
    return batch_plan(space).items_per_problem;
}

extern "C" sisso_status sisso_expand_score_batched(const sisso_space *space, const sisso_problem *problems,
                                                   int32_t n_problems, int32_t keep_max, int32_t grid, void *ws,
                                                   size_t ws_bytes, void *stream)
{
    if (!space || !problems || !ws) return SISSO_E_NULL;
    if (space->total <= 0 || space->levels < 1 || space->levels > SISSO_MAX_LEVELS) return SISSO_E_SHAPE;
    if (!batch_space_ok(space)) return SISSO_E_UNSUPPORTED;
    if (n_problems < 1 || n_problems > kMaxBatch || keep_max < 1 || keep_max > SISSO_MAX_KEEP || grid < 0)
        return SISSO_E_SHAPE;
    const BatchPlan b = batch_plan(space);
    if (ws_bytes < batch_ws_bytes(n_problems, (int64_t)n_problems * b.items_per_problem, keep_max))
        return SISSO_E_WORKSPACE;
    if ((int64_t)n_problems * b.items_per_problem > INT32_MAX / 2) return SISSO_E_SHAPE;
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, st, ws, problems, n_problems, b.items_per_problem,
                       b.pair_items, keep_max);
    const int cap = batch_list_cap(keep_max);
    const size_t smem = batch_smem(cap);
    const FormSlots fs = form_slots(space);
    const int n_items = n_problems * b.items_per_problem;
    auto launch = [&](auto kern) -> sisso_status {
        if (!allow_dynamic_lds(kern, smem)) return SISSO_E_UNSUPPORTED;
        int g = grid > 0 ? grid : resident_grid(kern, smem);
        if (g > n_items) g = n_items;
        hipLaunchKernelGGL(kern, dim3(g), dim3(256), smem, st, *space, fs, problems, ws, cap);
        return SISSO_OK;
    };
    sisso_status rs;
    if (space->n_unary == 0) rs = launch(k_score_batch<0>);
    else if (space->n_unary <= 3) rs = launch(k_score_batch<3>);
    else rs = launch(k_score_batch<8>);
    if (rs != SISSO_OK) return rs;
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_topk_batched(const sisso_problem *problems, int32_t n_problems, const void *ws,
                                           size_t ws_bytes, int64_t *out_ids, float *out_scores,
                                           int32_t *out_count, int32_t *out_status, void *stream)
{
    if (!problems || !ws || !out_ids || !out_scores || !out_count) return SISSO_E_NULL;
    if (n_problems < 1 || n_problems > kMaxBatch || ws_bytes < sizeof(BatchHeader)) return SISSO_E_SHAPE;
    const size_t smem = (size_t)kBatchFinalCap * (sizeof(float) + sizeof(int64_t));
    hipLaunchKernelGGL(k_topk_batch, dim3(n_problems), dim3(1024), smem, as_stream(stream), problems,
                       const_cast<void *>(ws), out_ids, out_scores, out_count, out_status);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
