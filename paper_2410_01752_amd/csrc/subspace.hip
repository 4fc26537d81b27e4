// subspace.hip -- subspace update S_t = S_{t-1} u SIS(r) (Sec. 2.3,
// eq. subspace-expansion) with the duplicate rule for non-unique features
// (Sec. 2.1: some combinations are not unique).
//
// The screened list is re-scored in FP64 (|corr| of the FP64 feature with the
// FP64 residual).  Duplicate classes are the connected components of
// 1 - |corr(f, g)| <= 1e-9 over list + current subspace; a class touching the
// subspace is dropped; a class is represented by its smallest id and scored by
// its best member; the best k classes (score desc, id asc) are appended.
// The components are formed by a lock-free union-find over the duplicate
// pairs as the pair kernel finds them (a root is hooked under the smaller of
// two roots, so every root is the smallest node of its component), which
// holds any number of duplicate pairs.
#include "linalg.hpp"

namespace sisso {

struct SubWs {
    double *Z;        // n x nodes, standardised (ld = ldz)
    double *zr;       // standardised residual
    double *score;    // FP64 score per node (candidates)
    int *ok;          // per node
    int *parent;      // union-find forest over the nodes
    const double *wt; // sample weights (nullable: unweighted)
    int ldz;
};

__host__ __device__ inline size_t sub_ws_bytes(int n, int nodes)
{
    const size_t ldz = (size_t)((n + 3) & ~3);
    size_t b = 0;
    b += ldz * nodes * sizeof(double);
    b += ldz * sizeof(double);
    b += (size_t)nodes * sizeof(double);
    b += (size_t)nodes * sizeof(int);
    b = (b + 255) & ~(size_t)255;
    b += (size_t)nodes * sizeof(int);
    b += 256;
    return b;
}

__host__ __device__ inline SubWs sub_ws_view(void *ws, int n, int nodes)
{
    SubWs w;
    w.ldz = (n + 3) & ~3;
    char *p = (char *)ws;
    w.Z = (double *)p; p += (size_t)w.ldz * nodes * sizeof(double);
    w.zr = (double *)p; p += (size_t)w.ldz * sizeof(double);
    w.score = (double *)p; p += (size_t)nodes * sizeof(double);
    w.ok = (int *)p; p += (size_t)nodes * sizeof(int);
    size_t off = (size_t)(p - (char *)ws);
    off = (off + 255) & ~(size_t)255;
    p = (char *)ws + off;
    w.parent = (int *)p;
    w.wt = nullptr;
    return w;
}

__device__ inline void sub_resid(const double *__restrict__ r, int n, SubWs w)
{
    __shared__ double red[16];
    standardize_column_w(r, w.wt, n, w.zr, nullptr, nullptr, nullptr, red);
}

// node q < m_prev: subspace column; else candidate q - m_prev.
__device__ inline void sub_standardize(const double *__restrict__ sub, int lds, int m_prev,
                                       const double *__restrict__ cand, int ldc, const int32_t *__restrict__ cvalid,
                                       const int32_t *__restrict__ count_dev, int n, SubWs w, int q)
{
    __shared__ double red[16];
    const bool is_c = q >= m_prev;
    const int ci = q - m_prev;
    const double *x = is_c ? cand + (size_t)ci * ldc : sub + (size_t)q * lds;
    double *z = w.Z + (size_t)q * w.ldz;
    if (threadIdx.x == 0) w.parent[q] = q;
    int ok_live = 1;
    if (is_c) ok_live = (ci < *count_dev) && cvalid[ci] != 0;
    if (!ok_live) {
        for (int t = threadIdx.x; t < n; t += blockDim.x) z[t] = 0.0;
        if (threadIdx.x == 0) { w.ok[q] = 0; w.score[q] = -1.0; }
        return;
    }
    int okc;
    __shared__ int okc_s;
    standardize_column_w(x, w.wt, n, z, nullptr, nullptr, &okc_s, red);
    okc = okc_s;
    double d = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) d += z[t] * w.zr[t];
    const double dot = block_sum(d, red);
    if (threadIdx.x == 0) {
        w.ok[q] = okc;
        w.score[q] = okc ? fabs(dot) : -1.0;
    }
}

// Root of node a (loads bypass the non-coherent caches: other blocks hook
// roots while this one walks).
__device__ __forceinline__ int uf_root(int *par, int a)
{
    int p = __hip_atomic_load(par + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (p != a) {
        a = p;
        p = __hip_atomic_load(par + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return a;
}

// Join the components of a and b: the larger root is hooked under the smaller
// one by compare-and-swap; a failed swap means another thread changed that
// root, and the walk starts again.  Hooks only point to smaller nodes, so no
// cycle forms and every loop ends.
__device__ inline void uf_join(int *par, int a, int b)
{
    for (;;) {
        a = uf_root(par, a);
        b = uf_root(par, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        if (atomicCAS(par + a, a, b) == a) return;
    }
}

// Duplicate pairs between candidate rows and all earlier nodes, joined in the
// union-find forest.
__device__ inline void sub_edges(int m_prev, int nodes, int n, SubWs w, int bi, int bj)
{
    __shared__ double As[kGK][kGT + 1];
    __shared__ double Bs[kGK][kGT + 1];
    // rows: nodes, cols: nodes
    if (bj > bi) return;                              // only j <= i tiles
    if ((bi + 1) * kGT <= m_prev) return;             // rows all subspace members
    double acc[2][2];
    gemm_tile_tn(w.Z, nodes, w.Z, nodes, n, w.ldz, bi, bj, acc, As, Bs);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int i = bi * kGT + ty * 2 + a, j = bj * kGT + tx * 2 + b;
            if (i < nodes && j < i && i >= m_prev && w.ok[i] && w.ok[j] && 1.0 - fabs(acc[a][b]) <= kDupTol)
                uf_join(w.parent, i, j);
        }
}

__device__ __forceinline__ bool rank64_before(double sa, int64_t ia, double sb, int64_t ib)
{
    return sa > sb || (sa == sb && ia < ib);
}

// Components, classes, ranking and the new members (one block).
__device__ inline void sub_classes(int m_prev, int nodes, const int64_t *__restrict__ cand_ids,
                                   int64_t *__restrict__ sub_ids, int k, int32_t *n_new, int32_t *n_classes,
                                   int *__restrict__ new_src, SubWs w, unsigned char *smem)
{
    int *label = (int *)smem;                                   // nodes
    unsigned long long *rep = (unsigned long long *)(label + ((nodes + 1) & ~1));   // min id per root
    unsigned long long *best = rep + nodes;                     // max score bits per root
    double *ksc = (double *)(best + nodes);                     // class list (pow2)
    int64_t *kid = (int64_t *)(ksc + next_pow2(nodes));
    __shared__ int ncls;
    // component label: the root, which is the component's smallest node
    for (int i = threadIdx.x; i < nodes; i += blockDim.x) {
        int r = i;
        while (w.parent[r] != r) r = w.parent[r];
        label[i] = r;
        rep[i] = ~0ull;
        best[i] = 0ull;
    }
    __syncthreads();
    // per root: min candidate id and max FP64 score over valid candidates
    for (int i = threadIdx.x; i < nodes; i += blockDim.x) {
        if (i >= m_prev && w.ok[i]) {
            const int r = label[i];
            atomicMin(&rep[r], (unsigned long long)cand_ids[i - m_prev]);
            atomicMax(&best[r], (unsigned long long)__double_as_longlong(w.score[i]));
        }
    }
    if (threadIdx.x == 0) ncls = 0;
    __syncthreads();
    // surviving classes: roots not touching the subspace (min label >= m_prev)
    for (int i = threadIdx.x; i < nodes; i += blockDim.x) {
        if (label[i] == i && i >= m_prev && rep[i] != ~0ull) {
            const int q = atomicAdd(&ncls, 1);
            ksc[q] = __longlong_as_double((long long)best[i]);
            kid[q] = (int64_t)rep[i];
        }
    }
    __syncthreads();
    const int nc = ncls;
    const int cap = next_pow2(nc > 1 ? nc : 2);
    for (int i = nc + threadIdx.x; i < cap; i += blockDim.x) { ksc[i] = -1.0; kid[i] = INT64_MAX; }
    __syncthreads();
    for (int size = 2; size <= cap; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (cap >> 1); t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1)), j = i + stride;
                const bool up = (i & size) == 0;
                if (rank64_before(ksc[j], kid[j], ksc[i], kid[i]) == up) {
                    const double ts = ksc[i]; ksc[i] = ksc[j]; ksc[j] = ts;
                    const int64_t ti = kid[i]; kid[i] = kid[j]; kid[j] = ti;
                }
            }
            __syncthreads();
        }
    const int take = nc < k ? nc : k;
    // source candidate of each new member: the candidate whose id is the rep
    for (int i = threadIdx.x; i < nodes; i += blockDim.x) {
        if (i >= m_prev && w.ok[i]) {
            const int64_t id = cand_ids[i - m_prev];
            // binary search is not possible (ksc order); scan the taken list
            for (int q = 0; q < take; ++q)
                if (kid[q] == id) new_src[q] = i - m_prev;
        }
    }
    for (int q = threadIdx.x; q < take; q += blockDim.x) sub_ids[m_prev + q] = kid[q];
    if (threadIdx.x == 0) { *n_new = take; *n_classes = nc; }
}

__device__ inline void sub_gather(const double *__restrict__ cand, int ldc, const int *__restrict__ new_src,
                                  const int32_t *__restrict__ n_new, int n, double *__restrict__ sub, int lds,
                                  int m_prev, int q)
{
    if (q >= *n_new) return;
    const double *src = cand + (size_t)new_src[q] * ldc;
    double *dst = sub + (size_t)(m_prev + q) * lds;
    for (int t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
}

// Sort ids ascending (one block) and record the permutation.
__device__ inline void sort_ids(const int64_t *__restrict__ ids, int m, int64_t *__restrict__ ids_sorted,
                                int32_t *__restrict__ perm)
{
    __shared__ int64_t key[SISSO_MAX_SUBSPACE];
    __shared__ int pos[SISSO_MAX_SUBSPACE];
    const int cap = next_pow2(m > 1 ? m : 2);
    for (int i = threadIdx.x; i < cap; i += blockDim.x) {
        key[i] = i < m ? ids[i] : INT64_MAX;
        pos[i] = i;
    }
    __syncthreads();
    for (int size = 2; size <= cap; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (cap >> 1); t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1)), j = i + stride;
                const bool up = (i & size) == 0;
                const bool j_first = key[j] < key[i] || (key[j] == key[i] && pos[j] < pos[i]);
                if (j_first == up) {
                    const int64_t tk = key[i]; key[i] = key[j]; key[j] = tk;
                    const int tp = pos[i]; pos[i] = pos[j]; pos[j] = tp;
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < m; i += blockDim.x) { ids_sorted[i] = key[i]; perm[i] = pos[i]; }
}

__device__ inline void gather_perm(const double *__restrict__ src, int lds, const int32_t *__restrict__ perm, int n,
                                   double *__restrict__ dst, int ldd, int q)
{
    const double *s = src + (size_t)perm[q] * lds;
    double *d = dst + (size_t)q * ldd;
    for (int t = threadIdx.x; t < n; t += blockDim.x) d[t] = s[t];
}


// ------------------------------------------------------- one problem

__global__ void __launch_bounds__(256) k_sub_resid(const double *__restrict__ r, int n, SubWs w) { sub_resid(r, n, w); }

__global__ void __launch_bounds__(256) k_sub_standardize(const double *__restrict__ sub, int lds, int m_prev,
                                                         const double *__restrict__ cand, int ldc,
                                                         const int32_t *__restrict__ cvalid,
                                                         const int32_t *__restrict__ count_dev, int n, SubWs w)
{
    sub_standardize(sub, lds, m_prev, cand, ldc, cvalid, count_dev, n, w, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_sub_edges(int m_prev, int nodes, int n, SubWs w)
{
    sub_edges(m_prev, nodes, n, w, blockIdx.y, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_sub_classes(int m_prev, int nodes, const int64_t *__restrict__ cand_ids,
                                                      int64_t *__restrict__ sub_ids, int k, int32_t *n_new,
                                                      int32_t *n_classes, int *__restrict__ new_src, SubWs w)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    sub_classes(m_prev, nodes, cand_ids, sub_ids, k, n_new, n_classes, new_src, w, smem);
}

__global__ void __launch_bounds__(256) k_sub_gather(const double *__restrict__ cand, int ldc,
                                                    const int *__restrict__ new_src, const int32_t *__restrict__ n_new,
                                                    int n, double *__restrict__ sub, int lds, int m_prev)
{
    sub_gather(cand, ldc, new_src, n_new, n, sub, lds, m_prev, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_sort_ids(const int64_t *__restrict__ ids, int m,
                                                   int64_t *__restrict__ ids_sorted, int32_t *__restrict__ perm)
{
    sort_ids(ids, m, ids_sorted, perm);
}

__global__ void __launch_bounds__(256) k_gather_perm(const double *__restrict__ src, int lds,
                                                     const int32_t *__restrict__ perm, int n,
                                                     double *__restrict__ dst, int ldd)
{
    gather_perm(src, lds, perm, n, dst, ldd, blockIdx.x);
}

// ------------------------------------------------------- many problems
//
// The same bodies over a table: blockIdx.y (edges: blockIdx.z) is the
// problem; blocks beyond a problem's own extent return at once.

__host__ __device__ inline size_t sub_ws_total(int n, int count_max, int m_prev)
{
    return sub_ws_bytes(n, m_prev + count_max) + (size_t)SISSO_MAX_SUBSPACE * sizeof(int) + 256;
}

__device__ inline bool subp_ok(const sisso_subspace_problem &P, int nodes_max, int k_max)
{
    return P.cand && P.cand_ids && P.cand_valid && P.count_dev && P.r && P.sub && P.sub_ids && P.n_new &&
           P.n_classes && P.ws && P.n >= 2 && P.n <= SISSO_MAX_N && P.ldc >= P.n && P.lds >= P.n &&
           P.count_max >= 1 && P.count_max <= SISSO_MAX_KEEP && P.m_prev >= 0 && P.k >= 1 && P.k <= k_max &&
           P.m_prev + P.k <= SISSO_MAX_SUBSPACE && P.m_prev + P.count_max <= nodes_max &&
           P.ws_bytes >= (int64_t)sub_ws_total(P.n, P.count_max, P.m_prev);
}

__device__ inline SubWs subp_ws(const sisso_subspace_problem &P)
{
    return sub_ws_view(P.ws, P.n, P.m_prev + P.count_max);
}

__device__ inline int *subp_new_src(const sisso_subspace_problem &P)
{
    return (int *)((char *)P.ws + sub_ws_bytes(P.n, P.m_prev + P.count_max));
}

__global__ void __launch_bounds__(256) k_subb_resid(const sisso_subspace_problem *__restrict__ T, int nodes_max,
                                                    int k_max, int32_t *__restrict__ status)
{
    const sisso_subspace_problem P = T[blockIdx.y];
    const bool ok = subp_ok(P, nodes_max, k_max);
    if (threadIdx.x == 0 && status) status[blockIdx.y] = ok ? SISSO_OK : SISSO_E_SHAPE;
    if (!ok) return;
    sub_resid(P.r, P.n, subp_ws(P));
}

__global__ void __launch_bounds__(256) k_subb_standardize(const sisso_subspace_problem *__restrict__ T, int nodes_max,
                                                          int k_max)
{
    const sisso_subspace_problem P = T[blockIdx.y];
    if (!subp_ok(P, nodes_max, k_max) || (int)blockIdx.x >= P.m_prev + P.count_max) return;
    sub_standardize(P.sub, P.lds, P.m_prev, P.cand, P.ldc, P.cand_valid, P.count_dev, P.n, subp_ws(P), blockIdx.x);
}

__global__ void __launch_bounds__(256) k_subb_edges(const sisso_subspace_problem *__restrict__ T, int nodes_max,
                                                    int k_max)
{
    const sisso_subspace_problem P = T[blockIdx.z];
    const int nodes = P.m_prev + P.count_max, tiles = (nodes + kGT - 1) / kGT;
    if (!subp_ok(P, nodes_max, k_max) || (int)blockIdx.x >= tiles || (int)blockIdx.y >= tiles) return;
    sub_edges(P.m_prev, nodes, P.n, subp_ws(P), blockIdx.y, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_subb_classes(const sisso_subspace_problem *__restrict__ T, int nodes_max,
                                                       int k_max)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const sisso_subspace_problem P = T[blockIdx.y];
    if (!subp_ok(P, nodes_max, k_max)) return;
    sub_classes(P.m_prev, P.m_prev + P.count_max, P.cand_ids, P.sub_ids, P.k, P.n_new, P.n_classes,
                subp_new_src(P), subp_ws(P), smem);
}

__global__ void __launch_bounds__(256) k_subb_gather(const sisso_subspace_problem *__restrict__ T, int nodes_max,
                                                     int k_max)
{
    const sisso_subspace_problem P = T[blockIdx.y];
    if (!subp_ok(P, nodes_max, k_max) || (int)blockIdx.x >= P.k) return;
    sub_gather(P.cand, P.ldc, subp_new_src(P), P.n_new, P.n, P.sub, P.lds, P.m_prev, blockIdx.x);
}

__device__ inline bool sortp_ok(const sisso_sort_problem &P, int m_max)
{
    return P.src && P.ids && P.dst && P.ids_sorted && P.perm && P.m >= 1 && P.m <= m_max && P.n >= 1 &&
           P.lds >= P.n && P.ldd >= P.n;
}

__global__ void __launch_bounds__(1024) k_sortb_ids(const sisso_sort_problem *__restrict__ T, int m_max,
                                                    int32_t *__restrict__ status)
{
    const sisso_sort_problem P = T[blockIdx.y];
    const bool ok = sortp_ok(P, m_max);
    if (threadIdx.x == 0 && status) status[blockIdx.y] = ok ? SISSO_OK : SISSO_E_SHAPE;
    if (!ok) return;
    sort_ids(P.ids, P.m, P.ids_sorted, P.perm);
}

__global__ void __launch_bounds__(256) k_sortb_gather(const sisso_sort_problem *__restrict__ T, int m_max)
{
    const sisso_sort_problem P = T[blockIdx.y];
    if (!sortp_ok(P, m_max) || (int)blockIdx.x >= P.m) return;
    gather_perm(P.src, P.lds, P.perm, P.n, P.dst, P.ldd, blockIdx.x);
}

}  // namespace sisso

using namespace sisso;

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" size_t sisso_subspace_workspace_size(int32_t n, int32_t count, int32_t m_prev)
{
    if (n < 2 || count < 0 || m_prev < 0) return 0;
    return sub_ws_total(n, count, m_prev);
}

static size_t classes_smem(int nodes)
{
    return (size_t)((nodes + 1) & ~1) * sizeof(int) + (size_t)nodes * 2 * sizeof(unsigned long long) +
           (size_t)next_pow2(nodes) * (sizeof(double) + sizeof(int64_t));
}

extern "C" sisso_status sisso_subspace_update_weighted(const double *cand, int32_t ldc, const int64_t *cand_ids,
                                                       const int32_t *cand_valid, const int32_t *count_dev,
                                                       int32_t count_max, const double *r, const double *wts,
                                                       int32_t n, double *sub, int32_t lds, int64_t *sub_ids,
                                                       int32_t m_prev, int32_t k, int32_t *n_new, int32_t *n_classes,
                                                       void *ws, size_t ws_bytes, void *stream)
{
    if (!cand || !cand_ids || !cand_valid || !count_dev || !r || !sub || !sub_ids || !n_new || !n_classes || !ws)
        return SISSO_E_NULL;
    if (n < 2 || n > SISSO_MAX_N || ldc < n || lds < n || count_max < 1 || count_max > SISSO_MAX_KEEP ||
        m_prev < 0 || k < 1 || m_prev + k > SISSO_MAX_SUBSPACE)
        return SISSO_E_SHAPE;
    const int nodes = m_prev + count_max;
    if (ws_bytes < sisso_subspace_workspace_size(n, count_max, m_prev)) return SISSO_E_WORKSPACE;
    hipStream_t st = as_stream(stream);
    SubWs w = sub_ws_view(ws, n, nodes);
    w.wt = wts;
    int *new_src = (int *)((char *)ws + sub_ws_bytes(n, nodes));
    hipLaunchKernelGGL(k_sub_resid, dim3(1), dim3(256), 0, st, r, n, w);
    hipLaunchKernelGGL(k_sub_standardize, dim3(nodes), dim3(256), 0, st, sub, lds, m_prev, cand, ldc, cand_valid,
                       count_dev, n, w);
    const int tiles = (nodes + kGT - 1) / kGT;
    hipLaunchKernelGGL(k_sub_edges, dim3(tiles, tiles), dim3(256), 0, st, m_prev, nodes, n, w);
    const size_t smem = classes_smem(nodes);
    if (smem > 160 * 1024) return SISSO_E_SHAPE;
    if (!allow_dynamic_lds(k_sub_classes, smem)) return SISSO_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_sub_classes, dim3(1), dim3(1024), smem, st, m_prev, nodes, cand_ids, sub_ids, k, n_new,
                       n_classes, new_src, w);
    hipLaunchKernelGGL(k_sub_gather, dim3(k), dim3(256), 0, st, cand, ldc, new_src, n_new, n, sub, lds, m_prev);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_subspace_update(const double *cand, int32_t ldc, const int64_t *cand_ids,
                                              const int32_t *cand_valid, const int32_t *count_dev,
                                              int32_t count_max, const double *r, int32_t n, double *sub,
                                              int32_t lds, int64_t *sub_ids, int32_t m_prev, int32_t k,
                                              int32_t *n_new, int32_t *n_classes, void *ws, size_t ws_bytes,
                                              void *stream)
{
    return sisso_subspace_update_weighted(cand, ldc, cand_ids, cand_valid, count_dev, count_max, r, nullptr, n, sub,
                                          lds, sub_ids, m_prev, k, n_new, n_classes, ws, ws_bytes, stream);
}

extern "C" sisso_status sisso_sort_subspace(const double *src, int32_t lds, const int64_t *ids, int32_t m,
                                            int32_t n, double *dst, int32_t ldd, int64_t *ids_sorted,
                                            int32_t *perm_out, void *stream)
{
    if (!src || !ids || !dst || !ids_sorted || !perm_out) return SISSO_E_NULL;
    if (m < 1 || m > SISSO_MAX_SUBSPACE || n < 1 || lds < n || ldd < n) return SISSO_E_SHAPE;
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_sort_ids, dim3(1), dim3(1024), 0, st, ids, m, ids_sorted, perm_out);
    hipLaunchKernelGGL(k_gather_perm, dim3(m), dim3(256), 0, st, src, lds, perm_out, n, dst, ldd);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_subspace_update_batched(const sisso_subspace_problem *problems, int32_t n_problems,
                                                      int32_t nodes_max, int32_t k_max, int32_t *out_status,
                                                      void *stream)
{
    if (!problems) return SISSO_E_NULL;
    if (n_problems < 1 || n_problems > SISSO_MAX_BATCH || nodes_max < 1 ||
        nodes_max > SISSO_MAX_SUBSPACE + SISSO_MAX_KEEP || k_max < 1 || k_max > SISSO_MAX_SUBSPACE)
        return SISSO_E_SHAPE;
    const size_t smem = classes_smem(nodes_max);
    if (smem > 160 * 1024) return SISSO_E_SHAPE;
    if (!allow_dynamic_lds(k_subb_classes, smem)) return SISSO_E_UNSUPPORTED;
    hipStream_t st = as_stream(stream);
    const unsigned P = (unsigned)n_problems;
    const int tiles = (nodes_max + kGT - 1) / kGT;
    hipLaunchKernelGGL(k_subb_resid, dim3(1, P), dim3(256), 0, st, problems, nodes_max, k_max, out_status);
    hipLaunchKernelGGL(k_subb_standardize, dim3(nodes_max, P), dim3(256), 0, st, problems, nodes_max, k_max);
    hipLaunchKernelGGL(k_subb_edges, dim3(tiles, tiles, P), dim3(256), 0, st, problems, nodes_max, k_max);
    hipLaunchKernelGGL(k_subb_classes, dim3(1, P), dim3(1024), smem, st, problems, nodes_max, k_max);
    hipLaunchKernelGGL(k_subb_gather, dim3(k_max, P), dim3(256), 0, st, problems, nodes_max, k_max);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_sort_subspace_batched(const sisso_sort_problem *problems, int32_t n_problems,
                                                    int32_t m_max, int32_t *out_status, void *stream)
{
    if (!problems) return SISSO_E_NULL;
    if (n_problems < 1 || n_problems > SISSO_MAX_BATCH || m_max < 1 || m_max > SISSO_MAX_SUBSPACE)
        return SISSO_E_SHAPE;
    hipStream_t st = as_stream(stream);
    const unsigned P = (unsigned)n_problems;
    hipLaunchKernelGGL(k_sortb_ids, dim3(1, P), dim3(1024), 0, st, problems, m_max, out_status);
    hipLaunchKernelGGL(k_sortb_gather, dim3(m_max, P), dim3(256), 0, st, problems, m_max);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
