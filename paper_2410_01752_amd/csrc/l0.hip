// l0.hip -- the sparsifying operator: exhaustive least squares over every
// D-subset of the subspace (Sec. 2.3, eq. residual, read with an inverse; the
// best model minimises the residual norm over all C(m, D) models).
//
// Columns and y are centred (the intercept is fitted and not counted in D) and
// columns are scaled to unit norm; their FP64 correlation Gram C and
// beta = Z^T y~ are formed once.  A tuple's SSE then follows from an
// incremental Cholesky factorisation of C restricted to the tuple:
//   D = 1: SSE = S_yy - b_i^2
//   D = 2: L22 = sqrt(1 - C_ij^2), z2 = (b_j - C_ij b_i) / L22,
//          SSE = S_yy - b_i^2 - z2^2
//   D = 3: L32 = (C_jl - C_il C_ij) / L22, q = 1 - C_il^2 - L32^2,
//          tau = b_l - C_il b_i - L32 z2, SSE = S_yy - b_i^2 - z2^2 - tau^2 / q
// A tuple whose pivot (L22^2 or q) is <= singular_tol is skipped.
// Pass 1 finds the minimum SSE; pass 2 the lexicographically first tuple whose
// SSE is within 1e-12 S_yy of it (columns arrive in ascending id order).
//
// One problem: the Gram is split over the samples across blocks (partial
// tiles summed in a fixed order, so the result does not depend on the launch);
// D = 2 takes one thread per pair; D = 3 one wave per first index, block of
// 64 second indices (one per lane) and block of third indices, pass 1 records
// each block's minimum SSE, and pass 2 revisits only the blocks whose minimum
// lies in the tie band.  Many problems (batched) keep one block per first index.
#include "linalg.hpp"

#include <mutex>

namespace sisso {

struct L0Ws {
    double *Z;         // n x m standardised
    double *C;         // m x m correlation Gram
    double *beta;      // m
    double *mean;      // m
    double *norm;      // m
    double *yt;        // n centred y
    double *scal;      // [0] ybar, [1] syy, [2] sum of the weights (n unweighted)
    unsigned long long *best;   // [0] min SSE bits, [1] lex key
    unsigned long long *skipped;
    double *pmin;      // per work item of the D = 3 search: its minimum SSE (one problem)
    double *part;      // split Gram: partial tiles
    const double *wt;  // sample weights (nullable: unweighted)
    int ldz;
};

// D = 3 work items: a first index, a block of 64 second indices and a block
// of kRunL third indices (one minimum per item is kept between the two
// passes), indexed over the full rectangle
constexpr int kRunL = 64;
__host__ __device__ inline int l0_jblocks(int m) { return (m + 63) / 64; }
__host__ __device__ inline int l0_lblocks(int m) { return (m + kRunL - 1) / kRunL; }
__host__ __device__ inline int64_t l0_items3(int m) { return (int64_t)m * l0_jblocks(m) * l0_lblocks(m); }
__host__ __device__ inline size_t l0_pmin_count(int m) { return (size_t)l0_items3(m); }

// Gram split over the samples: a part per 256 samples, at most 8, and no more
// than keep the partial tiles within 8 MB
constexpr int kGramSplitK = 256;
constexpr int kGramMaxSplit = 8;
constexpr size_t kGramPartBytes = (size_t)8 << 20;
__host__ __device__ inline int l0_gram_tiles(int m) { const int t = (m + kGT - 1) / kGT; return t * (t + 1) / 2; }
__host__ __device__ inline int l0_gram_split(int m, int n)
{
    int s = (n + kGramSplitK - 1) / kGramSplitK;
    const int cap = (int)(kGramPartBytes / ((size_t)l0_gram_tiles(m) * kGT * kGT * 8));
    s = s > cap ? cap : s;
    return s < 1 ? 1 : (s > kGramMaxSplit ? kGramMaxSplit : s);
}

__host__ __device__ inline size_t l0_ws_bytes(int m, int n)
{
    const size_t ldz = (size_t)((n + 3) & ~3);
    size_t b = ldz * m * 8 + (size_t)m * m * 8 + 3 * (size_t)m * 8 + ldz * 8 + 4 * 8 + 4 * 8;
    b += l0_pmin_count(m) * 8;
    b += (size_t)l0_gram_tiles(m) * l0_gram_split(m, n) * kGT * kGT * 8;
    return (b + 255) & ~(size_t)255;
}

__host__ __device__ inline L0Ws l0_ws_view(void *ws, int m, int n)
{
    L0Ws w;
    w.ldz = (n + 3) & ~3;
    char *p = (char *)ws;
    w.Z = (double *)p; p += (size_t)w.ldz * m * 8;
    w.C = (double *)p; p += (size_t)m * m * 8;
    w.beta = (double *)p; p += (size_t)m * 8;
    w.mean = (double *)p; p += (size_t)m * 8;
    w.norm = (double *)p; p += (size_t)m * 8;
    w.yt = (double *)p; p += (size_t)w.ldz * 8;
    w.scal = (double *)p; p += 4 * 8;
    w.best = (unsigned long long *)p; p += 2 * 8;
    w.skipped = (unsigned long long *)p; p += 2 * 8;
    w.pmin = (double *)p; p += l0_pmin_count(m) * 8;
    w.part = (double *)p;
    w.wt = nullptr;
    return w;
}

// Centred y (weighted: sqrt(w) (y - ybar_w), the whitened target of
// Sec. 2.4), ybar and S_yy = sum w (y - ybar)^2.
__device__ inline void l0_y(const double *__restrict__ y, int n, L0Ws w)
{
    __shared__ double red[16];
    double ym, syy, W;
    if (!w.wt) {
        double s = 0.0;
        for (int t = threadIdx.x; t < n; t += blockDim.x) s += y[t];
        ym = block_sum(s, red) / n;
        double ss = 0.0;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const double e = y[t] - ym;
            w.yt[t] = e;
            ss += e * e;
        }
        syy = block_sum(ss, red);
        W = (double)n;
    } else {
        double s = 0.0, sw = 0.0;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            s += w.wt[t] * y[t];
            sw += w.wt[t];
        }
        W = block_sum(sw, red);
        ym = block_sum(s, red) / W;
        double ss = 0.0;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const double e = y[t] - ym;
            w.yt[t] = sqrt(w.wt[t]) * e;
            ss += w.wt[t] * e * e;
        }
        syy = block_sum(ss, red);
    }
    if (threadIdx.x == 0) {
        w.scal[0] = ym;
        w.scal[1] = syy;
        w.scal[2] = W;
        w.best[0] = 0x7FF0000000000000ull;   // +inf
        w.best[1] = ~0ull;
        *w.skipped = 0ull;
    }
}

__device__ inline void l0_column(const double *__restrict__ F, int ld, int n, L0Ws w, int j)
{
    __shared__ double red[16];
    double *z = w.Z + (size_t)j * w.ldz;
    standardize_column_w(F + (size_t)j * ld, w.wt, n, z, &w.mean[j], &w.norm[j], nullptr, red);
    double d = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) d += z[t] * w.yt[t];
    const double b = block_sum(d, red);
    if (threadIdx.x == 0) w.beta[j] = b;
}

__device__ __forceinline__ unsigned long long sse_bits(double sse)
{
    return (unsigned long long)__double_as_longlong(sse > 0.0 ? sse : 0.0);
}

// Lower-triangle tile t (row-major over bi >= bj) of the Gram.
__device__ __forceinline__ void gram_tile(int t, int &bi, int &bj)
{
    int b = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((b + 1) * (b + 2) / 2 <= t) ++b;
    while (b * (b + 1) / 2 > t) --b;
    bi = b;
    bj = t - b * (b + 1) / 2;
}

// Split Gram: one block per lower-triangle 64 x 64 tile and part of the
// samples writes the part's dot products into the partial slots of the
// tile's 32 x 32 tiles (those above the diagonal of a diagonal 64 x 64 tile
// are not stored); each thread computes a 4 x 4 block of dot products.  Every
// dot product takes the part's samples in order, one fma each from 0.0, as
// gemm_tile_tn_range does, so the sums equal those of l0_gram bit for bit.
constexpr int kGT4 = 2 * kGT;
__host__ __device__ inline int l0_gram_tiles64(int m) { const int t = (m + kGT4 - 1) / kGT4; return t * (t + 1) / 2; }
__device__ inline void l0_gram_part64(int m, int n, L0Ws w, int split, int T, int sp)
{
    constexpr int KK = 16;
    __shared__ __attribute__((aligned(16))) double As[KK][kGT4 + 2];
    __shared__ __attribute__((aligned(16))) double Bs[KK][kGT4 + 2];
    int BI, BJ;
    gram_tile(T, BI, BJ);
    const int chunk = ((n + split - 1) / split + kGK - 1) / kGK * kGK;
    const int kb = sp * chunk, ke = kb + chunk < n ? kb + chunk : n;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    constexpr int Q = KK * kGT4 / 256;              // values of each operand per thread and chunk
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    double ra[Q], rb[Q];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q, c = e / KK, t = e % KK;
            const int ia = BI * kGT4 + c, ib = BJ * kGT4 + c;
            ra[q] = (ia < m && k0 + t < ke) ? w.Z[(size_t)ia * w.ldz + k0 + t] : 0.0;
            rb[q] = (ib < m && k0 + t < ke) ? w.Z[(size_t)ib * w.ldz + k0 + t] : 0.0;
        }
    };
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += KK) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q, c = e / KK, t = e % KK;
            As[t][c] = ra[q];
            Bs[t][c] = rb[q];
        }
        __syncthreads();
        if (k0 + KK < ke) load(k0 + KK);             // the next chunk's loads overlap this chunk's products
#pragma unroll
        for (int t = 0; t < KK; ++t) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) { av[a] = As[t][ty * 4 + a]; bv[a] = Bs[t][tx * 4 + a]; }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
    const int nt = (m + kGT - 1) / kGT;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = BI * kGT4 + ty * 4 + a, j = BJ * kGT4 + tx * 4 + b;
            const int bi = i / kGT, bj = j / kGT;
            if (bi < nt && bj <= bi) {
                const int t32 = bi * (bi + 1) / 2 + bj;
                w.part[((size_t)t32 * split + sp) * (kGT * kGT) + (i % kGT) * kGT + j % kGT] = acc[a][b];
            }
        }
}

// The parts of each tile summed in their order into the symmetric Gram (unit
// diagonal).
__device__ inline void l0_gram_sum(int m, L0Ws w, int split, int t)
{
    int bi, bj;
    gram_tile(t, bi, bj);
    const double *part = w.part + (size_t)t * split * (kGT * kGT);
    for (int e = threadIdx.x; e < kGT * kGT; e += blockDim.x) {
        const int i = bi * kGT + e / kGT, j = bj * kGT + e % kGT;
        if (i < m && j < m && j <= i) {
            double v = 0.0;
            for (int sp = 0; sp < split; ++sp) v += part[(size_t)sp * (kGT * kGT) + e];
            v = i == j ? 1.0 : v;
            w.C[(size_t)i * m + j] = v;
            w.C[(size_t)j * m + i] = v;
        }
    }
}

// Tile (bi, bj) of the Gram by one block, the sample parts of
// l0_gram_split taken one after another and summed in the order l0_gram_sum
// takes them, so both give the same values.
__device__ inline void l0_gram(int m, int n, L0Ws w, int bi, int bj)
{
    __shared__ double As[kGK][kGT + 1];
    __shared__ double Bs[kGK][kGT + 1];
    if (bj > bi) return;
    const int split = l0_gram_split(m, n);
    const int chunk = ((n + split - 1) / split + kGK - 1) / kGK * kGK;
    double v[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int sp = 0; sp < split; ++sp) {
        const int k0 = sp * chunk, k1 = k0 + chunk < n ? k0 + chunk : n;
        double acc[2][2];
        gemm_tile_tn_range(w.Z, m, w.Z, m, k0, k1, w.ldz, bi, bj, acc, As, Bs);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) v[a][b] += acc[a][b];
    }
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int i = bi * kGT + ty * 2 + a, j = bj * kGT + tx * 2 + b;
            if (i < m && j < m && j <= i) {
                const double c = i == j ? 1.0 : v[a][b];
                w.C[(size_t)i * m + j] = c;
                w.C[(size_t)j * m + i] = c;
            }
        }
}

// The double of lane k (wave-uniform k), moved bit for bit.
__device__ __forceinline__ double readlane_f64(double x, int k)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), k);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(v, o, 64);
        v = other < v ? other : v;
    }
    return v;
}

// Block minimum of a 64-bit key into *dst (atomic), and a skip count.
__device__ inline void block_min_to(unsigned long long mine, unsigned long long *dst, unsigned long long nskip,
                                    unsigned long long *skipped)
{
    __shared__ unsigned long long red64[16];
    __shared__ unsigned long long skip_s;
    if (threadIdx.x == 0) skip_s = 0;
    mine = wave_min_u64(mine);
    __syncthreads();
    if (nskip) atomicAdd(&skip_s, nskip);
    if ((threadIdx.x & 63) == 0) red64[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long v = red64[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) v = red64[q] < v ? red64[q] : v;
        // most blocks hold no improvement by the time they finish: they
        // leave the shared minimum alone (fewer atomics on one address)
        if (v < __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(dst, v);
        if (skipped && skip_s) atomicAdd(skipped, skip_s);
    }
}

// D = 2, one thread per pair (i, j): PASS 0 the minimum SSE, PASS 1 the
// smallest key i m + j with SSE in the tie band.  The arithmetic of a tuple is
// the batched kernels'.
template <int PASS>
__global__ void __launch_bounds__(256) k_l0_pairs2(int m, double tol, L0Ws w)
{
    const double syy = w.scal[1];
    const double band = PASS == 1 ? __longlong_as_double((long long)w.best[0]) + kTieRel * syy : 0.0;
    unsigned long long mine = PASS == 0 ? 0x7FF0000000000000ull : ~0ull, nskip = 0;
    const int64_t npairs = (int64_t)m * (m - 1) / 2;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        int64_t jj, ii;
        pair_from_index(p, &jj, &ii);
        const int i = (int)ii, j = (int)jj;
        const double bi = w.beta[i];
        const double cij = w.C[(size_t)i * m + j];
        const double p2 = fma(-cij, cij, 1.0);
        if (!(p2 > tol)) { nskip++; continue; }
        const double l22 = sqrt(p2);
        const double z2 = (w.beta[j] - cij * bi) / l22;
        const double sse = fma(-z2, z2, w.scal[1] - bi * bi);
        const unsigned long long sb = sse_bits(sse);
        if (PASS == 0) { if (sb < mine) mine = sb; }
        else if (__longlong_as_double((long long)sb) <= band) {
            const unsigned long long key = (unsigned long long)i * m + j;
            if (key < mine) mine = key;
        }
    }
    block_min_to(mine, &w.best[PASS], PASS == 0 ? nskip : 0, PASS == 0 ? w.skipped : nullptr);
}

// D = 3: a work item is a first index i, a block of 64 second indices j (one
// per lane) and a block of kRunL third indices l, looped over by the wave.
// Items are indexed over the rectangle (i, j block, l block); those with no
// tuple are skipped at once.  Per l the wave loads C_il and b_l once and the
// row C_l. (C_lj = C_jl, coalesced over the lanes' j).  PASS 0 records each
// item's minimum SSE and the global minimum; PASS 1 revisits only the items
// whose minimum lies in the tie band and finds the smallest key
// (i m + j) m + l there.  The arithmetic of a tuple is the batched kernels'.
template <int PASS>
__global__ void __launch_bounds__(256) k_l0_cols3(int m, double tol, L0Ws w)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const double syy = w.scal[1];
    const double band = PASS == 1 ? __longlong_as_double((long long)w.best[0]) + kTieRel * syy : 0.0;
    unsigned long long mine = PASS == 0 ? 0x7FF0000000000000ull : ~0ull, nskip = 0;
    const int nj = l0_jblocks(m), nl = l0_lblocks(m);
    const int64_t items = l0_items3(m);
    for (int64_t it = wave; it < items; it += nw) {
        const int i = (int)(it / ((int64_t)nj * nl));
        const int rem = (int)(it % ((int64_t)nj * nl));
        const int jb = rem / nl, lb = rem % nl;
        const int j0 = i + 1 + 64 * jb;                           // the block's first j
        const int lo = j0 + 1 + kRunL * lb;                        // its l range [lo, hi)
        const int hi = lo + kRunL < m ? lo + kRunL : m;
        if (j0 >= m - 1 || lo >= m) continue;                      // wave-uniform: no tuple
        if (PASS == 1 && !(w.pmin[it] <= band)) continue;          // wave-uniform
        const double *Ci = w.C + (size_t)i * m;
        const double bi = w.beta[i];
        const double base = syy - bi * bi;
        // this lane's pair (i, j): C_ij, 1 / L22, z2, S_yy - b_i^2 - z2^2
        const int j = j0 + lane;
        const bool jin = j < m - 1;
        const double cij = jin ? Ci[j] : 0.0;
        const double p2 = fma(-cij, cij, 1.0);
        const bool okj = jin && p2 > tol;
        const double l22 = sqrt(p2);
        const double iv = okj ? 1.0 / l22 : 0.0;
        const double z2 = okj ? (w.beta[jin ? j : 0] - cij * bi) / l22 : 0.0;
        const double bs = fma(-z2, z2, base);
        unsigned long long pm = 0x7FF0000000000000ull;
        // C_il and b_l of the block's l, one per lane, read back per l as scalars
        const int nlc = hi - lo;
        const double cil_v = lane < nlc ? Ci[lo + lane] : 0.0;
        const double bl_v = lane < nlc ? w.beta[lo + lane] : 0.0;
        for (int t = 0; t < nlc; t += 4) {
            double cjl[4];                                         // the loads of four l ahead
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int l = lo + t + u;
                cjl[u] = t + u < nlc && okj && l > j ? w.C[(size_t)l * m + j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (t + u >= nlc) break;                           // wave-uniform
                const int l = lo + t + u;
                const double cil = readlane_f64(cil_v, t + u);
                const double bl = readlane_f64(bl_v, t + u);
                const double r1 = fma(-cil, cil, 1.0);
                const double t1 = fma(-cil, bi, bl);
                if (l <= j) continue;                              // lanes past l hold no tuple
                if (!okj) {
                    if (PASS == 0 && jin) nskip++;                 // singular pair: every l skipped
                    continue;
                }
                const double l32 = fma(-cil, cij, cjl[u]) * iv;
                const double q = fma(-l32, l32, r1);
                if (!(q > tol)) { if (PASS == 0) nskip++; continue; }
                const double tau = fma(-l32, z2, t1);
                const double sse = bs - tau * tau / q;
                const unsigned long long sb = sse_bits(sse);
                if (PASS == 0) { if (sb < pm) pm = sb; }
                else if (__longlong_as_double((long long)sb) <= band) {
                    const unsigned long long key = ((unsigned long long)i * m + j) * m + l;
                    if (key < mine) mine = key;
                }
            }
        }
        if (PASS == 0) {
            pm = wave_min_u64(pm);
            if (lane == 0) w.pmin[it] = __longlong_as_double((long long)pm);
            if (pm < mine) mine = pm;
        }
    }
    block_min_to(mine, &w.best[PASS], PASS == 0 ? nskip : 0, PASS == 0 ? w.skipped : nullptr);
}

// Enumerate tuples with first index i = blockIdx.x.  PASS 0: minimum SSE;
// PASS 1: smallest lexicographic key (i, j, l) with SSE <= band.
template <int D, int PASS>
__device__ inline void l0_enum(int m, double tol, L0Ws w, int i)
{
    __shared__ double inv22[SISSO_MAX_SUBSPACE], z2s[SISSO_MAX_SUBSPACE];
    __shared__ unsigned long long red64[4];
    __shared__ unsigned long long skip_s;
    const double syy = w.scal[1];
    const double bi = w.beta[i];
    const double base = syy - bi * bi;
    double band = 0.0;
    if (PASS == 1) band = __longlong_as_double((long long)w.best[0]) + kTieRel * syy;
    unsigned long long mine = PASS == 0 ? 0x7FF0000000000000ull : ~0ull;
    unsigned long long nskip = 0;
    if (threadIdx.x == 0) skip_s = 0;
    if (D == 1) {
        if (threadIdx.x == 0) {
            const unsigned long long sb = sse_bits(base);
            if (PASS == 0) mine = sb;
            else if (__longlong_as_double((long long)sb) <= band) mine = (unsigned long long)i;
        }
    } else {
        const double *Ci = w.C + (size_t)i * m;
        // per-j quantities of the pair (i, j)
        for (int j = i + 1 + threadIdx.x; j < m; j += blockDim.x) {
            const double cij = Ci[j];
            const double p2 = fma(-cij, cij, 1.0);
            if (p2 > tol) {
                const double l22 = sqrt(p2);
                inv22[j] = 1.0 / l22;
                z2s[j] = (w.beta[j] - cij * bi) / l22;
            } else {
                inv22[j] = 0.0;     // singular pair
                z2s[j] = 0.0;
            }
        }
        __syncthreads();
        if (D == 2) {
            for (int j = i + 1 + threadIdx.x; j < m; j += blockDim.x) {
                if (inv22[j] == 0.0) { nskip++; continue; }
                const double z2 = z2s[j];
                const double sse = fma(-z2, z2, base);
                const unsigned long long sb = sse_bits(sse);
                if (PASS == 0) { if (sb < mine) mine = sb; }
                else if (__longlong_as_double((long long)sb) <= band) {
                    const unsigned long long key = (unsigned long long)i * m + j;
                    if (key < mine) mine = key;
                }
            }
        } else {
            for (int l = i + 2 + threadIdx.x; l < m; l += blockDim.x) {
                const double cil = Ci[l];
                const double bl = w.beta[l];
                const double r1 = fma(-cil, cil, 1.0);
                const double t1 = fma(-cil, bi, bl);
                for (int j = i + 1; j < l; ++j) {
                    const double iv = inv22[j];
                    if (iv == 0.0) { nskip++; continue; }
                    const double cij = Ci[j];
                    const double cjl = w.C[(size_t)j * m + l];
                    const double l32 = fma(-cil, cij, cjl) * iv;
                    const double q = fma(-l32, l32, r1);
                    if (!(q > tol)) { nskip++; continue; }
                    const double z2 = z2s[j];
                    const double tau = fma(-l32, z2, t1);
                    const double sse = fma(-z2, z2, base) - tau * tau / q;
                    const unsigned long long sb = sse_bits(sse);
                    if (PASS == 0) { if (sb < mine) mine = sb; }
                    else if (__longlong_as_double((long long)sb) <= band) {
                        const unsigned long long key = ((unsigned long long)i * m + j) * m + l;
                        if (key < mine) mine = key;
                    }
                }
            }
        }
    }
    // block min, then global atomic min
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(mine, o, 64);
        mine = other < mine ? other : mine;
    }
    if (PASS == 0 && nskip) atomicAdd(&skip_s, nskip);
    if ((threadIdx.x & 63) == 0) red64[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long v = red64[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) v = red64[q] < v ? red64[q] : v;
        atomicMin(&w.best[PASS], v);
        if (PASS == 0 && skip_s) atomicAdd(w.skipped, skip_s);
    }
}

// Decode the best tuple, solve for the coefficients, form the residual.
__device__ inline void l0_finish(const double *__restrict__ F, int ld, int n, int m, int D,
                                 const double *__restrict__ y, double n_tuples, L0Ws w,
                                 int32_t *__restrict__ out_tuple, double *__restrict__ out_sse,
                                 double *__restrict__ out_coef, double *__restrict__ out_resid,
                                 double *__restrict__ out_stats)
{
    __shared__ int tup[SISSO_MAX_D];
    __shared__ double coef[SISSO_MAX_D + 1];
    __shared__ double sse_chosen;
    __shared__ int found;
    __shared__ double red[16];
    if (threadIdx.x == 0) {
        const unsigned long long key = w.best[1];
        found = key != ~0ull;
        if (found) {
            unsigned long long k = key;
            for (int a = D - 1; a >= 0; --a) { tup[a] = (int)(k % (unsigned long long)m); k /= (unsigned long long)m; }
            // normal equations on the unit-diagonal system, Cholesky (D <= 3)
            double A[SISSO_MAX_D][SISSO_MAX_D], b[SISSO_MAX_D], L[SISSO_MAX_D][SISSO_MAX_D], zz[SISSO_MAX_D], c[SISSO_MAX_D];
            for (int a = 0; a < D; ++a) {
                b[a] = w.beta[tup[a]];
                for (int q = 0; q < D; ++q) A[a][q] = w.C[(size_t)tup[a] * m + tup[q]];
            }
            for (int a = 0; a < D; ++a) {
                for (int q = 0; q <= a; ++q) {
                    double s = A[a][q];
                    for (int p = 0; p < q; ++p) s -= L[a][p] * L[q][p];
                    if (a == q) L[a][a] = sqrt(s > 0.0 ? s : 0.0);
                    else L[a][q] = s / L[q][q];
                }
            }
            for (int a = 0; a < D; ++a) {
                double s = b[a];
                for (int p = 0; p < a; ++p) s -= L[a][p] * zz[p];
                zz[a] = s / L[a][a];
            }
            for (int a = D - 1; a >= 0; --a) {
                double s = zz[a];
                for (int p = a + 1; p < D; ++p) s -= L[p][a] * c[p];
                c[a] = s / L[a][a];
            }
            double fit = 0.0;
            for (int a = 0; a < D; ++a) fit += zz[a] * zz[a];
            const double e = w.scal[1] - fit;
            sse_chosen = e > 0.0 ? e : 0.0;            // SSE of the chosen tuple
            double icpt = w.scal[0];
            for (int a = 0; a < D; ++a) {
                const double ca = c[a] / w.norm[tup[a]];
                coef[1 + a] = ca;
                icpt -= ca * w.mean[tup[a]];
            }
            coef[0] = icpt;
        }
    }
    __syncthreads();
    if (!found) {
        for (int t = threadIdx.x; t < n; t += blockDim.x) out_resid[t] = y[t];
        if (threadIdx.x == 0) {
            for (int a = 0; a < D; ++a) out_tuple[a] = -1;
            for (int a = 0; a <= D; ++a) out_coef[a] = 0.0;
            out_sse[0] = INFINITY;
            out_stats[0] = NAN; out_stats[1] = NAN;
            out_stats[2] = n_tuples; out_stats[3] = (double)*w.skipped;
        }
        return;
    }
    double ss = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        double yh = coef[0];
        for (int a = 0; a < D; ++a) yh = fma(coef[1 + a], F[(size_t)tup[a] * ld + t], yh);
        const double r = y[t] - yh;
        out_resid[t] = r;
        ss += w.wt ? w.wt[t] * r * r : r * r;
    }
    const double sst = block_sum(ss, red);
    if (threadIdx.x == 0) {
        for (int a = 0; a < D; ++a) out_tuple[a] = tup[a];
        for (int a = 0; a <= D; ++a) out_coef[a] = coef[a];
        const double sse = sse_chosen;
        out_sse[0] = sse;
        out_stats[0] = w.wt ? sqrt(sst / w.scal[2]) : sqrt(sst / n);
        out_stats[1] = 1.0 - sse / w.scal[1];
        out_stats[2] = n_tuples;
        out_stats[3] = (double)*w.skipped;
    }
}

__host__ __device__ inline double n_choose(int m, int D)
{
    double r = 1.0;
    for (int a = 0; a < D; ++a) r = r * (m - a) / (a + 1);
    return r;
}

// ------------------------------------------------------- one problem

__global__ void __launch_bounds__(256) k_l0_y(const double *__restrict__ y, int n, L0Ws w) { l0_y(y, n, w); }

__global__ void __launch_bounds__(256) k_l0_columns(const double *__restrict__ F, int ld, int n, L0Ws w)
{
    l0_column(F, ld, n, w, blockIdx.x);
}


__global__ void __launch_bounds__(256) k_l0_gram_sum(int m, L0Ws w, int split) { l0_gram_sum(m, w, split, blockIdx.x); }
__global__ void __launch_bounds__(256) k_l0_gram_part64(int m, int n, L0Ws w, int split)
{
    l0_gram_part64(m, n, w, split, blockIdx.x, blockIdx.y);
}

template <int D, int PASS>
__global__ void __launch_bounds__(256) k_l0_enum(int m, double tol, L0Ws w)
{
    l0_enum<D, PASS>(m, tol, w, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_l0_finish(const double *__restrict__ F, int ld, int n, int m, int D,
                                                   const double *__restrict__ y, double n_tuples, L0Ws w,
                                                   int32_t *__restrict__ out_tuple, double *__restrict__ out_sse,
                                                   double *__restrict__ out_coef, double *__restrict__ out_resid,
                                                   double *__restrict__ out_stats)
{
    l0_finish(F, ld, n, m, D, y, n_tuples, w, out_tuple, out_sse, out_coef, out_resid, out_stats);
}

// ------------------------------------------------------- many problems
//
// The same bodies over a table of problems: blockIdx.y (gram: blockIdx.z)
// is the problem; blocks beyond a problem's own extent return at once.

__device__ inline bool l0p_ok(const sisso_l0_problem &P, int D, int m_max, int n_max)
{
    return P.F && P.y && P.out_tuple && P.out_sse && P.out_coef && P.out_resid && P.out_stats && P.ws &&
           P.m >= D && P.m <= m_max && P.n >= 2 && P.n <= n_max && P.ld >= P.n &&
           P.ws_bytes >= (int64_t)l0_ws_bytes(P.m, P.n);
}

__global__ void __launch_bounds__(256) k_l0b_y(const sisso_l0_problem *__restrict__ T, int D, int m_max, int n_max,
                                               int32_t *__restrict__ status)
{
    const sisso_l0_problem P = T[blockIdx.y];
    const bool ok = l0p_ok(P, D, m_max, n_max);
    if (threadIdx.x == 0 && status) status[blockIdx.y] = ok ? SISSO_OK : SISSO_E_SHAPE;
    if (!ok) return;
    l0_y(P.y, P.n, l0_ws_view(P.ws, P.m, P.n));
}

__global__ void __launch_bounds__(256) k_l0b_columns(const sisso_l0_problem *__restrict__ T, int D, int m_max,
                                                     int n_max)
{
    const sisso_l0_problem P = T[blockIdx.y];
    if (!l0p_ok(P, D, m_max, n_max) || (int)blockIdx.x >= P.m) return;
    l0_column(P.F, P.ld, P.n, l0_ws_view(P.ws, P.m, P.n), blockIdx.x);
}

__global__ void __launch_bounds__(256) k_l0b_gram(const sisso_l0_problem *__restrict__ T, int D, int m_max, int n_max)
{
    const sisso_l0_problem P = T[blockIdx.z];
    const int tiles = (P.m + kGT - 1) / kGT;
    if (!l0p_ok(P, D, m_max, n_max) || (int)blockIdx.x >= tiles || (int)blockIdx.y >= tiles) return;
    l0_gram(P.m, P.n, l0_ws_view(P.ws, P.m, P.n), blockIdx.y, blockIdx.x);
}

template <int D, int PASS>
__global__ void __launch_bounds__(256) k_l0b_enum(const sisso_l0_problem *__restrict__ T, int m_max, int n_max,
                                                  double tol)
{
    const sisso_l0_problem P = T[blockIdx.y];
    const int gb = D == 1 ? P.m : P.m - D + 1;
    if (!l0p_ok(P, D, m_max, n_max) || (int)blockIdx.x >= gb) return;
    l0_enum<D, PASS>(P.m, tol, l0_ws_view(P.ws, P.m, P.n), blockIdx.x);
}

__global__ void __launch_bounds__(256) k_l0b_finish(const sisso_l0_problem *__restrict__ T, int D, int m_max,
                                                    int n_max)
{
    const sisso_l0_problem P = T[blockIdx.x];
    if (!l0p_ok(P, D, m_max, n_max)) return;
    l0_finish(P.F, P.ld, P.n, P.m, D, P.y, n_choose(P.m, D), l0_ws_view(P.ws, P.m, P.n), P.out_tuple, P.out_sse,
              P.out_coef, P.out_resid, P.out_stats);
}

}  // namespace sisso

using namespace sisso;

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" sisso_status sisso_l0_outcome(const double *stats)
{
    if (!stats) return SISSO_E_NULL;
    // tuples evaluated == tuples skipped: no admissible model
    return stats[2] >= 1.0 && stats[3] >= stats[2] ? SISSO_E_NUMERIC : SISSO_OK;
}

extern "C" size_t sisso_l0_workspace_size(int32_t m, int32_t n, int32_t D)
{
    if (m < 1 || n < 2 || D < 1) return 0;
    return l0_ws_bytes(m, n);
}


extern "C" sisso_status sisso_l0_search_weighted(const double *F, int32_t m, int32_t ld, int32_t n,
                                                 const double *y, const double *wts, int32_t D, double singular_tol,
                                                 int32_t *out_tuple, double *out_sse, double *out_coef,
                                                 double *out_resid, double *out_stats, void *ws, size_t ws_bytes,
                                                 void *stream)
{
    if (!F || !y || !out_tuple || !out_sse || !out_coef || !out_resid || !out_stats || !ws) return SISSO_E_NULL;
    if (D < 1 || D > SISSO_MAX_D || m < D || m > SISSO_MAX_SUBSPACE || n < 2 || n > SISSO_MAX_N || ld < n)
        return SISSO_E_SHAPE;
    if (!(singular_tol >= 0.0) || singular_tol >= 1.0) return SISSO_E_RANGE;
    if (ws_bytes < l0_ws_bytes(m, n)) return SISSO_E_WORKSPACE;
    hipStream_t st = as_stream(stream);
    L0Ws w = l0_ws_view(ws, m, n);
    w.wt = wts;
    hipLaunchKernelGGL(k_l0_y, dim3(1), dim3(256), 0, st, y, n, w);
    hipLaunchKernelGGL(k_l0_columns, dim3(m), dim3(256), 0, st, F, ld, n, w);
    const int split = l0_gram_split(m, n), gtiles = l0_gram_tiles(m);
    hipLaunchKernelGGL(k_l0_gram_part64, dim3(l0_gram_tiles64(m), split), dim3(256), 0, st, m, n, w, split);
    hipLaunchKernelGGL(k_l0_gram_sum, dim3(gtiles), dim3(256), 0, st, m, w, split);
    const int64_t npairs = (int64_t)m * (m - 1) / 2;
    if (D == 1) {
        hipLaunchKernelGGL((k_l0_enum<1, 0>), dim3(m), dim3(64), 0, st, m, singular_tol, w);
        hipLaunchKernelGGL((k_l0_enum<1, 1>), dim3(m), dim3(64), 0, st, m, singular_tol, w);
    } else if (D == 2) {
        const unsigned g = (unsigned)((npairs + 255) / 256 < 1024 ? (npairs + 255) / 256 : 1024);
        hipLaunchKernelGGL(k_l0_pairs2<0>, dim3(g), dim3(256), 0, st, m, singular_tol, w);
        hipLaunchKernelGGL(k_l0_pairs2<1>, dim3(g), dim3(256), 0, st, m, singular_tol, w);
    } else {
        const int64_t items = l0_items3(m);
        // both passes over the items in 2048 persistent blocks (the tie pass
        // revisits only the few items whose minimum lies within the band)
        const unsigned g = (unsigned)((items + 3) / 4 < 2048 ? (items + 3) / 4 : 2048);
        hipLaunchKernelGGL(k_l0_cols3<0>, dim3(g), dim3(256), 0, st, m, singular_tol, w);
        hipLaunchKernelGGL(k_l0_cols3<1>, dim3(g), dim3(256), 0, st, m, singular_tol, w);
    }
    hipLaunchKernelGGL(k_l0_finish, dim3(1), dim3(256), 0, st, F, ld, n, m, D, y, n_choose(m, D), w, out_tuple,
                       out_sse, out_coef, out_resid, out_stats);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_l0_search(const double *F, int32_t m, int32_t ld, int32_t n, const double *y,
                                        int32_t D, double singular_tol, int32_t *out_tuple, double *out_sse,
                                        double *out_coef, double *out_resid, double *out_stats, void *ws,
                                        size_t ws_bytes, void *stream)
{
    return sisso_l0_search_weighted(F, m, ld, n, y, nullptr, D, singular_tol, out_tuple, out_sse, out_coef,
                                    out_resid, out_stats, ws, ws_bytes, stream);
}

// ------------------------------------------------- allocation-free search
//
// sisso_l0_search with its workspace in a file-scope device array instead of
// a caller-provided buffer.  The array's host-side name is not a device
// address: its address on each device is taken once with hipGetSymbolAddress
// (with that device current) and only that pointer is passed to kernels.

namespace {
constexpr size_t kL0ScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kL0ScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up on the first
// call per device), or nullptr if the runtime reports an error.
void *scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" size_t sisso_l0_scratch_capacity(void) { return kL0ScratchBytes; }

extern "C" sisso_status sisso_l0_search_noalloc(const double *F, int32_t m, int32_t ld, int32_t n, const double *y,
                                                int32_t D, double singular_tol, int32_t *out_tuple, double *out_sse,
                                                double *out_coef, double *out_resid, double *out_stats,
                                                void *stream)
{
    if (!F || !y || !out_tuple || !out_sse || !out_coef || !out_resid || !out_stats) return SISSO_E_NULL;
    if (D < 1 || D > SISSO_MAX_D || m < D || m > SISSO_MAX_SUBSPACE || n < 2 || n > SISSO_MAX_N || ld < n)
        return SISSO_E_SHAPE;
    if (l0_ws_bytes(m, n) > kL0ScratchBytes) return SISSO_E_WORKSPACE;
    void *ws = scratch_on_current_device();
    if (!ws) return SISSO_E_DEVICE;
    return sisso_l0_search(F, m, ld, n, y, D, singular_tol, out_tuple, out_sse, out_coef, out_resid, out_stats, ws,
                           kL0ScratchBytes, stream);
}

extern "C" sisso_status sisso_l0_search_batched(const sisso_l0_problem *problems, int32_t n_problems, int32_t D,
                                                int32_t m_max, int32_t n_max, double singular_tol,
                                                int32_t *out_status, void *stream)
{
    if (!problems) return SISSO_E_NULL;
    if (n_problems < 1 || n_problems > SISSO_MAX_BATCH || D < 1 || D > SISSO_MAX_D || m_max < D ||
        m_max > SISSO_MAX_SUBSPACE || n_max < 2 || n_max > SISSO_MAX_N)
        return SISSO_E_SHAPE;
    if (!(singular_tol >= 0.0) || singular_tol >= 1.0) return SISSO_E_RANGE;
    hipStream_t st = as_stream(stream);
    const unsigned P = (unsigned)n_problems;
    hipLaunchKernelGGL(k_l0b_y, dim3(1, P), dim3(256), 0, st, problems, D, m_max, n_max, out_status);
    hipLaunchKernelGGL(k_l0b_columns, dim3(m_max, P), dim3(256), 0, st, problems, D, m_max, n_max);
    const int tiles = (m_max + kGT - 1) / kGT;
    hipLaunchKernelGGL(k_l0b_gram, dim3(tiles, tiles, P), dim3(256), 0, st, problems, D, m_max, n_max);
    const unsigned gb = (unsigned)(D == 1 ? m_max : m_max - D + 1);
    if (D == 1) {
        hipLaunchKernelGGL((k_l0b_enum<1, 0>), dim3(gb, P), dim3(64), 0, st, problems, m_max, n_max, singular_tol);
        hipLaunchKernelGGL((k_l0b_enum<1, 1>), dim3(gb, P), dim3(64), 0, st, problems, m_max, n_max, singular_tol);
    } else if (D == 2) {
        hipLaunchKernelGGL((k_l0b_enum<2, 0>), dim3(gb, P), dim3(256), 0, st, problems, m_max, n_max, singular_tol);
        hipLaunchKernelGGL((k_l0b_enum<2, 1>), dim3(gb, P), dim3(256), 0, st, problems, m_max, n_max, singular_tol);
    } else {
        hipLaunchKernelGGL((k_l0b_enum<3, 0>), dim3(gb, P), dim3(256), 0, st, problems, m_max, n_max, singular_tol);
        hipLaunchKernelGGL((k_l0b_enum<3, 1>), dim3(gb, P), dim3(256), 0, st, problems, m_max, n_max, singular_tol);
    }
    hipLaunchKernelGGL(k_l0b_finish, dim3(P), dim3(256), 0, st, problems, D, m_max, n_max);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
