// prescreen.hip -- ranking of the base features before expansion, for problems
// with many primary features (Sec. 3.1, eq. mi-exact; the initial screening
// option of Sec. 3.3 with its two methods):
//   mutual information  the integral of p(x, y) log(p(x, y) / (p(x) p(y))),
//                       estimated by Gaussian kernel densities: both variables
//                       standardised, Silverman bandwidths h_k = (4 / (k + 2))^
//                       (1 / (k + 4)) n^(-1 / (k + 4)) (k = 1 marginals, k = 2
//                       the joint), the integral replaced by the mean over the
//                       observations of the log density ratio, each density
//                       the kernel average over all observations;
//   Spearman            |Pearson correlation| of the ranks (ties share their
//                       average rank);
// and the selection of the best ceil(q d) features by (score desc, index asc).
//
// MI: one block per feature computes, for its samples s, the kernel sums over
// all t of the marginal and the joint kernels (FP32 exponentials of FP64
// arguments, FP64 sums).  The y marginal, common to all features, is computed
// once.  Spearman: one block
// per feature sorts (value, index) pairs in LDS (bitonic) and assigns average
// ranks with two scans; the ranks of y are computed once the same way.
#include "linalg.hpp"

namespace sisso {

constexpr int kPsSortMax = 4096;          // Spearman: samples sorted in LDS
constexpr int kPsSelectMax = 8192;        // features ranked by the selection

__host__ __device__ inline double ps_bandwidth(int n, int k)
{
    return pow(4.0 / (k + 2.0), 1.0 / (k + 4.0)) * pow((double)n, -1.0 / (k + 4.0));
}

// ws: standardised y (n), its marginal densities (n) and its ranks (n);
// standardised features (ldz x d)
struct PsWs {
    double *ys, *py, *ry, *xs;
    int ldz;
};
__host__ __device__ inline size_t ps_ws_bytes(int n, int d)
{
    const size_t ldz = (size_t)((n + 1) & ~1);
    return (3 * ldz + ldz * (size_t)d) * sizeof(double) + 256;
}
__host__ __device__ inline PsWs ps_ws_view(void *p, int n)
{
    PsWs w;
    w.ldz = (n + 1) & ~1;
    double *c = (double *)p;
    w.ys = c; c += w.ldz;
    w.py = c; c += w.ldz;
    w.ry = c; c += w.ldz;
    w.xs = c;
    return w;
}

// standardised copy of a column (zeros for a constant one); flag: constant
__device__ inline void ps_standardise(const double *__restrict__ x, int n, double *__restrict__ z, int *constant)
{
    __shared__ double red[16];
    double s = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) s += x[t];
    const double mean = block_sum(s, red) / n;
    double q = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) q += (x[t] - mean) * (x[t] - mean);
    const double sd = sqrt(block_sum(q, red) / n);
    for (int t = threadIdx.x; t < n; t += blockDim.x) z[t] = sd > 0.0 ? (x[t] - mean) / sd : 0.0;
    if (threadIdx.x == 0 && constant) *constant = !(sd > 0.0);
}

// column c of X (c = d: y) standardised into the workspace
__global__ void __launch_bounds__(256) k_ps_standardise(const double *__restrict__ X, int n, int ldx, int d,
                                                        const double *__restrict__ y, PsWs w, int *__restrict__ flags)
{
    const int c = blockIdx.x;
    const double *src = c < d ? X + (size_t)c * ldx : y;
    double *dst = c < d ? w.xs + (size_t)c * w.ldz : w.ys;
    ps_standardise(src, n, dst, flags + c);
}

// y's marginal density at each observation (kernel average; normalisation
// applied by the MI kernel)
__global__ void __launch_bounds__(256) k_ps_py(int n, PsWs w)
{
    const double h1 = ps_bandwidth(n, 1), c1 = 1.0 / (2.0 * h1 * h1);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        const double ys = w.ys[s];
        double p = 0.0;
        for (int t = 0; t < n; ++t) {
            const double dy = ys - w.ys[t];
            p += (double)__expf((float)(-dy * dy * c1));
        }
        w.py[s] = p / n;
    }
}

// One block per feature: each thread takes samples s and sums the marginal and
// joint kernels over all t (wave-uniform loads of x_t, y_t).  With the
// kernels' normalisations 1 / (sqrt(2 pi) h1) per marginal and
// 1 / (2 pi h2^2) for the joint, log p(x, y) - log p(x) - log p(y) is the log
// ratio of the kernel averages plus 2 log(h1 / h2).
__global__ void __launch_bounds__(256) k_ps_mi(int n, PsWs w, const int *__restrict__ flags, int d,
                                               double *__restrict__ out)
{
    __shared__ double red[16];
    const int c = blockIdx.x;
    const double *x = w.xs + (size_t)c * w.ldz;
    const double h1 = ps_bandwidth(n, 1), h2 = ps_bandwidth(n, 2);
    const double c1 = 1.0 / (2.0 * h1 * h1), c2 = 1.0 / (2.0 * h2 * h2), lk = 2.0 * log(h1 / h2);
    double part = 0.0;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const double xs = x[s], ys = w.ys[s];
        double px = 0.0, pxy = 0.0;
        for (int t = 0; t < n; ++t) {
            const double dx = xs - x[t], dy = ys - w.ys[t];
            const double ex = dx * dx;
            px += (double)__expf((float)(-ex * c1));
            pxy += (double)__expf((float)(-fma(dy, dy, ex) * c2));
        }
        part += log(pxy / n) - log(px / n) - log(w.py[s]) + lk;
    }
    const double mi = block_sum(part, red) / n;
    if (threadIdx.x == 0) out[c] = flags[c] || flags[d] ? 0.0 : mi;
}

// ---------------------------------------------------------------- Spearman

// average ranks (1-based) of x[0..n) into r; one block, n <= kPsSortMax
__device__ inline void ps_ranks(const double *__restrict__ x, int n, double *__restrict__ r, double *key, int *idx,
                                int *lo, int *hi)
{
    const int cap = next_pow2(n > 1 ? n : 2);
    for (int i = threadIdx.x; i < cap; i += blockDim.x) {
        key[i] = i < n ? x[i] : INFINITY;
        idx[i] = i;
    }
    __syncthreads();
    for (int size = 2; size <= cap; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (cap >> 1); t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1)), j = i + stride;
                const bool up = (i & size) == 0;
                const bool j_first = key[j] < key[i] || (key[j] == key[i] && idx[j] < idx[i]);
                if (j_first == up) {
                    const double tk = key[i]; key[i] = key[j]; key[j] = tk;
                    const int ti = idx[i]; idx[i] = idx[j]; idx[j] = ti;
                }
            }
            __syncthreads();
        }
    // run of equal values around each sorted position: first position by a
    // max-scan of run starts, last by a min-scan of run ends
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        lo[p] = (p == 0 || key[p] != key[p - 1]) ? p : 0;
        hi[p] = (p == n - 1 || key[p] != key[p + 1]) ? p : n;
    }
    __syncthreads();
    for (int off = 1; off < n; off <<= 1) {
        int a[kPsSortMax / 256], b[kPsSortMax / 256];
        int m = 0;
        for (int p = threadIdx.x; p < n; p += blockDim.x, ++m) {
            a[m] = p >= off ? max(lo[p], lo[p - off]) : lo[p];
            b[m] = p + off < n ? min(hi[p], hi[p + off]) : hi[p];
        }
        __syncthreads();
        m = 0;
        for (int p = threadIdx.x; p < n; p += blockDim.x, ++m) { lo[p] = a[m]; hi[p] = b[m]; }
        __syncthreads();
    }
    for (int p = threadIdx.x; p < n; p += blockDim.x) r[idx[p]] = 0.5 * (lo[p] + hi[p]) + 1.0;
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_ps_rank_y(const double *__restrict__ y, int n, PsWs w)
{
    __shared__ double key[kPsSortMax];
    __shared__ int idx[kPsSortMax], lo[kPsSortMax], hi[kPsSortMax];
    ps_ranks(y, n, w.ry, key, idx, lo, hi);
}

// one block per feature: |Pearson correlation| of its ranks with y's ranks
__global__ void __launch_bounds__(256) k_ps_spearman(const double *__restrict__ X, int n, int ldx, PsWs w,
                                                     double *__restrict__ out)
{
    __shared__ double key[kPsSortMax], rx[kPsSortMax];
    __shared__ int idx[kPsSortMax], lo[kPsSortMax], hi[kPsSortMax];
    __shared__ double red[16];
    const int c = blockIdx.x;
    ps_ranks(X + (size_t)c * ldx, n, rx, key, idx, lo, hi);
    const double m = 0.5 * (n + 1);            // mean of any set of average ranks
    double sxy = 0.0, sxx = 0.0, syy = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double a = rx[t] - m, b = w.ry[t] - m;
        sxy += a * b; sxx += a * a; syy += b * b;
    }
    sxy = block_sum(sxy, red);
    sxx = block_sum(sxx, red);
    syy = block_sum(syy, red);
    if (threadIdx.x == 0) out[c] = sxx > 0.0 && syy > 0.0 ? fabs(sxy) / sqrt(sxx * syy) : 0.0;
}

// ---------------------------------------------------------------- selection

__global__ void __launch_bounds__(1024) k_ps_select(const double *__restrict__ sc, int d, int keep,
                                                    int32_t *__restrict__ out_idx, int32_t *__restrict__ out_count)
{
    __shared__ double key[kPsSelectMax];
    __shared__ int idx[kPsSelectMax];
    const int cap = next_pow2(d > 1 ? d : 2);
    for (int i = threadIdx.x; i < cap; i += blockDim.x) {
        key[i] = i < d ? sc[i] : -INFINITY;
        idx[i] = i < d ? i : INT32_MAX;
    }
    __syncthreads();
    // descending score, ascending index
    for (int size = 2; size <= cap; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (cap >> 1); t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1)), j = i + stride;
                const bool up = (i & size) == 0;
                const bool j_first = key[j] > key[i] || (key[j] == key[i] && idx[j] < idx[i]);
                if (j_first == up) {
                    const double tk = key[i]; key[i] = key[j]; key[j] = tk;
                    const int ti = idx[i]; idx[i] = idx[j]; idx[j] = ti;
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < keep; i += blockDim.x) out_idx[i] = idx[i];
    if (threadIdx.x == 0) *out_count = keep;
}

}  // namespace sisso

using namespace sisso;

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" size_t sisso_prescreen_workspace_size(int32_t n, int32_t d)
{
    if (n < 2 || d < 1) return 0;
    return ps_ws_bytes(n, d) + (size_t)(d + 1) * sizeof(int) + 256;
}

extern "C" sisso_status sisso_prescreen_scores(const double *X, int32_t n, int32_t ldx, int32_t d, const double *y,
                                               int32_t method, double *out, void *ws, size_t ws_bytes, void *stream)
{
    if (!X || !y || !out || !ws) return SISSO_E_NULL;
    if (n < 2 || d < 1 || ldx < n) return SISSO_E_SHAPE;
    if (method != SISSO_PRESCREEN_MI && method != SISSO_PRESCREEN_SPEARMAN) return SISSO_E_RANGE;
    if (method == SISSO_PRESCREEN_SPEARMAN && n > kPsSortMax) return SISSO_E_UNSUPPORTED;
    if (ws_bytes < sisso_prescreen_workspace_size(n, d)) return SISSO_E_WORKSPACE;
    hipStream_t st = as_stream(stream);
    PsWs w = ps_ws_view(ws, n);
    int *flags = (int *)((char *)ws + ps_ws_bytes(n, d));
    if (method == SISSO_PRESCREEN_MI) {
        hipLaunchKernelGGL(k_ps_standardise, dim3(d + 1), dim3(256), 0, st, X, n, ldx, d, y, w, flags);
        hipLaunchKernelGGL(k_ps_py, dim3((n + 255) / 256), dim3(256), 0, st, n, w);
        hipLaunchKernelGGL(k_ps_mi, dim3(d), dim3(256), 0, st, n, w, flags, d, out);
    } else {
        hipLaunchKernelGGL(k_ps_rank_y, dim3(1), dim3(256), 0, st, y, n, w);
        hipLaunchKernelGGL(k_ps_spearman, dim3(d), dim3(256), 0, st, X, n, ldx, w, out);
    }
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_prescreen_select(const double *scores, int32_t d, double quantile, int32_t *out_idx,
                                               int32_t *out_count, void *stream)
{
    if (!scores || !out_idx || !out_count) return SISSO_E_NULL;
    if (d < 1 || d > kPsSelectMax) return SISSO_E_SHAPE;
    if (!(quantile > 0.0) || quantile > 1.0) return SISSO_E_RANGE;
    double kq = ceil(quantile * d - 1e-12);
    const int keep = kq < 1.0 ? 1 : (kq > d ? d : (int)kq);
    hipLaunchKernelGGL(k_ps_select, dim3(1), dim3(1024), 0, as_stream(stream), scores, d, keep, out_idx, out_count);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
