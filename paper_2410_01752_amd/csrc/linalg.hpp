// linalg.hpp -- FP64 helpers shared by the subspace update and the SO search:
// column standardisation and a tiled Z_a^T Z_b product.
#pragma once

#include "common.hpp"

namespace sisso {

// Standardise column j of src (n x m, ld): z = (x - mean) / ||x - mean||.
// Writes z (ldz), mean and norm; ok = 0 if the column is constant or has a
// non-finite value (z is then zero).  One block per column.
__device__ inline void standardize_column(const double *x, int n, double *z, double *mean_out,
                                          double *norm_out, int *ok_out, double *red)
{
    double s = 0.0;
    int bad = 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double v = x[t];
        if (!isfinite(v)) bad = 1;
        s += v;
    }
    bad = __syncthreads_or(bad);
    const double mean = block_sum(s, red) / n;
    double ss = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double e = x[t] - mean;
        ss += e * e;
    }
    const double sst = block_sum(ss, red);
    const bool ok = !bad && sst > 0.0;
    const double inv = ok ? 1.0 / sqrt(sst) : 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) z[t] = ok ? (x[t] - mean) * inv : 0.0;
    if (threadIdx.x == 0) {
        if (mean_out) *mean_out = mean;
        if (norm_out) *norm_out = ok ? sqrt(sst) : 0.0;
        if (ok_out) *ok_out = ok ? 1 : 0;
    }
    __syncthreads();
}

// standardize_column under sample weights wt (nullable: the unweighted
// form): weighted mean mu = sum w x / sum w and
// z = sqrt(w) (x - mu) / sqrt(sum w (x - mu)^2), so that z_a . z_b is the
// weighted correlation of two columns (Sec. 2.4: whitening by
// W = Sigma^(-1/2) with the intercept whitened too).  norm_out receives
// sqrt(sum w (x - mu)^2).  Weights must be positive; `ok` also fails for a
// non-finite weight.
__device__ inline void standardize_column_w(const double *x, const double *wt, int n, double *z, double *mean_out,
                                            double *norm_out, int *ok_out, double *red)
{
    if (!wt) {
        standardize_column(x, n, z, mean_out, norm_out, ok_out, red);
        return;
    }
    double s = 0.0, sw = 0.0;
    int bad = 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double v = x[t], w = wt[t];
        if (!isfinite(v) || !isfinite(w)) bad = 1;
        s += w * v;
        sw += w;
    }
    bad = __syncthreads_or(bad);
    const double W = block_sum(sw, red);
    const double mean = block_sum(s, red) / W;
    double ss = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double e = x[t] - mean;
        ss += wt[t] * e * e;
    }
    const double sst = block_sum(ss, red);
    const bool ok = !bad && sst > 0.0;
    const double inv = ok ? 1.0 / sqrt(sst) : 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) z[t] = ok ? sqrt(wt[t]) * (x[t] - mean) * inv : 0.0;
    if (threadIdx.x == 0) {
        if (mean_out) *mean_out = mean;
        if (norm_out) *norm_out = ok ? sqrt(sst) : 0.0;
        if (ok_out) *ok_out = ok ? 1 : 0;
    }
    __syncthreads();
}

constexpr int kGT = 32;    // output tile
constexpr int kGK = 16;    // samples per LDS chunk

// Tile (bi, bj) of Z_a^T Z_b (a: ma columns, b: mb columns, both n x *,
// leading dim ldz) over the samples [kb, ke).  256 threads, 2 x 2 outputs
// each.  Returns the four dot products in acc; rows i = bi*32 + ty*2 + {0,1},
// cols j = bj*32 + tx*2 + {0,1}.
__device__ inline void gemm_tile_tn_range(const double *Za, int ma, const double *Zb, int mb, int kb, int ke,
                                          int ldz, int bi, int bj, double (&acc)[2][2], double (*As)[kGT + 1],
                                          double (*Bs)[kGT + 1])
{
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    acc[0][0] = acc[0][1] = acc[1][0] = acc[1][1] = 0.0;
    for (int k0 = kb; k0 < ke; k0 += kGK) {
        // load 32 columns x 16 samples of each operand: 512 values, 2 per thread
        for (int e = tid; e < kGT * kGK; e += blockDim.x) {
            const int c = e / kGK, t = e % kGK;
            const int ia = bi * kGT + c, ib = bj * kGT + c;
            As[t][c] = (ia < ma && k0 + t < ke) ? Za[(size_t)ia * ldz + k0 + t] : 0.0;
            Bs[t][c] = (ib < mb && k0 + t < ke) ? Zb[(size_t)ib * ldz + k0 + t] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kGK; ++t) {
            const double a0 = As[t][ty * 2], a1 = As[t][ty * 2 + 1];
            const double b0 = Bs[t][tx * 2], b1 = Bs[t][tx * 2 + 1];
            acc[0][0] = fma(a0, b0, acc[0][0]);
            acc[0][1] = fma(a0, b1, acc[0][1]);
            acc[1][0] = fma(a1, b0, acc[1][0]);
            acc[1][1] = fma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
}

// The same over all n samples.
__device__ inline void gemm_tile_tn(const double *Za, int ma, const double *Zb, int mb, int n, int ldz,
                                    int bi, int bj, double (&acc)[2][2], double (*As)[kGT + 1],
                                    double (*Bs)[kGT + 1])
{
    gemm_tile_tn_range(Za, ma, Zb, mb, 0, n, ldz, bi, bj, acc, As, Bs);
}

}  // namespace sisso
