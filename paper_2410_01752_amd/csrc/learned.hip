// learned.hip -- a learned proposal that prunes the one-sided rung-3 slice
// before exact SIS scoring (Sec. 2.2 scores every candidate; here a small
// network ranks the candidates op(u, v) and only those it ranks in the top
// fraction are scored exactly, with the FP32 path's arithmetic).
//
// Operand encoding enc(x), 64 values per pool column: one-hot classes of the
// column's operator and of its two operands (base feature, one of the 12
// operators, or none), then statistics against the residual: corr(x, r),
// |corr(x, r)|, corr(1/x, r), corr(log|x|, r), corr(x^2, r), |corr(1/x, r)|,
// |corr(log|x|, r)|, clip(log10(sd/|mean|), -4, 4)/4, clip(skew, -10, 10)/10,
// clip(log10|mean|, -6, 6)/6, clip(log10 sd, -6, 6)/6, [min > 0], [has a
// zero], 1; the rest 0.  Undefined or non-finite statistics are 0.
//
// Network (two layers, 256 hidden ReLU units): input x = [enc(u) | enc(v) |
// onehot(form) | 0] (144 values), z = W1 x + b1, s = w2 . relu(z) + b2.  The
// input products run on BF16 matrix cores (v_mfma_f32_32x32x16_bf16) with
// FP32 accumulation; everything else is FP32.  Training: weighted squared
// error against atanh(|corr|), Adam on FP32 master weights.
//
// Pruned screening factorises the first layer over the candidate's tree:
// W1 x = A_u + B_v + c_form with A_u = W1[:, 0:64] enc(u) and B_v =
// W1[:, 64:128] enc(v) computed once per residual as GEMMs over the pool
// columns.  Per (u, v) tile of 32 x 32 pairs a block evaluates the network on
// all 5120 candidates from LDS-resident A and B rows, collects those with
// s >= tau (tau: a quantile of s on a uniform sample of the slice) and scores
// only those exactly, staging the operand sample chunks through LDS as the
// plain FP32 kernel does and repeating its arithmetic per candidate, so every
// kept score is bit-identical to the exhaustive one.
#include "tiles.hpp"

namespace sisso {

constexpr int kE = 64;                                  // operand encoding width
constexpr int kIn = 144;                                // network input width
constexpr int kH = 256;                                 // hidden units
constexpr int kOffB1 = kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH;
constexpr int kParams = kOffB2 + 1;
constexpr int kTab = 5 * kH + kH + 1;                   // c_form rows, w2, b2
constexpr int kPS = kH + 4;                             // row stride of FP32 rows
constexpr int kPH = kH / 2 + 4;                         // LDS row stride of A / B rows (FP16 pairs)

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ int op_class(int op) { return op < 0 ? 0 : 1 + op; }

__device__ __forceinline__ float corr_of(double A, double B, double C, double nd, double R1, double Srr)
{
    const double var = B - A * (A / nd);
    if (!(var > 0.0) || !(Srr > 0.0)) return 0.0f;
    const double c = (C - A * (R1 / nd)) / sqrt(var * Srr);
    return isfinite(c) ? (float)c : 0.0f;
}

__device__ __forceinline__ float clipf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// ------------------------------------------------------------- encoding

// One wave per pool column c in [c_begin, c_end); row c - c_begin of enc.
__global__ void __launch_bounds__(256) k_encode(sisso_space s, int n, const float *__restrict__ pool32, int64_t ld32,
                                                const sisso_colstat *__restrict__ stats, const float *__restrict__ r32,
                                                const sisso_resid_info *__restrict__ info, int64_t c_begin,
                                                int64_t c_end, float *__restrict__ enc)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const double nd = (double)n, R1 = info->sum_r32, Srr = info->s_rr;
    for (int64_t c = c_begin + wave; c < c_end; c += nwaves) {
        const sisso_colstat st = stats[c];
        const float *col = pool32 + (size_t)c * ld32;
        const bool zero = st.minabs == 0.0f;
        const float mu = st.mean;
        // shifts of 1/x, log|x| and x^2: their means over the first 256 samples
        float sh[3];
        {
            const int t = lane * 4;
            float4 fv = make_float4(1, 1, 1, 1);
            if (t < n) fv = *reinterpret_cast<const float4 *>(col + t);
            const float fa[4] = {fv.x, fv.y, fv.z, fv.w};
            float p[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < n) {
                    const float x = fa[e];
                    p[0] += zero ? 0.f : __builtin_amdgcn_rcpf(x);
                    p[1] += zero ? 0.f : logf(fabsf(x));
                    p[2] += x * x;
                }
            const int cnt = n < 256 ? n : 256;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const float v = (float)(wave_sum((double)p[q]) / cnt);
                sh[q] = isfinite(v) ? v : 0.f;
            }
        }
        float a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0}, cc[4] = {0, 0, 0, 0}, m3 = 0.f;
        for (int t = lane * 4; t < n; t += 256) {
            const float4 fv = *reinterpret_cast<const float4 *>(col + t);
            const float4 rv = *reinterpret_cast<const float4 *>(r32 + t);
            const float fa[4] = {fv.x, fv.y, fv.z, fv.w};
            const float ra[4] = {rv.x, rv.y, rv.z, rv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (t + e < n) {
                    const float x = fa[e], r = ra[e];
                    const float g[4] = {x - mu, zero ? 0.f : __builtin_amdgcn_rcpf(x) - sh[0],
                                        zero ? 0.f : logf(fabsf(x)) - sh[1], x * x - sh[2]};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        a[q] += g[q];
                        b[q] = fmaf(g[q], g[q], b[q]);
                        cc[q] = fmaf(g[q], r, cc[q]);
                    }
                    m3 = fmaf(g[0] * g[0], g[0], m3);
                }
            }
        }
        double A[4], B[4], C[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            A[q] = wave_sum((double)a[q]);
            B[q] = wave_sum((double)b[q]);
            C[q] = wave_sum((double)cc[q]);
        }
        const double M3 = wave_sum((double)m3);
        float sv[14];
        const float c1 = corr_of(A[0], B[0], C[0], nd, R1, Srr);
        const float c2 = zero ? 0.f : corr_of(A[1], B[1], C[1], nd, R1, Srr);
        const float c3 = zero ? 0.f : corr_of(A[2], B[2], C[2], nd, R1, Srr);
        const float c4 = corr_of(A[3], B[3], C[3], nd, R1, Srr);
        // moments about the exact mean from the sums about mu
        const double dlt = A[0] / nd;
        const double var = B[0] / nd - dlt * dlt;
        const double sd = var > 0.0 ? sqrt(var) : 0.0;
        const double m3c = M3 / nd - 3.0 * dlt * (B[0] / nd) + 2.0 * dlt * dlt * dlt;
        const double skew = sd > 0.0 ? m3c / (sd * sd * sd) : 0.0;
        const double mean = (double)mu + dlt, am = fabs(mean);
        sv[0] = c1; sv[1] = fabsf(c1); sv[2] = c2; sv[3] = c3; sv[4] = c4; sv[5] = fabsf(c2); sv[6] = fabsf(c3);
        sv[7] = am > 0.0 ? clipf((float)log10(sd / am), -4.f, 4.f) / 4.f : 1.0f;
        if (sd == 0.0) sv[7] = am > 0.0 ? -1.0f : 1.0f;
        sv[8] = clipf((float)skew, -10.f, 10.f) / 10.f;
        sv[9] = am > 0.0 ? clipf((float)log10(am), -6.f, 6.f) / 6.f : -1.0f;
        sv[10] = sd > 0.0 ? clipf((float)log10(sd), -6.f, 6.f) / 6.f : -1.0f;
        sv[11] = st.minval > 0.0f ? 1.f : 0.f;
        sv[12] = zero ? 1.f : 0.f;
        sv[13] = 1.f;
        // operator classes of the column and of its operands
        int op, cls[3];
        int64_t l, r;
        decode_id(s, c, &op, &l, &r);
        cls[0] = op_class(op);
        if (op < 0) {
            cls[1] = cls[2] = 13;
        } else {
            int o2;
            int64_t x1, x2;
            decode_id(s, l, &o2, &x1, &x2);
            cls[1] = op_class(o2);
            if (r >= 0) {
                decode_id(s, r, &o2, &x1, &x2);
                cls[2] = op_class(o2);
            } else {
                cls[2] = 13;
            }
        }
        float v = 0.f;
        if (lane < 42) {
            const int slotc = lane / 14;
            const int want = slotc == 0 ? cls[0] : (slotc == 1 ? cls[1] : cls[2]);
            v = (lane - slotc * 14) == want ? 1.f : 0.f;
        }
        else if (lane < 56) {
#pragma unroll
            for (int q = 0; q < 14; ++q)
                if (lane == 42 + q) v = sv[q];
        }
        enc[(size_t)(c - c_begin) * kE + lane] = isfinite(v) ? v : 0.f;
    }
}

// Network input rows of candidate ids of the slice's binary block (one wave
// per id); an id outside the block gives a zero row.
__global__ void __launch_bounds__(256) k_inputs(sisso_space s, FormSlots fs, const float *__restrict__ enc,
                                                const int64_t *__restrict__ ids, int count, float *__restrict__ X)
{
    const int lane = threadIdx.x & 63;
    const int q = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (q >= count) return;
    const int Lv = s.levels;
    const int64_t binbase = s.pool[Lv] + s.rect_unary, vcount = s.pool[Lv - 1];
    const int64_t id = ids[q];
    float *row = X + (size_t)q * kIn;
    int k = -1;
    int64_t u = 0, v = 0;
    if (s.rect == 1 && id >= binbase && id < s.total) {
        const int64_t loc = id - binbase, pair = loc / s.n_slots;
        const int slot = (int)(loc % s.n_slots);
        u = s.pool[Lv - 1] + pair / vcount;
        v = pair % vcount;
        for (int f = 0; f < 5; ++f)
            if (fs.slot[f] == slot) k = f;
    }
    if (k < 0) {
        row[lane] = 0.f;
        row[64 + lane] = 0.f;
        if (lane < 16) row[128 + lane] = 0.f;
        return;
    }
    row[lane] = enc[(size_t)u * kE + lane];
    row[64 + lane] = enc[(size_t)v * kE + lane];
    if (lane < 16) row[128 + lane] = lane == k ? 1.f : 0.f;
}

// Exact FP32 scores of an id list (one thread per id; -1 = invalid).
__global__ void __launch_bounds__(256) k_score_ids(sisso_space s, FormSlots fs, int n, const float *__restrict__ pool32,
                                                   int64_t ld32, const sisso_colstat *__restrict__ stats,
                                                   const float *__restrict__ r32,
                                                   const sisso_resid_info *__restrict__ info,
                                                   const int64_t *__restrict__ ids, int count, float *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) out[q] = score_slice_id(s, fs, n, pool32, ld32, stats, r32, info, ids[q]);
}

// --------------------------------------------------------------- GEMM

// C[i][j] = sum_k A(i, k) B(j, k) (+ bias[j]) for i < M, j < N, with
// A(i, k) = A[i*sai + k*sak], B(j, k) = B[j*sbj + k*sbk] (FP32, rounded to BF16
// when staged), FP32 accumulation.  Block: 4 waves over a 64 x 64 tile of C,
// each wave one 32 x 32 MFMA accumulator; K in steps of 16.  grid.x: M tiles,
// grid.y: N tiles.
__global__ void __launch_bounds__(256) k_gemm_bf16(int64_t M, int N, int K, const float *__restrict__ A, int64_t sai,
                                                   int64_t sak, const float *__restrict__ B, int64_t sbj,
                                                   int64_t sbk, const float *__restrict__ bias, float *__restrict__ C,
                                                   int64_t ldc)
{
    __shared__ __attribute__((aligned(16))) __bf16 sA[64 * 24];
    __shared__ __attribute__((aligned(16))) __bf16 sB[64 * 24];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid * 4 + q, row = e >> 4, kk = e & 15;
            const int k = k0 + kk;
            const int64_t i = i0 + row;
            const int j = j0 + row;
            const float av = (i < M && k < K) ? A[i * sai + (int64_t)k * sak] : 0.f;
            const float bv = (j < N && k < K) ? B[(int64_t)j * sbj + (int64_t)k * sbk] : 0.f;
            sA[row * 24 + kk] = (__bf16)av;
            sB[row * 24 + kk] = (__bf16)bv;
        }
        __syncthreads();
        const int koff = (lane >> 5) * 8;
        const bf16x8 af = *reinterpret_cast<const bf16x8 *>(sA + (wm * 32 + (lane & 31)) * 24 + koff);
        const bf16x8 bfr = *reinterpret_cast<const bf16x8 *>(sB + (wn * 32 + (lane & 31)) * 24 + koff);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bfr, acc, 0, 0, 0);
        __syncthreads();
    }
    const int j = j0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = i0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i < M && j < N) C[i * ldc + j] = acc[r] + (bias ? bias[j] : 0.f);
    }
}

// ------------------------------------------------------------ training

// s_i = w2 . relu(z_i) + b2 (one wave per row).
__global__ void __launch_bounds__(256) k_mlp_out(const float *__restrict__ Z, const float *__restrict__ P, int batch,
                                                 float *__restrict__ s)
{
    const int lane = threadIdx.x & 63;
    const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (i >= batch) return;
    const float4 z = *reinterpret_cast<const float4 *>(Z + (size_t)i * kH + lane * 4);
    const float4 w = *reinterpret_cast<const float4 *>(P + kOffW2 + lane * 4);
    float acc = fmaxf(z.x, 0.f) * w.x;
    acc = fmaf(fmaxf(z.y, 0.f), w.y, acc);
    acc = fmaf(fmaxf(z.z, 0.f), w.z, acc);
    acc = fmaf(fmaxf(z.w, 0.f), w.w, acc);
    const double tot = wave_sum((double)acc);
    if (lane == 0) s[i] = (float)(tot + (double)P[kOffB2]);
}

struct MlpWs {
    double wsum, loss;
    float *ds;          // batch
    float *dz;          // batch x kH
};

__host__ __device__ inline size_t mlp_ws_bytes(int batch)
{
    return 256 + align256((size_t)batch * sizeof(float)) + align256((size_t)batch * kH * sizeof(float));
}

__host__ __device__ inline MlpWs *mlp_ws(void *ws) { return (MlpWs *)ws; }
__host__ __device__ inline float *mlp_ds(void *ws) { return (float *)((char *)ws + 256); }
__host__ __device__ inline float *mlp_dz(void *ws, int batch)
{
    return (float *)((char *)ws + 256 + align256((size_t)batch * sizeof(float)));
}

// Weighted loss sum w (s - t)^2 / sum w and sum w (one block).
__global__ void __launch_bounds__(1024) k_mlp_loss(const float *__restrict__ s, const float *__restrict__ t,
                                                   const float *__restrict__ w, int batch, void *ws,
                                                   float *__restrict__ loss)
{
    __shared__ double red[16];
    double sw = 0.0, sl = 0.0;
    for (int i = threadIdx.x; i < batch; i += blockDim.x) {
        const double e = (double)s[i] - (double)t[i];
        sw += (double)w[i];
        sl += (double)w[i] * e * e;
    }
    const double W = block_sum(sw, red);
    const double Ls = block_sum(sl, red);
    if (threadIdx.x == 0) {
        mlp_ws(ws)->wsum = W;
        mlp_ws(ws)->loss = W > 0.0 ? Ls / W : 0.0;
        if (loss) *loss = W > 0.0 ? (float)(Ls / W) : 0.f;
    }
}

// ds_i = 2 w_i (s_i - t_i) / sum w;  dz_ij = ds_i w2_j [z_ij > 0] (one wave per row).
__global__ void __launch_bounds__(256) k_mlp_dz(const float *__restrict__ Z, const float *__restrict__ P,
                                                const float *__restrict__ s, const float *__restrict__ t,
                                                const float *__restrict__ w, int batch, void *ws)
{
    const int lane = threadIdx.x & 63;
    const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (i >= batch) return;
    const double W = mlp_ws(ws)->wsum;
    const float ds = W > 0.0 ? (float)(2.0 * (double)w[i] * ((double)s[i] - (double)t[i]) / W) : 0.f;
    const float4 z = *reinterpret_cast<const float4 *>(Z + (size_t)i * kH + lane * 4);
    const float4 w2 = *reinterpret_cast<const float4 *>(P + kOffW2 + lane * 4);
    float4 d;
    d.x = z.x > 0.f ? ds * w2.x : 0.f;
    d.y = z.y > 0.f ? ds * w2.y : 0.f;
    d.z = z.z > 0.f ? ds * w2.z : 0.f;
    d.w = z.w > 0.f ? ds * w2.w : 0.f;
    *reinterpret_cast<float4 *>(mlp_dz(ws, batch) + (size_t)i * kH + lane * 4) = d;
    if (lane == 0) mlp_ds(ws)[i] = ds;
}

// db1_j = sum_i dz_ij, dw2_j = sum_i ds_i relu(z_ij), db2 = sum_i ds_i (FP64
// sums in row order; thread j of one block).
__global__ void __launch_bounds__(256) k_mlp_colsums(const float *__restrict__ Z, int batch, void *ws,
                                                     float *__restrict__ G)
{
    const int j = threadIdx.x;
    const float *dz = mlp_dz(ws, batch), *ds = mlp_ds(ws);
    double sb = 0.0, sw = 0.0, s2 = 0.0;
    // the rows in order; each group's loads are issued before its sums
    constexpr int U = 16;
    int i = 0;
    for (; i + U <= batch; i += U) {
        float a[U], b[U], c[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            a[q] = dz[(size_t)(i + q) * kH + j];
            b[q] = ds[i + q];
            c[q] = Z[(size_t)(i + q) * kH + j];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            sb += (double)a[q];
            sw += (double)b[q] * (double)fmaxf(c[q], 0.f);
            s2 += (double)b[q];
        }
    }
    for (; i < batch; ++i) {
        sb += (double)dz[(size_t)i * kH + j];
        sw += (double)ds[i] * (double)fmaxf(Z[(size_t)i * kH + j], 0.f);
        s2 += (double)ds[i];
    }
    G[kOffB1 + j] = (float)sb;
    G[kOffW2 + j] = (float)sw;
    if (j == 0) G[kOffB2] = (float)s2;
}

// Adam with bias-corrected moments (element per thread).
__global__ void __launch_bounds__(256) k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, int64_t count, float lr, float beta1, float beta2,
                                              float eps, float c1, float c2)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float gg = g[e];
    const float mm = beta1 * m[e] + (1.f - beta1) * gg;
    const float vv = beta2 * v[e] + (1.f - beta2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ----------------------------------------------------------- inference

// tables: c_form rows (5 x kH): BF16-rounded W1 column 128 + form plus b1;
// then w2 (kH) and b2.
__global__ void __launch_bounds__(256) k_mlp_tables(const float *__restrict__ P, float *__restrict__ tab)
{
    const int j = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 5; ++k) tab[k * kH + j] = (float)(__bf16)P[j * kIn + 2 * kE + k] + P[kOffB1 + j];
    tab[5 * kH + j] = P[kOffW2 + j];
    if (j == 0) tab[6 * kH] = P[kOffB2];
}

// The network score is evaluated in packed FP16 (two hidden units per
// instruction): the FP32 parts are rounded toward zero to FP16 pairs, then per
// pair t = a + b, z = t + c_form, h = max(z, 0), and the FP32 score accumulates
// h . w2 with a two-term dot product, pairs in ascending order.  The sampler
// and the pruned kernel perform this same instruction sequence per candidate.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __fp16 hp2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2 to_h2(float a, float b) { return __builtin_bit_cast(h2, __builtin_amdgcn_cvt_pkrtz(a, b)); }

__device__ __forceinline__ float net_step(h2 a, h2 b, h2 c, h2 w, float acc)
{
    const h2 z = (a + b) + c;
    const h2 h = __builtin_elementwise_max(z, (h2){(_Float16)0.0f, (_Float16)0.0f});
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(hp2, h), __builtin_bit_cast(hp2, w), acc, false);
}

// Network score of one candidate from its FP32 parts (sampler order).
__device__ __forceinline__ float net_score(const float *__restrict__ a, const float *__restrict__ b,
                                           const float *__restrict__ c, const float *__restrict__ w2, float b2)
{
    float acc = 0.f;
    for (int j = 0; j < kH; j += 2)
        acc = net_step(to_h2(a[j], a[j + 1]), to_h2(b[j], b[j + 1]), to_h2(c[j], c[j + 1]), to_h2(w2[j], w2[j + 1]),
                       acc);
    return acc + b2;
}

// Network scores of slice binary ids (thread per id; -inf outside the block).
__global__ void __launch_bounds__(256) k_mlp_score_ids(sisso_space s, FormSlots fs, const float *__restrict__ Au,
                                                       const float *__restrict__ Bv, const float *__restrict__ tab,
                                                       const int64_t *__restrict__ ids, int count,
                                                       float *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const int Lv = s.levels;
    const int64_t binbase = s.pool[Lv] + s.rect_unary, vcount = s.pool[Lv - 1];
    const int64_t id = ids[q];
    float sc = -INFINITY;
    if (s.rect == 1 && id >= binbase && id < s.total) {
        const int64_t loc = id - binbase, pair = loc / s.n_slots;
        const int slot = (int)(loc % s.n_slots);
        const int64_t ui = pair / vcount, v = pair % vcount;
        int k = -1;
        for (int f = 0; f < 5; ++f)
            if (fs.slot[f] == slot) k = f;
        if (k >= 0) sc = net_score(Au + (size_t)ui * kH, Bv + (size_t)v * kH, tab + k * kH, tab + 5 * kH, tab[6 * kH]);
    }
    out[q] = sc;
}

// Tail agreement of the proposal on a uniform sample: out[0] = number of
// sample ids whose exact score is >= *exact_thr, out[1] = how many of those
// have a network score >= *net_thr (one block; deterministic integer counts).
__global__ void __launch_bounds__(1024) k_count_pass(const float *__restrict__ exact, const float *__restrict__ net,
                                                     int count, const float *__restrict__ exact_thr,
                                                     const float *__restrict__ net_thr, int32_t *__restrict__ out)
{
    __shared__ int c0, c1;
    if (threadIdx.x == 0) { c0 = 0; c1 = 0; }
    __syncthreads();
    const float te = *exact_thr, tn = *net_thr;
    int a = 0, b = 0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        if (exact[i] >= te && exact[i] >= 0.0f) {
            ++a;
            if (net[i] >= tn) ++b;
        }
    }
    atomicAdd(&c0, a);
    atomicAdd(&c1, b);
    __syncthreads();
    if (threadIdx.x == 0) { out[0] = c0; out[1] = c1; }
}

// Order-preserving key of a float (NaN lowest).
__device__ __forceinline__ unsigned fkey(float f)
{
    if (isnan(f)) return 0u;
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_float(unsigned k)
{
    const unsigned u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
}

// q-th largest value (1-based) of x[0..count) by radix selection on the keys,
// 8 bits per pass (one block).
__global__ void __launch_bounds__(1024) k_select_kth(const float *__restrict__ x, int count, int q,
                                                     float *__restrict__ out)
{
    __shared__ unsigned hist[256];
    __shared__ unsigned s_prefix;
    __shared__ int s_need;
    if (threadIdx.x == 0) { s_prefix = 0u; s_need = q; }
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
        const unsigned pre = s_prefix;
        const unsigned mask = pass == 0 ? 0u : (0xFFFFFFFFu << (shift + 8));
        for (int e = threadIdx.x; e < count; e += blockDim.x) {
            const unsigned k = fkey(x[e]);
            if ((k & mask) == (pre & mask)) atomicAdd(&hist[(k >> shift) & 0xFFu], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int need = s_need, b = 255;
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
    if (threadIdx.x == 0) *out = key_float(s_prefix);
}

// Pruned screening of the slice's binary block (see the file comment).  A
// work item is a u tile of 32 operands times a v span of up to kVS operands
// (kVS / 32 sub-tiles).  Phase 1 evaluates the network on every candidate of
// the item, one 32 x 32 sub-tile at a time (A rows of the u tile and B rows of
// the sub-tile in LDS), and appends the passing ones to an LDS list.  Phase 2
// scores the list exactly: sample chunks of the item's raw operand columns
// (32 u + up to kVS v) and of r are staged through LDS with a register
// prefetch of the next chunk; each thread carries up to KPT candidates.  A full
// list is scored before phase 1 continues.
constexpr int kVS = 256;                      // v operands per work item
constexpr int kKeptCap = 8192;                // kept-list entries per block
constexpr int kSP = 32 + kVS + 4;             // LDS row stride of the staged chunk
constexpr int kStageFloats = kSC * kSP + kSC; // staged u/v values + r
constexpr int kRegion = kStageFloats > 32 * kPH ? kStageFloats : 32 * kPH;   // floats (a pair is 4 bytes)

template <int KPT>
__global__ void __launch_bounds__(256) k_score_pruned(
    sisso_space s, FormSlots fs, int n, const float *__restrict__ pool32, int64_t ld32,
    const sisso_colstat *__restrict__ stats, const float *__restrict__ r32,
    const sisso_resid_info *__restrict__ info, const int64_t *__restrict__ excl, int n_excl,
    const float *__restrict__ Au, const float *__restrict__ Bv, const float *__restrict__ tab,
    const float *__restrict__ tau_p, int64_t ut_lo, int64_t ut_hi, int64_t id_begin, int64_t id_end, int list_base,
    void *ws, int lists_total, int keep, int cap, unsigned long long *__restrict__ kept_total)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    h2 *sA = (h2 *)smem;                       // 32 x kPH pairs
    float *sR = (float *)(sA + 32 * kPH);      // B rows of a sub-tile (pairs), or the staged chunk
    h2 *sB = (h2 *)sR;
    h2 *sC = (h2 *)(sR + kRegion);             // 5 x kH/2 form rows, then w2
    unsigned short *kl = (unsigned short *)(sC + 3 * kH);
    float *lsc = (float *)(kl + kKeptCap);
    int64_t *lid = (int64_t *)(lsc + cap);
    __shared__ int lcnt, nkept, nuc, nvc;
    __shared__ float lthr;
    // operand columns referenced by the kept list (bitmaps), and their compact
    // staging order: u columns first, then v columns
    __shared__ unsigned ubits, vbits[kVS / 32], vpre[kVS / 32];
    __shared__ unsigned char umap[32], vmap[kVS];
    __shared__ short clist[32 + kVS];
    WsView W = ws_view(ws, lists_total, keep);
    BlockList L{lsc, lid, &lcnt, &lthr, cap, keep};
    list_init(L);

    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    for (int e = tid; e < 3 * kH; e += 256) sC[e] = to_h2(tab[2 * e], tab[2 * e + 1]);
    if (tid == 0) { nkept = 0; ubits = 0u; }
    if (tid < kVS / 32) vbits[tid] = 0u;
    const float b2 = tab[6 * kH], tau = *tau_p;
    const int Lv = s.levels;
    const int64_t vcount = s.pool[Lv - 1], ulo = s.pool[Lv - 1], uhi = s.pool[Lv];
    const int64_t binbase = s.pool[Lv] + s.rect_unary;
    const int S = s.n_slots;
    const double nd = (double)n, R1 = info->sum_r32, Srr = info->s_rr;
    const int nch = (n + kSC - 1) / kSC;
    const int64_t nvs = (vcount + kVS - 1) / kVS;
    unsigned long long kept_local = 0;

    // exact FP32 scores of the kept list of item (u0, vb, ve)
    auto exact = [&](int64_t u0, int64_t vb, int64_t ve) {
        const int nk = nkept;
        // compact staging order of the referenced columns
        if (tid == 0) {
            unsigned acc = __popc(ubits);
            nuc = (int)acc;
            for (int w = 0; w < kVS / 32; ++w) { vpre[w] = acc; acc += __popc(vbits[w]); }
            nvc = (int)acc - nuc;
        }
        __syncthreads();
        if (tid < 32) {
            const unsigned below = ubits & ((1u << tid) - 1u);
            umap[tid] = (unsigned char)__popc(below);
            if ((ubits >> tid) & 1u) clist[__popc(below)] = (short)tid;
        }
        if (tid < kVS) {
            const int w = tid >> 5, b = tid & 31;
            const unsigned below = vbits[w] & ((1u << b) - 1u);
            const int rank = (int)vpre[w] + __popc(below);          // includes the u columns
            vmap[tid] = (unsigned char)(rank - nuc);
            if ((vbits[w] >> b) & 1u) clist[rank] = (short)(32 + tid);
        }
        __syncthreads();
        const int ncols = nuc + nvc;
        if (tid == 0) kept_local += (unsigned long long)nk;
        float *St = sR;
        const float *Rr = sR + kSC * kSP;
        for (int p0 = 0; p0 < nk; p0 += 256 * KPT) {
            // candidates e = p0 + tid + 256 i; imax is uniform over the wave
            const int wave0 = tid & ~63;
            const int imax_w = (nk - p0 - wave0 + 255) / 256;
            const int imax = __builtin_amdgcn_readfirstlane(imax_w < KPT ? imax_w : KPT);
            int ul[KPT], vl[KPT], kf[KPT], ax[KPT], ay[KPT];
            bool has[KPT], rc[KPT], ad[KPT];
            float mx[KPT], my[KPT], sg[KPT];
#pragma unroll
            for (int i = 0; i < KPT; ++i) {
                const int e = p0 + tid + 256 * i;
                has[i] = e < nk;
                const unsigned code = has[i] ? kl[e] : 0u;
                ul[i] = code & 31;
                vl[i] = (code >> 5) & 255;
                kf[i] = (code >> 13) & 7;
                // form k from two staged values x, y (LDS offsets ax, ay):
                //   k < 2:  (x - mean_u) +- (y - mean_v)   (x = u, y = v)
                //   k >= 2: fma(x, y', -c), (x, y') = (u, v), (u, 1/v), (v, 1/u) for k = 2, 3, 4
                const bool sw = kf[i] == 4;
                const int cu = umap[ul[i]], cv = nuc + vmap[vl[i]];
                ax[i] = sw ? cv : cu;
                ay[i] = sw ? cu : cv;
                rc[i] = kf[i] >= 3;
                ad[i] = kf[i] < 2;
                sg[i] = kf[i] == 1 ? -1.0f : 1.0f;
                mx[i] = has[i] ? stats[u0 + ul[i]].mean : 0.f;
                my[i] = has[i] ? stats[vb + vl[i]].mean : 0.f;
            }
            float cc[KPT], fA[KPT], fB[KPT], fC[KPT];
            double dB[KPT], dC[KPT];
#pragma unroll
            for (int i = 0; i < KPT; ++i) {
                cc[i] = 0.f;
                fA[i] = fB[i] = fC[i] = 0.f;
                dB[i] = dC[i] = 0.0;
            }
            // staging roles: float4 q of this thread covers column e / 8, samples 4 (e % 8) ..
            constexpr int NQ = ((32 + kVS) * (kSC / 4) + 255) / 256;
            float4 pf[NQ];
            float4 pr = make_float4(0, 0, 0, 0);
            auto load = [&](int ch) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int e = q * 256 + tid, col = e >> 3, quad = e & 7;
                    const int t0 = ch * kSC + quad * 4;
                    int64_t c = -1;
                    if (col < ncols) {
                        const int src = clist[col];
                        if (src < 32) { if (u0 + src < uhi) c = u0 + src; }
                        else if (vb + (src - 32) < ve) c = vb + (src - 32);
                    }
                    pf[q] = (c >= 0 && t0 < n) ? *reinterpret_cast<const float4 *>(pool32 + (size_t)c * ld32 + t0)
                                               : make_float4(0, 0, 0, 0);
                }
                if (tid < kSC / 4) {
                    const int tr = ch * kSC + tid * 4;
                    pr = tr < n ? *reinterpret_cast<const float4 *>(r32 + tr) : make_float4(0, 0, 0, 0);
                }
            };
            auto store = [&]() {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int e = q * 256 + tid, col = e >> 3, quad = e & 7;
                    if (col < ncols) {
                        St[(quad * 4 + 0) * kSP + col] = pf[q].x;
                        St[(quad * 4 + 1) * kSP + col] = pf[q].y;
                        St[(quad * 4 + 2) * kSP + col] = pf[q].z;
                        St[(quad * 4 + 3) * kSP + col] = pf[q].w;
                    }
                }
                if (tid < kSC / 4) {
                    float *R = sR + kSC * kSP;
                    R[tid * 4 + 0] = pr.x; R[tid * 4 + 1] = pr.y; R[tid * 4 + 2] = pr.z; R[tid * 4 + 3] = pr.w;
                }
            };
            load(0);
            for (int ch = 0; ch < nch; ++ch) {
                __syncthreads();                 // the previous chunk (or phase 1's B rows) is consumed
                store();
                __syncthreads();
                if (ch + 1 < nch) load(ch + 1);  // in flight during this chunk
                if (ch == 0) {
                    // pilot shift of a multiplicative form: its mean over the first chunk
                    const int c0 = n < kSC ? n : kSC;
                    float pm[KPT];
#pragma unroll
                    for (int i = 0; i < KPT; ++i) pm[i] = 0.f;
                    for (int t = 0; t < c0; ++t) {
#pragma unroll
                        for (int i = 0; i < KPT; ++i) {
                            if (i >= imax) break;
                            const float x = St[t * kSP + ax[i]], y = St[t * kSP + ay[i]];
                            pm[i] = fmaf(x, rc[i] ? __builtin_amdgcn_rcpf(y) : y, pm[i]);
                        }
                    }
                    const float inv = 1.0f / (float)c0;
#pragma unroll
                    for (int i = 0; i < KPT; ++i) cc[i] = pm[i] * inv;
                }
                const int cnt = (n - ch * kSC) < kSC ? (n - ch * kSC) : kSC;
                auto step = [&](int t) {
                    const float r = Rr[t];
#pragma unroll
                    for (int i = 0; i < KPT; ++i) {
                        if (i >= imax) break;
                        const float x = St[t * kSP + ax[i]], y = St[t * kSP + ay[i]];
                        const float gm = fmaf(x, rc[i] ? __builtin_amdgcn_rcpf(y) : y, -cc[i]);
                        const float ga = fmaf(sg[i], y - my[i], x - mx[i]);
                        const float g = ad[i] ? ga : gm;
                        fA[i] += g;
                        fB[i] = fmaf(g, g, fB[i]);
                        fC[i] = fmaf(g, r, fC[i]);
                    }
                };
                if (cnt == kSC) {
#pragma unroll 8
                    for (int t = 0; t < kSC; ++t) step(t);
                } else {
                    for (int t = 0; t < cnt; ++t) step(t);
                }
#pragma unroll
                for (int i = 0; i < KPT; ++i) {
                    dB[i] += (double)fB[i];
                    dC[i] += (double)fC[i];
                    fB[i] = fC[i] = 0.f;
                }
            }
            float osc[KPT];
            int64_t oid[KPT];
#pragma unroll
            for (int i = 0; i < KPT; ++i) {
                osc[i] = -1.0f;
                oid[i] = INT64_MAX;
                if (!has[i]) continue;
                const int64_t u = u0 + ul[i], v = vb + vl[i];
                const sisso_colstat ust = stats[u], vst = stats[v];
                if (ust.valid == 0.0f || vst.valid == 0.0f) continue;
                const int k = kf[i];
                const double shifts[5] = {(double)ust.mean + (double)vst.mean, (double)ust.mean - (double)vst.mean,
                                          (double)cc[i], (double)cc[i], (double)cc[i]};
                oid[i] = binbase + ((u - ulo) * vcount + v) * S + fs.slot[k];
                osc[i] = form_score(k, fA[i], dB[i], dC[i], shifts[k], pool32 + (size_t)u * ld32,
                                    pool32 + (size_t)v * ld32, n, ust.maxabs, ust.minabs, ust.rms, vst.maxabs,
                                    vst.minabs, vst.rms, nd, R1, Srr);
            }
            list_offer<KPT>(L, osc, oid, &W.h->gthr, excl, n_excl);
        }
        __syncthreads();
        if (tid == 0) { nkept = 0; ubits = 0u; }
        if (tid < kVS / 32) vbits[tid] = 0u;
        __syncthreads();
    };

    const int64_t items_hi = ut_hi * nvs;
    for (int64_t item = ut_lo * nvs + blockIdx.x; item < items_hi; item += gridDim.x) {
        const int64_t ut = item / nvs, vsup = item % nvs;
        const int64_t u0 = ulo + ut * 32;
        const int64_t vb = vsup * kVS, ve = vb + kVS < vcount ? vb + kVS : vcount;
        __syncthreads();
        for (int e = tid; e < 32 * (kH / 4); e += 256) {
            const int row = e / (kH / 4), q = e % (kH / 4);
            const int64_t u = u0 + row;
            const float4 val = u < uhi ? reinterpret_cast<const float4 *>(Au + (size_t)(u - ulo) * kH)[q]
                                       : make_float4(0, 0, 0, 0);
            sA[row * kPH + 2 * q] = to_h2(val.x, val.y);
            sA[row * kPH + 2 * q + 1] = to_h2(val.z, val.w);
        }
        for (int64_t v0 = vb; v0 < ve; v0 += 32) {
            if (nkept > kKeptCap - 32 * 32 * 5) exact(u0, vb, ve);   // uniform: read after a barrier
            __syncthreads();
            for (int e = tid; e < 32 * (kH / 4); e += 256) {
                const int row = e / (kH / 4), q = e % (kH / 4);
                const int64_t v = v0 + row;
                const float4 val = v < ve ? reinterpret_cast<const float4 *>(Bv + (size_t)v * kH)[q]
                                          : make_float4(0, 0, 0, 0);
                sB[row * kPH + 2 * q] = to_h2(val.x, val.y);
                sB[row * kPH + 2 * q + 1] = to_h2(val.z, val.w);
            }
            __syncthreads();
            float acc[2][2][5];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int k = 0; k < 5; ++k) acc[a][b][k] = 0.f;
            for (int jp = 0; jp < kH / 2; jp += 4) {
                // four hidden-unit pairs of both u rows, both v rows, every form and w2
                h2 A[2][4], B[2][4], C[5][4], Wv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    A[0][q] = sA[(2 * ty) * kPH + jp + q];
                    A[1][q] = sA[(2 * ty + 1) * kPH + jp + q];
                    B[0][q] = sB[(2 * tx) * kPH + jp + q];
                    B[1][q] = sB[(2 * tx + 1) * kPH + jp + q];
                    Wv[q] = sC[5 * (kH / 2) + jp + q];
#pragma unroll
                    for (int k = 0; k < 5; ++k) C[k][q] = sC[k * (kH / 2) + jp + q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
#pragma unroll
                            for (int k = 0; k < 5; ++k)
                                acc[a][b][k] = net_step(A[a][q], B[b][q], C[k][q], Wv[q], acc[a][b][k]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int64_t u = u0 + 2 * ty + a, v = v0 + 2 * tx + b;
                    if (u >= uhi || v >= ve) continue;
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        if (fs.slot[k] < 0 || !(acc[a][b][k] + b2 >= tau)) continue;
                        const int64_t fid = binbase + ((u - ulo) * vcount + v) * S + fs.slot[k];
                        if (fid < id_begin || fid >= id_end) continue;
                        const int slot = atomicAdd(&nkept, 1);
                        atomicOr(&ubits, 1u << (2 * ty + a));
                        atomicOr(&vbits[(int)(v - vb) >> 5], 1u << ((int)(v - vb) & 31));
                        kl[slot] = (unsigned short)((2 * ty + a) | ((int)(v - vb) << 5) | (k << 13));
                    }
                }
            __syncthreads();
        }
        if (nkept > 0) exact(u0, vb, ve);
    }
    const int list = list_base + blockIdx.x;
    list_flush(L, &W.h->gthr, W.sc + (size_t)list * keep, W.id + (size_t)list * keep);
    if (tid == 0 && kept_total) atomicAdd(kept_total, kept_local);
}

}  // namespace sisso

// ------------------------------------------------------------------ C ABI

using namespace sisso;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

bool args_ok(const sisso_score_args *a)
{
    return a->n >= 2 && a->n <= SISSO_MAX_N && a->ld32 >= a->n && (a->ld32 % 4) == 0;
}

bool slice_ok(const sisso_space *s)
{
    return s && s->total > 0 && s->rect == 1 && s->levels >= 1 && s->levels <= SISSO_MAX_LEVELS &&
           s->pool[s->levels - 1] >= 1;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kPrunedMaxGrid = 1024;
constexpr int kPrunedKPT = 4;

size_t pruned_smem(int cap)
{
    return (size_t)(32 * kPH + kRegion + 3 * kH) * sizeof(float) + (size_t)kKeptCap * sizeof(unsigned short) +
           (size_t)cap * (sizeof(float) + sizeof(int64_t));
}

struct PrunedPlan {
    int64_t ut_lo = 0, ut_hi = 0;
    int grid = 0;
};

// Work items (u tile, v span) over the u tiles that [begin, end) touches; the
// grid stays within the list slots the workspace reserves for the block.
PrunedPlan pruned_plan(const sisso_space *s, const sisso_score_args *a, int64_t begin, int64_t end)
{
    PrunedPlan p;
    const int64_t bb = s->pool[s->levels] + s->rect_unary, be = s->total;
    const int64_t b = begin > bb ? begin : bb, e = end < be ? end : be;
    if (b >= e) return p;
    const int64_t vcount = s->pool[s->levels - 1];
    const int64_t per_u = vcount * s->n_slots;
    const int64_t ul = (b - bb) / per_u, uh = (e - 1 - bb) / per_u + 1;
    p.ut_lo = ul / 32;
    p.ut_hi = (uh + 31) / 32;
    const int64_t items = (p.ut_hi - p.ut_lo) * ((vcount + kVS - 1) / kVS);
    const int64_t all_ut = (s->pool[s->levels] - s->pool[s->levels - 1] + 31) / 32;
    const int mg = a->grid > 0 ? a->grid : kPrunedMaxGrid;
    int64_t slots = all_ut < mg ? all_ut : mg;
    if (slots < 32) slots = 32;
    p.grid = (int)(items < slots ? items : slots);
    return p;
}

}  // namespace

extern "C" int32_t sisso_mlp_param_count(void) { return kParams; }
extern "C" int32_t sisso_mlp_table_count(void) { return kTab; }

extern "C" sisso_status sisso_encode_operands(const sisso_space *space, const sisso_score_args *args,
                                              int64_t c_begin, int64_t c_end, float *enc, void *stream)
{
    if (args && (args->w32 || args->units)) return SISSO_E_UNSUPPORTED;   // weights, units: FP32 / 16-bit forms
    if (!space || !args || !enc || !args->pool32 || !args->stats || !args->r32 || !args->info) return SISSO_E_NULL;
    if (space->total <= 0 || !args_ok(args)) return SISSO_E_SHAPE;
    const int64_t pL = space->pool[space->levels];
    if (c_begin < 0 || c_end > pL || c_begin >= c_end) return SISSO_E_RANGE;
    const int64_t waves = c_end - c_begin;
    const int64_t blocks = cdiv(waves, 4);
    const int grid = (int)(blocks < 16384 ? blocks : 16384);
    hipLaunchKernelGGL(k_encode, dim3(grid), dim3(256), 0, as_stream(stream), *space, args->n, args->pool32,
                       args->ld32, args->stats, args->r32, args->info, c_begin, c_end, enc);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_candidate_inputs(const sisso_space *space, const float *enc, const int64_t *ids,
                                               int32_t count, float *X, void *stream)
{
    if (!space || !enc || !ids || !X) return SISSO_E_NULL;
    if (!slice_ok(space)) return SISSO_E_UNSUPPORTED;
    if (count < 0) return SISSO_E_SHAPE;
    if (count == 0) return SISSO_OK;
    hipLaunchKernelGGL(k_inputs, dim3((unsigned)cdiv(count, 4)), dim3(256), 0, as_stream(stream), *space,
                       form_slots(space), enc, ids, count, X);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_score_ids(const sisso_space *space, const sisso_score_args *args, const int64_t *ids,
                                        int32_t count, float *out, void *stream)
{
    if (args && (args->w32 || args->units)) return SISSO_E_UNSUPPORTED;   // weights, units: FP32 / 16-bit forms
    if (!space || !args || !ids || !out || !args->pool32 || !args->stats || !args->r32 || !args->info)
        return SISSO_E_NULL;
    if (!slice_ok(space)) return SISSO_E_UNSUPPORTED;
    if (!args_ok(args) || count < 0) return SISSO_E_SHAPE;
    if (count == 0) return SISSO_OK;
    hipLaunchKernelGGL(k_score_ids, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, as_stream(stream), *space,
                       form_slots(space), args->n, args->pool32, args->ld32, args->stats, args->r32, args->info, ids,
                       count, out);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_mlp_forward(const float *params, const float *X, int32_t batch, float *Z, float *s,
                                          void *stream)
{
    if (!params || !X || !Z || !s) return SISSO_E_NULL;
    if (batch < 1) return SISSO_E_SHAPE;
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)cdiv(batch, 64), kH / 64), dim3(256), 0, st, (int64_t)batch, kH,
                       kIn, X, (int64_t)kIn, (int64_t)1, params, (int64_t)kIn, (int64_t)1, params + kOffB1, Z,
                       (int64_t)kH);
    hipLaunchKernelGGL(k_mlp_out, dim3((unsigned)cdiv(batch, 4)), dim3(256), 0, st, Z, params, batch, s);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" size_t sisso_mlp_workspace_size(int32_t batch) { return batch < 1 ? 0 : mlp_ws_bytes(batch); }

extern "C" sisso_status sisso_mlp_backward(const float *params, const float *X, const float *Z, const float *s,
                                           const float *t, const float *w, int32_t batch, float *grads, float *loss,
                                           void *ws, size_t ws_bytes, void *stream)
{
    if (!params || !X || !Z || !s || !t || !w || !grads || !ws) return SISSO_E_NULL;
    if (batch < 1) return SISSO_E_SHAPE;
    if (ws_bytes < mlp_ws_bytes(batch)) return SISSO_E_WORKSPACE;
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(1024), 0, st, s, t, w, batch, ws, loss);
    hipLaunchKernelGGL(k_mlp_dz, dim3((unsigned)cdiv(batch, 4)), dim3(256), 0, st, Z, params, s, t, w, batch, ws);
    hipLaunchKernelGGL(k_mlp_colsums, dim3(1), dim3(kH), 0, st, Z, batch, ws, grads);
    // dW1 = dz^T X: A(i, k) = dz[k][i], B(j, k) = X[k][j]
    hipLaunchKernelGGL(k_gemm_bf16, dim3(kH / 64, (unsigned)cdiv(kIn, 64)), dim3(256), 0, st, (int64_t)kH, kIn,
                       batch, (const float *)mlp_dz(ws, batch), (int64_t)1, (int64_t)kH, X, (int64_t)1, (int64_t)kIn,
                       (const float *)nullptr, grads, (int64_t)kIn);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

namespace sisso {
// Regression target of the proposal network: the Fisher z-transform of a
// |correlation|, atanh(min(|c|, 1 - 1e-6)) (finite at |c| = 1), in FP64.
__global__ void __launch_bounds__(256) k_mlp_target(const float *__restrict__ sc, int count, float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double c = fmin(fabs((double)sc[i]), 0.999999);
    out[i] = (float)atanh(c);
}
}  // namespace sisso

extern "C" sisso_status sisso_mlp_target(const float *scores, int32_t count, float *out, void *stream)
{
    if (!scores || !out) return SISSO_E_NULL;
    if (count < 1) return SISSO_E_SHAPE;
    hipLaunchKernelGGL(k_mlp_target, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, as_stream(stream), scores,
                       count, out);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_adam_step(float *params, const float *grads, float *m, float *v, int64_t count,
                                        int32_t step, float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!params || !grads || !m || !v) return SISSO_E_NULL;
    if (count < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return SISSO_E_SHAPE;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, as_stream(stream), params, grads, m,
                       v, count, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_mlp_parts(const float *params, const float *enc, int64_t rows, int32_t side,
                                        float *out, void *stream)
{
    if (!params || !enc || !out) return SISSO_E_NULL;
    if (rows < 1 || side < 0 || side > 1) return SISSO_E_SHAPE;
    hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)cdiv(rows, 64), kH / 64), dim3(256), 0, as_stream(stream), rows,
                       kH, kE, enc, (int64_t)kE, (int64_t)1, params + side * kE, (int64_t)kIn, (int64_t)1,
                       (const float *)nullptr, out, (int64_t)kH);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_mlp_tables(const float *params, float *tables, void *stream)
{
    if (!params || !tables) return SISSO_E_NULL;
    hipLaunchKernelGGL(k_mlp_tables, dim3(1), dim3(kH), 0, as_stream(stream), params, tables);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_mlp_score_ids(const sisso_space *space, const float *Au, const float *Bv,
                                            const float *tables, const int64_t *ids, int32_t count, float *out,
                                            void *stream)
{
    if (!space || !Au || !Bv || !tables || !ids || !out) return SISSO_E_NULL;
    if (!slice_ok(space)) return SISSO_E_UNSUPPORTED;
    if (count < 0) return SISSO_E_SHAPE;
    if (count == 0) return SISSO_OK;
    hipLaunchKernelGGL(k_mlp_score_ids, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, as_stream(stream), *space,
                       form_slots(space), Au, Bv, tables, ids, count, out);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_select_kth(const float *x, int32_t count, int32_t q, float *out_value, void *stream)
{
    if (!x || !out_value) return SISSO_E_NULL;
    if (count < 1 || q < 1 || q > count) return SISSO_E_RANGE;
    hipLaunchKernelGGL(k_select_kth, dim3(1), dim3(1024), 0, as_stream(stream), x, count, q, out_value);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" int32_t sisso_expand_score_pruned_lists(const sisso_space *space, const sisso_score_args *args,
                                                   int64_t cand_begin, int64_t cand_end)
{
    if (!slice_ok(space) || !args || cand_begin < 0 || cand_end > space->total || cand_begin >= cand_end ||
        args->grid < 0)
        return -1;
    return pruned_plan(space, args, cand_begin, cand_end).grid;
}

extern "C" sisso_status sisso_expand_score_pruned(const sisso_space *space, const sisso_score_args *args,
                                                  const float *Au, const float *Bv, const float *tables,
                                                  const float *tau, int64_t cand_begin, int64_t cand_end, void *ws,
                                                  size_t ws_bytes, unsigned long long *kept, void *stream)
{
    if (args && (args->w32 || args->units)) return SISSO_E_UNSUPPORTED;   // weights, units: FP32 / 16-bit forms
    if (!space || !args || !Au || !Bv || !tables || !tau || !ws || !args->pool32 || !args->stats || !args->r32 ||
        !args->info)
        return SISSO_E_NULL;
    if (args->n_exclude > 0 && !args->exclude) return SISSO_E_NULL;
    if (!slice_ok(space)) return SISSO_E_UNSUPPORTED;
    if (!args_ok(args) || args->n_exclude < 0) return SISSO_E_SHAPE;
    if (args->keep < 1 || args->keep > SISSO_MAX_KEEP) return SISSO_E_RANGE;
    if (cand_begin < 0 || cand_end > space->total || cand_begin >= cand_end || args->grid < 0) return SISSO_E_RANGE;
    const int lists = score_lists_capacity(space, args);
    if (ws_bytes < ws_bytes_for(lists, args->keep)) return SISSO_E_WORKSPACE;
    const PrunedPlan p = pruned_plan(space, args, cand_begin, cand_end);
    if (args->list_base < 0 || args->list_base + p.grid > lists) return SISSO_E_WORKSPACE;
    hipStream_t st = as_stream(stream);
    if (!ws_begin_call(ws, args->keep, args->list_base, p.grid, lists, st)) return SISSO_E_DEVICE;
    if (p.grid == 0) return SISSO_OK;
    const int cap = next_pow2(args->keep + 256);
    const size_t smem = pruned_smem(cap);
    if (!allow_dynamic_lds(k_score_pruned<kPrunedKPT>, smem)) return SISSO_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_score_pruned<kPrunedKPT>, dim3(p.grid), dim3(256), smem, st, *space, form_slots(space),
                       args->n, args->pool32, args->ld32, args->stats, args->r32, args->info, args->exclude,
                       args->n_exclude, Au, Bv, tables, tau, p.ut_lo, p.ut_hi, cand_begin, cand_end, args->list_base,
                       ws, lists, args->keep, cap, kept);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_count_pass(const float *exact, const float *net, int32_t count, const float *exact_thr,
                                         const float *net_thr, int32_t *out, void *stream)
{
    if (!exact || !net || !exact_thr || !net_thr || !out) return SISSO_E_NULL;
    if (count < 1) return SISSO_E_SHAPE;
    hipLaunchKernelGGL(k_count_pass, dim3(1), dim3(1024), 0, as_stream(stream), exact, net, count, exact_thr, net_thr,
                       out);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
