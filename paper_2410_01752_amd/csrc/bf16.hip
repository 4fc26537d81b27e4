// bf16.hip -- 16-bit MFMA screening of the one-sided rung-3 slice, followed by
// an exact FP32 rescore of a band of candidates around the cutoff (Sec. 2.2,
// eq. sis-weight: the correlation of every candidate with the residual).
//
// With centred operands u~ = u - mean(u), z~ = 1/u - mean(1/u) and
// v~ = v - mean(v), w~ = 1/v - mean(1/v), the sums a score needs are
// contractions over the samples.  For u * v, with h = uv - mean(u) mean(v)
// = u~v~ + mean(v) u~ + mean(u) v~:
//   sum h      = G[U~, V~]
//   sum h r    = G[U~, V~ r] + mean(v) sum u~ r + mean(u) sum v~ r
//   sum h^2    = G[U~^2, V~ (V~ + 2 mean(v))] + 2 mean(u) G[U~, V~ (V~ + mean(v))]
//                + mean(v)^2 sum u~^2 + mean(u)^2 sum v~^2
// and likewise u/v (with W~) and v/u (with Z~ against V~); u + v and u - v
// need only G[U~, V~].  Twelve GEMMs over a tile of (u, v) pairs, with the
// per-column terms folded into the v-side operands, give all five forms.
//
// The operands are IEEE half precision (11-bit significand): every variant
// column is scaled by a power of two near the inverse of its root-mean-square
// (exact, undone on the FP32 accumulators), rounded to FP16 while a sample
// chunk is staged into LDS (nothing 16-bit is stored in HBM), and each GEMM is
// one v_mfma_f32_32x32x16_f16 per 16 samples with FP32 accumulation.  A single
// 16-bit product cannot resolve a variance whose expansion terms cancel (a
// ratio of strongly related operands, a sum or difference of nearly opposite
// operands): such a candidate is recognised per pair and form by a
// conditioning test -- its approximate variance is below kCondRel of the sum
// of the magnitudes of the terms it was formed from, where the rounding error
// of those terms is no longer negligible -- and is scored exactly instead
// (about 3 in 10^4 candidates at n = 2000, d = 20).  Every other candidate
// keeps its approximate score.  The approximate scores and the exact scores of
// the flagged candidates select a band (a margin wider than the list, since
// 16-bit noise reorders near-ties); every candidate of the band is rescored
// with the plain FP32 kernel's arithmetic (shared functions), so reported
// scores are the FP32 path's scores.
//
// The file is compiled twice.  The second translation unit (bf16_mfma.hip,
// which defines SISSO_BF16_MFMA_PART) holds only the plain form and the
// moments pass and is compiled with the scheduler that maximises
// instruction-level parallelism.
#include "tiles.hpp"

#include <cstdlib>
#include <type_traits>
#include <utility>

namespace sisso {

typedef _Float16 h16;
typedef h16 h16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef h16 h16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBT = 64;       // u operands per block tile (the tiling of the slice's u range)
// A form's approximate variance is trusted when it is at least kCondRel of the
// sum of the magnitudes of its expansion terms (each carries a relative
// rounding error of about 2^-12 from the FP16 operands); below it the
// candidate is scored exactly.
constexpr float kCondRel = 1e-2f;
constexpr int kKC = 16;       // samples per LDS stage (one MFMA k-step)
constexpr int kKR = kKC;      // 16-bit values per LDS row: one chunk of samples of one column
constexpr int kMom = 6;       // residual-independent moments kept per (u, v) pair
constexpr size_t kMomTile = (size_t)4 * 16 * kMom * 64;   // floats per (u tile, v tile)

// Forms of the screening kernel.  kBfFull runs all twelve GEMMs.  Within a
// fit, the first pass runs the moments pass (k_bf_moments below: the nine
// residual-independent GEMMs, reduced per pair to sum h of u v, u/v and v/u
// and their variances, stored with the u side's FP16 image), and every pass
// scores with kBfRead, which loads them and runs only the three residual
// GEMMs.
enum BfMode { kBfFull = 0, kBfRead = 2 };

// GEMM g multiplies u-side variant A(g) with v-side variant B(g).
//   full:  g:  0   1    2   3   4   5    6    7   8   9    10   11
//          A:  U~  U~   U~2 U~  U~  U~   U~2  U~  Z~  Z~   Z~2  Z~
//          B:  V~  V~r  P   Q   W~  W~r  Pw   Qw  V~  V~r  P    Q
//   read:  g:  0    1    2           (= full 1, 5, 9)
//          A:  U~   U~   Z~
//          B:  V~r  W~r  V~r
template <int MODE> struct BfShape {
    static constexpr bool kRead = MODE == kBfRead;
    static constexpr int kUVar = kRead ? 2 : 4;     // U~, [U~^2,] Z~, [Z~^2]
    static constexpr int kVVar = kRead ? 2 : 8;     // [V~,] V~ r, [P, Q, W~,] W~ r, [Pw, Qw]
    static constexpr int kNG = kRead ? 3 : 12;      // GEMMs per tile
    // Block tile: kBTU u columns x kBTV v columns; each wave owns kSubV
    // 32 x 32 sub-tiles along v.  The read form's few GEMMs leave registers for
    // two sub-tiles per wave at two waves per SIMD: its 128 x 128 block streams
    // each image once per 128 columns of the other side.
    static constexpr int kWU = kRead ? 4 : 2, kWV = 2;                 // waves along u and along v
    static constexpr int kSubV = kRead ? 2 : 1;                        // 32 x 32 sub-tiles per wave (along v)
    static constexpr int kBTU = 32 * kWU, kBTV = 32 * kWV * kSubV, kThreads = 64 * kWU * kWV;
    static constexpr int kSU = kBTU * kKC / kThreads;                  // u samples staged per thread
    static constexpr int kSV = kBTV * kKC / kThreads;                  // v samples staged per thread
    static constexpr int kPlaneU = kBTU * kKR, kPlaneV = kBTV * kKR;   // 16-bit values per staged plane
    static constexpr int kPA = kUVar, kPB = kVVar;                     // staged planes per side
    static constexpr int kStage = kPA * kPlaneU + kPB * kPlaneV;       // 16-bit values per staging buffer
    // The read form stages its u side as the image's 64-column tiles, each
    // with its planes: the stride of a u plane within a tile.
    static constexpr int kAPlane = kRead ? 64 * kKR : kPlaneU;
    static constexpr int kMinBlocks = 1;            // resident blocks per CU the registers are sized for
    static constexpr int kNStage = kRead ? 3 : 2;   // staging buffers
    static constexpr int kRing = 6;                 // the read form: chunks held in registers (loads in flight)
    // accumulator of the residual contraction of u v, u/v and v/u
    static constexpr int kCovUV = kRead ? 0 : 1, kCovUW = kRead ? 1 : 5, kCovZV = kRead ? 2 : 9;
};

// f(std::integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

__host__ __device__ inline size_t align256b(size_t x) { return (x + 255) & ~(size_t)255; }

// u-side per-column constants (residual-independent, once per problem).
struct BfOps {
    float4 *usum;     // mean(u), mean(1/u), sum u~^2, sum z~^2
};
__host__ __device__ inline size_t bf_ops_bytes(int64_t ucols) { return align256b((size_t)ucols * sizeof(float4)); }
__host__ __device__ inline BfOps bf_ops_view(void *p)
{
    BfOps o;
    o.usum = (float4 *)p;
    return o;
}

// Candidates the conditioning test flags, kept for exact scoring: a counter
// (which may exceed the capacity: the excess was not stored) and their ids.
// The capacity is proportional to the binary block (one in 1024 candidates).
struct BfSide {
    unsigned long long *cnt;
    int64_t *ids;
    int64_t cap;
};
__host__ __device__ inline int64_t bf_side_cap(const sisso_space &s)
{
    const int64_t c = s.rect_binary / 1024;
    return c < ((int64_t)1 << 16) ? ((int64_t)1 << 16) : (c > ((int64_t)1 << 26) ? ((int64_t)1 << 26) : c);
}
__host__ __device__ inline size_t bf_side_bytes(const sisso_space &s) { return 256 + (size_t)bf_side_cap(s) * 8; }
__host__ __device__ inline BfSide bf_side_view(void *p, const sisso_space &s)
{
    BfSide d;
    d.cnt = (unsigned long long *)p;
    d.ids = (int64_t *)((char *)p + 256);
    d.cap = bf_side_cap(s);
    return d;
}

// per-pass workspace of the 16-bit screen: v-side column sums, u-side residual
// sums, band lists (a screening workspace of its own, whose lists are those of
// the screen followed by the exact scores of the flagged candidates), the
// band ids, the read form's v-side image and the flagged candidates of a
// screen that stores no moments.
struct BfWs {
    float4 *vsum;     // 2 per column: (mean v, mean 1/v, sum v~^2, sum w~^2), (sum v~ r, sum w~ r, rms, 0)
    float2 *ures;     // per u column: sum u~ r, sum z~ r
    int64_t *band_ids;
    float *band_sc;
    int32_t *band_cnt;
    void *lists;      // screening workspace of the band lists
    h16 *vimg;        // the read form's v-side staging image (see k_bf16_v_image)
    void *side;       // BfSide storage of a screen without moments
};
// the read form's v-side image: per 128-column v tile and chunk of samples,
// the staged planes of V~ r and W~ r in their LDS layout
__host__ __device__ inline size_t bf_vimg_elems(int64_t vcols, int n)
{
    return (size_t)((vcols + 127) / 128) * (size_t)((n + kKC - 1) / kKC) * 2 * (128 * kKR);
}
// the u side's image (written before the moments pass, read by it and by the
// read form): per 64-column u tile and chunk of samples, the staged planes
// U~, Z~, U~^2 and Z~^2 (64 rows of 16 samples each, FP16, in their LDS layout)
constexpr int kUImgPlanes = 4;
__host__ __device__ inline size_t bf_uimg_elems(int64_t ucols, int n)
{
    return (size_t)((ucols + 63) / 64) * (size_t)((n + kKC - 1) / kKC) * kUImgPlanes * (64 * kKR);
}
// the v side's residual-independent image for the moments pass: per 128-column
// v tile and chunk, the staged planes V~, P, Q, W~, Pw, Qw (128 rows each)
constexpr int kVmPlanes = 6;
__host__ __device__ inline size_t bf_vmimg_elems(int64_t vcols, int n)
{
    return (size_t)((vcols + 127) / 128) * (size_t)((n + kKC - 1) / kKC) * kVmPlanes * (128 * kKR);
}
__host__ __device__ inline size_t bf_ws_bytes(const sisso_space &s, int64_t ucols, int64_t vcols, int n, int band,
                                              int lists, int keep)
{
    size_t b = align256b((size_t)vcols * 2 * sizeof(float4));
    b += align256b((size_t)ucols * sizeof(float2));
    b += align256b((size_t)band * sizeof(int64_t)) + align256b((size_t)band * sizeof(float)) + 256;
    b += align256b(ws_bytes_for(lists, keep));
    b += align256b(bf_vimg_elems(vcols, n) * sizeof(h16));
    b += align256b(bf_side_bytes(s));
    return b;
}
__host__ __device__ inline BfWs bf_ws_view(void *p, int64_t ucols, int64_t vcols, int n, int band, int lists, int keep)
{
    BfWs w;
    char *c = (char *)p;
    w.vsum = (float4 *)c; c += align256b((size_t)vcols * 2 * sizeof(float4));
    w.ures = (float2 *)c; c += align256b((size_t)ucols * sizeof(float2));
    w.band_ids = (int64_t *)c; c += align256b((size_t)band * sizeof(int64_t));
    w.band_sc = (float *)c; c += align256b((size_t)band * sizeof(float));
    w.band_cnt = (int32_t *)c; c += 256;
    w.lists = c; c += align256b(ws_bytes_for(lists, keep));
    w.vimg = (h16 *)c; c += align256b(bf_vimg_elems(vcols, n) * sizeof(h16));
    w.side = c;
    return w;
}

// Power of two nearest to 1 / x for x in [2^-56, 2^56], 1 otherwise: x times
// it lies in [2^-1/2, 2^1/2).  Every operand variant is scaled by such a
// factor of its root-mean-square (products of them by the product of the
// factors, which stays inside FP32's exponent range), so that FP16 holds it
// without overflow (|value| <= sqrt(n) times its rms) and with full relative
// precision; the FP32 accumulators are scaled back exactly.  A column whose
// rms lies outside that range is not scalable: the screen scores its
// candidates exactly.
__device__ __forceinline__ bool scalable(float x) { return x >= 0x1p-56f && x <= 0x1p56f; }
__device__ __forceinline__ float pow2_inv(float x)
{
    if (!scalable(x)) return 1.0f;
    int e;
    const float f = frexpf(x, &e);                // x = f 2^e, f in [1/2, 1)
    return ldexpf(1.0f, f < 0.70710678f ? 1 - e : -e);
}
// the root-mean-squares of a column's centred variants x~ and 1/x - mean(1/x)
// (the latter only when the column has no zero) are scalable
__device__ __forceinline__ bool col_scalable(float sxx, float srr, float fn, bool rcp)
{
    return scalable(sqrtf(sxx / fn)) && (!rcp || scalable(sqrtf(srr / fn)));
}

// Extra factor of the variants that are products of two centred values (their
// magnitude can reach 2n times the product of the factors): keeps them under
// 2^15 for any n.
__device__ __forceinline__ float sq_shift(int n)
{
    int e;
    frexpf((float)(2 * n), &e);                   // 2n < 2^e
    return e > 15 ? ldexpf(1.0f, 15 - e) : 1.0f;
}

// Scale factors of a u column (U~, Z~; U~^2 and Z~^2 take the squares times
// sq_shift) from its sums of squares.
struct UScale { float u, z; };
__device__ __forceinline__ UScale u_scales(float suu, float szz, float fn)
{
    return UScale{pow2_inv(sqrtf(suu / fn)), pow2_inv(sqrtf(szz / fn))};
}
// Scale factors of a v column: V~, P = V~ (V~ + 2 mean v), Q = V~ (V~ + mean v),
// V~ r; the same for W~ = 1/v - mean(1/v).  rs: the residual's factor.
struct VScale { float v, p, q, vr, w, pw, qw, wr; };
__device__ __forceinline__ VScale v_scales(float mv, float mw, float svv, float sww, float fn, float rs, float sh)
{
    const float sv = sqrtf(svv / fn), sw = sqrtf(sww / fn);
    VScale c;
    c.v = pow2_inv(sv);
    c.p = c.v * pow2_inv(sv + 2.0f * fabsf(mv)) * sh;
    c.q = c.v * pow2_inv(sv + fabsf(mv)) * sh;
    c.vr = c.v * rs * sh;
    c.w = pow2_inv(sw);
    c.pw = c.w * pow2_inv(sw + 2.0f * fabsf(mw)) * sh;
    c.qw = c.w * pow2_inv(sw + fabsf(mw)) * sh;
    c.wr = c.w * rs * sh;
    return c;
}
// the residual's factor from its sum of squares
__device__ __forceinline__ float r_scale(double srr, double n) { return pow2_inv((float)sqrt(srr / n)); }

// Element offset of samples k .. k + 3 (k % 4 == 0) of column `row` in a staged
// plane.  The two 8-sample halves of a row are swapped on rows whose bits 2 and
// 3 differ, so that the fragment reads (16 bytes of 32 consecutive rows) and
// the staging stores (8 bytes, 4 columns x 4 quads per 16 lanes) fall into
// distinct banks.
__device__ __forceinline__ int lds_off(int row, int k)
{
    return row * kKR + (k ^ ((((row >> 2) ^ (row >> 3)) & 1) << 3));
}

// A workgroup barrier after this wave's LDS stores have completed, which
// leaves its vector memory loads in flight (__syncthreads would wait for
// them); the clobber keeps the compiler from moving memory accesses across.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// N consecutive floats (N = 2 or 4, 4N-byte aligned) in one load.
template <int N>
__device__ __forceinline__ void load_floats(const float *p, float (&x)[N])
{
    static_assert(N == 2 || N == 4, "2 or 4 samples per thread");
    if constexpr (N == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
    } else {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        x[0] = t.x; x[1] = t.y;
    }
}

// Stores N consecutive samples rounded to FP16 (two per conversion).
template <int N>
__device__ __forceinline__ void put_h16(h16 *dst, const float (&x)[N])
{
    unsigned hw[N / 2];
#pragma unroll
    for (int e = 0; e < N; e += 2) {
        const h16x2 h = __builtin_convertvector((f32x2){x[e], x[e + 1]}, h16x2);
        __builtin_memcpy(&hw[e / 2], &h, 4);
    }
    if constexpr (N == 4) *reinterpret_cast<uint2 *>(dst) = make_uint2(hw[0], hw[1]);
    else *reinterpret_cast<unsigned *>(dst) = hw[0];
}

#ifndef SISSO_BF16_MFMA_PART
// ---------------------------------------------------------------- operands

// u side (newest pool level), independent of the residual: the column
// constants of the centred variants.  One wave per column.
__global__ void __launch_bounds__(256) k_bf16_u_prep(int n, const float *__restrict__ pool32, int64_t ld32,
                                                     const sisso_colstat *__restrict__ stats, int64_t col0,
                                                     int64_t ucols, BfOps ops)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = wave; c < ucols; c += nw) {
        const sisso_colstat st = stats[col0 + c];
        const float *col = pool32 + (size_t)(col0 + c) * ld32;
        const float mu = st.mean, mz = st.mean_rcp;
        const bool zok = st.minabs > 0.0f;
        double suu = 0.0, szz = 0.0;
        for (int t = lane * 4; t < n; t += 256) {     // 16-byte loads: samples t .. t + 3
            const float4 x4 = *reinterpret_cast<const float4 *>(col + t);
            const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < n) {
                    const float uu = xs[e] - mu;
                    const float zz = zok ? __builtin_amdgcn_rcpf(xs[e]) - mz : 0.f;
                    suu += (double)uu * uu;
                    szz += (double)zz * zz;
                }
        }
        suu = wave_sum_dpp(suu);
        szz = wave_sum_dpp(szz);
        if (lane == 0) ops.usum[c] = make_float4(mu, mz, (float)suu, (float)szz);
    }
}

// u side, per residual: sum u~ r and sum z~ r.
__global__ void __launch_bounds__(256) k_bf16_u_resid(int n, const float *__restrict__ pool32, int64_t ld32,
                                                      const sisso_colstat *__restrict__ stats, int64_t col0,
                                                      int64_t ucols, const float *__restrict__ r32,
                                                      float2 *__restrict__ ures)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = wave; c < ucols; c += nw) {
        const sisso_colstat st = stats[col0 + c];
        const float *col = pool32 + (size_t)(col0 + c) * ld32;
        const bool zok = st.minabs > 0.0f;
        float sur = 0.f, szr = 0.f;
        for (int t = lane * 4; t < n; t += 256) {     // 16-byte loads: samples t .. t + 3
            const float4 x4 = *reinterpret_cast<const float4 *>(col + t);
            const float4 r4 = *reinterpret_cast<const float4 *>(r32 + t);
            const float xs[4] = {x4.x, x4.y, x4.z, x4.w}, rs[4] = {r4.x, r4.y, r4.z, r4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < n) {
                    sur = fmaf(xs[e] - st.mean, rs[e], sur);
                    if (zok) szr = fmaf(__builtin_amdgcn_rcpf(xs[e]) - st.mean_rcp, rs[e], szr);
                }
        }
        const double a = wave_sum_dpp((double)sur), b = wave_sum_dpp((double)szr);
        if (lane == 0) ures[c] = make_float2((float)a, (float)b);
    }
}

// v side (previous pool), per residual: the column sums.
__global__ void __launch_bounds__(256) k_bf16_v_prep(int n, const float *__restrict__ pool32, int64_t ld32,
                                                     const sisso_colstat *__restrict__ stats, int64_t vcols,
                                                     const float *__restrict__ r32, BfWs w)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = wave; c < vcols; c += nw) {
        const sisso_colstat st = stats[c];
        const float *col = pool32 + (size_t)c * ld32;
        const float mv = st.mean, mw = st.mean_rcp;
        const bool wok = st.minabs > 0.0f;
        double svv = 0.0, sww = 0.0, svr = 0.0, swr = 0.0;
        for (int t = lane; t < n; t += 64) {
            const float x = col[t], r = r32[t];
            const float vv = x - mv;
            const float ww = wok ? __builtin_amdgcn_rcpf(x) - mw : 0.f;
            svv += (double)vv * vv;
            sww += (double)ww * ww;
            svr += (double)vv * r;
            swr += (double)ww * r;
        }
        svv = wave_sum_dpp(svv); sww = wave_sum_dpp(sww); svr = wave_sum_dpp(svr); swr = wave_sum_dpp(swr);
        if (lane == 0) {
            w.vsum[2 * c] = make_float4(mv, mw, (float)svv, (float)sww);
            w.vsum[2 * c + 1] = make_float4((float)svr, (float)swr, st.rms, 0.f);
        }
    }
}
#endif  // SISSO_BF16_MFMA_PART

// The residual-weighted centred v variants of one sample, V~ r and W~ r,
// scaled (0 for a sample past n).  The plain form forms them in its tile
// kernel and the read form takes them from the v-side image: one function, the
// same bits.
__device__ __forceinline__ void v_resid_vars(float x, float r, float smv, float smw, float cvr, float cwr, bool live,
                                             float &vr, float &wr)
{
#pragma clang fp contract(off)
    float vv = x - smv, ww = __builtin_amdgcn_rcpf(x) - smw;
    vv = live ? vv : 0.f; ww = live ? ww : 0.f; r = live ? r : 0.f;
    vr = (vv * r) * cvr;
    wr = (ww * r) * cwr;
}

#ifndef SISSO_BF16_MFMA_PART
// The read form's v-side staging image for one residual: for each 128-column
// v tile and chunk of 16 samples, the planes V~ r and W~ r (128 rows of 16
// samples each, FP16) exactly as the tile kernel lays them out in LDS, so that
// staging them is a copy.  Block (vt, ch); thread t forms column t / 2,
// samples 8 (t % 2) .. + 7.  Columns past |P_1| stage column 0's values
// (their scores are discarded), samples past n zeros.
__global__ void __launch_bounds__(256) k_bf16_v_image(int n, const float *__restrict__ pool32, int64_t ld32,
                                                      int64_t vcols, const float *__restrict__ r32,
                                                      const sisso_resid_info *__restrict__ info,
                                                      const float4 *__restrict__ vsum, h16 *__restrict__ img)
{
    constexpr int kRows = 128, kPlanes = 2;
    const int nch = (n + kKC - 1) / kKC;
    const int64_t vt = blockIdx.x / nch;
    const int ch = blockIdx.x % nch;
    const int c = threadIdx.x >> 1, k0 = (threadIdx.x & 1) * 8;
    const int64_t v = vt * kRows + c;
    const int64_t vv = v < vcols ? v : 0;
    const float4 vs = vsum[2 * vv];
    const VScale sc = v_scales(vs.x, vs.y, vs.z, vs.w, (float)n, r_scale(info->s_rr, (double)n), sq_shift(n));
    const float *col = pool32 + (size_t)vv * ld32;
    float vr[8], wr[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int t = ch * kKC + k0 + e;
        const int tc = t < n ? t : n - 1;
        v_resid_vars(col[tc], r32[tc], vs.x, vs.y, sc.vr, sc.wr, t < n, vr[e], wr[e]);
    }
    h16 *const out = img + (size_t)blockIdx.x * kPlanes * kRows * kKR + lds_off(c, k0);
    h16 hv[8], hw[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        hv[e] = (h16)vr[e];
        hw[e] = (h16)wr[e];
    }
    __builtin_memcpy(out, hv, 16);
    __builtin_memcpy(out + kRows * kKR, hw, 16);
}

// -------------------------------------------------------------- screening
#endif  // SISSO_BF16_MFMA_PART

// The v column of a pair as the five forms use it.
struct BfVCol {
    float mv, mw, Svv, Svr, Swr;   // mean v, mean 1/v, sum v~^2, sum v~ r, sum w~ r
    bool ok;                       // in the pool and valid
    bool nonzero;                  // no zero (v/u, u/v defined)
    bool scalable;                 // the column's variants fit the 16-bit operands
    uint4 unit;
};

// The five forms of one (u, v) pair from its column constants, the
// residual-independent moments m (sum h and variance of u v, u/v and v/u)
// and the three residual contractions c0, c1, c2 (of u v, u/v and v/u,
// unscaled): residual covariance, variance, whether the candidate is live
// (in the space and its form's domain, its variance resolved) and whether it
// is flagged (in the space, its variance not resolved by the 16-bit
// operands: scored exactly instead, never live).  ua = (mean u, mean 1/u,
// sum u~^2, .), ub = (sum u~ r, sum z~ r, ., flags: 1 valid, 2 no zero, 4 not
// scalable).  The plain form's epilogue and the scorer of stored
// contractions both call it: the same operations on the same bits.
__device__ __forceinline__ void bf_forms(float4 ua, float4 ub, uint4 uunit, const BfVCol &vc, const float (&m)[kMom],
                                         float c0, float c1, float c2, float rr, const FormSlots &fs,
                                         float (&cov)[5], float (&var)[5], bool (&live)[5], bool (&flag)[5])
{
#pragma clang fp contract(off)
    const float mu = ua.x, mz = ua.y, Suu = ua.z, Sur = ub.x, Szr = ub.y;
    // (the conditions combine with & and |, not && and ||: evaluated in full,
    // they stay lane masks instead of becoming branches)
    const int uflags = (int)ub.w;
    const bool ok = ((uflags & 1) != 0) & vc.ok;
    const bool unscal = ((uflags & 4) != 0) | !vc.scalable;
    const float g0 = m[0];
    var[0] = Suu + vc.Svv + 2.0f * g0;                  // u + v
    var[1] = Suu + vc.Svv - 2.0f * g0;                  // u - v
    cov[0] = Sur + vc.Svr;
    cov[1] = Sur - vc.Svr;
    var[2] = m[1];                                      // u v
    cov[2] = c0 + vc.mv * Sur + mu * vc.Svr - m[0] * rr;
    var[3] = m[3];                                      // u / v
    cov[3] = c1 + vc.mw * Sur + mu * vc.Swr - m[2] * rr;
    var[4] = m[5];                                      // v / u
    cov[4] = c2 + vc.mv * Szr + mz * vc.Svr - m[4] * rr;
    // a sum or difference needs operands of equal units
    const bool same_u = unit_eq(uunit, vc.unit);
    const bool dom[5] = {same_u, same_u, true, vc.nonzero, (uflags & 2) != 0};
    // u + v and u - v: trusted when the variance is at least kCondRel of
    // Suu + Svv (the error of 2 g0 is a fraction of it); the product forms
    // carry -1 when their test failed
    const float cth = kCondRel * (Suu + vc.Svv);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const bool cand = ok & dom[k] & (fs.slot[k] >= 0);
        const bool good = !unscal & (k < 2 ? var[k] >= cth : var[k] > 0.0f) & (var[k] < INFINITY);
        live[k] = cand & good & (var[k] > 0.0f);
        flag[k] = cand & !good;
    }
}

// Approximate scores of the five forms of a pair, -1 for a candidate that is
// not live; |cov| / sqrt(var Srr), clamped to 1 when rounding exceeds it.
__device__ __forceinline__ void bf_scores(const float (&cov)[5], const float (&var)[5], const bool (&live)[5],
                                          double Srr, float (&sc)[5])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float q = fabsf(cov[k]) * __builtin_amdgcn_rsqf(var[k] * (float)Srr);
        const float sk = q <= 1.0f ? q : (q > 1.0f ? 1.0f : -1.0f);   // rounding above 1, or NaN
        sc[k] = live[k] ? sk : -1.0f;
    }
}

// Admission of one 32 x 32 sub-tile's candidates into the block list, after
// each lane has tested its 16 rows (bit r of `rows`: row r may have a
// candidate at the bound tb).  Block-uniform: every wave of the block calls it
// with its own sub-tile (rows = 0 for none) and `pend` a shared counter that
// is zero on entry.  row_scores(r, sc) gives row r's scores, fid_of(r, k) a
// candidate's id, in_range(id) whether the id is in the slice.
template <class RowScores, class FidOf, class InRange>
__device__ __forceinline__ void bf_admit(BlockList &Lst, unsigned *gb, int *pend, unsigned rows, float tb,
                                         const int64_t *__restrict__ excl, int n_excl, RowScores &&row_scores,
                                         FidOf &&fid_of, InRange &&in_range)
{
    auto admit_id = [&](int64_t id) { return in_range(id) && (n_excl == 0 || !in_sorted_ids(excl, n_excl, id)); };
    // Count this lane's candidates at or above the admission bound (the
    // bounds only rise, so a stale read admits more, never fewer), in range
    // and not excluded, and the block's total.  When they all fit into the
    // list, every thread reserves its slots with one atomic and writes them:
    // no per-row barriers.
    int mine = 0;
    if (rows) {
#pragma unroll 1
        for (int r = 0; r < 16; ++r) {
            if (!((rows >> r) & 1u)) continue;
            float sc[5];
            row_scores(r, sc);
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (sc[k] >= 0.0f && sc[k] >= tb && admit_id(fid_of(r, k))) ++mine;
        }
    }
    if (mine) atomicAdd(pend, mine);
    __syncthreads();
    const int total = *pend;                  // the caller resets it after a later barrier
    if (total == 0) return;
    // Every thread takes the same branch only if every thread reads the
    // list's count before any thread reserves slots: read it, merge if the
    // candidates do not fit (block-uniform, ends with a barrier), read it
    // again, and meet at a barrier before reserving.
    int cnt0 = *Lst.cnt;
    if (cnt0 + total > Lst.cap) {
        list_merge(Lst, gb);
        cnt0 = *Lst.cnt;
    }
    __syncthreads();
    if (cnt0 + total <= Lst.cap) {
        if (mine) {
            int slot = atomicAdd(Lst.cnt, mine);
#pragma unroll 1
            for (int r = 0; r < 16; ++r) {
                if (!((rows >> r) & 1u)) continue;
                float sc[5];
                row_scores(r, sc);
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    if (!(sc[k] >= 0.0f && sc[k] >= tb)) continue;
                    const int64_t id = fid_of(r, k);
                    if (admit_id(id)) {
                        Lst.sc[slot] = sc[k];
                        Lst.id[slot] = id;
                        ++slot;
                    }
                }
            }
        }
        return;
    }
    // the list is filling: row by row, merging as needed
#pragma unroll 1
    for (int r = 0; r < 16; ++r) {
        float sc[5];
        int64_t fid[5];
        row_scores(r, sc);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            fid[k] = fid_of(r, k);
            if (!in_range(fid[k])) sc[k] = -1.0f;
        }
        __syncthreads();
        const int c = *Lst.cnt;
        __syncthreads();
        if (c + 5 * (int)blockDim.x <= Lst.cap) {
            const float t = fmaxf(*Lst.thr, load_gthr(gb));
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (sc[k] >= 0.0f && sc[k] >= t && (n_excl == 0 || !in_sorted_ids(excl, n_excl, fid[k]))) {
                    const int slot = atomicAdd(Lst.cnt, 1);
                    Lst.sc[slot] = sc[k];
                    Lst.id[slot] = fid[k];
                }
        } else {
            list_offer<5>(Lst, sc, fid, gb, excl, n_excl);
        }
    }
}

// mom: per 64 x 64 tile (ut64, vt64) of (u, v) pairs, its four 32 x 32
// sub-tiles w = su + 2 sv (su, sv: the 32-column half of the tile along u and
// along v), row slot r and moment k, the 64 lanes' values, at float offset
// (((ut64 * nvt64 + vt64) * 4 + w) * 16 + r) * kMom * 64 + k * 64 + lane
// (written by the moments pass, read by the scorer of stored contractions;
// nvt64 = ceil(|P_1| / 64)).  cst: the residual contractions of a pass in the
// same tiling, three per pair: (((ut64 * nvt64 + vt64) * 4 + w) * 16 + r) *
// 3 * 64 + k * 64 + lane (written by kBfRead).  Lane l holds column l % 32
// and row 8 (r / 4) + 4 (l / 32) + (r % 4) of its 32 x 32 sub-tile.
template <int MODE>
__global__ void __launch_bounds__(BfShape<MODE>::kThreads, BfShape<MODE>::kMinBlocks) k_score_rect_bf16(
    sisso_space s, FormSlots fs, int n, const float *__restrict__ pool32, int64_t ld32,
    const float *__restrict__ r32, const float4 *__restrict__ usum, const float4 *__restrict__ vsum,
    const float2 *__restrict__ ures, const sisso_colstat *__restrict__ stats,
    const sisso_resid_info *__restrict__ info, const int64_t *__restrict__ excl, int n_excl, int64_t ut_lo,
    int64_t ut_hi, int64_t id_begin, int64_t id_end, float *__restrict__ cst, const h16 *__restrict__ vimg,
    const h16 *uimg, const int16_t *__restrict__ units, BfSide side, void *lws, int lists_total,
    int keep, int cap, int publish)
{
    // (uimg is not restrict-qualified: the read form's loads of a u tile's
    // first chunks, the same for every v tile, must not be hoisted out of the
    // v-tile loop into registers the chunk loop needs)
    using Sh = BfShape<MODE>;
    constexpr int kUVar = Sh::kUVar, kVVar = Sh::kVVar, kNG = Sh::kNG, kPA = Sh::kPA, kPB = Sh::kPB,
                  kStage = Sh::kStage, kBTU = Sh::kBTU, kBTV = Sh::kBTV, kSU = Sh::kSU, kSV = Sh::kSV,
                  kPlaneU = Sh::kPlaneU, kPlaneV = Sh::kPlaneV, kAPlane = Sh::kAPlane, kSubV = Sh::kSubV;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    h16 *const stage = reinterpret_cast<h16 *>(smem);   // staging buffers (two; the read form's ring: kNStage)
    float *lsc = (float *)(stage + Sh::kNStage * kStage);
    int64_t *lid = (int64_t *)(lsc + cap);
    // u-tile column constants for the epilogue: (mean u, mean 1/u, sum u~^2,
    // sum z~^2), (sum u~ r, sum z~ r, rms, flags: 1 valid, 2 no zero) and the
    // inverse scale factors of U~, U~^2, Z~, Z~^2
    float4 *ucon_a = reinterpret_cast<float4 *>(lid + cap), *ucon_b = ucon_a + kBTU, *ucon_c = ucon_b + kBTU;
    uint4 *ucon_u = reinterpret_cast<uint4 *>(ucon_c + kBTU);      // the u columns' units (zero without units)
    __shared__ int lcnt, lpend[kSubV];            // lpend: candidates of each sub-tile's epilogue
    __shared__ float lthr;
    __shared__ unsigned gdummy;                   // bound of a block that must not publish (stays 0)
    WsView W = ws_view(lws, lists_total, keep);
    if (threadIdx.x == 0) gdummy = 0u;
    unsigned *const gb = publish ? &W.h->gthr : &gdummy;
    BlockList Lst{lsc, lid, &lcnt, &lthr, cap, keep};
    if (threadIdx.x < kSubV) lpend[threadIdx.x] = 0;
    list_init(Lst);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wu = w % Sh::kWU, wv = w / Sh::kWU;
    const int Lv = s.levels;
    const int64_t vcount = s.pool[Lv - 1], ulo = s.pool[Lv - 1], ucols = s.pool[Lv] - ulo;
    const int64_t binbase = s.pool[Lv] + s.rect_unary;
    const int S = s.n_slots;
    const double nd = (double)n, R1 = info->sum_r32, Srr = info->s_rr;
    const float fn = (float)n, rsc = r_scale(Srr, nd), shs = sq_shift(n);
    const int nch = (n + kKC - 1) / kKC;
    const int64_t nvt = (vcount + kBTV - 1) / kBTV, nvt64 = (vcount + 63) / 64, nut64 = (ucols + 63) / 64;
    // staging roles: u column ucs, samples uks .. uks + kSU - 1 of a chunk; v
    // column vcs, samples vks .. vks + kSV - 1
    const int ucs = tid / (kKC / kSU), uks = (tid % (kKC / kSU)) * kSU;
    const int vcs = tid / (kKC / kSV), vks = (tid % (kKC / kSV)) * kSV;
    const int tmax_u = ((n - 1) / kSU) * kSU, tmax_v = ((n - 1) / kSV) * kSV;   // loads stay inside a column
    const int sto_u = lds_off(ucs, uks), sto_v = lds_off(vcs, vks);              // store offsets within a plane
    // fragment role: lane reads 8 samples (koff ..) of row lane % 32 of its
    // wave's 32-row part (the read form: of its 64-column u tile), and of each
    // of its v sub-tiles
    const int koff = (lane >> 5) * 8;
    const int fa = Sh::kRead ? (wu >> 1) * (kPA * kAPlane) + lds_off((wu & 1) * 32 + (lane & 31), koff)
                             : lds_off(wu * 32 + (lane & 31), koff);
    int fb[kSubV];
#pragma unroll
    for (int s2 = 0; s2 < kSubV; ++s2) fb[s2] = lds_off((wv * kSubV + s2) * 32 + (lane & 31), koff);

    // Tile order.  The plain form: a block owns u tiles (strided over the
    // grid) and sweeps every v tile.  The read form: (u, v) tiles, v fastest,
    // in turns of eight consecutive runs of gridDim.x / 8 tiles, one run per
    // XCD (consecutive blocks are dispatched to the XCDs in turn): the blocks
    // of an XCD then work on few u tiles at a time and share their images in
    // that XCD's L2, where a block per u tile would stream its own from HBM.
    const int64_t T = Sh::kRead ? (ut_hi - ut_lo) * nvt : ut_hi - ut_lo;
    const bool by_xcd = Sh::kRead && gridDim.x % 8 == 0;
    const int64_t gx = blockIdx.x % 8, gk = blockIdx.x / 8, gn = gridDim.x / 8;
    for (int64_t it = 0;; ++it) {
        const int64_t t = by_xcd ? (it * 8 + gx) * gn + gk : it * gridDim.x + blockIdx.x;
        if (t >= T) break;
        const int64_t ut = Sh::kRead ? ut_lo + t / nvt : ut_lo + t;
        const int64_t vt_first = Sh::kRead ? t % nvt : 0, vt_end = Sh::kRead ? vt_first + 1 : nvt;
        const int64_t u0 = ut * kBTU;  // index into the newest level
        const int64_t su = u0 + ucs;
        const bool su_ok = su < ucols;
        const float4 us_c = usum[su_ok ? su : 0];
        const float smu = us_c.x, smz = us_c.y;
        const UScale usc = u_scales(us_c.z, us_c.w, fn);
        const float cu = usc.u, cz = usc.z, cu2 = usc.u * usc.u * shs, cz2 = usc.z * usc.z * shs;
        const float *ucol = pool32 + (size_t)(ulo + (su_ok ? su : 0)) * ld32;
        __syncthreads();                              // the previous tile's epilogue reads are done
        if (tid < kBTU) {
            const int64_t x = u0 + tid;
            const bool in = x < ucols;
            const sisso_colstat cs = stats[ulo + (in ? x : 0)];
            const float2 b = ures[in ? x : 0];
            const float4 ua = usum[in ? x : 0];
            ucon_a[tid] = ua;
            ucon_b[tid] = make_float4(b.x, b.y, cs.rms,
                                      (in && cs.valid != 0.0f ? 1.0f : 0.0f) + (cs.minabs > 0.0f ? 2.0f : 0.0f));
            const UScale c = u_scales(ua.z, ua.w, fn);
            ucon_c[tid] = make_float4(1.0f / c.u, 1.0f / (c.u * c.u * shs), 1.0f / c.z, 1.0f / (c.z * c.z * shs));
            if (!col_scalable(ua.z, ua.w, fn, cs.minabs > 0.0f)) ucon_b[tid].w += 4.0f;
            ucon_u[tid] = units ? unit_of(units, ulo + (in ? x : 0)) : make_uint4(0u, 0u, 0u, 0u);
        }
        for (int64_t vt = vt_first; vt < vt_end; ++vt) {
            const int64_t v0 = vt * kBTV;
            const int64_t sv = v0 + vcs;
            const bool sv_ok = sv < vcount;
            const float4 vs_c = vsum[2 * (sv_ok ? sv : 0)];
            const float smv = vs_c.x, smw = vs_c.y;
            const VScale vsc = v_scales(smv, smw, vs_c.z, vs_c.w, fn, rsc, shs);
            const float *vcol = pool32 + (size_t)(sv_ok ? sv : 0) * ld32;
            f32x16 acc[kSubV][kNG];
#pragma unroll
            for (int s2 = 0; s2 < kSubV; ++s2)
#pragma unroll
                for (int g = 0; g < kNG; ++g)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[s2][g][e] = 0.0f;
            // Raw FP32 values of one chunk are loaded two chunks ahead into
            // registers; the centred, scaled variants are formed, rounded to FP16
            // and stored into the other staging buffer while the MFMAs of the
            // current chunk run.  Out-of-range columns stage finite values of
            // column 0 (their rows and columns are dropped by the epilogue); a
            // zero in a column gives infinite reciprocal variants, which reach
            // only the accumulators of the form whose domain excludes it.
            // The read form copies its v side from the image (32 bytes per thread
            // and chunk); the other forms form it from v and r.
            constexpr int kRawV = Sh::kRead ? 1 : kSV;
            // the read form's image chunk: kPB planes of kPlaneV values, one
            // 16-byte vector per thread
            static_assert(!Sh::kRead || kPB * kPlaneV * sizeof(h16) == 16 * Sh::kThreads, "image chunk per thread");
            struct Raw {
                float u[kSU], v[kRawV], r[kRawV];
                u32x4 i0;                             // image bytes (read form)
            };
            Raw pr;                                   // the next chunk to stage
            auto load_chunk = [&](int ch, Raw &x) {
                const int tu = min(ch * kKC + uks, tmax_u);
                load_floats<kSU>(ucol + tu, x.u);
                if constexpr (Sh::kRead) {
                    const int cc = min(ch, nch - 1);
                    const u32x4 *src = reinterpret_cast<const u32x4 *>(vimg + (size_t)(vt * nch + cc) * kPB * kPlaneV);
                    x.i0 = src[tid];                  // each wave instruction: 1 KB contiguous
                } else {
                    const int tv = min(ch * kKC + vks, tmax_v);
                    load_floats<kSV>(vcol + tv, x.v);
                    load_floats<kSV>(r32 + tv, x.r);
                }
            };
            auto store_chunk = [&](int ch, h16 *buf, bool tail) {
                // no contraction: U~, Z~, V~ r and W~ r are the same bits in
                // every mode, so the residual GEMMs agree exactly
#pragma clang fp contract(off)
                float ua[kUVar][kSU], va[kVVar][kSV];
#pragma unroll
                for (int e = 0; e < kSU; ++e) {
                    float uu = pr.u[e] - smu, zz = __builtin_amdgcn_rcpf(pr.u[e]) - smz;
                    if (tail) {                       // samples past n contribute nothing
                        const bool live = ch * kKC + uks + e < n;
                        uu = live ? uu : 0.f; zz = live ? zz : 0.f;
                    }
                    if constexpr (Sh::kRead) {
                        ua[0][e] = uu * cu; ua[1][e] = zz * cz;
                    } else {
                        ua[0][e] = uu * cu; ua[1][e] = (uu * uu) * cu2; ua[2][e] = zz * cz; ua[3][e] = (zz * zz) * cz2;
                    }
                }
#pragma unroll
                for (int q = 0; q < kUVar; ++q) put_h16<kSU>(buf + q * kPlaneU + sto_u, ua[q]);
                if constexpr (Sh::kRead) {
                    u32x4 *dst = reinterpret_cast<u32x4 *>(buf + kPA * kPlaneU);
                    dst[tid] = pr.i0;
                } else {
#pragma unroll
                    for (int e = 0; e < kSV; ++e) {
                        float vv = pr.v[e] - smv, ww = __builtin_amdgcn_rcpf(pr.v[e]) - smw, r = pr.r[e];
                        if (tail) {
                            const bool live = ch * kKC + vks + e < n;
                            vv = live ? vv : 0.f; ww = live ? ww : 0.f; r = live ? r : 0.f;
                        }
                        va[0][e] = vv * vsc.v; va[2][e] = (vv * (vv + 2.f * smv)) * vsc.p;
                        va[3][e] = (vv * (vv + smv)) * vsc.q;
                        va[4][e] = ww * vsc.w; va[6][e] = (ww * (ww + 2.f * smw)) * vsc.pw;
                        va[7][e] = (ww * (ww + smw)) * vsc.qw;
                        // V~ r and W~ r as the read form's image has them
                        v_resid_vars(pr.v[e], pr.r[e], smv, smw, vsc.vr, vsc.wr, !tail || ch * kKC + vks + e < n,
                                     va[1][e], va[5][e]);
                    }
#pragma unroll
                    for (int q = 0; q < kVVar; ++q) put_h16<kSV>(buf + kPA * kPlaneU + q * kPlaneV + sto_v, va[q]);
                }
            };
            // GEMM g: u-side variant GA[g], v-side variant GB[g]
            constexpr int GAf[12] = {0, 0, 1, 0, 0, 0, 1, 0, 2, 2, 3, 2};
            constexpr int GBf[12] = {0, 1, 2, 3, 4, 5, 6, 7, 0, 1, 2, 3};
            constexpr int GAr[3] = {0, 0, 1}, GBr[3] = {0, 1, 0};
            auto GA = [&](int g) { return Sh::kRead ? GAr[g] : GAf[g]; };
            auto GB = [&](int g) { return Sh::kRead ? GBr[g] : GBf[g]; };
            // Fragments of the staged chunk, then its MFMAs.  With a single staging
            // buffer a barrier between the two frees the buffer for the next chunk
            // (every wave holds its fragments in registers by then).
            auto mfma_chunk = [&](const h16 *buf) {
                h16x8 af[kPA], bfr[kSubV][kPB];
#pragma unroll
                for (int a = 0; a < kPA; ++a) af[a] = *reinterpret_cast<const h16x8 *>(buf + a * kAPlane + fa);
#pragma unroll
                for (int s2 = 0; s2 < kSubV; ++s2)
#pragma unroll
                    for (int q = 0; q < kPB; ++q)
                        bfr[s2][q] = *reinterpret_cast<const h16x8 *>(buf + kPA * kPlaneU + q * kPlaneV + fb[s2]);
#pragma unroll
                for (int s2 = 0; s2 < kSubV; ++s2)
#pragma unroll
                    for (int g = 0; g < kNG; ++g)
                        acc[s2][g] =
                            __builtin_amdgcn_mfma_f32_32x32x16_f16(af[GA(g)], bfr[s2][GB(g)], acc[s2][g], 0, 0, 0);
            };
            // interleave: fragment reads first, then each MFMA followed by a share of
            // the staging work of the next chunk (VALU and LDS stores)
            auto interleave = [&]() {
                __builtin_amdgcn_sched_group_barrier(0x100, kPA + kPB, 0);   // LDS reads
                __builtin_amdgcn_sched_group_barrier(0x020, 3, 0);           // global loads
#pragma unroll
                for (int i = 0; i < kNG; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);       // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, Sh::kRead ? 6 : 12, 0);   // VALU
                    if (i < kPA + kPB) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0); // LDS stores
                }
            };
            auto buf_of = [&](int c) { return stage + (c & 1) * kStage; };   // two staging buffers
            __syncthreads();                          // the previous tile's fragment reads are done
            if (tid < kSubV) lpend[tid] = 0;          // every thread has read the previous totals
            if constexpr (Sh::kRead) {
                // Both sides are copies of FP16 images already in the staged
                // layout (u: written for the moments pass, of which the read
                // form takes the first two planes, U~ and Z~; v: per residual).
                // Chunk c's 8 KB of u (4 KB of two 64-column image tiles) and
                // its 8 KB of v are 1 KB pieces, one of each per wave: wave w's
                // u piece is piece w % 4 of tile w / 4, at stage offset 512 w
                // either way.  A tile past the last one re-reads the last (its
                // columns are outside the space).  The pieces travel through a
                // ring of kRing chunks in registers (the loads of kRing - 1
                // chunks stay in flight while a chunk is computed: the reads
                // come from L2 and the MALL, and their latency is hidden only by
                // many bytes in flight), then into the staging buffers.
                constexpr int kR = Sh::kRing;
                static_assert(!Sh::kRead || (kPA * kPlaneU == 8 * 512 && kPB * kPlaneV == 8 * 512 &&
                                             Sh::kThreads == 512 && kPA * kAPlane == 4 * 512),
                              "one 1 KB u piece and one v piece per wave");
                const int64_t utile = u0 / 64 + (w >> 2) < nut64 ? u0 / 64 + (w >> 2) : nut64 - 1;
                const h16 *const ub = uimg + (size_t)utile * nch * (kUImgPlanes * kAPlane) + (w & 3) * 512 + lane * 8;
                const h16 *const vb = vimg + (size_t)vt * nch * (kPB * kPlaneV) + w * 512 + lane * 8;
                u32x4 ru[kR], rv[kR];
                // (a chunk past the last loads the last one again; it is staged
                // as zeros, so its MFMAs add nothing)
                auto fetch = [&](int c, u32x4 &a, u32x4 &b) {
                    const size_t cc = (size_t)(c < nch ? c : nch - 1);
                    a = *reinterpret_cast<const u32x4 *>(ub + cc * (kUImgPlanes * kAPlane));
                    b = *reinterpret_cast<const u32x4 *>(vb + cc * (kPB * kPlaneV));
                };
                // Three staging buffers and two fragment sets: in the turn of
                // chunk ch, the fragments of chunk ch + 1 are read, the MFMAs of
                // chunk ch run on the fragments read in the previous turn, and
                // chunk ch + 2 goes from its ring slot to its buffer (that of
                // chunk ch - 1, whose fragments every wave has read: each turn
                // ends in a barrier after this wave's LDS operations are done);
                // the slot is refilled with chunk ch + 2 + kR.  The LDS traffic
                // of a turn overlaps its MFMAs.
                struct Frags {
                    h16x8 a[kPA], b[kSubV][kPB];
                };
                auto read_frags = [&](const h16 *buf, Frags &f) {
#pragma unroll
                    for (int q = 0; q < kPA; ++q) f.a[q] = *reinterpret_cast<const h16x8 *>(buf + q * kAPlane + fa);
#pragma unroll
                    for (int s2 = 0; s2 < kSubV; ++s2)
#pragma unroll
                        for (int q = 0; q < kPB; ++q)
                            f.b[s2][q] = *reinterpret_cast<const h16x8 *>(buf + kPA * kPlaneU + q * kPlaneV + fb[s2]);
                };
                auto mfma_frags = [&](const Frags &f) {
#pragma unroll
                    for (int s2 = 0; s2 < kSubV; ++s2)
#pragma unroll
                        for (int g = 0; g < kNG; ++g)
                            acc[s2][g] = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.a[GA(g)], f.b[s2][GB(g)], acc[s2][g],
                                                                               0, 0, 0);
                };
                auto put = [&](h16 *buf, const u32x4 &x, const u32x4 &y, bool past) {
                    const u32x4 zero = {0u, 0u, 0u, 0u};
                    *reinterpret_cast<u32x4 *>(buf + w * 512 + lane * 8) = past ? zero : x;
                    *reinterpret_cast<u32x4 *>(buf + kPA * kPlaneU + w * 512 + lane * 8) = past ? zero : y;
                };
                static_assert(!Sh::kRead || (kR % 6 == 0 && Sh::kNStage == 3), "ring slot, fragment set and buffer "
                                                                               "of a chunk fixed within a group");
                // the first kR chunks, in order (the compiler's waits in the
                // loop assume the oldest load is the one needed first)
                static_for<kR>([&](auto S) {
                    fetch(decltype(S)::value, ru[S], rv[S]);
                    __builtin_amdgcn_sched_barrier(0);
                });
                Frags F[2];
                put(stage, ru[0], rv[0], false);
                fetch(kR, ru[0], rv[0]);
                put(stage + kStage, ru[1], rv[1], nch < 2);
                fetch(kR + 1, ru[1], rv[1]);
                lds_barrier();
                read_frags(stage, F[0]);
                // whole groups of kR chunks without a branch (the compiler's
                // waits then leave the ring's chunks in flight): turns past the
                // last chunk compute on zeros
                for (int c0 = 0; c0 < nch; c0 += kR)
                    static_for<kR>([&](auto S) {
                        constexpr int sc = decltype(S)::value;
                        constexpr int sl = (sc + 2) % kR;
                        read_frags(stage + ((sc + 1) % 3) * kStage, F[(sc + 1) & 1]);
                        mfma_frags(F[sc & 1]);
                        put(stage + ((sc + 2) % 3) * kStage, ru[sl], rv[sl], c0 + sc + 2 >= nch);
                        fetch(c0 + sc + 2 + kR, ru[sl], rv[sl]);
                        lds_barrier();
                    });
            } else {
                // pr holds chunk ch + 1 while chunk ch + 2 loads (loads past the last
                // chunk re-read it); deeper load rings were slower
                load_chunk(0, pr);
                store_chunk(0, stage, nch == 1);
                load_chunk(1, pr);
                __syncthreads();
                int ch = 0;
                for (; ch + 2 < nch; ++ch) {              // chunk ch + 1 is full
                    Raw q;
                    load_chunk(ch + 2, q);
                    mfma_chunk(buf_of(ch));
                    store_chunk(ch + 1, buf_of(ch + 1), false);
                    interleave();
                    pr = q;
                    __syncthreads();
                }
                if (ch + 1 < nch) {                       // chunk ch + 1 is the last one
                    mfma_chunk(buf_of(ch));
                    store_chunk(ch + 1, buf_of(ch + 1), true);
                    __syncthreads();
                    ++ch;
                }
                mfma_chunk(buf_of(ch));
            }

            if constexpr (Sh::kRead) {
                // The pass's three residual contractions of every pair of this
                // wave's sub-tiles, unscaled, into the moments' tiling (the
                // scorer of stored contractions reads them beside the moments);
                // a sub-tile past the last 64-column tile has no pair in the space
                static_for<kSubV>([&](auto SV) {
#pragma clang fp contract(off)
                    constexpr int sv = decltype(SV)::value;
                    const int64_t v32 = vt * (Sh::kWV * kSubV) + wv * kSubV + sv;
                    const int64_t u64 = (u0 + wu * 32) / 64;
                    if ((v32 >> 1) < nvt64 && u64 < nut64) {
                        const int64_t v = v0 + (wv * kSubV + sv) * 32 + (lane & 31);
                        const float4 vs0 = vsum[2 * (v < vcount ? v : 0)];
                        const VScale vc = v_scales(vs0.x, vs0.y, vs0.z, vs0.w, fn, rsc, shs);
                        const float ivr = 1.0f / vc.vr, iwr = 1.0f / vc.wr;
                        float *const cp =
                            cst + (((size_t)u64 * nvt64 + (v32 >> 1)) * 4 + (wu & 1) + 2 * (int)(v32 & 1)) * (16 * 3 * 64) +
                            lane;
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                            const float4 ui = ucon_c[wu * 32 + i];
                            __builtin_nontemporal_store((acc[sv][Sh::kCovUV][r] * ui.x) * ivr, cp + (r * 3 + 0) * 64);
                            __builtin_nontemporal_store((acc[sv][Sh::kCovUW][r] * ui.x) * iwr, cp + (r * 3 + 1) * 64);
                            __builtin_nontemporal_store((acc[sv][Sh::kCovZV][r] * ui.z) * ivr, cp + (r * 3 + 2) * 64);
                        }
                    }
                });
                continue;
            } else {
                // The plain form's epilogue.  Its code is kept small (runtime
                // loops over the rows, a row's accumulator values taken by a
                // uniform register index): unrolled, it outgrows the instruction
                // cache and is fetched again for every tile.
                auto &acs = acc[0];
                // lane holds column j = lane % 32 and rows
                // i = 8 (r / 4) + 4 (lane / 32) + (r % 4) of each 32 x 32 result
                const int j = lane & 31;
                const int64_t v = v0 + wv * 32 + j;
                const bool vin = v < vcount;
                const sisso_colstat vst = stats[vin ? v : 0];
                const float4 vs0 = vsum[2 * (vin ? v : 0)], vs1 = vsum[2 * (vin ? v : 0) + 1];
                const float mv = vs0.x, mw = vs0.y, Svv = vs0.z, Sww = vs0.w;
                const float rr = (float)(R1 / nd);
                const BfVCol vcol{mv,
                                  mw,
                                  Svv,
                                  vs1.x,
                                  vs1.y,
                                  vin && vst.valid != 0.0f,
                                  vst.minabs > 0.0f,
                                  col_scalable(Svv, Sww, fn, vst.minabs > 0.0f),
                                  units ? unit_of(units, vin ? v : 0) : make_uint4(0u, 0u, 0u, 0u)};
                // inverse scale factors of this lane's v column: the accumulator of
                // GEMM g times iu(row) iv(column) is the unscaled contraction
                const VScale vc = v_scales(mv, mw, Svv, Sww, fn, rsc, shs);
                const float iv = 1.0f / vc.v, ip = 1.0f / vc.p, iq = 1.0f / vc.q, ivr = 1.0f / vc.vr, iw = 1.0f / vc.w,
                            ipw = 1.0f / vc.pw, iqw = 1.0f / vc.qw, iwr = 1.0f / vc.wr;
                // Residual-independent moments of row r, from the accumulators: sum h
                // of u v, its variance, then the same for u/v and v/u.  A variance
                // below kCondRel of the magnitude of its terms is not resolved by the
                // FP16 operands: it is -1 (the candidate is scored exactly).  The
                // moments pass stores exactly these values.
                auto moments_acc = [&](int r, float (&m)[kMom]) {
#pragma clang fp contract(off)
                    const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const float4 us = ucon_a[wu * 32 + i], ui = ucon_c[wu * 32 + i];
                    const float mu = us.x, mz = us.y, Suu = us.z, Szz = us.w;
                    auto var_of = [&](float s1, float g2, float g3, float ma, float mb, float sa, float sb) {
                        const float t2 = 2.0f * ma * g3, t3 = mb * mb * sa, t4 = ma * ma * sb;
                        const float var = (g2 + t2 + t3 + t4) - s1 * s1 / fn;
                        const float mag = fabsf(g2) + fabsf(t2) + t3 + t4;
                        return var >= kCondRel * mag && var < INFINITY ? var : -1.0f;
                    };
                    m[0] = (acs[0][r] * ui.x) * iv;                 // u v
                    m[1] = var_of(m[0], (acs[2][r] * ui.y) * ip, (acs[3][r] * ui.x) * iq, mu, mv, Suu, Svv);
                    m[2] = (acs[4][r] * ui.x) * iw;                 // u / v
                    m[3] = var_of(m[2], (acs[6][r] * ui.y) * ipw, (acs[7][r] * ui.x) * iqw, mu, mw, Suu, Sww);
                    m[4] = (acs[8][r] * ui.z) * iv;                 // v / u
                    m[5] = var_of(m[4], (acs[10][r] * ui.w) * ip, (acs[11][r] * ui.z) * iq, mz, mv, Szz, Svv);
                };
                // the five forms of row r (see bf_forms)
                auto row_sums = [&](int r, float (&cov)[5], float (&var)[5], bool (&live)[5], bool (&flag)[5]) {
#pragma clang fp contract(off)
                    const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const float4 ui = ucon_c[wu * 32 + i];
                    float m[kMom];
                    moments_acc(r, m);
                    const float c0 = (acs[Sh::kCovUV][r] * ui.x) * ivr, c1 = (acs[Sh::kCovUW][r] * ui.x) * iwr,
                                c2 = (acs[Sh::kCovZV][r] * ui.z) * ivr;
                    bf_forms(ucon_a[wu * 32 + i], ucon_b[wu * 32 + i], ucon_u[wu * 32 + i], vcol, m, c0, c1, c2, rr, fs,
                             cov, var, live, flag);
                };
                auto row_scores = [&](int r, float (&sc)[5]) {
                    float cov[5], var[5];
                    bool live[5], flag[5];
                    row_sums(r, cov, var, live, flag);
                    bf_scores(cov, var, live, Srr, sc);
                };
                auto fid_of = [&](int r, int k) -> int64_t {
                    const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    return binbase + ((u0 + wu * 32 + i) * vcount + v) * S + fs.slot[k];
                };
                // every id of the tile inside [id_begin, id_end) (the usual case): no
                // per-candidate range check
                const int64_t tile_lo = binbase + (u0 * vcount + v0) * S;
                const int64_t tile_hi = binbase + ((u0 + kBTU - 1) * vcount + v0 + kBTV - 1) * S + S;
                const bool tile_in = tile_lo >= id_begin && tile_hi <= id_end;
                auto in_range = [&](int64_t id) { return tile_in || (id >= id_begin && id < id_end); };
                const float tb = fmaxf(*Lst.thr, load_gthr(gb));
                // Rows with a candidate at the bound, by a test without the reciprocal
                // square root: |cov| / sqrt(var Srr) >= tb as cov^2 >= var Srr tb^2,
                // loosened by a margin above the rounding of rsq and of the squares.
                // It may flag a row whose scores all fall below the bound (the exact
                // test then admits nothing from it), never the reverse.
                const bool no_bound = !(tb > 0.0f);
                const float k2 = (float)Srr * tb * tb * (1.0f - 1e-5f);
                unsigned rows = 0;                        // bit r: row r may have a candidate at the bound
#pragma unroll 1
                for (int r = 0; r < 16; ++r) {
                    float cov[5], var[5];
                    bool live[5], flag[5];
                    row_sums(r, cov, var, live, flag);
                    bool hit = false, fl = false;
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        hit = hit | (live[k] & (no_bound | (cov[k] * cov[k] >= var[k] * k2)));
                        fl = fl | flag[k];
                    }
                    rows |= (hit ? 1u : 0u) << r;
                    // flagged candidates in range join the list of exact scoring
                    // (the exclusion list is applied when they are scored)
                    if (fl) {
#pragma unroll
                        for (int k = 0; k < 5; ++k) {
                            const int64_t id = fid_of(r, k);
                            if (flag[k] && in_range(id)) {
                                const unsigned long long q = atomicAdd(side.cnt, 1ull);
                                if (q < (unsigned long long)side.cap) side.ids[q] = id;
                            }
                        }
                    }
                }
                bf_admit(Lst, gb, &lpend[0], rows, tb, excl, n_excl, row_scores, fid_of, in_range);
            }
        }
    }
    if constexpr (!Sh::kRead)
        list_flush(Lst, gb, W.sc + (size_t)blockIdx.x * keep, W.id + (size_t)blockIdx.x * keep);
}

#ifndef SISSO_BF16_MFMA_PART
// ------------------------------------------- scorer of stored contractions
//
// The second kernel of a pass that reads the moments: the five forms of every
// pair from the stored moments and the pass's three residual contractions
// (written by kBfRead), through bf_forms as the plain form scores them.  No
// accumulators are held; a block of eight waves (two per SIMD: at four per
// SIMD the 128-register budget spills) keeps several rows' loads in flight
// per wave.  A block stages the row constants of kScU 64-column u tiles in
// LDS, then each wave takes 32 x 32 sub-tiles of them.  Modes:
//   0 lists    every block keeps its best `keep` candidates in its LDS list
//              (rounds of kScWaves sub-tiles, one per wave, then bf_admit), as
//              the plain form does;
//   1 append   every candidate at or above a bound tau (read from the device:
//              tau_sc[tau_k - 1] when tau_cnt >= tau_k, else 0) is appended to
//              the flat array of the workspace's lists, no per-round barrier;
//              past app_cap entries the workspace reports scr_status 6;
//   2 maxima   the best candidate of each sub-tile (if in the slice and not
//              excluded) is appended, while room lasts (a lower bound for
//              mode 1: the band-th best of any set of the slice's candidates
//              is at most the slice's band-th best);
//   3 redo     mode 0 if the workspace's redo flag is set (an append that
//              overflowed), else nothing.
// Only u tiles u64_lo + t u64_step (t = 0, 1, ...) below u64_hi are scored.
constexpr int kScWaves = 8, kScThreads = 64 * kScWaves, kScU = 4;

__global__ void __launch_bounds__(kScThreads, 1) k_bf_score_stored(
    sisso_space s, FormSlots fs, int n, const float4 *__restrict__ usum, const float4 *__restrict__ vsum,
    const float2 *__restrict__ ures, const sisso_colstat *__restrict__ stats,
    const sisso_resid_info *__restrict__ info, const int64_t *__restrict__ excl, int n_excl, int64_t u64_lo,
    int64_t u64_hi, int64_t u64_step, int64_t id_begin, int64_t id_end, const float *__restrict__ mom,
    const float *__restrict__ cst, const int16_t *__restrict__ units, void *lws, int lists_total, int keep, int cap,
    int mode, const float *__restrict__ tau_sc, const int32_t *__restrict__ tau_cnt, int tau_k,
    unsigned long long *__restrict__ app_cnt, int64_t app_cap)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    if (mode == 3) {
        if (reinterpret_cast<const WsHeader *>(lws)->redo == 0) return;   // uniform: every thread leaves
        mode = 0;
    }
    const bool append = mode != 0;
    float *lsc = (float *)smem;
    int64_t *lid = (int64_t *)(lsc + cap);
    // the staged u tiles' row constants (as bf_forms takes them) and units
    float4 *ucon_a = reinterpret_cast<float4 *>(lid + cap), *ucon_b = ucon_a + 64 * kScU;
    uint4 *ucon_u = reinterpret_cast<uint4 *>(ucon_b + 64 * kScU);
    __shared__ int lcnt, lpend[2];                // lpend: candidates of a round (two, alternating)
    __shared__ float lthr;
    WsView W = ws_view(lws, lists_total, keep);
    if (threadIdx.x == 0) { lpend[0] = 0; lpend[1] = 0; }
    BlockList Lst{lsc, lid, &lcnt, &lthr, cap, keep};
    list_init(Lst);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, j = lane & 31;
    const int Lv = s.levels;
    const int64_t vcount = s.pool[Lv - 1], ulo = s.pool[Lv - 1], ucols = s.pool[Lv] - ulo;
    const int64_t binbase = s.pool[Lv] + s.rect_unary;
    const int S = s.n_slots;
    const double nd = (double)n, R1 = info->sum_r32, Srr = info->s_rr;
    const float fn = (float)n, rr = (float)(R1 / nd);
    const int64_t nvt64 = (vcount + 63) / 64;
    const int nsub = (int)(nvt64 * 4);
    const int64_t n_u = u64_hi > u64_lo ? (u64_hi - u64_lo + u64_step - 1) / u64_step : 0;
    const float tau = mode == 1 ? (*tau_cnt >= tau_k ? tau_sc[tau_k - 1] : 0.0f) : 0.0f;
    int round = 0;
    for (int64_t g0 = (int64_t)blockIdx.x * kScU; g0 < n_u; g0 += (int64_t)gridDim.x * kScU) {
        const int nt = n_u - g0 < kScU ? (int)(n_u - g0) : kScU;      // u tiles of this step
        __syncthreads();                              // the previous step's reads of the row constants are done
        if (tid < 64 * kScU) {
            const int t = tid >> 6;
            const int64_t x = (u64_lo + (g0 + t) * u64_step) * 64 + (tid & 63);
            const bool in = t < nt && x < ucols;
            const sisso_colstat cs = stats[ulo + (in ? x : 0)];
            const float2 b = ures[in ? x : 0];
            const float4 ua = usum[in ? x : 0];
            float flags = (in && cs.valid != 0.0f ? 1.0f : 0.0f) + (cs.minabs > 0.0f ? 2.0f : 0.0f);
            if (!col_scalable(ua.z, ua.w, fn, cs.minabs > 0.0f)) flags += 4.0f;
            ucon_a[tid] = ua;
            ucon_b[tid] = make_float4(b.x, b.y, cs.rms, flags);
            ucon_u[tid] = units ? unit_of(units, ulo + (in ? x : 0)) : make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();
        const int nq = nt * nsub;
        // sub-tile q of the step: u tile t = q / nsub, then 4 vt64 + su + 2 sv;
        // rows: bit r of the result, row r may have a candidate at the bound tb
        auto sub_tile = [&](int q, float tb, auto MX, auto &&emit) -> unsigned {
            constexpr bool kMax = decltype(MX)::value;
            const bool act = q >= 0;
            const int qa = act ? q : 0;
            const int t = qa / nsub, qq = qa - t * nsub;
            const int64_t u64 = u64_lo + (g0 + t) * u64_step;
            const int64_t vt64 = qq >> 2;
            const int su = qq & 1, svh = (qq >> 1) & 1;
            const int64_t v = vt64 * 64 + svh * 32 + j;
            const bool vin = act && v < vcount;
            const sisso_colstat vst = stats[vin ? v : 0];
            const float4 vs0 = vsum[2 * (vin ? v : 0)], vs1 = vsum[2 * (vin ? v : 0) + 1];
            const BfVCol vcol{vs0.x,
                              vs0.y,
                              vs0.z,
                              vs1.x,
                              vs1.y,
                              vin && vst.valid != 0.0f,
                              vst.minabs > 0.0f,
                              col_scalable(vs0.z, vs0.w, fn, vst.minabs > 0.0f),
                              units ? unit_of(units, vin ? v : 0) : make_uint4(0u, 0u, 0u, 0u)};
            const size_t sub = ((size_t)u64 * nvt64 + vt64) * 4 + (qq & 3);
            const float *const mp = mom + sub * (16 * kMom * 64) + lane;
            const float *const cp = cst + sub * (16 * 3 * 64) + lane;
            const int64_t ub0 = u64 * 64 + su * 32, vb0 = vt64 * 64 + svh * 32;
            const int ucb = t * 64 + su * 32;
            auto forms = [&](int r, const float (&m)[kMom], float c0, float c1, float c2, float (&cov)[5],
                             float (&var)[5], bool (&live)[5], bool (&flag)[5]) {
                const int i = ucb + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                bf_forms(ucon_a[i], ucon_b[i], ucon_u[i], vcol, m, c0, c1, c2, rr, fs, cov, var, live, flag);
            };
            auto row_scores = [&](int r, float (&sc)[5]) {
                float m[kMom];
#pragma unroll
                for (int k = 0; k < kMom; ++k) m[k] = __builtin_nontemporal_load(mp + (r * kMom + k) * 64);
                const float c0 = __builtin_nontemporal_load(cp + (r * 3 + 0) * 64),
                            c1 = __builtin_nontemporal_load(cp + (r * 3 + 1) * 64),
                            c2 = __builtin_nontemporal_load(cp + (r * 3 + 2) * 64);
                float cov[5], var[5];
                bool live[5], flag[5];
                forms(r, m, c0, c1, c2, cov, var, live, flag);
                bf_scores(cov, var, live, Srr, sc);
            };
            auto fid_of = [&](int r, int k) -> int64_t {
                const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                return binbase + ((ub0 + i) * vcount + v) * S + fs.slot[k];
            };
            const int64_t tile_lo = binbase + (ub0 * vcount + vb0) * S;
            const int64_t tile_hi = binbase + ((ub0 + 31) * vcount + vb0 + 31) * S + S;
            const bool tile_in = tile_lo >= id_begin && tile_hi <= id_end;
            auto in_range = [&](int64_t id) { return tile_in || (id >= id_begin && id < id_end); };
            // the test of the plain form: cov^2 >= var Srr tb^2, loosened
            const bool no_bound = !(tb > 0.0f);
            const float k2 = (float)Srr * tb * tb * (1.0f - 1e-5f);
            unsigned rows = 0;
            float best = -1.0f;                       // maxima: this lane's best live score, row, form
            int best_r = 0, best_k = 0;
            if (act) {
                // four rows at a time, the next four rows' loads in flight
                constexpr int kG = 4 * (kMom + 3);
                float cur[kG], nxt[kG];
                auto load4 = [&](int g, float (&d)[kG]) {
#pragma unroll
                    for (int q2 = 0; q2 < 4 * kMom; ++q2) d[q2] = __builtin_nontemporal_load(mp + (g * 4 * kMom + q2) * 64);
#pragma unroll
                    for (int q2 = 0; q2 < 12; ++q2) d[4 * kMom + q2] = __builtin_nontemporal_load(cp + (g * 12 + q2) * 64);
                };
                load4(0, nxt);
                static_for<4>([&](auto G) {
                    constexpr int g = decltype(G)::value;
#pragma unroll
                    for (int e = 0; e < kG; ++e) cur[e] = nxt[e];
                    if constexpr (g + 1 < 4) load4(g + 1, nxt);
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4) {
                        const int r = 4 * g + r4;
                        float m[kMom];
#pragma unroll
                        for (int k = 0; k < kMom; ++k) m[k] = cur[r4 * kMom + k];
                        float cov[5], var[5];
                        bool live[5], flag[5];
                        forms(r, m, cur[4 * kMom + r4 * 3], cur[4 * kMom + r4 * 3 + 1], cur[4 * kMom + r4 * 3 + 2],
                              cov, var, live, flag);
                        if constexpr (kMax) {
                            float sc[5];
                            bf_scores(cov, var, live, Srr, sc);
#pragma unroll
                            for (int k = 0; k < 5; ++k) {
                                const bool b = sc[k] > best;
                                best = b ? sc[k] : best;
                                best_r = b ? r : best_r;
                                best_k = b ? k : best_k;
                            }
                        } else {
                            bool hit = false;
#pragma unroll
                            for (int k = 0; k < 5; ++k)
                                hit = hit | (live[k] & (no_bound | (cov[k] * cov[k] >= var[k] * k2)));
                            rows |= (hit ? 1u : 0u) << r;
                        }
                    }
                });
            }
            if constexpr (kMax) {
                // the sub-tile's best: the lowest lane holding the wave's maximum
                const float wm = wave_max(best);
                const unsigned long long who = __ballot(best == wm && wm >= 0.0f);
                if (who != 0ull && lane == __builtin_ctzll(who)) {
                    const int64_t id = fid_of(best_r, best_k);
                    if (in_range(id) && (n_excl == 0 || !in_sorted_ids(excl, n_excl, id))) {
                        const unsigned long long slot = atomicAdd(app_cnt, 1ull);
                        if (slot < (unsigned long long)app_cap) {
                            W.sc[slot] = wm;
                            W.id[slot] = id;
                        }
                    }
                }
            } else {
                emit(rows, row_scores, fid_of, in_range);
            }
            return rows;
        };
        if (append) {
            // every candidate at or above tau, in range and not excluded, to
            // the flat array; waves take the step's sub-tiles independently
            for (int q = w; q < nq; q += kScWaves) {
                if (mode == 2) {
                    sub_tile(q, 0.0f, std::true_type{}, [](unsigned, auto &, auto &, auto &) {});
                    continue;
                }
                sub_tile(q, tau, std::false_type{}, [&](unsigned rows, auto &row_scores, auto &fid_of, auto &in_range) {
#pragma unroll 1
                    for (int r = 0; r < 16; ++r) {
                        if (!((rows >> r) & 1u)) continue;
                        float sc[5];
                        row_scores(r, sc);
#pragma unroll
                        for (int k = 0; k < 5; ++k) {
                            if (!(sc[k] >= 0.0f && sc[k] >= tau)) continue;
                            const int64_t id = fid_of(r, k);
                            if (!in_range(id) || (n_excl != 0 && in_sorted_ids(excl, n_excl, id))) continue;
                            const unsigned long long slot = atomicAdd(app_cnt, 1ull);
                            if (slot < (unsigned long long)app_cap) {
                                W.sc[slot] = sc[k];
                                W.id[slot] = id;
                            } else {
                                W.h->scr_status = 6;
                            }
                        }
                    }
                });
            }
        } else {
            // rounds of sixteen sub-tiles, one per wave, each ending in bf_admit
            for (int q0 = 0; q0 < nq; q0 += kScWaves, ++round) {
                const int q = q0 + w < nq ? q0 + w : -1;
                const float tb = fmaxf(*Lst.thr, load_gthr(&W.h->gthr));
                sub_tile(q, tb, std::false_type{}, [&](unsigned rows, auto &row_scores, auto &fid_of, auto &in_range) {
                    bf_admit(Lst, &W.h->gthr, &lpend[round & 1], rows, tb, excl, n_excl, row_scores, fid_of,
                             in_range);
                });
                // every thread read this round's count before the barrier below;
                // the next round's counter was last read before the previous round's
                if (tid == 0) lpend[(round + 1) & 1] = 0;
                __syncthreads();
            }
        }
    }
    if (!append) list_flush(Lst, &W.h->gthr, W.sc + (size_t)blockIdx.x * keep, W.id + (size_t)blockIdx.x * keep);
}

// Fill of a workspace's first n_entries list entries with empty slots (score
// -1, id INT64_MAX) before an append-mode scorer writes into them.
__global__ void k_bf_lists_clear(void *lws, int lists_total, int keep, int64_t n_entries)
{
    WsView W = ws_view(lws, lists_total, keep);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_entries; e += (int64_t)gridDim.x * blockDim.x) {
        W.sc[e] = -1.0f;
        W.id[e] = INT64_MAX;
    }
}
#endif  // SISSO_BF16_MFMA_PART

#ifdef SISSO_BF16_MFMA_PART
// ----------------------------------------------------------- moments pass
//
// The first pass of a fit: per (u, v) pair of the binary block, the six
// residual-independent moments the read form's scorer loads (sum h and the
// variance of u v, u/v and v/u), from the nine residual-independent
// contractions of the full form, and the conditioning flags of the five forms
// (the flagged candidates join the list of exact scoring).  Both sides'
// operands are first written once as FP16 images in the staged layout (the u
// side's four planes, which the read form reuses, and the v side's six), so
// that the pass itself only copies chunks into LDS and runs MFMAs: block tile
// 64 u x 128 v (one u image tile, one v image tile), eight waves (two along u,
// four along v), one 32 x 32 sub-tile each.  Every staged value takes the
// full form's operations and every accumulator its order, so the moments and
// flags are the bits the full form computes.
//   g:  0   1    2   3   4    5    6   7    8
//   A:  U~  U~2  U~  U~  U~2  U~   Z~  Z~2  Z~
//   B:  V~  P    Q   W~  Pw   Qw   V~  P    Q

// The u side's image over the 64-column tiles [ut_lo, ut_hi): per tile and
// chunk, the planes U~, Z~, U~^2, Z~^2 as the full form stages them (columns
// past the last take column 0's values, samples past n zeros).  Block: one
// tile at a time; thread t: column t / 4, samples 4 (t % 4) .. + 3 of a chunk.
__global__ void __launch_bounds__(256) k_bf16_u_image(int n, const float *__restrict__ pool32, int64_t ld32,
                                                      int64_t ulo, int64_t ucols, const float4 *__restrict__ usum,
                                                      int64_t ut_lo, int64_t ut_hi, h16 *__restrict__ uimg)
{
#pragma clang fp contract(off)
    const int c = threadIdx.x >> 2, k0 = (threadIdx.x & 3) * 4;
    const int nch = (n + kKC - 1) / kKC, tmax = ((n - 1) / 4) * 4;
    const float fn = (float)n, shs = sq_shift(n);
    const int off = lds_off(c, k0);
    for (int64_t ut = ut_lo + blockIdx.x; ut < ut_hi; ut += gridDim.x) {
        const int64_t su = ut * 64 + c;
        const bool su_ok = su < ucols;
        const float4 us = usum[su_ok ? su : 0];
        const float smu = us.x, smz = us.y;
        const UScale usc = u_scales(us.z, us.w, fn);
        const float cu = usc.u, cz = usc.z, cu2 = usc.u * usc.u * shs, cz2 = usc.z * usc.z * shs;
        const float *col = pool32 + (size_t)(ulo + (su_ok ? su : 0)) * ld32;
        h16 *const dst = uimg + (size_t)ut * nch * (kUImgPlanes * 64 * kKR) + off;
        for (int ch = 0; ch < nch; ++ch) {
            float x[4], ua[kUImgPlanes][4];
            load_floats<4>(col + min(ch * kKC + k0, tmax), x);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float uu = x[e] - smu, zz = __builtin_amdgcn_rcpf(x[e]) - smz;
                const bool live = ch * kKC + k0 + e < n;
                uu = live ? uu : 0.f; zz = live ? zz : 0.f;
                ua[0][e] = uu * cu; ua[1][e] = zz * cz; ua[2][e] = (uu * uu) * cu2; ua[3][e] = (zz * zz) * cz2;
            }
#pragma unroll
            for (int q = 0; q < kUImgPlanes; ++q) put_h16<4>(dst + (size_t)ch * (kUImgPlanes * 64 * kKR) + q * (64 * kKR), ua[q]);
        }
    }
}

// The v side's image for the moments pass: per 128-column tile and chunk, the
// planes V~, P, Q, W~, Pw, Qw.  Block (vt, ch); thread t: column t / 2,
// samples 8 (t % 2) .. + 7.
__global__ void __launch_bounds__(256) k_bf16_vm_image(int n, const float *__restrict__ pool32, int64_t ld32,
                                                       int64_t vcols, const float4 *__restrict__ vsum,
                                                       h16 *__restrict__ img)
{
#pragma clang fp contract(off)
    const int nch = (n + kKC - 1) / kKC;
    const int64_t vt = blockIdx.x / nch;
    const int ch = blockIdx.x % nch;
    const int c = threadIdx.x >> 1, k0 = (threadIdx.x & 1) * 8;
    const int64_t v = vt * 128 + c;
    const int64_t vv = v < vcols ? v : 0;
    const float4 vs = vsum[2 * vv];
    const float smv = vs.x, smw = vs.y;
    const VScale vsc = v_scales(smv, smw, vs.z, vs.w, (float)n, 1.0f, sq_shift(n));
    const float *col = pool32 + (size_t)vv * ld32;
    float va[kVmPlanes][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int t = ch * kKC + k0 + e;
        const float x = col[t < n ? t : n - 1];
        float d = x - smv, w = __builtin_amdgcn_rcpf(x) - smw;
        const bool live = t < n;
        d = live ? d : 0.f; w = live ? w : 0.f;
        va[0][e] = d * vsc.v; va[1][e] = (d * (d + 2.f * smv)) * vsc.p; va[2][e] = (d * (d + smv)) * vsc.q;
        va[3][e] = w * vsc.w; va[4][e] = (w * (w + 2.f * smw)) * vsc.pw; va[5][e] = (w * (w + smw)) * vsc.qw;
    }
    h16 *const out = img + (size_t)blockIdx.x * (kVmPlanes * 128 * kKR) + lds_off(c, k0);
#pragma unroll
    for (int q = 0; q < kVmPlanes; ++q) {
        h16 hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[e] = (h16)va[q][e];
        __builtin_memcpy(out + q * (128 * kKR), hv, 16);
    }
}

struct MomShape {
    static constexpr int kWU = 2, kWV = 4, kBTU = 32 * kWU, kBTV = 32 * kWV, kThreads = 64 * kWU * kWV;
    static constexpr int kPA = kUImgPlanes, kPB = kVmPlanes, kNG = 9;
    static constexpr int kPlaneU = kBTU * kKR, kPlaneV = kBTV * kKR;
    static constexpr int kStage = kPA * kPlaneU;                   // the u image's tile-chunk (LDS)
    static constexpr int kRing = 2;                                // chunks held in registers
};
static_assert(8 * MomShape::kThreads == MomShape::kStage, "one 16-byte u piece per thread and chunk");

__global__ void __launch_bounds__(MomShape::kThreads, 1) k_bf_moments(
    sisso_space s, FormSlots fs, int n, const float4 *__restrict__ usum, const float4 *__restrict__ vsum,
    const sisso_colstat *__restrict__ stats, int64_t ut_lo, int64_t ut_hi, int64_t id_begin, int64_t id_end,
    float *__restrict__ mom, const h16 *uimg, const h16 *vmimg, const int16_t *__restrict__ units, BfSide side)
{
    using Sh = MomShape;
    constexpr int kPA = Sh::kPA, kPB = Sh::kPB, kNG = Sh::kNG, kStage = Sh::kStage, kBTU = Sh::kBTU,
                  kBTV = Sh::kBTV, kPlaneU = Sh::kPlaneU, kPlaneV = Sh::kPlaneV, kR = Sh::kRing;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    h16 *const stage = reinterpret_cast<h16 *>(smem);            // two staging buffers
    // u-tile constants: (mean u, mean 1/u, sum u~^2, sum z~^2), the inverse
    // scale factors of U~, U~^2, Z~, Z~^2, flags (1 valid, 2 no zero, 4 not
    // scalable), units (zero without units)
    float4 *ucon_a = reinterpret_cast<float4 *>(stage + 2 * kStage), *ucon_c = ucon_a + kBTU;
    uint4 *ucon_u = reinterpret_cast<uint4 *>(ucon_c + kBTU);
    int *ucon_f = reinterpret_cast<int *>(ucon_u + kBTU);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wu = w % Sh::kWU, wv = w / Sh::kWU;
    const int Lv = s.levels;
    const int64_t vcount = s.pool[Lv - 1], ulo = s.pool[Lv - 1], ucols = s.pool[Lv] - ulo;
    const int64_t binbase = s.pool[Lv] + s.rect_unary;
    const int S = s.n_slots;
    const float fn = (float)n, shs = sq_shift(n);
    const int nch = (n + kKC - 1) / kKC;
    const int64_t nvt = (vcount + kBTV - 1) / kBTV, nvt64 = (vcount + 63) / 64;
    const int koff = (lane >> 5) * 8;
    const int fa = lds_off(wu * 32 + (lane & 31), koff), fb = lds_off(wv * 32 + (lane & 31), koff);
    // A plane of GEMM g in the image's order (U~, Z~, U~^2, Z~^2); B plane
    constexpr int GA[kNG] = {0, 2, 0, 0, 2, 0, 1, 3, 1};
    constexpr int GB[kNG] = {0, 1, 2, 3, 4, 5, 0, 1, 2};
    // (u, v) tiles, v fastest, in turns of eight runs of gridDim.x / 8, one
    // run per XCD (the blocks of an XCD share their u images in its L2)
    const int64_t T = (ut_hi - ut_lo) * nvt;
    const bool by_xcd = gridDim.x % 8 == 0;
    const int64_t gx = blockIdx.x % 8, gk = blockIdx.x / 8, gn = gridDim.x / 8;
    int64_t ut_cur = -1;
    for (int64_t it = 0;; ++it) {
        const int64_t t = by_xcd ? (it * 8 + gx) * gn + gk : it * gridDim.x + blockIdx.x;
        if (t >= T) break;
        const int64_t ut = ut_lo + t / nvt, vt = t % nvt;
        const int64_t u0 = ut * kBTU, v0 = vt * kBTV;
        __syncthreads();                              // the previous tile's reads of LDS are done
        if (ut != ut_cur && tid < kBTU) {
            const int64_t x = u0 + tid;
            const bool in = x < ucols;
            const sisso_colstat cs = stats[ulo + (in ? x : 0)];
            const float4 ua = usum[in ? x : 0];
            ucon_a[tid] = ua;
            const UScale c = u_scales(ua.z, ua.w, fn);
            ucon_c[tid] = make_float4(1.0f / c.u, 1.0f / (c.u * c.u * shs), 1.0f / c.z, 1.0f / (c.z * c.z * shs));
            ucon_f[tid] = (in && cs.valid != 0.0f ? 1 : 0) + (cs.minabs > 0.0f ? 2 : 0) +
                          (col_scalable(ua.z, ua.w, fn, cs.minabs > 0.0f) ? 0 : 4);
            ucon_u[tid] = units ? unit_of(units, ulo + (in ? x : 0)) : make_uint4(0u, 0u, 0u, 0u);
        }
        ut_cur = ut;
        f32x16 acc[kNG];
#pragma unroll
        for (int g = 0; g < kNG; ++g)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[g][e] = 0.0f;
        // Chunks.  The u side (shared by the four waves along v) goes through
        // LDS: its image tile-chunk, one 16-byte piece per thread, through a
        // ring of kR chunks in registers into two staging buffers (a chunk
        // past the last is staged as zeros: its MFMAs add nothing; no branch
        // around a load).  The v side (shared by two waves only) is loaded by
        // each wave as its own MFMA fragments straight from the image, whose
        // layout is the staged one: no LDS traffic for it.
        const h16 *const ub = uimg + (size_t)ut * nch * kStage + tid * 8;
        const h16 *const vb = vmimg + (size_t)vt * nch * (kPB * kPlaneV) + fb;
        struct Slot {
            u32x4 u;
            h16x8 b[kPB];
        };
        Slot ring[kR];
        auto fetch = [&](int c, Slot &d) {
            const size_t cc = (size_t)(c < nch ? c : nch - 1);
            d.u = *reinterpret_cast<const u32x4 *>(ub + cc * kStage);
#pragma unroll
            for (int q = 0; q < kPB; ++q)
                d.b[q] = *reinterpret_cast<const h16x8 *>(vb + cc * (kPB * kPlaneV) + q * kPlaneV);
        };
        static_for<kR>([&](auto S2) {
            fetch(decltype(S2)::value, ring[S2]);
            __builtin_amdgcn_sched_barrier(0);
        });
        static_assert(kR == 2, "ring slot and buffer of a chunk fixed within a group");
        for (int c0 = 0; c0 < nch; c0 += kR)
            static_for<kR>([&](auto S2) {
                constexpr int sc = decltype(S2)::value;
                h16 *const buf = stage + sc * kStage;
                const u32x4 zero = {0u, 0u, 0u, 0u};
                *reinterpret_cast<u32x4 *>(buf + tid * 8) = c0 + sc >= nch ? zero : ring[sc].u;
                // this wave's store is done and every wave is past the
                // fragment reads of chunk c - 2 (the buffer's previous user)
                lds_barrier();
                h16x8 af[kPA];
#pragma unroll
                for (int q = 0; q < kPA; ++q) af[q] = *reinterpret_cast<const h16x8 *>(buf + q * kPlaneU + fa);
#pragma unroll
                for (int g = 0; g < kNG; ++g)
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[GA[g]], ring[sc].b[GB[g]], acc[g], 0, 0, 0);
                fetch(c0 + sc + kR, ring[sc]);
            });

        // epilogue: lane holds column j = lane % 32 and rows
        // i = 8 (r / 4) + 4 (lane / 32) + (r % 4) of each 32 x 32 result
        const int j = lane & 31;
        const int64_t v = v0 + wv * 32 + j;
        const bool vin = v < vcount;
        const sisso_colstat vst = stats[vin ? v : 0];
        const float4 vs0 = vsum[2 * (vin ? v : 0)];
        const float mv = vs0.x, mw = vs0.y, Svv = vs0.z, Sww = vs0.w;
        const VScale vc = v_scales(mv, mw, Svv, Sww, fn, 1.0f, shs);
        const float iv = 1.0f / vc.v, ip = 1.0f / vc.p, iq = 1.0f / vc.q, iw = 1.0f / vc.w, ipw = 1.0f / vc.pw,
                    iqw = 1.0f / vc.qw;
        const bool vscal = col_scalable(Svv, Sww, fn, vst.minabs > 0.0f);
        const uint4 vunit = units ? unit_of(units, vin ? v : 0) : make_uint4(0u, 0u, 0u, 0u);
        const int64_t v32 = vt * Sh::kWV + wv;
        const int64_t u64 = ut;
        const bool mom_in = (v32 >> 1) < nvt64;
        float *const mp = mom + (((size_t)u64 * nvt64 + (v32 >> 1)) * 4 + wu + 2 * (int)(v32 & 1)) *
                                    (16 * kMom * 64) + lane;
        const int64_t tile_lo = binbase + (u0 * vcount + v0) * S;
        const int64_t tile_hi = binbase + ((u0 + kBTU - 1) * vcount + v0 + kBTV - 1) * S + S;
        const bool tile_in = tile_lo >= id_begin && tile_hi <= id_end;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma clang fp contract(off)
            const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const float4 us = ucon_a[wu * 32 + i], ui = ucon_c[wu * 32 + i];
            const int uf = ucon_f[wu * 32 + i];
            const float mu = us.x, mz = us.y, Suu = us.z, Szz = us.w;
            auto var_of = [&](float s1, float g2, float g3, float ma, float mb, float sa, float sb) {
                const float t2 = 2.0f * ma * g3, t3 = mb * mb * sa, t4 = ma * ma * sb;
                const float var = (g2 + t2 + t3 + t4) - s1 * s1 / fn;
                const float mag = fabsf(g2) + fabsf(t2) + t3 + t4;
                return var >= kCondRel * mag && var < INFINITY ? var : -1.0f;
            };
            float m[kMom];
            m[0] = (acc[0][r] * ui.x) * iv;                 // u v
            m[1] = var_of(m[0], (acc[1][r] * ui.y) * ip, (acc[2][r] * ui.x) * iq, mu, mv, Suu, Svv);
            m[2] = (acc[3][r] * ui.x) * iw;                 // u / v
            m[3] = var_of(m[2], (acc[4][r] * ui.y) * ipw, (acc[5][r] * ui.x) * iqw, mu, mw, Suu, Sww);
            m[4] = (acc[6][r] * ui.z) * iv;                 // v / u
            m[5] = var_of(m[4], (acc[7][r] * ui.w) * ip, (acc[8][r] * ui.z) * iq, mz, mv, Szz, Svv);
            if (mom_in) {
#pragma unroll
                for (int k = 0; k < kMom; ++k) __builtin_nontemporal_store(m[k], mp + (r * kMom + k) * 64);
            }
            // the read form's conditioning decision, from the same values
            const bool ok = ((uf & 1) != 0) & vin & (vst.valid != 0.0f);
            const bool unscal = ((uf & 4) != 0) | !vscal;
            const float var[5] = {Suu + Svv + 2.0f * m[0], Suu + Svv - 2.0f * m[0], m[1], m[3], m[5]};
            const bool same_u = unit_eq(ucon_u[wu * 32 + i], vunit);   // sums and differences
            const bool dom[5] = {same_u, same_u, true, vst.minabs > 0.f, (uf & 2) != 0};
            const float cth = kCondRel * (Suu + Svv);
            bool any = false, flag[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const bool cand = ok & dom[k] & (fs.slot[k] >= 0);
                const bool good = !unscal & (k < 2 ? var[k] >= cth : var[k] > 0.0f) & (var[k] < INFINITY);
                flag[k] = cand & !good;
                any = any | flag[k];
            }
            if (any) {
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const int64_t id = binbase + ((u0 + wu * 32 + i) * vcount + v) * S + fs.slot[k];
                    if (flag[k] && (tile_in || (id >= id_begin && id < id_end))) {
                        const unsigned long long q = atomicAdd(side.cnt, 1ull);
                        if (q < (unsigned long long)side.cap) side.ids[q] = id;
                    }
                }
            }
        }
    }
}
#endif  // SISSO_BF16_MFMA_PART

#ifndef SISSO_BF16_MFMA_PART
// --------------------------------------------------------------- rescore

// Exact FP32 score of every band id, with the plain kernel's arithmetic: the
// same staged values, pilot shifts, chunked FP32 partial sums carried in FP64
// and validity rules.  One thread per candidate.
__global__ void __launch_bounds__(256) k_rescore_ids(sisso_space s, FormSlots fs, int n,
                                                     const float *__restrict__ pool32, int64_t ld32,
                                                     const sisso_colstat *__restrict__ stats,
                                                     const float *__restrict__ r32,
                                                     const sisso_resid_info *__restrict__ info,
                                                     const int64_t *__restrict__ ids, const int32_t *__restrict__ count,
                                                     const int64_t *__restrict__ excl, int n_excl, int list_base,
                                                     void *ws, int lists_total, int keep, int cap)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *lsc = (float *)smem;
    int64_t *lid = (int64_t *)(smem + cap * sizeof(float));
    __shared__ int lcnt;
    __shared__ float lthr;
    WsView W = ws_view(ws, lists_total, keep);
    BlockList L{lsc, lid, &lcnt, &lthr, cap, keep};
    list_init(L);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    float osc[1] = {-1.0f};
    int64_t oid[1] = {INT64_MAX};
    if (q < *count) {
        const int64_t id = ids[q];
        const float sc = score_slice_id(s, fs, n, pool32, ld32, stats, r32, info, id);
        if (sc >= 0.0f) { osc[0] = sc; oid[0] = id; }
    }
    list_offer<1>(L, osc, oid, &W.h->gthr, excl, n_excl);
    const int list = list_base + blockIdx.x;
    list_flush(L, &W.h->gthr, W.sc + (size_t)list * keep, W.id + (size_t)list * keep);
}

// Score of binary slice candidate `id` by one wave (lanes over the samples,
// FP32 partial sums per lane, FP64 wave sums), with the validity, magnitude and
// cancellation rules of the exact kernels; -1 if invalid.  Used for the
// candidates the 16-bit screen cannot rank; the band rescore then gives every
// reported candidate its exact FP32 score.
__device__ inline float score_slice_id_wave(const sisso_space &s, const FormSlots &fs, int n,
                                            const float *__restrict__ pool32, int64_t ld32,
                                            const sisso_colstat *__restrict__ stats, const float *__restrict__ r32,
                                            double nd, double R1, double Srr, int64_t id)
{
    const int lane = threadIdx.x & 63;
    const int Lv = s.levels;
    const int64_t binbase = s.pool[Lv] + s.rect_unary;
    if (s.rect != 1 || id < binbase || id >= s.total) return -1.0f;
    const int64_t loc = id - binbase, vcount = s.pool[Lv - 1];
    const int slot = (int)(loc % s.n_slots);
    const int64_t pair = loc / s.n_slots;
    const int64_t u = s.pool[Lv - 1] + pair / vcount, v = pair % vcount;
    int k = -1;
    for (int f = 0; f < 5; ++f)
        if (fs.slot[f] == slot) k = f;
    const sisso_colstat ust = stats[u], vst = stats[v];
    if (k < 0 || ust.valid == 0.0f || vst.valid == 0.0f) return -1.0f;
    if ((k == 3 && !(vst.minabs > 0.0f)) || (k == 4 && !(ust.minabs > 0.0f))) return -1.0f;
    const float *cu = pool32 + (size_t)u * ld32, *cv = pool32 + (size_t)v * ld32;
    const float cm = ust.mean * vst.mean, c3 = ust.mean * vst.mean_rcp, c4 = vst.mean * ust.mean_rcp;
    float fA = 0.f, fB = 0.f, fC = 0.f;
    auto step = [&](float ur, float vr, float r) {
        const float g = binary_form(k, ur, ur - ust.mean, __builtin_amdgcn_rcpf(ur), vr, vr - vst.mean,
                                    __builtin_amdgcn_rcpf(vr), cm, c3, c4);
        fA += g;
        fB = fmaf(g, g, fB);
        fC = fmaf(g, r, fC);
    };
    for (int t = lane * 4; t < n; t += 256) {     // 16-byte loads: samples t .. t + 3
        const float4 a4 = *reinterpret_cast<const float4 *>(cu + t);
        const float4 b4 = *reinterpret_cast<const float4 *>(cv + t);
        const float4 r4 = *reinterpret_cast<const float4 *>(r32 + t);
        const float ua[4] = {a4.x, a4.y, a4.z, a4.w}, va[4] = {b4.x, b4.y, b4.z, b4.w};
        const float ra[4] = {r4.x, r4.y, r4.z, r4.w};
        if (t + 3 < n) {                           // the lane's four samples all lie below n
#pragma unroll
            for (int e = 0; e < 4; ++e) step(ua[e], va[e], ra[e]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < n) step(ua[e], va[e], ra[e]);
        }
    }
    const double A = wave_sum_dpp((double)fA), B = wave_sum_dpp((double)fB), C = wave_sum_dpp((double)fC);
    const double shifts[5] = {(double)ust.mean + (double)vst.mean, (double)ust.mean - (double)vst.mean,
                              (double)cm, (double)c3, (double)c4};
    return form_score(k, (float)A, B, C, shifts[k], cu, cv, n, ust.maxabs, ust.minabs, ust.rms, vst.maxabs,
                      vst.minabs, vst.rms, nd, R1, Srr);
}

// Scores of the flagged candidates, one wave per candidate, written as extra
// lists of the band workspace after the screen's l0 lists: entry e at list
// l0 + e / keep, slot e % keep (-1 for an entry outside [id_begin, id_end)
// or excluded, and for the padding of the last list).  Every flagged
// candidate is kept, so the band's merge does not depend on the order in
// which the screen stored them.  An overflowing list is reported (3).
__global__ void __launch_bounds__(256) k_bf_side(sisso_space s, FormSlots fs, int n, const float *__restrict__ pool32,
                                                 int64_t ld32, const sisso_colstat *__restrict__ stats,
                                                 const float *__restrict__ r32,
                                                 const sisso_resid_info *__restrict__ info,
                                                 const int64_t *__restrict__ excl, int n_excl, int64_t id_begin,
                                                 int64_t id_end, BfSide side, void *lws, int lists_total, int keep,
                                                 int l0)
{
    WsView W = ws_view(lws, lists_total, keep);
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const unsigned long long c = *side.cnt;
    const int64_t cnt = c < (unsigned long long)side.cap ? (int64_t)c : side.cap;
    const int64_t nl = (cnt + keep - 1) / keep;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        W.h->n_lists = l0 + (int)nl;
        if (c > (unsigned long long)side.cap) W.h->scr_status = 3;
    }
    const double nd = (double)n, R1 = info->sum_r32, Srr = info->s_rr;
    float *const osc = W.sc + (size_t)l0 * keep;
    int64_t *const oid = W.id + (size_t)l0 * keep;
    for (int64_t e = wave; e < nl * keep; e += nw) {
        float sc = -1.0f;
        int64_t id = INT64_MAX;
        if (e < cnt) {
            // one id per wave: decoded on the scalar unit
            const int64_t raw = side.ids[e];
            id = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(raw >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)raw));
            if (id >= id_begin && id < id_end && (n_excl == 0 || !in_sorted_ids(excl, n_excl, id)))
                sc = score_slice_id_wave(s, fs, n, pool32, ld32, stats, r32, nd, R1, Srr, id);
        }
        if (lane == 0) {
            osc[e] = sc;
            oid[e] = id;
        }
    }
}

__global__ void k_bf_side_reset(BfSide side)
{
    if (threadIdx.x == 0) *side.cnt = 0ull;
}

// the screening status of the band workspace joins the main workspace's
__global__ void k_bf_status(WsHeader *h, const WsHeader *band)
{
    if (threadIdx.x == 0 && band->scr_status != 0) h->scr_status = band->scr_status;
}

__global__ void k_bf_append(WsHeader *h, int n_lists)
{
    if (threadIdx.x == 0) h->n_lists = n_lists;
}

__global__ void k_bf_reset(WsHeader *h, int keep, int n_lists, int lists_cap)
{
    if (threadIdx.x == 0) {
        h->gthr = 0u; h->keep = keep; h->n_lists = n_lists; h->lists_cap = lists_cap; h->status = 0;
        h->scr_status = 0; h->app = 0ull; h->redo = 0;
    }
}

// After an append pass: if it overflowed app_cap entries, the workspace is
// reset for a pass in lists and flagged for it (k_bf_score_stored mode 3).
__global__ void k_bf_redo_reset(WsHeader *h, int keep, int n_lists, int lists_cap, int64_t app_cap)
{
    if (threadIdx.x == 0 && h->app > (unsigned long long)app_cap) {
        h->gthr = 0u; h->keep = keep; h->n_lists = n_lists; h->lists_cap = lists_cap; h->status = 0;
        h->scr_status = 0; h->app = 0ull; h->redo = 1;
    }
}
#else
__global__ void k_bf_reset(WsHeader *h, int keep, int n_lists, int lists_cap);   // defined in the main build
__global__ void k_bf_redo_reset(WsHeader *h, int keep, int n_lists, int lists_cap, int64_t app_cap);
#endif  // SISSO_BF16_MFMA_PART

}  // namespace sisso

using namespace sisso;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }


struct BfPlan {
    int64_t ut_lo = 0, ut_hi = 0;
    int grid = 0;
};

constexpr int kMaxBfGrid = 1024;

// u tiles of `tile` columns (the form's kBTU) covering the ids [begin, end)
BfPlan bf_plan(const sisso_space *s, int64_t begin, int64_t end, int max_grid = kMaxBfGrid, int tile = kBT)
{
    BfPlan p;
    const int L = s->levels;
    const int64_t bb = s->pool[L] + s->rect_unary, be = s->total;
    const int64_t b = begin > bb ? begin : bb, e = end < be ? end : be;
    if (b >= e) return p;
    const int64_t per_u = s->pool[L - 1] * s->n_slots;
    const int64_t ul = (b - bb) / per_u, uh = (e - 1 - bb) / per_u + 1;
    p.ut_lo = ul / tile;
    p.ut_hi = (uh + tile - 1) / tile;
    const int64_t tiles = p.ut_hi - p.ut_lo;
    p.grid = (int)(tiles < max_grid ? tiles : max_grid);
    return p;
}

// band lists: those of the screen (one per block) and those of the exact
// scores of the flagged candidates
int bf_lists_cap(const sisso_space *s) { return bf_plan(s, 0, s->total).grid; }
int bf_lists_total(const sisso_space *s, int keep_b)
{
    return bf_lists_cap(s) + (int)((bf_side_cap(*s) + keep_b - 1) / keep_b);
}

// a block list holds keep entries plus one offer per thread between merges
int bf_list_cap(int keep, int threads) { return next_pow2(keep + threads); }

// Per-block list length of a band: every block keeps its best `band` (the
// LDS list) and publishes its bound, so the grid-wide merge takes the exact
// `band` best approximate scores of the slice, whatever the grid and tiles.
int bf_block_keep(int band) { return band; }

bool space_ok(const sisso_space *s)
{
    return s && s->total > 0 && s->rect == 1 && s->levels >= 1 && s->levels <= SISSO_MAX_LEVELS &&
           s->pool[s->levels - 1] > 0;
}

}  // namespace

#ifndef SISSO_BF16_MFMA_PART
extern "C" size_t sisso_bf16_operands_size(const sisso_space *space, int32_t n)
{
    if (!space_ok(space) || n < 2 || n > SISSO_MAX_N) return 0;
    const int64_t ucols = space->pool[space->levels] - space->pool[space->levels - 1];
    return bf_ops_bytes(ucols);
}

extern "C" sisso_status sisso_prepare_bf16(const sisso_space *space, const sisso_score_args *args, void *ops,
                                           size_t ops_bytes, void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;   // weighted passes run in the FP32 form
    if (!space || !args || !ops || !args->pool32 || !args->stats) return SISSO_E_NULL;
    if (!space_ok(space)) return SISSO_E_UNSUPPORTED;
    if (args->n < 2 || args->n > SISSO_MAX_N || args->ld32 < args->n || (args->ld32 % 4) != 0) return SISSO_E_SHAPE;
    if (ops_bytes < sisso_bf16_operands_size(space, args->n)) return SISSO_E_WORKSPACE;
    const int L = space->levels;
    const int64_t col0 = space->pool[L - 1], ucols = space->pool[L] - col0;
    const BfOps o = bf_ops_view(ops);
    const int64_t blocks = (ucols + 3) / 4;
    hipLaunchKernelGGL(k_bf16_u_prep, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, as_stream(stream),
                       args->n, args->pool32, args->ld32, args->stats, col0, ucols, o);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" size_t sisso_bf16_workspace_size(const sisso_space *space, const sisso_score_args *args, int32_t band)
{
    if (!space_ok(space) || !args || args->n < 2 || band < 1 || band > SISSO_MAX_BAND) return 0;
    const int L = space->levels;
    const int64_t ucols = space->pool[L] - space->pool[L - 1], vcols = space->pool[L - 1];
    return bf_ws_bytes(*space, ucols, vcols, args->n, band, bf_lists_total(space, bf_block_keep(band)),
                       bf_block_keep(band));
}

extern "C" int32_t sisso_expand_score_bf16_lists(const sisso_space *space, const sisso_score_args *args,
                                                 int32_t band)
{
    (void)space;
    (void)args;
    if (band < 1 || band > SISSO_MAX_BAND) return -1;
    return (band + 255) / 256;
}

namespace {

sisso_status bf_check(const sisso_space *space, const sisso_score_args *args, int32_t band, size_t bws_bytes)
{
    if (!space || !args || !args->pool32 || !args->stats || !args->r32 || !args->info) return SISSO_E_NULL;
    if (args->n_exclude > 0 && !args->exclude) return SISSO_E_NULL;
    if (!space_ok(space)) return SISSO_E_UNSUPPORTED;
    const int n = args->n;
    if (n < 2 || n > SISSO_MAX_N || args->ld32 < n || (args->ld32 % 4) != 0 || args->n_exclude < 0)
        return SISSO_E_SHAPE;
    if (args->keep < 1 || args->keep > SISSO_MAX_KEEP || band < args->keep || band > SISSO_MAX_BAND)
        return SISSO_E_RANGE;
    if (bws_bytes < sisso_bf16_workspace_size(space, args, band)) return SISSO_E_WORKSPACE;
    return SISSO_OK;
}

}  // namespace

extern "C" sisso_status sisso_bf16_residual(const sisso_space *space, const sisso_score_args *args, int32_t band,
                                            void *bws, size_t bws_bytes, void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;   // weighted passes run in the FP32 form
    if (!bws) return SISSO_E_NULL;
    const sisso_status c = bf_check(space, args, band, bws_bytes);
    if (c != SISSO_OK) return c;
    hipStream_t st = as_stream(stream);
    const int L = space->levels, n = args->n;
    const int64_t col0 = space->pool[L - 1], ucols = space->pool[L] - col0, vcols = space->pool[L - 1];
    BfWs w = bf_ws_view(bws, ucols, vcols, n, band, bf_lists_total(space, bf_block_keep(band)), bf_block_keep(band));
    const int64_t vb = (vcols + 3) / 4, ub = (ucols + 3) / 4;
    hipLaunchKernelGGL(k_bf16_v_prep, dim3((unsigned)(vb < 65536 ? vb : 65536)), dim3(256), 0, st, n, args->pool32,
                       args->ld32, args->stats, vcols, args->r32, w);
    hipLaunchKernelGGL(k_bf16_u_resid, dim3((unsigned)(ub < 65536 ? ub : 65536)), dim3(256), 0, st, n, args->pool32,
                       args->ld32, args->stats, col0, ucols, args->r32, w.ures);
    const int64_t img_blocks = ((vcols + 127) / 128) * (int64_t)((n + kKC - 1) / kKC);
    hipLaunchKernelGGL(k_bf16_v_image, dim3((unsigned)img_blocks), dim3(256), 0, st, n, args->pool32, args->ld32,
                       vcols, args->r32, args->info, w.vsum, w.vimg);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

#endif  // SISSO_BF16_MFMA_PART

namespace sisso {

// One launch of a 16-bit screening form (after the workspace reset).  The
// plain form is instantiated by the second build only.
template <int MODE>
sisso_status bf_launch(const sisso_space *space, const sisso_score_args *args, const BfOps &o, BfWs &w,
                       int32_t band, int64_t cand_begin, int64_t cand_end, float *mom, const h16 *uimg, BfSide side,
                       hipStream_t st)
{
    using Sh = BfShape<MODE>;
    const int n = args->n;
    const FormSlots fs = form_slots(space);
    static_assert(!Sh::kRead, "the read form launches through bf_launch_read");
    const int max_grid = args->grid > 0 && args->grid < kMaxBfGrid ? args->grid : kMaxBfGrid;
    const BfPlan p = bf_plan(space, cand_begin, cand_end, max_grid, Sh::kBTU);
    // Every block keeps the whole band and may publish its threshold as the
    // grid-wide bound (a lower bound of the band-th best score).
    const int keep_b = bf_block_keep(band);
    const int cap_b = bf_list_cap(keep_b, Sh::kThreads);
    const int publish = keep_b >= band ? 1 : 0;
    const int lcap = bf_lists_total(space, keep_b);
    hipLaunchKernelGGL(k_bf_reset, dim3(1), dim3(64), 0, st, (WsHeader *)w.lists, keep_b, p.grid, lcap);
    if (p.grid > 0) {
        const size_t smem = (size_t)Sh::kNStage * Sh::kStage * sizeof(h16) + 4 * Sh::kBTU * sizeof(float4) +
                            (size_t)cap_b * (sizeof(float) + sizeof(int64_t));
        if (!allow_dynamic_lds(k_score_rect_bf16<MODE>, smem)) return SISSO_E_UNSUPPORTED;
        hipLaunchKernelGGL(k_score_rect_bf16<MODE>, dim3(p.grid), dim3(Sh::kThreads), smem, st, *space, fs, n,
                           args->pool32, args->ld32, args->r32, o.usum, w.vsum, w.ures, args->stats, args->info,
                           args->exclude, args->n_exclude, p.ut_lo, p.ut_hi, cand_begin, cand_end, mom, w.vimg,
                           uimg, args->units, side, w.lists, lcap, keep_b, cap_b, publish);
    }
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

// The screen's lists come first in the band workspace: the number it writes.
template <int MODE>
int bf_screen_lists(const sisso_space *space, const sisso_score_args *args, int64_t cand_begin, int64_t cand_end,
                    int cus)
{
    if (BfShape<MODE>::kRead)   // the scorer of stored contractions: one block per CU, 64-column u tiles
        return bf_plan(space, cand_begin, cand_end, cus < kMaxBfGrid ? cus : kMaxBfGrid, 64).grid;
    const int max_grid = args->grid > 0 && args->grid < kMaxBfGrid ? args->grid : kMaxBfGrid;
    return bf_plan(space, cand_begin, cand_end, max_grid, BfShape<MODE>::kBTU).grid;
}

#ifndef SISSO_BF16_MFMA_PART
// A pass that reads the moments: the residual contractions of the u tiles
// covering [cand_begin, cand_end) (kBfRead, 128 x 128 block tiles, one block
// per CU sweeping its share), then their scores from the stored moments and
// contractions into the band lists (one block per CU).
// Sampling step of the read pass's bound: every step-th u tile (default 8;
// SISSO_BF16_BOUND_STEP in the environment, 1 .. 1024, overrides it).  A
// sparser sample costs less but gives a lower bound, so more candidates are
// appended.
inline int64_t bf_bound_step()
{
    const char *e = getenv("SISSO_BF16_BOUND_STEP");
    const long v = e ? strtol(e, nullptr, 10) : 8;
    return v >= 1 && v <= 1024 ? v : 8;
}

sisso_status bf_launch_read(const sisso_space *space, const sisso_score_args *args, const BfOps &o, BfWs &w,
                            int32_t band, int64_t cand_begin, int64_t cand_end, const float *mom, float *cst,
                            const h16 *uimg, BfSide side, hipStream_t st)
{
    using Sh = BfShape<kBfRead>;
    const int n = args->n;
    const FormSlots fs = form_slots(space);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return SISSO_E_DEVICE;
    const int grid_max = cus < kMaxBfGrid ? cus : kMaxBfGrid;
    const BfPlan p = bf_plan(space, cand_begin, cand_end, grid_max, Sh::kBTU);
    if (p.grid > 0) {
        // one block per CU over the (u, v) tiles, a multiple of the eight XCDs
        const int64_t tiles = (p.ut_hi - p.ut_lo) * ((space->pool[space->levels - 1] + Sh::kBTV - 1) / Sh::kBTV);
        int g = (int)(tiles < grid_max ? tiles : grid_max);
        if (g >= 8) g -= g % 8;
        const size_t smem = (size_t)Sh::kNStage * Sh::kStage * sizeof(h16) + 4 * Sh::kBTU * sizeof(float4);
        if (!allow_dynamic_lds(k_score_rect_bf16<kBfRead>, smem)) return SISSO_E_UNSUPPORTED;
        hipLaunchKernelGGL(k_score_rect_bf16<kBfRead>, dim3(g), dim3(Sh::kThreads), smem, st, *space, fs, n,
                           args->pool32, args->ld32, args->r32, o.usum, w.vsum, w.ures, args->stats, args->info,
                           args->exclude, args->n_exclude, p.ut_lo, p.ut_hi, cand_begin, cand_end, cst, w.vimg,
                           uimg, args->units, side, w.lists, 0, 1, 0, 0);
    }
    // The scores.  Over a large slice: first the best candidate of every
    // 32 x 32 sub-tile of a sample of the u tiles (every step-th), whose
    // band-th best score tau is a lower bound of the slice's band-th best (the
    // sample is part of the slice); then every candidate at or above tau
    // appended, without lists.  The band of the appended candidates is the
    // slice's band, whatever the sample.  If more candidates reach tau than
    // the workspace holds, the pass is scored again in lists (the redo
    // kernels do nothing otherwise).  Over a small slice: lists (every block
    // keeps the whole band).
    const BfPlan q = bf_plan(space, cand_begin, cand_end, grid_max, 64);
    if (q.grid == 0) {
        hipLaunchKernelGGL(k_bf_reset, dim3(1), dim3(64), 0, st, (WsHeader *)w.lists, bf_block_keep(band), 0,
                           bf_lists_total(space, bf_block_keep(band)));
        return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
    }
    const int keep_b = bf_block_keep(band);
    const int cap_b = bf_list_cap(keep_b, kScThreads);
    const int lcap = bf_lists_total(space, keep_b);
    WsHeader *const wh = (WsHeader *)w.lists;
    const size_t smem = (size_t)cap_b * (sizeof(float) + sizeof(int64_t)) + 64 * kScU * (2 * sizeof(float4) + sizeof(uint4));
    if (!allow_dynamic_lds(k_bf_score_stored, smem)) return SISSO_E_UNSUPPORTED;
    const int64_t n_u = q.ut_hi - q.ut_lo, step = bf_bound_step();
    const int64_t nsub = 4 * ((space->pool[space->levels - 1] + 63) / 64);   // sub-tiles per u tile
    const bool sampled = (n_u / step) * nsub >= (int64_t)4 * band;
    auto score = [&](int grid, int64_t u_step, int mode) {
        hipLaunchKernelGGL(k_bf_score_stored, dim3(grid), dim3(kScThreads), smem, st, *space, fs, n, o.usum, w.vsum,
                           w.ures, args->stats, args->info, args->exclude, args->n_exclude, q.ut_lo, q.ut_hi, u_step,
                           cand_begin, cand_end, mom, cst, args->units, w.lists, lcap, keep_b, cap_b, mode,
                           w.band_sc, w.band_cnt, band, &wh->app, (int64_t)q.grid * keep_b);
    };
    if (sampled) {
        // tau: the band-th best of the sub-tile maxima of every step-th u tile
        const int64_t n_s = (n_u + step - 1) / step;
        const int g_s = (int)((n_s + kScU - 1) / kScU < grid_max ? (n_s + kScU - 1) / kScU : grid_max);
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_bf_reset, dim3(1), dim3(64), 0, st, wh, keep_b, q.grid, lcap);
            hipLaunchKernelGGL(k_bf_lists_clear, dim3(1024), dim3(256), 0, st, w.lists, lcap, keep_b,
                               (int64_t)q.grid * keep_b);
            if (pass == 0) {
                score(g_s, step, 2);
                const sisso_status rs = topk_launch(w.lists, band, w.band_ids, w.band_sc, w.band_cnt, st, false);
                if (rs != SISSO_OK) return rs;
            } else {
                score(q.grid, 1, 1);
            }
        }
        hipLaunchKernelGGL(k_bf_redo_reset, dim3(1), dim3(64), 0, st, wh, keep_b, q.grid, lcap,
                           (int64_t)q.grid * keep_b);
        score(q.grid, 1, 3);
    } else {
        hipLaunchKernelGGL(k_bf_reset, dim3(1), dim3(64), 0, st, wh, keep_b, q.grid, lcap);
        score(q.grid, 1, 0);
    }
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
#endif  // SISSO_BF16_MFMA_PART

}  // namespace sisso

namespace sisso {
// The moments pass over the u tiles covering [cand_begin, cand_end): one
// block per CU (its registers allow no more), each sweeping its share.
// images: the operand images of the pass (before it), else the pass itself
sisso_status bf_launch_moments(const sisso_space *space, const sisso_score_args *args, const BfOps &o, BfWs &w,
                               int64_t cand_begin, int64_t cand_end, float *mom, h16 *uimg, h16 *vmimg, BfSide side,
                               bool images, hipStream_t st)
#ifdef SISSO_BF16_MFMA_PART
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return SISSO_E_DEVICE;
    const int n = args->n, L = space->levels, nch = (n + kKC - 1) / kKC;
    const int64_t ulo = space->pool[L - 1], ucols = space->pool[L] - ulo, vcols = space->pool[L - 1];
    const BfPlan p = bf_plan(space, cand_begin, cand_end, cus, MomShape::kBTU);
    if (p.grid == 0) return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
    const int64_t nvt = (vcols + MomShape::kBTV - 1) / MomShape::kBTV;
    if (images) {
        // the u tiles of the pass, widened to the read form's 128-column
        // tiles; every v tile
        const int64_t nut64 = (ucols + 63) / 64, ilo = p.ut_lo & ~(int64_t)1,
                      ihi = ((p.ut_hi + 1) & ~(int64_t)1) < nut64 ? ((p.ut_hi + 1) & ~(int64_t)1) : nut64;
        hipLaunchKernelGGL(k_bf16_u_image, dim3((unsigned)(ihi - ilo < 8192 ? ihi - ilo : 8192)), dim3(256), 0, st,
                           n, args->pool32, args->ld32, ulo, ucols, o.usum, ilo, ihi, uimg);
        hipLaunchKernelGGL(k_bf16_vm_image, dim3((unsigned)(nvt * nch)), dim3(256), 0, st, n, args->pool32,
                           args->ld32, vcols, w.vsum, vmimg);
        return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
    }
    // one block per CU over the (u, v) tiles, a multiple of the eight XCDs
    const int64_t tiles = (p.ut_hi - p.ut_lo) * nvt;
    int g = (int)(tiles < cus ? tiles : cus);
    if (g >= 8) g -= g % 8;
    const size_t smem = 2 * (size_t)MomShape::kStage * sizeof(h16) +
                        MomShape::kBTU * (2 * sizeof(float4) + sizeof(uint4) + sizeof(int));   // staging, u constants
    if (!allow_dynamic_lds(k_bf_moments, smem)) return SISSO_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_bf_moments, dim3(g), dim3(MomShape::kThreads), smem, st, *space, form_slots(space), n, o.usum,
                       w.vsum, args->stats, p.ut_lo, p.ut_hi, cand_begin, cand_end, mom, uimg, vmimg, args->units,
                       side);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
#else
    ;
#endif
}  // namespace sisso

#ifdef SISSO_BF16_MFMA_PART
template sisso_status sisso::bf_launch<kBfFull>(const sisso_space *, const sisso_score_args *, const BfOps &,
                                                BfWs &, int32_t, int64_t, int64_t, float *, const h16 *, BfSide,
                                                hipStream_t);
#else
extern template sisso_status sisso::bf_launch<kBfFull>(const sisso_space *, const sisso_score_args *, const BfOps &,
                                                       BfWs &, int32_t, int64_t, int64_t, float *, const h16 *,
                                                       BfSide, hipStream_t);

namespace {

int64_t bf_tiles(int64_t cols) { return (cols + kBT - 1) / kBT; }

// the moments of every pair, 256-byte aligned (the flagged candidates and
// the u side's image follow)
size_t bf_moments_bytes(const sisso_space *space)
{
    const int L = space->levels;
    const int64_t ucols = space->pool[L] - space->pool[L - 1], vcols = space->pool[L - 1];
    return align256b((size_t)bf_tiles(ucols) * (size_t)bf_tiles(vcols) * kMomTile * sizeof(float));
}
size_t bf_uimg_offset(const sisso_space *space) { return bf_moments_bytes(space) + align256b(bf_side_bytes(*space)); }
// the pass's residual contractions (three per pair, the moments' tiling)
size_t bf_cst_offset(const sisso_space *space, int n)
{
    const int L = space->levels;
    return bf_uimg_offset(space) + align256b(bf_uimg_elems(space->pool[L] - space->pool[L - 1], n) * sizeof(h16));
}
// the moments pass's v image
size_t bf_vmimg_offset(const sisso_space *space, int n)
{
    const int L = space->levels;
    const int64_t ucols = space->pool[L] - space->pool[L - 1], vcols = space->pool[L - 1];
    return bf_cst_offset(space, n) + align256b((size_t)bf_tiles(ucols) * (size_t)bf_tiles(vcols) * (kMomTile / kMom) *
                                               3 * sizeof(float));
}
size_t bf_moments_total(const sisso_space *space, int n)
{
    const int L = space->levels;
    return bf_vmimg_offset(space, n) + align256b(bf_vmimg_elems(space->pool[L - 1], n) * sizeof(h16));
}

// internal modes of bf_screen beside the public three: the two halves of the
// moments work of a WRITE screen, for callers that time them
constexpr int32_t kMomentsImages = 100, kMomentsPass = 101;

sisso_status bf_screen(const sisso_space *space, const sisso_score_args *args, const void *ops, size_t ops_bytes,
                       int32_t band, int64_t cand_begin, int64_t cand_end, void *moments, size_t moments_bytes,
                       int32_t mode, void *bws, size_t bws_bytes, void *stream)
{
    if (!ops || !bws) return SISSO_E_NULL;
    const sisso_status c = bf_check(space, args, band, bws_bytes);
    if (c != SISSO_OK) return c;
    const int L = space->levels, n = args->n;
    const int64_t bb = space->pool[L] + space->rect_unary;
    if (cand_begin < bb || cand_end > space->total || cand_begin >= cand_end) return SISSO_E_RANGE;
    if (ops_bytes < sisso_bf16_operands_size(space, n)) return SISSO_E_WORKSPACE;
    if (mode != SISSO_MOMENTS_NONE && mode != SISSO_MOMENTS_WRITE && mode != SISSO_MOMENTS_READ &&
        mode != kMomentsImages && mode != kMomentsPass)
        return SISSO_E_RANGE;
    if (mode != SISSO_MOMENTS_NONE) {
        if (!moments) return SISSO_E_NULL;
        if (moments_bytes < sisso_bf16_moments_size(space, n)) return SISSO_E_WORKSPACE;
    }
    hipStream_t st = as_stream(stream);
    const int64_t col0 = space->pool[L - 1], ucols = space->pool[L] - col0, vcols = space->pool[L - 1];
    const BfOps o = bf_ops_view(const_cast<void *>(ops));
    const int keep_b = bf_block_keep(band);
    BfWs w = bf_ws_view(bws, ucols, vcols, n, band, bf_lists_total(space, keep_b), keep_b);
    float *mom = (float *)moments;
    h16 *const uimg = mode == SISSO_MOMENTS_NONE ? nullptr : (h16 *)((char *)moments + bf_uimg_offset(space));
    float *const cst = mode == SISSO_MOMENTS_NONE ? nullptr : (float *)((char *)moments + bf_cst_offset(space, n));
    h16 *const vmimg = mode == SISSO_MOMENTS_NONE ? nullptr : (h16 *)((char *)moments + bf_vmimg_offset(space, n));
    // the flagged candidates: beside the moments (every pass of a fit scores
    // those its first pass stored), else in the workspace
    const BfSide side = bf_side_view(mode == SISSO_MOMENTS_NONE ? w.side : (char *)moments + bf_moments_bytes(space),
                                     *space);
    if (mode != SISSO_MOMENTS_READ && mode != kMomentsImages)
        hipLaunchKernelGGL(k_bf_side_reset, dim3(1), dim3(64), 0, st, side);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return SISSO_E_DEVICE;
    sisso_status rc;
    int l0;
    switch (mode) {
    case SISSO_MOMENTS_WRITE:
        // the moments pass stores the moments, the flagged candidates and the
        // u side's image; the read form then scores the pass from them
        rc = bf_launch_moments(space, args, o, w, cand_begin, cand_end, mom, uimg, vmimg, side, true, st);
        if (rc == SISSO_OK) rc = bf_launch_moments(space, args, o, w, cand_begin, cand_end, mom, uimg, vmimg, side, false, st);
        if (rc == SISSO_OK) rc = bf_launch_read(space, args, o, w, band, cand_begin, cand_end, mom, cst, uimg, side, st);
        l0 = bf_screen_lists<kBfRead>(space, args, cand_begin, cand_end, cus);
        break;
    case kMomentsImages:
        return bf_launch_moments(space, args, o, w, cand_begin, cand_end, mom, uimg, vmimg, side, true, st);
    case kMomentsPass:
        return bf_launch_moments(space, args, o, w, cand_begin, cand_end, mom, uimg, vmimg, side, false, st);
    case SISSO_MOMENTS_READ:
        rc = bf_launch_read(space, args, o, w, band, cand_begin, cand_end, mom, cst, uimg, side, st);
        l0 = bf_screen_lists<kBfRead>(space, args, cand_begin, cand_end, cus);
        break;
    default:
        rc = bf_launch<kBfFull>(space, args, o, w, band, cand_begin, cand_end, nullptr, nullptr, side, st);
        l0 = bf_screen_lists<kBfFull>(space, args, cand_begin, cand_end, cus);
    }
    if (rc != SISSO_OK) return rc;
    const FormSlots fs = form_slots(space);
    hipLaunchKernelGGL(k_bf_side, dim3(1024), dim3(256), 0, st, *space, fs, n, args->pool32, args->ld32, args->stats,
                       args->r32, args->info, args->exclude, args->n_exclude, cand_begin, cand_end, side, w.lists,
                       bf_lists_total(space, keep_b), keep_b, l0);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

}  // namespace

extern "C" size_t sisso_bf16_moments_size(const sisso_space *space, int32_t n)
{
    if (!space_ok(space) || n < 2 || n > SISSO_MAX_N) return 0;
    return bf_moments_total(space, n);
}

extern "C" sisso_status sisso_bf16_screen(const sisso_space *space, const sisso_score_args *args, const void *ops,
                                          size_t ops_bytes, int32_t band, int64_t cand_begin, int64_t cand_end,
                                          void *bws, size_t bws_bytes, void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;   // weighted passes run in the FP32 form
    return bf_screen(space, args, ops, ops_bytes, band, cand_begin, cand_end, nullptr, 0, SISSO_MOMENTS_NONE, bws,
                     bws_bytes, stream);
}

extern "C" sisso_status sisso_bf16_screen_moments(const sisso_space *space, const sisso_score_args *args,
                                                  const void *ops, size_t ops_bytes, int32_t band,
                                                  int64_t cand_begin, int64_t cand_end, void *moments,
                                                  size_t moments_bytes, int32_t mode, void *bws, size_t bws_bytes,
                                                  void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;   // weighted passes run in the FP32 form
    return bf_screen(space, args, ops, ops_bytes, band, cand_begin, cand_end, moments, moments_bytes, mode, bws,
                     bws_bytes, stream);
}

extern "C" sisso_status sisso_bf16_moments_images(const sisso_space *space, const sisso_score_args *args,
                                                  const void *ops, size_t ops_bytes, int32_t band,
                                                  int64_t cand_begin, int64_t cand_end, void *moments,
                                                  size_t moments_bytes, void *bws, size_t bws_bytes, void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;
    return bf_screen(space, args, ops, ops_bytes, band, cand_begin, cand_end, moments, moments_bytes, kMomentsImages,
                     bws, bws_bytes, stream);
}

extern "C" sisso_status sisso_bf16_moments_pass(const sisso_space *space, const sisso_score_args *args,
                                                const void *ops, size_t ops_bytes, int32_t band, int64_t cand_begin,
                                                int64_t cand_end, void *moments, size_t moments_bytes, void *bws,
                                                size_t bws_bytes, void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;
    return bf_screen(space, args, ops, ops_bytes, band, cand_begin, cand_end, moments, moments_bytes, kMomentsPass,
                     bws, bws_bytes, stream);
}

extern "C" sisso_status sisso_bf16_rescore(const sisso_space *space, const sisso_score_args *args, int32_t band,
                                           void *bws, size_t bws_bytes, void *ws, size_t ws_bytes, void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;   // weighted passes run in the FP32 form
    if (!bws || !ws) return SISSO_E_NULL;
    const sisso_status c = bf_check(space, args, band, bws_bytes);
    if (c != SISSO_OK) return c;
    const int lists_main = score_lists_capacity(space, args);
    const int n_resc = (band + 255) / 256;
    if (ws_bytes < ws_bytes_for(lists_main, args->keep)) return SISSO_E_WORKSPACE;
    if (args->list_base < 0 || args->list_base + n_resc > lists_main) return SISSO_E_WORKSPACE;
    hipStream_t st = as_stream(stream);
    const int L = space->levels, n = args->n;
    const int64_t ucols = space->pool[L] - space->pool[L - 1], vcols = space->pool[L - 1];
    BfWs w = bf_ws_view(bws, ucols, vcols, n, band, bf_lists_total(space, bf_block_keep(band)), bf_block_keep(band));
    const FormSlots fs = form_slots(space);
    sisso_status rs = topk_launch(w.lists, band, w.band_ids, w.band_sc, w.band_cnt, st, band > bf_block_keep(band));
    if (rs != SISSO_OK) return rs;
    const int keep = args->keep, cap = next_pow2(keep + 256);
    if (args->list_base == 0)
        hipLaunchKernelGGL(k_bf_reset, dim3(1), dim3(64), 0, st, (WsHeader *)ws, keep, n_resc, lists_main);
    else
        hipLaunchKernelGGL(k_bf_append, dim3(1), dim3(64), 0, st, (WsHeader *)ws, args->list_base + n_resc);
    hipLaunchKernelGGL(k_bf_status, dim3(1), dim3(64), 0, st, (WsHeader *)ws, (const WsHeader *)w.lists);
    const size_t smem = (size_t)cap * (sizeof(float) + sizeof(int64_t));
    hipLaunchKernelGGL(k_rescore_ids, dim3(n_resc), dim3(256), smem, st, *space, fs, n, args->pool32, args->ld32,
                       args->stats, args->r32, args->info, w.band_ids, w.band_cnt, args->exclude, args->n_exclude,
                       args->list_base, ws, lists_main, keep, cap);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_expand_score_bf16(const sisso_space *space, const sisso_score_args *args,
                                                const void *ops, size_t ops_bytes, int32_t band, int64_t cand_begin,
                                                int64_t cand_end, void *bws, size_t bws_bytes, void *ws,
                                                size_t ws_bytes, void *stream)
{
    if (args && args->w32) return SISSO_E_UNSUPPORTED;   // weighted passes run in the FP32 form
    sisso_status st = sisso_bf16_residual(space, args, band, bws, bws_bytes, stream);
    if (st != SISSO_OK) return st;
    st = sisso_bf16_screen(space, args, ops, ops_bytes, band, cand_begin, cand_end, bws, bws_bytes, stream);
    if (st != SISSO_OK) return st;
    return sisso_bf16_rescore(space, args, band, bws, bws_bytes, ws, ws_bytes, stream);
}
#endif  // SISSO_BF16_MFMA_PART
