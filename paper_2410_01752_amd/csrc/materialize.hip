// materialize.hip -- operand pools and FP64 feature evaluation.
//
// Feature expansion (Sec. 2.1, eq. feature-exp): the pool levels P_0, P_1,
// P_2 are evaluated in FP64 from the base features, one wave per column,
// and stored column-major in FP32 (the screening operands) together with
// per-column statistics.  Level-1 values are also kept in FP64 so that any
// feature of the space (pool or one-sided slice) can be re-evaluated exactly
// in FP64 for the subspace and the SO step.
#include "common.hpp"

namespace sisso {

struct BlockStats {
    double red[16];
    float fmx[16], fmn[16], fmv[16];
    int bad[16];
};

__device__ inline void block_minmax(float &mx, float &mn, float &mv, int &bad, BlockStats &bs)
{
    mx = wave_max(mx); mn = wave_min(mn); mv = wave_min(mv); bad = wave_or(bad);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { bs.fmx[w] = mx; bs.fmn[w] = mn; bs.fmv[w] = mv; bs.bad[w] = bad; }
    __syncthreads();
    for (int i = 0; i < nw; ++i) {
        mx = fmaxf(mx, bs.fmx[i]); mn = fminf(mn, bs.fmn[i]); mv = fminf(mv, bs.fmv[i]);
        bad |= bs.bad[i];
    }
}

// One level of the pool: columns [c_begin, c_end), one wave per column.
// Level 0 copies the base features; operands of levels >= 1 are read from
// the FP64 level-1 pool.  For n <= 64 kPoolRegs the column's FP64 values stay
// in registers between the two passes (the mean is needed before the sum of
// squared deviations); longer columns are evaluated twice.
constexpr int kPoolRegs = 32;

// Pass 1 over the register-resident part of a column for a compile-time
// operator OP (-1: copy of a base feature): values, domain and magnitude
// flags, and the sums of f, x^2 and y^2.
template <int OP>
__device__ __forceinline__ void pool_values(const double *__restrict__ A, const double *__restrict__ B, int n,
                                            double (&fr)[kPoolRegs], double &sum, double &sa2, double &sb2,
                                            int &bad)
{
    const int lane = threadIdx.x & 63;
    constexpr bool binary = OP == SISSO_ADD || OP == SISSO_SUB || OP == SISSO_MUL || OP == SISSO_DIV;
#pragma unroll
    for (int i = 0; i < kPoolRegs; ++i) {
        const int t = lane + 64 * i;
        fr[i] = 0.0;
        if (t < n) {
            bool ok = true;
            const double x = A[t], y = binary ? B[t] : 0.0;
            const double f = OP < 0 ? x : apply64(OP, x, y, ok);
            if (!ok || !(fabs(f) <= kValueCap)) bad = 1;   // also catches NaN
            fr[i] = f;
            sum += f;
            sa2 += x * x;
            sb2 += y * y;
        }
    }
}

__global__ void __launch_bounds__(256) k_pool_level(sisso_space s, const double *__restrict__ X,
                                                    int n, int ldx, float *__restrict__ pool32,
                                                    int64_t ld32, double *__restrict__ p1,
                                                    int64_t ld64, sisso_colstat *__restrict__ stats,
                                                    int64_t c_begin, int64_t c_end)
{
    const int lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * nwv + (threadIdx.x >> 6), wstride = (int64_t)gridDim.x * nwv;
    const bool regs = n <= 64 * kPoolRegs;
    for (int64_t c = c_begin + wid; c < c_end; c += wstride) {
        int op;
        int64_t a, b;
        decode_id(s, c, &op, &a, &b);
        bool opok = true;
        if (op >= 0) {
            opok = stats[a].valid != 0.0f;
            if (b >= 0) opok = opok && stats[b].valid != 0.0f;
        }
        const double *A = op < 0 ? X + (size_t)c * ldx : p1 + (size_t)a * ld64;
        const double *B = (op >= 0 && b >= 0) ? p1 + (size_t)b * ld64 : nullptr;
        auto value = [&](int t, bool &ok, double &x, double &y) {
            x = A[t];
            y = B ? B[t] : 0.0;
            return op < 0 ? x : apply64(op, x, y, ok);
        };
        // pass 1: values, domain, magnitude, sums
        double fr[kPoolRegs];
        double sum = 0.0, sa2 = 0.0, sb2 = 0.0;
        int bad = opok ? 0 : 1;
        auto pass1 = [&](int t, double &f) {
            bool ok = true;
            double x, y;
            f = value(t, ok, x, y);
            if (!ok || !(fabs(f) <= kValueCap)) bad = 1;   // also catches NaN
            sum += f;
            sa2 += x * x;
            sb2 += y * y;
        };
        switch (op < 0 ? -1 : op) {
        case -1: pool_values<-1>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_ADD: pool_values<SISSO_ADD>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_SUB: pool_values<SISSO_SUB>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_MUL: pool_values<SISSO_MUL>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_DIV: pool_values<SISSO_DIV>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_SQ: pool_values<SISSO_SQ>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_CUBE: pool_values<SISSO_CUBE>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_SQRT: pool_values<SISSO_SQRT>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_INV: pool_values<SISSO_INV>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_EXP: pool_values<SISSO_EXP>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_NEXP: pool_values<SISSO_NEXP>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_LOG: pool_values<SISSO_LOG>(A, B, n, fr, sum, sa2, sb2, bad); break;
        case SISSO_SIN: pool_values<SISSO_SIN>(A, B, n, fr, sum, sa2, sb2, bad); break;
        default:
#pragma unroll
            for (int i = 0; i < kPoolRegs; ++i) {
                fr[i] = 0.0;
                const int t = lane + 64 * i;
                if (t < n) pass1(t, fr[i]);
            }
        }
        if (!regs)
            for (int t = lane + 64 * kPoolRegs; t < n; t += 64) {
                double f;
                pass1(t, f);
            }
        const double mean = wave_sum_dpp(sum) / n;
        const double ra = sqrt(wave_sum_dpp(sa2) / n), rb = sqrt(wave_sum_dpp(sb2) / n);
        // pass 2: sum of squares, extremes, reciprocal mean, stores
        double ss = 0.0, srcp = 0.0, sf2 = 0.0;
        float mx = 0.0f, mn = INFINITY, mv = INFINITY;
        float *out32 = pool32 + (size_t)c * ld32;
        double *out64 = (c < s.pool[1 < s.levels ? 1 : s.levels]) ? p1 + (size_t)c * ld64 : nullptr;
        auto pass2 = [&](int t, double f) {
            const double e = f - mean;
            ss += e * e;
            sf2 += f * f;
            srcp += 1.0 / f;
            const float af = (float)fabs(f);
            mx = fmaxf(mx, af); mn = fminf(mn, af); mv = fminf(mv, (float)f);
            out32[t] = (float)f;
            if (out64) out64[t] = f;
        };
#pragma unroll
        for (int i = 0; i < kPoolRegs; ++i) {
            const int t = lane + 64 * i;
            if (t < n) pass2(t, fr[i]);
        }
        if (!regs)
            for (int t = lane + 64 * kPoolRegs; t < n; t += 64) {
                bool ok = true;
                double x, y;
                pass2(t, value(t, ok, x, y));
            }
        for (int64_t t = n + lane; t < ld32; t += 64) out32[t] = 0.0f;
        const double sst = wave_sum_dpp(ss);
        const double mrcp = wave_sum_dpp(srcp) / n;
        const double msq = wave_sum_dpp(sf2) / n;
        mx = wave_max_dpp(mx); mn = wave_min_dpp(mn); mv = wave_min_dpp(mv); bad = wave_or_dpp(bad);
        if (lane == 0) {
            const double sd = sqrt(sst / n);
            bool valid = !bad && sd != 0.0 && sd > kConstRel * fabs(mean);
            if (op == SISSO_ADD || op == SISSO_SUB) valid = valid && sd > kCancelRel * fmax(ra, rb);
            sisso_colstat st;
            st.mean = (float)mean;
            st.sd = (float)sd;
            st.mean_rcp = mn > 0.0f ? (float)mrcp : INFINITY;
            st.maxabs = mx;
            st.minabs = mn;
            st.minval = mv;
            st.valid = valid ? 1.0f : 0.0f;
            st.rms = (float)sqrt(msq);
            stats[c] = st;
        }
    }
}

// One operand of a feature, evaluated from the FP64 level-1 pool: a pool-1
// column, or a level-2 column op(P1[a], P1[b]).
struct Node {
    int op;          // -1: leaf P1[a]
    int64_t a, b;
};

__device__ inline Node make_node(const sisso_space &s, int64_t id)
{
    Node nd;
    if (id < s.pool[1]) { nd.op = -1; nd.a = id; nd.b = -1; return nd; }
    int op;
    int64_t a, b;
    decode_id(s, id, &op, &a, &b);
    nd.op = op; nd.a = a; nd.b = b;
    return nd;
}

__device__ __forceinline__ double eval_node(const Node &nd, const double *p1, int64_t ld64, int t,
                                            bool &ok)
{
    const double x = p1[(size_t)nd.a * ld64 + t];
    if (nd.op < 0) return x;
    const double y = nd.b >= 0 ? p1[(size_t)nd.b * ld64 + t] : 0.0;
    return apply64(nd.op, x, y, ok);
}

// FP64 values of arbitrary features, one block per id (ids q0, q0 + qstep, ..).
__device__ inline void eval_ids(const sisso_space &s, int stored, int n, const double *__restrict__ p1,
                                int64_t ld64, const sisso_colstat *__restrict__ stats,
                                const int64_t *__restrict__ ids, int count, double *__restrict__ out, int ldo,
                                int32_t *__restrict__ valid, int q0, int qstep)
{
    __shared__ BlockStats bs;
    for (int q = q0; q < count; q += qstep) {
        const int64_t id = ids[q];
        double *o = out + (size_t)q * ldo;
        if (id < 0 || id >= s.total) {
            for (int t = threadIdx.x; t < n; t += blockDim.x) o[t] = NAN;
            if (threadIdx.x == 0) valid[q] = 0;
            continue;
        }
        int top = -1;
        Node L, R;
        bool opok = true;
        R.op = -1; R.a = -1; R.b = -1;
        if (id < s.pool[stored]) {
            L = make_node(s, id);
            opok = stats[id].valid != 0.0f;   // pool columns: decided at materialisation
        } else {
            int64_t u, v;
            decode_id(s, id, &top, &u, &v);
            L = make_node(s, u);
            opok = stats[u].valid != 0.0f;
            if (v >= 0) { R = make_node(s, v); opok = opok && stats[v].valid != 0.0f; }
        }
        double sum = 0.0, sa2 = 0.0, sb2 = 0.0;
        int bad = opok ? 0 : 1;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            bool ok = true;
            double f = eval_node(L, p1, ld64, t, ok);
            if (top >= 0) {
                const double g = R.a >= 0 ? eval_node(R, p1, ld64, t, ok) : 0.0;
                sa2 += f * f;
                sb2 += g * g;
                f = apply64(top, f, g, ok);
            }
            if (!ok || !(fabs(f) <= kValueCap)) bad = 1;
            o[t] = f;
            sum += f;
        }
        const double mean = block_sum(sum, bs.red) / n;
        const double ra = sqrt(block_sum(sa2, bs.red) / n), rb = sqrt(block_sum(sb2, bs.red) / n);
        double ss = 0.0;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const double e = o[t] - mean;
            ss += e * e;
        }
        const double sst = block_sum(ss, bs.red);
        float mx = 0, mn = 0, mv = 0;
        block_minmax(mx, mn, mv, bad, bs);
        const double sd = sqrt(sst / n);
        bool ok = !bad && sd != 0.0 && sd > kConstRel * fabs(mean);
        if (top == SISSO_ADD || top == SISSO_SUB) ok = ok && sd > kCancelRel * fmax(ra, rb);
        if (!ok)
            for (int t = threadIdx.x; t < n; t += blockDim.x) o[t] = NAN;
        if (threadIdx.x == 0) valid[q] = ok ? 1 : 0;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_eval_ids(sisso_space s, int stored, int n, const double *__restrict__ p1,
                                                  int64_t ld64, const sisso_colstat *__restrict__ stats,
                                                  const int64_t *__restrict__ ids, int count,
                                                  double *__restrict__ out, int ldo,
                                                  int32_t *__restrict__ valid)
{
    eval_ids(s, stored, n, p1, ld64, stats, ids, count, out, ldo, valid, blockIdx.x, gridDim.x);
}

// The same over a table of problems (blockIdx.y = problem).
__device__ inline bool evalp_ok(const sisso_eval_problem &P, int count_max)
{
    return P.pool1_64 && P.stats && P.ids && P.out && P.valid && P.n >= 2 && P.n <= SISSO_MAX_N &&
           P.ld64 >= P.n && P.ldo >= P.n && P.count >= 0 && P.count <= count_max;
}

__global__ void __launch_bounds__(256) k_eval_ids_batch(sisso_space s, int stored,
                                                        const sisso_eval_problem *__restrict__ T, int count_max,
                                                        int32_t *__restrict__ status)
{
    const sisso_eval_problem P = T[blockIdx.y];
    const bool ok = evalp_ok(P, count_max);
    if (blockIdx.x == 0 && threadIdx.x == 0 && status) status[blockIdx.y] = ok ? SISSO_OK : SISSO_E_SHAPE;
    if (!ok) return;
    eval_ids(s, stored, P.n, P.pool1_64, P.ld64, P.stats, P.ids, P.count, P.out, P.ldo, P.valid, blockIdx.x,
             gridDim.x);
}

// Centre a residual, round it to FP32 and record its sums (one block).
__device__ inline void prepare_residual_block(const double *__restrict__ r, int n, float *__restrict__ r32,
                                              sisso_resid_info *__restrict__ info, double *red)
{
    double s = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) s += r[t];
    const double mean = block_sum(s, red) / n;
    double s32 = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const float v = (float)(r[t] - mean);
        r32[t] = v;
        s32 += (double)v;
    }
    const double sum32 = block_sum(s32, red);
    const double m32 = sum32 / n;
    double ss = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double e = (double)r32[t] - m32;
        ss += e * e;
    }
    const double srr = block_sum(ss, red);
    if (threadIdx.x == 0) {
        info->sum_r32 = sum32;
        info->s_rr = srr;
        info->mean_r = mean;
        info->n = (double)n;
    }
}

__global__ void __launch_bounds__(1024) k_prepare_residual(const double *__restrict__ r, int n,
                                                           float *__restrict__ r32,
                                                           sisso_resid_info *__restrict__ info)
{
    __shared__ double red[16];
    prepare_residual_block(r, n, r32, info, red);
}

// Weighted residual of a pass under sample weights (Sec. 2.4, whitening with
// a diagonal covariance): weights scaled to mean 1 (wn = w n / sum w), the
// weighted mean mu of r, r32 = wn (r - mu) in FP32 and its sums (one block).
// A weight that is not positive and finite poisons s_rr with NaN.
__global__ void __launch_bounds__(1024) k_prepare_residual_weighted(const double *__restrict__ r,
                                                                    const double *__restrict__ w, int n,
                                                                    float *__restrict__ r32,
                                                                    float *__restrict__ w32,
                                                                    sisso_resid_info *__restrict__ info)
{
    __shared__ double red[16];
    double sw = 0.0, swr = 0.0;
    int bad = 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double wt = w[t];
        if (!(wt > 0.0) || !isfinite(wt)) bad = 1;
        sw += wt;
        swr += wt * r[t];
    }
    bad = __syncthreads_or(bad);
    const double W = block_sum(sw, red);
    const double mean = block_sum(swr, red) / W;
    const double scale = (double)n / W;
    double s32 = 0.0, ss = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double wn = w[t] * scale;
        const double e = r[t] - mean;
        const float v = (float)(wn * e);
        r32[t] = v;
        w32[t] = (float)wn;
        s32 += (double)v;
        ss += wn * e * e;
    }
    const double sum32 = block_sum(s32, red);
    const double srr = block_sum(ss, red);
    if (threadIdx.x == 0) {
        info->sum_r32 = sum32;
        info->s_rr = bad ? NAN : srr;
        info->mean_r = mean;
        info->n = (double)n;
    }
}

// One block per problem of a batch; entries with a bad n or a null pointer
// are left untouched (the batched screening flags them).
__global__ void __launch_bounds__(1024) k_prepare_residual_batch(const sisso_problem *__restrict__ probs)
{
    __shared__ double red[16];
    const sisso_problem P = probs[blockIdx.x];
    if (P.n < 2 || P.n > SISSO_MAX_N || !P.r64 || !P.r32 || !P.info) return;
    prepare_residual_block(P.r64, P.n, P.r32, P.info, red);
}

}  // namespace sisso

using namespace sisso;

namespace sisso {
// Units of the pool columns [lo, hi) of one level from those of the earlier
// levels (level 0: copied from the base features); a column that breaks a
// rule gets kUnitNone and loses its validity.  One thread per column.
__global__ void __launch_bounds__(256) k_pool_units(sisso_space s, const int16_t *__restrict__ base,
                                                    int16_t *__restrict__ units, sisso_colstat *__restrict__ stats,
                                                    int64_t lo, int64_t hi)
{
    constexpr int K = SISSO_UNIT_DIMS;
    for (int64_t c = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < hi;
         c += (int64_t)gridDim.x * blockDim.x) {
        int32_t e[K];
        bool ok = true;
        int op;
        int64_t a, b;
        if (c < s.d) {
            for (int q = 0; q < K; ++q) e[q] = base[c * K + q];
            ok = e[0] != kUnitNone;
        } else {
            decode_id(s, c, &op, &a, &b);
            const int16_t *ua = units + a * K, *ub = b >= 0 ? units + b * K : nullptr;
            ok = ua[0] != kUnitNone && (!ub || ub[0] != kUnitNone);
            bool dimless = true;
            for (int q = 0; q < K; ++q) dimless = dimless && ua[q] == 0;
            for (int q = 0; q < K && ok; ++q) {
                const int x = ua[q];
                switch (op) {
                case SISSO_ADD: case SISSO_SUB: ok = x == ub[q]; e[q] = x; break;
                case SISSO_MUL: e[q] = x + ub[q]; break;
                case SISSO_DIV: e[q] = x - ub[q]; break;
                case SISSO_SQ: e[q] = 2 * x; break;
                case SISSO_CUBE: e[q] = 3 * x; break;
                case SISSO_SQRT: ok = (x & 1) == 0; e[q] = x / 2; break;
                case SISSO_INV: e[q] = -x; break;
                default: ok = dimless; e[q] = 0; break;       // exp, exp(-x), ln, sin
                }
                ok = ok && e[q] >= -(1 << 14) && e[q] <= (1 << 14);
            }
        }
        int16_t *out = units + c * K;
        for (int q = 0; q < K; ++q) out[q] = ok ? (int16_t)e[q] : (q == 0 ? (int16_t)kUnitNone : (int16_t)0);
        if (!ok) stats[c].valid = 0.0f;
    }
}
}  // namespace sisso

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" sisso_status sisso_pool_units(const sisso_space *space, const int16_t *base_units, int16_t *units,
                                         sisso_colstat *stats, void *stream)
{
    if (!space || !base_units || !units || !stats) return SISSO_E_NULL;
    if (space->total <= 0 || space->levels < 1 || space->levels > SISSO_MAX_LEVELS) return SISSO_E_SHAPE;
    hipStream_t st = as_stream(stream);
    for (int lev = 0; lev <= space->levels; ++lev) {
        const int64_t lo = lev == 0 ? 0 : space->pool[lev - 1], hi = space->pool[lev];
        const int64_t blocks = (hi - lo + 255) / 256;
        const int grid = (int)(blocks < 16384 ? blocks : 16384);
        hipLaunchKernelGGL(k_pool_units, dim3(grid), dim3(256), 0, st, *space, base_units, units, stats, lo, hi);
        if (hipGetLastError() != hipSuccess) return SISSO_E_DEVICE;
    }
    return SISSO_OK;
}

extern "C" sisso_status sisso_materialize_pools(const sisso_space *space, const double *X, int32_t n,
                                                int32_t ldx, float *pool32, int64_t ld32,
                                                double *pool1_64, int64_t ld64, sisso_colstat *stats,
                                                void *stream)
{
    if (!space || !X || !pool32 || !pool1_64 || !stats) return SISSO_E_NULL;
    if (space->total <= 0 || space->levels < 1 || space->levels > SISSO_MAX_LEVELS) return SISSO_E_SHAPE;
    if (n < 2 || n > SISSO_MAX_N || ldx < n || ld32 < n || (ld32 % 4) != 0 || ld64 < n)
        return SISSO_E_SHAPE;
    hipStream_t st = as_stream(stream);
    for (int lev = 0; lev <= space->levels; ++lev) {
        const int64_t lo = lev == 0 ? 0 : space->pool[lev - 1], hi = space->pool[lev];
        const int64_t cols = hi - lo;
        const int64_t blocks = (cols + 3) / 4;   // four waves (columns) per block
        const int grid = (int)(blocks < 16384 ? blocks : 16384);
        hipLaunchKernelGGL(k_pool_level, dim3(grid), dim3(256), 0, st, *space, X, n, ldx, pool32, ld32,
                           pool1_64, ld64, stats, lo, hi);
        if (hipGetLastError() != hipSuccess) return SISSO_E_DEVICE;
    }
    return SISSO_OK;
}

extern "C" sisso_status sisso_materialize_ids_stored(const sisso_space *space, int32_t stored_levels, int32_t n,
                                                     const double *pool1_64, int64_t ld64,
                                                     const sisso_colstat *stats, const int64_t *ids,
                                                     int32_t count, double *out, int32_t ldo,
                                                     int32_t *valid, void *stream)
{
    if (!space || !pool1_64 || !stats || !ids || !out || !valid) return SISSO_E_NULL;
    if (space->total <= 0 || n < 2 || n > SISSO_MAX_N || ld64 < n || ldo < n || count < 0)
        return SISSO_E_SHAPE;
    if (stored_levels < 1 || stored_levels > space->levels) return SISSO_E_SHAPE;
    if (count == 0) return SISSO_OK;
    const int grid = count < 4096 ? count : 4096;
    hipLaunchKernelGGL(k_eval_ids, dim3(grid), dim3(256), 0, as_stream(stream), *space, stored_levels, n,
                       pool1_64, ld64, stats, ids, count, out, ldo, valid);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_materialize_ids(const sisso_space *space, int32_t n,
                                              const double *pool1_64, int64_t ld64,
                                              const sisso_colstat *stats, const int64_t *ids,
                                              int32_t count, double *out, int32_t ldo,
                                              int32_t *valid, void *stream)
{
    if (!space) return SISSO_E_NULL;
    return sisso_materialize_ids_stored(space, space->levels, n, pool1_64, ld64, stats, ids, count, out, ldo,
                                        valid, stream);
}

extern "C" sisso_status sisso_prepare_residual(const double *r, int32_t n, float *r32,
                                               sisso_resid_info *info, void *stream)
{
    if (!r || !r32 || !info) return SISSO_E_NULL;
    if (n < 2 || n > SISSO_MAX_N) return SISSO_E_SHAPE;
    hipLaunchKernelGGL(k_prepare_residual, dim3(1), dim3(1024), 0, as_stream(stream), r, n, r32, info);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_prepare_residual_weighted(const double *r, const double *w, int32_t n, float *r32,
                                                        float *w32, sisso_resid_info *info, void *stream)
{
    if (!r || !w || !r32 || !w32 || !info) return SISSO_E_NULL;
    if (n < 2 || n > SISSO_MAX_N) return SISSO_E_SHAPE;
    hipLaunchKernelGGL(k_prepare_residual_weighted, dim3(1), dim3(1024), 0, as_stream(stream), r, w, n, r32, w32,
                       info);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_prepare_residual_batched(const sisso_problem *problems, int32_t n_problems,
                                                       void *stream)
{
    if (!problems) return SISSO_E_NULL;
    if (n_problems < 1 || n_problems > SISSO_MAX_BATCH) return SISSO_E_SHAPE;
    hipLaunchKernelGGL(k_prepare_residual_batch, dim3(n_problems), dim3(1024), 0, as_stream(stream), problems);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}

extern "C" sisso_status sisso_materialize_ids_batched(const sisso_space *space, int32_t stored_levels,
                                                      const sisso_eval_problem *problems, int32_t n_problems,
                                                      int32_t count_max, int32_t *out_status, void *stream)
{
    if (!space || !problems) return SISSO_E_NULL;
    if (space->total <= 0 || stored_levels < 1 || stored_levels > space->levels || n_problems < 1 ||
        n_problems > SISSO_MAX_BATCH || count_max < 1 || count_max > SISSO_MAX_KEEP)
        return SISSO_E_SHAPE;
    const int gx = count_max < 256 ? count_max : 256;
    hipLaunchKernelGGL(k_eval_ids_batch, dim3(gx, n_problems), dim3(256), 0, as_stream(stream), *space,
                       stored_levels, problems, count_max, out_status);
    return hipGetLastError() == hipSuccess ? SISSO_OK : SISSO_E_DEVICE;
}
