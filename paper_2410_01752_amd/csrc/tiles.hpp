// tiles.hpp -- the per-column and per-pair-tile scoring steps of SIS
// (Sec. 2.2, eq. sis-weight), shared by the single-problem kernels and the
// batched persistent kernel so that both compute every score with the same
// sequence of FP32/FP64 operations.
#pragma once
#include "screen.hpp"

namespace sisso {

constexpr int kColWaves = 4;       // waves per block of the column kernels
constexpr int kColBatch = 16;      // columns per wave between list merges
constexpr int kColRegs = 8;        // float4 per lane of a register-resident column (n <= 2048)

// ------------------------------------------------------------ columns

// Score of a stored column (scs[0]) and of its unary children (scs[1 + o] for
// the o-th unary operator, when do_unary), -1 where invalid.  One wave per
// column; every lane returns the same values.  The column's shift is its mean;
// a unary child's shift is its mean over the first 256 samples.  WT: sample
// weights w32 (mean 1) enter the sums A and B (the residual of a weighted
// pass already carries them).
template <int NU, bool WT = false>
__device__ __forceinline__ void score_column(const float *__restrict__ col, const sisso_colstat &st,
                                             const float *__restrict__ r32, int n, double nd, double R1,
                                             double Srr, const int (&uop)[NU > 0 ? NU : 1], int nu,
                                             bool do_unary, float (&scs)[1 + NU],
                                             const float *__restrict__ w32 = nullptr)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 0; o < 1 + NU; ++o) scs[o] = -1.0f;
    if (NU == 0 || !do_unary) {
        scs[0] = score_stored_column_t<WT>(col, r32, w32, n, st.mean, st.valid != 0.0f, nd, R1, Srr);
        return;
    }
    const float f0 = st.mean;
    float a0 = 0.f, b0s = 0.f, c0 = 0.f;
    float au[NU > 0 ? NU : 1], bu[NU > 0 ? NU : 1], cu[NU > 0 ? NU : 1], sh[NU > 0 ? NU : 1];
    int badu = 0;
#pragma unroll
    for (int o = 0; o < (NU > 0 ? NU : 1); ++o) au[o] = bu[o] = cu[o] = sh[o] = 0.f;
    {
        const int t = lane * 4;
        float4 fv = make_float4(0, 0, 0, 0);
        if (t < n) fv = *reinterpret_cast<const float4 *>(col + t);
        const float fa[4] = {fv.x, fv.y, fv.z, fv.w};
        const int cnt = n < 256 ? n : 256;
#pragma unroll
        for (int o = 0; o < NU; ++o) {
            float acc = 0.f;
            if (o < nu) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (t + e < n) {
                        const float h = unary32(uop[o], fa[e]);
                        acc += fabsf(h) <= 1e15f ? h : 0.f;
                    }
            }
            sh[o] = (float)(wave_sum_dpp((double)acc) / cnt);
        }
    }
    for (int t = lane * 4; t < n; t += 256) {
        const float4 fv = *reinterpret_cast<const float4 *>(col + t);
        const float4 rv = *reinterpret_cast<const float4 *>(r32 + t);
        float4 wv = make_float4(1.f, 1.f, 1.f, 1.f);
        if (WT) wv = *reinterpret_cast<const float4 *>(w32 + t);
        const float fa[4] = {fv.x, fv.y, fv.z, fv.w};
        const float ra[4] = {rv.x, rv.y, rv.z, rv.w};
        const float wa[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (t + e < n) {
                const float g = fa[e] - f0;
                const float wg = WT ? wa[e] * g : g;
                a0 += wg; b0s = fmaf(wg, g, b0s); c0 = fmaf(g, ra[e], c0);
#pragma unroll
                for (int o = 0; o < NU; ++o) {
                    if (o < nu) {
                        const float h = unary32(uop[o], fa[e]);
                        badu |= (!(fabsf(h) <= 1e15f)) << o;
                        const float gu = h - sh[o];
                        const float wgu = WT ? wa[e] * gu : gu;
                        au[o] += wgu; bu[o] = fmaf(wgu, gu, bu[o]); cu[o] = fmaf(gu, ra[e], cu[o]);
                    }
                }
            }
        }
    }
    const double A = wave_sum_dpp((double)a0), B = wave_sum_dpp((double)b0s), C = wave_sum_dpp((double)c0);
    if (st.valid != 0.0f) scs[0] = score_from_sums(A, B, C, (double)f0, nd, R1, Srr);
    badu = wave_or_dpp(badu);
#pragma unroll
    for (int o = 0; o < NU; ++o) {
        if (o < nu) {
            const double Au = wave_sum_dpp((double)au[o]), Bu = wave_sum_dpp((double)bu[o]), Cu = wave_sum_dpp((double)cu[o]);
            float bound;
            const bool dom = unary_domain_bound(uop[o], st, &bound);
            if (st.valid != 0.0f && dom && !((badu >> o) & 1))
                scs[1 + o] = score_from_sums(Au, Bu, Cu, (double)sh[o], nd, R1, Srr);
        }
    }
}

// Sums of a unary child of a register-resident column (see
// score_column_regs): the shift (mean of the first 256 samples), then
// sum g, sum g^2, sum g r of g = op(f) - shift, in the order score_column
// takes them.  OP is a compile-time operator so the loop stays small enough
// to unroll and the column stays in registers.
template <int OP, int KR, bool WT = false>
__device__ __forceinline__ void unary_child_sums(const float4 (&fv)[KR], const float4 (&rv)[KR],
                                                 const float4 (&wv)[KR], int n, float &shift, float &au, float &bu,
                                                 float &cu, bool &bad)
{
    const int lane = threadIdx.x & 63;
    {
        const int t = lane * 4;
        const float fa[4] = {fv[0].x, fv[0].y, fv[0].z, fv[0].w};
        const int cnt = n < 256 ? n : 256;
        float acc = 0.f;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (t + e < n) {
                const float h = unary32(OP, fa[e]);
                acc += fabsf(h) <= 1e15f ? h : 0.f;
            }
        shift = (float)(wave_sum_dpp((double)acc) / cnt);
    }
    au = bu = cu = 0.f;
    bad = false;
    auto step = [&](float f, float r, float w) {
        const float h = unary32(OP, f);
        bad |= !(fabsf(h) <= 1e15f);
        const float gu = h - shift;
        const float wgu = WT ? w * gu : gu;
        au += wgu; bu = fmaf(wgu, gu, bu); cu = fmaf(gu, r, cu);
    };
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int t = lane * 4 + 256 * k;
        const float fa[4] = {fv[k].x, fv[k].y, fv[k].z, fv[k].w};
        const float ra[4] = {rv[k].x, rv[k].y, rv[k].z, rv[k].w};
        const float wa[4] = {wv[k].x, wv[k].y, wv[k].z, wv[k].w};
        if (t + 3 < n) {            // the lane's four samples all lie below n
#pragma unroll
            for (int e = 0; e < 4; ++e) step(fa[e], ra[e], wa[e]);
        } else if (t < n) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < n) step(fa[e], ra[e], wa[e]);
        }
    }
}

// score_column with the column's and the residual's samples already in
// registers: float4 k of a lane holds samples lane * 4 + 256 k .. + 3
// (zero past n), for n <= 256 * KR.  Every sum takes the same operations in
// the same order as score_column, so the two give identical scores.
template <int NU, int KR, bool WT = false>
__device__ __forceinline__ void score_column_regs(const float4 (&fv)[KR], const float4 (&rv)[KR],
                                                  const float4 (&wv)[KR], const sisso_colstat &st, int n,
                                                  double nd, double R1, double Srr,
                                                  const int (&uop)[NU > 0 ? NU : 1], int nu, bool do_unary,
                                                  float (&scs)[1 + NU])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 0; o < 1 + NU; ++o) scs[o] = -1.0f;
    const float f0 = st.mean;
    float a0 = 0.f, b0s = 0.f, c0 = 0.f;
    auto step = [&](float f, float r, float w) {
        const float g = f - f0;
        const float wg = WT ? w * g : g;
        a0 += wg; b0s = fmaf(wg, g, b0s); c0 = fmaf(g, r, c0);
    };
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int t = lane * 4 + 256 * k;
        const float fa[4] = {fv[k].x, fv[k].y, fv[k].z, fv[k].w};
        const float ra[4] = {rv[k].x, rv[k].y, rv[k].z, rv[k].w};
        const float wa[4] = {wv[k].x, wv[k].y, wv[k].z, wv[k].w};
        if (t + 3 < n) {            // the lane's four samples all lie below n
#pragma unroll
            for (int e = 0; e < 4; ++e) step(fa[e], ra[e], wa[e]);
        } else if (t < n) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t + e < n) step(fa[e], ra[e], wa[e]);
        }
    }
    const double A = wave_sum_dpp((double)a0), B = wave_sum_dpp((double)b0s), C = wave_sum_dpp((double)c0);
    if (st.valid != 0.0f) scs[0] = score_from_sums(A, B, C, (double)f0, nd, R1, Srr);
    if (NU == 0 || !do_unary) return;
#pragma unroll
    for (int o = 0; o < (NU > 0 ? NU : 1); ++o) {
        if (o >= nu) continue;
        float sh = 0.f, au = 0.f, bu = 0.f, cu = 0.f;
        bool bad = false;
        switch (uop[o]) {
        case SISSO_SQ: unary_child_sums<SISSO_SQ, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        case SISSO_CUBE: unary_child_sums<SISSO_CUBE, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        case SISSO_SQRT: unary_child_sums<SISSO_SQRT, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        case SISSO_INV: unary_child_sums<SISSO_INV, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        case SISSO_EXP: unary_child_sums<SISSO_EXP, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        case SISSO_NEXP: unary_child_sums<SISSO_NEXP, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        case SISSO_LOG: unary_child_sums<SISSO_LOG, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        case SISSO_SIN: unary_child_sums<SISSO_SIN, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        default: unary_child_sums<-1, KR, WT>(fv, rv, wv, n, sh, au, bu, cu, bad); break;
        }
        const bool anybad = wave_or_dpp(bad ? 1 : 0) != 0;
        const double Au = wave_sum_dpp((double)au), Bu = wave_sum_dpp((double)bu), Cu = wave_sum_dpp((double)cu);
        float bound;
        const bool dom = unary_domain_bound(uop[o], st, &bound);
        if (st.valid != 0.0f && dom && !anybad) scs[1 + o] = score_from_sums(Au, Bu, Cu, (double)sh, nd, R1, Srr);
    }
}

// ---------------------------------------------------------- pair tiles

template <int RU, int RV>
struct RectCfg {
    static constexpr int TU = 16 * RU, TV = 16 * RV;
    static constexpr int TUP = TU + 4, TVP = TV + 4;
    static constexpr int BUF = kSC * (3 * TUP + 3 * TVP) + 2 * kSC;   // floats per buffer (+ r, w chunks)
};

// Canonical id of binary candidate (u, v, slot) of a pair block.
//   RECT (one-sided slice): u in N_L, v in P_{L-1}; row(u) = (u - u_first) * vcount
//   TRI  (last TRI level):  u in N_{L-1}, v < u;   row(u) = C(u,2) - C(u_first,2)
struct PairIds {
    int64_t base;       // id of (u_first, v = 0, slot 0)
    int64_t u_first;
    int64_t vcount;     // RECT only
    int S;              // slots per pair
    bool tri;
    __device__ __forceinline__ int64_t row(int64_t u) const
    {
        return tri ? choose2(u) - choose2(u_first) : (u - u_first) * vcount;
    }
};

// Operand statistics of a tile's u rows (thread role: rows ty*RU + a) and the
// staging column of this thread.
template <int RU, int RV>
struct USide {
    float fo[RU], mx[RU], mn[RU], rm[RU];
    bool val[RU];
    int64_t row[RU];
    int64_t su;
    bool su_ok;
    float smean;
};

template <int RU, int RV>
__device__ __forceinline__ void load_uside(USide<RU, RV> &U, const sisso_colstat *__restrict__ stats,
                                           const PairIds &ids, int64_t u0, int64_t uhi)
{
    using Cfg = RectCfg<RU, RV>;
    const int tid = threadIdx.x, ty = tid >> 4;
    const int scol = tid / (kSC / 4);
    U.su = u0 + (scol < Cfg::TU ? scol : 0);
    U.su_ok = scol < Cfg::TU && U.su < uhi;
    U.smean = stats[U.su_ok ? U.su : u0].mean;
#pragma unroll
    for (int a = 0; a < RU; ++a) {
        const int64_t u = u0 + ty * RU + a;
        const bool in = u < uhi;
        const sisso_colstat st = stats[in ? u : u0];
        U.val[a] = in && st.valid != 0.0f;
        U.fo[a] = st.mean; U.mx[a] = st.maxabs; U.mn[a] = st.minabs; U.rm[a] = st.rms;
        U.row[a] = ids.row(in ? u : u0);
    }
}

// Scores of the RU*RV*5 candidates of this thread in the tile (u rows
// [u0, u0 + TU), v columns [v0, v0 + TV) below vcount): binary form k of
// (u, v) goes to osc[(a*RV + b)*5 + k], its id to oid (-1 / INT64_MAX where
// invalid, outside [id_begin, id_end), or not an operator of the space).  In
// TRI mode only v < u is a candidate.  Sample chunks of kSC samples of both
// operand tiles and of r are staged through LDS (buf0/buf1, double
// buffered); the forms are evaluated in registers.  Block-uniform call.
template <int RU, int RV, bool WT = false>
__device__ __forceinline__ void score_pair_tile(
    const float *__restrict__ pool32, int64_t ld32, const sisso_colstat *__restrict__ stats,
    const float *__restrict__ r32, int n, double nd, double R1, double Srr, const FormSlots &fs,
    const PairIds &ids, int64_t u0, const USide<RU, RV> &U, int64_t v0, int64_t vcount, int64_t id_begin,
    int64_t id_end, float *buf0, float *buf1, float (&osc)[RU * RV * 5], int64_t (&oid)[RU * RV * 5],
    const float *__restrict__ w32 = nullptr, const int16_t *__restrict__ units = nullptr)
{
    using Cfg = RectCfg<RU, RV>;
    constexpr int TU = Cfg::TU, TV = Cfg::TV, TUP = Cfg::TUP, TVP = Cfg::TVP;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int nch = (n + kSC - 1) / kSC;
    const int scol = tid / (kSC / 4), squad = tid % (kSC / 4);
    const int64_t su = U.su;
    const bool su_ok = U.su_ok;

    const int64_t sv = v0 + (scol < TV ? scol : 0);
    const bool sv_ok = scol < TV && sv < vcount;
    const float svmean = stats[sv_ok ? sv : 0].mean;
    float vfo[RV], vmx[RV], vmn[RV], vrm[RV];
    bool vval[RV];
#pragma unroll
    for (int b = 0; b < RV; ++b) {
        const int64_t v = v0 + tx * RV + b;
        vval[b] = v < vcount;
        const sisso_colstat st = stats[vval[b] ? v : 0];
        vval[b] = vval[b] && st.valid != 0.0f;
        vfo[b] = st.mean; vmx[b] = st.maxabs; vmn[b] = st.minabs; vrm[b] = st.rms;
    }
    // shift constants of the multiplicative forms (set by the pilot below);
    // sums and differences use the operands' exact means
    float cm[RU][RV], c3[RU][RV], c4[RU][RV];
    // A stays small (the shifts are means) and is kept in FP32; B and C are
    // carried in FP64 across chunks
    double dB[RU][RV][5], dC[RU][RV][5];
    float fA[RU][RV][5], fB[RU][RV][5], fC[RU][RV][5];
#pragma unroll
    for (int a = 0; a < RU; ++a)
#pragma unroll
        for (int b = 0; b < RV; ++b)
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                dB[a][b][k] = dC[a][b][k] = 0.0;
                fA[a][b][k] = fB[a][b][k] = fC[a][b][k] = 0.0f;
            }

    // register prefetch of one chunk
    float4 pu = make_float4(0, 0, 0, 0), pv = make_float4(0, 0, 0, 0), pr = make_float4(0, 0, 0, 0);
    float4 pw = make_float4(0, 0, 0, 0);
    auto load_chunk = [&](int ch) {
        const int t0 = ch * kSC + squad * 4;
        pu = make_float4(0, 0, 0, 0);
        pv = make_float4(0, 0, 0, 0);
        if (t0 < n) {
            if (su_ok) pu = *reinterpret_cast<const float4 *>(pool32 + (size_t)su * ld32 + t0);
            if (sv_ok) pv = *reinterpret_cast<const float4 *>(pool32 + (size_t)sv * ld32 + t0);
        }
        if (tid < kSC / 4) {
            const int tr = ch * kSC + tid * 4;
            pr = tr < n ? *reinterpret_cast<const float4 *>(r32 + tr) : make_float4(0, 0, 0, 0);
            if (WT) pw = tr < n ? *reinterpret_cast<const float4 *>(w32 + tr) : make_float4(0, 0, 0, 0);
        }
    };
    auto store_chunk = [&](float *bf) {
        float *Ur = bf, *Us = Ur + kSC * TUP, *Uq = Us + kSC * TUP;
        float *Vr = Uq + kSC * TUP, *Vs = Vr + kSC * TVP, *Vq = Vs + kSC * TVP;
        float *R = Vq + kSC * TVP;
        const float uv[4] = {pu.x, pu.y, pu.z, pu.w};
        const float vv[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int srow = squad * 4 + e;
            if (scol < TU) {
                Ur[srow * TUP + scol] = uv[e];
                Us[srow * TUP + scol] = uv[e] - U.smean;
                Uq[srow * TUP + scol] = __builtin_amdgcn_rcpf(uv[e]);
            }
            if (scol < TV) {
                Vr[srow * TVP + scol] = vv[e];
                Vs[srow * TVP + scol] = vv[e] - svmean;
                Vq[srow * TVP + scol] = __builtin_amdgcn_rcpf(vv[e]);
            }
        }
        if (tid < kSC / 4) {
            R[tid * 4 + 0] = pr.x; R[tid * 4 + 1] = pr.y;
            R[tid * 4 + 2] = pr.z; R[tid * 4 + 3] = pr.w;
            if (WT) {
                float *Wc = R + kSC;
                Wc[tid * 4 + 0] = pw.x; Wc[tid * 4 + 1] = pw.y;
                Wc[tid * 4 + 2] = pw.z; Wc[tid * 4 + 3] = pw.w;
            }
        }
    };

    __syncthreads();
    load_chunk(0);
    store_chunk(buf0);
    __syncthreads();
    {
        // pilot: shift of the multiplicative forms = their mean over the first
        // chunk, so that B - A^2/n does not cancel
        const float *Ur = buf0, *Uq = Ur + 2 * kSC * TUP;
        const float *Vr = Uq + kSC * TUP, *Vq = Vr + 2 * kSC * TVP;
        const int c0 = n < kSC ? n : kSC;
        float pm[RU][RV], p3[RU][RV], p4[RU][RV];
#pragma unroll
        for (int a = 0; a < RU; ++a)
#pragma unroll
            for (int b = 0; b < RV; ++b) pm[a][b] = p3[a][b] = p4[a][b] = 0.0f;
        for (int t = 0; t < c0; ++t) {
#pragma unroll
            for (int a = 0; a < RU; ++a)
#pragma unroll
                for (int b = 0; b < RV; ++b) {
                    const float ur = Ur[t * TUP + ty * RU + a], uq = Uq[t * TUP + ty * RU + a];
                    const float vr = Vr[t * TVP + tx * RV + b], vq = Vq[t * TVP + tx * RV + b];
                    pm[a][b] = fmaf(ur, vr, pm[a][b]);
                    p3[a][b] = fmaf(ur, vq, p3[a][b]);
                    p4[a][b] = fmaf(vr, uq, p4[a][b]);
                }
        }
        const float inv = 1.0f / (float)c0;
#pragma unroll
        for (int a = 0; a < RU; ++a)
#pragma unroll
            for (int b = 0; b < RV; ++b) {
                cm[a][b] = pm[a][b] * inv;
                c3[a][b] = p3[a][b] * inv;
                c4[a][b] = p4[a][b] * inv;
            }
    }
    for (int ch = 0; ch < nch; ++ch) {
        float *bf = (ch & 1) ? buf1 : buf0;
        if (ch + 1 < nch) load_chunk(ch + 1);
        const float *Ur = bf, *Us = Ur + kSC * TUP, *Uq = Us + kSC * TUP;
        const float *Vr = Uq + kSC * TUP, *Vs = Vr + kSC * TVP, *Vq = Vs + kSC * TVP;
        const float *R = Vq + kSC * TVP;
        const int cnt = (n - ch * kSC) < kSC ? (n - ch * kSC) : kSC;
        auto step = [&](int t) {
            float ur[RU], us[RU], uq[RU], vr[RV], vs[RV], vq[RV];
#pragma unroll
            for (int a = 0; a < RU; ++a) {
                ur[a] = Ur[t * TUP + ty * RU + a];
                us[a] = Us[t * TUP + ty * RU + a];
                uq[a] = Uq[t * TUP + ty * RU + a];
            }
#pragma unroll
            for (int b = 0; b < RV; ++b) {
                vr[b] = Vr[t * TVP + tx * RV + b];
                vs[b] = Vs[t * TVP + tx * RV + b];
                vq[b] = Vq[t * TVP + tx * RV + b];
            }
            const float r = R[t];
            const float wt = WT ? R[kSC + t] : 1.0f;
#pragma unroll
            for (int a = 0; a < RU; ++a)
#pragma unroll
                for (int b = 0; b < RV; ++b) {
                    float g[5];
#pragma unroll
                    for (int k = 0; k < 5; ++k)
                        g[k] = binary_form(k, ur[a], us[a], uq[a], vr[b], vs[b], vq[b], cm[a][b], c3[a][b],
                                           c4[a][b]);
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        const float wg = WT ? wt * g[k] : g[k];
                        fA[a][b][k] += wg;
                        fB[a][b][k] = fmaf(wg, g[k], fB[a][b][k]);
                        fC[a][b][k] = fmaf(g[k], r, fC[a][b][k]);
                    }
                }
        };
        if (cnt == kSC) {
#pragma unroll 4
            for (int t = 0; t < kSC; ++t) step(t);
        } else {
            for (int t = 0; t < cnt; ++t) step(t);
        }
        // carry the chunk's FP32 partial sums in FP64
#pragma unroll
        for (int a = 0; a < RU; ++a)
#pragma unroll
            for (int b = 0; b < RV; ++b)
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    dB[a][b][k] += (double)fB[a][b][k];
                    dC[a][b][k] += (double)fC[a][b][k];
                    fB[a][b][k] = fC[a][b][k] = 0.0f;
                }
        if (ch + 1 < nch) store_chunk((ch & 1) ? buf0 : buf1);
        __syncthreads();
    }

    // scores, validity and ids of the tile's candidates
#pragma unroll
    for (int a = 0; a < RU; ++a)
#pragma unroll
        for (int b = 0; b < RV; ++b) {
            const int64_t v = v0 + tx * RV + b;
            const int64_t u = u0 + ty * RU + a;
            const bool ok = U.val[a] && vval[b] && (!ids.tri || v < u);
            // dimensional analysis: a sum or difference needs equal units
            const bool same_units = !units || unit_eq(unit_of(units, ok ? u : 0), unit_of(units, ok ? v : 0));
            const double shifts[5] = {(double)U.fo[a] + (double)vfo[b], (double)U.fo[a] - (double)vfo[b],
                                      (double)cm[a][b], (double)c3[a][b], (double)c4[a][b]};
            const float *cu = pool32 + (size_t)(ok ? u : 0) * ld32;
            const float *cv = pool32 + (size_t)(ok ? v : 0) * ld32;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int e = (a * RV + b) * 5 + k;
                float sc = -1.0f;
                int64_t fid = INT64_MAX;
                if (fs.slot[k] >= 0 && ok && (k >= 2 || same_units)) {
                    fid = ids.base + (U.row[a] + v) * ids.S + fs.slot[k];
                    if (fid >= id_begin && fid < id_end)
                        sc = form_score(k, fA[a][b][k], dB[a][b][k], dC[a][b][k], shifts[k], cu, cv, n, U.mx[a],
                                        U.mn[a], U.rm[a], vmx[b], vmn[b], vrm[b], nd, R1, Srr);
                }
                osc[e] = sc;
                oid[e] = fid;
            }
        }
}

// Exact FP32 score of one candidate of the one-sided slice's binary block,
// by one thread, with the pair-tile kernel's sequence of operations (pilot
// over the first chunk, FP32 chunk sums carried in FP64), so the value is
// bit-identical to the tile kernel's.  -1 for an invalid candidate or an id
// outside the binary block.
__device__ inline float score_slice_id(const sisso_space &s, const FormSlots &fs, int n,
                                       const float *__restrict__ pool32, int64_t ld32,
                                       const sisso_colstat *__restrict__ stats, const float *__restrict__ r32,
                                       const sisso_resid_info *__restrict__ info, int64_t id,
                                       const int16_t *__restrict__ units = nullptr)
{
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
    if (units && k < 2 && !unit_eq(unit_of(units, u), unit_of(units, v))) return -1.0f;
    const float *cu = pool32 + (size_t)u * ld32, *cv = pool32 + (size_t)v * ld32;
    const int c0 = n < kSC ? n : kSC;
    float pm = 0.f, p3 = 0.f, p4 = 0.f;
    for (int t = 0; t < c0; ++t) {
        const float ur = cu[t], vr = cv[t];
        const float uq = __builtin_amdgcn_rcpf(ur), vq = __builtin_amdgcn_rcpf(vr);
        pm = fmaf(ur, vr, pm);
        p3 = fmaf(ur, vq, p3);
        p4 = fmaf(vr, uq, p4);
    }
    const float inv = 1.0f / (float)c0;
    const float cm = pm * inv, c3 = p3 * inv, c4 = p4 * inv;
    float fA = 0.f, fB = 0.f, fC = 0.f;
    double dB = 0.0, dC = 0.0;
    for (int t0 = 0; t0 < n; t0 += kSC) {
        const int te = t0 + kSC < n ? t0 + kSC : n;
        for (int t = t0; t < te; ++t) {
            const float ur = cu[t], vr = cv[t];
            const float us = ur - ust.mean, vs = vr - vst.mean;
            const float uq = __builtin_amdgcn_rcpf(ur), vq = __builtin_amdgcn_rcpf(vr);
            const float g = binary_form(k, ur, us, uq, vr, vs, vq, cm, c3, c4);
            fA += g;
            fB = fmaf(g, g, fB);
            fC = fmaf(g, r32[t], fC);
        }
        dB += (double)fB;
        dC += (double)fC;
        fB = fC = 0.0f;
    }
    const double shifts[5] = {(double)ust.mean + (double)vst.mean, (double)ust.mean - (double)vst.mean,
                              (double)cm, (double)c3, (double)c4};
    return form_score(k, fA, dB, dC, shifts[k], cu, cv, n, ust.maxabs, ust.minabs, ust.rms, vst.maxabs, vst.minabs,
                      vst.rms, (double)n, info->sum_r32, info->s_rr);
}

}  // namespace sisso
