// The quadratic fractional-delay table in LDS and the two-outputs-per-lane tap
// sums over it, shared by the forward synthesis and the gain/delay adjoint.
#pragma once

#include "msim_device.h"
#include "msim_internal.h"

#include <hip/hip_runtime.h>

namespace msim {

// Pointers to row 0 of quad 0 of the three table arrays in LDS (qtab_pitch rows
// per quad, the first of them row -1).
struct QTab {
    const float4* Y;
    const float4* D1;
    const uint2* D2;
};

template <int T>
__device__ __forceinline__ QTab qtab_view(const float4* tab, int LP)
{
    constexpr int NG = T / 8;
    return {tab + 1, tab + NG * LP + 1, (const uint2*)(tab + 2 * NG * LP) + 1};
}

// Copies the quadratic table (qtab_bytes) from global memory into LDS.
template <int T>
__device__ __forceinline__ void load_qtab(const float4* __restrict__ table, float4* tab, int Lq, int nthreads)
{
    const int n = (int)(qtab_bytes(T, Lq) / 16);
    for (int i = threadIdx.x; i < n; i += nthreads) tab[i] = table[i];
}

// Stages the source window of a tile: xw[p] = x[ws+p .. ws+p+3], zero outside [0, n_in).
__device__ __forceinline__ void stage_window(const float* __restrict__ xs, int n_in, int ws, int W, float4* xw,
                                             int nthreads)
{
    for (int p = threadIdx.x; p < W; p += nthreads) {
        const int q = ws + p;
        float4 v;
        v.x = (q >= 0 && q < n_in) ? xs[q] : 0.0f;
        v.y = (q + 1 >= 0 && q + 1 < n_in) ? xs[q + 1] : 0.0f;
        v.z = (q + 2 >= 0 && q + 2 < n_in) ? xs[q + 2] : 0.0f;
        v.w = (q + 3 >= 0 && q + 3 < n_in) ? xs[q + 3] : 0.0f;
        xw[p] = v;
    }
}

// The two-outputs-per-lane window layout.  Lane l's outputs sit two positions
// after lane l-1's, so with contiguous quads the 16 lanes of a quarter-wave read
// 32 B apart and meet every bank slot twice.  Even positions are kept in the first
// half of the entries and odd ones in the second: position p at entry
// (p & 1) * half + (p >> 1), half = (W + 1) / 2 (W + 1 entries at most).  Positions
// of one parity 4 apart are then 2 entries apart, and the lanes of a quarter-wave
// (mostly one parity) read 16 B apart.
__device__ __forceinline__ int split_half(int W) { return (W + 1) >> 1; }

__device__ __forceinline__ const float4* split_at(const float4* xw, int half, int p)
{
    // byte offset (p >> 1) * 16 + (p & 1) * half * 16, p >= 0
    const uint32_t up = (uint32_t)p;
    const uint32_t odd = (uint32_t)(((int)(up << 31)) >> 31);          // all ones for odd p
    return (const float4*)((const char*)xw + (((up << 3) & ~15u) + (odd & (uint32_t)(half * 16))));
}

// f (f - 1) / 2, the weight of the quadratic term, in two instructions.
__device__ __forceinline__ float qweight(float f)
{
    const float t = 0.5f * f;
    return fmaf(t, f, -t);
}

__device__ __forceinline__ void stage_window_split(const float* __restrict__ xs, int n_in, int ws, int W, float4* xw,
                                                   int nthreads)
{
    const int half = split_half(W);
    for (int p = threadIdx.x; p < W; p += nthreads) {
        const int q = ws + p;
        float4 v;
        v.x = (q >= 0 && q < n_in) ? xs[q] : 0.0f;
        v.y = (q + 1 >= 0 && q + 1 < n_in) ? xs[q + 1] : 0.0f;
        v.z = (q + 2 >= 0 && q + 2 < n_in) ? xs[q + 2] : 0.0f;
        v.w = (q + 3 >= 0 && q + 3 < n_in) ? xs[q + 3] : 0.0f;
        xw[(p & 1) * half + (p >> 1)] = v;
    }
}

// The frame of a lane's outputs n, n+1 for one image with delays D_m = K_ms + d_m
// (integer base plus a small FP32 offset).  Both read the table rows of one
// frame: K, the smaller of the two integer delays, with phases q_m = (D_m - K) Lq
// in table rows (in [0, 2 Lq)); the near side's base row floor(min q) and the far
// side's Lq-1-floor(max q) (down to -1), so each output's fractions on those rows,
// f_m = q_m - kq and h_m = Lq - q_m - kp, stay within [0, 2] while the delay moves
// by less than one row per sample.
struct PairFrame {
    int K;
    float q0, q1;
    int kq, kp;
};

__device__ __forceinline__ PairFrame pair_frame(float d0, int K0s, float d1, int K1s, int L, float Lf)
{
    const float fl0 = floorf(d0), fl1 = floorf(d1);
    const int i0 = K0s + (int)fl0, i1 = K1s + (int)fl1;
    PairFrame fr;
    fr.K = min(i0, i1);
    fr.q0 = ((d0 - fl0) + (float)(i0 - fr.K)) * Lf;
    fr.q1 = ((d1 - fl1) + (float)(i1 - fr.K)) * Lf;
    fr.kq = min((int)fminf(fr.q0, fr.q1), L - 1);
    fr.kp = max(L - 1 - (int)fmaxf(fr.q0, fr.q1), -1);
    return fr;
}

// Tap sums of one image for outputs n (0) and n+1 (1) in the frame K, with xq the
// split source window's entry of position n - K (split_at), written into ps (by reference: returning the sums by
// value made the register allocator spill).  Near side (taps j = -(4g+e),
// |u| = 4g+e + mu, base row kq): A += Y x, B += D1 x, C += D2 x; far side (taps
// j = 1+4g+e, |u| = 4g+e + 1-mu, base row kp): A += Y x, Bm += D1 x, Cm += D2 x.
// The value is then
//   s = A + f B + h Bm + f (f-1)/2 C + h (h-1)/2 Cm.
// Output n reads x[n-K+4g+e] on the near side and x[n-K-1-4g-e] on the far side
// (quads 4g and -4-4g, entries 2g and -2-2g of the split window); output n+1 the
// next position.  One table read (Y, D1, D2 of four taps) and one
// new source quad serve eight taps of both outputs.  The 2 T/8 steps are
// software-pipelined one deep: the rows and the source quad of step st+1 are read
// while step st is summed, and scheduling barriers keep the pipeline at that depth
// (so the values in flight stay within the register budget).
struct PairSums {
    float A0, B0, Bm0, C0, Cm0;
    float A1, B1, Bm1, C1, Cm1;
};

template <int NG, int NC = qcorr_quads(8 * NG)>
__device__ __forceinline__ void pair_sums(const QTab& tq, int LP, int kq, int kp, const float4* xq, PairSums& ps)
{
    float& A0 = ps.A0; float& B0 = ps.B0; float& Bm0 = ps.Bm0; float& C0 = ps.C0; float& Cm0 = ps.Cm0;
    float& A1 = ps.A1; float& B1 = ps.B1; float& Bm1 = ps.Bm1; float& C1 = ps.C1; float& Cm1 = ps.Cm1;
    A0 = B0 = Bm0 = C0 = Cm0 = A1 = B1 = Bm1 = C1 = Cm1 = 0.0f;
    // each side's rows of quad 0 (the steps add whole quads, LP rows each)
    const float4* Yn = tq.Y + kq;
    const float4* D1n = tq.D1 + kq;
    const uint2* D2n = tq.D2 + kq;
    const float4* Yf = tq.Y + kp;          // kp >= -1 (row -1 exists)
    const float4* D1f = tq.D1 + kp;
    const uint2* D2f = tq.D2 + kp;
    float4 xo = xq[0];                  // the previous step's source quad
    float4 xc = xq[2], Yc = Yn[0], D1c = D1n[0];
    uint2 D2c = D2n[0];
#pragma unroll
    for (int st = 0; st < 2 * NG; ++st) {
        float4 xnx = xc, Ynx = Yc, D1nx = D1c, x0 = xo;
        uint2 D2nx = D2c;
        if (st + 1 == NG) x0 = xq[0];
        if (st + 1 < 2 * NG) {
            const int s1 = st + 1;
            const int g1 = s1 < NG ? s1 : s1 - NG;
            xnx = s1 < NG ? xq[2 * s1 + 2] : xq[-2 - 2 * (s1 - NG)];
            Ynx = s1 < NG ? Yn[g1 * LP] : Yf[g1 * LP];
            D1nx = s1 < NG ? D1n[g1 * LP] : D1f[g1 * LP];
            if (g1 < NC) D2nx = s1 < NG ? D2n[g1 * LP] : D2f[g1 * LP];
        }
        const float c0 = h16_lo(D2c.x), c1 = h16_hi(D2c.x), c2 = h16_lo(D2c.y), c3 = h16_hi(D2c.y);
        // quads from NC on have no quadratic term (their table values are zero)
        const bool qc = (st < NG ? st : st - NG) < NC;
        if (st < NG) {
            // near side: output n reads quad 4g (xo, component e), output n+1 the
            // next position (the last from quad 4g+4 = xc)
            const float4 xn = xo, xa = xc;
            A0 = fmaf(Yc.x, xn.x, A0); B0 = fmaf(D1c.x, xn.x, B0);
            A1 = fmaf(Yc.x, xn.y, A1); B1 = fmaf(D1c.x, xn.y, B1);
            A0 = fmaf(Yc.y, xn.y, A0); B0 = fmaf(D1c.y, xn.y, B0);
            A1 = fmaf(Yc.y, xn.z, A1); B1 = fmaf(D1c.y, xn.z, B1);
            A0 = fmaf(Yc.z, xn.z, A0); B0 = fmaf(D1c.z, xn.z, B0);
            A1 = fmaf(Yc.z, xn.w, A1); B1 = fmaf(D1c.z, xn.w, B1);
            A0 = fmaf(Yc.w, xn.w, A0); B0 = fmaf(D1c.w, xn.w, B0);
            A1 = fmaf(Yc.w, xa.x, A1); B1 = fmaf(D1c.w, xa.x, B1);
            if (qc) {
                C0 = fmaf(c0, xn.x, C0); C1 = fmaf(c0, xn.y, C1);
                C0 = fmaf(c1, xn.y, C0); C1 = fmaf(c1, xn.z, C1);
                C0 = fmaf(c2, xn.z, C0); C1 = fmaf(c2, xn.w, C1);
                C0 = fmaf(c3, xn.w, C0); C1 = fmaf(c3, xa.x, C1);
            }
        } else {
            // far side: output n reads quad -4-4g (xc, component 3-e), output n+1
            // the next position (the first from quad -4g = xo)
            const float4 xp = xc, xr = xo;
            A0 = fmaf(Yc.x, xp.w, A0); Bm0 = fmaf(D1c.x, xp.w, Bm0);
            A1 = fmaf(Yc.x, xr.x, A1); Bm1 = fmaf(D1c.x, xr.x, Bm1);
            A0 = fmaf(Yc.y, xp.z, A0); Bm0 = fmaf(D1c.y, xp.z, Bm0);
            A1 = fmaf(Yc.y, xp.w, A1); Bm1 = fmaf(D1c.y, xp.w, Bm1);
            A0 = fmaf(Yc.z, xp.y, A0); Bm0 = fmaf(D1c.z, xp.y, Bm0);
            A1 = fmaf(Yc.z, xp.z, A1); Bm1 = fmaf(D1c.z, xp.z, Bm1);
            A0 = fmaf(Yc.w, xp.x, A0); Bm0 = fmaf(D1c.w, xp.x, Bm0);
            A1 = fmaf(Yc.w, xp.y, A1); Bm1 = fmaf(D1c.w, xp.y, Bm1);
            if (qc) {
                Cm0 = fmaf(c0, xp.w, Cm0); Cm1 = fmaf(c0, xr.x, Cm1);
                Cm0 = fmaf(c1, xp.z, Cm0); Cm1 = fmaf(c1, xp.w, Cm1);
                Cm0 = fmaf(c2, xp.y, Cm0); Cm1 = fmaf(c2, xp.z, Cm1);
                Cm0 = fmaf(c3, xp.x, Cm0); Cm1 = fmaf(c3, xp.y, Cm1);
            }
        }
        xo = st + 1 == NG ? x0 : xc;
        xc = xnx;
        Yc = Ynx;
        D1c = D1nx;
        D2c = D2nx;
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace msim
