// gfx950 kernels of the Farrow form of the fractional delay (Sec. II-B, Eq. 3-5).
//
// The T-tap kernel h(j - mu) is replaced, for every tap j, by a degree-M
// polynomial in s = 2 mu - 1, h(j - mu) ~ sum_k c_k(j) s^k.  Then
//   sum_j h(j - mu) x[P - j] = sum_k s^k v_k[P],   v_k[P] = sum_j c_k(j) x[P - j],
// so the M+1 filtered signals v_k are computed once per source (k_farrow_conv) and
// every image sample reads v_0..v_M at P = n - floor(D) and runs Horner's rule:
// one convolution shared by all images and mics instead of T taps per image sample.
#include "msim_device.h"
#include "msim_internal.h"

#include <hip/hip_runtime.h>

namespace msim {

// v[v_off + (P + T/2) * kFarrowStride + k] for source positions P in [-T/2, n_in + T/2).
// One thread per position of every scene (prefix: first position of each scene).
__global__ __launch_bounds__(256) void k_farrow_conv(const DScene* __restrict__ scenes, int n_scenes,
                                                     const int64_t* __restrict__ prefix, int64_t total, int T,
                                                     const float* __restrict__ coef, const float* __restrict__ x,
                                                     float* __restrict__ v)
{
    __shared__ float c[kFarrowStride * 128];
    for (int i = threadIdx.x; i < kFarrowStride * T; i += blockDim.x) c[i] = coef[i];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const DScene& S = scenes[lo];
    const int64_t P = i - prefix[lo] - T / 2;
    const float* xs = x + S.x_off;
    float acc[kFarrowStride];
#pragma unroll
    for (int k = 0; k < kFarrowStride; ++k) acc[k] = 0.0f;
    // taps j = -T/2+1 .. T/2 read x[P - j]
    for (int t = 0; t < T; ++t) {
        const int64_t m = P - (t - T / 2 + 1);
        const float xv = (m >= 0 && m < S.n_in) ? xs[m] : 0.0f;
#pragma unroll
        for (int k = 0; k < kFarrowStride; ++k) acc[k] = fmaf(c[k * T + t], xv, acc[k]);
    }
    float4* out = (float4*)(v + S.v_off + (P + T / 2) * kFarrowStride);
    out[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    out[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    out[2] = make_float4(acc[8], acc[9], acc[10], acc[11]);
}

hipError_t launch_farrow_conv(const DScene* d_scenes, int n_scenes, const int64_t* d_vprefix, int64_t total, int taps,
                              const float* d_coef, const float* x, float* v, hipStream_t st)
{
    hipLaunchKernelGGL(k_farrow_conv, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, d_scenes, n_scenes,
                       d_vprefix, total, taps, d_coef, x, v);
    return hipGetLastError();
}

// Image descriptors staged in LDS per chunk of a group (one-output tile).
constexpr int kFarrowDescChunk = 256;

// LDS of the Farrow forward: a chunk of image descriptors, then the window of
// v_0..v_11 (48 B per source position).
size_t farrow_lds_bytes(int window)
{
    return (size_t)kFarrowDescChunk * 16 + (size_t)window * kFarrowStride * sizeof(float);
}

// Stages v_0..v_11 of source positions [ws, ws + W) in LDS (zero outside the
// stored positions [-T/2, n_in + T/2)).
__device__ inline void stage_v(const DScene& S, const float* __restrict__ v, int T, int ws, int W, float4* vw,
                               int nthreads)
{
    const int plo = -T / 2, phi = (int)S.n_in + T / 2;
    const float4* vs = (const float4*)(v + S.v_off);
    for (int p = threadIdx.x; p < W; p += nthreads) {
        const int P = ws + p;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a;
        if (P >= plo && P < phi) {
            const float4* q = vs + (int64_t)(P + T / 2) * 3;
            a = q[0];
            b = q[1];
            c = q[2];
        }
        vw[3 * p] = a;
        vw[3 * p + 1] = b;
        vw[3 * p + 2] = c;
    }
}

// Horner's rule for sum_k v_k s^k over the 10 (12 with HI) stored coefficients.
template <bool HI>
__device__ __forceinline__ float farrow_horner(const float4* vp, float s)
{
    const float4 a = vp[0], b = vp[1];
    float r;
    if constexpr (HI) {
        const float4 c = vp[2];
        r = fmaf(c.w, s, c.z);
        r = fmaf(r, s, c.y);
        r = fmaf(r, s, c.x);
        r = fmaf(r, s, b.w);
    } else {
        const float2 c = *(const float2*)&vp[2];
        r = fmaf(c.y, s, c.x);
        r = fmaf(r, s, b.w);
    }
    r = fmaf(r, s, b.z);
    r = fmaf(r, s, b.y);
    r = fmaf(r, s, b.x);
    r = fmaf(r, s, a.w);
    r = fmaf(r, s, a.z);
    r = fmaf(r, s, a.y);
    r = fmaf(r, s, a.x);
    return r;
}

// One delay group of an output tile [n0, n0 + TO) of one mic, Farrow form:
// stages v_k over the group's source-position window in LDS, then each of the
// TO/RB lanes adds the group's images for RB consecutive outputs to acc.  The RB
// outputs of a lane share one track segment when the image is decimated (the
// planner only picks RB > 1 when every decimation is a multiple of RB), so the
// segment fetch and its index arithmetic are paid once per RB image samples.
// HI selects Horner over all 12 stored coefficients (orders 10-11) instead of
// the first 10.  Ends with a barrier.
template <int TO, int RB, bool HI>
__device__ inline void farrow_group(const DScene& S, const DGroup& G, int n0, int T, Slot sl,
                                    const DImage* __restrict__ I, const PermEntry* __restrict__ perm, float4* vw, const float* __restrict__ v,
                                    float (&acc)[RB], int& bad)
{
    constexpr int NT = TO / RB;
    const int tid = threadIdx.x;
    const int ws = n0 - G.dmax - 4;                    // source position of window slot 0
    const int W = TO + (G.dmax - G.dmin) + 9;
    stage_v(S, v, T, ws, W, vw, NT);
    __syncthreads();

    const int nf = n0 + RB * tid;                       // first output of this lane
    const int n_out = (int)S.n_out;
    if (nf < n_out) {
        // slot indices of the lane's segments, kept for the last decimation seen
        int cR = 0, cl[RB];
        float cv = 0.0f;
        auto fetch = [&](const DImage& im, Seg (&q)[RB], int (&K)[RB], float& vv) {
            if (im.R != cR) {
                cR = im.R;
                if (cR == 1) {
#pragma unroll
                    for (int j = 0; j < RB; ++j) cl[j] = min(nf + j, n_out - 1) - n0;
                    cv = 0.0f;
                } else {
                    const int k = div_exact(nf, cR, im.invR);
                    cl[0] = k - div_exact(n0, cR, im.invR);
                    cv = (float)(nf - k * cR);
                }
            }
            if (im.R == 1) {
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    q[j] = sl.seg[im.loc + cl[j]];
                    K[j] = sl.K[im.loc + cl[j]];
                }
            } else {
                q[0] = sl.seg[im.loc + cl[0]];
                K[0] = sl.K[im.loc + cl[0]];
            }
            vv = cv;
        };
        auto body = [&](const DImage& im, const Seg (&q)[RB], const int (&Kq)[RB], float v0) {
            float d[RB];
            int Ks[RB];
            if (im.R == 1) {
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    d[j] = q[j].a0;
                    Ks[j] = Kq[j];
                }
            } else {
                const Seg sg = q[0];
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    const float vv = v0 + (float)j;
                    d[j] = fmaf(vv, fmaf(vv, fmaf(vv, sg.b3, sg.b2), sg.b1), sg.a0);
                    Ks[j] = Kq[0];
                }
            }
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                // positions outside the stored range read the window's zeros
                const float fl = floorf(d[j]);
                const int p = nf + j - (Ks[j] + (int)fl) - ws;
                if ((unsigned)p >= (unsigned)W) {
                    bad = 1;
                    continue;
                }
                const float r = farrow_horner<HI>(vw + __mul24(p, 3), 2.0f * (d[j] - fl) - 1.0f);
                acc[j] = fmaf(im.gfac * __builtin_amdgcn_rcpf((float)Ks[j] + d[j]), r, acc[j]);
            }
        };
        // three buffers in turn: image ii is summed while ii+1 and ii+2 are in flight
        Seg q0[RB] = {}, q1[RB] = {}, q2[RB] = {};
        int K0[RB] = {}, K1[RB] = {}, K2[RB] = {};
        float k0 = 0.0f, k1 = 0.0f, k2 = 0.0f;
        const int e = G.img_end;
        DImage i0 = perm_image(I, perm, G.img_begin), i1 = i0, i2 = i0;
        fetch(i0, q0, K0, k0);
        if (G.img_begin + 1 < e) {
            i1 = perm_image(I, perm, G.img_begin + 1);
            fetch(i1, q1, K1, k1);
        }
        int ii = G.img_begin;
        for (; ii + 2 < e; ii += 3) {
            i2 = perm_image(I, perm, ii + 2);
            fetch(i2, q2, K2, k2);
            body(i0, q0, K0, k0);
            if (ii + 3 < e) {
                i0 = perm_image(I, perm, ii + 3);
                fetch(i0, q0, K0, k0);
            }
            body(i1, q1, K1, k1);
            if (ii + 4 < e) {
                i1 = perm_image(I, perm, ii + 4);
                fetch(i1, q1, K1, k1);
            }
            body(i2, q2, K2, k2);
        }
        if (ii < e) body(i0, q0, K0, k0);
        if (ii + 1 < e) body(i1, q1, K1, k1);
    }
    __syncthreads();
}

// The same with one output per lane, branch-free per image.  A full-rate track
// segment carries zero cubic terms, so the decimated formula gives its delay
// too, and the lane's slot index depends only on the decimation R, so it is
// kept for the last R seen (images of a group mostly share a tier).  The group's
// image descriptors (slot offset of the lane's segment base, R, gain factor) are
// staged in LDS a chunk at a time: read there, they keep scalar memory loads out
// of the image loop (a scalar load's wait also drains every LDS read in flight).
// dsc: kFarrowDescChunk int4 in LDS; vw: the window after it.  Ends with a barrier.
template <int TO, bool HI>
__device__ inline void farrow_group1(const DScene& S, const DGroup& G, int n0, int T, Slot sl,
                                     const DImage* __restrict__ I, const PermEntry* __restrict__ perm, int4* dsc, float4* vw,
                                     const float* __restrict__ v, float& acc, int& bad)
{
    const int tid = threadIdx.x;
    const int ws = n0 - G.dmax - 4;                    // source position of window slot 0
    const int W = TO + (G.dmax - G.dmin) + 9;
    stage_v(S, v, T, ws, W, vw, TO);

    const int n = n0 + tid;
    const bool active = n < (int)S.n_out;
    int cR = 0, cl = 0;
    float cv = 0.0f;
    // descriptor j of the chunk: slot offset of segment k_lo, R, gfac, k_lo
    auto fetch = [&](int j, Seg& q, int& K, float& vv, float& gf) {
        const int4 d = dsc[j];
        const int R = __builtin_amdgcn_readfirstlane(d.y);
        if (R != cR) {
            cR = R;
            const int k = n / R;
            cl = k - d.w;
            cv = (float)(n - k * R);
        }
        const int off = __builtin_amdgcn_readfirstlane(d.x);
        q = ld_at(sl.seg, (uint32_t)(off + cl));
        K = ld_at(sl.K, (uint32_t)(off + cl));
        vv = cv;
        gf = __int_as_float(d.z);
    };
    // positions outside the stored range read the window's zeros; a position
    // outside the window (never, for a correct plan) is read clamped to it and
    // flagged after the group (pmax: the largest window index seen, unsigned)
    const int nws = n - ws;
    uint32_t pmax = 0;
    auto body = [&](const Seg& sg, int Ks, float vv, float gf) {
        const float dl = fmaf(vv, fmaf(vv, fmaf(vv, sg.b3, sg.b2), sg.b1), sg.a0);
        const float fl = floorf(dl);
        const uint32_t p = (uint32_t)(nws - Ks - (int)fl);
        pmax = max(pmax, p);
        const float r = farrow_horner<HI>(vw + 3 * min(p, (uint32_t)(W - 1)), 2.0f * (dl - fl) - 1.0f);
        acc = fmaf(gf * __builtin_amdgcn_rcpf((float)Ks + dl), r, acc);
    };
    for (int c0 = G.img_begin; c0 < G.img_end; c0 += kFarrowDescChunk) {
        const int nc = min(kFarrowDescChunk, G.img_end - c0);
        __syncthreads();                 // window staged; the previous chunk's descriptors read
        for (int i = tid; i < nc; i += TO) {
            const PermEntry e = perm[c0 + i];
            const DImage& im = I[e.img];
            const int klo = n0 / im.R;
            dsc[i] = make_int4(e.loc, im.R, __float_as_int(im.gfac), klo);
        }
        __syncthreads();
        if (!active) continue;
        // three buffers in turn: image j is summed while j+1 and j+2 are in flight
        Seg q0{}, q1{}, q2{};
        int K0 = 0, K1 = 0, K2 = 0;
        float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        fetch(0, q0, K0, v0, g0);
        if (nc > 1) fetch(1, q1, K1, v1, g1);
        int j = 0;
        for (; j + 2 < nc; j += 3) {
            fetch(j + 2, q2, K2, v2, g2);
            body(q0, K0, v0, g0);
            if (j + 3 < nc) fetch(j + 3, q0, K0, v0, g0);
            body(q1, K1, v1, g1);
            if (j + 4 < nc) fetch(j + 4, q1, K1, v1, g1);
            body(q2, K2, v2, g2);
        }
        if (j < nc) body(q0, K0, v0, g0);
        if (j + 1 < nc) body(q1, K1, v1, g1);
    }
    bad |= pmax >= (uint32_t)W;
    __syncthreads();
}

// Farrow forward, persistent: work items (scene, mic, tile, supergroup) from the
// ticket counter; per delay group of the supergroup the tracks over the tile go
// to the workgroup's slot (tile_tracks) and the group's images are added to the
// lane's accumulators; the item's sum is written once.
template <int TO, int RB, bool HI>
__global__ __launch_bounds__(TO / RB) void k_farrow(PlanView pv, int T, const WorkItem* __restrict__ items,
                                                     int n_items, int32_t* __restrict__ ticket, TrackArgs ta,
                                                     const float* __restrict__ v, float* __restrict__ part,
                                                     int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int NT = TO / RB;
    const Slot sl = slot_at(ta.slots, ta.slot_bytes, ta.slot_segs, blockIdx.x);
    for_each_item(ticket, n_items, [&](int it) {
        const WorkItem w = items[it];
        const DScene& S = pv.scenes[w.scene];
        const DImage* I = pv.imgs + S.img_begin;
        const DBlock B = pv.blocks[S.blk_begin + w.tile / S.blk_tiles];
        const int n0 = w.tile * TO;
        const int n_out = (int)S.n_out;
        const int n_hi = min(n0 + TO, n_out);
        const int gb = sg_begin(B.n_grp, S.n_sg, w.sg), ge = sg_begin(B.n_grp, S.n_sg, w.sg + 1);
        float acc[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[j] = 0.0f;
        int bad = 0;
        for (int g = gb; g < ge; ++g) {
            const DGroup G = pv.groups[B.grp_begin + g];
            tile_tracks<NT>(S, w.mic, I, pv.perm, G.img_begin, G.img_end, n0, n_hi, group_span(TO, G.dmin, G.dmax),
                            sl, (int*)(lds + kFarrowDescChunk), ta.knots, ta.mics, ta.c, ta.fs, ta.model);
            if constexpr (RB == 1)
                farrow_group1<TO, HI>(S, G, n0, T, sl, I, pv.perm, (int4*)lds, lds + kFarrowDescChunk, v, acc[0],
                                      bad);
            else
                farrow_group<TO, RB, HI>(S, G, n0, T, sl, I, pv.perm, lds + kFarrowDescChunk, v, acc, bad);
        }
        float* out = part + S.part_base + ((int64_t)w.mic * S.n_sg + w.sg) * S.n_out;
        const int nf = n0 + RB * (int)threadIdx.x;
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if (nf + j < n_out) out[nf + j] = acc[j];
        if (bad) atomicOr(status, kStatusWindow);
    });
}

template <int TO, int RB>
static hipError_t launch_farrow_t(int n_wg, int window, int taps, int hi, const PlanView& pv,
                                  const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta,
                                  const float* v, float* part, int32_t* d_status, hipStream_t st)
{
    const size_t lds = farrow_lds_bytes(window);
    auto kern = hi ? k_farrow<TO, RB, true> : k_farrow<TO, RB, false>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(64), 0, st, ticket);
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(TO / RB), lds, st, pv, taps, items, n_items, ticket, ta, v,
                       part, d_status);
    return hipGetLastError();
}

// Outputs per lane the Farrow forward may use: every decimation must be 1 or a
// multiple of it (so a lane's outputs share a segment), and tiles must split evenly.
int farrow_outputs_per_lane(const int32_t* decim, int n_tiers)
{
    for (int rb : {4, 2}) {
        bool ok = true;
        for (int t = 0; t < n_tiers; ++t) ok = ok && (decim[t] == 1 || decim[t] % rb == 0);
        if (ok) return rb;
    }
    return 1;
}

hipError_t launch_farrow(int nthreads, int rb, int n_wg, int window, int taps, int order, const PlanView& pv,
                         const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* v,
                         float* part, int32_t* d_status, hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
    const int hi = order > 9;
#define MSIM_CALL(TO, RB)                                                                                      \
    launch_farrow_t<TO, RB>(n_wg, window, taps, hi, pv, items, n_items, ticket, ta, v, part, d_status, st)
    if (nthreads == 1024 && rb == 4) return MSIM_CALL(1024, 4);
    if (nthreads == 1024 && rb == 2) return MSIM_CALL(1024, 2);
    if (nthreads == 1024 && rb == 1) return MSIM_CALL(1024, 1);
    if (nthreads == 512 && rb == 4) return MSIM_CALL(512, 4);
    if (nthreads == 512 && rb == 2) return MSIM_CALL(512, 2);
    if (nthreads == 512 && rb == 1) return MSIM_CALL(512, 1);
#undef MSIM_CALL
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ adjoints

// Reverse of the Farrow forward y_c[n] = sum_i g_i(n) sum_k s^k v_k[P_i(n)],
// P_i(n) = n - floor(D_i(n)), s = 2 mu - 1, v_k = x * c_k:
//   u_k[P]  = sum over (mic, i, n) with P_i(n) = P of gy_c[n] g_i(n) s^k,
//   dL/dx[m] = sum_k sum_j c_k(j) u_k[m + j]          (the filter bank's transpose),
//   dL/dbeta_i = sum gy s_i(n) fs/(4 pi c D),  dL/dD = gy g (ds/dD - s/D),  ds/dD = 2 dr/ds.

// (window: the Farrow forward's, TILE + delay spread + 9 positions), then the
// track offsets, the parameter sums and a chunk of image descriptors.
constexpr int kGdDescChunk = 256;
size_t farrow_gd_lds_bytes(int window)
{
    return (size_t)window * kFarrowStride * sizeof(float) + kLscBytes + kParamLdsBytes +
           (size_t)kGdDescChunk * 2 * sizeof(int4);
}

// LDS of the dL/dx gather: the gy window, the track offsets, then the image
// descriptors of a chunk (two int4 each).
constexpr int kUDescChunk = 256;
size_t farrow_u_lds_bytes(int window)
{
    return (size_t)window * sizeof(float) + kLscBytes + (size_t)kUDescChunk * 2 * sizeof(int4);
}

// Gain and delay adjoints of one delay group, Farrow form, one output per lane of
// the tile [n0, n0 + NT): per image sample r = sum_k v_k s^k and dr/ds by Horner's
// rule for value and derivative; dL/dD into the image's Catmull-Rom partials in
// the slot (cr_partials), the wave sums of dL/dbeta_i to esum.  Ends with a
// barrier.
template <int TILE, bool HI>
__device__ inline void farrow_gd_group(const DScene& S, const DGroup& G, int n0, int T, Slot sl, AdjSlot as,
                                       const DImage* __restrict__ I, const PermEntry* __restrict__ perm, float4* vw,
                                       int4* dsc, const float* __restrict__ v, const float* __restrict__ gyc,
                                       float ghat, int& bad)
{
    constexpr int NT = kAdjThreads;
    constexpr int WAVES = NT / 64;
    constexpr int HV = TILE / NT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ws = n0 - G.dmax - 4;
    const int W = TILE + (G.dmax - G.dmin) + 9;
    stage_v(S, v, T, ws, W, vw, NT);
    const int n_out = (int)S.n_out;
    // The group's image descriptors a chunk at a time in LDS (slot offset, R, gain
    // factor, 1/R; k_lo = n0 / R), read there as wave-uniform values.
    for (int c0 = G.img_begin; c0 < G.img_end; c0 += kGdDescChunk) {
        const int nc = min(kGdDescChunk, G.img_end - c0);
        __syncthreads();                 // window staged; the previous chunk's descriptors read
        for (int i = tid; i < nc; i += NT) {
            const PermEntry e = perm[c0 + i];
            const DImage& im = I[e.img];
            dsc[2 * i] = make_int4(e.loc, im.R, __float_as_int(im.gfac), __float_as_int(im.invR));
            dsc[2 * i + 1] = make_int4(div_exact(n0, im.R, im.invR), 0, 0, 0);
        }
        __syncthreads();
        for (int hv = 0; hv < HV; ++hv) {
            const int n = n0 + hv * NT + tid;
            const bool valid = n < n_out;
            const int nc_out = valid ? n : n_out - 1;
            const float wy = valid ? gyc[n] : 0.0f;
            int cR = 0, cl = 0;
            float cv = 0.0f;
            CrLane<1> crl;
            for (int j = 0; j < nc; ++j) {
                const int4 d0 = dsc[2 * j];
                const int loc = __builtin_amdgcn_readfirstlane(d0.x);
                const int R = __builtin_amdgcn_readfirstlane(d0.y);
                const float gfac = __int_as_float(d0.z), invR = __int_as_float(d0.w);
                if (R != cR) {
                    cR = R;
                    const int k = div_exact(nc_out, R, invR);
                    const int k_lo = __builtin_amdgcn_readfirstlane(dsc[2 * j + 1].x);
                    cl = k - k_lo;
                    cv = (float)(nc_out - k * R);
                    cr_lane<1>(crl, n, nc_out, n_out, R, invR, k, k_lo, hv * WAVES + wave, lane);
                }
                const Seg sg = ld_at(sl.seg, (uint32_t)(loc + cl));
                const int Ks = ld_at(sl.K, (uint32_t)(loc + cl));
                const float dl = fmaf(cv, fmaf(cv, fmaf(cv, sg.b3, sg.b2), sg.b1), sg.a0);
                const float fl = floorf(dl);
                const int p = nc_out - (Ks + (int)fl) - ws;
                const bool inb = p >= 0 && p < W;
                if (valid && !inb) bad = 1;
                float E = 0.0f, Db = 0.0f;
                if (valid && inb && wy != 0.0f) {
                    const float s = 2.0f * (dl - fl) - 1.0f;
                    const float4 a = vw[3 * p], b = vw[3 * p + 1], c = vw[3 * p + 2];
                    const float cf[kFarrowStride] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
                    // orders up to 9 leave the last two coefficients zero
                    constexpr int KT = HI ? kFarrowStride : 10;
                    float r = cf[KT - 1], dr = 0.0f;
#pragma unroll
                    for (int k = KT - 2; k >= 0; --k) {
                        dr = fmaf(dr, s, r);
                        r = fmaf(r, s, cf[k]);
                    }
                    const float iD = __builtin_amdgcn_rcpf((float)Ks + dl);
                    E = wy * r * ghat * iD;
                    Db = wy * gfac * iD * fmaf(2.0f, dr, -r * iD);
                }
                const int li = c0 + j - G.img_begin;
                const float db[1] = {valid ? Db : 0.0f};
                cr_partials<1>(crl, db, as.dpart + loc + li * (TILE / 64));
                E = wave_sum_dpp(E);
                if (lane == 0) as.esum[li * (TILE / 64) + hv * WAVES + wave] = E;
            }
        }
    }
    __syncthreads();
}

// The same with two consecutive outputs per lane (n0 + 2 tid and the next) over
// a tile of 2 kAdjThreads outputs: both lie on one track segment (every
// decimation is 1 or even), so they share the image's descriptor, segment fetch
// and Catmull-Rom lane state, and one segmented scan and one wave sum serve both.
// wy0, wy1: dL/dy at the lane's outputs (0 past the end).  Ends with a barrier.
template <bool HI>
__device__ inline void farrow_gd_group2(const DScene& S, const DGroup& G, int n0, int T, Slot sl, AdjSlot as,
                                        const DImage* __restrict__ I, const PermEntry* __restrict__ perm,
                                        float4* vw, int4* dsc, const float* __restrict__ v, float wy0, float wy1,
                                        float ghat, int& bad)
{
    constexpr int NT = kAdjThreads;
    constexpr int TO = 2 * NT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ws = n0 - G.dmax - 4;
    const int W = TO + (G.dmax - G.dmin) + 9;
    stage_v(S, v, T, ws, W, vw, NT);
    const int n_out = (int)S.n_out;
    const int n = n0 + 2 * tid;
    const bool ok0 = n < n_out, ok1 = n + 1 < n_out;
    const int nc = ok0 ? n : n_out - 1;           // lanes past the end follow the last output
    const int nc1 = min(nc + 1, n_out - 1);
    for (int c0 = G.img_begin; c0 < G.img_end; c0 += kGdDescChunk) {
        const int nchunk = min(kGdDescChunk, G.img_end - c0);
        __syncthreads();                 // window staged; the previous chunk's descriptors read
        for (int i = tid; i < nchunk; i += NT) {
            const PermEntry e = perm[c0 + i];
            const DImage& im = I[e.img];
            dsc[2 * i] = make_int4(e.loc, im.R, __float_as_int(im.gfac), __float_as_int(im.invR));
            dsc[2 * i + 1] = make_int4(div_exact(n0, im.R, im.invR), 0, 0, 0);
        }
        __syncthreads();
        int cR = 0, cs0 = 0, cs1 = 0;
        float cv = 0.0f;
        CrLane<2> crl;
        for (int j = 0; j < nchunk; ++j) {
            const int4 d0 = dsc[2 * j];
            const int loc = __builtin_amdgcn_readfirstlane(d0.x);
            const int R = __builtin_amdgcn_readfirstlane(d0.y);
            const float gfac = __int_as_float(d0.z), invR = __int_as_float(d0.w);
            if (R != cR) {
                cR = R;
                if (R == 1) {
                    cs0 = nc - n0;
                    cs1 = nc1 - n0;
                    cv = 0.0f;
                    cr_lane<2>(crl, n, nc, n_out, 1, 1.0f, nc, n0, wave, lane);
                } else {
                    const int k = div_exact(nc, R, invR);
                    const int k_lo = __builtin_amdgcn_readfirstlane(dsc[2 * j + 1].x);
                    cs0 = cs1 = k - k_lo;
                    cv = (float)(nc - k * R);
                    cr_lane<2>(crl, n, nc, n_out, R, invR, k, k_lo, wave, lane);
                }
            }
            const Seg sg = ld_at(sl.seg, (uint32_t)(loc + cs0));
            const float a1 = ld_at(sl.seg, (uint32_t)(loc + cs1)).a0;
            const int K0s = ld_at(sl.K, (uint32_t)(loc + cs0)), K1s = ld_at(sl.K, (uint32_t)(loc + cs1));
            const float dl0 = fmaf(cv, fmaf(cv, fmaf(cv, sg.b3, sg.b2), sg.b1), sg.a0);
            const float v1 = cv + 1.0f;
            const float dl1 = R == 1 ? a1 : fmaf(v1, fmaf(v1, fmaf(v1, sg.b3, sg.b2), sg.b1), sg.a0);
            // value r and dr/ds of one output; E and dL/dD accumulate its terms
            float E = 0.0f, Db[2] = {0.0f, 0.0f};
            auto one = [&](int c, int Ks, float dl, float wy, bool ok, int r) {
                const float fl = floorf(dl);
                const int p = c - (Ks + (int)fl) - ws;
                const bool inb = p >= 0 && p < W;
                if (ok && !inb) bad = 1;
                if (ok && inb && wy != 0.0f) {
                    const float s = 2.0f * (dl - fl) - 1.0f;
                    const float4 a = vw[3 * p], b = vw[3 * p + 1], cc = vw[3 * p + 2];
                    const float cf[kFarrowStride] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, cc.x, cc.y, cc.z, cc.w};
                    constexpr int KT = HI ? kFarrowStride : 10;
                    float rv = cf[KT - 1], dr = 0.0f;
#pragma unroll
                    for (int k = KT - 2; k >= 0; --k) {
                        dr = fmaf(dr, s, rv);
                        rv = fmaf(rv, s, cf[k]);
                    }
                    const float iD = __builtin_amdgcn_rcpf((float)Ks + dl);
                    E = fmaf(wy * rv * ghat, iD, E);
                    Db[r] = wy * gfac * iD * fmaf(2.0f, dr, -rv * iD);
                }
            };
            one(nc, K0s, dl0, wy0, ok0, 0);
            one(nc1, K1s, dl1, wy1, ok1, 1);
            const int li = c0 + j - G.img_begin;
            cr_partials<2>(crl, Db, as.dpart + loc + li * (TO / 128));
            E = wave_sum_dpp(E);
            if (lane == 0) {
                as.esum[li * (TO / 64) + 2 * wave] = E;
                as.esum[li * (TO / 64) + 2 * wave + 1] = 0.0f;
            }
        }
    }
    __syncthreads();
}

// Gain/delay adjoint and parameter partials, Farrow form, persistent over work
// items (scene, mic, tile, supergroup): one row of parameter partials per item.
// kAdjThreads lanes, TILE / kAdjThreads outputs per lane in turn (RB 1), or two
// consecutive outputs per lane at once (RB 2, TILE = 2 kAdjThreads).
template <int TILE, bool HI, int RB>
__global__ __launch_bounds__(kAdjThreads) void k_farrow_gd(PlanView pv, int T, const WorkItem* __restrict__ items,
                                                           int n_items, int32_t* __restrict__ ticket, TrackArgs ta,
                                                           int window, const float* __restrict__ v,
                                                           const float* __restrict__ gy, ParamArgs pa,
                                                           int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int NT = kAdjThreads;
    float4* vw = lds;
    int* lsc = (int*)(lds + 3 * window);
    double* pl = (double*)((char*)lsc + kLscBytes);
    int4* dsc = (int4*)((char*)pl + kParamLdsBytes);
    const Slot sl = slot_at(ta.slots, ta.slot_bytes, ta.slot_segs, blockIdx.x);
    const AdjSlot as = adj_slot_at(ta, pa.gmax, TILE, blockIdx.x);
    for_each_item(ticket, n_items, [&](int it) {
        const WorkItem w = items[it];
        const DScene& S = pv.scenes[w.scene];
        const DImage* I = pv.imgs + S.img_begin;
        const DBlock B = pv.blocks[S.blk_begin + w.tile / S.blk_tiles];
        const int n0 = w.tile * TILE;
        const int n_out = (int)S.n_out;
        const int n_hi = min(n0 + TILE, n_out);
        const float* gyc = gy + S.y_off + (int64_t)w.mic * S.n_out;
        ParamAcc acc;
        param_item_begin<NT>(pl, acc);
        const int gb = sg_begin(B.n_grp, S.n_sg, w.sg), ge = sg_begin(B.n_grp, S.n_sg, w.sg + 1);
        int bad = 0;
        for (int g = gb; g < ge; ++g) {
            const DGroup G = pv.groups[B.grp_begin + g];
            tile_tracks<NT>(S, w.mic, I, pv.perm, G.img_begin, G.img_end, n0, n_hi,
                            group_span(TILE, G.dmin, G.dmax), sl, lsc, ta.knots, ta.mics, ta.c, ta.fs, ta.model);
            if constexpr (RB == 1) {
                farrow_gd_group<TILE, HI>(S, G, n0, T, sl, as, I, pv.perm, vw, dsc, v, gyc, pa.ghat, bad);
            } else {
                static_assert(TILE == 2 * NT, "two outputs per lane cover the tile");
                const int n = n0 + 2 * (int)threadIdx.x;
                const float wy0 = n < n_out ? gyc[n] : 0.0f;
                const float wy1 = n + 1 < n_out ? gyc[n + 1] : 0.0f;
                farrow_gd_group2<HI>(S, G, n0, T, sl, as, I, pv.perm, vw, dsc, v, wy0, wy1, pa.ghat, bad);
            }
            param_group<NT, TILE, RB>(S, w.mic, G, n0, n_hi, sl, as, lsc, I, pv.perm, ta, pa, pl, acc);
        }
        param_item_end<NT>(S, w, pl, acc, pa);
        if (bad) atomicOr(status, kStatusWindow);
    });
}

template <int TILE, int RB>
static hipError_t launch_farrow_gd_t(int n_wg, int window, int taps, int hi, const PlanView& pv,
                                     const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta,
                                     const float* v, const float* gy, const ParamArgs& pa, int32_t* d_status,
                                     hipStream_t st)
{
    const size_t lds = farrow_gd_lds_bytes(window);
    auto kern = hi ? k_farrow_gd<TILE, true, RB> : k_farrow_gd<TILE, false, RB>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(64), 0, st, ticket);
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(kAdjThreads), lds, st, pv, taps, items, n_items, ticket, ta,
                       window, v, gy, pa, d_status);
    return hipGetLastError();
}

hipError_t launch_farrow_gd(int tile, int rb, int n_wg, int window, int taps, int order, const PlanView& pv,
                            const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* v,
                            const float* gy, const ParamArgs& pa, int32_t* d_status, hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
    const int hi = order > 9;
    if (tile == 2 * kAdjThreads && rb == 2)
        return launch_farrow_gd_t<2 * kAdjThreads, 2>(n_wg, window, taps, hi, pv, items, n_items, ticket, ta, v, gy,
                                                      pa, d_status, st);
    if (tile == 1024 && rb == 1)
        return launch_farrow_gd_t<1024, 1>(n_wg, window, taps, hi, pv, items, n_items, ticket, ta, v, gy, pa,
                                           d_status, st);
    if (tile == 512 && rb == 1)
        return launch_farrow_gd_t<512, 1>(n_wg, window, taps, hi, pv, items, n_items, ticket, ta, v, gy, pa,
                                          d_status, st);
    return hipErrorInvalidValue;
}

// dL/dx gather, Farrow form, persistent over items (scene, mic, position tile,
// supergroup of each delay block's groups).  One lane per source position P of
// the tile [P0, P0 + NT) of the positions [-T/2, n_in + T/2).  The outputs of
// image i that read P are the n with n - floor(D_i(n)) = P; n - D_i(n) increases
// for a subsonic image, so they form a band of at most two consecutive samples
// (none where the integer delay steps down).  Per image the lane takes one
// Newton step on n - D_i(n) = P - 1/2 from the previous image's integer delay
// (the images are sorted by delay), evaluates the rounded solution and its two
// neighbours on the (at most two) track segments they lie on, and takes
// fixed-point steps n <- P + floor(D_i(n)) from there in the rare case the band
// is not inside them (a full-rate track carries no slope, so there the Newton
// step is a fixed-point step too).  It
// accumulates u_k += gy g s^k in registers over every group of the supergroup.
// Per group the tracks cover the outputs of the block that can read the tile,
// and gy over them is staged in LDS.
// upart[S.u_base + ((mic n_sgw + sgw) (n_in + T) + P + T/2) 12 + k].
// Four waves per SIMD (at most 128 VGPRs): the per-image search waits on track
// segment loads, and the extra waves hide them (26 % faster than at 144 VGPRs).
template <int NT, bool HI>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_farrow_u(PlanView pv, int T, int fwd_tile, const WorkItem* __restrict__ items,
                                                  int n_items, int32_t* __restrict__ ticket, TrackArgs ta, int window,
                                                  const float* __restrict__ gy, float* __restrict__ upart,
                                                  int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int NU = HI ? kFarrowStride : 10;       // polynomial orders summed
    float* gw = (float*)lds;
    const Slot sl = slot_at(ta.slots, ta.slot_bytes, ta.slot_segs, blockIdx.x);
    for_each_item(ticket, n_items, [&](int it) {
        const WorkItem w = items[it];
        const DScene& S = pv.scenes[w.scene];
        const DImage* I = pv.imgs + S.img_begin;
        const int tid = threadIdx.x;
        const int P0 = w.tile * NT - T / 2;
        const int P = P0 + tid;
        const bool act = P < (int)S.n_in + T / 2;
        const int n_out = (int)S.n_out;
        int* lsc = (int*)(gw + window);
        int4* dsc = (int4*)((char*)lsc + kLscBytes);
        float u[kFarrowStride];
#pragma unroll
        for (int k = 0; k < kFarrowStride; ++k) u[k] = 0.0f;
        int bad = 0;
        // the outputs that can read the tile, and the delay blocks holding them
        const int blk_len = S.blk_tiles * fwd_tile;
        const int r_lo = max(0, P0 + S.dlo_all - 4), r_hi = min(n_out, P0 + NT + S.dhi_all + 5);
        const int b0 = r_lo / blk_len, b1 = r_lo < r_hi ? min(S.n_blk - 1, (r_hi - 1) / blk_len) : -1;
        for (int b = b0; b <= b1; ++b) {
        const DBlock B = pv.blocks[S.blk_begin + b];
        const int bl = b * blk_len, bh = min(n_out, bl + blk_len);
        const int gb = sg_begin(B.n_grp, S.n_sgw, w.sg), ge = sg_begin(B.n_grp, S.n_sgw, w.sg + 1);
        for (int g = gb; g < ge; ++g) {
            const DGroup G = pv.groups[B.grp_begin + g];
            const int nw = P0 + G.dmin - 4;                  // output of gy window slot 0
            const int W = NT + (G.dmax - G.dmin) + 9;
            // this block's outputs only: every output is gathered in its own block
            const int n_lo = max(bl, nw), n_hi = min(bh, nw + W);
            if (n_lo >= n_hi) continue;
            tile_tracks<NT>(S, w.mic, I, pv.perm, G.img_begin, G.img_end, n_lo, n_hi, group_span(NT, G.dmin, G.dmax),
                            sl, lsc, ta.knots, ta.mics, ta.c, ta.fs, ta.model);
            const float* gys = gy + S.y_off + (int64_t)w.mic * S.n_out;
            for (int p = tid; p < W; p += NT) {
                const int n = nw + p;
                gw[p] = (n >= n_lo && n < n_hi) ? gys[n] : 0.0f;
            }
            // the images are sorted by delay: each search starts from the integer
            // delay the previous image ended with
            int Kguess = (G.dmin + G.dmax) / 2;
            for (int c0 = G.img_begin; c0 < G.img_end; c0 += kUDescChunk) {
                const int nc = min(kUDescChunk, G.img_end - c0);
                if (c0 > G.img_begin) __syncthreads();      // the previous chunk's descriptors read
                // per image: first segment's slot index minus k_lo, R, gain factor,
                // 1/R; then k_lo, k_hi - k_lo
                for (int i = tid; i < nc; i += NT) {
                    const PermEntry e = pv.perm[c0 + i];
                    const DImage& im = I[e.img];
                    const int klo = n_lo / im.R, khi = (n_hi - 1) / im.R;
                    dsc[2 * i] = make_int4(e.loc - klo, im.R, __float_as_int(im.gfac), __float_as_int(im.invR));
                    dsc[2 * i + 1] = make_int4(klo, khi, 0, 0);
                }
                __syncthreads();
                if (!act) continue;
                // image j's descriptor, read from LDS as wave-uniform values
                struct Desc {
                    int base, R, klo, khi;
                    float gfac, invR;
                };
                auto desc = [&](int j) {
                    const int4 d0 = dsc[2 * j], d1 = dsc[2 * j + 1];
                    Desc d;
                    d.base = __builtin_amdgcn_readfirstlane(d0.x);
                    d.R = __builtin_amdgcn_readfirstlane(d0.y);
                    d.gfac = __int_as_float(d0.z);
                    d.invR = __int_as_float(d0.w);
                    d.klo = __builtin_amdgcn_readfirstlane(d1.x);
                    d.khi = __builtin_amdgcn_readfirstlane(d1.y);
                    return d;
                };
                // segment k of an image (klo <= k <= khi): slot entry base + k
                auto seg = [&](const Desc& d, int k) { return ld_at(sl.seg, (uint32_t)(d.base + k)); };
                auto kint = [&](const Desc& d, int k) { return ld_at(sl.K, (uint32_t)(d.base + k)); };
                // integer delay, offset and delay of output c on its segment k
                auto at = [&](const Desc& d, const Seg& sg, int Kb, int k, int c, int& K, float& off, float& D) {
                    const float vv = (float)(c - k * d.R);
                    const float dl = fmaf(vv, fmaf(vv, fmaf(vv, sg.b3, sg.b2), sg.b1), sg.a0);
                    const float fl = floorf(dl);
                    K = Kb + (int)fl;
                    off = dl - fl;
                    D = (float)Kb + dl;
                };
                auto clampn = [&](int n) { return min(max(n, n_lo), n_hi - 1); };
                for (int j = 0; j < nc; ++j) {
                    const Desc d = desc(j);
                    // u_k += gy g s^k for output c (n_lo <= c < n_hi: inside the gy window)
                    auto add = [&](int c, float off, float D, bool hit = true) {
                        const float sv = 2.0f * off - 1.0f;
                        float wv = hit ? gw[c - nw] * d.gfac * __builtin_amdgcn_rcpf(D) : 0.0f;
#pragma unroll
                        for (int k = 0; k < NU; ++k) {
                            u[k] += wv;
                            wv *= sv;
                        }
                    };
                    // The outputs reading P are the integers n with n - D(n) in
                    // (P - 1, P]: a band of width 1 / (1 - dD/dn) around the solution
                    // x of x - D(x) = P - 1/2.  One Newton step from the guess n0
                    // (the previous image's integer delay) puts n1 = round(x)
                    // within a fraction of a sample of it for a smooth track, so
                    // the band lies in n1 - 1 .. n1 + 1 (it holds at most two
                    // outputs below |dD/dn| = 1/2).
                    const int n0 = clampn(P + Kguess);
                    int n1;
                    {
                        const int k0 = div_exact(n0, d.R, d.invR);
                        const Seg sg = seg(d, k0);
                        const int Kb = kint(d, k0);
                        const float vv = (float)(n0 - k0 * d.R);
                        const float dl = fmaf(vv, fmaf(vv, fmaf(vv, sg.b3, sg.b2), sg.b1), sg.a0);
                        const float dd = fmaf(vv, fmaf(vv, 3.0f * sg.b3, 2.0f * sg.b2), sg.b1);
                        const float e = (float)(n0 - Kb - P) - dl + 0.5f;   // x - D(x) - (P - 1/2) at n0
                        n1 = clampn(n0 + (int)floorf(0.5f - e * __builtin_amdgcn_rcpf(1.0f - dd)));
                    }
                    // n1 - 1 .. n1 + 1 on two segments (three when R = 1); outside
                    // [n_lo, n_hi) a candidate reads nothing (position -inf / +inf)
                    for (int itr = 0;; ++itr) {
                        const int q = div_exact(n1, d.R, d.invR), r = n1 - q * d.R;
                        const int ka = max(r == 0 ? q - 1 : q, d.klo), kb = min(r == d.R - 1 ? q + 1 : q, d.khi);
                        const Seg sa = seg(d, ka), sb = seg(d, kb);
                        const int Ka = kint(d, ka), Kb = kint(d, kb);
                        Seg sm = r == 0 ? sb : sa;
                        int Km = r == 0 ? Kb : Ka;
                        if (d.R == 1) {
                            sm = seg(d, q);
                            Km = kint(d, q);
                        }
                        int Kc, Km1, Kp1;
                        float offc, Dc, offm, Dm, offp, Dp;
                        at(d, sm, Km, q, n1, Kc, offc, Dc);
                        at(d, sa, Ka, ka, n1 - 1, Km1, offm, Dm);
                        at(d, sb, Kb, kb, n1 + 1, Kp1, offp, Dp);
                        const int pc = n1 - Kc;
                        const int pm = n1 > n_lo ? n1 - 1 - Km1 : INT_MIN;
                        const int pp = n1 + 1 < n_hi ? n1 + 1 - Kp1 : INT_MAX;
                        // the band is inside the candidates when n1 is in it (it then
                        // holds n1 and at most one neighbour), or when it falls
                        // strictly between n1 - 1 and n1 + 1 without n1 (empty)
                        const bool inside = pc == P || (pm < P && pp > P);
                        if (inside || itr == 8) {
                            bad |= !inside;
                            Kguess = Kc;
                            add(n1, offc, Dc, pc == P);
                            const bool hm = pm == P, hp = pp == P;
                            if (hm || hp) add(hm ? n1 - 1 : n1 + 1, hm ? offm : offp, hm ? Dm : Dp);
                            break;
                        }
                        // a fixed-point step n <- P + K(n) (a contraction)
                        n1 = clampn(n1 + (P - pc));
                    }
                }
            }
        }
        }
        if (bad) atomicOr(status, kStatusWindow);
        if (act) {
            const int64_t npos = S.n_in + T;
            float4* out = (float4*)(upart + S.u_base +
                                    (((int64_t)w.mic * S.n_sgw + w.sg) * npos + (P + T / 2)) * kFarrowStride);
            out[0] = make_float4(u[0], u[1], u[2], u[3]);
            out[1] = make_float4(u[4], u[5], u[6], u[7]);
            out[2] = make_float4(u[8], u[9], u[10], u[11]);
        }
    });
}

template <int NT, bool HI>
static hipError_t launch_farrow_u_t(int n_wg, int window, int taps, int fwd_tile, const PlanView& pv, const WorkItem* items,
                                    int n_items, int32_t* ticket, const TrackArgs& ta, const float* gy, float* upart,
                                    int32_t* d_status, hipStream_t st)
{
    const size_t lds = farrow_u_lds_bytes(window);
    auto kern = k_farrow_u<NT, HI>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(64), 0, st, ticket);
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(NT), lds, st, pv, taps, fwd_tile, items, n_items, ticket, ta,
                       window, gy, upart, d_status);
    return hipGetLastError();
}

hipError_t launch_farrow_u(int nthreads, int n_wg, int window, int taps, int order, int fwd_tile, const PlanView& pv,
                           const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* gy,
                           float* upart, int32_t* d_status, hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
    if (nthreads != kAdjThreads) return hipErrorInvalidValue;
    if (order > 9)
        return launch_farrow_u_t<kAdjThreads, true>(n_wg, window, taps, fwd_tile, pv, items, n_items, ticket, ta, gy,
                                                    upart, d_status, st);
    return launch_farrow_u_t<kAdjThreads, false>(n_wg, window, taps, fwd_tile, pv, items, n_items, ticket, ta, gy,
                                                 upart, d_status, st);
}

// u = sum over (mic, supergroup) of the partial sums, in that order; one thread per
// (position, k) of every scene (prefix: first position of each scene).
__global__ __launch_bounds__(256) void k_farrow_u_reduce(PlanView pv, int n_scenes, const int64_t* __restrict__ prefix,
                                                         int64_t total, int T, const float* __restrict__ upart,
                                                         float* __restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total * kFarrowStride) return;
    const int64_t pos = i / kFarrowStride;
    const int s = scene_of(prefix, n_scenes, pos);
    const DScene& S = pv.scenes[s];
    const int64_t npos = S.n_in + T;
    const int64_t j = i - prefix[s] * kFarrowStride;       // (position, k) within the scene
    u[S.v_off + j] = strided_sum<16>(upart + S.u_base + j, S.n_mics * S.n_sgw, npos * kFarrowStride);
}

hipError_t launch_farrow_u_reduce(const PlanView& pv, int n_scenes, const int64_t* d_vprefix, int64_t vtotal, int taps,
                                  const float* upart, float* u, hipStream_t st)
{
    const int64_t n = vtotal * kFarrowStride;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_farrow_u_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pv, n_scenes, d_vprefix,
                       vtotal, taps, upart, u);
    return hipGetLastError();
}

// dL/dx[m] = sum_k sum_j c_k(j) u_k[m + j], taps j = -T/2+1 .. T/2; block (x, s):
// inputs [256 x, 256 x + 256) of scene s0 + s.
__global__ __launch_bounds__(256) void k_farrow_corr(PlanView pv, int s0, int T, const float* __restrict__ coef,
                                                     const float* __restrict__ u, float* __restrict__ gx)
{
    __shared__ float c[kFarrowStride * 128];
    __shared__ float4 us[(256 + 128) * 3];
    const DScene& S = pv.scenes[s0 + blockIdx.y];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * 256;
    if (m0 >= S.n_in) return;
    for (int i = tid; i < kFarrowStride * T; i += blockDim.x) c[i] = coef[i];
    // positions m0 + j for j in [-T/2+1, 256 + T/2): stored index m + j + T/2
    const int span = 256 + T;
    const int64_t npos = S.n_in + T;
    const float4* u4 = (const float4*)(u + S.v_off);
    for (int i = tid; i < span; i += blockDim.x) {
        const int64_t q = m0 + 1 + i;                   // stored index of position m0 - T/2 + 1 + i
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, d = a;
        if (q >= 0 && q < npos) {
            a = u4[q * 3];
            b = u4[q * 3 + 1];
            d = u4[q * 3 + 2];
        }
        us[3 * i] = a;
        us[3 * i + 1] = b;
        us[3 * i + 2] = d;
    }
    __syncthreads();
    const int64_t m = m0 + tid;
    if (m >= S.n_in) return;
    float acc = 0.0f;
    for (int t = 0; t < T; ++t) {
        // tap j = t - T/2 + 1 reads u at m + j = m0 - T/2 + 1 + (tid + t)
        const float4 a = us[3 * (tid + t)], b = us[3 * (tid + t) + 1], d = us[3 * (tid + t) + 2];
        acc = fmaf(c[0 * T + t], a.x, acc);
        acc = fmaf(c[1 * T + t], a.y, acc);
        acc = fmaf(c[2 * T + t], a.z, acc);
        acc = fmaf(c[3 * T + t], a.w, acc);
        acc = fmaf(c[4 * T + t], b.x, acc);
        acc = fmaf(c[5 * T + t], b.y, acc);
        acc = fmaf(c[6 * T + t], b.z, acc);
        acc = fmaf(c[7 * T + t], b.w, acc);
        acc = fmaf(c[8 * T + t], d.x, acc);
        acc = fmaf(c[9 * T + t], d.y, acc);
        acc = fmaf(c[10 * T + t], d.z, acc);
        acc = fmaf(c[11 * T + t], d.w, acc);
    }
    gx[S.x_off + m] = acc;
}

hipError_t launch_farrow_corr(const PlanView& pv, int s0, int n_scenes, int64_t max_in, int taps, const float* d_coef,
                              const float* u, float* gx, hipStream_t st)
{
    if (max_in == 0) return hipSuccess;
    hipLaunchKernelGGL(k_farrow_corr, dim3((unsigned)((max_in + 255) / 256), (unsigned)n_scenes), dim3(256), 0, st,
                       pv, s0, taps, d_coef, u, gx);
    return hipGetLastError();
}

}  // namespace msim
