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

size_t farrow_lds_bytes(int window) { return (size_t)window * kFarrowStride * sizeof(float); }

// One output tile of one delay group for one mic, Farrow form: stages v_k over the
// group's source-position window in LDS, then one output sample per lane sums the
// group's images.  Ends with a barrier.
template <int NT>
__device__ inline void farrow_tile(const DScene& S, const DGroup& G, int g, int tile, int mic, int T,
                                   const DImage* __restrict__ imgs, float4* vw, const Seg* __restrict__ seg,
                                   const int32_t* __restrict__ segK, const float* __restrict__ v,
                                   float* __restrict__ part, int32_t* __restrict__ status)
{
    const int tid = threadIdx.x;
    const int64_t n0 = (int64_t)tile * NT;
    const int64_t ws = n0 - G.dmax - 4;                 // source position of window slot 0
    const int W = NT + (G.dmax - G.dmin) + 9;
    const int64_t plo = -T / 2, phi = S.n_in + T / 2;    // positions with stored v
    const float4* vs = (const float4*)(v + S.v_off);
    for (int p = tid; p < W; p += NT) {
        const int64_t P = ws + p;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a;
        if (P >= plo && P < phi) {
            const float4* q = vs + (P + T / 2) * 3;
            a = q[0];
            b = q[1];
            c = q[2];
        }
        vw[3 * p] = a;
        vw[3 * p + 1] = b;
        vw[3 * p + 2] = c;
    }
    __syncthreads();

    const int64_t n = n0 + tid;
    if (n < S.n_out) {
        const int64_t trk = S.trk_base + (int64_t)mic * S.seg_per_mic;
        const DImage* I = imgs + S.img_begin;
        const float fn = (float)n + 0.5f;
        float acc = 0.0f;
        int bad = 0;
        auto seg_index = [&](const DImage& im, int* kout) {
            int k = (int)(fn * im.invR);
            k = min(max(k, 0), im.n_seg - 1);
            *kout = k;
            return trk + im.seg_off + k;
        };
        DImage nim = I[G.img_begin];
        int nk;
        int64_t nsidx = seg_index(nim, &nk);
        Seg nsg = seg[nsidx];
        int nKs = segK[nsidx];
        for (int ii = G.img_begin; ii < G.img_end; ++ii) {
            const DImage im = nim;
            const int k = nk;
            const Seg sg = nsg;
            const int Ks = nKs;
            if (ii + 1 < G.img_end) {
                nim = I[ii + 1];
                nsidx = seg_index(nim, &nk);
                nsg = seg[nsidx];
                nKs = segK[nsidx];
            }
            const float vv = (float)(n - (int64_t)k * im.R);
            const float d = sg.a0 + vv * (sg.b1 + vv * (sg.b2 + vv * sg.b3));
            const float fl = floorf(d);
            const int64_t P = n - (Ks + (int)fl);
            if (!__any(P >= plo && P < phi)) continue;
            const int p = (int)(P - ws);
            if (p < 0 || p >= W) {
                bad = 1;
                continue;
            }
            const float s = 2.0f * (d - fl) - 1.0f;
            const float4 a = vw[3 * p], b = vw[3 * p + 1], c = vw[3 * p + 2];
            float r = c.w;
            r = fmaf(r, s, c.z);
            r = fmaf(r, s, c.y);
            r = fmaf(r, s, c.x);
            r = fmaf(r, s, b.w);
            r = fmaf(r, s, b.z);
            r = fmaf(r, s, b.y);
            r = fmaf(r, s, b.x);
            r = fmaf(r, s, a.w);
            r = fmaf(r, s, a.z);
            r = fmaf(r, s, a.y);
            r = fmaf(r, s, a.x);
            acc = fmaf(im.gfac * __builtin_amdgcn_rcpf((float)Ks + d), r, acc);
        }
        if (bad) atomicOr(status, kStatusWindow);
        part[S.part_base + ((int64_t)mic * S.n_grp + g) * S.n_out + n] = acc;
    }
    __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_farrow_fwd(DScene S, const DImage* __restrict__ imgs,
                                                    const DGroup* __restrict__ groups, int T,
                                                    const Seg* __restrict__ seg, const int32_t* __restrict__ segK,
                                                    const float* __restrict__ v, float* __restrict__ part,
                                                    int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    const int g = blockIdx.y;
    farrow_tile<NT>(S, groups[S.grp_begin + g], g, blockIdx.x, blockIdx.z, T, imgs, lds, seg, segK, v, part, status);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_farrow_persistent(const DScene* __restrict__ scenes,
                                                           const DImage* __restrict__ imgs,
                                                           const DGroup* __restrict__ groups, int T,
                                                           const WorkItem* __restrict__ items, int n_items,
                                                           int32_t* __restrict__ ticket, const Seg* __restrict__ seg,
                                                           const int32_t* __restrict__ segK,
                                                           const float* __restrict__ v, float* __restrict__ part,
                                                           int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(ticket, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const DScene& S = scenes[w.scene];
        farrow_tile<NT>(S, groups[S.grp_begin + w.group], w.group, w.tile, w.mic, T, imgs, lds, seg, segK, v, part,
                        status);
    }
}

__global__ void k_zero_ticket(int32_t* p)
{
    if (threadIdx.x == 0) p[0] = 0;
}

template <int NT>
static hipError_t launch_farrow_fwd_t(const DScene& hs, int taps, const DImage* d_imgs, const DGroup* d_groups,
                                      const Seg* seg, const int32_t* segK, const float* v, float* part,
                                      int32_t* d_status, hipStream_t st)
{
    const size_t lds = farrow_lds_bytes(hs.window);
    auto kern = k_farrow_fwd<NT>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)hs.n_tiles, (unsigned)hs.n_grp, (unsigned)hs.n_mics);
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, hs, d_imgs, d_groups, taps, seg, segK, v, part, d_status);
    return hipGetLastError();
}

template <int NT>
static hipError_t launch_farrow_pers_t(int n_wg, int window, int taps, const DScene* d_scenes, const DImage* d_imgs,
                                       const DGroup* d_groups, const WorkItem* items, int n_items, int32_t* ticket,
                                       const Seg* seg, const int32_t* segK, const float* v, float* part,
                                       int32_t* d_status, hipStream_t st)
{
    const size_t lds = farrow_lds_bytes(window);
    auto kern = k_farrow_persistent<NT>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(64), 0, st, ticket);
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(NT), lds, st, d_scenes, d_imgs, d_groups, taps, items, n_items,
                       ticket, seg, segK, v, part, d_status);
    return hipGetLastError();
}

hipError_t launch_farrow_fwd(int nthreads, int taps, const DScene& hs, const DImage* d_imgs, const DGroup* d_groups,
                             const Seg* seg, const int32_t* segK, const float* v, float* part, int32_t* d_status,
                             hipStream_t st)
{
    if (nthreads == 1024) return launch_farrow_fwd_t<1024>(hs, taps, d_imgs, d_groups, seg, segK, v, part, d_status, st);
    if (nthreads == 512) return launch_farrow_fwd_t<512>(hs, taps, d_imgs, d_groups, seg, segK, v, part, d_status, st);
    return hipErrorInvalidValue;
}

hipError_t launch_farrow_persistent(int nthreads, int n_wg, int window, int taps, const DScene* d_scenes,
                                    const DImage* d_imgs, const DGroup* d_groups, const WorkItem* items, int n_items,
                                    int32_t* ticket, const Seg* seg, const int32_t* segK, const float* v, float* part,
                                    int32_t* d_status, hipStream_t st)
{
    if (nthreads == 1024)
        return launch_farrow_pers_t<1024>(n_wg, window, taps, d_scenes, d_imgs, d_groups, items, n_items, ticket, seg,
                                          segK, v, part, d_status, st);
    if (nthreads == 512)
        return launch_farrow_pers_t<512>(n_wg, window, taps, d_scenes, d_imgs, d_groups, items, n_items, ticket, seg,
                                         segK, v, part, d_status, st);
    return hipErrorInvalidValue;
}

}  // namespace msim
