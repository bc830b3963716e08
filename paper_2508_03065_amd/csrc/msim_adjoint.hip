// gfx950 adjoint (reverse-mode) kernels of the moving image-source synthesis.
//
// The forward map is y_c[n] = sum_i g_i(n) s_i(n),  s_i(n) = sum_j h(j - mu_i(n)) x[n - K_i(n) - j],
// with D_i(n) = K_i(n) + mu_i(n) the Catmull-Rom interpolated delay and
// g_i(n) = beta_i fs / (4 pi c D_i(n))  (Eq. 2 / Eq. 8, Sec. II-B, Sec. II-C-3),
// with h the forward's quadratic interpolation of the Kaiser-windowed sinc.  Given gy = dL/dy:
//   adj_x      : dL/dx[m] = sum_{c,i,n} gy_c[n] g_i(n) h(n - D_i(n) - m), the transpose
//                time-varying fractional delay, accumulated per wave in a shifting
//                register accumulator, per (mic, output tile, delay group) in LDS,
//                and gathered in fixed order.
//   adj_track  : per image sample, s and ds/dmu from the same table sums:
//                dL/dbeta_i += gy s fs / (4 pi c D),  dL/dD_i(n) = gy g (ds/dmu - s / D).
//   seg/grid   : transpose of the Catmull-Rom interpolation (dL/dD on the delay
//                grid), then the implicit-function derivative of the retarded
//                delay c tau = |S_i p(t - tau) + O_i - r(t)| with respect to the
//                source position at the emission time, split onto the two
//                knots of its path segment.
//   reduce     : fixed-order reductions to dL/dbeta_w and dL/dP_knot.
#include "msim_device.h"
#include "msim_internal.h"
#include "msim_pair.h"

#include <hip/hip_runtime.h>

namespace msim {

namespace {

// Delay of image `im` at output n from its track segment.
struct ImageSample {
    int K;        // integer delay
    float mu;     // fractional delay in [0, 1)
    float D;      // delay in samples (FP32, for the gain)
};

__device__ inline ImageSample sample_of(const DImage& im, int k, const Seg& sg, int Ks, int64_t n)
{
    const float v = (float)(n - (int64_t)k * im.R);
    const float d = sg.a0 + v * (sg.b1 + v * (sg.b2 + v * sg.b3));
    const float fl = floorf(d);
    ImageSample r;
    r.K = Ks + (int)fl;
    r.mu = d - fl;
    r.D = (float)Ks + d;
    return r;
}

}  // namespace

// The transpose reads the forward's quadratic table, rearranged tap-major:
// three arrays Y, D1, D2 of [T/2][Lq] floats (a packed
// {Y, D1, D2, 0} per tap and row, one b96 read instead of three b32, measured 25 %
// slower); then each wave owns a window of (window - NT + 64) samples: its 64
// outputs' taps under every delay of the group.  (Two outputs per lane, as in the
// forward, cut the instructions per tap by a third but halve the waves a CU holds
// within this LDS, and measured no faster.)
size_t adj_x_lds_bytes(int taps, int Lq, int window, int nthreads)
{
    return (size_t)3 * (taps / 2) * (size_t)Lq * sizeof(float) +
           (size_t)(nthreads / 64) * (size_t)(window - nthreads + 64) * sizeof(float);
}

size_t adj_track_lds_bytes(int taps, int Lq, int window)
{
    return qtab_bytes(taps, Lq) + (size_t)(window + 1) * sizeof(float4);
}

// ------------------------------------------------------------ transpose delay

// Transpose of the time-varying fractional delay of the table form:
//   dL/dx[m] += w h_q(j - mu)  for every image sample (w = gy g) and tap j, m = n - K - j,
// with h_q the forward's quadratic interpolation of h, so this is its exact transpose.
//
// Systolic form.  A wave holds 64 consecutive outputs of one image; their integer
// delays differ by at most one (K_ref = the smallest, dK = K - K_ref in {0, 1}),
// so at step s (s = 0 .. T) lane l's tap lands on relative source position
// l + s - T/2 - 1 (relative to n0 - K_ref).  The wave keeps one register
// accumulator per lane for that position; between steps it moves one lane down
// (DPP wave_shl:1, fused into the add), the value leaving lane 0 is complete and
// is parked in a second register that shifts the same way.  Each image's 64 + T
// positions then reach the wave's LDS window with two read-add-writes per lane
// (the old per-tap scatter needed one per tap).  Waves whose integer delay spans
// more than one sample (relative speeds above ~fs/64 samples per sample) take a
// per-tap scatter instead.  The wave windows are summed in wave order: no
// atomics, and the result does not depend on scheduling.
template <int T, int NT, int LQC>
__global__ __launch_bounds__(NT) void k_adj_x(DScene S, const DImage* __restrict__ imgs,
                                               const DGroup* __restrict__ groups, const float* __restrict__ atab,
                                               int Lr, const Seg* __restrict__ seg, const int32_t* __restrict__ segK,
                                               const float* __restrict__ gy, float* __restrict__ xpart,
                                               int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int WAVES = NT / 64;
    constexpr int H = T / 2;
    const int LQ = LQC > 0 ? LQC : Lr;
    float* tY = (float*)lds;
    float* tD1 = tY + H * LQ;
    float* tD2 = tD1 + H * LQ;
    float* wbase = tD2 + H * LQ;
    // the interpolated tap weight a Y + b D1 + c D2 at table index i (tap-major;
    // row r of tap d at d LQ + r)
    auto wt = [&](int i, float a, float b, float c) { return fmaf(a, tY[i], fmaf(b, tD1[i], c * tD2[i])); };

    const int tile = blockIdx.x, g = blockIdx.y, mic = blockIdx.z, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const DGroup G = groups[S.grp_begin + g];
    const int n0 = tile * NT;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = NT + (G.dmax - G.dmin) + T + 8;       // the tile's window
    const int Wstride = S.window - NT + 64;             // per-wave window slot
    const int Ww = W - NT + 64;                         // per-wave window used by this group
    for (int i = tid; i < 3 * H * LQ; i += NT) tY[i] = atab[i];
    for (int p = tid; p < WAVES * Wstride; p += NT) wbase[p] = 0.0f;
    __syncthreads();

    // read-add-writes of successive images stay in program order (lanes of one
    // wave may touch the same position for different images)
    volatile float* xb = wbase + wave * Wstride;        // covers source positions ws + 64 wave + [0, Ww)
    const int wsw = ws + 64 * wave;
    const int n0w = n0 + 64 * wave;
    const int n = n0w + lane;
    const int n_out = (int)S.n_out;
    const bool valid = n < n_out;
    const float wy = valid ? gy[S.y_off + (int64_t)mic * S.n_out + n] : 0.0f;
    const int nc = valid ? n : n_out - 1;
    const Seg* sgm = seg + (int64_t)mic * S.seg_per_mic;
    const int32_t* sgk = segK + (int64_t)mic * S.seg_per_mic;
    const DImage* I = imgs + S.img_begin;
    const float fn = (float)nc + 0.5f;
    const float LQf = (float)LQ;
    const int n_in = (int)S.n_in;
    int bad = 0;
    for (int ii = G.img_begin; ii < G.img_end; ++ii) {
        const DImage im = I[ii];
        const int k = min(max((int)(fn * im.invR), 0), im.n_seg - 1);
        const Seg sg = sgm[im.seg_off + k];
        const int Ks = sgk[im.seg_off + k];
        const float v = (float)(nc - __mul24(k, im.R));
        const float d = fmaf(v, fmaf(v, fmaf(v, sg.b3, sg.b2), sg.b1), sg.a0);
        const float fl = floorf(d);
        const int K = Ks + (int)fl;
        const int P = nc - K;
        const bool reach = valid && wy != 0.0f && P + T / 2 - 1 >= 0 && P - T / 2 < n_in;
        if (!__any(reach)) continue;
        // every lane's taps must fall inside the wave's window
        const int p0 = P - wsw;
        if (__any(valid && (p0 < T / 2 + 1 || p0 > Ww - T / 2 - 1))) {
            bad = 1;
            continue;
        }
        const float w = reach ? wy * im.gfac * __builtin_amdgcn_rcpf((float)Ks + d) : 0.0f;
        const float mu = d - fl;
        const float q = mu * LQf;
        const int kq = min((int)q, LQ - 1);
        const float f = q - (float)kq;
        const float A = w, Bn = w * f, Bf = w * (1.0f - f), C = w * (0.5f * f * (f - 1.0f));
        const int rf = LQ - 1 - kq;
        const int kmin = wave_min_i(K), kmax = wave_max_i(K);
        if (kmax - kmin > 1) {
            // per-tap scatter; lanes sharing a source position (the integer delay
            // stepped between them) take a second pass
            const int prevP = __shfl_up(P, 1, 64);
            const bool dup = lane > 0 && prevP == P;
            for (int pass = 0; pass < 2; ++pass) {
                if (!reach || (pass == 0 ? dup : !dup)) continue;
                for (int dd = 0; dd < H; ++dd) {
                    const int in = dd * LQ + kq, ifr = dd * LQ + rf;
                    xb[p0 + dd] += wt(in, A, Bn, C);
                    xb[p0 - 1 - dd] += wt(ifr, A, Bf, C);
                    __builtin_amdgcn_wave_barrier();
                }
            }
            continue;
        }
        const int dK = K - kmin;
        // table indices at step s: far side (d = H - s - dK) pF + (H-1-s) LQ; near side
        // (d = s - H - 1 + dK) pN + (s-H-1) LQ
        const int pF = (1 - dK) * LQ + rf;
        const int pN = dK * LQ + kq;
        // steps whose taps lie beyond the quadratic term's quads for either dK
        // (zero second differences) skip that read
        constexpr int DQ = 4 * qcorr_quads(T);
        auto far = [&](int s) {
            const int i = pF + (H - 1 - s) * LQ;
            return H - 1 - s >= DQ ? fmaf(A, tY[i], Bf * tD1[i]) : wt(i, A, Bf, C);
        };
        auto near = [&](int s) {
            const int i = pN + (s - H - 1) * LQ;
            return s - H - 1 >= DQ ? fmaf(A, tY[i], Bn * tD1[i]) : wt(i, A, Bn, C);
        };
        // relative position (to n0w - kmin) of lane l at step s: l + s - H - 1
        const int rel0 = n0w - kmin - wsw;               // window index of relative position 0
        float acc, out = 0.0f;
        int ndep = 0;                                    // departures parked in `out`
        auto step = [&](int s, float c) {
            if (s == 0) {
                acc = c;
                return;
            }
            // the value leaving lane 0 is parked in lane (s-1) mod 64 of `out`
            // (v_writelane takes the lane from a scalar and ignores EXEC; every
            // lane of the wave runs this path)
            const int dep = __builtin_amdgcn_readlane(__float_as_int(acc), 0);
            acc = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), 0x130, 0xF, 0xF, true)) + c;
            asm("v_writelane_b32 %0, %1, %2" : "+v"(out) : "s"(dep), "i"((s - 1) & 63));
            if (++ndep == 64) {
                // departures of steps s-64 .. s-1 sit in lanes 0..63
                const int pw = rel0 + (s - 64 + lane) - H - 1;
                xb[pw] += out;
                ndep = 0;
            }
        };
        step(0, dK ? far(0) : 0.0f);
#pragma unroll
        for (int s = 1; s < H; ++s) step(s, far(s));
        step(H, wt(dK ? kq : rf, A, dK ? Bn : Bf, C));
#pragma unroll
        for (int s = H + 1; s < T; ++s) step(s, near(s));
        step(T, dK ? 0.0f : near(T));
        // remaining departures (steps T-ndep .. T-1) in lanes 0 .. ndep-1
        if (lane < ndep) xb[rel0 + (T - ndep + lane) - H - 1] += out;
        xb[rel0 + lane + T - H - 1] += acc;
        __builtin_amdgcn_wave_barrier();
    }
    if (bad) atomicOr(status, kStatusWindow);
    __syncthreads();
    // tile window position p = wave window position p - 64 w, summed in wave order
    float* outp = xpart + (((int64_t)mic * S.n_grp + g) * S.n_tiles + tile) * S.window;
    for (int p = tid; p < W; p += NT) {
        float a = 0.0f;
        for (int w2 = 0; w2 < WAVES; ++w2) {
            const int pw = p - 64 * w2;
            if (pw >= 0 && pw < Ww) a += wbase[w2 * Wstride + pw];
        }
        outp[p] = a;
    }
}

template <int T, int NT>
static hipError_t launch_adj_x_t(const DScene& hs, const DImage* d_imgs, const DGroup* d_groups,
                                 const float* d_atab, int Lq, const Seg* seg, const int32_t* segK, const float* gy,
                                 float* xpart, int32_t* d_status, hipStream_t st)
{
    const size_t lds = adj_x_lds_bytes(T, Lq, hs.window, NT);
    auto kern = Lq == 128 ? k_adj_x<T, NT, 128> : k_adj_x<T, NT, 0>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)hs.n_tiles, (unsigned)hs.n_grp, (unsigned)hs.n_mics);
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, hs, d_imgs, d_groups, d_atab, Lq, seg, segK, gy, xpart,
                       d_status);
    return hipGetLastError();
}

hipError_t launch_adj_x(int taps, int nthreads, const DScene& hs, const DImage* d_imgs, const DGroup* d_groups,
                        const float* d_atab, int Lq, const Seg* seg, const int32_t* segK, const float* gy,
                        float* xpart, int32_t* d_status, hipStream_t st)
{
#define MSIM_ADJX_CASE(TT, NN)                                                                                 \
    if (taps == TT && nthreads == NN)                                                                          \
        return launch_adj_x_t<TT, NN>(hs, d_imgs, d_groups, d_atab, Lq, seg, segK, gy, xpart, d_status, st);
    MSIM_ADJX_CASE(32, 1024)
    MSIM_ADJX_CASE(64, 1024)
    MSIM_ADJX_CASE(96, 1024)
    MSIM_ADJX_CASE(128, 1024)
    MSIM_ADJX_CASE(32, 512)
    MSIM_ADJX_CASE(64, 512)
    MSIM_ADJX_CASE(96, 512)
    MSIM_ADJX_CASE(128, 512)
#undef MSIM_ADJX_CASE
    return hipErrorInvalidValue;
}

// Gathers the partial windows that cover each input sample, in a fixed order
// (mic, group, tile).  Window (mic, g, tile) covers inputs
// [tile*NT - c_g, tile*NT - c_g + W_g),  c_g = dmax_g + T/2 + 4.
__global__ __launch_bounds__(256) void k_reduce_x(DScene S, const DGroup* __restrict__ groups, int lg_nt, int T,
                                                  const float* __restrict__ xpart, float* __restrict__ gx)
{
    // 32-bit sample indices (inputs are capped at 2^23 samples); NT = 2^lg_nt, so
    // floor division by NT is an arithmetic shift
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= (int)S.n_in) return;
    const int NT = 1 << lg_nt;
    const int nt_last = (int)S.n_tiles - 1;
    float acc = 0.0f;
    // the windows of group g that cover m: tiles t_lo .. t_hi
    auto span = [&](int g, int& t_lo, int& t_hi, int& cg) {
        const DGroup G = groups[S.grp_begin + g];
        cg = G.dmax + T / 2 + 4;
        const int Wg = NT + (G.dmax - G.dmin) + T + 8;
        t_lo = max((m + cg - Wg + NT) >> lg_nt, 0);
        t_hi = min((m + cg) >> lg_nt, nt_last);
    };
    for (int mic = 0; mic < S.n_mics; ++mic) {
        const float* xm = xpart + (int64_t)mic * S.n_grp * S.n_tiles * S.window;
        auto at = [&](int g, int t, int cg) {
            return xm[((int64_t)g * S.n_tiles + t) * S.window + (m - (t * NT - cg))];
        };
        int g = 0;
        // eight groups at a time with their (at most two) windows' loads issued
        // together, then added in the plain loop's order (masked loads add zero)
        for (; g + 8 <= S.n_grp; g += 8) {
            float a0[8], a1[8];
            bool wide = false;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                int t_lo, t_hi, cg;
                span(g + u, t_lo, t_hi, cg);
                a0[u] = t_lo <= t_hi ? at(g + u, t_lo, cg) : 0.0f;
                a1[u] = t_lo + 1 <= t_hi ? at(g + u, t_lo + 1, cg) : 0.0f;
                wide |= t_hi - t_lo >= 2;
            }
            if (!wide) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    acc += a0[u];
                    acc += a1[u];
                }
                continue;
            }
            for (int u = 0; u < 8; ++u) {
                int t_lo, t_hi, cg;
                span(g + u, t_lo, t_hi, cg);
                for (int t = t_lo; t <= t_hi; ++t) acc += at(g + u, t, cg);
            }
        }
        for (; g < S.n_grp; ++g) {
            int t_lo, t_hi, cg;
            span(g, t_lo, t_hi, cg);
            for (int t = t_lo; t <= t_hi; ++t) acc += at(g, t, cg);
        }
    }
    gx[S.x_off + m] = acc;
}

hipError_t launch_reduce_x(const DScene& hs, const DGroup* d_groups, int nthreads, int taps, const float* xpart,
                           float* gx, hipStream_t st)
{
    int lg = 0;
    while ((1 << lg) < nthreads) ++lg;
    if ((1 << lg) != nthreads) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce_x, dim3((unsigned)((hs.n_in + 255) / 256)), dim3(256), 0, st, hs, d_groups, lg,
                       taps, xpart, gx);
    return hipGetLastError();
}

// --------------------------------------------------- gain and delay adjoints

// Per image sample the forward's quadratic-table sums give the filtered value
//   s = A + f B + (1-f) Bm + f (f-1)/2 C
// (A over both sides' Y, B and Bm over the near and far sides' first differences,
// C over both sides' second differences), and its derivative in mu, the exact
// derivative of the same interpolant:
//   ds/dmu = Lq (B - Bm + (f - 1/2) C)
// (the near side's fraction is f, the far side's 1 - f and runs the other way).
// Then dL/dbeta_i += gy s fs / (4 pi c D) and dL/dD = gy g (ds/dmu - s / D).
// dbar [mic][image][n_out]; gpart [image][(mic*n_tiles + tile)*waves + wave].
template <int T, int NT, int LC>
__global__ __launch_bounds__(NT) void k_adj_track(DScene S, const DImage* __restrict__ imgs,
                                                   const DGroup* __restrict__ groups,
                                                   const float4* __restrict__ table, int Lr,
                                                   const Seg* __restrict__ seg, const int32_t* __restrict__ segK,
                                                   const float* __restrict__ x, const float* __restrict__ gy,
                                                   float ghat, float* __restrict__ dbar, float* __restrict__ gpart,
                                                   int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int NG = T / 8;
    constexpr int WAVES = NT / 64;
    const int L = LC > 0 ? LC : Lr;
    const int LP = LC > 0 ? LC + 1 : Lr + 1;      // rows per quad: -1 .. L-1
    float4* tab = lds;
    const float4* tabY = tab + 1;
    const float4* tabD1 = tab + NG * LP + 1;
    const uint2* tabD2 = (const uint2*)(tab + 2 * NG * LP) + 1;
    float4* xw = lds + qtab_bytes(T, L) / 16;

    const int tile = blockIdx.x, g = blockIdx.y, mic = blockIdx.z, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const DGroup G = groups[S.grp_begin + g];
    const int n0 = tile * NT;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = NT + (G.dmax - G.dmin) + T + 8;
    for (int i = tid; i < (int)(qtab_bytes(T, L) / 16); i += NT) tab[i] = table[i];
    const float* xs = x + S.x_off;
    const int n_in = (int)S.n_in;
    for (int p = tid; p < W; p += NT) {
        const int q = ws + p;
        float4 v;
        v.x = (q >= 0 && q < n_in) ? xs[q] : 0.0f;
        v.y = (q + 1 >= 0 && q + 1 < n_in) ? xs[q + 1] : 0.0f;
        v.z = (q + 2 >= 0 && q + 2 < n_in) ? xs[q + 2] : 0.0f;
        v.w = (q + 3 >= 0 && q + 3 < n_in) ? xs[q + 3] : 0.0f;
        xw[p] = v;
    }
    __syncthreads();

    const int n = n0 + tid;
    const int n_out = (int)S.n_out;
    const bool valid = n < n_out;
    const float wy = valid ? gy[S.y_off + (int64_t)mic * S.n_out + n] : 0.0f;
    const int nc = valid ? n : n_out - 1;
    const Seg* sgm = seg + (int64_t)mic * S.seg_per_mic;
    const int32_t* sgk = segK + (int64_t)mic * S.seg_per_mic;
    const DImage* I = imgs + S.img_begin;
    const float fn = (float)nc + 0.5f;
    const float Lf = (float)L;
    float* dout = dbar + (int64_t)mic * S.n_img * S.n_out + n;
    const int64_t nrow = (int64_t)S.n_mics * S.n_tiles * WAVES;
    float* gout = gpart + ((int64_t)mic * S.n_tiles + tile) * WAVES + wave;
    int bad = 0;
    for (int ii = G.img_begin; ii < G.img_end; ++ii) {
        const DImage im = I[ii];
        const int k = min(max((int)(fn * im.invR), 0), im.n_seg - 1);
        const Seg sg = sgm[im.seg_off + k];
        const int Ks = sgk[im.seg_off + k];
        const float v = (float)(nc - __mul24(k, im.R));
        const float d = fmaf(v, fmaf(v, fmaf(v, sg.b3, sg.b2), sg.b1), sg.a0);
        const float fl = floorf(d);
        const int K = Ks + (int)fl;
        const bool act = valid && wy != 0.0f && nc - K + T / 2 - 1 >= 0 && nc - K - T / 2 < n_in;
        float E = 0.0f, Db = 0.0f;
        if (__any(act)) {
            const int p0 = nc - K - ws;
            const bool inb = p0 >= T / 2 && p0 <= W - T / 2 + 3;
            if (act && !inb) bad = 1;
            if (act && inb) {
                const float mu = d - fl;
                const float q = mu * Lf;
                const int kq = min((int)q, L - 1);
                const float f = q - (float)kq;
                const int kp = L - 1 - kq;
                const float4* xq = xw + p0;
                float A = 0.0f, B = 0.0f, Bm = 0.0f, C = 0.0f;
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    const float4 xn = xq[4 * gi];
                    const float4 Y = tabY[gi * LP + kq], D1 = tabD1[gi * LP + kq];
                    A = fmaf(Y.x, xn.x, A); B = fmaf(D1.x, xn.x, B);
                    A = fmaf(Y.y, xn.y, A); B = fmaf(D1.y, xn.y, B);
                    A = fmaf(Y.z, xn.z, A); B = fmaf(D1.z, xn.z, B);
                    A = fmaf(Y.w, xn.w, A); B = fmaf(D1.w, xn.w, B);
                    if (gi < qcorr_quads(T)) {  // further out the quadratic term is zero
                        const uint2 D2 = tabD2[gi * LP + kq];
                        C = fmaf(h16_lo(D2.x), xn.x, C); C = fmaf(h16_hi(D2.x), xn.y, C);
                        C = fmaf(h16_lo(D2.y), xn.z, C); C = fmaf(h16_hi(D2.y), xn.w, C);
                    }
                    const float4 xp = xq[-4 - 4 * gi];
                    const float4 Ym = tabY[gi * LP + kp], E1 = tabD1[gi * LP + kp];
                    A = fmaf(Ym.x, xp.w, A); Bm = fmaf(E1.x, xp.w, Bm);
                    A = fmaf(Ym.y, xp.z, A); Bm = fmaf(E1.y, xp.z, Bm);
                    A = fmaf(Ym.z, xp.y, A); Bm = fmaf(E1.z, xp.y, Bm);
                    A = fmaf(Ym.w, xp.x, A); Bm = fmaf(E1.w, xp.x, Bm);
                    if (gi < qcorr_quads(T)) {
                        const uint2 E2 = tabD2[gi * LP + kp];
                        C = fmaf(h16_lo(E2.x), xp.w, C); C = fmaf(h16_hi(E2.x), xp.z, C);
                        C = fmaf(h16_lo(E2.y), xp.y, C); C = fmaf(h16_hi(E2.y), xp.x, C);
                    }
                }
                const float s = fmaf(0.5f * f * (f - 1.0f), C, fmaf(1.0f - f, Bm, fmaf(f, B, A)));
                const float sd = Lf * fmaf(f - 0.5f, C, B - Bm);
                const float iD = __builtin_amdgcn_rcpf((float)Ks + d);
                const float gain = im.gfac * iD;
                E = wy * s * ghat * iD;
                Db = wy * gain * fmaf(-s, iD, sd);
            }
        }
        if (valid) dout[(int64_t)ii * S.n_out] = Db;
        E = wave_sum_dpp(E);
        if (lane == 0) gout[(int64_t)ii * nrow] = E;
    }
    if (bad) atomicOr(status, kStatusWindow);
}

// The same with two adjacent outputs per lane (NT lanes, 2 NT outputs per tile),
// on the forward's shared-row tap sums (pair_frame, pair_sums).  With f and h the
// near and far fractions,
//   s     = A + f B + h Bm + f (f-1)/2 C + h (h-1)/2 Cm,
//   ds/dmu = Lq (B + (f - 1/2) C - Bm - (h - 1/2) Cm)
// (h runs against mu).  gpart keeps its 2 NT / 64 slots per tile: each wave
// writes its sum to the first of its two slots and zero to the second.
template <int T, int NT, int LC>
__global__ __launch_bounds__(NT, 4) void k_adj_track2(DScene S, const DImage* __restrict__ imgs,
                                                      const DGroup* __restrict__ groups,
                                                      const float4* __restrict__ table, int Lr,
                                                      const Seg* __restrict__ seg,
                                                      const int32_t* __restrict__ segK, const float* __restrict__ x,
                                                      const float* __restrict__ gy, float ghat,
                                                      float* __restrict__ dbar, float* __restrict__ gpart,
                                                      int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int NG = T / 8;
    constexpr int TO = 2 * NT;
    constexpr int SLOTS = TO / 64;
    const int L = LC > 0 ? LC : Lr;
    const int LP = LC > 0 ? LC + 1 : Lr + 1;
    float4* tab = lds;
    const QTab tq = qtab_view<T>(tab, LP);
    float4* xw = lds + qtab_bytes(T, L) / 16;

    const int tile = blockIdx.x, g = blockIdx.y, mic = blockIdx.z, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const DGroup G = groups[S.grp_begin + g];
    const int n0 = tile * TO;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = TO + (G.dmax - G.dmin) + T + 8;
    const int n_in = (int)S.n_in;
    const int half = split_half(W);
    load_qtab<T>(table, tab, L, NT);
    stage_window_split(x + S.x_off, n_in, ws, W, xw, NT);
    __syncthreads();

    const int n_out = (int)S.n_out;
    const int n = n0 + 2 * tid;
    const bool ok0 = n < n_out, ok1 = n + 1 < n_out;
    const float* gyc = gy + S.y_off + (int64_t)mic * S.n_out;
    const float wy0 = ok0 ? gyc[n] : 0.0f, wy1 = ok1 ? gyc[n + 1] : 0.0f;
    const int nc = ok0 ? n : n_out - 1;           // lanes past the end follow the last output
    const Seg* sgm = seg + (int64_t)mic * S.seg_per_mic;
    const int32_t* sgk = segK + (int64_t)mic * S.seg_per_mic;
    const DImage* I = imgs + S.img_begin;
    const float fn = (float)nc + 0.5f;
    const float Lf = (float)L;
    float* dout = dbar + (int64_t)mic * S.n_img * S.n_out + n;
    const int64_t nrow = (int64_t)S.n_mics * S.n_tiles * SLOTS;
    float* gout = gpart + ((int64_t)mic * S.n_tiles + tile) * SLOTS + 2 * wave;
    int bad = 0;
    for (int ii = G.img_begin; ii < G.img_end; ++ii) {
        const DImage im = I[ii];
        float d0, d1;
        int K0s, K1s;
        if (im.R == 1) {
            const int k0 = min(nc, im.n_seg - 1), k1 = min(nc + 1, im.n_seg - 1);
            d0 = sgm[im.seg_off + k0].a0;
            d1 = sgm[im.seg_off + k1].a0;
            K0s = sgk[im.seg_off + k0];
            K1s = sgk[im.seg_off + k1];
        } else {
            const int k = min(max((int)(fn * im.invR), 0), im.n_seg - 1);
            const Seg sg = sgm[im.seg_off + k];
            K0s = K1s = sgk[im.seg_off + k];
            const float v = (float)(nc - __mul24(k, im.R)), v1 = v + 1.0f;
            d0 = fmaf(v, fmaf(v, fmaf(v, sg.b3, sg.b2), sg.b1), sg.a0);
            d1 = fmaf(v1, fmaf(v1, fmaf(v1, sg.b3, sg.b2), sg.b1), sg.a0);
        }
        const PairFrame fr = pair_frame(d0, K0s, d1, K1s, L, Lf);
        const int K = fr.K;
        const bool act = (wy0 != 0.0f || wy1 != 0.0f) && nc - K + T / 2 >= 0 && nc - K - T / 2 < n_in;
        float E = 0.0f, Db0 = 0.0f, Db1 = 0.0f;
        if (__any(act)) {
            const int p0 = nc - K - ws;
            const bool inb = p0 >= T / 2 && p0 <= W - 1 - T / 2;
            if (act && !inb) bad = 1;
            if (act && inb) {
                PairSums ps;
                pair_sums<NG>(tq, LP, fr.kq, fr.kp, split_at(xw, half, p0), ps);
                const float f0 = fr.q0 - (float)fr.kq, f1 = fr.q1 - (float)fr.kq;
                const float h0 = (Lf - fr.q0) - (float)fr.kp, h1 = (Lf - fr.q1) - (float)fr.kp;
                const float s0 =
                    fmaf(qweight(h0), ps.Cm0, fmaf(qweight(f0), ps.C0, fmaf(h0, ps.Bm0, fmaf(f0, ps.B0, ps.A0))));
                const float s1 =
                    fmaf(qweight(h1), ps.Cm1, fmaf(qweight(f1), ps.C1, fmaf(h1, ps.Bm1, fmaf(f1, ps.B1, ps.A1))));
                const float sd0 = Lf * (fmaf(f0 - 0.5f, ps.C0, ps.B0) - fmaf(h0 - 0.5f, ps.Cm0, ps.Bm0));
                const float sd1 = Lf * (fmaf(f1 - 0.5f, ps.C1, ps.B1) - fmaf(h1 - 0.5f, ps.Cm1, ps.Bm1));
                const float iD0 = __builtin_amdgcn_rcpf((float)K0s + d0);
                const float iD1 = __builtin_amdgcn_rcpf((float)K1s + d1);
                E = ghat * fmaf(wy0 * s0, iD0, wy1 * s1 * iD1);
                Db0 = wy0 * im.gfac * iD0 * fmaf(-s0, iD0, sd0);
                Db1 = wy1 * im.gfac * iD1 * fmaf(-s1, iD1, sd1);
            }
        }
        if (ok0) dout[(int64_t)ii * S.n_out] = Db0;
        if (ok1) dout[(int64_t)ii * S.n_out + 1] = Db1;
        E = wave_sum_dpp(E);
        if (lane == 0) {
            gout[(int64_t)ii * nrow] = E;
            gout[(int64_t)ii * nrow + 1] = 0.0f;
        }
    }
    if (bad) atomicOr(status, kStatusWindow);
}

template <int T, int TO, int RB>
static hipError_t launch_adj_track_t(const DScene& hs, const DImage* d_imgs, const DGroup* d_groups,
                                     const float4* d_qtable, int Lq, const Seg* seg, const int32_t* segK,
                                     const float* x, const float* gy, float ghat, float* dbar, float* gpart,
                                     int32_t* d_status, hipStream_t st)
{
    constexpr int NT = TO / RB;
    const size_t lds = adj_track_lds_bytes(T, Lq, hs.window);
    decltype(&k_adj_track<T, NT, 0>) kern;
    if constexpr (RB == 2)
        kern = Lq == 128 ? k_adj_track2<T, NT, 128> : k_adj_track2<T, NT, 0>;
    else
        kern = Lq == 128 ? k_adj_track<T, NT, 128> : k_adj_track<T, NT, 0>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)hs.n_tiles, (unsigned)hs.n_grp, (unsigned)hs.n_mics);
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, hs, d_imgs, d_groups, d_qtable, Lq, seg, segK, x, gy, ghat,
                       dbar, gpart, d_status);
    return hipGetLastError();
}

hipError_t launch_adj_track(int taps, int nthreads, int rb, const DScene& hs, const DImage* d_imgs,
                            const DGroup* d_groups, const float4* d_qtable, int Lq, const Seg* seg,
                            const int32_t* segK, const float* x, const float* gy, float ghat, float* dbar,
                            float* gpart, int32_t* d_status, hipStream_t st)
{
#define MSIM_ADJT_CASE(TT, NN, RR)                                                                             \
    if (taps == TT && nthreads == NN && rb == RR)                                                             \
        return launch_adj_track_t<TT, NN, RR>(hs, d_imgs, d_groups, d_qtable, Lq, seg, segK, x, gy, ghat, dbar, \
                                              gpart, d_status, st);
#define MSIM_ADJT_TAPS(TT)                                                                                     \
    MSIM_ADJT_CASE(TT, 512, 1) MSIM_ADJT_CASE(TT, 1024, 1) MSIM_ADJT_CASE(TT, 512, 2) MSIM_ADJT_CASE(TT, 1024, 2)
    MSIM_ADJT_TAPS(32)
    MSIM_ADJT_TAPS(64)
    MSIM_ADJT_TAPS(96)
    MSIM_ADJT_TAPS(128)
#undef MSIM_ADJT_TAPS
#undef MSIM_ADJT_CASE
    return hipErrorInvalidValue;
}

// ------------------------------------------- Catmull-Rom transpose, retarded delay

// Per (mic, segment): the segment's outputs n = kR + v weight the grid delays
// D_{k-1..k+2} by the Catmull-Rom basis at u = v/R; sum dL/dD(n) times each
// weight.  One block per run of seg_adj_block_segs(R) segments of one image:
// the run's outputs are loaded coalesced into LDS (segment stride R+1, so the
// per-segment reads below fall in distinct banks), then TPS consecutive threads
// per segment (a power of two, as many as the block holds, at most 64) each sum
// every TPS-th output of it, and the TPS partial sums are combined in a fixed
// order within the wave.
__global__ __launch_bounds__(kSegAdjThreads) void k_seg_adj(DScene S, const DImage* __restrict__ imgs,
                                                            const float* __restrict__ dbar,
                                                            float4* __restrict__ dseg)
{
    __shared__ float st[kSegAdjStage + kSegAdjStage / 16 + kSegAdjThreads];
    const int64_t bid = blockIdx.x;
    const int mic = (int)(bid / S.sadj_per_mic);
    const int ridx = (int)(bid - (int64_t)mic * S.sadj_per_mic);
    const DImage* I = imgs + S.img_begin;
    int lo = 0, hi = S.n_img - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (I[mid].sadj_off <= ridx) lo = mid; else hi = mid - 1;
    }
    const DImage im = I[lo];
    const int R = im.R;
    const int per = seg_adj_block_segs(R);
    const int k0 = (ridx - im.sadj_off) * per;
    const int nseg = min(per, im.n_seg - k0);
    const int n0 = k0 * R;
    const int nv = min(nseg * R, (int)S.n_out - n0);       // outputs of this run
    const float* Db = dbar + ((int64_t)mic * S.n_img + lo) * S.n_out + n0;
    // i / R as umulhi(i, ceil(2^32 / R)) for R >= 2 (the constant fits 32 bits there):
    // exact for i < 2^32 / R (i < kSegAdjStage here); R = 1 is i itself
    const uint32_t rmag = R > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)R - 1) / (uint64_t)R) : 0u;
    // eight independent loads in flight per thread
    for (int i0 = threadIdx.x; i0 < nseg * R; i0 += 8 * kSegAdjThreads) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * kSegAdjThreads;
            t[u] = i < nv ? Db[i] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * kSegAdjThreads;
            if (i < nseg * R) {
                const int kk = R > 1 ? (int)__umulhi((uint32_t)i, rmag) : i;     // segment of i
                st[i + kk] = t[u];                                    // row kk, column i - kk R
            }
        }
    }
    __syncthreads();
    int tps = 1;
    while (tps < 64 && tps * 2 * per <= kSegAdjThreads && tps * 2 <= R) tps *= 2;
    const int kk = threadIdx.x / tps, j = threadIdx.x % tps;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    if (kk < nseg) {
        const float* row = st + kk * (R + 1);
        const float iR = 1.0f / (float)R;
        for (int v = j; v < R; v += tps) {
            const float d = row[v];
            const float u = (float)v * iR;
            s0 = fmaf(d, 0.5f * u * fmaf(u, 2.0f - u, -1.0f), s0);
            s1 = fmaf(d, fmaf(u * u, fmaf(1.5f, u, -2.5f), 1.0f), s1);
            s2 = fmaf(d, 0.5f * u * fmaf(u, fmaf(-3.0f, u, 4.0f), 1.0f), s2);
            s3 = fmaf(d, 0.5f * u * u * (u - 1.0f), s3);
        }
    }
    // groups of tps lanes are aligned within a wave: halve them in a fixed order
    for (int o = tps / 2; o > 0; o >>= 1) {
        s0 += __shfl_down(s0, o, 64);
        s1 += __shfl_down(s1, o, 64);
        s2 += __shfl_down(s2, o, 64);
        s3 += __shfl_down(s3, o, 64);
    }
    if (kk < nseg && j == 0)
        dseg[(int64_t)mic * S.seg_per_mic + im.seg_off + k0 + kk] = make_float4(s0, s1, s2, s3);
}

// Per (mic, grid point k of an image): dL/dtau_k = fs * sum of the segment
// weights that reference D_k; then dtau_k / d p(t_e) for the source position
// at the emission time t_e = t_k - tau_k:
//   retarded:       S^T u / (c + u . S p'(t_e)),  u = unit vector mic -> image
//   instantaneous:  S^T u / c
// and the knot a of t_e's path segment with the weight lam of knot a+1.
__global__ __launch_bounds__(256) void k_grid_adj(const DScene* __restrict__ scenes, int scene,
                                                  const DImage* __restrict__ imgs, const double* __restrict__ knots,
                                                  const double* __restrict__ mics, const double* __restrict__ grid,
                                                  const float4* __restrict__ dseg, double4* __restrict__ pgc,
                                                  int32_t* __restrict__ pga, double c, double fs, int model)
{
    const DScene& S = scenes[scene];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_mic = S.seg_per_mic + 3 * (int64_t)S.n_img;
    if (gid >= per_mic * S.n_mics) return;
    const int mic = S.n_mics == 1 ? 0 : (int)(gid / per_mic);
    const int64_t idx = gid - (int64_t)mic * per_mic;
    const DImage* I = imgs + S.img_begin;
    // the lanes of a wave hold consecutive grid points: when they share one mic, one
    // search for the first active lane's point (wave-uniform), then each lane steps
    // over the few images that end before its own point
    int ii;
    const int mic0 = __builtin_amdgcn_readfirstlane(mic);
    if (__all(mic == mic0)) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)idx);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)idx >> 32));
        ii = owner(I, S.n_img, (int64_t)(((uint64_t)hi << 32) | lo), 3);
        while (ii + 1 < S.n_img && (int64_t)I[ii + 1].seg_off + 3 * (int64_t)(ii + 1) <= idx) ++ii;
    } else {
        ii = owner(I, S.n_img, idx, 3);
    }
    const DImage im = I[ii];
    const int64_t k = idx - ((int64_t)im.seg_off + 3 * (int64_t)ii) - 1;
    const float4* ds = dseg + (int64_t)mic * S.seg_per_mic + im.seg_off;
    double dD = 0.0;
    // segment s uses grid point k with basis index q = k - s + 1
    for (int q = 0; q < 4; ++q) {
        const int64_t s = k + 1 - q;
        if (s < 0 || s >= im.n_seg) continue;
        const float4 w = ds[s];
        dD += (q == 0) ? w.x : (q == 1) ? w.y : (q == 2) ? w.z : w.w;
    }
    const double taubar = fs * dD;
    double4 out = make_double4(0.0, 0.0, 0.0, 0.0);
    int a = -1;
    if (S.src.kind == 0 && taubar != 0.0) {
        const double tk = (double)(k * im.R) / fs;
        const double tau = grid[gid] / fs;
        const double te = model == 0 ? tk - tau : tk;
        double q[3], r[3], v[3], lam;
        pwl_eval(S.src, knots, te, q, v, &a, &lam);        // a PWL path (kind 0)
        mic_pos(S, knots, mics, mic, tk, r);
        double e[3], d2 = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            e[ax] = image_coord(im.m[ax], S.size[ax], q[ax]) - r[ax];
            d2 += e[ax] * e[ax];
        }
        const double id = 1.0 / sqrt(d2);
        double denom = c;
        double sgn[3];
        for (int ax = 0; ax < 3; ++ax) sgn[ax] = (im.m[ax] & 1) ? -1.0 : 1.0;
        if (model == 0)
            for (int ax = 0; ax < 3; ++ax) denom += e[ax] * id * sgn[ax] * v[ax];
        const double sc = taubar * id / denom;
        out.x = sc * sgn[0] * e[0];
        out.y = sc * sgn[1] * e[1];
        out.z = sc * sgn[2] * e[2];
        out.w = lam;
    }
    pgc[gid] = out;
    pga[gid] = a;
}

hipError_t launch_adj_params(const DScene* d_scenes, int scene, const DScene& hs, const DImage* d_imgs,
                             const double* d_knots, const double* d_mics, const double* grid, const float* dbar,
                             float4* dseg, double4* pgc, int32_t* pga, double c, double fs, int delay_model,
                             int want_src, hipStream_t st)
{
    const int64_t nb = hs.sadj_per_mic * hs.n_mics;
    hipLaunchKernelGGL(k_seg_adj, dim3((unsigned)nb), dim3(kSegAdjThreads), 0, st, hs, d_imgs, dbar, dseg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !want_src) return e;
    const int64_t ng = (hs.seg_per_mic + 3 * (int64_t)hs.n_img) * hs.n_mics;
    hipLaunchKernelGGL(k_grid_adj, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, d_scenes, scene, d_imgs,
                       d_knots, d_mics, grid, dseg, pgc, pga, c, fs, delay_model);
    return hipGetLastError();
}

// ------------------------------------------------------------- reductions

constexpr int kMaxGradKnots = 32;
constexpr int kRedThreads = 256;

// Fixed-order block sum of one double per thread; every thread returns the total.
__device__ inline double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ inline double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block b of NB (4 waves): images ii = 4b + wave (+ k*4*NB), one wave per image,
// give dL/dbeta_w partials sum_i (d beta_i / d beta_w) G_i, G_i = dL/dbeta_i summed
// over its [mic][tile][wave] rows; grid points i = b*256 + t (+ k*NB*256) give
// dL/dP_a partials, accumulated in NK >= src_knots registers per axis.
// partial: [NB][6 + 3*kMaxGradKnots].
template <int NK>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(const DScene* __restrict__ scenes, int scene,
                                                                const DImage* __restrict__ imgs,
                                                                const float* __restrict__ gpart, int gstride,
                                                                const double4* __restrict__ pgc,
                                                                const int32_t* __restrict__ pga, int want_beta,
                                                                int want_src, double* __restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    const DScene& S = scenes[scene];
    const int t = threadIdx.x, b = blockIdx.x, NB = gridDim.x;
    const int wave = t >> 6, lane = t & 63;
    constexpr int WPB = kRedThreads / 64;
    const int64_t stride = (int64_t)NB * kRedThreads;
    double* out = partial + (int64_t)b * (6 + 3 * kMaxGradKnots);
    const DImage* I = imgs + S.img_begin;
    if (want_beta) {
        double bw[6] = {0, 0, 0, 0, 0, 0};
        const int64_t nrow = (int64_t)S.n_mics * gstride;
        for (int64_t ii = (int64_t)b * WPB + wave; ii < S.n_img; ii += (int64_t)NB * WPB) {
            double Gi = 0.0;
            for (int64_t r = lane; r < nrow; r += 64) Gi += gpart[ii * nrow + r];
            Gi = wave_sum_d(Gi);
            const DImage im = I[ii];
            for (int w = 0; w < 6; ++w) {
                const int h = im.hits[w];
                if (h == 0) continue;
                double d = (double)h;
                for (int r = 0; r < h - 1; ++r) d *= S.beta[w];
                for (int v = 0; v < 6; ++v) {
                    if (v == w) continue;
                    for (int r = 0; r < im.hits[v]; ++r) d *= S.beta[v];
                }
                bw[w] += d * Gi;
            }
        }
        // every lane of a wave holds the same bw; combine the waves in order
        for (int w = 0; w < 6; ++w) {
            if (lane == 0) sh[wave] = bw[w];
            __syncthreads();
            if (t == 0) {
                double v = 0.0;
                for (int k = 0; k < WPB; ++k) v += sh[k];
                out[w] = v;
            }
            __syncthreads();
        }
    }
    if (want_src && S.src_knots > 0) {
        const int nk = min(S.src_knots, NK);
        double acc[NK][3];
#pragma unroll
        for (int j = 0; j < NK; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
        const int64_t total = (S.seg_per_mic + 3 * (int64_t)S.n_img) * S.n_mics;
        // four items' loads go out together; the items are added in the plain
        // grid-stride order
        for (int64_t i0 = (int64_t)b * kRedThreads + t; i0 < total; i0 += 4 * stride) {
            int aa[4];
            double4 vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t i = i0 + u * stride;
                aa[u] = i < total ? pga[i] : -1;
                vv[u] = i < total ? pgc[i] : make_double4(0.0, 0.0, 0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int a = aa[u];
                if (a < 0) continue;
                const double4 v = vv[u];
                const double wa = 1.0 - v.w, wb = v.w;
#pragma unroll
                for (int j = 0; j < NK; ++j) {
                    const double f = (j == a) ? wa : (j == a + 1) ? wb : 0.0;
                    acc[j][0] += f * v.x;
                    acc[j][1] += f * v.y;
                    acc[j][2] += f * v.z;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            if (j >= nk) break;
            for (int ax = 0; ax < 3; ++ax) {
                const double tot = block_sum(acc[j][ax], sh);
                if (t == 0) out[6 + 3 * j + ax] = tot;
            }
        }
    }
}

// One wave per output value: the NB block partials, lane-strided, then a
// fixed butterfly.
__global__ __launch_bounds__(64) void k_reduce_final(const DScene* __restrict__ scenes, int scene, int NB,
                                                     const double* __restrict__ partial, int want_beta,
                                                     int want_src, double* __restrict__ gbeta,
                                                     double* __restrict__ gsrc)
{
    const DScene& S = scenes[scene];
    const int v = blockIdx.x, lane = threadIdx.x;
    const int row = 6 + 3 * kMaxGradKnots;
    const int nk = min(S.src_knots, kMaxGradKnots);
    const bool is_beta = v < 6;
    if (is_beta ? !want_beta : (!want_src || v - 6 >= 3 * nk)) return;
    double acc = 0.0;
    for (int b = lane; b < NB; b += 64) acc += partial[(int64_t)b * row + v];
    acc = wave_sum_d(acc);
    if (lane == 0) {
        if (is_beta) gbeta[(int64_t)scene * 6 + v] = acc;
        else gsrc[(int64_t)S.src_grad_off * 3 + (v - 6)] = acc;
    }
}

int reduce_blocks(const DScene& hs)
{
    const int64_t total = (hs.seg_per_mic + 3 * (int64_t)hs.n_img) * hs.n_mics;
    int64_t nb = (total + 8191) / 8192;
    nb = nb < 1 ? 1 : nb > 512 ? 512 : nb;
    return (int)nb;
}

size_t reduce_partial_bytes(const DScene& hs) { return (size_t)reduce_blocks(hs) * (6 + 3 * kMaxGradKnots) * 8; }

int max_grad_knots() { return kMaxGradKnots; }

hipError_t launch_reduce_params(const DScene* d_scenes, int scene, const DScene& hs, const DImage* d_imgs,
                                const float* gpart, int gpart_stride, const double4* pgc, const int32_t* pga,
                                double* partial, double* gbeta, double* gsrc, hipStream_t st)
{
    const int NB = reduce_blocks(hs);
    const int wb = gbeta != nullptr, wsrc = gsrc != nullptr && hs.src_knots > 0;
    const int nk = hs.src_knots;
    auto kern = nk <= 4 ? k_reduce_partial<4> : nk <= 8 ? k_reduce_partial<8> : nk <= 16 ? k_reduce_partial<16>
                                                                                          : k_reduce_partial<kMaxGradKnots>;
    hipLaunchKernelGGL(kern, dim3(NB), dim3(kRedThreads), 0, st, d_scenes, scene, d_imgs, gpart, gpart_stride, pgc,
                       pga, wb, wsrc, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(6 + 3 * kMaxGradKnots), dim3(64), 0, st, d_scenes, scene, NB, partial,
                       wb, wsrc, gbeta, gsrc);
    return hipGetLastError();
}

}  // namespace msim
