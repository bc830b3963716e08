// gfx950 adjoint (reverse-mode) kernels of the moving image-source synthesis.
//
// The forward map is y_c[n] = sum_i g_i(n) s_i(n),  s_i(n) = sum_j h(j - mu_i(n)) x[n - K_i(n) - j],
// with D_i(n) = K_i(n) + mu_i(n) the Catmull-Rom interpolated delay and
// g_i(n) = beta_i fs / (4 pi c D_i(n))  (Eq. 2 / Eq. 8, Sec. II-B, Sec. II-C-3),
// with h the forward's quadratic interpolation of the Kaiser-windowed sinc.  Given gy = dL/dy:
//   k_adjx     : dL/dx[m] = sum_{c,i,n} gy_c[n] g_i(n) h(n - D_i(n) - m), the transpose
//                time-varying fractional delay, accumulated per wave in a shifting
//                register accumulator, per delay group in LDS, per work item
//                (mic, output tile, supergroup) in a window of source positions,
//                and gathered over the windows in a fixed order (k_reduce_x).
//   k_adjp     : per image sample, s and ds/dmu from the forward's table sums:
//                dL/dbeta_i += gy s fs / (4 pi c D),  dL/dD_i(n) = gy g (ds/dmu - s / D),
//                then, inside the tile, the transpose of the Catmull-Rom
//                interpolation (dL/dD on the delay grid), the implicit-function
//                derivative of the retarded delay c tau = |S_i p(t - tau) + O_i - r(t)|
//                with respect to the source position at the emission time, split
//                onto the two knots of its path segment, and dL/dbeta_w through
//                beta_i = prod_w beta_w^hits_w: one row of parameter partials per
//                work item.
//   k_reduce_rows : the rows of each scene summed in a fixed order.
// Every kernel solves its delay tracks per tile (tile_tracks): nothing is stored
// at the audio rate, and every sum runs in a fixed order.
#include "msim_device.h"
#include "msim_internal.h"
#include "msim_pair.h"

#include <hip/hip_runtime.h>

namespace msim {

// ------------------------------------------------------------------ sizes

// The transpose reads the forward's quadratic table rearranged tap-major: three
// arrays Y, D1, D2 of [T/2][Lq] floats; then each of its kAdjThreads/64 waves
// owns a window of (window - tile + 64 h) source positions (its 64 h outputs' taps
// under every delay of the group, h = tile / kAdjThreads); then the group's slot
// offsets.
size_t adj_x_lds_bytes(int taps, int Lq, int window, int tile)
{
    const int h = tile / kAdjThreads;
    return (size_t)3 * (taps / 2) * (size_t)Lq * sizeof(float) +
           (size_t)(kAdjThreads / 64) * (size_t)(window - tile + 64 * h) * sizeof(float) + kLscBytes;
}

// Image descriptors staged in LDS at a time by the table form's gain/delay
// kernel at two outputs per lane (one chunk covers a delay group at the table
// form's default cap of 96 images).
constexpr int kAdjDescChunk = 96;

// The gain/delay kernels: the forward's LDS, then the slot offsets, the
// parameter accumulators and a chunk of image descriptors.
size_t adj_track_lds_bytes(int taps, int Lq, int window)
{
    return qtab_bytes(taps, Lq) + (size_t)(window + 1) * sizeof(float4) + kLscBytes + kParamLdsBytes +
           (size_t)kAdjDescChunk * 2 * sizeof(int4);
}

// ------------------------------------------------------------ transpose delay

// One delay group of the transpose, table form, on the tile [n0, n0 + NT) of one
// mic (one output per lane):
//   dL/dx[m] += w h_q(j - mu)  for every image sample (w = gy g) and tap j, m = n - K - j,
// with h_q the forward's quadratic interpolation of h, so this is its exact transpose.
//
// Systolic form.  A wave holds 64 consecutive outputs of one image; their integer
// delays differ by at most one (K_ref = the smallest, dK = K - K_ref in {0, 1}),
// so at step s (s = 0 .. T) lane l's tap lands on relative source position
// l + s - T/2 - 1 (relative to n0 - K_ref).  The wave keeps one register
// accumulator per lane for that position; between steps it moves one lane down
// (DPP wave_shl:1, fused into the add), the value leaving lane 0 is complete and
// is parked in a second register.  Each image's 64 + T positions then reach the
// wave's LDS window with two read-add-writes per lane.  Waves whose integer delay
// spans more than one sample (relative speeds above ~fs/64 samples per sample)
// take a per-tap scatter instead.  The wave windows are then summed in wave order
// and added to the item's window xo (global, this workgroup's alone; position
// p of xo is source position xws + p).
template <int T, int TILE, int LQC>
__device__ inline void adjx_group(const DScene& S, const DGroup& G, int n0, int mic, Slot sl,
                                  const DImage* __restrict__ I, const PermEntry* __restrict__ perm, const float* tY,
                                  const float* tD1, const float* tD2, int Lr, float* wbase, int Wstride,
                                  const float* __restrict__ gyc, float* xo, int xws, int& bad)
{
    constexpr int NT = kAdjThreads;
    constexpr int WAVES = NT / 64;
    constexpr int HV = TILE / NT;                       // 64-output blocks per wave
    constexpr int H = T / 2;
    const int LQ = LQC > 0 ? LQC : Lr;
    auto wt = [&](int i, float a, float b, float c) { return fmaf(a, tY[i], fmaf(b, tD1[i], c * tD2[i])); };
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = TILE + (G.dmax - G.dmin) + T + 8;     // the tile's window
    const int Ww = W - TILE + 64 * HV;                  // per-wave window used by this group
    for (int p = tid; p < WAVES * Wstride; p += NT) wbase[p] = 0.0f;
    __syncthreads();

    // read-add-writes of successive images stay in program order (lanes of one
    // wave may touch the same position for different images)
    volatile float* xb = wbase + wave * Wstride;        // covers source positions ws + 64 HV wave + [0, Ww)
    const int wsw = ws + 64 * HV * wave;
    const int n_out = (int)S.n_out;
    const float LQf = (float)LQ;
    const int n_in = (int)S.n_in;
    for (int hv = 0; hv < HV; ++hv) {
    const int n0w = n0 + 64 * (HV * wave + hv);
    const int n = n0w + lane;
    const bool valid = n < n_out;
    const int nc = valid ? n : n_out - 1;
    const float wy = valid ? gyc[n] : 0.0f;
    int cR = 0, cl = 0;
    float cv = 0.0f;
    for (int ii = G.img_begin; ii < G.img_end; ++ii) {
        const DImage im = perm_image(I, perm, ii);
        if (im.R != cR) {
            cR = im.R;
            const int k = div_exact(nc, cR, im.invR);
            cl = k - div_exact(n0, cR, im.invR);
            cv = (float)(nc - k * cR);
        }
        const Seg sg = sl.seg[im.loc + cl];
        const int Ks = sl.K[im.loc + cl];
        const float d = fmaf(cv, fmaf(cv, fmaf(cv, sg.b3, sg.b2), sg.b1), sg.a0);
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
    }
    __syncthreads();
    // tile window position p = wave window position p - 64 HV w, summed in wave
    // order, added to the item's window (the groups in order)
    const int off = ws - xws;
    for (int p = tid; p < W; p += NT) {
        float a = 0.0f;
        for (int w2 = 0; w2 < WAVES; ++w2) {
            const int pw = p - 64 * HV * w2;
            if (pw >= 0 && pw < Ww) a += wbase[w2 * Wstride + pw];
        }
        xo[off + p] += a;
    }
    __syncthreads();
}

// Delay bounds [dmin, dmax] of the groups of a supergroup.
__device__ inline int2 sg_bounds(const DGroup* __restrict__ groups, const DBlock& B, int n_sg, int sg)
{
    const int gb = sg_begin(B.n_grp, n_sg, sg), ge = sg_begin(B.n_grp, n_sg, sg + 1);
    int lo = INT32_MAX, hi = INT32_MIN;
    for (int g = gb; g < ge; ++g) {
        lo = min(lo, groups[B.grp_begin + g].dmin);
        hi = max(hi, groups[B.grp_begin + g].dmax);
    }
    return make_int2(lo, hi);
}

// dL/dx partial windows, persistent over work items (scene, mic, tile,
// supergroup): window (mic, sg, tile) of a scene covers source positions
// [tile TILE - c, tile TILE - c + W), c = dmax + T/2 + 4, W = TILE + dmax - dmin + T + 8
// with [dmin, dmax] the supergroup's delay bounds in the tile's block.
// kAdjThreads lanes; each wave takes TILE / kAdjThreads consecutive blocks of 64
// outputs (the transpose's register accumulators and parked departures need the
// kernel within its register budget at this size).
template <int T, int TILE, int LQC>
__global__ __launch_bounds__(kAdjThreads) void k_adjx(PlanView pv, const float* __restrict__ atab, int Lr,
                                                      const WorkItem* __restrict__ items, int n_items,
                                                      int32_t* __restrict__ ticket, TrackArgs ta, int window,
                                                      const float* __restrict__ gy, float* __restrict__ xwin,
                                                      int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int NT = kAdjThreads;
    constexpr int H = T / 2;
    const int LQ = LQC > 0 ? LQC : Lr;
    float* tY = (float*)lds;
    float* tD1 = tY + H * LQ;
    float* tD2 = tD1 + H * LQ;
    float* wbase = tD2 + H * LQ;
    const int Wstride = window - TILE + 64 * (TILE / NT);
    int* lsc = (int*)(wbase + (NT / 64) * Wstride);
    for (int i = threadIdx.x; i < 3 * H * LQ; i += NT) tY[i] = atab[i];
    const Slot sl = slot_at(ta.slots, ta.slot_bytes, ta.slot_segs, blockIdx.x);
    for_each_item(ticket, n_items, [&](int it) {
        const WorkItem w = items[it];
        const DScene& S = pv.scenes[w.scene];
        const DImage* I = pv.imgs + S.img_begin;
        const DBlock B = pv.blocks[S.blk_begin + w.tile / S.blk_tiles];
        const int n0 = w.tile * TILE;
        const int n_out = (int)S.n_out;
        const int n_hi = min(n0 + TILE, n_out);
        const int2 bd = sg_bounds(pv.groups, B, S.n_sg, w.sg);
        const int xws = n0 - bd.y - T / 2 - 4;
        const int Wi = TILE + (bd.y - bd.x) + T + 8;
        float* xo = xwin + S.xw_base + (((int64_t)w.mic * S.n_sg + w.sg) * S.n_tiles + w.tile) * S.xw_stride;
        for (int p = threadIdx.x; p < Wi; p += NT) xo[p] = 0.0f;
        const float* gyc = gy + S.y_off + (int64_t)w.mic * S.n_out;
        const int gb = sg_begin(B.n_grp, S.n_sg, w.sg), ge = sg_begin(B.n_grp, S.n_sg, w.sg + 1);
        int bad = 0;
        for (int g = gb; g < ge; ++g) {
            const DGroup G = pv.groups[B.grp_begin + g];
            tile_tracks<NT>(S, w.mic, I, pv.perm, G.img_begin, G.img_end, n0, n_hi,
                            group_span(TILE, G.dmin, G.dmax), sl, lsc, ta.knots, ta.mics, ta.c, ta.fs, ta.model);
            adjx_group<T, TILE, LQC>(S, G, n0, w.mic, sl, I, pv.perm, tY, tD1, tD2, LQ, wbase, Wstride, gyc, xo,
                                     xws, bad);
        }
        if (bad) atomicOr(status, kStatusWindow);
    });
}

template <int T, int TILE>
static hipError_t launch_adjx_t(int n_wg, int window, const PlanView& pv, const float* d_atab, int Lq,
                                const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta,
                                const float* gy, float* xwin, int32_t* d_status, hipStream_t st)
{
    const size_t lds = adj_x_lds_bytes(T, Lq, window, TILE);
    auto kern = Lq == 128 ? k_adjx<T, TILE, 128> : k_adjx<T, TILE, 0>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(64), 0, st, ticket);
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(kAdjThreads), lds, st, pv, d_atab, Lq, items, n_items, ticket,
                       ta, window, gy, xwin, d_status);
    return hipGetLastError();
}

hipError_t launch_adjx(int taps, int tile, int n_wg, int window, const PlanView& pv, const float* d_atab, int Lq,
                       const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* gy,
                       float* xwin, int32_t* d_status, hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
#define MSIM_ADJX_CASE(TT, NN)                                                                                 \
    if (taps == TT && tile == NN)                                                                              \
        return launch_adjx_t<TT, NN>(n_wg, window, pv, d_atab, Lq, items, n_items, ticket, ta, gy, xwin,       \
                                     d_status, st);
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

// Gathers the partial windows that cover each input sample of every scene, in a
// fixed order (mic, supergroup, tile).  prefix[s]: first input of scene s.
__global__ __launch_bounds__(256) void k_reduce_x(PlanView pv, int n_scenes, const int64_t* __restrict__ prefix,
                                                  int64_t x_total, int NT, int T, const int2* __restrict__ sgb,
                                                  const float* __restrict__ xwin, float* __restrict__ gx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= x_total) return;
    const int s = scene_of(prefix, n_scenes, i);
    const DScene& S = pv.scenes[s];
    const int m = (int)(i - prefix[s]);
    // tiles whose windows can hold m: tile NT in [m - T/2 - 4 + dmin_lo - NT, m + dmax_hi + T/2 + 4]
    const int t_lo = max(0, (m - T / 2 - 8 + S.dlo_all - NT) / NT);
    const int t_hi = min(S.n_tiles - 1, (m + S.dhi_all + T / 2 + 4) / NT);
    float acc = 0.0f;
    for (int mic = 0; mic < S.n_mics; ++mic)
        for (int sg = 0; sg < S.n_sg; ++sg)
            for (int t = t_lo; t <= t_hi; ++t) {
                const int2 bd = sgb[(S.blk_begin + t / S.blk_tiles) * S.sgb_stride + sg];
                const int p = m - (t * NT - bd.y - T / 2 - 4);
                const int Wi = NT + (bd.y - bd.x) + T + 8;
                if (p >= 0 && p < Wi)
                    acc += xwin[S.xw_base + (((int64_t)mic * S.n_sg + sg) * S.n_tiles + t) * S.xw_stride + p];
            }
    gx[S.x_off + m] = acc;
}

hipError_t launch_reduce_x(const PlanView& pv, int n_scenes, const int64_t* d_x_prefix, int64_t x_total, int nthreads,
                           int taps, const int2* d_sgb, const float* xwin, float* gx, hipStream_t st)
{
    if (x_total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_x, dim3((unsigned)((x_total + 255) / 256)), dim3(256), 0, st, pv, n_scenes,
                       d_x_prefix, x_total, nthreads, taps, d_sgb, xwin, gx);
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
// One output per lane; dL/dD goes into the image's Catmull-Rom partials in the
// slot (cr_partials), the wave sums of dL/dbeta_i to esum[(ii - ib) WAVES + wave].
// Ends with a barrier.
template <int T, int TILE, int LC>
__device__ inline void gd_group(const DScene& S, const DGroup& G, int n0, Slot sl, AdjSlot as,
                                const DImage* __restrict__ I, const PermEntry* __restrict__ perm, const float4* tab,
                                float4* xw, int Lr, const float* __restrict__ x, const float* __restrict__ gyc,
                                float ghat, int& bad)
{
    constexpr int NG = T / 8;
    constexpr int NT = kAdjThreads;
    constexpr int WAVES = NT / 64;
    constexpr int HV = TILE / NT;
    const int L = LC > 0 ? LC : Lr;
    const int LP = LC > 0 ? LC + 1 : Lr + 1;
    const QTab tq = qtab_view<T>(tab, LP);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = TILE + (G.dmax - G.dmin) + T + 8;
    const int n_in = (int)S.n_in;
    stage_window(x + S.x_off, n_in, ws, W, xw, NT);
    __syncthreads();
    const int n_out = (int)S.n_out;
    const float Lf = (float)L;
    for (int hv = 0; hv < HV; ++hv) {
    const int n = n0 + hv * NT + tid;
    const bool valid = n < n_out;
    const int nc = valid ? n : n_out - 1;
    const float wy = valid ? gyc[n] : 0.0f;
    int cR = 0, cl = 0;
    float cv = 0.0f;
    CrLane<1> crl;
    for (int ii = G.img_begin; ii < G.img_end; ++ii) {
        const DImage im = perm_image(I, perm, ii);
        if (im.R != cR) {
            cR = im.R;
            const int k = div_exact(nc, cR, im.invR);
            const int k_lo = div_exact(n0, cR, im.invR);
            cl = k - k_lo;
            cv = (float)(nc - k * cR);
            cr_lane<1>(crl, n, nc, n_out, cR, im.invR, k, k_lo, hv * WAVES + wave, lane);
        }
        const Seg sg = sl.seg[im.loc + cl];
        const int Ks = sl.K[im.loc + cl];
        const float d = fmaf(cv, fmaf(cv, fmaf(cv, sg.b3, sg.b2), sg.b1), sg.a0);
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
                    const float4 Y = tq.Y[gi * LP + kq], D1 = tq.D1[gi * LP + kq];
                    A = fmaf(Y.x, xn.x, A); B = fmaf(D1.x, xn.x, B);
                    A = fmaf(Y.y, xn.y, A); B = fmaf(D1.y, xn.y, B);
                    A = fmaf(Y.z, xn.z, A); B = fmaf(D1.z, xn.z, B);
                    A = fmaf(Y.w, xn.w, A); B = fmaf(D1.w, xn.w, B);
                    if (gi < qcorr_quads(T)) {  // further out the quadratic term is zero
                        const uint2 D2 = tq.D2[gi * LP + kq];
                        C = fmaf(h16_lo(D2.x), xn.x, C); C = fmaf(h16_hi(D2.x), xn.y, C);
                        C = fmaf(h16_lo(D2.y), xn.z, C); C = fmaf(h16_hi(D2.y), xn.w, C);
                    }
                    const float4 xp = xq[-4 - 4 * gi];
                    const float4 Ym = tq.Y[gi * LP + kp], E1 = tq.D1[gi * LP + kp];
                    A = fmaf(Ym.x, xp.w, A); Bm = fmaf(E1.x, xp.w, Bm);
                    A = fmaf(Ym.y, xp.z, A); Bm = fmaf(E1.y, xp.z, Bm);
                    A = fmaf(Ym.z, xp.y, A); Bm = fmaf(E1.z, xp.y, Bm);
                    A = fmaf(Ym.w, xp.x, A); Bm = fmaf(E1.w, xp.x, Bm);
                    if (gi < qcorr_quads(T)) {
                        const uint2 E2 = tq.D2[gi * LP + kp];
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
        const int li = ii - G.img_begin;
        const float db[1] = {valid ? Db : 0.0f};
        cr_partials<1>(crl, db, as.dpart + im.loc + li * (TILE / 64));
        E = wave_sum_dpp(E);
        if (lane == 0) as.esum[li * (TILE / 64) + hv * WAVES + wave] = E;
    }
    }
    __syncthreads();
}

// The same with two adjacent outputs per lane (NT lanes, 2 NT outputs per tile),
// on the forward's shared-row tap sums (pair_frame, pair_sums).  With f and h the
// near and far fractions,
//   s     = A + f B + h Bm + f (f-1)/2 C + h (h-1)/2 Cm,
//   ds/dmu = Lq (B + (f - 1/2) C - Bm - (h - 1/2) Cm)
// (h runs against mu).  Ends with a barrier.
template <int T, int NT, int LC>
__device__ inline void gd_group2(const DScene& S, const DGroup& G, int n0, Slot sl, AdjSlot as,
                                 const DImage* __restrict__ I, const PermEntry* __restrict__ perm, const float4* tab,
                                 float4* xw, int4* dsc, int Lr, const float* __restrict__ x, float wy0, float wy1,
                                 float ghat, int& bad)
{
    constexpr int NG = T / 8;
    constexpr int TO = 2 * NT;
    const int L = LC > 0 ? LC : Lr;
    const int LP = LC > 0 ? LC + 1 : Lr + 1;
    const QTab tq = qtab_view<T>(tab, LP);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = TO + (G.dmax - G.dmin) + T + 8;
    const int n_in = (int)S.n_in;
    const int half = split_half(W);
    stage_window_split(x + S.x_off, n_in, ws, W, xw, NT);
    const int n_out = (int)S.n_out;
    const int n = n0 + 2 * tid;
    const bool ok0 = n < n_out, ok1 = n + 1 < n_out;
    const int nc = ok0 ? n : n_out - 1;           // lanes past the end follow the last output
    const float Lf = (float)L;
    // the group's image descriptors a chunk at a time in LDS (slot offset, R, gain
    // factor, 1/R; k_lo = n0 / R), read there as wave-uniform values
    for (int cb = G.img_begin; cb < G.img_end; cb += kAdjDescChunk) {
    const int nch = min(kAdjDescChunk, G.img_end - cb);
    __syncthreads();                 // window staged; the previous chunk's descriptors read
    for (int i = tid; i < nch; i += NT) {
        const PermEntry e = perm[cb + i];
        const DImage& im = I[e.img];
        dsc[2 * i] = make_int4(e.loc, im.R, __float_as_int(im.gfac), __float_as_int(im.invR));
        dsc[2 * i + 1] = make_int4(div_exact(n0, im.R, im.invR), 0, 0, 0);
    }
    __syncthreads();
    int cR = 0, c0 = 0, c1 = 0;
    float cv = 0.0f;
    CrLane<2> crl;
    for (int j = 0; j < nch; ++j) {
        const int4 dd = dsc[2 * j];
        const int loc = __builtin_amdgcn_readfirstlane(dd.x);
        const int R = __builtin_amdgcn_readfirstlane(dd.y);
        const float gfac = __int_as_float(dd.z), invR = __int_as_float(dd.w);
        if (R != cR) {
            cR = R;
            if (cR == 1) {
                c0 = nc - n0;
                c1 = min(nc + 1, n_out - 1) - n0;
                cv = 0.0f;
                cr_lane<2>(crl, n, nc, n_out, 1, 1.0f, nc, n0, wave, lane);
            } else {
                const int k0 = div_exact(nc, cR, invR);
                const int k_lo = __builtin_amdgcn_readfirstlane(dsc[2 * j + 1].x);
                c0 = c1 = k0 - k_lo;
                cv = (float)(nc - k0 * cR);
                cr_lane<2>(crl, n, nc, n_out, cR, invR, k0, k_lo, wave, lane);
            }
        }
        const Seg sg = ld_at(sl.seg, (uint32_t)(loc + c0));
        const float a1 = ld_at(sl.seg, (uint32_t)(loc + c1)).a0;
        const int K0s = ld_at(sl.K, (uint32_t)(loc + c0)), K1s = ld_at(sl.K, (uint32_t)(loc + c1));
        const float d0 = fmaf(cv, fmaf(cv, fmaf(cv, sg.b3, sg.b2), sg.b1), sg.a0);
        const float v1 = cv + 1.0f;
        const float d1 = R == 1 ? a1 : fmaf(v1, fmaf(v1, fmaf(v1, sg.b3, sg.b2), sg.b1), sg.a0);
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
                Db0 = wy0 * gfac * iD0 * fmaf(-s0, iD0, sd0);
                Db1 = wy1 * gfac * iD1 * fmaf(-s1, iD1, sd1);
            }
        }
        const int li = cb + j - G.img_begin;
        const float db[2] = {ok0 ? Db0 : 0.0f, ok1 ? Db1 : 0.0f};
        cr_partials<2>(crl, db, as.dpart + loc + li * (TO / 128));
        E = wave_sum_dpp(E);
        if (lane == 0) {
            as.esum[li * (TO / 64) + 2 * wave] = E;
            as.esum[li * (TO / 64) + 2 * wave + 1] = 0.0f;
        }
    }
    }
    __syncthreads();
}

// Gain/delay adjoint and parameter partials, table form, persistent over work
// items (scene, mic, tile, supergroup): per delay group the tracks, then
// gd_group(2), then the in-tile parameter reductions (param_group); one row of
// parameter partials per item.
template <int T, int TO, int LC, int RB>
__global__ __launch_bounds__(RB == 1 ? kAdjThreads : TO / 2) void k_adjp(
    PlanView pv, const float4* __restrict__ table, int L, const WorkItem* __restrict__ items, int n_items,
    int32_t* __restrict__ ticket, TrackArgs ta, int window, const float* __restrict__ x, const float* __restrict__ gy,
    ParamArgs pa, int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int NT = RB == 1 ? kAdjThreads : TO / 2;
    float4* tab = lds;
    float4* xw = lds + qtab_bytes(T, L) / 16;
    int* lsc = (int*)(xw + window + 1);
    double* pl = (double*)((char*)lsc + kLscBytes);
    int4* dsc = (int4*)((char*)pl + kParamLdsBytes);
    load_qtab<T>(table, tab, L, NT);
    const Slot sl = slot_at(ta.slots, ta.slot_bytes, ta.slot_segs, blockIdx.x);
    const AdjSlot as = adj_slot_at(ta, pa.gmax, TO, blockIdx.x);
    for_each_item(ticket, n_items, [&](int it) {
        const WorkItem w = items[it];
        const DScene& S = pv.scenes[w.scene];
        const DImage* I = pv.imgs + S.img_begin;
        const DBlock B = pv.blocks[S.blk_begin + w.tile / S.blk_tiles];
        const int n0 = w.tile * TO;
        const int n_out = (int)S.n_out;
        const int n_hi = min(n0 + TO, n_out);
        const float* gyc = gy + S.y_off + (int64_t)w.mic * S.n_out;
        ParamAcc acc;
        param_item_begin<NT>(pl, acc);
        const int gb = sg_begin(B.n_grp, S.n_sg, w.sg), ge = sg_begin(B.n_grp, S.n_sg, w.sg + 1);
        int bad = 0;
        for (int g = gb; g < ge; ++g) {
            const DGroup G = pv.groups[B.grp_begin + g];
            const int span = group_span(TO, G.dmin, G.dmax);
            tile_tracks<NT>(S, w.mic, I, pv.perm, G.img_begin, G.img_end, n0, n_hi, span, sl, lsc, ta.knots, ta.mics,
                            ta.c, ta.fs, ta.model);
            if constexpr (RB == 1) {
                gd_group<T, TO, LC>(S, G, n0, sl, as, I, pv.perm, tab, xw, L, x, gyc, pa.ghat, bad);
            } else {
                const int n = n0 + 2 * (int)threadIdx.x;
                const float wy0 = n < n_out ? gyc[n] : 0.0f;
                const float wy1 = n + 1 < n_out ? gyc[n + 1] : 0.0f;
                gd_group2<T, NT, LC>(S, G, n0, sl, as, I, pv.perm, tab, xw, dsc, L, x, wy0, wy1, pa.ghat, bad);
            }
            param_group<NT, TO, RB>(S, w.mic, G, n0, n_hi, sl, as, lsc, I, pv.perm, ta, pa, pl, acc);
        }
        param_item_end<NT>(S, w, pl, acc, pa);
        if (bad) atomicOr(status, kStatusWindow);
    });
}

template <int T, int TO, int RB>
static hipError_t launch_adjp_t(int n_wg, int window, const PlanView& pv, const float4* d_qtable, int Lq,
                                const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta,
                                const float* x, const float* gy, const ParamArgs& pa, int32_t* d_status,
                                hipStream_t st)
{
    constexpr int NT = RB == 1 ? kAdjThreads : TO / 2;
    const size_t lds = adj_track_lds_bytes(T, Lq, window);
    auto kern = Lq == kTablePhases ? k_adjp<T, TO, kTablePhases, RB> : k_adjp<T, TO, 0, RB>;
    if constexpr (RB == 2)
        if (Lq == kPairTablePhases) kern = k_adjp<T, TO, kPairTablePhases, RB>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(64), 0, st, ticket);
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(NT), lds, st, pv, d_qtable, Lq, items, n_items, ticket, ta,
                       window, x, gy, pa, d_status);
    return hipGetLastError();
}

hipError_t launch_adjp(int taps, int nthreads, int rb, int n_wg, int window, const PlanView& pv,
                       const float4* d_qtable, int Lq, const WorkItem* items, int n_items, int32_t* ticket,
                       const TrackArgs& ta, const float* x, const float* gy, const ParamArgs& pa, int32_t* d_status,
                       hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
#define MSIM_ADJP_CASE(TT, NN, RR)                                                                             \
    if (taps == TT && nthreads == NN && rb == RR)                                                             \
        return launch_adjp_t<TT, NN, RR>(n_wg, window, pv, d_qtable, Lq, items, n_items, ticket, ta, x, gy, pa, \
                                         d_status, st);
#define MSIM_ADJP_TAPS(TT)                                                                                     \
    MSIM_ADJP_CASE(TT, 512, 1) MSIM_ADJP_CASE(TT, 1024, 1) MSIM_ADJP_CASE(TT, 512, 2) MSIM_ADJP_CASE(TT, 1024, 2)
    MSIM_ADJP_TAPS(32)
    MSIM_ADJP_TAPS(64)
    MSIM_ADJP_TAPS(96)
    MSIM_ADJP_TAPS(128)
#undef MSIM_ADJP_TAPS
#undef MSIM_ADJP_CASE
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------- reductions

// One wave per (scene, value): value v < 6 is dL/dbeta_v, value 6 + 3 j + a is
// dL/d(source knot j, axis a); the scene's rows summed lane-strided in row order,
// then by a fixed butterfly.  prefix[s]: the scene's first row.
__global__ __launch_bounds__(64) void k_reduce_rows(PlanView pv, int n_values, const double* __restrict__ rows,
                                                    int want_beta, int want_src, double* __restrict__ gbeta,
                                                    double* __restrict__ gsrc)
{
    const int s = blockIdx.y, v = blockIdx.x, lane = threadIdx.x;
    const DScene& S = pv.scenes[s];
    const bool is_beta = v < 6;
    if (is_beta ? !want_beta : (!want_src || v - 6 >= 3 * S.src_knots)) return;
    const int64_t nr = (int64_t)S.n_mics * S.n_sg * S.n_tiles;
    const double* r = rows + S.row_base * kRowWidth + v;
    double acc = 0.0;
    for (int64_t k = lane; k < nr; k += 64) acc += r[k * kRowWidth];
    acc = wave_sum_d(acc);
    if (lane == 0) {
        if (is_beta) gbeta[(int64_t)s * 6 + v] = acc;
        else gsrc[(int64_t)S.src_grad_off * 3 + (v - 6)] = acc;
    }
}

hipError_t launch_reduce_rows(const PlanView& pv, int n_scenes, int scene0, const double* rows, double* gbeta,
                              double* gsrc, hipStream_t st)
{
    // scene0 > 0 only for a one-scene launch: its outputs go to row scene0 of gbeta
    PlanView v = pv;
    hipLaunchKernelGGL(k_reduce_rows, dim3(kRowWidth, (unsigned)n_scenes), dim3(64), 0, st, v, kRowWidth, rows,
                       gbeta != nullptr, gsrc != nullptr, gbeta ? gbeta + (int64_t)scene0 * 6 : nullptr, gsrc);
    return hipGetLastError();
}

int max_grad_knots() { return kMaxGradKnots; }

}  // namespace msim
