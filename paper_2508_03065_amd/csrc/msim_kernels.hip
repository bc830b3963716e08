// gfx950 kernels of the moving image-source synthesis.
//
//   tracks      : exact delays of every image on its tier's grid (FP64 retarded
//                 solve), turned into per-segment Catmull-Rom cubics stored as an
//                 integer base plus FP32 offsets (Sec. II-C-3: decimated delays
//                 of high-order images, upsampled to the audio rate).
//   synth_fwd   : the gather-reduce y[n] = sum_i g_i(n) sum_j h(j - mu_i(n)) x[n - K_i(n) - j]
//                 (Eq. 2 / Eq. 8 with the FIR fractional delay of Sec. II-B), one
//                 output sample per lane, images of one delay group per
//                 workgroup, source window and fractional-delay table in LDS.
//   reduce      : fixed-order sum of the per-group partial outputs.
#include "msim_device.h"
#include "msim_internal.h"
#include "msim_pair.h"

#include <hip/hip_runtime.h>

namespace msim {

// -------------------------------------------------------------- forward synth

// LDS: the half table of h(v) = h(-v), v in [0, T/2], for quadratic
// interpolation between Lq phases, grouped by four taps, as three arrays over
// (g, r), r in [-1, Lq) (qtab_pitch(Lq) rows per quad, row r at index r + 1):
// Y(r) (float4), Y(r+1) - Y(r) (float4), Y(r+2) - 2 Y(r+1) + Y(r) (four fp16),
// Y(r) = (h((4g+e) + r/Lq)), e = 0..3; then the source window as overlapping
// quads xw[p] = x[ws+p .. ws+p+3] (split by parity at two outputs per lane, one
// entry more).
// Image descriptors of a delay group staged in LDS at a time by the two-outputs
// kernel (one chunk covers a group at the table form's default cap of 96 images).
constexpr int kSynDescChunk = 96;

size_t synth_lds_bytes(int taps, int Lq, int window)
{
    return qtab_bytes(taps, Lq) + (size_t)kSynDescChunk * 2 * sizeof(int4) + (size_t)(window + 1) * sizeof(float4);
}

// One delay group of an output tile [n0, n0 + NT) of one mic: stages the group's
// source window in LDS (the table must already be there, the group's tracks in
// the slot), then one output sample per lane adds every image of the group to
// acc.  The tap weights come from the quadratic table: with q = mu Lq = k + f, the
// taps on the delay's near side (|u| = 4g+e + mu) read base row k at fraction f,
// the mirrored ones (|u| = 4g+e + 1 - mu) base row Lq-1-k at fraction 1-f, and
// both second-difference terms carry the same weight f (f - 1) / 2.  LC is Lq
// when known at compile time (then every table read has an immediate offset),
// else 0 and Lr is used.  Ends with a barrier.
template <int T, int NT, int LC>
__device__ inline void synth_group(const DScene& S, const DGroup& G, int n0, Slot sl, const DImage* __restrict__ I,
                                   const PermEntry* __restrict__ perm, const float4* tab, float4* xw, int Lr, const float* __restrict__ x, float& acc,
                                   int& bad)
{
    constexpr int NG = T / 8;          // tap quads per side
    const int L = LC > 0 ? LC : Lr;
    const int LP = LC > 0 ? LC + 1 : Lr + 1;
    const QTab tq = qtab_view<T>(tab, LP);
    const int tid = threadIdx.x;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = NT + (G.dmax - G.dmin) + T + 8;
    const int n_in = (int)S.n_in;
    stage_window(x + S.x_off, n_in, ws, W, xw, NT);
    __syncthreads();

    const int n = n0 + tid;
    if (n < (int)S.n_out) {
        const float Lf = (float)L;
        // The lane's segment (slot index relative to the image's first) and its
        // offset depend only on the decimation: kept for the last R seen.  Track
        // data of the next image is fetched while the current one is filtered.
        int cR = 0, cl = 0;
        float cv = 0.0f;
        auto fetch = [&](const DImage& im, Seg& q, int& K, float& v) {
            if (im.R != cR) {
                cR = im.R;
                const int k = div_exact(n, cR, im.invR);
                cl = k - div_exact(n0, cR, im.invR);
                cv = (float)(n - k * cR);
            }
            q = sl.seg[im.loc + cl];
            K = sl.K[im.loc + cl];
            v = cv;
        };
        auto body = [&](const DImage& im, const Seg& sg, int Ks, float v) {
            const float d = fmaf(v, fmaf(v, fmaf(v, sg.b3, sg.b2), sg.b1), sg.a0);
            const float fl = floorf(d);
            const int K = Ks + (int)fl;
            // skip the image when no lane's taps reach a source sample
            if (!__any(n - K + T / 2 - 1 >= 0 && n - K - T / 2 < n_in)) return;
            const int p0 = n - K - ws;
            if (p0 < T / 2 || p0 > W - T / 2 + 3) {
                bad = 1;
                return;
            }
            const float mu = d - fl;
            const float gain = im.gfac * __builtin_amdgcn_rcpf((float)Ks + d);
            const float q = mu * Lf;
            const int kq = min((int)q, L - 1);
            const float f = q - (float)kq;
            const int kp = L - 1 - kq;
            const float4* xq = xw + p0;
            float A = 0.0f, B = 0.0f, Bm = 0.0f, C = 0.0f;
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                // taps j = -(4gi+e): x[n-K+4gi+e], |u| = 4gi+e + mu -> base row kq, fraction f
                const float4 xn = xq[4 * gi];
                const float4 Y = tq.Y[gi * LP + kq], D1 = tq.D1[gi * LP + kq];
                A = fmaf(Y.x, xn.x, A); B = fmaf(D1.x, xn.x, B);
                A = fmaf(Y.y, xn.y, A); B = fmaf(D1.y, xn.y, B);
                A = fmaf(Y.z, xn.z, A); B = fmaf(D1.z, xn.z, B);
                A = fmaf(Y.w, xn.w, A); B = fmaf(D1.w, xn.w, B);
                if (gi < qcorr_quads(T)) {      // further out the quadratic term is zero
                    const uint2 D2 = tq.D2[gi * LP + kq];
                    C = fmaf(h16_lo(D2.x), xn.x, C); C = fmaf(h16_hi(D2.x), xn.y, C);
                    C = fmaf(h16_lo(D2.y), xn.z, C); C = fmaf(h16_hi(D2.y), xn.w, C);
                }
                // taps j = 1+4gi+e: x[n-K-1-4gi-e] (quad component 3-e), |u| = 4gi+e + 1-mu
                //   -> base row L-1-kq, fraction 1-f
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
            acc = fmaf(gain, s, acc);
        };
        Seg qa{}, qb{};
        int Ka = 0, Kb = 0;
        float va = 0.0f, vb = 0.0f;
        DImage ia = perm_image(I, perm, G.img_begin), ib;
        fetch(ia, qa, Ka, va);
        int ii = G.img_begin;
        for (; ii + 1 < G.img_end; ii += 2) {
            ib = perm_image(I, perm, ii + 1);
            fetch(ib, qb, Kb, vb);
            body(ia, qa, Ka, va);
            if (ii + 2 < G.img_end) {
                ia = perm_image(I, perm, ii + 2);
                fetch(ia, qa, Ka, va);
            }
            body(ib, qb, Kb, vb);
        }
        if (ii < G.img_end) body(ia, qa, Ka, va);
    }
    __syncthreads();
}

// The same group with two adjacent outputs n, n+1 per lane (NT lanes, 2 NT outputs
// per tile), which take their tap weights from the same table rows (pair_frame,
// pair_sums): half the LDS bytes per tap.  Output n+1's taps are output n's shifted
// by one source position; in the shared frame its far-side tap -T/2+1 and near-side
// tap T/2+1 fall outside or at the kernel's edge.  The plan uses it only while the
// delay drifts by well under two table rows per sample and that edge tap's weight
// is below its accuracy bound.  Ends with a barrier.
template <int T, int NT, int LC>
__device__ inline void synth_group2(const DScene& S, const DGroup& G, int n0, Slot sl, const DImage* __restrict__ I,
                                    const PermEntry* __restrict__ perm, const float4* tab, float4* xw, int4* dsc,
                                    int Lr, const float* __restrict__ x, float& acc0, float& acc1, int& bad)
{
    constexpr int NG = T / 8;
    constexpr int TO = 2 * NT;
    const int L = LC > 0 ? LC : Lr;
    const int LP = LC > 0 ? LC + 1 : Lr + 1;
    const QTab tq = qtab_view<T>(tab, LP);
    const int tid = threadIdx.x;
    const int ws = n0 - G.dmax - T / 2 - 4;
    const int W = TO + (G.dmax - G.dmin) + T + 8;
    const int half = split_half(W);
    const int n_in = (int)S.n_in;
    stage_window_split(x + S.x_off, n_in, ws, W, xw, NT);

    const int n = n0 + 2 * tid;
    const int n_out = (int)S.n_out;
    const bool active = n < n_out;
    // every lane's taps reach source samples for every image of the group (integer
    // delays within [dmin, dmax]): the per-image check is skipped
    const bool all_reach = n0 - G.dmax + T / 2 >= 0 && n0 + TO - G.dmin - T / 2 < n_in;
    const float Lf = (float)L;
    // The group's image descriptors a chunk at a time in LDS (slot offset, R, gain
    // factor, 1/R; k_lo = n0 / R), read there as wave-uniform values.  Track data
    // for both outputs: one segment when the image is decimated (every decimation
    // is even, so n and n+1 share it), else the two full-rate delays (full-rate
    // segments carry zero cubic terms, so the segment of n gives D(n) either way).
    // The lane's slot offsets depend only on the decimation R: they are kept for
    // the last R seen (images of a group mostly share a tier).  Two buffers in
    // turn, as in the one-output group.
    for (int cb = G.img_begin; cb < G.img_end; cb += kSynDescChunk) {
        const int nch = min(kSynDescChunk, G.img_end - cb);
        __syncthreads();                 // window staged; the previous chunk's descriptors read
        for (int i = tid; i < nch; i += NT) {
            const PermEntry e = perm[cb + i];
            const DImage& im = I[e.img];
            dsc[2 * i] = make_int4(e.loc, im.R, __float_as_int(im.gfac), __float_as_int(im.invR));
            dsc[2 * i + 1] = make_int4(div_exact(n0, im.R, im.invR), 0, 0, 0);
        }
        __syncthreads();
        if (!active) continue;
        int cR = 0, c0 = 0, c1 = 0;        // slot indices of the segments of n and n+1
        float cv = 0.0f;                    // n relative to its segment start
        struct Img {
            int R;
            float gfac;
            Seg q;
            float a1;
            int K0, K1;
            float v;
        };
        auto fetch = [&](int j, Img& m) {
            const int4 d0 = dsc[2 * j];
            const int loc = __builtin_amdgcn_readfirstlane(d0.x);
            const int R = __builtin_amdgcn_readfirstlane(d0.y);
            if (R != cR) {
                cR = R;
                if (R == 1) {
                    c0 = n - n0;
                    c1 = min(n + 1, n_out - 1) - n0;
                    cv = 0.0f;
                } else {
                    const int k0 = div_exact(n, R, __int_as_float(d0.w));
                    c0 = c1 = k0 - __builtin_amdgcn_readfirstlane(dsc[2 * j + 1].x);
                    cv = (float)(n - k0 * R);
                }
            }
            m.R = R;
            m.gfac = __int_as_float(d0.z);
            m.q = ld_at(sl.seg, (uint32_t)(loc + c0));
            m.K0 = ld_at(sl.K, (uint32_t)(loc + c0));
            if (R == 1) {
                m.a1 = ld_at(sl.seg, (uint32_t)(loc + c1)).a0;
                m.K1 = ld_at(sl.K, (uint32_t)(loc + c1));
            } else {
                m.a1 = 0.0f;
                m.K1 = m.K0;
            }
            m.v = cv;
        };
        auto body = [&](const Img& m) {
            const Seg& sg = m.q;
            const float v = m.v;
            const float d0 = fmaf(v, fmaf(v, fmaf(v, sg.b3, sg.b2), sg.b1), sg.a0);
            const float v1 = v + 1.0f;
            const float d1 = m.R == 1 ? m.a1 : fmaf(v1, fmaf(v1, fmaf(v1, sg.b3, sg.b2), sg.b1), sg.a0);
            const PairFrame fr = pair_frame(d0, m.K0, d1, m.K1, L, Lf);
            const int K = fr.K;
            // skip the image when no lane's taps reach a source sample
            if (!all_reach && !__any(n - K + T / 2 >= 0 && n - K - T / 2 < n_in)) return;
            const int p0 = n - K - ws;
            if (p0 < T / 2 || p0 > W - 1 - T / 2) {
                bad = 1;
                return;
            }
            PairSums ps;
            pair_sums<NG>(tq, LP, fr.kq, fr.kp, split_at(xw, half, p0), ps);
            const float f0 = fr.q0 - (float)fr.kq, f1 = fr.q1 - (float)fr.kq;                   // near side
            const float h0 = (Lf - fr.q0) - (float)fr.kp, h1 = (Lf - fr.q1) - (float)fr.kp;     // far side
            const float s0 = fmaf(qweight(h0), ps.Cm0, fmaf(qweight(f0), ps.C0, fmaf(h0, ps.Bm0, fmaf(f0, ps.B0, ps.A0))));
            const float s1 = fmaf(qweight(h1), ps.Cm1, fmaf(qweight(f1), ps.C1, fmaf(h1, ps.Bm1, fmaf(f1, ps.B1, ps.A1))));
            acc0 = fmaf(m.gfac * __builtin_amdgcn_rcpf((float)m.K0 + d0), s0, acc0);
            acc1 = fmaf(m.gfac * __builtin_amdgcn_rcpf((float)m.K1 + d1), s1, acc1);
        };
        Img ia, ib;
        fetch(0, ia);
        int j = 0;
        for (; j + 1 < nch; j += 2) {
            fetch(j + 1, ib);
            body(ia);
            if (j + 2 < nch) fetch(j + 2, ia);
            body(ib);
        }
        if (j < nch) body(ia);
    }
    __syncthreads();
}

// Forward synthesis, persistent: a fixed grid of workgroups loads the table once,
// then takes work items (scene, mic, tile, supergroup).  For each delay group of
// the item's supergroup it solves the group's delay tracks over the tile into the
// workgroup's slot (tile_tracks) and adds the group's images to the lane's
// register accumulators; the item's sum over its groups (in group order) is
// written once.  RB outputs per lane (1 or 2), NT lanes, NT * RB outputs per tile.
template <int T, int NT, int LC, int RB>
__global__ __launch_bounds__(NT, 4) void k_synth(PlanView pv, const float4* __restrict__ table, int L,
                                                 const WorkItem* __restrict__ items, int n_items,
                                                 int32_t* __restrict__ ticket, TrackArgs ta,
                                                 const float* __restrict__ x, float* __restrict__ part,
                                                 int32_t* __restrict__ status)
{
    extern __shared__ float4 lds[];
    constexpr int TO = NT * RB;
    float4* tab = lds;
    int4* dsc = (int4*)(lds + qtab_bytes(T, L) / 16);
    float4* xw = (float4*)(dsc + 2 * kSynDescChunk);
    load_qtab<T>(table, tab, L, NT);
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
        float acc0 = 0.0f, acc1 = 0.0f;
        int bad = 0;
        for (int g = gb; g < ge; ++g) {
            const DGroup G = pv.groups[B.grp_begin + g];
            tile_tracks<NT>(S, w.mic, I, pv.perm, G.img_begin, G.img_end, n0, n_hi, group_span(TO, G.dmin, G.dmax),
                            sl, (int*)xw, ta.knots, ta.mics, ta.c, ta.fs, ta.model);
            if constexpr (RB == 1)
                synth_group<T, NT, LC>(S, G, n0, sl, I, pv.perm, tab, xw, L, x, acc0, bad);
            else
                synth_group2<T, NT, LC>(S, G, n0, sl, I, pv.perm, tab, xw, dsc, L, x, acc0, acc1, bad);
        }
        float* out = part + S.part_base + ((int64_t)w.mic * S.n_sg + w.sg) * S.n_out;
        const int n = n0 + RB * (int)threadIdx.x;
        if (n < n_out) out[n] = acc0;
        if (RB == 2 && n + 1 < n_out) out[n + 1] = acc1;
        if (bad) atomicOr(status, kStatusWindow);
    });
}

template <int T, int TO, int RB>
static hipError_t launch_synth_t(int n_wg, int window, const PlanView& pv, const float4* d_table, int L,
                                 const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta,
                                 const float* x, float* part, int32_t* d_status, hipStream_t st)
{
    constexpr int NT = TO / RB;
    const size_t lds = synth_lds_bytes(T, L, window);
    auto kern = L == kTablePhases ? k_synth<T, NT, kTablePhases, RB> : k_synth<T, NT, 0, RB>;
    if constexpr (RB == 2)
        if (L == kPairTablePhases) kern = k_synth<T, NT, kPairTablePhases, RB>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_ticket, dim3(1), dim3(64), 0, st, ticket);
    hipLaunchKernelGGL(kern, dim3((unsigned)n_wg), dim3(NT), lds, st, pv, d_table, L, items, n_items, ticket, ta, x,
                       part, d_status);
    return hipGetLastError();
}

hipError_t launch_synth(int taps, int nthreads, int rb, int n_wg, int window, const PlanView& pv,
                        const float4* d_table, int L, const WorkItem* items, int n_items, int32_t* ticket,
                        const TrackArgs& ta, const float* x, float* part, int32_t* d_status, hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
#define MSIM_SYN_CASE(TT, NN, RR)                                                                              \
    if (taps == TT && nthreads == NN && rb == RR)                                                             \
        return launch_synth_t<TT, NN, RR>(n_wg, window, pv, d_table, L, items, n_items, ticket, ta, x, part,   \
                                          d_status, st);
#define MSIM_SYN_TAPS(TT)                                                                                      \
    MSIM_SYN_CASE(TT, 512, 1) MSIM_SYN_CASE(TT, 1024, 1) MSIM_SYN_CASE(TT, 512, 2) MSIM_SYN_CASE(TT, 1024, 2)
    MSIM_SYN_TAPS(32)
    MSIM_SYN_TAPS(64)
    MSIM_SYN_TAPS(96)
    MSIM_SYN_TAPS(128)
#undef MSIM_SYN_TAPS
#undef MSIM_SYN_CASE
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ reduction

// Partial outputs [mic][supergroup][n_out] summed in supergroup order, one thread
// per output sample of every scene (y packed scene-major); prefix[s] is scene s's
// first output.
__global__ __launch_bounds__(256) void k_reduce_sg(const DScene* __restrict__ scenes, int n_scenes,
                                                   const int64_t* __restrict__ y_prefix, int64_t y_total,
                                                   const float* __restrict__ part, float* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= y_total) return;
    const int s = scene_of(y_prefix, n_scenes, i);
    const DScene& S = scenes[s];
    const int64_t j = i - y_prefix[s];
    const int mic = (int)(j / S.n_out);
    const int64_t n = j - (int64_t)mic * S.n_out;
    y[S.y_off + j] = strided_sum<16>(part + S.part_base + (int64_t)mic * S.n_sg * S.n_out + n, S.n_sg, S.n_out);
}

hipError_t launch_reduce_sg(const DScene* d_scenes, int n_scenes, const int64_t* d_y_prefix, int64_t y_total,
                            const float* part, float* y, hipStream_t st)
{
    if (y_total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_sg, dim3((unsigned)((y_total + 255) / 256)), dim3(256), 0, st, d_scenes, n_scenes,
                       d_y_prefix, y_total, part, y);
    return hipGetLastError();
}

}  // namespace msim
