// Device-side geometry shared by the forward and adjoint kernels: trajectories,
// image positions and the retarded-delay solve.
#pragma once

#include "msim_internal.h"

#include <hip/hip_runtime.h>

namespace msim {

// ------------------------------------------------------------------ arithmetic

// 1/x and sqrt(x) (x > 0) from the hardware estimates refined by Newton's method
// (two steps each): within a few ulp of the correctly rounded results, in fewer
// instructions than the IEEE division and square-root sequences.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ double sqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);                 // ~1/sqrt(x)
    y = y * fma(-0.5 * x * y, y, 1.5);
    double s = x * y;                                    // ~sqrt(x)
    s = fma(fma(-s, s, x), 0.5 * y, s);
    return s;
}

// The low and high fp16 halves of a 32-bit word as floats (the conversion folds
// into a mixed-precision FMA).
__device__ __forceinline__ float h16_lo(unsigned v)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu));
}

__device__ __forceinline__ float h16_hi(unsigned v)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
}

// p[0] + p[stride] + ... + p[(n - 1) stride], added in that order.  The loads go out
// B at a time so their latencies overlap; slots past n add an exact zero, so the
// result is the plain loop's (up to the sign of a zero total).
template <int B>
__device__ __forceinline__ float strided_sum(const float* __restrict__ p, int n, int64_t stride)
{
    float s = 0.0f;
    for (int g = 0; g < n; g += B) {
        float t[B];
#pragma unroll
        for (int u = 0; u < B; ++u) t[u] = g + u < n ? p[(int64_t)(g + u) * stride] : 0.0f;
#pragma unroll
        for (int u = 0; u < B; ++u) s += t[u];
    }
    return s;
}

// Sum over the 64 lanes of a wave by DPP (no LDS traffic): pairs and quads by
// quad permutes, rows of 16 by mirrors, then rows combined by row broadcasts;
// lane 63 ends with the total, which is returned to every lane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float wave_sum_dpp(float v)
{
    v += dpp_mov<0xB1, 0xF>(v);      // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E, 0xF>(v);      // quad_perm [2,3,0,1]
    v += dpp_mov<0x141, 0xF>(v);     // row_half_mirror
    v += dpp_mov<0x140, 0xF>(v);     // row_mirror
    v += dpp_mov<0x142, 0xA>(v);     // row_bcast:15 into rows 1 and 3
    v += dpp_mov<0x143, 0xC>(v);     // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Minimum and maximum over the 64 lanes of a wave by DPP (the same pattern;
// lanes a step does not write keep their own value).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_self_i(int x)
{
    return __builtin_amdgcn_update_dpp(x, x, CTRL, ROW_MASK, 0xF, false);
}

__device__ __forceinline__ int wave_min_i(int v)
{
    v = min(v, dpp_self_i<0xB1, 0xF>(v));
    v = min(v, dpp_self_i<0x4E, 0xF>(v));
    v = min(v, dpp_self_i<0x141, 0xF>(v));
    v = min(v, dpp_self_i<0x140, 0xF>(v));
    v = min(v, dpp_self_i<0x142, 0xA>(v));
    v = min(v, dpp_self_i<0x143, 0xC>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int wave_max_i(int v)
{
    v = max(v, dpp_self_i<0xB1, 0xF>(v));
    v = max(v, dpp_self_i<0x4E, 0xF>(v));
    v = max(v, dpp_self_i<0x141, 0xF>(v));
    v = max(v, dpp_self_i<0x140, 0xF>(v));
    v = max(v, dpp_self_i<0x142, 0xA>(v));
    v = max(v, dpp_self_i<0x143, 0xC>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// ------------------------------------------------------------------ geometry

// Segment of a PWL path holding t, T[0] <= t: the largest a <= n-2 with T[a] <= t
// (binary search, so dense band-limited paths cost log2 of their knot count).
__device__ __forceinline__ int pwl_find(const double* __restrict__ T, int n, double t)
{
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void traj_pos(const DTraj& tr, const double* __restrict__ knots, double t, double out[3])
{
    if (tr.kind == 1) {
        double s, c;
        sincos(tr.omega * t + tr.phase0, &s, &c);
        out[0] = tr.center[0] + tr.radius * c;
        out[1] = tr.center[1] + tr.radius * s;
        out[2] = tr.center[2];
        return;
    }
    const double* T = knots + tr.knot_off;
    const double* P = knots + tr.pos_off;
    const int n = tr.n_points;
    int a;
    double lam;
    if (n == 1 || t <= T[0]) {
        a = 0;
        lam = 0.0;
    } else if (t >= T[n - 1]) {
        a = n - 1;
        lam = 0.0;
    } else {
        a = pwl_find(T, n, t);
        lam = (t - T[a]) / (T[a + 1] - T[a]);
    }
    const int b = (lam > 0.0) ? a + 1 : a;
    for (int k = 0; k < 3; ++k) out[k] = P[3 * a + k] + lam * (P[3 * b + k] - P[3 * a + k]);
}

// Position and velocity of a trajectory at time t, and the index of the PWL
// segment holding t (-1 before the first knot, n-1 after the last; 0 for circles).
__device__ __forceinline__ int traj_pos_vel_seg(const DTraj& tr, const double* __restrict__ knots, double t, double p[3],
                                       double v[3])
{
    if (tr.kind == 1) {
        double s, c;
        sincos(tr.omega * t + tr.phase0, &s, &c);
        p[0] = tr.center[0] + tr.radius * c;
        p[1] = tr.center[1] + tr.radius * s;
        p[2] = tr.center[2];
        const double sp = tr.radius * tr.omega;
        v[0] = -sp * s;
        v[1] = sp * c;
        v[2] = 0.0;
        return 0;
    }
    const double* T = knots + tr.knot_off;
    const double* P = knots + tr.pos_off;
    const int n = tr.n_points;
    if (n == 1 || t <= T[0] || t >= T[n - 1]) {
        const int a = (n == 1 || t <= T[0]) ? 0 : n - 1;
        for (int k = 0; k < 3; ++k) {
            p[k] = P[3 * a + k];
            v[k] = 0.0;
        }
        return (n == 1 || t <= T[0]) ? -1 : n - 1;
    }
    const int a = pwl_find(T, n, t);
    const double idt = rcp_nr(T[a + 1] - T[a]);
    const double lam = (t - T[a]) * idt;
    for (int k = 0; k < 3; ++k) {
        const double dp = P[3 * (a + 1) + k] - P[3 * a + k];
        p[k] = P[3 * a + k] + lam * dp;
        v[k] = dp * idt;
    }
    return a;
}

// The PWL segment holding t, numbered as traj_pos_vel_seg does (0 for circles).
__device__ __forceinline__ int traj_seg(const DTraj& tr, const double* __restrict__ knots, double t)
{
    if (tr.kind == 1) return 0;
    const double* T = knots + tr.knot_off;
    const int n = tr.n_points;
    if (n == 1 || t <= T[0]) return -1;
    if (t >= T[n - 1]) return n - 1;
    const int a = pwl_find(T, n, t);
    return a;
}

__device__ __forceinline__ double image_coord(int m, double L, double q)
{
    return (m & 1) ? (double)(m + 1) * L - q : (double)m * L + q;
}

__device__ __forceinline__ double dist_to(const DScene& S, const int16_t m[3], const double* knots, const double r[3], double te)
{
    double q[3];
    traj_pos(S.src, knots, te, q);
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double e = image_coord(m[a], S.size[a], q[a]) - r[a];
        d2 += e * e;
    }
    return sqrt(d2);
}

// Position and velocity of a trajectory at time t (velocity zero where a PWL
// path is held at its end knots).
__device__ __forceinline__ void traj_pos_vel(const DTraj& tr, const double* __restrict__ knots, double t, double p[3],
                                    double v[3])
{
    if (tr.kind == 1) {
        double s, c;
        sincos(tr.omega * t + tr.phase0, &s, &c);
        p[0] = tr.center[0] + tr.radius * c;
        p[1] = tr.center[1] + tr.radius * s;
        p[2] = tr.center[2];
        const double sp = tr.radius * tr.omega;
        v[0] = -sp * s;
        v[1] = sp * c;
        v[2] = 0.0;
        return;
    }
    const double* T = knots + tr.knot_off;
    const double* P = knots + tr.pos_off;
    const int n = tr.n_points;
    if (n == 1 || t <= T[0] || t >= T[n - 1]) {
        const int a = (n == 1 || t <= T[0]) ? 0 : n - 1;
        for (int k = 0; k < 3; ++k) {
            p[k] = P[3 * a + k];
            v[k] = 0.0;
        }
        return;
    }
    const int a = pwl_find(T, n, t);
    const double dt = T[a + 1] - T[a];
    const double lam = (t - T[a]) / dt;
    for (int k = 0; k < 3; ++k) {
        const double dp = P[3 * (a + 1) + k] - P[3 * a + k];
        p[k] = P[3 * a + k] + lam * dp;
        v[k] = dp / dt;
    }
}

// Propagation delay (s) for sound received at time t by mic position r.
// Retarded: the root of f(tau) = tau - |p_i(t - tau) - r(t)| / c, by Newton's
// method from the instantaneous delay; f' = 1 + u . S p'(t - tau) / c lies in
// [0.9, 1.1] (speeds below c/10 by validation), so the steps contract even
// across the kinks of a piecewise-linear path.  Instantaneous: |p_i(t) - r(t)| / c.
__device__ __forceinline__ double solve_tau(const DScene& S, const int16_t m[3], const double* knots, const double* mics,
                                   int mic, double t, double inv_c, int model)
{
    double r[3];
    traj_pos(S.rcv, knots, t, r);
    const double* off = mics + 3 * (S.mic_off + mic);
    r[0] += off[0];
    r[1] += off[1];
    r[2] += off[2];
    double tau = dist_to(S, m, knots, r, t) * inv_c;
    if (model == 0) {
        for (int it = 0; it < 30; ++it) {
            double q[3], v[3], e[3];
            traj_pos_vel(S.src, knots, t - tau, q, v);
            double d2 = 0.0, ev = 0.0;
            for (int a = 0; a < 3; ++a) {
                e[a] = image_coord(m[a], S.size[a], q[a]) - r[a];
                d2 += e[a] * e[a];
                ev += e[a] * ((m[a] & 1) ? -v[a] : v[a]);
            }
            const double d = sqrt(d2);
            const double f = tau - d * inv_c;
            const double fp = 1.0 + ev * inv_c / d;
            const double step = f / fp;
            tau -= step;
            if (fabs(step) <= 1e-15 * tau) break;
        }
    }
    return tau;
}

// ------------------------------------------------------------------- tracks

// Position (traj_pos's arithmetic), velocity (zero outside the knot range) and
// PWL segment of a path at t by one search: knot a and the weight lam of knot a+1
// (lam = 0 outside the knot range or for a static path; then only knot a moves it).
__device__ __forceinline__ void pwl_eval(const DTraj& tr, const double* __restrict__ knots, double t, double p[3],
                                double v[3], int* a_out, double* lam_out)
{
    const double* T = knots + tr.knot_off;
    const double* P = knots + tr.pos_off;
    const int n = tr.n_points;
    if (n == 1 || t <= T[0] || t >= T[n - 1]) {
        const int a = (n == 1 || t <= T[0]) ? 0 : n - 1;
        for (int k = 0; k < 3; ++k) {
            p[k] = P[3 * a + k];
            v[k] = 0.0;
        }
        *a_out = a;
        *lam_out = 0.0;
        return;
    }
    const int a = pwl_find(T, n, t);
    const double lam = (t - T[a]) / (T[a + 1] - T[a]);
    const double idt = 1.0 / (T[a + 1] - T[a]);
    for (int k = 0; k < 3; ++k) {
        const double dp = P[3 * (a + 1) + k] - P[3 * a + k];
        p[k] = P[3 * a + k] + lam * dp;
        v[k] = dp * idt;
    }
    *a_out = a;
    *lam_out = lam;
}

__device__ __forceinline__ void mic_pos(const DScene& S, const double* __restrict__ knots, const double* __restrict__ mics,
                               int mic, double t, double r[3])
{
    traj_pos(S.rcv, knots, t, r);
    const double* off = mics + 3 * (S.mic_off + mic);
    r[0] += off[0];
    r[1] += off[1];
    r[2] += off[2];
}


// ------------------------------------------------------- retarded delay

// Distance term of the retarded-delay equation at emission time te: returns
// |p_i(te) - r| and sets ev = (p_i(te) - r) . S p'(te) and the PWL segment of te.
__device__ __forceinline__ double image_dist(const DScene& S, const int16_t m[3], const double* __restrict__ knots,
                                    const double r[3], double te, double* ev, int* seg)
{
    double q[3], v[3];
    *seg = traj_pos_vel_seg(S.src, knots, te, q, v);
    double d2 = 0.0, e_v = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double e = image_coord(m[a], S.size[a], q[a]) - r[a];
        d2 += e * e;
        e_v += e * ((m[a] & 1) ? -v[a] : v[a]);
    }
    *ev = e_v;
    return sqrt_nr(d2);
}

// Retarded delay at reception time t for mic position r: the root of
// f(tau) = tau - |p_i(t - tau) - r| / c, by Newton's method from `tau`
// (f' = 1 + u . S p'(t - tau) / c, in [0.9, 1.1] for speeds below c/10).  A step
// below 1e-9 s ends it; so does one below 1e-5 s whose emission time stayed on
// the same piece of the path: the error left is then the curvature of
// |p_i(t - tau) - r| (below 0.02 / s for the validated speeds and distances)
// times the step squared, under 1e-11 s.
__device__ __forceinline__ double newton_tau(const DScene& S, const int16_t m[3], const double* __restrict__ knots,
                                    const double r[3], double t, double c, double tau)
{
    for (int it = 0; it < 30; ++it) {
        double ev;
        int sg0;
        const double d = image_dist(S, m, knots, r, t - tau, &ev, &sg0);
        const double step = (c * tau - d) * d * rcp_nr(c * d + ev);
        tau -= step;
        const double as = fabs(step);
        if (as <= 1e-9) break;
        if (as <= 1e-5 && traj_seg(S.src, knots, t - tau) == sg0) break;
    }
    return tau;
}

// First guess of the retarded delay: the equation solved with the image moving on
// its tangent at time t, c tau = d - (u . S p'(t)) tau, which is off by
// O((v/c)^2) tau.  Instantaneous model: d / c exactly.
__device__ __forceinline__ double first_tau(const DScene& S, const int16_t m[3], const double* __restrict__ knots,
                                   const double r[3], double t, double c, int model)
{
    double ev;
    int sg;
    const double d = image_dist(S, m, knots, r, t, &ev, &sg);
    return model == 1 ? d / c : d * d * rcp_nr(c * d + ev);
}


// Retarded delay of a piecewise-linear source, by the closed form on each piece
// of the path.  On piece a (knots a, a+1) the image moves linearly,
// S p(t - u) + O - r = W - U u with W the image position extrapolated along the
// piece to the reception time minus r, and U the image velocity; c u = |W - U u|
// is the quadratic (|U|^2 - c^2) u^2 - 2 (W.U) u + |W|^2 = 0, whose positive root
// (|U| < c) is u = |W|^2 / (W.U + sqrt((W.U)^2 + (c^2 - |U|^2) |W|^2)) (a form
// without cancellation).  Before the first knot and after the last the source is
// held still (U = 0).  If the emission time t - u falls outside piece a, the next
// piece towards it is tried; *a carries the piece between calls (-1: before the
// first knot, n-1: after the last; any value is a valid start).
__device__ __forceinline__ double pwl_retarded(const DScene& S, const int16_t m[3], const double* __restrict__ knots,
                                               const double r[3], double t, double c, int* a_io)
{
    const double* T = knots + S.src.knot_off;
    const double* P = knots + S.src.pos_off;
    const int n = S.src.n_points;
    double sg[3], of[3];
    for (int k = 0; k < 3; ++k) {
        sg[k] = (m[k] & 1) ? -1.0 : 1.0;
        of[k] = (m[k] & 1) ? (double)(m[k] + 1) * S.size[k] : (double)m[k] * S.size[k];
    }
    int a = min(max(*a_io, -1), n - 1);
    double u = 0.0;
    for (int it = 0; it < 2 * n + 2; ++it) {
        double W[3], U[3];
        if (a < 0 || a >= n - 1) {
            const int q = a < 0 ? 0 : n - 1;
            for (int k = 0; k < 3; ++k) {
                W[k] = sg[k] * P[3 * q + k] + of[k] - r[k];
                U[k] = 0.0;
            }
        } else {
            const double idt = 1.0 / (T[a + 1] - T[a]);
            const double dt = t - T[a];
            for (int k = 0; k < 3; ++k) {
                const double v = (P[3 * (a + 1) + k] - P[3 * a + k]) * idt;
                W[k] = sg[k] * (P[3 * a + k] + v * dt) + of[k] - r[k];
                U[k] = sg[k] * v;
            }
        }
        const double ww = W[0] * W[0] + W[1] * W[1] + W[2] * W[2];
        const double wu = W[0] * U[0] + W[1] * U[1] + W[2] * U[2];
        const double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
        u = ww / (wu + sqrt_nr(fma(wu, wu, (c * c - uu) * ww)));
        const double te = t - u;
        if (a >= 0 && te < T[a]) {
            --a;                              // emitted on an earlier piece
        } else if (a < n - 1 && te > T[a + 1]) {
            ++a;                              // emitted on a later piece
        } else {
            break;
        }
    }
    *a_io = a;
    return u;
}

// The delay of image m for mic position r at reception time t: the closed form
// above for a piecewise-linear source with retarded delays, else Newton's method
// (circles) or the instantaneous distance.  *a: the path piece hint.
__device__ __forceinline__ double image_delay(const DScene& S, const int16_t m[3], const double* __restrict__ knots,
                                              const double r[3], double t, double c, int model, int* a)
{
    if (model == 0 && S.src.kind == kTrajPwl) return pwl_retarded(S, m, knots, r, t, c, a);
    const double tau = first_tau(S, m, knots, r, t, c, model);
    return model == 0 ? newton_tau(S, m, knots, r, t, c, tau) : tau;
}

// Last scene whose prefix start is <= i (prefix[0] = 0, ascending).
__device__ __forceinline__ int scene_of(const int64_t* __restrict__ prefix, int n, int64_t i)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Clears a persistent launch's ticket counter (a kernel, so graphs hold no memset).
static __global__ void k_zero_ticket(int32_t* p)
{
    if (threadIdx.x == 0) p[0] = 0;
}

// Fixed-order butterfly sum over the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------- persistent kernels

// Work-item loop shared by the persistent kernels: takes items from the ticket
// counter until the list is exhausted and calls fn(item).  Items write disjoint
// outputs, so the result does not depend on which workgroup ran which item.
template <typename F>
__device__ __forceinline__ void for_each_item(int32_t* ticket, int n_items, F&& fn)
{
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(ticket, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        fn(it);
    }
}

// ------------------------------------------------------- tile-local tracks

// The workgroup's track slot: Seg[slot_segs], int32[slot_segs], double[slot_segs
// + 3 gmax] (grid delays), each part 256-byte aligned, then kernel-specific
// scratch at slot_extra_off.  Written and read by one workgroup only, through
// plain (non-restrict) pointers, between barriers.
__device__ inline Slot slot_at(char* slots, int64_t slot_bytes, int slot_segs, int wg)
{
    char* b = slots + (int64_t)wg * slot_bytes;
    Slot s;
    s.seg = (Seg*)b;
    s.K = (int32_t*)(b + slot_al((int64_t)slot_segs * 16));
    s.grid = (double*)(b + slot_al((int64_t)slot_segs * 16) + slot_al((int64_t)slot_segs * 4));
    return s;
}

// p[i] through a 32-bit byte offset from a base that is the same for the whole
// block (the load then takes the scalar-base, vector-offset form).
template <class T>
__device__ __forceinline__ T ld_at(const T* p, uint32_t i)
{
    return *(const T*)((const char*)p + i * (uint32_t)sizeof(T));
}

// k / R for k >= 0 from a float estimate, corrected once (the estimate is within
// one of the quotient for k < 2^24).
__device__ __forceinline__ int div_exact(int k, int R, float invR)
{
    int q = (int)(((float)k + 0.5f) * invR);
    const int r = k - q * R;
    q += r < 0 ? -1 : (r >= R ? 1 : 0);
    return q;
}

// The image of index f in a group's offset table off[0 .. cnt): the last i with
// off[i] <= f.
__device__ __forceinline__ int off_index(const int* off, int cnt, int f)
{
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= f) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Image k of the plan's group permutation, with its slot offset.
__device__ __forceinline__ DImage perm_image(const DImage* __restrict__ I, const PermEntry* __restrict__ perm, int k)
{
    const PermEntry e = perm[k];
    DImage im = I[e.img];
    im.loc = e.loc;
    return im;
}

// Delay tracks of images perm[ib .. ie) of scene S (I: the scene's images), mic `mic`,
// over outputs [n_lo, n_hi) (n_hi <= n_out): segment k of image ii, k_lo <= k <= k_hi
// with k_lo = n_lo / R, k_hi = (n_hi - 1) / R, at slot seg[loc + k - k_lo] (loc: the
// image's permutation entry's slot offset)
// (Seg and integer base, as in the stored form: the exact delay at the audio rate,
// else the uniform Catmull-Rom cubic through D_{k-1} .. D_{k+2}, Sec. II-C-3), and
// the exact grid delays D_g, g = g_lo .. g_hi (k_lo - 1 .. k_hi + 2 when R > 1,
// else k_lo .. k_hi), at grid[loc + 3 (ii - ib) + g - g_lo].
//
// Image ii holds slot_segs_of(R, span) segments and 3 more grid points, so the
// group's grid points form one index space (each image's share at its grid
// offset); every thread takes a run of consecutive indices and solves its points
// in time order, each from the delays before it.  lsc: 2 (ie - ib) + 2 ints of LDS
// for the images' grid and segment offsets.  Starts and ends with a barrier.
template <int NT>
__device__ __forceinline__ void tile_tracks(const DScene& S, int mic, const DImage* __restrict__ I,
                                            const PermEntry* __restrict__ perm, int ib, int ie, int n_lo,
                            int n_hi, int span, Slot sl, int* lsc, const double* __restrict__ knots,
                            const double* __restrict__ mics, double c, double fs, int model)
{
    const int cnt = ie - ib;
    int* goff = lsc;               // [cnt + 1]: first grid index of each image, then the total
    int* soff = lsc + cnt + 1;     // [cnt + 1]: first segment index of each image, then the total
    const double inv_fs = 1.0 / fs;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += NT) {
        const PermEntry e = perm[ib + i];
        goff[i] = e.loc + 3 * i;
        soff[i] = e.loc;
        if (i == cnt - 1) {
            soff[cnt] = e.loc + slot_segs_of(I[e.img].R, span);
            goff[cnt] = soff[cnt] + 3 * cnt;
        }
    }
    __syncthreads();
    auto image_at = [&](const int* off, int f) { return off_index(off, cnt, f); };
    {
        const int total = goff[cnt];
        const int run = (total + NT - 1) / NT;
        const int f0 = threadIdx.x * run, f1 = min(f0 + run, total);
        int ii = f0 < f1 ? image_at(goff, f0) : 0;
        int last_j = -2;               // grid point solved before
        int apiece = 0;                // path piece of its emission time
        int g_lo = 0, npts = 0, R = 1, cur = -1;
        int16_t m[3] = {0, 0, 0};
        for (int f = f0; f < f1; ++f) {
            while (ii + 1 < cnt && f >= goff[ii + 1]) ++ii;
            if (ii != cur) {
                cur = ii;
                const DImage& im = I[perm[ib + ii].img];
                R = im.R;
                m[0] = im.m[0];
                m[1] = im.m[1];
                m[2] = im.m[2];
                const int k_lo = n_lo / R, k_hi = (n_hi - 1) / R;
                g_lo = R == 1 ? k_lo : k_lo - 1;
                npts = (R == 1 ? k_hi : k_hi + 2) - g_lo + 1;
                last_j = -2;
            }
            const int j = f - goff[ii];
            if (j >= npts) continue;
            const double t = (double)(g_lo + j) * (double)R * inv_fs;
            double r[3];
            mic_pos(S, knots, mics, mic, t, r);
            if (last_j != j - 1) apiece = S.src.kind == kTrajPwl ? traj_seg(S.src, knots, t) : 0;
            const double tau = image_delay(S, m, knots, r, t, c, model, &apiece);
            last_j = j;
            sl.grid[f] = fs * tau;
        }
    }
    __syncthreads();
    {
        const int total = soff[cnt];
        for (int f = threadIdx.x; f < total; f += NT) {
            const int i = image_at(soff, f);
            const int R = I[perm[ib + i].img].R;
            const int k_lo = n_lo / R, k_hi = (n_hi - 1) / R;
            const int j = f - soff[i];
            if (j > k_hi - k_lo) continue;
            const double* gd = sl.grid + goff[i];
            if (R == 1) {
                const double D = gd[j];
                const double Kd = floor(D);
                sl.seg[f] = Seg{(float)(D - Kd), 0.0f, 0.0f, 0.0f};
                sl.K[f] = (int32_t)Kd;
            } else {
                // grid index of D_{k-1} is (k - 1) - g_lo = j
                const double iR = 1.0 / (double)R;
                const double D0 = gd[j], D1 = gd[j + 1], D2 = gd[j + 2], D3 = gd[j + 3];
                const double Kd = floor(D1);
                const double a1 = 0.5 * (D2 - D0);
                const double a2 = 0.5 * (2.0 * D0 - 5.0 * D1 + 4.0 * D2 - D3);
                const double a3 = 0.5 * (3.0 * D1 - D0 - 3.0 * D2 + D3);
                sl.seg[f] = Seg{(float)(D1 - Kd), (float)(a1 * iR), (float)(a2 * iR * iR), (float)(a3 * iR * iR * iR)};
                sl.K[f] = (int32_t)Kd;
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------- parameter reductions

__device__ inline AdjSlot adj_slot_at(const TrackArgs& ta, int gmax, int TO, int wg)
{
    char* b = ta.slots + (int64_t)wg * ta.slot_bytes + slot_extra_off(ta.slot_segs, gmax);
    const int64_t np = slot_al(((int64_t)ta.slot_segs + (int64_t)gmax * (TO / 64)) * 16);
    AdjSlot a;
    a.dpart = (float4*)b;
    a.esum = (float*)(b + np);
    a.dseg = (float4*)(b + np + slot_al((int64_t)gmax * 16 * 4));
    return a;
}

// Catmull-Rom transpose partials.  The track parameters need, per segment k of
// an image (outputs n in [kR, kR + R)), the sums
//   S_q(k) = sum_n w_q(u_n) dL/dD(n),  u_n = (n - kR) / R,  q = 0..3,
// w_q the uniform Catmull-Rom basis weights of D_{k-1} .. D_{k+2}.  The gain and
// delay adjoints hold dL/dD with one lane per output, or per pair of outputs
// (RB = 2: the second output of a pair that starts the next segment is taken at
// u = 1 of the first one's, which weights the same grid point).  Over a chunk of
// 64 lanes the lanes' segment index does not decrease, so a segmented inclusive
// scan by DPP leaves the sum of each run of equal segments in the run's last
// lane, which stores it as the (segment, chunk) partial at index (k - k_lo) + c
// of the image's partials: consecutive chunks share at most one segment, so
// distinct pairs get distinct indices.  The per-lane state depends only on the
// lane's output, R and the tile, and is kept while consecutive images share R.
template <int RB>
struct CrLane {
    float w[RB][4];   // basis weights at the lane's outputs
    float m[6];       // scan masks: 1 where the step's source lane is in this lane's segment
    int pidx;         // partial index (k - k_lo) + chunk, or -1 when the lane ends no run
};

__device__ __forceinline__ void cr_weights(float u, float* w)
{
    w[0] = 0.5f * u * fmaf(u, 2.0f - u, -1.0f);
    w[1] = fmaf(u * u, fmaf(1.5f, u, -2.5f), 1.0f);
    w[2] = 0.5f * u * fmaf(u, fmaf(-3.0f, u, 4.0f), 1.0f);
    w[3] = 0.5f * u * u * (u - 1.0f);
}

// State of the lane whose first output is n (unclamped; nc = min(n, n_out - 1)),
// in chunk c of the tile, for an image at rate R: k = nc / R its segment, k_lo
// the tile's first, cv = nc - kR.
template <int RB>
__device__ __forceinline__ void cr_lane(CrLane<RB>& L, int n, int nc, int n_out, int R, float invR, int k, int k_lo,
                                        int c, int lane)
{
    const float cv = (float)(nc - k * R);
#pragma unroll
    for (int r = 0; r < RB; ++r) cr_weights((cv + (float)r) * invR, L.w[r]);
    // source lane l - s is in this lane's segment iff its first output n - s RB
    // (clamped like n) is >= kR, i.e. iff n - kR >= s RB
    const int jj = n - k * R;
    L.m[0] = jj >= RB ? 1.0f : 0.0f;
    L.m[1] = jj >= 2 * RB ? 1.0f : 0.0f;
    L.m[2] = jj >= 4 * RB ? 1.0f : 0.0f;
    L.m[3] = jj >= 8 * RB ? 1.0f : 0.0f;
    L.m[4] = jj >= ((lane & 15) + 1) * RB ? 1.0f : 0.0f;   // from lane 15 of the row before (rows 1, 3)
    L.m[5] = jj >= (lane - 31) * RB ? 1.0f : 0.0f;         // from lane 31 (rows 2, 3)
    const int nn = min(n + RB, n_out - 1);
    const bool end = lane == 63 || nn - k * R >= R;
    L.pidx = end ? (k - k_lo) + c : -1;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void cr_step(float (&v)[4], float m)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = fmaf(dpp_mov<CTRL, ROW_MASK>(v[q]), m, v[q]);
}

// Adds the lane's dL/dD values db[r] (its RB outputs) into the image's partials
// (dpart: the image's first partial).
template <int RB>
__device__ __forceinline__ void cr_partials(const CrLane<RB>& L, const float* db, float4* dpart)
{
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = L.w[0][q] * db[0];
#pragma unroll
        for (int r = 1; r < RB; ++r) v[q] = fmaf(L.w[r][q], db[r], v[q]);
    }
    cr_step<0x111, 0xF>(v, L.m[0]);   // row_shr:1
    cr_step<0x112, 0xF>(v, L.m[1]);   // row_shr:2
    cr_step<0x114, 0xF>(v, L.m[2]);   // row_shr:4
    cr_step<0x118, 0xF>(v, L.m[3]);   // row_shr:8
    cr_step<0x142, 0xA>(v, L.m[4]);   // row_bcast:15 into rows 1 and 3
    cr_step<0x143, 0xC>(v, L.m[5]);   // row_bcast:31 into rows 2 and 3
    if (L.pidx >= 0) dpart[L.pidx] = make_float4(v[0], v[1], v[2], v[3]);
}

// Per-thread dL/dbeta_w partials of a work item.
struct ParamAcc {
    double bw[6];
};

// Knots summed per pass of the grid-point loop (a group's emission times touch a
// few path pieces; more take further passes).
constexpr int kKnotWin = 4;

// pl (LDS): per wave [3 kMaxGradKnots] knot sums (each wave adds its own), then
// [waves][12] reduction scratch.
template <int NT>
__device__ inline void param_item_begin(double* pl, ParamAcc& acc)
{
    static_assert(NT / 64 <= kParamWaves, "parameter LDS holds kParamWaves waves");
    for (int k = threadIdx.x; k < (NT / 64) * 3 * kMaxGradKnots; k += NT) pl[k] = 0.0;
#pragma unroll
    for (int w = 0; w < 6; ++w) acc.bw[w] = 0.0;
}

// Adds n values per thread (n <= 12) of the workgroup in a fixed order: each
// wave's by a butterfly, the waves in order; thread v < n gets total v.
template <int NT>
__device__ inline double block_sum12(const double* v, int n, double* red, int v_out)
{
    constexpr int WAVES = NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = 0; k < n; ++k) {
        const double s = wave_sum_d(v[k]);
        if (lane == 0) red[wave * 12 + k] = s;
    }
    __syncthreads();
    double t = 0.0;
    if (v_out < n)
        for (int w = 0; w < WAVES; ++w) t += red[w * 12 + v_out];
    __syncthreads();
    return t;
}

// The in-tile parameter reductions of one delay group (its tracks in the slot,
// the Catmull-Rom partials of its images over the tile [n0, n_hi) in as.dpart,
// the wave sums of dL/dbeta_i in as.esum; lsc: the group's grid and segment
// offsets; RB outputs per lane in the adjoint that wrote the partials):
//  1. dL/dbeta_w += (d beta_i / d beta_w) dL/dbeta_i, per image (thread-owned);
//  2. per segment k of the tile, S_q(k) = the sum of its (segment, chunk)
//     partials in chunk order (as.dseg);
//  3. per grid point g, dL/dtau_g = fs * the weights of the segments that use
//     D_g, then dtau_g / d p(t_e) for the source position at the emission time
//     t_e = t_g - tau_g (retarded: S^T u / (c + u . S p'(t_e)), u the unit vector
//     mic -> image; instantaneous: S^T u / c), split onto the two knots of t_e's
//     path piece and summed by each wave into its knot sums in LDS (pl).
// The tile's outputs of a segment belong to this item; the other outputs of a
// segment that straddles the tile belong to the neighbouring item, whose row
// holds their part.  Starts after and ends with a barrier.
template <int NT, int TO, int RB>
__device__ inline void param_group(const DScene& S, int mic, const DGroup& G, int n0, int n_hi, Slot sl, AdjSlot as,
                                   const int* lsc, const DImage* __restrict__ I, const PermEntry* __restrict__ perm,
                                   const TrackArgs& ta, const ParamArgs& pa, double* pl, ParamAcc& acc)
{
    constexpr int NCH = TO / (64 * RB);         // 64-lane chunks of the tile
    const int tid = threadIdx.x;
    const int ib = G.img_begin, cnt = G.img_end - ib;
    const int* goff = lsc;
    const int* soff = lsc + cnt + 1;
    constexpr int SL = TO / 64;                 // dL/dbeta_i wave-sum slots per image
    if (pa.want_beta)
        for (int i = tid; i < cnt; i += NT) {
            float e = 0.0f;
            for (int w = 0; w < SL; ++w) e += as.esum[i * SL + w];
            const DImage& im = I[perm[ib + i].img];
            for (int w = 0; w < 6; ++w) {
                const int h = im.hits[w];
                if (h == 0) continue;
                double dv = (double)h;
                for (int r = 0; r < h - 1; ++r) dv *= S.beta[w];
                for (int v = 0; v < 6; ++v) {
                    if (v == w) continue;
                    for (int r = 0; r < im.hits[v]; ++r) dv *= S.beta[v];
                }
                acc.bw[w] += dv * (double)e;
            }
        }
    const bool src = pa.want_src && S.src.kind == kTrajPwl && S.src_knots > 0;
    if (!src) return;
    const int n_out = (int)S.n_out;
    {
        // each thread a run of consecutive segments, walking the image index
        const int total = soff[cnt];
        const int run = (total + NT - 1) / NT;
        const int f0 = tid * run, f1 = min(f0 + run, total);
        int i = f0 < f1 ? off_index(soff, cnt, f0) : 0;
        for (int f = f0; f < f1; ++f) {
            while (i + 1 < cnt && f >= soff[i + 1]) ++i;
            const int R = I[perm[ib + i].img].R;
            const int k_lo = n0 / R, k_hi = (n_hi - 1) / R;
            const int j = f - soff[i];
            if (j > k_hi - k_lo) continue;
            const int k = k_lo + j;
            // chunk c holds the lanes with first outputs n0 + 64 RB c + RB l; it has
            // a partial of segment k iff one of them lies in [kR, kR + R)
            const float4* dp = as.dpart + soff[i] + i * NCH + j;
            float4 t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            for (int c = max(0, (k * R - n0 - 63 * RB) / (64 * RB)); c < NCH; ++c) {
                const int first = n0 + 64 * RB * c;
                if (first > k * R + R - 1 || first >= n_hi) break;
                const int last = min(first + 63 * RB, n_out - 1);
                const int a = max(k * R, first), b = min(k * R + R - 1, last);
                const int na = RB == 1 ? a : a + ((first - a) % RB + RB) % RB;
                if (na > b) continue;
                const float4 p = dp[c];
                t.x += p.x;
                t.y += p.y;
                t.z += p.z;
                t.w += p.w;
            }
            as.dseg[f] = t;
        }
    }
    __syncthreads();
    // knots this group's emission times can touch
    const double fs = ta.fs, c = ta.c;
    const double t_min = ((double)(n0 - 2 * pa.rmax) - (ta.model == 0 ? (double)G.dmax + 1.0 : 0.0)) / fs;
    const double t_max = ((double)(n_hi + 2 * pa.rmax) - (ta.model == 0 ? (double)G.dmin - 1.0 : 0.0)) / fs;
    const int nk = S.src.n_points;
    const int a_lo = max(0, traj_seg(S.src, ta.knots, t_min));
    const int a_hi = min(nk - 1, max(0, traj_seg(S.src, ta.knots, t_max)) + 1);
    const int wave = tid >> 6, lane = tid & 63;
    double* pw = pl + wave * 3 * kMaxGradKnots;
    const int total = goff[cnt];
    const int run = (total + NT - 1) / NT;
    const int f0 = tid * run, f1 = min(f0 + run, total);
    const int i0 = f0 < f1 ? off_index(goff, cnt, f0) : 0;
    for (int kb = a_lo; kb <= a_hi; kb += kKnotWin) {
        double ak[kKnotWin * 3];
#pragma unroll
        for (int q = 0; q < kKnotWin * 3; ++q) ak[q] = 0.0;
        int i = i0;
        for (int f = f0; f < f1; ++f) {
            while (i + 1 < cnt && f >= goff[i + 1]) ++i;
            const DImage& im = I[perm[ib + i].img];
            const int R = im.R;
            const int k_lo = n0 / R, k_hi = (n_hi - 1) / R;
            const int g_lo = R == 1 ? k_lo : k_lo - 1;
            const int npts = (R == 1 ? k_hi : k_hi + 2) - g_lo + 1;
            const int j = f - goff[i];
            if (j >= npts) continue;
            const int g = g_lo + j;
            double dD = 0.0;
            for (int q = 0; q < 4; ++q) {
                const int s = g + 1 - q;                 // segment s uses grid point g with basis index q
                if (s < k_lo || s > k_hi) continue;
                const float4 w4 = as.dseg[soff[i] + s - k_lo];
                dD += (double)(q == 0 ? w4.x : q == 1 ? w4.y : q == 2 ? w4.z : w4.w);
            }
            if (dD == 0.0) continue;
            const double taubar = fs * dD;
            const double tk = (double)g * (double)R / fs;
            const double te = ta.model == 0 ? tk - sl.grid[f] / fs : tk;
            double qp[3], vp[3], r[3], lam;
            int a;
            pwl_eval(S.src, ta.knots, te, qp, vp, &a, &lam);
            mic_pos(S, ta.knots, ta.mics, mic, tk, r);
            double e[3], d2 = 0.0, sgn[3];
            for (int ax = 0; ax < 3; ++ax) {
                sgn[ax] = (im.m[ax] & 1) ? -1.0 : 1.0;
                e[ax] = image_coord(im.m[ax], S.size[ax], qp[ax]) - r[ax];
                d2 += e[ax] * e[ax];
            }
            const double id = 1.0 / sqrt(d2);
            double denom = c;
            if (ta.model == 0)
                for (int ax = 0; ax < 3; ++ax) denom += e[ax] * id * sgn[ax] * vp[ax];
            const double sc = taubar * id / denom;
            const double wa = 1.0 - lam, wb = lam;
#pragma unroll
            for (int jj = 0; jj < kKnotWin; ++jj) {
                const int kk = kb + jj;
                const double fw = (kk == a) ? wa : (kk == a + 1) ? wb : 0.0;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) ak[3 * jj + ax] += fw * (sc * sgn[ax] * e[ax]);
            }
        }
        // the wave's sums into its own knot sums (no other wave writes them)
#pragma unroll
        for (int q = 0; q < kKnotWin * 3; ++q) {
            const int kk = kb + q / 3;
            if (kk >= nk || kk >= kMaxGradKnots) break;
            const double s = wave_sum_d(ak[q]);
            if (lane == 0) pw[3 * kb + q] += s;
        }
    }
    __syncthreads();
}

// Writes the item's row of parameter partials: dL/dbeta_w (summed over the
// workgroup in a fixed order) and the knot sums (the waves' in order).
template <int NT>
__device__ inline void param_item_end(const DScene& S, const WorkItem& w, double* pl, ParamAcc& acc,
                                      const ParamArgs& pa)
{
    constexpr int WAVES = NT / 64;
    double* red = pl + WAVES * 3 * kMaxGradKnots;
    __syncthreads();
    const double tb = block_sum12<NT>(acc.bw, 6, red, threadIdx.x);
    double* row = pa.rows + (S.row_base + ((int64_t)w.mic * S.n_sg + w.sg) * S.n_tiles + w.tile) * kRowWidth;
    if (threadIdx.x < 6) row[threadIdx.x] = tb;
    for (int k = threadIdx.x; k < 3 * kMaxGradKnots; k += NT) {
        double t = 0.0;
        for (int v = 0; v < WAVES; ++v) t += pl[v * 3 * kMaxGradKnots + k];
        row[6 + k] = t;
    }
    __syncthreads();
}

}  // namespace msim
