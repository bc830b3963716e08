// Host side of the msim C-ABI: validation, image enumeration, delay-sorted
// grouping, the fractional-delay table, workspace sizing and launch order.
#include "../../include/msim.h"
#include "msim_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace msim;

namespace {

thread_local std::string g_err;

msim_status fail(msim_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

// A failed HIP call is reported as MSIM_E_HIP and HIP's last-error state is
// cleared, so the caller's next HIP call does not see it again.
#define HIP_OK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            (void)hipGetLastError();                                                               \
            return fail(MSIM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));                      \
        }                                                                                          \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
constexpr int64_t kMaxOut = int64_t(1) << 23;
constexpr size_t kLdsLimit = 160 * 1024 - 256;   // dynamic LDS (a little is static)
constexpr int kSlotSegCap = 4096;                   // track segments per workgroup slot (unless one image needs more)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

// Scratch of msim_forward_noalloc: a fixed array on every GPU the library runs
// on, held until the process ends.  Host code uses only its per-device address
// from hipGetSymbolAddress (the array's name is a host-side stand-in).
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The address of `scratch` on device dev (which must be current), looked up once.
msim_status scratch_on(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(MSIM_E_UNSUPPORTED, "device %d: beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(MSIM_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MSIM_OK;
}

// Modified Bessel function I0 by its power series sum_k ((x/2)^k / k!)^2.
double bessel_i0(double x)
{
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 1000 && term > 1e-17 * sum; ++k) {
        term *= q / (double(k) * double(k));
        sum += term;
    }
    return sum;
}

// Kaiser-windowed sinc fractional-delay kernel, h(v) on |v| <= T/2.
double fd_kernel(double v, int T, double kbeta, double fc, double i0b)
{
    if (std::fabs(v) > 0.5 * T) return 0.0;
    const double z = 2.0 * fc * v;
    const double sinc = (z == 0.0) ? 1.0 : std::sin(kPi * z) / (kPi * z);
    const double r = 2.0 * v / T;
    const double w = bessel_i0(kbeta * std::sqrt(std::max(0.0, 1.0 - r * r))) / i0b;
    return 2.0 * fc * sinc * w;
}

struct Box {
    double lo[3], hi[3];
};

Box traj_box(const msim_traj& tr)
{
    Box b;
    if (tr.kind == MSIM_TRAJ_CIRCLE) {
        for (int a = 0; a < 2; ++a) {
            b.lo[a] = tr.center[a] - tr.radius;
            b.hi[a] = tr.center[a] + tr.radius;
        }
        b.lo[2] = b.hi[2] = tr.center[2];
        return b;
    }
    for (int a = 0; a < 3; ++a) b.lo[a] = b.hi[a] = tr.p[a];
    for (int k = 1; k < tr.n_points; ++k)
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = std::min(b.lo[a], tr.p[3 * k + a]);
            b.hi[a] = std::max(b.hi[a], tr.p[3 * k + a]);
        }
    return b;
}

bool inside(const double p[3], const double L[3])
{
    for (int a = 0; a < 3; ++a)
        if (!(p[a] > 0.0 && p[a] < L[a])) return false;
    return true;
}

void traj_at(const msim_traj& tr, double t, double out[3])
{
    if (tr.kind == MSIM_TRAJ_CIRCLE) {
        const double w = tr.speed / tr.radius;
        out[0] = tr.center[0] + tr.radius * std::cos(w * t + tr.phase0);
        out[1] = tr.center[1] + tr.radius * std::sin(w * t + tr.phase0);
        out[2] = tr.center[2];
        return;
    }
    const int n = tr.n_points;
    if (n == 1 || t <= tr.t[0]) {
        for (int a = 0; a < 3; ++a) out[a] = tr.p[a];
        return;
    }
    if (t >= tr.t[n - 1]) {
        for (int a = 0; a < 3; ++a) out[a] = tr.p[3 * (n - 1) + a];
        return;
    }
    int k = 0;
    while (k + 2 < n && t >= tr.t[k + 1]) ++k;
    const double lam = (t - tr.t[k]) / (tr.t[k + 1] - tr.t[k]);
    for (int a = 0; a < 3; ++a) out[a] = tr.p[3 * k + a] + lam * (tr.p[3 * (k + 1) + a] - tr.p[3 * k + a]);
}

// Box of a trajectory over the times [ta, tb]: the end points and the knots in
// between (PWL), or the arc sampled at 64 steps padded by the sagitta of a step
// (circle; the whole circle when the arc is a full turn).
Box traj_box_range(const msim_traj& tr, double ta, double tb)
{
    Box b;
    double q[3];
    traj_at(tr, ta, q);
    for (int a = 0; a < 3; ++a) b.lo[a] = b.hi[a] = q[a];
    auto add = [&](const double* v) {
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = std::min(b.lo[a], v[a]);
            b.hi[a] = std::max(b.hi[a], v[a]);
        }
    };
    if (tr.kind == MSIM_TRAJ_CIRCLE) {
        const double w = tr.speed / tr.radius, span = (tb - ta) * w;
        if (span >= 2.0 * kPi) return traj_box(tr);
        const int steps = 64;
        for (int k = 1; k <= steps; ++k) {
            traj_at(tr, ta + (tb - ta) * k / steps, q);
            add(q);
        }
        const double dth = span / steps, sag = tr.radius * dth * dth / 8.0 + 1e-9;
        for (int a = 0; a < 2; ++a) {
            b.lo[a] -= sag;
            b.hi[a] += sag;
        }
        return b;
    }
    traj_at(tr, tb, q);
    add(q);
    for (int k = 0; k < tr.n_points; ++k)
        if (tr.t[k] > ta && tr.t[k] < tb) add(tr.p + 3 * k);
    return b;
}

msim_status check_traj(const msim_traj& tr, const double L[3], double c, const char* what)
{
    if (tr.kind == MSIM_TRAJ_PWL) {
        if (tr.n_points < 1 || !tr.t || !tr.p) return fail(MSIM_E_INVALID_ARG, "%s: PWL needs >= 1 knot", what);
        for (int k = 0; k < tr.n_points; ++k) {
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(tr.p[3 * k + a])) return fail(MSIM_E_INVALID_ARG, "%s: non-finite knot", what);
            if (!std::isfinite(tr.t[k])) return fail(MSIM_E_INVALID_ARG, "%s: non-finite knot time", what);
            if (k > 0) {
                const double dt = tr.t[k] - tr.t[k - 1];
                if (!(dt > 0.0)) return fail(MSIM_E_INVALID_ARG, "%s: knot times must increase strictly", what);
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double e = tr.p[3 * k + a] - tr.p[3 * (k - 1) + a];
                    d2 += e * e;
                }
                if (std::sqrt(d2) / dt >= 0.1 * c)
                    return fail(MSIM_E_SUPERSONIC, "%s: segment %d moves at >= c/10", what, k - 1);
            }
        }
        return MSIM_OK;
    }
    if (tr.kind == MSIM_TRAJ_CIRCLE) {
        if (!(tr.radius > 0.0) || !(tr.speed >= 0.0) || !std::isfinite(tr.phase0))
            return fail(MSIM_E_INVALID_ARG, "%s: circle needs radius > 0 and speed >= 0", what);
        if (tr.speed >= 0.1 * c) return fail(MSIM_E_SUPERSONIC, "%s: circle speed >= c/10", what);
        return MSIM_OK;
    }
    return fail(MSIM_E_INVALID_ARG, "%s: unknown trajectory kind %d", what, tr.kind);
}

// Largest speed along a trajectory (m/s): the fastest PWL segment, or the circle's speed.
double traj_max_speed(const msim_traj& tr)
{
    if (tr.kind == MSIM_TRAJ_CIRCLE) return tr.speed;
    double v = 0.0;
    if (tr.kind == MSIM_TRAJ_PWL)
        for (int k = 1; k < tr.n_points; ++k) {
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double e = tr.p[3 * k + a] - tr.p[3 * (k - 1) + a];
                d2 += e * e;
            }
            v = std::max(v, std::sqrt(d2) / (tr.t[k] - tr.t[k - 1]));
        }
    return v;
}

msim_status check_params(const msim_params* p)
{
    if (!p) return fail(MSIM_E_INVALID_ARG, "params is NULL");
    if (!(p->c > 0.0) || !(p->fs > 0.0)) return fail(MSIM_E_INVALID_ARG, "c and fs must be > 0");
    if (p->taps < 8 || p->taps > 128 || p->taps % 8 != 0)
        return fail(MSIM_E_INVALID_ARG, "taps must be a multiple of 8 in 8..128 (got %d)", p->taps);
    if (p->taps != 32 && p->taps != 64 && p->taps != 96 && p->taps != 128)
        return fail(MSIM_E_UNSUPPORTED, "the library is compiled for taps 32, 64, 96, 128 (got %d)", p->taps);
    if (!(p->kaiser_beta >= 0.0) || !(p->cutoff > 0.0 && p->cutoff <= 0.5))
        return fail(MSIM_E_INVALID_ARG, "kaiser_beta >= 0 and cutoff in (0, 0.5] required");
    const int L = p->table_phases;
    if (L != 0 && (L < 16 || L > 1024 || (L & (L - 1)) != 0))
        return fail(MSIM_E_INVALID_ARG, "table_phases must be 0 (chosen by the planner) or a power of two in 16..1024");
    if (p->n_tiers < 0 || p->n_tiers > 4) return fail(MSIM_E_INVALID_ARG, "n_tiers must be 0..4");
    for (int k = 0; k < p->n_tiers; ++k) {
        if (p->tier_decim[k] < 1 || p->tier_decim[k] > 4096)
            return fail(MSIM_E_INVALID_ARG, "tier_decim must be 1..4096");
        if (k > 0 && p->tier_max_order[k] < p->tier_max_order[k - 1])
            return fail(MSIM_E_INVALID_ARG, "tier_max_order must not decrease");
    }
    if (p->delay_model != MSIM_DELAY_RETARDED && p->delay_model != MSIM_DELAY_INSTANTANEOUS)
        return fail(MSIM_E_INVALID_ARG, "unknown delay_model");
    if (p->fd_kind != MSIM_FD_TABLE && p->fd_kind != MSIM_FD_FARROW) return fail(MSIM_E_INVALID_ARG, "unknown fd_kind");
    if (p->farrow_order < 4 || p->farrow_order > 11) return fail(MSIM_E_INVALID_ARG, "farrow_order must be 4..11");
    if (!(p->knot_slack >= 0.0 && p->knot_slack <= 10.0))
        return fail(MSIM_E_INVALID_ARG, "knot_slack must be in [0, 10] m");
    if (p->adjx_mode != MSIM_ADJX_GATHER && p->adjx_mode != MSIM_ADJX_TRANSPOSE)
        return fail(MSIM_E_INVALID_ARG, "adjx_mode must be MSIM_ADJX_GATHER or MSIM_ADJX_TRANSPOSE");
    if (p->tier_mode != MSIM_TIER_ORDER && p->tier_mode != MSIM_TIER_ADAPTIVE)
        return fail(MSIM_E_INVALID_ARG, "tier_mode must be MSIM_TIER_ORDER or MSIM_TIER_ADAPTIVE");
    if (p->tier_mode == MSIM_TIER_ADAPTIVE && (!(p->tier_tol > 0.0) || p->tier_rmax < 1 || p->tier_rmax > 4096))
        return fail(MSIM_E_INVALID_ARG, "adaptive tiers need tier_tol > 0 and tier_rmax in 1..4096");
    return MSIM_OK;
}

msim_status check_scene(const msim_scene& s, const msim_params* p, int idx)
{
    for (int a = 0; a < 3; ++a)
        if (!(s.size[a] > 0.0) || !std::isfinite(s.size[a]))
            return fail(MSIM_E_INVALID_ARG, "scene %d: room size must be > 0", idx);
    for (int w = 0; w < 6; ++w)
        if (!(s.beta[w] >= 0.0 && s.beta[w] <= 1.0))
            return fail(MSIM_E_INVALID_ARG, "scene %d: beta[%d] outside [0, 1]", idx, w);
    if (s.n_mics < 1 || !s.mic_offset) return fail(MSIM_E_INVALID_ARG, "scene %d: needs >= 1 mic", idx);
    if (s.max_order < 0 || s.max_order > 64) return fail(MSIM_E_INVALID_ARG, "scene %d: max_order in 0..64", idx);
    if (s.n_in < 1 || s.n_out < 1) return fail(MSIM_E_INVALID_ARG, "scene %d: n_in and n_out must be >= 1", idx);
    if (s.n_out > kMaxOut || s.n_in > kMaxOut)
        return fail(MSIM_E_UNSUPPORTED, "scene %d: n_in or n_out above 2^23", idx);
    msim_status st;
    if ((st = check_traj(s.src, s.size, p->c, "source")) != MSIM_OK) return st;
    if ((st = check_traj(s.rcv, s.size, p->c, "receiver")) != MSIM_OK) return st;
    // every knot (or the circle's extent) inside the room; mics too
    auto traj_inside = [&](const msim_traj& tr, const double* off) {
        double q[3];
        if (tr.kind == MSIM_TRAJ_CIRCLE) {
            for (int k = 0; k < 4; ++k) {
                const double ang = k * 0.5 * kPi;
                q[0] = tr.center[0] + tr.radius * std::cos(ang) + (off ? off[0] : 0.0);
                q[1] = tr.center[1] + tr.radius * std::sin(ang) + (off ? off[1] : 0.0);
                q[2] = tr.center[2] + (off ? off[2] : 0.0);
                if (!inside(q, s.size)) return false;
            }
            return true;
        }
        for (int k = 0; k < tr.n_points; ++k) {
            for (int a = 0; a < 3; ++a) q[a] = tr.p[3 * k + a] + (off ? off[a] : 0.0);
            if (!inside(q, s.size)) return false;
        }
        return true;
    };
    if (!traj_inside(s.src, nullptr)) return fail(MSIM_E_OUTSIDE_ROOM, "scene %d: source leaves the room", idx);
    for (int c = 0; c < s.n_mics; ++c)
        if (!traj_inside(s.rcv, s.mic_offset + 3 * c))
            return fail(MSIM_E_OUTSIDE_ROOM, "scene %d: mic %d leaves the room", idx, c);
    // source-mic separation at every knot time of either path (and t = 0)
    std::vector<double> times{0.0};
    if (s.src.kind == MSIM_TRAJ_PWL) times.insert(times.end(), s.src.t, s.src.t + s.src.n_points);
    if (s.rcv.kind == MSIM_TRAJ_PWL) times.insert(times.end(), s.rcv.t, s.rcv.t + s.rcv.n_points);
    for (double t : times) {
        double ps[3], pr[3];
        traj_at(s.src, t, ps);
        traj_at(s.rcv, t, pr);
        for (int c = 0; c < s.n_mics; ++c) {
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double e = ps[a] - pr[a] - s.mic_offset[3 * c + a];
                d2 += e * e;
            }
            if (std::sqrt(d2) < 1e-3) return fail(MSIM_E_TOO_CLOSE, "scene %d: source within 1 mm of mic %d", idx, c);
        }
    }
    return MSIM_OK;
}

int64_t count_images(int K)
{
    // points of the L1 ball: sum over |mx| of the 2D diamond of radius K-|mx|
    int64_t n = 0;
    for (int a = -K; a <= K; ++a) {
        const int r = K - std::abs(a);
        n += 2 * int64_t(r) * r + 2 * r + 1;
    }
    return n;
}

struct HostImage {
    int m[3];
    int hits[6];
    double beta;
    int tier;
    int R;
    double dlo, dhi;   // delay bounds in samples over every mic and time
};

int tier_of(const msim_params* p, int order, int* R)
{
    if (p->n_tiers == 0) {
        *R = 1;
        return 0;
    }
    for (int k = 0; k < p->n_tiers; ++k)
        if (order <= p->tier_max_order[k]) {
            *R = p->tier_decim[k];
            return k;
        }
    *R = p->tier_decim[p->n_tiers - 1];
    return p->n_tiers - 1;
}

// Largest of the adaptive decimations 1, 4, 8, 16, ... not above rmax.
int largest_ladder(int rmax)
{
    int R = 1;
    for (int r = 4; r <= rmax; r *= 2) R = r;
    return R;
}

// Largest speed, acceleration and jerk of a path, and its largest velocity
// change at an inner knot (a PWL path read as samples of a smooth one: that
// change spread over the mean of its two pieces' durations is the acceleration;
// no jerk; a circle: v, v^2/r, v^3/r^2 and no knots).
struct Kin {
    double v = 0.0, a = 0.0, j = 0.0, dv = 0.0;
};

Kin traj_kin(const msim_traj& tr)
{
    Kin k;
    if (tr.kind == MSIM_TRAJ_CIRCLE) {
        k.v = tr.speed;
        k.a = tr.speed * tr.speed / tr.radius;
        k.j = k.a * tr.speed / tr.radius;
        return k;
    }
    std::vector<double> vel;
    for (int i = 0; i + 1 < tr.n_points; ++i) {
        const double dt = tr.t[i + 1] - tr.t[i];
        double s2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double v = (tr.p[3 * (i + 1) + a] - tr.p[3 * i + a]) / dt;
            vel.push_back(v);
            s2 += v * v;
        }
        k.v = std::max(k.v, std::sqrt(s2));
    }
    for (int i = 1; i + 1 < tr.n_points; ++i) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double e = vel[3 * i + a] - vel[3 * (i - 1) + a];
            d2 += e * e;
        }
        k.dv = std::max(k.dv, std::sqrt(d2));
        k.a = std::max(k.a, std::sqrt(d2) / (0.5 * (tr.t[i + 1] - tr.t[i - 1])));
    }
    return k;
}

// Decimation of an image (MSIM_TIER_ADAPTIVE, documented at msim_plan_create):
// d its distance bound (m), beta_i its reflection product; u, a, j, dv the
// relative motion bounds and the largest velocity change at a knot.
int adaptive_decim(const msim_params& p, double u, double a, double j, double dv, double d, double beta_i)
{
    if (beta_i == 0.0) return largest_ladder(p.tier_rmax);
    if (!(d > 0.0)) return 1;
    const double tol = p.tier_tol * std::max(d, 0.1) / beta_i;       // this image's error budget
    const double k3 = ((2.0 / std::sqrt(3.0)) * u * u * u / (d * d) + 3.0 * u * a / d + j) /
                      std::pow(1.0 - u / p.c, 3);
    const double d3 = k3 / (p.c * p.fs * p.fs);
    const double kink = 0.1875 * dv / (p.c - u);
    int R = 1;
    for (int r = 4; r <= p.tier_rmax; r *= 2)
        if ((double)r * r * r * d3 <= 24.0 * tol && (double)r * kink <= tol) R = r;
    return R;
}

// Interval of image coordinates along one axis for source coordinates in [lo, hi].
void image_interval(int m, double L, double lo, double hi, double* out_lo, double* out_hi)
{
    if (m & 1) {
        *out_lo = (m + 1) * L - hi;
        *out_hi = (m + 1) * L - lo;
    } else {
        *out_lo = m * L + lo;
        *out_hi = m * L + hi;
    }
}

// Delay bounds (samples) of image m for a source in box sb and mics in box mb:
// the nearest and farthest points of the image box from the mic box.
void image_bounds(const int m[3], const double L[3], const Box& sb, const Box& mb, double fs, double c, double* dlo,
                  double* dhi)
{
    double dmin2 = 0.0, dmax2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double lo, hi;
        image_interval(m[a], L[a], sb.lo[a], sb.hi[a], &lo, &hi);
        const double gap = std::max(0.0, std::max(lo - mb.hi[a], mb.lo[a] - hi));
        const double far = std::max(std::fabs(hi - mb.lo[a]), std::fabs(mb.hi[a] - lo));
        dmin2 += gap * gap;
        dmax2 += far * far;
    }
    *dlo = fs * std::sqrt(dmin2) / c;
    *dhi = fs * std::sqrt(dmax2) / c;
}

}  // namespace

// ---------------------------------------------------------------- the plan

// One delay block of a scene: its images sorted by the lower bound of their
// delay over the block, with both bounds (samples).
struct BlockOrder {
    std::vector<int32_t> idx;
    std::vector<float> lo, hi;
};

struct msim_plan {
    msim_params par{};
    int n_scenes = 0;
    int threads = 1024;                   // outputs per workgroup (the tile)
    int rb = 1;                           // outputs per lane of the forward (table form: two by
    int rb_max = 1;                       //   default, sharing table rows; Farrow form: one, as
                                          //   occupancy wins over shared segment fetches), and the
                                          //   largest the form and the tier decimations allow
    double err_table = 0.0, err_pair = 0.0, err_farrow = 0.0;   // predicted fractional-delay errors
    bool ugather = false;                 // dL/dx by the Farrow gather (both forms; else the table transpose)
    int slot_segs_fwd = 1, gmax_fwd = 1;  // the forward's slots (block groups only)
    std::vector<DScene> scenes;           // host copies
    std::vector<DImage> images;
    std::vector<DGroup> groups;
    std::vector<double> knots, mics;
    std::vector<double> knots_ref;        // knot positions the delay bounds were planned for
    std::vector<uint8_t> qtable;          // the quadratic FD table: [Y | D1 | D2] bytes
    std::vector<float> atable;            // the same values tap-major (Y, D1, D2 of [T/2][Lq]) for the transpose
    std::vector<int64_t> n_img;
    int64_t src_grad_total = 0;           // knots in the packed d/dsource array
    std::vector<bool> grad_ok;            // the adjoint's LDS fits this scene's windows
    std::vector<std::vector<std::pair<double, double>>> bounds;   // per scene, per image: delay bounds over the whole path
    // Delay blocks: every blk_len outputs of a scene, the images sorted by a lower
    // bound of their delay over the block (from the source's box over the
    // emission times and the mics' box over the block), grouped per tuning.
    int64_t blk_len = 0;
    std::vector<std::vector<BlockOrder>> orders;   // per scene, per block
    std::vector<DBlock> blocks;
    std::vector<PermEntry> perm;
    DBlock* d_blocks = nullptr;
    PermEntry* d_perm = nullptr;
    // work items of the Farrow dL/dx gather (scene, mic, position tile, supergroup of
    // each block's groups); supergroup delay bounds per block (table dL/dx windows)
    std::vector<WorkItem> uitems, uitems_plain;
    std::vector<int> uplain_off, uplain_cnt;
    std::vector<int2> sgb;
    int sgb_stride = 1, uwin = 0, rmax = 1;
    int64_t b_rows = 0, max_rows = 0, b_xw = 0, max_xw = 0, b_upart = 0, max_upart = 0;
    int adj_wgs = 0;
    WorkItem* d_uitems = nullptr;
    WorkItem* d_uitems_plain = nullptr;
    int2* d_sgb = nullptr;
    int64_t* d_x_prefix = nullptr;
    // graph of the batched backward, valid for one argument set
    hipGraphExec_t bgraph_exec = nullptr;
    bool bgraph_valid = false;
    const void* bgraph_key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int group_cap = 0;                    // images per delay group (0: the form's default)
    // work items: every scene's (mic, tile, supergroup) in decreasing-cost order
    // (batched), and per scene (plain: scene s's items at plain_off[s])
    std::vector<DScene> scenes_b;         // with batched partial-output bases set
    std::vector<int64_t> y_prefix;
    std::vector<WorkItem> items, items_plain;
    std::vector<int> plain_off, plain_cnt;
    int64_t b_part_total = 0, max_part = 0;   // partial outputs: all scenes / the largest scene
    int b_window = 0, b_wgs = 0;
    int slot_segs = 0, gmax = 0;          // track slot: segments, and images of the largest group
    DScene* d_scenes_b = nullptr;
    int64_t* d_y_prefix = nullptr;
    int64_t* d_zero = nullptr;
    WorkItem* d_items = nullptr;
    WorkItem* d_items_plain = nullptr;
    // graph of the batched forward, valid for one (x, y, workspace) triple
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_valid = false;
    const void* graph_key[3] = {nullptr, nullptr, nullptr};
    double fwd_taps = 0.0;
    int64_t x_total = 0, y_total = 0;
    // device
    DScene* d_scenes = nullptr;
    DImage* d_images = nullptr;
    DGroup* d_groups = nullptr;
    double* d_knots = nullptr;
    double* d_mics = nullptr;
    float4* d_qtable = nullptr;           // (16-byte aligned bytes of qtable)
    float* d_atable = nullptr;
    std::vector<float> fcoef;             // Farrow coefficients [kFarrowStride][T]
    std::vector<int64_t> vpos_prefix;     // first Farrow source position of each scene
    int64_t vpos_total = 0;
    float* d_fcoef = nullptr;
    int64_t* d_vpos_prefix = nullptr;
    int32_t* d_status = nullptr;
    int device = 0;
    // profiling: (kind, start, stop) per launch while enabled
    bool profiling = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

enum { kKindSynth = 0, kKindReduce, kKindAdjX, kKindAdjP, kKindParams, kKindGraph, kKindFilter, kKinds };

hipEvent_t pool_event(msim_plan* P)
{
    if (!P->pool.empty()) {
        hipEvent_t e = P->pool.back();
        P->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when the plan is profiling.
struct LaunchTimer {
    msim_plan* P;
    hipStream_t st;
    msim_plan::Rec r{};
    bool on;
    LaunchTimer(msim_plan* p, int kind, hipStream_t s) : P(p), st(s), on(p->profiling)
    {
        if (!on) return;
        r.kind = kind;
        r.a = pool_event(P);
        r.b = pool_event(P);
        on = r.a && r.b && hipEventRecord(r.a, st) == hipSuccess;
    }
    ~LaunchTimer()
    {
        if (on && hipEventRecord(r.b, st) == hipSuccess) P->recs.push_back(r);
    }
};

}  // namespace

namespace {

// Quadratic-interpolation half table, grouped by tap quads, as three arrays:
// for quad g and row r in [-1, Lq), Y(r), Y(r+1) - Y(r) (float4 each) and
// Y(r+2) - 2 Y(r+1) + Y(r) (four fp16: it is below 1e-3, so fp16 keeps it to
// ~3e-7 absolute; zero for g >= qcorr_quads(T)), with Y(r) = h((4g+e) + r/Lq),
// e = 0..3 (differences in double),
// stored at row index r + 1 of a quad's qtab_pitch(Lq) rows.  Row -1 serves a lane
// whose two outputs straddle an integer delay (the far side's base row sits one
// below row 0).  qtable holds the bytes [Y | D1 | D2]; y_out, d1_out and d2_out
// return the same values as floats in the same order (the fp16 values as rounded).
void build_qtable(std::vector<uint8_t>& out, std::vector<float>& y_out, std::vector<float>& d1_out,
                  std::vector<float>& d2_out, int T, int Lq, double kbeta, double fc)
{
    const int NG = T / 8, LP = qtab_pitch(Lq);
    const size_t np = (size_t)NG * LP * 4;
    const double i0b = bessel_i0(kbeta);
    y_out.assign(np, 0.0f);
    d1_out.assign(np, 0.0f);
    d2_out.assign(np, 0.0f);
    std::vector<uint16_t> d2h(np, 0);
    for (int g = 0; g < NG; ++g)
        for (int row = -1; row < Lq; ++row)
            for (int e = 0; e < 4; ++e) {
                double y[3];
                for (int i = 0; i < 3; ++i) y[i] = fd_kernel((4 * g + e) + double(row + i) / Lq, T, kbeta, fc, i0b);
                const size_t o = ((size_t)g * LP + row + 1) * 4 + e;
                y_out[o] = (float)y[0];
                d1_out[o] = (float)(y[1] - y[0]);
                const _Float16 h = g < qcorr_quads(T) ? (_Float16)(y[2] - 2.0 * y[1] + y[0]) : (_Float16)0.0;
                std::memcpy(&d2h[o], &h, sizeof h);
                d2_out[o] = (float)h;
            }
    out.resize(np * 4 * 2 + np * 2);
    std::memcpy(out.data(), y_out.data(), np * 4);
    std::memcpy(out.data() + np * 4, d1_out.data(), np * 4);
    std::memcpy(out.data() + np * 8, d2h.data(), np * 2);
}

void build_table(msim_plan* P)
{
    const int T = P->par.taps, Lq = P->par.table_phases, LP = qtab_pitch(Lq);
    std::vector<float> y, d1, d2;
    build_qtable(P->qtable, y, d1, d2, T, Lq, P->par.kaiser_beta, P->par.cutoff);
    // the same values tap-major for the transpose: [Y | D1 | D2] of [T/2][Lq] floats
    // (rows 0 .. Lq-1)
    P->atable.assign((size_t)3 * (T / 2) * Lq, 0.0f);
    const std::vector<float>* src[3] = {&y, &d1, &d2};
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < T / 2; ++d)
            for (int r = 0; r < Lq; ++r)
                P->atable[((size_t)c * (T / 2) + d) * Lq + r] =
                    (*src[c])[((size_t)(d / 4) * LP + r + 1) * 4 + d % 4];
}

// Farrow coefficients: for every tap j = -T/2+1 .. T/2, the degree-M polynomial in
// s = 2 mu - 1 interpolating h(j - mu) at the M+1 Chebyshev points of [-1, 1],
// converted to monomials.  coef[k*T + t], t = j + T/2 - 1; rows k > M are zero.
void build_farrow(msim_plan* P)
{
    const int T = P->par.taps, M = P->par.farrow_order, N = M + 1;
    const double i0b = bessel_i0(P->par.kaiser_beta);
    P->fcoef.assign((size_t)kFarrowStride * T, 0.0f);
    std::vector<std::vector<double>> mono(N, std::vector<double>(N, 0.0));   // T_l(s) = sum_k mono[l][k] s^k
    mono[0][0] = 1.0;
    if (N > 1) mono[1][1] = 1.0;
    for (int l = 2; l < N; ++l)
        for (int k = 0; k < N; ++k)
            mono[l][k] = (k > 0 ? 2.0 * mono[l - 1][k - 1] : 0.0) - mono[l - 2][k];
    std::vector<double> f(N), a(N);
    for (int t = 0; t < T; ++t) {
        const int j = t - T / 2 + 1;
        for (int i = 0; i < N; ++i) {
            const double s = std::cos(kPi * (i + 0.5) / N);
            f[i] = fd_kernel(j - 0.5 * (s + 1.0), T, P->par.kaiser_beta, P->par.cutoff, i0b);
        }
        for (int l = 0; l < N; ++l) {
            double acc = 0.0;
            for (int i = 0; i < N; ++i) acc += f[i] * std::cos(kPi * l * (i + 0.5) / N);
            a[l] = (l == 0 ? 1.0 : 2.0) * acc / N;
        }
        for (int k = 0; k < N; ++k) {
            double c = 0.0;
            for (int l = k; l < N; ++l) c += a[l] * mono[l][k];
            P->fcoef[(size_t)k * T + t] = (float)c;
        }
    }
}

// Predicted relative L2 error of one image's output for a white source signal,
// per approximation of the fractional-delay kernel h (Sec. II-B): the mean square
// over the fractional delay of (approximation - exact h) per tap, summed over the
// T taps, over the kernel's energy (sum of h^2 over the taps).  Both sides of a
// tap window have the same errors, so half the taps are evaluated, twice.
constexpr double kFdErrBudget = 5e-6;   // half the 1e-5 FP32 target

double fd_energy(const msim_params& p)
{
    const double i0b = bessel_i0(p.kaiser_beta);
    double e = 0.0;
    for (int d = 0; d < p.taps / 2; ++d) {
        const double h = fd_kernel(d + 0.5, p.taps, p.kaiser_beta, p.cutoff, i0b);
        e += 2.0 * h * h;
    }
    return e;
}

// The quadratic phase table as stored (FP32 values and first differences, FP16
// second differences, zero beyond qcorr_quads): tap offset d + (r + f) / Lq is
// read as Y + f D1 + f (f - 1) / 2 D2, at eight fractions f per row.
double table_error(const msim_plan* P)
{
    const int T = P->par.taps, Lq = P->par.table_phases, H = T / 2;
    const double i0b = bessel_i0(P->par.kaiser_beta);
    double se = 0.0;
    for (int d = 0; d < H; ++d) {
        double sq = 0.0;
        for (int r = 0; r < Lq; ++r) {
            const double Y = P->atable[(size_t)d * Lq + r];
            const double D1 = P->atable[((size_t)H + d) * Lq + r];
            const double D2 = P->atable[((size_t)2 * H + d) * Lq + r];
            for (int k = 0; k < 8; ++k) {
                const double f = (k + 0.5) / 8.0;
                const double ex = fd_kernel(d + (r + f) / Lq, T, P->par.kaiser_beta, P->par.cutoff, i0b);
                const double ap = Y + f * D1 + 0.5 * f * (f - 1.0) * D2;
                sq += (ap - ex) * (ap - ex);
            }
        }
        se += 2.0 * sq / (8.0 * Lq);
    }
    return std::sqrt(se / fd_energy(P->par));
}

// Two outputs per lane omit the edge tap u in (T/2 - 1, T/2] of the output whose
// integer delay differs from its partner's; that happens for at most a fraction
// |dD/dn| <= 1.5 v / (c - v) of the lanes (v the source plus receiver speed, 1.5
// for the cubic delay interpolation's slope).
double pair_error(const msim_params& p, double v)
{
    const double i0b = bessel_i0(p.kaiser_beta);
    double sq = 0.0;
    for (int k = 0; k < 64; ++k) {
        const double h = fd_kernel(0.5 * p.taps - 1.0 + (k + 0.5) / 64.0, p.taps, p.kaiser_beta, p.cutoff, i0b);
        sq += h * h / 64.0;
    }
    const double frac = std::min(1.0, 1.5 * v / (p.c - v));
    return std::sqrt(frac * sq / fd_energy(p));
}

// The Farrow polynomials (FP32 coefficients, evaluated exactly) against h at 64
// fractional delays per tap.
double farrow_error(const msim_plan* P)
{
    const int T = P->par.taps;
    const double i0b = bessel_i0(P->par.kaiser_beta);
    double se = 0.0;
    for (int t = 0; t < T; ++t) {
        const int j = t - T / 2 + 1;
        for (int k = 0; k < 64; ++k) {
            const double mu = (k + 0.5) / 64.0, sv = 2.0 * mu - 1.0;
            double a = 0.0;
            for (int q = kFarrowStride - 1; q >= 0; --q) a = a * sv + P->fcoef[(size_t)q * T + t];
            const double ex = fd_kernel(j - mu, T, P->par.kaiser_beta, P->par.cutoff, i0b);
            se += (a - ex) * (a - ex) / 64.0;
        }
    }
    return std::sqrt(se / fd_energy(P->par));
}

int push_traj(msim_plan* P, const msim_traj& tr, DTraj* d)
{
    d->kind = tr.kind;
    d->n_points = tr.kind == MSIM_TRAJ_PWL ? tr.n_points : 0;
    d->knot_off = (int)P->knots.size();
    if (tr.kind == MSIM_TRAJ_PWL) {
        P->knots.insert(P->knots.end(), tr.t, tr.t + tr.n_points);
        d->pos_off = (int)P->knots.size();
        P->knots.insert(P->knots.end(), tr.p, tr.p + 3 * tr.n_points);
    } else {
        d->pos_off = d->knot_off;
    }
    for (int a = 0; a < 3; ++a) d->center[a] = tr.center[a];
    d->radius = tr.radius;
    d->omega = tr.kind == MSIM_TRAJ_CIRCLE ? tr.speed / tr.radius : 0.0;
    d->phase0 = tr.phase0;
    return 0;
}

template <typename TT>
msim_status upload(TT** dst, const std::vector<TT>& v)
{
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(TT);
    HIP_OK(hipMalloc((void**)dst, bytes));
    if (!v.empty()) HIP_OK(hipMemcpy(*dst, v.data(), v.size() * sizeof(TT), hipMemcpyHostToDevice));
    return MSIM_OK;
}

// Plan one scene: images sorted by their lower delay bound, split into groups
// of consecutive delays; the group count is raised until the source window of a
// group fits LDS beside the table, and to give enough workgroups.
msim_status plan_scene(msim_plan* P, const msim_scene& s, int si, int64_t x_off, int64_t y_off)
{
    const msim_params& p = P->par;
    const int K = s.max_order;
    std::vector<HostImage> imgs;
    imgs.reserve((size_t)count_images(K));
    Box sb = traj_box(s.src), rb = traj_box(s.rcv);
    const Box sb0 = sb;             // the path itself (adaptive decimations)
    const Kin ks = traj_kin(s.src), kr = traj_kin(s.rcv);
    for (int a = 0; a < 3; ++a) {   // knots may later move by up to the slack
        sb.lo[a] -= p.knot_slack;
        sb.hi[a] += p.knot_slack;
    }
    // receiver box grown by the mic offsets
    Box mb = rb;
    for (int a = 0; a < 3; ++a) {
        double lo = 1e300, hi = -1e300;
        for (int c = 0; c < s.n_mics; ++c) {
            lo = std::min(lo, s.mic_offset[3 * c + a]);
            hi = std::max(hi, s.mic_offset[3 * c + a]);
        }
        mb.lo[a] = rb.lo[a] + lo;
        mb.hi[a] = rb.hi[a] + hi;
    }
    for (int mx = -K; mx <= K; ++mx)
        for (int my = -(K - std::abs(mx)); my <= K - std::abs(mx); ++my) {
            const int rz = K - std::abs(mx) - std::abs(my);
            for (int mz = -rz; mz <= rz; ++mz) {
                HostImage h;
                h.m[0] = mx; h.m[1] = my; h.m[2] = mz;
                double b = 1.0;
                for (int a = 0; a < 3; ++a) {
                    const int m = h.m[a], am = std::abs(m);
                    const int far = m >= 0 ? (am + 1) / 2 : am / 2;
                    const int near = am - far;
                    h.hits[2 * a] = near;
                    h.hits[2 * a + 1] = far;
                    b *= std::pow(s.beta[2 * a], near) * std::pow(s.beta[2 * a + 1], far);
                }
                h.beta = b;
                if (p.tier_mode == MSIM_TIER_ADAPTIVE) {
                    double g2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double lo, hi;
                        image_interval(h.m[a], s.size[a], sb0.lo[a], sb0.hi[a], &lo, &hi);
                        const double gap = std::max(0.0, std::max(lo - mb.hi[a], mb.lo[a] - hi));
                        g2 += gap * gap;
                    }
                    h.tier = 0;
                    h.R = adaptive_decim(p, ks.v + kr.v, ks.a + kr.a, ks.j + kr.j, ks.dv + kr.dv, std::sqrt(g2), b);
                } else {
                    h.tier = tier_of(&p, std::abs(mx) + std::abs(my) + std::abs(mz), &h.R);
                }
                double dmin2 = 0.0, dmax2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double lo, hi;
                    image_interval(h.m[a], s.size[a], sb.lo[a], sb.hi[a], &lo, &hi);
                    const double gap = std::max(0.0, std::max(lo - mb.hi[a], mb.lo[a] - hi));
                    const double far = std::max(std::fabs(hi - mb.lo[a]), std::fabs(mb.hi[a] - lo));
                    dmin2 += gap * gap;
                    dmax2 += far * far;
                }
                h.dlo = p.fs * std::sqrt(dmin2) / p.c;
                h.dhi = p.fs * std::sqrt(dmax2) / p.c;
                imgs.push_back(h);
            }
        }
    std::stable_sort(imgs.begin(), imgs.end(), [](const HostImage& a, const HostImage& b) {
        return a.dlo < b.dlo || (a.dlo == b.dlo && a.dhi < b.dhi);
    });
    const int I = (int)imgs.size();
    DScene d{};
    for (int a = 0; a < 3; ++a) d.size[a] = s.size[a];
    push_traj(P, s.src, &d.src);
    push_traj(P, s.rcv, &d.rcv);
    d.n_mics = s.n_mics;
    d.mic_off = (int)(P->mics.size() / 3);
    P->mics.insert(P->mics.end(), s.mic_offset, s.mic_offset + 3 * s.n_mics);
    d.n_in = s.n_in;
    d.n_out = s.n_out;
    d.x_off = x_off;
    d.y_off = y_off;
    d.img_begin = (int)P->images.size();
    d.n_img = I;
    for (const HostImage& h : imgs) {
        DImage di{};
        for (int a = 0; a < 3; ++a) di.m[a] = (int16_t)h.m[a];
        di.tier = (int16_t)h.tier;
        di.R = h.R;
        di.invR = 1.0f / (float)h.R;
        di.gfac = (float)(h.beta * p.fs / (4.0 * kPi * p.c));
        di.n_seg = (int32_t)((s.n_out + h.R - 1) / h.R);
        for (int w = 0; w < 6; ++w) di.hits[w] = (int8_t)h.hits[w];
        P->images.push_back(di);
    }
    for (int w = 0; w < 6; ++w) d.beta[w] = s.beta[w];
    d.src_grad_off = (int32_t)P->src_grad_total;
    d.src_knots = s.src.kind == MSIM_TRAJ_PWL ? s.src.n_points : 0;
    P->src_grad_total += d.src_knots;
    P->scenes.push_back(d);
    P->n_img.push_back(I);
    std::vector<std::pair<double, double>> bnd((size_t)I);
    for (int i = 0; i < I; ++i) bnd[i] = {imgs[i].dlo, imgs[i].dhi};
    P->bounds.push_back(std::move(bnd));
    P->fwd_taps += (double)s.n_mics * I * double(s.n_in + p.taps - 1) * p.taps;
    return MSIM_OK;
}

// Host view of a device trajectory (its knots in the plan's knot array).
msim_traj host_traj(const msim_plan* P, const DTraj& d)
{
    msim_traj t{};
    t.kind = d.kind;
    t.n_points = d.kind == MSIM_TRAJ_PWL ? d.n_points : 0;
    t.t = d.kind == MSIM_TRAJ_PWL ? P->knots.data() + d.knot_off : nullptr;
    t.p = d.kind == MSIM_TRAJ_PWL ? P->knots.data() + d.pos_off : nullptr;
    for (int a = 0; a < 3; ++a) t.center[a] = d.center[a];
    t.radius = d.radius;
    t.speed = d.omega * d.radius;
    t.phase0 = d.phase0;
    return t;
}

// Orders the images of scene si in each of its delay blocks.  The delay of an
// image at an output of block [t0, t1) (interpolated from grid delays up to two
// decimations outside it) lies within the bounds from the mics' box over the
// padded block and the source's box over the emission times the image's
// whole-path bounds allow.
void order_blocks(msim_plan* P, int si)
{
    const DScene& d = P->scenes[si];
    const msim_traj src = host_traj(P, d.src), rcv = host_traj(P, d.rcv);
    const double fs = P->par.fs, c = P->par.c;
    const int I = d.n_img;
    const int nb = (int)((d.n_out + P->blk_len - 1) / P->blk_len);
    int rmax = 1;
    for (int i = 0; i < I; ++i) rmax = std::max(rmax, P->images[d.img_begin + i].R);
    const double pad = 2.0 * rmax / fs + 1e-6;
    double olo[3], ohi[3];
    for (int a = 0; a < 3; ++a) {
        olo[a] = 1e300;
        ohi[a] = -1e300;
        for (int m = 0; m < d.n_mics; ++m) {
            olo[a] = std::min(olo[a], P->mics[3 * (d.mic_off + m) + a]);
            ohi[a] = std::max(ohi[a], P->mics[3 * (d.mic_off + m) + a]);
        }
    }
    const auto& whole = P->bounds[si];
    std::vector<BlockOrder>& out = P->orders[si];
    out.assign(nb, BlockOrder{});
    std::vector<std::pair<double, int>> key(I);
    std::vector<double> hi(I);
    for (int b = 0; b < nb; ++b) {
        const double t0 = (double)((int64_t)b * P->blk_len) / fs - pad;
        const double t1 = (double)std::min<int64_t>(d.n_out, (int64_t)(b + 1) * P->blk_len) / fs + pad;
        Box mb = traj_box_range(rcv, t0, t1);
        for (int a = 0; a < 3; ++a) {
            mb.lo[a] += olo[a];
            mb.hi[a] += ohi[a];
        }
        for (int i = 0; i < I; ++i) {
            const DImage& im = P->images[d.img_begin + i];
            Box sb = traj_box_range(src, t0 - whole[i].second / fs - 1e-6, t1 - whole[i].first / fs + 1e-6);
            for (int a = 0; a < 3; ++a) {
                sb.lo[a] -= P->par.knot_slack;
                sb.hi[a] += P->par.knot_slack;
            }
            const int m[3] = {im.m[0], im.m[1], im.m[2]};
            double lo, h;
            image_bounds(m, d.size, sb, mb, fs, c, &lo, &h);
            key[i] = {std::max(lo, whole[i].first), i};
            hi[i] = std::min(h, whole[i].second);
        }
        std::sort(key.begin(), key.end());
        BlockOrder& o = out[b];
        o.idx.resize(I);
        o.lo.resize(I);
        o.hi.resize(I);
        for (int j = 0; j < I; ++j) {
            o.idx[j] = key[j].second;
            o.lo[j] = (float)key[j].first;
            o.hi[j] = (float)hi[key[j].second];
        }
    }
}

// Splits every delay block's sorted images into groups for the current tile
// size (threads) and group cap, sizes the LDS windows and track slots, and lays
// out the work items: supergroups, partial-output bases and the cost-ordered
// work lists.
msim_status regroup(msim_plan* P)
{
    const int NT = P->threads, T = P->par.taps, L = P->par.table_phases;
    const bool farrow = P->par.fd_kind == MSIM_FD_FARROW;
    // dL/dx through the Farrow gather: always in the Farrow form; in the table form
    // unless asked for its own transpose, or the Farrow fit misses the budget, or a
    // delay group's gather window does not fit LDS (then the table's transpose is used)
    P->ugather = farrow || (P->par.adjx_mode == MSIM_ADJX_GATHER && P->err_farrow <= kFdErrBudget);
    bool ugather = P->ugather;
    P->groups.clear();
    P->blocks.clear();
    P->perm.clear();
    P->uwin = 0;
    P->grad_ok.clear();
    int slot_segs = 1, gmax = 1, slot_segs_fwd = 1, gmax_fwd = 1;
    for (int s = 0; s < P->n_scenes; ++s) {
        DScene& d = P->scenes[s];
        const int I = d.n_img;
        d.n_tiles = (int)((d.n_out + NT - 1) / NT);
        d.blk_tiles = (int)(P->blk_len / NT);
        d.blk_begin = (int)P->blocks.size();
        d.n_blk = (int)P->orders[s].size();
        // Group windows are sized so the adjoint's LDS (the table beside the source
        // window, or beside the per-wave windows) fits too; failing that, the forward's alone.
        bool grad_fit = true;
        auto fits = [&](int window) {
            if (farrow)
                return farrow_lds_bytes(window) <= kLdsLimit && (!grad_fit || farrow_gd_lds_bytes(window) <= kLdsLimit);
            if (!grad_fit) return synth_lds_bytes(T, L, window) <= kLdsLimit;
            return adj_track_lds_bytes(T, L, window) <= kLdsLimit &&
                   adj_x_lds_bytes(T, L, window, NT) <= kLdsLimit;
        };
        int window = 0;
        for (int b = 0; b < d.n_blk; ++b) {
            const BlockOrder& o = P->orders[s][b];
            // Greedy groups in the block's delay order: an image joins the current
            // group while the group keeps to the image cap (table form 96 images:
            // against 24, the large workload's forward 2 %, dL/dx 7 % and gain/delay
            // 15 % faster, the paper-scale scene's forward 9 %; Farrow form, whose
            // 48-byte window costs more to stage, 256) and its window (tile, delay
            // spread, filter) to the preferred limit: the largest that lets two
            // workgroups share one CU's LDS, unless that leaves more than 2.5 times
            // the cap's group count (a long filter's table leaves room for little
            // delay spread), then the LDS limit.  A gap in the delays (the sparse
            // early reflections) so ends a group where it occurs, and every other
            // group stays full.  An image whose own window exceeds the preferred
            // limit gets a group of its own, up to the LDS limit.
            const int cap = std::min(kMaxGroup, P->group_cap > 0 ? P->group_cap : (farrow ? 256 : 96));
            auto window_of = [&](double lo, double hi) {
                return NT + (((int)std::ceil(hi) + 4) - ((int)std::floor(lo) - 4)) + T + 8;
            };
            auto largest = [&](auto ok) {   // largest window ok() accepts (ok is monotone)
                int lo_w = 0, hi_w = 1 << 22;
                while (lo_w < hi_w) {
                    const int mid = lo_w + (hi_w - lo_w + 1) / 2;
                    if (ok(mid)) lo_w = mid; else hi_w = mid - 1;
                }
                return lo_w;
            };
            std::vector<DGroup> gr;
            int bw = 0;
            for (;;) {
                const int w_full = largest([&](int w) { return fits(w); });
                const int w_half = largest([&](int w) {
                    return fits(w) && (farrow ? farrow_lds_bytes(w) : synth_lds_bytes(T, L, w)) <= kLdsLimit / 2;
                });
                bool ok = true;
                auto greedy = [&](int w_pref) {
                    gr.clear();
                    bw = 0;
                    ok = true;
                    int ib = 0;
                    double glo = o.lo[0], ghi = o.hi[0];
                    for (int i = 1; i <= I; ++i) {
                        const bool join =
                            i < I && i - ib < cap && window_of(glo, std::max(ghi, (double)o.hi[i])) <= w_pref;
                        if (join) {
                            ghi = std::max(ghi, (double)o.hi[i]);
                            continue;
                        }
                        const int wg = window_of(glo, ghi);
                        if (wg > w_full) ok = false;
                        gr.push_back(DGroup{ib, i, (int)std::floor(glo) - 4, (int)std::ceil(ghi) + 4});
                        bw = std::max(bw, wg);
                        if (i < I) {
                            ib = i;
                            glo = o.lo[i];
                            ghi = o.hi[i];
                        }
                    }
                };
                greedy(w_half);
                if (gr.size() * 2 > (size_t)5 * ((I + cap - 1) / cap)) greedy(w_full);
                if (ok) break;
                if (!grad_fit) return fail(MSIM_E_UNSUPPORTED, "scene %d: one image's delay span exceeds LDS", s);
                grad_fit = false;
            }
            // groups whose tracks exceed a slot of kSlotSegCap segments (audio-rate
            // images hold a tile's worth each) are split into consecutive parts
            {
                std::vector<DGroup> out;
                for (const DGroup& g : gr) {
                    const int span = group_span(NT, g.dmin, g.dmax);
                    int ib = g.img_begin;
                    int64_t segs = 0;
                    for (int i = g.img_begin; i <= g.img_end; ++i) {
                        const int add = i < g.img_end ? slot_segs_of(P->images[d.img_begin + o.idx[i]].R, span) : 0;
                        if (i == g.img_end || (segs + add > kSlotSegCap && i > ib)) {
                            double lo = 1e300, hi = -1e300;
                            for (int k = ib; k < i; ++k) {
                                lo = std::min(lo, (double)o.lo[k]);
                                hi = std::max(hi, (double)o.hi[k]);
                            }
                            out.push_back(DGroup{ib, i, (int)std::floor(lo) - 4, (int)std::ceil(hi) + 4});
                            ib = i;
                            segs = 0;
                        }
                        segs += add;
                    }
                }
                gr.swap(out);
            }
            window = std::max(window, bw);
            P->blocks.push_back(DBlock{(int)P->groups.size(), (int)gr.size()});
            // permutation entries with their slot offsets: slot_segs_of(R, span)
            // segments per image, span the group's tile plus its delay spread
            for (DGroup g : gr) {
                const int span = group_span(NT, g.dmin, g.dmax);
                const int base = (int)P->perm.size();
                int64_t loc = 0;
                for (int i = g.img_begin; i < g.img_end; ++i) {
                    const int img = o.idx[i];
                    P->perm.push_back(PermEntry{img, (int32_t)loc});
                    loc += slot_segs_of(P->images[d.img_begin + img].R, span);
                }
                if (loc > INT32_MAX / 4)
                    return fail(MSIM_E_UNSUPPORTED, "scene %d: a delay group's tracks exceed a slot", s);
                slot_segs_fwd = std::max(slot_segs_fwd, (int)loc);
                gmax_fwd = std::max(gmax_fwd, g.img_end - g.img_begin);
                g.img_end = base + (g.img_end - g.img_begin);
                g.img_begin = base;
                P->groups.push_back(g);
            }
        }
        if (P->perm.size() > (size_t)INT32_MAX) return fail(MSIM_E_UNSUPPORTED, "too many delay-block entries");
        P->grad_ok.push_back(grad_fit);
        d.window = window;
        d.dlo_all = INT32_MAX;
        d.dhi_all = INT32_MIN;
        for (int g = P->blocks[d.blk_begin].grp_begin; g < (int)P->groups.size(); ++g) {
            d.dlo_all = std::min(d.dlo_all, P->groups[g].dmin);
            d.dhi_all = std::max(d.dhi_all, P->groups[g].dmax);
        }
        // the dL/dx gather takes the block groups too: per position tile, the
        // outputs of each block that can read it; its window is the group's spread
        // plus the position tile
        if (ugather)
            for (int g = P->blocks[d.blk_begin].grp_begin; g < (int)P->groups.size(); ++g)
                P->uwin = std::max(P->uwin, kAdjThreads + (P->groups[g].dmax - P->groups[g].dmin) + 9);
    }
    if (farrow_u_lds_bytes(std::max(1, P->uwin)) > kLdsLimit) {
        if (farrow) return fail(MSIM_E_UNSUPPORTED, "a delay group's gather window exceeds LDS");
        ugather = false;   // the table form falls back to its own transpose
    }
    if (P->ugather && !ugather) {
        P->ugather = false;
        P->uwin = 0;
    }
    P->slot_segs = std::max(slot_segs, slot_segs_fwd);
    P->gmax = std::max(gmax, gmax_fwd);
    P->slot_segs_fwd = slot_segs_fwd;
    P->gmax_fwd = gmax_fwd;
    // Supergroups: a work item sums the groups of one supergroup of one (mic, tile)
    // in registers and writes one partial output row.  Each scene gets items
    // enough to fill the persistent grid several times on its own (the plain path
    // runs scenes one at a time), as long as all partial outputs stay within 2 GiB.
    const int64_t want = 8 * 512;
    std::vector<int> nsg(P->n_scenes);
    int64_t total = 0;
    for (int s = 0; s < P->n_scenes; ++s) {
        const DScene& d = P->scenes[s];
        const int64_t tm = std::max<int64_t>(1, (int64_t)d.n_tiles * d.n_mics);
        int min_grp = INT32_MAX;
        for (int b = 0; b < d.n_blk; ++b) min_grp = std::min(min_grp, P->blocks[d.blk_begin + b].n_grp);
        nsg[s] = (int)std::min<int64_t>(min_grp, std::max<int64_t>(1, (want + tm - 1) / tm));
        total += (int64_t)d.n_mics * d.n_out * nsg[s];
    }
    const int64_t budget = (int64_t)1 << 29;
    if (total > budget)
        for (int s = 0; s < P->n_scenes; ++s) nsg[s] = (int)std::max<int64_t>(1, (int64_t)nsg[s] * budget / total);
    P->scenes_b = P->scenes;
    P->y_prefix.assign(P->n_scenes, 0);
    int64_t po = 0, pmax = 0;
    int wmax = 0;
    for (int s = 0; s < P->n_scenes; ++s) {
        DScene& d = P->scenes[s];
        d.n_sg = nsg[s];
        d.part_base = 0;
        DScene& b = P->scenes_b[s];
        b.n_sg = d.n_sg;
        b.part_base = po;
        P->y_prefix[s] = b.y_off;
        const int64_t pr = (int64_t)b.n_mics * b.n_sg * b.n_out;
        po += pr;
        pmax = std::max(pmax, pr);
        wmax = std::max(wmax, b.window);
    }
    P->b_part_total = po;
    P->max_part = pmax;
    P->b_window = wmax;
    std::vector<std::pair<double, WorkItem>> it;
    P->plain_off.assign(P->n_scenes, 0);
    P->plain_cnt.assign(P->n_scenes, 0);
    P->items_plain.clear();
    for (int s = 0; s < P->n_scenes; ++s) {
        const DScene& d = P->scenes[s];
        std::vector<std::pair<double, WorkItem>> its;
        for (int t = 0; t < d.n_tiles; ++t) {
            const DBlock& B = P->blocks[d.blk_begin + t / d.blk_tiles];
            const int64_t len = std::min<int64_t>(NT, d.n_out - (int64_t)t * NT);
            for (int sg = 0; sg < d.n_sg; ++sg) {
                const int gb = sg_begin(B.n_grp, d.n_sg, sg), ge = sg_begin(B.n_grp, d.n_sg, sg + 1);
                double per_out = 0.0, stage = 0.0;
                for (int g = gb; g < ge; ++g) {
                    const DGroup& G = P->groups[B.grp_begin + g];
                    per_out += (double)(G.img_end - G.img_begin) * T;
                    stage += 4.0 * (NT + (G.dmax - G.dmin) + T + 8);
                }
                for (int m = 0; m < d.n_mics; ++m) its.push_back({per_out * len + stage, WorkItem{s, m, t, sg}});
            }
        }
        std::stable_sort(its.begin(), its.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
        P->plain_off[s] = (int)P->items_plain.size();
        P->plain_cnt[s] = (int)its.size();
        for (const auto& e : its) P->items_plain.push_back(e.second);
        it.insert(it.end(), its.begin(), its.end());
    }
    if (it.size() > (size_t)INT32_MAX) return fail(MSIM_E_UNSUPPORTED, "too many work items");
    std::stable_sort(it.begin(), it.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    P->items.resize(it.size());
    for (size_t i = 0; i < it.size(); ++i) P->items[i] = it[i].second;
    const size_t lds =
        P->par.fd_kind == MSIM_FD_FARROW ? farrow_lds_bytes(wmax) : synth_lds_bytes(T, L, wmax);
    const int wg_threads = NT / P->rb;
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(2048 / wg_threads, kLdsLimit / lds));
    P->b_wgs = (int)std::min<int64_t>((int64_t)256 * per_cu, (int64_t)P->items.size());

    // ---- backward layout
    // supergroup delay bounds per block (the table dL/dx windows)
    P->sgb_stride = 1;
    for (const DScene& d : P->scenes) P->sgb_stride = std::max(P->sgb_stride, d.n_sg);
    P->sgb.assign(P->blocks.size() * (size_t)P->sgb_stride, make_int2(0, 0));
    P->rmax = 1;
    for (const DImage& im : P->images) P->rmax = std::max(P->rmax, im.R);
    int64_t rows = 0, xw = 0, up = 0;
    P->max_rows = P->max_xw = P->max_upart = 0;
    P->uitems.clear();
    P->uitems_plain.clear();
    P->uplain_off.assign(P->n_scenes, 0);
    P->uplain_cnt.assign(P->n_scenes, 0);
    std::vector<std::pair<double, WorkItem>> uit;
    for (int s = 0; s < P->n_scenes; ++s) {
        DScene& d = P->scenes[s];
        DScene& b = P->scenes_b[s];
        int xs = 0;
        for (int k = 0; k < d.n_blk; ++k) {
            const DBlock& B = P->blocks[d.blk_begin + k];
            for (int sg = 0; sg < d.n_sg; ++sg) {
                const int gb = sg_begin(B.n_grp, d.n_sg, sg), ge = sg_begin(B.n_grp, d.n_sg, sg + 1);
                int lo = INT32_MAX, hi = INT32_MIN;
                for (int g = gb; g < ge; ++g) {
                    lo = std::min(lo, P->groups[B.grp_begin + g].dmin);
                    hi = std::max(hi, P->groups[B.grp_begin + g].dmax);
                }
                P->sgb[(size_t)(d.blk_begin + k) * P->sgb_stride + sg] = make_int2(lo, hi);
                xs = std::max(xs, NT + (hi - lo) + T + 8);
            }
        }
        d.sgb_stride = b.sgb_stride = P->sgb_stride;
        d.xw_stride = b.xw_stride = xs;
        const int64_t nr = (int64_t)d.n_mics * d.n_sg * d.n_tiles;
        const int64_t nx = P->ugather ? 0 : nr * xs;
        // dL/dx gather: items per (mic, position tile, share of each block's groups)
        d.n_ptiles = b.n_ptiles = (int)((d.n_in + T + kAdjThreads - 1) / kAdjThreads);
        int nsgw = 0;
        if (P->ugather) {
            int gmax_blk = 1;
            for (int k = 0; k < d.n_blk; ++k) gmax_blk = std::max(gmax_blk, P->blocks[d.blk_begin + k].n_grp);
            const int64_t tm = std::max<int64_t>(1, (int64_t)d.n_ptiles * d.n_mics);
            nsgw = (int)std::min<int64_t>(gmax_blk, std::max<int64_t>(1, (want + tm - 1) / tm));
            const int64_t per = (int64_t)d.n_mics * (d.n_in + T) * kFarrowStride;
            nsgw = (int)std::max<int64_t>(1, std::min<int64_t>(nsgw, budget / std::max<int64_t>(1, per * P->n_scenes)));
        }
        d.n_sgw = b.n_sgw = nsgw;
        const int64_t nu = P->ugather ? (int64_t)d.n_mics * nsgw * (d.n_in + T) * kFarrowStride : 0;
        d.row_base = 0;
        d.xw_base = 0;
        d.u_base = 0;
        b.row_base = rows;
        b.xw_base = xw;
        b.u_base = up;
        rows += nr;
        xw += nx;
        up += nu;
        P->max_rows = std::max(P->max_rows, nr);
        P->max_xw = std::max(P->max_xw, nx);
        P->max_upart = std::max(P->max_upart, nu);
        if (P->ugather) {
            std::vector<std::pair<double, WorkItem>> its;
            for (int sg = 0; sg < nsgw; ++sg)
                for (int m = 0; m < d.n_mics; ++m)
                    for (int t = 0; t < d.n_ptiles; ++t) its.push_back({(double)d.n_img, WorkItem{s, m, t, sg}});
            P->uplain_off[s] = (int)P->uitems_plain.size();
            P->uplain_cnt[s] = (int)its.size();
            for (const auto& e : its) P->uitems_plain.push_back(e.second);
            uit.insert(uit.end(), its.begin(), its.end());
        }
        b.dlo_all = d.dlo_all;
        b.dhi_all = d.dhi_all;
    }
    std::stable_sort(uit.begin(), uit.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
    for (const auto& e : uit) P->uitems.push_back(e.second);
    P->b_rows = rows;
    P->b_xw = xw;
    P->b_upart = up;
    // persistent grid of the backward kernels: the largest any of them runs
    {
        auto grid = [&](size_t l, int threads) {
            return 256 * (int)std::max<size_t>(1, std::min<size_t>(2048 / threads, kLdsLimit / std::max<size_t>(1, l)));
        };
        int g = 1;
        if (P->ugather)
            g = std::max(g, grid(farrow_u_lds_bytes(std::max(1, P->uwin)), kAdjThreads));
        else
            g = std::max(g, grid(adj_x_lds_bytes(T, L, wmax, NT), kAdjThreads));
        if (farrow)
            g = std::max(g, grid(farrow_gd_lds_bytes(wmax), kAdjThreads));
        else
            g = std::max(g, grid(adj_track_lds_bytes(T, L, wmax), P->rb == 1 ? kAdjThreads : NT / 2));
        P->adj_wgs = g;
    }
    P->graph_valid = false;
    P->bgraph_valid = false;
    return MSIM_OK;
}

void free_layout(msim_plan* P)
{
    (void)hipFree(P->d_scenes);
    (void)hipFree(P->d_groups);
    (void)hipFree(P->d_scenes_b);
    (void)hipFree(P->d_y_prefix);
    (void)hipFree(P->d_items);
    (void)hipFree(P->d_items_plain);
    (void)hipFree(P->d_blocks);
    (void)hipFree(P->d_perm);
    (void)hipFree(P->d_uitems);
    (void)hipFree(P->d_uitems_plain);
    (void)hipFree(P->d_sgb);
    P->d_blocks = nullptr;
    P->d_perm = nullptr;
    P->d_uitems = P->d_uitems_plain = nullptr;
    P->d_sgb = nullptr;
    P->d_scenes = nullptr;
    P->d_groups = nullptr;
    P->d_scenes_b = nullptr;
    P->d_y_prefix = nullptr;
    P->d_items = P->d_items_plain = nullptr;
}

// (Re)uploads everything regroup() decides: scene descriptors, groups, the images
// (their slot offsets), the batched descriptors, prefix arrays and the work lists.
msim_status upload_layout(msim_plan* P)
{
    free_layout(P);
    msim_status st;
    if ((st = upload(&P->d_scenes, P->scenes)) != MSIM_OK || (st = upload(&P->d_groups, P->groups)) != MSIM_OK ||
        (st = upload(&P->d_scenes_b, P->scenes_b)) != MSIM_OK ||
        (st = upload(&P->d_y_prefix, P->y_prefix)) != MSIM_OK || (st = upload(&P->d_items, P->items)) != MSIM_OK ||
        (st = upload(&P->d_items_plain, P->items_plain)) != MSIM_OK ||
        (st = upload(&P->d_blocks, P->blocks)) != MSIM_OK || (st = upload(&P->d_perm, P->perm)) != MSIM_OK ||
        (st = upload(&P->d_uitems, P->uitems)) != MSIM_OK ||
        (st = upload(&P->d_uitems_plain, P->uitems_plain)) != MSIM_OK || (st = upload(&P->d_sgb, P->sgb)) != MSIM_OK)
        return st;
    if (P->d_images)
        HIP_OK(hipMemcpy(P->d_images, P->images.data(), P->images.size() * sizeof(DImage), hipMemcpyHostToDevice));
    return MSIM_OK;
}

PlanView plan_view(const msim_plan* P, const DScene* scenes)
{
    return PlanView{scenes, P->d_images, P->d_blocks, P->d_groups, P->d_perm};
}

// Bytes of one workgroup's track slot for the forward.
int64_t fwd_slot_bytes(const msim_plan* P) { return slot_extra_off(P->slot_segs_fwd, P->gmax_fwd); }

TrackArgs track_args(const msim_plan* P, char* slots, int64_t slot_bytes, bool fwd)
{
    TrackArgs ta;
    ta.knots = P->d_knots;
    ta.mics = P->d_mics;
    ta.c = P->par.c;
    ta.fs = P->par.fs;
    ta.model = P->par.delay_model;
    ta.slot_segs = fwd ? P->slot_segs_fwd : P->slot_segs;
    ta.slots = slots;
    ta.slot_bytes = slot_bytes;
    return ta;
}

// Farrow-filtered source signals of every scene, ahead of the per-scene scratch.
size_t farrow_v_bytes(const msim_plan* P)
{
    return P->par.fd_kind == MSIM_FD_FARROW ? align_up((size_t)P->vpos_total * kFarrowStride * sizeof(float)) : 0;
}

// Forward workspace: the Farrow-filtered sources (Farrow form), one track slot
// per persistent workgroup, the partial outputs of every scene (batched) or of the
// largest scene (plain: scenes run one after another), and the ticket counter.
struct FwdWs2 {
    float* v;
    char* slots;
    float* part;
    int32_t* ticket;
};

size_t carve_fwd_ws(const msim_plan* P, bool batched, char* base, FwdWs2* w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    char* v = take(farrow_v_bytes(P));
    char* sl = take((size_t)P->b_wgs * (size_t)fwd_slot_bytes(P));
    char* pa = take((size_t)(batched ? P->b_part_total : P->max_part) * sizeof(float));
    char* t = take(sizeof(int32_t));
    if (w) {
        w->v = (float*)v;
        w->slots = sl;
        w->part = (float*)pa;
        w->ticket = (int32_t*)t;
    }
    return off;
}

// The forward's launches: the Farrow filter bank (Farrow form), then the
// persistent synthesis and the supergroup reduction, over every scene at once
// (batched) or scene by scene (plain).
msim_status enqueue_forward(msim_plan* P, const float* x, float* y, const FwdWs2& w, bool batched, hipStream_t st)
{
    const bool farrow = P->par.fd_kind == MSIM_FD_FARROW;
    const TrackArgs ta = track_args(P, w.slots, fwd_slot_bytes(P), true);
    if (farrow) {
        LaunchTimer t(P, kKindFilter, st);
        HIP_OK(launch_farrow_conv(P->d_scenes, P->n_scenes, P->d_vpos_prefix, P->vpos_total, P->par.taps,
                                  P->d_fcoef, x, w.v, st));
    }
    auto run = [&](const DScene* scenes, const WorkItem* items, int n_items, int n_wg) -> msim_status {
        LaunchTimer t(P, kKindSynth, st);
        const PlanView pv = plan_view(P, scenes);
        if (farrow)
            HIP_OK(launch_farrow(P->threads, P->rb, n_wg, P->b_window, P->par.taps, P->par.farrow_order, pv, items,
                                 n_items, w.ticket, ta, w.v, w.part, P->d_status, st));
        else
            HIP_OK(launch_synth(P->par.taps, P->threads, P->rb, n_wg, P->b_window, pv, P->d_qtable,
                                P->par.table_phases, items, n_items, w.ticket, ta, x, w.part, P->d_status, st));
        return MSIM_OK;
    };
    msim_status s;
    if (batched) {
        if ((s = run(P->d_scenes_b, P->d_items, (int)P->items.size(), P->b_wgs)) != MSIM_OK) return s;
        LaunchTimer t(P, kKindReduce, st);
        HIP_OK(launch_reduce_sg(P->d_scenes_b, P->n_scenes, P->d_y_prefix, P->y_total, w.part, y, st));
        return MSIM_OK;
    }
    for (int sc = 0; sc < P->n_scenes; ++sc) {
        const int cnt = P->plain_cnt[sc];
        if ((s = run(P->d_scenes, P->d_items_plain + P->plain_off[sc], cnt, std::min(cnt, P->b_wgs))) != MSIM_OK)
            return s;
        const DScene& d = P->scenes[sc];
        LaunchTimer t(P, kKindReduce, st);
        HIP_OK(launch_reduce_sg(P->d_scenes + sc, 1, P->d_zero, (int64_t)d.n_mics * d.n_out, w.part, y, st));
    }
    return MSIM_OK;
}

// Backward workspace: the Farrow-filtered sources and the gathered sums u
// (Farrow form), one adjoint slot per persistent workgroup, the dL/dx windows
// (table form) or the partial sums u (Farrow form), the rows of parameter
// partials, and the ticket counter; all scenes' (batched) or the largest scene's
// (plain).
struct BwdWs {
    float* v;
    float* u;
    char* slots;
    float* xwin;
    float* upart;
    double* rows;
    int32_t* ticket;
};

int64_t adj_slot_size(const msim_plan* P) { return adj_slot_bytes(P->slot_segs, P->gmax, P->threads); }

// Outputs per lane of the Farrow gain/delay adjoint: two where the tile is two
// lanes' worth and every decimation is 1 or even (a lane's outputs then share a
// track segment), else one.
int farrow_gd_rb(const msim_plan* P)
{
    return P->threads == 2 * kAdjThreads && P->rb_max % 2 == 0 ? 2 : 1;
}

size_t carve_bwd_ws(const msim_plan* P, bool batched, char* base, BwdWs* w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    char* v = take(farrow_v_bytes(P));
    char* u = take(P->ugather ? align_up((size_t)P->vpos_total * kFarrowStride * sizeof(float)) : 0);
    char* sl = take((size_t)P->adj_wgs * (size_t)adj_slot_size(P));
    char* xw = take((size_t)(batched ? P->b_xw : P->max_xw) * sizeof(float));
    char* up = take((size_t)(batched ? P->b_upart : P->max_upart) * sizeof(float));
    char* r = take((size_t)(batched ? P->b_rows : P->max_rows) * kRowWidth * sizeof(double));
    char* t = take(sizeof(int32_t));
    if (w) {
        w->v = (float*)v;
        w->u = (float*)u;
        w->slots = sl;
        w->xwin = (float*)xw;
        w->upart = (float*)up;
        w->rows = (double*)r;
        w->ticket = (int32_t*)t;
    }
    return off;
}

msim_status check_backward(msim_plan* P, const float* x, const float* gy, double* gsrc)
{
    if (!P || !x || !gy) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != P->device) return fail(MSIM_E_INVALID_ARG, "plan was created on device %d, current is %d", P->device, dev);
    for (int s = 0; s < P->n_scenes; ++s) {
        if (!P->grad_ok[s]) return fail(MSIM_E_UNSUPPORTED, "scene %d: adjoint LDS does not fit its delay groups", s);
        if (gsrc && P->scenes[s].src_knots > max_grad_knots())
            return fail(MSIM_E_UNSUPPORTED, "scene %d: more than %d source knots", s, max_grad_knots());
    }
    return MSIM_OK;
}

// The backward's launches, over every scene at once (batched) or scene by scene
// (plain): dL/dx (table: the transpose delay into windows, then their gather;
// Farrow: the gathered sums u, their reduction and the transposed filter bank),
// then the gain/delay adjoint with the in-tile parameter reductions and the
// reduction of the rows.
msim_status enqueue_backward(msim_plan* P, const float* x, const float* gy, float* gx, double* gbeta, double* gsrc,
                             const BwdWs& w, bool batched, hipStream_t st)
{
    const bool farrow = P->par.fd_kind == MSIM_FD_FARROW;
    const int T = P->par.taps, L = P->par.table_phases, NT = P->threads;
    const TrackArgs ta = track_args(P, w.slots, adj_slot_size(P), false);
    ParamArgs pa;
    pa.rows = w.rows;
    pa.gmax = P->gmax;
    pa.rmax = P->rmax;
    pa.ghat = (float)(P->par.fs / (4.0 * kPi * P->par.c));
    pa.want_beta = gbeta != nullptr;
    pa.want_src = gsrc != nullptr;
    const bool want_p = gbeta || gsrc;
    if (farrow && want_p) {
        LaunchTimer t(P, kKindFilter, st);
        HIP_OK(launch_farrow_conv(P->d_scenes, P->n_scenes, P->d_vpos_prefix, P->vpos_total, T, P->d_fcoef, x, w.v,
                                  st));
    }
    const int ns = batched ? 1 : P->n_scenes;
    for (int k = 0; k < ns; ++k) {
        const DScene* scenes = batched ? P->d_scenes_b : P->d_scenes + k;
        const PlanView pv = plan_view(P, batched ? P->d_scenes_b : P->d_scenes);
        const int nsc = batched ? P->n_scenes : 1;
        const int64_t* xpre = batched ? P->d_x_prefix : P->d_zero;
        const int64_t xtot = batched ? P->x_total : P->scenes[k].n_in;
        PlanView one = pv;
        one.scenes = scenes;
        if (gx) {
            LaunchTimer t(P, kKindAdjX, st);
            if (P->ugather) {
                const WorkItem* it = batched ? P->d_uitems : P->d_uitems_plain + P->uplain_off[k];
                const int n = batched ? (int)P->uitems.size() : P->uplain_cnt[k];
                HIP_OK(launch_farrow_u(kAdjThreads, std::min(n, P->adj_wgs), P->uwin, T, P->par.farrow_order, NT, pv,
                                       it, n, w.ticket, ta, gy, w.upart, P->d_status, st));
                const int64_t vtot = batched ? P->vpos_total : P->scenes[k].n_in + T;
                HIP_OK(launch_farrow_u_reduce(one, nsc, batched ? P->d_vpos_prefix : P->d_zero, vtot, T, w.upart,
                                              w.u, st));
                int64_t max_in = 0;
                for (int s = 0; s < P->n_scenes; ++s)
                    if (batched || s == k) max_in = std::max(max_in, P->scenes[s].n_in);
                HIP_OK(launch_farrow_corr(pv, batched ? 0 : k, nsc, max_in, T, P->d_fcoef, w.u, gx, st));
            } else {
                const WorkItem* it = batched ? P->d_items : P->d_items_plain + P->plain_off[k];
                const int n = batched ? (int)P->items.size() : P->plain_cnt[k];
                HIP_OK(launch_adjx(T, NT, std::min(n, P->adj_wgs), P->b_window, pv, P->d_atable, L, it, n, w.ticket,
                                   ta, gy, w.xwin, P->d_status, st));
                HIP_OK(launch_reduce_x(one, nsc, xpre, xtot, NT, T, P->d_sgb, w.xwin, gx, st));
            }
        }
        if (want_p) {
            const WorkItem* it = batched ? P->d_items : P->d_items_plain + P->plain_off[k];
            const int n = batched ? (int)P->items.size() : P->plain_cnt[k];
            {
                LaunchTimer t(P, kKindAdjP, st);
                if (farrow)
                    HIP_OK(launch_farrow_gd(NT, farrow_gd_rb(P), std::min(n, P->adj_wgs), P->b_window, T,
                                            P->par.farrow_order, pv, it, n, w.ticket, ta, w.v, gy, pa, P->d_status,
                                            st));
                else
                    HIP_OK(launch_adjp(T, NT, P->rb, std::min(n, P->adj_wgs), P->b_window, pv, P->d_qtable, L, it, n,
                                       w.ticket, ta, x, gy, pa, P->d_status, st));
            }
            LaunchTimer t(P, kKindParams, st);
            HIP_OK(launch_reduce_rows(one, nsc, batched ? 0 : k, w.rows, gbeta, gsrc, st));
        }
    }
    return MSIM_OK;
}

}  // namespace

// ------------------------------------------------------------------ C-ABI

extern "C" {

const char* msim_last_error(void) { return g_err.c_str(); }

msim_status msim_default_params(msim_params* p)
{
    if (!p) return fail(MSIM_E_INVALID_ARG, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->c = 343.0;
    p->fs = 16000.0;
    p->taps = 64;
    p->kaiser_beta = 8.0;
    p->cutoff = 0.5;
    p->table_phases = 0;
    p->n_tiers = 3;
    p->tier_max_order[0] = 2;
    p->tier_decim[0] = 1;
    p->tier_max_order[1] = 6;
    p->tier_decim[1] = 16;
    p->tier_max_order[2] = 1 << 20;
    p->tier_decim[2] = 160;
    p->delay_model = MSIM_DELAY_RETARDED;
    p->fd_kind = MSIM_FD_TABLE;
    p->farrow_order = 9;
    p->knot_slack = 0.0;
    p->tier_mode = MSIM_TIER_ORDER;
    p->tier_tol = 1e-3;
    p->tier_rmax = 1024;
    p->adjx_mode = MSIM_ADJX_GATHER;
    return MSIM_OK;
}

msim_status msim_count_images(int32_t max_order, int64_t* n)
{
    if (!n || max_order < 0 || max_order > 64) return fail(MSIM_E_INVALID_ARG, "max_order in 0..64, n non-NULL");
    *n = count_images(max_order);
    return MSIM_OK;
}

msim_status msim_suggest_n_out(const msim_scene* s, const msim_params* p, int64_t* n_out)
{
    if (!s || !n_out) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    msim_status st = check_params(p);
    if (st != MSIM_OK) return st;
    if (s->max_order < 0 || s->n_in < 1) return fail(MSIM_E_INVALID_ARG, "max_order >= 0 and n_in >= 1 required");
    // farthest image cell of order <= K: all of the order on the longest axis
    double L[3] = {s->size[0], s->size[1], s->size[2]};
    std::sort(L, L + 3);
    const double d = std::sqrt(std::pow(L[2] * (s->max_order + 1), 2) + L[1] * L[1] + L[0] * L[0]);
    *n_out = s->n_in + (int64_t)std::ceil(p->fs * d / p->c) + p->taps;
    return MSIM_OK;
}

msim_status msim_plan_create(const msim_scene* scenes, int32_t n_scenes, const msim_params* p, msim_plan** out)
{
    if (!out) return fail(MSIM_E_INVALID_ARG, "plan pointer is NULL");
    *out = nullptr;
    if (!scenes || n_scenes < 1) return fail(MSIM_E_INVALID_ARG, "need >= 1 scene");
    msim_status st = check_params(p);
    if (st != MSIM_OK) return st;
    for (int s = 0; s < n_scenes; ++s)
        if ((st = check_scene(scenes[s], p, s)) != MSIM_OK) return st;
    msim_plan* P = new msim_plan();
    P->par = *p;
    {
        // adaptive decimations are 1 or multiples of 4
        const int32_t four[1] = {4};
        P->rb_max = p->tier_mode == MSIM_TIER_ADAPTIVE ? farrow_outputs_per_lane(four, 1)
                                                        : farrow_outputs_per_lane(p->tier_decim, p->n_tiers);
    }
    if (p->fd_kind != MSIM_FD_FARROW) {
        // Two outputs per lane read the table rows of the earlier one: fine while
        // the delay drifts by well under two rows per sample.  An image moves no
        // faster than its source, so |dD/dn| <= v / (c - v) with v the source plus
        // receiver speed; allowing 1.5x for the cubic delay interpolation's slope,
        // the pair is used up to 1.25 rows per sample (the quadratic then reads at
        // fractions within [-0.25, 2.25], at most 1.8x its interpolation error).
        double v = 0.0;
        for (int s = 0; s < n_scenes; ++s)
            v = std::max(v, traj_max_speed(scenes[s].src) + traj_max_speed(scenes[s].rcv));
        auto pair_fits = [&](int L) { return 1.5 * v / (p->c - v) * L <= 1.25; };
        P->err_pair = pair_error(*p, v);
        if (p->table_phases == 0) {
            // Phases chosen by the planner: 128 (compiled in) where the pair fits
            // there; else 64 where the pair fits at 64 and the coarser table plus the
            // pair's edge tap stay within the error budget (the pair halves the
            // table and source reads per tap); else 128 at one output per lane.
            P->par.table_phases = kTablePhases;
            if (P->rb_max >= 2 && !pair_fits(kTablePhases) && pair_fits(kPairTablePhases)) {
                P->par.table_phases = kPairTablePhases;
                build_table(P);
                if (std::hypot(table_error(P), P->err_pair) > kFdErrBudget) P->par.table_phases = kTablePhases;
            }
        }
        P->rb_max = pair_fits(P->par.table_phases) ? std::min(P->rb_max, 2) : 1;
    }
    build_table(P);
    build_farrow(P);
    if (p->fd_kind == MSIM_FD_FARROW) {
        P->err_farrow = farrow_error(P);
        if (P->err_farrow > kFdErrBudget) {
            const double e = P->err_farrow;
            delete P;
            return fail(MSIM_E_UNSUPPORTED,
                        "Farrow form: predicted relative error %.2e of order-%d polynomials exceeds %.0e at "
                        "kaiser_beta %g, cutoff %g, taps %d (raise farrow_order or kaiser_beta)",
                        e, p->farrow_order, kFdErrBudget, p->kaiser_beta, p->cutoff, p->taps);
        }
    } else {
        P->err_table = table_error(P);
        P->err_farrow = farrow_error(P);   // its dL/dx goes through the Farrow gather
        if (P->err_table > kFdErrBudget) {
            const double e = P->err_table;
            const int L = P->par.table_phases;
            delete P;
            return fail(MSIM_E_UNSUPPORTED,
                        "table form: predicted relative error %.2e of the %d-phase table exceeds %.0e at "
                        "kaiser_beta %g, cutoff %g, taps %d (raise table_phases or use the Farrow form)",
                        e, L, kFdErrBudget, p->kaiser_beta, p->cutoff, p->taps);
        }
        // the pair's omitted edge tap on top of the table's error
        if (std::hypot(P->err_table, P->err_pair) > kFdErrBudget) P->rb_max = 1;
    }
    P->rb = p->fd_kind != MSIM_FD_FARROW ? P->rb_max : 1;
    P->n_scenes = n_scenes;
    int64_t xo = 0, yo = 0;
    for (int s = 0; s < n_scenes; ++s) {
        if ((st = plan_scene(P, scenes[s], s, xo, yo)) != MSIM_OK) {
            delete P;
            return st;
        }
        xo += scenes[s].n_in;
        yo += (int64_t)scenes[s].n_mics * scenes[s].n_out;
    }
    P->x_total = xo;
    P->y_total = yo;
    P->knots_ref = P->knots;
    // delay blocks of about a quarter second, a whole number of 1024-output tiles
    P->blk_len = std::max<int64_t>(1024, (int64_t)std::llround(0.25 * p->fs / 1024.0) * 1024);
    P->orders.assign(n_scenes, {});
    {
        const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        std::atomic<int> next{0};
        for (unsigned k = 0; k < hw; ++k)
            pool.emplace_back([&] {
                for (int s = next++; s < n_scenes; s = next++) order_blocks(P, s);
            });
        for (auto& th : pool) th.join();
    }
    // Farrow-filtered source positions [-T/2, n_in + T/2) of every scene, packed
    int64_t vo = 0;
    P->vpos_prefix.assign(n_scenes, 0);
    for (int s = 0; s < n_scenes; ++s) {
        P->vpos_prefix[s] = vo;
        P->scenes[s].v_off = vo * kFarrowStride;
        vo += P->scenes[s].n_in + p->taps;
    }
    P->vpos_total = vo;
    if ((st = regroup(P)) != MSIM_OK) {
        delete P;
        return st;
    }
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return fail(MSIM_E_HIP, "no HIP device");
    }
    {
        void* sp = nullptr;
        if ((st = scratch_on(P->device, &sp)) != MSIM_OK) {
            delete P;
            return st;
        }
    }
    std::vector<float4> qtab4((P->qtable.size() + 15) / 16);
    std::memcpy(qtab4.data(), P->qtable.data(), P->qtable.size());
    std::vector<int32_t> zero(1, 0);
    std::vector<int64_t> x_prefix(n_scenes);
    for (int sc = 0; sc < n_scenes; ++sc) x_prefix[sc] = P->scenes[sc].x_off;
    if ((st = upload(&P->d_fcoef, P->fcoef)) != MSIM_OK || (st = upload(&P->d_vpos_prefix, P->vpos_prefix)) != MSIM_OK ||
        (st = upload(&P->d_images, P->images)) != MSIM_OK ||
        (st = upload(&P->d_knots, P->knots)) != MSIM_OK || (st = upload(&P->d_mics, P->mics)) != MSIM_OK ||
        (st = upload(&P->d_status, zero)) != MSIM_OK || (st = upload(&P->d_zero, std::vector<int64_t>(1, 0))) != MSIM_OK ||
        (st = upload(&P->d_x_prefix, x_prefix)) != MSIM_OK ||
        (st = upload(&P->d_qtable, qtab4)) != MSIM_OK || (st = upload(&P->d_atable, P->atable)) != MSIM_OK ||
        (st = upload_layout(P)) != MSIM_OK) {
        msim_plan_destroy(P);
        return st;
    }
    *out = P;
    return MSIM_OK;
}

msim_status msim_plan_destroy(msim_plan* P)
{
    if (!P) return MSIM_OK;
    for (auto& r : P->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : P->pool) (void)hipEventDestroy(e);
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    free_layout(P);
    (void)hipFree(P->d_images);
    (void)hipFree(P->d_knots);
    (void)hipFree(P->d_mics);
    (void)hipFree(P->d_qtable);
    (void)hipFree(P->d_atable);
    (void)hipFree(P->d_fcoef);
    (void)hipFree(P->d_vpos_prefix);
    (void)hipFree(P->d_status);
    (void)hipFree(P->d_zero);
    (void)hipFree(P->d_x_prefix);
    if (P->bgraph_exec) (void)hipGraphExecDestroy(P->bgraph_exec);
    delete P;
    return MSIM_OK;
}

msim_status msim_plan_layout(const msim_plan* P, int64_t* x_off, int64_t* y_off, int64_t* x_total, int64_t* y_total)
{
    if (!P) return fail(MSIM_E_INVALID_ARG, "plan is NULL");
    for (int s = 0; s < P->n_scenes; ++s) {
        if (x_off) x_off[s] = P->scenes[s].x_off;
        if (y_off) y_off[s] = P->scenes[s].y_off;
    }
    if (x_total) *x_total = P->x_total;
    if (y_total) *y_total = P->y_total;
    return MSIM_OK;
}

msim_status msim_plan_stats(const msim_plan* P, int64_t* n_images, double* forward_taps)
{
    if (!P) return fail(MSIM_E_INVALID_ARG, "plan is NULL");
    if (n_images)
        for (int s = 0; s < P->n_scenes; ++s) n_images[s] = P->n_img[s];
    if (forward_taps) *forward_taps = P->fwd_taps;
    return MSIM_OK;
}

msim_status msim_workspace_size(const msim_plan* P, int32_t with_grad, size_t* bytes)
{
    if (!P || !bytes) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    if (!with_grad) {
        *bytes = carve_fwd_ws(P, false, nullptr, nullptr);
        return MSIM_OK;
    }
    *bytes = carve_bwd_ws(P, false, nullptr, nullptr);
    return MSIM_OK;
}

msim_status msim_plan_grad_layout(const msim_plan* P, int64_t* src_off, int64_t* src_total)
{
    if (!P) return fail(MSIM_E_INVALID_ARG, "plan is NULL");
    for (int s = 0; s < P->n_scenes; ++s)
        if (src_off) src_off[s] = P->scenes[s].src_grad_off;
    if (src_total) *src_total = P->src_grad_total;
    return MSIM_OK;
}

msim_status msim_backward(msim_plan* P, const float* x, const float* gy, float* gx, double* gbeta, double* gsrc,
                          void* ws, size_t ws_bytes, hipStream_t stream)
{
    msim_status st = check_backward(P, x, gy, gsrc);
    if (st != MSIM_OK) return st;
    const size_t need = carve_bwd_ws(P, false, nullptr, nullptr);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0)
        return fail(MSIM_E_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned", need);
    BwdWs w;
    carve_bwd_ws(P, false, (char*)ws, &w);
    return enqueue_backward(P, x, gy, gx, gbeta, gsrc, w, false, stream);
}

msim_status msim_forward(msim_plan* P, const float* x, float* y, void* ws, size_t ws_bytes, hipStream_t stream)
{
    if (!P || !x || !y) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    const size_t need = carve_fwd_ws(P, false, nullptr, nullptr);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0)
        return fail(MSIM_E_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned", need);
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != P->device) return fail(MSIM_E_INVALID_ARG, "plan was created on device %d, current is %d", P->device, dev);
    FwdWs2 w;
    carve_fwd_ws(P, false, (char*)ws, &w);
    return enqueue_forward(P, x, y, w, false, stream);
}

msim_status msim_forward_noalloc(msim_plan* P, const float* x, float* y, hipStream_t stream)
{
    if (!P || !x || !y) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    const size_t need = carve_fwd_ws(P, false, nullptr, nullptr);
    if (need > kNoAllocBytes)
        return fail(MSIM_E_WORKSPACE,
                    "msim_forward_noalloc: this plan needs %zu bytes of scratch, the fixed per-GPU scratch holds %zu",
                    need, kNoAllocBytes);
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != P->device) return fail(MSIM_E_INVALID_ARG, "plan was created on device %d, current is %d", P->device, dev);
    void* sp = nullptr;
    msim_status st = scratch_on(dev, &sp);
    if (st != MSIM_OK) return st;
    FwdWs2 w;
    carve_fwd_ws(P, false, (char*)sp, &w);
    // no per-launch timing events here: they would be created on the first use
    const bool prof = P->profiling;
    P->profiling = false;
    st = enqueue_forward(P, x, y, w, false, stream);
    P->profiling = prof;
    return st;
}

msim_status msim_profile_begin(msim_plan* P)
{
    if (!P) return fail(MSIM_E_INVALID_ARG, "plan is NULL");
    P->profiling = true;
    return MSIM_OK;
}

msim_status msim_profile_end(msim_plan* P, msim_profile* out)
{
    if (!P || !out) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    P->profiling = false;
    double ms[kKinds] = {0};
    int32_t cnt[kKinds] = {0};
    msim_status st = MSIM_OK;
    for (auto& r : P->recs) {
        float v = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&v, r.a, r.b) != hipSuccess)
            st = fail(MSIM_E_HIP, "profiling event failed");
        ms[r.kind] += v;
        cnt[r.kind] += 1;
        P->pool.push_back(r.a);
        P->pool.push_back(r.b);
    }
    P->recs.clear();
    out->synth_ms = ms[kKindSynth];
    out->reduce_ms = ms[kKindReduce];
    out->adjx_ms = ms[kKindAdjX];
    out->adjp_ms = ms[kKindAdjP];
    out->params_ms = ms[kKindParams];
    out->graph_ms = ms[kKindGraph];
    out->filter_ms = ms[kKindFilter];
    out->synth_launches = cnt[kKindSynth];
    out->reduce_launches = cnt[kKindReduce];
    out->adjx_launches = cnt[kKindAdjX];
    out->adjp_launches = cnt[kKindAdjP];
    out->params_launches = cnt[kKindParams];
    out->graph_launches = cnt[kKindGraph];
    out->filter_launches = cnt[kKindFilter];
    return st;
}

}  // extern "C"

namespace {

msim_status check_batched_call(msim_plan* P, const float* x, float* y, void* ws, size_t ws_bytes)
{
    if (!P || !x || !y) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    const size_t need = carve_fwd_ws(P, true, nullptr, nullptr);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0)
        return fail(MSIM_E_WORKSPACE, "batched workspace needs %zu bytes, 256-byte aligned", need);
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != P->device) return fail(MSIM_E_INVALID_ARG, "plan was created on device %d, current is %d", P->device, dev);
    return MSIM_OK;
}

const int kTuneThreads[] = {512, 1024};
const int kTuneCaps[] = {0, 16, 32, 64, 128, 256, 512};

std::string tune_key(const msim_plan* P)
{
    int64_t imgs = 0;
    for (int64_t v : P->n_img) imgs += v;
    char buf[256];
    snprintf(buf, sizeof buf, "gfx950/F%d/M%d/T%d/L%d/S%d/I%lld/Y%lld", P->par.fd_kind, P->par.farrow_order,
             P->par.taps, P->par.table_phases, P->n_scenes, (long long)imgs, (long long)P->y_total);
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, int* threads, int* cap, int* rb)
{
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[256];
        int t = 0, c = 0, r = 0;
        // {"key": "...", "threads": N, "group_cap": N, "outputs_per_lane": N, ...}
        if (sscanf(line, " {\"key\": \"%255[^\"]\", \"threads\": %d, \"group_cap\": %d, \"outputs_per_lane\": %d",
                   k, &t, &c, &r) == 4 &&
            key == k && (t == 512 || t == 1024) && c >= 0 && (r == 1 || r == 2 || r == 4)) {
            *threads = t;
            *cap = c;
            *rb = r;
            found = true;
        }
    }
    fclose(f);
    return found;
}

}  // namespace

extern "C" {

msim_status msim_batched_workspace_size(const msim_plan* P, size_t* bytes)
{
    if (!P || !bytes) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    *bytes = std::max(carve_fwd_ws(P, true, nullptr, nullptr), carve_bwd_ws(P, true, nullptr, nullptr));
    return MSIM_OK;
}

msim_status msim_forward_batched(msim_plan* P, const float* x, float* y, void* ws, size_t ws_bytes,
                                 hipStream_t stream, int32_t use_graph)
{
    msim_status st = check_batched_call(P, x, y, ws, ws_bytes);
    if (st != MSIM_OK) return st;
    FwdWs2 w;
    carve_fwd_ws(P, true, (char*)ws, &w);
    if (!use_graph) return enqueue_forward(P, x, y, w, true, stream);
    const void* key[3] = {x, y, ws};
    if (!P->graph_valid || std::memcmp(key, P->graph_key, sizeof key) != 0) {
        if (!P->cap_stream) HIP_OK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
        if (P->graph_exec) {
            HIP_OK(hipGraphExecDestroy(P->graph_exec));
            P->graph_exec = nullptr;
        }
        P->graph_valid = false;
        const bool prof = P->profiling;
        P->profiling = false;
        HIP_OK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed));
        st = enqueue_forward(P, x, y, w, true, P->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(P->cap_stream, &graph);
        P->profiling = prof;
        if (st != MSIM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(MSIM_E_HIP, "graph capture: %s", hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&P->graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) return fail(MSIM_E_HIP, "graph instantiate: %s", hipGetErrorString(e2));
        std::memcpy(P->graph_key, key, sizeof key);
        P->graph_valid = true;
    }
    LaunchTimer t(P, kKindGraph, stream);
    HIP_OK(hipGraphLaunch(P->graph_exec, stream));
    return MSIM_OK;
}

msim_status msim_backward_batched(msim_plan* P, const float* x, const float* gy, float* gx, double* gbeta,
                                  double* gsrc, void* ws, size_t ws_bytes, hipStream_t stream, int32_t use_graph)
{
    msim_status st = check_backward(P, x, gy, gsrc);
    if (st != MSIM_OK) return st;
    const size_t need = carve_bwd_ws(P, true, nullptr, nullptr);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0)
        return fail(MSIM_E_WORKSPACE, "batched workspace needs %zu bytes, 256-byte aligned", need);
    BwdWs w;
    carve_bwd_ws(P, true, (char*)ws, &w);
    if (!use_graph) return enqueue_backward(P, x, gy, gx, gbeta, gsrc, w, true, stream);
    const void* key[6] = {x, gy, gx, gbeta, gsrc, ws};
    if (!P->bgraph_valid || std::memcmp(key, P->bgraph_key, sizeof key) != 0) {
        if (!P->cap_stream) HIP_OK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
        if (P->bgraph_exec) {
            HIP_OK(hipGraphExecDestroy(P->bgraph_exec));
            P->bgraph_exec = nullptr;
        }
        P->bgraph_valid = false;
        const bool prof = P->profiling;
        P->profiling = false;
        HIP_OK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed));
        st = enqueue_backward(P, x, gy, gx, gbeta, gsrc, w, true, P->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(P->cap_stream, &graph);
        P->profiling = prof;
        if (st != MSIM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(MSIM_E_HIP, "graph capture: %s", hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&P->bgraph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) return fail(MSIM_E_HIP, "graph instantiate: %s", hipGetErrorString(e2));
        std::memcpy(P->bgraph_key, key, sizeof key);
        P->bgraph_valid = true;
    }
    LaunchTimer t(P, kKindGraph, stream);
    HIP_OK(hipGraphLaunch(P->bgraph_exec, stream));
    return MSIM_OK;
}

msim_status msim_get_tuning(const msim_plan* P, msim_tuning* out)
{
    if (!P || !out) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    out->threads = P->threads;
    out->group_cap = P->group_cap;
    out->outputs_per_lane = P->rb;
    out->workgroups = P->b_wgs;
    out->ms = 0.0;
    out->adjx_gather = P->ugather ? 1 : 0;
    return MSIM_OK;
}

msim_status msim_plan_update(msim_plan* P, const double* beta, const double* knots, hipStream_t stream)
{
    if (!P) return fail(MSIM_E_INVALID_ARG, "plan is NULL");
    if (!beta && !knots) return MSIM_OK;
    std::vector<DScene> sc = P->scenes, scb = P->scenes_b;
    std::vector<double> kn = P->knots;
    for (int s = 0; s < P->n_scenes; ++s) {
        DScene& d = sc[s];
        if (beta)
            for (int w = 0; w < 6; ++w) d.beta[w] = beta[6 * s + w];
        if (knots && d.src_knots > 0) {
            for (int k = 0; k < d.src_knots; ++k)
                for (int a = 0; a < 3; ++a) {
                    const double v = knots[3 * ((int64_t)d.src_grad_off + k) + a];
                    const double ref = P->knots_ref[d.src.pos_off + 3 * k + a];
                    if (!(std::fabs(v - ref) <= P->par.knot_slack))
                        return fail(MSIM_E_UNSUPPORTED,
                                    "scene %d: knot %d moved %.3g m from the planned path, beyond knot_slack %.3g m "
                                    "(create a new plan)",
                                    s, k, std::fabs(v - ref), P->par.knot_slack);
                    kn[d.src.pos_off + 3 * k + a] = v;
                }
        }
        // the scene as updated passes the same checks as at plan creation
        msim_scene h{};
        for (int a = 0; a < 3; ++a) h.size[a] = d.size[a];
        for (int w = 0; w < 6; ++w) h.beta[w] = d.beta[w];
        msim_traj src{}, rcv{};
        {
            std::swap(P->knots, kn);
            src = host_traj(P, d.src);
            rcv = host_traj(P, d.rcv);
            std::swap(P->knots, kn);
        }
        std::vector<double> tk(src.t ? src.t : nullptr, src.t ? src.t + src.n_points : nullptr);
        std::vector<double> pk(kn.begin() + (src.kind == MSIM_TRAJ_PWL ? d.src.pos_off : 0),
                               kn.begin() + (src.kind == MSIM_TRAJ_PWL ? d.src.pos_off + 3 * src.n_points : 0));
        std::vector<double> tr(rcv.t ? rcv.t : nullptr, rcv.t ? rcv.t + rcv.n_points : nullptr);
        std::vector<double> pr(rcv.p ? rcv.p : nullptr, rcv.p ? rcv.p + 3 * rcv.n_points : nullptr);
        if (src.kind == MSIM_TRAJ_PWL) {
            src.t = tk.data();
            src.p = pk.data();
        }
        if (rcv.kind == MSIM_TRAJ_PWL) {
            rcv.t = tr.data();
            rcv.p = pr.data();
        }
        h.src = src;
        h.rcv = rcv;
        h.n_mics = d.n_mics;
        h.mic_offset = P->mics.data() + 3 * (size_t)d.mic_off;
        h.max_order = 0;
        h.n_in = d.n_in;
        h.n_out = d.n_out;
        msim_status st = check_scene(h, &P->par, s);
        if (st != MSIM_OK) return st;
        for (int w = 0; w < 6; ++w) scb[s].beta[w] = d.beta[w];
    }
    std::vector<DImage> im = P->images;
    if (beta)
        for (int s = 0; s < P->n_scenes; ++s)
            for (int i = sc[s].img_begin; i < sc[s].img_begin + sc[s].n_img; ++i) {
                double b = 1.0;
                for (int w = 0; w < 6; ++w) b *= std::pow(sc[s].beta[w], im[i].hits[w]);
                im[i].gfac = (float)(b * P->par.fs / (4.0 * kPi * P->par.c));
            }
    P->scenes.swap(sc);
    P->scenes_b.swap(scb);
    P->knots.swap(kn);
    P->images.swap(im);
    auto put = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream) == hipSuccess;
    };
    const bool ok = put(P->d_scenes, P->scenes.data(), P->scenes.size() * sizeof(DScene)) &&
                    put(P->d_scenes_b, P->scenes_b.data(), P->scenes_b.size() * sizeof(DScene)) &&
                    put(P->d_knots, P->knots.data(), P->knots.size() * sizeof(double)) &&
                    put(P->d_images, P->images.data(), P->images.size() * sizeof(DImage)) &&
                    hipStreamSynchronize(stream) == hipSuccess;
    if (!ok) return fail(MSIM_E_HIP, "plan update upload failed");
    return MSIM_OK;
}

msim_status msim_get_images(const msim_plan* P, int32_t scene, int32_t* out, int64_t capacity, int64_t* n_img)
{
    if (!P || !n_img) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    if (scene < 0 || scene >= P->n_scenes) return fail(MSIM_E_INVALID_ARG, "scene %d out of range", scene);
    const DScene& d = P->scenes[scene];
    *n_img = d.n_img;
    if (!out) return MSIM_OK;
    if (capacity < d.n_img) return fail(MSIM_E_INVALID_ARG, "capacity %lld < %d images", (long long)capacity, d.n_img);
    for (int i = 0; i < d.n_img; ++i) {
        const DImage& im = P->images[d.img_begin + i];
        out[4 * i] = im.m[0];
        out[4 * i + 1] = im.m[1];
        out[4 * i + 2] = im.m[2];
        out[4 * i + 3] = im.R;
    }
    return MSIM_OK;
}

msim_status msim_get_fd_error(const msim_plan* P, msim_fd_error* out)
{
    if (!P || !out) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    out->table = P->err_table;
    out->pair = P->err_pair;
    out->farrow = P->err_farrow;
    out->budget = kFdErrBudget;
    out->table_phases = P->par.table_phases;
    return MSIM_OK;
}

msim_status msim_set_tuning(msim_plan* P, const msim_tuning* t)
{
    if (!P || !t) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    if (t->threads != 512 && t->threads != 1024) return fail(MSIM_E_INVALID_ARG, "threads must be 512 or 1024");
    if (t->group_cap < 0) return fail(MSIM_E_INVALID_ARG, "group_cap must be >= 0");
    const int rb = t->outputs_per_lane != 0 ? t->outputs_per_lane
                                            : (P->par.fd_kind == MSIM_FD_FARROW ? 1 : P->rb_max);
    if (rb != 1 && rb != 2 && rb != 4) return fail(MSIM_E_INVALID_ARG, "outputs_per_lane must be 0, 1, 2 or 4");
    if (P->rb_max % rb != 0)
        return fail(MSIM_E_INVALID_ARG,
                    "outputs_per_lane %d: the form, the tier decimations and the speeds allow at most %d", rb,
                    P->rb_max);
    const int ot = P->threads, oc = P->group_cap, orb = P->rb;
    P->threads = t->threads;
    P->group_cap = t->group_cap;
    P->rb = rb;
    msim_status st = regroup(P);
    if (st != MSIM_OK) {
        P->threads = ot;
        P->group_cap = oc;
        P->rb = orb;
        regroup(P);
        return st;
    }
    return upload_layout(P);
}

msim_status msim_autotune_workspace_size(msim_plan* P, size_t* bytes)
{
    if (!P || !bytes) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    const int ot = P->threads, oc = P->group_cap;
    size_t m = 0;
    for (int t : kTuneThreads)
        for (int c : kTuneCaps) {
            P->threads = t;
            P->group_cap = c;
            if (regroup(P) == MSIM_OK) m = std::max(m, carve_fwd_ws(P, true, nullptr, nullptr));
        }
    P->threads = ot;
    P->group_cap = oc;
    msim_status st = regroup(P);
    if (st != MSIM_OK) return st;
    *bytes = m;
    return MSIM_OK;
}

msim_status msim_autotune(msim_plan* P, const float* x, float* y, void* ws, size_t ws_bytes, hipStream_t stream,
                          const char* cache_path, msim_tuning* best_out)
{
    if (!P || !x || !y || !ws) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    const std::string key = tune_key(P);
    int bt = 0, bc = 0, brb = 1;
    // a cached shape this plan accepts is used as it is; one it refuses (another
    // build's limits, a hand-edited line) is timed again
    if (cache_lookup(cache_path, key, &bt, &bc, &brb)) {
        msim_tuning t{bt, bc, brb, 0, 0.0, 0};
        if (msim_set_tuning(P, &t) == MSIM_OK) {
            if (best_out) msim_get_tuning(P, best_out);
            return MSIM_OK;
        }
    }
    // Every exit restores the plan's launch shape (regrouped and uploaded) and
    // its profiling flag, and frees the events, unless a tuning was applied.
    struct Guard {
        msim_plan* P;
        int t, c, rb;
        bool prof, applied = false;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        explicit Guard(msim_plan* p) : P(p), t(p->threads), c(p->group_cap), rb(p->rb), prof(p->profiling) {}
        ~Guard()
        {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            P->profiling = prof;
            if (!applied) {
                P->threads = t;
                P->group_cap = c;
                P->rb = rb;
                if (regroup(P) == MSIM_OK) (void)upload_layout(P);
            }
        }
    } guard(P);
    HIP_OK(hipEventCreate(&guard.e0));
    HIP_OK(hipEventCreate(&guard.e1));
    P->profiling = false;
    double best = 1e300;
    bt = 0;
    for (int t : kTuneThreads)
        for (int c : kTuneCaps)
            for (int rb : {1, 2, 4}) {
                if (P->rb_max % rb != 0) continue;
                P->threads = t;
                P->group_cap = c;
                P->rb = rb;
                if (regroup(P) != MSIM_OK || carve_fwd_ws(P, true, nullptr, nullptr) > ws_bytes) continue;
                msim_status st = upload_layout(P);
                if (st != MSIM_OK) return st;
                FwdWs2 w;
                carve_fwd_ws(P, true, (char*)ws, &w);
                if ((st = enqueue_forward(P, x, y, w, true, stream)) != MSIM_OK) return st;
                HIP_OK(hipEventRecord(guard.e0, stream));
                for (int r = 0; r < 3; ++r)
                    if ((st = enqueue_forward(P, x, y, w, true, stream)) != MSIM_OK) return st;
                HIP_OK(hipEventRecord(guard.e1, stream));
                HIP_OK(hipEventSynchronize(guard.e1));
                float ms = 0.0f;
                HIP_OK(hipEventElapsedTime(&ms, guard.e0, guard.e1));
                if (ms / 3.0 < best) {
                    best = ms / 3.0;
                    bt = t;
                    bc = c;
                    brb = rb;
                }
            }
    if (bt == 0) return fail(MSIM_E_WORKSPACE, "no tuning candidate fits the workspace");
    msim_tuning t{bt, bc, brb, 0, best, 0};
    P->profiling = guard.prof;
    msim_status st = msim_set_tuning(P, &t);
    if (st != MSIM_OK) return st;
    guard.applied = true;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"key\": \"%s\", \"threads\": %d, \"group_cap\": %d, \"outputs_per_lane\": %d, "
                    "\"ms\": %.4f}\n", key.c_str(), bt, bc, brb, best);
            fclose(f);
        }
    }
    if (best_out) {
        msim_get_tuning(P, best_out);
        best_out->ms = best;
    }
    return MSIM_OK;
}

msim_status msim_device_status(msim_plan* P, hipStream_t stream, int32_t* flags)
{
    if (!P || !flags) return fail(MSIM_E_INVALID_ARG, "NULL argument");
    int32_t v = 0;
    HIP_OK(hipMemcpyAsync(&v, P->d_status, sizeof v, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    HIP_OK(hipMemsetAsync(P->d_status, 0, sizeof v, stream));
    HIP_OK(hipStreamSynchronize(stream));
    *flags = v;
    return v ? fail(MSIM_E_DEVICE, "device status flags 0x%x", v) : MSIM_OK;
}

}  // extern "C"
