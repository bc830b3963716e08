/*
 * FP64 CPU oracle for moving-source image-source synthesis.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library; it is written from the paper's
 * definitions, plainly and slowly, in double precision.
 *
 * What it computes (paper: "Fast Algorithm for Moving Sound Source",
 * arXiv 2508.03065):
 *   - Image sources of a shoebox room (image-source method, Sec. II-A, the
 *     static RIR of Eq. (1)); gain A_i = beta_i / (4 pi d_i) with beta_i the
 *     product of the wall coefficients along the path (Sec. II-A, the text
 *     after Eq. (2)).
 *   - Moving-image output v(t) = sum_i A_i(t) s(t - tau_i(t))  (Eq. (2), Eq. (8)),
 *     with tau_i = d_i / c (Sec. II-C-3) taken at the emission time (retarded
 *     reading) or at the reception time (instantaneous reading).
 *   - The fractional delay is an FIR truncation of the ideal sinc response
 *     (Sec. II-B); here a T-tap Kaiser-windowed sinc, evaluated exactly from
 *     its formula at every tap (no table).
 *   - Order-tiered trajectory sampling (Sec. II-C-3): delays solved exactly on a
 *     decimated grid and brought back to the audio rate by uniform Catmull-Rom
 *     interpolation of tau ("tier-emulating" mode).  With no tiers every
 *     image's exact delay is solved at every output sample ("full-rate" mode).
 *   - Adjoints: the exact transpose of the time-varying delay (d loss / d x) and
 *     d loss / d beta_w via the product structure of beta_i.
 *
 * Parity pins live in tests/test_oracle_pins.py.  Every function is pinned
 * there by a closed form, a library routine, an independent brute force or an
 * invariant; none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ types */

typedef struct {
    int32_t kind;        /* 0: piecewise linear through knots (1 knot = static), 1: horizontal circle */
    int32_t n_points;    /* number of knots (kind 0) */
    const double* t;     /* [n_points] knot times in s, strictly increasing */
    const double* p;     /* [n_points*3] knot positions in m */
    double center[3];    /* circle centre (kind 1); motion in the plane z = center[2] */
    double radius;       /* circle radius, m */
    double speed;        /* speed along the circle, m/s */
    double phase0;       /* angle at t = 0, rad */
} orc_traj;

typedef struct {
    double size[3];          /* room Lx, Ly, Lz in m */
    double beta[6];          /* wall coefficients: x=0, x=Lx, y=0, y=Ly, z=0, z=Lz */
    orc_traj src, rcv;
    int32_t n_mics;
    const double* mic_offset;    /* [n_mics*3], added to the receiver position */
    int64_t n_in, n_out;
} orc_scene;

typedef struct {
    double c, fs;
    int32_t max_order;       /* K: images with |mx|+|my|+|mz| <= K */
    int32_t taps;            /* T (even) */
    double kaiser_beta;
    double cutoff;           /* normalised cutoff f_c in cycles/sample (0.5 = full band) */
    int32_t n_tiers;         /* 0: full rate; else tiers as below */
    int32_t tier_max_order[4];
    int32_t tier_decim[4];
    int32_t delay_model;     /* 0: retarded (emission-time) delay, 1: instantaneous */
    int32_t tier_mode;       /* 0: decimation by reflection order (tiers above); 1: per image from
                                the delay track's third-derivative bound (see adaptive_decim) */
    double tier_tol;         /* mode 1: allowed error of the interpolated delay, samples */
    int32_t tier_rmax;       /* mode 1: largest decimation */
} orc_params;

/* ----------------------------------------------------- image enumeration */

/* Number of integer triples with |mx|+|my|+|mz| <= K, counted one by one. */
int64_t orc_count_images(int32_t K)
{
    int64_t n = 0;
    for (int mx = -K; mx <= K; ++mx)
        for (int my = -K; my <= K; ++my)
            for (int mz = -K; mz <= K; ++mz)
                if (abs(mx) + abs(my) + abs(mz) <= K) ++n;
    return n;
}

/* Wall hits of an axis index m: the image at index m along an axis is reached
 * after |m| reflections alternating between the two walls of that axis.  For
 * m > 0 the first reflection is on the far wall (coordinate L), for m < 0 on
 * the near wall (coordinate 0). */
static void axis_hits(int m, int* n_near, int* n_far)
{
    int a = abs(m);
    if (m >= 0) { *n_far = (a + 1) / 2; *n_near = a / 2; }
    else        { *n_near = (a + 1) / 2; *n_far = a / 2; }
}

/* Fills m[n*3] and hits[n*6] (wall order x0,xL,y0,yL,z0,zL) and beta_i[n];
 * returns the image count.  Any of the output pointers may be NULL. */
int64_t orc_images(const double* beta, int32_t K, int32_t* m, int32_t* hits, double* beta_i)
{
    int64_t n = 0;
    for (int mx = -K; mx <= K; ++mx)
        for (int my = -K; my <= K; ++my)
            for (int mz = -K; mz <= K; ++mz) {
                if (abs(mx) + abs(my) + abs(mz) > K) continue;
                int mm[3] = {mx, my, mz};
                int h[6];
                for (int a = 0; a < 3; ++a) axis_hits(mm[a], &h[2 * a], &h[2 * a + 1]);
                double b = 1.0;
                for (int w = 0; w < 6; ++w)
                    for (int r = 0; r < h[w]; ++r) b *= beta[w];
                if (m) { m[3 * n] = mx; m[3 * n + 1] = my; m[3 * n + 2] = mz; }
                if (hits) for (int w = 0; w < 6; ++w) hits[6 * n + w] = h[w];
                if (beta_i) beta_i[n] = b;
                ++n;
            }
    return n;
}

/* Position of image m of a point q: per axis, the mirrored copy in cell m. */
static void image_point(const double L[3], const int m[3], const double q[3], double out[3])
{
    for (int a = 0; a < 3; ++a) {
        if (m[a] % 2 == 0) out[a] = m[a] * L[a] + q[a];
        else               out[a] = (m[a] + 1) * L[a] - q[a];
    }
}

/* Exported for the tests: image of point q in cell m. */
void orc_image_pos(const double* size, const int32_t* m, const double* q, double* out)
{
    int mm[3] = {m[0], m[1], m[2]};
    image_point(size, mm, q, out);
}

/* ---------------------------------------------------------- trajectories */

void orc_traj_pos(const orc_traj* tr, double t, double out[3])
{
    if (tr->kind == 1) {
        double w = tr->speed / tr->radius;
        out[0] = tr->center[0] + tr->radius * cos(w * t + tr->phase0);
        out[1] = tr->center[1] + tr->radius * sin(w * t + tr->phase0);
        out[2] = tr->center[2];
        return;
    }
    int np = tr->n_points;
    const double* P = tr->p;
    if (np == 1 || t <= tr->t[0]) { out[0] = P[0]; out[1] = P[1]; out[2] = P[2]; return; }
    if (t >= tr->t[np - 1]) {
        out[0] = P[3 * (np - 1)]; out[1] = P[3 * (np - 1) + 1]; out[2] = P[3 * (np - 1) + 2];
        return;
    }
    int a = 0;
    while (!(t >= tr->t[a] && t < tr->t[a + 1])) ++a;
    double lam = (t - tr->t[a]) / (tr->t[a + 1] - tr->t[a]);
    for (int k = 0; k < 3; ++k) out[k] = P[3 * a + k] + lam * (P[3 * (a + 1) + k] - P[3 * a + k]);
}

static void mic_pos(const orc_scene* s, int mic, double t, double out[3])
{
    orc_traj_pos(&s->rcv, t, out);
    for (int k = 0; k < 3; ++k) out[k] += s->mic_offset[3 * mic + k];
}

/* Distance from mic (at reception time t) to the image of the source at time te. */
static double image_dist(const orc_scene* s, const int m[3], const double r[3], double te)
{
    double q[3], pi[3];
    orc_traj_pos(&s->src, te, q);
    image_point(s->size, m, q, pi);
    double dx = pi[0] - r[0], dy = pi[1] - r[1], dz = pi[2] - r[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Propagation delay (s) of image m to mic `mic` for sound received at time t.
 * Retarded: the unique tau > 0 with c tau = |p_i(t - tau) - r(t)| (the wave
 * received at t left the image at t - tau); solved by fixed-point iteration,
 * which contracts with factor |source speed| / c.  Instantaneous:
 * tau = |p_i(t) - r(t)| / c. */
double orc_tau(const orc_scene* s, const orc_params* p, const int32_t m[3], int mic, double t)
{
    double r[3];
    mic_pos(s, mic, t, r);
    int mm[3] = {m[0], m[1], m[2]};
    double tau = image_dist(s, mm, r, t) / p->c;
    if (p->delay_model == 1) return tau;
    for (int it = 0; it < 200; ++it) {
        double nt = image_dist(s, mm, r, t - tau) / p->c;
        double d = fabs(nt - tau);
        tau = nt;
        if (d <= 2e-15 * tau) break;
    }
    return tau;
}

/* ------------------------------------------------- fractional delay kernel */

/* Modified Bessel function of the first kind, order 0: sum_k ((x/2)^k / k!)^2. */
double orc_i0(double x)
{
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

/* Kaiser-windowed sinc: h(u) = 2 fc sinc(2 fc u) w(u), with
 * w(u) = I0(beta sqrt(1 - (2u/T)^2)) / I0(beta) on |u| <= T/2, zero outside. */
double orc_kernel(double u, int32_t T, double kbeta, double fc)
{
    double half = 0.5 * T;
    if (fabs(u) > half) return 0.0;
    double z = 2.0 * fc * u;
    double sinc = (z == 0.0) ? 1.0 : sin(M_PI * z) / (M_PI * z);
    double r = 2.0 * u / T;
    double arg = 1.0 - r * r;
    if (arg < 0.0) arg = 0.0;
    double w = orc_i0(kbeta * sqrt(arg)) / orc_i0(kbeta);
    return 2.0 * fc * sinc * w;
}

/* ----------------------------------------------------------- tiered delays */

/* Uniform Catmull-Rom through v[0..3] (knots at -1, 0, 1, 2), evaluated at u in [0,1). */
double orc_catmull_rom(const double v[4], double u)
{
    double a = v[0], b = v[1], c = v[2], d = v[3];
    return 0.5 * (2.0 * b + (c - a) * u + (2.0 * a - 5.0 * b + 4.0 * c - d) * u * u
                  + (3.0 * b - a - 3.0 * c + d) * u * u * u);
}

static int order_of(const int32_t m[3]) { return abs(m[0]) + abs(m[1]) + abs(m[2]); }

/* Whether delays are decimated at all (tier-emulating mode). */
static int tiered(const orc_params* p) { return p->n_tiers > 0 || p->tier_mode == 1; }

/* Bounding box of a path: its knots, or the circle's square in its plane. */
static void path_box(const orc_traj* tr, double lo[3], double hi[3])
{
    if (tr->kind == 1) {
        for (int a = 0; a < 2; ++a) {
            lo[a] = tr->center[a] - tr->radius;
            hi[a] = tr->center[a] + tr->radius;
        }
        lo[2] = hi[2] = tr->center[2];
        return;
    }
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = tr->p[a];
    for (int k = 1; k < tr->n_points; ++k)
        for (int a = 0; a < 3; ++a) {
            if (tr->p[3 * k + a] < lo[a]) lo[a] = tr->p[3 * k + a];
            if (tr->p[3 * k + a] > hi[a]) hi[a] = tr->p[3 * k + a];
        }
}

/* Largest speed v, acceleration acc and jerk jrk of a path, and its largest
 * velocity change dv at an inner knot.  A circle of radius r at speed v: v,
 * v^2/r, v^3/r^2, no knots.  A PWL path, read as samples of a smooth path: the
 * largest piece speed; at each inner knot the change of velocity divided by half
 * the time between its neighbouring knots; no jerk. */
static void path_kinematics(const orc_traj* tr, double* v, double* acc, double* jrk, double* dv)
{
    *v = *acc = *jrk = *dv = 0.0;
    if (tr->kind == 1) {
        *v = tr->speed;
        *acc = tr->speed * tr->speed / tr->radius;
        *jrk = *acc * tr->speed / tr->radius;
        return;
    }
    for (int k = 0; k + 1 < tr->n_points; ++k) {
        double w = 0.0;
        for (int a = 0; a < 3; ++a) {
            double va = (tr->p[3 * (k + 1) + a] - tr->p[3 * k + a]) / (tr->t[k + 1] - tr->t[k]);
            w += va * va;
        }
        if (sqrt(w) > *v) *v = sqrt(w);
        if (k == 0) continue;
        double ch = 0.0;
        for (int a = 0; a < 3; ++a) {
            double v1 = (tr->p[3 * (k + 1) + a] - tr->p[3 * k + a]) / (tr->t[k + 1] - tr->t[k]);
            double v0 = (tr->p[3 * k + a] - tr->p[3 * (k - 1) + a]) / (tr->t[k] - tr->t[k - 1]);
            ch += (v1 - v0) * (v1 - v0);
        }
        ch = sqrt(ch);
        if (ch > *dv) *dv = ch;
        if (ch / (0.5 * (tr->t[k + 1] - tr->t[k - 1])) > *acc) *acc = ch / (0.5 * (tr->t[k + 1] - tr->t[k - 1]));
    }
}

/* Adaptive decimation (mode 1), the reading of Sec. II-C-1/2 that the delay of
 * a far image carries the motion's own bandwidth while a close image (near
 * field) needs a higher rate, and that faint (high-order) images can be sampled
 * sparsely.  Image m may err in delay by tier_tol * max(d, 0.1 m) / beta_m
 * samples (its gain beta_m / (4 pi d) against that of a unit source at 1 m),
 * d the gap between the image's box over the path and the mics' box.  For
 * d(t) = |r(t)|, r the image-to-mic vector, the third derivative is at most
 * (2/sqrt 3) u^3/d^2 + 3 u a/d + j (u, a, j: relative speed, acceleration and
 * jerk bounds; the first term is the largest value of 3 u^3 sin^2 cos / d^2, the
 * straight-motion case), divided by (1 - u/c)^3 for the emission-time reading.
 * In samples the bound is D3 = K3 / (c fs^2); uniform Catmull-Rom at decimation R
 * errs by at most about R^3 D3 / 24 on smooth motion, and by up to 3/16 of R
 * times the delay slope's jump dv / (c - u) at a knot (the largest error of the
 * interpolated ramp max(0, x) at unit spacing is 3/16).  Take the largest R of
 * 1, 4, 8, 16, ... up to tier_rmax that keeps both within the budget. */
static int adaptive_decim(const orc_scene* s, const orc_params* p, const int32_t m[3])
{
    double slo[3], shi[3], rlo[3], rhi[3];
    path_box(&s->src, slo, shi);
    path_box(&s->rcv, rlo, rhi);
    double d2 = 0.0, beta_m = 1.0;
    for (int a = 0; a < 3; ++a) {
        int n_near, n_far;
        axis_hits(m[a], &n_near, &n_far);
        for (int r = 0; r < n_near; ++r) beta_m *= s->beta[2 * a];
        for (int r = 0; r < n_far; ++r) beta_m *= s->beta[2 * a + 1];
        double olo = s->mic_offset[a], ohi = s->mic_offset[a];
        for (int c = 1; c < s->n_mics; ++c) {
            if (s->mic_offset[3 * c + a] < olo) olo = s->mic_offset[3 * c + a];
            if (s->mic_offset[3 * c + a] > ohi) ohi = s->mic_offset[3 * c + a];
        }
        double mlo = rlo[a] + olo, mhi = rhi[a] + ohi;
        double L = s->size[a], ilo, ihi;
        if (m[a] % 2 == 0) { ilo = m[a] * L + slo[a]; ihi = m[a] * L + shi[a]; }
        else               { ilo = (m[a] + 1) * L - shi[a]; ihi = (m[a] + 1) * L - slo[a]; }
        double gap = 0.0;
        if (ilo - mhi > gap) gap = ilo - mhi;
        if (mlo - ihi > gap) gap = mlo - ihi;
        d2 += gap * gap;
    }
    int top = 1;
    for (int r = 4; r <= p->tier_rmax; r *= 2) top = r;
    if (beta_m == 0.0) return top;
    double d = sqrt(d2);
    if (!(d > 0.0)) return 1;
    double budget = p->tier_tol * (d > 0.1 ? d : 0.1) / beta_m;
    double vs, as, js, dvs, vr, ar, jr, dvr;
    path_kinematics(&s->src, &vs, &as, &js, &dvs);
    path_kinematics(&s->rcv, &vr, &ar, &jr, &dvr);
    double u = vs + vr, acc = as + ar, jrk = js + jr;
    double k3 = (2.0 / sqrt(3.0)) * u * u * u / (d * d) + 3.0 * u * acc / d + jrk;
    k3 /= pow(1.0 - u / p->c, 3);
    double d3 = k3 / (p->c * p->fs * p->fs);
    double kink = 0.1875 * (dvs + dvr) / (p->c - u);
    int R = 1;
    for (int r = 4; r <= p->tier_rmax; r *= 2)
        if ((double)r * r * r * d3 <= 24.0 * budget && (double)r * kink <= budget) R = r;
    return R;
}

/* Decimation factor of an image: by order, the first tier whose max order
 * covers it; adaptive, from its distance and the motion. */
static int decim_of(const orc_scene* s, const orc_params* p, const int32_t m[3])
{
    if (p->tier_mode == 1) return adaptive_decim(s, p, m);
    if (p->n_tiers <= 0) return 0;
    int o = order_of(m);
    for (int k = 0; k < p->n_tiers; ++k)
        if (o <= p->tier_max_order[k]) return p->tier_decim[k];
    return p->tier_decim[p->n_tiers - 1];
}

/* Exported for the tests: the decimation the oracle uses for image m. */
int32_t orc_image_decim(const orc_scene* s, const orc_params* p, const int32_t* m)
{
    return decim_of(s, p, m);
}

/* Delay of image m at output sample n: exact (full rate) or Catmull-Rom of the
 * exact delays at grid samples kR (tier-emulating). */
static double tau_at(const orc_scene* s, const orc_params* p, const int32_t m[3], int mic, int64_t n)
{
    int R = decim_of(s, p, m);
    if (R <= 1) return orc_tau(s, p, m, mic, (double)n / p->fs);
    int64_t k = n / R;
    double u = (double)(n - k * R) / (double)R;
    double v[4];
    for (int q = 0; q < 4; ++q) v[q] = orc_tau(s, p, m, mic, (double)((k - 1 + q) * R) / p->fs);
    return orc_catmull_rom(v, u);
}

/* Grid of exact delays for one (image, mic): g[k+1] = tau(kR/fs), k = -1 .. nk+1. */
static double* tau_grid(const orc_scene* s, const orc_params* p, const int32_t m[3], int mic, int R, int64_t* len)
{
    int64_t nk = (s->n_out + R - 1) / R;
    int64_t L = nk + 3;
    double* g = (double*)malloc(sizeof(double) * L);
    for (int64_t k = -1; k <= nk + 1; ++k) g[k + 1] = orc_tau(s, p, m, mic, (double)(k * R) / p->fs);
    *len = L;
    return g;
}

/* ------------------------------------------------------------- synthesis */

typedef struct {
    int64_t n_img;
    int32_t* m;
    int32_t* hits;
    double* beta;
} img_set;

static img_set make_images(const orc_scene* s, const orc_params* p)
{
    img_set I;
    I.n_img = orc_count_images(p->max_order);
    I.m = (int32_t*)malloc(sizeof(int32_t) * 3 * I.n_img);
    I.hits = (int32_t*)malloc(sizeof(int32_t) * 6 * I.n_img);
    I.beta = (double*)malloc(sizeof(double) * I.n_img);
    orc_images(s->beta, p->max_order, I.m, I.hits, I.beta);
    return I;
}

static void free_images(img_set* I) { free(I->m); free(I->hits); free(I->beta); }

/* Per-(image, mic) delay source: cached grid (tiered, all outputs) or on the fly. */
typedef struct {
    const orc_scene* s;
    const orc_params* p;
    double** grid;   /* [n_img] or NULL */
    int* R;          /* [n_img] */
} delay_src;

static double delay_of(const delay_src* ds, const img_set* I, int64_t i, int mic, int64_t n)
{
    const int32_t* m = I->m + 3 * i;
    if (ds->grid && ds->grid[i]) {
        int R = ds->R[i];
        int64_t k = n / R;
        double u = (double)(n - k * R) / (double)R;
        return orc_catmull_rom(ds->grid[i] + k, u);   /* grid[k] holds tau at (k-1)R */
    }
    return tau_at(ds->s, ds->p, m, mic, n);
}

static void build_grids(delay_src* ds, const img_set* I, int mic)
{
    ds->grid = (double**)calloc(I->n_img, sizeof(double*));
    ds->R = (int*)calloc(I->n_img, sizeof(int));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < I->n_img; ++i) {
        int R = decim_of(ds->s, ds->p, I->m + 3 * i);
        ds->R[i] = R;
        if (R > 1) {
            int64_t len;
            ds->grid[i] = tau_grid(ds->s, ds->p, I->m + 3 * i, mic, R, &len);
        }
    }
}

static void free_grids(delay_src* ds, int64_t n)
{
    if (!ds->grid) return;
    for (int64_t i = 0; i < n; ++i) free(ds->grid[i]);
    free(ds->grid); free(ds->R);
    ds->grid = NULL; ds->R = NULL;
}

/* Contribution of image i to output n of one mic: gain and filtered signal.
 * s_i(n) = sum_j h(j - mu) x[n - floor(D) - j], j = -T/2+1 .. T/2, D = fs tau, mu = D - floor(D). */
static double filtered(const orc_params* p, const double* x, int64_t n_in, int64_t n, double tau)
{
    double D = p->fs * tau;
    double Kf = floor(D);
    double mu = D - Kf;
    int64_t K = (int64_t)Kf;
    int T = p->taps;
    double acc = 0.0;
    for (int j = -T / 2 + 1; j <= T / 2; ++j) {
        int64_t idx = n - K - j;
        if (idx < 0 || idx >= n_in) continue;
        acc += orc_kernel((double)j - mu, T, p->kaiser_beta, p->cutoff) * x[idx];
    }
    return acc;
}

/* y[mic][k] for output samples idx[k] (or all n_out samples when idx is NULL). */
int orc_forward(const orc_scene* s, const orc_params* p, const double* x,
                int64_t n_idx, const int64_t* idx, double* y)
{
    img_set I = make_images(s, p);
    int64_t ny = idx ? n_idx : s->n_out;
    if (idx) {
        /* listed outputs: every (mic, output) pair is one task (delays solved where
         * needed); each output's sum over images runs in image order */
        delay_src ds = {s, p, NULL, NULL};
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t t = 0; t < (int64_t)s->n_mics * ny; ++t) {
            const int mic = (int)(t / ny);
            const int64_t k = t - (int64_t)mic * ny;
            const int64_t n = idx[k];
            double acc = 0.0;
            for (int64_t i = 0; i < I.n_img; ++i) {
                if (I.beta[i] == 0.0) continue;
                double tau = delay_of(&ds, &I, i, mic, n);
                double g = I.beta[i] / (4.0 * M_PI * p->c * tau);
                acc += g * filtered(p, x, s->n_in, n, tau);
            }
            y[(int64_t)mic * ny + k] = acc;
        }
        free_images(&I);
        return 0;
    }
    for (int mic = 0; mic < s->n_mics; ++mic) {
        delay_src ds = {s, p, NULL, NULL};
        if (tiered(p)) build_grids(&ds, &I, mic);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < ny; ++k) {
            int64_t n = k;
            double acc = 0.0;
            for (int64_t i = 0; i < I.n_img; ++i) {
                if (I.beta[i] == 0.0) continue;
                double tau = delay_of(&ds, &I, i, mic, n);
                double g = I.beta[i] / (4.0 * M_PI * p->c * tau);
                acc += g * filtered(p, x, s->n_in, n, tau);
            }
            y[(int64_t)mic * ny + k] = acc;
        }
        free_grids(&ds, I.n_img);
    }
    free_images(&I);
    return 0;
}

/* With few non-zero output gradients the tier-emulating delays are evaluated
 * where needed (tau_at: the same Catmull-Rom of the same exact grid delays)
 * instead of over every grid point first. */
static int sparse_ok(const orc_scene* s, int64_t n_nz) { return n_nz * 64 < s->n_out; }

/* Exact transpose of the forward map x -> y:
 * gx[m] = sum_{mic,i,n} gy[mic][n] g_i(n) h(j - mu_i(n)) where m = n - floor(D_i(n)) - j. */
int orc_adjoint_x(const orc_scene* s, const orc_params* p, const double* gy, double* gx)
{
    img_set I = make_images(s, p);
    int T = p->taps;
    memset(gx, 0, sizeof(double) * s->n_in);
    int64_t* nz = (int64_t*)malloc(sizeof(int64_t) * (s->n_out > 0 ? s->n_out : 1));
    for (int mic = 0; mic < s->n_mics; ++mic) {
        const double* g_y = gy + (int64_t)mic * s->n_out;
        /* the outputs with a non-zero gradient, in increasing n */
        int64_t n_nz = 0;
        for (int64_t n = 0; n < s->n_out; ++n)
            if (g_y[n] != 0.0) nz[n_nz++] = n;
        if (n_nz == 0) continue;
        delay_src ds = {s, p, NULL, NULL};
        if (tiered(p) && sparse_ok(s, n_nz) == 0) build_grids(&ds, &I, mic);
#pragma omp parallel
        {
            double* part = (double*)calloc(s->n_in, sizeof(double));
#pragma omp for schedule(dynamic, 4)
            for (int64_t i = 0; i < I.n_img; ++i) {
                if (I.beta[i] == 0.0) continue;
                for (int64_t q = 0; q < n_nz; ++q) {
                    const int64_t n = nz[q];
                    double tau = delay_of(&ds, &I, i, mic, n);
                    double g = I.beta[i] / (4.0 * M_PI * p->c * tau);
                    double D = p->fs * tau;
                    double Kf = floor(D), mu = D - Kf;
                    int64_t K = (int64_t)Kf;
                    for (int j = -T / 2 + 1; j <= T / 2; ++j) {
                        int64_t m = n - K - j;
                        if (m < 0 || m >= s->n_in) continue;
                        part[m] += g_y[n] * g * orc_kernel((double)j - mu, T, p->kaiser_beta, p->cutoff);
                    }
                }
            }
#pragma omp critical
            for (int64_t m = 0; m < s->n_in; ++m) gx[m] += part[m];
            free(part);
        }
        free_grids(&ds, I.n_img);
    }
    free(nz);
    free_images(&I);
    return 0;
}

/* d loss / d beta_w for loss gradient gy = dL/dy.  The output is linear in each
 * image gain, and beta_i = prod_w beta_w^{n_w}; so
 * dL/dbeta_w = sum_i (d beta_i / d beta_w) * sum_{mic,n} gy[n] s_i(n) / (4 pi c tau_i(n)),
 * with d beta_i / d beta_w = n_w beta_w^{n_w-1} prod_{w' != w} beta_w'^{n_w'}. */
int orc_grad_beta(const orc_scene* s, const orc_params* p, const double* x, const double* gy, double* gbeta)
{
    img_set I = make_images(s, p);
    double* G = (double*)calloc(I.n_img, sizeof(double));
    int64_t* nz = (int64_t*)malloc(sizeof(int64_t) * (s->n_out > 0 ? s->n_out : 1));
    for (int mic = 0; mic < s->n_mics; ++mic) {
        const double* g_y = gy + (int64_t)mic * s->n_out;
        int64_t n_nz = 0;
        for (int64_t n = 0; n < s->n_out; ++n)
            if (g_y[n] != 0.0) nz[n_nz++] = n;
        if (n_nz == 0) continue;
        delay_src ds = {s, p, NULL, NULL};
        if (tiered(p) && sparse_ok(s, n_nz) == 0) build_grids(&ds, &I, mic);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t i = 0; i < I.n_img; ++i) {
            double acc = 0.0;
            for (int64_t q = 0; q < n_nz; ++q) {
                const int64_t n = nz[q];
                double tau = delay_of(&ds, &I, i, mic, n);
                acc += g_y[n] * filtered(p, x, s->n_in, n, tau) / (4.0 * M_PI * p->c * tau);
            }
            G[i] += acc;
        }
        free_grids(&ds, I.n_img);
    }
    free(nz);
    for (int w = 0; w < 6; ++w) {
        double acc = 0.0;
        for (int64_t i = 0; i < I.n_img; ++i) {
            const int32_t* h = I.hits + 6 * i;
            if (h[w] == 0) continue;
            double d = (double)h[w];
            for (int r = 0; r < h[w] - 1; ++r) d *= s->beta[w];
            for (int v = 0; v < 6; ++v) {
                if (v == w) continue;
                for (int r = 0; r < h[v]; ++r) d *= s->beta[v];
            }
            acc += d * G[i];
        }
        gbeta[w] = acc;
    }
    free(G);
    free_images(&I);
    return 0;
}

/* Exact delays of every image at the given output samples for one mic:
 * tau[i * n_idx + k].  Used to time and inspect the delay model alone. */
int orc_delays(const orc_scene* s, const orc_params* p, int mic, int64_t n_idx, const int64_t* idx, double* tau)
{
    img_set I = make_images(s, p);
    delay_src ds = {s, p, NULL, NULL};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < I.n_img; ++i)
        for (int64_t k = 0; k < n_idx; ++k) tau[i * n_idx + k] = delay_of(&ds, &I, i, mic, idx[k]);
    free_images(&I);
    return 0;
}
