// Internal structures shared by the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace msim {

// Trajectory kinds (as in the C-ABI): piecewise linear, horizontal circle.
constexpr int kTrajPwl = 0, kTrajCircle = 1;

// A trajectory as the kernels see it: knot times and positions live in the
// plan's knot array (times at knot_off, xyz triples at pos_off).
struct DTraj {
    int32_t kind;
    int32_t n_points;
    int32_t knot_off;
    int32_t pos_off;
    double center[3];
    double radius;
    double omega;     // angular rate speed/radius (circle)
    double phase0;
};

struct DScene {
    double size[3];
    DTraj src;
    DTraj rcv;
    int32_t n_mics;
    int32_t mic_off;      // index of this scene's first offset triple in the mic array
    int64_t n_in;
    int64_t n_out;
    int64_t x_off;        // packed signal offsets
    int64_t y_off;
    int32_t img_begin;    // this scene's images in the plan's image table
    int32_t n_img;
    int32_t grp_begin;    // this scene's delay groups
    int32_t n_grp;
    int32_t n_sg;         // supergroups per mic: contiguous runs of delay groups, one work item each
    int32_t pad_sg;
    int64_t seg_per_mic;  // track segments of one mic (sum over images)
    int64_t runs_per_mic; // track-kernel blocks of one mic
    int64_t sadj_per_mic; // Catmull-Rom-transpose blocks of one mic
    int32_t n_tiles;
    int32_t window;       // LDS source window (positions) the plan sized for this scene
    double beta[6];       // wall coefficients (for d/dbeta)
    int32_t src_grad_off; // this scene's first knot in the packed d/dsource array
    int32_t src_knots;    // source knots with a gradient (PWL sources; 0 for circles)
    int64_t v_off;        // this scene's Farrow-filtered source v_k in the workspace (floats)
    int64_t grid_base;    // offsets of this scene's delay grid, track segments and partial
    int64_t trk_base;     //   outputs in the workspace (0 when scenes run one at a time)
    int64_t part_base;
};

// One work item of the persistent kernels: an output tile of one mic, summed over
// the delay groups of one supergroup (groups [n_grp sg / n_sg, n_grp (sg+1) / n_sg)).
struct WorkItem {
    int32_t scene;
    int32_t mic;
    int32_t tile;
    int32_t sg;
};

__host__ __device__ inline int sg_begin(int n_grp, int n_sg, int sg) { return (int)((int64_t)n_grp * sg / n_sg); }

// Delay of an image over one grid segment [kR, (k+1)R):
//   D(kR + v) = K + a0 + v (b1 + v (b2 + v b3)),  v = 0 .. R-1,
// the uniform Catmull-Rom cubic through the exact delays at (k-1)R .. (k+2)R.
struct Seg {
    float a0, b1, b2, b3;
};

// One image source.  Position of image m of point q, per axis a:
//   m_a even: m_a L_a + q_a ;  m_a odd: (m_a + 1) L_a - q_a.
struct DImage {
    int16_t m[3];
    int16_t tier;
    int32_t R;            // decimation of its delay grid
    float invR;
    float gfac;           // beta_i * fs / (4 pi c): gain = gfac / D
    int32_t seg_off;      // first track segment within one mic's track
    int32_t n_seg;        // ceil(n_out / R)
    int8_t hits[6];       // reflections on each wall (beta_i = prod beta_w^hits_w)
    int8_t pad[2];
    int32_t run_off;      // first track-kernel block within one mic
    int32_t sadj_off;     // first Catmull-Rom-transpose block within one mic
    int32_t loc;          // first segment of this image in a workgroup's track slot: the
                          // images of a delay group hold slot_segs_of(R, span) segments each,
                          // in group order (grid delays: 3 more per image)
    int32_t pad2;
};

// Segments of decimation R that outputs [n, n + span) touch, for any n: at most this many.
__host__ __device__ constexpr int slot_segs_of(int R, int span) { return (span - 1) / R + 2; }
// Outputs a delay group's track slot covers: an output tile plus the group's delay
// spread and margin (the Farrow dL/dx gather reads the outputs that reach a tile
// of source positions through any delay of the group).
__host__ __device__ constexpr int group_span(int tile, int dmin, int dmax) { return tile + (dmax - dmin) + 16; }

// A workgroup's track slot in global memory (one per workgroup of a persistent
// launch; written and read by that workgroup only): per segment a Seg and its
// integer base, then the FP64 grid delays.
struct Slot {
    Seg* seg;
    int32_t* K;
    double* grid;
};

// Slot layout: Seg[slot_segs], int32[slot_segs], double[slot_segs + 3 gmax] (the
// grid delays), each part 256-byte aligned; kernel-specific scratch follows at
// slot_extra_off.
__host__ __device__ constexpr int64_t slot_al(int64_t b) { return (b + 255) / 256 * 256; }
__host__ __device__ constexpr int64_t slot_extra_off(int slot_segs, int gmax)
{
    return slot_al((int64_t)slot_segs * 16) + slot_al((int64_t)slot_segs * 4) +
           slot_al(((int64_t)slot_segs + 3 * (int64_t)gmax) * 8);
}

// Floats per source position of the Farrow-filtered signals (v_0..v_11, zero padded).
constexpr int kFarrowStride = 12;

// A track-kernel block: kTrackThreads threads, each solving kTrackWalk
// consecutive grid points in time order.  A block emits every segment of an
// audio-rate image (R = 1) it solves, and all but three of a decimated image's,
// whose cubics also need the next two grid points and the one before.
constexpr int kTrackThreads = 256;
constexpr int kTrackWalk = 4;
constexpr int kTrackPoints = kTrackThreads * kTrackWalk;
__host__ __device__ constexpr int track_block_segs(int R) { return R == 1 ? kTrackPoints : kTrackPoints - 3; }

// Segments one block of the Catmull-Rom transpose sums: its outputs (segments x R)
// are staged in LDS, at most kSegAdjStage of them.
constexpr int kSegAdjThreads = 256;
constexpr int kSegAdjStage = 4096;
static_assert(kSegAdjStage >= 4096, "a segment of the largest decimation (4096) must fit the stage");
__host__ __device__ constexpr int seg_adj_block_segs(int R)
{
    return R * kSegAdjThreads <= kSegAdjStage ? kSegAdjThreads : (kSegAdjStage / R > 0 ? kSegAdjStage / R : 1);
}

// Images [img_begin, img_end) of a scene (sorted by delay) whose delays, in
// samples, are bounded by [dmin, dmax] for every mic at every time.
struct DGroup {
    int32_t img_begin;
    int32_t img_end;
    int32_t dmin;
    int32_t dmax;
};


constexpr int kStatusWindow = 1;

// ---- kernel launchers (msim_kernels.hip) ----
hipError_t launch_tracks(const DScene* d_scenes, int scene, const DScene& hs, const DImage* d_imgs,
                         const double* d_knots, const double* d_mics, double* grid, Seg* seg, int32_t* segK,
                         double c, double fs, int delay_model, hipStream_t st);

// What a persistent kernel needs to solve its tracks tile by tile: the plan's
// knots and mic offsets, the physics, and the per-workgroup slots.
struct TrackArgs {
    const double* knots;
    const double* mics;
    double c, fs;
    int model;
    int slot_segs;        // segments per slot
    char* slots;          // n_wg slots of slot_bytes each
    int64_t slot_bytes;
};

hipError_t launch_synth(int taps, int nthreads, int rb, int n_wg, int window, const DScene* d_scenes,
                        const DImage* d_imgs, const DGroup* d_groups, const float4* d_table, int L,
                        const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* x,
                        float* part, int32_t* d_status, hipStream_t st);
hipError_t launch_reduce_sg(const DScene* d_scenes, int n_scenes, const int64_t* d_y_prefix, int64_t y_total,
                            const float* part, float* y, hipStream_t st);

// Tap quads of the half table that carry the quadratic term: those within 3/4 of
// the half-width.  Further out the kernel's second differences are below 1.3e-6
// at 128 phases (taps 3T/8 .. T/2 of a Kaiser-windowed sinc with beta = 8); their
// term, at most 1.5e-7 of the kernel's energy for fractions in [0, 1], is below the
// FP32 rounding of the tap sum, and the table stores them as zero.
__host__ __device__ constexpr int qcorr_quads(int taps) { return taps / 8 - taps / 32; }
// Rows per tap quad of the quadratic FD table: rows -1 .. Lq-1.
__host__ __device__ constexpr int qtab_pitch(int Lq) { return Lq + 1; }
// Bytes of the quadratic FD table ([Y | D1 | D2], 40 B per quad row).
__host__ __device__ constexpr size_t qtab_bytes(int taps, int Lq)
{
    return (size_t)(taps / 8) * (size_t)qtab_pitch(Lq) * 40;
}
size_t synth_lds_bytes(int taps, int Lq, int window);

// ---- adjoint launchers (msim_adjoint.hip) ----
// Scratch of the adjoint of one scene (all carved from the caller's workspace).
struct AdjBufs {
    float* xpart;     // table: [mic][group][tile][window], transpose-delay partial windows;
                      // Farrow: [mic][group][position][12], per-group sums u_k
    float* u;         // Farrow: [position][12], u_k summed over mics and groups
    float* dbar;      // [mic][image][n_out]: d loss / d D_i(n)
    float* gpart;     // [mic][tile * waves][image]: partial sums of d loss / d beta_i
    float4* dseg;     // [mic][segment]: Catmull-Rom transpose weights summed per segment
    double4* pgc;     // [mic][grid point]: d loss / d source position at emission time, and lambda
    int32_t* pga;     // [mic][grid point]: knot index of that emission time
};

size_t adj_x_lds_bytes(int taps, int L, int window, int nthreads);
size_t adj_track_lds_bytes(int taps, int Lq, int window);

hipError_t launch_adj_x(int taps, int nthreads, const DScene& hs, const DImage* d_imgs, const DGroup* d_groups,
                        const float* d_atab, int Lq, const Seg* seg, const int32_t* segK, const float* gy,
                        float* xpart, int32_t* d_status, hipStream_t st);
hipError_t launch_reduce_x(const DScene& hs, const DGroup* d_groups, int nthreads, int taps, const float* xpart,
                           float* gx, hipStream_t st);
hipError_t launch_adj_track(int taps, int nthreads, int rb, const DScene& hs, const DImage* d_imgs,
                            const DGroup* d_groups, const float4* d_qtable, int Lq, const Seg* seg,
                            const int32_t* segK, const float* x, const float* gy, float ghat, float* dbar,
                            float* gpart, int32_t* d_status, hipStream_t st);
hipError_t launch_adj_params(const DScene* d_scenes, int scene, const DScene& hs, const DImage* d_imgs,
                             const double* d_knots, const double* d_mics, const double* grid, const float* dbar,
                             float4* dseg, double4* pgc, int32_t* pga, double c, double fs, int delay_model,
                             int want_src, hipStream_t st);
hipError_t launch_reduce_params(const DScene* d_scenes, int scene, const DScene& hs, const DImage* d_imgs,
                                const float* gpart, int gpart_stride, const double4* pgc, const int32_t* pga,
                                double* partial, double* gbeta, double* gsrc, hipStream_t st);
size_t reduce_partial_bytes(const DScene& hs);
int max_grad_knots();

// ---- Farrow launchers (msim_farrow.hip) ----
size_t farrow_lds_bytes(int window);
hipError_t launch_farrow_conv(const DScene* d_scenes, int n_scenes, const int64_t* d_vprefix, int64_t total, int taps,
                              const float* d_coef, const float* x, float* v, hipStream_t st);
int farrow_outputs_per_lane(const int32_t* decim, int n_tiers);
hipError_t launch_farrow(int nthreads, int rb, int n_wg, int window, int taps, int order, const DScene* d_scenes,
                         const DImage* d_imgs, const DGroup* d_groups, const WorkItem* items, int n_items,
                         int32_t* ticket, const TrackArgs& ta, const float* v, float* part, int32_t* d_status,
                         hipStream_t st);
hipError_t launch_farrow_adjoint(int nthreads, int taps, int order, const DScene& hs, const DImage* d_imgs,
                                 const DGroup* d_groups, const Seg* seg, const int32_t* segK, const float* d_coef,
                                 const float* v, const float* gy, float ghat, float* upart, float* u, float* gx,
                                 float* dbar, float* gpart, int32_t* d_status, hipStream_t st);

}  // namespace msim
