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
    int32_t n_sg;         // supergroups per mic and block: contiguous runs of a block's delay groups
    int32_t blk_begin;    // this scene's delay blocks in the plan's block table
    int32_t n_blk;
    int32_t blk_tiles;    // output tiles per delay block
    int32_t n_tiles;
    int32_t window;       // LDS source window (positions) the plan sized for this scene
    double beta[6];       // wall coefficients (for d/dbeta)
    int32_t src_grad_off; // this scene's first knot in the packed d/dsource array
    int32_t src_knots;    // source knots with a gradient (PWL sources; 0 for circles)
    int64_t v_off;        // this scene's Farrow-filtered source v_k in the workspace (floats)
    int64_t part_base;    // this scene's partial outputs [mic][sg][n_out] in the workspace
    int64_t xw_base;      // its dL/dx windows [mic][sg][tile][xw_stride] (table form)
    int64_t row_base;     // its first row of parameter partials ([mic][sg][tile])
    int64_t u_base;       // its Farrow dL/dx sums [mic][sgw][position][12]
    int32_t xw_stride;    // floats per dL/dx window
    int32_t sgb_stride;   // supergroup bounds per delay block (the plan's stride)
    int32_t dlo_all;      // delay bounds of every group of every block (samples)
    int32_t dhi_all;
    int32_t n_sgw;        // shares of each block's groups in the dL/dx gather's items
    int32_t n_ptiles;     // source-position tiles of the Farrow dL/dx gather
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
    int32_t n_seg;        // ceil(n_out / R)
    int8_t hits[6];       // reflections on each wall (beta_i = prod beta_w^hits_w)
    int8_t pad[2];
    int32_t loc;          // kernels: the image's slot offset (from its PermEntry)
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

// Adjoint slot, after the tracks: the Catmull-Rom transpose partials of the
// group's images, one float4 per (segment, 64-lane chunk of the tile) pair an
// image touches (at most its slot segments plus TO / 64 more), the per-wave sums
// of dL/dbeta_i ([gmax][16]), and the segments' transpose sums (float4 per slot
// segment).
__host__ __device__ constexpr int64_t adj_slot_bytes(int slot_segs, int gmax, int TO)
{
    return slot_extra_off(slot_segs, gmax) + slot_al(((int64_t)slot_segs + (int64_t)gmax * (TO / 64)) * 16) +
           slot_al((int64_t)gmax * 16 * 4) + slot_al((int64_t)slot_segs * 16);
}

// Threads of the backward kernels' workgroups (their register budget needs it).
constexpr int kAdjThreads = 512;

// Images per delay group at most (their slot offsets are staged in LDS).
constexpr int kMaxGroup = 512;
// LDS for a group's slot offsets (grid and segment offsets, with totals).
constexpr size_t kLscBytes = (size_t)8 * (kMaxGroup + 2);
// Source knots with a gradient per scene at most, and a parameter row: dL/dbeta_w
// (6) then dL/d(knot j, axis a) at 6 + 3 j + a.
constexpr int kMaxGradKnots = 32;
constexpr int kRowWidth = 6 + 3 * kMaxGradKnots;
// LDS of the parameter accumulators: per wave its knot sums, then per wave 12
// doubles of block-reduction scratch (backward workgroups have at most 8 waves).
constexpr int kParamWaves = 8;
constexpr size_t kParamLdsBytes = (size_t)8 * kParamWaves * (3 * kMaxGradKnots + 12);

// Floats per source position of the Farrow-filtered signals (v_0..v_11, zero padded).
constexpr int kFarrowStride = 12;

// A delay group: the images perm[img_begin .. img_end) of the plan's permutation
// (consecutive in the block's delay order) whose delays, in samples, are bounded
// by [dmin, dmax] for every mic at every output of the block.
struct DGroup {
    int32_t img_begin;
    int32_t img_end;
    int32_t dmin;
    int32_t dmax;
};

// A delay block of a scene (blk_tiles output tiles): its delay groups.
struct DBlock {
    int32_t grp_begin;
    int32_t n_grp;
};

// An image of a delay group: its index among the scene's images, and its first
// segment in a workgroup's track slot (the images of a group hold
// slot_segs_of(R, span) segments each, in group order).
struct PermEntry {
    int32_t img;
    int32_t loc;
};


constexpr int kStatusWindow = 1;

// ---- kernel launchers (msim_kernels.hip) ----
// The plan's device tables the kernels read: scenes, images, delay blocks, delay
// groups and the groups' image permutation.
struct PlanView {
    const DScene* scenes;
    const DImage* imgs;
    const DBlock* blocks;
    const DGroup* groups;
    const PermEntry* perm;
};

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

// The adjoint part of a workgroup's slot.
struct AdjSlot {
    float4* dpart;
    float* esum;
    float4* dseg;
};

// What the parameter reductions need: the rows of partials, the largest group,
// the largest decimation, dL/dbeta_i's constant fs / (4 pi c), and which
// gradients are wanted.
struct ParamArgs {
    double* rows;
    int gmax;
    int rmax;
    float ghat;
    int want_beta;
    int want_src;
};

hipError_t launch_synth(int taps, int nthreads, int rb, int n_wg, int window, const PlanView& pv,
                        const float4* d_table, int L, const WorkItem* items, int n_items, int32_t* ticket,
                        const TrackArgs& ta, const float* x, float* part, int32_t* d_status, hipStream_t st);
hipError_t launch_reduce_sg(const DScene* d_scenes, int n_scenes, const int64_t* d_y_prefix, int64_t y_total,
                            const float* part, float* y, hipStream_t st);

// Tap quads of the half table that carry the quadratic term: those within 3/4 of
// the half-width for 32 and 64 taps, within half of it for 96 and 128.  Further
// out the table stores zero second differences: the kernel's curvature there is
// small against its edge values (a Kaiser-windowed sinc, beta = 8), and the
// predicted table error (fd error model, which reads the stored values) grows by
// at most 0.9e-6 at 64 phases and 0.3e-6 at 128 for 96 and 128 taps, while the
// longer filters' tap loops drop a third of their second-difference FMAs.
__host__ __device__ constexpr int qcorr_quads(int taps) { return taps >= 96 ? taps / 16 : taps / 8 - taps / 32; }
// Phase counts of the quadratic FD table compiled into the kernels (immediate
// table offsets; other counts read it at run time): the default, and the coarser
// one the planner may take so that two outputs per lane fit a faster path.
constexpr int kTablePhases = 128;
constexpr int kPairTablePhases = 64;
// Rows per tap quad of the quadratic FD table: rows -1 .. Lq-1.
__host__ __device__ constexpr int qtab_pitch(int Lq) { return Lq + 1; }
// Bytes of the quadratic FD table ([Y | D1 | D2], 40 B per quad row).
__host__ __device__ constexpr size_t qtab_bytes(int taps, int Lq)
{
    return (size_t)(taps / 8) * (size_t)qtab_pitch(Lq) * 40;
}
size_t synth_lds_bytes(int taps, int Lq, int window);

// ---- adjoint launchers (msim_adjoint.hip) ----
size_t adj_x_lds_bytes(int taps, int L, int window, int tile);
size_t adj_track_lds_bytes(int taps, int Lq, int window);
hipError_t launch_adjx(int taps, int tile, int n_wg, int window, const PlanView& pv, const float* d_atab, int Lq,
                       const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* gy,
                       float* xwin, int32_t* d_status, hipStream_t st);
hipError_t launch_reduce_x(const PlanView& pv, int n_scenes, const int64_t* d_x_prefix, int64_t x_total, int nthreads,
                           int taps, const int2* d_sgb, const float* xwin, float* gx, hipStream_t st);
hipError_t launch_adjp(int taps, int nthreads, int rb, int n_wg, int window, const PlanView& pv,
                       const float4* d_qtable, int Lq, const WorkItem* items, int n_items, int32_t* ticket,
                       const TrackArgs& ta, const float* x, const float* gy, const ParamArgs& pa, int32_t* d_status,
                       hipStream_t st);
hipError_t launch_reduce_rows(const PlanView& pv, int n_scenes, int scene0, const double* rows, double* gbeta,
                              double* gsrc, hipStream_t st);
int max_grad_knots();

// ---- Farrow launchers (msim_farrow.hip) ----
size_t farrow_lds_bytes(int window);
hipError_t launch_farrow_conv(const DScene* d_scenes, int n_scenes, const int64_t* d_vprefix, int64_t total, int taps,
                              const float* d_coef, const float* x, float* v, hipStream_t st);
int farrow_outputs_per_lane(const int32_t* decim, int n_tiers);
hipError_t launch_farrow(int nthreads, int rb, int n_wg, int window, int taps, int order, const PlanView& pv,
                         const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* v,
                         float* part, int32_t* d_status, hipStream_t st);
// LDS of the Farrow gain/delay adjoint and of the dL/dx gather.
size_t farrow_gd_lds_bytes(int window);
size_t farrow_u_lds_bytes(int window);
// rb: outputs per lane (2 needs tile = 2 kAdjThreads and every decimation 1 or even).
hipError_t launch_farrow_gd(int tile, int rb, int n_wg, int window, int taps, int order, const PlanView& pv,
                            const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* v,
                            const float* gy, const ParamArgs& pa, int32_t* d_status, hipStream_t st);
// The dL/dx gather over the delay blocks' groups; order: the Farrow degree M.
hipError_t launch_farrow_u(int nthreads, int n_wg, int window, int taps, int order, int fwd_tile, const PlanView& pv,
                           const WorkItem* items, int n_items, int32_t* ticket, const TrackArgs& ta, const float* gy,
                           float* upart, int32_t* d_status, hipStream_t st);
hipError_t launch_farrow_u_reduce(const PlanView& pv, int n_scenes, const int64_t* d_vprefix, int64_t vtotal, int taps,
                                  const float* upart, float* u, hipStream_t st);
// scenes s0 .. s0 + n_scenes - 1 (max_in: their largest input length)
hipError_t launch_farrow_corr(const PlanView& pv, int s0, int n_scenes, int64_t max_in, int taps, const float* d_coef,
                              const float* u, float* gx, hipStream_t st);

}  // namespace msim
