// vi_internal.h -- shared host/device declarations of libvi (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vi.h"

namespace vi {

constexpr int kMaxTF = 1024;     // transfer-function entries staged in LDS
constexpr int kMaxTaps = 49;     // largest gather (7 x 7 lattice)

// ---------------------------------------------------------------------------
// Build pass parameters.  Positions are carried in "offset voxel"
// coordinates h = p*N - 1/2 - M, with M = floor(N/2) an integer, so that
// floor/fraction of the voxel index g = h + M are exact and |h| <= ~0.9 N.
// Column (i,j) at slab k sits at h = B(i,j) + k * AL.  The build carries h as
// a fixed-point number h * 2^kQBits in an int64 (Q40: |h| < 2^23 voxels,
// resolution 2^-40 voxel); the host derives the light frame (Eq. 8, Eq. 10)
// in double and rounds every coefficient to Q40 once.
// ---------------------------------------------------------------------------
constexpr int kQBits = 40;

// Empty-space map: per cell of 2^shift voxels, (min, max) of the normalised
// values over the cell's voxels and the next one along each axis.
// Optional occupancy bits for the frame's transfer function: one bit per
// cell (1 = may hold opacity), staged in LDS by every workgroup.  Used only
// when they fit in kMaxLdsOccWords; larger maps are decided from mm.
// Behind the cell bits lie the bits of the super-cells (4 x 4 x 4 cells):
// set where any of their cells is set, so a ray in empty space can jump a
// whole empty super-cell at once.
struct OccMap {
    const float2* mm;   // nullptr: no skipping
    int shift;
    uint32_t nc;        // cells per axis
    const uint32_t* bits;  // nullptr: decide from mm and the transfer function
    uint32_t words;        // 32-bit words of cell bits (the super-cell bits follow)
    uint32_t snc;          // super-cells per axis, ceil(nc / 4)
    uint32_t swords;       // 32-bit words of super-cell bits
};
constexpr uint32_t kMaxLdsOccWords = 2304;  // 9 KiB of bits (65536 cells and their super-cells)

struct BuildParams {
    const void* vol;
    int vol_dtype;
    int vol_layout;
    uint32_t vsy, vsz;  // per-axis offset strides of the volume layout
    OccMap occ;
    int N, M;
    float scale;
    const float* tf;   // K x 4
    int K;
    void* out;
    int out_dtype;     // VI_F32 transmittance / VI_BF16 optical depth
    int n, res;
    int out_layout;    // VI_STACK_TILED / VI_STACK_ROWS
    uint32_t layer, row_tiles32;  // tiled: R8*R4 per layer, (R8/8)*32 per tile row
    uint32_t rlayer, rpitch, rorg;  // rows: elements per layer, pitch P, element of texel (0,0,0)
    int64_t B0q[3];    // h at (i,j,k) = (0,0,0), Q40
    int64_t BUq[3];    // d h / d i
    int64_t BVq[3];    // d h / d j
    int64_t ALq[3];    // d h / d k (point light: at column (0,0))
    float e;           // slab thickness in voxels: exponent of (1-a)
    float darken;      // exponent m of the (1+alpha)^m slab compensation, 0 = off
    int64_t loq, hiq;  // cube in h coordinates: [-1/2 - M, N - 1/2 - M], Q40
    // point light: column (i,j) advances by ALq + i ALUq + j ALVq per slab,
    // and its slab exponent is that step's length (the ray crosses the
    // slab obliquely)
    int point;
    int64_t ALUq[3], ALVq[3];
};

// ---------------------------------------------------------------------------
// Render pass parameters (one frame).
// ---------------------------------------------------------------------------
struct RenderFrame {
    // volume
    const void* vol;
    int vol_dtype;
    int vol_layout;
    uint32_t vsy, vsz;
    OccMap occ;
    int N, M;
    float scale;
    // transfer function
    const float* tf;
    int K;
    // stack
    const void* stack;
    // rows: the stack advanced by one row, one layer, and one layer and one
    // row, so that the four loads of a lookup share one offset
    const void* stack_r1;
    const void* stack_l1;
    const void* stack_l1r1;
    uint32_t rbase;  // rows: element of light-grid cell (iz, iy, ix) = rbase + iz rlayer + iy rpitch + ix
    int stack_dtype;
    int n, res;
    int stack_layout;
    uint32_t layer, row_tiles32;
    uint32_t rlayer, rpitch, rorg;  // rows: elements per layer, pitch, element of texel (0,0,0)
    int Mz, Mr;          // integer offsets of the light-grid coordinates
    int nearest;         // 1: every lookup reads the face nearest its depth index
    // Light grid as affine maps of the offset-voxel position h; every
    // coefficient is a float pair (value, remainder), so that the per-ray
    // offsets are as accurate as a double set-up would make them:
    float Lq[3], Lql[3], Lq0, Lq0l;  // z = Lq . h + Lq0   (Eq. 9 index minus one, minus Mz)
    float Ux[3], Uxl[3], Ux0, Ux0l;  // x = Ux . h + Ux0   (Eq. 10 texel column minus Mr)
    float Vy[3], Vyl[3], Vy0, Vy0l;  // y = Vy . h + Vy0
    float L[3], U[3], V[3];
    float Ll[3], Ul[3], Vl[3];
    float ds, ids;       // slab thickness in voxels (cone ring radii) and its inverse
    // point light: depth d = L.(h - Ph) and lateral u = U.(h - Ph),
    // v = V.(h - Ph) (voxels) map to x = (u / d) sc + xo, y = (v / d) sc + xo
    int point;
    float Ph[3], Phl[3]; // light position in offset-voxel coordinates
    float sc, xo;
    // camera, in offset-voxel coordinates (float pairs): pixel (px, py)
    // maps to b = cam_b + px cam_sx + py cam_sy; a pinhole ray leaves cam_o
    // along b (normalised), an orthographic ray leaves b along cam_f
    int cam_kind;
    int width, height;
    float cam_o[3], cam_ol[3], cam_f[3], cam_fl[3];
    float cam_b[3], cam_bl[3], cam_sx[3], cam_sxl[3], cam_sy[3], cam_syl[3];
    float lo, hi;        // the cube in h coordinates: [-1/2 - M, N - 1/2 - M]
    // march
    int mode;
    float dt;            // step in voxels (= the reference length of Eq. 6's exponent)
    float idt, idtl;     // 1 / dt as a float pair
    float ambient, light[3], bg[4], term_eps;
    float phong_ka, phong_kd, phong_ks, phong_shin, grad_eps;
    // gather taps in light-grid units (shell: fixed; cone: per ray)
    int ntaps;
    float tap_w;
    float tz[kMaxTaps], tx_[kMaxTaps], ty_[kMaxTaps];  // shell offsets
    float tw[kMaxTaps];                                 // shell tap weights (sum 1)
    float td_[kMaxTaps];                                // point light: depth offsets (tx_, ty_ then
                                                        // hold lateral offsets), voxels
    int cone_rings, cone_angles, cone_grid;
    float cone_tan;
    float cone_cos[16], cone_sin[16];
    // output
    float4* out;
    unsigned long long* samples;  // [0] segments marched, [1] (count_opaque) segments composited with alpha > 0
    int count_opaque;
};

// launchers (vi_build.hip / vi_render.hip / vi_layout.hip)
hipError_t launch_build(const BuildParams& p, hipStream_t s);
hipError_t launch_render(const RenderFrame& f, hipStream_t s);
// one launch over `ntiles` tiles whose frames all have kernel_mode() `mode`
// (maxK / max_occ_words: the largest transfer function and LDS occupancy
// bits of the frames, which size the launch's LDS)
hipError_t launch_render_batch(int vol_dtype, int layout, int stack_dtype, int stack_layout, int mode,
                               const RenderFrame* d_frames, const uint32_t* d_tiles, uint32_t ntiles, int maxK,
                               uint32_t max_occ_words, hipStream_t s);
hipError_t launch_to_bricks(const void* src, void* dst, int dtype, int N, hipStream_t s);
hipError_t launch_to_quads(const void* src, void* dst, int dtype, int N, hipStream_t s);
hipError_t launch_minmax(const void* vol, int dtype, int layout, uint32_t vsy, uint32_t vsz, int N, float scale,
                         int shift, float* out, hipStream_t s);
hipError_t launch_occupancy(const float* minmax, uint32_t nc, const float* tf, int K, uint32_t* bits,
                            hipStream_t s);

// Kernel variants beyond the public modes: for a point light the light grid
// is a perspective frustum (every stack lookup divides by its depth),
// Phong's light vector points at the light from each sample and the cone's
// axis is the light's direction at each sample (ring and lattice forms in
// one kernel); the directional cone's lattice form is a kernel of its own
// (its best tap batching and register budget differ from the ring form's).
constexpr int kModePointShadow = 5, kModePointShell = 6, kModePointPhong = 7, kModeConeGrid = 8,
              kModePointCone = 9, kKernelModes = 10;
inline int kernel_mode(const RenderFrame& f)
{
    if (f.point && f.mode == VI_MODE_SHADOW) return kModePointShadow;
    if (f.point && f.mode == VI_MODE_SHELL) return kModePointShell;
    if (f.point && f.mode == VI_MODE_PHONG) return kModePointPhong;
    if (f.point && f.mode == VI_MODE_CONE) return kModePointCone;
    if (f.mode == VI_MODE_CONE && f.cone_grid > 0) return kModeConeGrid;
    return f.mode;
}

// host helpers shared by the API and the server
int make_frame(const vi_volume* vol, const vi_tf* tf, const vi_slices* sl, const vi_camera* cam, int mode,
               float step_vox, const vi_render_opts* opts, float* d_rgba, unsigned long long* d_samples,
               RenderFrame* out);
int fail_msg(int code, const char* msg);  // set the thread's vi_last_error message
inline uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }

}  // namespace vi
