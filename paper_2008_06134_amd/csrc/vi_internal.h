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
// Column (i,j) at slab k sits at h = B(i,j) + k * AL, with B evaluated in
// double on the device once per column.
// ---------------------------------------------------------------------------
// Empty-space map: per cell of 2^shift voxels, (min, max) of the normalised
// values over the cell's voxels and the next one along each axis.
// Optional occupancy bits for the frame's transfer function: one bit per
// cell (1 = may hold opacity), staged in LDS by every workgroup.  Used only
// when they fit in kMaxLdsOccWords; larger maps are decided from mm.
struct OccMap {
    const float2* mm;   // nullptr: no skipping
    int shift;
    uint32_t nc;        // cells per axis
    const uint32_t* bits;  // nullptr: decide from mm and the transfer function
    uint32_t words;        // 32-bit words of bits
};
constexpr uint32_t kMaxLdsOccWords = 2048;  // 8 KiB of bits (65536 cells)

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
    uint32_t rlayer, rpitch, rorg;  // rows: (res+2)*P elements per layer, pitch P, texel 0 at column rorg
    double B0[3];      // h at (i,j,k) = (0,0,0)
    double BU[3];      // d h / d i
    double BV[3];      // d h / d j
    float AL[3];       // d h / d k
    float e;           // slab thickness in voxels: exponent of (1-a)
    float darken;      // exponent m of the (1+alpha)^m slab compensation, 0 = off
    float lo, hi;      // cube in h coordinates: [-1/2 - M, N - 1/2 - M]
    // point light: column (i,j) advances by AL0 + i ALU + j ALV per slab,
    // and its slab exponent is that step's length (the ray crosses the
    // slab obliquely)
    int point;
    double AL0[3], ALU[3], ALV[3];
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
    int stack_dtype;
    int n, res;
    int stack_layout;
    uint32_t layer, row_tiles32;
    uint32_t rlayer, rpitch, rorg;
    int Mz, Mr;          // integer offsets of the light-grid coordinates
    double Lq[3], Lq0;   // z = Lq . p + Lq0 - Mz       (Eq. 9 index minus one)
    double Ux[3], Ux0;   // x = Ux . p + Ux0 - Mr       (Eq. 10 texel column)
    double Vy[3], Vy0;   // y = Vy . p + Vy0 - Mr
    double L[3], U[3], V[3];
    double ds;
    // point light: depth d = L.(p - P) and lateral u = U.(p - P), v = V.(p - P)
    // map to z = (d - dmin) zs - 1 - Mz, x = (u / d) sc + xo, y = (v / d) sc + yo
    int point;
    double P[3], dmin;
    float zs, sc, xo;
    // camera
    int cam_kind;
    int width, height;
    double eye[3], fwd[3], right[3], up[3];
    double tx, ty;       // persp: tan(fovy/2)*W/H, tan(fovy/2); ortho: h*W/H, h
    // march
    int mode;
    double dt;           // step in world units
    float N_f;           // voxels per world unit (segment exponent scale)
    float ambient, light[3], bg[4], term_eps;
    float phong_ka, phong_kd, phong_ks, phong_shin, grad_eps;
    // gather taps in light-grid units (shell: fixed; cone: per ray)
    int ntaps;
    float tap_w;
    float tz[kMaxTaps], tx_[kMaxTaps], ty_[kMaxTaps];  // shell offsets
    float tw[kMaxTaps];                                 // shell tap weights (sum 1)
    float td_[kMaxTaps];                                // point light: depth offsets (tx_, ty_ then
                                                        // hold world-frame lateral offsets)
    int cone_rings, cone_angles, cone_grid;
    float cone_tan;
    float cone_cos[16], cone_sin[16];
    // output
    float4* out;
    unsigned long long* samples;
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
hipError_t launch_occupancy(const float* minmax, uint32_t cells, const float* tf, int K, uint32_t* bits,
                            hipStream_t s);

// Kernel variants beyond the public modes: for a point light the light grid
// is a perspective frustum (every stack lookup divides by its depth) and
// Phong's light vector points at the light from each sample; the cone's
// lattice form is a kernel of its own (its best tap batching and register
// budget differ from the ring form's).
constexpr int kModePointShadow = 5, kModePointShell = 6, kModePointPhong = 7, kModeConeGrid = 8,
              kKernelModes = 9;
inline int kernel_mode(const RenderFrame& f)
{
    if (f.point && f.mode == VI_MODE_SHADOW) return kModePointShadow;
    if (f.point && f.mode == VI_MODE_SHELL) return kModePointShell;
    if (f.point && f.mode == VI_MODE_PHONG) return kModePointPhong;
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
