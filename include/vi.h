/*
 * vi.h -- C ABI of libvi: slice-based ray-casting volume illumination on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: D. Luo, "Interactive volume illumination of slice-based ray
 * casting" (arXiv 2008.06134).  Two passes:
 *   1. vi_build_attenuation -- the light-space illumination attenuation
 *      buffer (section 3.2.1, Alg. 1): the volume is cut into n slabs
 *      perpendicular to the light between the minimum and maximum light
 *      distances of the unit cube (Eq. 8); opacity is composited slab by
 *      slab (Eq. 4 applied to opacity) and the running transmittance after
 *      every slab is stored as one res x res layer.
 *   2. vi_render -- single-pass ray casting from the camera (section 4):
 *      per sample a trilinear volume fetch, a transfer-function lookup,
 *      the illumination coefficient gathered from the stack (section 3:
 *      direct shadow; section 3.2.3: shell or cone distribution; slice
 *      index by Eq. 9, slice UV by Eq. 10), emission weighted by that
 *      coefficient (Eq. 7) and front-to-back compositing (Eq. 3) with
 *      early ray termination.
 *
 * Geometry conventions (the paper leaves these open; the library fixes):
 *   - the volume fills the unit cube [0,1]^3; voxel (x,y,z) is centred at
 *     ((x+1/2)/N, (y+1/2)/N, (z+1/2)/N); cubic volumes only (N^3), stored
 *     linearly (x fastest) or in 4x4x4 bricks (vi_layout);
 *   - sampling is trilinear with clamp-to-edge; value = clamp(raw*scale,0,1)
 *     per voxel before interpolation;
 *   - the transfer function holds K RGBA float entries (non-premultiplied
 *     colour, alpha per one voxel of path length) looked up linearly at
 *     x = value*(K-1); a segment of length l has opacity 1-(1-a)^(l*N)
 *     (the extinction form of Eq. 6);
 *   - light_dir is the direction the light travels; slab k spans
 *     [dmin + k ds, dmin + (k+1) ds] along it and is sampled at its middle;
 *     layer k holds the transmittance after slab k;
 *   - the light projection is orthographic over the square of half-width
 *     sqrt(3)/2 about the cube centre in the (U,V) plane, V = L x U, U from
 *     the coordinate axis least aligned with L;
 *   - a stack lookup interpolates linearly in depth between layer faces
 *     (index q of Eq. 9 lies between faces floor(q) and ceil(q); face f
 *     holds layer f-1, face 0 is fully transmitting) and bilinearly inside
 *     a layer; outside the texel grid the stack transmits fully;
 *   - rays: pixel centres, y = 0 on top; segments of step_vox/N from the
 *     cube entry with a shorter last segment, sampled at their middles;
 *     termination once 1 - alpha_dst <= term_eps; premultiplied RGBA out,
 *     background composited last.
 *
 * Memory: every large buffer (volume, transfer function, stack, image,
 * sample counter) is a DEVICE pointer owned by the caller; the library
 * allocates nothing for vi_build_attenuation / vi_render.  All work is
 * enqueued asynchronously on `stream` (a hipStream_t; NULL = the null
 * stream); the call returns after the launch.  Buffers must stay valid
 * until that work completes.
 *
 * Errors: every int-returning call returns VI_OK (0) or a negative code;
 * nothing throws across the ABI.  vi_last_error() returns a message for
 * the calling thread's last failure.  Launch failures are reported as
 * VI_E_DEVICE with the HIP error text in the message.
 */
#ifndef VI_H
#define VI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VI_OK 0
#define VI_E_INVALID_ARG (-1)
#define VI_E_UNSUPPORTED (-2)
#define VI_E_NO_MEMORY (-3)
#define VI_E_DEVICE (-4)
#define VI_E_BUSY (-5)
#define VI_E_CANCELLED (-6)

typedef void* vi_stream_t; /* a hipStream_t */

typedef enum {
    VI_U8 = 0,   /* volume: unsigned 8-bit                              */
    VI_U16 = 1,  /* volume: unsigned 16-bit                             */
    VI_F16 = 2,  /* volume: IEEE half; stack: half transmittance (rows)  */
    VI_F32 = 3,  /* volume: float; stack: float transmittance           */
    VI_BF16 = 4  /* stack: bfloat16 optical depth -log2 T (precision form) */
} vi_dtype;

typedef enum {
    VI_MODE_NONE = 0,   /* coefficient 1: unlit emission-absorption        */
    VI_MODE_SHADOW = 1, /* transmittance at the sample itself (section 3)  */
    VI_MODE_SHELL = 2,  /* shell distribution (section 3.2.3)              */
    VI_MODE_CONE = 3,   /* cone distribution (section 3.2.3, Eq. 11)       */
    VI_MODE_PHONG = 4   /* local Phong model, the comparison mode of section 4:
                           central-difference normals, no stack read       */
} vi_mode;

typedef enum { VI_CAM_ORTHO = 0, VI_CAM_PERSP = 1 } vi_camera_kind;

/* Volume layouts in device memory (N = edge, NP = N rounded up to 4,
 * nb = NP / 4):
 *   VI_LAYOUT_LINEAR: raw[z][y][x], element (x,y,z) at (z*N + y)*N + x;
 *   VI_LAYOUT_BRICK4: 4x4x4 bricks, bricks ordered z,y,x; element (x,y,z)
 *     at ((z/4)*nb*nb + (y/4)*nb + x/4)*64 + (z%4)*16 + (y%4)*4 + x%4,
 *     NP^3 elements (padding never read).  A trilinear footprint then
 *     touches one to eight 64-element bricks instead of four rows, which is
 *     what the gathers of both passes pay for.
 *   VI_LAYOUT_QUAD4: the slots of VI_LAYOUT_BRICK4, each holding the 2x2
 *     neighbourhood of its voxel in one 4-element unit: slot (x,y,z) =
 *     { v(x,y,z), v(x+1,y,z), v(x,y+1,z), v(x+1,y+1,z) } with indices
 *     clamped to N-1, at elements 4*brick_offset(x,y,z) + 0..3 (4*NP^3
 *     elements, 4x the bytes).  A trilinear footprint is then two loads (one
 *     per z) instead of eight; results are the same bit for bit. */
typedef enum { VI_LAYOUT_LINEAR = 0, VI_LAYOUT_BRICK4 = 1, VI_LAYOUT_QUAD4 = 2 } vi_layout;

/* A cubic volume in device memory.  `scale` maps raw values to [0,1]
 * (u8: 1/255, u16 12-bit data: 1/4095, f16/f32 normalised: 1).
 *
 * Optional empty-space map (`minmax`, from vi_volume_minmax): for every
 * cell of `cell`^3 voxels, the minimum and maximum normalised voxel value
 * over the cell's voxels plus the next voxel along each axis, i.e. over
 * every trilinear footprint whose lower corner lies in the cell.  Where all
 * transfer-function entries that such values can reach have zero opacity, a
 * segment's opacity is exactly zero and both passes skip its volume fetch:
 * results are unchanged bit for bit. */
typedef struct {
    const void* data;
    int dtype;  /* VI_U8, VI_U16, VI_F16 or VI_F32 */
    int n;      /* edge length N >= 2; < 2^32 bytes per copy of the voxels */
    float scale;
    int layout; /* VI_LAYOUT_LINEAR (0), VI_LAYOUT_BRICK4 or VI_LAYOUT_QUAD4 */
    const float* minmax; /* NULL, or ceil(n/cell)^3 (min, max) float pairs, cells x fastest */
    int cell;            /* cell edge in voxels (4, 8, 16 or 32) when minmax is set */
    const uint32_t* occ; /* NULL, or occupancy bits from vi_volume_occupancy (needs minmax) */
    uint64_t occ_tag;    /* identity of the (volume, map, transfer function) the bits were made for */
} vi_volume;

/* Transfer function: `n_entries` x 4 floats (r,g,b,a) in device memory,
 * 2 <= n_entries <= 1024.  Opacities outside [0, 1] are clamped to it.
 * `tag` names the table's contents: vi_tf_tag() of the same table in host
 * memory, set by the caller whenever it writes the table.  Stacks and
 * occupancy bits made with one table are then refused with another, also
 * one that reuses the device address of a freed table.  tag = 0 leaves the
 * table identified by its device pointer alone (a table rewritten in place
 * then goes undetected). */
typedef struct {
    const float* rgba;
    int n_entries;
    uint64_t tag;
} vi_tf;

/* Stack layouts.  Texel (k, j, i): layer k, row j (along V), column i
 * (along U); T = 1 outside the res x res grid.
 *   VI_STACK_TILED: every layer in 8 x 4 texel tiles; with R8 = res rounded
 *     up to 8 and R4 = res rounded up to 4, texel (k, j, i) is element
 *       k*R8*R4 + ((j/4)*(R8/8) + i/8)*32 + (j%4)*8 + i%8
 *     (padding never read).  n*R8*R4 elements.
 *   VI_STACK_ROWS: every layer row-major with a border two texels wide of
 *     fully transmitting texels (T = 1, optical depth 0) around the grid,
 *     one leading layer k = -1 that transmits fully everywhere (face 0 of
 *     the depth index of Eq. 9), and one trailing layer k = n equal to
 *     layer n-1 (the light leaving the last slab).  The two texels of a
 *     bilinear row, (k, j, i) and (k, j, i+1), are adjacent, so one load
 *     per row reads them, and every footprint of a lookup, clamped to i, j
 *     in [-2, res] and k in [-1, n-1] (with its second layer k+1), reads
 *     stored texels only.  With row pitch P = res+4 rounded up to 4 and
 *     LS = the least odd multiple of h from (res+4)*P up, h = 16 for VI_F32
 *     and 32 for the 2-byte dtypes (half a 128-byte line), texel (k, j, i),
 *     k in [-1, n], i and j in [-2, res+1], is element
 *     (k+1)*LS + (j+2)*P + (i+2); (n+2)*LS elements
 *     (columns res+4 .. P-1 and a layer's last LS - (res+4)*P elements are
 *     never read).  The same texel of neighbouring layers lies half a line
 *     apart; in a buffer aligned to 128 bytes every other layer starts on a
 *     line and the build writes whole lines but for two half-lines per
 *     workgroup and layer (any 16-byte aligned buffer is correct, more
 *     slowly). */
typedef enum { VI_STACK_TILED = 0, VI_STACK_ROWS = 1 } vi_stack_layout;

/* Attenuation stack descriptor, filled by vi_build_attenuation (or by
 * vi_light_frame for the geometry alone).  `data` points at the caller's
 * buffer of vi_slices_bytes(n, res, dtype, layout) bytes in `layout`.  F32
 * stores transmittance T_k; BF16 stores optical depth in base-2 units,
 * tau_k = -log2 T_k, so T_k = 2^-tau_k (0 outside the grid).
 * Geometry is kept in double as computed on the host (Eq. 8). */
typedef struct {
    void* data;
    int dtype;          /* VI_F32, VI_BF16 or VI_F16 (VI_F16: row layout only) */
    int layout;         /* VI_STACK_TILED or VI_STACK_ROWS */
    int n, res;         /* slabs, texels per side */
    double L[3];        /* unit propagation direction */
    double U[3], V[3];  /* light-plane basis */
    double c[3];        /* cube centre */
    double dmin, dmax;  /* Eq. 8 */
    double ds;          /* slab thickness (dmax - dmin) / n */
    double R;           /* half-width of the light square: sqrt(3)/2, or at unit depth for a point light */
    int vol_n;          /* edge of the volume it was built from */
    uint64_t tag;       /* identity of (volume, transfer function); 0 = unchecked */
    float darken;       /* build option it was built with (vi_build_opts) */
    int positional;     /* 1: point light at P; L is then its axis (toward the cube centre) */
    double P[3];
} vi_slices;

/* Build options; NULL means all defaults. */
typedef struct {
    /* 0: plain Eq. 4 product.  m > 0: the compensation of section 4 --
     * every slab's transmitted fraction (1-alpha) is multiplied by
     * (1+alpha)^m and capped at 1 (a slab never adds light).  0 <= m <= 64. */
    float darken;
    /* 0: directional light along `light_dir`.  1: point light at `position`
     * (world, outside the sphere circumscribing the unit cube; `light_dir`
     * is then ignored and may be NULL): the light's view looks at the cube
     * centre, slabs are planes of constant depth along that axis, the light
     * projection is perspective (section 3.2.1's L_p with a point light),
     * and each texel column is the ray from the light through the texel. */
    int positional;
    double position[3];
} vi_build_opts;

/* Camera: orthographic (view along target-eye, half image height
 * ortho_half_h in world units) or pinhole (full vertical field of view
 * fovy_deg).  World = the unit-cube frame of the volume. */
typedef struct {
    int kind; /* VI_CAM_ORTHO or VI_CAM_PERSP */
    double eye[3], target[3], up[3];
    double fovy_deg;
    double ortho_half_h;
    int width, height; /* 1 .. 16384 each */
} vi_camera;

/* Render options; vi_default_render_opts fills the defaults shown. */
typedef struct {
    float ambient;      /* 0: shade = ambient + (1-ambient) * A            */
    float light_rgb[3]; /* (1,1,1)                                          */
    float bg[4];        /* (0,0,0,0), premultiplied, composited last       */
    float term_eps;     /* 2^-15: stop once 1 - alpha_dst <= term_eps       */
    int shell_count;    /* 1: cuboid shells, 6 taps each                    */
    float shell_w[8];   /* 0s: equal weights; else weight of shell r: A = sum w_r mean_r / sum w_r */
    float shell_h_vox;  /* 1: shell r samples at +-(r+1)*h voxels along x,y,z */
    int cone_rings;     /* 2: rings m = 1..rings, m slabs toward the light (ds each along L) */
    int cone_angles;    /* 4: taps per ring, angles 2*pi*q/angles           */
    int cone_grid;      /* 0: ring form; G in 1..7: G x G lattice one slab toward the light */
    float cone_tan;     /* 1: ring radius m*ds*cone_tan; lattice pitch ds*cone_tan/2 */
    /* VI_MODE_PHONG: emission alpha*(sd*rgb + ss)*light_rgb with
     * sd = phong_ka + phong_kd*max(0, n.l), ss = phong_ks*max(0, r.v)^phong_shininess,
     * n = -g / max(|g|, grad_eps) from central differences g (value per
     * voxel) one voxel either side along x, y, z; l = -L, v = -ray
     * direction, r = 2(n.l)n - (n.n)l. */
    float phong_ka;        /* 0.1 */
    float phong_kd;        /* 0.9 */
    float phong_ks;        /* 0.4 */
    float phong_shininess; /* 20  */
    float grad_eps;        /* 0.02 */
    int samples_opaque;    /* 0: d_samples of vi_render is one counter; 1: two, [0] as
                              described there and [1] the segments composited with
                              non-zero opacity (those whose coefficient is gathered) */
    int nearest_layer;     /* 0: depth-continuous lookups (the index q of Eq. 9 lies
                              between faces floor(q) and ceil(q), linear between them);
                              1: each lookup reads the single layer of the face nearest
                              to q, floor(q + 1/2) (face 0 = 1, face f = layer f-1), as a
                              texture array indexed by Eq. 9 would, bilinear within it */
} vi_render_opts;

/* Library version string. */
const char* vi_version(void);

/* Message for the calling thread's last failed call ("" if none). */
const char* vi_last_error(void);

/* Fill `o` with the defaults listed above.  Returns VI_E_INVALID_ARG on NULL. */
int vi_default_render_opts(vi_render_opts* o);

/* Bytes of a stack buffer (element 4 bytes for VI_F32, 2 for VI_BF16 and
 * VI_F16): tiled n*R8*R4 elements, rows (n+2)*LS elements; 0 for invalid
 * arguments (VI_F16 with the tiled layout included). */
size_t vi_slices_bytes(int n_slices, int slice_res, int slice_dtype, int slice_layout);

/* Bytes of a volume of edge n, dtype and layout (0 for invalid arguments). */
size_t vi_volume_bytes(int n, int dtype, int layout);

/* Copy a linear volume into the 4x4x4 brick layout: `d_dst` (device,
 * vi_volume_bytes(n, dtype, VI_LAYOUT_BRICK4) bytes, caller-owned) receives
 * the bricks and `out` describes them (same dtype, edge and scale).  One
 * kernel launch on `stream`; values are copied bit for bit, so every result
 * computed from the bricked volume equals the one from the linear volume.
 * Errors: VI_E_INVALID_ARG for NULL pointers or a source that is not
 * linear; VI_E_UNSUPPORTED for sizes beyond the limits; VI_E_DEVICE. */
int vi_volume_to_bricks(const vi_volume* src, void* d_dst, vi_volume* out, vi_stream_t stream);

/* Copy a linear volume into the quad layout (VI_LAYOUT_QUAD4): `d_dst`
 * (device, vi_volume_bytes(n, dtype, VI_LAYOUT_QUAD4) bytes, aligned to
 * 4 elements, caller-owned) receives every voxel's 2x2 neighbourhood and
 * `out` describes it.  One kernel launch on `stream`; results computed from
 * it equal those from the linear volume bit for bit.  Errors as
 * vi_volume_to_bricks. */
int vi_volume_to_quads(const vi_volume* src, void* d_dst, vi_volume* out, vi_stream_t stream);

/* Bytes of the empty-space map of a volume of edge n with cells of `cell`
 * voxels: ceil(n/cell)^3 * 8 (0 for invalid arguments). */
size_t vi_volume_minmax_bytes(int n, int cell);

/* Compute the empty-space map of `vol` (any layout) into `d_minmax`
 * (device, vi_volume_minmax_bytes bytes, caller-owned) and return in `out`
 * a copy of `vol` that refers to it.  cell: 4, 8, 16 or 32.  One kernel
 * launch on `stream`.  The map depends on the volume only; the transfer
 * function is applied when rendering, so one map serves every TF.
 * Errors: VI_E_INVALID_ARG for NULL pointers or a bad cell size. */
int vi_volume_minmax(const vi_volume* vol, int cell, float* d_minmax, vi_volume* out, vi_stream_t stream);

/* Bytes of the occupancy bits of a volume of edge n with cells of `cell`
 * voxels: ceil(ceil(n/cell)^3 / 32) * 4 (0 for invalid arguments). */
size_t vi_volume_occupancy_bytes(int n, int cell);

/* For a volume with an empty-space map and one transfer function, write to
 * `d_bits` (device, vi_volume_occupancy_bytes bytes, 4-byte aligned,
 * caller-owned) one bit per cell -- bit c%32 of word c/32 is 1 where the
 * cell may hold opacity under `tf`, i.e. the negation of the map's
 * emptiness test -- and return in `out` a copy of `vol` that refers to them.
 * Both passes then answer the empty-space question with one bit, held in
 * LDS when the bits fit in 8 KiB (65536 cells), instead of a map entry and a
 * transfer-function table lookup: a shorter chain of dependent reads per
 * cell; results are unchanged bit for bit.  The passes accept the bits only
 * with the transfer function (and map) they were made for.  One kernel
 * launch on `stream`.
 * Errors: VI_E_INVALID_ARG for NULL pointers, a volume without a map or a
 * misaligned buffer; VI_E_DEVICE. */
int vi_volume_occupancy(const vi_volume* vol, const vi_tf* tf, uint32_t* d_bits, vi_volume* out,
                        vi_stream_t stream);

/* Host only: compute the light frame of Eq. 8 and the light projection
 * for `light_dir` (need not be unit length; finite, non-zero), or for the
 * point light of `opts` (may be NULL), and fill the geometry fields of
 * `out` (data = NULL, tag = 0).  1 <= n_slices <= 4096, 1 <= slice_res <= 8192. */
int vi_light_frame(const double light_dir[3], int n_slices, int slice_res, int slice_dtype, int slice_layout,
                   const vi_build_opts* opts, vi_slices* out);

/* Build the attenuation stack (section 3.2.1, Alg. 1) for light direction
 * `light_dir` into `d_slices` (device, vi_slices_bytes bytes, 16-byte
 * aligned -- 128-byte aligned for whole-line writes in the row layout --,
 * layout `slice_layout`) and describe it in `out_desc` (host).  One kernel
 * launch on `stream`, which writes every element of the row layout that a
 * lookup can read (the border and the leading layer included).  slice_dtype: VI_F32 (transmittance, product of per-slab
 * (1-alpha)), VI_BF16 (optical depth in base-2 units, -log2 T: the
 * per-slab extinction over ln 2 summed in float and rounded to bfloat16 per
 * layer; each slab adds at most 64 / ln 2, a factor e^-64) or VI_F16 (row
 * layout only: the same float optical depth stored as its transmittance
 * 2^-tau rounded to half precision, so that lookups need no exponential;
 * transmittances below 2^-24 round to 0).
 * `opts` may be NULL (directional light, plain product).
 * Errors: VI_E_INVALID_ARG for NULL pointers, bad sizes, a degenerate
 * light or options out of range; VI_E_UNSUPPORTED for dtypes or sizes
 * outside the limits above or a stack of 4 GiB or more; VI_E_DEVICE if the
 * launch fails. */
int vi_build_attenuation(const vi_volume* vol, const vi_tf* tf, const double light_dir[3], int n_slices,
                         int slice_res, int slice_dtype, int slice_layout, const vi_build_opts* opts,
                         void* d_slices, vi_slices* out_desc, vi_stream_t stream);

/* Ray-cast `cam` through the volume with the illumination coefficient
 * `mode` gathered from `slices` (section 3.2.2 and 3.2.3) and write
 * width*height premultiplied RGBA floats to `d_rgba` (device, 16-byte
 * aligned, row-major, y = 0 on top).  step_vox > 0 is the ray step in
 * voxels.  `opts` may be NULL (defaults).  `slices` may be NULL only for
 * VI_MODE_NONE; VI_MODE_PHONG reads only its light, so a descriptor from
 * vi_light_frame (data NULL) serves.  With a point light's descriptor
 * every stack lookup projects through its depth from the light, and a
 * lookup at or behind the light's depth plane reads transmittance 1;
 * Phong's light vector points at the light from each sample, and the
 * cone's axis is the light's direction at each sample, L_s = (p - P)/|p - P|:
 * ring m is centred on that line m slabs of depth toward the light, in the
 * plane across L_s, radius (that distance) * cone_tan; the lattice lies one
 * slab toward the light in the same way.
 * If `d_samples` (device) is non-NULL the number of segments composited
 * (stopping at termination; segments that empty-space skipping steps over
 * count too) is ADDED to d_samples[0]; with opts->samples_opaque = 1 the
 * number of those segments whose opacity is non-zero is added to
 * d_samples[1] as well.
 * Errors: VI_E_INVALID_ARG for NULL/misaligned pointers, bad sizes, a
 * descriptor whose vol_n differs from the volume or whose non-zero tag
 * names another (volume, transfer function); VI_E_UNSUPPORTED for dtypes
 * outside the list; VI_E_DEVICE if the launch fails. */
int vi_render(const vi_volume* vol, const vi_tf* tf, const vi_slices* slices, const vi_camera* cam, int mode,
              float step_vox, const vi_render_opts* opts, float* d_rgba, unsigned long long* d_samples,
              vi_stream_t stream);

/* Identity tag vi_build_attenuation stores in vi_slices.tag for (vol, tf):
 * a hash of the volume's pointer, edge, dtype and scale and of the table's
 * content tag (its pointer when the tag is 0) and size. */
uint64_t vi_tag(const vi_volume* vol, const vi_tf* tf);

/* Content tag of a transfer function: FNV-1a over the bytes of the
 * n_entries x 4 floats at `host_rgba` (HOST memory) and n_entries; never 0.
 * Returns 0 for a NULL table or n_entries < 1. */
uint64_t vi_tf_tag(const float* host_rgba, int n_entries);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * The stack depends only on (volume, transfer function, light, n, res,
 * dtype), not on the camera (the paper builds it once and reuses it while
 * only the view changes, section 4), so the server keeps stacks resident
 * in a device pool and reuses them across requests.  A scheduler thread
 *   - admits requests first come first served while fewer than max_inflight
 *     frames are unfinished and their stack is cached or fits in the pool
 *     (least recently used unpinned stacks are evicted to make room; a stack
 *     larger than the whole pool is rejected with VI_E_NO_MEMORY);
 *   - builds missing stacks on its own build stream;
 *   - renders 16x16-pixel tiles of all admitted frames, oldest first, in
 *     launches of at most tiles_per_launch tiles that mix frames of
 *     different volumes, sizes, cameras and modes; a launch waits on the
 *     device (not the host) for the builds it needs, so builds overlap
 *     renders; up to two launches are in flight;
 *   - completes a frame when the launch holding its last tile finishes, and
 *     admits waiting requests as slots and pool memory free up.
 * Every pixel is computed by the same per-ray code as vi_render, so a
 * frame is bit-identical whether rendered alone or in any mix.
 * Memory: the library allocates the stack pool (stack_budget bytes, once,
 * at creation) and small staging buffers; volumes, transfer functions,
 * images and sample counters stay caller-owned device buffers that must
 * outlive the requests using them.
 * ---------------------------------------------------------------------- */
typedef struct vi_server vi_server;

typedef struct {
    size_t stack_budget;       /* bytes of the device stack pool (> 0)                 */
    int max_inflight;          /* admitted, unfinished frames: 1..256 (default 16)     */
    int tiles_per_launch;      /* 16x16-pixel tiles per render launch (default 8192)   */
    int device;                /* HIP device ordinal                                   */
} vi_server_cfg;

typedef struct {
    int vol_id;                /* from vi_server_register_volume                        */
    double light_dir[3];
    int n_slices, slice_res, slice_dtype, slice_layout;
    vi_build_opts build;       /* stack build options (part of the stack's identity)   */
    vi_camera camera;
    int mode;
    float step_vox;
    vi_render_opts opts;       /* all fields used; start from vi_default_render_opts    */
    float* d_rgba;             /* caller-owned device image, width*height*4 floats     */
    unsigned long long* d_samples; /* optional device counter (added to), or NULL      */
} vi_request;

/* Request states reported by vi_server_poll / vi_server_wait. */
#define VI_REQ_PENDING 0
#define VI_REQ_ADMITTED 1
#define VI_REQ_DONE 2

typedef struct {
    uint64_t submitted, completed, rejected, cancelled;
    uint64_t stack_hits, stack_builds, evictions;
    uint64_t launches, tiles;
    double mean_frames_per_launch;     /* distinct frames per render launch               */
    double p50_ms, p99_ms, mean_ms, max_ms; /* completion - submission, completed frames */
    double frames_per_s;               /* completed / (last completion - first submission) */
    size_t pool_bytes, pool_in_use, pool_peak;
} vi_stats;

/* Create a server on cfg->device: allocates the stack pool and staging
 * buffers, creates a render and a build stream (default priority) and
 * starts the scheduler thread.  VI_E_NO_MEMORY if the pool cannot be
 * allocated, VI_E_INVALID_ARG for bad sizes. */
int vi_server_create(const vi_server_cfg* cfg, vi_server** out);

/* Make a resident volume and transfer function known to the server (both
 * stay caller-owned).  Returns its id in *vol_id. */
int vi_server_register_volume(vi_server* srv, const vi_volume* vol, const vi_tf* tf, int* vol_id);

/* Queue a frame; returns at once with its ticket.  Arguments are validated
 * here (VI_E_INVALID_ARG / VI_E_UNSUPPORTED); VI_E_NO_MEMORY if its stack
 * can never fit the pool. */
int vi_server_submit(vi_server* srv, const vi_request* req, uint64_t* ticket);

/* State of a ticket: VI_REQ_PENDING, VI_REQ_ADMITTED, VI_REQ_DONE, or a
 * negative error code (e.g. VI_E_CANCELLED, VI_E_DEVICE). */
int vi_server_poll(vi_server* srv, uint64_t ticket, int* state);

/* Block until the ticket is done or failed, or timeout_ms passes (< 0:
 * no limit).  Returns VI_OK when done, VI_E_BUSY on timeout, or the
 * request's error code. */
int vi_server_wait(vi_server* srv, uint64_t ticket, int timeout_ms);

/* Cancel a request that has not been admitted yet (VI_E_BUSY if it has). */
int vi_server_cancel(vi_server* srv, uint64_t ticket);

/* Counters and latency percentiles since creation or the last reset. */
int vi_server_stats(vi_server* srv, vi_stats* out);
int vi_server_reset_stats(vi_server* srv);

/* Finish all admitted and queued work, stop the thread, free the pool. */
void vi_server_destroy(vi_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* VI_H */
