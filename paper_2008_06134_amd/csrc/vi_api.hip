// vi_api.hip -- host side of the libvi C ABI: validation, the light frame in
// double (Eq. 8, light projection of Eq. 10), kernel parameter set-up and
// launches.  No allocation, no synchronisation.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "vi_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_err() { g_err[0] = 0; }

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
void cross3(const double* a, const double* b, double* r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

size_t elem_size(int dt)
{
    switch (dt) {
    case VI_U8: return 1;
    case VI_U16: case VI_F16: case VI_BF16: return 2;
    case VI_F32: return 4;
    default: return 0;
    }
}

bool known_layout(int layout)
{
    return layout == VI_LAYOUT_LINEAR || layout == VI_LAYOUT_BRICK4 || layout == VI_LAYOUT_QUAD4;
}

// bytes of one copy of the voxels (the quad layout stores four copies):
// kernels index voxels (quad slots) with 32-bit offsets, so this stays
// below 4 GiB
double voxel_storage(int n, int dtype, int layout)
{
    const double e = (double)(layout == VI_LAYOUT_LINEAR ? (uint32_t)n : vi::round_up((uint32_t)n, 4u));
    return e * e * e * (double)elem_size(dtype);
}
double volume_storage(int n, int dtype, int layout)
{
    return voxel_storage(n, dtype, layout) * (layout == VI_LAYOUT_QUAD4 ? 4.0 : 1.0);
}

int check_volume(const vi_volume* v)
{
    if (!v || !v->data) return fail(VI_E_INVALID_ARG, "volume or its data pointer is NULL");
    if (v->dtype != VI_U8 && v->dtype != VI_U16 && v->dtype != VI_F16 && v->dtype != VI_F32)
        return fail(VI_E_UNSUPPORTED, "volume dtype %d not supported", v->dtype);
    if (!known_layout(v->layout)) return fail(VI_E_UNSUPPORTED, "volume layout %d not supported", v->layout);
    if (v->n < 2) return fail(VI_E_INVALID_ARG, "volume edge %d < 2", v->n);
    const double bytes = voxel_storage(v->n, v->dtype, v->layout);
    if (bytes >= 4294967296.0) return fail(VI_E_UNSUPPORTED, "volume of %.0f bytes exceeds 4 GiB", bytes);
    const size_t align = elem_size(v->dtype) * (v->layout == VI_LAYOUT_QUAD4 ? 4 : 1);
    if (((uintptr_t)v->data) % align) return fail(VI_E_INVALID_ARG, "volume pointer misaligned");
    if (!(v->scale > 0.0f) || !isfinite(v->scale)) return fail(VI_E_INVALID_ARG, "volume scale must be > 0");
    if (v->minmax) {
        if (v->cell != 4 && v->cell != 8 && v->cell != 16 && v->cell != 32)
            return fail(VI_E_INVALID_ARG, "empty-space cell %d must be 4, 8, 16 or 32", v->cell);
        if (((uintptr_t)v->minmax) % 8) return fail(VI_E_INVALID_ARG, "empty-space map misaligned");
    }
    if (v->occ) {
        if (!v->minmax) return fail(VI_E_INVALID_ARG, "occupancy bits without an empty-space map");
        if (((uintptr_t)v->occ) % 4) return fail(VI_E_INVALID_ARG, "occupancy bits misaligned");
    }
    return VI_OK;
}

int cell_shift(int cell) { return cell == 4 ? 2 : cell == 8 ? 3 : cell == 16 ? 4 : 5; }

uint32_t cells_of(int n, int cell)
{
    const uint32_t nc = ((uint32_t)n + (uint32_t)cell - 1) / (uint32_t)cell;
    return nc * nc * nc;
}

vi::OccMap occ_of(const vi_volume* v)
{
    vi::OccMap o;
    o.mm = v->minmax ? (const float2*)v->minmax : nullptr;
    o.shift = v->minmax ? cell_shift(v->cell) : 0;
    o.nc = v->minmax ? ((uint32_t)v->n + (uint32_t)v->cell - 1) / (uint32_t)v->cell : 0;
    const uint32_t words = v->minmax ? (cells_of(v->n, v->cell) + 31u) / 32u : 0;
    const uint32_t snc = (o.nc + 3u) / 4u, swords = v->minmax ? (snc * snc * snc + 31u) / 32u : 0;
    // bits that do not fit in LDS are not used: the map decides instead
    o.bits = v->minmax && v->occ && words + swords <= vi::kMaxLdsOccWords ? v->occ : nullptr;
    o.words = o.bits ? words : 0;
    o.snc = o.bits ? snc : 0;
    o.swords = o.bits ? swords : 0;
    return o;
}

// Identity of the (volume, map, transfer function) occupancy bits belong to.
uint64_t occ_tag_of(const vi_volume* v, const vi_tf* tf)
{
    uint64_t h = vi_tag(v, tf);
    const uint64_t parts[2] = {(uint64_t)(uintptr_t)v->minmax, (uint64_t)v->cell};
    for (uint64_t x : parts)
        for (int b = 0; b < 8; ++b) {
            h ^= (x >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    return h ? h : 1;
}

int check_occ(const vi_volume* v, const vi_tf* tf)
{
    if (v->occ && v->occ_tag != occ_tag_of(v, tf))
        return fail(VI_E_INVALID_ARG, "occupancy bits were made for another transfer function or map");
    return VI_OK;
}

int check_tf(const vi_tf* tf)
{
    if (!tf || !tf->rgba) return fail(VI_E_INVALID_ARG, "transfer function or its pointer is NULL");
    if (tf->n_entries < 2 || tf->n_entries > vi::kMaxTF)
        return fail(VI_E_INVALID_ARG, "transfer function needs 2..%d entries, got %d", vi::kMaxTF, tf->n_entries);
    if (((uintptr_t)tf->rgba) % 4) return fail(VI_E_INVALID_ARG, "transfer function pointer misaligned");
    return VI_OK;
}

// per-axis offset strides of a volume layout (y, z)
void volume_strides(const vi_volume* v, uint32_t* sy, uint32_t* sz)
{
    if (v->layout != VI_LAYOUT_LINEAR) {  // bricks, or quads in brick order
        const uint32_t nb = vi::round_up((uint32_t)v->n, 4u) / 4u;
        *sy = nb * 64u;
        *sz = nb * nb * 64u;
    } else {
        *sy = (uint32_t)v->n;
        *sz = (uint32_t)v->n * (uint32_t)v->n;
    }
}

// Kernels index stacks with 32-bit element offsets: stacks stay below 4 GiB.
bool stack_size_ok(int n, int res, int dt, int sl) { return (double)vi_slices_bytes(n, res, dt, sl) < 4294967296.0; }

// Row layout: every layer has rows -2 .. res+1 and columns -2 .. res+1 of
// texels, the two outermost rings a fully transmitting border; one extra
// leading layer (-1, face 0 of Eq. 9's index) transmits fully too, and one
// trailing layer n repeats layer n - 1 (the light leaving the last slab), so
// that a lookup's second layer k0 + 1 needs no clamp.  The
// pitch P is res + 4 rounded up to 4.  A layer holds the least number of
// elements from (res + 4) P up that is an odd multiple of half a 128-byte
// line (16 floats, 32 two-byte texels): the same texel of two neighbouring
// layers then lies half a line apart, which keeps the render's reads of
// neighbouring layers from colliding in the L1 tags (whole-line layer
// strides measured 6-8 % slower frames), and every other layer starts on a
// line, which the build's line-aligned stores rely on.
uint32_t row_pitch(int res, int) { return vi::round_up((uint32_t)res + 4u, 4u); }
uint32_t row_layer(int res, int dt)
{
    const uint32_t half = dt == VI_F32 ? 16u : 32u, w = ((uint32_t)res + 4u) * row_pitch(res, dt);
    const uint32_t m = (w + half - 1) / half;  // least multiple of half from w up, made odd
    return (m | 1u) * half;
}
// element of texel (k, j, i) = (0, 0, 0): past the front layer, two rows and two columns of border
uint32_t row_origin(int res, int dt) { return row_layer(res, dt) + 2u * row_pitch(res, dt) + 2u; }

// A position or step in voxels as a Q40 fixed-point number (the build's
// slab positions): |x| < 2^23 voxels, rounded to the nearest 2^-40 voxel.
int64_t to_q40(double x) { return (int64_t)llround(ldexp(x, vi::kQBits)); }

// A double as a float pair: hi = x rounded to float, lo = the remainder
// rounded to float (together about 48 significant bits).
void split_float(double x, float* hi, float* lo)
{
    *hi = (float)x;
    *lo = (float)(x - (double)*hi);
}

// Light-plane basis (U from the axis least aligned with L, Gram-Schmidt;
// V = L x U).
void plane_basis(const double L[3], double U[3], double V[3])
{
    int js = 0;
    for (int a = 1; a < 3; ++a)
        if (fabs(L[a]) < fabs(L[js])) js = a;
    double u[3] = {-L[js] * L[0], -L[js] * L[1], -L[js] * L[2]};
    u[js] += 1.0;
    const double nu = sqrt(dot3(u, u));
    for (int a = 0; a < 3; ++a) U[a] = u[a] / nu;
    cross3(L, U, V);
}

// A point light's frame: axis from the light to the cube centre, slab
// planes of constant depth along it between the nearest and farthest cube
// vertices, and the smallest square on the unit-depth plane that holds
// every vertex's perspective projection.
int fill_point_frame(const double P[3], int n, int res, int dt, int sl, vi_slices* f)
{
    if (!isfinite(P[0]) || !isfinite(P[1]) || !isfinite(P[2]))
        return fail(VI_E_INVALID_ARG, "light position is not finite");
    const double w[3] = {0.5 - P[0], 0.5 - P[1], 0.5 - P[2]};
    const double nw = sqrt(dot3(w, w));
    if (!(nw > 0.5 * sqrt(3.0) * 1.0001))
        return fail(VI_E_INVALID_ARG, "a point light must lie outside the cube's circumscribed sphere");
    memset(f, 0, sizeof *f);
    f->dtype = dt;
    f->layout = sl;
    f->positional = 1;
    for (int a = 0; a < 3; ++a) {
        f->L[a] = w[a] / nw;
        f->P[a] = P[a];
        f->c[a] = 0.5;
    }
    plane_basis(f->L, f->U, f->V);
    f->dmin = 1e300;
    f->dmax = -1e300;
    f->R = 0.0;
    for (int vtx = 0; vtx < 8; ++vtx) {
        const double r[3] = {(double)(vtx & 1) - P[0], (double)((vtx >> 1) & 1) - P[1], (double)((vtx >> 2) & 1) - P[2]};
        const double d = dot3(f->L, r);
        f->dmin = fmin(f->dmin, d);
        f->dmax = fmax(f->dmax, d);
        f->R = fmax(f->R, fmax(fabs(dot3(f->U, r)), fabs(dot3(f->V, r))) / d);
    }
    f->ds = (f->dmax - f->dmin) / n;
    f->n = n;
    f->res = res;
    return VI_OK;
}

// Eq. 8 and the light projection: geometry of the stack in double.
int fill_frame(const double l[3], int n, int res, int dt, int sl, const vi_build_opts* o, vi_slices* f)
{
    const bool point = o && o->positional;
    if (o && o->positional != 0 && o->positional != 1) return fail(VI_E_INVALID_ARG, "positional must be 0 or 1");
    if ((!l && !point) || !f) return fail(VI_E_INVALID_ARG, "NULL light direction or descriptor");
    if (n < 1 || n > 4096) return fail(VI_E_INVALID_ARG, "n_slices %d outside 1..4096", n);
    if (res < 1 || res > 8192) return fail(VI_E_INVALID_ARG, "slice_res %d outside 1..8192", res);
    if (dt != VI_F32 && dt != VI_BF16 && dt != VI_F16) return fail(VI_E_UNSUPPORTED, "slice dtype %d not supported", dt);
    if (sl != VI_STACK_TILED && sl != VI_STACK_ROWS) return fail(VI_E_UNSUPPORTED, "slice layout %d not supported", sl);
    if (dt == VI_F16 && sl != VI_STACK_ROWS) return fail(VI_E_UNSUPPORTED, "a half-precision stack needs the row layout");
    if (point) return fill_point_frame(o->position, n, res, dt, sl, f);
    if (!isfinite(l[0]) || !isfinite(l[1]) || !isfinite(l[2]))
        return fail(VI_E_INVALID_ARG, "light direction is not finite");
    const double nl = sqrt(dot3(l, l));
    if (!(nl > 0.0) || !isfinite(nl)) return fail(VI_E_INVALID_ARG, "light direction is zero");
    memset(f, 0, sizeof *f);
    f->dtype = dt;
    f->layout = sl;
    for (int a = 0; a < 3; ++a) f->L[a] = l[a] / nl;
    f->c[0] = f->c[1] = f->c[2] = 0.5;
    // extreme distances along L over the cube's vertices: the vertex picks
    // 0 or 1 per axis by the sign of L
    f->dmin = f->dmax = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (f->L[a] < 0.0) f->dmin += f->L[a];
        else f->dmax += f->L[a];
    }
    f->ds = (f->dmax - f->dmin) / n;
    plane_basis(f->L, f->U, f->V);
    f->R = sqrt(3.0) / 2.0;
    f->n = n;
    f->res = res;
    f->dtype = dt;
    return VI_OK;
}

}  // namespace

extern "C" {

const char* vi_version(void) { return "libvi 0.1 gfx950"; }

const char* vi_last_error(void) { return g_err; }

int vi_default_render_opts(vi_render_opts* o)
{
    if (!o) return fail(VI_E_INVALID_ARG, "NULL options");
    o->ambient = 0.0f;
    o->light_rgb[0] = o->light_rgb[1] = o->light_rgb[2] = 1.0f;
    o->bg[0] = o->bg[1] = o->bg[2] = o->bg[3] = 0.0f;
    o->term_eps = ldexpf(1.0f, -15);
    o->shell_count = 1;
    o->shell_h_vox = 1.0f;
    o->cone_rings = 2;
    o->cone_angles = 4;
    o->cone_grid = 0;
    o->cone_tan = 1.0f;
    for (int r = 0; r < 8; ++r) o->shell_w[r] = 0.0f;
    o->phong_ka = 0.1f;
    o->phong_kd = 0.9f;
    o->phong_ks = 0.4f;
    o->phong_shininess = 20.0f;
    o->grad_eps = 0.02f;
    o->samples_opaque = 0;
    o->nearest_layer = 0;
    return VI_OK;
}

size_t vi_slices_bytes(int n, int res, int dt, int sl)
{
    if (n < 1 || res < 1 || (dt != VI_F32 && dt != VI_BF16 && dt != VI_F16)) return 0;
    if (sl == VI_STACK_TILED && dt == VI_F16) return 0;
    if (sl == VI_STACK_TILED)
        return (size_t)n * vi::round_up((uint32_t)res, 8u) * vi::round_up((uint32_t)res, 4u) * elem_size(dt);
    if (sl == VI_STACK_ROWS) return ((size_t)n + 2u) * row_layer(res, dt) * elem_size(dt);
    return 0;
}

size_t vi_volume_bytes(int n, int dtype, int layout)
{
    if (n < 2 || elem_size(dtype) == 0 || dtype == VI_BF16) return 0;
    if (!known_layout(layout)) return 0;
    return (size_t)volume_storage(n, dtype, layout);
}

static int relayout(const vi_volume* src, void* d_dst, vi_volume* out, vi_stream_t stream, int layout)
{
    clear_err();
    int rc;
    if ((rc = check_volume(src)) != VI_OK) return rc;
    if (src->layout != VI_LAYOUT_LINEAR) return fail(VI_E_INVALID_ARG, "source volume is not linear");
    if (!d_dst || !out) return fail(VI_E_INVALID_ARG, "NULL destination or descriptor");
    const size_t align = elem_size(src->dtype) * (layout == VI_LAYOUT_QUAD4 ? 4 : 1);
    if (((uintptr_t)d_dst) % align) return fail(VI_E_INVALID_ARG, "destination misaligned");
    if (voxel_storage(src->n, src->dtype, layout) >= 4294967296.0)
        return fail(VI_E_UNSUPPORTED, "bricked volume exceeds 4 GiB per copy of the voxels");
    hipError_t e = layout == VI_LAYOUT_QUAD4
                       ? vi::launch_to_quads(src->data, d_dst, src->dtype, src->n, (hipStream_t)stream)
                       : vi::launch_to_bricks(src->data, d_dst, src->dtype, src->n, (hipStream_t)stream);
    if (e != hipSuccess) return fail(VI_E_DEVICE, "layout launch failed: %s", hipGetErrorString(e));
    *out = *src;
    out->data = d_dst;
    out->layout = layout;
    out->occ = nullptr;  // bits are tied to the source's identity (the map stays valid)
    out->occ_tag = 0;
    return VI_OK;
}

int vi_volume_to_bricks(const vi_volume* src, void* d_dst, vi_volume* out, vi_stream_t stream)
{
    return relayout(src, d_dst, out, stream, VI_LAYOUT_BRICK4);
}

int vi_volume_to_quads(const vi_volume* src, void* d_dst, vi_volume* out, vi_stream_t stream)
{
    return relayout(src, d_dst, out, stream, VI_LAYOUT_QUAD4);
}

size_t vi_volume_minmax_bytes(int n, int cell)
{
    if (n < 2 || (cell != 4 && cell != 8 && cell != 16 && cell != 32)) return 0;
    const size_t nc = ((size_t)n + cell - 1) / cell;
    return nc * nc * nc * 8;
}

size_t vi_volume_occupancy_bytes(int n, int cell)
{
    if (n < 2 || (cell != 4 && cell != 8 && cell != 16 && cell != 32)) return 0;
    const size_t nc = ((size_t)n + cell - 1) / cell, snc = (nc + 3) / 4;
    return ((size_t)cells_of(n, cell) + 31) / 32 * 4 + (snc * snc * snc + 31) / 32 * 4;
}

int vi_volume_occupancy(const vi_volume* vol, const vi_tf* tf, uint32_t* d_bits, vi_volume* out,
                        vi_stream_t stream)
{
    clear_err();
    int rc;
    if ((rc = check_volume(vol)) != VI_OK) return rc;
    if ((rc = check_tf(tf)) != VI_OK) return rc;
    if (!vol->minmax) return fail(VI_E_INVALID_ARG, "the volume has no empty-space map");
    if (!d_bits || !out) return fail(VI_E_INVALID_ARG, "NULL bits or descriptor");
    if (((uintptr_t)d_bits) % 4) return fail(VI_E_INVALID_ARG, "bits pointer must be 4-byte aligned");
    const uint32_t nc = ((uint32_t)vol->n + (uint32_t)vol->cell - 1u) / (uint32_t)vol->cell;
    hipError_t e = vi::launch_occupancy(vol->minmax, nc, tf->rgba, tf->n_entries, d_bits, (hipStream_t)stream);
    if (e != hipSuccess) return fail(VI_E_DEVICE, "occupancy launch failed: %s", hipGetErrorString(e));
    *out = *vol;
    out->occ = d_bits;
    out->occ_tag = occ_tag_of(vol, tf);
    return VI_OK;
}

int vi_volume_minmax(const vi_volume* vol, int cell, float* d_minmax, vi_volume* out, vi_stream_t stream)
{
    clear_err();
    int rc;
    if ((rc = check_volume(vol)) != VI_OK) return rc;
    if (cell != 4 && cell != 8 && cell != 16 && cell != 32)
        return fail(VI_E_INVALID_ARG, "cell %d must be 4, 8, 16 or 32", cell);
    if (!d_minmax || !out) return fail(VI_E_INVALID_ARG, "NULL map or descriptor");
    if (((uintptr_t)d_minmax) % 8) return fail(VI_E_INVALID_ARG, "map pointer must be 8-byte aligned");
    uint32_t sy, sz;
    volume_strides(vol, &sy, &sz);
    hipError_t e = vi::launch_minmax(vol->data, vol->dtype, vol->layout, sy, sz, vol->n, vol->scale,
                                     cell_shift(cell), d_minmax, (hipStream_t)stream);
    if (e != hipSuccess) return fail(VI_E_DEVICE, "min/max launch failed: %s", hipGetErrorString(e));
    *out = *vol;
    out->minmax = d_minmax;
    out->cell = cell;
    out->occ = nullptr;  // bits belong to the previous map
    out->occ_tag = 0;
    return VI_OK;
}

uint64_t vi_tag(const vi_volume* vol, const vi_tf* tf)
{
    // FNV-1a over the identity of the inputs (pointers, sizes, dtype, scale)
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t x) {
        for (int b = 0; b < 8; ++b) {
            h ^= (x >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    if (vol) {
        mix((uint64_t)(uintptr_t)vol->data);
        mix((uint64_t)vol->n);
        mix((uint64_t)vol->dtype);
        uint32_t sb;
        memcpy(&sb, &vol->scale, 4);
        mix(sb);
    }
    if (tf) {
        mix(tf->tag ? tf->tag : (uint64_t)(uintptr_t)tf->rgba);
        mix((uint64_t)tf->n_entries);
    }
    return h ? h : 1;
}

uint64_t vi_tf_tag(const float* host_rgba, int n_entries)
{
    if (!host_rgba || n_entries < 1) return 0;
    uint64_t h = 1469598103934665603ull;
    const unsigned char* b = (const unsigned char*)host_rgba;
    for (size_t i = 0; i < (size_t)n_entries * 4u * sizeof(float); ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    for (int k = 0; k < 4; ++k) {
        h ^= ((uint32_t)n_entries >> (8 * k)) & 0xffu;
        h *= 1099511628211ull;
    }
    return h ? h : 1;
}

int vi_light_frame(const double light_dir[3], int n, int res, int dt, int sl, const vi_build_opts* opts,
                   vi_slices* out)
{
    clear_err();
    return fill_frame(light_dir, n, res, dt, sl, opts, out);
}

int vi_build_attenuation(const vi_volume* vol, const vi_tf* tf, const double light_dir[3], int n, int res,
                         int dt, int sl, const vi_build_opts* opts, void* d_slices, vi_slices* out_desc,
                         vi_stream_t stream)
{
    clear_err();
    int rc;
    if ((rc = check_volume(vol)) != VI_OK) return rc;
    if ((rc = check_tf(tf)) != VI_OK) return rc;
    if ((rc = check_occ(vol, tf)) != VI_OK) return rc;
    if (!d_slices) return fail(VI_E_INVALID_ARG, "NULL stack buffer");
    if (!out_desc) return fail(VI_E_INVALID_ARG, "NULL stack descriptor");
    vi_slices f;
    if ((rc = fill_frame(light_dir, n, res, dt, sl, opts, &f)) != VI_OK) return rc;
    if (((uintptr_t)d_slices) % 16) return fail(VI_E_INVALID_ARG, "stack buffer must be 16-byte aligned");
    if (!stack_size_ok(n, res, dt, sl))
        return fail(VI_E_UNSUPPORTED, "stack of %zu bytes exceeds the layout's limit", vi_slices_bytes(n, res, dt, sl));
    const float darken = opts ? opts->darken : 0.0f;
    if (!(darken >= 0.0f && darken <= 64.0f)) return fail(VI_E_INVALID_ARG, "darken must be in [0, 64]");

    vi::BuildParams p;
    memset(&p, 0, sizeof p);
    p.vol = vol->data;
    p.vol_dtype = vol->dtype;
    p.vol_layout = vol->layout;
    volume_strides(vol, &p.vsy, &p.vsz);
    p.occ = occ_of(vol);
    p.N = vol->n;
    p.M = vol->n / 2;
    p.scale = vol->scale;
    p.tf = tf->rgba;
    p.K = tf->n_entries;
    p.out = d_slices;
    p.out_dtype = dt;
    p.n = n;
    p.res = res;
    p.out_layout = sl;
    p.layer = vi::round_up((uint32_t)res, 8u) * vi::round_up((uint32_t)res, 4u);
    p.row_tiles32 = vi::round_up((uint32_t)res, 8u) * 4u;
    p.rpitch = row_pitch(res, dt);
    p.rorg = row_origin(res, dt);
    p.rlayer = row_layer(res, dt);
    const double N = vol->n, texel = 2.0 * f.R / res, u0 = -f.R + 0.5 * texel;
    const double d0 = f.dmin + 0.5 * f.ds, Lc = dot3(f.L, f.c);
    if (f.positional) {
        // column (i,j) is the ray P + d D(i,j), D = L + u U + v V on the
        // unit-depth plane; slab k's mid-plane at depth d0 + k ds
        p.point = 1;
        for (int a = 0; a < 3; ++a) {
            const double D00 = f.L[a] + u0 * f.U[a] + u0 * f.V[a];
            p.B0q[a] = to_q40((f.P[a] + d0 * D00) * N - 0.5 - p.M);
            p.BUq[a] = to_q40(d0 * texel * f.U[a] * N);
            p.BVq[a] = to_q40(d0 * texel * f.V[a] * N);
            p.ALq[a] = to_q40(f.ds * D00 * N);
            p.ALUq[a] = to_q40(f.ds * texel * f.U[a] * N);
            p.ALVq[a] = to_q40(f.ds * texel * f.V[a] * N);
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            const double p0 = f.c[a] + u0 * f.U[a] + u0 * f.V[a] + (d0 - Lc) * f.L[a];
            p.B0q[a] = to_q40(p0 * N - 0.5 - p.M);
            p.BUq[a] = to_q40(f.U[a] * texel * N);
            p.BVq[a] = to_q40(f.V[a] * texel * N);
            p.ALq[a] = to_q40(f.L[a] * f.ds * N);
        }
    }
    p.e = (float)(f.ds * N);
    p.darken = darken;
    p.loq = to_q40(-0.5 - p.M);
    p.hiq = to_q40(N - 0.5 - p.M);
    hipError_t e = vi::launch_build(p, (hipStream_t)stream);
    if (e != hipSuccess) return fail(VI_E_DEVICE, "build launch failed: %s", hipGetErrorString(e));
    f.data = d_slices;
    f.vol_n = vol->n;
    f.tag = vi_tag(vol, tf);
    f.darken = darken;
    *out_desc = f;
    return VI_OK;
}

int vi_render(const vi_volume* vol, const vi_tf* tf, const vi_slices* sl, const vi_camera* cam, int mode,
              float step_vox, const vi_render_opts* opts, float* d_rgba, unsigned long long* d_samples,
              vi_stream_t stream)
{
    clear_err();
    vi::RenderFrame F;
    int rc = vi::make_frame(vol, tf, sl, cam, mode, step_vox, opts, d_rgba, d_samples, &F);
    if (rc != VI_OK) return rc;
    hipError_t e = vi::launch_render(F, (hipStream_t)stream);
    if (e != hipSuccess) return fail(VI_E_DEVICE, "render launch failed: %s", hipGetErrorString(e));
    return VI_OK;
}

}  // extern "C"

namespace vi {

// Validate a render request and fill its kernel parameters (shared by
// vi_render and the server, so a frame is computed identically by both).
int make_frame(const vi_volume* vol, const vi_tf* tf, const vi_slices* sl, const vi_camera* cam, int mode,
               float step_vox, const vi_render_opts* opts, float* d_rgba, unsigned long long* d_samples,
               RenderFrame* out)
{
    int rc;
    if ((rc = check_volume(vol)) != VI_OK) return rc;
    if ((rc = check_tf(tf)) != VI_OK) return rc;
    if ((rc = check_occ(vol, tf)) != VI_OK) return rc;
    if (mode < VI_MODE_NONE || mode > VI_MODE_PHONG) return fail(VI_E_UNSUPPORTED, "mode %d not supported", mode);
    if (!cam) return fail(VI_E_INVALID_ARG, "NULL camera");
    if (!d_rgba) return fail(VI_E_INVALID_ARG, "NULL output image");
    if (((uintptr_t)d_rgba) % 16) return fail(VI_E_INVALID_ARG, "output image must be 16-byte aligned");
    if (d_samples && ((uintptr_t)d_samples) % 8) return fail(VI_E_INVALID_ARG, "sample counter misaligned");
    if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
        return fail(VI_E_INVALID_ARG, "image size %dx%d outside 1..16384", cam->width, cam->height);
    if (cam->kind != VI_CAM_ORTHO && cam->kind != VI_CAM_PERSP)
        return fail(VI_E_INVALID_ARG, "camera kind %d", cam->kind);
    if (!(step_vox > 0.0f) || !isfinite(step_vox)) return fail(VI_E_INVALID_ARG, "step_vox must be > 0");
    vi_render_opts o;
    if (opts) o = *opts;
    else vi_default_render_opts(&o);
    if (!(o.term_eps >= 0.0f && o.term_eps < 1.0f) || !(o.ambient >= 0.0f && o.ambient <= 1.0f))
        return fail(VI_E_INVALID_ARG, "term_eps must be in [0,1) and ambient in [0,1]");
    const bool reads_stack = mode != VI_MODE_NONE && mode != VI_MODE_PHONG;
    if (mode == VI_MODE_PHONG) {
        if (!sl) return fail(VI_E_INVALID_ARG, "Phong mode needs a light frame");
        const double l2 = dot3(sl->L, sl->L);
        if (!(fabs(l2 - 1.0) < 1e-6)) return fail(VI_E_INVALID_ARG, "light frame has no unit direction");
        if (!(o.phong_ka >= 0.0f && o.phong_kd >= 0.0f && o.phong_ks >= 0.0f) || !isfinite(o.phong_ka) ||
            !isfinite(o.phong_kd) || !isfinite(o.phong_ks))
            return fail(VI_E_INVALID_ARG, "Phong coefficients must be finite and >= 0");
        if (!(o.phong_shininess >= 0.0f && o.phong_shininess <= 1024.0f))
            return fail(VI_E_INVALID_ARG, "phong_shininess must be in [0, 1024]");
        if (!(o.grad_eps > 0.0f) || !isfinite(o.grad_eps)) return fail(VI_E_INVALID_ARG, "grad_eps must be > 0");
    }
    const bool point = sl && sl->positional;
    if (point) {
        if (!isfinite(sl->P[0]) || !isfinite(sl->P[1]) || !isfinite(sl->P[2]))
            return fail(VI_E_INVALID_ARG, "point light position is not finite");
        if (reads_stack && !(sl->dmin > 0.0 && sl->R > 0.0))
            return fail(VI_E_INVALID_ARG, "point-light frame must have dmin > 0 and R > 0");
    }
    if (reads_stack) {
        if (!sl || !sl->data) return fail(VI_E_INVALID_ARG, "mode %d needs a stack", mode);
        if (sl->dtype != VI_F32 && sl->dtype != VI_BF16 && sl->dtype != VI_F16)
            return fail(VI_E_UNSUPPORTED, "stack dtype %d", sl->dtype);
        if (sl->layout != VI_STACK_TILED && sl->layout != VI_STACK_ROWS)
            return fail(VI_E_UNSUPPORTED, "stack layout %d", sl->layout);
        if (sl->dtype == VI_F16 && sl->layout != VI_STACK_ROWS)
            return fail(VI_E_UNSUPPORTED, "a half-precision stack needs the row layout");
        if (((uintptr_t)sl->data) % 16) return fail(VI_E_INVALID_ARG, "stack buffer must be 16-byte aligned");
        if (sl->n < 1 || sl->res < 1) return fail(VI_E_INVALID_ARG, "stack descriptor has no size");
        if (sl->vol_n != vol->n)
            return fail(VI_E_INVALID_ARG, "stack built for a volume of edge %d, rendering %d", sl->vol_n, vol->n);
        if (sl->tag != 0 && sl->tag != vi_tag(vol, tf))
            return fail(VI_E_INVALID_ARG, "stack was built from another volume or transfer function");
        if (!stack_size_ok(sl->n, sl->res, sl->dtype, sl->layout))
            return fail(VI_E_UNSUPPORTED, "stack exceeds the layout's limit");
    }

    vi::RenderFrame& F = *out;
    memset(&F, 0, sizeof F);
    F.vol = vol->data;
    F.vol_dtype = vol->dtype;
    F.vol_layout = vol->layout;
    volume_strides(vol, &F.vsy, &F.vsz);
    F.occ = occ_of(vol);
    F.N = vol->n;
    F.M = vol->n / 2;
    F.scale = vol->scale;
    F.tf = tf->rgba;
    F.K = tf->n_entries;
    F.mode = mode;
    // Geometry is derived in double here and handed to the kernels as float
    // affine coefficients of the offset-voxel position h = p N - 1/2 - M
    // (p = (h + 1/2 + M) / N), so that no GPU step needs double.
    const double Nd = vol->n, hoff = 0.5 + F.M;
    if (mode == VI_MODE_PHONG)
        for (int a = 0; a < 3; ++a) F.L[a] = (float)sl->L[a];
    if (point) {
        F.point = 1;
        for (int a = 0; a < 3; ++a) split_float(sl->P[a] * Nd - hoff, &F.Ph[a], &F.Phl[a]);
    }
    double Lq[3] = {0, 0, 0}, Ux[3] = {0, 0, 0}, Vy[3] = {0, 0, 0};  // per world unit
    if (reads_stack) {
        F.stack = sl->data;
        F.stack_dtype = sl->dtype;
        F.n = sl->n;
        F.res = sl->res;
        F.stack_layout = sl->layout;
        F.layer = vi::round_up((uint32_t)sl->res, 8u) * vi::round_up((uint32_t)sl->res, 4u);
        F.row_tiles32 = vi::round_up((uint32_t)sl->res, 8u) * 4u;
        F.rpitch = row_pitch(sl->res, sl->dtype);
        F.rorg = row_origin(sl->res, sl->dtype);
        F.rlayer = row_layer(sl->res, sl->dtype);
        F.Mz = sl->n / 2;
        F.Mr = sl->res / 2;
        // rows: the shifted bases and the element of light-grid cell (0, 0, 0)
        const size_t es = elem_size(sl->dtype);
        F.stack_r1 = (const char*)sl->data + (size_t)F.rpitch * es;
        F.stack_l1 = (const char*)sl->data + (size_t)F.rlayer * es;
        F.stack_l1r1 = (const char*)sl->data + ((size_t)F.rlayer + F.rpitch) * es;
        F.rbase = F.rorg + (uint32_t)F.Mr * F.rpitch + (uint32_t)F.Mr + (uint32_t)F.Mz * F.rlayer;
        const double span = sl->dmax - sl->dmin, sc = sl->res / (2.0 * sl->R);
        for (int a = 0; a < 3; ++a) {
            Lq[a] = sl->n * sl->L[a] / span;
            Ux[a] = sl->U[a] * sc;
            Vy[a] = sl->V[a] * sc;
            split_float(sl->L[a], &F.L[a], &F.Ll[a]);
            split_float(sl->U[a], &F.U[a], &F.Ul[a]);
            split_float(sl->V[a], &F.V[a], &F.Vl[a]);
        }
        // world-unit offsets of the three maps (Eq. 9 index minus one; a
        // point light's depth is measured from the light: d = L.p - L.P)
        double Lq0 = point ? -sl->n * (sl->dmin + dot3(sl->L, sl->P)) / span - 1.0 : -sl->n * sl->dmin / span - 1.0;
        double Ux0 = (-dot3(sl->U, sl->c) + sl->R) * sc - 0.5;
        double Vy0 = (-dot3(sl->V, sl->c) + sl->R) * sc - 0.5;
        // the same maps of h, less the integer offsets Mz, Mr
        for (int a = 0; a < 3; ++a) {
            Lq0 += Lq[a] * hoff / Nd;
            Ux0 += Ux[a] * hoff / Nd;
            Vy0 += Vy[a] * hoff / Nd;
            split_float(Lq[a] / Nd, &F.Lq[a], &F.Lql[a]);
            split_float(Ux[a] / Nd, &F.Ux[a], &F.Uxl[a]);
            split_float(Vy[a] / Nd, &F.Vy[a], &F.Vyl[a]);
        }
        split_float(Lq0 - F.Mz, &F.Lq0, &F.Lq0l);
        split_float(Ux0 - F.Mr, &F.Ux0, &F.Ux0l);
        split_float(Vy0 - F.Mr, &F.Vy0, &F.Vy0l);
        F.ds = (float)(sl->ds * Nd);
        F.ids = (float)(1.0 / (sl->ds * Nd));
        if (point) {
            F.sc = (float)sc;
            F.xo = (float)(0.5 * sl->res - 0.5 - F.Mr);
        }
    }
    // camera basis
    double fwd[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1], cam->target[2] - cam->eye[2]};
    const double nf = sqrt(dot3(fwd, fwd));
    if (!(nf > 0.0) || !isfinite(nf)) return fail(VI_E_INVALID_ARG, "camera eye equals target");
    for (int a = 0; a < 3; ++a) fwd[a] /= nf;
    double right[3], up2[3];
    cross3(fwd, cam->up, right);
    const double nr = sqrt(dot3(right, right));
    if (!(nr > 1e-12) || !isfinite(nr)) return fail(VI_E_INVALID_ARG, "camera up is parallel to the view");
    for (int a = 0; a < 3; ++a) right[a] /= nr;
    cross3(right, fwd, up2);
    F.cam_kind = cam->kind;
    F.width = cam->width;
    F.height = cam->height;
    const double aspect = (double)cam->width / cam->height;
    double tx, ty;
    if (cam->kind == VI_CAM_PERSP) {
        if (!(cam->fovy_deg > 0.0 && cam->fovy_deg < 180.0)) return fail(VI_E_INVALID_ARG, "fovy outside (0,180)");
        const double th = tan(0.5 * cam->fovy_deg * M_PI / 180.0);
        tx = th * aspect;
        ty = th;
    } else {
        if (!(cam->ortho_half_h > 0.0)) return fail(VI_E_INVALID_ARG, "ortho_half_h must be > 0");
        // the image plane's extent in voxels
        tx = cam->ortho_half_h * aspect * Nd;
        ty = cam->ortho_half_h * Nd;
    }
    // pixel (px, py): xn = (2 px + 1 - W) / W, yn = (H - 2 py - 1) / H, and
    // b = base + xn R + yn U (base: the eye, or for a pinhole the forward
    // direction) = (base + R (1 - W) / W + U (H - 1) / H) + px (2 R / W) - py (2 U / H)
    const double Wd = cam->width, Hd = cam->height;
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(cam->eye[a])) return fail(VI_E_INVALID_ARG, "camera eye is not finite");
        const double eye_h = cam->eye[a] * Nd - hoff, R = right[a] * tx, U = up2[a] * ty;
        const double base = cam->kind == VI_CAM_PERSP ? fwd[a] : eye_h;
        split_float(eye_h, &F.cam_o[a], &F.cam_ol[a]);
        split_float(fwd[a], &F.cam_f[a], &F.cam_fl[a]);
        split_float(base + R * (1.0 - Wd) / Wd + U * (Hd - 1.0) / Hd, &F.cam_b[a], &F.cam_bl[a]);
        split_float(2.0 * R / Wd, &F.cam_sx[a], &F.cam_sxl[a]);
        split_float(-2.0 * U / Hd, &F.cam_sy[a], &F.cam_syl[a]);
    }
    F.lo = (float)(-hoff);
    F.hi = (float)(Nd - hoff);
    // segments per ray stay below 2^24, where float segment positions are exact
    if (sqrt(3.0) * Nd / step_vox > 16777216.0)
        return fail(VI_E_INVALID_ARG, "step_vox %g gives more than 2^24 segments per ray", (double)step_vox);
    F.dt = step_vox;
    split_float(1.0 / (double)step_vox, &F.idt, &F.idtl);
    F.ambient = o.ambient;
    for (int c = 0; c < 3; ++c) F.light[c] = o.light_rgb[c];
    for (int c = 0; c < 4; ++c) F.bg[c] = o.bg[c];
    F.term_eps = o.term_eps;
    F.phong_ka = o.phong_ka;
    F.phong_kd = o.phong_kd;
    F.phong_ks = o.phong_ks;
    F.phong_shin = o.phong_shininess;
    F.grad_eps = o.grad_eps;
    if (o.samples_opaque != 0 && o.samples_opaque != 1) return fail(VI_E_INVALID_ARG, "samples_opaque must be 0 or 1");
    F.count_opaque = o.samples_opaque;
    if (o.nearest_layer != 0 && o.nearest_layer != 1) return fail(VI_E_INVALID_ARG, "nearest_layer must be 0 or 1");
    F.nearest = o.nearest_layer;

    if (mode == VI_MODE_SHELL) {
        if (o.shell_count < 1 || 6 * o.shell_count > vi::kMaxTaps)
            return fail(VI_E_INVALID_ARG, "shell_count must be 1..%d", vi::kMaxTaps / 6);
        if (!(o.shell_h_vox >= 0.0f)) return fail(VI_E_INVALID_ARG, "shell_h_vox must be >= 0");
        // shell weights: all zero = equal; else w_r >= 0 with a positive sum
        double wsum = 0.0;
        bool weighted = false;
        for (int r = 0; r < 8; ++r) {
            if (!(o.shell_w[r] >= 0.0f) || !isfinite(o.shell_w[r]))
                return fail(VI_E_INVALID_ARG, "shell weights must be finite and >= 0");
            if (r < o.shell_count) {
                weighted |= o.shell_w[r] != 0.0f;
                wsum += o.shell_w[r];
            }
        }
        if (!weighted) wsum = o.shell_count;
        const double h = (double)o.shell_h_vox / vol->n;  // world units
        int t = 0;
        for (int r = 1; r <= o.shell_count; ++r)
            for (int a = 0; a < 3; ++a)
                for (int sg = -1; sg <= 1; sg += 2) {
                    const double off = sg * r * h;
                    F.tz[t] = (float)(off * Lq[a]);
                    if (point) {
                        // world-frame offsets in voxels: the projection
                        // divides by depth per tap
                        F.td_[t] = (float)(off * Nd * sl->L[a]);
                        F.tx_[t] = (float)(off * Nd * sl->U[a]);
                        F.ty_[t] = (float)(off * Nd * sl->V[a]);
                    } else {
                        F.tx_[t] = (float)(off * Ux[a]);
                        F.ty_[t] = (float)(off * Vy[a]);
                    }
                    F.tw[t] = (float)((weighted ? o.shell_w[r - 1] : 1.0) / (6.0 * wsum));
                    ++t;
                }
        F.ntaps = t;
        F.tap_w = 1.0f / t;
    } else if (mode == VI_MODE_CONE) {
        if (!(o.cone_tan >= 0.0f) || !isfinite(o.cone_tan)) return fail(VI_E_INVALID_ARG, "cone_tan must be >= 0");
        F.cone_tan = o.cone_tan;
        F.cone_grid = o.cone_grid;
        if (o.cone_grid > 0) {
            if (o.cone_grid > 7) return fail(VI_E_INVALID_ARG, "cone_grid must be 0..7");
            F.ntaps = o.cone_grid * o.cone_grid;
        } else {
            if (o.cone_rings < 1 || o.cone_rings > 8 || o.cone_angles < 1 || o.cone_angles > 16)
                return fail(VI_E_INVALID_ARG, "cone needs 1..8 rings and 1..16 angles");
            F.cone_rings = o.cone_rings;
            F.cone_angles = o.cone_angles;
            for (int q = 0; q < o.cone_angles; ++q) {
                const double th = 2.0 * M_PI * q / o.cone_angles;
                F.cone_cos[q] = (float)cos(th);
                F.cone_sin[q] = (float)sin(th);
            }
            F.ntaps = o.cone_rings * o.cone_angles;
        }
        F.tap_w = 1.0f / F.ntaps;
    }
    F.out = (float4*)d_rgba;
    F.samples = d_samples;
    return VI_OK;
}

int fail_msg(int code, const char* msg) { return fail(code, "%s", msg); }

}  // namespace vi

extern "C" {

}  // extern "C"
