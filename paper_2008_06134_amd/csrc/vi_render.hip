// vi_render.hip -- eye-space ray march with the slice-based illumination
// coefficient (sections 3.2.2, 3.2.3 and 4).
//
// Four lanes march one ray together (each takes every fourth segment; the
// four segments of a step are composited by an in-group scan).  Per ray, once
// (float): the camera ray, the slab test against the unit cube, the entry
// point in volume and light-grid coordinates and the increments of both per
// voxel of path; for the cone, the per-ray frame (B, L x B) in texel units.
// Per segment: position = entry + s * direction in offset coordinates (so
// the fraction of every interpolation is taken on small magnitudes),
// trilinear fetch, transfer function from LDS, extinction-corrected opacity,
// and -- only when the opacity is non-zero -- the coefficient gather from the
// stack, then the front-to-back update (Eq. 3) with the coefficient weighting
// the emission (Eq. 7).  A ray stops when it exits the cube or its remaining
// transmittance drops to term_eps.
//
// A wave covers 4 x 4 pixels (16 rays x 4 lanes), a workgroup 8 x 8 pixels,
// so the rays of a wave sample neighbouring voxels and texels.
#include "vi_device.h"
#include "vi_internal.h"

namespace vi {

// --------------------------------------------------------------------------
// stack access
// --------------------------------------------------------------------------
// A float stack holds transmittance T; a bfloat16 stack holds optical depth
// in base-2 units, tau2 = -log2 T (Eq. 6's exponent summed over the slabs in
// front, over ln 2), so that each texel converts to T = 2^-tau2 with one
// exponential before the interpolation; a half-precision stack holds T
// (from the float optical depth), converted with no exponential.
template <int SDT>
__device__ __forceinline__ float stack_texel(const void* __restrict__ S, uint32_t idx);

template <>
__device__ __forceinline__ float stack_texel<VI_F32>(const void* __restrict__ S, uint32_t idx)
{
    return ((const float*)S)[idx];
}
template <>
__device__ __forceinline__ float stack_texel<VI_BF16>(const void* __restrict__ S, uint32_t idx)
{
    return fast_exp2(-bf16_to_f32(((const uint16_t*)S)[idx]));
}
template <>
__device__ __forceinline__ float stack_texel<VI_F16>(const void* __restrict__ S, uint32_t idx)
{
    return __half2float(((const __half*)S)[idx]);
}

// Row layout: the two texels (i, i+1) of one bilinear row, element e and
// e+1, with one load: 8 bytes (4-byte aligned) for float, 4 bytes (2-byte
// aligned, which global loads allow) for bfloat16.
typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32_a2 __attribute__((aligned(2)));

// The load and the conversion are separate steps (PairRaw holds the loaded
// bits), so that a gather can issue the loads of several taps before it
// converts any of them.
template <int SDT> struct PairRaw;
template <> struct PairRaw<VI_F32> { f32x2_a4 v; };
template <> struct PairRaw<VI_BF16> { uint32_t w; };
template <> struct PairRaw<VI_F16> { uint32_t w; };

template <int SDT>
__device__ __forceinline__ PairRaw<SDT> pair_load(const void* __restrict__ S, uint32_t e);
// (Byte offsets are formed in 32 bits -- a stack is below 4 GiB -- so that
// each load takes the stack's base from scalar registers and a 32-bit
// offset, with no 64-bit address arithmetic per load.)
template <>
__device__ __forceinline__ PairRaw<VI_F32> pair_load<VI_F32>(const void* __restrict__ S, uint32_t e)
{
    return PairRaw<VI_F32>{*(const f32x2_a4*)((const char*)S + (e << 2))};
}
template <>
__device__ __forceinline__ PairRaw<VI_BF16> pair_load<VI_BF16>(const void* __restrict__ S, uint32_t e)
{
    return PairRaw<VI_BF16>{*(const u32_a2*)((const char*)S + (e << 1))};
}
template <>
__device__ __forceinline__ PairRaw<VI_F16> pair_load<VI_F16>(const void* __restrict__ S, uint32_t e)
{
    return PairRaw<VI_F16>{*(const u32_a2*)((const char*)S + (e << 1))};
}
__device__ __forceinline__ float2 pair_value(const PairRaw<VI_F32>& r) { return make_float2(r.v.x, r.v.y); }
__device__ __forceinline__ float2 pair_value(const PairRaw<VI_F16>& r)
{
    return make_float2(__half2float(__ushort_as_half((unsigned short)(r.w & 0xffffu))),
                       __half2float(__ushort_as_half((unsigned short)(r.w >> 16))));
}
__device__ __forceinline__ float2 pair_value(const PairRaw<VI_BF16>& r)
{
    // element e in the low half, e + 1 in the high half (little-endian)
    return make_float2(fast_exp2(-__uint_as_float(r.w << 16)), fast_exp2(-__uint_as_float(r.w & 0xffff0000u)));
}

// One row-layout lookup split into its four loads (rows j, j+1 of layers k0
// and k1) and its arithmetic.  The layout makes every footprint a plain read:
// layer -1 (face 0) transmits fully, so a depth index in front of the first
// face needs no test, and the two-texel border lets a footprint that reaches
// past the grid clamp onto border texels only (a column a < -2 reads the
// pair (-2, -1), a > res the pair (res, res+1): both 1).  No selects, no
// branches; the four loads go out together.
template <int SDT>
struct RowTap {
    PairRaw<SDT> a0, a1, b0, b1;  // layer k0 rows j, j+1; layer k1 rows j, j+1
    float wx, wy, wz;
};
template <int SDT, bool NEAR>
__device__ __forceinline__ void rowtap_load(const RenderFrame& F, float z, float x, float y, RowTap<SDT>& t)
{
    if (NEAR) z = floorf(z + 0.5f);
    // clamping the coordinates (not the texel indices) keeps every footprint
    // on stored texels: beyond the grid both texels of a row are border
    // texels (1), so the value is the same 1 whatever the weight
    z = __builtin_amdgcn_fmed3f(z, (float)(-1 - F.Mz), (float)(F.n - 1 - F.Mz));
    x = __builtin_amdgcn_fmed3f(x, (float)(-2 - F.Mr), (float)(F.res - F.Mr));
    y = __builtin_amdgcn_fmed3f(y, (float)(-2 - F.Mr), (float)(F.res - F.Mr));
    const float fz = floorf(z), fx = floorf(x), fy = floorf(y);
    t.wz = z - fz;
    t.wx = x - fx;
    t.wy = y - fy;
    // texel (k0, b, a) of the footprint, k0 = iz + Mz in -1 .. n-1 and
    // a, b = ix, iy + Mr in -2 .. res: one offset for all four loads, whose
    // next row and next layer come from the shifted bases (layer n repeats
    // layer n-1, so k0 + 1 needs no clamp)
    const int iz = (int)fz, ix = (int)fx, iy = (int)fy;
    const uint32_t e = F.rbase + (uint32_t)(iz * (int)F.rlayer) + (uint32_t)__mul24(iy, (int)F.rpitch) + (uint32_t)ix;
    t.a0 = pair_load<SDT>(F.stack, e);
    t.a1 = pair_load<SDT>(F.stack_r1, e);
    t.b0 = pair_load<SDT>(F.stack_l1, e);
    t.b1 = pair_load<SDT>(F.stack_l1r1, e);
}
template <int SDT>
__device__ __forceinline__ float rowtap_value(const RowTap<SDT>& t)
{
    float2 r0 = pair_value(t.a0), r1 = pair_value(t.a1);
    float ab = fmaf(t.wx, r0.y - r0.x, r0.x), cd = fmaf(t.wx, r1.y - r1.x, r1.x);
    const float t0 = fmaf(t.wy, cd - ab, ab);
    r0 = pair_value(t.b0);
    r1 = pair_value(t.b1);
    ab = fmaf(t.wx, r0.y - r0.x, r0.x);
    cd = fmaf(t.wx, r1.y - r1.x, r1.x);
    const float t1 = fmaf(t.wy, cd - ab, ab);
    return fmaf(t.wz, t1 - t0, t0);
}

// Transmittance at light-grid offset coordinates (z, x, y): depth between
// faces (layer z and z+1 in stack order, layer -1 = 1), bilinear in the
// layer, fully transmitting outside the texel grid.
template <int SDT, int SL, bool NEAR>
__device__ __forceinline__ float stack_lookup(const RenderFrame& F, float z, float x, float y)
{
    if (SL == VI_STACK_ROWS) {
        RowTap<SDT> t;
        rowtap_load<SDT, NEAR>(F, z, x, y, t);
        return rowtap_value<SDT>(t);
    }
    if (NEAR) z = floorf(z + 0.5f);
    z = fminf(fmaxf(z, (float)(-1 - F.Mz)), (float)(F.n - 1 - F.Mz));
    const float fz = floorf(z), fx = floorf(x), fy = floorf(y);
    const float wz = z - fz, wx = x - fx, wy = y - fy;
    const int k0 = (int)fz + F.Mz;
    const int k1 = min(k0 + 1, F.n - 1);
    const int i0 = (int)fx + F.Mr, j0 = (int)fy + F.Mr;
    const int res = F.res;
    const bool vi0 = (unsigned)i0 < (unsigned)res, vi1 = (unsigned)(i0 + 1) < (unsigned)res;
    const bool vj0 = (unsigned)j0 < (unsigned)res, vj1 = (unsigned)(j0 + 1) < (unsigned)res;
    const uint32_t oi0 = stack_oi(clampi(i0, 0, res - 1)), oi1 = stack_oi(clampi(i0 + 1, 0, res - 1));
    const uint32_t oj0 = stack_oj(clampi(j0, 0, res - 1), F.row_tiles32);
    const uint32_t oj1 = stack_oj(clampi(j0 + 1, 0, res - 1), F.row_tiles32);

    constexpr float one = 1.0f;
    float t0 = one;
    if (k0 >= 0) {
        const uint32_t base = (uint32_t)k0 * F.layer;
        const uint32_t r0 = base + oj0, r1 = base + oj1;
        float a = stack_texel<SDT>(F.stack, r0 + oi0), b = stack_texel<SDT>(F.stack, r0 + oi1);
        float c = stack_texel<SDT>(F.stack, r1 + oi0), d = stack_texel<SDT>(F.stack, r1 + oi1);
        a = (vi0 && vj0) ? a : one;
        b = (vi1 && vj0) ? b : one;
        c = (vi0 && vj1) ? c : one;
        d = (vi1 && vj1) ? d : one;
        const float ab = fmaf(wx, b - a, a), cd = fmaf(wx, d - c, c);
        t0 = fmaf(wy, cd - ab, ab);
    }
    float t1;
    {
        const uint32_t base = (uint32_t)k1 * F.layer;
        const uint32_t r0 = base + oj0, r1 = base + oj1;
        float a = stack_texel<SDT>(F.stack, r0 + oi0), b = stack_texel<SDT>(F.stack, r0 + oi1);
        float c = stack_texel<SDT>(F.stack, r1 + oi0), d = stack_texel<SDT>(F.stack, r1 + oi1);
        a = (vi0 && vj0) ? a : one;
        b = (vi1 && vj0) ? b : one;
        c = (vi0 && vj1) ? c : one;
        d = (vi1 && vj1) ? d : one;
        const float ab = fmaf(wx, b - a, a), cd = fmaf(wx, d - c, c);
        t1 = fmaf(wy, cd - ab, ab);
    }
    return fmaf(wz, t1 - t0, t0);
}

// --------------------------------------------------------------------------
// one ray
// --------------------------------------------------------------------------
struct ConeFrame {
    float bx, by;  // B in texels per world unit (x, y)
    float px, py;  // L x B in texels per world unit
};

// NB stack lookups at once: all their loads are issued before any of them
// is converted (row layout; the tiled layout looks up one at a time), so a
// gather waits on one round trip per batch of taps.  Larger batches keep
// more loads in flight per wave but take registers, i.e. resident waves;
// measured on the 512^3 workload: the ring cone and the float-stack shell
// (the latter held to six waves per SIMD) run fastest with two taps per
// batch, the 5 x 5 lattice with one (four loads); the bfloat16 shell, whose
// decoding takes more registers, keeps one.
template <int MODE, int SDT>
constexpr int tap_batch()
{
    return (MODE == VI_MODE_CONE || (MODE == VI_MODE_SHELL && SDT == VI_F32)) ? 2 : 1;
}

template <int SDT, int SL, bool NEAR, int NB>
__device__ __forceinline__ void lookup_batch(const RenderFrame& F, const float (&z)[NB], const float (&x)[NB],
                                             const float (&y)[NB], float (&out)[NB])
{
    if constexpr (SL == VI_STACK_ROWS) {
        RowTap<SDT> t[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) rowtap_load<SDT, NEAR>(F, z[u], x[u], y[u], t[u]);
#pragma unroll
        for (int u = 0; u < NB; ++u) out[u] = rowtap_value<SDT>(t[u]);
    } else {
#pragma unroll
        for (int u = 0; u < NB; ++u) out[u] = stack_lookup<SDT, SL, NEAR>(F, z[u], x[u], y[u]);
    }
}

template <int MODE, int SDT, int SL, bool NEAR>
__device__ __forceinline__ float gather(const RenderFrame& F, const ConeFrame& cf, float z, float x, float y)
{
    if (MODE == VI_MODE_SHADOW) return stack_lookup<SDT, SL, NEAR>(F, z, x, y);
    // Taps go in batches; a batch running past the last tap repeats it and
    // leaves the sum alone for the repeats, so every tap is added once, in
    // order, as a one-at-a-time loop adds it.
    constexpr int NB = tap_batch<MODE, SDT>();
    float zz[NB], xx[NB], yy[NB], v[NB];
    if (MODE == VI_MODE_SHELL) {
        // weighted taps (shell r's six taps share w_r / (6 sum w))
        float s = 0.0f;
        for (int t = 0; t < F.ntaps; t += NB) {
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int i = min(t + u, F.ntaps - 1);
                zz[u] = z + F.tz[i];
                xx[u] = x + F.tx_[i];
                yy[u] = y + F.ty_[i];
            }
            lookup_batch<SDT, SL, NEAR>(F, zz, xx, yy, v);
#pragma unroll
            for (int u = 0; u < NB; ++u)
                if (t + u < F.ntaps) s = fmaf(F.tw[t + u], v[u], s);
        }
        return s;
    }
    // cone: rings (Eq. 11), or the lattice form in a kernel of its own
    float s = 0.0f;
    if (MODE == VI_MODE_CONE) {
        for (int m = 1; m <= F.cone_rings; ++m) {
            const float r = (float)m * F.ds * F.cone_tan;
            for (int q = 0; q < F.cone_angles; q += NB) {
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int i = min(q + u, F.cone_angles - 1);
                    const float ca = F.cone_cos[i] * r, sa = F.cone_sin[i] * r;
                    zz[u] = z - (float)m;
                    xx[u] = x + ca * cf.bx + sa * cf.px;
                    yy[u] = y + ca * cf.by + sa * cf.py;
                }
                lookup_batch<SDT, SL, NEAR>(F, zz, xx, yy, v);
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    if (q + u < F.cone_angles) s += v[u];
            }
        }
    } else if (MODE == kModeConeGrid) {
        const int G = F.cone_grid;
        const float rho = F.ds * F.cone_tan * 0.5f, half = 0.5f * (float)(G - 1);
        for (int ia = 0; ia < G; ++ia) {
            const float a = ((float)ia - half) * rho;
            for (int ib = 0; ib < G; ib += NB) {
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const float b = ((float)min(ib + u, G - 1) - half) * rho;
                    zz[u] = z - 1.0f;
                    xx[u] = x + a * cf.bx + b * cf.px;
                    yy[u] = y + a * cf.by + b * cf.py;
                }
                lookup_batch<SDT, SL, NEAR>(F, zz, xx, yy, v);
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    if (ib + u < G) s += v[u];
            }
        }
    }
    return s * F.tap_w;
}

// Point light: the light grid is a frustum with its apex at P.  A lookup at
// depth d = L.(p - P) and lateral offsets (u, v) = (U, V).(p - P) reads texel
// column (u / d) sc + xo; a point at or behind the apex's plane (d <= 0) lies
// outside every texel, where the stack reads 1.  The column is clamped to a
// band just outside the grid, which keeps huge quotients finite.
__device__ __forceinline__ float frustum_col(const RenderFrame& F, float u, float rd, bool ahead)
{
    const float x = ahead ? fmaf(u * rd, F.sc, F.xo) : -3.0e38f;
    return fminf(fmaxf(x, (float)(-3 - F.Mr)), (float)(F.res + 2 - F.Mr));
}

// Cone (Eq. 11) about the light's direction at the sample.  With r = (d, u,
// v) the sample's offset from the light in the light frame (voxels), the
// axis is L_s = r / |r|, and one slab of depth toward the light lies
// S = ds |r| / d along it.  Tap (c, a, b) sits at
//   r - c S L_s + S (a B + b L_s x B) = r (1 - c ds / d) + S (a B + b L_s x B),
// B the view vector w = (wd, wu, wv) with its L_s part removed (U's, when w
// runs along L_s), of unit length; ring m has c = m and (a, b) = m tan phi
// (cos, sin) theta, the lattice c = 1 and (a, b) on a grid of spacing
// tan phi / 2.  The tap's slab index moves with its depth: c slabs, plus
// the depth part of the lateral offset.  Taps are summed in the order rings
// (or lattice rows), then angles (or columns), in batches as in gather().
template <int SDT, int SL, bool NEAR>
__device__ __forceinline__ float gather_point_cone(const RenderFrame& F, float z, float d, float u, float v, float wd,
                                                   float wu, float wv)
{
    const float r2 = fmaf(d, d, fmaf(u, u, v * v)), ir = __builtin_amdgcn_rsqf(r2);
    const float ld = d * ir, lu = u * ir, lv = v * ir;
    const float wl = fmaf(wd, ld, fmaf(wu, lu, wv * lv));
    float bd = fmaf(-wl, ld, wd), bu = fmaf(-wl, lu, wu), bv = fmaf(-wl, lv, wv);
    float nb = fmaf(bd, bd, fmaf(bu, bu, bv * bv));
    if (nb < 1e-12f) {
        // U is (0, 1, 0) in the light frame
        bd = -lu * ld;
        bu = fmaf(-lu, lu, 1.0f);
        bv = -lu * lv;
        nb = fmaf(bd, bd, fmaf(bu, bu, bv * bv));
    }
    const float q = F.ds * __builtin_amdgcn_rcpf(d);                  // ds / d
    const float sb = (q * r2 * ir) * __builtin_amdgcn_rsqf(nb);       // S / |B|
    bd *= sb;
    bu *= sb;
    bv *= sb;
    const float cd = fmaf(lu, bv, -lv * bu), cu = fmaf(lv, bd, -ld * bv), cv = fmaf(ld, bu, -lu * bd);
    const auto tap = [&](float c, float a, float b, float& zz, float& xx, float& yy) {
        const float k = fmaf(-c, q, 1.0f);
        const float od = fmaf(a, bd, b * cd);
        const float dd = fmaf(d, k, od);
        const float rd = __builtin_amdgcn_rcpf(dd);
        zz = fmaf(od, F.ids, z - c);
        xx = frustum_col(F, fmaf(u, k, fmaf(a, bu, b * cu)), rd, dd > 0.0f);
        yy = frustum_col(F, fmaf(v, k, fmaf(a, bv, b * cv)), rd, dd > 0.0f);
    };
    constexpr int NB = 2;
    float zz[NB], xx[NB], yy[NB], val[NB];
    float s = 0.0f;
    if (F.cone_grid == 0) {
        for (int m = 1; m <= F.cone_rings; ++m) {
            const float c = (float)m, r = c * F.cone_tan;
            for (int t = 0; t < F.cone_angles; t += NB) {
#pragma unroll
                for (int w = 0; w < NB; ++w) {
                    const int i = min(t + w, F.cone_angles - 1);
                    tap(c, F.cone_cos[i] * r, F.cone_sin[i] * r, zz[w], xx[w], yy[w]);
                }
                lookup_batch<SDT, SL, NEAR>(F, zz, xx, yy, val);
#pragma unroll
                for (int w = 0; w < NB; ++w)
                    if (t + w < F.cone_angles) s += val[w];
            }
        }
    } else {
        const int G = F.cone_grid;
        const float rho = 0.5f * F.cone_tan, half = 0.5f * (float)(G - 1);
        for (int ia = 0; ia < G; ++ia) {
            const float a = ((float)ia - half) * rho;
            for (int ib = 0; ib < G; ib += NB) {
#pragma unroll
                for (int w = 0; w < NB; ++w)
                    tap(1.0f, a, ((float)min(ib + w, G - 1) - half) * rho, zz[w], xx[w], yy[w]);
                lookup_batch<SDT, SL, NEAR>(F, zz, xx, yy, val);
#pragma unroll
                for (int w = 0; w < NB; ++w)
                    if (ib + w < G) s += val[w];
            }
        }
    }
    return s * F.tap_w;
}

template <int MODE, int SDT, int SL, bool NEAR>
__device__ __forceinline__ float gather_point(const RenderFrame& F, float z, float d, float u, float v, float wd,
                                              float wu, float wv)
{
    if (MODE == kModePointShadow) {
        const float rd = __builtin_amdgcn_rcpf(d);
        return stack_lookup<SDT, SL, NEAR>(F, z, frustum_col(F, u, rd, d > 0.0f), frustum_col(F, v, rd, d > 0.0f));
    }
    if constexpr (MODE == kModePointCone) return gather_point_cone<SDT, SL, NEAR>(F, z, d, u, v, wd, wu, wv);
    // shell taps: world-frame offsets, each projected through its own depth
    // (batched as in gather())
    float s = 0.0f;
    constexpr int NB = tap_batch<MODE, SDT>();
    float zz[NB], xx[NB], yy[NB], val[NB];
    for (int t = 0; t < F.ntaps; t += NB) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int i = min(t + q, F.ntaps - 1);
            const float dt = d + F.td_[i], rd = __builtin_amdgcn_rcpf(dt);
            zz[q] = z + F.tz[i];
            xx[q] = frustum_col(F, u + F.tx_[i], rd, dt > 0.0f);
            yy[q] = frustum_col(F, v + F.ty_[i], rd, dt > 0.0f);
        }
        lookup_batch<SDT, SL, NEAR>(F, zz, xx, yy, val);
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (t + q < F.ntaps) s = fmaf(F.tw[t + q], val[q], s);
    }
    return s;
}

// G lanes march one ray together: lane g of the group takes segment k + g of
// every group step, the G segments are composited front to back with a scan
// over the group (inclusive product of (1 - alpha), then the emission of each
// segment weighted by the transmittance in front of it), and the ray stops
// exactly at the first segment after which 1 - alpha_dst <= term_eps.  All
// lanes of a group carry identical ray state.  G = 1 is the plain sequential
// march; larger G shortens the longest waves (rays of ~1000 non-empty
// segments) and packs the G samples of a step within a couple of voxels.
template <int G>
__device__ __forceinline__ float group_scan_mul(float x, int g)
{
    for (int d = 1; d < G; d <<= 1) {
        const float t = __shfl_up(x, d, G);
        if (g >= d) x *= t;
    }
    return x;
}
template <int G>
__device__ __forceinline__ float group_sum(float x)
{
    for (int d = G / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, G);
    return x;
}
template <int G>
__device__ __forceinline__ uint32_t group_bits(bool p, int base)
{
    const unsigned long long m = __ballot(p);
    return (uint32_t)((m >> base) & ((G == 32 ? 0xffffffffull : ((1ull << G) - 1ull))));
}

// Per-ray march state (identical in the G lanes of a ray's group): the ray
// in offset-voxel coordinates, its light-grid maps, the cone basis or Phong
// vectors, the empty-space cache and the compositing state.
struct RayState {
    float hx0, hy0, hz0, hdx, hdy, hdz;  // entry point and direction
    float Df;                            // chord length, voxels
    int K;                               // segments
    float qz0, qx0, qy0, qdz, qdx, qdy, pd0, pdd;
    ConeFrame cf;
    float lx, ly, lz, vx, vy, vz, lv;
    float ihx, ihy, ihz;
    float Cr, Cg, Cb, T;
    uint32_t last_cell;
    bool cell_is_empty;
    int k, count;
};

constexpr bool is_point_gather(int mode)
{
    return mode == kModePointShadow || mode == kModePointShell || mode == kModePointCone;
}

// Ray set-up for pixel (px, py): false if the ray misses the cube (the pixel
// is then the background).
template <typename VT, int LAYOUT, int MODE, int SDT, int SL, int G>
__device__ __forceinline__ bool ray_setup(const RenderFrame& F, int px, int py, RayState& S)
{
    // ---- camera ray, in offset-voxel coordinates, in float pairs (the
    // host folded the camera and the light grid into float-pair
    // coefficients of h; see F2): pixel (px, py) -> b = base + px sx + py sy
    F2 o[3], d[3];
    {
        const F2 fx = f2((float)px), fy = f2((float)py);
        for (int a = 0; a < 3; ++a) {
            const F2 b = f2_add(F2{F.cam_b[a], F.cam_bl[a]},
                                f2_add(f2_mul(fx, F2{F.cam_sx[a], F.cam_sxl[a]}), f2_mul(fy, F2{F.cam_sy[a], F.cam_syl[a]})));
            if (F.cam_kind == VI_CAM_PERSP) {
                o[a] = F2{F.cam_o[a], F.cam_ol[a]};
                d[a] = b;
            } else {
                o[a] = b;
                d[a] = F2{F.cam_f[a], F.cam_fl[a]};
            }
        }
        if (F.cam_kind == VI_CAM_PERSP) {
            const F2 inv = f2_rsqrt(f2_dot3(d, d));
            for (int a = 0; a < 3; ++a) d[a] = f2_mul(d[a], inv);
        }
    }
    // ---- slab test against the cube [lo, hi]^3 (distances in voxels): the
    // entry and exit faces are picked in float, their distances then taken on
    // the pairs
    float tn = -3.0e38f, tf_ = 3.0e38f, bn = 0.0f, bf = 0.0f;
    int an = -1, af = -1;
    bool hit = true;
    for (int a = 0; a < 3; ++a) {
        if (d[a].hi == 0.0f) {
            if (o[a].hi < F.lo || o[a].hi > F.hi) hit = false;
            continue;
        }
        const float r = __builtin_amdgcn_rcpf(d[a].hi);
        const float near = d[a].hi > 0.0f ? F.lo : F.hi, far = d[a].hi > 0.0f ? F.hi : F.lo;
        const float t1 = (near - o[a].hi) * r, t2 = (far - o[a].hi) * r;
        if (t1 > tn) tn = t1, an = a, bn = near;
        if (t2 < tf_) tf_ = t2, af = a, bf = far;
    }
    if (!hit || af < 0 || !(tf_ > fmaxf(tn, 0.0f))) return false;
    // the chosen faces' numerators and denominators, gathered with constant
    // indices (a variable index would put o and d in scratch memory)
    F2 on = f2(0.0f), dn = f2(1.0f), of = f2(0.0f), df = f2(1.0f);
    for (int a = 0; a < 3; ++a) {
        on = a == an ? o[a] : on;
        dn = a == an ? d[a] : dn;
        of = a == af ? o[a] : of;
        df = a == af ? d[a] : df;
    }
    const F2 ti = (an >= 0 && tn > 0.0f) ? f2_div(f2_sub(f2(bn), on), dn) : f2(0.0f);
    const F2 tf = f2_div(f2_sub(f2(bf), of), df);
    if (!f2_lt(ti, tf)) return false;

    const F2 Dc = f2_sub(tf, ti);  // chord length, voxels
    S.Df = Dc.hi;
    int K;
    {
        // K = ceil(D / dt), decided on the pair
        const F2 q = f2_mul(Dc, F2{F.idt, F.idtl});
        float c = ceilf(q.hi);
        if (c == q.hi && q.lo > 0.0f) c += 1.0f;
        else if (c - 1.0f - q.hi >= q.lo) c -= 1.0f;
        K = (int)c;
        S.K = K;
    }
    // volume: entry point (value, remainder) and direction (value, remainder)
    F2 pin[3];
    for (int a = 0; a < 3; ++a) pin[a] = f2_add(o[a], f2_mul(ti, d[a]));
    S.hx0 = pin[0].hi, S.hy0 = pin[1].hi, S.hz0 = pin[2].hi;
    const float hdx = d[0].hi, hdy = d[1].hi, hdz = d[2].hi;
    S.hdx = hdx, S.hdy = hdy, S.hdz = hdz;
    // light grid: depth index (Eq. 9, minus one) and texel coordinates (Eq. 10)
    // (point light: qx / qy hold the lateral offsets U.(h - Ph), V.(h - Ph)
    // and pd the depth L.(h - Ph), all affine along the ray)
    constexpr bool PT = is_point_gather(MODE);
    constexpr bool PTP = MODE == kModePointPhong, PHONG = MODE == VI_MODE_PHONG || PTP;
    float& qz0 = S.qz0; float& qx0 = S.qx0; float& qy0 = S.qy0; float& qdz = S.qdz; float& qdx = S.qdx;
    float& qdy = S.qdy; float& pd0 = S.pd0; float& pdd = S.pdd;
    ConeFrame& cf = S.cf;
    qz0 = qx0 = qy0 = qdz = qdx = qdy = pd0 = pdd = 0.f;
    cf = ConeFrame{0.f, 0.f, 0.f, 0.f};
    // Phong: light vector l = -L and, folded in, l.v with v = -d
    // (point light: l is taken per sample toward P, and lx, ly, lz hold h_in - Ph)
    float& lx = S.lx; float& ly = S.ly; float& lz = S.lz; float& vx = S.vx; float& vy = S.vy; float& vz = S.vz;
    float& lv = S.lv;
    lx = ly = lz = vx = vy = vz = lv = 0.f;
    if (PHONG) {
        lx = -F.L[0];
        ly = -F.L[1];
        lz = -F.L[2];
        vx = -hdx;
        vy = -hdy;
        vz = -hdz;
        lv = fmaf(F.L[0], hdx, fmaf(F.L[1], hdy, F.L[2] * hdz));
        if (PTP) {
            lx = f2_sub(pin[0], F2{F.Ph[0], F.Phl[0]}).hi;
            ly = f2_sub(pin[1], F2{F.Ph[1], F.Phl[1]}).hi;
            lz = f2_sub(pin[2], F2{F.Ph[2], F.Phl[2]}).hi;
        }
    }
    if (MODE != VI_MODE_NONE && !PHONG) {
        const F2 Lq[3] = {F2{F.Lq[0], F.Lql[0]}, F2{F.Lq[1], F.Lql[1]}, F2{F.Lq[2], F.Lql[2]}};
        qz0 = f2_add(f2_dot3(Lq, pin), F2{F.Lq0, F.Lq0l}).hi;
        qdz = fmaf(F.Lq[0], hdx, fmaf(F.Lq[1], hdy, F.Lq[2] * hdz));
        if (PT) {
            const F2 r[3] = {f2_sub(pin[0], F2{F.Ph[0], F.Phl[0]}), f2_sub(pin[1], F2{F.Ph[1], F.Phl[1]}),
                             f2_sub(pin[2], F2{F.Ph[2], F.Phl[2]})};
            const F2 L[3] = {F2{F.L[0], F.Ll[0]}, F2{F.L[1], F.Ll[1]}, F2{F.L[2], F.Ll[2]}};
            const F2 U[3] = {F2{F.U[0], F.Ul[0]}, F2{F.U[1], F.Ul[1]}, F2{F.U[2], F.Ul[2]}};
            const F2 V[3] = {F2{F.V[0], F.Vl[0]}, F2{F.V[1], F.Vl[1]}, F2{F.V[2], F.Vl[2]}};
            pd0 = f2_dot3(L, r).hi;
            pdd = fmaf(F.L[0], hdx, fmaf(F.L[1], hdy, F.L[2] * hdz));
            qx0 = f2_dot3(U, r).hi;
            qdx = fmaf(F.U[0], hdx, fmaf(F.U[1], hdy, F.U[2] * hdz));
            qy0 = f2_dot3(V, r).hi;
            qdy = fmaf(F.V[0], hdx, fmaf(F.V[1], hdy, F.V[2] * hdz));
        } else {
            const F2 Ux[3] = {F2{F.Ux[0], F.Uxl[0]}, F2{F.Ux[1], F.Uxl[1]}, F2{F.Ux[2], F.Uxl[2]}};
            const F2 Vy[3] = {F2{F.Vy[0], F.Vyl[0]}, F2{F.Vy[1], F.Vyl[1]}, F2{F.Vy[2], F.Vyl[2]}};
            qx0 = f2_add(f2_dot3(Ux, pin), F2{F.Ux0, F.Ux0l}).hi;
            qy0 = f2_add(f2_dot3(Vy, pin), F2{F.Vy0, F.Vy0l}).hi;
            qdx = fmaf(F.Ux[0], hdx, fmaf(F.Ux[1], hdy, F.Ux[2] * hdz));
            qdy = fmaf(F.Vy[0], hdx, fmaf(F.Vy[1], hdy, F.Vy[2] * hdz));
        }
        if (MODE == VI_MODE_CONE || MODE == kModeConeGrid) {
            // B: direction toward the viewer with its L component removed
            // (U when the view runs along L)
            const float wl = -fmaf(hdx, F.L[0], fmaf(hdy, F.L[1], hdz * F.L[2]));
            float B[3] = {fmaf(-wl, F.L[0], -hdx), fmaf(-wl, F.L[1], -hdy), fmaf(-wl, F.L[2], -hdz)};
            const float nb = sqrtf(fmaf(B[0], B[0], fmaf(B[1], B[1], B[2] * B[2])));
            if (nb < 1e-6f) {
                for (int a = 0; a < 3; ++a) B[a] = F.U[a];
            } else {
                const float inb = 1.0f / nb;
                for (int a = 0; a < 3; ++a) B[a] *= inb;
            }
            const float P[3] = {F.L[1] * B[2] - F.L[2] * B[1], F.L[2] * B[0] - F.L[0] * B[2],
                                F.L[0] * B[1] - F.L[1] * B[0]};
            // B and L x B in texels per voxel
            cf.bx = fmaf(F.Ux[0], B[0], fmaf(F.Ux[1], B[1], F.Ux[2] * B[2]));
            cf.by = fmaf(F.Vy[0], B[0], fmaf(F.Vy[1], B[1], F.Vy[2] * B[2]));
            cf.px = fmaf(F.Ux[0], P[0], fmaf(F.Ux[1], P[1], F.Ux[2] * P[2]));
            cf.py = fmaf(F.Vy[0], P[0], fmaf(F.Vy[1], P[1], F.Vy[2] * P[2]));
        }
    }

    // C: premultiplied colour so far; T = 1 - alpha_dst, the transmittance in
    // front of the next segment (kept as a product of exact per-segment
    // factors, which keeps its relative precision down to term_eps).
    S.Cr = S.Cg = S.Cb = 0.f;
    S.T = 1.0f;
    S.ihx = hdx != 0.f ? __builtin_amdgcn_rcpf(hdx) : 0.f;
    S.ihy = hdy != 0.f ? __builtin_amdgcn_rcpf(hdy) : 0.f;
    S.ihz = hdz != 0.f ? __builtin_amdgcn_rcpf(hdz) : 0.f;
    S.last_cell = 0xffffffffu;
    S.cell_is_empty = false;
    S.k = 0;
    S.count = K;
    return true;
}

// One step of G segments of the ray's march (the G lanes of its group take
// one segment each); true once the ray is done.
template <typename VT, int LAYOUT, int MODE, int SDT, int SL, int G>
__device__ __forceinline__ bool ray_step(const RenderFrame& F, const float4* __restrict__ s_tf,
                                         const int* __restrict__ s_next, const uint32_t* __restrict__ s_bits,
                                         RayState& S, uint32_t& nop)
{
    const int lane = threadIdx.x & 63, g = lane % G, gbase = lane - g;
    constexpr bool PT = is_point_gather(MODE);
    constexpr bool PTP = MODE == kModePointPhong, PHONG = MODE == VI_MODE_PHONG || PTP;
    const float hx0 = S.hx0, hy0 = S.hy0, hz0 = S.hz0, hdx = S.hdx, hdy = S.hdy, hdz = S.hdz;
    const float qz0 = S.qz0, qx0 = S.qx0, qy0 = S.qy0, qdz = S.qdz, qdx = S.qdx, qdy = S.qdy, pd0 = S.pd0,
                pdd = S.pdd;
    const ConeFrame cf = S.cf;
    const float lx = S.lx, ly = S.ly, lz = S.lz, vx = S.vx, vy = S.vy, vz = S.vz, lv = S.lv;
    const float Df = S.Df, ihx = S.ihx, ihy = S.ihy, ihz = S.ihz;
    const int K = S.K;
    float& Cr = S.Cr; float& Cg = S.Cg; float& Cb = S.Cb; float& T = S.T;
    uint32_t& last_cell = S.last_cell;
    bool& cell_is_empty = S.cell_is_empty;
    int& k = S.k;
    int& count = S.count;
    const VT* __restrict__ vol = (const VT*)F.vol;
    const VolIndex VI_ = {1u, F.vsy, F.vsz};
    const float dtf = F.dt;
    const float Km1 = (float)(F.K - 1);
    // Empty-space traversal.  A group whose G segments all lie in
    // zero-opacity cells jumps to the last segment midpoint inside the empty
    // box around its last segment -- the segment's cell, or the cell's
    // super-cell (4 x 4 x 4 cells) when that is empty too -- with the box's
    // faces moved inward by kEps voxels (far above the float position
    // error), so no segment with non-zero opacity is ever skipped.  Faces of
    // boxes at the volume's edge toward the outside are at infinity (edge
    // cells also hold the clamped positions beyond the last voxel centre).
    const float kEps = 0.02f;
    const float Mf = (float)F.M;
    const int kk = k + g;
    const bool in = kk < K;
    float om = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;  // om = 1 - alpha of the segment
    bool empty = true;
    int cx = 0, cy = 0, cz = 0;  // the segment's cell
    if (in) {
        const float s0 = (float)kk * dtf;
        const float s1 = fminf((float)(kk + 1) * dtf, Df);
        const float len = s1 - s0;
        const float sm = 0.5f * (s0 + s1);
        const float hx = fmaf(sm, hdx, hx0), hy = fmaf(sm, hdy, hy0), hz = fmaf(sm, hdz, hz0);
        empty = false;
        if (F.occ.mm) {
            const int gx = clampi((int)floorf(hx) + F.M, 0, F.N - 1),
                      gy = clampi((int)floorf(hy) + F.M, 0, F.N - 1),
                      gz = clampi((int)floorf(hz) + F.M, 0, F.N - 1);
            cx = gx >> F.occ.shift, cy = gy >> F.occ.shift, cz = gz >> F.occ.shift;
            const uint32_t c = __umul24(__umul24((uint32_t)cz, F.occ.nc) + (uint32_t)cy, F.occ.nc) + (uint32_t)cx;
            if (c != last_cell) {
                last_cell = c;
                cell_is_empty = !cell_occupied(F.occ, s_bits, c, s_next, Km1, F.K);
            }
            empty = cell_is_empty;
        }
        if (!empty) {
            const float v = sample_volume<VT, LAYOUT>(vol, VI_, F.N, F.M, F.scale, hx, hy, hz);
            const float x = v * Km1;
            const int e0 = min((int)x, F.K - 2);
            const float w = x - (float)e0;
            const float4 ta = s_tf[e0], tb = s_tf[e0 + 1];
            const float a = clampf01(fmaf(w, tb.w - ta.w, ta.w));
            // (1 - alpha) of a segment of length len: (1 - a)^(len / dref)
            if (len > 0.0f && a > 0.0f) om = fast_exp2(len * fast_log2(1.0f - a));
            const float alpha = 1.0f - om;
            if (alpha > 0.0f) {
                // emission alpha (sd rgb + ss) light: Eq. 7 with the
                // coefficient A, or the local Phong terms
                float sd, ss = 0.0f;
                if (PHONG) {
                    // central differences one voxel either side (exact
                    // offsets in voxel units)
                    const float gx = 0.5f * (sample_volume<VT, LAYOUT>(vol, VI_, F.N, F.M, F.scale, hx + 1.f, hy, hz) -
                                             sample_volume<VT, LAYOUT>(vol, VI_, F.N, F.M, F.scale, hx - 1.f, hy, hz));
                    const float gy = 0.5f * (sample_volume<VT, LAYOUT>(vol, VI_, F.N, F.M, F.scale, hx, hy + 1.f, hz) -
                                             sample_volume<VT, LAYOUT>(vol, VI_, F.N, F.M, F.scale, hx, hy - 1.f, hz));
                    const float gz = 0.5f * (sample_volume<VT, LAYOUT>(vol, VI_, F.N, F.M, F.scale, hx, hy, hz + 1.f) -
                                             sample_volume<VT, LAYOUT>(vol, VI_, F.N, F.M, F.scale, hx, hy, hz - 1.f));
                    const float gn = sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
                    const float inv = -1.0f / fmaxf(gn, F.grad_eps);  // n = -g / max(|g|, eps)
                    const float nx = gx * inv, ny = gy * inv, nz = gz * inv;
                    float llx = lx, lly = ly, llz = lz, llv = lv;
                    if (PTP) {
                        // l = (P - p) / |P - p|
                        const float rx = fmaf(sm, -vx, lx), ry = fmaf(sm, -vy, ly), rz = fmaf(sm, -vz, lz);
                        const float ir = -__builtin_amdgcn_rsqf(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
                        llx = rx * ir;
                        lly = ry * ir;
                        llz = rz * ir;
                        llv = fmaf(llx, vx, fmaf(lly, vy, llz * vz));
                    }
                    const float nl = fmaf(nx, llx, fmaf(ny, lly, nz * llz));
                    const float nv = fmaf(nx, vx, fmaf(ny, vy, nz * vz));
                    const float nn = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
                    const float rv = fmaf(2.0f * nl, nv, -nn * llv);  // r.v, r = 2(n.l)n - (n.n)l
                    sd = fmaf(F.phong_kd, fmaxf(nl, 0.0f), F.phong_ka);
                    if (rv > 0.0f) ss = F.phong_ks * fast_exp2(F.phong_shin * fast_log2(rv));
                } else {
                    // (the nearest-face form is a second copy of the
                    // gather behind a branch that is uniform per frame)
                    float A = 1.0f;
                    const float qz = fmaf(sm, qdz, qz0), qx = fmaf(sm, qdx, qx0), qy = fmaf(sm, qdy, qy0);
                    if (PT) {
                        const float pd = fmaf(sm, pdd, pd0);
                        A = F.nearest ? gather_point<MODE, SDT, SL, true>(F, qz, pd, qx, qy, -pdd, -qdx, -qdy)
                                      : gather_point<MODE, SDT, SL, false>(F, qz, pd, qx, qy, -pdd, -qdx, -qdy);
                    } else if (MODE != VI_MODE_NONE) {
                        A = F.nearest ? gather<MODE, SDT, SL, true>(F, cf, qz, qx, qy)
                                      : gather<MODE, SDT, SL, false>(F, cf, qz, qx, qy);
                    }
                    sd = fmaf(1.0f - F.ambient, A, F.ambient);
                }
                cr = alpha * F.light[0] * fmaf(sd, fmaf(w, tb.x - ta.x, ta.x), ss);
                cg = alpha * F.light[1] * fmaf(sd, fmaf(w, tb.y - ta.y, ta.y), ss);
                cb = alpha * F.light[2] * fmaf(sd, fmaf(w, tb.z - ta.z, ta.z), ss);
            }
        }
    }
    if (group_bits<G>(empty, gbase) == ((G == 32) ? 0xffffffffu : ((1u << G) - 1u))) {
        // every segment of this step is empty (or past the exit): jump,
        // staying on multiples of G so that the steps group segments as a
        // march without the map would (the products then round alike and
        // the map changes no bit of the result).  Each lane finds the
        // last segment inside the empty box around its own segment; the
        // group takes its last lane's.
        int jl = K;
        if (in && F.occ.mm) {
            int sh = F.occ.shift, bx = cx, by = cy, bz = cz, last = (int)F.occ.nc - 1;
            if (F.occ.bits) {
                const int sx = cx >> 2, sy = cy >> 2, sz = cz >> 2;
                const uint32_t sc =
                    __umul24(__umul24((uint32_t)sz, F.occ.snc) + (uint32_t)sy, F.occ.snc) + (uint32_t)sx;
                if (!occupancy_bit(s_bits + F.occ.words, sc)) {
                    sh += 2;
                    bx = sx, by = sy, bz = sz;
                    last = (int)F.occ.snc - 1;
                }
            }
            // distance along the ray to the box's exit faces, moved inward
            const float edge = (float)(1 << sh) - kEps;
            float se = 3.4e38f;
            if (hdx > 0.f && bx < last) se = fminf(se, ((float)(bx << sh) - Mf + edge - hx0) * ihx);
            if (hdx < 0.f && bx > 0) se = fminf(se, ((float)(bx << sh) - Mf + kEps - hx0) * ihx);
            if (hdy > 0.f && by < last) se = fminf(se, ((float)(by << sh) - Mf + edge - hy0) * ihy);
            if (hdy < 0.f && by > 0) se = fminf(se, ((float)(by << sh) - Mf + kEps - hy0) * ihy);
            if (hdz > 0.f && bz < last) se = fminf(se, ((float)(bz << sh) - Mf + edge - hz0) * ihz);
            if (hdz < 0.f && bz > 0) se = fminf(se, ((float)(bz << sh) - Mf + kEps - hz0) * ihz);
            // last full segment whose midpoint (j + 1/2) dt is <= se
            const float jf = floorf(fmaf(se, F.idt, -0.5f));
            jl = jf >= (float)(K - 1) ? K - 1 : (int)jf;
        }
        const int jlast = G == 1 ? jl : __shfl(jl, gbase + G - 1);
        k = max(k + G, ((jlast + 1) / G) * G);
        if (k >= K) return true;
        return false;
    }
    // front-to-back over the G segments of this step (Eq. 3 in product form)
    const float incl = group_scan_mul<G>(om, g);                  // prod_{h<=g} (1 - alpha_h)
    // every lane of the group takes part in the shuffle (a lane that sat
    // out would hand its neighbour no value)
    const float up = G == 1 ? 1.0f : __shfl_up(incl, 1, G);
    const float excl = g == 0 ? 1.0f : up;
    const uint32_t tb_ = group_bits<G>(in && T * incl <= F.term_eps, gbase);
    const int gs = tb_ ? __ffs(tb_) - 1 : G;                     // terminating segment, G if none
    const float keep = (g <= gs) ? T * excl : 0.0f;
    nop += (in && g <= gs && om < 1.0f) ? 1u : 0u;  // composited with non-zero opacity
    Cr += group_sum<G>(keep * cr);
    Cg += group_sum<G>(keep * cg);
    Cb += group_sum<G>(keep * cb);
    const float prod = G == 1 ? incl : __shfl(incl, gbase + min(gs, G - 1));
    T *= prod;
    if (gs < G) {
        count = k + gs + 1;
        return true;
    }
    k += G;
    return k >= K;
}

// The finished ray's colour over the background, and its segment count.
__device__ __forceinline__ float4 ray_result(const RenderFrame& F, const RayState& S)
{
    return make_float4(fmaf(S.T, F.bg[0], S.Cr), fmaf(S.T, F.bg[1], S.Cg), fmaf(S.T, F.bg[2], S.Cb),
                       fmaf(S.T, F.bg[3], 1.0f - S.T));
}

template <typename VT, int LAYOUT, int MODE, int SDT, int SL, int G>
__device__ __forceinline__ float4 render_ray(const RenderFrame& F, const float4* __restrict__ s_tf,
                                             const int* __restrict__ s_next, const uint32_t* __restrict__ s_bits,
                                             int px, int py, uint32_t& nsamp, uint32_t& nop)
{
    RayState S;
    if (!ray_setup<VT, LAYOUT, MODE, SDT, SL, G>(F, px, py, S))
        return make_float4(F.bg[0], F.bg[1], F.bg[2], F.bg[3]);
    while (!ray_step<VT, LAYOUT, MODE, SDT, SL, G>(F, s_tf, s_next, s_bits, S, nop)) {
    }
    if ((threadIdx.x & 63) % G == 0) nsamp += (uint32_t)min(S.count, S.K);
    return ray_result(F, S);
}

// --------------------------------------------------------------------------
// lane -> pixel mapping: kG lanes per ray; a wave covers WX x WY pixels, a
// workgroup 2 x 2 waves = BX x BY pixels.
// --------------------------------------------------------------------------
// optional lower bound on resident waves per SIMD for the render kernels
// (caps their registers)
#ifdef VI_RENDER_WAVES
#define VI_RENDER_OCCUPANCY __attribute__((amdgpu_waves_per_eu(VI_RENDER_WAVES)))
#else
#define VI_RENDER_OCCUPANCY
#endif
#ifndef VI_RAY_LANES
#define VI_RAY_LANES 4
#endif
constexpr int kG = VI_RAY_LANES;  // lanes per ray: 1, 2, 4, 8 or 16
static_assert(kG == 1 || kG == 2 || kG == 4 || kG == 8 || kG == 16, "lanes per ray");
constexpr int kWX = (64 / kG) >= 32 ? 8 : 4, kWY = (64 / kG) / kWX;
constexpr int kBX = 2 * kWX, kBY = 2 * kWY;

__device__ __forceinline__ void block_pixel(uint32_t tx, uint32_t ty, int* px, int* py)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane / kG;
    *px = (int)tx * kBX + (wave & 1) * kWX + r % kWX;
    *py = (int)ty * kBY + (wave >> 1) * kWY + r / kWX;
}

// Segment counters: a wave sums its lanes' counts, the workgroup's waves add
// theirs in LDS, and the last wave to finish adds the workgroup's totals to
// the frame's counters -- one global atomic per workgroup and counter (one
// per wave measured up to twice the unlit frame's time: every wave of the
// frame hits the same two words).  No barrier: finished waves still leave.
struct GroupCount {
    unsigned long long ns, nop;
    uint32_t waves_done;
};
__device__ __forceinline__ void group_count_init(GroupCount* g)
{
    if (threadIdx.x == 0) {
        g->ns = 0;
        g->nop = 0;
        g->waves_done = 0;
    }
}
__device__ __forceinline__ void group_count_add(const RenderFrame& F, GroupCount* g, uint32_t ns, uint32_t nop)
{
    if (!F.samples) return;
    for (int off = 32; off > 0; off >>= 1) {
        ns += __shfl_xor(ns, off);
        nop += __shfl_xor(nop, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&g->ns, (unsigned long long)ns);
        atomicAdd(&g->nop, (unsigned long long)nop);
        __threadfence_block();
        if (atomicAdd(&g->waves_done, 1u) == blockDim.x / 64u - 1u) {
            const unsigned long long tn = atomicAdd(&g->ns, 0ull), to = atomicAdd(&g->nop, 0ull);
            if (tn) atomicAdd(F.samples, tn);
            if (to && F.count_opaque) atomicAdd(F.samples + 1, to);
        }
    }
}

template <typename VT, int LAYOUT, int MODE, int SDT, int SL>
__device__ __forceinline__ void shade_pixel(const RenderFrame& F, const float4* s_tf, const int* s_next,
                                            const uint32_t* s_bits, GroupCount* gc, int px, int py)
{
    uint32_t ns = 0, nop = 0;
    const int lane = threadIdx.x & 63;
    if (px < F.width && py < F.height) {
        const float4 c = render_ray<VT, LAYOUT, MODE, SDT, SL, kG>(F, s_tf, s_next, s_bits, px, py, ns, nop);
        if (lane % kG == 0) F.out[(size_t)py * F.width + px] = c;
    }
    group_count_add(F, gc, ns, nop);
}

// Ray compaction (VI_RENDER_COMPACT = 1): a wave owns four blocks of
// (64 / kG) rays and its groups take the next ray of the wave's list as they
// finish, a refill at a time once at least VI_COMPACT_REFILL groups are idle
// (a refill runs the set-up code for the whole wave, so one per finished
// ray would cost more than the idle lanes it saves).  The per-ray
// arithmetic is unchanged, so the image and counts are the same bits as
// with one block per wave.
#ifndef VI_RENDER_COMPACT
#define VI_RENDER_COMPACT 0
#endif
#ifndef VI_COMPACT_REFILL
#define VI_COMPACT_REFILL 8
#endif
constexpr bool kCompact = VI_RENDER_COMPACT != 0;

template <typename VT, int LAYOUT, int MODE, int SDT, int SL>
__device__ __forceinline__ void shade_region_compact(const RenderFrame& F, const float4* s_tf, const int* s_next,
                                                     const uint32_t* s_bits, GroupCount* gc, int x0, int y0)
{
    constexpr int kGroups = 64 / kG, kRays = 4 * kGroups;
    const int lane = threadIdx.x & 63, g = lane % kG, grp = lane / kG;
    RayState S;
    bool live = false;
    int px = 0, py = 0, next = 0;  // next: the wave's next ray (uniform)
    uint32_t ns = 0, nop = 0;
    for (;;) {
        const uint64_t idle = __ballot(!live && g == 0);
        const int nidle = __popcll(idle);
        if (next < kRays && (nidle >= VI_COMPACT_REFILL || nidle == kGroups)) {
            if (!live) {
                const int r = next + __popcll(idle & ((1ull << (grp * kG)) - 1ull));
                if (r < kRays) {
                    const int b = r / kGroups, i = r % kGroups;
                    px = x0 + (b & 1) * kWX + i % kWX;
                    py = y0 + (b >> 1) * kWY + i / kWX;
                    if (px < F.width && py < F.height) {
                        live = ray_setup<VT, LAYOUT, MODE, SDT, SL, kG>(F, px, py, S);
                        if (!live && g == 0)
                            F.out[(size_t)py * F.width + px] = make_float4(F.bg[0], F.bg[1], F.bg[2], F.bg[3]);
                    }
                }
            }
            next += nidle;
            continue;
        }
        if (nidle == kGroups) break;  // nothing live, nothing left
        if (live && ray_step<VT, LAYOUT, MODE, SDT, SL, kG>(F, s_tf, s_next, s_bits, S, nop)) {
            if (g == 0) {
                ns += (uint32_t)min(S.count, S.K);
                F.out[(size_t)py * F.width + px] = ray_result(F, S);
            }
            live = false;
        }
    }
    group_count_add(F, gc, ns, nop);
}

// --------------------------------------------------------------------------
// single-frame kernel
// --------------------------------------------------------------------------
template <typename VT, int LAYOUT, int MODE, int SDT, int SL>
__device__ __forceinline__ void render_frame(const RenderFrame& F)
{
    extern __shared__ float4 s_tf[];  // K entries, K next-opaque indices, then the occupancy bits
    int* s_next = (int*)(s_tf + F.K);
    uint32_t* s_bits = (uint32_t*)(s_next + F.K);
    __shared__ GroupCount gc;
    group_count_init(&gc);
    for (int t = threadIdx.x; t < F.K; t += blockDim.x)
        s_tf[t] = make_float4(F.tf[4 * t], F.tf[4 * t + 1], F.tf[4 * t + 2], F.tf[4 * t + 3]);
    if (F.occ.mm && !F.occ.bits) build_next_opaque(s_next, F.tf, F.K);
    stage_occupancy(F.occ, s_bits);
    __syncthreads();

    if constexpr (kCompact) {
        // workgroup tile of 2 x 2 waves, each 2 x 2 blocks of kWX x kWY pixels
        const uint32_t tiles_x = (F.width + 4 * kWX - 1) / (4 * kWX), tiles_y = (F.height + 4 * kWY - 1) / (4 * kWY);
        uint32_t tx, ty;
        if (!supertile_of(blockIdx.x, tiles_x, tiles_y, &tx, &ty)) return;
        const int wave = threadIdx.x >> 6;
        shade_region_compact<VT, LAYOUT, MODE, SDT, SL>(F, s_tf, s_next, s_bits, &gc,
                                                        (int)tx * 4 * kWX + (wave & 1) * 2 * kWX,
                                                        (int)ty * 4 * kWY + (wave >> 1) * 2 * kWY);
    } else {
        const uint32_t tiles_x = (F.width + kBX - 1) / kBX, tiles_y = (F.height + kBY - 1) / kBY;
        uint32_t tx, ty;
        if (!supertile_of(blockIdx.x, tiles_x, tiles_y, &tx, &ty)) return;
        int px, py;
        block_pixel(tx, ty, &px, &py);
        shade_pixel<VT, LAYOUT, MODE, SDT, SL>(F, s_tf, s_next, s_bits, &gc, px, py);
    }
}

// --------------------------------------------------------------------------
// batched kernel (serving): the launch lists 16 x 16-pixel tiles of any frames
// of one mode; each tile is covered by (16/BX) x (16/BY) workgroups, each
// reading its frame's parameters from device memory.  Per pixel it runs the
// same render_ray as render_kernel, so a frame is bit-identical alone and in a
// mix.  (One kernel per mode keeps each mode's register budget: a kernel
// holding every mode runs all of them at the occupancy of the largest.)
// --------------------------------------------------------------------------
constexpr uint32_t kSubX = 16 / kBX, kSubY = 16 / kBY, kSub = kSubX * kSubY;

template <typename VT, int LAYOUT, int MODE, int SDT, int SL>
__device__ __forceinline__ void render_tiles(const RenderFrame* __restrict__ frames, const uint32_t* __restrict__ tiles,
                                             uint32_t ntiles)
{
    extern __shared__ float4 s_tf[];
    uint32_t q;
    if (!list_of(blockIdx.x, ntiles * kSub, &q)) return;
    const uint32_t t = tiles[q / kSub], sub = q % kSub;
    const RenderFrame& F = frames[t >> 22];
    int* s_next = (int*)(s_tf + F.K);
    uint32_t* s_bits = (uint32_t*)(s_next + F.K);
    __shared__ GroupCount gc;
    group_count_init(&gc);
    for (int i = threadIdx.x; i < F.K; i += blockDim.x)
        s_tf[i] = make_float4(F.tf[4 * i], F.tf[4 * i + 1], F.tf[4 * i + 2], F.tf[4 * i + 3]);
    if (F.occ.mm && !F.occ.bits) build_next_opaque(s_next, F.tf, F.K);
    stage_occupancy(F.occ, s_bits);
    __syncthreads();
    int px, py;
    block_pixel((t & 2047u) * kSubX + sub % kSubX, ((t >> 11) & 2047u) * kSubY + sub / kSubX, &px, &py);
    shade_pixel<VT, LAYOUT, MODE, SDT, SL>(F, s_tf, s_next, s_bits, &gc, px, py);
}

// The kernels.  The float-stack shell's two-tap batches fit six waves per
// SIMD (at most 80 VGPRs, no spills), which measured faster than the five
// the compiler picks for them; the other cases keep the compiler's budget.
template <typename VT, int LAYOUT, int MODE, int SDT, int SL>
__global__ __launch_bounds__(256) VI_RENDER_OCCUPANCY void render_kernel(RenderFrame F)
{
    render_frame<VT, LAYOUT, MODE, SDT, SL>(F);
}
template <typename VT, int LAYOUT, int SDT, int SL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void render_kernel_shell(RenderFrame F)
{
    render_frame<VT, LAYOUT, VI_MODE_SHELL, SDT, SL>(F);
}
template <typename VT, int LAYOUT, int MODE, int SDT, int SL>
__global__ __launch_bounds__(256) VI_RENDER_OCCUPANCY void render_batch_kernel(const RenderFrame* __restrict__ frames,
                                                                               const uint32_t* __restrict__ tiles,
                                                                               uint32_t ntiles)
{
    render_tiles<VT, LAYOUT, MODE, SDT, SL>(frames, tiles, ntiles);
}
template <typename VT, int LAYOUT, int SDT, int SL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void render_batch_kernel_shell(
    const RenderFrame* __restrict__ frames, const uint32_t* __restrict__ tiles, uint32_t ntiles)
{
    render_tiles<VT, LAYOUT, VI_MODE_SHELL, SDT, SL>(frames, tiles, ntiles);
}

template <typename VT, int LAYOUT, int SDT, int SL>
static hipError_t launch_batch_t(int mode, const RenderFrame* d_frames, const uint32_t* d_tiles, uint32_t ntiles,
                                 int maxK, uint32_t occ_words, hipStream_t s)
{
    const size_t lds = (sizeof(float4) + sizeof(int)) * (size_t)maxK + sizeof(uint32_t) * (size_t)occ_words;
    const dim3 grid(list_grid(ntiles * kSub)), block(256);
    switch (mode) {
    case VI_MODE_NONE:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, VI_MODE_NONE, SDT, SL>), grid, block, lds, s, d_frames,
                           d_tiles, ntiles);
        break;
    case VI_MODE_SHADOW:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, VI_MODE_SHADOW, SDT, SL>), grid, block, lds, s, d_frames,
                           d_tiles, ntiles);
        break;
    case VI_MODE_SHELL:
        if constexpr (SDT == VI_F32)
            hipLaunchKernelGGL((render_batch_kernel_shell<VT, LAYOUT, SDT, SL>), grid, block, lds, s, d_frames,
                               d_tiles, ntiles);
        else
            hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, VI_MODE_SHELL, SDT, SL>), grid, block, lds, s,
                               d_frames, d_tiles, ntiles);
        break;
    case VI_MODE_CONE:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, VI_MODE_CONE, SDT, SL>), grid, block, lds, s, d_frames,
                           d_tiles, ntiles);
        break;
    case kModePointShadow:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, kModePointShadow, SDT, SL>), grid, block, lds, s,
                           d_frames, d_tiles, ntiles);
        break;
    case kModePointShell:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, kModePointShell, SDT, SL>), grid, block, lds, s,
                           d_frames, d_tiles, ntiles);
        break;
    case kModePointPhong:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, kModePointPhong, SDT, SL>), grid, block, lds, s,
                           d_frames, d_tiles, ntiles);
        break;
    case kModeConeGrid:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, kModeConeGrid, SDT, SL>), grid, block, lds, s,
                           d_frames, d_tiles, ntiles);
        break;
    case kModePointCone:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, kModePointCone, SDT, SL>), grid, block, lds, s,
                           d_frames, d_tiles, ntiles);
        break;
    default:
        hipLaunchKernelGGL((render_batch_kernel<VT, LAYOUT, VI_MODE_PHONG, SDT, SL>), grid, block, lds, s, d_frames,
                           d_tiles, ntiles);
        break;
    }
    return hipGetLastError();
}

template <typename VT, int LAYOUT>
static hipError_t launch_batch_l(int sdt, int sl, int mode, const RenderFrame* f, const uint32_t* t, uint32_t n,
                                 int K, uint32_t w, hipStream_t s)
{
    if (sdt == VI_BF16)
        return sl == VI_STACK_ROWS ? launch_batch_t<VT, LAYOUT, VI_BF16, VI_STACK_ROWS>(mode, f, t, n, K, w, s)
                                   : launch_batch_t<VT, LAYOUT, VI_BF16, VI_STACK_TILED>(mode, f, t, n, K, w, s);
    if (sdt == VI_F16)  // row layout only
        return launch_batch_t<VT, LAYOUT, VI_F16, VI_STACK_ROWS>(mode, f, t, n, K, w, s);
    return sl == VI_STACK_ROWS ? launch_batch_t<VT, LAYOUT, VI_F32, VI_STACK_ROWS>(mode, f, t, n, K, w, s)
                               : launch_batch_t<VT, LAYOUT, VI_F32, VI_STACK_TILED>(mode, f, t, n, K, w, s);
}

template <typename VT>
static hipError_t launch_batch_vt(int layout, int sdt, int sl, int mode, const RenderFrame* f, const uint32_t* t,
                                  uint32_t n, int K, uint32_t w, hipStream_t s)
{
    if (layout == VI_LAYOUT_QUAD4) return launch_batch_l<VT, VI_LAYOUT_QUAD4>(sdt, sl, mode, f, t, n, K, w, s);
    return layout == VI_LAYOUT_BRICK4 ? launch_batch_l<VT, VI_LAYOUT_BRICK4>(sdt, sl, mode, f, t, n, K, w, s)
                                      : launch_batch_l<VT, VI_LAYOUT_LINEAR>(sdt, sl, mode, f, t, n, K, w, s);
}

hipError_t launch_render_batch(int vol_dtype, int layout, int stack_dtype, int stack_layout, int mode,
                               const RenderFrame* d_frames, const uint32_t* d_tiles, uint32_t ntiles, int maxK,
                               uint32_t max_occ_words, hipStream_t s)
{
    const uint32_t w = max_occ_words;
    switch (vol_dtype) {
    case VI_U8: return launch_batch_vt<uint8_t>(layout, stack_dtype, stack_layout, mode, d_frames, d_tiles, ntiles, maxK, w, s);
    case VI_U16:
        return launch_batch_vt<uint16_t>(layout, stack_dtype, stack_layout, mode, d_frames, d_tiles, ntiles, maxK, w, s);
    case VI_F16:
        return launch_batch_vt<__half>(layout, stack_dtype, stack_layout, mode, d_frames, d_tiles, ntiles, maxK, w, s);
    default: return launch_batch_vt<float>(layout, stack_dtype, stack_layout, mode, d_frames, d_tiles, ntiles, maxK, w, s);
    }
}

template <typename VT, int LAYOUT, int SDT, int SL>
static hipError_t launch_mode(const RenderFrame& f, hipStream_t s)
{
    const uint32_t tw = kCompact ? 4 * kWX : kBX, th = kCompact ? 4 * kWY : kBY;
    dim3 grid(supertile_grid((f.width + tw - 1) / tw, (f.height + th - 1) / th)), block(256);
    const size_t lds =
        (sizeof(float4) + sizeof(int)) * (size_t)f.K + (f.occ.bits ? sizeof(uint32_t) * (f.occ.words + f.occ.swords) : 0);
    switch (kernel_mode(f)) {
    case VI_MODE_NONE:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, VI_MODE_NONE, SDT, SL>), grid, block, lds, s, f);
        break;
    case VI_MODE_SHADOW:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, VI_MODE_SHADOW, SDT, SL>), grid, block, lds, s, f);
        break;
    case VI_MODE_SHELL:
        if constexpr (SDT == VI_F32)
            hipLaunchKernelGGL((render_kernel_shell<VT, LAYOUT, SDT, SL>), grid, block, lds, s, f);
        else
            hipLaunchKernelGGL((render_kernel<VT, LAYOUT, VI_MODE_SHELL, SDT, SL>), grid, block, lds, s, f);
        break;
    case VI_MODE_CONE:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, VI_MODE_CONE, SDT, SL>), grid, block, lds, s, f);
        break;
    case kModePointShadow:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, kModePointShadow, SDT, SL>), grid, block, lds, s, f);
        break;
    case kModePointShell:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, kModePointShell, SDT, SL>), grid, block, lds, s, f);
        break;
    case kModePointPhong:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, kModePointPhong, SDT, SL>), grid, block, lds, s, f);
        break;
    case kModeConeGrid:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, kModeConeGrid, SDT, SL>), grid, block, lds, s, f);
        break;
    case kModePointCone:
        hipLaunchKernelGGL((render_kernel<VT, LAYOUT, kModePointCone, SDT, SL>), grid, block, lds, s, f);
        break;
    default: hipLaunchKernelGGL((render_kernel<VT, LAYOUT, VI_MODE_PHONG, SDT, SL>), grid, block, lds, s, f); break;
    }
    return hipGetLastError();
}

template <typename VT, int LAYOUT>
static hipError_t launch_sdt(const RenderFrame& f, hipStream_t s)
{
    const bool q = f.stack_layout == VI_STACK_ROWS;
    if (f.stack_dtype == VI_BF16)
        return q ? launch_mode<VT, LAYOUT, VI_BF16, VI_STACK_ROWS>(f, s) : launch_mode<VT, LAYOUT, VI_BF16, VI_STACK_TILED>(f, s);
    if (f.stack_dtype == VI_F16)  // row layout only
        return launch_mode<VT, LAYOUT, VI_F16, VI_STACK_ROWS>(f, s);
    return q ? launch_mode<VT, LAYOUT, VI_F32, VI_STACK_ROWS>(f, s) : launch_mode<VT, LAYOUT, VI_F32, VI_STACK_TILED>(f, s);
}

template <typename VT>
static hipError_t launch_vt(const RenderFrame& f, hipStream_t s)
{
    if (f.vol_layout == VI_LAYOUT_QUAD4) return launch_sdt<VT, VI_LAYOUT_QUAD4>(f, s);
    return f.vol_layout == VI_LAYOUT_BRICK4 ? launch_sdt<VT, VI_LAYOUT_BRICK4>(f, s)
                                            : launch_sdt<VT, VI_LAYOUT_LINEAR>(f, s);
}

hipError_t launch_render(const RenderFrame& f, hipStream_t s)
{
    switch (f.vol_dtype) {
    case VI_U8: return launch_vt<uint8_t>(f, s);
    case VI_U16: return launch_vt<uint16_t>(f, s);
    case VI_F16: return launch_vt<__half>(f, s);
    default: return launch_vt<float>(f, s);
    }
}

}  // namespace vi
