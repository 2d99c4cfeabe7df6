// vi_build.hip -- light-space attenuation build (section 3.2.1, Alg. 1).
//
// Every texel column of the light square is scanned over the n slabs from
// the light (Eq. 8 ordering): per slab the volume is sampled at the slab
// midpoint, the transfer-function opacity is looked up and corrected to the
// slab thickness (extinction form, Eq. 6), and the running transmittance is
// multiplied by (1 - alpha) -- Eq. 4 applied to opacity.  Every layer is
// written within a few slabs of being known (the row layout holds the layers
// of four slab pairs in LDS before storing them), so the pass is one
// streaming sweep: the volume is read through the caches and the stack is
// written once.
//
// Mapping: one workgroup per run of consecutive elements of a layer, one
// column per lane (in the tiled layout optionally C columns).  In the row
// layout a run is a stretch of the layer's element range, border included
// (build_rows); in the tiled layout a run of one stack row (build_tiled).
// At every slab a workgroup stores its run as one contiguous stretch of the
// layer (4 KiB for 1024 float texels); many short runs spread over the layer
// (64 x 4 texel tiles per workgroup) measured at half that write rate.  The
// 64 lanes of a wave hold 64 neighbouring columns (of at most two rows), so
// each volume gather of a wave stays compact.
//
// Per column the slabs whose midpoints lie in the cube form one interval
// [k_in, k_out], found once by exact integer division; a wave runs the full
// per-slab work (fetch, transfer function, Eq. 6 correction, product) only
// for slabs in its columns' union of intervals, and otherwise only stores
// (the unattenuated value in front, the final transmittance behind).
// Empty-space verdicts come from the occupancy bits in LDS (without bits
// every slab in the cube is fetched).
//
// Slab-midpoint positions are fixed-point numbers (h * 2^40 in an int64, h
// the offset-voxel coordinate), so stepping from slab to slab is an exact
// integer add and the voxel index and trilinear weight are exact bit fields
// of the position: no rounding accumulates over the 512 slabs, and a float
// would resolve |h| ~ N/2 only to 2^-16 voxel.
#include <algorithm>

#include "vi_device.h"
#include "vi_internal.h"

namespace vi {

// Workgroup b -> (row, run): rows (in the row layout, runs of about a row
// of the layer's element range) are dealt to the 8 XCDs in groups of 4
// consecutive ones (neighbouring rows sample the same voxels and share an
// L2), the groups of an XCD spread over the whole light square.
constexpr uint32_t kRowGroup = 4;
__device__ __forceinline__ bool row_run_of(uint32_t b, uint32_t rows, uint32_t runs, uint32_t* row, uint32_t* run)
{
    const uint32_t x = b % kXcds, q = b / kXcds;  // XCD, index within it
    const uint32_t unit = q / runs, r = q % runs;
    const uint32_t grp = unit / kRowGroup, within = unit % kRowGroup;
    *row = (grp * kXcds + x) * kRowGroup + within;
    *run = r;
    return *row < rows;
}
inline uint32_t row_run_grid(uint32_t rows, uint32_t runs)
{
    const uint32_t groups = (rows + kRowGroup - 1) / kRowGroup;
    return (groups + kXcds - 1) / kXcds * kRowGroup * runs * kXcds;
}

// Q40 positions: floor(h) and the trilinear weight h - floor(h) (its top 24
// bits, exact in a float).
__device__ __forceinline__ int q_floor(int64_t H) { return (int)(H >> kQBits); }
__device__ __forceinline__ float q_frac(int64_t H)
{
    return (float)((uint32_t)((uint64_t)H >> (kQBits - 24)) & 0xFFFFFFu) * (1.0f / 16777216.0f);
}
__device__ __forceinline__ float q_to_float(int64_t H) { return (float)H * (1.0f / 1099511627776.0f); }

// (NT, C, B): threads per workgroup, columns per lane, slabs per batch;
// a lane's C columns are NT apart (CONSEC = 0: each store instruction of a
// wave covers 64 neighbouring texels) or adjacent (CONSEC = 1: one
// C-element store per lane)
#ifndef VI_BUILD_NT
#define VI_BUILD_NT 1024
#endif
#ifndef VI_BUILD_C
#define VI_BUILD_C 1
#endif
#ifndef VI_BUILD_BATCH
#define VI_BUILD_BATCH 2
#endif
#ifndef VI_BUILD_CONSEC
#define VI_BUILD_CONSEC 0
#endif
// row layout: pairs of slabs per LDS exchange (one barrier each)
#ifndef VI_BUILD_EXCH
#define VI_BUILD_EXCH 4
#endif
constexpr int kBuildNT = VI_BUILD_NT, kBuildC = VI_BUILD_C, kBuildB = VI_BUILD_BATCH;
constexpr bool kBuildConsec = VI_BUILD_CONSEC != 0;
constexpr int kBuildExch = VI_BUILD_EXCH;
constexpr int kRowsX = 2;  // exchange rows per slab pair: both of its layers

// The slabs of a column whose midpoints lie in the cube: k in [k_in, k_out]
// (empty when k_in > k_out), exactly as the per-slab test lo <= h_k <= hi
// on all three axes decides it: per axis a half-line or interval of k from
// an exact integer division of Q40 values.
__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}
__device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }
__device__ __forceinline__ void slab_range(const int64_t H[3], const int64_t A[3], int n, int64_t lo, int64_t hi,
                                           int* k_in, int* k_out)
{
    int64_t kl = 0, kh = n - 1;
    for (int a = 0; a < 3; ++a) {
        if (A[a] == 0) {
            if (H[a] < lo || H[a] > hi) kl = n;  // never inside along this axis
        } else if (A[a] > 0) {
            kl = max(kl, ceil_div(lo - H[a], A[a]));
            kh = min(kh, floor_div(hi - H[a], A[a]));
        } else {
            kl = max(kl, ceil_div(hi - H[a], A[a]));
            kh = min(kh, floor_div(lo - H[a], A[a]));
        }
    }
    if (kl > kh) {
        *k_in = n;
        *k_out = -1;
    } else {
        *k_in = (int)kl;
        *k_out = (int)kh;
    }
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// One stack texel: transmittance (F32), optical depth in base-2 units
// -log2 T (BF16), or the transmittance 2^-tau of the float optical depth
// rounded to half precision (F16).
// (The stack is below 4 GiB: byte offsets in 32 bits, so a store takes the
// stack's base from scalar registers.)
template <int OUT_DTYPE>
__device__ __forceinline__ void put_texel(void* out, uint32_t at, float T, float tau)
{
    if (OUT_DTYPE == VI_F32) *(float*)((char*)out + (at << 2)) = T;
    else if (OUT_DTYPE == VI_BF16) *(uint16_t*)((char*)out + (at << 1)) = f32_to_bf16(tau);
    else *(__half*)((char*)out + (at << 1)) = __float2half_rn(fast_exp2(-tau));
}

// An empty statement that reads a fetched footprint's registers.  Placed
// after all loads of a pair of slabs, it is the one point where they must
// have arrived, so the compiler waits there once for all of them; without it
// the loads of a slab fetched only by some lanes left their registers pending
// across the loop's back edge, and the compiler waited for the first slab's
// loads before issuing the second slab's (8 % slower).
template <typename T>
__device__ __forceinline__ void keep_value(const T& x)
{
    if constexpr (sizeof(T) == 8) asm volatile("" ::"v"(__builtin_bit_cast(uint64_t, x)));
    else if constexpr (sizeof(T) == 4) asm volatile("" ::"v"(__builtin_bit_cast(uint32_t, x)));
    else if constexpr (sizeof(T) == 2) asm volatile("" ::"v"((uint32_t)__builtin_bit_cast(uint16_t, x)));
    else if constexpr (sizeof(T) == 1) asm volatile("" ::"v"((uint32_t)__builtin_bit_cast(uint8_t, x)));
    else {
        struct W { uint64_t lo, hi; };
        const W w = __builtin_bit_cast(W, x);
        asm volatile("" ::"v"(w.lo), "v"(w.hi));
    }
}
template <typename VT, int LAYOUT>
__device__ __forceinline__ void keep_foot(const RawFoot<VT, LAYOUT>& r)
{
    if constexpr (LAYOUT == VI_LAYOUT_QUAD4) {
        keep_value(r.a);
        keep_value(r.b);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) keep_value(r.v[i]);
    }
}

// Shared set-up of both layouts: the TF's opacities and the occupancy bits
// in LDS.  Empty-space verdicts come from the bits; without them one set bit
// stands for "every cell may hold opacity" (cell index 0).  Returns the
// number of 32-bit words the bits take.
__device__ __forceinline__ uint32_t stage_build_tables(const BuildParams& P, float* s_alpha, uint32_t* s_bits)
{
    for (int t = threadIdx.x; t < P.K; t += blockDim.x) s_alpha[t] = P.tf[4 * t + 3];
    if (P.occ.bits != nullptr) {
        stage_occupancy(P.occ, s_bits);
        return P.occ.words + P.occ.swords;
    }
    if (threadIdx.x == 0) s_bits[0] = 1u;
    return 1u;
}

// The slab-0 midpoint of column (i, j) and (point light) its step, in Q40,
// the step's length in voxels, and the column's slabs inside the cube.
template <bool PT>
__device__ __forceinline__ void column_setup(const BuildParams& P, int i, int j, bool grid, int64_t H[3], int64_t A[3],
                                             float* e, int* kin, int* kout)
{
    for (int a = 0; a < 3; ++a) H[a] = P.B0q[a] + (int64_t)i * P.BUq[a] + (int64_t)j * P.BVq[a];
    if constexpr (PT) {
        for (int a = 0; a < 3; ++a) A[a] = P.ALq[a] + (int64_t)i * P.ALUq[a] + (int64_t)j * P.ALVq[a];
        const float ax = q_to_float(A[0]), ay = q_to_float(A[1]), az = q_to_float(A[2]);
        *e = sqrtf(fmaf(ax, ax, fmaf(ay, ay, az * az)));
    } else {
        for (int a = 0; a < 3; ++a) A[a] = P.ALq[a];
        *e = P.e;
    }
    if (grid) {
        slab_range(H, A, P.n, P.loq, P.hiq, kin, kout);
    } else {
        *kin = P.n;  // border, padding or past the grid: no slab
        *kout = -1;
    }
}

// A slab midpoint in Q40: its footprint's lower voxel, trilinear weights and
// whether it must be fetched (slab k inside the column's cube interval and
// its cell possibly opaque; a zero-opacity cell leaves T unchanged exactly).
struct SlabProbe {
    int gx, gy, gz;
    float wx, wy, wz;
    bool fetch;
};
__device__ __forceinline__ SlabProbe probe_slab(const BuildParams& P, int64_t hx, int64_t hy, int64_t hz, int k, int kin,
                                                int kout, const uint32_t* s_bits, int cshift, uint32_t cnc)
{
    SlabProbe s;
    s.gx = q_floor(hx) + P.M;
    s.gy = q_floor(hy) + P.M;
    s.gz = q_floor(hz) + P.M;
    s.wx = q_frac(hx);
    s.wy = q_frac(hy);
    s.wz = q_frac(hz);
    const uint32_t cell = cell_of(s.gx, s.gy, s.gz, P.N, cshift, cnc);
    s.fetch = k >= kin && k <= kout && occupancy_bit(s_bits, cell);
    return s;
}

// One slab of a column (Alg. 1): the volume value at the slab midpoint, the
// TF opacity clamped to [0, 1] as the render clamps it, corrected to the
// slab thickness (Eq. 6, extinction form: e = ds / dref), applied to the
// transmittance T (F32) or added to the optical depth tau in base-2 units
// (2-byte stacks).  `darken` applies the section 4 compensation
// (1 + alpha)^m; m = 0 leaves every factor unchanged exactly.
template <typename VT, int LAYOUT, int OUT_DTYPE>
__device__ __forceinline__ void slab_step(const BuildParams& P, const float* s_alpha, const RawFoot<VT, LAYOUT>& raw,
                                          const SlabProbe& s, float e, bool darken, float& T, float& tau)
{
    const float v = foot_value<VT, LAYOUT>(raw, s.wx, s.wy, s.wz, P.scale);
    const float x = v * (float)(P.K - 1);
    const int e0 = min((int)x, P.K - 2);
    const float w = x - (float)e0;
    const float a = clampf01(fmaf(w, s_alpha[e0 + 1] - s_alpha[e0], s_alpha[e0]));
    const float l2 = fast_log2(1.0f - a);  // -inf for a = 1
    if (OUT_DTYPE == VI_F32) {
        // (1 - alpha(ds)) = (1 - a)^(ds / dref) = 2^(e log2(1 - a))
        float f = fast_exp2(e * l2);
        // section 4 compensation: times (1 + alpha)^m, at most 1
        if (darken) f = fminf(f * fast_exp2(P.darken * fast_log2(2.0f - f)), 1.0f);
        T *= f;
    } else {
        // optical depth in base-2 units: sigma ds / ln 2 = -e log2(1 - a),
        // capped at 64 / ln 2 per slab (a factor e^-64); the compensation
        // subtracts m log2(1 + alpha), floored at 0
        float dtau = -e * l2;
        if (darken) dtau = fmaxf(dtau - P.darken * fast_log2(2.0f - fast_exp2(e * l2)), 0.0f);
        tau += fminf(dtau, 92.332482616893656f);
    }
}

// Tiled layout: one workgroup per run of NT * C texels of one stack row,
// lane l owning columns l, l + NT, ..., l + NT (C - 1) of the run (or C
// adjacent ones).  Slabs in front of a wave's columns' union of cube
// intervals and behind it are stored without touching the volume; inside,
// batches of B slabs: positions and empty-space verdicts, then every volume
// load of the batch, and only then the arithmetic and the stores -- one
// wait per batch, with C * B footprints in flight.
template <typename VT, int LAYOUT, int OUT_DTYPE, bool PT>
__device__ __forceinline__ void build_tiled(const BuildParams& P)
{
    constexpr int NT = kBuildNT, C = kBuildC, B = kBuildB;
    constexpr int CS = kBuildConsec ? 1 : NT;  // stride between a lane's columns
    extern __shared__ float s_alpha[];  // K alphas, then the occupancy bits
    uint32_t* s_bits = (uint32_t*)(s_alpha + P.K);
    stage_build_tables(P, s_alpha, s_bits);
    const bool use_bits = P.occ.bits != nullptr;
    const int cshift = use_bits ? P.occ.shift : 30;
    const uint32_t cnc = use_bits ? P.occ.nc : 1u;
    __syncthreads();

    const uint32_t runs = ((uint32_t)P.res + NT * C - 1) / (NT * C);
    uint32_t row, run;
    if (!row_run_of(blockIdx.x, (uint32_t)P.res, runs, &row, &run)) return;
    const int i0 = (int)(run * NT * C) + (kBuildConsec ? C * (int)threadIdx.x : (int)threadIdx.x);
    const int j = (int)row;

    int64_t H[C][3], A[C][3];
    float ex[C];
    int kin[C], kout[C];
    bool col[C];
    uint32_t at[C];
    int kmin = P.n, kmax = -1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int i = i0 + CS * c;
        col[c] = i < P.res;
        column_setup<PT>(P, i, j, col[c], H[c], A[c], &ex[c], &kin[c], &kout[c]);
        at[c] = stack_oj(j, P.row_tiles32) + stack_oi(i);
        kmin = min(kmin, kin[c]);
        kmax = max(kmax, kout[c]);
    }
    // the wave's slabs with any midpoint in the cube: [kmin, kmax]
    kmin = __builtin_amdgcn_readfirstlane(wave_min(kmin));
    kmax = __builtin_amdgcn_readfirstlane(wave_max(kmax));
    const uint32_t layer = P.layer;

    // slabs in front of the cube: the light arrives unattenuated
    for (int k = 0; k < min(kmin, P.n); ++k)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (col[c]) put_texel<OUT_DTYPE>(P.out, at[c], 1.0f, 0.0f);
            at[c] += layer;
        }

    const VT* __restrict__ vol = (const VT*)P.vol;
    const VolIndex VI_ = {1u, P.vsy, P.vsz};
    float T[C], tau[C];
    const int kstart = kmin < P.n ? kmin : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T[c] = 1.0f, tau[c] = 0.0f;
        for (int a = 0; a < 3; ++a) H[c][a] += (int64_t)kstart * A[c][a];  // positions at slab kmin
    }
    const bool darken = P.darken > 0.0f;

    for (int k0 = kmin; k0 <= kmax; k0 += B) {
        SlabProbe sp[C][B];
        RawFoot<VT, LAYOUT> raw[C][B];
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
            for (int u = 0; u < B; ++u)
                sp[c][u] = probe_slab(P, H[c][0] + (int64_t)u * A[c][0], H[c][1] + (int64_t)u * A[c][1],
                                      H[c][2] + (int64_t)u * A[c][2], k0 + u, kin[c], kout[c], s_bits, cshift, cnc);
            for (int a = 0; a < 3; ++a) H[c][a] += (int64_t)B * A[c][a];
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (sp[c][u].fetch)
                    foot_load_g<VT, LAYOUT>(raw[c][u], sp[c][u].wx, sp[c][u].wy, vol, VI_, P.N, sp[c][u].gx,
                                            sp[c][u].gy, sp[c][u].gz);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (k0 + u > kmax) break;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (sp[c][u].fetch) slab_step<VT, LAYOUT, OUT_DTYPE>(P, s_alpha, raw[c][u], sp[c][u], ex[c], darken,
                                                                     T[c], tau[c]);
                if (col[c]) put_texel<OUT_DTYPE>(P.out, at[c], T[c], tau[c]);
                at[c] += layer;
            }
        }
    }

    // slabs behind the cube: the transmittance stays as it left the cube
    for (int k = max(kmax + 1, kmin < P.n ? kmin : P.n); k < P.n; ++k)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (col[c]) put_texel<OUT_DTYPE>(P.out, at[c], T[c], tau[c]);
            at[c] += layer;
        }
}

// Row layout.  A layer, border and padding included, is one run of LS
// elements, LS times the element size an odd multiple of 64 bytes: the same
// texel of two neighbouring layers lies half a 128-byte line apart, as the
// render's lookups need (the lanes of a ray group read neighbouring layers
// at one texel position in the same load instruction; a whole-line layer
// stride made those reads collide in the L1 tags, 6-8 % slower frames).  In
// a buffer aligned to 128 bytes layers -1, 1, 3, ... then start on a line
// and layers 0, 2, 4, ... half a line past one.
//
// The workgroup owns NT consecutive elements of a layer's run, one column
// per lane, in every layer from the leading layer -1 to the trailing layer n
// (a copy of layer n - 1); border and padding lanes store the fully
// transmitting value without touching the volume.  It walks the slabs two at a time, in step
// across the workgroup: layer k0 + 1 (on the line grid) is stored by the
// lane that owns each element, layer k0 (half a line off) goes through LDS
// rotated by half a line, so that every wave's store there starts on a line
// too; only the two half-lines at the ends of the workgroup's run are
// written in part.  (Stores straddling lines measured at half the write
// rate.)  Both layers of E pairs wait in LDS for one barrier, which every
// wave reaches the same number of times, and all their stores go out after
// it (E = 4: a barrier per pair held the 2-byte stacks 8 % back): CDNA
// counts loads and stores on one counter, so a wait for a pair's loads also
// waits for every store issued before them, and with no store between the
// batch's loads only its first pair pays for the previous batch's stores
// (float 0.76 -> 0.73 ms together with the single wait per pair below).  A
// wave with no slab inside the cube in a pair only stores.  (Issuing the
// next pair's loads before this pair's stores measured 6-13 % slower: the
// compiler then waited for every load at each pair.)
template <typename VT, int LAYOUT, int OUT_DTYPE, bool PT>
__device__ __forceinline__ void build_rows(const BuildParams& P)
{
    static_assert(kBuildC == 1 && !kBuildConsec, "the row-layout build runs one column per lane");
    constexpr uint32_t NT = kBuildNT;
    constexpr uint32_t HALF = OUT_DTYPE == VI_F32 ? 16u : 32u;  // half a 128-byte line, in elements
    extern __shared__ float s_alpha[];  // K alphas, the occupancy bits, then two sets of 2E exchange rows of NT
    uint32_t* s_bits = (uint32_t*)(s_alpha + P.K);
    float* s_x = (float*)(s_bits + stage_build_tables(P, s_alpha, s_bits));
    const bool use_bits = P.occ.bits != nullptr;
    const int cshift = use_bits ? P.occ.shift : 30;
    const uint32_t cnc = use_bits ? P.occ.nc : 1u;
    __syncthreads();

    const uint32_t span = P.rlayer;
    uint32_t unit, one;
    if (!row_run_of(blockIdx.x, (span + NT - 1) / NT, 1u, &unit, &one)) return;  // uniform per workgroup
    const uint32_t t = threadIdx.x, f = unit * NT + t;
    // in layers half a line off, lane t stores the element of lane tr
    const uint32_t tr = (t + HALF) % NT, fr = unit * NT + tr;
    const int i = (int)(f % P.rpitch) - 2, j = (int)(f / P.rpitch) - 2;
    const bool col = f < span, col_r = fr < span;
    const bool grid = col && i >= 0 && i < P.res && j >= 0 && j < P.res;

    int64_t H[3], A[3];
    float ex;
    int kin, kout;
    column_setup<PT>(P, i, j, grid, H, A, &ex, &kin, &kout);
    // the wave's slabs with any midpoint in the cube: [kmin, kmax]
    const int kmin = __builtin_amdgcn_readfirstlane(wave_min(kin));
    const int kmax = __builtin_amdgcn_readfirstlane(wave_max(kout));
    const uint32_t layer = P.rlayer;
    uint32_t at = layer + f, at_r = layer + fr;  // elements of layer 0

    // the leading layer -1 (face 0) transmits fully
    if (col) put_texel<OUT_DTYPE>(P.out, f, 1.0f, 0.0f);

    const VT* __restrict__ vol = (const VT*)P.vol;
    const VolIndex VI_ = {1u, P.vsy, P.vsz};
    const bool darken = P.darken > 0.0f;
    float T = 1.0f, tau = 0.0f;  // transmittance (float stack), optical depth (2-byte stacks)
    // E pairs of slabs per exchange: their layers wait in 2E LDS rows and
    // are stored after one barrier (two sets of rows in turn, so that one
    // barrier per E pairs keeps writes and reads apart)
    constexpr int E = kBuildExch;
    for (int k0 = 0; k0 < P.n; k0 += 2 * E) {
        float* xs = s_x + ((uint32_t)(k0 / (2 * E)) & 1u) * (kRowsX * E * NT);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int kk = k0 + 2 * e;  // this pair: layers kk (half a line off) and kk + 1
            if (kk >= P.n) break;       // uniform
            float v0;                   // the value of layer kk: T or tau
            if (kk + 1 >= kmin && kk <= kmax) {  // uniform per wave
                SlabProbe sp[2];
                RawFoot<VT, LAYOUT> raw[2];
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    sp[u] = probe_slab(P, H[0] + (int64_t)u * A[0], H[1] + (int64_t)u * A[1],
                                       H[2] + (int64_t)u * A[2], kk + u, kin, kout, s_bits, cshift, cnc);
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (sp[u].fetch)
                        foot_load_g<VT, LAYOUT>(raw[u], sp[u].wx, sp[u].wy, vol, VI_, P.N, sp[u].gx, sp[u].gy,
                                                sp[u].gz);
                keep_foot<VT, LAYOUT>(raw[0]);
                keep_foot<VT, LAYOUT>(raw[1]);
                if (sp[0].fetch) slab_step<VT, LAYOUT, OUT_DTYPE>(P, s_alpha, raw[0], sp[0], ex, darken, T, tau);
                v0 = OUT_DTYPE == VI_F32 ? T : tau;
                if (sp[1].fetch) slab_step<VT, LAYOUT, OUT_DTYPE>(P, s_alpha, raw[1], sp[1], ex, darken, T, tau);
            } else {
                v0 = OUT_DTYPE == VI_F32 ? T : tau;
            }
            for (int a = 0; a < 3; ++a) H[a] += 2 * A[a];
            xs[e * NT + t] = v0;                                 // layer kk
            xs[(E + e) * NT + t] = OUT_DTYPE == VI_F32 ? T : tau;  // layer kk + 1
        }
        __syncthreads();
        // the layers half a line off, rotated by half a line
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (k0 + 2 * e >= P.n) break;  // uniform
            const float w = xs[e * NT + tr];
            if (col_r) put_texel<OUT_DTYPE>(P.out, at_r, w, w);
            at_r += 2 * layer;
            // layer kk + 1, on the line grid: each lane its own element
            const float o = xs[(E + e) * NT + t];
            if (k0 + 2 * e + 1 < P.n && col) put_texel<OUT_DTYPE>(P.out, at + layer, o, o);
            at += 2 * layer;
        }
    }
    // the trailing layer n repeats layer n - 1
    if (col) put_texel<OUT_DTYPE>(P.out, (uint32_t)(P.n + 1) * layer + f, T, tau);
}

template <typename VT, int LAYOUT, int OUT_DTYPE, int SL, bool PT>
__global__ __launch_bounds__(kBuildNT) void build_kernel(BuildParams P)
{
    if constexpr (SL == VI_STACK_ROWS) build_rows<VT, LAYOUT, OUT_DTYPE, PT>(P);
    else build_tiled<VT, LAYOUT, OUT_DTYPE, PT>(P);
}

template <typename VT, int LAYOUT, int SL, bool PT>
static void launch_build_k(const BuildParams& p, dim3 grid, size_t lds, hipStream_t s)
{
    if (p.out_dtype == VI_F32)
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F32, SL, PT>), grid, dim3(kBuildNT), lds, s, p);
    else if (p.out_dtype == VI_BF16)
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_BF16, SL, PT>), grid, dim3(kBuildNT), lds, s, p);
    else if constexpr (SL == VI_STACK_ROWS)
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F16, SL, PT>), grid, dim3(kBuildNT), lds, s, p);
}

template <typename VT, int LAYOUT>
static hipError_t launch_build_t(const BuildParams& p, hipStream_t s)
{
    constexpr uint32_t per_group = (uint32_t)kBuildNT * kBuildC;
    // (at least one word of bits: without them word 0 says "occupied")
    const size_t lds = sizeof(float) * (size_t)p.K + sizeof(uint32_t) * std::max(p.occ.words + p.occ.swords, 1u);
    if (p.out_layout == VI_STACK_ROWS) {
        // runs of a layer's element range, border and padding included; two
        // sets of exchange rows of floats
        const dim3 grid(row_run_grid((p.rlayer + per_group - 1) / per_group, 1u));
        const size_t lds_rows = lds + 2 * sizeof(float) * (size_t)kRowsX * kBuildExch * kBuildNT;
        if (p.point) launch_build_k<VT, LAYOUT, VI_STACK_ROWS, true>(p, grid, lds_rows, s);
        else launch_build_k<VT, LAYOUT, VI_STACK_ROWS, false>(p, grid, lds_rows, s);
    } else {
        const uint32_t runs = ((uint32_t)p.res + per_group - 1) / per_group;
        const dim3 grid(row_run_grid((uint32_t)p.res, runs));
        if (p.point) launch_build_k<VT, LAYOUT, VI_STACK_TILED, true>(p, grid, lds, s);
        else launch_build_k<VT, LAYOUT, VI_STACK_TILED, false>(p, grid, lds, s);
    }
    return hipGetLastError();
}

template <typename VT>
static hipError_t launch_build_l(const BuildParams& p, hipStream_t s)
{
    if (p.vol_layout == VI_LAYOUT_QUAD4) return launch_build_t<VT, VI_LAYOUT_QUAD4>(p, s);
    return p.vol_layout == VI_LAYOUT_BRICK4 ? launch_build_t<VT, VI_LAYOUT_BRICK4>(p, s)
                                            : launch_build_t<VT, VI_LAYOUT_LINEAR>(p, s);
}

hipError_t launch_build(const BuildParams& p, hipStream_t s)
{
    switch (p.vol_dtype) {
    case VI_U8: return launch_build_l<uint8_t>(p, s);
    case VI_U16: return launch_build_l<uint16_t>(p, s);
    case VI_F16: return launch_build_l<__half>(p, s);
    default: return launch_build_l<float>(p, s);
    }
}

}  // namespace vi
