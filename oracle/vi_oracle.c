/*
 * vi_oracle.c -- FP64 CPU oracle for slice-based ray-casting volume
 * illumination (Luo, arXiv 2008.06134).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Independent of
 * the HIP library: no shared code, headers or tables.
 *
 * Each function follows one step of the method and says which passage of
 * the paper it states.  Where the paper is silent the reading used is named
 * (R-numbers, listed with reasons in the design notes).  No blocking, fusion
 * or reordering: every quantity is evaluated from its definition.
 *
 * Parity-pin status: every function here is pinned by the CPU tests
 * (closed forms, special cases, invariants, brute force against an
 * independent NumPy statement).  Not pinned ("parity unpinned"): agreement
 * with the intent of the paper's shell/cone figures, whose images are not
 * available.
 */
#include "vi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <sched.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define VIO_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

int vio_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void vio_default_opts(vio_opts* o)
{
    /* Defaults of the readings: no ambient term and a white light (R16,
     * R17), transparent black background (R23), termination threshold 2^-15
     * (R20), one shell at one voxel with six taps (section 3.2.3, R13), a
     * two-ring, four-angle cone with a 45 degree half-angle (section 3.2.3,
     * R14). */
    o->ambient = 0.0;
    o->light_rgb[0] = o->light_rgb[1] = o->light_rgb[2] = 1.0;
    o->bg[0] = o->bg[1] = o->bg[2] = o->bg[3] = 0.0;
    o->term_eps = ldexp(1.0, -15);
    o->shell_count = 1;
    o->shell_h_vox = 1.0;
    o->cone_rings = 2;
    o->cone_angles = 4;
    o->cone_grid = 0;
    o->cone_tan = 1.0;
    /* the local-illumination comparison mode (section 4, Fig. 7 (b)):
     * readings R29-R32 */
    o->phong_ka = 0.1;
    o->phong_kd = 0.9;
    o->phong_ks = 0.4;
    o->phong_shininess = 20.0;
    o->grad_eps = 0.02;
    /* continuous depth (R11); the nearest-layer reading R25 is an option */
    o->nearest_layer = 0;
    o->nearest_shift = 0.0;
}

/* ------------------------------------------------------------------ */
/* Light frame: Eq. 8 (min/max of L.V[i] over the cube vertices, slab    */
/* increment (max-min)/n) and Eq. 10 (light view/projection), readings  */
/* R4 (L is the propagation direction), R9 (orthographic light square of */
/* half-width sqrt(3)/2 about the cube centre), R10 (basis choice).      */
/* ------------------------------------------------------------------ */
/* R10: seed the plane basis with the coordinate axis least aligned with
 * L (ties to the lowest index), Gram-Schmidt it against L. */
static void plane_basis(vio_frame* f)
{
    int js = 0;
    for (int a = 1; a < 3; ++a)
        if (fabs(f->L[a]) < fabs(f->L[js])) js = a;
    double e[3] = {0.0, 0.0, 0.0};
    e[js] = 1.0;
    double el = dot3(e, f->L);
    double u[3] = {e[0] - el * f->L[0], e[1] - el * f->L[1], e[2] - el * f->L[2]};
    double nu = norm3(u);
    for (int a = 0; a < 3; ++a) f->U[a] = u[a] / nu;
    cross3(f->L, f->U, f->V);
}

int vio_light_frame(const double l[3], int n, int res, vio_frame* f)
{
    double nl = norm3(l);
    if (!(nl > 0.0) || !isfinite(nl) || n < 1 || res < 1) return -1;
    for (int a = 0; a < 3; ++a) f->L[a] = l[a] / nl;
    f->c[0] = f->c[1] = f->c[2] = 0.5;
    f->darken = 0.0;
    f->positional = 0;
    f->P[0] = f->P[1] = f->P[2] = 0.0;

    /* Eq. 8: distances of the eight unit-cube vertices along L */
    f->dmin = INFINITY;
    f->dmax = -INFINITY;
    for (int vtx = 0; vtx < 8; ++vtx) {
        double V[3] = {(double)(vtx & 1), (double)((vtx >> 1) & 1), (double)((vtx >> 2) & 1)};
        double d = dot3(f->L, V);
        if (d < f->dmin) f->dmin = d;
        if (d > f->dmax) f->dmax = d;
    }
    f->n = n;
    f->res = res;
    f->ds = (f->dmax - f->dmin) / n;

    plane_basis(f);

    /* R9: the square [-R,R]^2 in the (U,V) plane covers the cube for any L */
    f->R = sqrt(3.0) / 2.0;
    return 0;
}

/* Point light (R34-R36): the light's view looks from P at the cube centre
 * (axis L = (c - P)/|c - P|); slabs are planes of constant depth
 * d = L.(p - P) between the nearest and farthest cube vertices (Eq. 8 with
 * distances measured from the light); the light projection is the
 * perspective one onto the plane d = 1, whose square [-R,R]^2 is the
 * smallest that holds every cube vertex's projection. */
int vio_light_frame_point(const double pos[3], int n, int res, vio_frame* f)
{
    if (!isfinite(pos[0]) || !isfinite(pos[1]) || !isfinite(pos[2]) || n < 1 || res < 1) return -1;
    f->c[0] = f->c[1] = f->c[2] = 0.5;
    double w[3] = {f->c[0] - pos[0], f->c[1] - pos[1], f->c[2] - pos[2]};
    double nw = norm3(w);
    if (!(nw > 0.5 * sqrt(3.0) * 1.0001)) return -1; /* inside the circumscribed sphere */
    for (int a = 0; a < 3; ++a) {
        f->L[a] = w[a] / nw;
        f->P[a] = pos[a];
    }
    f->darken = 0.0;
    f->positional = 1;
    plane_basis(f);
    f->dmin = INFINITY;
    f->dmax = -INFINITY;
    f->R = 0.0;
    for (int vtx = 0; vtx < 8; ++vtx) {
        double V[3] = {(double)(vtx & 1) - pos[0], (double)((vtx >> 1) & 1) - pos[1], (double)((vtx >> 2) & 1) - pos[2]};
        double d = dot3(f->L, V);
        if (d < f->dmin) f->dmin = d;
        if (d > f->dmax) f->dmax = d;
        double u = fabs(dot3(f->U, V)) / d, v = fabs(dot3(f->V, V)) / d;
        if (u > f->R) f->R = u;
        if (v > f->R) f->R = v;
    }
    f->n = n;
    f->res = res;
    f->ds = (f->dmax - f->dmin) / n;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Volume sampling (section 3: the volume as a 3D texture), readings R1, */
/* R2 (texel-centre convention, trilinear, clamp to edge), R22           */
/* (normalisation, clamped per voxel before interpolation).             */
/* ------------------------------------------------------------------ */
static double half_bits_to_double(uint16_t h)
{
    int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(m + 1024), e - 25);
    return s ? -v : v;
}

static double voxel(const vio_volume* v, int x, int y, int z)
{
    size_t N = (size_t)v->N;
    size_t idx = ((size_t)z * N + (size_t)y) * N + (size_t)x;
    double raw;
    switch (v->dtype) {
    case VIO_U8: raw = ((const uint8_t*)v->data)[idx]; break;
    case VIO_U16: raw = ((const uint16_t*)v->data)[idx]; break;
    case VIO_F16: raw = half_bits_to_double(((const uint16_t*)v->data)[idx]); break;
    default: raw = ((const float*)v->data)[idx]; break;
    }
    double s = raw * v->scale;
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    return s;
}

static int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

double vio_volume_sample(const vio_volume* v, const double p[3])
{
    int N = v->N;
    int i0[3], i1[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        double g = p[a] * N - 0.5; /* continuous voxel index */
        double fl = floor(g);
        w[a] = g - fl;
        i0[a] = clampi((int)fl, 0, N - 1);
        i1[a] = clampi((int)fl + 1, 0, N - 1);
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
                acc += wt * voxel(v, dx ? i1[0] : i0[0], dy ? i1[1] : i0[1], dz ? i1[2] : i0[2]);
            }
    return acc;
}

/* Transfer function (section 3.1.1: colour C_i and opacity A_i assigned to
 * the data value), reading R21: linear lookup at x = value * (K-1). */
void vio_tf_lookup(const vio_tf* tf, double value, double rgba[4])
{
    double x = value * (tf->K - 1);
    int i = (int)floor(x);
    if (i > tf->K - 2) i = tf->K - 2;
    if (i < 0) i = 0;
    double w = x - i;
    for (int c = 0; c < 4; ++c) rgba[c] = (1.0 - w) * tf->rgba[4 * i + c] + w * tf->rgba[4 * (i + 1) + c];
}

/* Opacity of a segment of length len (Eq. 6: extinction exp(-sum dt tau)),
 * reading R8: the table alpha a is the opacity of one reference length dref,
 * so the extinction is sigma = -ln(1-a)/dref and the segment opacity is
 * 1 - exp(-sigma len) = 1 - (1-a)^(len/dref). */
double vio_segment_alpha(double a, double len, double dref)
{
    if (!(len > 0.0) || !(a > 0.0)) return 0.0;
    if (a >= 1.0) return 1.0;
    return 1.0 - pow(1.0 - a, len / dref);
}

/* ------------------------------------------------------------------ */
/* Attenuation build: Alg. 1 with Eq. 4 blending, readings R3 (outside  */
/* the cube is empty), R5 (slabs of thickness ds from dmin, sampled at  */
/* their midpoints), R6 (one channel, the transmittance product), R7     */
/* (layer k holds the transmittance after slab k).                        */
/* ------------------------------------------------------------------ */
static int inside_cube(const double p[3])
{
    return p[0] >= 0.0 && p[0] <= 1.0 && p[1] >= 0.0 && p[1] <= 1.0 && p[2] >= 0.0 && p[2] <= 1.0;
}

void vio_build_column(const vio_volume* v, const vio_tf* tf, const vio_frame* f, int i, int j, double* col)
{
    double dref = 1.0 / v->N;
    double ui = -f->R + (i + 0.5) * (2.0 * f->R / f->res); /* texel centre, R9 */
    double vj = -f->R + (j + 0.5) * (2.0 * f->R / f->res);
    double Lc = dot3(f->L, f->c);
    /* point light (R37): the column is the ray from P through the texel
     * (u, v) of the unit-depth plane, D = L + u U + v V (L.D = 1); it meets
     * the mid-plane of slab k at P + d_k D and crosses the slab over a
     * length ds |D| */
    double D[3], seg = f->ds;
    for (int a = 0; a < 3; ++a) D[a] = f->L[a] + ui * f->U[a] + vj * f->V[a];
    if (f->positional) seg = f->ds * norm3(D);
    double T = 1.0;
    for (int k = 0; k < f->n; ++k) {
        double dk = f->dmin + (k + 0.5) * f->ds;
        double p[3];
        for (int a = 0; a < 3; ++a)
            p[a] = f->positional ? f->P[a] + dk * D[a] : f->c[a] + ui * f->U[a] + vj * f->V[a] + (dk - Lc) * f->L[a];
        double alpha = 0.0;
        if (inside_cube(p)) {
            double rgba[4];
            vio_tf_lookup(tf, vio_volume_sample(v, p), rgba);
            alpha = vio_segment_alpha(rgba[3], seg, dref);
        }
        /* Eq. 4 on opacity: (1-a_dst)(1-a_src) is what stays transmitted;
         * with the section 4 compensation every slab's factor is also
         * multiplied by (1+alpha)^m, capped at 1 so that no slab adds
         * light (R24) */
        double f_slab = 1.0 - alpha;
        if (f->darken > 0.0) {
            f_slab *= pow(1.0 + alpha, f->darken);
            if (f_slab > 1.0) f_slab = 1.0;
        }
        T = T * f_slab;
        col[k] = T;
    }
}

struct vio_stack {
    vio_volume vol;
    vio_tf tf;
    vio_frame f;
    double* data;           /* column-major [j][i][k] */
    unsigned char* state;   /* 0 empty, 1 being built, 2 ready */
    int64_t built;
};

vio_stack* vio_stack_create(const vio_volume* v, const vio_tf* tf, const vio_frame* f)
{
    vio_stack* s = (vio_stack*)calloc(1, sizeof(vio_stack));
    if (!s) return NULL;
    s->vol = *v;
    s->tf = *tf;
    s->f = *f;
    size_t cols = (size_t)f->res * (size_t)f->res;
    s->data = (double*)calloc(cols * (size_t)f->n, sizeof(double));
    s->state = (unsigned char*)calloc(cols, 1);
    if (!s->data || !s->state) {
        free(s->data);
        free(s->state);
        free(s);
        return NULL;
    }
    return s;
}

void vio_stack_destroy(vio_stack* s)
{
    if (!s) return;
    free(s->data);
    free(s->state);
    free(s);
}

const double* vio_stack_column(vio_stack* s, int i, int j)
{
    size_t c = (size_t)j * s->f.res + (size_t)i;
    double* col = s->data + c * (size_t)s->f.n;
    unsigned char st = __atomic_load_n(&s->state[c], __ATOMIC_ACQUIRE);
    if (st == 2) return col;
    unsigned char expect = 0;
    if (__atomic_compare_exchange_n(&s->state[c], &expect, 1, 0, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) {
        vio_build_column(&s->vol, &s->tf, &s->f, i, j, col);
        __atomic_fetch_add(&s->built, 1, __ATOMIC_RELAXED);
        __atomic_store_n(&s->state[c], 2, __ATOMIC_RELEASE);
        return col;
    }
    while (__atomic_load_n(&s->state[c], __ATOMIC_ACQUIRE) != 2) sched_yield();
    return col;
}

int64_t vio_stack_columns_built(const vio_stack* s) { return __atomic_load_n(&s->built, __ATOMIC_RELAXED); }

void vio_stack_fill(vio_stack* s, int nthreads)
{
    int res = s->f.res;
    long long cols = (long long)res * res;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
    for (long long c = 0; c < cols; ++c) vio_stack_column(s, (int)(c % res), (int)(c / res));
    (void)nthreads;
}

void vio_stack_export(vio_stack* s, double* out, int nthreads)
{
    vio_stack_fill(s, nthreads);
    int n = s->f.n, res = s->f.res;
    for (int j = 0; j < res; ++j)
        for (int i = 0; i < res; ++i) {
            const double* col = s->data + ((size_t)j * res + i) * (size_t)n;
            for (int k = 0; k < n; ++k) out[((size_t)k * res + j) * res + i] = col[k];
        }
}

/* Extended stack S^: layer -1 is fully transmitting, texels outside the
 * res x res grid are fully transmitting (reading R12). */
static double stack_ext(vio_stack* s, int k, int j, int i)
{
    if (k < 0) return 1.0;
    if (i < 0 || j < 0 || i >= s->f.res || j >= s->f.res) return 1.0;
    if (k > s->f.n - 1) k = s->f.n - 1;
    return vio_stack_column(s, i, j)[k];
}

/* Transmittance at a world point: slice index by Eq. 9, light-space UV by
 * Eq. 10 (an orthographic light projection, R9), continuous in depth
 * (reading R11: the index q lies between faces q-1 and q, so the lookup
 * interpolates layers S[q-1] ... with S[-1] = 1), bilinear in the slice,
 * clamped beyond the last face (R12). */
double vio_stack_lookup(vio_stack* s, const double p[3]) { return vio_stack_lookup_layer(s, p, 0, 0.0); }

/* The same lookup, or with nearest = 1 the nearest-layer reading R25 of
 * Eq. 9: the index q picks one layer of the texture array, the face nearest
 * to q, f = floor(q + 1/2 + shift) clamped to 0..n (face 0 = 1, face f holds
 * S[f-1]), read bilinearly in that layer.  shift = 0 is the reading; a
 * small non-zero shift moves every rounding boundary, which the tests use
 * to tell which results depend on a depth index lying within |shift| of a
 * half-integer. */
double vio_stack_lookup_layer(vio_stack* s, const double p[3], int nearest, double shift)
{
    const vio_frame* f = &s->f;
    double q, x, y;
    if (f->positional) {
        /* R38: depth from the light and the perspective projection; a
         * point at or behind the light's depth plane lies outside every
         * frustum texel and is lit (R40) */
        double r[3] = {p[0] - f->P[0], p[1] - f->P[1], p[2] - f->P[2]};
        double d = dot3(f->L, r);
        if (!(d > 0.0)) return 1.0;
        q = f->n * (d - f->dmin) / (f->dmax - f->dmin); /* Eq. 9 */
        x = (dot3(f->U, r) / d + f->R) / (2.0 * f->R) * f->res - 0.5;
        y = (dot3(f->V, r) / d + f->R) / (2.0 * f->R) * f->res - 0.5;
    } else {
        q = f->n * (dot3(f->L, p) - f->dmin) / (f->dmax - f->dmin); /* Eq. 9 */
        double r[3] = {p[0] - f->c[0], p[1] - f->c[1], p[2] - f->c[2]};
        x = (dot3(f->U, r) + f->R) / (2.0 * f->R) * f->res - 0.5;
        y = (dot3(f->V, r) + f->R) / (2.0 * f->R) * f->res - 0.5;
    }
    double z = q - 1.0;
    if (nearest) z = floor(q + 0.5 + shift) - 1.0;
    if (z < -1.0) z = -1.0;
    if (z > f->n - 1.0) z = f->n - 1.0;

    double kf = floor(z), xf = floor(x), yf = floor(y);
    double wz = z - kf, wx = x - xf, wy = y - yf;
    int k0 = (int)kf, x0 = (int)xf, y0 = (int)yf;
    double acc = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wt = (dk ? wz : 1.0 - wz) * (dy ? wy : 1.0 - wy) * (dx ? wx : 1.0 - wx);
                if (wt == 0.0) continue; /* e.g. layer n when z = n-1 exactly */
                acc += wt * stack_ext(s, k0 + dk, y0 + dy, x0 + dx);
            }
    return acc;
}

/* ------------------------------------------------------------------ */
/* Coefficient A at a sample (section 3: direct shadow; section 3.2.3:   */
/* shell and cone scattering distributions; Eq. 7 uses A as the weight). */
/* ------------------------------------------------------------------ */
double vio_coefficient(vio_stack* s, int mode, const vio_opts* o, int N, const double p[3], const double d[3])
{
    if (mode == VIO_MODE_NONE) return 1.0;
    if (mode == VIO_MODE_SHADOW) return vio_stack_lookup_layer(s, p, o->nearest_layer, o->nearest_shift);

    if (mode == VIO_MODE_SHELL) {
        /* Cuboid shells: the sample moved by +-(r+1) h along x, y and z;
         * shell r weighted w_r (section 3.2.3: each neighbourhood gets a
         * weight), equal weights when none is given (reading R13):
         * A = sum_r w_r mean_r / sum_r w_r. */
        double h = o->shell_h_vox / N, num = 0.0, wsum = 0.0;
        int weighted = 0;
        for (int r = 0; r < o->shell_count && r < 8; ++r) weighted |= o->shell_w[r] != 0.0;
        for (int r = 0; r < o->shell_count; ++r) {
            double w = weighted ? o->shell_w[r] : 1.0, sum = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int sg = -1; sg <= 1; sg += 2) {
                    double q[3] = {p[0], p[1], p[2]};
                    q[a] += sg * (r + 1) * h;
                    sum += vio_stack_lookup_layer(s, q, o->nearest_layer, o->nearest_shift);
                }
            num += w * sum / 6.0;
            wsum += w;
        }
        return num / wsum;
    }

    double taps[VIO_MAX_CONE_TAPS][3];
    int nt = vio_cone_taps(s, o, p, d, taps);
    if (nt == 0) return 1.0;
    double sum = 0.0;
    for (int t = 0; t < nt; ++t) sum += vio_stack_lookup_layer(s, taps[t], o->nearest_layer, o->nearest_shift);
    return sum / nt;
}

/* Cone tap positions at sample p viewed along d (section 3.2.3, Eq. 11).
 * The light at p travels along L_s: the stack's direction L for a
 * directional light; for a point light (reading R39) the direction from the
 * light to p, L_s = (p - P)/|p - P|.  B_proj lies in the plane of sample,
 * light and viewer: the direction toward the viewer with its component
 * along L_s removed (reading R14); when the view runs along L_s it is U with
 * its L_s component removed.  Ring m lies toward the light along L_s, at the
 * point t_m whose depth is m slabs less than p's: t_m = m ds / (L . L_s)
 * (= m ds for a directional light); its radius is t_m tan(phi), its axis
 * B_proj rotated about L_s by theta (Rodrigues, Eq. 11).  The lattice form
 * (R15) puts G x G points one slab toward the light, spacing t_1 tan(phi)/2
 * in the (B_proj, L_s x B_proj) plane.  Returns the tap count. */
int vio_cone_taps(vio_stack* s, const vio_opts* o, const double p[3], const double d[3],
                  double taps[][3])
{
    const vio_frame* f = &s->f;
    double Ls[3] = {f->L[0], f->L[1], f->L[2]};
    if (f->positional) {
        double r[3] = {p[0] - f->P[0], p[1] - f->P[1], p[2] - f->P[2]};
        double nr = norm3(r);
        for (int a = 0; a < 3; ++a) Ls[a] = r[a] / nr;
    }
    /* t_1: one slab toward the light along L_s */
    double step = f->positional ? f->ds / dot3(f->L, Ls) : f->ds;
    double wv[3] = {-d[0], -d[1], -d[2]};
    double wl = dot3(wv, Ls);
    double B[3] = {wv[0] - wl * Ls[0], wv[1] - wl * Ls[1], wv[2] - wl * Ls[2]};
    double nb = norm3(B);
    if (nb < 1e-6) {
        double ul = dot3(f->U, Ls);
        for (int a = 0; a < 3; ++a) B[a] = f->U[a] - ul * Ls[a];
        nb = norm3(B);
    }
    for (int a = 0; a < 3; ++a) B[a] /= nb;
    double LxB[3];
    cross3(Ls, B, LxB);
    double LdotB = dot3(Ls, B);
    int nt = 0;
    if (o->cone_grid <= 0) {
        if (o->cone_rings * o->cone_angles > VIO_MAX_CONE_TAPS) return 0;
        for (int m = 1; m <= o->cone_rings; ++m) {
            double cm = m * step, rm = cm * o->cone_tan;
            for (int qa = 0; qa < o->cone_angles; ++qa) {
                double th = 2.0 * VIO_PI * qa / o->cone_angles;
                double ct = cos(th), st = sin(th), Ap[3];
                for (int a = 0; a < 3; ++a) Ap[a] = B[a] * ct + LxB[a] * st + LdotB * Ls[a] * (1.0 - ct);
                for (int a = 0; a < 3; ++a) taps[nt][a] = p[a] - cm * Ls[a] + rm * Ap[a];
                ++nt;
            }
        }
    } else {
        int G = o->cone_grid;
        if (G * G > VIO_MAX_CONE_TAPS) return 0;
        double rho = step * o->cone_tan / 2.0, half = (G - 1) / 2.0;
        for (int ia = 0; ia < G; ++ia)
            for (int ib = 0; ib < G; ++ib) {
                double a_ = ia - half, b_ = ib - half;
                for (int a = 0; a < 3; ++a) taps[nt][a] = p[a] - step * Ls[a] + a_ * rho * B[a] + b_ * rho * LxB[a];
                ++nt;
            }
    }
    return nt;
}

/* ------------------------------------------------------------------ */
/* Local illumination (section 4's Phong comparison mode).  The normal   */
/* comes from central differences of the reconstructed field one voxel  */
/* either side along each axis (R29); n = -g / max(|g|, grad_eps), so it */
/* is a unit vector wherever the field changes by at least grad_eps per  */
/* voxel and shrinks smoothly to zero in flat regions (R30).  Light      */
/* vector l = -L, view vector v = -d (R31); Phong reflection            */
/* r = 2 (n.l) n - (n.n) l, which is the mirror of l for a unit n (R32). */
/* ------------------------------------------------------------------ */
void vio_gradient(const vio_volume* v, const double p[3], double g[3])
{
    double h = 1.0 / v->N;
    for (int a = 0; a < 3; ++a) {
        double q1[3] = {p[0], p[1], p[2]}, q0[3] = {p[0], p[1], p[2]};
        q1[a] += h;
        q0[a] -= h;
        g[a] = 0.5 * (vio_volume_sample(v, q1) - vio_volume_sample(v, q0));
    }
}

void vio_phong(const vio_volume* v, const vio_opts* o, const double L[3], const double p[3], const double d[3],
               double* sd, double* ss)
{
    double g[3], n[3], l[3], w[3], r[3];
    vio_gradient(v, p, g);
    double gn = norm3(g), den = gn > o->grad_eps ? gn : o->grad_eps;
    for (int a = 0; a < 3; ++a) {
        n[a] = -g[a] / den;
        l[a] = -L[a];
        w[a] = -d[a];
    }
    double nl = dot3(n, l), nn = dot3(n, n);
    for (int a = 0; a < 3; ++a) r[a] = 2.0 * nl * n[a] - nn * l[a];
    double rv = dot3(r, w);
    *sd = o->phong_ka + o->phong_kd * (nl > 0.0 ? nl : 0.0);
    *ss = o->phong_ks * (rv > 0.0 ? pow(rv, o->phong_shininess) : 0.0);
}

/* ------------------------------------------------------------------ */
/* Camera rays (Eq. 10's camera matrices E_mv, E_vi; reading R27).       */
/* ------------------------------------------------------------------ */
int vio_camera_ray(const vio_camera* cam, int px, int py, double o[3], double d[3])
{
    double W = cam->width, H = cam->height;
    double xn = 2.0 * (px + 0.5) / W - 1.0;
    double yn = 1.0 - 2.0 * (py + 0.5) / H;
    double fwd[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1], cam->target[2] - cam->eye[2]};
    double nf = norm3(fwd);
    for (int a = 0; a < 3; ++a) fwd[a] /= nf;
    double right[3], up2[3];
    cross3(fwd, cam->up, right);
    double nr = norm3(right);
    for (int a = 0; a < 3; ++a) right[a] /= nr;
    cross3(right, fwd, up2);
    if (cam->kind == VIO_CAM_PERSP) {
        double th = tan(0.5 * cam->fovy_deg * VIO_PI / 180.0);
        for (int a = 0; a < 3; ++a) {
            o[a] = cam->eye[a];
            d[a] = fwd[a] + xn * th * (W / H) * right[a] + yn * th * up2[a];
        }
        double nd = norm3(d);
        for (int a = 0; a < 3; ++a) d[a] /= nd;
    } else {
        double h = cam->ortho_half_h;
        for (int a = 0; a < 3; ++a) {
            d[a] = fwd[a];
            o[a] = cam->eye[a] + xn * h * (W / H) * right[a] + yn * h * up2[a];
        }
    }
    return 0;
}

/* Slab test against [0,1]^3; entry clamped at t = 0 (R27). */
int vio_cube_hit(const double o[3], const double d[3], double* t_in, double* t_far)
{
    double tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > 1.0) return 0;
            continue;
        }
        double t1 = (0.0 - o[a]) / d[a], t2 = (1.0 - o[a]) / d[a];
        double lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
        if (lo > tn) tn = lo;
        if (hi < tf) tf = hi;
    }
    double ti = tn > 0.0 ? tn : 0.0;
    *t_in = ti;
    *t_far = tf;
    return tf > ti;
}

/* ------------------------------------------------------------------ */
/* Render: single-pass ray casting (section 4), segments of length       */
/* step from the entry point with a partial last segment (R19), sampled  */
/* at midpoints; emission weighted by A (Eq. 7, R16); front-to-back      */
/* compositing (Eq. 3); termination once the remaining transmittance is */
/* at most term_eps (R20); premultiplied background last (R23).          */
/* ------------------------------------------------------------------ */
static void render_pixel(const vio_volume* v, const vio_tf* tf, vio_stack* s, const vio_camera* cam, int mode,
                         double step_vox, const vio_opts* o, int px, int py, int want_full, double out_full[4],
                         double out_term[4], int64_t* ns_term, int64_t* ns_full)
{
    double dref = 1.0 / v->N, dt = step_vox / v->N;
    double ro[3], rd[3], ti, tfar;
    double C[3] = {0.0, 0.0, 0.0}, ad = 0.0;
    double Ct[3] = {0.0, 0.0, 0.0}, adt = 0.0;
    int terminated = 0;
    int64_t kt = 0, K = 0;
    vio_camera_ray(cam, px, py, ro, rd);
    if (vio_cube_hit(ro, rd, &ti, &tfar)) {
        K = (int64_t)ceil((tfar - ti) / dt);
        for (int64_t k = 0; k < K; ++k) {
            double t0 = ti + k * dt, t1 = ti + (k + 1) * dt;
            if (t1 > tfar) t1 = tfar;
            double len = t1 - t0, tm = 0.5 * (t0 + t1), p[3];
            for (int a = 0; a < 3; ++a) p[a] = ro[a] + tm * rd[a];
            double rgba[4];
            vio_tf_lookup(tf, vio_volume_sample(v, p), rgba);
            double alpha = vio_segment_alpha(rgba[3], len, dref);
            /* The coefficient only scales an emission that is zero when
             * alpha is zero, so it is gathered only where alpha > 0. */
            double sd = 1.0, ss = 0.0;
            if (alpha > 0.0) {
                if (mode == VIO_MODE_PHONG) {
                    /* the light travels along L, or from P to p for a point light */
                    double Lp[3] = {s->f.L[0], s->f.L[1], s->f.L[2]};
                    if (s->f.positional) {
                        for (int a = 0; a < 3; ++a) Lp[a] = p[a] - s->f.P[a];
                        double nl = norm3(Lp);
                        for (int a = 0; a < 3; ++a) Lp[a] /= nl;
                    }
                    vio_phong(v, o, Lp, p, rd, &sd, &ss);
                } else {
                    double A = vio_coefficient(s, mode, o, v->N, p, rd);
                    sd = o->ambient + (1.0 - o->ambient) * A;
                }
            }
            /* emission alpha (sd rgb + ss) (x) light: Eq. 7 with the
             * coefficient, or the Phong terms (specular uncoloured) */
            for (int c = 0; c < 3; ++c)
                C[c] += (1.0 - ad) * (alpha * (sd * rgba[c] + ss) * o->light_rgb[c]);
            ad += (1.0 - ad) * alpha;
            if (!terminated && 1.0 - ad <= o->term_eps) {
                terminated = 1;
                kt = k + 1;
                for (int c = 0; c < 3; ++c) Ct[c] = C[c];
                adt = ad;
                if (!want_full) break;
            }
        }
    }
    if (!terminated) {
        kt = K;
        for (int c = 0; c < 3; ++c) Ct[c] = C[c];
        adt = ad;
    }
    if (out_full) {
        for (int c = 0; c < 3; ++c) out_full[c] = C[c] + (1.0 - ad) * o->bg[c];
        out_full[3] = ad + (1.0 - ad) * o->bg[3];
    }
    for (int c = 0; c < 3; ++c) out_term[c] = Ct[c] + (1.0 - adt) * o->bg[c];
    out_term[3] = adt + (1.0 - adt) * o->bg[3];
    *ns_term = kt;
    *ns_full = K;
}

int vio_render(const vio_volume* v, const vio_tf* tf, vio_stack* s, const vio_camera* cam, int mode,
               double step_vox, const vio_opts* o, const int64_t* pix, int64_t npix, double* out_full,
               double* out_term, int64_t* samples_term, int64_t* samples_full, int nthreads)
{
    if (!v || !tf || !cam || !o || !out_term || !(step_vox > 0.0)) return -1;
    if (mode != VIO_MODE_NONE && !s) return -1;  /* Phong takes its light from the stack's frame */
    int64_t W = cam->width;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t q = 0; q < npix; ++q) {
        int64_t id = pix ? pix[q] : q;
        int64_t nt, nf;
        render_pixel(v, tf, s, cam, mode, step_vox, o, (int)(id % W), (int)(id / W), out_full != NULL,
                     out_full ? out_full + 4 * q : NULL, out_term + 4 * q, &nt, &nf);
        if (samples_term) samples_term[q] = nt;
        if (samples_full) samples_full[q] = nf;
    }
    (void)nthreads;
    return 0;
}
