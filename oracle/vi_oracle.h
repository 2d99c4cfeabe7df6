/*
 * vi_oracle.h -- FP64 CPU oracle for slice-based ray-casting volume
 * illumination (Luo, "Interactive volume illumination of slice-based ray
 * casting", arXiv 2008.06134).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * statement of what the method computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library and includes nothing
 * from it.
 *
 * Everything is IEEE double with libm exp/log/pow.  Loops are scalar; the
 * only parallelism is an OpenMP split over independent light columns and
 * independent pixels, which does not change any result.
 *
 * Conventions (readings of the paper, listed with reasons in the design
 * notes of the repository):
 *   - the volume fills the unit cube [0,1]^3 (section 3.2.1, "unit cube");
 *     voxel (x,y,z) has its centre at ((x+1/2)/N, (y+1/2)/N, (z+1/2)/N);
 *     storage is raw[z][y][x] with x fastest; only cubic volumes N^3;
 *   - the light direction is the propagation direction; the first slab lies
 *     at the minimum distance (Eq. 8);
 *   - the transfer-function alpha is defined per reference length dref =
 *     one voxel = 1/N and corrected per segment length (Eq. 6);
 *   - the attenuation stack stores the transmittance after each slab,
 *     S[k][j][i], k = 0..n-1 (Alg. 1, Eq. 4);
 *   - rendering composites front to back (Eq. 3) with the gathered
 *     coefficient A weighting the emission (Eq. 7).
 */
#ifndef VI_ORACLE_H
#define VI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VIO_U8 = 0, VIO_U16 = 1, VIO_F16 = 2, VIO_F32 = 3 };
enum { VIO_MODE_NONE = 0, VIO_MODE_SHADOW = 1, VIO_MODE_SHELL = 2, VIO_MODE_CONE = 3, VIO_MODE_PHONG = 4 };
enum { VIO_CAM_ORTHO = 0, VIO_CAM_PERSP = 1 };

typedef struct {
    const void* data;   /* raw[z][y][x], x fastest                      */
    int dtype;          /* VIO_U8 / VIO_U16 / VIO_F16 (IEEE half bits) / VIO_F32 */
    int N;              /* edge length in voxels (cubic volumes only)   */
    double scale;       /* value = clamp(raw * scale, 0, 1)             */
} vio_volume;

typedef struct {
    const double* rgba; /* K x 4, non-premultiplied rgb, alpha per dref */
    int K;              /* number of entries, >= 2                      */
} vio_tf;

typedef struct {
    double L[3];        /* unit propagation direction of the light      */
    double U[3], V[3];  /* orthonormal light-plane basis, V = L x U      */
    double c[3];        /* cube centre (1/2,1/2,1/2)                     */
    double dmin, dmax;  /* min / max of L.v over the 8 cube vertices     */
    double ds;          /* slab thickness (dmax - dmin) / n              */
    double R;           /* half-width of the light-plane square          */
    int n, res;         /* slab count and texels per side                */
    double darken;      /* build: exponent m of the (1+alpha)^m slab
                           compensation of section 4 (0 = off, R24)      */
    int positional;     /* 1: point light at P (R34-R38); L is then the
                           light's axis and R the half-width of the
                           texel square at unit depth                    */
    double P[3];
} vio_frame;

typedef struct {
    int kind;           /* VIO_CAM_ORTHO or VIO_CAM_PERSP                */
    double eye[3], target[3], up[3];
    double fovy_deg;    /* perspective: full vertical field of view      */
    double ortho_half_h;/* orthographic: half image height, world units  */
    int width, height;
} vio_camera;

typedef struct {
    double ambient;       /* k_a: s = k_a + (1 - k_a) A                   */
    double light_rgb[3];  /* light colour                                 */
    double bg[4];         /* premultiplied background                     */
    double term_eps;      /* terminate once 1 - alpha_dst <= term_eps     */
    int shell_count;      /* number of cuboid shells                      */
    double shell_w[8];    /* weight of shell r (all 0: equal weights)     */
    double shell_h_vox;   /* shell step in voxels                         */
    int cone_rings;       /* rings toward the light (ring form)           */
    int cone_angles;      /* taps per ring (ring form)                    */
    int cone_grid;        /* 0: ring form, G > 0: G x G lattice form      */
    double cone_tan;      /* tan of the cone half-angle                   */
    double phong_ka, phong_kd, phong_ks; /* local Phong model (no stack)  */
    double phong_shininess;
    double grad_eps;      /* gradient magnitude (per voxel) below which the
                             normal shrinks toward zero                     */
    int nearest_layer;    /* 1: lookups read the layer nearest Eq. 9's index (R25) */
    double nearest_shift; /* moves the nearest-layer rounding boundary (tests) */
} vio_opts;

/* Stack of light-space transmittance slices.  Columns are built on demand
 * (each one exactly as the full build would) so that a sampled render at
 * full size touches only the columns it needs. */
typedef struct vio_stack vio_stack;

int    vio_threads(void); /* OpenMP threads the oracle uses by default */
void   vio_default_opts(vio_opts* o);
int    vio_light_frame(const double l[3], int n, int res, vio_frame* f);
/* point light at `pos` (outside the cube's circumscribed sphere) */
int    vio_light_frame_point(const double pos[3], int n, int res, vio_frame* f);
double vio_volume_sample(const vio_volume* v, const double p[3]);
void   vio_tf_lookup(const vio_tf* tf, double value, double rgba[4]);
double vio_segment_alpha(double a, double len, double dref);
void   vio_build_column(const vio_volume* v, const vio_tf* tf, const vio_frame* f,
                        int i, int j, double* col /* n values */);

vio_stack* vio_stack_create(const vio_volume* v, const vio_tf* tf, const vio_frame* f);
void       vio_stack_destroy(vio_stack* s);
/* build every column (OpenMP over columns) */
void       vio_stack_fill(vio_stack* s, int nthreads);
/* copy the whole stack out as S[k][j][i] */
void       vio_stack_export(vio_stack* s, double* out, int nthreads);
/* column (i,j): n transmittances, built on first use */
const double* vio_stack_column(vio_stack* s, int i, int j);
double     vio_stack_lookup(vio_stack* s, const double p[3]);
double     vio_stack_lookup_layer(vio_stack* s, const double p[3], int nearest, double shift);
int64_t    vio_stack_columns_built(const vio_stack* s);

/* camera ray through pixel (px,py); returns 1 and the entry/exit distances
 * if it hits the unit cube, else 0 */
int  vio_camera_ray(const vio_camera* cam, int px, int py, double o[3], double d[3]);
int  vio_cube_hit(const double o[3], const double d[3], double* t_in, double* t_far);

/* central-difference gradient of the reconstructed field at p, in value
 * per voxel */
void vio_gradient(const vio_volume* v, const double p[3], double g[3]);
/* local Phong terms at p for a ray of direction d and light propagation
 * direction L: diffuse factor sd = ka + kd max(0, n.l) and specular term
 * ss = ks max(0, r.v)^shininess */
void vio_phong(const vio_volume* v, const vio_opts* o, const double L[3], const double p[3], const double d[3],
               double* sd, double* ss);

/* coefficient A at p for a ray of direction d */
/* Cone tap positions at sample p for view direction d (reading R14, R15,
 * R39): at most VIO_MAX_CONE_TAPS rows of world xyz; returns the count. */
#define VIO_MAX_CONE_TAPS 128
int vio_cone_taps(vio_stack* s, const vio_opts* o, const double p[3], const double d[3], double taps[][3]);

double vio_coefficient(vio_stack* s, int mode, const vio_opts* o, int N,
                       const double p[3], const double d[3]);

/* Render the listed pixels (pix = y*W + x; NULL with npix = W*H renders all).
 * out_full: no termination; out_term: terminated at term_eps.
 * Both W*H-ordered as the list, 4 doubles per pixel, premultiplied.
 * samples_term / samples_full: segments composited per pixel (may be NULL). */
int vio_render(const vio_volume* v, const vio_tf* tf, vio_stack* s,
               const vio_camera* cam, int mode, double step_vox, const vio_opts* o,
               const int64_t* pix, int64_t npix,
               double* out_full, double* out_term,
               int64_t* samples_term, int64_t* samples_full, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
