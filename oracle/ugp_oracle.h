/*
 * ugp_oracle.h -- interface of the FP64 CPU oracle (test infrastructure only).
 *
 * Used by the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark.  Not part of the product; shares nothing with the GPU library.
 * Arrays are host memory.  Rays are float32 [o.xyz, w.xyz, t0, t1] exactly as
 * the GPU receives them; all arithmetic is double precision.
 */
#ifndef UGP_ORACLE_H
#define UGP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_scene orc_scene;

typedef struct {
    double origin[3], target[3], up[3];
    double vfov_deg;
    int32_t width, height;
} orc_camera;

typedef struct {
    int32_t spp, max_depth;
    uint64_t seed;
    int64_t sample_offset;
    double env_radiance[3];
    int32_t mis_mode; /* 0 balance heuristic, 1 phase sampling only, 2 light sampling only */
    /* radiance cache: mode 0 off; 1 training paths (chosen with probability
     * nrc_train_frac) run to max_depth, the others end in the cache; 2 every
     * path ends in the cache; 3 paths end after nrc_terminate_after scattering
     * events with nothing added.  nrc_weights: double [orc_nrc_num_params()];
     * nrc_box: lo[3], hi[3] of the position encoding. */
    int32_t nrc_mode, nrc_terminate_after;
    double nrc_train_frac;
    const double *nrc_weights;
    double nrc_box[6];
    /* transport model: 0 linear transmittance (Sec. 4); 1 the exponential
     * variant (App. D): collisions and light samples by analog decomposition
     * tracking, environment samples by exp(-sum I_k), no primitive excluded
     * from a path's next segment */
    int32_t transport;
} orc_render_params;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox4x32_10_batch(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out);
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

int orc_scene_create(int64_t n, const float *mean, const float *scale, const float *rotation,
                     const float *density, const float *albedo, const float *roughness,
                     const float *emission, const int32_t *material, double eps, orc_scene **out);
void orc_scene_destroy(orc_scene *S);
int orc_scene_build_bvh(orc_scene *S);
double orc_cutoff_radius(const orc_scene *S);
void orc_prim_frame(const orc_scene *S, int64_t k, double M[9], double normal[3], double lo[3],
                    double hi[3]);

int orc_chord(const orc_scene *S, int64_t k, const float ray[8], double out[2]);
double orc_ray_integral(const orc_scene *S, int64_t k, const double ray[8], double x, double y);

void orc_transmittance(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                       int use_bvh, double *F_out, double *T_out);
void orc_F_at(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
              const double *t, int use_bvh, double *F_out);
void orc_saturation(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                    int use_bvh, double *tsat_out);
void orc_rf_radiance(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                     const double *tsat, int use_bvh, double *L_out);
void orc_exp_transmittance(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                           int use_bvh, double *T_out);
void orc_exp_sample(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude, uint64_t seed,
                    int use_bvh, int32_t *prim_out, double *t_out, double *margin_out);
void orc_sample_collision(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                          const double *u, int use_bvh, int32_t *prim_out, double *t_out,
                          double *F_out, double *tsat_out, double *margin_out);
void orc_emitter_query(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                       const int32_t *target, int use_bvh, double *L_out);
/* light sampling of the path tracer: solid-angle pdf of direction w from x
 * toward emissive primitive k (times the uniform choice 1/n_emit), and the
 * direction toward a Gaussian point of emitter slot j from uniforms u[4]
 * (returns 0 if none) */
double orc_light_pdf(const orc_scene *S, int64_t k, const double *x, const double *w);
int orc_light_dir(const orc_scene *S, int64_t j, const double *x, const double *u, double *w);

void orc_phase_eval(int mat, const double alb[3], double rough, const double nrm[3],
                    const double wo[3], const double wi[3], double f[3], double *pdf);
void orc_phase_sample(int mat, const double alb[3], double rough, const double nrm[3],
                      const double wo[3], double u1, double u2, double wi[3], double wgt[3],
                      double *pdf);

/* SGGX microflake phase function with a Lambertian base BSDF (Sec. 4.2,
 * eq. vndf, eq. phase_function, App. B); s6 = (xx, yy, zz, xy, xz, yz) of the
 * symmetric positive-definite matrix S in the world frame; values per unit
 * albedo.  what: 0 sigma(v), 1 D(v), 2 D_wo(v). */
double orc_sggx_sigma(const double s6[6], const double w[3]);
double orc_sggx_D(const double s6[6], const double n[3]);
double orc_sggx_vndf(const double s6[6], const double wo[3], const double n[3]);
void orc_sggx_sample_vndf(const double s6[6], const double wo[3], double u1, double u2, double n[3]);
double orc_sggx_phase_est(const double s6[6], const double wo[3], const double wi[3], const double u[4]);
double orc_sggx_phase_quad(const double s6[6], const double wo[3], const double wi[3], int nz, int nphi);
double orc_sggx_pdf_approx(const double wo[3], const double wi[3]);
void orc_sggx_eval_n(const double s6[6], int64_t n, const double *wo, const double *v, int what, double *out);
void orc_sggx_sample_vndf_n(const double s6[6], const double wo[3], int64_t n, const double *u, double *nrm);
void orc_sggx_sample_dir_n(const double s6[6], const double wo[3], int64_t n, const double *u, double *wi);
void orc_sggx_phase_est_n(const double s6[6], const double wo[3], const double wi[3], int64_t n,
                          const double *u, double *out);
/* per-primitive SGGX matrices [n][6] (copied); materials 2 and 3 need them */
int orc_scene_set_sggx(orc_scene *S, const float *sggx);
/* metallic [n] of material 3 (copied; default 0) */
int orc_scene_set_metallic(orc_scene *S, const float *met);
/* material 3: SGGX microflakes with a Disney-style base BSDF (diffuse with
 * retro-reflection + GGX specular, metallic m); c = base colour */
double orc_disney_spec_prob(const double c[3], double met);
void orc_disney_base(const double c[3], double rough, double met, const double n[3], const double wo[3],
                     const double wi[3], double fs[3], double fd[3]);
void orc_sggx_disney_est(const double s6[6], const double c[3], double rough, double met, const double wo[3],
                         const double wi[3], const double u[6], double f[3]);
int orc_sggx_disney_sample(const double s6[6], const double c[3], double rough, double met, const double wo[3],
                           double u0, double u1, const double v[3], double wi[3], double wgt[3]);
void orc_sggx_roughened(const double s6[6], double rough, double out6[6]);
double orc_sggx_disney_pdf_approx(const double s6[6], const double c[3], double rough, double met,
                                  const double wo[3], const double wi[3]);
void orc_sggx_disney_quad(const double s6[6], const double c[3], double rough, double met, const double wo[3],
                          const double wi[3], int nz, int nphi, double f[3]);

void orc_camera_rays(const orc_camera *cam, uint64_t seed, uint32_t sample, float *rays);
int64_t orc_render(const orc_scene *S, const orc_camera *cam, const orc_render_params *p,
                   int64_t n_pix, const int64_t *pixels, int nthreads, double *sum, double *sumsq);
void orc_path_radiance(const orc_scene *S, const orc_camera *cam, const orc_render_params *p,
                       uint32_t pix, uint32_t sample, double L[3]);
/* radiance of one path and its cache-training records: per scattering vertex
 * of a training path, 24 doubles = network inputs (position, outgoing
 * direction, facet normal, roughness, albedo, 3 zeros), throughput, pixel,
 * path radiance before the vertex's scattered light, vertex index.  Returns
 * the number of records (at most max_rec are written). */
int orc_path_records(const orc_scene *S, const orc_camera *cam, const orc_render_params *p, uint32_t pix,
                     uint32_t sample, double *rec, int max_rec, double L[3]);

/* neural radiance cache (double precision reference) */
int orc_nrc_num_params(void);
void orc_nrc_encode(int64_t n, const float *in, const double lo[3], const double hi[3], double *feat);
void orc_nrc_forward(int64_t n, const double *W, const double *feat, double *y);
double orc_nrc_loss_grad(int64_t n, const double *W, const double *feat, const double *target, double *grad);
void orc_nrc_adam(int64_t np, double *W, double *m, double *v, const double *g, int t, double lr, double b1,
                  double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
