/*
 * ugp_oracle.c -- FP64 CPU oracle for Monte Carlo path tracing of scenes made of
 * linear-transmittance Gaussian primitives.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no source, header, table
 * or helper with the HIP library, and it never calls it.
 *
 * Source: "Unified Gaussian Primitives for Scene Representation and Rendering"
 * (arXiv 2406.09733).  Each routine names the section / equation it follows.
 * Where the paper is silent or garbled the adopted reading is stated inline.
 *
 * Everything is double precision.  Inputs arrive as the same float32 values the
 * GPU receives and are widened exactly.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ugp_oracle.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 and Philox4x64-10 counter-based generators, written from the */
/* definition in Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3" (SC'11): N rounds of (multiply-hi/lo S-box, word          */
/* permutation, xor with a round key), the key bumped by a Weyl sequence      */
/* between rounds.                                                            */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* the same generator over n counters [n][4] (one key) */
void orc_philox4x32_10_batch(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out) {
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four uniforms in [0,1) from one counter: the top 24 bits of each word. */
static void rng4(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t vertex, uint32_t group,
                 double u[4]) {
    uint32_t ctr[4] = {pixel, sample, vertex, group};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = (double)(x[i] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------- */
/* Small vector helpers.                                                      */
/* ------------------------------------------------------------------------- */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(double a[3]) {
    double l = sqrt(dot3(a, a));
    a[0] /= l; a[1] /= l; a[2] /= l;
}

/* Orthonormal basis (b1, b2, n) around a unit vector n: Duff, Burgess,
 * Christensen, Hery, Kensler, Liani, Villemin, "Building an Orthonormal Basis,
 * Revisited" (JCGT 2017). */
static void onb(const double n[3], double b1[3], double b2[3]) {
    double sign = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a; b1[1] = sign * b; b1[2] = -sign * n[0];
    b2[0] = b; b2[1] = sign + n[1] * n[1] * a; b2[2] = -n[1];
}

/* ------------------------------------------------------------------------- */
/* Scene: the primitives of Sec. 3.1 / Sec. 4 with the cut-off of            */
/* eq. (cutoff_threshold).                                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t left, right; /* children (internal) or -1 */
    int32_t first, count; /* primitive range in perm (leaf) */
    double lo[3], hi[3];
} onode;

struct orc_scene {
    int64_t n;
    double r;      /* Mahalanobis radius of the cut-off ellipsoid */
    double *mu;    /* [n][3] mean */
    double *M;     /* [n][9] row-major S^-1 R^T: world offset -> unit-Gaussian frame */
    double *d;     /* [n] peak density G(mu) */
    double *nrm;   /* [n][3] R e_argmin(s): the facet normal of the delta NDF */
    double *alb;   /* [n][3] */
    double *rough; /* [n] */
    double *emis;  /* [n][3] */
    int32_t *mat;  /* [n] 0 Lambert, 1 GGX (delta NDF), 2 / 3 microflakes with an SGGX NDF and a
                      Lambertian / Disney-style base BSDF */
    double *sggx;  /* [n][6] SGGX matrix (xx, yy, zz, xy, xz, yz), world frame; NULL if none */
    double *met;   /* [n] metallic of material 3's base BSDF; NULL = 0 */
    double *lo, *hi;  /* [n][3] axis-aligned box of the cut-off ellipsoid */
    int64_t *emitters;
    double *emA;   /* [n_emit][9] row-major R S of emitter slot j (unit frame -> world offset) */
    int64_t n_emit;
    /* acceleration structure: a plain median-split BVH, used only to find the
       candidate set; results are independent of it (checked against brute force) */
    onode *nodes;
    int64_t n_nodes;
    int64_t *perm;
};

/* Primitive set-up (Sec. 3.1, eq. covariance_decomposition): unit quaternion
 * (w,x,y,z) -> rotation R; Sigma = (R S)(R S)^T, so the map that sends the
 * Gaussian to the unit isotropic one is M = S^-1 R^T.  The cut-off ellipsoid of
 * eq. (cutoff_threshold) is |M (x - mu)| = r with r = sqrt(-2 ln eps). */
int orc_scene_create(int64_t n, const float *mean, const float *scale, const float *rotation,
                     const float *density, const float *albedo, const float *roughness,
                     const float *emission, const int32_t *material, double eps,
                     orc_scene **out) {
    if (n < 0 || !out || !(eps > 0.0 && eps < 1.0)) return 1;
    orc_scene *S = (orc_scene *)calloc(1, sizeof(orc_scene));
    S->n = n;
    S->r = sqrt(-2.0 * log(eps));
    size_t nn = (size_t)(n > 0 ? n : 1);
    S->mu = (double *)malloc(sizeof(double) * 3 * nn);
    S->M = (double *)malloc(sizeof(double) * 9 * nn);
    S->d = (double *)malloc(sizeof(double) * nn);
    S->nrm = (double *)malloc(sizeof(double) * 3 * nn);
    S->alb = (double *)malloc(sizeof(double) * 3 * nn);
    S->rough = (double *)malloc(sizeof(double) * nn);
    S->emis = (double *)malloc(sizeof(double) * 3 * nn);
    S->mat = (int32_t *)malloc(sizeof(int32_t) * nn);
    S->lo = (double *)malloc(sizeof(double) * 3 * nn);
    S->hi = (double *)malloc(sizeof(double) * 3 * nn);
    S->emitters = (int64_t *)malloc(sizeof(int64_t) * nn);
    S->emA = (double *)malloc(sizeof(double) * 9 * nn);
    S->n_emit = 0;
    for (int64_t k = 0; k < n; ++k) {
        double qw = rotation[4 * k + 0], qx = rotation[4 * k + 1], qy = rotation[4 * k + 2],
               qz = rotation[4 * k + 3];
        double ql = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= ql; qx /= ql; qy /= ql; qz /= ql;
        double R[3][3] = {
            {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy)},
            {2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx)},
            {2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)}};
        double s[3] = {scale[3 * k + 0], scale[3 * k + 1], scale[3 * k + 2]};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S->M[9 * k + 3 * i + j] = R[j][i] / s[i];
        int m = 0;
        if (s[1] < s[m]) m = 1;
        if (s[2] < s[m]) m = 2;
        for (int j = 0; j < 3; ++j) S->nrm[3 * k + j] = R[j][m];
        for (int j = 0; j < 3; ++j) {
            double h2 = 0.0;
            for (int i = 0; i < 3; ++i) h2 += (R[j][i] * s[i]) * (R[j][i] * s[i]);
            double h = S->r * sqrt(h2);
            S->mu[3 * k + j] = mean[3 * k + j];
            /* a relative 1e-12 widening keeps the box conservative under rounding */
            S->lo[3 * k + j] = mean[3 * k + j] - h * (1.0 + 1e-12) - 1e-300;
            S->hi[3 * k + j] = mean[3 * k + j] + h * (1.0 + 1e-12) + 1e-300;
            S->alb[3 * k + j] = albedo[3 * k + j];
            S->emis[3 * k + j] = emission[3 * k + j];
        }
        S->d[k] = density[k];
        S->rough[k] = roughness[k];
        S->mat[k] = material[k];
        if (S->emis[3 * k] > 0.0 || S->emis[3 * k + 1] > 0.0 || S->emis[3 * k + 2] > 0.0) {
            double *A = S->emA + 9 * S->n_emit;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) A[3 * i + j] = R[i][j] * s[j];
            S->emitters[S->n_emit++] = k;
        }
    }
    if (S->n_emit > 0) S->emA = (double *)realloc(S->emA, sizeof(double) * 9 * (size_t)S->n_emit);
    *out = S;
    return 0;
}

void orc_scene_destroy(orc_scene *S) {
    if (!S) return;
    free(S->mu); free(S->M); free(S->d); free(S->nrm); free(S->alb); free(S->rough);
    free(S->emis); free(S->mat); free(S->lo); free(S->hi); free(S->emitters); free(S->emA);
    free(S->sggx); free(S->met);
    free(S->nodes); free(S->perm);
    free(S);
}

double orc_cutoff_radius(const orc_scene *S) { return S->r; }

void orc_prim_frame(const orc_scene *S, int64_t k, double M[9], double normal[3], double lo[3],
                    double hi[3]) {
    for (int i = 0; i < 9; ++i) M[i] = S->M[9 * k + i];
    for (int i = 0; i < 3; ++i) {
        normal[i] = S->nrm[3 * k + i];
        lo[i] = S->lo[3 * k + i];
        hi[i] = S->hi[3 * k + i];
    }
}

/* ------------------------------------------------------------------------- */
/* Ray / primitive: chord of the cut-off ellipsoid and the ray integral.      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t k;
    double a, b;   /* chord clipped to [t0, t1] */
    double tc;     /* parameter of the closest approach in the unit frame */
    double A;      /* |M w|^2 */
    double rho2;   /* squared distance of closest approach in the unit frame */
} ohit;

/* Chord of the cut-off ellipsoid (Sec. 4.1, eq. cutoff_threshold): in the unit
 * frame o' = M(o - mu), w' = M w, the ray point is o' + t w' and the ellipsoid
 * is |.| = r.  Closest approach t_c = -(o'.w')/A with A = w'.w', squared
 * distance rho^2 = |o' x w'|^2 / A; the chord is t_c -/+ sqrt((r^2-rho^2)/A). */
static int ray_prim(const orc_scene *S, int64_t k, const double o[3], const double w[3], double t0,
                    double t1, ohit *h) {
    const double *M = S->M + 9 * k, *mu = S->mu + 3 * k;
    double dlt[3] = {o[0] - mu[0], o[1] - mu[1], o[2] - mu[2]};
    double op[3], wp[3];
    for (int i = 0; i < 3; ++i) {
        op[i] = M[3 * i] * dlt[0] + M[3 * i + 1] * dlt[1] + M[3 * i + 2] * dlt[2];
        wp[i] = M[3 * i] * w[0] + M[3 * i + 1] * w[1] + M[3 * i + 2] * w[2];
    }
    double A = dot3(wp, wp);
    if (!(A > 0.0)) return 0;
    double cr[3];
    cross3(op, wp, cr);
    double rho2 = dot3(cr, cr) / A;
    double r2 = S->r * S->r;
    if (!(rho2 < r2)) return 0;
    double tc = -dot3(op, wp) / A;
    double half = sqrt((r2 - rho2) / A);
    double a = fmax(t0, tc - half), b = fmin(t1, tc + half);
    if (!(a < b)) return 0;
    h->k = k; h->a = a; h->b = b; h->tc = tc; h->A = A; h->rho2 = rho2;
    return 1;
}

/* Ray integral I(x, y) = int_x^y G(o + t w) dt, closed form of App. A with its
 * garbled square corrected: the exponent is -(A/2)(t - t_c)^2 - rho^2/2, so
 * I = d sqrt(pi/(2A)) exp(-rho^2/2) [erf(tau_y) - erf(tau_x)],
 * tau_t = sqrt(A/2)(t - t_c).  x and y lie inside the chord, where the
 * truncated kernel equals the Gaussian.  The difference of erf is taken as a
 * difference of erfc when both arguments have the same sign, to avoid
 * cancellation in the tails. */
static double seg_integral(const orc_scene *S, const ohit *h, double x, double y) {
    if (!(x < y)) return 0.0;
    double s = sqrt(0.5 * h->A);
    double tx = s * (x - h->tc), ty = s * (y - h->tc);
    double diff;
    if (tx >= 0.0) diff = erfc(tx) - erfc(ty);
    else if (ty <= 0.0) diff = erfc(-ty) - erfc(-tx);
    else diff = erf(ty) - erf(tx);
    return S->d[h->k] * sqrt(M_PI / (2.0 * h->A)) * exp(-0.5 * h->rho2) * diff;
}

/* Kernel value G(o + t w) inside the chord: d exp(-(A (t-t_c)^2 + rho^2)/2). */
static double kernel_at(const orc_scene *S, const ohit *h, double t) {
    double q = h->A * (t - h->tc) * (t - h->tc) + h->rho2;
    return S->d[h->k] * exp(-0.5 * q);
}

int orc_chord(const orc_scene *S, int64_t k, const float ray[8], double out[2]) {
    double o[3] = {ray[0], ray[1], ray[2]}, w[3] = {ray[3], ray[4], ray[5]};
    ohit h;
    if (!ray_prim(S, k, o, w, ray[6], ray[7], &h)) return 0;
    out[0] = h.a;
    out[1] = h.b;
    return 1;
}

double orc_ray_integral(const orc_scene *S, int64_t k, const double ray[8], double x, double y) {
    ohit h;
    if (!ray_prim(S, k, ray, ray + 3, ray[6], ray[7], &h)) return 0.0;
    double a = fmax(x, h.a), b = fmin(y, h.b);
    return seg_integral(S, &h, a, b);
}

/* ------------------------------------------------------------------------- */
/* Candidate gathering: brute force, or a median-split BVH over the boxes.    */
/* Either way the result is the set H = {k != exclude : a_k < b_k}.           */
/* ------------------------------------------------------------------------- */
typedef struct {
    ohit *v;
    int64_t n, cap;
} hitvec;

static void hv_push(hitvec *hv, const ohit *h) {
    if (hv->n == hv->cap) {
        hv->cap = hv->cap ? 2 * hv->cap : 64;
        hv->v = (ohit *)realloc(hv->v, sizeof(ohit) * (size_t)hv->cap);
    }
    hv->v[hv->n++] = *h;
}

static int box_hit(const double lo[3], const double hi[3], const double o[3], const double w[3],
                   double t0, double t1) {
    for (int i = 0; i < 3; ++i) {
        if (w[i] != 0.0) {
            double ta = (lo[i] - o[i]) / w[i], tb = (hi[i] - o[i]) / w[i];
            if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        } else if (o[i] < lo[i] || o[i] > hi[i]) {
            return 0;
        }
    }
    return t0 <= t1;
}

typedef struct {
    const orc_scene *S;
    int axis;
} sortctx;

static double centroid(const orc_scene *S, int64_t k, int axis) {
    return 0.5 * (S->lo[3 * k + axis] + S->hi[3 * k + axis]);
}

/* quickselect on perm[first..last) so that element nth is in sorted place */
static void select_nth(const orc_scene *S, int64_t *p, int64_t first, int64_t last, int64_t nth,
                       int axis) {
    while (last - first > 1) {
        int64_t mid = first + (last - first) / 2;
        double pivot = centroid(S, p[mid], axis);
        int64_t i = first, j = last - 1;
        while (i <= j) {
            while (centroid(S, p[i], axis) < pivot) ++i;
            while (centroid(S, p[j], axis) > pivot) --j;
            if (i <= j) {
                int64_t t = p[i]; p[i] = p[j]; p[j] = t;
                ++i; --j;
            }
        }
        if (nth <= j) last = j + 1;
        else if (nth >= i) first = i;
        else return;
    }
}

int orc_scene_build_bvh(orc_scene *S) {
    free(S->nodes); free(S->perm);
    int64_t n = S->n;
    S->perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) S->perm[i] = i;
    int64_t cap = 2 * (n > 0 ? n : 1);
    S->nodes = (onode *)malloc(sizeof(onode) * (size_t)cap);
    S->n_nodes = 0;
    if (n == 0) return 0;
    /* explicit work stack of (node, first, count) */
    typedef struct { int64_t node, first, count; } job;
    job *stack = (job *)malloc(sizeof(job) * 128);
    int sp = 0;
    S->n_nodes = 1;
    stack[sp++] = (job){0, 0, n};
    while (sp) {
        job jb = stack[--sp];
        onode *nd = &S->nodes[jb.node];
        for (int i = 0; i < 3; ++i) { nd->lo[i] = INFINITY; nd->hi[i] = -INFINITY; }
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = jb.first; i < jb.first + jb.count; ++i) {
            int64_t k = S->perm[i];
            for (int a = 0; a < 3; ++a) {
                nd->lo[a] = fmin(nd->lo[a], S->lo[3 * k + a]);
                nd->hi[a] = fmax(nd->hi[a], S->hi[3 * k + a]);
                double c = centroid(S, k, a);
                clo[a] = fmin(clo[a], c);
                chi[a] = fmax(chi[a], c);
            }
        }
        if (jb.count <= 4) {
            nd->left = nd->right = -1;
            nd->first = (int32_t)jb.first;
            nd->count = (int32_t)jb.count;
            continue;
        }
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
        int64_t half = jb.count / 2;
        select_nth(S, S->perm, jb.first, jb.first + jb.count, jb.first + half, axis);
        int64_t l = S->n_nodes++, r = S->n_nodes++;
        nd->left = (int32_t)l;
        nd->right = (int32_t)r;
        nd->first = 0;
        nd->count = 0;
        stack[sp++] = (job){l, jb.first, half};
        stack[sp++] = (job){r, jb.first + half, jb.count - half};
    }
    free(stack);
    return 0;
}

static void gather(const orc_scene *S, const double o[3], const double w[3], double t0, double t1,
                   int64_t exclude, int use_bvh, hitvec *out) {
    out->n = 0;
    ohit h;
    if (!use_bvh || !S->nodes || S->n_nodes == 0) {
        for (int64_t k = 0; k < S->n; ++k)
            if (k != exclude && ray_prim(S, k, o, w, t0, t1, &h)) hv_push(out, &h);
        return;
    }
    int64_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp) {
        const onode *nd = &S->nodes[stack[--sp]];
        if (!box_hit(nd->lo, nd->hi, o, w, t0, t1)) continue;
        if (nd->left < 0) {
            for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
                int64_t k = S->perm[i];
                if (k != exclude && ray_prim(S, k, o, w, t0, t1, &h)) hv_push(out, &h);
            }
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Transmittance (Sec. 4, eq. transmittance): F = 1/2 sum_k I_k(a_k, b_k) over */
/* the clipped chords, T = max(0, 1 - F).  Order independent.                 */
/* ------------------------------------------------------------------------- */
static double accumulated_F(const orc_scene *S, const hitvec *H) {
    double F = 0.0;
    for (int64_t i = 0; i < H->n; ++i) F += seg_integral(S, &H->v[i], H->v[i].a, H->v[i].b);
    return 0.5 * F;
}

/* F(t) = 1/2 sum_k I_k(a_k, min(b_k, t)), the free-flight CDF before clamping */
static double F_at(const orc_scene *S, const hitvec *H, double t) {
    double F = 0.0;
    for (int64_t i = 0; i < H->n; ++i)
        if (H->v[i].a < t) F += seg_integral(S, &H->v[i], H->v[i].a, fmin(H->v[i].b, t));
    return 0.5 * F;
}

/* dF/dt = 1/2 sum of the kernels active at t (eq. free_flight_pdf) */
static double dF_at(const orc_scene *S, const hitvec *H, double t) {
    double g = 0.0;
    for (int64_t i = 0; i < H->n; ++i)
        if (H->v[i].a < t && t < H->v[i].b) g += kernel_at(S, &H->v[i], t);
    return 0.5 * g;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Saturating distance (Sec. 4, below eq. free_flight_pdf; Sec. 4.1 eq.
 * sampling_overlaps with u = 1): the smallest t with F(t) = 1.  F is
 * continuous and non-decreasing; the chord end points split [t0, t1] into
 * pieces on which the active set is fixed.  The first end point with F >= 1
 * brackets the root, F is strictly increasing inside, and a bisection-guarded
 * Newton iteration with dF/dt = 1/2 sum G_k converges to full precision. */
static double solve_tsat(const orc_scene *S, const hitvec *H, double t0) {
    int64_t m = 2 * H->n;
    double *bp = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < H->n; ++i) { bp[2 * i] = H->v[i].a; bp[2 * i + 1] = H->v[i].b; }
    qsort(bp, (size_t)m, sizeof(double), cmp_double);
    double lo = t0, hi = t0;
    for (int64_t i = 0; i < m; ++i) {
        if (bp[i] <= lo) continue;
        if (F_at(S, H, bp[i]) >= 1.0) { hi = bp[i]; break; }
        lo = bp[i];
    }
    free(bp);
    if (!(hi > lo)) return hi;
    double t = 0.5 * (lo + hi);
    for (int it = 0; it < 300; ++it) {
        double f = F_at(S, H, t) - 1.0;
        if (f >= 0.0) hi = t; else lo = t;
        double g = dF_at(S, H, t);
        double tn = (g > 0.0) ? t - f / g : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - t) <= 1e-16 * fmax(1.0, fabs(t)) || hi - lo <= 4e-16 * fmax(1.0, fabs(hi))) {
            t = tn;
            break;
        }
        t = tn;
    }
    return t;
}

void orc_transmittance(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                       int use_bvh, double *F_out, double *T_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        gather(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, use_bvh, &H);
        double F = accumulated_F(S, &H);
        if (F_out) F_out[i] = F;
        if (T_out) T_out[i] = fmax(0.0, 1.0 - F);
    }
    free(H.v);
}

/* F(t) = 1/2 sum_k I_k(a_k, min(b_k, t)) along each ray (t inside [t0, t1]) */
void orc_F_at(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
              const double *t, int use_bvh, double *F_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        gather(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, use_bvh, &H);
        F_out[i] = F_at(S, &H, t[i]);
    }
    free(H.v);
}

void orc_saturation(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                    int use_bvh, double *tsat_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        gather(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, use_bvh, &H);
        double F = accumulated_F(S, &H);
        tsat_out[i] = (F < 1.0) ? (double)r[7] : solve_tsat(S, &H, r[6]);
    }
    free(H.v);
}

/* Radiance-field mode (Sec. 8, eq. rf): with emission and absorption only
 * the radiance along a ray is the sum over the primitives it meets of their
 * free-flight probability up to the saturating distance times their emission,
 *   L = sum_k 1/2 I_k(a_k, min(b_k, t_sat)) L_e,k,
 * with no Monte Carlo (u = 1 exhausts every contributing primitive).  t_sat
 * as orc_saturation unless given (tsat may be NULL).  L_out [n][3]. */
void orc_rf_radiance(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                     const double *tsat, int use_bvh, double *L_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        gather(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, use_bvh, &H);
        double ts;
        if (tsat) ts = tsat[i];
        else ts = accumulated_F(S, &H) < 1.0 ? (double)r[7] : solve_tsat(S, &H, r[6]);
        double L[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < H.n; ++j) {
            const ohit *h = &H.v[j];
            if (!(h->a < ts)) continue;
            const double W = 0.5 * seg_integral(S, h, h->a, fmin(h->b, ts));
            for (int c = 0; c < 3; ++c) L[c] += W * S->emis[3 * h->k + c];
        }
        for (int c = 0; c < 3; ++c) L_out[3 * i + c] = L[c];
    }
    free(H.v);
}

/* Exponential variant (App. D; eq. exp_ff): the same Gaussians as a
 * heterogeneous exponential medium, sigma_t = sum_k G_k, so the optical depth
 * of a ray is sum_k I_k over the clipped chords and T = exp(-depth). */
void orc_exp_transmittance(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                           int use_bvh, double *T_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        gather(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, use_bvh, &H);
        double depth = 0.0;
        for (int64_t j = 0; j < H.n; ++j) depth += seg_integral(S, &H.v[j], H.v[j].a, H.v[j].b);
        T_out[i] = exp(-depth);
    }
    free(H.v);
}

/* The uniform of primitive k on ray i for analog decomposition tracking:
 * Philox4x32-10 with counter (i low, i high, k, 0) and key (seed low, seed
 * high); the top 24 bits of the first word. */
static double exp_uniform(uint64_t seed, int64_t i, int64_t k) {
    const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)k, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    return (double)(x[0] >> 8) * (1.0 / 16777216.0);
}

/* Where the uniform of primitive k comes from in one decomposition-tracking
 * query: ray i of a per-ray query (exp_uniform), or vertex v of a path of the
 * exponential render mode -- counter (pixel, sample, v, 16 + 2k + which)
 * under the path tracer's key, first word, which = 0 for the path's next
 * collision and 1 for its light sample. */
typedef struct {
    int path;
    uint64_t seed;
    int64_t i;
    uint32_t pix, sample, v, which;
} exp_key;

static double exp_u(const exp_key *q, int64_t k) {
    if (!q->path) return exp_uniform(q->seed, q->i, k);
    double u[4];
    rng4(q->seed, q->pix, q->sample, q->v, (uint32_t)(16 + 2 * k + q->which), u);
    return u[0];
}

/* Free-flight sampling of the exponential variant by analog decomposition
 * tracking (App. D, after Kutz et al. 2017): every Gaussian the ray meets
 * draws its own exponential free flight y_k = -ln(1 - u_k); it collides where
 * its optical depth from the chord entry reaches y_k, t_k = I_k^-1(y_k; a_k),
 * if y_k is below its whole chord's depth; the ray collides at the nearest
 * t_k, else escapes (returns -1).  The inversion here is a bisection on the
 * monotone I_k(a_k, t).  margin: the smallest of |y_k - I_k(a_k, b_k)| / y_k
 * and, when two collide, the relative gap of the two nearest t_k. */
static int64_t exp_track(const orc_scene *S, const hitvec *H, const exp_key *q, double *t_out,
                         double *margin_out) {
    double best = INFINITY, second = INFINITY, margin = INFINITY;
    int64_t bk = -1;
    for (int64_t j = 0; j < H->n; ++j) {
        const ohit *h = &H->v[j];
        const double y = -log1p(-exp_u(q, h->k));
        const double total = seg_integral(S, h, h->a, h->b);
        margin = fmin(margin, fabs(y - total) / fmax(y, 1e-30));
        if (!(y < total)) continue;
        double lo = h->a, hi = h->b;
        for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(1.0, fabs(hi)); ++it) {
            const double mid = 0.5 * (lo + hi);
            if (seg_integral(S, h, h->a, mid) < y) lo = mid;
            else hi = mid;
        }
        const double t = 0.5 * (lo + hi);
        if (t < best) {
            second = best;
            best = t;
            bk = h->k;
        } else if (t < second) {
            second = t;
        }
    }
    if (second < INFINITY) margin = fmin(margin, (second - best) / fmax(fabs(best), 1e-30));
    *t_out = bk >= 0 ? best : NAN;
    if (margin_out) *margin_out = margin;
    return bk;
}

void orc_exp_sample(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude, uint64_t seed,
                    int use_bvh, int32_t *prim_out, double *t_out, double *margin_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        gather(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, use_bvh, &H);
        const exp_key q = {0, seed, i, 0, 0, 0, 0};
        prim_out[i] = (int32_t)exp_track(S, &H, &q, &t_out[i], margin_out ? &margin_out[i] : NULL);
    }
    free(H.v);
}

/* ------------------------------------------------------------------------- */
/* Free-flight (primitive) sampling, Sec. 5.2.                                */
/* The paper samples primitive k with probability equal to its share of the   */
/* free-flight pdf up to the saturating distance:                             */
/*   W_k = 1/2 I_k(a_k, min(b_k, t_sat)),  P(escape) = 1 - sum W = T(t1).     */
/* One uniform u picks an outcome by walking a fixed ordering of H and        */
/* returning the first k whose running sum of W exceeds u.  The ordering is   */
/* canonical (independent of any tree): exit order, key (min(b_k, t_sat), k), */
/* so primitives that straddle t_sat come last, by index.  The disambiguation */
/* step of Sec. 5.2 is subsumed: straddlers get their exact clipped weights.  */
/* ------------------------------------------------------------------------- */
typedef struct {
    double key;
    int64_t k;
    double W, a, b;
} wentry;

static int cmp_wentry(const void *x, const void *y) {
    const wentry *a = (const wentry *)x, *b = (const wentry *)y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->k > b->k) - (a->k < b->k);
}

typedef struct {
    int64_t prim;
    double t_hit, F_end, t_sat, margin, W_total;
} ocoll;

static void collide(const orc_scene *S, const hitvec *H, double t0, double t1, double u, ocoll *c) {
    double Fend = accumulated_F(S, H);
    double tsat = (Fend < 1.0) ? t1 : solve_tsat(S, H, t0);
    wentry *E = (wentry *)malloc(sizeof(wentry) * (size_t)(H->n > 0 ? H->n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < H->n; ++i) {
        const ohit *h = &H->v[i];
        if (!(h->a < tsat)) continue;
        double e = fmin(h->b, tsat);
        E[m].key = e;
        E[m].k = h->k;
        E[m].W = 0.5 * seg_integral(S, h, h->a, e);
        E[m].a = h->a;
        E[m].b = h->b;
        ++m;
    }
    qsort(E, (size_t)m, sizeof(wentry), cmp_wentry);
    c->prim = -1;
    c->t_hit = NAN;
    c->F_end = Fend;
    c->t_sat = tsat;
    double run = 0.0, margin = fabs(u);
    for (int64_t i = 0; i < m; ++i) {
        run += E[i].W;
        margin = fmin(margin, fabs(u - run));
        if (c->prim < 0 && run > u) {
            c->prim = E[i].k;
            c->t_hit = 0.5 * (E[i].a + E[i].b);
        }
    }
    c->margin = margin;
    c->W_total = run;
    free(E);
}

void orc_sample_collision(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                          const double *u, int use_bvh, int32_t *prim_out, double *t_out,
                          double *F_out, double *tsat_out, double *margin_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        gather(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, use_bvh, &H);
        ocoll c;
        collide(S, &H, r[6], r[7], u[i], &c);
        if (prim_out) prim_out[i] = (int32_t)c.prim;
        if (t_out) t_out[i] = c.t_hit;
        if (F_out) F_out[i] = c.F_end;
        if (tsat_out) tsat_out[i] = c.t_sat;
        if (margin_out) margin_out[i] = c.margin;
    }
    free(H.v);
}

/* Emission carried by primitive k along a ray (eq. rte: emission rides on the
 * free-flight pdf, so k contributes 1/2 L_e int_0^{t_sat} G_k dt).  The ray is
 * (x, w, 0, b_k) with b_k the exit of k's chord; t_sat is taken over every
 * primitive except `exclude`, k included.  Returns the factor multiplying
 * L_e: 1/2 I_k(a_k, min(b_k, t_sat)), 0 when the ray misses k.  The ray is
 * clipped to [t0, min(t1, b_k)]. */
static double emitter_factor(const orc_scene *S, const double x[3], const double w[3], double t0,
                             double t1, int64_t exclude, int64_t k, int use_bvh, hitvec *H) {
    ohit hk;
    if (k < 0 || k >= S->n || k == exclude || !ray_prim(S, k, x, w, t0, t1, &hk)) return 0.0;
    double tend = hk.b;
    gather(S, x, w, t0, tend, exclude, use_bvh, H);
    double F = accumulated_F(S, H);
    double tsat = (F < 1.0) ? tend : solve_tsat(S, H, t0);
    if (!(hk.a < tsat)) return 0.0;
    return 0.5 * seg_integral(S, &hk, hk.a, fmin(hk.b, tsat));
}

void orc_emitter_query(const orc_scene *S, int64_t n, const float *rays, const int32_t *exclude,
                       const int32_t *target, int use_bvh, double *L_out) {
    hitvec H = {0};
    for (int64_t i = 0; i < n; ++i) {
        const float *r = rays + 8 * i;
        double o[3] = {r[0], r[1], r[2]}, w[3] = {r[3], r[4], r[5]};
        L_out[i] = emitter_factor(S, o, w, r[6], r[7], exclude ? exclude[i] : -1, target[i], use_bvh, &H);
    }
    free(H.v);
}

/* ------------------------------------------------------------------------- */
/* Phase function in the delta-NDF limit (Sec. 6: with a single facet normal  */
/* eq. phase_function reduces to the surface BSDF times the foreshortening    */
/* cosine).  Normal n = R e_argmin(s), flipped toward w_o; reflection only.   */
/*   Lambert:  f = albedo/pi cos_i,             pdf = cos_i/pi                */
/*   GGX:      f = F D G2 / (4 cos_o),          pdf = G1(w_o) D(h) / (4 cos_o) */
/* with alpha = roughness^2 (floored at 1e-4), height-correlated Smith G2,    */
/* Schlick Fresnel with F0 = albedo, sampling by visible normals (Heitz,      */
/* "Sampling the GGX Distribution of Visible Normals", JCGT 2018).            */
/* All vectors are in the local frame (z = n).                                */
/* ------------------------------------------------------------------------- */
static double ggx_alpha(double rough) { return fmax(rough * rough, 1e-4); }

static double ggx_D(double a, double cos_h) {
    double a2 = a * a;
    double t = cos_h * cos_h * (a2 - 1.0) + 1.0;
    return a2 / (M_PI * t * t);
}

static double ggx_lambda(double a, double c) {
    double c2 = c * c;
    double tan2 = fmax(0.0, 1.0 - c2) / c2;
    return 0.5 * (-1.0 + sqrt(1.0 + a * a * tan2));
}

/* local-frame eval; returns f (rgb) and the sampling pdf */
static void phase_eval_local(int mat, const double alb[3], double rough, const double wo[3],
                             const double wi[3], double f[3], double *pdf) {
    f[0] = f[1] = f[2] = 0.0;
    *pdf = 0.0;
    if (wo[2] <= 0.0 || wi[2] <= 0.0) return;
    if (mat == 0) {
        for (int c = 0; c < 3; ++c) f[c] = alb[c] / M_PI * wi[2];
        *pdf = wi[2] / M_PI;
        return;
    }
    double a = ggx_alpha(rough);
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    normalize3(h);
    double D = ggx_D(a, h[2]);
    double lo = ggx_lambda(a, wo[2]), li = ggx_lambda(a, wi[2]);
    double G2 = 1.0 / (1.0 + lo + li), G1 = 1.0 / (1.0 + lo);
    double c = dot3(wi, h);
    double sch = pow(1.0 - fmax(0.0, c), 5.0);
    for (int k = 0; k < 3; ++k) {
        double F = alb[k] + (1.0 - alb[k]) * sch;
        f[k] = F * D * G2 / (4.0 * wo[2]);
    }
    *pdf = G1 * D / (4.0 * wo[2]);
}

/* local-frame sample; returns wi, weight f/pdf and pdf (pdf 0 = no sample) */
static void phase_sample_local(int mat, const double alb[3], double rough, const double wo[3],
                               double u1, double u2, double wi[3], double wgt[3], double *pdf) {
    wgt[0] = wgt[1] = wgt[2] = 0.0;
    *pdf = 0.0;
    if (wo[2] <= 0.0) return;
    if (mat == 0) {
        double rr = sqrt(u1), ph = 2.0 * M_PI * u2;
        wi[0] = rr * cos(ph);
        wi[1] = rr * sin(ph);
        wi[2] = sqrt(fmax(0.0, 1.0 - u1));
        if (wi[2] <= 0.0) return;
        *pdf = wi[2] / M_PI;
        for (int c = 0; c < 3; ++c) wgt[c] = alb[c];
        return;
    }
    double a = ggx_alpha(rough);
    /* visible-normal sampling: stretch, sample the projected hemisphere, unstretch */
    double Vh[3] = {a * wo[0], a * wo[1], wo[2]};
    normalize3(Vh);
    double lensq = Vh[0] * Vh[0] + Vh[1] * Vh[1];
    double T1[3];
    if (lensq > 0.0) {
        double il = 1.0 / sqrt(lensq);
        T1[0] = -Vh[1] * il; T1[1] = Vh[0] * il; T1[2] = 0.0;
    } else {
        T1[0] = 1.0; T1[1] = 0.0; T1[2] = 0.0;
    }
    double T2[3];
    cross3(Vh, T1, T2);
    double rr = sqrt(u1), ph = 2.0 * M_PI * u2;
    double p1 = rr * cos(ph), p2 = rr * sin(ph);
    double sv = 0.5 * (1.0 + Vh[2]);
    p2 = (1.0 - sv) * sqrt(fmax(0.0, 1.0 - p1 * p1)) + sv * p2;
    double p3 = sqrt(fmax(0.0, 1.0 - p1 * p1 - p2 * p2));
    double Nh[3];
    for (int i = 0; i < 3; ++i) Nh[i] = p1 * T1[i] + p2 * T2[i] + p3 * Vh[i];
    double h[3] = {a * Nh[0], a * Nh[1], fmax(0.0, Nh[2])};
    normalize3(h);
    double c = dot3(wo, h);
    for (int i = 0; i < 3; ++i) wi[i] = 2.0 * c * h[i] - wo[i];
    if (wi[2] <= 0.0) return;
    double D = ggx_D(a, h[2]);
    double lo = ggx_lambda(a, wo[2]), li = ggx_lambda(a, wi[2]);
    double G2 = 1.0 / (1.0 + lo + li), G1 = 1.0 / (1.0 + lo);
    *pdf = G1 * D / (4.0 * wo[2]);
    double sch = pow(1.0 - fmax(0.0, c), 5.0);
    for (int k = 0; k < 3; ++k) {
        double F = alb[k] + (1.0 - alb[k]) * sch;
        wgt[k] = F * G2 / G1;
    }
}

static void to_local(const double b1[3], const double b2[3], const double n[3], const double v[3],
                     double l[3]) {
    l[0] = dot3(v, b1); l[1] = dot3(v, b2); l[2] = dot3(v, n);
}

/* world-frame wrappers: n is the stored facet normal, flipped toward wo */
static void facet_frame(const double nrm[3], const double wo[3], double n[3], double b1[3],
                        double b2[3]) {
    double s = dot3(nrm, wo) >= 0.0 ? 1.0 : -1.0;
    n[0] = s * nrm[0]; n[1] = s * nrm[1]; n[2] = s * nrm[2];
    onb(n, b1, b2);
}

void orc_phase_eval(int mat, const double alb[3], double rough, const double nrm[3],
                    const double wo[3], const double wi[3], double f[3], double *pdf) {
    double n[3], b1[3], b2[3], lo[3], li[3];
    facet_frame(nrm, wo, n, b1, b2);
    to_local(b1, b2, n, wo, lo);
    to_local(b1, b2, n, wi, li);
    phase_eval_local(mat, alb, rough, lo, li, f, pdf);
}

void orc_phase_sample(int mat, const double alb[3], double rough, const double nrm[3],
                      const double wo[3], double u1, double u2, double wi[3], double wgt[3],
                      double *pdf) {
    double n[3], b1[3], b2[3], lo[3], li[3] = {0.0, 0.0, 0.0};
    facet_frame(nrm, wo, n, b1, b2);
    to_local(b1, b2, n, wo, lo);
    phase_sample_local(mat, alb, rough, lo, u1, u2, li, wgt, pdf);
    for (int i = 0; i < 3; ++i) wi[i] = li[0] * b1[i] + li[1] * b2[i] + li[2] * n[i];
}

/* ------------------------------------------------------------------------- */
/* SGGX microflake phase function (Sec. 4.2, eq. vndf and eq. phase_function) */
/* with a Lambertian base BSDF.  The NDF of a symmetric positive-definite S   */
/* (Heitz et al. 2015) is D(n) = 1 / (pi sqrt(det S) (n^T S^-1 n)^2); the     */
/* projected area is sigma(w) = sqrt(w^T S w); the visible NDF is             */
/* D_wo(n) = <wo.n> D(n) / sigma(wo).  f_p(wi, wo) = int D_wo(n) f(wi; n) dn  */
/* with the cosine-weighted Lambert f(wi; n) = albedo/pi <wi.n>.  Functions  */
/* below are per unit albedo.                                                 */
/* ------------------------------------------------------------------------- */

static void sggx_full(const double s6[6], double S[3][3]) {
    S[0][0] = s6[0]; S[1][1] = s6[1]; S[2][2] = s6[2];
    S[0][1] = S[1][0] = s6[3]; S[0][2] = S[2][0] = s6[4]; S[1][2] = S[2][1] = s6[5];
}

/* inverse and determinant of a symmetric 3x3 (cofactors) */
static double inv3(const double A[3][3], double Ai[3][3]) {
    double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    double id = 1.0 / det;
    Ai[0][0] = c00 * id; Ai[1][0] = c01 * id; Ai[2][0] = c02 * id;
    Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    return det;
}

static double quad_form(const double A[3][3], const double v[3]) {
    double r = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r += v[i] * A[i][j] * v[j];
    return r;
}

double orc_sggx_sigma(const double s6[6], const double w[3]) {
    double S[3][3];
    sggx_full(s6, S);
    return sqrt(fmax(0.0, quad_form(S, w)));
}

double orc_sggx_D(const double s6[6], const double n[3]) {
    double S[3][3], Si[3][3];
    sggx_full(s6, S);
    double det = inv3(S, Si);
    double q = quad_form(Si, n);
    return 1.0 / (M_PI * sqrt(det) * q * q);
}

double orc_sggx_vndf(const double s6[6], const double wo[3], const double n[3]) {
    double c = dot3(wo, n);
    if (c <= 0.0) return 0.0;
    return c * orc_sggx_D(s6, n) / orc_sggx_sigma(s6, wo);
}

/* A visible normal: the microflakes' normals are those of the ellipsoid
 * x^T S x = 1 (its projected area along w is proportional to
 * sqrt(w^T S w)), and the visible ones, weighted by projected area, are the
 * normals at the front surface above a point uniform in the ellipsoid's
 * shadow along wo.  The shadow of {B y : |y| <= 1} (B B^T = S^-1) on the
 * plane of an orthonormal pair (e1, e2) orthogonal to wo is the ellipse of
 * the 2x2 matrix [e_a^T S^-1 e_b]: a point u uniform in the unit disk maps
 * to q = L u (L its Cholesky factor); the front surface point is q + s wo
 * with s the larger root of (q + s wo)^T S (q + s wo) = 1; its normal is
 * S x normalised. */
void orc_sggx_sample_vndf(const double s6[6], const double wo[3], double u1, double u2, double n[3]) {
    double S[3][3], Si[3][3], e1[3], e2[3];
    sggx_full(s6, S);
    inv3(S, Si);
    onb(wo, e1, e2);
    double s11 = quad_form(Si, e1), s22 = quad_form(Si, e2), s12 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s12 += e1[i] * Si[i][j] * e2[j];
    double l11 = sqrt(s11), l21 = s12 / l11, l22 = sqrt(fmax(0.0, s22 - l21 * l21));
    double r = sqrt(u1), ph = 2.0 * M_PI * u2;
    double a = r * cos(ph), b = r * sin(ph);
    double qa = l11 * a, qb = l21 * a + l22 * b;
    double q[3];
    for (int i = 0; i < 3; ++i) q[i] = qa * e1[i] + qb * e2[i];
    double A = quad_form(S, wo), B = 0.0, Cq = quad_form(S, q) - 1.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B += q[i] * S[i][j] * wo[j];
    double sroot = (-B + sqrt(fmax(0.0, B * B - A * Cq))) / A;
    double x[3];
    for (int i = 0; i < 3; ++i) x[i] = q[i] + sroot * wo[i];
    for (int i = 0; i < 3; ++i) n[i] = S[i][0] * x[0] + S[i][1] * x[1] + S[i][2] * x[2];
    normalize3(n);
}

/* a direction cosine-distributed about the unit vector m */
static void cosine_about(const double m[3], double u1, double u2, double w[3]) {
    double b1[3], b2[3];
    onb(m, b1, b2);
    double r = sqrt(u1), ph = 2.0 * M_PI * u2, z = sqrt(fmax(0.0, 1.0 - u1));
    for (int i = 0; i < 3; ++i) w[i] = r * cos(ph) * b1[i] + r * sin(ph) * b2[i] + z * m[i];
}

/* The stochastic evaluation of f_p (Sec. 4.2, "Evaluation"): one normal from
 * the visible NDF and one from the base BSDF's sampling reversed (for the
 * Lambertian base: cosine-distributed about wi), combined by the one-sample
 * balance heuristic.  u[0..1] drive the first, u[2..3] the second.  An
 * unbiased estimate of f_p / albedo. */
double orc_sggx_phase_est(const double s6[6], const double wo[3], const double wi[3], const double u[4]) {
    double n1[3], n3[3];
    orc_sggx_sample_vndf(s6, wo, u[0], u[1], n1);
    double p1 = orc_sggx_vndf(s6, wo, n1);
    double f1 = fmax(0.0, dot3(wi, n1)) / M_PI; /* base f(wi; n1), also n1's density about wi */
    double est = p1 > 0.0 ? f1 * p1 / (p1 + f1) : 0.0;
    cosine_about(wi, u[2], u[3], n3);
    double p3 = orc_sggx_vndf(s6, wo, n3);
    double c3 = fmax(0.0, dot3(n3, wi)) / M_PI;
    if (c3 > 0.0 && p3 > 0.0) est += p3 * c3 / (c3 + p3);
    return est;
}

/* f_p / albedo by quadrature on a (cos theta, phi) midpoint grid: the plain
 * definition, for checks */
double orc_sggx_phase_quad(const double s6[6], const double wo[3], const double wi[3], int nz, int nphi) {
    double acc = 0.0;
    for (int a = 0; a < nz; ++a) {
        double z = -1.0 + (a + 0.5) * 2.0 / nz, rr = sqrt(fmax(0.0, 1.0 - z * z));
        for (int b = 0; b < nphi; ++b) {
            double ph = (b + 0.5) * 2.0 * M_PI / nphi;
            double n[3] = {rr * cos(ph), rr * sin(ph), z};
            acc += orc_sggx_vndf(s6, wo, n) * fmax(0.0, dot3(wi, n)) / M_PI;
        }
    }
    return acc * (2.0 / nz) * (2.0 * M_PI / nphi);
}

/* The approximate MIS pdf of the Lambertian component (App. B): a
 * cosine-weighted lobe of the half vector, <wh.wo>/pi. */
double orc_sggx_pdf_approx(const double wo[3], const double wi[3]) {
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    double l = sqrt(dot3(h, h));
    if (!(l > 0.0)) return 0.0;
    return fmax(0.0, dot3(h, wo) / l) / M_PI;
}

/* ------------------------------------------------------------------------- */
/* SGGX microflakes with a Disney-style base BSDF (material 3; Sec. 4.2: a    */
/* microfacet specular component and a diffuse component with empirical       */
/* retro-reflection, Burley 2012/2015).  The base BSDF at a flake normal n,   */
/* cosine-weighted, for base colour c, roughness r (alpha = r^2 for the       */
/* specular lobe, r itself in the diffuse retro-reflection) and metallic m:   */
/*   specular: F D G2 / (4 <n.wo>), GGX D and height-correlated Smith G2 in   */
/*             the frame of n, Schlick F with F0 = 0.04 (1 - m) + c m;        */
/*   diffuse : (1 - m) c / pi (1 + (F_D90 - 1)(1 - <n.wi>)^5)                 */
/*             (1 + (F_D90 - 1)(1 - <n.wo>)^5) <n.wi>,                        */
/*             F_D90 = 1/2 + 2 r <wi.h>^2;                                    */
/* zero unless wi and wo are both on the side of n.                           */
/* ------------------------------------------------------------------------- */

static void disney_base(const double c[3], double rough, double met, const double n[3], const double wo[3],
                        const double wi[3], double fs[3], double fd[3]) {
    double b1[3], b2[3], lo[3], li[3];
    for (int k = 0; k < 3; ++k) fs[k] = fd[k] = 0.0;
    onb(n, b1, b2);
    to_local(b1, b2, n, wo, lo);
    to_local(b1, b2, n, wi, li);
    if (lo[2] <= 0.0 || li[2] <= 0.0) return;
    double a = ggx_alpha(rough);
    double h[3] = {lo[0] + li[0], lo[1] + li[1], lo[2] + li[2]};
    normalize3(h);
    double D = ggx_D(a, h[2]);
    double G2 = 1.0 / (1.0 + ggx_lambda(a, lo[2]) + ggx_lambda(a, li[2]));
    double cd = fmax(0.0, dot3(li, h));
    double sch = pow(1.0 - cd, 5.0);
    double fd90 = 0.5 + 2.0 * rough * cd * cd;
    double rl = 1.0 + (fd90 - 1.0) * pow(1.0 - li[2], 5.0), rv = 1.0 + (fd90 - 1.0) * pow(1.0 - lo[2], 5.0);
    for (int k = 0; k < 3; ++k) {
        double F0 = 0.04 * (1.0 - met) + c[k] * met;
        fs[k] = (F0 + (1.0 - F0) * sch) * D * G2 / (4.0 * lo[2]);
        fd[k] = (1.0 - met) * c[k] / M_PI * rl * rv * li[2];
    }
}

/* probability of choosing the specular lobe when sampling the base BSDF:
 * weights 1 (specular) and (1 - m) times the base colour's luminance (diffuse) */
double orc_disney_spec_prob(const double c[3], double met) {
    double lum = 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2];
    return 1.0 / (1.0 + (1.0 - met) * lum);
}

/* pdf of sampling the base BSDF at n: the lobe mixture of GGX visible-normal
 * reflection, G1(wo) D / (4 <n.wo>), and cosine sampling, <n.wi> / pi */
static double disney_base_pdf(double ps, double rough, const double n[3], const double wo[3], const double wi[3]) {
    double b1[3], b2[3], lo[3], li[3];
    onb(n, b1, b2);
    to_local(b1, b2, n, wo, lo);
    to_local(b1, b2, n, wi, li);
    if (lo[2] <= 0.0 || li[2] <= 0.0) return 0.0;
    double a = ggx_alpha(rough);
    double h[3] = {lo[0] + li[0], lo[1] + li[1], lo[2] + li[2]};
    normalize3(h);
    double G1 = 1.0 / (1.0 + ggx_lambda(a, lo[2]));
    return ps * G1 * ggx_D(a, h[2]) / (4.0 * lo[2]) + (1.0 - ps) * li[2] / M_PI;
}

/* a normal n about the half vector h with density D(<n.h>) <n.h> (the GGX
 * normal distribution's own sampling, Walter et al. 2007, with the roles of
 * normal and half vector exchanged) */
static void ggx_ndf_about(const double h[3], double a, double u1, double u2, double n[3]) {
    double b1[3], b2[3];
    onb(h, b1, b2);
    double t2 = a * a * u1 / (1.0 - u1);
    double ct = 1.0 / sqrt(1.0 + t2), st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * M_PI * u2;
    for (int i = 0; i < 3; ++i) n[i] = st * cos(ph) * b1[i] + st * sin(ph) * b2[i] + ct * h[i];
}

/* Improved stochastic evaluation of f_p (Sec. 4.2, "Evaluation"): per lobe,
 * one normal from the visible NDF (u0, u1) combined by the one-sample balance
 * heuristic with one normal from the lobe's own sampling reversed -- for the
 * specular lobe a GGX normal about the half vector (u2, u3), for the diffuse
 * lobe a normal cosine-distributed about wi (u4, u5).  f[3] = estimate. */
void orc_sggx_disney_est(const double s6[6], const double c[3], double rough, double met, const double wo[3],
                         const double wi[3], const double u[6], double f[3]) {
    double a = ggx_alpha(rough);
    double n1[3], n2[3], n3[3], fs[3], fd[3], h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    for (int k = 0; k < 3; ++k) f[k] = 0.0;
    orc_sggx_sample_vndf(s6, wo, u[0], u[1], n1);
    double p1 = orc_sggx_vndf(s6, wo, n1);
    if (p1 > 0.0) {
        disney_base(c, rough, met, n1, wo, wi, fs, fd);
        double hl = sqrt(dot3(h, h)), hn = 0.0;
        if (hl > 0.0) hn = dot3(h, n1) / hl;
        double pm = hn > 0.0 ? ggx_D(a, hn) * hn : 0.0;
        double pc = fmax(0.0, dot3(wi, n1)) / M_PI;
        for (int k = 0; k < 3; ++k) f[k] += fs[k] * p1 / (p1 + pm) + fd[k] * p1 / (p1 + pc);
    }
    double hl = sqrt(dot3(h, h));
    if (hl > 0.0) {
        for (int i = 0; i < 3; ++i) h[i] /= hl;
        ggx_ndf_about(h, a, u[2], u[3], n2);
        double hn = dot3(n2, h);
        double p2 = hn > 0.0 ? ggx_D(a, hn) * hn : 0.0;
        double v2 = orc_sggx_vndf(s6, wo, n2);
        if (p2 > 0.0 && v2 > 0.0) {
            disney_base(c, rough, met, n2, wo, wi, fs, fd);
            for (int k = 0; k < 3; ++k) f[k] += v2 * fs[k] / (p2 + v2);
        }
    }
    cosine_about(wi, u[4], u[5], n3);
    double p3 = fmax(0.0, dot3(n3, wi)) / M_PI;
    double v3 = orc_sggx_vndf(s6, wo, n3);
    if (p3 > 0.0 && v3 > 0.0) {
        disney_base(c, rough, met, n3, wo, wi, fs, fd);
        for (int k = 0; k < 3; ++k) f[k] += v3 * fd[k] / (p3 + v3);
    }
}

/* Importance sampling (Sec. 4.2): a visible normal n (u0, u1), then the base
 * BSDF at n: the specular lobe with probability ps (GGX visible normals of n,
 * v1, v2, reflected) else cosine about n (v1, v2), chosen by v0.  Weight =
 * base f / mixture pdf (zero below n).  Returns 0 when no direction. */
int orc_sggx_disney_sample(const double s6[6], const double c[3], double rough, double met, const double wo[3],
                           double u0, double u1, const double v[3], double wi[3], double wgt[3]) {
    double n[3], b1[3], b2[3], lo[3], li[3], fs[3], fd[3], dummy[3], dp;
    double ps = orc_disney_spec_prob(c, met);
    for (int k = 0; k < 3; ++k) wgt[k] = 0.0;
    orc_sggx_sample_vndf(s6, wo, u0, u1, n);
    if (v[0] < ps) {
        onb(n, b1, b2);
        to_local(b1, b2, n, wo, lo);
        double one[3] = {1.0, 1.0, 1.0};
        phase_sample_local(1, one, rough, lo, v[1], v[2], li, dummy, &dp);
        if (!(dp > 0.0)) { wi[0] = wi[1] = 0.0; wi[2] = 1.0; return 0; }
        for (int i = 0; i < 3; ++i) wi[i] = li[0] * b1[i] + li[1] * b2[i] + li[2] * n[i];
    } else {
        cosine_about(n, v[1], v[2], wi);
    }
    double pdf = disney_base_pdf(ps, rough, n, wo, wi);
    if (!(pdf > 0.0)) return 0;
    disney_base(c, rough, met, n, wo, wi, fs, fd);
    for (int k = 0; k < 3; ++k) wgt[k] = (fs[k] + fd[k]) / pdf;
    return 1;
}

/* Symmetric eigen-decomposition by cyclic Jacobi rotations: eigenvalues w,
 * eigenvectors in the columns of V. */
static void jacobi3(const double A0[3][3], double w[3], double V[3][3]) {
    double A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) { A[i][j] = A0[i][j]; V[i][j] = i == j ? 1.0 : 0.0; }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        if (off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                double th = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
                double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {  /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq; A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {  /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk; A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = cs * vkp - sn * vkq; V[k][q] = sn * vkp + cs * vkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

/* The roughened SGGX of App. B: eigenvalues (s1 + a^2 s3, s2 + a^2 s3, s3)
 * for the eigenvalues s1 <= s2 <= s3 of S, same eigenvectors:
 * S~ = S + a^2 s3 (I - v3 v3^T) with v3 the eigenvector of s3. */
void orc_sggx_roughened(const double s6[6], double rough, double out6[6]) {
    double S[3][3], V[3][3], w[3];
    sggx_full(s6, S);
    jacobi3(S, w, V);
    int t = 0;
    if (w[1] > w[t]) t = 1;
    if (w[2] > w[t]) t = 2;
    double a = ggx_alpha(rough), cc = a * a * w[t];
    double v[3] = {V[0][t], V[1][t], V[2][t]};
    double R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = S[i][j] + cc * ((i == j ? 1.0 : 0.0) - v[i] * v[j]);
    out6[0] = R[0][0]; out6[1] = R[1][1]; out6[2] = R[2][2];
    out6[3] = R[0][1]; out6[4] = R[0][2]; out6[5] = R[1][2];
}

/* Approximate MIS pdf (App. B): ps times the roughened SGGX's visible NDF at
 * the half vector plus (1 - ps) times <w_h . w_o> / pi. */
double orc_sggx_disney_pdf_approx(const double s6[6], const double c[3], double rough, double met,
                                  const double wo[3], const double wi[3]) {
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    double l = sqrt(dot3(h, h));
    if (!(l > 0.0)) return 0.0;
    for (int i = 0; i < 3; ++i) h[i] /= l;
    double r6[6];
    orc_sggx_roughened(s6, rough, r6);
    double ps = orc_disney_spec_prob(c, met);
    return ps * orc_sggx_vndf(r6, wo, h) + (1.0 - ps) * fmax(0.0, dot3(h, wo)) / M_PI;
}

/* f_p of material 3 by quadrature on a (cos theta, phi) midpoint grid of normals */
void orc_sggx_disney_quad(const double s6[6], const double c[3], double rough, double met, const double wo[3],
                          const double wi[3], int nz, int nphi, double f[3]) {
    double acc[3] = {0.0, 0.0, 0.0}, fs[3], fd[3];
    for (int a = 0; a < nz; ++a) {
        double z = -1.0 + (a + 0.5) * 2.0 / nz, rr = sqrt(fmax(0.0, 1.0 - z * z));
        for (int b = 0; b < nphi; ++b) {
            double ph = (b + 0.5) * 2.0 * M_PI / nphi;
            double n[3] = {rr * cos(ph), rr * sin(ph), z};
            double dv = orc_sggx_vndf(s6, wo, n);
            if (dv <= 0.0) continue;
            disney_base(c, rough, met, n, wo, wi, fs, fd);
            for (int k = 0; k < 3; ++k) acc[k] += dv * (fs[k] + fd[k]);
        }
    }
    for (int k = 0; k < 3; ++k) f[k] = acc[k] * (2.0 / nz) * (2.0 * M_PI / nphi);
}

/* the base BSDF alone at a given normal (for checks): fs, fd */
void orc_disney_base(const double c[3], double rough, double met, const double n[3], const double wo[3],
                     const double wi[3], double fs[3], double fd[3]) {
    disney_base(c, rough, met, n, wo, wi, fs, fd);
}

/* metallic per primitive (copied; values outside [0, 1] rejected) */
int orc_scene_set_metallic(orc_scene *S, const float *met) {
    if (!S || !met) return 1;
    for (int64_t k = 0; k < S->n; ++k)
        if (!(met[k] >= 0.0f && met[k] <= 1.0f)) return 1;
    free(S->met);
    S->met = (double *)malloc(sizeof(double) * (size_t)(S->n > 0 ? S->n : 1));
    for (int64_t k = 0; k < S->n; ++k) S->met[k] = met[k];
    return 0;
}

/* Copies the matrices; returns 1 (and keeps none) unless every one is finite
 * and positive definite (Sylvester: leading minors > 0). */
int orc_scene_set_sggx(orc_scene *S, const float *sggx) {
    if (!S || !sggx) return 1;
    for (int64_t k = 0; k < S->n; ++k) {
        double A[3][3], s6[6];
        for (int i = 0; i < 6; ++i) s6[i] = sggx[6 * k + i];
        sggx_full(s6, A);
        double m2 = A[0][0] * A[1][1] - A[0][1] * A[0][1];
        double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[1][2]) - A[0][1] * (A[0][1] * A[2][2] - A[1][2] * A[0][2]) +
                     A[0][2] * (A[0][1] * A[1][2] - A[1][1] * A[0][2]);
        if (!(A[0][0] > 0.0) || !(m2 > 0.0) || !(det > 0.0) || !isfinite(det)) return 1;
    }
    free(S->sggx);
    S->sggx = (double *)malloc(sizeof(double) * 6 * (size_t)(S->n > 0 ? S->n : 1));
    for (int64_t i = 0; i < 6 * S->n; ++i) S->sggx[i] = sggx[i];
    return 0;
}

/* Phase function of primitive k for (wo, wi): the delta-NDF materials in
 * closed form with their exact pdf; SGGX microflakes (material 2) by the
 * stochastic estimate from u[0..3] with the approximate MIS pdf. */
static void prim_phase_eval(const orc_scene *S, int64_t k, const double wo[3], const double wi[3],
                            const double u[6], double f[3], double *pdf) {
    const double *alb = S->alb + 3 * k;
    if (S->mat[k] == 3) {
        if (!S->sggx) { f[0] = f[1] = f[2] = 0.0; *pdf = 0.0; return; }
        double met = S->met ? S->met[k] : 0.0;
        orc_sggx_disney_est(S->sggx + 6 * k, alb, S->rough[k], met, wo, wi, u, f);
        *pdf = orc_sggx_disney_pdf_approx(S->sggx + 6 * k, alb, S->rough[k], met, wo, wi);
        return;
    }
    if (S->mat[k] == 2) {
        if (!S->sggx) { f[0] = f[1] = f[2] = 0.0; *pdf = 0.0; return; }
        double e = orc_sggx_phase_est(S->sggx + 6 * k, wo, wi, u);
        for (int c = 0; c < 3; ++c) f[c] = alb[c] * e;
        *pdf = orc_sggx_pdf_approx(wo, wi);
        return;
    }
    orc_phase_eval(S->mat[k], alb, S->rough[k], S->nrm + 3 * k, wo, wi, f, pdf);
}

/* Sampling the phase function of primitive k (Sec. 4.2, "Importance
 * Sampling"): for SGGX microflakes a visible normal from (u1, u2), then the
 * base BSDF's sampling about it from v (Lambertian: cosine from v[0..1], the
 * weight is the albedo; Disney-style: lobe choice v[0], direction v[1..2],
 * the weight f / pdf of the base); the pdf reported for MIS is the
 * approximate one. */
static void prim_phase_sample(const orc_scene *S, int64_t k, const double wo[3], double u1, double u2,
                              const double v[3], double wi[3], double wgt[3], double *pdf) {
    const double *alb = S->alb + 3 * k;
    if (S->mat[k] == 3) {
        *pdf = 0.0;
        if (!S->sggx) return;
        double met = S->met ? S->met[k] : 0.0;
        if (!orc_sggx_disney_sample(S->sggx + 6 * k, alb, S->rough[k], met, wo, u1, u2, v, wi, wgt)) return;
        *pdf = orc_sggx_disney_pdf_approx(S->sggx + 6 * k, alb, S->rough[k], met, wo, wi);
        return;
    }
    if (S->mat[k] == 2) {
        double m[3];
        if (!S->sggx) { *pdf = 0.0; return; }
        orc_sggx_sample_vndf(S->sggx + 6 * k, wo, u1, u2, m);
        cosine_about(m, v[0], v[1], wi);
        for (int c = 0; c < 3; ++c) wgt[c] = alb[c];
        *pdf = orc_sggx_pdf_approx(wo, wi);
        return;
    }
    orc_phase_sample(S->mat[k], alb, S->rough[k], S->nrm + 3 * k, wo, u1, u2, wi, wgt, pdf);
}

/* vectorised forms for the checks: n directions or normals in, n values out */
void orc_sggx_eval_n(const double s6[6], int64_t n, const double *wo, const double *v, int what, double *out) {
    for (int64_t i = 0; i < n; ++i) {
        if (what == 0) out[i] = orc_sggx_sigma(s6, v + 3 * i);
        else if (what == 1) out[i] = orc_sggx_D(s6, v + 3 * i);
        else out[i] = orc_sggx_vndf(s6, wo, v + 3 * i);
    }
}

void orc_sggx_sample_vndf_n(const double s6[6], const double wo[3], int64_t n, const double *u, double *nrm) {
    for (int64_t i = 0; i < n; ++i) orc_sggx_sample_vndf(s6, wo, u[2 * i], u[2 * i + 1], nrm + 3 * i);
}

/* importance samples: visible normal from u[0..1], then cosine about it from u[2..3] */
void orc_sggx_sample_dir_n(const double s6[6], const double wo[3], int64_t n, const double *u, double *wi) {
    for (int64_t i = 0; i < n; ++i) {
        double m[3];
        orc_sggx_sample_vndf(s6, wo, u[4 * i], u[4 * i + 1], m);
        cosine_about(m, u[4 * i + 2], u[4 * i + 3], wi + 3 * i);
    }
}

void orc_sggx_phase_est_n(const double s6[6], const double wo[3], const double wi[3], int64_t n, const double *u,
                          double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = orc_sggx_phase_est(s6, wo, wi, u + 4 * i);
}

/* ------------------------------------------------------------------------- */
/* Path tracer (Sec. 5, Table tab:highlevel, right column; eq. rte), with     */
/* next-event estimation to emissive primitives and to a constant environment */
/* and the balance heuristic between light and phase sampling.                */
/* ------------------------------------------------------------------------- */

/* the radiance cache's network (defined with the cache below) */
void orc_nrc_encode(int64_t n, const float *in, const double lo[3], const double hi[3], double *feat);
static void nrc_predict(const double *W, const float in[16], const double box[6], double y[3]);

/* Light sampling (reading C12): pick an emissive primitive uniformly, draw a
 * point y of its untruncated Gaussian N(mu_k, Sigma_k), Sigma_k = (R S)(R S)^T,
 * and aim at it from x.  The direction's solid-angle density is the density
 * of y integrated along the ray, int_0^inf N(x + t w) t^2 dt.  In the unit
 * frame of k (x' = M (x - mu), w' = M w, a = |w'|) the point x + t w maps to
 * x' + t w', on a line that passes the centre at distance rho, at signed
 * position s = s0 + a t along it (s0 = x'.w' / a), so |x' + t w'|^2 =
 * rho^2 + s^2; the density of y is |det M| (2 pi)^(-3/2) exp(-|M (y - mu)|^2/2), so
 *   p(w) = |det M| exp(-rho^2/2) / ((2 pi)^(3/2) a^3) K(s0),
 *   K(s0) = int_{s0}^inf exp(-s^2/2) (s - s0)^2 ds
 *         = (1 + s0^2) sqrt(pi/2) erfc(s0/sqrt 2) - s0 exp(-s0^2/2).
 * Returned times the uniform emitter-choice probability.  From a point inside
 * the emitter's cut-off ellipsoid no light sample is taken toward it (pdf 0):
 * there the directions that leave a flat emitter's plane would have a density
 * far below their share of its emission, and phase sampling covers them. */
static double nee_pdf(const orc_scene *S, int64_t k, const double x[3], const double w[3]) {
    const double *M = S->M + 9 * k, *mu = S->mu + 3 * k;
    double c[3] = {x[0] - mu[0], x[1] - mu[1], x[2] - mu[2]}, xp[3], wp[3];
    for (int i = 0; i < 3; ++i) {
        xp[i] = M[3 * i] * c[0] + M[3 * i + 1] * c[1] + M[3 * i + 2] * c[2];
        wp[i] = M[3 * i] * w[0] + M[3 * i + 1] * w[1] + M[3 * i + 2] * w[2];
    }
    if (dot3(xp, xp) <= S->r * S->r) return 0.0;
    double a = sqrt(dot3(wp, wp));
    if (!(a > 0.0)) return 0.0;
    double s0 = dot3(xp, wp) / a;
    double perp[3];
    for (int i = 0; i < 3; ++i) perp[i] = xp[i] - s0 * wp[i] / a;
    double rho2 = dot3(perp, perp);
    double K = (1.0 + s0 * s0) * sqrt(M_PI / 2.0) * erfc(s0 / sqrt(2.0)) - s0 * exp(-0.5 * s0 * s0);
    double detM = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                  M[2] * (M[3] * M[7] - M[4] * M[6]);
    double p = fabs(detM) * exp(-0.5 * rho2) * fmax(K, 0.0) / (pow(2.0 * M_PI, 1.5) * a * a * a);
    return p / (double)S->n_emit;
}

/* The light-sampled direction from x toward emitter slot j: y = mu + (R S) n
 * with n three standard normals from the uniforms u[0..3] (Box-Muller);
 * returns 0 when x is inside the emitter's cut-off ellipsoid or y coincides
 * with x. */
static int nee_dir(const orc_scene *S, int64_t j, const double x[3], const double u[4], double w[3]) {
    int64_t e = S->emitters[j];
    const double *A = S->emA + 9 * j, *mu = S->mu + 3 * e, *M = S->M + 9 * e;
    double c[3] = {x[0] - mu[0], x[1] - mu[1], x[2] - mu[2]}, q2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        double xi = M[3 * i] * c[0] + M[3 * i + 1] * c[1] + M[3 * i + 2] * c[2];
        q2 += xi * xi;
    }
    if (q2 <= S->r * S->r) return 0;
    double r1 = sqrt(-2.0 * log(1.0 - u[0])), r2 = sqrt(-2.0 * log(1.0 - u[2]));
    double n[3] = {r1 * cos(2.0 * M_PI * u[1]), r1 * sin(2.0 * M_PI * u[1]), r2 * cos(2.0 * M_PI * u[3])};
    double y[3];
    for (int i = 0; i < 3; ++i) y[i] = mu[i] + A[3 * i] * n[0] + A[3 * i + 1] * n[1] + A[3 * i + 2] * n[2];
    for (int i = 0; i < 3; ++i) w[i] = y[i] - x[i];
    double l = sqrt(dot3(w, w));
    if (!(l > 0.0)) return 0;
    for (int i = 0; i < 3; ++i) w[i] /= l;
    return 1;
}

/* exported for the tests: light pdf of primitive k and the light-sampled
 * direction toward emitter slot j */
double orc_light_pdf(const orc_scene *S, int64_t k, const double *x, const double *w) {
    return nee_pdf(S, k, x, w);
}

int orc_light_dir(const orc_scene *S, int64_t j, const double *x, const double *u, double *w) {
    if (j < 0 || j >= S->n_emit) return 0;
    return nee_dir(S, j, x, u, w);
}

typedef struct {
    const orc_scene *S;
    orc_camera cam;
    orc_render_params p;
    const int64_t *pixels; /* NULL = all */
    int64_t n_pix;
    double *sum, *sumsq;
    int nthreads, tid;
    int64_t rays;
} rjob;

static void camera_ray(const orc_camera *cam, int64_t px, int64_t py, double jx, double jy,
                       double o[3], double w[3]) {
    double f[3] = {cam->target[0] - cam->origin[0], cam->target[1] - cam->origin[1],
                   cam->target[2] - cam->origin[2]};
    normalize3(f);
    double up[3] = {cam->up[0], cam->up[1], cam->up[2]};
    double rgt[3];
    cross3(f, up, rgt);
    normalize3(rgt);
    double u[3];
    cross3(rgt, f, u);
    double th = tan(0.5 * cam->vfov_deg * M_PI / 180.0);
    double asp = (double)cam->width / (double)cam->height;
    double sx = (2.0 * ((double)px + jx) / (double)cam->width - 1.0) * th * asp;
    double sy = (1.0 - 2.0 * ((double)py + jy) / (double)cam->height) * th;
    for (int i = 0; i < 3; ++i) {
        o[i] = cam->origin[i];
        w[i] = f[i] + sx * rgt[i] + sy * u[i];
    }
    normalize3(w);
}

/* The camera rays of one sample of every pixel (the jitter of vertex 0,
 * group 0, as the path tracer draws it), rounded to float [npix][8] =
 * (origin, direction, t0 = 0, t1 = inf). */
void orc_camera_rays(const orc_camera *cam, uint64_t seed, uint32_t sample, float *rays) {
    const int64_t npix = (int64_t)cam->width * cam->height;
    for (int64_t i = 0; i < npix; ++i) {
        double u[4], o[3], w[3];
        rng4(seed, (uint32_t)i, sample, 0, 0, u);
        camera_ray(cam, i % cam->width, i / cam->width, u[0], u[1], o, w);
        float *r = rays + 8 * i;
        for (int k = 0; k < 3; ++k) {
            r[k] = (float)o[k];
            r[3 + k] = (float)w[k];
        }
        r[6] = 0.f;
        r[7] = (float)INFINITY;
    }
}

/* Radiance of one camera path (Sec. 5 table tab:highlevel, eq. rte; vertex
 * v = 1, 2, ...: collide, pick up emission, stop after max_depth scattering
 * events, else NEE and phase sampling).  transport 1 runs the same loop in
 * the exponential variant (App. D): decomposition tracking for collisions and
 * light samples, exp(-sum I_k) for environment samples, no primitive skipped
 * after a scatter. */
static void trace_path(const orc_scene *S, const orc_render_params *P, const orc_camera *cam,
                       uint32_t pix, uint32_t sample, hitvec *H, hitvec *H2, double L[3],
                       int64_t *rays, double *rec, int max_rec, int *n_rec) {
    const uint64_t seed = P->seed;
    double u[4], g[4];
    rng4(seed, pix, sample, 0, 0, u);
    double o[3], w[3];
    camera_ray(cam, pix % (uint32_t)cam->width, pix / (uint32_t)cam->width, u[0], u[1], o, w);
    double beta[3] = {1.0, 1.0, 1.0};
    L[0] = L[1] = L[2] = 0.0;
    int64_t self = -1;
    double p_prev = 0.0, x_prev[3] = {0, 0, 0};
    const int env = (P->env_radiance[0] > 0.0 || P->env_radiance[1] > 0.0 || P->env_radiance[2] > 0.0);
    const double p_env = 1.0 / (4.0 * M_PI);
    /* radiance cache: a training path runs to max_depth and records its
     * vertices; any other path ends at collision nrc_terminate_after + 1 */
    int train = 0;
    if (P->nrc_mode == 1) {
        double t4[4];
        rng4(seed, pix, sample, 0, 2, t4);
        train = t4[0] < P->nrc_train_frac;
    }
    if (n_rec) *n_rec = 0;
    for (uint32_t v = 1;; ++v) {
        /* SGGX: uniforms of the light and environment estimates (groups 3, 4,
           and 6 for material 3's third normal) and of the base BSDF's sample
           about the visible normal (group 5) */
        double q3[4] = {0}, q4[4] = {0}, q5[4] = {0}, q6[4] = {0}, e3[6], e4[6];
        rng4(seed, pix, sample, v, 0, u);
        rng4(seed, pix, sample, v, 1, g);
        gather(S, o, w, 0.0, INFINITY, self, 1, H);
        ocoll c;
        if (P->transport == 1) {
            /* exponential variant: the nearest of the Gaussians' own free flights */
            const exp_key q = {1, seed, 0, pix, sample, v, 0};
            c.prim = exp_track(S, H, &q, &c.t_hit, NULL);
        } else {
            collide(S, H, 0.0, INFINITY, u[0], &c);
        }
        ++*rays;
        if (c.prim < 0) {
            if (env) {
                double wt;
                if (v == 1) wt = 1.0;
                else if (P->mis_mode == 1) wt = 1.0;
                else if (P->mis_mode == 2) wt = 0.0;
                else wt = p_prev / (p_prev + p_env);
                for (int i = 0; i < 3; ++i) L[i] += beta[i] * P->env_radiance[i] * wt;
            }
            break;
        }
        int64_t k = c.prim;
        double x[3] = {o[0] + c.t_hit * w[0], o[1] + c.t_hit * w[1], o[2] + c.t_hit * w[2]};
        const double *Le = S->emis + 3 * k;
        if (Le[0] > 0.0 || Le[1] > 0.0 || Le[2] > 0.0) {
            double wt;
            if (v == 1) wt = 1.0;
            else {
                double pn = nee_pdf(S, k, x_prev, w);
                if (P->mis_mode == 1) wt = 1.0;
                else if (P->mis_mode == 2) wt = (pn > 0.0) ? 0.0 : 1.0;
                else wt = p_prev / (p_prev + pn);
            }
            for (int i = 0; i < 3; ++i) L[i] += beta[i] * Le[i] * wt;
        }
        if ((int)v == P->max_depth + 1) break;
        double wo[3] = {-w[0], -w[1], -w[2]};
        if (S->mat[k] >= 2) {  /* drawn only where an SGGX phase function uses them */
            rng4(seed, pix, sample, v, 3, q3);
            rng4(seed, pix, sample, v, 4, q4);
            rng4(seed, pix, sample, v, 5, q5);
            rng4(seed, pix, sample, v, 6, q6);
        }
        for (int i = 0; i < 4; ++i) { e3[i] = q3[i]; e4[i] = q4[i]; }
        e3[4] = q6[0]; e3[5] = q6[1]; e4[4] = q6[2]; e4[5] = q6[3];
        const double *nrm = S->nrm + 3 * k, *alb = S->alb + 3 * k;
        double rough = S->rough[k];
        if (P->nrc_mode != 0) {
            /* cache inputs at this vertex: position, outgoing direction, facet
             * normal turned toward it, roughness, albedo */
            double nf[3] = {nrm[0], nrm[1], nrm[2]};
            if (dot3(nf, wo) < 0.0) for (int i = 0; i < 3; ++i) nf[i] = -nf[i];
            float in[16] = {(float)x[0], (float)x[1], (float)x[2], (float)wo[0], (float)wo[1], (float)wo[2],
                            (float)nf[0], (float)nf[1], (float)nf[2], (float)rough, (float)alb[0],
                            (float)alb[1], (float)alb[2], 0.f, 0.f, 0.f};
            if (!train && (int)v == P->nrc_terminate_after + 1) {
                if (P->nrc_mode == 1 || P->nrc_mode == 2) {
                    double y[3];
                    nrc_predict(P->nrc_weights, in, P->nrc_box, y);
                    for (int i = 0; i < 3; ++i) L[i] += beta[i] * fmax(0.0, y[i]);
                }
                break;
            }
            if (train && n_rec) {
                if (*n_rec < max_rec) {
                    double *r = rec + 24 * (*n_rec);
                    for (int i = 0; i < 16; ++i) r[i] = in[i];
                    for (int i = 0; i < 3; ++i) { r[16 + i] = beta[i]; r[20 + i] = L[i]; }
                    r[19] = (double)pix;
                    r[23] = (double)v;
                }
                ++*n_rec;
            }
        }
        /* NEE to one emissive primitive: uniform pick (group 0), a point of its
           Gaussian to aim at (group 7) */
        if (S->n_emit > 0 && P->mis_mode != 1) {
            int64_t j = (int64_t)(u[1] * (double)S->n_emit);
            if (j >= S->n_emit) j = S->n_emit - 1;
            int64_t e = S->emitters[j];
            double q7[4], wl[3];
            rng4(seed, pix, sample, v, 7, q7);
            if (e != k && nee_dir(S, j, x, q7, wl)) {
                double f[3], pph;
                prim_phase_eval(S, k, wo, wl, e3, f, &pph);
                ohit he;
                if ((f[0] > 0.0 || f[1] > 0.0 || f[2] > 0.0) && ray_prim(S, e, x, wl, 0.0, INFINITY, &he)) {
                    double pn = nee_pdf(S, e, x, wl);
                    if (pn > 0.0) {
                        double fac;
                        if (P->transport == 1) {
                            /* exponential variant: one decomposition-tracking draw along the
                             * segment to e's chord exit scores 1 if e is hit first, an
                             * unbiased estimate of the probability that it is */
                            gather(S, x, wl, 0.0, he.b, -1, 1, H2);
                            const exp_key q = {1, seed, 0, pix, sample, v, 1};
                            double th;
                            fac = exp_track(S, H2, &q, &th, NULL) == e ? 1.0 : 0.0;
                        } else {
                            fac = emitter_factor(S, x, wl, 0.0, INFINITY, k, e, 1, H2);
                        }
                        ++*rays;
                        double wt = (P->mis_mode == 2) ? 1.0 : pn / (pn + pph);
                        for (int i = 0; i < 3; ++i)
                            L[i] += beta[i] * f[i] * S->emis[3 * e + i] * fac * wt / pn;
                    }
                }
            }
        }
        /* NEE to the constant environment */
        if (env && P->mis_mode != 1) {
            double z = 1.0 - 2.0 * g[2];
            double rr = sqrt(fmax(0.0, 1.0 - z * z));
            double ph = 2.0 * M_PI * g[3];
            double wl[3] = {rr * cos(ph), rr * sin(ph), z};
            double f[3], pph;
            prim_phase_eval(S, k, wo, wl, e4, f, &pph);
            if (f[0] > 0.0 || f[1] > 0.0 || f[2] > 0.0) {
                double T;
                if (P->transport == 1) {
                    /* exponential variant: exp of the optical depth, nothing excluded */
                    gather(S, x, wl, 0.0, INFINITY, -1, 1, H2);
                    double depth = 0.0;
                    for (int64_t j = 0; j < H2->n; ++j) depth += seg_integral(S, &H2->v[j], H2->v[j].a, H2->v[j].b);
                    T = exp(-depth);
                } else {
                    gather(S, x, wl, 0.0, INFINITY, k, 1, H2);
                    T = fmax(0.0, 1.0 - accumulated_F(S, H2));
                }
                ++*rays;
                double wt = (P->mis_mode == 2) ? 1.0 : p_env / (p_env + pph);
                for (int i = 0; i < 3; ++i) L[i] += beta[i] * f[i] * T * P->env_radiance[i] * wt / p_env;
            }
        }
        /* continue by phase sampling from the collision point */
        double wi[3], wgt[3], pdf;
        prim_phase_sample(S, k, wo, g[0], g[1], q5, wi, wgt, &pdf);
        if (!(pdf > 0.0)) break;
        for (int i = 0; i < 3; ++i) beta[i] *= wgt[i];
        if (beta[0] == 0.0 && beta[1] == 0.0 && beta[2] == 0.0) break;
        for (int i = 0; i < 3; ++i) { o[i] = x[i]; w[i] = wi[i]; x_prev[i] = x[i]; }
        /* the linear model's scatter point is the chord centre, and the
         * primitive is skipped from there; an exponential medium scatters
         * inside the Gaussian, whose rest still attenuates */
        self = P->transport == 1 ? -1 : k;
        p_prev = pdf;
    }
}

static void *render_worker(void *arg) {
    rjob *J = (rjob *)arg;
    hitvec H = {0}, H2 = {0};
    int64_t npix = J->pixels ? J->n_pix : (int64_t)J->cam.width * J->cam.height;
    for (int64_t i = J->tid; i < npix; i += J->nthreads) {
        int64_t pix = J->pixels ? J->pixels[i] : i;
        double s[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
        for (int32_t sp = 0; sp < J->p.spp; ++sp) {
            double L[3];
            uint32_t sample = (uint32_t)(J->p.sample_offset + sp);
            trace_path(J->S, &J->p, &J->cam, (uint32_t)pix, sample, &H, &H2, L, &J->rays, NULL, 0, NULL);
            for (int c = 0; c < 3; ++c) { s[c] += L[c]; s2[c] += L[c] * L[c]; }
        }
        for (int c = 0; c < 3; ++c) {
            J->sum[3 * i + c] += s[c];
            if (J->sumsq) J->sumsq[3 * i + c] += s2[c];
        }
    }
    free(H.v);
    free(H2.v);
    return NULL;
}

int64_t orc_render(const orc_scene *S, const orc_camera *cam, const orc_render_params *p,
                   int64_t n_pix, const int64_t *pixels, int nthreads, double *sum, double *sumsq) {
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    rjob *jobs = (rjob *)malloc(sizeof(rjob) * (size_t)nthreads);
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (rjob){S, *cam, *p, pixels, n_pix, sum, sumsq, nthreads, t, 0};
        pthread_create(&th[t], NULL, render_worker, &jobs[t]);
    }
    int64_t rays = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        rays += jobs[t].rays;
    }
    free(th);
    free(jobs);
    return rays;
}

/* single path, for expected-value tests: radiance of (pixel, sample) */
void orc_path_radiance(const orc_scene *S, const orc_camera *cam, const orc_render_params *p,
                       uint32_t pix, uint32_t sample, double L[3]) {
    hitvec H = {0}, H2 = {0};
    int64_t rays = 0;
    trace_path(S, p, cam, pix, sample, &H, &H2, L, &rays, NULL, 0, NULL);
    free(H.v);
    free(H2.v);
}

int orc_path_records(const orc_scene *S, const orc_camera *cam, const orc_render_params *p, uint32_t pix,
                     uint32_t sample, double *rec, int max_rec, double L[3]) {
    hitvec H = {0}, H2 = {0};
    int64_t rays = 0;
    int n = 0;
    trace_path(S, p, cam, pix, sample, &H, &H2, L, &rays, rec, max_rec, &n);
    free(H.v);
    free(H2.v);
    return n;
}

/* ------------------------------------------------------------------------- */
/* Neural radiance cache (the learned radiance cache that terminates paths):  */
/* input encoding, MLP 96 -> 64 -> 64 -> 64 -> 64 -> 3 with ReLU and no       */
/* biases, relative-L2 loss and Adam, all in double precision.  Weights are   */
/* stored per layer as [n_out][n_in], layers back to back.                    */
/* ------------------------------------------------------------------------- */
#define NRC_IN 96
#define NRC_H 64
#define NRC_OUT 3
#define NRC_NPARAM (NRC_H * NRC_IN + 3 * NRC_H * NRC_H + NRC_OUT * NRC_H)

int orc_nrc_num_params(void) { return NRC_NPARAM; }

/* Encoding: position normalised to the scene box, x_hat in [0,1]^3, as
 * sin / cos(2^j pi x_hat) for j = 0..11 per axis (72); the outgoing direction
 * as real spherical harmonics of bands 0..3 (16); the facet normal (3),
 * roughness (1) and albedo (3); one zero pad.  in[16] = pos, wo, normal,
 * roughness, albedo, unused. */
void orc_nrc_encode(int64_t n, const float *in, const double lo[3], const double hi[3], double *feat) {
    for (int64_t r = 0; r < n; ++r) {
        const float *p = in + 16 * r;
        double *f = feat + NRC_IN * r;
        int o = 0;
        for (int a = 0; a < 3; ++a) {
            double xh = ((double)p[a] - lo[a]) / (hi[a] - lo[a]);
            for (int j = 0; j < 12; ++j) {
                double arg = ldexp(M_PI * xh, j);
                f[o++] = sin(arg);
                f[o++] = cos(arg);
            }
        }
        double x = p[3], y = p[4], z = p[5];
        double x2 = x * x, y2 = y * y, z2 = z * z;
        f[o++] = 0.28209479177387814;
        f[o++] = -0.48860251190291987 * y;
        f[o++] = 0.48860251190291987 * z;
        f[o++] = -0.48860251190291987 * x;
        f[o++] = 1.0925484305920792 * x * y;
        f[o++] = -1.0925484305920792 * y * z;
        f[o++] = 0.31539156525252005 * (3.0 * z2 - 1.0);
        f[o++] = -1.0925484305920792 * x * z;
        f[o++] = 0.5462742152960396 * (x2 - y2);
        f[o++] = -0.5900435899266435 * y * (3.0 * x2 - y2);
        f[o++] = 2.890611442640554 * x * y * z;
        f[o++] = -0.4570457994644658 * y * (5.0 * z2 - 1.0);
        f[o++] = 0.3731763325901154 * z * (5.0 * z2 - 3.0);
        f[o++] = -0.4570457994644658 * x * (5.0 * z2 - 1.0);
        f[o++] = 1.445305721320277 * z * (x2 - y2);
        f[o++] = -0.5900435899266435 * x * (x2 - 3.0 * y2);
        for (int k = 6; k < 13; ++k) f[o++] = p[k];
        f[o++] = 0.0;
    }
}

static const int nrc_nin[5] = {NRC_IN, NRC_H, NRC_H, NRC_H, NRC_H};
static const int nrc_nout[5] = {NRC_H, NRC_H, NRC_H, NRC_H, NRC_OUT};

static int nrc_offset(int l) {
    int o = 0;
    for (int k = 0; k < l; ++k) o += nrc_nin[k] * nrc_nout[k];
    return o;
}

/* forward: act[l] holds the input of layer l (act[0] = features); out = y */
static void nrc_forward_one(const double *W, const double *x, double act[5][NRC_IN], double y[3]) {
    for (int i = 0; i < NRC_IN; ++i) act[0][i] = x[i];
    for (int l = 0; l < 5; ++l) {
        const double *w = W + nrc_offset(l);
        for (int o = 0; o < nrc_nout[l]; ++o) {
            double s = 0.0;
            for (int i = 0; i < nrc_nin[l]; ++i) s += w[o * nrc_nin[l] + i] * act[l][i];
            if (l < 4) act[l + 1][o] = s > 0.0 ? s : 0.0;
            else y[o] = s;
        }
    }
}

void orc_nrc_forward(int64_t n, const double *W, const double *feat, double *y) {
    double act[5][NRC_IN];
    for (int64_t r = 0; r < n; ++r) nrc_forward_one(W, feat + NRC_IN * r, act, y + 3 * r);
}

/* Relative L2 loss mean over records and channels of (y - t)^2 / (sg(y)^2 +
 * 0.01), its gradient with respect to W (back-propagation through the ReLU
 * network, y in the denominator held constant). */
/* cache prediction for one vertex: encode, then the network */
static void nrc_predict(const double *W, const float in[16], const double box[6], double y[3]) {
    double feat[NRC_IN], act[5][NRC_IN];
    orc_nrc_encode(1, in, box, box + 3, feat);
    nrc_forward_one(W, feat, act, y);
}

double orc_nrc_loss_grad(int64_t n, const double *W, const double *feat, const double *target,
                         double *grad) {
    double act[5][NRC_IN], y[3], d[5][NRC_IN];
    memset(grad, 0, sizeof(double) * NRC_NPARAM);
    double loss = 0.0;
    const double scale = 1.0 / (3.0 * (double)n);
    for (int64_t r = 0; r < n; ++r) {
        nrc_forward_one(W, feat + NRC_IN * r, act, y);
        double dy[3];
        for (int c = 0; c < 3; ++c) {
            double den = y[c] * y[c] + 0.01;
            double e = y[c] - target[3 * r + c];
            loss += e * e / den * scale;
            dy[c] = 2.0 * e / den * scale;
        }
        /* output layer */
        for (int c = 0; c < 3; ++c) d[4][c] = dy[c];
        for (int l = 4; l >= 0; --l) {
            const double *w = W + nrc_offset(l);
            double *g = grad + nrc_offset(l);
            for (int o = 0; o < nrc_nout[l]; ++o)
                for (int i = 0; i < nrc_nin[l]; ++i) g[o * nrc_nin[l] + i] += d[l][o] * act[l][i];
            if (l == 0) break;
            /* delta of the layer input, through the ReLU that produced it */
            for (int i = 0; i < nrc_nin[l]; ++i) {
                double s = 0.0;
                for (int o = 0; o < nrc_nout[l]; ++o) s += w[o * nrc_nin[l] + i] * d[l][o];
                d[l - 1][i] = act[l][i] > 0.0 ? s : 0.0;
            }
        }
    }
    return loss;
}

/* one Adam step (Kingma and Ba, 2015) with bias correction, step t >= 1 */
void orc_nrc_adam(int64_t np, double *W, double *m, double *v, const double *g, int t, double lr, double b1,
                  double b2, double eps) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t i = 0; i < np; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        W[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
