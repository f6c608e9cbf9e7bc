/*
 * FP64 CPU oracle for stochastic ray tracing of transparent 3D Gaussians
 * (Sun, Georgiev, Fei, Hasan, "Stochastic Ray Tracing of Transparent 3D
 * Gaussians", EGSR 2025).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * reference against which the GPU library is checked. Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it. It shares
 * no code, header, table or helper with the GPU library.
 *
 * Every ray is tested against EVERY Gaussian (brute force, no acceleration
 * structure), in FP64. What each function follows:
 *   - records:   Sec. 3.1, eqn "gaussian" (G(x) with Sigma = R^T S^2 R).
 *   - isect:     Sec. 3.1 (the ray/Gaussian intersection is a 1D Gaussian;
 *                its mean is the depth) and eqn "cuboid" (cull outside the
 *                k-sigma ellipsoid, s = 2 sqrt 2), with the open ray range of
 *                Alg. "intersect".
 *   - acceptance: eqn "rr" (binary opacity, P(1) = alpha) drawn with
 *                Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 *   - selection: eqn "cloest" (the estimate is the colour of the closest
 *                accepted intersection) and eqn "multisample" (N independent
 *                instances; pixel = mean).
 *   - composite: eqn "accumulated" (exact front-to-back compositing).
 *   - gradients: the paper gives none (Sec. 7 names differentiable rendering
 *                as future work); the exact gradient is the derivative of
 *                eqn "accumulated" and the estimator is derived from it.
 *
 * Readings taken where the paper is silent (shared with the GPU library by
 * specification, not by code):
 *   alpha = opacity * peak of the 1D Gaussian = o * exp(-q/2), q the squared
 *   Mahalanobis distance of the 1D mean; accept iff u < alpha (the figure and
 *   eqn "rr" fix this direction; the printed listing has it inverted);
 *   the ellipsoid test is q <= s^2 = 8; a candidate's depth key is its FP64
 *   depth rounded to FP32, ties broken by Gaussian id; colour is the real
 *   SH expansion at the ray direction, offset by 0.5 and clamped at 0.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SRTO_S2 8.0 /* s^2 with s = 2 sqrt 2 */
#define SRTO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: 10 rounds of the Philox S-P network, 4x32-bit counter,    */
/* 2x32-bit key, multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key bumps        */
/* 0x9E3779B9 / 0xBB67AE85.                                                 */
/* ------------------------------------------------------------------------ */
void srto_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)b;
        uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void srto_philox_many(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i)
        srto_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* Acceptance number of (ray, sample, gaussian) for one ray purpose:
 * counter (ray_id, sample / 4, gid, purpose), key (seed lo, seed hi);
 * u = (word[sample mod 4] >> 8) * 2^-24, exact in FP32 and FP64. */
static double accept_u(uint64_t seed, uint32_t ray_id, uint32_t sample, uint32_t gid,
                       uint32_t purpose)
{
    uint32_t ctr[4] = {ray_id, sample >> 2, gid, purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    srto_philox4x32_10(ctr, key, w);
    return (double)(w[sample & 3u] >> 8) * (1.0 / 16777216.0);
}

double srto_accept_u(uint64_t seed, uint32_t ray_id, uint32_t sample, uint32_t gid,
                     uint32_t purpose)
{
    return accept_u(seed, ray_id, sample, gid, purpose);
}

/* ------------------------------------------------------------------------ */
/* Gaussian records (eqn "gaussian").                                        */
/* ------------------------------------------------------------------------ */

/* Rotation matrix (row-major, local -> world) of the unit Hamilton
 * quaternion (w, x, y, z). */
static void quat_to_rot(double w, double x, double y, double z, double R[9])
{
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

void srto_quat_to_rot(const double q[4], double R[9])
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    quat_to_rot(q[0] / n, q[1] / n, q[2] / n, q[3] / n, R);
}

/* The whitening matrix M = S^-1 R^T maps x - mu to the Gaussian's unit-sphere
 * frame, so (x-mu)^T Sigma^-1 (x-mu) = |M (x-mu)|^2 with Sigma = R S^2 R^T
 * (the paper's R is this R transposed). Opacity o = sigmoid(logit).
 * With round_f32 != 0 the record is rounded to FP32, which is the canonical
 * record both implementations intersect against. */
void srto_records(int64_t G, const float* means, const float* log_scales,
                  const float* quats, const float* logits, int round_f32,
                  double* mu, double* M, double* op)
{
    for (int64_t g = 0; g < G; ++g) {
        double qw = quats[4 * g + 0], qx = quats[4 * g + 1];
        double qy = quats[4 * g + 2], qz = quats[4 * g + 3];
        double n = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        double R[9];
        if (n > 0.0)
            quat_to_rot(qw / n, qx / n, qy / n, qz / n, R);
        else
            quat_to_rot(1.0, 0.0, 0.0, 0.0, R);
        for (int i = 0; i < 3; ++i) {
            double inv_s = exp(-(double)log_scales[3 * g + i]);
            for (int j = 0; j < 3; ++j) {
                double v = R[3 * j + i] * inv_s; /* (R^T)_ij / s_i */
                M[9 * g + 3 * i + j] = round_f32 ? (double)(float)v : v;
            }
            mu[3 * g + i] = (double)means[3 * g + i];
        }
        double o = 1.0 / (1.0 + exp(-(double)logits[g]));
        op[g] = round_f32 ? (double)(float)o : o;
    }
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3, orthonormal on the sphere, index */
/* l*l + l + m with m = -l..l; m > 0 is sqrt2 * Re and m < 0 is sqrt2 * Im   */
/* of the complex harmonic carrying the Condon-Shortley phase.               */
/* ------------------------------------------------------------------------ */
void srto_sh_basis(int deg, const double dir[3], double* Y)
{
    double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double x = dir[0] / n, y = dir[1] / n, z = dir[2] / n;
    Y[0] = 0.5 * sqrt(1.0 / SRTO_PI);
    if (deg < 1) return;
    double c1 = sqrt(3.0 / (4.0 * SRTO_PI));
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    double c2a = 0.5 * sqrt(15.0 / SRTO_PI);
    double c2b = 0.25 * sqrt(5.0 / SRTO_PI);
    double c2c = 0.25 * sqrt(15.0 / SRTO_PI);
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0 * z * z - x * x - y * y);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (x * x - y * y);
    if (deg < 3) return;
    double c3a = 0.25 * sqrt(35.0 / (2.0 * SRTO_PI));
    double c3b = 0.5 * sqrt(105.0 / SRTO_PI);
    double c3c = 0.25 * sqrt(21.0 / (2.0 * SRTO_PI));
    double c3d = 0.25 * sqrt(7.0 / SRTO_PI);
    double c3e = 0.25 * sqrt(105.0 / SRTO_PI);
    Y[9] = -c3a * y * (3.0 * x * x - y * y);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0 * z * z - x * x - y * y);
    Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = -c3c * x * (4.0 * z * z - x * x - y * y);
    Y[14] = c3e * z * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3.0 * y * y);
}

/* Colour of Gaussian g seen along direction dir: max(0, 0.5 + sum k Y).
 * pre[3] receives the unclamped value when non-null. */
static void gauss_colour(int deg, const float* sh, int64_t g, const double* Y,
                         double c[3], double pre[3])
{
    int K = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double s = 0.5;
        for (int j = 0; j < K; ++j) s += (double)sh[((int64_t)g * K + j) * 3 + ch] * Y[j];
        if (pre) pre[ch] = s;
        c[ch] = s > 0.0 ? s : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Ray / Gaussian intersection (Sec. 3.1 and eqn "cuboid").                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    double t;     /* mean of the 1D Gaussian along the ray (the depth) */
    double q;     /* squared Mahalanobis distance at t (peak = exp(-q/2)) */
    double p[3];  /* whitened position M (o + t d - mu) */
    double w[3];  /* world offset o + t d - mu */
} isect_t;

/* Along x(t) = o + t d the exponent is -|M(o - mu) + t M d|^2 / 2, a 1D
 * Gaussian in t with mean t* = -(o'.d')/(d'.d'), o' = M(o-mu), d' = M d. */
static void isect(const double* mu, const double* M, const float* o, const float* d,
                  isect_t* r)
{
    double w0 = (double)o[0] - mu[0], w1 = (double)o[1] - mu[1], w2 = (double)o[2] - mu[2];
    double d0 = d[0], d1 = d[1], d2 = d[2];
    double op[3], dp[3];
    for (int i = 0; i < 3; ++i) {
        op[i] = M[3 * i] * w0 + M[3 * i + 1] * w1 + M[3 * i + 2] * w2;
        dp[i] = M[3 * i] * d0 + M[3 * i + 1] * d1 + M[3 * i + 2] * d2;
    }
    double dd = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
    double od = op[0] * dp[0] + op[1] * dp[1] + op[2] * dp[2];
    double t = -od / dd;
    r->t = t;
    for (int i = 0; i < 3; ++i) r->p[i] = op[i] + t * dp[i];
    r->q = r->p[0] * r->p[0] + r->p[1] * r->p[1] + r->p[2] * r->p[2];
    r->w[0] = w0 + t * d0;
    r->w[1] = w1 + t * d1;
    r->w[2] = w2 + t * d2;
}

/* Single-candidate probe for tests: t, q, alpha and validity. */
int srto_isect_one(const double* mu, const double* M, double op, const float* o,
                   const float* d, double tmin, double tmax, double* out /*t,q,alpha*/)
{
    isect_t r;
    isect(mu, M, o, d, &r);
    out[0] = r.t;
    out[1] = r.q;
    out[2] = op * exp(-0.5 * r.q);
    return (r.t > tmin && r.t < tmax && r.q <= SRTO_S2) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Candidate lists.                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    double t, q, alpha;
    float t32;
    int32_t gid;
    int valid;      /* strictly inside the range and the ellipsoid */
    int borderline; /* within 1e-9 (relative) of a validity boundary */
} cand_t;

typedef struct {
    cand_t* v;
    int64_t n, cap;
} clist_t;

static void cl_push(clist_t* l, const cand_t* c)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 64;
        l->v = (cand_t*)realloc(l->v, (size_t)l->cap * sizeof(cand_t));
    }
    l->v[l->n++] = *c;
}

static int key_less(float ta, int32_t ga, float tb, int32_t gb)
{
    return ta < tb || (ta == tb && ga < gb);
}

static int cmp_cand(const void* a, const void* b)
{
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (key_less(x->t32, x->gid, y->t32, y->gid)) return -1;
    if (key_less(y->t32, y->gid, x->t32, x->gid)) return 1;
    return 0;
}

static int near_rel(double a, double b)
{
    double s = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
    if (s < 1.0) s = 1.0;
    return fabs(a - b) <= 1e-9 * s;
}

/* Depth of a candidate (Sec. 3.1 and Sec. 4.1). Mode 0 ("mean"): the mean
 * of the 1D Gaussian along the ray. Mode 1 ("center"): the Gaussian centre
 * projected onto a viewing axis a, expressed as the ray parameter with the
 * same depth along a: t = ((mu - o) . a) / (d . a); a = (0,0,0) means the
 * ray's own direction. Opacity stays at the 1D peak in both modes. The mode
 * is an argument of every call that collects candidates (no global state). */
typedef struct {
    int mode;
    double axis[3];
} depth_t;

static depth_t depth_of(int mode, const double* axis)
{
    depth_t dm;
    dm.mode = mode;
    for (int i = 0; i < 3; ++i) dm.axis[i] = (mode != 0 && axis) ? axis[i] : 0.0;
    return dm;
}

static double depth_key(const depth_t* dm, const isect_t* r, const double* mu, const float* o,
                        const float* d)
{
    if (dm->mode == 0) return r->t;
    double a[3] = {dm->axis[0], dm->axis[1], dm->axis[2]};
    if (a[0] == 0.0 && a[1] == 0.0 && a[2] == 0.0) {
        a[0] = d[0];
        a[1] = d[1];
        a[2] = d[2];
    }
    double num = 0.0, den = 0.0;
    for (int i = 0; i < 3; ++i) {
        num += (mu[i] - (double)o[i]) * a[i];
        den += (double)d[i] * a[i];
    }
    return num / den;
}

/* Brute-force candidate collection for one ray: every Gaussian whose depth
 * is in the open ray range and whose 1D mean is inside the ellipsoid, plus
 * borderline ones (kept for flagging, never selected). */
static void collect(const depth_t* dm, int64_t G, const double* mu, const double* M,
                    const double* op, const float* o, const float* d, double tmin, double tmax,
                    int32_t ignore_gid, clist_t* out)
{
    out->n = 0;
    for (int64_t g = 0; g < G; ++g) {
        if ((int32_t)g == ignore_gid) continue;
        isect_t r;
        isect(mu + 3 * g, M + 9 * g, o, d, &r);
        const double t = depth_key(dm, &r, mu + 3 * g, o, d);
        int valid = (t > tmin && t < tmax && r.q <= SRTO_S2);
        int border = near_rel(r.q, SRTO_S2) || near_rel(t, tmin) ||
                     (isfinite(tmax) && near_rel(t, tmax));
        if (!valid && !border) continue;
        if (!(t == t)) continue;
        cand_t c;
        c.t = t;
        c.q = r.q;
        c.alpha = op[g] * exp(-0.5 * r.q);
        c.t32 = (float)t;
        c.gid = (int32_t)g;
        c.valid = valid;
        c.borderline = border;
        cl_push(out, &c);
    }
}

/* ------------------------------------------------------------------------ */
/* Stochastic trace (eqns "rr", "cloest", "multisample").                    */
/* ------------------------------------------------------------------------ */
enum { FLAG_U = 1, FLAG_GEO = 2 };

typedef struct {
    int64_t count;
    const float *o, *d, *tmin, *tmax;
    const int32_t* ignore_gid;
    const uint32_t *ray_id, *sample_base;
} rays_t;

static void ray_get(const rays_t* R, int64_t i, double* tmin, double* tmax, int32_t* ign,
                    uint32_t* rid, uint32_t* sbase)
{
    *tmin = R->tmin ? (double)R->tmin[i] : 0.0;
    *tmax = R->tmax ? (double)R->tmax[i] : INFINITY;
    *ign = R->ignore_gid ? R->ignore_gid[i] : -1;
    *rid = R->ray_id ? R->ray_id[i] : (uint32_t)i;
    *sbase = R->sample_base ? R->sample_base[i] : 0u;
}

/* Resolve one sample of one ray from its candidate list. `u_override`, when
 * non-null, replaces the Philox number by u_override[gid] (tests inject
 * binary outcomes this way). Returns the index of the chosen candidate or -1,
 * and sets flags / margin. */
static int64_t resolve(const clist_t* cl, uint64_t seed, uint32_t rid, uint32_t sample,
                       uint32_t purpose, int any_hit, const double* u_override,
                       uint8_t* flags, double* margin)
{
    int64_t best = -1;
    int64_t n_acc = 0;
    double* u = (double*)malloc((size_t)(cl->n > 0 ? cl->n : 1) * sizeof(double));
    for (int64_t i = 0; i < cl->n; ++i) {
        const cand_t* c = &cl->v[i];
        u[i] = u_override ? u_override[c->gid] : accept_u(seed, rid, sample, (uint32_t)c->gid, purpose);
        if (!c->valid) continue;
        if (u[i] < c->alpha) {
            ++n_acc;
            if (best < 0 || key_less(c->t32, c->gid, cl->v[best].t32, cl->v[best].gid)) best = i;
        }
    }
    uint8_t f = 0;
    double mu_ = INFINITY;
    for (int64_t i = 0; i < cl->n; ++i) {
        const cand_t* c = &cl->v[i];
        int in_front = best < 0 || !key_less(cl->v[best].t32, cl->v[best].gid, c->t32, c->gid);
        if (any_hit) in_front = 1;
        if (!in_front) continue;
        if (c->valid) {
            double m = fabs(c->alpha - u[i]);
            if (m < mu_) mu_ = m;
        }
        if (c->borderline && u[i] < c->alpha) f |= FLAG_GEO;
    }
    if (mu_ < 1e-6) f |= FLAG_U;
    if (any_hit && n_acc > 1) f &= (uint8_t)~FLAG_U; /* one flip cannot clear occlusion */
    if (!any_hit && best >= 0) {
        /* another accepted candidate within one FP32 ulp of the result's depth */
        const cand_t* b = &cl->v[best];
        for (int64_t i = 0; i < cl->n; ++i) {
            const cand_t* c = &cl->v[i];
            if (i == best || !c->valid || !(u[i] < c->alpha)) continue;
            if (c->t != b->t && fabsf(c->t32 - b->t32) <= nextafterf(fabsf(b->t32), INFINITY) - fabsf(b->t32))
                f |= FLAG_GEO;
        }
    }
    free(u);
    *flags = f;
    *margin = mu_;
    return best;
}

/* Trace R rays with spp samples each against all G Gaussians.
 * Outputs: rgb [R,3] (mean over samples of the shaded colour, bg on miss),
 * hit_gid [R,spp] (-1 on miss), hit_t [R,spp] (FP32 key, +inf on miss),
 * flags [R,spp], margin [R,spp] (min |alpha - u| in front of the result).
 * In any-hit mode the sample's hit is any accepted candidate (the oracle
 * reports the nearest) and rgb is the fraction of unoccluded samples. */
void srto_trace(int64_t G, const double* mu, const double* M, const double* op, int deg,
                const float* sh, int64_t R, const float* o, const float* d, const float* tmin,
                const float* tmax, const int32_t* ignore_gid, const uint32_t* ray_id,
                const uint32_t* sample_base, int32_t spp, uint64_t seed, uint32_t purpose,
                int any_hit, const double* bg, const double* u_override, int depth_mode,
                const double* depth_axis, double* rgb, int32_t* hit_gid, float* hit_t,
                uint8_t* flags, double* margin, int threads)
{
    rays_t RR = {R, o, d, tmin, tmax, ignore_gid, ray_id, sample_base};
    const depth_t dm = depth_of(depth_mode, depth_axis);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
    {
        clist_t cl = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < R; ++i) {
            double t0, t1;
            int32_t ign;
            uint32_t rid, sb;
            ray_get(&RR, i, &t0, &t1, &ign, &rid, &sb);
            collect(&dm, G, mu, M, op, o + 3 * i, d + 3 * i, t0, t1, ign, &cl);
            double Y[16], dir[3] = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
            srto_sh_basis(deg, dir, Y);
            double acc[3] = {0, 0, 0};
            for (int32_t s = 0; s < spp; ++s) {
                uint8_t f;
                double m;
                int64_t b = resolve(&cl, seed, rid, sb + (uint32_t)s, purpose, any_hit,
                                    u_override, &f, &m);
                int64_t k = i * spp + s;
                if (hit_gid) hit_gid[k] = b >= 0 ? cl.v[b].gid : -1;
                if (hit_t) hit_t[k] = b >= 0 ? cl.v[b].t32 : INFINITY;
                if (flags) flags[k] = f;
                if (margin) margin[k] = m;
                if (any_hit) {
                    double v = b >= 0 ? 0.0 : 1.0;
                    for (int ch = 0; ch < 3; ++ch) acc[ch] += v;
                } else if (b >= 0) {
                    double c[3];
                    gauss_colour(deg, sh, cl.v[b].gid, Y, c, 0);
                    for (int ch = 0; ch < 3; ++ch) acc[ch] += c[ch];
                } else {
                    for (int ch = 0; ch < 3; ++ch) acc[ch] += bg[ch];
                }
            }
            if (rgb)
                for (int ch = 0; ch < 3; ++ch) rgb[3 * i + ch] = acc[ch] / (double)spp;
        }
        free(cl.v);
    }
}

/* Valid candidates of one ray in (depth key, id) order: for tests. Returns
 * the number written (at most cap). */
int64_t srto_candidates(int64_t G, const double* mu, const double* M, const double* op,
                        const float* o, const float* d, double tmin, double tmax,
                        int32_t ignore_gid, int depth_mode, const double* depth_axis,
                        int64_t cap, double* t, double* q, double* alpha, float* t32,
                        int32_t* gid)
{
    clist_t cl = {0, 0, 0};
    const depth_t dm = depth_of(depth_mode, depth_axis);
    collect(&dm, G, mu, M, op, o, d, tmin, tmax, ignore_gid, &cl);
    int64_t n = 0;
    for (int64_t i = 0; i < cl.n; ++i)
        if (cl.v[i].valid) cl.v[n++] = cl.v[i];
    if (n > 1) qsort(cl.v, (size_t)n, sizeof(cand_t), cmp_cand); /* v may be null when n = 0 */
    int64_t m = n < cap ? n : cap;
    for (int64_t i = 0; i < m; ++i) {
        t[i] = cl.v[i].t;
        q[i] = cl.v[i].q;
        alpha[i] = cl.v[i].alpha;
        t32[i] = cl.v[i].t32;
        gid[i] = cl.v[i].gid;
    }
    free(cl.v);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Exact compositing (eqn "accumulated") and its gradient.                   */
/* ------------------------------------------------------------------------ */

/* Sorted valid candidates of ray i with their colours. */
typedef struct {
    clist_t cl;
    double* c;   /* [n,3] clamped colour */
    double* pre; /* [n,3] unclamped */
} sorted_t;

static void sorted_build(sorted_t* S, const depth_t* dm, int64_t G, const double* mu,
                         const double* M, const double* op, int deg, const float* sh,
                         const float* o, const float* d, double tmin, double tmax, int32_t ign,
                         const double* Y)
{
    collect(dm, G, mu, M, op, o, d, tmin, tmax, ign, &S->cl);
    int64_t n = 0;
    for (int64_t i = 0; i < S->cl.n; ++i)
        if (S->cl.v[i].valid) S->cl.v[n++] = S->cl.v[i];
    S->cl.n = n;
    if (n > 1) qsort(S->cl.v, (size_t)n, sizeof(cand_t), cmp_cand); /* v may be null when n = 0 */
    S->c = (double*)realloc(S->c, (size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    S->pre = (double*)realloc(S->pre, (size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    for (int64_t k = 0; k < n; ++k)
        gauss_colour(deg, sh, S->cl.v[k].gid, Y, S->c + 3 * k, S->pre + 3 * k);
}

/* L = sum_k T_k alpha_k c_k + T_{M+1} bg, T_k = prod_{j<k} (1 - alpha_j).
 * var = E[Lhat^2] - L^2 for the single-sample estimator, per channel. */
void srto_composite(int64_t G, const double* mu, const double* M, const double* op, int deg,
                    const float* sh, int64_t R, const float* o, const float* d,
                    const float* tmin, const float* tmax, const int32_t* ignore_gid,
                    const double* bg, int depth_mode, const double* depth_axis, double* L,
                    double* var, double* T_end, int32_t* n_cand, int threads)
{
    rays_t RR = {R, o, d, tmin, tmax, ignore_gid, 0, 0};
    const depth_t dm = depth_of(depth_mode, depth_axis);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
    {
        sorted_t S = {{0, 0, 0}, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < R; ++i) {
            double t0, t1;
            int32_t ign;
            uint32_t rid, sb;
            ray_get(&RR, i, &t0, &t1, &ign, &rid, &sb);
            double Y[16], dir[3] = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
            srto_sh_basis(deg, dir, Y);
            sorted_build(&S, &dm, G, mu, M, op, deg, sh, o + 3 * i, d + 3 * i, t0, t1, ign, Y);
            double T = 1.0, l[3] = {0, 0, 0}, l2[3] = {0, 0, 0};
            for (int64_t k = 0; k < S.cl.n; ++k) {
                double a = S.cl.v[k].alpha;
                for (int ch = 0; ch < 3; ++ch) {
                    double c = S.c[3 * k + ch];
                    l[ch] += T * a * c;
                    l2[ch] += T * a * c * c;
                }
                T *= (1.0 - a);
            }
            for (int ch = 0; ch < 3; ++ch) {
                double Lc = l[ch] + T * bg[ch];
                if (L) L[3 * i + ch] = Lc;
                if (var) var[3 * i + ch] = l2[ch] + T * bg[ch] * bg[ch] - Lc * Lc;
            }
            if (T_end) T_end[i] = T;
            if (n_cand) n_cand[i] = (int32_t)S.cl.n;
        }
        free(S.cl.v);
        free(S.c);
        free(S.pre);
    }
}

/* Chain rule from d(loss)/d(alpha) of one candidate of one ray to the raw
 * parameters of its Gaussian. alpha = o exp(-q/2), o = sigmoid(logit),
 * q = |M (x* - mu)|^2 with x* = o_ray + t* d at the 1D mean; because t*
 * minimises q along the ray, dq/dt* = 0 (envelope) and only the explicit
 * dependence on mu and M remains:
 *   dq/dmu = -2 M^T p,  dq/dM = 2 p w^T,  p = M w,  w = x* - mu.
 * M = S^-1 R^T with S = diag(exp(ls)), R = R(quat / |quat|). */
static void chain_alpha(int64_t g, double s_alpha, double alpha, const isect_t* r,
                        const float* log_scales, const float* quats, const float* logits,
                        double* g_means, double* g_ls, double* g_quats, double* g_logits)
{
    double o = 1.0 / (1.0 + exp(-(double)logits[g]));
    double s_q = s_alpha * (-0.5 * alpha);
    double qw = quats[4 * g], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
    double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    double R[9];
    quat_to_rot(w, x, y, z, R);
    double inv_s[3], Mx[9];
    for (int i = 0; i < 3; ++i) {
        inv_s[i] = exp(-(double)log_scales[3 * g + i]);
        for (int j = 0; j < 3; ++j) Mx[3 * i + j] = R[3 * j + i] * inv_s[i];
    }
    /* d loss / d M_ij */
    double GM[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) GM[3 * i + j] = s_q * 2.0 * r->p[i] * r->w[j];
    double gmu[3], gls[3], GR[9];
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i) s += Mx[3 * i + j] * r->p[i];
        gmu[j] = s_q * (-2.0) * s;
    }
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) s += GM[3 * i + j] * (-Mx[3 * i + j]);
        gls[i] = s;
    }
    /* M_ij = R_ji inv_s_i  =>  dL/dR_ji = GM_ij inv_s_i */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) GR[3 * j + i] = GM[3 * i + j] * inv_s[i];
    /* dR/d(w,x,y,z) of the unit quaternion */
    double gq[4];
    gq[0] = GR[1] * (-2 * z) + GR[2] * (2 * y) + GR[3] * (2 * z) + GR[5] * (-2 * x) +
            GR[6] * (-2 * y) + GR[7] * (2 * x);
    gq[1] = GR[1] * (2 * y) + GR[2] * (2 * z) + GR[3] * (2 * y) + GR[4] * (-4 * x) +
            GR[5] * (-2 * w) + GR[6] * (2 * z) + GR[7] * (2 * w) + GR[8] * (-4 * x);
    gq[2] = GR[0] * (-4 * y) + GR[1] * (2 * x) + GR[2] * (2 * w) + GR[3] * (2 * x) +
            GR[5] * (2 * z) + GR[6] * (-2 * w) + GR[7] * (2 * z) + GR[8] * (-4 * y);
    gq[3] = GR[0] * (-4 * z) + GR[1] * (-2 * w) + GR[2] * (2 * x) + GR[3] * (2 * w) +
            GR[4] * (-4 * z) + GR[5] * (2 * y) + GR[6] * (2 * x) + GR[7] * (2 * y);
    /* through the normalisation q / |q| */
    double dotq = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
    double uq[4] = {w, x, y, z};
    for (int k = 0; k < 4; ++k) {
        double v = (gq[k] - uq[k] * dotq) / qn;
#pragma omp atomic
        g_quats[4 * g + k] += v;
    }
    for (int k = 0; k < 3; ++k) {
#pragma omp atomic
        g_means[3 * g + k] += gmu[k];
#pragma omp atomic
        g_ls[3 * g + k] += gls[k];
    }
    double gl = s_alpha * alpha * (1.0 - o);
#pragma omp atomic
    g_logits[g] += gl;
}

static void chain_colour(int deg, int64_t g, const double* Y, const double* pre,
                         const double gc[3], double* g_sh)
{
    int K = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        if (!(pre[ch] > 0.0)) continue;
        for (int j = 0; j < K; ++j) {
            double v = Y[j] * gc[ch];
#pragma omp atomic
            g_sh[((int64_t)g * K + j) * 3 + ch] += v;
        }
    }
}

/* Re-intersect to recover the geometry of candidate k of the sorted list. */
static void regeo(const double* mu, const double* M, int64_t g, const float* o,
                  const float* d, isect_t* r)
{
    isect(mu + 3 * g, M + 9 * g, o, d, r);
}

/* Exact gradient of sum_i <dL_i, L_i> through eqn "accumulated":
 *   dL/dalpha_k = T_k (c_k - B_k), B_k = colour expected behind k
 *   (B_last = bg, B_{k-1} = alpha_k c_k + (1 - alpha_k) B_k),
 *   dL/dc_k = T_k alpha_k. Gradients are ADDED to the outputs. */
void srto_composite_grad(int64_t G, const double* mu, const double* M, const double* op,
                         int deg, const float* sh, const float* log_scales,
                         const float* quats, const float* logits, int64_t R, const float* o,
                         const float* d, const float* tmin, const float* tmax,
                         const int32_t* ignore_gid, const double* bg, int depth_mode,
                         const double* depth_axis, const double* dL, double* g_means,
                         double* g_ls, double* g_quats, double* g_logits, double* g_sh,
                         int threads)
{
    rays_t RR = {R, o, d, tmin, tmax, ignore_gid, 0, 0};
    const depth_t dm = depth_of(depth_mode, depth_axis);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
    {
        sorted_t S = {{0, 0, 0}, 0, 0};
        double* B = 0;
        int64_t Bcap = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < R; ++i) {
            double t0, t1;
            int32_t ign;
            uint32_t rid, sb;
            ray_get(&RR, i, &t0, &t1, &ign, &rid, &sb);
            double Y[16], dir[3] = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
            srto_sh_basis(deg, dir, Y);
            sorted_build(&S, &dm, G, mu, M, op, deg, sh, o + 3 * i, d + 3 * i, t0, t1, ign, Y);
            int64_t n = S.cl.n;
            if (n == 0) continue;
            if (Bcap < n) {
                Bcap = n;
                B = (double*)realloc(B, (size_t)Bcap * 3 * sizeof(double));
            }
            for (int ch = 0; ch < 3; ++ch) B[3 * (n - 1) + ch] = bg[ch];
            for (int64_t k = n - 1; k > 0; --k) {
                double a = S.cl.v[k].alpha;
                for (int ch = 0; ch < 3; ++ch)
                    B[3 * (k - 1) + ch] = a * S.c[3 * k + ch] + (1.0 - a) * B[3 * k + ch];
            }
            double T = 1.0;
            for (int64_t k = 0; k < n; ++k) {
                const cand_t* c = &S.cl.v[k];
                double s_alpha = 0.0, gc[3];
                for (int ch = 0; ch < 3; ++ch) {
                    s_alpha += dL[3 * i + ch] * T * (S.c[3 * k + ch] - B[3 * k + ch]);
                    gc[ch] = dL[3 * i + ch] * T * c->alpha;
                }
                isect_t r;
                regeo(mu, M, c->gid, o + 3 * i, d + 3 * i, &r);
                chain_alpha(c->gid, s_alpha, c->alpha, &r, log_scales, quats, logits, g_means,
                            g_ls, g_quats, g_logits);
                chain_colour(deg, c->gid, Y, S.pre + 3 * k, gc, g_sh);
                T *= (1.0 - c->alpha);
            }
        }
        free(S.cl.v);
        free(S.c);
        free(S.pre);
        free(B);
    }
}

/* The unbiased stochastic gradient estimator, evaluated on the SAME
 * realisation the trace draws (same Philox numbers). For a sample whose
 * result is a (colour X = c_a, or bg on a miss), every valid candidate k in
 * front of a was rejected; its alpha receives <dL, c_k - X> / (1 - alpha_k),
 * whose expectation T_k (1 - alpha_k) (c_k - B_k) / (1 - alpha_k) is exactly
 * dL/dalpha_k. The result receives the colour gradient dL. Each sample is
 * weighted 1/spp (eqn "multisample"). Gradients are ADDED to the outputs. */
void srto_estimator_grad(int64_t G, const double* mu, const double* M, const double* op,
                         int deg, const float* sh, const float* log_scales,
                         const float* quats, const float* logits, int64_t R, const float* o,
                         const float* d, const float* tmin, const float* tmax,
                         const int32_t* ignore_gid, const uint32_t* ray_id,
                         const uint32_t* sample_base, int32_t spp, uint64_t seed,
                         uint32_t purpose, const double* bg, int depth_mode,
                         const double* depth_axis, const double* dL, double* g_means,
                         double* g_ls, double* g_quats, double* g_logits, double* g_sh,
                         int threads)
{
    rays_t RR = {R, o, d, tmin, tmax, ignore_gid, ray_id, sample_base};
    const depth_t dm = depth_of(depth_mode, depth_axis);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
    {
        sorted_t S = {{0, 0, 0}, 0, 0};
        double* sa = 0;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < R; ++i) {
            double t0, t1;
            int32_t ign;
            uint32_t rid, sb;
            ray_get(&RR, i, &t0, &t1, &ign, &rid, &sb);
            double Y[16], dir[3] = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
            srto_sh_basis(deg, dir, Y);
            sorted_build(&S, &dm, G, mu, M, op, deg, sh, o + 3 * i, d + 3 * i, t0, t1, ign, Y);
            int64_t n = S.cl.n;
            if (n == 0) continue;
            if (cap < n) {
                cap = n;
                sa = (double*)realloc(sa, (size_t)cap * sizeof(double));
            }
            memset(sa, 0, (size_t)n * sizeof(double));
            const double* g = dL + 3 * i;
            for (int32_t s = 0; s < spp; ++s) {
                uint32_t sample = sb + (uint32_t)s;
                /* the list is sorted: the result is the first accepted */
                int64_t a = -1;
                for (int64_t k = 0; k < n; ++k) {
                    double u = accept_u(seed, rid, sample, (uint32_t)S.cl.v[k].gid, purpose);
                    if (u < S.cl.v[k].alpha) {
                        a = k;
                        break;
                    }
                }
                double X[3];
                for (int ch = 0; ch < 3; ++ch) X[ch] = a >= 0 ? S.c[3 * a + ch] : bg[ch];
                int64_t front = a >= 0 ? a : n;
                for (int64_t k = 0; k < front; ++k) {
                    double v = 0.0;
                    for (int ch = 0; ch < 3; ++ch) v += g[ch] * (S.c[3 * k + ch] - X[ch]);
                    sa[k] += v / ((1.0 - S.cl.v[k].alpha) * (double)spp);
                }
                if (a >= 0) {
                    double gc[3] = {g[0] / spp, g[1] / spp, g[2] / spp};
                    chain_colour(deg, S.cl.v[a].gid, Y, S.pre + 3 * a, gc, g_sh);
                }
            }
            for (int64_t k = 0; k < n; ++k) {
                if (sa[k] == 0.0) continue;
                isect_t r;
                regeo(mu, M, S.cl.v[k].gid, o + 3 * i, d + 3 * i, &r);
                chain_alpha(S.cl.v[k].gid, sa[k], S.cl.v[k].alpha, &r, log_scales, quats,
                            logits, g_means, g_ls, g_quats, g_logits);
            }
        }
        free(S.cl.v);
        free(S.c);
        free(S.pre);
        free(sa);
    }
}

/* A lower-variance form of the same estimator (the paper leaves lower-
 * variance gradient estimators open, Sec. 7): each candidate's term is
 * averaged over its own acceptance number. With the candidates in depth
 * order, candidate k's term in the estimator above is
 *   [all j < k rejected] [u_k >= alpha_k] <dL, c_k - X_k> / (1 - alpha_k),
 * X_k the colour of the first accepted candidate behind k (bg if none),
 * which does not depend on u_k. Its mean over u_k is
 *   [all j < k rejected] <dL, c_k - X_k>,
 * still with expectation T_k (c_k - B_k) = dL/dalpha_k and, by the
 * Rao-Blackwell theorem, no larger variance. On a sample whose first and
 * second accepted candidates are a and a2: every k in front of a gets
 * <dL, c_k - c_a>, a gets <dL, c_a - c_a2> (c_a2 = bg if a has no accepted
 * candidate behind it), and the colour gradient still goes to a. */
void srto_estimator_grad_rb(int64_t G, const double* mu, const double* M, const double* op,
                            int deg, const float* sh, const float* log_scales,
                            const float* quats, const float* logits, int64_t R,
                            const float* o, const float* d, const float* tmin,
                            const float* tmax, const int32_t* ignore_gid,
                            const uint32_t* ray_id, const uint32_t* sample_base, int32_t spp,
                            uint64_t seed, uint32_t purpose, const double* bg,
                            int depth_mode, const double* depth_axis, const double* dL,
                            double* g_means, double* g_ls, double* g_quats, double* g_logits,
                            double* g_sh, int threads)
{
    rays_t RR = {R, o, d, tmin, tmax, ignore_gid, ray_id, sample_base};
    const depth_t dm = depth_of(depth_mode, depth_axis);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
    {
        sorted_t S = {{0, 0, 0}, 0, 0};
        double* sa = 0;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < R; ++i) {
            double t0, t1;
            int32_t ign;
            uint32_t rid, sb;
            ray_get(&RR, i, &t0, &t1, &ign, &rid, &sb);
            double Y[16], dir[3] = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
            srto_sh_basis(deg, dir, Y);
            sorted_build(&S, &dm, G, mu, M, op, deg, sh, o + 3 * i, d + 3 * i, t0, t1, ign, Y);
            int64_t n = S.cl.n;
            if (n == 0) continue;
            if (cap < n) {
                cap = n;
                sa = (double*)realloc(sa, (size_t)cap * sizeof(double));
            }
            memset(sa, 0, (size_t)n * sizeof(double));
            const double* g = dL + 3 * i;
            for (int32_t s = 0; s < spp; ++s) {
                uint32_t sample = sb + (uint32_t)s;
                /* first and second accepted candidates in depth order */
                int64_t a = -1, a2 = -1;
                for (int64_t k = 0; k < n; ++k) {
                    double u = accept_u(seed, rid, sample, (uint32_t)S.cl.v[k].gid, purpose);
                    if (u < S.cl.v[k].alpha) {
                        if (a < 0) {
                            a = k;
                        } else {
                            a2 = k;
                            break;
                        }
                    }
                }
                double X[3], X2[3];
                for (int ch = 0; ch < 3; ++ch) {
                    X[ch] = a >= 0 ? S.c[3 * a + ch] : bg[ch];
                    X2[ch] = a2 >= 0 ? S.c[3 * a2 + ch] : bg[ch];
                }
                int64_t front = a >= 0 ? a : n;
                for (int64_t k = 0; k < front; ++k) {
                    double v = 0.0;
                    for (int ch = 0; ch < 3; ++ch) v += g[ch] * (S.c[3 * k + ch] - X[ch]);
                    sa[k] += v / (double)spp;
                }
                if (a >= 0) {
                    double v = 0.0;
                    for (int ch = 0; ch < 3; ++ch) v += g[ch] * (X[ch] - X2[ch]);
                    sa[a] += v / (double)spp;
                    double gc[3] = {g[0] / spp, g[1] / spp, g[2] / spp};
                    chain_colour(deg, S.cl.v[a].gid, Y, S.pre + 3 * a, gc, g_sh);
                }
            }
            for (int64_t k = 0; k < n; ++k) {
                if (sa[k] == 0.0) continue;
                isect_t r;
                regeo(mu, M, S.cl.v[k].gid, o + 3 * i, d + 3 * i, &r);
                chain_alpha(S.cl.v[k].gid, sa[k], S.cl.v[k].alpha, &r, log_scales, quats,
                            logits, g_means, g_ls, g_quats, g_logits);
            }
        }
        free(S.cl.v);
        free(S.c);
        free(S.pre);
        free(sa);
    }
}

/* ------------------------------------------------------------------------ */
/* Path-tracer mix: Gaussians inside a renderer with shadows and mirror      */
/* reflections (Sec. 1 and Sec. 5: secondary rays go through the same       */
/* traversal). Per camera sample the shading point P is the nearer of the    */
/* accepted Gaussian and the ground plane y = plane_y; P spawns an any-hit   */
/* shadow ray toward a point light and, on the plane, a mirror ray.          */
/* Secondary rays are built with single correctly rounded FP32 operations in */
/* a fixed order (compiled without contraction), so an implementation that   */
/* performs the same operations obtains the same bits:                       */
/*   P = o + t*d (per component: o_i + (t*d_i)); on the plane P_y = plane_y; */
/*   v = light - P; len = sqrt((vx*vx + vy*vy) + vz*vz); l = v / len;        */
/*   shadow: (P, l, tmin = 1e-4, tmax = len, ignore = the spawning Gaussian) */
/*   mirror: (P, (dx, -dy, dz), tmin = 1e-4, tmax = inf).                    */
/* Colour: Gaussian c * (0.3 + 0.7 V); plane 0.5 V max(0, l_y) + 0.5 Lm,     */
/* Lm the mirror ray's Gaussian colour (bg on a miss); a miss of both: bg.   */
/* Secondary rays reuse the camera sample's ray id and sample index with     */
/* Philox purposes 2 (shadow) and 3 (mirror). `u_override`, when non-null,   */
/* replaces every acceptance number of Gaussian g (any ray, any purpose) by  */
/* u_override[g] (tests inject binary outcomes this way).                    */
/* ------------------------------------------------------------------------ */
void srto_pathmix(int64_t G, const double* mu, const double* M, const double* op, int deg,
                  const float* sh, int64_t R, const float* o, const float* d,
                  const uint32_t* ray_id, int32_t spp, uint64_t seed, const float* light,
                  float plane_y, const double* bg, const double* u_override, double* rgb,
                  int32_t* cam_gid, float* cam_t, uint8_t* shadow_vis, int32_t* mirror_gid,
                  uint8_t* flags, int threads)
{
    const depth_t dm = depth_of(0, 0);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
    {
        clist_t cam = {0, 0, 0}, sec = {0, 0, 0};
        const float tmin_sec = 1e-4f;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < R; ++i) {
            const float* oi = o + 3 * i;
            const float* di = d + 3 * i;
            uint32_t rid = ray_id ? ray_id[i] : (uint32_t)i;
            collect(&dm, G, mu, M, op, oi, di, 0.0, INFINITY, -1, &cam);
            double Y[16], dir[3] = {di[0], di[1], di[2]};
            srto_sh_basis(deg, dir, Y);
            float tp = INFINITY;
            if (di[1] < 0.0f) {
                float num = plane_y - oi[1];
                float tt = num / di[1];
                if (tt > 0.0f) tp = tt;
            }
            double acc[3] = {0, 0, 0};
            for (int32_t s = 0; s < spp; ++s) {
                int64_t k = i * spp + s;
                uint8_t f = 0, f2 = 0;
                double m;
                int64_t b = resolve(&cam, seed, rid, (uint32_t)s, 0u, 0, u_override, &f, &m);
                float tg = b >= 0 ? cam.v[b].t32 : INFINITY;
                int32_t gg = b >= 0 ? cam.v[b].gid : -1;
                if (cam_gid) cam_gid[k] = gg;
                if (cam_t) cam_t[k] = tg;
                uint8_t vis = 255;
                int32_t mg = -2;
                double col[3];
                int on_gauss = b >= 0 && tg <= tp;
                int on_plane = !on_gauss && tp < INFINITY;
                if (on_gauss || on_plane) {
                    float t = on_gauss ? tg : tp;
                    float P[3];
                    for (int c = 0; c < 3; ++c) {
                        float prod = t * di[c];
                        P[c] = oi[c] + prod;
                    }
                    if (on_plane) P[1] = plane_y;
                    float v[3] = {light[0] - P[0], light[1] - P[1], light[2] - P[2]};
                    float len2 = v[0] * v[0];
                    len2 = len2 + v[1] * v[1];
                    len2 = len2 + v[2] * v[2];
                    float len = sqrtf(len2);
                    float l[3] = {v[0] / len, v[1] / len, v[2] / len};
                    /* shadow ray: (P, l, tmin_sec, len, gg), any hit */
                    collect(&dm, G, mu, M, op, P, l, (double)tmin_sec, (double)len,
                            on_gauss ? gg : -1, &sec);
                    int64_t sb = resolve(&sec, seed, rid, (uint32_t)s, 2u, 1, u_override, &f2, &m);
                    f |= f2;
                    vis = sb >= 0 ? 0 : 1;
                    double V = (double)vis;
                    if (on_gauss) {
                        double c[3];
                        gauss_colour(deg, sh, gg, Y, c, 0);
                        for (int ch = 0; ch < 3; ++ch) col[ch] = c[ch] * (0.3 + 0.7 * V);
                    } else {
                        float md[3] = {di[0], -di[1], di[2]};
                        collect(&dm, G, mu, M, op, P, md, (double)tmin_sec, INFINITY, -1, &sec);
                        int64_t mb = resolve(&sec, seed, rid, (uint32_t)s, 3u, 0, u_override, &f2, &m);
                        f |= f2;
                        double Lm[3];
                        if (mb >= 0) {
                            double Ym[16], mdir[3] = {md[0], md[1], md[2]};
                            srto_sh_basis(deg, mdir, Ym);
                            gauss_colour(deg, sh, sec.v[mb].gid, Ym, Lm, 0);
                            mg = sec.v[mb].gid;
                        } else {
                            for (int ch = 0; ch < 3; ++ch) Lm[ch] = bg[ch];
                            mg = -1;
                        }
                        double nl = l[1] > 0.0f ? (double)l[1] : 0.0;
                        for (int ch = 0; ch < 3; ++ch) col[ch] = 0.5 * V * nl + 0.5 * Lm[ch];
                    }
                } else {
                    for (int ch = 0; ch < 3; ++ch) col[ch] = bg[ch];
                }
                for (int ch = 0; ch < 3; ++ch) acc[ch] += col[ch];
                if (shadow_vis) shadow_vis[k] = vis;
                if (mirror_gid) mirror_gid[k] = mg;
                if (flags) flags[k] = f;
            }
            if (rgb)
                for (int ch = 0; ch < 3; ++ch) rgb[3 * i + ch] = acc[ch] / (double)spp;
        }
        free(cam.v);
        free(sec.v);
    }
}
