/*
 * oracle.c -- plain FP64 CPU reference of the spherical 2D-Gaussian-surfel
 * rasterizer of Splat-LOAM (Giacomini et al., arXiv 2503.17491).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library; both sides are written from the paper and from the conventions
 * listed under "Readings" in the design notes.
 *
 * What each part follows:
 *   or_camera_matrix     Supp. A, equation for K({p_q}).
 *   or_pixel_basis       Sec. 3.1 (psi, phi^-1) and Sec. 3.2.2 (planes h_x, h_y).
 *   or_surfel_frame      Sec. 3.2 Eq. (world_T_splat) and Supp. D (T = T_cw H).
 *   pair_eval            Supp. D "Forward Process" (h_alpha, h_beta, p_hat,
 *                        s_hat, nu, d, alpha = o G(s_hat)).
 *   or_render_pixels     Sec. 3.2.1 Eqs. (ab_depth), (ab_normal), (ab_opacity),
 *                        brute force: every pixel ray against every surfel.
 *   or_backward_pixels   Supp. D "Gradient Computation", with the garbled
 *                        formulas read as the exact chain rule, the opacity
 *                        channel added, and the se(3) pose gradient for the
 *                        update T <- T exp(delta) of Sec. 3.3.3.
 *   *_mode(cull = 1)     the same render / backward with an angular cull that
 *                        skips only pairs whose support test must fail (the
 *                        ray's line misses the bounding sphere of the 3-sigma
 *                        square); pinned identical to brute force.
 *   or_render_variants   the admissible results of a pixel whose decisions lie
 *                        within rounding distance of a threshold: each such
 *                        decision taken both ways (Sec. 3.2.1 blending rules).
 *   or_bin               Sec. 3.2.1 (16x16 tiles, per-tile lists sorted by
 *                        range) and Sec. 3.2.3 / Supp. B (3-sigma splat box,
 *                        centre-relative azimuth extent, seam propagation),
 *                        computed as the exact angular box of the 3-sigma square.
 *
 * Parity pins (tests/test_oracle_*.py): closed forms for one and two surfels,
 * an independent textbook ray-plane solve, compositing invariants, seam mirror
 * symmetry and rotation equivariance, pose consistency, FP64 central finite
 * differences for every gradient, brute-force conservativeness of the box and
 * brute-force checks of the binning.  Nothing here is "parity unpinned" except
 * the conventions the paper leaves open (pixel centres, tie order, thresholds).
 *
 * Surfel parameters enter as FP64 arrays; the library's FP32 inputs are
 * promoted exactly by the Python front end, and finite-difference pins pass
 * FP64 values directly.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC.
 * Contraction must stay off: or_bin mirrors a fixed FP64 operation order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t height, width;
    double fu, cu, fv, cv, near_m;
} or_sensor;

/* Blending conventions taken from the 3DGS rasterizer that Sec. 3.2.1 says it
 * follows: skip alpha < 1/255, clamp alpha to 0.99, stop before T < 1e-4. */
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_ALPHA_MAX 0.99
#define OR_T_MIN 1e-4
/* 3-sigma support of the splat-space kernel (Sec. 3.2.3). */
#define OR_SUPPORT 3.0

/* guard-band flag bits reported per pixel */
#define OR_FLAG_SUPPORT 1
#define OR_FLAG_NEAR 2
#define OR_FLAG_AMIN 4
#define OR_FLAG_TSTOP 8
#define OR_FLAG_CLAMP 16
#define OR_FLAG_KEYTIE 32

/* ------------------------------------------------------------------------ */
/* Supp. A: camera matrix from the angular extent of a cloud and (H, W).     */
/* out = (fu, cu, fv, cv):  u = fu*azimuth + cu,  v = fv*elevation + cv.     */
/* ------------------------------------------------------------------------ */
void or_camera_matrix(double az_min, double az_max, double el_min, double el_max,
                      int32_t H, int32_t W, double *out)
{
    double fov_h = az_max - az_min;
    double fov_v = el_max - el_min;
    out[0] = -((double)W - 1.0) / fov_h;
    out[1] = (double)W / 2.0 * (1.0 + (az_max + az_min) / fov_h);
    out[2] = -((double)H - 1.0) / fov_v;
    out[3] = (double)H / 2.0 * (1.0 + (el_max + el_min) / fov_v);
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.1 / 3.2.2: direction of pixel (i, j) and its two planes.          */
/* Pixel centre convention: (u, v) = (j + 1/2, i + 1/2).                    */
/* ------------------------------------------------------------------------ */
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

void or_pixel_basis(const or_sensor *s, int32_t i, int32_t j, double *v, double *hx, double *hy)
{
    double u = (double)j + 0.5, vv = (double)i + 0.5;
    double az = (u - s->cu) / s->fu;     /* K^-1 u */
    double el = (vv - s->cv) / s->fv;
    v[0] = cos(el) * cos(az);           /* phi^-1 at unit range */
    v[1] = cos(el) * sin(az);
    v[2] = sin(el);
    double uz[3] = {0.0, 0.0, 1.0}, c[3];
    cross3(v, uz, c);                    /* h_x = v x u_z / |v x u_z| */
    double nc = sqrt(dot3(c, c));
    hx[0] = c[0] / nc; hx[1] = c[1] / nc; hx[2] = c[2] / nc;
    cross3(hx, v, hy);                   /* h_y = h_x x v */
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.2 / Supp. D: splat-to-sensor transform of one surfel.             */
/* Raw parameters: mean[3], quaternion (w,x,y,z) unnormalised, log-scales[2],*/
/* opacity logit.  Pose: T_cw as R (row-major 3x3) followed by t (3).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double ba[3], bb[3], bc[3], n[3];   /* T = T_cw H = (b_alpha b_beta b_c); n = R_cw t_n */
    double R[9];                         /* world rotation (t_alpha t_beta t_n) row-major */
    double qhat[4], qnorm;
    double s[2], o;
    float key;                           /* range sort key */
    int valid;
} or_frame;

static void quat_to_rot(const double *q, double *R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Range key of a surfel: FP32 rounding of |b_c| with b_c = R_cw mu + t_cw,
 * evaluated in FP64 in this exact order (shared convention with the GPU). */
static float mirror_key(const double *mu, const double *pose)
{
    double m0 = mu[0], m1 = mu[1], m2 = mu[2];
    double c[3];
    for (int r = 0; r < 3; ++r)
        c[r] = ((pose[3 * r + 0] * m0 + pose[3 * r + 1] * m1) + pose[3 * r + 2] * m2) + pose[9 + r];
    double r2 = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
    return (float)sqrt(r2);
}

static int finite_params(const double *mu, const double *q, const double *ls, double lo)
{
    for (int k = 0; k < 3; ++k) if (!isfinite(mu[k])) return 0;
    for (int k = 0; k < 4; ++k) if (!isfinite(q[k])) return 0;
    if (!isfinite(ls[0]) || !isfinite(ls[1]) || !isfinite(lo)) return 0;
    return 1;
}

void or_surfel_frame(const double *mu, const double *q, const double *ls, double logit,
                     const double *pose, double near_m, or_frame *f)
{
    memset(f, 0, sizeof(*f));
    if (!finite_params(mu, q, ls, logit)) return;
    double qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(qq > 0.0)) return;
    f->qnorm = sqrt(qq);
    for (int k = 0; k < 4; ++k) f->qhat[k] = q[k] / f->qnorm;
    quat_to_rot(f->qhat, f->R);
    f->s[0] = exp(ls[0]);
    f->s[1] = exp(ls[1]);
    f->o = 1.0 / (1.0 + exp(-logit));
    const double *Rc = pose, *tc = pose + 9;
    for (int r = 0; r < 3; ++r) {
        double a = 0, b = 0, c = 0, nn = 0;
        for (int k = 0; k < 3; ++k) {
            a += Rc[3 * r + k] * f->s[0] * f->R[3 * k + 0];
            b += Rc[3 * r + k] * f->s[1] * f->R[3 * k + 1];
            c += Rc[3 * r + k] * mu[k];
            nn += Rc[3 * r + k] * f->R[3 * k + 2];
        }
        f->ba[r] = a; f->bb[r] = b; f->bc[r] = c + tc[r]; f->n[r] = nn;
    }
    f->key = mirror_key(mu, pose);
    /* cull: centre at or inside the near range */
    f->valid = sqrt(dot3(f->bc, f->bc)) > near_m;
}

/* ------------------------------------------------------------------------ */
/* Supp. D forward process for one (pixel, surfel) pair.                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t id;
    float key;
    double alpha, G, d;
    int clamped;
    double sh[2], ph[3], ha[3], hb[3], nu[3];
} or_pair;

/* Returns 1 when the pair contributes. *flags collects guard-band bits. */
static int pair_eval(const or_frame *f, const double *v, const double *hx, const double *hy,
                     double near_m, const double *guard, or_pair *p, int *flags)
{
    /* h_alpha = T^T h_x, h_beta = T^T h_y (planes through the origin: 4th coordinate 0) */
    p->ha[0] = dot3(hx, f->ba); p->ha[1] = dot3(hx, f->bb); p->ha[2] = dot3(hx, f->bc);
    p->hb[0] = dot3(hy, f->ba); p->hb[1] = dot3(hy, f->bb); p->hb[2] = dot3(hy, f->bc);
    cross3(p->ha, p->hb, p->ph);                        /* p_hat = h_alpha x h_beta */
    if (p->ph[2] == 0.0) return 0;
    p->sh[0] = p->ph[0] / p->ph[2];                     /* s_hat = (p_x, p_y) / p_z */
    p->sh[1] = p->ph[1] / p->ph[2];
    double m = fmax(fabs(p->sh[0]), fabs(p->sh[1]));
    if (guard && fabs(m - OR_SUPPORT) < guard[0]) *flags |= OR_FLAG_SUPPORT;
    if (!(m <= OR_SUPPORT)) return 0;                   /* 3-sigma square support */
    for (int k = 0; k < 3; ++k) p->nu[k] = p->sh[0] * f->ba[k] + p->sh[1] * f->bb[k] + f->bc[k];
    double t = dot3(p->nu, v);
    if (guard && fabs(t - near_m) < guard[1]) *flags |= OR_FLAG_NEAR;
    if (!(t > near_m)) return 0;                        /* intersection in front of the near range */
    p->d = sqrt(dot3(p->nu, p->nu));                    /* d = |nu| */
    p->G = exp(-0.5 * (p->sh[0] * p->sh[0] + p->sh[1] * p->sh[1]));
    double a = f->o * p->G;
    if (guard && fabs(a - OR_ALPHA_MIN) < guard[2] * OR_ALPHA_MIN) *flags |= OR_FLAG_AMIN;
    if (guard && fabs(a - OR_ALPHA_MAX) < guard[2] * OR_ALPHA_MAX) *flags |= OR_FLAG_CLAMP;
    if (a < OR_ALPHA_MIN) return 0;
    p->clamped = a > OR_ALPHA_MAX;
    p->alpha = p->clamped ? OR_ALPHA_MAX : a;
    p->key = f->key;
    return 1;
}

static int pair_cmp(const void *a, const void *b)
{
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct { or_pair *p; int64_t n, cap; } pair_list;
static void list_push(pair_list *L, const or_pair *p)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->p = (or_pair *)realloc(L->p, (size_t)L->cap * sizeof(or_pair));
    }
    L->p[L->n++] = *p;
}

/* ------------------------------------------------------------------------ */
/* Angular-cull mode: the same lists as brute force, found faster.           */
/*                                                                          */
/* A pair passes the support test only if the ray meets the splat square     */
/* {b_c + a b_alpha + b b_beta : |a|, |b| <= 3} (Sec. 3.2.3), whose points lie */
/* within r = 3 sqrt(s_alpha^2 + s_beta^2) of b_c (b_alpha, b_beta are       */
/* orthogonal).  The support test meets the plane along the whole line of   */
/* the ray (in front of or behind the sensor), so the line's direction +-v    */
/* lies in the cone of half-angle asin(r / |b_c|) around b_c when |b_c| > r: */
/* the test |v . c_hat| >= sqrt(1 - (r/|b_c|)^2) can only drop pairs whose   */
/* support test fails.                                                       */
/* r is taken 0.1 % larger (plus 1e-9 m) so that no pair near the support    */
/* threshold, which the guard band reports, is dropped either.  Directions    */
/* are bucketed in 2-degree azimuth x elevation bins: a surfel goes into every */
/* bin its cone's elevation interval [el_c - th, el_c + th] and azimuth      */
/* interval [az_c - asin(sin th / cos el_c), az_c + ...] (the extent of a     */
/* spherical cap) overlap, both widened by 1e-6 rad for rounding; caps that  */
/* reach a pole span every azimuth.  Angular distance bounds the elevation    */
/* difference, so the bin of a ray holds every surfel whose cone holds it;   */
/* a surfel also goes into the mirrored bins of the antipodal cone (the bin  */
/* grid is symmetric under v -> -v: elevation bin e -> NEL-1-e, azimuth bin  */
/* a -> a + NAZ/2), each bin at most once.                                   */
/* ------------------------------------------------------------------------ */
#define CULL_NAZ 180
#define CULL_NEL 90
#define CULL_MARGIN 1e-6
typedef struct cull_index {
    int64_t *start;   /* [CULL_NAZ * CULL_NEL + 1] */
    int32_t *ids;
    double *cone;     /* [n, 4]: c_hat, cosine limit (-2: no cull) */
} cull_index;

static int64_t cull_bin(const cull_index *cx, const double *v)
{
    (void)cx;
    const double PI = 3.14159265358979323846;
    double az = atan2(v[1], v[0]), el = atan2(v[2], hypot(v[0], v[1]));
    int ia = (int)floor((az + PI) / (2.0 * PI / CULL_NAZ));
    int ie = (int)floor((el + 0.5 * PI) / (PI / CULL_NEL));
    ia = ia < 0 ? 0 : (ia >= CULL_NAZ ? CULL_NAZ - 1 : ia);
    ie = ie < 0 ? 0 : (ie >= CULL_NEL ? CULL_NEL - 1 : ie);
    return (int64_t)ie * CULL_NAZ + ia;
}

/* Bin ranges of one surfel's cone: elevation bins [*e0, *e1], azimuth bins
 * [*a0, *a1] taken modulo CULL_NAZ (*a1 - *a0 + 1 >= CULL_NAZ: all). */
static void cull_ranges(const double *c, double sin_th, int *e0, int *e1, int *a0, int *a1)
{
    const double PI = 3.14159265358979323846;
    const double del = PI / CULL_NEL, daz = 2.0 * PI / CULL_NAZ;
    double th = asin(sin_th);
    double el_c = atan2(c[2], hypot(c[0], c[1])), az_c = atan2(c[1], c[0]);
    double lo = el_c - th - CULL_MARGIN, hi = el_c + th + CULL_MARGIN;
    *e0 = (int)floor((lo + 0.5 * PI) / del);
    *e1 = (int)floor((hi + 0.5 * PI) / del);
    if (*e0 < 0) *e0 = 0;
    if (*e1 >= CULL_NEL) *e1 = CULL_NEL - 1;
    if (lo <= -0.5 * PI || hi >= 0.5 * PI || !(cos(el_c) > sin_th)) { *a0 = 0; *a1 = CULL_NAZ - 1; return; }
    double r = sin_th / cos(el_c);
    double dz = (r >= 1.0 ? 0.5 * PI : asin(r)) * (1.0 + 1e-9) + CULL_MARGIN;
    *a0 = (int)floor((az_c - dz + PI) / daz);
    *a1 = (int)floor((az_c + dz + PI) / daz);
    if (*a1 - *a0 + 1 >= CULL_NAZ) { *a0 = 0; *a1 = CULL_NAZ - 1; }
}

static void cull_build(const or_frame *F, int64_t n, cull_index *cx)
{
    const int64_t NB = (int64_t)CULL_NAZ * CULL_NEL;
    cx->start = (int64_t *)calloc((size_t)NB + 1, sizeof(int64_t));
    cx->cone = (double *)malloc((size_t)(n > 0 ? n : 1) * 4 * sizeof(double));
    double *sth = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t k = 0; k < n; ++k) {
        double *c = cx->cone + 4 * k;
        c[0] = c[1] = c[2] = 0.0; c[3] = -2.0; sth[k] = -1.0;
        if (!F[k].valid) continue;
        const double *b = F[k].bc;
        double d = sqrt(dot3(b, b));
        double r = 3.0 * sqrt(F[k].s[0] * F[k].s[0] + F[k].s[1] * F[k].s[1]) * 1.001 + 1e-9;
        for (int q = 0; q < 3; ++q) c[q] = b[q] / d;
        if (d > r) {
            sth[k] = r / d;
            c[3] = sqrt(1.0 - sth[k] * sth[k]) - 1e-12;
        } else {
            sth[k] = 2.0;   /* the sensor lies inside the ball: every direction */
        }
    }
    /* two passes: count the bins of every surfel, then fill */
    unsigned char *mark = (unsigned char *)calloc((size_t)NB, 1);
    int64_t *touched = (int64_t *)malloc((size_t)NB * sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
        int64_t *fill = NULL;
        if (pass == 1) {
            for (int64_t b = 0; b < NB; ++b) cx->start[b + 1] += cx->start[b];
            cx->ids = (int32_t *)malloc((size_t)(cx->start[NB] > 0 ? cx->start[NB] : 1) * sizeof(int32_t));
            fill = (int64_t *)malloc((size_t)NB * sizeof(int64_t));
            memcpy(fill, cx->start, (size_t)NB * sizeof(int64_t));
        }
        for (int64_t k = 0; k < n; ++k) {
            if (!(sth[k] >= 0.0)) continue;
            int e0, e1, a0, a1;
            if (sth[k] >= 1.0) { e0 = 0; e1 = CULL_NEL - 1; a0 = 0; a1 = CULL_NAZ - 1; }
            else cull_ranges(cx->cone + 4 * k, sth[k], &e0, &e1, &a0, &a1);
            int64_t nt = 0;
            for (int mirror = 0; mirror < 2; ++mirror)
                for (int e = e0; e <= e1; ++e)
                    for (int a = a0; a <= a1; ++a) {
                        int ee = mirror ? CULL_NEL - 1 - e : e;
                        int aa = (((a + (mirror ? CULL_NAZ / 2 : 0)) % CULL_NAZ) + CULL_NAZ) % CULL_NAZ;
                        int64_t b = (int64_t)ee * CULL_NAZ + aa;
                        if (mark[b]) continue;
                        mark[b] = 1;
                        touched[nt++] = b;
                        if (pass == 0) cx->start[b + 1] += 1;
                        else cx->ids[fill[b]++] = (int32_t)k;
                    }
            for (int64_t t = 0; t < nt; ++t) mark[touched[t]] = 0;
        }
        free(fill);
    }
    free(mark);
    free(touched);
    free(sth);
}

static void cull_free(cull_index *cx) { free(cx->start); free(cx->ids); free(cx->cone); }

/* Gather and sort the contributors of one pixel ray; returns the number of
 * pairs kept after the front-to-back stop rule (T_before * (1 - alpha) < 1e-4
 * ends the list before that pair). */
static int64_t pixel_list(const or_frame *F, int64_t n, const double *v, const double *hx,
                          const double *hy, double near_m, const double *guard, pair_list *L,
                          int *flags, const struct cull_index *cx)
{
    L->n = 0;
    if (cx) {
        /* angular-cull mode: only the surfels of the pixel's direction bin whose
         * bounding cone holds the ray (a superset of the pairs that can pass the
         * support test, so the list below is the brute-force list) */
        int64_t b = cull_bin(cx, v), e = cx->start[b + 1];
        for (int64_t q = cx->start[b]; q < e; ++q) {
            int32_t k = cx->ids[q];
            const double *c = cx->cone + 4 * (int64_t)k;
            if (fabs(v[0] * c[0] + v[1] * c[1] + v[2] * c[2]) < c[3]) continue;
            or_pair p;
            if (pair_eval(&F[k], v, hx, hy, near_m, guard, &p, flags)) { p.id = k; list_push(L, &p); }
        }
    } else {
        for (int64_t k = 0; k < n; ++k) {
            if (!F[k].valid) continue;
            or_pair p;
            if (pair_eval(&F[k], v, hx, hy, near_m, guard, &p, flags)) { p.id = (int32_t)k; list_push(L, &p); }
        }
    }
    qsort(L->p, (size_t)L->n, sizeof(or_pair), pair_cmp);
    for (int64_t c = 1; c < L->n; ++c)
        if (L->p[c].key == L->p[c - 1].key) *flags |= OR_FLAG_KEYTIE;
    double T = 1.0;
    int64_t m = 0;
    for (; m < L->n; ++m) {
        double test_T = T * (1.0 - L->p[m].alpha);
        if (guard && fabs(test_T - OR_T_MIN) < guard[3] * OR_T_MIN) *flags |= OR_FLAG_TSTOP;
        if (test_T < OR_T_MIN) break;
        T = test_T;
    }
    return m;
}

static or_frame *build_frames(int64_t n, const double *means, const double *quats, const double *ls,
                              const double *logits, const double *pose, double near_m)
{
    or_frame *F = (or_frame *)malloc((size_t)(n > 0 ? n : 1) * sizeof(or_frame));
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k)
        or_surfel_frame(means + 3 * k, quats + 4 * k, ls + 2 * k, logits[k], pose, near_m, &F[k]);
    return F;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.2.1 Eqs. (ab_depth)/(ab_normal)/(ab_opacity) for a list of pixels. */
/* guard (nullable): widths of the guard bands {support, near [m],          */
/* alpha (relative), T-stop (relative)}.                                     */
/* ------------------------------------------------------------------------ */
/* cull = 1: the angular-cull mode (identical results, fewer pairs tested). */
int or_render_pixels_mode(int64_t n, const double *means, const double *quats, const double *log_scales,
                          const double *logits, const double *pose, const or_sensor *s,
                          int64_t P, const int32_t *pix, const double *guard,
                          double *depth, double *normal, double *alpha, double *T_final,
                          int32_t *n_contrib, int32_t *flags, int32_t cull)
{
    if (n < 0 || P < 0 || !s) return -1;
    or_frame *F = build_frames(n, means, quats, log_scales, logits, pose, s->near_m);
    cull_index cxs, *cx = NULL;
    if (cull) { cull_build(F, n, &cxs); cx = &cxs; }
    #pragma omp parallel
    {
        pair_list L = {0, 0, 0};
        #pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < P; ++q) {
            double v[3], hx[3], hy[3];
            or_pixel_basis(s, pix[2 * q], pix[2 * q + 1], v, hx, hy);
            int fl = 0;
            int64_t m = pixel_list(F, n, v, hx, hy, s->near_m, guard, &L, &fl, cx);
            double T = 1.0, D = 0.0, N[3] = {0, 0, 0}, O = 0.0;
            for (int64_t c = 0; c < m; ++c) {
                const or_pair *p = &L.p[c];
                double w = p->alpha * T;                 /* o_i G_i prod_{j<i} (1 - o_j G_j) */
                D += w * p->d;
                for (int k = 0; k < 3; ++k) N[k] += w * F[p->id].n[k];
                O += w;
                T *= 1.0 - p->alpha;
            }
            depth[q] = D; alpha[q] = O;
            for (int k = 0; k < 3; ++k) normal[3 * q + k] = N[k];
            if (T_final) T_final[q] = T;
            if (n_contrib) n_contrib[q] = (int32_t)m;
            if (flags) flags[q] = fl;
        }
        free(L.p);
    }
    if (cx) cull_free(cx);
    free(F);
    return 0;
}

int or_render_pixels(int64_t n, const double *means, const double *quats, const double *log_scales,
                     const double *logits, const double *pose, const or_sensor *s,
                     int64_t P, const int32_t *pix, const double *guard,
                     double *depth, double *normal, double *alpha, double *T_final,
                     int32_t *n_contrib, int32_t *flags)
{
    return or_render_pixels_mode(n, means, quats, log_scales, logits, pose, s, P, pix, guard, depth, normal,
                                 alpha, T_final, n_contrib, flags, 0);
}

/* ------------------------------------------------------------------------ */
/* Guard-band variants of a pixel.                                          */
/*                                                                          */
/* Where the FP64 value of a decision lies within rounding distance of its  */
/* threshold (the guard band: the 3-sigma support, the near range, the      */
/* 1/255 alpha floor, the 1e-4 transmittance stop), an FP32 evaluation may   */
/* take it either way, and both outcomes are results of the method.  For a  */
/* pixel, the pairs whose inclusion hangs on such decisions and the stop    */
/* tests that fall in the band are branched on, both ways, in list order (a */
/* depth-first walk of Eqs. ab_depth / ab_normal / ab_opacity); every leaf  */
/* is one admissible (D, N, O).  The walk with no branch taken is the plain */
/* render of or_render_pixels, bit for bit (slot 0).  At most max_flips     */
/* branches are taken along a path; a pixel that needs more reports         */
/* overflow.  The alpha clamp is continuous in the forward and not branched. */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t id;
    float key;
    int contrib;     /* the decisions as evaluated */
    int flip_inc;    /* a flagged decision can turn the inclusion around */
    double alpha, d;
} ext_pair;

static int ext_cmp(const void *a, const void *b)
{
    const ext_pair *x = (const ext_pair *)a, *y = (const ext_pair *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;   /* near to far, then by index */
    return (x->id > y->id) - (x->id < y->id);
}

/* Evaluates every decision of one pair; returns 1 if the pair contributes or
 * a flagged decision could make it contribute (then *e is filled). */
static int pair_eval_ext(const or_frame *f, const double *v, const double *hx, const double *hy, double near_m,
                         const double *guard, ext_pair *e)
{
    double ha[3], hb[3], ph[3], sh[2], nu[3];
    ha[0] = dot3(hx, f->ba); ha[1] = dot3(hx, f->bb); ha[2] = dot3(hx, f->bc);
    hb[0] = dot3(hy, f->ba); hb[1] = dot3(hy, f->bb); hb[2] = dot3(hy, f->bc);
    cross3(ha, hb, ph);
    if (ph[2] == 0.0) return 0;
    sh[0] = ph[0] / ph[2];
    sh[1] = ph[1] / ph[2];
    double m = fmax(fabs(sh[0]), fabs(sh[1]));
    int sup = m <= OR_SUPPORT, fsup = fabs(m - OR_SUPPORT) < guard[0];
    for (int k = 0; k < 3; ++k) nu[k] = sh[0] * f->ba[k] + sh[1] * f->bb[k] + f->bc[k];
    double t = dot3(nu, v);
    int nr = t > near_m, fnr = fabs(t - near_m) < guard[1];
    double d = sqrt(dot3(nu, nu));
    double G = exp(-0.5 * (sh[0] * sh[0] + sh[1] * sh[1]));
    double a = f->o * G;
    int am = !(a < OR_ALPHA_MIN), fam = fabs(a - OR_ALPHA_MIN) < guard[2] * OR_ALPHA_MIN;
    e->contrib = sup && nr && am;
    if (e->contrib)
        e->flip_inc = fsup || fnr || fam;
    else
        e->flip_inc = (sup || fsup) && (nr || fnr) && (am || fam);
    if (!e->contrib && !e->flip_inc) return 0;
    e->alpha = a > OR_ALPHA_MAX ? OR_ALPHA_MAX : a;
    e->d = d;
    e->key = f->key;
    return 1;
}

typedef struct {
    const ext_pair *p;
    int64_t n;
    const or_frame *F;
    double gT;
    int max_flips, cap, nout, overflow;
    double *D, *N, *O;   /* [cap], [cap, 3], [cap]; slot 0 = no branch taken */
    int have_base;
} vwalk_ctx;

static void vwalk_emit(vwalk_ctx *c, int flips, double D, const double *N, double O)
{
    int slot;
    if (flips == 0) { slot = 0; c->have_base = 1; }
    else {
        if (c->nout >= c->cap) { c->overflow = 1; return; }
        slot = c->nout;
    }
    c->D[slot] = D; c->O[slot] = O;
    for (int k = 0; k < 3; ++k) c->N[3 * slot + k] = N[k];
    if (flips != 0) c->nout++;
}

/* Composites from list position i with state (T, D, N, O); force_inc /
 * force_stop (-1: none) impose the outcome of pair i's decisions. */
static void vwalk(vwalk_ctx *c, int64_t i, double T, double D, const double *N0, double O, int flips,
                  int force_inc, int force_stop)
{
    double N[3] = {N0[0], N0[1], N0[2]};
    for (; i < c->n; ++i) {
        const ext_pair *p = &c->p[i];
        int inc = p->contrib;
        if (force_inc >= 0) {
            inc = force_inc;
            force_inc = -1;
        } else if (p->flip_inc) {
            if (flips < c->max_flips) vwalk(c, i, T, D, N, O, flips + 1, !inc, -1);
            else c->overflow = 1;
        }
        if (!inc) continue;
        double tT = T * (1.0 - p->alpha);
        int stop = tT < OR_T_MIN;
        if (force_stop >= 0) {
            stop = force_stop;
            force_stop = -1;
        } else if (fabs(tT - OR_T_MIN) < c->gT * OR_T_MIN) {
            if (flips < c->max_flips) vwalk(c, i, T, D, N, O, flips + 1, 1, !stop);
            else c->overflow = 1;
        }
        if (stop) break;
        double w = p->alpha * T;
        D += w * p->d;
        for (int k = 0; k < 3; ++k) N[k] += w * c->F[p->id].n[k];
        O += w;
        T = tT;
    }
    vwalk_emit(c, flips, D, N, O);
}

/* For each listed pixel: nvar[q] admissible results (slot 0 = the plain
 * render) in depth [P, cap], normal [P, cap, 3], alpha [P, cap], with
 * cap = 2^max_flips (max_flips in [0, 6]); overflow[q] = 1 when a path needed
 * more than max_flips branches or more than cap results. */
int or_render_variants(int64_t n, const double *means, const double *quats, const double *log_scales,
                       const double *logits, const double *pose, const or_sensor *s, int64_t P, const int32_t *pix,
                       const double *guard, int32_t max_flips, double *depth, double *normal, double *alpha,
                       int32_t *nvar, int32_t *overflow, int32_t cull)
{
    if (n < 0 || P < 0 || !s || !guard || max_flips < 0 || max_flips > 6) return -1;
    const int cap = 1 << max_flips;
    or_frame *F = build_frames(n, means, quats, log_scales, logits, pose, s->near_m);
    cull_index cxs, *cx = NULL;
    if (cull) { cull_build(F, n, &cxs); cx = &cxs; }
    #pragma omp parallel
    {
        ext_pair *buf = NULL;
        int64_t nb = 0, cb = 0;
        #pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < P; ++q) {
            double v[3], hx[3], hy[3];
            or_pixel_basis(s, pix[2 * q], pix[2 * q + 1], v, hx, hy);
            nb = 0;
            int64_t b0 = 0, b1 = n;
            if (cx) { int64_t b = cull_bin(cx, v); b0 = cx->start[b]; b1 = cx->start[b + 1]; }
            for (int64_t r = b0; r < b1; ++r) {
                int32_t k = cx ? cx->ids[r] : (int32_t)r;
                if (!F[k].valid) continue;
                if (cx) {
                    const double *c = cx->cone + 4 * (int64_t)k;
                    if (fabs(v[0] * c[0] + v[1] * c[1] + v[2] * c[2]) < c[3]) continue;
                }
                ext_pair e;
                if (!pair_eval_ext(&F[k], v, hx, hy, s->near_m, guard, &e)) continue;
                e.id = k;
                if (nb == cb) { cb = cb ? 2 * cb : 64; buf = (ext_pair *)realloc(buf, (size_t)cb * sizeof(ext_pair)); }
                buf[nb++] = e;
            }
            qsort(buf, (size_t)nb, sizeof(ext_pair), ext_cmp);
            vwalk_ctx c = {buf, nb, F, guard[3], max_flips, cap, 1, 0,
                           depth + (int64_t)cap * q, normal + 3 * (int64_t)cap * q, alpha + (int64_t)cap * q, 0};
            const double N0[3] = {0.0, 0.0, 0.0};
            vwalk(&c, 0, 1.0, 0.0, N0, 0.0, 0, -1, -1);
            nvar[q] = c.nout;
            overflow[q] = c.overflow || !c.have_base;
        }
        free(buf);
    }
    if (cx) cull_free(cx);
    free(F);
    return 0;
}

/* Supp. D, last block: gradients w.r.t. the raw parameters of one surfel from
 * its sensor-frame gradients g13 = (dL/db_alpha, dL/db_beta, dL/db_c, dL/dn,
 * dL/do).  out10 = (mean[3], quaternion[4], log-scales[2], logit[1]). */
static void raw_from_frame(const or_frame *f, const double *Rc, const double *g, double *out10)
{
    double *gm = out10, *gq = out10 + 3, *gl = out10 + 7;
    /* world-frame vectors: R_cw^T g */
    double wA[3], wB[3], wC[3], wN[3];
    for (int c = 0; c < 3; ++c) {
        wA[c] = Rc[c] * g[0] + Rc[3 + c] * g[1] + Rc[6 + c] * g[2];
        wB[c] = Rc[c] * g[3] + Rc[3 + c] * g[4] + Rc[6 + c] * g[5];
        wC[c] = Rc[c] * g[6] + Rc[3 + c] * g[7] + Rc[6 + c] * g[8];
        wN[c] = Rc[c] * g[9] + Rc[3 + c] * g[10] + Rc[6 + c] * g[11];
    }
    for (int c = 0; c < 3; ++c) gm[c] = wC[c];                       /* dL/dmu */
    double ta[3] = {f->R[0], f->R[3], f->R[6]}, tb[3] = {f->R[1], f->R[4], f->R[7]};
    gl[0] = f->s[0] * dot3(wA, ta);                                  /* dL/dlog s_alpha */
    gl[1] = f->s[1] * dot3(wB, tb);
    out10[9] = f->o * (1.0 - f->o) * g[12];                          /* dL/dlogit */
    /* dL/dR with columns (s_a wA, s_b wB, wN) */
    double GR[9];
    for (int r = 0; r < 3; ++r) {
        GR[3 * r + 0] = f->s[0] * wA[r];
        GR[3 * r + 1] = f->s[1] * wB[r];
        GR[3 * r + 2] = wN[r];
    }
    double w = f->qhat[0], x = f->qhat[1], y = f->qhat[2], z = f->qhat[3];
    double dRw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    double dRx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    double dRy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    double dRz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    double gh[4] = {0, 0, 0, 0};
    for (int e = 0; e < 9; ++e) {
        gh[0] += GR[e] * dRw[e]; gh[1] += GR[e] * dRx[e];
        gh[2] += GR[e] * dRy[e]; gh[3] += GR[e] * dRz[e];
    }
    double proj = gh[0] * w + gh[1] * x + gh[2] * y + gh[3] * z;   /* through q / |q| */
    for (int c = 0; c < 4; ++c) gq[c] = (gh[c] - proj * f->qhat[c]) / f->qnorm;
}

/* ------------------------------------------------------------------------ */
/* Supp. D gradient computation for the pixels in the list, with upstream   */
/* dL/dD, dL/dN (3) and dL/dO per listed pixel.  Outputs are overwritten:    */
/* gradients w.r.t. the raw parameters (mean, unnormalised quaternion,       */
/* log-scales, opacity logit) and w.r.t. delta = (rho; phi) in se(3) for     */
/* T_cw(delta) = exp(-delta^) T_cw, i.e. the sensor pose update              */
/* T_wc <- T_wc exp(delta) of Sec. 3.3.3.  g_abs (nullable, [n,10]) receives */
/* per surfel the sum over pixels of |per-pixel contribution| to each raw    */
/* parameter gradient: the scale an FP32 accumulation error is measured by.  */
/* ------------------------------------------------------------------------ */
int or_backward_pixels_mode(int64_t n, const double *means, const double *quats, const double *log_scales,
                            const double *logits, const double *pose, const or_sensor *s,
                            int64_t P, const int32_t *pix,
                            const double *dL_dD, const double *dL_dN, const double *dL_dO,
                            double *g_means, double *g_quats, double *g_log_scales, double *g_logits,
                            double *g_pose, double *g_abs, int32_t cull)
{
    if (n < 0 || P < 0 || !s) return -1;
    or_frame *F = build_frames(n, means, quats, log_scales, logits, pose, s->near_m);
    cull_index cxs, *cx = NULL;
    if (cull) { cull_build(F, n, &cxs); cx = &cxs; }
    /* per-surfel sensor-frame accumulators: g_alpha, g_beta, g_c, g_n (3 each), g_o */
    double *acc = (double *)calloc((size_t)(n > 0 ? n : 1) * 13, sizeof(double));
    if (g_abs) memset(g_abs, 0, (size_t)(n > 0 ? n : 0) * 10 * sizeof(double));
    #pragma omp parallel
    {
        pair_list L = {0, 0, 0};
        double *Apre = NULL; int64_t Acap = 0;
        #pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < P; ++q) {
            double gD = dL_dD ? dL_dD[q] : 0.0, gO = dL_dO ? dL_dO[q] : 0.0;
            double gN[3] = {0, 0, 0};
            if (dL_dN) for (int k = 0; k < 3; ++k) gN[k] = dL_dN[3 * q + k];
            double v[3], hx[3], hy[3];
            or_pixel_basis(s, pix[2 * q], pix[2 * q + 1], v, hx, hy);
            int fl = 0;
            int64_t m = pixel_list(F, n, v, hx, hy, s->near_m, NULL, &L, &fl, cx);
            if (m + 1 > Acap) { Acap = 2 * (m + 1); Apre = (double *)realloc(Apre, (size_t)Acap * sizeof(double)); }
            /* A_k = prod_{i<k} (1 - alpha_i), by definition (forward prefix products) */
            Apre[0] = 1.0;
            for (int64_t c = 0; c < m; ++c) Apre[c + 1] = Apre[c] * (1.0 - L.p[c].alpha);
            double Tfin = Apre[m];
            double Bd = 0.0, Bn[3] = {0, 0, 0};          /* suffix sums over i > k */
            for (int64_t c = m - 1; c >= 0; --c) {
                const or_pair *p = &L.p[c];
                const or_frame *f = &F[p->id];
                double A = Apre[c], a = p->alpha, om = 1.0 - a;
                /* dL/dalpha_k: depth, normal and opacity channels */
                double dA = gD * (p->d * A - Bd / om);
                for (int k = 0; k < 3; ++k) dA += gN[k] * (f->n[k] * A - Bn[k] / om);
                dA += gO * Tfin / om;
                double w = a * A;
                Bd += p->d * w;
                for (int k = 0; k < 3; ++k) Bn[k] += f->n[k] * w;
                double gd = gD * w;                      /* dL/dd_k */
                /* dL/ds_hat: through alpha = o G(s_hat) and through d = |nu| */
                double gs[2];
                double nba = dot3(p->nu, f->ba), nbb = dot3(p->nu, f->bb);
                gs[0] = gd * nba / p->d; gs[1] = gd * nbb / p->d;
                if (!p->clamped) { gs[0] -= dA * a * p->sh[0]; gs[1] -= dA * a * p->sh[1]; }
                /* dL/dp_hat through s_hat = (p_x, p_y) / p_z */
                double pz = p->ph[2];
                double gp[3] = {gs[0] / pz, gs[1] / pz, -(p->ph[0] * gs[0] + p->ph[1] * gs[1]) / (pz * pz)};
                double ra[3], rb[3];
                cross3(gp, p->ha, ra);                   /* rho_alpha */
                cross3(gp, p->hb, rb);                   /* rho_beta */
                double gA[3], gB[3], gC[3];
                for (int k = 0; k < 3; ++k) {
                    gA[k] = -rb[0] * hx[k] + ra[0] * hy[k] + gd * p->sh[0] * p->nu[k] / p->d;
                    gB[k] = -rb[1] * hx[k] + ra[1] * hy[k] + gd * p->sh[1] * p->nu[k] / p->d;
                    gC[k] = -rb[2] * hx[k] + ra[2] * hy[k] + gd * p->nu[k] / p->d;
                }
                double go = p->clamped ? 0.0 : dA * p->G;
                double *g = acc + 13 * (int64_t)p->id;
                if (g_abs) {
                    double g13[13], r10[10];
                    for (int k = 0; k < 3; ++k) {
                        g13[k] = gA[k]; g13[3 + k] = gB[k]; g13[6 + k] = gC[k]; g13[9 + k] = gN[k] * w;
                    }
                    g13[12] = go;
                    raw_from_frame(f, pose, g13, r10);
                    double *ga = g_abs + 10 * (int64_t)p->id;
                    for (int k = 0; k < 10; ++k) {
                        #pragma omp atomic
                        ga[k] += fabs(r10[k]);
                    }
                }
                for (int k = 0; k < 3; ++k) {
                    #pragma omp atomic
                    g[k] += gA[k];
                    #pragma omp atomic
                    g[3 + k] += gB[k];
                    #pragma omp atomic
                    g[6 + k] += gC[k];
                    #pragma omp atomic
                    g[9 + k] += gN[k] * w;               /* dL/dn_k */
                }
                #pragma omp atomic
                g[12] += go;
            }
        }
        free(L.p);
        free(Apre);
    }
    /* per-surfel parameter gradients (Supp. D, last block) and the pose gradient */
    const double *Rc = pose;
    double gpose[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = 0; k < n; ++k) {
        const or_frame *f = &F[k];
        const double *g = acc + 13 * k;
        double *gm = g_means + 3 * k, *gq = g_quats + 4 * k, *gl = g_log_scales + 2 * k;
        memset(gm, 0, 3 * sizeof(double)); memset(gq, 0, 4 * sizeof(double));
        gl[0] = gl[1] = 0.0; g_logits[k] = 0.0;
        if (!f->valid) continue;
        double r10[10];
        raw_from_frame(f, Rc, g, r10);
        for (int c = 0; c < 3; ++c) gm[c] = r10[c];
        for (int c = 0; c < 4; ++c) gq[c] = r10[3 + c];
        gl[0] = r10[7]; gl[1] = r10[8];
        g_logits[k] = r10[9];
        /* pose: d b / d rho = -I, d b / d phi = [b]_x for every sensor-frame vector */
        double t1[3], t2[3], t3[3], t4[3];
        cross3(g + 6, f->bc, t1); cross3(g + 0, f->ba, t2);
        cross3(g + 3, f->bb, t3); cross3(g + 9, f->n, t4);
        for (int c = 0; c < 3; ++c) {
            gpose[c] -= g[6 + c];
            gpose[3 + c] += t1[c] + t2[c] + t3[c] + t4[c];
        }
    }
    if (g_pose) memcpy(g_pose, gpose, sizeof(gpose));
    free(acc);
    if (cx) cull_free(cx);
    free(F);
    return 0;
}

int or_backward_pixels(int64_t n, const double *means, const double *quats, const double *log_scales,
                       const double *logits, const double *pose, const or_sensor *s,
                       int64_t P, const int32_t *pix,
                       const double *dL_dD, const double *dL_dN, const double *dL_dO,
                       double *g_means, double *g_quats, double *g_log_scales, double *g_logits,
                       double *g_pose, double *g_abs)
{
    return or_backward_pixels_mode(n, means, quats, log_scales, logits, pose, s, P, pix, dL_dD, dL_dN, dL_dO,
                                   g_means, g_quats, g_log_scales, g_logits, g_pose, g_abs, 0);
}

/* ======================================================================== */
/* Binning (Sec. 3.2.1, Sec. 3.2.3, Supp. B).                               */
/*                                                                          */
/* The box is the exact angular box of the 3-sigma splat square            */
/* {b_c + a A + b B : |a|,|b| <= 1}, A = 3 s_a R_cw t_a, B = 3 s_b R_cw t_b,  */
/* widened by an angular margin.  Every step uses only IEEE-exact FP64       */
/* +,-,*,/,sqrt in a fixed order plus the sensor direction tables, so that   */
/* the integer outputs are reproducible bit for bit.                         */
/* ======================================================================== */

/* exp for the box scales: range reduction by ln 2 and a degree-13 Taylor
 * polynomial (textbook method; accurate to a few ulp, reproducible). */
static double box_exp(double x)
{
    const double LN2 = 0.6931471805599453;
    const double INV_LN2 = 1.4426950408889634;
    double k = floor(x * INV_LN2 + 0.5);
    double r = x - k * LN2;
    double p = 1.0 / 6227020800.0;            /* 1/13! */
    p = p * r + 1.0 / 479001600.0;            /* 1/12! */
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

static double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

/* angle(a) <= angle(b) for angles in (-pi, pi] */
static int ang_le(double ax, double ay, double bx, double by)
{
    int ha = (ay > 0.0) || (ay == 0.0 && ax < 0.0);
    int hb = (by > 0.0) || (by == 0.0 && bx < 0.0);
    if (ha != hb) return ha < hb;
    return cross2(ax, ay, bx, by) >= 0.0;
}

/* Sensor direction tables (FP64, host libm). */
typedef struct {
    int32_t H, W;
    double *col;     /* [W][2]  (cos az_j, sin az_j) of column centres */
    double *rlo;     /* [H][2]  (cos, sin) of el_i - margin */
    double *rhi;     /* [H][2]  (cos, sin) of el_i + margin */
    double cm, sm;   /* cos, sin of the margin */
} box_tables;

static void tables_make(const or_sensor *s, double margin, box_tables *T)
{
    T->H = s->height; T->W = s->width;
    T->col = (double *)malloc(sizeof(double) * 2 * (size_t)s->width);
    T->rlo = (double *)malloc(sizeof(double) * 2 * (size_t)s->height);
    T->rhi = (double *)malloc(sizeof(double) * 2 * (size_t)s->height);
    for (int32_t j = 0; j < s->width; ++j) {
        double az = (((double)j + 0.5) - s->cu) / s->fu;
        T->col[2 * j] = cos(az); T->col[2 * j + 1] = sin(az);
    }
    for (int32_t i = 0; i < s->height; ++i) {
        double el = (((double)i + 0.5) - s->cv) / s->fv;
        T->rlo[2 * i] = cos(el - margin); T->rlo[2 * i + 1] = sin(el - margin);
        T->rhi[2 * i] = cos(el + margin); T->rhi[2 * i + 1] = sin(el + margin);
    }
    T->cm = cos(margin); T->sm = sin(margin);
}
static void tables_free(box_tables *T) { free(T->col); free(T->rlo); free(T->rhi); }

/* Elevation order of two points given as (r, z) with r >= 0:  el(a) < el(b). */
static int el_lt(double ra, double za, double rb, double zb) { return za * rb - ra * zb < 0.0; }

/* Per-surfel box.  Writes rows [r0, r1] and up to two column intervals.
 * Returns the number of column intervals (0 = culled). */
/* Box modes: 0 the exact angular box of the 3-sigma square (R12); 1 the same
 * box of the opacity-aware square below; 2 the paper's relaxed box (Supp. B):
 * the angular extent of the four projected vertices only, which can miss
 * pixels where an edge bulges beyond its vertices or the sensor's axis
 * pierces the square.
 *
 * Opacity-aware support radius (box mode 1).  A pair contributes only when
 * alpha = o G >= 1/255 (R7), i.e. inside the disk |s_hat|^2 <= 2 ln(255 o);
 * the square of half-side r = k/16 bounds it for the smallest integer k with
 * 255 o exp(-(k/16)^2 / 2) <= 0.999 (a 0.1 % margin over the threshold),
 * found by binary search with the reproducible exp, so that both sides take
 * the same integer decision.  Returns 0 when no pixel can reach the threshold
 * (255 o <= 0.999) and 3 when the disk is not smaller than the 3-sigma
 * square. */
static double support_radius(double logit)
{
    double o = 1.0 / (1.0 + box_exp(-logit));
    double c = 255.0 * o;
    if (c <= 0.999) return 0.0;
    if (!(c * box_exp(-(48.0 * 48.0) / 512.0) <= 0.999)) return 3.0;
    int lo = 1, hi = 48;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (c * box_exp(-(double)(mid * mid) / 512.0) <= 0.999) hi = mid; else lo = mid + 1;
    }
    return (double)lo / 16.0;
}

static int surfel_box(const double *mu, const double *q, const double *ls, double logit, const double *pose,
                      double near_m, const box_tables *T, int32_t box_mode, int32_t *rows, int32_t *cols)
{
    if (!finite_params(mu, q, ls, logit)) return 0;
    double rad = 3.0;
    if (box_mode == 1) {
        rad = support_radius(logit);
        if (rad == 0.0) return 0;
    }
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double qq = ((w * w + x * x) + y * y) + z * z;
    if (!(qq > 0.0)) return 0;
    double qn = sqrt(qq);
    w = w / qn; x = x / qn; y = y / qn; z = z / qn;
    /* first two columns of R(q) */
    double ta[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
    double tb[3] = {2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x)};
    double sa = rad * box_exp(ls[0]), sb = rad * box_exp(ls[1]);
    double Aw[3] = {sa * ta[0], sa * ta[1], sa * ta[2]};
    double Bw[3] = {sb * tb[0], sb * tb[1], sb * tb[2]};
    double A[3], B[3], C[3];
    double m0 = mu[0], m1 = mu[1], m2 = mu[2];
    for (int r = 0; r < 3; ++r) {
        const double *Rr = pose + 3 * r;
        A[r] = (Rr[0] * Aw[0] + Rr[1] * Aw[1]) + Rr[2] * Aw[2];
        B[r] = (Rr[0] * Bw[0] + Rr[1] * Bw[1]) + Rr[2] * Bw[2];
        C[r] = ((Rr[0] * m0 + Rr[1] * m1) + Rr[2] * m2) + pose[9 + r];
    }
    double range = sqrt((C[0] * C[0] + C[1] * C[1]) + C[2] * C[2]);
    if (!(range > near_m)) return 0;

    const int32_t H = T->H, W = T->W;
    int full_az = 0, rows_top = 0, rows_bot = 0;   /* rows_top: extend to row 0; rows_bot: to row H-1 */
    /* Does the sensor's z-axis meet the square?  With n = A x B (det = n_z) the
     * axis meets the plane at height z* = (n.C)/det, and every point of the
     * square lies within Rb = |C| + |A| + |B| of the sensor.  E bounds the
     * rounding of n.C and det; each undecidable case widens the box. */
    double det = A[0] * B[1] - A[1] * B[0];
    double n0 = A[1] * B[2] - A[2] * B[1], n1 = A[2] * B[0] - A[0] * B[2];
    double sc = (n0 * C[0] + n1 * C[1]) + det * C[2];
    double an = sqrt((A[0] * A[0] + A[1] * A[1]) + A[2] * A[2]);
    double bn = sqrt((B[0] * B[0] + B[1] * B[1]) + B[2] * B[2]);
    double nn = sqrt((n0 * n0 + n1 * n1) + det * det);
    double Rb = (range + an) + bn;
    double E = 4e-15 * (an * bn);
    double as = fabs(sc);
    if (box_mode == 2) {
        /* vertex-only box (Supp. B's relaxed box): no pierce test */
    } else if (!(as > (1e-9 * Rb) * nn + E * range)) {
        full_az = 1; rows_top = 1; rows_bot = 1;      /* sensor (nearly) in the square's plane */
    } else if (as - E * range > Rb * (fabs(det) + E)) {
        /* the axis meets the plane beyond the square, or never (plane parallel to it) */
    } else if (!(fabs(det) >= 1e-6 * nn)) {
        full_az = 1; rows_top = 1; rows_bot = 1;      /* ill-conditioned solve */
    } else {
        double a = (B[0] * C[1] - B[1] * C[0]) / det;
        double b = (A[1] * C[0] - A[0] * C[1]) / det;
        if (fabs(a) <= 1.0 + 1e-6 && fabs(b) <= 1.0 + 1e-6) {   /* z-axis pierces the square */
            double zp = (C[2] + a * A[2]) + b * B[2];
            full_az = 1;
            if (zp >= 0.0) rows_top = 1;
            if (zp <= 0.0) rows_bot = 1;
        }
    }
    /* vertices in cyclic order */
    double V[4][3];
    const double sg[4][2] = {{-1.0, -1.0}, {1.0, -1.0}, {1.0, 1.0}, {-1.0, 1.0}};
    for (int k = 0; k < 4; ++k)
        for (int r = 0; r < 3; ++r) V[k][r] = (C[r] + sg[k][0] * A[r]) + sg[k][1] * B[r];

    /* elevation extremes over the boundary: vertices and one stationary point per edge */
    double rmax = 0, zmax = 0, rmin = 0, zmin = 0;
    int have = 0;
    for (int k = 0; k < 4; ++k) {
        double cand[2][3];
        int nc = 0;
        cand[nc][0] = V[k][0]; cand[nc][1] = V[k][1]; cand[nc][2] = V[k][2]; ++nc;
        const double *P0 = V[k], *P1 = V[(k + 1) & 3];
        double dx = P1[0] - P0[0], dy = P1[1] - P0[1], dz = P1[2] - P0[2];
        double qd = P0[0] * dx + P0[1] * dy;
        double q2 = P0[0] * P0[0] + P0[1] * P0[1];
        double d2 = dx * dx + dy * dy;
        double den = dz * qd - P0[2] * d2;
        if (box_mode != 2 && den != 0.0) {   /* the vertex-only box skips the edges' stationary points */
            double ts = (P0[2] * qd - dz * q2) / den;
            if (ts > 0.0 && ts < 1.0) {
                cand[nc][0] = P0[0] + ts * dx; cand[nc][1] = P0[1] + ts * dy; cand[nc][2] = P0[2] + ts * dz; ++nc;
            }
        }
        for (int c = 0; c < nc; ++c) {
            double r = sqrt(cand[c][0] * cand[c][0] + cand[c][1] * cand[c][1]), zz = cand[c][2];
            if (!have) { rmax = rmin = r; zmax = zmin = zz; have = 1; continue; }
            if (el_lt(rmax, zmax, r, zz)) { rmax = r; zmax = zz; }
            if (el_lt(r, zz, rmin, zmin)) { rmin = r; zmin = zz; }
        }
    }
    /* rows: elevation decreases with the row index (fv < 0) */
    int32_t r0, r1;
    if (rows_top) r0 = 0;
    else {   /* first i with el_i - margin <= el_max */
        int32_t lo = 0, hi = H;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if (zmax * T->rlo[2 * mid] - rmax * T->rlo[2 * mid + 1] >= 0.0) hi = mid; else lo = mid + 1;
        }
        r0 = lo;
    }
    if (rows_bot) r1 = H - 1;
    else {   /* last i with el_i + margin >= el_min */
        int32_t lo = 0, hi = H;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if (!(zmin * T->rhi[2 * mid] - rmin * T->rhi[2 * mid + 1] <= 0.0)) hi = mid; else lo = mid + 1;
        }
        r1 = lo - 1;
    }
    if (r0 > r1) return 0;
    rows[0] = r0; rows[1] = r1;

    if (!full_az) {
        /* azimuth extent: extreme vertices relative to each other (no angles, no seam) */
        int klo = 0, khi = 0;
        for (int k = 1; k < 4; ++k) {
            if (cross2(V[klo][0], V[klo][1], V[k][0], V[k][1]) < 0.0) klo = k;
            if (cross2(V[khi][0], V[khi][1], V[k][0], V[k][1]) > 0.0) khi = k;
        }
        double lx = V[klo][0] * T->cm + V[klo][1] * T->sm, ly = V[klo][1] * T->cm - V[klo][0] * T->sm;
        double ux = V[khi][0] * T->cm - V[khi][1] * T->sm, uy = V[khi][0] * T->sm + V[khi][1] * T->cm;
        if (!(cross2(lx, ly, ux, uy) > 0.0)) full_az = 1;    /* widened arc reaches pi */
        else {
            /* columns are ordered by decreasing azimuth (fu < 0) */
            int32_t lo = 0, hi = W;                 /* first j with az_j <= az(upper) */
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (ang_le(T->col[2 * mid], T->col[2 * mid + 1], ux, uy)) hi = mid; else lo = mid + 1;
            }
            int32_t jf = lo;
            lo = 0; hi = W;                         /* last j with az_j >= az(lower) */
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (!ang_le(lx, ly, T->col[2 * mid], T->col[2 * mid + 1])) hi = mid; else lo = mid + 1;
            }
            int32_t jl = lo - 1;
            if (ang_le(lx, ly, ux, uy)) {           /* arc does not cross the seam */
                if (jf > jl) return 0;
                cols[0] = jf; cols[1] = jl;
                return 1;
            }
            int nint = 0;                           /* arc crosses the seam: two pieces */
            if (jl >= 0) { cols[0] = 0; cols[1] = jl; nint = 1; }
            if (jf <= W - 1) { cols[2 * nint] = jf; cols[2 * nint + 1] = W - 1; ++nint; }
            return nint;
        }
    }
    cols[0] = 0; cols[1] = W - 1;
    return 1;
}

/* Pixel intervals -> tile rectangles (tx0, tx1, ty0, ty1); two pieces whose tile
 * columns overlap are merged.  Returns the rectangle count. */
static int box_rects(int nint, const int32_t *rows, const int32_t *cols, int32_t th, int32_t tw,
                     int32_t *rect)
{
    if (nint == 0) return 0;
    int32_t ty0 = rows[0] / th, ty1 = rows[1] / th;
    rect[0] = cols[0] / tw; rect[1] = cols[1] / tw; rect[2] = ty0; rect[3] = ty1;
    if (nint == 1) return 1;
    int32_t bx0 = cols[2] / tw, bx1 = cols[3] / tw;
    if (bx0 <= rect[1]) { rect[1] = bx1 > rect[1] ? bx1 : rect[1]; return 1; }
    rect[4] = bx0; rect[5] = bx1; rect[6] = ty0; rect[7] = ty1;
    return 2;
}

typedef struct { int32_t tile; uint32_t key; int32_t id; } bin_pair;
static int bin_cmp(const void *a, const void *b)
{
    const bin_pair *x = (const bin_pair *)a, *y = (const bin_pair *)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Per-surfel keys, pixel boxes, tile rectangles and counts; then the per-tile
 * lists sorted by range (ties by surfel index) and the tile ranges.
 *   keys[n]       bit pattern of the FP32 range key
 *   counts[n]     number of tiles (0 = culled)
 *   pixbox[n][6]  r0, r1, c0, c1, c2, c3 (c2 = c3 = -1 for a single interval)
 *   rects[n][8]   (tx0, tx1, ty0, ty1) x 2, unused entries -1
 *   *K            number of (tile, surfel) pairs; sorted_* are written only
 *                 when *K <= capacity
 *   ranges[T][2]  [start, end) per tile, T = tiles_y * tiles_x
 * Returns 0, or 1 when the pair capacity is too small (K still reported). */
int or_bin(int64_t n, const double *means, const double *quats, const double *log_scales,
           const double *logits, const double *pose, const or_sensor *s, int32_t tile_h, int32_t tile_w, double margin,
           int32_t box_mode, uint32_t *keys, int32_t *counts, int32_t *pixbox, int32_t *rects,
           int64_t capacity, int64_t *K, int32_t *sorted_tile, int32_t *sorted_id, int32_t *ranges)
{
    if (n < 0 || !s || tile_h <= 0 || tile_w <= 0) return -1;
    box_tables T;
    tables_make(s, margin, &T);
    int32_t tiles_x = (s->width + tile_w - 1) / tile_w, tiles_y = (s->height + tile_h - 1) / tile_h;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        const double *mu = means + 3 * k;
        float key = mirror_key(mu, pose);
        uint32_t kb;
        memcpy(&kb, &key, 4);
        keys[k] = kb;
        int32_t rows[2] = {-1, -1}, cols[4] = {-1, -1, -1, -1}, rc[8];
        for (int e = 0; e < 8; ++e) rc[e] = -1;
        int nint = surfel_box(mu, quats + 4 * k, log_scales + 2 * k, logits[k], pose, s->near_m, &T, box_mode, rows, cols);
        int nr = box_rects(nint, rows, cols, tile_h, tile_w, rc);
        int32_t cnt = 0;
        for (int r = 0; r < nr; ++r) cnt += (rc[4 * r + 1] - rc[4 * r] + 1) * (rc[4 * r + 3] - rc[4 * r + 2] + 1);
        counts[k] = cnt;
        if (pixbox) {
            int32_t *pb = pixbox + 6 * k;
            pb[0] = nint ? rows[0] : -1; pb[1] = nint ? rows[1] : -1;
            for (int e = 0; e < 4; ++e) pb[2 + e] = (e < 2 * nint) ? cols[e] : -1;
        }
        if (rects) for (int e = 0; e < 8; ++e) rects[8 * k + e] = rc[e];
    }
    tables_free(&T);
    int64_t tot = 0;
    for (int64_t k = 0; k < n; ++k) tot += counts[k];
    *K = tot;
    int32_t ntiles = tiles_x * tiles_y;
    if (tot > capacity) return 1;
    bin_pair *bp = (bin_pair *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(bin_pair));
    int64_t e = 0;
    box_tables T2;
    tables_make(s, margin, &T2);
    for (int64_t k = 0; k < n; ++k) {
        if (!counts[k]) continue;
        int32_t rows[2], cols[4] = {-1, -1, -1, -1}, rc[8];
        int nint = surfel_box(means + 3 * k, quats + 4 * k, log_scales + 2 * k, logits[k], pose, s->near_m, &T2, box_mode,
                              rows, cols);
        int nr = box_rects(nint, rows, cols, tile_h, tile_w, rc);
        for (int r = 0; r < nr; ++r)
            for (int32_t ty = rc[4 * r + 2]; ty <= rc[4 * r + 3]; ++ty)
                for (int32_t tx = rc[4 * r]; tx <= rc[4 * r + 1]; ++tx) {
                    bp[e].tile = ty * tiles_x + tx; bp[e].key = keys[k]; bp[e].id = (int32_t)k; ++e;
                }
    }
    tables_free(&T2);
    qsort(bp, (size_t)tot, sizeof(bin_pair), bin_cmp);
    for (int32_t t = 0; t < ntiles; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t p = 0; p < tot; ++p) {
        sorted_tile[p] = bp[p].tile; sorted_id[p] = bp[p].id;
        if (p == 0 || bp[p].tile != bp[p - 1].tile) ranges[2 * bp[p].tile] = (int32_t)p;
        if (p == tot - 1 || bp[p].tile != bp[p + 1].tile) ranges[2 * bp[p].tile + 1] = (int32_t)(p + 1);
    }
    free(bp);
    return 0;
}

/* Support test of one (pixel, surfel) pair in the oracle's FP64 geometry, for
 * the box-conservativeness check: 1 if the ray meets the 3-sigma square in
 * front of the near range. */
int or_pair_support(const double *mu, const double *q, const double *ls, double logit,
                    const double *pose, const or_sensor *s, int32_t i, int32_t j, double *sh_out)
{
    or_frame f;
    or_surfel_frame(mu, q, ls, logit, pose, s->near_m, &f);
    if (!f.valid) return 0;
    double v[3], hx[3], hy[3];
    or_pixel_basis(s, i, j, v, hx, hy);
    or_pair p;
    int fl = 0;
    /* evaluate geometry only: opacity thresholds are not part of the box */
    p.ha[0] = dot3(hx, f.ba); p.ha[1] = dot3(hx, f.bb); p.ha[2] = dot3(hx, f.bc);
    p.hb[0] = dot3(hy, f.ba); p.hb[1] = dot3(hy, f.bb); p.hb[2] = dot3(hy, f.bc);
    cross3(p.ha, p.hb, p.ph);
    (void)fl;
    if (p.ph[2] == 0.0) return 0;
    double s0 = p.ph[0] / p.ph[2], s1 = p.ph[1] / p.ph[2];
    if (sh_out) { sh_out[0] = s0; sh_out[1] = s1; }
    if (!(fmax(fabs(s0), fabs(s1)) <= OR_SUPPORT)) return 0;
    double nu[3];
    for (int k = 0; k < 3; ++k) nu[k] = s0 * f.ba[k] + s1 * f.bb[k] + f.bc[k];
    return dot3(nu, v) > s->near_m;
}

/* Exposed for the tests: the oracle's per-surfel frame quantities
 * (ba, bb, bc, n, o, s_a, s_b) as 15 doubles, and the range key bits. */
int or_frames(int64_t n, const double *means, const double *quats, const double *log_scales,
              const double *logits, const double *pose, double near_m, double *out15,
              uint32_t *keys, int32_t *valid)
{
    for (int64_t k = 0; k < n; ++k) {
        or_frame f;
        or_surfel_frame(means + 3 * k, quats + 4 * k, log_scales + 2 * k, logits[k], pose, near_m, &f);
        double *o = out15 + 15 * k;
        for (int c = 0; c < 3; ++c) { o[c] = f.ba[c]; o[3 + c] = f.bb[c]; o[6 + c] = f.bc[c]; o[9 + c] = f.n[c]; }
        o[12] = f.o; o[13] = f.s[0]; o[14] = f.s[1];
        if (keys) memcpy(&keys[k], &f.key, 4);
        if (valid) valid[k] = f.valid;
    }
    return 0;
}

/* Exposed for the tests: the reproducible exp used by the box. */
double or_box_exp(double x) { return box_exp(x); }
double or_support_radius(double logit) { return support_radius(logit); }
