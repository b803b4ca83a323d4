/*
 * tsr_oracle.c -- plain, slow FP64 CPU reference of the differentiable triangle-soup
 * rasterizer of "Triangle Splatting SLAM" (Sec. 3.1-3.3, eqs. 1-7).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  It shares no code, header, table or helper
 * with the HIP path; the two only see the same seeded float32 inputs.
 *
 * What it computes, per pixel, by brute force over every face (no tiles, no binning):
 *   1. v_C = R v_W + t                                   (eq. 1, world -> camera)
 *   2. cull a face if any vertex has z_C < z_near
 *   3. q = (fx x/z + cx, fy y/z + cy)                    (eq. 1, pinhole reading of pi)
 *   4. edge lines L_k(p) = n_k . p + d_k with outward unit normals n_k  (eq. 2)
 *      inradius r = |A2| / perimeter; cull if r < r_min (phi(s) = -r at the incentre s)
 *   5. window I(p) = min(1, max(0, phi(p)/phi(s)))^sigma, phi = max_k L_k  (eq. 3)
 *   6. colour c(p) = sum_i lambda_i c_i with screen-space barycentrics (Sec. 3.1)
 *   7. face opacity o_F = (o_i + o_j + o_k)/3, alpha = o_F I(p)             (Sec. 3.1)
 *   8. faces with alpha > 0 sorted ascending by (float32(z_F), face index),
 *      z_F = mean camera-space vertex depth                                 (eq. 4 "depth order")
 *   9. C = sum c alpha T, D = sum z_F alpha T, T <- T (1 - alpha), T starts at 1 (eq. 4)
 * and the gradient of any loss whose per-pixel derivatives (dL/dC, dL/dD, dL/dT) are given,
 * with respect to vertex positions, colours, opacities and the left se(3) perturbation
 * tau = (rho, theta) of T_CW (eqs. 5-7: dv_C/dtau = [I, -[v_C]x]).
 *
 * Derivatives of the per-face quantities are taken with forward-mode dual numbers seeded on
 * the nine camera-space vertex coordinates; the compositing derivative uses stored per-pixel
 * lists.  The per-face pixel-rectangle test below only skips pixels where the window is
 * exactly zero (outside the closed bounding box of the projected triangle).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ECAP -2

/* ------------------------------------------------------------------------- inputs */
typedef struct {
    const double *pos;  /* [3][N] */
    const double *col;  /* [3][N] */
    const double *opa;  /* [N]    */
    const int32_t *faces; /* [M][3] or NULL for a soup */
    int64_t n_vertices, n_faces;
    const double *face_sigma; /* [M] per-face window exponents, or NULL: every face uses the
                                 parameters' sigma (Sec. 3.2: learnable per triangle in Triangle
                                 Splatting, one global constant in Mesh Splatting) */
} orc_scene;

typedef struct { int32_t width, height; double fx, fy, cx, cy; } orc_cam;
/* opa_min: 0 = face opacity is the mean of its vertex opacities (Sec. 3.1); 1 = their minimum
 * (the Mesh Splatting rule the paper departs from), whose derivative goes to the vertex of
 * lowest opacity (lowest index on ties). */
/* tight_tiles: 0 = a face is listed in every tile of its pixel rectangle (the conservative
 * bounding-box rule); 1 = only in the tiles whose pixel centres inside that rectangle can be
 * inside the face: for each edge k the smallest L_k over the tile's box of pixel centres is
 * below 0 (the triangle-tile binning variant). */
/* persp: 0 = colour interpolated with the screen-space (affine) barycentrics of the projected
 * triangle and depth z_F (the reading of Sec. 3.1 and eq. 4); 1 = perspective-correct
 * barycentrics mu_i = (lambda_i / z_i) / sum_j (lambda_j / z_j) for the colour and the depth of
 * the face's plane along the pixel's ray, 1 / sum_j (lambda_j / z_j), in D (the variant).  The
 * depth order stays that of z_F. */
typedef struct { double sigma, z_near, r_min, opa_min, tight_tiles, persp; } orc_par;

static int64_t vid(const orc_scene *s, int64_t m, int k) {
    return s->faces ? (int64_t)s->faces[3 * m + k] : 3 * m + k;
}

/* ------------------------------------------------------------------------- face geometry */
typedef struct {
    int ok;
    int64_t v[3];
    double vc[3][3];      /* camera-space vertices */
    double q[3][2];       /* projected vertices */
    double n[3][2], d[3], len[3];
    double area2, perim, r;
    double zf, of;
    double sig;           /* the face's window exponent sigma (eq. 3) */
    int persp;            /* perspective-correct interpolation (orc_par.persp) */
    int kmin;             /* vertex of lowest opacity (lowest index on ties) */
    float zkey;
    double umin, umax, vmin, vmax;
} face_t;

static void rot(const double *pose, double R[3][3], double t[3]) {
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) R[i][j] = pose[3 * i + j];
        t[i] = pose[9 + i];
    }
}

/* Steps 1-4 and 7-8 for face m. */
static void face_setup(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                       int64_t m, face_t *f) {
    double R[3][3], t[3];
    rot(pose, R, t);
    int64_t N = s->n_vertices;
    f->ok = 0;
    f->sig = s->face_sigma ? s->face_sigma[m] : p->sigma;
    f->persp = p->persp != 0.0;
    for (int k = 0; k < 3; k++) {
        int64_t i = vid(s, m, k);
        f->v[k] = i;
        double w[3] = {s->pos[i], s->pos[N + i], s->pos[2 * N + i]};
        for (int a = 0; a < 3; a++)
            f->vc[k][a] = R[a][0] * w[0] + R[a][1] * w[1] + R[a][2] * w[2] + t[a];
    }
    for (int k = 0; k < 3; k++)
        if (!(f->vc[k][2] >= p->z_near)) return;           /* near-plane cull (NaN culls too) */
    for (int k = 0; k < 3; k++) {
        f->q[k][0] = c->fx * f->vc[k][0] / f->vc[k][2] + c->cx;
        f->q[k][1] = c->fy * f->vc[k][1] / f->vc[k][2] + c->cy;
    }
    double a2 = (f->q[1][0] - f->q[0][0]) * (f->q[2][1] - f->q[0][1])
              - (f->q[1][1] - f->q[0][1]) * (f->q[2][0] - f->q[0][0]);
    double so = a2 >= 0 ? 1.0 : -1.0;
    f->area2 = fabs(a2);
    f->perim = 0;
    for (int k = 0; k < 3; k++) {
        int k1 = (k + 1) % 3;
        double ex = f->q[k1][0] - f->q[k][0], ey = f->q[k1][1] - f->q[k][1];
        f->len[k] = sqrt(ex * ex + ey * ey);
        f->perim += f->len[k];
    }
    f->r = f->area2 / f->perim;
    if (!(f->r >= p->r_min)) return;                       /* degenerate cull */
    for (int k = 0; k < 3; k++) {
        int k1 = (k + 1) % 3;
        double ex = f->q[k1][0] - f->q[k][0], ey = f->q[k1][1] - f->q[k][1];
        f->n[k][0] = so * ey / f->len[k];
        f->n[k][1] = -so * ex / f->len[k];
        f->d[k] = -(f->n[k][0] * f->q[k][0] + f->n[k][1] * f->q[k][1]);
    }
    f->zf = (f->vc[0][2] + f->vc[1][2] + f->vc[2][2]) / 3.0;
    f->zkey = (float)f->zf;
    f->kmin = 0;
    for (int k = 1; k < 3; k++)
        if (s->opa[f->v[k]] < s->opa[f->v[f->kmin]]) f->kmin = k;
    f->of = p->opa_min != 0.0 ? s->opa[f->v[f->kmin]]
                              : (s->opa[f->v[0]] + s->opa[f->v[1]] + s->opa[f->v[2]]) / 3.0;
    f->umin = fmin(f->q[0][0], fmin(f->q[1][0], f->q[2][0]));
    f->umax = fmax(f->q[0][0], fmax(f->q[1][0], f->q[2][0]));
    f->vmin = fmin(f->q[0][1], fmin(f->q[1][1], f->q[2][1]));
    f->vmax = fmax(f->q[0][1], fmax(f->q[1][1], f->q[2][1]));
    f->ok = 1;
}

/* Steps 4-6 at pixel centre (u, v).  Returns I(p); writes rho and the barycentrics. */
static double face_window(const face_t *f, double u, double v, double *rho_out, double lam[3]) {
    double L[3];
    for (int k = 0; k < 3; k++) L[k] = f->n[k][0] * u + f->n[k][1] * v + f->d[k];
    int ks = 0;
    for (int k = 1; k < 3; k++)
        if (L[k] > L[ks]) ks = k;                          /* lowest k on ties */
    double rho = -L[ks] / f->r;                            /* phi(p)/phi(s), phi(s) = -r */
    *rho_out = rho;
    /* lambda_i is the signed distance to the opposite edge over the vertex's distance to it */
    lam[0] = -L[1] * f->len[1] / f->area2;
    lam[1] = -L[2] * f->len[2] / f->area2;
    lam[2] = -L[0] * f->len[0] / f->area2;
    if (!(rho > 0)) return 0.0;
    if (rho >= 1) return 1.0;
    return pow(rho, f->sig);
}

static int in_box(const face_t *f, double u, double v) {
    return u > f->umin && u < f->umax && v > f->vmin && v < f->vmax;
}

/* ------------------------------------------------------------------------- per-pixel lists */
typedef struct {
    float zkey;
    int64_t m;
    double alpha, I, rho, zf, c[3], lam[3];
} hit_t;

static int hit_cmp(const void *a, const void *b) {
    const hit_t *x = (const hit_t *)a, *y = (const hit_t *)b;
    if (x->zkey < y->zkey) return -1;
    if (x->zkey > y->zkey) return 1;
    return (x->m > y->m) - (x->m < y->m);
}

/* Collect and depth-sort every face covering pixel (u, v).  Caller frees *out. */
static int64_t pixel_hits(const orc_scene *s, const face_t *F, int u, int v, hit_t **out) {
    int64_t cap = 16, n = 0;
    hit_t *h = (hit_t *)malloc(sizeof(hit_t) * cap);
    for (int64_t m = 0; m < s->n_faces; m++) {
        const face_t *f = &F[m];
        if (!f->ok || !in_box(f, u, v)) continue;
        double rho, lam[3];
        double I = face_window(f, u, v, &rho, lam);
        double alpha = f->of * I;
        if (!(alpha > 0)) continue;
        if (n == cap) { cap *= 2; h = (hit_t *)realloc(h, sizeof(hit_t) * cap); }
        hit_t *e = &h[n++];
        e->zkey = f->zkey; e->m = m; e->alpha = alpha; e->I = I; e->rho = rho; e->zf = f->zf;
        if (f->persp) {
            /* perspective-correct weights and the plane's depth along the ray (1/z is affine) */
            double w[3], W = 0;
            for (int i = 0; i < 3; i++) { w[i] = lam[i] / f->vc[i][2]; W += w[i]; }
            for (int i = 0; i < 3; i++) lam[i] = w[i] / W;
            e->zf = 1.0 / W;
        }
        for (int i = 0; i < 3; i++) e->lam[i] = lam[i];
        for (int ch = 0; ch < 3; ch++) {
            double acc = 0;
            for (int i = 0; i < 3; i++)
                acc += lam[i] * s->col[(int64_t)ch * s->n_vertices + f->v[i]];
            e->c[ch] = acc;
        }
    }
    qsort(h, (size_t)n, sizeof(hit_t), hit_cmp);
    *out = h;
    return n;
}

static void setup_all(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                      face_t *F) {
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < s->n_faces; m++) face_setup(s, pose, c, p, m, &F[m]);
}

static int check_args(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p) {
    if (!s || !pose || !c || !p || !s->pos || !s->col || !s->opa) return ORC_EINVAL;
    if (s->n_faces < 0 || s->n_vertices < 0 || c->width <= 0 || c->height <= 0 || !(p->sigma > 0))
        return ORC_EINVAL;
    if (!s->faces && s->n_vertices < 3 * s->n_faces) return ORC_EINVAL;
    if (s->face_sigma)
        for (int64_t m = 0; m < s->n_faces; m++)
            if (!(s->face_sigma[m] > 0)) return ORC_EINVAL;
    return ORC_OK;
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Forward render of the listed pixels (pixel index = y*W + x; pix == NULL means every pixel,
 * npix = W*H).  Outputs color[3][npix], depth[npix], trans[npix]. */
int orc_render(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
               const int64_t *pix, int64_t npix, double *color, double *depth, double *trans) {
    int rc = check_args(s, pose, c, p);
    if (rc) return rc;
    face_t *F = (face_t *)calloc((size_t)(s->n_faces ? s->n_faces : 1), sizeof(face_t));
    setup_all(s, pose, c, p, F);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; k++) {
        int64_t id = pix ? pix[k] : k;
        int u = (int)(id % c->width), v = (int)(id / c->width);
        hit_t *h;
        int64_t n = pixel_hits(s, F, u, v, &h);
        double C[3] = {0, 0, 0}, D = 0, T = 1;
        for (int64_t j = 0; j < n; j++) {
            double w = h[j].alpha * T;
            for (int ch = 0; ch < 3; ch++) C[ch] += h[j].c[ch] * w;
            D += h[j].zf * w;
            T *= 1.0 - h[j].alpha;
        }
        free(h);
        for (int ch = 0; ch < 3; ch++) color[ch * npix + k] = C[ch];
        depth[k] = D;
        trans[k] = T;
    }
    free(F);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- dual numbers */
#define NT 9
typedef struct { double v, d[NT]; } dn;

static dn dn_const(double v) { dn r; r.v = v; memset(r.d, 0, sizeof r.d); return r; }
static dn dn_var(double v, int i) { dn r = dn_const(v); r.d[i] = 1.0; return r; }
static dn dn_add(dn a, dn b) { dn r; r.v = a.v + b.v; for (int i = 0; i < NT; i++) r.d[i] = a.d[i] + b.d[i]; return r; }
static dn dn_sub(dn a, dn b) { dn r; r.v = a.v - b.v; for (int i = 0; i < NT; i++) r.d[i] = a.d[i] - b.d[i]; return r; }
static dn dn_mul(dn a, dn b) { dn r; r.v = a.v * b.v; for (int i = 0; i < NT; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
static dn dn_div(dn a, dn b) {
    dn r; r.v = a.v / b.v;
    for (int i = 0; i < NT; i++) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r;
}
static dn dn_scale(dn a, double k) { dn r; r.v = a.v * k; for (int i = 0; i < NT; i++) r.d[i] = a.d[i] * k; return r; }
static dn dn_sqrt(dn a) {
    dn r; r.v = sqrt(a.v);
    for (int i = 0; i < NT; i++) r.d[i] = a.d[i] / (2.0 * r.v);
    return r;
}

/* Window, barycentrics and depth of face f at (u, v) as functions of its nine camera-space
 * vertex coordinates (tangent index 3*vertex + axis).  Same steps as face_setup/face_window. */
static void face_local_dual(const face_t *f, const orc_cam *c, double u, double v,
                            dn *I_out, dn lam[3], dn *zf_out) {
    const double sigma = f->sig;
    dn q[3][2];
    for (int k = 0; k < 3; k++) {
        dn x = dn_var(f->vc[k][0], 3 * k), y = dn_var(f->vc[k][1], 3 * k + 1),
           z = dn_var(f->vc[k][2], 3 * k + 2);
        q[k][0] = dn_add(dn_scale(dn_div(x, z), c->fx), dn_const(c->cx));
        q[k][1] = dn_add(dn_scale(dn_div(y, z), c->fy), dn_const(c->cy));
    }
    dn a2 = dn_sub(dn_mul(dn_sub(q[1][0], q[0][0]), dn_sub(q[2][1], q[0][1])),
                   dn_mul(dn_sub(q[1][1], q[0][1]), dn_sub(q[2][0], q[0][0])));
    double so = a2.v >= 0 ? 1.0 : -1.0;
    dn area = dn_scale(a2, so);
    dn len[3], L[3], perim = dn_const(0);
    for (int k = 0; k < 3; k++) {
        int k1 = (k + 1) % 3;
        dn ex = dn_sub(q[k1][0], q[k][0]), ey = dn_sub(q[k1][1], q[k][1]);
        len[k] = dn_sqrt(dn_add(dn_mul(ex, ex), dn_mul(ey, ey)));
        perim = dn_add(perim, len[k]);
        dn nx = dn_scale(dn_div(ey, len[k]), so), ny = dn_scale(dn_div(ex, len[k]), -so);
        /* L_k(p) = n_k . (p - q_k) */
        L[k] = dn_add(dn_mul(nx, dn_sub(dn_const(u), q[k][0])), dn_mul(ny, dn_sub(dn_const(v), q[k][1])));
    }
    int ks = 0;
    for (int k = 1; k < 3; k++)
        if (L[k].v > L[ks].v) ks = k;
    dn r = dn_div(area, perim);
    dn rho = dn_scale(dn_div(L[ks], r), -1.0);
    if (!(rho.v > 0)) *I_out = dn_const(0.0);
    else if (rho.v >= 1) *I_out = dn_const(1.0);
    else {
        dn I = dn_const(pow(rho.v, sigma));
        double dIdr = sigma * pow(rho.v, sigma - 1.0);
        for (int i = 0; i < NT; i++) I.d[i] = dIdr * rho.d[i];
        *I_out = I;
    }
    lam[0] = dn_scale(dn_div(dn_mul(L[1], len[1]), area), -1.0);
    lam[1] = dn_scale(dn_div(dn_mul(L[2], len[2]), area), -1.0);
    lam[2] = dn_scale(dn_div(dn_mul(L[0], len[0]), area), -1.0);
    if (f->persp) {
        dn w[3], W = dn_const(0);
        for (int i = 0; i < 3; i++) {
            w[i] = dn_div(lam[i], dn_var(f->vc[i][2], 3 * i + 2));
            W = dn_add(W, w[i]);
        }
        for (int i = 0; i < 3; i++) lam[i] = dn_div(w[i], W);
        *zf_out = dn_div(dn_const(1.0), W);
        return;
    }
    dn zf = dn_const(0);
    for (int k = 0; k < 3; k++) zf = dn_add(zf, dn_var(f->vc[k][2], 3 * k + 2));
    *zf_out = dn_scale(zf, 1.0 / 3.0);
}

/* Backward of the render over the listed pixels, given per-pixel upstream gradients
 * gC[3][npix], gD[npix], gT[npix] (gT may be NULL).  Accumulates (+=) into
 * grad_pos[3][N], grad_col[3][N], grad_opa[N] and grad_pose[6] = (rho, theta); the caller
 * zeroes them.  Only contributions of the listed pixels are included.
 * abs_pos / abs_col / abs_opa (nullable, same shapes) receive the sums over pixels of the
 * absolute per-pixel contributions: the conditioning of each gradient element, which bounds
 * the rounding error of any implementation that forms per-pixel terms in lower precision. */
static int backward_impl(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                         const int64_t *pix, int64_t npix, const double *gC, const double *gD,
                         const double *gT, double *grad_pos, double *grad_col, double *grad_opa,
                         double *grad_pose, double *abs_pos, double *abs_col, double *abs_opa,
                         double *grad_sigma, double *abs_sigma) {
    int rc = check_args(s, pose, c, p);
    if (rc) return rc;
    int64_t M = s->n_faces, N = s->n_vertices;
    face_t *F = (face_t *)calloc((size_t)(M ? M : 1), sizeof(face_t));
    setup_all(s, pose, c, p, F);
    double *gvc = (double *)calloc((size_t)(M ? M : 1) * 9, sizeof(double)); /* dL/dv_C per face */
    double Rw[3][3], tw[3];
    rot(pose, Rw, tw);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; k++) {
        int64_t id = pix ? pix[k] : k;
        int u = (int)(id % c->width), v = (int)(id / c->width);
        double g[3] = {gC[k], gC[npix + k], gC[2 * npix + k]};
        double gd = gD[k], gt = gT ? gT[k] : 0.0;
        hit_t *h;
        int64_t n = pixel_hits(s, F, u, v, &h);
        double *Tn = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
        double T = 1;
        for (int64_t j = 0; j < n; j++) { Tn[j] = T; T *= 1.0 - h[j].alpha; }
        /* back to front: B = what lies behind face j, composited from transmittance 1 */
        double B[3] = {0, 0, 0}, BD = 0, BA = 0;
        for (int64_t j = n - 1; j >= 0; j--) {
            const hit_t *e = &h[j];
            const face_t *f = &F[e->m];
            double w = e->alpha * Tn[j];
            /* dC/dalpha_j = T_j (c_j - B), dD/dalpha_j = T_j (z_j - BD), dT_fin/dalpha_j = -T_j (1 - BA) */
            double galpha = Tn[j] * (g[0] * (e->c[0] - B[0]) + g[1] * (e->c[1] - B[1]) +
                                     g[2] * (e->c[2] - B[2]) + gd * (e->zf - BD) - gt * (1.0 - BA));
            double gcol[3] = {g[0] * w, g[1] * w, g[2] * w};
            double gz = gd * w;
            dn I, lam[3], zf;
            face_local_dual(f, c, u, v, &I, lam, &zf);
            double acc[9];
            for (int t = 0; t < 9; t++) {
                double dc = 0;
                for (int i = 0; i < 3; i++) {
                    double ci = 0;
                    for (int ch = 0; ch < 3; ch++) ci += gcol[ch] * s->col[(int64_t)ch * N + f->v[i]];
                    dc += ci * lam[i].d[t];
                }
                acc[t] = galpha * f->of * I.d[t] + dc + gz * zf.d[t];
            }
            for (int t = 0; t < 9; t++) {
                #pragma omp atomic
                gvc[9 * e->m + t] += acc[t];
            }
            if (abs_pos)
                for (int k = 0; k < 3; k++)
                    for (int a = 0; a < 3; a++) {
                        double w = fabs(Rw[0][a] * acc[3 * k] + Rw[1][a] * acc[3 * k + 1] + Rw[2][a] * acc[3 * k + 2]);
                        #pragma omp atomic
                        abs_pos[(int64_t)a * N + f->v[k]] += w;
                    }
            for (int i = 0; i < 3; i++) {
                int64_t vi = f->v[i];
                for (int ch = 0; ch < 3; ch++) {
                    double val = gcol[ch] * e->lam[i];
                    #pragma omp atomic
                    grad_col[(int64_t)ch * N + vi] += val;
                    if (abs_col) {
                        #pragma omp atomic
                        abs_col[(int64_t)ch * N + vi] += fabs(val);
                    }
                }
                double go = p->opa_min != 0.0 ? (i == f->kmin ? galpha * e->I : 0.0) : galpha * e->I / 3.0;
                #pragma omp atomic
                grad_opa[vi] += go;
                if (abs_opa) {
                    #pragma omp atomic
                    abs_opa[vi] += fabs(go);
                }
            }
            /* per-face exponent: dI/dsigma = I ln(rho) inside (0 < rho < 1), 0 where I is 0 or 1 */
            if (grad_sigma && e->rho > 0 && e->rho < 1) {
                double gs = galpha * f->of * e->I * log(e->rho);
                #pragma omp atomic
                grad_sigma[e->m] += gs;
                if (abs_sigma) {
                    #pragma omp atomic
                    abs_sigma[e->m] += fabs(gs);
                }
            }
            for (int ch = 0; ch < 3; ch++) B[ch] = e->c[ch] * e->alpha + (1.0 - e->alpha) * B[ch];
            BD = e->zf * e->alpha + (1.0 - e->alpha) * BD;
            BA = e->alpha + (1.0 - e->alpha) * BA;
        }
        free(Tn);
        free(h);
    }
    /* camera -> world (R^T) and the se(3) pose gradient (eq. 7) */
    double R[3][3], t[3];
    rot(pose, R, t);
    double pg[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t m = 0; m < M; m++) {
        const face_t *f = &F[m];
        if (!f->ok) continue;
        for (int k = 0; k < 3; k++) {
            const double *gc = &gvc[9 * m + 3 * k];
            const double *vc = f->vc[k];
            for (int a = 0; a < 3; a++)
                grad_pos[(int64_t)a * N + f->v[k]] += R[0][a] * gc[0] + R[1][a] * gc[1] + R[2][a] * gc[2];
            pg[0] += gc[0]; pg[1] += gc[1]; pg[2] += gc[2];
            pg[3] += vc[1] * gc[2] - vc[2] * gc[1];
            pg[4] += vc[2] * gc[0] - vc[0] * gc[2];
            pg[5] += vc[0] * gc[1] - vc[1] * gc[0];
        }
    }
    for (int i = 0; i < 6; i++) grad_pose[i] += pg[i];
    free(gvc);
    free(F);
    return ORC_OK;
}

int orc_backward_abs(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                     const int64_t *pix, int64_t npix, const double *gC, const double *gD,
                     const double *gT, double *grad_pos, double *grad_col, double *grad_opa,
                     double *grad_pose, double *abs_pos, double *abs_col, double *abs_opa) {
    return backward_impl(s, pose, c, p, pix, npix, gC, gD, gT, grad_pos, grad_col, grad_opa, grad_pose,
                         abs_pos, abs_col, abs_opa, NULL, NULL);
}

int orc_backward(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                 const int64_t *pix, int64_t npix, const double *gC, const double *gD,
                 const double *gT, double *grad_pos, double *grad_col, double *grad_opa,
                 double *grad_pose) {
    return backward_impl(s, pose, c, p, pix, npix, gC, gD, gT, grad_pos, grad_col, grad_opa, grad_pose,
                         NULL, NULL, NULL, NULL, NULL);
}

/* As orc_backward_abs, plus (+=) the gradient with respect to each face's window exponent,
 * grad_sigma[M] = sum over blended pixels of dL/dalpha o_F I ln(rho), and (abs_sigma,
 * nullable) the sums of its absolute per-pixel terms. */
int orc_backward_sigma(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                       const int64_t *pix, int64_t npix, const double *gC, const double *gD,
                       const double *gT, double *grad_pos, double *grad_col, double *grad_opa,
                       double *grad_pose, double *grad_sigma, double *abs_pos, double *abs_col,
                       double *abs_opa, double *abs_sigma) {
    return backward_impl(s, pose, c, p, pix, npix, gC, gD, gT, grad_pos, grad_col, grad_opa, grad_pose,
                         abs_pos, abs_col, abs_opa, grad_sigma, abs_sigma);
}

/* L1 loss of eqs. (8)-(10) without the D-SSIM term, as means over pixels (and channels):
 *   L = w_c mean|C - Cbar| + w_d mean([Dbar > 0] |D - Dbar|)
 * and its per-pixel derivatives.  `norm_pix` is the full frame's pixel count H*W (the listed
 * pixels may be a subset).  sign(0) = 0.  Returns L restricted to the listed pixels. */
double orc_l1_seeds(const double *C, const double *D, const float *Cbar, const float *Dbar,
                    int64_t npix, int64_t norm_pix, double w_c, double w_d, double *gC, double *gD) {
    double L = 0;
    for (int64_t k = 0; k < npix; k++) {
        for (int ch = 0; ch < 3; ch++) {
            double dlt = C[ch * npix + k] - (double)Cbar[ch * npix + k];
            L += w_c * fabs(dlt) / (3.0 * norm_pix);
            gC[ch * npix + k] = w_c * ((dlt > 0) - (dlt < 0)) / (3.0 * norm_pix);
        }
        double db = (double)Dbar[k];
        double dlt = D[k] - db;
        double msk = db > 0 ? 1.0 : 0.0;
        L += w_d * msk * fabs(dlt) / (double)norm_pix;
        gD[k] = w_d * msk * ((dlt > 0) - (dlt < 0)) / (double)norm_pix;
    }
    return L;
}

/* ------------------------------------------------------------------------- reference binner */
/* Per face: visibility, float32 depth key, pixel rectangle and tile rectangle, using the
 * binning rule: pixel range [ceil(max(umin,-1)), floor(min(umax,W))] clipped to [0, W-1]
 * (likewise v), tiles of 16x16 pixels.  rect[m] = (u0,u1,v0,v1) or (-1,...) when empty. */
static int face_rect(const face_t *f, const orc_cam *c, int r[4]) {
    if (!f->ok) return 0;
    double lo_u = ceil(fmax(f->umin, -1.0)), hi_u = floor(fmin(f->umax, (double)c->width));
    double lo_v = ceil(fmax(f->vmin, -1.0)), hi_v = floor(fmin(f->vmax, (double)c->height));
    int u0 = (int)fmax(lo_u, 0.0), u1 = (int)fmin(hi_u, (double)(c->width - 1));
    int v0 = (int)fmax(lo_v, 0.0), v1 = (int)fmin(hi_v, (double)(c->height - 1));
    if (u0 > u1 || v0 > v1) return 0;
    r[0] = u0; r[1] = u1; r[2] = v0; r[3] = v1;
    return 1;
}

/* Per-face projection records for parity of the projection step.
 * out_q[6][M] projected vertices, out_f[4][M] = (r, o_F, z_F, float32 z key), rect[4][M],
 * tiles[M] = number of 16x16 tiles overlapped (0 when culled or off-screen). */
int orc_project(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                double *out_q, double *out_f, int32_t *rect, int64_t *tiles) {
    int rc = check_args(s, pose, c, p);
    if (rc) return rc;
    int64_t M = s->n_faces;
    face_t *F = (face_t *)calloc((size_t)(M ? M : 1), sizeof(face_t));
    setup_all(s, pose, c, p, F);
    for (int64_t m = 0; m < M; m++) {
        const face_t *f = &F[m];
        int r[4] = {-1, -1, -1, -1};
        int vis = face_rect(f, c, r);
        for (int k = 0; k < 3; k++) {
            out_q[(2 * k) * M + m] = f->ok ? f->q[k][0] : NAN;
            out_q[(2 * k + 1) * M + m] = f->ok ? f->q[k][1] : NAN;
        }
        out_f[0 * M + m] = f->ok ? f->r : NAN;
        out_f[1 * M + m] = f->ok ? f->of : NAN;
        out_f[2 * M + m] = f->ok ? f->zf : NAN;
        out_f[3 * M + m] = f->ok ? (double)f->zkey : NAN;
        for (int i = 0; i < 4; i++) rect[i * M + m] = vis ? r[i] : -1;
        tiles[m] = vis ? (int64_t)((r[1] >> 4) - (r[0] >> 4) + 1) * ((r[3] >> 4) - (r[2] >> 4) + 1) : 0;
    }
    free(F);
    return ORC_OK;
}

typedef struct { int64_t tile; uint32_t zbits; int64_t face; } pair_t;

static int pair_cmp(const void *a, const void *b) {
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->zbits != y->zbits) return x->zbits < y->zbits ? -1 : 1;
    return (x->face > y->face) - (x->face < y->face);
}

/* Can tile (x, y) of face f's pixel rectangle r = [u0, u1, v0, v1] hold a pixel the face
 * covers?  Every covered pixel p has L_k(p) < 0 for all three edges (eq. 2: rho > 0 needs
 * phi < 0), and an affine L_k is smallest over the tile's box of pixel centres at one corner;
 * the tile is kept when that smallest value is below 0 for every edge. */
static int tile_may_cover(const face_t *f, const int r[4], int x, int y) {
    double ulo = fmax(16.0 * x, r[0]), uhi = fmin(16.0 * x + 15.0, r[1]);
    double vlo = fmax(16.0 * y, r[2]), vhi = fmin(16.0 * y + 15.0, r[3]);
    for (int k = 0; k < 3; k++) {
        double u = f->n[k][0] > 0 ? ulo : uhi, v = f->n[k][1] > 0 ? vlo : vhi;
        double lmin = f->n[k][0] * u + f->n[k][1] * v + f->d[k];
        if (!(lmin < 0)) return 0;
    }
    return 1;
}

/* Tile lists for views v = 0..n_views-1 (poses [V][12], cams [V]).  Every (tile, face) pair
 * of every face's tile rectangle (with tight_tiles, those tile_may_cover keeps), sorted by
 * (view-major global tile, float32 z bits, face);
 * faces are numbered v*M + m.  Writes *K; if cap >= K also writes tile_out[K], zbits_out[K],
 * face_out[K] and ranges[2*T_total] (start, end per global tile).  Returns ORC_ECAP when the
 * arrays are too small (K is still set). */
int orc_bin(const orc_scene *s, const double *poses, const orc_cam *cams, int n_views,
            const orc_par *p, int64_t cap, int64_t *K, int64_t *tile_out, uint32_t *zbits_out,
            int64_t *face_out, int64_t *ranges) {
    if (n_views <= 0) return ORC_EINVAL;
    for (int v = 0; v < n_views; v++) {
        int rc = check_args(s, poses + 12 * v, &cams[v], p);
        if (rc) return rc;
    }
    int64_t M = s->n_faces;
    face_t *F = (face_t *)calloc((size_t)(M ? M : 1), sizeof(face_t));
    int64_t total = 0, tile_base = 0;
    pair_t *pairs = NULL;
    int64_t pcap = 0;
    int64_t T_total = 0;
    for (int v = 0; v < n_views; v++)
        T_total += (int64_t)((cams[v].width + 15) / 16) * ((cams[v].height + 15) / 16);
    for (int v = 0; v < n_views; v++) {
        const orc_cam *c = &cams[v];
        int tx = (c->width + 15) / 16, ty = (c->height + 15) / 16;
        setup_all(s, poses + 12 * v, c, p, F);
        for (int64_t m = 0; m < M; m++) {
            int r[4];
            if (!face_rect(&F[m], c, r)) continue;
            uint32_t zb;
            memcpy(&zb, &F[m].zkey, 4);
            for (int y = r[2] >> 4; y <= r[3] >> 4; y++)
                for (int x = r[0] >> 4; x <= r[1] >> 4; x++) {
                    if (p->tight_tiles != 0.0 && !tile_may_cover(&F[m], r, x, y)) continue;
                    if (total == pcap) {
                        pcap = pcap ? 2 * pcap : 1024;
                        pairs = (pair_t *)realloc(pairs, sizeof(pair_t) * (size_t)pcap);
                    }
                    pairs[total].tile = tile_base + (int64_t)y * tx + x;
                    pairs[total].zbits = zb;
                    pairs[total].face = (int64_t)v * M + m;
                    total++;
                }
        }
        tile_base += (int64_t)tx * ty;
    }
    free(F);
    *K = total;
    if (cap < total) { free(pairs); return ORC_ECAP; }
    if (!tile_out || !zbits_out || !face_out || !ranges) { free(pairs); return ORC_OK; }  /* size query */
    qsort(pairs, (size_t)total, sizeof(pair_t), pair_cmp);
    for (int64_t t = 0; t < T_total; t++) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t i = 0; i < total; i++) {
        tile_out[i] = pairs[i].tile;
        zbits_out[i] = pairs[i].zbits;
        face_out[i] = pairs[i].face;
    }
    /* ranges: [start, end) of each tile's run; empty tiles get start = end = first index after
     * the preceding tiles' runs */
    int64_t i = 0;
    for (int64_t t = 0; t < T_total; t++) {
        ranges[2 * t] = i;
        while (i < total && pairs[i].tile == t) i++;
        ranges[2 * t + 1] = i;
    }
    free(pairs);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- discrete state */
/* Per listed pixel, a hash of everything that is piecewise constant in the inputs: the
 * depth-ordered covering set, the maximising edge of phi for each covering face, whether
 * the window is clamped (rho >= 1) and whether rho < rho_eps (steep edge band for sigma < 1).
 * A finite difference is only meaningful when the hash is equal at both ends. */
int orc_state(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
              const int64_t *pix, int64_t npix, double rho_eps, uint64_t *hash) {
    int rc = check_args(s, pose, c, p);
    if (rc) return rc;
    face_t *F = (face_t *)calloc((size_t)(s->n_faces ? s->n_faces : 1), sizeof(face_t));
    setup_all(s, pose, c, p, F);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; k++) {
        int64_t id = pix ? pix[k] : k;
        int u = (int)(id % c->width), v = (int)(id / c->width);
        hit_t *h;
        int64_t n = pixel_hits(s, F, u, v, &h);
        uint64_t x = 1469598103934665603ull;                 /* FNV-1a over the state words */
        for (int64_t j = 0; j < n; j++) {
            const face_t *f = &F[h[j].m];
            double L[3];
            for (int e = 0; e < 3; e++) L[e] = f->n[e][0] * u + f->n[e][1] * v + f->d[e];
            int ks = 0;
            for (int e = 1; e < 3; e++)
                if (L[e] > L[ks]) ks = e;
            uint64_t w = (uint64_t)h[j].m * 16u + (uint64_t)ks * 4u + (h[j].rho >= 1 ? 2u : 0u) +
                         (h[j].rho < rho_eps ? 1u : 0u);
            for (int b = 0; b < 8; b++) { x ^= (w >> (8 * b)) & 0xffu; x *= 1099511628211ull; }
        }
        free(h);
        hash[k] = x;
    }
    free(F);
    return ORC_OK;
}

/* Smallest |rho| = |phi/phi(s)| (eq. 3) over the faces whose bounding box contains each listed
 * pixel (faces that pass the culls), +infinity where there is none.  For sigma < 1 the
 * window's slope grows without bound as rho -> 0+, so pixels near any face's edge -- on
 * either side, since an implementation that rounds rho differently may blend a face there
 * that this oracle does not -- are where the gradient cannot be compared at a relative bar;
 * tests exclude them on both sides. */
int orc_min_rho(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                const int64_t *pix, int64_t npix, double *min_rho) {
    int rc = check_args(s, pose, c, p);
    if (rc) return rc;
    face_t *F = (face_t *)calloc((size_t)(s->n_faces ? s->n_faces : 1), sizeof(face_t));
    setup_all(s, pose, c, p, F);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; k++) {
        int64_t id = pix ? pix[k] : k;
        int u = (int)(id % c->width), v = (int)(id / c->width);
        double r = INFINITY;
        for (int64_t m = 0; m < s->n_faces; m++) {
            const face_t *f = &F[m];
            if (!f->ok || !in_box(f, u, v)) continue;
            double rho, lam[3];
            face_window(f, u, v, &rho, lam);
            if (fabs(rho) < r) r = fabs(rho);
        }
        min_rho[k] = r;
    }
    free(F);
    return ORC_OK;
}

/* Smallest ridge gap over the faces blended at each listed pixel: for a face, the distance in
 * rho units between its two smallest normalised edge distances E_k = -L_k / r (eq. 3 takes the
 * smallest), +infinity where no face is blended.  Where the gap is tiny the pixel lies on a
 * ridge of phi (an angle bisector from the incentre), where which edge attains the minimum --
 * and so which edge's parameters receive the window gradient -- flips under rounding; tests
 * exclude such pixels on both sides like the other discrete-state flips. */
int orc_ridge_gap(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p,
                  const int64_t *pix, int64_t npix, double *gap) {
    int rc = check_args(s, pose, c, p);
    if (rc) return rc;
    face_t *F = (face_t *)calloc((size_t)(s->n_faces ? s->n_faces : 1), sizeof(face_t));
    setup_all(s, pose, c, p, F);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; k++) {
        int64_t id = pix ? pix[k] : k;
        int u = (int)(id % c->width), v = (int)(id / c->width);
        hit_t *h;
        int64_t n = pixel_hits(s, F, u, v, &h);
        double best = INFINITY;
        for (int64_t j = 0; j < n; j++) {
            const face_t *f = &F[h[j].m];
            double E[3];
            for (int e = 0; e < 3; e++) E[e] = -(f->n[e][0] * u + f->n[e][1] * v + f->d[e]) / f->r;
            double lo = fmin(E[0], fmin(E[1], E[2]));
            double mid = E[0] + E[1] + E[2] - lo - fmax(E[0], fmax(E[1], E[2]));
            if (mid - lo < best) best = mid - lo;
        }
        free(h);
        gap[k] = best;
    }
    free(F);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- per-face screen statistics */
/* Map-management statistics of one view (Sec. 3.4: pruning by projected area, densification by
 * pixel coverage, keyframing by visibility), with the blending decisions of eq. 4 and the early
 * stop (a pixel blends while T >= t_min and T > 0):
 *   area[m]   projected area (half the absolute cross product of the projected edges) of faces
 *             that pass the culls and overlap the image, else 0;
 *   coverage  pixels at which the face has the largest weight alpha T (first in depth order on
 *             ties), returned as an interval [cov_lo, cov_hi]: a pixel counts in cov_lo only
 *             when its maximum is certain (a margin of 1e-4 relative + 1e-6 over every other
 *             candidate, and the face's blend certain), and in cov_hi for every face that is
 *             a possible blend within that margin of the maximum;
 *   visible   vis_certain / vis_possible: blended at one pixel with certainty / possibly.
 * "Certain" blends have rho >= 1e-4 and T >= 1.001 t_min; "possible" ones rho > -1e-4 and
 * T >= 0.999 t_min.  An implementation that rounds differently must land inside these
 * intervals; near-ties are the only freedom.  Candidates are the faces whose bounding box,
 * widened by 1e-3 pixel, contains the pixel. */
typedef struct { float zkey; int64_t m; double rho, alpha; } cand_t;

static int cand_cmp(const void *a, const void *b) {
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->zkey < y->zkey) return -1;
    if (x->zkey > y->zkey) return 1;
    return (x->m > y->m) - (x->m < y->m);
}

int orc_face_stats(const orc_scene *s, const double *pose, const orc_cam *c, const orc_par *p, double t_min,
                   double *area, int32_t *cov_lo, int32_t *cov_hi, int32_t *vis_certain, int32_t *vis_possible) {
    int rc = check_args(s, pose, c, p);
    if (rc) return rc;
    const int64_t M = s->n_faces;
    face_t *F = (face_t *)calloc((size_t)(M ? M : 1), sizeof(face_t));
    setup_all(s, pose, c, p, F);
    for (int64_t m = 0; m < M; m++) {
        int r[4];
        area[m] = face_rect(&F[m], c, r) ? 0.5 * F[m].area2 : 0.0;
        cov_lo[m] = cov_hi[m] = vis_certain[m] = vis_possible[m] = 0;
    }
    const int64_t npix = (int64_t)c->width * c->height;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; k++) {
        const int u = (int)(k % c->width), v = (int)(k / c->width);
        int64_t cap = 16, n = 0;
        cand_t *h = (cand_t *)malloc(sizeof(cand_t) * cap);
        for (int64_t m = 0; m < M; m++) {
            const face_t *f = &F[m];
            if (!f->ok) continue;
            if (!(u >= f->umin - 1e-3 && u <= f->umax + 1e-3 && v >= f->vmin - 1e-3 && v <= f->vmax + 1e-3)) continue;
            double rho, lam[3];
            const double I = face_window(f, u, v, &rho, lam);
            if (!(rho > -1e-4)) continue;
            if (n == cap) { cap *= 2; h = (cand_t *)realloc(h, sizeof(cand_t) * cap); }
            h[n].zkey = f->zkey; h[n].m = m; h[n].rho = rho; h[n].alpha = f->of * I;
            n++;
        }
        qsort(h, (size_t)n, sizeof(cand_t), cand_cmp);
        double *w = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
        char *poss = (char *)malloc((size_t)(n ? n : 1)), *cert = (char *)malloc((size_t)(n ? n : 1));
        double T = 1.0, best_w = 0.0;
        int64_t best = -1;
        for (int64_t j = 0; j < n; j++) {
            const int live = T >= t_min && T > 0.0;
            const int blend = live && h[j].rho > 0.0 && h[j].alpha > 0.0;
            poss[j] = (char)(T > 0.0 && T >= 0.999 * t_min);
            cert[j] = (char)(blend && h[j].rho >= 1e-4 && T >= 1.001 * t_min);
            w[j] = blend ? h[j].alpha * T : 0.0;
            if (blend && w[j] > best_w) { best_w = w[j]; best = j; }
            if (blend) T *= 1.0 - h[j].alpha;
        }
        const double slack = 1e-4 * best_w + 1e-6;
        int unique = best >= 0 && cert[best] && best_w > slack;
        for (int64_t j = 0; j < n; j++) {
            if (!poss[j]) continue;
            if (w[j] >= best_w - slack) {
                #pragma omp atomic
                cov_hi[h[j].m] += 1;
                if (j != best) unique = 0;
            }
            if (cert[j]) {
                #pragma omp atomic write
                vis_certain[h[j].m] = 1;
            }
            #pragma omp atomic write
            vis_possible[h[j].m] = 1;
        }
        if (unique) {
            #pragma omp atomic
            cov_lo[h[best].m] += 1;
        }
        free(w); free(poss); free(cert); free(h);
    }
    free(F);
    return ORC_OK;
}
