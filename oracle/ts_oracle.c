/*
 * ts_oracle.c -- plain FP64 CPU oracle of the Triangle Splatting
 * differentiable rasterizer (arXiv 2505.19175).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the package smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header, table or constant with the
 * HIP path.
 *
 * What it computes, and where the paper defines it:
 *   - projection q_i = K(R v_i + t) with the perspective divide      (Sec. 3.1)
 *   - the 2D signed distance phi(p) = max_k (n_k . p + d_k), unit outward
 *     normals n_k, and its value phi(s) at the incentre s            (Sec. 3.1, "A new window function")
 *   - the window I(p) = ReLU(phi(p)/phi(s))^sigma                    (Eq. 1)
 *   - the two alternatives the paper discusses and sets aside: the
 *     sigmoid window I(p) = sigmoid(-phi(p)/sigma), and the SDF with the
 *     max replaced by LogSumExp, phi(p) = log sum_k exp L_k(p), inside
 *     the window of Eq. 1                                            (Sec. 3.1, discussion; Eq. 2)
 *   - front-to-back alpha blending in depth order with I as opacity
 *     modulated by o (the blending weight T*o of Sec. 3.2)           (Sec. 3.1)
 *   - depth order by the triangle centre                             (Supp., "Depth sorting")
 *   - the tight tile bounding box: every edge line moved inward by
 *     d = L(s) (tau_cutoff/o)^(1/sigma), then the bbox of the new
 *     edge intersections                                            (Supp., "Tile assignment")
 *   - view-dependent colour from real spherical harmonics of degree
 *     <= 3 (59 parameters per triangle at degree 3)                  (Sec. 4, "Implementation details")
 *   - the analytic gradient of the above, end to end                 (Sec. 3.3)
 *
 * It is brute force: for every pixel it walks ALL triangles in global depth
 * order (no tiles), in double precision.  Everything the paper leaves open
 * (perspective divide, pixel centres, near plane, alpha clamp, cut-off
 * value, early termination, background, depth key, SH convention) follows
 * one fixed reading shared with the GPU path by specification only.
 *
 * Parallelism: OpenMP over pixels; the per-triangle gradient accumulators
 * use atomic adds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXK 16

/* ------------------------------------------------------------------------ */
/* Inputs                                                                    */
/* ------------------------------------------------------------------------ */

/* cam[16] = R[9] (row-major, world->camera), t[3], fx, fy, cx, cy */
typedef struct {
    double R[9], t[3], fx, fy, cx, cy;
    int W, H;
} ocam;

/* cfg[9] = alpha_min, alpha_max, T_min, z_near, r_min, bg[3], window */
enum { WIN_PAPER = 0, WIN_SIGMOID = 1, WIN_LSE = 2 };

typedef struct {
    double alpha_min, alpha_max, T_min, z_near, r_min, bg[3];
    int window;         /* WIN_PAPER (Eq. 1), WIN_SIGMOID (Eq. 2), WIN_LSE */
    int deg;
    double band_alpha, band_T; /* widths of the "decision too close to call" flags */
} ocfg;

static void load_cam(const double* c, int W, int H, ocam* cam)
{
    memcpy(cam->R, c, 9 * sizeof(double));
    memcpy(cam->t, c + 9, 3 * sizeof(double));
    cam->fx = c[12]; cam->fy = c[13]; cam->cx = c[14]; cam->cy = c[15];
    cam->W = W; cam->H = H;
}

static void load_cfg(const double* g, int deg, ocfg* cfg)
{
    cfg->alpha_min = g[0]; cfg->alpha_max = g[1]; cfg->T_min = g[2];
    cfg->z_near = g[3]; cfg->r_min = g[4];
    cfg->bg[0] = g[5]; cfg->bg[1] = g[6]; cfg->bg[2] = g[7];
    cfg->window = (int)g[8];
    cfg->deg = deg;
    cfg->band_alpha = 1e-6;
    cfg->band_T = 5e-9;
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, from their definition                           */
/* ------------------------------------------------------------------------ */
/*
 * Real orthonormal SH, index l*l + l + m, without the Condon-Shortley phase:
 *   Y_l^0      = N_l^0 P_l(z)
 *   Y_l^{m>0}  = sqrt(2) N_l^m  Re((x+iy)^m)   P_l^{(m)}(z)
 *   Y_l^{m<0}  = sqrt(2) N_l^|m| Im((x+iy)^|m|) P_l^{(|m|)}(z)
 * with N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^{(m)} the m-th
 * derivative of the Legendre polynomial.  This is the usual
 * Y = N P_l^m(cos theta) {cos, sin}(m phi) written in Cartesian form, since
 * P_l^m(z) = (1-z^2)^{m/2} P_l^{(m)}(z) and sin^m(theta) e^{i m phi} = (x+iy)^m.
 * The colour convention of the prior work the paper follows adds 0.5 and
 * clamps at zero.
 */
static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

static double binom(int n, int k)
{
    return factorial(n) / (factorial(k) * factorial(n - k));
}

/* coefficients c[0..l] of P_l(z) = sum_n c[n] z^n */
static void legendre_coeffs(int l, double* c)
{
    for (int n = 0; n <= l; ++n) c[n] = 0.0;
    for (int k = 0; 2 * k <= l; ++k) {
        double s = (k & 1) ? -1.0 : 1.0;
        c[l - 2 * k] = s * binom(l, k) * binom(2 * l - 2 * k, l) / pow(2.0, (double)l);
    }
}

/* m-th derivative of sum_n c[n] z^n at z */
static double poly_deriv(const double* c, int l, int m, double z)
{
    double acc = 0.0;
    for (int n = m; n <= l; ++n) {
        double fall = 1.0;
        for (int j = 0; j < m; ++j) fall *= (double)(n - j);
        acc += c[n] * fall * pow(z, (double)(n - m));
    }
    return acc;
}

/* (x + i y)^m as (re, im) */
static void cpow_xy(double x, double y, int m, double* re, double* im)
{
    double a = 1.0, b = 0.0;
    for (int j = 0; j < m; ++j) {
        double na = a * x - b * y;
        double nb = a * y + b * x;
        a = na; b = nb;
    }
    *re = a; *im = b;
}

/* Y[k] and, if dY != NULL, the gradient dY[k][0..2] of the polynomial
 * extension in (x,y,z). */
static void sh_eval(int deg, const double d[3], double* Y, double (*dY)[3])
{
    const double x = d[0], y = d[1], z = d[2];
    for (int l = 0; l <= deg; ++l) {
        double c[MAXK];
        legendre_coeffs(l, c);
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            const int k = l * l + l + m;
            const double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            const double Pm = poly_deriv(c, l, am, z);
            const double Pm1 = (am + 1 <= l) ? poly_deriv(c, l, am + 1, z) : 0.0;
            double re, im, re1 = 0.0, im1 = 0.0;
            cpow_xy(x, y, am, &re, &im);
            if (am >= 1) cpow_xy(x, y, am - 1, &re1, &im1);
            if (m == 0) {
                Y[k] = N * Pm;
                if (dY) { dY[k][0] = 0.0; dY[k][1] = 0.0; dY[k][2] = N * Pm1; }
            } else if (m > 0) {
                const double a = sqrt(2.0) * N;
                Y[k] = a * re * Pm;
                if (dY) {
                    dY[k][0] = a * am * re1 * Pm;
                    dY[k][1] = -a * am * im1 * Pm;
                    dY[k][2] = a * re * Pm1;
                }
            } else {
                const double a = sqrt(2.0) * N;
                Y[k] = a * im * Pm;
                if (dY) {
                    dY[k][0] = a * am * im1 * Pm;
                    dY[k][1] = a * am * re1 * Pm;
                    dY[k][2] = a * im * Pm1;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Per-triangle setup (Sec. 3.1)                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int visible;        /* survives the near-plane, degeneracy and opacity culls */
    double xc[3][3];    /* camera-space vertices */
    double q[3][2];     /* projected 2D vertices (pixels) */
    double e[3][2];     /* edge k: from q_k to q_{k+1} */
    double len[3];
    double area2;       /* signed doubled area */
    double perim;
    double sgn;         /* orientation */
    double n[3][2];     /* unit outward normals */
    double d[3];        /* offsets: L_k(p) = n_k . p + d_k */
    double s[2];        /* incentre */
    double phis;        /* phi(s) */
    double phis_lse;    /* LogSumExp SDF at s (WIN_LSE) */
    double r;           /* inradius */
    double zc;          /* depth of the centre */
    float key;          /* depth sort key */
    double dir[3], dnorm;
    double Y[MAXK];
    double rgb_raw[3], rgb[3];
    double o, sigma;
    int rect[4];        /* px0, px1, py0, py1 of the tight region */
    int ntiles;
} otri;

static double phi_at(const otri* T, double px, double py, int* kmax)
{
    int best = 0;
    double m = T->n[0][0] * px + T->n[0][1] * py + T->d[0];
    for (int k = 1; k < 3; ++k) {
        double L = T->n[k][0] * px + T->n[k][1] * py + T->d[k];
        if (L > m) { m = L; best = k; }
    }
    if (kmax) *kmax = best;
    return m;
}

/* The SDF with the max replaced by LogSumExp: log sum_k exp L_k(p), written
 * as m + log sum_k exp(L_k - m) with m = max_k L_k so no term overflows;
 * w[k] (if not NULL) receives the softmax weights dphi/dL_k. */
static double lse_at(const otri* T, double px, double py, double w[3])
{
    double L[3], m = -1e300, sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        L[k] = T->n[k][0] * px + T->n[k][1] * py + T->d[k];
        if (L[k] > m) m = L[k];
    }
    for (int k = 0; k < 3; ++k) sum += exp(L[k] - m);
    if (w)
        for (int k = 0; k < 3; ++k) w[k] = exp(L[k] - m) / sum;
    return m + log(sum);
}

static void setup_tri(const double* v, double o, double sigma, const double* sh,
                      const ocam* cam, const ocfg* cfg, otri* T)
{
    memset(T, 0, sizeof(*T));
    T->o = o; T->sigma = sigma;
    T->rect[0] = 0; T->rect[1] = -1; T->rect[2] = 0; T->rect[3] = -1;

    /* camera space x = R v + t */
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a)
            T->xc[i][a] = cam->R[3 * a + 0] * v[3 * i + 0] + cam->R[3 * a + 1] * v[3 * i + 1]
                        + cam->R[3 * a + 2] * v[3 * i + 2] + cam->t[a];
    T->zc = (T->xc[0][2] + T->xc[1][2] + T->xc[2][2]) / 3.0;
    T->key = (float)T->zc;

    T->visible = 1;
    for (int i = 0; i < 3; ++i)
        if (!(T->xc[i][2] > cfg->z_near)) T->visible = 0;
    if (!T->visible) return;

    /* pinhole projection with the perspective divide */
    for (int i = 0; i < 3; ++i) {
        T->q[i][0] = cam->fx * T->xc[i][0] / T->xc[i][2] + cam->cx;
        T->q[i][1] = cam->fy * T->xc[i][1] / T->xc[i][2] + cam->cy;
    }
    T->perim = 0.0;
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3;
        T->e[k][0] = T->q[k1][0] - T->q[k][0];
        T->e[k][1] = T->q[k1][1] - T->q[k][1];
        T->len[k] = sqrt(T->e[k][0] * T->e[k][0] + T->e[k][1] * T->e[k][1]);
        T->perim += T->len[k];
    }
    T->area2 = T->e[0][0] * (T->q[2][1] - T->q[0][1]) - T->e[0][1] * (T->q[2][0] - T->q[0][0]);
    T->sgn = T->area2 >= 0.0 ? 1.0 : -1.0;
    T->r = T->perim > 0.0 ? fabs(T->area2) / T->perim : 0.0;
    /* the sigmoid stays below 1, so it needs o > alpha_min strictly */
    const int o_ok = cfg->window == WIN_SIGMOID ? o > cfg->alpha_min : o >= cfg->alpha_min;
    if (!(T->r >= cfg->r_min) || !o_ok) { T->visible = 0; return; }

    /* edge lines with unit normals pointing out of the triangle */
    for (int k = 0; k < 3; ++k) {
        T->n[k][0] = T->sgn * T->e[k][1] / T->len[k];
        T->n[k][1] = -T->sgn * T->e[k][0] / T->len[k];
        T->d[k] = -(T->n[k][0] * T->q[k][0] + T->n[k][1] * T->q[k][1]);
    }
    /* incentre: vertices weighted by the length of the opposite edge */
    T->s[0] = (T->len[1] * T->q[0][0] + T->len[2] * T->q[1][0] + T->len[0] * T->q[2][0]) / T->perim;
    T->s[1] = (T->len[1] * T->q[0][1] + T->len[2] * T->q[1][1] + T->len[0] * T->q[2][1]) / T->perim;
    T->phis = phi_at(T, T->s[0], T->s[1], NULL);
    if (cfg->window == WIN_LSE) {
        /* a triangle whose LogSumExp SDF is not negative at s has no inside */
        T->phis_lse = lse_at(T, T->s[0], T->s[1], NULL);
        if (!(T->phis_lse < 0.0)) { T->visible = 0; return; }
    }

    /* colour: SH along the direction from the camera centre to the centroid */
    double cc[3], cen[3];
    for (int a = 0; a < 3; ++a)
        cc[a] = -(cam->R[0 + a] * cam->t[0] + cam->R[3 + a] * cam->t[1] + cam->R[6 + a] * cam->t[2]);
    for (int a = 0; a < 3; ++a) cen[a] = (v[a] + v[3 + a] + v[6 + a]) / 3.0;
    double dv[3] = {cen[0] - cc[0], cen[1] - cc[1], cen[2] - cc[2]};
    T->dnorm = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int a = 0; a < 3; ++a) T->dir[a] = dv[a] / T->dnorm;
    const int K = (cfg->deg + 1) * (cfg->deg + 1);
    sh_eval(cfg->deg, T->dir, T->Y, NULL);
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += sh[3 * k + c] * T->Y[k];
        T->rgb_raw[c] = acc + 0.5;
        T->rgb[c] = T->rgb_raw[c] > 0.0 ? T->rgb_raw[c] : 0.0;
    }

    /* tight bounding box (Supp., "Tile assignment"): move every edge line
     * inward by d = L(s) (tau/o)^(1/sigma), with L(s) = -phi(s) the distance
     * from the edges to the incentre; the shrunk triangle's corners are the
     * pairwise intersections of consecutive moved lines.
     * Sigmoid window: o sigmoid(-phi/sigma) >= tau where
     * phi <= sigma log(o/tau - 1), so the lines move by d = -sigma log(o/tau - 1)
     * (outward when d < 0); nothing is left when d >= r.
     * LogSumExp SDF: it is at least the max, so {o I >= tau} lies inside
     * {phi <= phi_lse(s) (tau/o)^(1/sigma)}: d = -phi_lse(s) (tau/o)^(1/sigma). */
    double dist;
    if (cfg->window == WIN_SIGMOID) {
        dist = -sigma * log(o / cfg->alpha_min - 1.0);
        if (!(dist < T->r)) { T->visible = 0; return; }
    } else if (cfg->window == WIN_LSE) {
        dist = -T->phis_lse * pow(cfg->alpha_min / o, 1.0 / sigma);
    } else {
        dist = -T->phis * pow(cfg->alpha_min / o, 1.0 / sigma);
    }
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    if (isinf(dist)) {   /* sigmoid with alpha_min = 0: unbounded support */
        xmin = ymin = -1e300;
        xmax = ymax = 1e300;
    }
    for (int k = 0; k < 3 && !isinf(dist); ++k) {
        int j = (k + 2) % 3;                 /* edges j and k meet at vertex k */
        double a1 = T->n[j][0], b1 = T->n[j][1], c1 = -(T->d[j] + dist);
        double a2 = T->n[k][0], b2 = T->n[k][1], c2 = -(T->d[k] + dist);
        double det = a1 * b2 - b1 * a2;
        double x = (c1 * b2 - b1 * c2) / det;
        double y = (a1 * c2 - c1 * a2) / det;
        if (x < xmin) xmin = x;
        if (x > xmax) xmax = x;
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
    }
    /* pixel (i,j) is sampled at its centre (i+1/2, j+1/2) */
    double fx0 = ceil(xmin - 0.5), fx1 = floor(xmax - 0.5);
    double fy0 = ceil(ymin - 0.5), fy1 = floor(ymax - 0.5);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > cam->W - 1) fx1 = cam->W - 1;
    if (fy1 > cam->H - 1) fy1 = cam->H - 1;
    if (fx0 <= fx1 && fy0 <= fy1) {
        T->rect[0] = (int)fx0; T->rect[1] = (int)fx1;
        T->rect[2] = (int)fy0; T->rect[3] = (int)fy1;
        T->ntiles = (T->rect[1] / 16 - T->rect[0] / 16 + 1) * (T->rect[3] / 16 - T->rect[2] / 16 + 1);
    }
}

typedef struct {
    int n;          /* triangles */
    int K;
    otri* tri;
    int* order;     /* visible triangles, front to back */
    int nvis;
} oscene;

static const otri* g_sort_tri;
static int cmp_depth(const void* a, const void* b)
{
    int i = *(const int*)a, j = *(const int*)b;
    float ki = g_sort_tri[i].key, kj = g_sort_tri[j].key;
    if (ki < kj) return -1;
    if (ki > kj) return 1;
    return (i > j) - (i < j);
}

static int build_scene(int N, const double* v, const double* o, const double* sigma,
                       const double* sh, const ocam* cam, const ocfg* cfg, oscene* S)
{
    S->n = N;
    S->K = (cfg->deg + 1) * (cfg->deg + 1);
    S->tri = (otri*)malloc(sizeof(otri) * (size_t)(N > 0 ? N : 1));
    S->order = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    if (!S->tri || !S->order) return -1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        setup_tri(v + 9 * (size_t)i, o[i], sigma[i], sh + (size_t)S->K * 3 * i, cam, cfg, &S->tri[i]);
    S->nvis = 0;
    for (int i = 0; i < N; ++i)
        if (S->tri[i].visible) S->order[S->nvis++] = i;
    g_sort_tri = S->tri;
    qsort(S->order, (size_t)S->nvis, sizeof(int), cmp_depth);
    return 0;
}

static void free_scene(oscene* S)
{
    free(S->tri);
    free(S->order);
}

/* ------------------------------------------------------------------------ */
/* Per-pixel forward: front-to-back compositing                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int tri, kmax, clamped;
    double u, I, a, T;  /* T = transmittance before this fragment */
} frag;

typedef struct {
    double C[3], D, T;
    int nfrag;
    int flag;           /* bit0 alpha near alpha_min, bit1 T near T_min, bit2 depth tie */
    int ndec;           /* decisions taken within a band (bits 0 and 1), in walk order */
    uint64_t hash;      /* discrete state: composited set, argmax edges, clamps, stop */
} pixout;

static uint64_t fnv(uint64_t h, uint64_t x)
{
    for (int b = 0; b < 8; ++b) {
        h ^= (x >> (8 * b)) & 0xffu;
        h *= 1099511628211ull;
    }
    return h;
}

/* frags == NULL: forward only.  Otherwise the composited fragments are
 * stored (capacity cap) and their count returned through *nf.
 *
 * A decision taken within its band (alpha against alpha_min, T(1 - alpha)
 * against T_min) could go either way under rounding, and both outcomes are
 * correct renders of the pixel.  Such decisions are numbered in walk order
 * (out->ndec counts them); bit d of `flip` takes the other outcome of the
 * d-th one, so the alternatives a rounding difference can produce are
 * enumerable. */
static void shade_pixel_flip(const oscene* S, const ocfg* cfg, double px, double py,
                             pixout* out, frag* frags, int cap, int* nf, uint32_t flip)
{
    double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
    int nfrag = 0, flag = 0, ndec = 0;
    uint64_t h = 1469598103934665603ull;
    float prev_key = -1.0f;
    int have_prev = 0;
    for (int oi = 0; oi < S->nvis; ++oi) {
        const int i = S->order[oi];
        const otri* tr = &S->tri[i];
        int k;
        double phi = phi_at(tr, px, py, &k);
        double u, I;
        if (cfg->window == WIN_SIGMOID) {          /* Eq. 2; u holds phi */
            u = phi;
            I = 1.0 / (1.0 + exp(phi / tr->sigma));
        } else {
            if (cfg->window == WIN_LSE) phi = lse_at(tr, px, py, NULL);
            u = phi / (cfg->window == WIN_LSE ? tr->phis_lse : tr->phis);
            if (!(u > 0.0)) continue;
            I = pow(u, tr->sigma);
        }
        double a = tr->o * I;
        int clamped = 0;
        if (a > cfg->alpha_max) { a = cfg->alpha_max; clamped = 1; }
        int skip = a < cfg->alpha_min;
        if (fabs(a - cfg->alpha_min) < cfg->band_alpha) {
            flag |= 1;
            if (ndec < 32 && ((flip >> ndec) & 1u)) skip = !skip;
            ++ndec;
        }
        if (skip) continue;
        if (have_prev && (double)tr->key - (double)prev_key <= 2.0 * (double)(nextafterf(prev_key, 1e30f) - prev_key))
            flag |= 4;
        prev_key = tr->key; have_prev = 1;
        double Tn = T * (1.0 - a);
        int stop = Tn < cfg->T_min;
        if (fabs(Tn - cfg->T_min) < cfg->band_T) {
            flag |= 2;
            if (ndec < 32 && ((flip >> ndec) & 1u)) stop = !stop;
            ++ndec;
        }
        if (stop) {
            h = fnv(h, ((uint64_t)i << 8) | 0xffu);
            break;
        }
        if (frags && nfrag < cap) {
            frag* f = &frags[nfrag];
            f->tri = i; f->kmax = k; f->clamped = clamped;
            f->u = u; f->I = I; f->a = a; f->T = T;
        }
        double w = a * T;
        for (int c = 0; c < 3; ++c) C[c] += w * tr->rgb[c];
        D += w * tr->zc;
        T = Tn;
        ++nfrag;
        h = fnv(h, ((uint64_t)i << 8) | ((uint64_t)k << 1) | (uint64_t)clamped);
    }
    for (int c = 0; c < 3; ++c) out->C[c] = C[c] + cfg->bg[c] * T;
    out->D = D;
    out->T = T;
    out->nfrag = nfrag;
    out->flag = flag;
    out->ndec = ndec;
    out->hash = h;
    if (nf) *nf = nfrag;
}

static void shade_pixel(const oscene* S, const ocfg* cfg, double px, double py,
                        pixout* out, frag* frags, int cap, int* nf)
{
    shade_pixel_flip(S, cfg, px, py, out, frags, cap, nf, 0u);
}

/* ------------------------------------------------------------------------ */
/* Exported API                                                              */
/* ------------------------------------------------------------------------ */

/* Per-triangle setup dump.  Arrays have N (or N*x) entries:
 *   vis[N], q[N*6], r[N], s[N*2], phis[N], zc[N], key[N] (float), rgb[N*3],
 *   rect[N*4], ntiles[N]. Any pointer may be NULL. */
int oracle_setup(int N, const double* v, const double* o, const double* sigma,
                 const double* sh, int deg, const double* cam16, int W, int H,
                 const double* cfg9, int* vis, double* q, double* r, double* s,
                 double* phis, double* zc, float* key, double* rgb, int* rect, int* ntiles)
{
    ocam cam; ocfg cfg;
    load_cam(cam16, W, H, &cam);
    load_cfg(cfg9, deg, &cfg);
    const int K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i) {
        otri T;
        setup_tri(v + 9 * (size_t)i, o[i], sigma[i], sh + (size_t)K * 3 * i, &cam, &cfg, &T);
        if (vis) vis[i] = T.visible;
        if (q) for (int a = 0; a < 6; ++a) q[6 * (size_t)i + a] = T.q[a / 2][a % 2];
        if (r) r[i] = T.r;
        if (s) { s[2 * (size_t)i] = T.s[0]; s[2 * (size_t)i + 1] = T.s[1]; }
        if (phis) phis[i] = T.phis;
        if (zc) zc[i] = T.zc;
        if (key) key[i] = T.key;
        if (rgb) for (int c = 0; c < 3; ++c) rgb[3 * (size_t)i + c] = T.rgb[c];
        int vis_rect = T.visible && T.ntiles > 0;
        if (rect) for (int a = 0; a < 4; ++a) rect[4 * (size_t)i + a] = vis_rect ? T.rect[a] : (a & 1 ? -1 : 0);
        if (ntiles) ntiles[i] = vis_rect ? T.ntiles : 0;
    }
    return 0;
}

/* Window at one point for one 2D triangle q[6].  window 0: u = phi(p)/phi(s)
 * and I = ReLU(u)^sigma; 1: u = phi(p) and I = sigmoid(-phi(p)/sigma);
 * 2: u = phi_lse(p)/phi_lse(s) and I = ReLU(u)^sigma (u = 0 when
 * phi_lse(s) >= 0). */
int oracle_window(const double* q6, double px, double py, double sigma, int window,
                  double* u_out, double* I_out)
{
    otri T;
    memset(&T, 0, sizeof T);
    for (int a = 0; a < 6; ++a) T.q[a / 2][a % 2] = q6[a];
    T.perim = 0.0;
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3;
        T.e[k][0] = T.q[k1][0] - T.q[k][0];
        T.e[k][1] = T.q[k1][1] - T.q[k][1];
        T.len[k] = sqrt(T.e[k][0] * T.e[k][0] + T.e[k][1] * T.e[k][1]);
        T.perim += T.len[k];
    }
    T.area2 = T.e[0][0] * (T.q[2][1] - T.q[0][1]) - T.e[0][1] * (T.q[2][0] - T.q[0][0]);
    T.sgn = T.area2 >= 0.0 ? 1.0 : -1.0;
    for (int k = 0; k < 3; ++k) {
        T.n[k][0] = T.sgn * T.e[k][1] / T.len[k];
        T.n[k][1] = -T.sgn * T.e[k][0] / T.len[k];
        T.d[k] = -(T.n[k][0] * T.q[k][0] + T.n[k][1] * T.q[k][1]);
    }
    T.s[0] = (T.len[1] * T.q[0][0] + T.len[2] * T.q[1][0] + T.len[0] * T.q[2][0]) / T.perim;
    T.s[1] = (T.len[1] * T.q[0][1] + T.len[2] * T.q[1][1] + T.len[0] * T.q[2][1]) / T.perim;
    T.phis = phi_at(&T, T.s[0], T.s[1], NULL);
    if (window == WIN_SIGMOID) {
        const double phi = phi_at(&T, px, py, NULL);
        *u_out = phi;
        *I_out = 1.0 / (1.0 + exp(phi / sigma));
        return 0;
    }
    double u;
    if (window == WIN_LSE) {
        const double ps = lse_at(&T, T.s[0], T.s[1], NULL);
        u = ps < 0.0 ? lse_at(&T, px, py, NULL) / ps : 0.0;
    } else {
        u = phi_at(&T, px, py, NULL) / T.phis;
    }
    *u_out = u;
    *I_out = u > 0.0 ? pow(u, sigma) : 0.0;
    return 0;
}

/* Real SH basis (and gradient) at a unit direction. Y[K], dY[K*3]. */
int oracle_sh(int deg, const double* dir3, double* Y, double* dY)
{
    if (deg < 0 || deg > 3) return -1;
    sh_eval(deg, dir3, Y, (double (*)[3])dY);
    return 0;
}

/* Forward render of npix pixels (pix = linear indices y*W+x, or NULL for the
 * full frame in row-major order).  Outputs per pixel: rgb[3*npix] (planar:
 * channel c at rgb[c*npix + p]), alpha, depth, T_final, nfrag, flag, hash. */
int oracle_render(int N, const double* v, const double* o, const double* sigma,
                  const double* sh, int deg, const double* cam16, int W, int H,
                  const double* cfg9, int64_t npix, const int64_t* pix,
                  double* rgb, double* alpha, double* depth, double* T_final,
                  int* nfrag, int* flag, uint64_t* hash)
{
    ocam cam; ocfg cfg; oscene S;
    load_cam(cam16, W, H, &cam);
    load_cfg(cfg9, deg, &cfg);
    if (build_scene(N, v, o, sigma, sh, &cam, &cfg, &S)) return -1;
    if (!pix) npix = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
        int64_t lin = pix ? pix[p] : p;
        double px = (double)(lin % W) + 0.5, py = (double)(lin / W) + 0.5;
        pixout po;
        shade_pixel(&S, &cfg, px, py, &po, NULL, 0, NULL);
        for (int c = 0; c < 3; ++c) rgb[c * npix + p] = po.C[c];
        alpha[p] = 1.0 - po.T;
        depth[p] = po.D;
        T_final[p] = po.T;
        if (nfrag) nfrag[p] = po.nfrag;
        if (flag) flag[p] = po.flag;
        if (hash) hash[p] = po.hash;
    }
    free_scene(&S);
    return 0;
}

/* The same forward on npix listed pixels, each with its own mask of
 * near-threshold decisions to take the other way (see shade_pixel_flip):
 * flips[p] for pixel pix[p].  ndec[p] receives the number of such decisions
 * met on the way (in the flipped walk). */
int oracle_render_flip(int N, const double* v, const double* o, const double* sigma,
                       const double* sh, int deg, const double* cam16, int W, int H,
                       const double* cfg9, int64_t npix, const int64_t* pix,
                       const uint32_t* flips, double* rgb, double* alpha, double* depth,
                       double* T_final, int* ndec)
{
    ocam cam; ocfg cfg; oscene S;
    if (!pix || !flips) return -2;
    load_cam(cam16, W, H, &cam);
    load_cfg(cfg9, deg, &cfg);
    if (build_scene(N, v, o, sigma, sh, &cam, &cfg, &S)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < npix; ++p) {
        int64_t lin = pix[p];
        double px = (double)(lin % W) + 0.5, py = (double)(lin / W) + 0.5;
        pixout po;
        shade_pixel_flip(&S, &cfg, px, py, &po, NULL, 0, NULL, flips[p]);
        for (int c = 0; c < 3; ++c) rgb[c * npix + p] = po.C[c];
        alpha[p] = 1.0 - po.T;
        depth[p] = po.D;
        T_final[p] = po.T;
        if (ndec) ndec[p] = po.ndec;
    }
    free_scene(&S);
    return 0;
}

/* Pruning statistics (Sec. 3.2, "Pruning"): over the given pixels (all of
 * them when pix is NULL), for every triangle the largest blending weight
 * T * o at a fragment of it that is composited (T the transmittance in front
 * of the fragment, o the triangle's opacity) and the number of pixels where
 * it is composited.  maxw[N] and npix[N] are overwritten (0 where never
 * composited). */
int oracle_prune_stats(int N, const double* v, const double* o, const double* sigma,
                       const double* sh, int deg, const double* cam16, int W, int H,
                       const double* cfg9, int64_t npix, const int64_t* pix,
                       double* maxw, int* npx)
{
    ocam cam; ocfg cfg; oscene S;
    load_cam(cam16, W, H, &cam);
    load_cfg(cfg9, deg, &cfg);
    if (build_scene(N, v, o, sigma, sh, &cam, &cfg, &S)) return -1;
    if (!pix) npix = (int64_t)W * H;
    for (int i = 0; i < N; ++i) { maxw[i] = 0.0; npx[i] = 0; }
    const int cap = S.nvis > 0 ? S.nvis : 1;
#pragma omp parallel
    {
        double* lw = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
        int* ln = (int*)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
        frag* fr = (frag*)malloc(sizeof(frag) * (size_t)cap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            int64_t lin = pix ? pix[p] : p;
            double px = (double)(lin % W) + 0.5, py = (double)(lin / W) + 0.5;
            pixout po;
            int nf = 0;
            shade_pixel(&S, &cfg, px, py, &po, fr, cap, &nf);
            for (int f = 0; f < nf; ++f) {
                const int i = fr[f].tri;
                const double wt = fr[f].T * S.tri[i].o;
                if (wt > lw[i]) lw[i] = wt;
                ln[i] += 1;
            }
        }
#pragma omp critical
        for (int i = 0; i < N; ++i) {
            if (lw[i] > maxw[i]) maxw[i] = lw[i];
            npx[i] += ln[i];
        }
        free(lw); free(ln); free(fr);
    }
    free_scene(&S);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Analytic gradient (FP64)                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    double gq[3][2];    /* dL/dq_i */
    double gzc;         /* dL/dz_centre */
    double grgb[3];     /* dL/drgb (after the clamp at zero) */
    double go, gsig;
} tacc;

static void atomic_add(double* p, double x)
{
#pragma omp atomic
    *p += x;
}

/* d r / d q for r = |2A| / P */
static void dr_dq(const otri* T, double g[3][2])
{
    const double* q0 = T->q[0]; const double* q1 = T->q[1]; const double* q2 = T->q[2];
    double dA[3][2] = {
        {q1[1] - q2[1], q2[0] - q1[0]},
        {q2[1] - q0[1], q0[0] - q2[0]},
        {q0[1] - q1[1], q1[0] - q0[0]},
    };
    double dP[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3;
        for (int a = 0; a < 2; ++a) {
            dP[k1][a] += T->e[k][a] / T->len[k];
            dP[k][a] -= T->e[k][a] / T->len[k];
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 2; ++a)
            g[i][a] = T->sgn * dA[i][a] / T->perim - T->r / T->perim * dP[i][a];
}

/* d L_k(p) / d q for L_k(p) = n_k . (p - q_k), n_k = sgn * (e_y, -e_x)/|e| */
static void dL_dq(const otri* T, int k, double px, double py, double g[3][2])
{
    int k1 = (k + 1) % 3;
    const double ex = T->e[k][0], ey = T->e[k][1], l = T->len[k];
    const double wx = px - T->q[k][0], wy = py - T->q[k][1];
    /* (dn/de)^T w = sgn * (R^T w / l - e ((R e) . w) / l^3), R e = (ey, -ex) */
    const double Re_w = ey * wx - ex * wy;
    const double jx = T->sgn * (-wy / l - ex * Re_w / (l * l * l));
    const double jy = T->sgn * (wx / l - ey * Re_w / (l * l * l));
    for (int i = 0; i < 3; ++i) g[i][0] = g[i][1] = 0.0;
    g[k][0] = -T->n[k][0] - jx;
    g[k][1] = -T->n[k][1] - jy;
    g[k1][0] += jx;
    g[k1][1] += jy;
}

/* Gradient of L = sum_p [ dC_p . rgb_p + dA_p alpha_p + dD_p depth_p ] over
 * the given pixels.  dC is planar [3][npix]; dA, dD may be NULL.
 * Outputs (overwritten): gv[N*9], go[N], gsig[N], gsh[N*K*3]. */
int oracle_backward(int N, const double* v, const double* o, const double* sigma,
                    const double* sh, int deg, const double* cam16, int W, int H,
                    const double* cfg9, int64_t npix, const int64_t* pix,
                    const double* dC, const double* dA, const double* dD,
                    double* gv, double* go, double* gsig, double* gsh)
{
    ocam cam; ocfg cfg; oscene S;
    load_cam(cam16, W, H, &cam);
    load_cfg(cfg9, deg, &cfg);
    if (build_scene(N, v, o, sigma, sh, &cam, &cfg, &S)) return -1;
    const int K = S.K;
    tacc* acc = (tacc*)calloc((size_t)(N > 0 ? N : 1), sizeof(tacc));
    if (!acc) { free_scene(&S); return -1; }
    if (!pix) npix = (int64_t)W * H;

#pragma omp parallel
    {
        int cap = 4096;
        frag* fr = (frag*)malloc(sizeof(frag) * (size_t)cap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            int64_t lin = pix ? pix[p] : p;
            double px = (double)(lin % W) + 0.5, py = (double)(lin / W) + 0.5;
            pixout po;
            int nf = 0;
            shade_pixel(&S, &cfg, px, py, &po, fr, cap, &nf);
            if (nf > cap) {
                while (cap < nf) cap *= 2;
                free(fr);
                fr = (frag*)malloc(sizeof(frag) * (size_t)cap);
                shade_pixel(&S, &cfg, px, py, &po, fr, cap, &nf);
            }
            const double gC[3] = {dC[p], dC[npix + p], dC[2 * npix + p]};
            const double gA = dA ? dA[p] : 0.0;
            const double gD = dD ? dD[p] : 0.0;
            const double Tf = po.T;
            double SC[3] = {0, 0, 0}, SD = 0.0;   /* sum over later fragments of w c, w z */
            for (int f = nf - 1; f >= 0; --f) {
                const frag* F = &fr[f];
                const otri* tr = &S.tri[F->tri];
                tacc* A = &acc[F->tri];
                const double a = F->a, Ti = F->T, w = a * Ti, om = 1.0 - a;
                /* colour and depth */
                for (int c = 0; c < 3; ++c) atomic_add(&A->grgb[c], gC[c] * w);
                atomic_add(&A->gzc, gD * w);
                /* alpha: C = sum c_i a_i T_i + bg T_final, D likewise, alpha = 1 - T_final */
                double ga = 0.0;
                for (int c = 0; c < 3; ++c) ga += gC[c] * (tr->rgb[c] * Ti - SC[c] / om);
                ga += gD * (tr->zc * Ti - SD / om);
                double gbg = 0.0;
                for (int c = 0; c < 3; ++c) gbg += gC[c] * cfg.bg[c];
                ga += (gA - gbg) * Tf / om;
                for (int c = 0; c < 3; ++c) SC[c] += w * tr->rgb[c];
                SD += w * tr->zc;
                if (F->clamped) continue;             /* alpha = alpha_max: flat */
                /* a = o I */
                atomic_add(&A->go, ga * F->I);
                const double gI = ga * tr->o;
                double gL[3][2], gr[3][2];
                dL_dq(tr, F->kmax, px, py, gL);
                if (cfg.window == WIN_SIGMOID) {
                    /* I = 1/(1 + exp(phi/sigma)), phi = L_k(p):
                     * dI/dphi = -I(1-I)/sigma, dI/dsigma = I(1-I) phi/sigma^2 */
                    const double s = tr->sigma, g = gI * F->I * (1.0 - F->I);
                    atomic_add(&A->gsig, g * F->u / (s * s));
                    for (int i = 0; i < 3; ++i)
                        for (int c = 0; c < 2; ++c) atomic_add(&A->gq[i][c], -g / s * gL[i][c]);
                    continue;
                }
                /* I = u^sigma */
                atomic_add(&A->gsig, gI * F->I * log(F->u));
                const double gu = gI * tr->sigma * F->I / F->u;
                double phis = tr->phis;
                if (cfg.window == WIN_LSE) {
                    /* phi = log sum_k exp L_k(p): dphi = sum_k w_k dL_k (softmax
                     * weights); at s every L_k equals -r, so phi_lse(s) =
                     * log 3 - r and dphi_lse(s) = -dr, as for the max */
                    double w[3], gk[3][2];
                    lse_at(tr, px, py, w);
                    for (int i = 0; i < 3; ++i) gL[i][0] = gL[i][1] = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        dL_dq(tr, k, px, py, gk);
                        for (int i = 0; i < 3; ++i)
                            for (int c = 0; c < 2; ++c) gL[i][c] += w[k] * gk[i][c];
                    }
                    phis = tr->phis_lse;
                }
                /* u = phi(p) / phi(s),  dphi(s) = -dr */
                dr_dq(tr, gr);
                for (int i = 0; i < 3; ++i)
                    for (int c = 0; c < 2; ++c) {
                        /* du = (dphi - u dphis)/phis, dphis = -dr */
                        double du = (gL[i][c] + F->u * gr[i][c]) / phis;
                        atomic_add(&A->gq[i][c], gu * du);
                    }
            }
        }
        free(fr);
    }

    /* per triangle: 2D -> camera space -> world, colour -> SH */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i) {
        const otri* tr = &S.tri[i];
        const tacc* A = &acc[i];
        double* gvi = gv + 9 * (size_t)i;
        double* gshi = gsh + (size_t)K * 3 * i;
        for (int a = 0; a < 9; ++a) gvi[a] = 0.0;
        for (int a = 0; a < K * 3; ++a) gshi[a] = 0.0;
        go[i] = 0.0; gsig[i] = 0.0;
        if (!tr->visible) continue;
        go[i] = A->go;
        gsig[i] = A->gsig;
        for (int j = 0; j < 3; ++j) {
            const double x = tr->xc[j][0], y = tr->xc[j][1], z = tr->xc[j][2];
            double gx[3];
            gx[0] = cam.fx / z * A->gq[j][0];
            gx[1] = cam.fy / z * A->gq[j][1];
            gx[2] = -cam.fx * x / (z * z) * A->gq[j][0] - cam.fy * y / (z * z) * A->gq[j][1]
                  + A->gzc / 3.0;
            for (int b = 0; b < 3; ++b)                      /* R^T gx */
                gvi[3 * j + b] += cam.R[0 + b] * gx[0] + cam.R[3 + b] * gx[1] + cam.R[6 + b] * gx[2];
        }
        double Y[MAXK], dY[MAXK][3];
        sh_eval(cfg.deg, tr->dir, Y, dY);
        double geff[3];
        for (int c = 0; c < 3; ++c) geff[c] = tr->rgb_raw[c] > 0.0 ? A->grgb[c] : 0.0;
        double gdir[3] = {0, 0, 0};
        for (int k = 0; k < K; ++k)
            for (int c = 0; c < 3; ++c) {
                gshi[3 * k + c] = geff[c] * Y[k];
                const double shc = sh[(size_t)K * 3 * i + 3 * k + c];
                for (int b = 0; b < 3; ++b) gdir[b] += geff[c] * shc * dY[k][b];
            }
        /* dir = dv/|dv|, dv = centroid - camera centre */
        const double dd = tr->dir[0] * gdir[0] + tr->dir[1] * gdir[1] + tr->dir[2] * gdir[2];
        for (int b = 0; b < 3; ++b) {
            const double gdv = (gdir[b] - tr->dir[b] * dd) / tr->dnorm;
            for (int j = 0; j < 3; ++j) gvi[3 * j + b] += gdv / 3.0;
        }
    }
    free(acc);
    free_scene(&S);
    return 0;
}

/* Number of OpenMP threads the oracle runs with. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
