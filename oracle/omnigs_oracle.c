/*
 * omnigs_oracle.c -- plain FP64 CPU oracle of the omnidirectional (ERP) Gaussian
 * rasterizer of OmniGS (arXiv 2404.03202).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * implementation.  It is deliberately slow and literal: every quantity is
 * computed in double precision in the order the paper states it, with no
 * blocking or fusion beyond the tile-based pipeline the paper itself describes
 * (Sec. 3.3, the paragraph on tile-based forward rendering).
 *
 * Paper sections followed (numbering of the paper):
 *   Eq. 1        t = W m + t_cw                                 (Sec. 3.2)
 *   Eq. 3        lon = atan2(t_x, t_z), lat = asin(t_y / t_r)    (Sec. 3.2)
 *   Eq. 4        s = (lon / pi, 2 lat / pi)                     (Sec. 3.2)
 *   Eq. 5        p = ((s_x + 1) W / 2, (s_y + 1) H / 2)          (Sec. 3.2)
 *   Eq. 6        C = sum_i c_i a_i prod_{j<i} (1 - a_j), sorted by t_r (Sec. 3.3)
 *   Eq. 7, 8     a_i = o_i exp(-1/2 dp^T Sigma2D^-1 dp)          (Sec. 3.3)
 *   Eq. 9        Sigma2D = J W Sigma W^T J^T, 3rd row/col dropped (Sec. 3.3)
 *   Eq. 10-16    the spherical Jacobian J                        (Sec. 3.3)
 *   Eq. 17       L1 photometric term                             (Sec. 3.4)
 *   Eq. 18-20    chain rule to m, q, S through the replaced
 *                omnidirectional terms dSigma2D/dSigma, dJ/dt,
 *                dp/ds, ds/dt                                    (Sec. 3.4)
 *   Eq. 2        the perspective (pinhole) camera the paper starts from,
 *                p = (f_x t_x / t_z + c_x, f_y t_y / t_z + c_y), with its
 *                Jacobian in Eq. 9 and instances ordered by t_z (Sec. 3.2,
 *                3.3); selected per camera
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - atan2 takes (t_x, t_z); lon = +pi is mapped to -pi (Eq. 3 range).
 *   - J's (2,3) entry is dp_y/dt_z (Eq. 16; the matrix of Eq. 10 misprints it).
 *   - pixel (x, y) samples the continuous image at (x + 1/2, y + 1/2).
 *   - the longitude seam: the x offset to a Gaussian is taken as the shortest
 *     signed offset on the circle of circumference W, in [-W/2, W/2); tile
 *     columns wrap modulo W/16; rows do not wrap (they clamp at the poles).
 *   - Sigma = R diag(S)^2 R^T with R from the normalised quaternion (w,x,y,z).
 *   - a low-pass "dilation" is added to the diagonal of Sigma2D.
 *   - a Gaussian's radius of influence is the axis-aligned box of its
 *     alpha = alpha_min iso-ellipse, so the tiled result equals the
 *     per-pixel brute-force result.
 *   - alpha is clamped to alpha_max; alpha < alpha_min is skipped; blending
 *     stops before an instance that would bring T below T_min.
 *   - colour = real spherical harmonics (Condon-Shortley phase, m = -l..l
 *     ordering, z polar) of the world-frame unit direction from the camera
 *     centre to m, plus 1/2, clamped below at 0.
 *   - gradient is taken w.r.t. activated scales and opacities, the raw
 *     quaternion (normalised inside), means and SH coefficients.
 *   - pinhole camera: J is the derivative of Eq. 2 evaluated at the
 *     Gaussian's direction with t_x / t_z and t_y / t_z clamped to 1.3 times
 *     the image's angular half-extent around its middle (3DGS's guard against
 *     the affine approximation's blow-up near the image plane; p itself is not
 *     clamped, and J's derivative is that of the clamped function);
 *     Gaussians with t_z <= near_plane are
 *     culled; the depth order is (t_z, index); pixel (x, y) samples at
 *     (x + 1/2, y + 1/2); nothing wraps: columns clamp like rows, and the
 *     width need not be a multiple of 16 (the last tile column is ragged);
 *     the screen-space gradient is (W/2, H/2) * dL/dp as for the ERP image.
 *   - loss masks (Sec. 4, the 360Roam evaluation skips the images' bottom
 *     rows): a camera may render only its top `rows` rows (the mapping still
 *     uses the full height H); the image then has `rows` rows.
 *   - auxiliary outputs of the same blend: the depth image
 *     D = sum_i d_i alpha_i T_i (d = the sort depth, t_r or t_z) and the
 *     alpha image A = 1 - T_final = sum_i alpha_i T_i; both back-propagate
 *     like colour channels with colour d_i (respectively 1) and a zero
 *     background, and dL/dd_i reaches the mean through d(t_r)/dt = t / t_r or
 *     d(t_z)/dt = (0, 0, 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16
#define ORC_MAXK 16
#define ORC_ERP 0
#define ORC_PINHOLE 1

typedef struct {
    int64_t n;
    const double *means;  /* [n][3] world positions m                    */
    const double *scales; /* [n][3] activated scales S (> 0)              */
    const double *quats;  /* [n][4] raw quaternion (w, x, y, z)           */
    const double *opac;   /* [n]    activated opacity o in (0, 1)         */
    const double *sh;     /* [n][sh_coeffs][3] SH coefficients, RGB last  */
    int32_t sh_degree;    /* active degree D, 0..3                         */
    int32_t sh_coeffs;    /* stored coefficients per Gaussian, >= (D+1)^2  */
    int32_t width, height;
    double R[9];          /* W of Eq. 1, row-major                         */
    double t[3];          /* t_cw of Eq. 1                                 */
    double alpha_min, alpha_max, T_min, dilation, near_plane;
    double bg[3];
    /* near-tie flagging margins (relative for alpha, T, depth; absolute
     * pixels for the rect bounds) */
    double flag_rel_alpha, flag_rel_T, flag_rel_depth, flag_abs_rect;
    int32_t model;        /* ORC_ERP or ORC_PINHOLE                         */
    int32_t reserved;
    double fx, fy, cx, cy; /* pinhole intrinsics of Eq. 2 (pixels)         */
    int32_t rows;         /* rendered rows: the top `rows` rows (0: all)   */
    int32_t reserved2;
    /* [n][2] pixel offsets added to each projected centre p (NULL: none).
     * Not part of the method: it lets a finite difference move p alone, with
     * the 2D covariance, colour and depth held, to check dL/dp and dL/ds. */
    const double *screen_shift;
} orc_scene;

/* rows of the rendered image */
static int orc_rows(const orc_scene *s) { return s->rows > 0 ? s->rows : s->height; }

/* tile columns: W / 16 for the ERP image (W a multiple of 16, the columns
 * wrap), ceil(W / 16) for the pinhole image */
static int orc_tiles_x(const orc_scene *s) {
    return s->model == ORC_PINHOLE ? (s->width + ORC_TILE - 1) / ORC_TILE : s->width / ORC_TILE;
}

static int orc_valid(const orc_scene *s) {
    if (s->height < 1 || s->width < 1 || s->rows < 0 || s->rows > s->height) return 0;
    if (s->model == ORC_ERP) return s->width % ORC_TILE == 0;
    if (s->model == ORC_PINHOLE) return isfinite(s->fx) && isfinite(s->fy) && s->fx > 0.0 && s->fy > 0.0 &&
                                        isfinite(s->cx) && isfinite(s->cy);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, evaluated from their definition.                */
/* Y_l^0  = N_l^0 P_l(z)                                                      */
/* Y_l^m  = sqrt2 (-1)^m N_l^m  d^m P_l/dz^m (z) Re[(x + i y)^m]      m > 0   */
/* Y_l^-m = sqrt2 (-1)^m N_l^m  d^m P_l/dz^m (z) Im[(x + i y)^m]      m > 0   */
/* N_l^m  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)                                 */
/* Legendre polynomials from Bonnet's recursion.  A forward-mode dual number  */
/* carries d/d(x, y, z) for the backward pass.                                */
/* ------------------------------------------------------------------------ */
typedef struct { double v, d[3]; } dual;

static dual dconst(double v) { dual r = {v, {0, 0, 0}}; return r; }
static dual dadd(dual a, dual b) {
    dual r = {a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
    return r;
}
static dual dsub(dual a, dual b) {
    dual r = {a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
    return r;
}
static dual dmul(dual a, dual b) {
    dual r;
    r.v = a.v * b.v;
    for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
static dual dscale(dual a, double s) {
    dual r = {a.v * s, {a.d[0] * s, a.d[1] * s, a.d[2] * s}};
    return r;
}

static double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return f;
}

/* coefficients of P_l (ascending powers of z), l <= 3 */
static void legendre_coeffs(int l, double c[4]) {
    double P[4][4];
    memset(P, 0, sizeof(P));
    P[0][0] = 1.0;
    P[1][1] = 1.0;
    for (int n = 1; n < 3; ++n) {
        /* (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1} */
        for (int k = 0; k < 4; ++k) {
            double v = 0.0;
            if (k >= 1) v += (2.0 * n + 1.0) * P[n][k - 1];
            v -= (double)n * P[n - 1][k];
            P[n + 1][k] = v / (n + 1.0);
        }
    }
    for (int k = 0; k < 4; ++k) c[k] = P[l][k];
}

/* Y[(l*l + l + m)] for l <= degree, as duals in the direction components */
static void sh_basis_dual(int degree, const double dir[3], dual *Y) {
    dual x = {dir[0], {1, 0, 0}};
    dual y = {dir[1], {0, 1, 0}};
    dual z = {dir[2], {0, 0, 1}};
    for (int l = 0; l <= degree; ++l) {
        double pc[4];
        legendre_coeffs(l, pc);
        for (int m = 0; m <= l; ++m) {
            /* m-th derivative of P_l, evaluated at z (Horner) */
            double dc[4] = {0, 0, 0, 0};
            for (int k = m; k <= l; ++k) dc[k - m] = pc[k] * factorial(k) / factorial(k - m);
            dual poly = dconst(0.0);
            for (int k = l - m; k >= 0; --k) poly = dadd(dmul(poly, z), dconst(dc[k]));
            /* (x + i y)^m */
            dual re = dconst(1.0), im = dconst(0.0);
            for (int k = 0; k < m; ++k) {
                dual nre = dsub(dmul(re, x), dmul(im, y));
                dual nim = dadd(dmul(re, y), dmul(im, x));
                re = nre;
                im = nim;
            }
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            if (m == 0) {
                Y[l * l + l] = dscale(poly, N);
            } else {
                double s = sqrt(2.0) * N * ((m % 2) ? -1.0 : 1.0);
                Y[l * l + l + m] = dscale(dmul(poly, re), s);
                Y[l * l + l - m] = dscale(dmul(poly, im), s);
            }
        }
    }
}

/* exported for the orthonormality pin: Y[(D+1)^2], dY[(D+1)^2][3] */
void orc_sh_eval(int degree, const double *dir, double *Y, double *dY) {
    dual Yd[ORC_MAXK];
    sh_basis_dual(degree, dir, Yd);
    int K = (degree + 1) * (degree + 1);
    for (int i = 0; i < K; ++i) {
        Y[i] = Yd[i].v;
        if (dY)
            for (int k = 0; k < 3; ++k) dY[i * 3 + k] = Yd[i].d[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Per-Gaussian projection (Eq. 1, 3-5, 9-16, SH colour)                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int visible;
    double tc[3], tr, rho;
    double depth;      /* sort key: t_r (ERP) or t_z (pinhole) */
    double dir_c[2];   /* pinhole: t_x / t_z, t_y / t_z after clamping */
    int clamped[2];    /* pinhole: whether each was clamped */
    double lon, lat, px, py;
    double J[6];       /* 2x3, row-major (third row of Eq. 10 is zero) */
    double Jp[6];      /* dp/dt: J itself, except for a guarded pinhole direction */
    double M[6];       /* J W, 2x3 */
    double qn[4], qnorm, Rq[9];
    double Sig[9];     /* 3D covariance */
    double a, b, c, det, Q[3]; /* Sigma2D = [[a,b],[b,c]], Q = inverse: Q00,Q01,Q11 */
    double kcut, ex, ey;
    int full_x;
    int64_t xs, xe, ys, ye;
    int tx0, ntx, ty0, nty;
    int64_t ntiles;
    double dir[3], rgb_raw[3], rgb[3];
    int clamp[3];
    int flag; /* a near-threshold discrete decision in this Gaussian's projection */
} orc_proj;

static int near_int(double v, double tol) { return fabs(v - nearbyint(v)) < tol; }

static int64_t floordiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

static void project_one(const orc_scene *s, int64_t i, orc_proj *P) {
    memset(P, 0, sizeof(*P));
    const double *m = s->means + 3 * i;
    const double W = (double)s->width, H = (double)s->height;
    const double o = s->opac[i];
    /* Eq. 1 */
    for (int r = 0; r < 3; ++r)
        P->tc[r] = s->R[3 * r + 0] * m[0] + s->R[3 * r + 1] * m[1] + s->R[3 * r + 2] * m[2] + s->t[r];
    const double tx = P->tc[0], ty = P->tc[1], tz = P->tc[2];
    P->tr = sqrt(tx * tx + ty * ty + tz * tz);
    P->rho = sqrt(tx * tx + tz * tz);
    if (fabs(o - s->alpha_min) < 1e-9 * s->alpha_min) P->flag = 1;
    if (s->model == ORC_PINHOLE) {
        /* culling: behind the near plane or too transparent */
        if (fabs(tz - s->near_plane) < 1e-9 * s->near_plane) P->flag = 1;
        if (tz <= s->near_plane || o <= s->alpha_min) return;
        P->depth = tz;
        /* Eq. 2 */
        P->px = s->fx * tx / tz + s->cx;
        P->py = s->fy * ty / tz + s->cy;
        /* its Jacobian d p / d t, at the direction clamped to 1.3 x the
         * image's angular half-extent around its middle */
        const double ax = tx / tz, ay = ty / tz;
        const double mx = (0.5 * W - s->cx) / s->fx, hx = 1.3 * 0.5 * W / s->fx;
        const double my = (0.5 * H - s->cy) / s->fy, hy = 1.3 * 0.5 * H / s->fy;
        P->dir_c[0] = ax < mx - hx ? mx - hx : (ax > mx + hx ? mx + hx : ax);
        P->dir_c[1] = ay < my - hy ? my - hy : (ay > my + hy ? my + hy : ay);
        P->clamped[0] = P->dir_c[0] != ax;
        P->clamped[1] = P->dir_c[1] != ay;
        P->J[0] = s->fx / tz;
        P->J[1] = 0.0;
        P->J[2] = -s->fx * P->dir_c[0] / tz;
        P->J[3] = 0.0;
        P->J[4] = s->fy / tz;
        P->J[5] = -s->fy * P->dir_c[1] / tz;
        /* the centre itself moves with the unclamped derivative of Eq. 2 */
        for (int k = 0; k < 6; ++k) P->Jp[k] = P->J[k];
        P->Jp[2] = -s->fx * ax / tz;
        P->Jp[5] = -s->fy * ay / tz;
    } else {
        /* culling: behind the near sphere, too transparent to ever pass
         * alpha_min, or on the polar axis where Eq. 11-16 diverge */
        if (fabs(P->tr - s->near_plane) < 1e-9 * s->near_plane) P->flag = 1;
        if (P->tr <= s->near_plane || o <= s->alpha_min || P->rho <= 1e-6 * P->tr) return;
        P->depth = P->tr;
        /* Eq. 3 */
        P->lon = atan2(tx, tz);
        if (P->lon >= M_PI) P->lon = -M_PI;
        P->lat = asin(ty / P->tr);
        /* Eq. 4, 5 */
        const double sx = P->lon / M_PI, sy = 2.0 * P->lat / M_PI;
        P->px = (sx + 1.0) * W / 2.0;
        P->py = (sy + 1.0) * H / 2.0;
        /* Eq. 11-16 */
        const double rho2 = P->rho * P->rho, r2 = P->tr * P->tr;
        const double kx = W / (2.0 * M_PI), ky = H / M_PI;
        P->J[0] = kx * tz / rho2;
        P->J[1] = 0.0;
        P->J[2] = -kx * tx / rho2;
        P->J[3] = -ky * tx * ty / (r2 * P->rho);
        P->J[4] = ky * P->rho / r2;
        P->J[5] = -ky * tz * ty / (r2 * P->rho);
        for (int k = 0; k < 6; ++k) P->Jp[k] = P->J[k];
    }
    if (s->screen_shift) {
        P->px += s->screen_shift[2 * i];
        P->py += s->screen_shift[2 * i + 1];
    }
    /* M = J W */
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k) {
            double v = 0.0;
            for (int j = 0; j < 3; ++j) v += P->J[3 * a + j] * s->R[3 * j + k];
            P->M[3 * a + k] = v;
        }
    /* Sigma = R diag(S^2) R^T */
    const double *q = s->quats + 4 * i;
    P->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) P->qn[k] = q[k] / P->qnorm;
    const double w = P->qn[0], x = P->qn[1], y = P->qn[2], z = P->qn[3];
    double *Rq = P->Rq;
    Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
    Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
    Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
    const double *S = s->scales + 3 * i;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += Rq[3 * a + k] * S[k] * S[k] * Rq[3 * b + k];
            P->Sig[3 * a + b] = v;
        }
    /* Eq. 9: Sigma2D = M Sigma M^T (+ dilation on the diagonal) */
    double T2[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double v = 0.0;
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) v += P->M[3 * a + j] * P->Sig[3 * j + k] * P->M[3 * b + k];
            T2[a][b] = v;
        }
    P->a = T2[0][0] + s->dilation;
    P->b = T2[0][1];
    P->c = T2[1][1] + s->dilation;
    P->det = P->a * P->c - P->b * P->b;
    if (P->det <= 0.0) return;
    P->Q[0] = P->c / P->det;
    P->Q[1] = -P->b / P->det;
    P->Q[2] = P->a / P->det;
    /* radius of influence: box of the alpha = alpha_min iso-ellipse */
    P->kcut = 2.0 * log(o / s->alpha_min);
    P->ex = sqrt(P->kcut * P->a);
    P->ey = sqrt(P->kcut * P->c);
    const double bx0 = P->px - P->ex - 0.5, bx1 = P->px + P->ex - 0.5;
    const double by0 = P->py - P->ey - 0.5, by1 = P->py + P->ey - 0.5;
    double tol = s->flag_abs_rect;
    if (near_int(bx0, tol + 1e-12 * P->ex) || near_int(bx1, tol + 1e-12 * P->ex) ||
        near_int(by0, tol + 1e-12 * P->ey) || near_int(by1, tol + 1e-12 * P->ey))
        P->flag = 1;
    double cxs = ceil(bx0), cxe = floor(bx1);
    if (s->model == ORC_PINHOLE) {
        /* no seam: columns clamp to the image */
        if (cxs < 0.0) cxs = 0.0;
        if (cxe > W - 1.0) cxe = W - 1.0;
        if (cxe < cxs) return;
        P->xs = (int64_t)cxs;
        P->xe = (int64_t)cxe;
    } else if (cxe - cxs + 1.0 >= W) {
        P->full_x = 1;
        P->xs = 0;
        P->xe = s->width - 1;
    } else {
        if (cxe < cxs) return;
        P->xs = (int64_t)cxs;
        P->xe = (int64_t)cxe;
    }
    double cys = ceil(by0), cye = floor(by1);
    if (cys < 0.0) cys = 0.0;
    if (cye > orc_rows(s) - 1.0) cye = orc_rows(s) - 1.0;
    if (cye < cys) return;
    P->ys = (int64_t)cys;
    P->ye = (int64_t)cye;
    const int tiles_x = orc_tiles_x(s);
    if (s->model == ORC_PINHOLE) {
        P->tx0 = (int)(P->xs / ORC_TILE);
        P->ntx = (int)(P->xe / ORC_TILE) - P->tx0 + 1;
    } else if (P->full_x) {
        P->tx0 = 0;
        P->ntx = tiles_x;
    } else {
        int64_t t0 = floordiv(P->xs, ORC_TILE), t1 = floordiv(P->xe, ORC_TILE);
        int64_t cnt = t1 - t0 + 1;
        if (cnt >= tiles_x) {
            P->tx0 = 0;
            P->ntx = tiles_x;
        } else {
            P->tx0 = (int)(((t0 % tiles_x) + tiles_x) % tiles_x);
            P->ntx = (int)cnt;
        }
    }
    P->ty0 = (int)(P->ys / ORC_TILE);
    P->nty = (int)(P->ye / ORC_TILE) - P->ty0 + 1;
    P->ntiles = (int64_t)P->ntx * P->nty;
    /* colour from SH along the world-frame direction camera centre -> m */
    double cpos[3];
    for (int k = 0; k < 3; ++k)
        cpos[k] = -(s->R[0 * 3 + k] * s->t[0] + s->R[1 * 3 + k] * s->t[1] + s->R[2 * 3 + k] * s->t[2]);
    double v[3] = {m[0] - cpos[0], m[1] - cpos[1], m[2] - cpos[2]};
    double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; ++k) P->dir[k] = v[k] / vn;
    dual Y[ORC_MAXK];
    sh_basis_dual(s->sh_degree, P->dir, Y);
    const int K = (s->sh_degree + 1) * (s->sh_degree + 1);
    const double *shi = s->sh + (int64_t)i * s->sh_coeffs * 3;
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += Y[k].v * shi[3 * k + ch];
        P->rgb_raw[ch] = acc + 0.5;
        P->clamp[ch] = P->rgb_raw[ch] < 0.0;
        P->rgb[ch] = P->clamp[ch] ? 0.0 : P->rgb_raw[ch];
        if (fabs(P->rgb_raw[ch]) < 1e-9) P->flag = 1;
    }
    P->visible = 1;
}

/* ------------------------------------------------------------------------ */
/* Instance lists: one instance per (Gaussian, covered tile), sorted by       */
/* (tile, depth, Gaussian index); depth = t_r (ERP) or t_z (pinhole).         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t tile;
    int32_t gid;
    double tr;
} orc_inst;

static int inst_cmp(const void *pa, const void *pb) {
    const orc_inst *a = (const orc_inst *)pa, *b = (const orc_inst *)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->tr != b->tr) return a->tr < b->tr ? -1 : 1;
    if (a->gid != b->gid) return a->gid < b->gid ? -1 : 1;
    return 0;
}

typedef struct {
    orc_proj *P;
    orc_inst *inst;
    int64_t n_inst;
    int64_t *tstart, *tend;
    int tiles_x, tiles_y;
} orc_lists;

static void lists_free(orc_lists *L) {
    free(L->P);
    free(L->inst);
    free(L->tstart);
    free(L->tend);
    memset(L, 0, sizeof(*L));
}

/* tile_mask may be NULL (all tiles) */
static int build_lists(const orc_scene *s, const uint8_t *tile_mask, orc_lists *L) {
    memset(L, 0, sizeof(*L));
    L->tiles_x = orc_tiles_x(s);
    L->tiles_y = (orc_rows(s) + ORC_TILE - 1) / ORC_TILE;
    const int64_t n = s->n, ntiles = (int64_t)L->tiles_x * L->tiles_y;
    L->P = (orc_proj *)malloc(sizeof(orc_proj) * (size_t)(n > 0 ? n : 1));
    L->tstart = (int64_t *)calloc((size_t)ntiles, sizeof(int64_t));
    L->tend = (int64_t *)calloc((size_t)ntiles, sizeof(int64_t));
    if (!L->P || !L->tstart || !L->tend) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) project_one(s, i, &L->P[i]);
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const orc_proj *P = &L->P[i];
        if (!P->visible) continue;
        if (!tile_mask) {
            total += P->ntiles;
            continue;
        }
        for (int ty = P->ty0; ty < P->ty0 + P->nty; ++ty)
            for (int k = 0; k < P->ntx; ++k) {
                int tx = (P->tx0 + k) % L->tiles_x;
                if (tile_mask[(int64_t)ty * L->tiles_x + tx]) ++total;
            }
    }
    L->inst = (orc_inst *)malloc(sizeof(orc_inst) * (size_t)(total > 0 ? total : 1));
    if (!L->inst) return -1;
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        const orc_proj *P = &L->P[i];
        if (!P->visible) continue;
        for (int ty = P->ty0; ty < P->ty0 + P->nty; ++ty)
            for (int k = 0; k < P->ntx; ++k) {
                int tx = (P->tx0 + k) % L->tiles_x;
                int32_t tid = (int32_t)((int64_t)ty * L->tiles_x + tx);
                if (tile_mask && !tile_mask[tid]) continue;
                L->inst[w].tile = tid;
                L->inst[w].gid = (int32_t)i;
                L->inst[w].tr = P->depth;
                ++w;
            }
    }
    L->n_inst = w;
    qsort(L->inst, (size_t)w, sizeof(orc_inst), inst_cmp);
    for (int64_t k = 0; k < w; ++k) {
        int32_t t = L->inst[k].tile;
        if (k == 0 || L->inst[k - 1].tile != t) L->tstart[t] = k;
        if (k == w - 1 || L->inst[k + 1].tile != t) L->tend[t] = k + 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel front-to-back blending (Eq. 6-8, stop rule)                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t gid;
    double dx, dy, G, alpha_raw, alpha, T; /* T = transmittance before this instance */
} orc_contrib;

typedef struct {
    double C[3], T;
    double D;             /* depth image: sum of d_i alpha_i T_i */
    int32_t n_contrib;    /* 1 + list position of the last blended instance */
    int32_t n_flags;      /* near-threshold decisions met */
    int32_t n_grad_flags; /* also counts alpha_max-clamp kinks */
    int32_t n_blended;    /* instances blended (entries written to contrib) */
    uint64_t sig;         /* hash of the discrete decisions */
} orc_pixel;

static uint64_t fnv(uint64_t h, uint64_t v) {
    for (int k = 0; k < 8; ++k) {
        h ^= (v >> (8 * k)) & 0xffu;
        h *= 1099511628211ull;
    }
    return h;
}

/* shortest signed offset on the circle of circumference W, in [-W/2, W/2) */
static double wrap_dx(double d, double W) {
    while (d >= 0.5 * W) d -= W;
    while (d < -0.5 * W) d += W;
    return d;
}

/* alpha of one Gaussian at pixel (x, y) (Eq. 7, 8): the pixel offset (the
 * shortest one across the seam for the ERP image), G, and the alpha before
 * and after the alpha_max clamp */
typedef struct {
    double dx, dy, G, araw, alpha;
} orc_eval;

static void eval_at(const orc_scene *s, const orc_proj *P, double opac, int x, int y, orc_eval *e) {
    const double W = (double)s->width;
    e->dx = s->model == ORC_PINHOLE ? (x + 0.5) - P->px : wrap_dx((x + 0.5) - P->px, W);
    e->dy = (y + 0.5) - P->py;
    const double power = -0.5 * (P->Q[0] * e->dx * e->dx + 2.0 * P->Q[1] * e->dx * e->dy + P->Q[2] * e->dy * e->dy);
    e->G = exp(power);
    e->araw = opac * e->G;
    e->alpha = e->araw < s->alpha_max ? e->araw : s->alpha_max;
}

/* state of one pixel's front-to-back walk */
typedef struct {
    double T, C[3], D;
    int32_t last, nflag, ngflag, ncon, stopped;
    uint64_t sig;
    uint64_t flips; /* bit j set: the j-th flagged decision of the walk goes the other way */
} orc_walk;

/* the decision of the walk's next flagged decision: taken as computed, or
 * inverted when its bit of flips is set */
static int flagged(orc_walk *w, int decision) {
    const int inv = w->nflag < 64 && ((w->flips >> w->nflag) & 1u);
    ++w->nflag;
    ++w->ngflag;
    return inv ? !decision : decision;
}

/* one instance met at walk position pos (0-based in the tile list): skip
 * below alpha_min, stop before T would drop below T_min, else blend (Eq. 6) */
static void walk_one(const orc_scene *s, const orc_proj *P, int32_t gid, const orc_eval *e, int64_t pos,
                     orc_walk *w, orc_contrib *contrib) {
    int pass = e->alpha >= s->alpha_min;
    if (fabs(e->araw / s->alpha_min - 1.0) < s->flag_rel_alpha) pass = flagged(w, pass);
    if (!pass) return;
    if (fabs(e->araw / s->alpha_max - 1.0) < s->flag_rel_alpha) ++w->ngflag;
    const double Tn = w->T * (1.0 - e->alpha);
    int stop = Tn < s->T_min;
    if (fabs(Tn / s->T_min - 1.0) < s->flag_rel_T) stop = flagged(w, stop);
    if (stop) {
        w->sig = fnv(w->sig, 0xffffffffull);
        w->stopped = 1;
        return;
    }
    if (contrib) {
        orc_contrib *c = &contrib[w->ncon];
        c->gid = gid;
        c->dx = e->dx;
        c->dy = e->dy;
        c->G = e->G;
        c->alpha_raw = e->araw;
        c->alpha = e->alpha;
        c->T = w->T;
    }
    ++w->ncon;
    w->sig = fnv(w->sig, ((uint64_t)(uint32_t)gid << 1) | (uint64_t)(e->araw >= s->alpha_max));
    for (int ch = 0; ch < 3; ++ch) w->C[ch] += P->rgb[ch] * e->alpha * w->T;
    w->D += P->depth * e->alpha * w->T;
    w->T = Tn;
    w->last = (int32_t)(pos + 1);
}

/* flips: bit j inverts the j-th flagged decision met along the walk (0: the
 * FP64 decisions).  Flagged decisions: alpha within a relative margin of
 * alpha_min, T(1 - alpha) within one of T_min, and the order of two list
 * neighbours whose depths agree to within the float32 resolution of the
 * depth key when this pixel may blend either of them (inverted: the pair is
 * walked swapped; with one of them blended, only its position changes).  contrib (may be NULL) receives the blended instances in order. */
static void render_pixel(const orc_scene *s, const orc_lists *L, int64_t start, int64_t end, int x, int y,
                         uint64_t flips, orc_pixel *out, orc_contrib *contrib) {
    orc_walk w;
    memset(&w, 0, sizeof(w));
    w.T = 1.0;
    w.sig = 1469598103934665603ull;
    w.flips = flips;
    const double lo = s->alpha_min * (1.0 - s->flag_rel_alpha);
    for (int64_t k = start; k < end && !w.stopped;) {
        const orc_inst *I = &L->inst[k];
        const orc_proj *P = &L->P[I->gid];
        orc_eval e;
        eval_at(s, P, s->opac[I->gid], x, y, &e);
        if (k + 1 < end && fabs(L->inst[k + 1].tr / I->tr - 1.0) < s->flag_rel_depth) {
            const orc_inst *J = &L->inst[k + 1];
            const orc_proj *PJ = &L->P[J->gid];
            orc_eval f;
            eval_at(s, PJ, s->opac[J->gid], x, y, &f);
            /* the order matters when either may blend: with both, the
             * image; with one, its list position (the contributor count) */
            if ((e.araw >= lo || f.araw >= lo) && flagged(&w, 0)) {
                walk_one(s, PJ, J->gid, &f, k - start, &w, contrib);
                if (!w.stopped) walk_one(s, P, I->gid, &e, k + 1 - start, &w, contrib);
                k += 2;
                continue;
            }
        }
        walk_one(s, P, I->gid, &e, k - start, &w, contrib);
        ++k;
    }
    for (int ch = 0; ch < 3; ++ch) out->C[ch] = w.C[ch] + w.T * s->bg[ch];
    out->D = w.D;
    out->T = w.T;
    out->n_contrib = w.last;
    out->n_flags = w.nflag;
    out->n_grad_flags = w.ngflag;
    out->n_blended = w.ncon;
    out->sig = w.sig;
}

static int64_t tile_of_pixel(const orc_lists *L, int x, int y) {
    return (int64_t)(y / ORC_TILE) * L->tiles_x + (x / ORC_TILE);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

/* Per-Gaussian projection records for the pins.  Layout of each record (48
 * doubles): 0 visible, 1-3 t, 4 depth (t_r or t_z), 5 lon, 6 lat, 7 px, 8 py, 9-14 J,
 * 15-17 Sigma2D (a, b, c), 18-20 Q (00, 01, 11), 21 e_x, 22 e_y, 23 xs, 24 xe,
 * 25 ys, 26 ye, 27 full_x, 28 tx0, 29 ntx, 30 ty0, 31 nty, 32 ntiles,
 * 33-35 rgb, 36-38 clamp, 39 flag, 40-42 dir, 43 det, 44 t_r, 45-47 unused. */
#define ORC_REC 48
int orc_project(const orc_scene *s, double *rec) {
    if (!orc_valid(s)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->n; ++i) {
        orc_proj P;
        project_one(s, i, &P);
        double *r = rec + i * ORC_REC;
        memset(r, 0, sizeof(double) * ORC_REC);
        r[0] = P.visible;
        for (int k = 0; k < 3; ++k) r[1 + k] = P.tc[k];
        r[4] = P.depth;
        r[44] = P.tr;
        r[5] = P.lon;
        r[6] = P.lat;
        r[7] = P.px;
        r[8] = P.py;
        for (int k = 0; k < 6; ++k) r[9 + k] = P.J[k];
        r[15] = P.a;
        r[16] = P.b;
        r[17] = P.c;
        for (int k = 0; k < 3; ++k) r[18 + k] = P.Q[k];
        r[21] = P.ex;
        r[22] = P.ey;
        r[23] = (double)P.xs;
        r[24] = (double)P.xe;
        r[25] = (double)P.ys;
        r[26] = (double)P.ye;
        r[27] = P.full_x;
        r[28] = P.tx0;
        r[29] = P.ntx;
        r[30] = P.ty0;
        r[31] = P.nty;
        r[32] = (double)P.ntiles;
        for (int k = 0; k < 3; ++k) r[33 + k] = P.rgb[k];
        for (int k = 0; k < 3; ++k) r[36 + k] = P.clamp[k];
        r[39] = P.flag;
        for (int k = 0; k < 3; ++k) r[40 + k] = P.dir[k];
        r[43] = P.det;
    }
    return 0;
}

/* Sorted instance list of the tiles set in tile_mask (NULL: all tiles).
 * Returns M, or -1 on error; writes at most cap entries. */
int64_t orc_tile_lists(const orc_scene *s, const uint8_t *tile_mask, int64_t cap, int32_t *tile_out, int32_t *gid_out,
                       double *tr_out) {
    if (!orc_valid(s)) return -1;
    orc_lists L;
    if (build_lists(s, tile_mask, &L) != 0) {
        lists_free(&L);
        return -1;
    }
    int64_t M = L.n_inst;
    for (int64_t k = 0; k < M && k < cap; ++k) {
        tile_out[k] = L.inst[k].tile;
        gid_out[k] = L.inst[k].gid;
        tr_out[k] = L.inst[k].tr;
    }
    lists_free(&L);
    return M;
}

/* Forward render of the tiles set in tile_mask (NULL: all tiles; pixels of
 * other tiles are left untouched).  image [3][H][W], final_T [H][W], n_contrib [H][W],
 * n_flags [H][W] (flagged decisions met: see render_pixel and orc_branches);
 * n_grad_flags (may be NULL) also counts alpha_max-clamp near-ties, where
 * the gradient (not the value) changes; n_blended (may be NULL) counts the
 * instances blended into each pixel; depth (may be NULL) receives the depth
 * image. */
int orc_render(const orc_scene *s, const uint8_t *tile_mask, double *image, double *final_T, int32_t *n_contrib,
               int32_t *n_flags, int32_t *n_grad_flags, int32_t *n_blended, double *depth) {
    if (!orc_valid(s)) return -1;
    orc_lists L;
    if (build_lists(s, tile_mask, &L) != 0) {
        lists_free(&L);
        return -1;
    }
    const int Wd = s->width, Hd = orc_rows(s);
    const int64_t HW = (int64_t)Wd * Hd;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < HW; ++p) {
        const int x = (int)(p % Wd), y = (int)(p / Wd);
        const int64_t t = tile_of_pixel(&L, x, y);
        if (tile_mask && !tile_mask[t]) continue;
        orc_pixel px;
        render_pixel(s, &L, L.tstart[t], L.tend[t], x, y, 0, &px, NULL);
        for (int ch = 0; ch < 3; ++ch) image[ch * HW + p] = px.C[ch];
        final_T[p] = px.T;
        n_contrib[p] = px.n_contrib;
        n_flags[p] = px.n_flags;
        if (n_grad_flags) n_grad_flags[p] = px.n_grad_flags;
        if (n_blended) n_blended[p] = px.n_blended;
        if (depth) depth[p] = px.D;
    }
    lists_free(&L);
    return 0;
}

/* depth-first enumeration of the flip masks of one pixel: the walk with
 * mask m meets some number f of flagged decisions; each of those past the
 * highest bit of m may also go the other way */
typedef struct {
    const orc_scene *s;
    const orc_lists *L;
    int64_t start, end;
    int x, y;
    int32_t max_b, count;
    double *image, *T;
    int32_t *n_contrib, *n_blended;
} orc_branch_ctx;

static void explore(orc_branch_ctx *c, uint64_t mask, int hb) {
    if (c->count > c->max_b) return;
    orc_pixel px;
    render_pixel(c->s, c->L, c->start, c->end, c->x, c->y, mask, &px, NULL);
    if (c->count == c->max_b) {
        c->count = c->max_b + 1; /* more branches than room: the caller excludes the pixel */
        return;
    }
    const int b = c->count++;
    for (int ch = 0; ch < 3; ++ch) c->image[3 * b + ch] = px.C[ch];
    c->T[b] = px.T;
    c->n_contrib[b] = px.n_contrib;
    c->n_blended[b] = px.n_blended;
    for (int j = hb + 1; j < px.n_flags && j < 64; ++j) explore(c, mask | (1ull << j), j);
}

/* Every result a pixel may take when its flagged decisions (alpha vs
 * alpha_min, T vs T_min, the order of two near-tied depths) go either way,
 * for the npix pixels pix[] (flat indices y * W + x of the rendered image;
 * only their tiles need be set in tile_mask, NULL: all).  Per pixel, up to
 * max_b branches: image [npix][max_b][3], final_T, n_contrib and n_blended
 * [npix][max_b]; count[k] receives the number of branches (the first is the
 * FP64 walk), or -1 when the pixel has more than max_b. */
int orc_branches(const orc_scene *s, const uint8_t *tile_mask, int64_t npix, const int64_t *pix, int32_t max_b,
                 int32_t *count, double *image, double *final_T, int32_t *n_contrib, int32_t *n_blended) {
    if (!orc_valid(s) || max_b < 1) return -1;
    orc_lists L;
    if (build_lists(s, tile_mask, &L) != 0) {
        lists_free(&L);
        return -1;
    }
    const int Wd = s->width, Hd = orc_rows(s);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t k = 0; k < npix; ++k) {
        const int x = (int)(pix[k] % Wd), y = (int)(pix[k] / Wd);
        if (pix[k] < 0 || y >= Hd) {
            bad = 1;
            continue;
        }
        const int64_t t = tile_of_pixel(&L, x, y);
        if (tile_mask && !tile_mask[t]) {
            bad = 1;
            continue;
        }
        orc_branch_ctx c = {s, &L, L.tstart[t], L.tend[t], x, y, max_b, 0, image + k * max_b * 3,
                            final_T + k * max_b, n_contrib + k * max_b, n_blended + k * max_b};
        explore(&c, 0ull, -1);
        count[k] = c.count > max_b ? -1 : c.count;
    }
    lists_free(&L);
    return bad ? -1 : 0;
}

/* L1 loss sum over the pixels of the masked tiles: sum w |C - target| / (3HW)
 * (w = weight[H][W], or 1 when weight is NULL),
 * plus a hash of every discrete decision taken there (for finite-difference
 * validity checks). */
int orc_l1_tiles(const orc_scene *s, const double *target, const double *weight, const uint8_t *tile_mask,
                 double *loss, uint64_t *signature) {
    if (!orc_valid(s)) return -1;
    orc_lists L;
    if (build_lists(s, tile_mask, &L) != 0) {
        lists_free(&L);
        return -1;
    }
    const int Wd = s->width, Hd = orc_rows(s);
    const int64_t HW = (int64_t)Wd * Hd;
    double total = 0.0;
    uint64_t sig = 1469598103934665603ull;
    for (int64_t t = 0; t < (int64_t)L.tiles_x * L.tiles_y; ++t) {
        if (!tile_mask[t]) continue;
        const int tx = (int)(t % L.tiles_x), ty = (int)(t / L.tiles_x);
        for (int y = ty * ORC_TILE; y < ty * ORC_TILE + ORC_TILE && y < Hd; ++y)
            for (int x = tx * ORC_TILE; x < tx * ORC_TILE + ORC_TILE && x < Wd; ++x) {
                orc_pixel px;
                render_pixel(s, &L, L.tstart[t], L.tend[t], x, y, 0, &px, NULL);
                const int64_t p = (int64_t)y * Wd + x;
                sig = fnv(sig, px.sig);
                for (int ch = 0; ch < 3; ++ch) {
                    const double r = px.C[ch] - target[ch * HW + p];
                    total += (weight ? weight[p] : 1.0) * fabs(r);
                    sig = fnv(sig, (uint64_t)(r > 0.0 ? 1 : (r < 0.0 ? 2 : 0)));
                }
            }
    }
    *loss = total / (3.0 * (double)HW);
    *signature = sig;
    lists_free(&L);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward (Eq. 18-20)                                                       */
/* ------------------------------------------------------------------------ */
/* per-Gaussian accumulator layout: dL/dp (2), dL/dQ (00, 01, 11), dL/do,
 * dL/drgb (3), dL/dd (the depth value of the depth image) */
#define ORC_NACC 10

/* dJ_{a,j}/dt_n for the pinhole Jacobian J00 = fx / tz, J02 = -fx a / tz,
 * J11 = fy / tz, J12 = -fy b / tz with a = t_x / t_z, b = t_y / t_z, each
 * clamped: a clamped direction is constant in t */
static void jacobian_dt_pinhole(const orc_proj *P, double fx, double fy, double dJ[6][3]) {
    const double tz = P->tc[2], tz2 = tz * tz;
    for (int e = 0; e < 6; ++e) dJ[e][0] = dJ[e][1] = dJ[e][2] = 0.0;
    dJ[0][2] = -fx / tz2;
    dJ[4][2] = -fy / tz2;
    /* J02: d/dt_x (-fx t_x / t_z^2) = -fx / t_z^2, d/dt_z = 2 fx t_x / t_z^3;
     * clamped: d/dt_z (-fx a / t_z) = fx a / t_z^2 */
    if (P->clamped[0]) {
        dJ[2][2] = fx * P->dir_c[0] / tz2;
    } else {
        dJ[2][0] = -fx / tz2;
        dJ[2][2] = 2.0 * fx * P->tc[0] / (tz2 * tz);
    }
    if (P->clamped[1]) {
        dJ[5][2] = fy * P->dir_c[1] / tz2;
    } else {
        dJ[5][1] = -fy / tz2;
        dJ[5][2] = 2.0 * fy * P->tc[1] / (tz2 * tz);
    }
}

/* dJ_{a,j}/dt_n for the spherical Jacobian (derivatives of Eq. 11-16) */
static void jacobian_dt(const double t[3], double W, double H, double dJ[6][3]) {
    const double tx = t[0], ty = t[1], tz = t[2];
    const double rho2 = tx * tx + tz * tz, rho = sqrt(rho2), r2 = rho2 + ty * ty;
    const double kx = W / (2.0 * M_PI), ky = H / M_PI;
    const double rho4 = rho2 * rho2, r4 = r2 * r2, rho3 = rho2 * rho;
    /* J00 = kx tz / rho^2 */
    dJ[0][0] = -2.0 * kx * tx * tz / rho4;
    dJ[0][1] = 0.0;
    dJ[0][2] = kx * (rho2 - 2.0 * tz * tz) / rho4;
    /* J01 = 0 */
    dJ[1][0] = dJ[1][1] = dJ[1][2] = 0.0;
    /* J02 = -kx tx / rho^2 */
    dJ[2][0] = -kx * (rho2 - 2.0 * tx * tx) / rho4;
    dJ[2][1] = 0.0;
    dJ[2][2] = 2.0 * kx * tx * tz / rho4;
    /* J10 = -ky tx ty / (r^2 rho) = -ky u, u = tx ty r^-2 rho^-1 */
    dJ[3][0] = -ky * (ty / (r2 * rho) - tx * ty * 2.0 * tx / (r4 * rho) - tx * ty * tx / (r2 * rho3));
    dJ[3][1] = -ky * (tx / (r2 * rho) - tx * ty * 2.0 * ty / (r4 * rho));
    dJ[3][2] = -ky * (-tx * ty * 2.0 * tz / (r4 * rho) - tx * ty * tz / (r2 * rho3));
    /* J11 = ky rho / r^2 */
    dJ[4][0] = ky * (tx / (rho * r2) - rho * 2.0 * tx / r4);
    dJ[4][1] = ky * (-rho * 2.0 * ty / r4);
    dJ[4][2] = ky * (tz / (rho * r2) - rho * 2.0 * tz / r4);
    /* J12 = -ky tz ty / (r^2 rho) */
    dJ[5][0] = -ky * (-tz * ty * 2.0 * tx / (r4 * rho) - tz * ty * tx / (r2 * rho3));
    dJ[5][1] = -ky * (tz / (r2 * rho) - tz * ty * 2.0 * ty / (r4 * rho));
    dJ[5][2] = -ky * (ty / (r2 * rho) - tz * ty * 2.0 * tz / (r4 * rho) - tz * ty * tz / (r2 * rho3));
}

/* The per-Gaussian chain from the screen-space accumulators to the
 * parameter gradients.  It is linear in acc.  Outputs (all overwritten):
 * dm[3], dS[3], dq[4], do_[1], dsh[K*3], dscreen[2]. */
static void chain_one(const orc_scene *s, int64_t i, const orc_proj *P, const double acc[ORC_NACC], double dm[3],
                      double dS[3], double dq[4], double *do_, double *dsh, double dscreen[2]) {
    const double W = (double)s->width, H = (double)s->height;
    const double *gp = acc, *gQ = acc + 2;
    /* Q = adj(Sigma2D) / det: dL/d(a, b, c) */
    const double det = P->det, det2 = det * det;
    double gabc[3];
    for (int v = 0; v < 3; ++v) {
        const double ddet = (v == 0) ? P->c : (v == 1 ? -2.0 * P->b : P->a);
        const double dQ00 = (v == 2 ? 1.0 / det : 0.0) - P->c * ddet / det2;
        const double dQ01 = (v == 1 ? -1.0 / det : 0.0) + P->b * ddet / det2;
        const double dQ11 = (v == 0 ? 1.0 / det : 0.0) - P->a * ddet / det2;
        gabc[v] = gQ[0] * dQ00 + gQ[1] * dQ01 + gQ[2] * dQ11;
    }
    const double ga = gabc[0], gb = gabc[1], gc = gabc[2];
    const double *M0 = P->M, *M1 = P->M + 3;
    /* dL/dSigma (all nine entries as independent intermediates) */
    double gSig[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            gSig[3 * a + b] = ga * M0[a] * M0[b] + gb * M0[a] * M1[b] + gc * M1[a] * M1[b];
    /* dL/dM */
    double SM0[3], SM1[3], SM0t[3];
    for (int k = 0; k < 3; ++k) {
        SM0[k] = SM1[k] = SM0t[k] = 0.0;
        for (int j = 0; j < 3; ++j) {
            SM0[k] += P->Sig[3 * k + j] * M0[j];
            SM1[k] += P->Sig[3 * k + j] * M1[j];
            SM0t[k] += P->Sig[3 * j + k] * M0[j];
        }
    }
    double gM[6];
    for (int k = 0; k < 3; ++k) {
        /* a = M0 Sig M0^T, b = M0 Sig M1^T, c = M1 Sig M1^T */
        double SM1t = 0.0;
        for (int j = 0; j < 3; ++j) SM1t += P->Sig[3 * j + k] * M1[j];
        gM[k] = ga * (SM0[k] + SM0t[k]) + gb * SM1[k];
        gM[3 + k] = gb * SM0t[k] + gc * (SM1[k] + SM1t);
    }
    /* M = J W  ->  dL/dJ_{a,i} = sum_k dL/dM_{a,k} W_{i,k} */
    double gJ[6];
    for (int a = 0; a < 2; ++a)
        for (int ii = 0; ii < 3; ++ii) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += gM[3 * a + k] * s->R[3 * ii + k];
            gJ[3 * a + ii] = v;
        }
    /* dL/dt: through p (dp/dt), through J(t) and through the depth d of the
     * depth image (d = t_r: dd/dt = t / t_r; d = t_z: dd/dt = (0, 0, 1)) */
    double dJdt[6][3];
    if (s->model == ORC_PINHOLE)
        jacobian_dt_pinhole(P, s->fx, s->fy, dJdt);
    else
        jacobian_dt(P->tc, W, H, dJdt);
    double gt[3];
    for (int nn = 0; nn < 3; ++nn) {
        double v = gp[0] * P->Jp[nn] + gp[1] * P->Jp[3 + nn];
        for (int e = 0; e < 6; ++e) v += gJ[e] * dJdt[e][nn];
        if (s->model == ORC_PINHOLE)
            v += nn == 2 ? acc[9] : 0.0;
        else
            v += acc[9] * P->tc[nn] / P->tr;
        gt[nn] = v;
    }
    /* t = W m + t_cw */
    for (int k = 0; k < 3; ++k) dm[k] = s->R[0 * 3 + k] * gt[0] + s->R[1 * 3 + k] * gt[1] + s->R[2 * 3 + k] * gt[2];
    /* Sigma = Rq diag(S^2) Rq^T */
    const double *S = s->scales + 3 * i;
    const double *Rq = P->Rq;
    for (int k = 0; k < 3; ++k) {
        double v = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) v += gSig[3 * a + b] * 2.0 * S[k] * Rq[3 * a + k] * Rq[3 * b + k];
        dS[k] = v;
    }
    double gR[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int j = 0; j < 3; ++j) v += (gSig[3 * a + j] + gSig[3 * j + a]) * S[b] * S[b] * Rq[3 * j + b];
            gR[3 * a + b] = v;
        }
    /* rotation matrix entries as functions of the unit quaternion */
    const double w = P->qn[0], x = P->qn[1], y = P->qn[2], z = P->qn[3];
    const double dR[9][4] = {
        {0, 0, -4 * y, -4 * z},      {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
        {2 * z, 2 * y, 2 * x, 2 * w}, {0, -4 * x, 0, -4 * z},        {-2 * x, -2 * w, 2 * z, 2 * y},
        {-2 * y, 2 * z, -2 * w, 2 * x}, {2 * x, 2 * w, 2 * z, 2 * y}, {0, -4 * x, -4 * y, 0},
    };
    double gqn[4] = {0, 0, 0, 0};
    for (int e = 0; e < 9; ++e)
        for (int k = 0; k < 4; ++k) gqn[k] += gR[e] * dR[e][k];
    double dotq = 0.0;
    for (int k = 0; k < 4; ++k) dotq += P->qn[k] * gqn[k];
    for (int k = 0; k < 4; ++k) dq[k] = (gqn[k] - P->qn[k] * dotq) / P->qnorm;
    /* opacity */
    *do_ = acc[5];
    /* SH colour: d rgb / d sh and d rgb / d dir */
    dual Y[ORC_MAXK];
    sh_basis_dual(s->sh_degree, P->dir, Y);
    const int K = (s->sh_degree + 1) * (s->sh_degree + 1);
    const double *shi = s->sh + i * s->sh_coeffs * 3;
    double gdir[3] = {0, 0, 0};
    for (int k = 0; k < s->sh_coeffs * 3; ++k) dsh[k] = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        const double grgb = P->clamp[ch] ? 0.0 : acc[6 + ch];
        for (int k = 0; k < K; ++k) {
            dsh[3 * k + ch] = Y[k].v * grgb;
            for (int d = 0; d < 3; ++d) gdir[d] += grgb * shi[3 * k + ch] * Y[k].d[d];
        }
    }
    /* dir = v / |v|, v = m - camera centre, |v| = t_r */
    double ddot = P->dir[0] * gdir[0] + P->dir[1] * gdir[1] + P->dir[2] * gdir[2];
    for (int d = 0; d < 3; ++d) dm[d] += (gdir[d] - P->dir[d] * ddot) / P->tr;
    /* screen-space gradient: p = (s + 1) (W/2, H/2) */
    dscreen[0] = gp[0] * W / 2.0;
    dscreen[1] = gp[1] * H / 2.0;
}

/* Backward of image = render(params) for a given dL/dimage [3][H][W] and,
 * each may be NULL, dL/ddepth [H][W] and dL/dalpha [H][W] (alpha = 1 - T_final),
 * restricted to the tiles set in tile_mask (NULL: all); exact when dL/dimage
 * vanishes outside them.
 * Gradient outputs are overwritten: dmeans [n][3], dscales [n][3],
 * dquats [n][4], dopac [n], dsh [n][sh_coeffs][3], dscreen [n][2].
 * acc_out (may be NULL): [n][10] screen-space accumulators.
 * abs_* (may all be NULL): sums of |per-pixel contributions| propagated
 * through |chain|: the scale against which float32 sums are judged. */
int orc_backward(const orc_scene *s, const uint8_t *tile_mask, const double *dLdC, const double *dLdD,
                 const double *dLdA, double *dmeans, double *dscales,
                 double *dquats, double *dopac, double *dsh, double *dscreen, double *acc_out, double *abs_means,
                 double *abs_scales, double *abs_quats, double *abs_opac, double *abs_sh, double *abs_screen) {
    if (!orc_valid(s)) return -1;
    orc_lists L;
    if (build_lists(s, tile_mask, &L) != 0) {
        lists_free(&L);
        return -1;
    }
    const int64_t n = s->n;
    const int Wd = s->width, Hd = orc_rows(s);
    const int64_t HW = (int64_t)Wd * Hd;
    const int64_t ntiles = (int64_t)L.tiles_x * L.tiles_y;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)(n * ORC_NACC * 2 * nthreads + 1), sizeof(double));
    int64_t maxlen = 1;
    for (int64_t t = 0; t < ntiles; ++t)
        if (L.tend[t] - L.tstart[t] > maxlen) maxlen = L.tend[t] - L.tstart[t];
    if (!acc) {
        lists_free(&L);
        return -1;
    }
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *A = acc + (int64_t)tid * n * ORC_NACC * 2; /* [n][10] signed then [n][10] abs */
        double *Aabs = A + n * ORC_NACC;
        orc_contrib *con = (orc_contrib *)malloc(sizeof(orc_contrib) * (size_t)maxlen);
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < ntiles; ++t) {
            if (tile_mask && !tile_mask[t]) continue;
            const int tx = (int)(t % L.tiles_x), ty = (int)(t / L.tiles_x);
            for (int y = ty * ORC_TILE; y < ty * ORC_TILE + ORC_TILE && y < Hd; ++y)
                for (int x = tx * ORC_TILE; x < tx * ORC_TILE + ORC_TILE && x < Wd; ++x) {
                    const int64_t p = (int64_t)y * Wd + x;
                    orc_pixel px;
                    render_pixel(s, &L, L.tstart[t], L.tend[t], x, y, 0, &px, con);
                    const int ncon = px.n_blended;
                    const double g[3] = {dLdC[p], dLdC[HW + p], dLdC[2 * HW + p]};
                    const double gD = dLdD ? dLdD[p] : 0.0, gA = dLdA ? dLdA[p] : 0.0;
                    /* S = colour blended behind the current instance, plus
                     * the background seen through the final transmittance */
                    double Sb[3], SD = 0.0, SA = 0.0; /* depth and alpha: zero background */
                    for (int ch = 0; ch < 3; ++ch) Sb[ch] = px.T * s->bg[ch];
                    for (int j = ncon - 1; j >= 0; --j) {
                        const orc_contrib *c = &con[j];
                        const orc_proj *P = &L.P[c->gid];
                        double *a = A + (int64_t)c->gid * ORC_NACC;
                        double *aa = Aabs + (int64_t)c->gid * ORC_NACC;
                        double dalpha = 0.0;
                        for (int ch = 0; ch < 3; ++ch) {
                            const double term = g[ch] * c->alpha * c->T;
                            a[6 + ch] += term;
                            aa[6 + ch] += fabs(term);
                            dalpha += g[ch] * (P->rgb[ch] * c->T - Sb[ch] / (1.0 - c->alpha));
                        }
                        for (int ch = 0; ch < 3; ++ch) Sb[ch] += P->rgb[ch] * c->alpha * c->T;
                        /* depth and alpha channels: colour d_i and 1 */
                        const double tD = gD * c->alpha * c->T;
                        a[9] += tD;
                        aa[9] += fabs(tD);
                        dalpha += gD * (P->depth * c->T - SD / (1.0 - c->alpha));
                        dalpha += gA * (c->T - SA / (1.0 - c->alpha));
                        SD += P->depth * c->alpha * c->T;
                        SA += c->alpha * c->T;
                        if (c->alpha_raw >= s->alpha_max) continue; /* clamped: no gradient */
                        const double o = s->opac[c->gid];
                        const double gO = c->G * dalpha;
                        const double gpow = o * c->G * dalpha; /* dalpha/dpower = alpha_raw */
                        const double t0 = -0.5 * c->dx * c->dx * gpow, t1 = -c->dx * c->dy * gpow,
                                     t2 = -0.5 * c->dy * c->dy * gpow;
                        /* power depends on p through dx = x + 1/2 - p_x */
                        const double tpx = (P->Q[0] * c->dx + P->Q[1] * c->dy) * gpow;
                        const double tpy = (P->Q[1] * c->dx + P->Q[2] * c->dy) * gpow;
                        a[0] += tpx; aa[0] += fabs(tpx);
                        a[1] += tpy; aa[1] += fabs(tpy);
                        a[2] += t0;  aa[2] += fabs(t0);
                        a[3] += t1;  aa[3] += fabs(t1);
                        a[4] += t2;  aa[4] += fabs(t2);
                        a[5] += gO;  aa[5] += fabs(gO);
                    }
                }
        }
        free(con);
    }
    /* reduce thread-local accumulators in fixed order */
    for (int th = 1; th < nthreads; ++th) {
        const double *src = acc + (int64_t)th * n * ORC_NACC * 2;
        for (int64_t k = 0; k < n * ORC_NACC * 2; ++k) acc[k] += src[k];
    }
    const int K = s->sh_coeffs;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const orc_proj *P = &L.P[i];
        double *gm = dmeans + 3 * i, *gs = dscales + 3 * i, *gq = dquats + 4 * i, *gsh = dsh + i * K * 3,
               *gscr = dscreen + 2 * i;
        const double *a = acc + i * ORC_NACC;
        const double *aa = acc + n * ORC_NACC + i * ORC_NACC;
        if (acc_out)
            for (int k = 0; k < ORC_NACC; ++k) acc_out[i * ORC_NACC + k] = a[k];
        if (!P->visible) {
            memset(gm, 0, 3 * sizeof(double));
            memset(gs, 0, 3 * sizeof(double));
            memset(gq, 0, 4 * sizeof(double));
            dopac[i] = 0.0;
            memset(gsh, 0, (size_t)K * 3 * sizeof(double));
            gscr[0] = gscr[1] = 0.0;
            if (abs_means) {
                memset(abs_means + 3 * i, 0, 3 * sizeof(double));
                memset(abs_scales + 3 * i, 0, 3 * sizeof(double));
                memset(abs_quats + 4 * i, 0, 4 * sizeof(double));
                abs_opac[i] = 0.0;
                memset(abs_sh + i * K * 3, 0, (size_t)K * 3 * sizeof(double));
                abs_screen[2 * i] = abs_screen[2 * i + 1] = 0.0;
            }
            continue;
        }
        chain_one(s, i, P, a, gm, gs, gq, &dopac[i], gsh, gscr);
        if (abs_means) {
            /* |chain| applied to the |contribution| sums, one accumulator
             * column at a time (the chain is linear in acc) */
            double *bm = abs_means + 3 * i, *bs = abs_scales + 3 * i, *bq = abs_quats + 4 * i, *bo = abs_opac + i,
                   *bsh = abs_sh + i * K * 3, *bscr = abs_screen + 2 * i;
            memset(bm, 0, 3 * sizeof(double));
            memset(bs, 0, 3 * sizeof(double));
            memset(bq, 0, 4 * sizeof(double));
            *bo = 0.0;
            memset(bsh, 0, (size_t)K * 3 * sizeof(double));
            bscr[0] = bscr[1] = 0.0;
            double *csh = (double *)malloc(sizeof(double) * (size_t)K * 3);
            for (int col = 0; col < ORC_NACC; ++col) {
                if (aa[col] == 0.0) continue;
                double e[ORC_NACC] = {0};
                e[col] = 1.0;
                double cm[3], cs[3], cq[4], co, cscr[2];
                chain_one(s, i, P, e, cm, cs, cq, &co, csh, cscr);
                for (int k = 0; k < 3; ++k) bm[k] += fabs(cm[k]) * aa[col];
                for (int k = 0; k < 3; ++k) bs[k] += fabs(cs[k]) * aa[col];
                for (int k = 0; k < 4; ++k) bq[k] += fabs(cq[k]) * aa[col];
                *bo += fabs(co) * aa[col];
                for (int k = 0; k < K * 3; ++k) bsh[k] += fabs(csh[k]) * aa[col];
                for (int k = 0; k < 2; ++k) bscr[k] += fabs(cscr[k]) * aa[col];
            }
            free(csh);
        }
    }
    free(acc);
    lists_free(&L);
    return 0;
}

/* L1 photometric term of Eq. 17 (lambda = 0): mean |C - C_gt| over 3HW and
 * its gradient sign(C - C_gt) / (3HW), sign(0) = 0. */
double orc_l1(int64_t count, const double *image, const double *target, double *grad) {
    double total = 0.0;
    for (int64_t k = 0; k < count; ++k) {
        const double r = image[k] - target[k];
        total += fabs(r);
        if (grad) grad[k] = (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0)) / (double)count;
    }
    return total / (double)count;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by later calls (n >= 1); used to time the oracle on one
 * core beside all of them. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
