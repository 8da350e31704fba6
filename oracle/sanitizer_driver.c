/*
 * sanitizer_driver.c -- TEST INFRASTRUCTURE: drives every entry point of the
 * FP64 oracle (omnigs_oracle.c, included whole) on small seeded scenes, so
 * that a build with AddressSanitizer and UndefinedBehaviorSanitizer checks
 * the oracle's memory accesses and arithmetic: an ERP scene with seam
 * straddlers, near-pole and culled Gaussians, exact depth ties and alpha
 * near-ties; a ragged pinhole image; a row crop.  Exit status 0 when every
 * call succeeds (the sanitizers abort on the first error).
 */
#include <stdio.h>

#include "omnigs_oracle.c"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* splitmix64 -> [0, 1) */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int run_scene(orc_scene *s) {
    const int64_t n = s->n;
    const int W = s->width, H = orc_rows(s);
    const int64_t HW = (int64_t)W * H;
    const int tiles = orc_tiles_x(s) * ((H + ORC_TILE - 1) / ORC_TILE);
    double *rec = calloc((size_t)(n * ORC_REC + 1), sizeof(double));
    if (orc_project(s, rec) != 0) return 1;
    int64_t M = orc_tile_lists(s, NULL, 0, NULL, NULL, NULL);
    if (M < 0) return 2;
    int32_t *tl = malloc(sizeof(int32_t) * (size_t)(M + 1)), *gl = malloc(sizeof(int32_t) * (size_t)(M + 1));
    double *trl = malloc(sizeof(double) * (size_t)(M + 1));
    if (orc_tile_lists(s, NULL, M, tl, gl, trl) != M) return 3;
    double *img = calloc((size_t)(3 * HW), sizeof(double)), *T = calloc((size_t)HW, sizeof(double));
    double *D = calloc((size_t)HW, sizeof(double));
    int32_t *nc = calloc((size_t)HW, sizeof(int32_t)), *nf = calloc((size_t)HW, sizeof(int32_t));
    int32_t *ngf = calloc((size_t)HW, sizeof(int32_t)), *nb = calloc((size_t)HW, sizeof(int32_t));
    if (orc_render(s, NULL, img, T, nc, nf, ngf, nb, D) != 0) return 4;
    /* a masked render of every other tile */
    uint8_t *mask = calloc((size_t)tiles, 1);
    for (int t = 0; t < tiles; t += 2) mask[t] = 1;
    if (orc_render(s, mask, img, T, nc, nf, ngf, nb, NULL) != 0) return 5;
    /* branches of every flagged pixel and of a few others */
    int64_t np = 0;
    int64_t *pix = malloc(sizeof(int64_t) * (size_t)(HW + 1));
    for (int64_t p = 0; p < HW; ++p)
        if (nf[p] > 0 || p % 97 == 0) pix[np++] = p;
    const int B = 16;
    int32_t *cnt = calloc((size_t)(np + 1), sizeof(int32_t));
    double *bimg = calloc((size_t)((np + 1) * B * 3), sizeof(double)), *bT = calloc((size_t)((np + 1) * B), sizeof(double));
    int32_t *bnc = calloc((size_t)((np + 1) * B), sizeof(int32_t)), *bnb = calloc((size_t)((np + 1) * B), sizeof(int32_t));
    if (np && orc_branches(s, NULL, np, pix, B, cnt, bimg, bT, bnc, bnb) != 0) return 6;
    /* backward with every cotangent and the abs sums */
    double *dC = malloc(sizeof(double) * (size_t)(3 * HW)), *dD = malloc(sizeof(double) * (size_t)HW);
    double *dA = malloc(sizeof(double) * (size_t)HW);
    for (int64_t k = 0; k < 3 * HW; ++k) dC[k] = urand() - 0.5;
    for (int64_t k = 0; k < HW; ++k) {
        dD[k] = urand() - 0.5;
        dA[k] = urand() - 0.5;
    }
    const int K = s->sh_coeffs;
    double *g[12];
    const size_t sz[6] = {3, 3, 4, 1, (size_t)K * 3, 2};
    for (int k = 0; k < 12; ++k) g[k] = calloc((size_t)n * sz[k % 6] + 1, sizeof(double));
    double *acc = calloc((size_t)(n * ORC_NACC + 1), sizeof(double));
    if (orc_backward(s, NULL, dC, dD, dA, g[0], g[1], g[2], g[3], g[4], g[5], acc, g[6], g[7], g[8], g[9], g[10],
                     g[11]) != 0)
        return 7;
    if (orc_backward(s, mask, dC, NULL, NULL, g[0], g[1], g[2], g[3], g[4], g[5], NULL, NULL, NULL, NULL, NULL, NULL,
                     NULL) != 0)
        return 8;
    double loss;
    uint64_t sig;
    if (orc_l1_tiles(s, img, NULL, mask, &loss, &sig) != 0) return 9;
    if (orc_l1_tiles(s, img, T, mask, &loss, &sig) != 0) return 10;
    (void)orc_l1(3 * HW, img, dC, dC);
    for (int k = 0; k < 12; ++k) free(g[k]);
    free(acc); free(dC); free(dD); free(dA); free(cnt); free(bimg); free(bT); free(bnc); free(bnb); free(pix);
    free(mask); free(img); free(T); free(D); free(nc); free(nf); free(ngf); free(nb); free(tl); free(gl); free(trl);
    free(rec);
    return 0;
}

int main(void) {
    const int64_t n = 400;
    double *m = malloc(sizeof(double) * n * 3), *sc = malloc(sizeof(double) * n * 3), *q = malloc(sizeof(double) * n * 4);
    double *o = malloc(sizeof(double) * n), *sh = malloc(sizeof(double) * n * 48);
    for (int64_t i = 0; i < n; ++i) {
        const double r = 1.0 + 6.0 * urand(), lon = (urand() * 2.0 - 1.0) * M_PI, lat = (urand() - 0.5) * M_PI;
        m[3 * i] = r * cos(lat) * sin(lon);
        m[3 * i + 1] = r * sin(lat);
        m[3 * i + 2] = r * cos(lat) * cos(lon);
        for (int k = 0; k < 3; ++k) sc[3 * i + k] = exp(log(0.005) + urand() * log(80.0));
        for (int k = 0; k < 4; ++k) q[4 * i + k] = urand() - 0.5;
        o[i] = 0.02 + 0.97 * urand();
        for (int k = 0; k < 48; ++k) sh[48 * i + k] = (k < 3 ? 0.5 : 0.0) + 0.2 * (urand() - 0.5);
    }
    /* seam straddlers, a near-pole Gaussian, culled ones, an exact depth tie,
       an alpha near-tie (opacity at alpha_min just above) */
    m[0] = 0.0; m[1] = 0.0; m[2] = -3.0;          /* on the seam behind the camera */
    m[3] = 0.001; m[4] = 4.0; m[5] = 0.0;         /* near the pole */
    m[6] = 0.05; m[7] = 0.0; m[8] = 0.05;         /* inside the near sphere */
    o[3] = 1.0 / 300.0;                           /* below alpha_min */
    for (int k = 0; k < 3; ++k) m[3 * 5 + k] = m[3 * 4 + k];
    o[6] = (1.0 / 255.0) * (1.0 + 1e-7);
    orc_scene s;
    memset(&s, 0, sizeof(s));
    s.n = n;
    s.means = m; s.scales = sc; s.quats = q; s.opac = o; s.sh = sh;
    s.sh_degree = 3; s.sh_coeffs = 16;
    s.width = 64; s.height = 32;
    s.R[0] = s.R[4] = s.R[8] = 1.0;
    s.t[0] = 0.1; s.t[1] = -0.05; s.t[2] = 0.02;
    s.alpha_min = 1.0 / 255.0; s.alpha_max = 0.99; s.T_min = 1e-4; s.dilation = 0.3; s.near_plane = 0.2;
    s.bg[0] = 0.1; s.bg[1] = 0.2; s.bg[2] = 0.3;
    s.flag_rel_alpha = 1e-5; s.flag_rel_T = 1e-4; s.flag_rel_depth = 0x1p-22; s.flag_abs_rect = 1e-6;
    int rc = run_scene(&s);
    if (rc) { fprintf(stderr, "ERP scene: step %d failed\n", rc); return rc; }
    /* screen shifts (the finite-difference handle) */
    double *shift = calloc((size_t)(2 * n), sizeof(double));
    shift[2 * 7] = 0.25;
    s.screen_shift = shift;
    rc = run_scene(&s);
    if (rc) { fprintf(stderr, "shifted scene: step %d failed\n", rc); return rc; }
    s.screen_shift = NULL;
    /* a row crop */
    s.rows = 20;
    rc = run_scene(&s);
    if (rc) { fprintf(stderr, "row crop: step %d failed\n", rc); return rc; }
    /* a ragged pinhole image, degree 1 with 4 stored coefficients */
    s.rows = 0;
    s.model = ORC_PINHOLE;
    s.width = 50; s.height = 40;
    s.fx = 40.0; s.fy = 42.0; s.cx = 24.5; s.cy = 21.0;
    s.sh_degree = 1;
    rc = run_scene(&s);
    if (rc) { fprintf(stderr, "pinhole scene: step %d failed\n", rc); return rc; }
    double Y[16], dY[48], dir[3] = {0.3, -0.4, 0.866};
    orc_sh_eval(3, dir, Y, dY);
    free(shift); free(m); free(sc); free(q); free(o); free(sh);
    printf("sanitized oracle run ok\n");
    return 0;
}
