/* Sanitizer driver for the FP64 oracle (test infrastructure): compiled together with
 * oracle/tsr_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers_cpu.py, it runs every entry point of the oracle on a small seeded
 * scene -- the global, per-face exponent, perspective-correct and tight-binning variants, an
 * indexed mesh, pixel subsets and the argument errors -- and exits non-zero on any unexpected
 * return code.  The sanitizers abort the run on the first memory or undefined-behaviour error. */
#include "../../oracle/tsr_oracle.c"

#include <stdio.h>

static uint64_t lcg = 12345u;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) / 9007199254740992.0;
}

#define CHECK(expr, want)                                                       \
    do {                                                                        \
        int rc_ = (expr);                                                       \
        if (rc_ != (want)) {                                                    \
            fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, #expr, rc_, (want)); \
            return 1;                                                           \
        }                                                                       \
    } while (0)

int main(void) {
    enum { M = 40, N = 3 * M, W = 48, H = 36 };
    static double pos[3 * N], col[3 * N], opa[N], fsig[M];
    for (int m = 0; m < M; m++) {
        double cx = urand() * 1.6 - 0.8, cy = urand() * 1.2 - 0.6, z = 1.0 + 2.0 * urand();
        for (int k = 0; k < 3; k++) {
            int i = 3 * m + k;
            pos[i] = (cx + 0.25 * (urand() - 0.5)) * z;
            pos[N + i] = (cy + 0.25 * (urand() - 0.5)) * z;
            pos[2 * N + i] = z + 0.2 * (urand() - 0.5);
            for (int ch = 0; ch < 3; ch++) col[ch * N + i] = urand();
            opa[i] = 0.3 + 0.7 * urand();
        }
        fsig[m] = 0.4 + 2.0 * urand();
    }
    /* one face behind the camera and one degenerate face */
    for (int k = 0; k < 3; k++) pos[2 * N + k] = -1.0;
    for (int k = 0; k < 3; k++) { pos[3 + k] = 0.1; pos[N + 3 + k] = 0.1; pos[2 * N + 3 + k] = 2.0; }
    int32_t faces[3 * M];
    for (int i = 0; i < 3 * M; i++) faces[i] = (int32_t)((i * 7) % N);
    orc_scene soup = {pos, col, opa, NULL, N, M, NULL};
    orc_scene mesh = {pos, col, opa, faces, N, M, NULL};
    orc_scene sig = {pos, col, opa, NULL, N, M, fsig};
    orc_cam cam = {W, H, 40.0, 42.0, (W - 1) / 2.0, (H - 1) / 2.0};
    orc_cam cams[2] = {cam, {33, 17, 25.0, 25.0, 16.0, 8.0}};
    double pose[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0.01, -0.02, 0.03};
    double poses[24];
    for (int i = 0; i < 12; i++) poses[i] = poses[12 + i] = pose[i];
    static double C[3 * W * H], D[W * H], T[W * H], gC[3 * W * H], gD[W * H], gT[W * H];
    static double gp[3 * N], gc[3 * N], go[N], gs[M], ap[3 * N], ac[3 * N], ao[N], as[M], gpose[6], mr[W * H];
    static uint64_t hash[W * H];
    for (int i = 0; i < 3 * W * H; i++) gC[i] = urand() - 0.5;
    for (int i = 0; i < W * H; i++) { gD[i] = urand() - 0.5; gT[i] = urand() - 0.5; }
    int64_t pix[5] = {0, 17, W * H / 2, W * H - 2, W * H - 1};
    for (int variant = 0; variant < 4; variant++) {
        orc_par par = {variant == 1 ? 0.5 : 1.0, 0.1, 1e-3, variant == 2 ? 1.0 : 0.0, variant == 3 ? 1.0 : 0.0,
                       variant == 2 ? 1.0 : 0.0};
        const orc_scene *scs[3] = {&soup, &mesh, &sig};
        for (int s = 0; s < 3; s++) {
            const orc_scene *sc = scs[s];
            CHECK(orc_render(sc, pose, &cam, &par, NULL, W * H, C, D, T), ORC_OK);
            CHECK(orc_render(sc, pose, &cam, &par, pix, 5, C, D, T), ORC_OK);
            memset(gp, 0, sizeof gp); memset(gc, 0, sizeof gc); memset(go, 0, sizeof go); memset(gpose, 0, sizeof gpose);
            CHECK(orc_backward_abs(sc, pose, &cam, &par, NULL, W * H, gC, gD, gT, gp, gc, go, gpose, ap, ac, ao), ORC_OK);
            CHECK(orc_backward(sc, pose, &cam, &par, pix, 5, gC, gD, NULL, gp, gc, go, gpose), ORC_OK);
            CHECK(orc_backward_sigma(sc, pose, &cam, &par, NULL, W * H, gC, gD, gT, gp, gc, go, gpose, gs, ap, ac, ao, as),
                  ORC_OK);
            CHECK(orc_state(sc, pose, &cam, &par, NULL, W * H, 1e-3, hash), ORC_OK);
            CHECK(orc_min_rho(sc, pose, &cam, &par, NULL, W * H, mr), ORC_OK);
            int64_t K = 0;
            int rc = orc_bin(sc, poses, cams, 2, &par, 0, &K, NULL, NULL, NULL, NULL);
            if (rc != ORC_OK && rc != ORC_ECAP) { fprintf(stderr, "orc_bin count: %d\n", rc); return 1; }
            int64_t T_total = 0;
            for (int v = 0; v < 2; v++) T_total += (int64_t)((cams[v].width + 15) / 16) * ((cams[v].height + 15) / 16);
            int64_t *tile = malloc(sizeof(int64_t) * (size_t)(K + 1)), *face = malloc(sizeof(int64_t) * (size_t)(K + 1));
            uint32_t *zb = malloc(sizeof(uint32_t) * (size_t)(K + 1));
            int64_t *ranges = malloc(sizeof(int64_t) * 2 * (size_t)T_total);
            CHECK(orc_bin(sc, poses, cams, 2, &par, K, &K, tile, zb, face, ranges), ORC_OK);
            free(tile); free(face); free(zb); free(ranges);
            double area[M];
            int32_t lo[M], hi[M], vc[M], vp[M];
            CHECK(orc_face_stats(sc, pose, &cam, &par, 0.3, area, lo, hi, vc, vp), ORC_OK);
            double q[6 * M], f4[4 * M];
            int32_t rect[4 * M];
            int64_t tiles[M];
            CHECK(orc_project(sc, pose, &cam, &par, q, f4, rect, tiles), ORC_OK);
        }
    }
    float tc[3 * W * H], td[W * H];
    for (int i = 0; i < 3 * W * H; i++) tc[i] = (float)urand();
    for (int i = 0; i < W * H; i++) td[i] = (float)(urand() * 3.0 - 0.5);
    (void)orc_l1_seeds(C, D, tc, td, W * H, W * H, 0.8, 0.05, gC, gD);
    /* argument errors */
    orc_par bad = {0.0, 0.1, 1e-3, 0.0, 0.0, 0.0};
    CHECK(orc_render(&soup, pose, &cam, &bad, NULL, W * H, C, D, T), ORC_EINVAL);
    CHECK(orc_render(NULL, pose, &cam, &bad, NULL, W * H, C, D, T), ORC_EINVAL);
    fsig[5] = -1.0;
    orc_par ok = {1.0, 0.1, 1e-3, 0.0, 0.0, 0.0};
    CHECK(orc_render(&sig, pose, &cam, &ok, NULL, W * H, C, D, T), ORC_EINVAL);
    orc_scene short_soup = {pos, col, opa, NULL, 10, M, NULL};
    CHECK(orc_render(&short_soup, pose, &cam, &ok, NULL, W * H, C, D, T), ORC_EINVAL);
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
