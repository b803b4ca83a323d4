/* Sanitizer driver for the host half of the C ABI (test infrastructure): linked against a
 * build of the library whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers_cpu.py), it calls the sizing entry points and every entry point's
 * argument validation -- the paths that return before any device work, so no GPU is needed --
 * and checks the return codes and the error message.  Exits non-zero on any surprise. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tsr.h"

#define CHECK(expr, want)                                                                   \
    do {                                                                                    \
        int rc_ = (expr);                                                                   \
        if (rc_ != (want)) {                                                                \
            fprintf(stderr, "%s:%d: %s returned %d, expected %d (%s)\n", __FILE__, __LINE__, #expr, rc_, (want), \
                    tsr_last_error());                                                      \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

int main(void) {
    static char dummy[4096];
    tsr_scene sc = {(const float *)dummy, (const float *)dummy, (const float *)dummy, NULL, 3000, 1000, NULL, NULL};
    tsr_intrinsics intr[3] = {{64, 48, 50.f, 50.f, 31.5f, 23.5f}, {1200, 680, 600.f, 600.f, 599.5f, 339.5f},
                              {1, 1, 1.f, 1.f, 0.f, 0.f}};
    tsr_params par = {1.0f, 1e-6f, 0.1f, 1e-3f, 0.8f, 0.05f, 0, 0, 0};
    size_t bytes = 0, more = 0;
    CHECK(tsr_workspace_size(&sc, intr, 3, 0, &bytes), TSR_OK);
    CHECK(tsr_workspace_size(&sc, intr, 3, 100000, &more), TSR_OK);
    if (more < bytes + 16 * 100000) { fprintf(stderr, "pair capacity not sized\n"); return 1; }
    CHECK(tsr_workspace_size(&sc, intr, 0, 0, &bytes), TSR_EINVAL);
    CHECK(tsr_workspace_size(&sc, intr, TSR_MAX_VIEWS + 1, 0, &bytes), TSR_EINVAL);
    CHECK(tsr_workspace_size(NULL, intr, 1, 0, &bytes), TSR_EINVAL);
    tsr_intrinsics big = {16385, 4, 1.f, 1.f, 0.f, 0.f};
    CHECK(tsr_workspace_size(&sc, &big, 1, 0, &bytes), TSR_EINVAL);
    if (strlen(tsr_last_error()) == 0) { fprintf(stderr, "no error message\n"); return 1; }
    CHECK(tsr_dssim_scratch_size(intr, 3, &bytes), TSR_OK);
    CHECK(tsr_dssim_scratch_size(intr, 0, &bytes), TSR_EINVAL);
    CHECK(tsr_equilateral_scratch_size(1000, &bytes), TSR_OK);
    CHECK(tsr_equilateral_scratch_size(-1, &bytes), TSR_EINVAL);
    CHECK(tsr_normal_scratch_size(&sc, intr, 3, &bytes), TSR_OK);
    size_t dss = 0;
    CHECK(tsr_dssim_scratch_size(intr, 3, &dss), TSR_OK);
    CHECK(tsr_mapping_scratch_size(&sc, intr, 3, &bytes), TSR_OK);
    if (bytes < dss + 32 * 1000) { fprintf(stderr, "mapping scratch not sized\n"); return 1; }
    CHECK(tsr_mapping_scratch_size(&sc, intr, 0, &bytes), TSR_EINVAL);
    CHECK(tsr_mapping_scratch_size(&sc, intr, 1, NULL), TSR_EINVAL);
    /* argument validation of the device entry points: every call below fails before any
       device work */
    float poses[36] = {0};
    CHECK(tsr_bin_and_sort(&sc, poses, intr, 1, &par, NULL, 0, NULL), TSR_EINVAL);            /* no workspace */
    CHECK(tsr_bin_and_sort(&sc, NULL, intr, 1, &par, dummy, sizeof dummy, NULL), TSR_EINVAL);  /* no poses */
    CHECK(tsr_bin_and_sort(&sc, poses, intr, 1, &par, dummy, 16, NULL), TSR_EWORKSPACE);        /* too small */
    tsr_params badp = par;
    badp.sigma = 0.f;
    CHECK(tsr_bin_and_sort(&sc, poses, intr, 1, &badp, dummy, sizeof dummy, NULL), TSR_EINVAL);
    badp = par;
    badp.t_min = 1.f;
    CHECK(tsr_render_forward(&sc, poses, intr, 1, &badp, dummy, sizeof dummy, NULL, NULL, NULL, NULL), TSR_EINVAL);
    badp = par;
    badp.perspective = 2;
    CHECK(tsr_render_forward(&sc, poses, intr, 1, &badp, dummy, sizeof dummy, NULL, NULL, NULL, NULL), TSR_EINVAL);
    badp = par;
    badp.tight_tiles = -1;
    CHECK(tsr_bin_and_sort(&sc, poses, intr, 1, &badp, dummy, sizeof dummy, NULL), TSR_EINVAL);
    tsr_scene sig = sc;
    sig.face_sigma = (const float *)dummy;
    badp = par;
    badp.perspective = 1;
    CHECK(tsr_bin_and_sort(&sig, poses, intr, 1, &badp, dummy, sizeof dummy, NULL), TSR_EINVAL);
    tsr_scene short_soup = sc;
    short_soup.n_vertices = 20;
    CHECK(tsr_bin_and_sort(&short_soup, poses, intr, 1, &par, dummy, sizeof dummy, NULL), TSR_EINVAL);
    CHECK(tsr_render_backward(&sc, poses, intr, 1, &par, dummy, 16, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL),
          TSR_EWORKSPACE);
    CHECK(tsr_render_train_l1(&sc, poses, intr, 1, &par, NULL, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL,
                              NULL, NULL, NULL), TSR_EINVAL);
    CHECK(tsr_pose_step(NULL, poses, 1, 0.001f, 0.003f, NULL), TSR_EINVAL);
    CHECK(tsr_pose_compose(poses, poses, 0, poses, NULL), TSR_EINVAL);
    CHECK(tsr_pose_tau_grad(NULL, poses, 1, poses, NULL), TSR_EINVAL);
    CHECK(tsr_dssim(intr, 1, NULL, NULL, 1.f, 0, NULL, NULL, NULL, 0, NULL), TSR_EINVAL);
    CHECK(tsr_equilateral(&sc, 1.f, 0, NULL, NULL, NULL, 0, NULL), TSR_EINVAL);
    CHECK(tsr_face_stats(&sc, poses, intr, 1, &par, NULL, 0, NULL, NULL, NULL, NULL), TSR_EINVAL);
    CHECK(tsr_sensor_normals(NULL, intr, 1, NULL, NULL), TSR_EINVAL);
    /* the mapping step: every refusal below comes before the first launch; the buffers are
       host memory, which the validation never dereferences */
    size_t wsb = 0, msb = 0;
    CHECK(tsr_workspace_size(&sc, intr, 1, 0, &wsb), TSR_OK);
    CHECK(tsr_mapping_scratch_size(&sc, intr, 1, &msb), TSR_OK);
    char *ws = malloc(wsb), *scr = malloc(msb + 512);
    float *f = (float *)dummy;
    if (!ws || !scr) { fprintf(stderr, "host allocation failed\n"); return 1; }
    char *scr_al = scr + (256 - ((size_t)scr & 255)) % 256;
#define MAP(scene_, poses_, ws_, wsb_, tc_, col_, scr_, scrb_) \
    tsr_render_train_mapping(scene_, poses_, intr, 1, &par, ws_, wsb_, tc_, f, f, 0.2f, 0.1f, col_, f, f, f, f, f, f, \
                             f, f, f, scr_, scrb_, NULL)
    CHECK(MAP(&sc, NULL, ws, wsb, f, f, scr_al, msb), TSR_EINVAL);            /* no poses */
    CHECK(MAP(&sc, poses, NULL, wsb, f, f, scr_al, msb), TSR_EINVAL);         /* no workspace */
    CHECK(MAP(&sc, poses, ws, 16, f, f, scr_al, msb), TSR_EWORKSPACE);        /* workspace too small */
    tsr_scene indexed = sc;
    indexed.faces = (const int32_t *)dummy;
    indexed.n_vertices = 600;
    CHECK(MAP(&indexed, poses, ws, wsb, f, f, scr_al, msb), TSR_EINVAL);      /* indexed mesh */
    CHECK(MAP(&sc, poses, ws, wsb, NULL, f, scr_al, msb), TSR_EINVAL);        /* no colour target */
    CHECK(MAP(&sc, poses, ws, wsb, f, NULL, scr_al, msb), TSR_EINVAL);        /* no colour output */
    CHECK(MAP(&sc, poses, ws, wsb, f, f, NULL, msb), TSR_EINVAL);             /* no scratch */
    CHECK(MAP(&sc, poses, ws, wsb, f, f, scr_al, msb - 1), TSR_EWORKSPACE);   /* scratch too small */
    CHECK(MAP(&sc, poses, ws, wsb, f, f, scr_al + 4, msb), TSR_EINVAL);       /* scratch misaligned */
#undef MAP
    free(ws);
    free(scr);
    CHECK(tsr_profile_reset(), TSR_OK);
    char buf[256];
    CHECK(tsr_profile_read(buf, sizeof buf), TSR_OK);
    printf("C ABI host sanitizer driver: ok\n");
    return 0;
}
