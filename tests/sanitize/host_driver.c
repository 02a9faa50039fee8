/* Drives the library's host code through the entry points that need no GPU,
 * under AddressSanitizer and UndefinedBehaviorSanitizer (built by
 * tests/test_sanitizers.py): grid and frame checks over valid, invalid and
 * unsupported inputs, the marching-cubes table, tuning set / get / clear with
 * good and bad parameters, status strings, timing names, and every entry
 * point given NULL handles.  Prints "ok" and returns 0 when every status is
 * the documented one. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "fvr.h"

#define CHECK(expr, want)                                                                   \
    do {                                                                                    \
        const int got_ = (int)(expr);                                                      \
        if (got_ != (int)(want)) {                                                          \
            fprintf(stderr, "%s:%d: %s = %d, expected %d\n", __FILE__, __LINE__, #expr, got_, \
                    (int)(want));                                                           \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

int main(void) {
    const float box[6] = {-1, -1, -1, 1, 1, 1};
    const int32_t good[][3] = {{64, 64, 64}, {8, 8, 8}, {512, 96, 30}, {256, 256, 256}};
    for (size_t i = 0; i < sizeof good / sizeof good[0]; ++i) CHECK(fvr_check_grid(good[i], box), FVR_OK);
    const int32_t odd[3] = {63, 64, 64}, small[3] = {4, 64, 64}, seven[3] = {56, 64, 64}, big[3] = {64, 64, 1024};
    CHECK(fvr_check_grid(odd, box), FVR_E_INVALID);
    CHECK(fvr_check_grid(small, box), FVR_E_INVALID);
    CHECK(fvr_check_grid(seven, box), FVR_E_UNSUPPORTED);
    CHECK(fvr_check_grid(big, box), FVR_E_UNSUPPORTED);
    const float flat[6] = {-1, -1, 1, 1, 1, 1}, nan_box[6] = {-1, -1, -1, 1, 1, 0.0f / 0.0f};
    CHECK(fvr_check_grid(good[0], flat), FVR_E_INVALID);
    CHECK(fvr_check_grid(good[0], nan_box), FVR_E_INVALID);
    CHECK(fvr_check_grid(NULL, box), FVR_E_INVALID);
    CHECK(fvr_check_grid(good[0], NULL), FVR_E_INVALID);

    float p[3] = {0, 0, 0};
    fvr_frame f;
    memset(&f, 0, sizeof f);
    f.points = p;
    f.normals = p;
    f.n_points = 1;
    memcpy(f.dims, good[0], sizeof f.dims);
    memcpy(f.bbox, box, sizeof f.bbox);
    CHECK(fvr_check_frame(&f), FVR_OK);
    f.options = FVR_SPLAT_NEAREST | FVR_STORAGE_FP16;
    CHECK(fvr_check_frame(&f), FVR_OK);
    f.options = FVR_STORAGE_BF16 | FVR_STORAGE_FP16;
    CHECK(fvr_check_frame(&f), FVR_E_INVALID);
    f.options = 64;
    CHECK(fvr_check_frame(&f), FVR_E_INVALID);
    f.options = 0;
    f.n_points = FVR_MAX_POINTS + 1;
    CHECK(fvr_check_frame(&f), FVR_E_INVALID);
    f.n_points = -1;
    CHECK(fvr_check_frame(&f), FVR_E_INVALID);
    f.n_points = 1;
    f.normals = NULL;
    CHECK(fvr_check_frame(&f), FVR_E_INVALID);
    f.n_points = 0;  /* an empty frame needs no arrays */
    CHECK(fvr_check_frame(&f), FVR_OK);
    CHECK(fvr_check_frame(NULL), FVR_E_INVALID);

    uint8_t counts[256];
    int8_t edges[256 * 15];
    CHECK(fvr_mc_table(counts, edges), FVR_OK);
    int tri = 0;
    for (int c = 0; c < 256; ++c) tri += counts[c];
    if (counts[0] != 0 || counts[255] != 0 || tri == 0) {
        fprintf(stderr, "implausible table\n");
        return 1;
    }

    /* tuning: a valid order and tile, read back, an invalid product, cleared */
    const int32_t d96[3] = {96, 160, 192};
    fvr_tuning t, u;
    memset(&t, 0, sizeof t);
    t.nstages[0] = 3;
    t.radices[0][0] = 4;
    t.radices[0][1] = 8;
    t.radices[0][2] = 3;
    t.splat_ty = 2;
    t.splat_tz = 2;
    CHECK(fvr_set_tuning(d96, &t), FVR_OK);
    CHECK(fvr_get_tuning(d96, &u), FVR_OK);
    if (u.nstages[0] != 3 || u.radices[0][1] != 8 || u.splat_ty != 2) {
        fprintf(stderr, "tuning not read back\n");
        return 1;
    }
    t.radices[0][2] = 5; /* 4 * 8 * 5 != 96 */
    CHECK(fvr_set_tuning(d96, &t), FVR_E_INVALID);
    CHECK(fvr_set_tuning(d96, NULL), FVR_OK);
    CHECK(fvr_get_tuning(d96, &u), FVR_OK);

    for (int s = -6; s <= 0; ++s)
        if (!fvr_status_string((fvr_status)s) || !strcmp(fvr_status_string((fvr_status)s), "unknown status")) {
            fprintf(stderr, "no string for status %d\n", s);
            return 1;
        }
    if (strcmp(fvr_status_string((fvr_status)-99), "unknown status")) return 1;
    for (int i = 0; i < fvr_timing_count(); ++i)
        if (!fvr_timing_name(i) || !fvr_timing_name(i)[0]) return 1;

    /* NULL handles: documented errors, no crash */
    fvr_mesh mesh;
    memset(&mesh, 0, sizeof mesh);
    CHECK(fvr_reconstruct(NULL, &f, &mesh), FVR_E_INVALID);
    CHECK(fvr_reconstruct_noalloc(NULL, &f, &mesh), FVR_E_INVALID);
    CHECK(fvr_indicator(NULL, &f, NULL, NULL), FVR_E_INVALID);
    CHECK(fvr_last_stats(NULL, NULL), FVR_E_INVALID);
    CHECK(fvr_timing_enable(NULL, 1), FVR_E_INVALID);
    CHECK(fvr_batch_reconstruct(NULL, &f, &mesh, 1), FVR_E_INVALID);
    CHECK(fvr_server_poll(NULL, NULL, 0, NULL), FVR_E_INVALID);
    if (!fvr_last_error(NULL)) return 1;
    fvr_destroy(NULL);
    fvr_batch_destroy(NULL);
    fvr_server_destroy(NULL);
    printf("ok\n");
    return 0;
}
