/* Host-side argument validation of every C-ABI entry point, for the AddressSanitizer and
 * UndefinedBehaviorSanitizer build of the library's host code in tests/test_sanitizers.py.  Every
 * call here is rejected (or has nothing to do) before any device work, so it runs without a GPU;
 * the pointers are never dereferenced.  Exit 0 and no sanitizer report is a pass. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include "degraf_flow.h"

static int fails = 0;
#define EXPECT(call, want)                                                                                         \
    do {                                                                                                           \
        const long long got_ = (long long)(call);                                                                  \
        if (got_ != (long long)(want)) {                                                                           \
            fprintf(stderr, "line %d: %s = %lld, expected %lld\n", __LINE__, #call, got_, (long long)(want));      \
            ++fails;                                                                                               \
        }                                                                                                          \
    } while (0)

int main(void)
{
    void *P = (void *)(uintptr_t)0x100000; /* never dereferenced: every call below stops first */
    float *F = (float *)P;
    uint8_t *U = (uint8_t *)P;
    dgf_image im = {P, 64, 48, 64, DGF_U8}, small = {P, 63, 48, 64, DGF_U8}, f32 = {P, 64, 48, 256, DGF_F32};
    dgf_image bad = {P, 64, 48, 32, DGF_U8}, huge = {P, 64, 1 << 24, 64, DGF_U8};

    for (int c = 1; c >= -8; --c) EXPECT(dgf_strerror(c) != NULL, 1);
    EXPECT(dgf_version() >= 100, 1);
    dgf_track_opts o;
    EXPECT(dgf_track_opts_default(&o), DGF_OK);
    EXPECT(dgf_track_opts_default(NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_detect_count(1242, 375, 9, 5), 18278);
    EXPECT(dgf_detect_count(8, 8, 9, 1), 0);
    EXPECT(dgf_detect_count(8, 8, 0, 1), -1);
    int64_t off[DGF_MAX_LEVELS], pitch[DGF_MAX_LEVELS];
    EXPECT(dgf_pyramid_layout(1242, 375, 5, DGF_U8, off, pitch) > 0, 1);
    EXPECT(dgf_pyramid_layout(1242, 375, 13, DGF_U8, off, pitch), 0);
    EXPECT(dgf_track_workspace_bytes(1242, 375, 5, 7), 0);
    EXPECT(dgf_gm_workspace_bytes() > 0, 1);
    EXPECT(dgf_epic_workspace_bytes(64, 48, 10) > 0, 1);

    /* detection */
    EXPECT(dgf_detect(&bad, 9, 8, F, NULL, NULL, 100, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_detect(&huge, 9, 8, F, NULL, NULL, 100, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_detect(&im, 0, 8, F, NULL, NULL, 100, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_detect(&im, 9, 8, F, NULL, NULL, 3, NULL), DGF_ERR_CAPACITY);
    EXPECT(dgf_detect(&im, 9, 8, NULL, NULL, NULL, 100, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_pyramid(&im, 3, NULL, 0, NULL), DGF_ERR_WORKSPACE);
    EXPECT(dgf_pyramid(&im, 1, NULL, 0, NULL), DGF_OK);

    /* tracking: every argument check, every flag, n = 0 */
    const size_t ws = dgf_track_workspace_bytes(64, 48, 3, DGF_U8);
    EXPECT(dgf_track(&im, &small, F, 10, 3, 9, 10, NULL, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track(&im, &im, F, 10, 0, 9, 10, NULL, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track(&im, &im, F, 10, 3, 8, 10, NULL, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track(&im, &im, F, 10, 3, 9, 0, NULL, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track(&im, &im, F, -1, 3, 9, 10, NULL, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track(&im, &im, F, 10, 3, 9, 10, NULL, NULL, 0, F, U, NULL, NULL, NULL), DGF_ERR_WORKSPACE);
    EXPECT(dgf_track(&im, &im, F, 10, 3, 9, 10, NULL, P, ws - 1, F, U, NULL, NULL, NULL), DGF_ERR_WORKSPACE);
    EXPECT(dgf_track(&im, &im, NULL, 0, 3, 9, 10, NULL, P, ws, NULL, NULL, NULL, NULL, NULL), DGF_OK);
    dgf_track_opts t = o;
    t.flags = 8;
    EXPECT(dgf_track(&im, &im, F, 10, 3, 9, 10, &t, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_UNSUPPORTED);
    t.flags = DGF_TRACK_CROSS;
    t.cross_tau = NAN;
    EXPECT(dgf_track(&im, &im, F, 10, 3, 9, 10, &t, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    t.cross_tau = 25.0f;
    EXPECT(dgf_track(&im, &im, F, 10, 3, 13, 10, &t, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_UNSUPPORTED);
    t.flags = DGF_TRACK_GLOBAL;
    EXPECT(dgf_track(&im, &im, NULL, 0, 1, 9, 10, &t, NULL, 0, NULL, NULL, NULL, NULL, NULL), DGF_ERR_WORKSPACE);
    t = o;
    t.sigma1 = NAN;
    EXPECT(dgf_track(&im, &im, F, 10, 3, 9, 10, &t, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track_run(&im, &im, F, 10, 3, 9, 10, NULL, P, ws, F, U, NULL, F, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track_pyramids(&im, &small, 3, P, ws, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track_pyramids(&im, &im, 3, NULL, 0, NULL), DGF_ERR_WORKSPACE);
    EXPECT(dgf_detect_pyramids(&im, &im, 9, 8, 3, NULL, 0, F, NULL, NULL, 100, NULL), DGF_ERR_WORKSPACE);
    EXPECT(dgf_detect_pyramids(&f32, &f32, 9, 8, 3, P, ws, F, NULL, NULL, 100, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track_static(&im, &im, F, 10, 0, 9, 10, NULL, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_track_static(&im, &im, NULL, 0, 3, 9, 10, NULL, NULL, NULL, NULL, NULL, NULL), DGF_OK);
    dgf_image big = {P, 4096, 4096, 4 * 4096, DGF_F32};
    EXPECT(dgf_track_static(&big, &big, F, 10, 3, 9, 10, NULL, F, U, NULL, NULL, NULL), DGF_ERR_SCRATCH);

    /* gradients, global fit, interpolation, tuning */
    EXPECT(dgf_track_backward(&im, &im, F, 10, 9, NULL, F, U, F, F, F, NULL, NULL, NULL), DGF_ERR_UNSUPPORTED);
    EXPECT(dgf_track_backward(&f32, &f32, F, 10, 8, NULL, F, U, F, F, F, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    t = o;
    t.flags = DGF_TRACK_CROSS;
    EXPECT(dgf_track_backward(&f32, &f32, F, 10, 9, &t, F, U, F, F, F, NULL, NULL, NULL), DGF_ERR_UNSUPPORTED);
    EXPECT(dgf_track_backward(&f32, &f32, NULL, 0, 9, NULL, NULL, NULL, NULL, F, F, NULL, NULL, NULL), DGF_OK);
    EXPECT(dgf_detect_backward(&im, 9, 8, U, F, 5, F, 64, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_gm_fit(F, F, U, 10, 0, 5, 1.0, P, dgf_gm_workspace_bytes(), (double *)P, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_gm_fit(F, F, U, 10, 5, 5, 0.0, P, dgf_gm_workspace_bytes(), (double *)P, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_gm_fit(F, F, U, 10, 5, 5, 1.0, P, 16, (double *)P, NULL), DGF_ERR_WORKSPACE);
    dgf_epic_opts eo;
    EXPECT(dgf_epic_opts_default(&eo), DGF_OK);
    EXPECT(dgf_epic_opts_default(NULL), DGF_ERR_INVALID_ARG);
    dgf_tuning tu;
    EXPECT(dgf_get_tuning(21, 5, DGF_U8, 18278, &tu), DGF_OK);
    EXPECT(dgf_set_tuning(8, DGF_U8, &tu), DGF_ERR_INVALID_ARG);
    tu.lanes_per_point = 7;
    EXPECT(dgf_set_tuning(21, DGF_U8, &tu), DGF_ERR_UNSUPPORTED);
    EXPECT(dgf_autotune(&im, &im, F, 0, 3, 9, 10, NULL, P, ws, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);

    /* batch plans: rejected descriptions allocate nothing */
    dgf_batch *b = NULL;
    dgf_pair_desc d = {im, small, 9, 8};
    EXPECT(dgf_batch_create(&d, 1, 3, 9, 10, NULL, &b), DGF_ERR_INVALID_ARG);
    d.I1 = im;
    EXPECT(dgf_batch_create(&d, 0, 3, 9, 10, NULL, &b), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_batch_create(&d, 1, 13, 9, 10, NULL, &b), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_batch_create(&d, 1, 3, 9, 10, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(b == NULL, 1);
    EXPECT(dgf_batch_num_points(NULL), -1);
    EXPECT(dgf_batch_grad_size(NULL, NULL), -1);
    EXPECT(dgf_batch_run(NULL, F, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_batch_front(NULL, F, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_batch_track(NULL, F, F, U, NULL, NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_batch_replay(NULL, NULL), DGF_ERR_INVALID_ARG);
    EXPECT(dgf_batch_destroy(NULL), DGF_OK);
    if (fails) return 1;
    printf("abi checks passed\n");
    return 0;
}
