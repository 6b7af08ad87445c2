/* Compile-only check of include/cgh.h as C11: every declared function is called
 * once with arguments of exactly the declared types.  Built with
 * `gcc -std=c11 -Wall -Wextra -Werror -c` by tests/test_c_header.py; never run. */
#include <stddef.h>
#include <stdint.h>

#include "cgh.h"

int cgh_header_calls(void);

int cgh_header_calls(void) {
    const float* cf = NULL;
    float* f = NULL;
    const uint8_t* u8 = NULL;
    const double z[1] = {0.2};
    const float thr[3] = {0.9f, 0.7f, 0.5f};
    void* ws = NULL;
    void* stream = NULL;
    size_t bytes = 0;
    double flops = 0.0;
    double ms[CGH_STAGE_COUNT];
    long long launches[CGH_STAGE_COUNT];
    cgh_stats stats;
    cgh_plan_info info;
    cgh_layout_info layout;
    cgh_plan* plan = NULL;
    cgh_scene scene = {cf, u8, 1, z, cf, 64, 64, f};
    int st = 0;

    st |= (cgh_status_string(CGH_SUCCESS) == NULL);
    st |= cgh_last_hip_error();
    st |= cgh_version();
    st |= cgh_haar_dwt(cf, 64, 64, 3, f, stream);
    st |= cgh_haar_idwt(cf, 64, 64, 3, f, stream);
    st |= cgh_workspace_size(64, 64, 1, 3, CGH_FP32, &bytes);
    st |= cgh_workspace_layout(64, 64, 1, 3, CGH_FP16_SPLIT, &layout);
    st |= cgh_progressive_hologram(cf, u8, 1, z, cf, thr, 532e-9, 8e-6, 64, 64, 3, CGH_BF16_SPLIT,
                                   CGH_FLAG_ACCUMULATE, ws, bytes, f, stream);
    st |= cgh_progressive_hologram_noalloc(cf, u8, 1, z, cf, thr, 532e-9, 8e-6, 64, 64, 3,
                                           CGH_FP16_SPLIT, 0u, f, stream);
    st |= cgh_progressive_stages(cf, u8, 1, z, cf, thr, 532e-9, 8e-6, 64, 64, 3, CGH_FP32, 0u, ws,
                                 bytes, f, stream);
    st |= cgh_literal_hologram(cf, u8, 1, z, cf, thr, 532e-9, 8e-6, 64, 64, 3, CGH_FP16_SPLIT,
                               CGH_FLAG_EQ1_PREFACTOR, ws, bytes, f, stream);
    st |= cgh_fused_hologram(cf, u8, 1, z, cf, thr, 532e-9, 8e-6, 64, 64, 3, CGH_FP32, 0u, ws,
                             bytes, f, stream);
    st |= cgh_exact_hologram(cf, u8, 1, z, cf, thr, 532e-9, 8e-6, 64, 64, 3, 0u, ws, bytes, f,
                             stream);
    st |= cgh_hologram_backward(cf, u8, 1, z, cf, thr, 532e-9, 8e-6, 64, 64, 3, CGH_FP32, 0u, ws,
                                bytes, f, stream);
    st |= cgh_fresnel_backpropagate(cf, 64, 64, 532e-9, 8e-6, 0.2, CGH_FP32, 0, ws, bytes, f,
                                    stream);
    bytes = cgh_angular_spectrum_workspace_size(64, 64);
    st |= cgh_angular_spectrum(cf, 64, 64, 532e-9, 8e-6, -0.2, ws, bytes, f, stream);
    st |= cgh_plan_create(&scene, 1, 3, 532e-9, 8e-6, thr, CGH_FP32, 0u, NULL, stream, &plan);
    st |= cgh_plan_execute(plan, stream);
    st |= cgh_plan_get_info(plan, &info);
    st |= cgh_plan_get_stats(plan, &stats, stream);
    st |= cgh_plan_destroy(plan);
    st |= cgh_profile_enable(1);
    st |= cgh_profile_stages(1u << CGH_STAGE_SECOND);
    st |= cgh_profile_read(ms, launches, 1);
    st |= cgh_workspace_stats(ws, 64, 64, 1, 3, CGH_FP32, &stats, stream);
    st |= cgh_mfma_peak(CGH_PEAK_BF16, 0, 256, 16, f, &flops, stream);
    return st;
}
