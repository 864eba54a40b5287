/* Host-side argument validation of libxsec, driven through the C ABI without a GPU: every
 * call below must return its documented status (no device work is reached, or the missing
 * device is reported as XS_ERR_HIP) and leave no memory error behind.  Built and run under
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "xsec.h"

static int failures = 0;

#define EXPECT(call, want)                                                                      \
    do {                                                                                        \
        xs_status s_ = (call);                                                                  \
        if (s_ != (want)) {                                                                     \
            printf("FAIL %s:%d %s -> %d (want %d): %s\n", __FILE__, __LINE__, #call, (int)s_,   \
                   (int)(want), xs_last_error());                                               \
            ++failures;                                                                         \
        }                                                                                       \
    } while (0)

static xs_opts good(void) {
    xs_opts o;
    xs_opts_default(&o);
    o.nu_a = 0.0;
    o.nu_b = 100.0;
    o.n_points = 10001;
    o.mass_da = 18.0;
    return o;
}

int main(void) {
    xs_plan* p = (xs_plan*)0;
    xs_opts o;
    EXPECT(xs_opts_default(NULL), XS_ERR_ARG);
    EXPECT(xs_plan_create(NULL, &p), XS_ERR_ARG);
    o = good();
    EXPECT(xs_plan_create(&o, NULL), XS_ERR_ARG);
    /* one bad field at a time */
    o = good(); o.n_points = 1;                 EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.n_points = (int64_t)1 << 40;  EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.nu_b = o.nu_a;                EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.nu_b = NAN;                   EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.cutoff = 0.0;                 EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.cutoff = INFINITY;            EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.cutoff = 1e12;                EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.mass_da = -1.0;               EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.T0 = 0.0;                     EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.profile = 99;                 EXPECT(xs_plan_create(&o, &p), XS_ERR_UNSUPPORTED);
    o = good(); o.profile = -1;                 EXPECT(xs_plan_create(&o, &p), XS_ERR_UNSUPPORTED);
    o = good(); o.precision = 7;                EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.broadening = 9;               EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.index_base = 2;               EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.profile = XS_GAUSS_FIXED;     EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.broadening = XS_BROAD_CONST; o.gamma_const = -1.0; EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.slices_per_wave = 3;          EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.waves_per_block = 3;          EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.a_is_log = 2;                 EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.n_split = 65;                 EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.tp_block = 257;               EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.vv_beta = 2;                  EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.vv_radius = -1.0;             EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    o = good(); o.gh_nodes = 65;                EXPECT(xs_plan_create(&o, &p), XS_ERR_ARG);
    if (p) { printf("FAIL a plan was returned for bad options\n"); ++failures; }
    /* a valid plan needs the device (its quadrature tables): without one, XS_ERR_HIP or
       XS_ERR_OOM and no plan */
    o = good();
    {
        xs_status s = xs_plan_create(&o, &p);
        if (s == XS_OK) {
            xs_plan_destroy(p);
            p = (xs_plan*)0;
        } else if (s != XS_ERR_HIP && s != XS_ERR_OOM) {
            printf("FAIL valid plan without a device -> %d: %s\n", (int)s, xs_last_error());
            ++failures;
        }
    }
    /* every entry point refuses NULL handles on the host */
    double T[2] = {296.0, 1000.0}, P[2] = {1.0, 1.0}, bad[2] = {-1.0, NAN};
    double q;
    int32_t cfg[6];
    int64_t st3[3];
    EXPECT(xs_plan_destroy(NULL), XS_OK);
    EXPECT(xs_set_states(NULL, 10, NULL, NULL, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_set_broadening_table(NULL, 5, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_set_lines(NULL, 10, NULL, NULL, NULL, NULL, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_lines_kept(NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_set_intensity_threshold(NULL, 1, 1e-29, 2000.0), XS_ERR_ARG);
    EXPECT(xs_set_intensity_kind(NULL, 1), XS_ERR_ARG);
    EXPECT(xs_partition_function(NULL, 2, T, &q, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_partition_function_noalloc(NULL, 2, T, &q, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_partition_function_noalloc(NULL, XS_NOALLOC_MAX_T + 1, T, &q, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_partition_moments(NULL, 2, T, NULL, NULL, NULL, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_cross_section(NULL, 2, T, P, &q, NULL), XS_ERR_ARG);
    EXPECT(xs_cross_section_nlte(NULL, 2, T, T, P, &q, NULL), XS_ERR_ARG);
    EXPECT(xs_cross_section_adjoint(NULL, 296.0, 1.0, &q, NULL, NULL, NULL, NULL, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_graph_create(NULL, 2, T, P, &q, NULL), XS_ERR_ARG);
    EXPECT(xs_graph_launch(NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_graph_set_tp(NULL, T, P, NULL), XS_ERR_ARG);
    EXPECT(xs_graph_destroy(NULL), XS_OK);
    EXPECT(xs_set_tile_config(NULL, 1, 4, 0, 0), XS_ERR_ARG);
    EXPECT(xs_get_tile_config(NULL, cfg), XS_ERR_ARG);
    EXPECT(xs_autotune(NULL, 2, T, P, 10.0, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_stream_begin(NULL, 2, T, P, &q, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_stream_chunk(NULL, 1, NULL, NULL, NULL, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_stream_chunk_device(NULL, 1, NULL, NULL, NULL, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_stream_end(NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_stream_checkpoint(NULL, "x"), XS_ERR_ARG);
    EXPECT(xs_stream_resume(NULL, "x", &q, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_stream_stats(NULL, st3), XS_ERR_ARG);
    EXPECT(xs_set_timing(NULL, 1), XS_ERR_ARG);
    EXPECT(xs_kernel_times(NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_lifetimes(NULL, 1, NULL, NULL, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_cooling_function(NULL, 1, NULL, NULL, NULL, 1, T, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_set_vibrational_labels(NULL, 1, NULL, NULL), XS_ERR_ARG);
    EXPECT(xs_partition_function_nlte(NULL, 1, T, T, &q, NULL), XS_ERR_ARG);
    (void)bad;
    if (xs_workspace_bytes(NULL) != 0) { printf("FAIL workspace of NULL\n"); ++failures; }
    if (xs_graph_workspace_bytes(NULL) != 0) { printf("FAIL graph workspace of NULL\n"); ++failures; }
    if (xs_version() != XS_ABI_VERSION) { printf("FAIL version\n"); ++failures; }
    if (strlen(xs_last_error()) == 0) { printf("FAIL empty error text after a failure\n"); ++failures; }
    printf("%s: %d failure(s)\n", failures ? "FAILED" : "OK", failures);
    return failures ? 1 : 0;
}
