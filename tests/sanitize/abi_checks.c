/*
 * Host-side argument validation of libzeta3 under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_sanitizers.py builds a host-only, instrumented copy of the library
 * and this driver).  Every call here is rejected, or completes, before any device work, so
 * the driver runs on a machine without a GPU.  Exit status 0 when every status code is the
 * expected one; a sanitizer report aborts with a non-zero status.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "zeta3.h"

static int failures = 0;

static void expect(const char *what, z3_status got, z3_status want)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, z3_last_error());
        ++failures;
    }
}

int main(void)
{
    const double edges[3] = {1e-6, 4e-6, 1e-5};
    const double unsorted[3] = {1e-6, 1e-5, 4e-6};
    const double zero_first[3] = {0.0, 4e-6, 1e-5};
    /* a non-NULL stand-in for device arrays: never dereferenced on these paths */
    double *fake = (double *)(uintptr_t)0x1000;
    z3_index idx = NULL;

    expect("build n < 0", z3_build_index(-1, fake, NULL, 2, edges, 0.0, NULL, &idx), Z3_ERR_INVALID_ARG);
    expect("build xyz NULL", z3_build_index(10, NULL, NULL, 2, edges, 0.0, NULL, &idx), Z3_ERR_INVALID_ARG);
    expect("build nbins 0", z3_build_index(10, fake, NULL, 0, edges, 0.0, NULL, &idx), Z3_ERR_INVALID_ARG);
    expect("build nbins too many", z3_build_index(10, fake, NULL, Z3_MAX_NBINS + 1, edges, 0.0, NULL, &idx),
           Z3_ERR_INVALID_ARG);
    expect("build unsorted", z3_build_index(10, fake, NULL, 2, unsorted, 0.0, NULL, &idx), Z3_ERR_INVALID_ARG);
    expect("build E_0 = 0", z3_build_index(10, fake, NULL, 2, zero_first, 0.0, NULL, &idx), Z3_ERR_INVALID_ARG);
    expect("build out NULL", z3_build_index(10, fake, NULL, 2, edges, 0.0, NULL, NULL), Z3_ERR_INVALID_ARG);
    expect("planar n < 0", z3_build_index_planar(-5, fake, NULL, 2, edges, 0.0, NULL, &idx), Z3_ERR_INVALID_ARG);
    if (idx) { fprintf(stderr, "index handle written on failure\n"); ++failures; }

    /* allocation limit: refused before the first device call, no handle */
    z3_set_device_alloc_limit(0);
    expect("build under a zero allocation limit", z3_build_index(10, fake, NULL, 2, edges, 0.0, NULL, &idx),
           Z3_ERR_OUT_OF_MEMORY);
    if (idx || !strstr(z3_last_error(), "allocation limit")) { fprintf(stderr, "limit path\n"); ++failures; }
    const double nu[4] = {-1.3, -2.5, -1.3, -1.3};
    expect("fftlog under a zero allocation limit",
           z3_fftlog_a_functions(64, fake, 1e-6, 30.0, nu, 100, 1e-4, 60.0, 2, fake, 8, fake, fake, NULL, 0, NULL),
           Z3_ERR_OUT_OF_MEMORY);
    z3_set_device_alloc_limit(SIZE_MAX);

    expect("set_values idx NULL", z3_index_set_values(NULL, 1, fake, NULL), Z3_ERR_INVALID_ARG);
    expect("update_values idx NULL", z3_index_update_values(NULL, fake, NULL), Z3_ERR_INVALID_ARG);
    expect("prepare_capture idx NULL", z3_index_prepare_capture(NULL, 0, NULL), Z3_ERR_INVALID_ARG);
    expect("perm idx NULL", z3_index_perm(NULL, (int64_t *)fake, NULL), Z3_ERR_INVALID_ARG);
    expect("estimate idx NULL", z3_estimate(NULL, 0, 10, Z3_PREC_FP64, 0, 1, fake, NULL, NULL), Z3_ERR_INVALID_ARG);
    expect("estimate_ex idx NULL", z3_estimate_ex(NULL, 0, 10, Z3_PREC_FP64, 0, 0, 1, fake, NULL, NULL),
           Z3_ERR_INVALID_ARG);
    expect("estimate_static idx NULL", z3_estimate_static(NULL, 0, 10, Z3_PREC_FP64, 0, 0, 1, fake, NULL, NULL),
           Z3_ERR_INVALID_ARG);
    expect("estimate_histogram idx NULL", z3_estimate_histogram(NULL, 0, 10, Z3_PREC_FP64, 0, 1, fake, NULL, NULL),
           Z3_ERR_INVALID_ARG);
    expect("set_phi_bins idx NULL", z3_index_set_phi_bins(NULL, 8, fake), Z3_ERR_INVALID_ARG);
    expect("adjoint idx NULL", z3_adjoint(NULL, 0, 10, 0, 1, fake, 1.0, fake, NULL), Z3_ERR_INVALID_ARG);
    expect("weight_sum idx NULL", z3_pivot_weight_sum(NULL, 0, 1, fake, NULL), Z3_ERR_INVALID_ARG);

    expect("contract npiv < 0", z3_contract(-1, 10, 4, Z3_PREC_FP64, fake, fake, fake, NULL), Z3_ERR_INVALID_ARG);
    expect("contract m_max too large", z3_contract(10, 1000, 4, Z3_PREC_FP64, fake, fake, fake, NULL),
           Z3_ERR_INVALID_ARG);
    expect("finalize nmaps 0", z3_finalize(0, 10, 4, fake, fake, NULL), Z3_ERR_INVALID_ARG);
    expect("finalize zeta NULL", z3_finalize(1, 10, 4, NULL, fake, NULL), Z3_ERR_INVALID_ARG);
    expect("resum m_max < 0", z3_resum(-1, 4, fake, 8, fake, fake, NULL), Z3_ERR_INVALID_ARG);
    expect("resum no angles", z3_resum(10, 4, fake, 0, fake, fake, NULL), Z3_OK);

    expect("fftlog odd N", z3_fftlog_a_functions(63, fake, 1e-6, 30.0, nu, 100, 1e-4, 60.0, 2, fake, 8, fake, fake,
                                                 NULL, 0, NULL),
           Z3_ERR_INVALID_ARG);
    const double pole[4] = {0.0, -2.5, -1.3, -1.3};
    expect("fftlog Gamma pole", z3_fftlog_a_functions(64, fake, 1e-6, 30.0, pole, 100, 1e-4, 60.0, 2, fake, 8, fake,
                                                      fake, NULL, 0, NULL),
           Z3_ERR_INVALID_ARG);
    expect("fftlog no models", z3_fftlog_a_functions(64, fake, 1e-6, 30.0, nu, 100, 1e-4, 60.0, 0, fake, 8, fake,
                                                     fake, NULL, 0, NULL),
           Z3_OK);
    size_t bytes = 0;
    expect("fftlog workspace size", z3_fftlog_workspace_size(256, 512, 64, 4, &bytes), Z3_OK);
    if (bytes == 0) { fprintf(stderr, "workspace size 0\n"); ++failures; }
    expect("fftlog workspace size NULL", z3_fftlog_workspace_size(256, 512, 64, 4, NULL), Z3_ERR_INVALID_ARG);

    int64_t launches = -1;
    double ms = -1.0;
    expect("profile enable", z3_profile_enable(1), Z3_OK);
    expect("profile read", z3_profile_read(&launches, &ms, 1), Z3_OK);
    expect("profile disable", z3_profile_enable(0), Z3_OK);
    for (int s = 0; s <= 5; ++s)
        if (!z3_status_string((z3_status)s)) { fprintf(stderr, "status string %d\n", s); ++failures; }
    z3_index_free(NULL);

    if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
    else printf("abi checks ok\n");
    return failures ? 1 : 0;
}
