/* c_abi_demo.c -- the thermal lattice Boltzmann library from C, without
 * Python or torch: the library allocates its own device memory (dev_buf =
 * NULL), the caller hands in the initial fields as a device FP64 array.
 *
 *   c_abi_demo [N] [Ra] [storage]      (defaults 33 1e4 1 = FP32)
 *
 * Runs the side-heated cell (Sec. 3) with U = 0.1 from rest with the
 * temperature perturbation T = 1e-3 ((7x + 13y + 29z) mod 17 - 8) / 8 to the
 * steady-state criterion max |dT| < 1e-6 over 1000 steps (at most 200 000
 * steps) and prints one JSON line: steps, final max |dT|, and the
 * nondimensional Nu (mean of the two isothermal walls, link flux), Re,
 * eps_u, eps_T.  Exit status 0
 * on success, 1 on any library or HIP error (message on stderr). */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "lbm.h"

static int fail(const char *what, int rc, const lbm_t *h) {
    fprintf(stderr, "%s: %s (%s)\n", what, lbm_strerror(rc), h ? lbm_last_error(h) : "");
    return 1;
}

int main(int argc, char **argv) {
    const int N = argc > 1 ? atoi(argv[1]) : 33;
    const double Ra = argc > 2 ? atof(argv[2]) : 1e4;
    const int storage = argc > 3 ? atoi(argv[3]) : LBM_FP32;
    const size_t V = (size_t)N * N * N;

    lbm_opts o;
    lbm_default_opts(&o);
    o.U = 0.1;
    lbm_t *h = NULL;
    int rc = lbm_create(N, Ra, 0.71, LBM_SIDE_HEATED, storage, &o, NULL, 0, &h);
    if (rc != LBM_OK) return fail("lbm_create", rc, NULL);

    double *host = (double *)calloc(4 * V, sizeof(double));
    if (!host) return 1;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x)
                host[3 * V + ((size_t)z * N + y) * N + x] = 1e-3 * (double)((7 * x + 13 * y + 29 * z) % 17 - 8) / 8.0;
    double *dev = NULL;
    if (hipMalloc((void **)&dev, 4 * V * sizeof(double)) != hipSuccess ||
        hipMemcpy(dev, host, 4 * V * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        fprintf(stderr, "HIP allocation or copy failed\n");
        return 1;
    }
    free(host);
    if ((rc = lbm_set_fields(h, dev, NULL)) != LBM_OK) return fail("lbm_set_fields", rc, h);
    hipFree(dev);

    int64_t steps = 0;
    double res = 0.0, Nu, Re, eps_u, eps_T;
    if ((rc = lbm_run_to_steady(h, 1000, 1e-6, 200000, NULL, &steps, &res, NULL, 0)) != LBM_OK)
        return fail("lbm_run_to_steady", rc, h);
    if ((rc = lbm_observables(h, NULL, &Nu, &Re, &eps_u, &eps_T)) != LBM_OK)
        return fail("lbm_observables", rc, h);
    printf("{\"N\": %d, \"Ra\": %.17g, \"storage\": %d, \"steps\": %lld, \"max_dT\": %.17g, "
           "\"Nu\": %.17g, \"Re\": %.17g, \"eps_u\": %.17g, \"eps_T\": %.17g}\n",
           N, Ra, storage, (long long)steps, res, Nu, Re, eps_u, eps_T);
    return lbm_destroy(h) == LBM_OK ? 0 : 1;
}
