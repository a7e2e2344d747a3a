/* A plain C program that uses libdnb through the headers alone (no torch, no
 * C++): it checks the two-body accelerations, a row block of them and their
 * vector-Jacobian product against Newton's closed forms, runs a short
 * integration with its gradient, and checks that a bad call is refused with a
 * message.  Exit status 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "dnb.h"
#include "dnb_orbitfit.h"

#define FAIL(...) do { fprintf(stderr, __VA_ARGS__); fputc('\n', stderr); return 1; } while (0)

int main(void) {
    const int64_t n = 2;
    const double G = 4.3009e-6, m = 1.0e4, d = 0.5;
    /* [3][n]: x then y then z */
    double pos[6] = {-0.5 * d, 0.5 * d, 0.0, 0.0, 0.0, 0.0};
    double vel[6] = {0.0, 0.0, -1.0, 1.0, 0.0, 0.0};
    double mass[2] = {m, m};
    double acc[6];
    dnb_pot pot = {G, 0.0, 0.0, 16.0, 0.0, 3.0, 0.28};   /* no host potential, no softening */

    dnb_ctx* ctx = NULL;
    if (dnb_create(&ctx, 16, DNB_FP64) != DNB_OK) FAIL("create: %s", dnb_last_error());
    double *dpos, *dvel, *dmass, *dacc, *tape, *work, *g0, *gv0, *gpar;
    const int64_t T = 20, K = 1;
    const int64_t tape_n = dnb_tape_doubles(n, T, K), work_n = dnb_vjp_workspace_doubles(n, K);
    if (hipMalloc((void**)&dpos, sizeof pos) || hipMalloc((void**)&dvel, sizeof vel) ||
        hipMalloc((void**)&dmass, sizeof mass) || hipMalloc((void**)&dacc, sizeof acc) ||
        hipMalloc((void**)&tape, sizeof(double) * tape_n) ||
        hipMalloc((void**)&work, sizeof(double) * work_n) ||
        hipMalloc((void**)&g0, sizeof pos) || hipMalloc((void**)&gv0, sizeof pos) ||
        hipMalloc((void**)&gpar, sizeof(double) * 7))
        FAIL("hipMalloc failed");
    hipMemcpy(dpos, pos, sizeof pos, hipMemcpyHostToDevice);
    hipMemcpy(dvel, vel, sizeof vel, hipMemcpyHostToDevice);
    hipMemcpy(dmass, mass, sizeof mass, hipMemcpyHostToDevice);

    if (dnb_accelerations(ctx, n, dpos, dmass, &pot, 1, dacc, NULL) != DNB_OK)
        FAIL("accelerations: %s", dnb_last_error());
    hipMemcpy(acc, dacc, sizeof acc, hipMemcpyDeviceToHost);
    const double a = G * m / (d * d);
    if (fabs(acc[0] - a) > 1e-14 * a || fabs(acc[1] + a) > 1e-14 * a || acc[2] != 0.0)
        FAIL("two-body acceleration %.17g %.17g, expected +-%.17g", acc[0], acc[1], a);

    /* one row of the same accelerations, and their vector-Jacobian product with
     * w = unit x on particle 0: d(a_0x)/dx_0 = 2 G m / d^3 = -d(a_0x)/dx_1 and
     * d(a_0x)/dm_1 = G / d^2 (a_0 does not depend on m_0) */
    double row[3], gx[6], gm[2], w0[6] = {1, 0, 0, 0, 0, 0};
    double *drow, *dw0, *dgx, *dgm;
    if (hipMalloc((void**)&drow, sizeof row) || hipMalloc((void**)&dw0, sizeof w0) ||
        hipMalloc((void**)&dgx, sizeof gx) || hipMalloc((void**)&dgm, sizeof gm))
        FAIL("hipMalloc failed");
    hipMemcpy(dw0, w0, sizeof w0, hipMemcpyHostToDevice);
    if (dnb_accelerations_rows(ctx, n, dpos, dmass, &pot, 1, 1, 1, drow, NULL) != DNB_OK)
        FAIL("accelerations_rows: %s", dnb_last_error());
    hipMemcpy(row, drow, sizeof row, hipMemcpyDeviceToHost);
    if (row[0] != acc[1] || row[1] != acc[3] || row[2] != acc[5])
        FAIL("row 1: %.17g, full call %.17g", row[0], acc[1]);
    if (dnb_accelerations_vjp(ctx, n, dpos, dmass, &pot, 1, dw0, 0, n, dgx, dgm, NULL) != DNB_OK)
        FAIL("accelerations_vjp: %s", dnb_last_error());
    hipMemcpy(gx, dgx, sizeof gx, hipMemcpyDeviceToHost);
    hipMemcpy(gm, dgm, sizeof gm, hipMemcpyDeviceToHost);
    const double h = 2.0 * G * m / (d * d * d);
    if (fabs(gx[0] - h) > 1e-13 * h || fabs(gx[1] + h) > 1e-13 * h || gm[0] != 0.0 ||
        fabs(gm[1] - G / (d * d)) > 1e-13 * G / (d * d))
        FAIL("accelerations vjp %.17g %.17g %.17g %.17g", gx[0], gx[1], gm[0], gm[1]);

    if (dnb_simulate(ctx, n, dpos, dvel, dmass, &pot, 0.01, T, K, tape, NULL) != DNB_OK)
        FAIL("simulate: %s", dnb_last_error());
    /* gradient of L = sum of final x coordinates */
    double w[6] = {1, 1, 0, 0, 0, 0};
    double *dw;
    if (hipMalloc((void**)&dw, sizeof w)) FAIL("hipMalloc failed");
    hipMemcpy(dw, w, sizeof w, hipMemcpyHostToDevice);
    if (dnb_simulate_vjp(ctx, n, dmass, &pot, 0.01, T, K, tape, dpos, dw, NULL, work, g0, gv0,
                         NULL, gpar, NULL) != DNB_OK)
        FAIL("simulate_vjp: %s", dnb_last_error());
    double g[6], gv[6];
    hipMemcpy(g, g0, sizeof g, hipMemcpyDeviceToHost);
    hipMemcpy(gv, gv0, sizeof gv, hipMemcpyDeviceToHost);
    /* internal forces cancel in the sum of x: d(sum x_T)/d(x_0) = (1, 1) and
     * d(sum x_T)/d(v_0) = (T dt, T dt) exactly, up to rounding */
    for (int i = 0; i < 2; ++i) {
        if (fabs(g[i] - 1.0) > 1e-12 || fabs(gv[i] - T * 0.01) > 1e-12)
            FAIL("gradient %d: %.17g %.17g", i, g[i], gv[i]);
    }

    /* the sweep that steps the trajectory backward between checkpoints every 5
     * steps, from the final velocities the forward run left in dvel: the same
     * closed form */
    const int64_t K2 = 5;
    double* work2;
    if (hipMalloc((void**)&work2, sizeof(double) * dnb_vjp_reversed_workspace_doubles(n)))
        FAIL("hipMalloc failed");
    if (dnb_simulate(ctx, n, dpos, dvel, dmass, &pot, 0.01, T, K2, tape, NULL) != DNB_OK)
        FAIL("simulate: %s", dnb_last_error());
    if (dnb_simulate_vjp_reversed(ctx, n, dmass, &pot, 0.01, T, K2, tape, dpos, dvel, dw, NULL,
                                  work2, g0, gv0, NULL, gpar, NULL) != DNB_OK)
        FAIL("simulate_vjp_reversed: %s", dnb_last_error());
    hipMemcpy(g, g0, sizeof g, hipMemcpyDeviceToHost);
    hipMemcpy(gv, gv0, sizeof gv, hipMemcpyDeviceToHost);
    for (int i = 0; i < 2; ++i) {
        if (fabs(g[i] - 1.0) > 1e-12 || fabs(gv[i] - T * 0.01) > 1e-12)
            FAIL("reversed-sweep gradient %d: %.17g %.17g", i, g[i], gv[i]);
    }

    /* a refused call: negative step count */
    if (dnb_simulate(ctx, n, dpos, dvel, dmass, &pot, 0.01, -1, 1, NULL, NULL) != DNB_ERR_ARG)
        FAIL("negative n_steps was accepted");
    if (dnb_last_error()[0] == '\0') FAIL("no error message");
    dnb_destroy(ctx);
    printf("abi consumer ok (%s)\n", dnb_version());
    return 0;
}
