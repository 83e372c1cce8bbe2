/*
 * A plain C caller of the library (no Python, no torch in the process): builds
 * a quadrature, initialises the populations from given fields, advances the
 * requested number of steps and writes the macroscopic fields back out.  The
 * library allocates and owns the device workspace (d_workspace = NULL) and
 * works on the default stream.
 *
 * Usage: step_from_c IN OUT
 *   IN   int32 Np, K, N, nx, ny, steps, precision, bc_x, bc_y; float64 tau, dt;
 *        then float64 n, T, ux, uy, each [ny][nx]
 *   OUT  int32 status of rlbm_moments; float64 n, eps, ux, uy, each [ny][nx];
 *        float64 charges[4]
 * Exit status 0 when every call succeeded (rlbm_moments may report
 * RLBM_ENONPHYS, which is written to OUT), else 1 with the library's message
 * on stderr.
 */
#include <stdio.h>
#include <stdlib.h>

#include "rlbm.h"

static int read_all(FILE* f, void* p, size_t size, size_t count)
{
    return fread(p, size, count, f) == count;
}

int main(int argc, char** argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
        return 1;
    }
    FILE* in = fopen(argv[1], "rb");
    if (!in) {
        perror(argv[1]);
        return 1;
    }
    int32_t hdr[9];
    double par[2];
    if (!read_all(in, hdr, sizeof hdr[0], 9) || !read_all(in, par, sizeof par[0], 2)) {
        fprintf(stderr, "short header\n");
        return 1;
    }
    const int Np = hdr[0], K = hdr[1], N = hdr[2], nx = hdr[3], ny = hdr[4], steps = hdr[5];
    const int prec = hdr[6], bcx = hdr[7], bcy = hdr[8];
    if (nx <= 0 || ny <= 0 || nx > 4096 || ny > 4096) {
        fprintf(stderr, "grid out of range\n");
        return 1;
    }
    const size_t S = (size_t)nx * ny;
    double* buf = (double*)malloc(8 * S * sizeof(double));
    if (!buf) {
        fprintf(stderr, "out of host memory\n");
        return 1;
    }
    double *n = buf, *T = buf + S, *ux = buf + 2 * S, *uy = buf + 3 * S;
    if (!read_all(in, n, sizeof(double), 4 * S)) {
        fprintf(stderr, "short fields\n");
        return 1;
    }
    fclose(in);

    rlbm_ctx ctx = NULL;
    int rc = rlbm_init_quadrature(&ctx, Np, K, N, 1);
    if (rc != RLBM_OK) {
        fprintf(stderr, "rlbm_init_quadrature: %d\n", rc);
        return 1;
    }
    rc = rlbm_init_fields(ctx, nx, ny, n, T, ux, uy, par[0], par[1], bcx, bcy, prec, NULL, NULL);
    if (rc != RLBM_OK) {
        fprintf(stderr, "rlbm_init_fields: %d %s\n", rc, rlbm_last_error(ctx));
        rlbm_destroy(ctx);
        return 1;
    }
    rc = rlbm_step(ctx, steps);
    if (rc != RLBM_OK) {
        fprintf(stderr, "rlbm_step: %d %s\n", rc, rlbm_last_error(ctx));
        rlbm_destroy(ctx);
        return 1;
    }
    double* fo = buf + 4 * S;
    double charges[4];
    const int32_t mrc = rlbm_moments(ctx, fo, fo + S, fo + 2 * S, fo + 3 * S, charges);
    if (mrc != RLBM_OK && mrc != RLBM_ENONPHYS) {
        fprintf(stderr, "rlbm_moments: %d %s\n", (int)mrc, rlbm_last_error(ctx));
        rlbm_destroy(ctx);
        return 1;
    }
    rlbm_destroy(ctx);

    FILE* out = fopen(argv[2], "wb");
    if (!out) {
        perror(argv[2]);
        return 1;
    }
    const int ok = fwrite(&mrc, sizeof mrc, 1, out) == 1 && fwrite(fo, sizeof(double), 4 * S, out) == 4 * S &&
                   fwrite(charges, sizeof(double), 4, out) == 4;
    if (fclose(out) != 0 || !ok) {
        fprintf(stderr, "write failed\n");
        return 1;
    }
    free(buf);
    return 0;
}
