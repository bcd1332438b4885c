/* A plain C client of libhalfwave: no Python, no torch.  It reads a problem,
 * its material and its initial fields from a binary file, runs them on the
 * current GPU through the C ABI of halfwave.h alone (the arena comes from
 * hipMalloc), and writes the final fields, compensation terms and energy
 * trace.  The tests run it and compare its output with the oracle.
 *
 *   halfwave_run INPUT OUTPUT
 *
 * INPUT, little-endian: int64 physics, order, storage, comp, nx, ny, nz,
 * nsteps, energy_every, tile (-1: the default shape), trace_cap; double dx,
 * dt; then hw_num_materials(physics) and hw_num_fields(physics) arrays of
 * nx*ny*nz doubles, row-major, in the header's orders.
 * OUTPUT: the hw_num_fields field arrays, the hw_num_fields compensation
 * arrays (fp64), int64 n (the energies held, at most trace_cap), then n
 * doubles.
 * Exit status 0 on success; otherwise the failing call and hw_last_error()
 * go to stderr and the status is 1 (2 for a usage or file error). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "halfwave.h"

static int fail_hw(const char *what, hw_status st)
{
    fprintf(stderr, "%s: status %d: %s\n", what, (int)st, hw_last_error());
    return 1;
}

static int read_all(FILE *f, void *dst, size_t bytes)
{
    return fread(dst, 1, bytes, f) == bytes;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s INPUT OUTPUT\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) {
        perror(argv[1]);
        return 2;
    }
    int64_t h[11];
    double dxdt[2];
    if (!read_all(in, h, sizeof h) || !read_all(in, dxdt, sizeof dxdt)) {
        fprintf(stderr, "%s: short header\n", argv[1]);
        return 2;
    }
    hw_problem pb = {0};
    pb.abi_version = HW_ABI_VERSION;
    pb.physics = (int32_t)h[0];
    pb.order = (int32_t)h[1];
    pb.storage = (int32_t)h[2];
    pb.comp = (int32_t)h[3];
    pb.nx = h[4];
    pb.ny = h[5];
    pb.nz = h[6];
    pb.dx = dxdt[0];
    pb.dt = dxdt[1];
    pb.trace_cap = h[10];
    const int64_t nsteps = h[7], every = h[8], tile = h[9];

    /* validation happens on the host, before any device memory exists */
    size_t bytes = 0;
    hw_status st = hw_footprint(&pb, &bytes);
    if (st != HW_OK)
        return fail_hw("hw_footprint", st);
    const int nm = hw_num_materials(pb.physics), nf = hw_num_fields(pb.physics);
    const size_t cells = (size_t)(pb.nx * pb.ny * pb.nz);
    double *host = (double *)malloc(sizeof(double) * cells * (size_t)(nm + 2 * nf));
    if (!host) {
        fprintf(stderr, "out of host memory\n");
        return 2;
    }
    const double *mat[8];
    const double *fin[16];
    double *fout[16], *cout[16];
    for (int i = 0; i < nm; ++i)
        mat[i] = host + (size_t)i * cells;
    for (int i = 0; i < nf; ++i) {
        fin[i] = host + (size_t)(nm + i) * cells;
        fout[i] = host + (size_t)i * cells;      /* after the upload, reused */
        cout[i] = host + (size_t)(nm + nf + i) * cells;
    }
    if (!read_all(in, host, sizeof(double) * cells * (size_t)(nm + nf))) {
        fprintf(stderr, "%s: short data\n", argv[1]);
        return 2;
    }
    fclose(in);

    void *arena = NULL;
    if (hipMalloc(&arena, bytes) != hipSuccess) {
        fprintf(stderr, "hipMalloc of %zu bytes failed\n", bytes);
        return 1;
    }
    hw_plan *plan = NULL;
    int rc = 0;
    double *energy = NULL;
    int64_t n_energy = 0;
    if ((st = hw_plan_create(&pb, arena, bytes, &plan)) != HW_OK) {
        rc = fail_hw("hw_plan_create", st);
        goto out;
    }
    if (tile >= 0 && (st = hw_plan_set_tile(plan, (int32_t)tile)) != HW_OK) {
        rc = fail_hw("hw_plan_set_tile", st);
        goto out;
    }
    if ((st = hw_set_material(plan, mat, NULL)) != HW_OK) {
        rc = fail_hw("hw_set_material", st);
        goto out;
    }
    if ((st = hw_set_fields(plan, fin, NULL)) != HW_OK) {
        rc = fail_hw("hw_set_fields", st);
        goto out;
    }
    /* the uploads are asynchronous: the host arrays are reused only after
     * the stream has drained */
    if (hipDeviceSynchronize() != hipSuccess) {
        fprintf(stderr, "hipDeviceSynchronize failed\n");
        rc = 1;
        goto out;
    }
    if ((st = hw_advance(plan, nsteps, every, NULL)) != HW_OK) {
        rc = fail_hw("hw_advance", st);
        goto out;
    }
    if ((st = hw_get_fields(plan, fout, cout, NULL)) != HW_OK) {
        rc = fail_hw("hw_get_fields", st);
        goto out;
    }
    energy = (double *)malloc(sizeof(double) * (size_t)(pb.trace_cap > 0 ? pb.trace_cap : 1));
    if ((st = hw_energy_trace(plan, energy, NULL, pb.trace_cap, &n_energy, NULL)) != HW_OK) {
        rc = fail_hw("hw_energy_trace", st);
        goto out;
    }
    {
        FILE *o = fopen(argv[2], "wb");
        if (!o) {
            perror(argv[2]);
            rc = 2;
            goto out;
        }
        fwrite(host, sizeof(double), cells * (size_t)nf, o);
        fwrite(host + (size_t)(nm + nf) * cells, sizeof(double), cells * (size_t)nf, o);
        const int64_t n_out = n_energy < pb.trace_cap ? n_energy : pb.trace_cap;
        fwrite(&n_out, sizeof n_out, 1, o);
        fwrite(energy, sizeof(double), (size_t)n_out, o);
        if (fclose(o) != 0) {
            perror(argv[2]);
            rc = 2;
        }
    }
out:
    if (plan) {
        hipDeviceSynchronize();
        hw_plan_destroy(plan);
    }
    hipFree(arena);
    free(energy);
    free(host);
    return rc;
}
