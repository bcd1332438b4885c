// Internal structures shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "halfwave.h"

namespace hw {

constexpr int kMaxBatch = 64;     // shots per batched launch
constexpr int kThreads = 256;     // threads per workgroup (4 wavefronts)
constexpr int kNumXcd = 8;        // MI355X: 8 accelerator complex dies

// Device-resident description of one 2D acoustic plan.  Buffers are
// row-major with a padded row pitch (elements).  With compensation, every
// field value is stored next to its compensation term (one word of two
// storage-format values per cell), so a cell's state of a field is one
// memory access.  The fields ping-pong between two sets so that a tile can
// recompute its neighbours' new velocities from old values.
struct Ac2dDesc {
    int64_t nx, ny, pitch;
    float w1, w2;                 // stencil weights c_k * dt/dx (fp32)
    const float *b;               // 1/rho at p points
    const float *k;               // kappa at p points
    void *vx[2], *vy[2], *p[2];   // field sets (storage words)
    int64_t comp_off;             // 8-bit compensation words: their bytes
                                  // start this many bytes after each value
                                  // array (0 when unused)
    // point source and receivers (src_n == 0 and rec_n == 0 when unused)
    const int64_t *step;          // device count of steps since the upload
    const float *src;             // per-step source samples (fp32)
    int64_t src_n;                // samples; step n < src_n adds src[n]
    int32_t src_x, src_y;         // source cell
    int32_t rec_n;                // receivers
    const int32_t *rec_xy;        // receiver cells (x, y) pairs
    double *rec;                  // trace [rec_rows][rec_n][3] (p, vx, vy)
    int64_t rec_rows;
    double rec_scale;             // 2^-scale_log2 (unscales the record)
};

// Device-resident description of one 3D elastic plan; same word layout.
// The nine fields ping-pong between two sets like the 2D fields: a step
// reads set n and writes set n+1.
struct El3dDesc {
    int64_t nx, ny, nz, pitch, slab;
    float w;                      // dt/dx (fp32)
    const float *b, *lam, *mu;    // at cell centres
    void *f[2][9];                // vx vy vz sxx syy szz sxy sxz syz
};

// Device-resident description of one 2D elastic plan (periodic in x, free
// surfaces on rows 0 and ny-1); same word layout and ping-pong as above.
// The material arrives as the per-cell fp32 coefficients of the step: b =
// 1/rho; l2m = lambda + 2 mu and lam = lambda, except on the surface rows
// where l2m is the plate modulus and lam = 0; mxy = the shear modulus at the
// sxy point (i+1/2, j+1/2), the mean of the four cells around it.
struct El2dDesc {
    int64_t nx, ny, pitch;
    float w;                      // dt/dx (fp32)
    const float *b, *l2m, *lam, *mxy;
    void *f[2][5];                // vx vy sxx syy sxy
    // point source on vy and receivers, as for Ac2dDesc (trace rows hold
    // the five fields)
    const int64_t *step;
    const float *src;
    int64_t src_n;
    int32_t src_x, src_y;
    int32_t rec_n;
    const int32_t *rec_xy;
    double *rec;
    int64_t rec_rows;
    double rec_scale;
};

// Arguments of one batched launch: the shots it covers, the parity (which
// field set is current) of each, the first global tile of each shot and
// its tile counts along x and y (for the launch's tile shape; 3D shots have
// tiles_x * tiles_y tiles per z slice).
template <class Desc>
struct BatchArgs {
    int32_t nshots;
    int32_t total_tiles;
    int32_t parity[kMaxBatch];
    int32_t tiles_x[kMaxBatch];
    int32_t tiles_y[kMaxBatch];
    int32_t tile_start[kMaxBatch + 1];
    const Desc *desc[kMaxBatch];
};

using Ac2dBatch = BatchArgs<Ac2dDesc>;

// Arguments of a launch for one plan: the descriptor travels by value.
struct Ac2dOne {
    Ac2dDesc d;
    int32_t parity, tiles_x, total_tiles;
};
using El3dBatch = BatchArgs<El3dDesc>;
struct El3dOne {
    El3dDesc d;
    int32_t parity, tiles_x, tiles_y, total_tiles;
};

// Tile shapes compiled into the library (x by y cells per workgroup, and
// the z planes one workgroup walks through for the marching 3D kernel).
//   2D kind 0: a workgroup of 4 wavefronts owns a tx by ty tile;
//   2D kind 1: a workgroup marches down a strip tx wide and ty rows tall;
//   2D kind 3: as kind 0 with 8 wavefronts (two rows of the tile per
//              wavefront fewer; faster for bf16 and fp32);
//   2D kind 4: two time steps per launch (temporal blocking): a workgroup
//              of 4 wavefronts advances its tx by ty tile from step n to
//              n+2, recomputing the cells around it the second step needs
//              (tz holds the steps per launch); kind 5: the same with 8
//              wavefronts;
//   3D kind 0: two passes (velocities, then stresses), one tx by ty tile of
//              one z plane per workgroup;
//   3D kind 2: one fused pass, a workgroup walks a tx by ty column through
//              tz planes.
struct TileShape { int tx, ty, kind, tz; };

// 2D: the width is 64 lanes times 1, 2 or 4 cells per lane
constexpr TileShape kTiles2D[] = {{64, 16, 0, 1}, {64, 32, 0, 1}, {128, 16, 0, 1},
                                  {64, 64, 1, 1}, {64, 128, 1, 1}, {128, 64, 1, 1},
                                  {128, 128, 1, 1}, {64, 16, 3, 1}, {128, 16, 3, 1},
                                  {64, 16, 4, 2}, {64, 32, 5, 2}, {64, 24, 5, 2}};
// Time steps one launch of a 2D shape advances.
constexpr int steps_per_launch2d(const TileShape &t)
{
    return t.kind == 4 || t.kind == 5 ? 2 : 1;
}
constexpr TileShape kTiles3D[] = {{64, 4, 0, 1},    {256, 1, 0, 1},   {64, 6, 2, 128},
                                  {64, 6, 2, 64},   {64, 6, 2, 512},  {64, 10, 2, 128},
                                  {64, 14, 2, 128}};
// 2D elastic: one 64 x 4 tile per workgroup, kind 1 = one fused pass,
// kind 0 = two passes (velocities, then stresses)
constexpr TileShape kTilesEl2D[] = {{64, 4, 1, 1}, {64, 4, 0, 1}};
constexpr int kNumTiles2D = sizeof(kTiles2D) / sizeof(kTiles2D[0]);
constexpr int kNumTiles3D = sizeof(kTiles3D) / sizeof(kTiles3D[0]);
constexpr int kNumTilesEl2D = sizeof(kTilesEl2D) / sizeof(kTilesEl2D[0]);

// Launchers (one translation unit per physics).
// one: the host copy of the descriptor when the launch covers a single plan
// (it is then passed by value), else nullptr
// forced: some plan of the launch has a point source or receivers;
// stencil: the stencil precision of the launch's plans (enum hw_stencil).
// Forced launches and those with a non-default stencil use tile shape 0.
hipError_t launch_ac2d_step(const Ac2dBatch &a, const Ac2dDesc *one, int storage,
                            int comp, int order, int tile, bool forced, int stencil,
                            hipStream_t s);
// The kernel variants with a point source, receivers and stencil
// precisions (tile shape 0); format is the storage format's id (F32::id ...).
hipError_t launch_ac2d_variant(const Ac2dBatch &a, const Ac2dDesc *one, int format,
                               int comp, int order, int tile, int stencil,
                               hipStream_t s);
// Two steps per launch (tile shapes of kind 4 and 5; every storage and
// compensation, no stencil variants).  `forced`: some shot has a point
// source or receivers (their plans' step counters then advance by two per
// launch).  The forcing kernels sit in their own translation unit.
hipError_t launch_ac2d_step2(const Ac2dBatch &a, const Ac2dDesc *one, int storage,
                             int comp, int order, int tile, bool forced, hipStream_t s);
hipError_t launch_ac2d_step2_forcing(const Ac2dBatch &a, const Ac2dDesc *one, int storage,
                                     int comp, int order, int tile, hipStream_t s);
hipError_t launch_ac2d_energy(const Ac2dDesc *d_desc, int parity,
                              int64_t ny, int storage, int order, int stride,
                              double *partial, hipStream_t s);
hipError_t launch_el3d_step(const El3dBatch &a, const El3dDesc *one, int storage,
                            int comp, int tile, hipStream_t s);
hipError_t launch_el3d_energy(const El3dDesc *d_desc, int parity, int64_t rows,
                              int storage, int stride, double *partial,
                              hipStream_t s);
// One step of one 2D elastic plan (descriptor by value, field set parity
// current, tile an index of kTilesEl2D); forced: the plan has a point source
// or receivers.
hipError_t launch_el2d_step(const El2dDesc &d, int parity, int storage, int comp,
                            bool forced, int tile, hipStream_t s);
hipError_t launch_el2d_energy(const El2dDesc *d_desc, int parity, int64_t ny,
                              int storage, int stride, double *partial,
                              hipStream_t s);
hipError_t launch_energy_finish(const double *partial, int64_t n,
                                double factor, double *out, int32_t *flag,
                                hipStream_t s);
// Advance the device step counters of n plans by one (n <= kMaxBatch);
// set one counter to a value.
// Step counters of plans with a source or receivers, each advanced by `by`
// (the steps of the launch before it).
struct StepCounters { int64_t *c[kMaxBatch]; int32_t n; int32_t by = 1; };
hipError_t launch_tick(const StepCounters &c, hipStream_t s);
hipError_t launch_set_counter(int64_t *c, int64_t value, hipStream_t s);

// Conversions between fp64 host-layout arrays and the device layouts:
// storage element (r*pitch + i)*stride + offset holds host value r*nx + i.
hipError_t launch_to_storage(const double *src, void *dst, int storage,
                             int64_t nx, int64_t rows, int64_t pitch,
                             int stride, int offset, double scale,
                             hipStream_t s);
hipError_t launch_from_storage(const void *src, double *dst, int storage,
                               int64_t nx, int64_t rows, int64_t pitch,
                               int stride, int offset, double scale,
                               hipStream_t s);
hipError_t launch_fill_zero(void *dst, size_t bytes, hipStream_t s);
// The compensation terms of a field held as 8-bit words (comp_off bytes
// after its value array) as fp64: q * ulp(value) / 2^7, times scale.
hipError_t launch_comp8_to_double(const void *values, size_t comp_off, double *dst,
                                  int storage, int64_t nx, int64_t rows,
                                  int64_t pitch, double scale, hipStream_t s);
hipError_t launch_material(const double *src, float *dst, int reciprocal,
                           int64_t nx, int64_t rows, int64_t pitch,
                           hipStream_t s);

}  // namespace hw
