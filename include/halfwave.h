/*
 * halfwave.h -- C ABI of the MI355X (gfx950) library for staggered-grid
 * leapfrog wave propagation with half-precision state and compensated
 * updates (Gao & Harms, "Half precision wave simulation").
 *
 * The library computes, on one GPU:
 *   - the 2D acoustic system of Eq. (1) (Sec. 3): rho dvx/dt = dp/dx,
 *     rho dvy/dt = dp/dy, beta dp/dt = dvx/dx + dvy/dy, with the signs as
 *     printed; staggered grid, 2nd- or 4th-order staggered stencil (the 4th
 *     order one has coefficients [1/24, -9/8, 9/8, -1/24], Sec. 3), periodic
 *     in both directions, 2nd-order staggered leapfrog in time;
 *   - the 3D velocity-stress elastic system, the 3D form of Eq. (A1)
 *     (App. A), 2nd order, on the standard staggered layout, periodic;
 *   - the 2D velocity-stress elastic system of Eq. (A1) (App. A), 2nd
 *     order, periodic in x and bounded in y by two free surfaces, with the
 *     point source on the vertical velocity (the s^{vy} term);
 *   - per step and per field, the update of Alg. 1 (plain, V += R) or of
 *     Alg. 2 (compensated, Sec. 4) with the 3-operation sum (Code 1) or the
 *     6-operation sum (Code 2), the fields and compensation terms held in
 *     fp32, fp16 or bf16;
 *   - the discrete energy of the scheme, in fp64 (Sec. 3 uses it as the
 *     diagnosis tool; its formula is given at hw_record_energy).
 *
 * Grid and layout.  2D arrays are row-major [ny][nx] (x fastest); p[j][i] is
 * at (i dx, j dx), vx[j][i] at ((i+1/2) dx, j dx), vy[j][i] at
 * (i dx, (j+1/2) dx).  3D arrays are [nz][ny][nx]; normal stresses and the
 * material at (i, j, k), vx at (i+1/2, j, k), vy at (i, j+1/2, k), vz at
 * (i, j, k+1/2), sxy at (i+1/2, j+1/2, k), sxz at (i+1/2, j, k+1/2), syz at
 * (i, j+1/2, k+1/2).  All indices wrap periodically, except y of the 2D
 * elastic system.  The state at the top of a step is (v^{n-1/2}, p^n) (or
 * sigma^n): velocities are updated first.
 *
 * 2D elastic layout ([ny][nx]): sxx, syy and the material at (i, j), vx at
 * (i+1/2, j), vy at (i, j+1/2), sxy at (i+1/2, j+1/2); x wraps.  Rows 0 and
 * ny-1 of the normal stresses are free surfaces (zero traction): syy is
 * zero there and never updated; sxy half a cell outside a surface is minus
 * sxy half a cell inside; on the surface rows sxx changes by the plate
 * modulus 4 mu (lambda + mu) / (lambda + 2 mu) times the horizontal strain
 * rate (the vertical strain rate eliminated through syy = 0).  vy and sxy
 * live on rows 0 .. ny-2; their row ny-1 lies outside the body, is zero and
 * stays zero.  ny >= 3.
 *
 * Field order:     acoustic  {vx, vy, p}
 *                  elastic   {vx, vy, vz, sxx, syy, szz, sxy, sxz, syz}
 *                  elastic2d {vx, vy, sxx, syy, sxy}
 * Material order:  acoustic  {rho, kappa} at p points, kappa = 1/beta
 *                  elastic, elastic2d  {rho, lambda, mu} at cell centres
 * The material is used as fp32 values b = fp32(1/rho), kappa, lambda, mu;
 * staggered buoyancy is the mean of the two adjacent b, the shear modulus on
 * an edge the mean of the four adjacent mu (2D elastic: fp32 of the fp64
 * mean; lambda + 2 mu, lambda and the plate modulus likewise rounded once
 * from fp64).  dt and dx enter through the stencil weights
 * w_k = fp32(c_k * (dt/dx)).
 *
 * Memory.  The library allocates no device memory.  The caller provides one
 * device buffer (the arena) per plan, at least hw_footprint() bytes, 256-byte
 * aligned, which must outlive the plan; the plan carves fields, compensation
 * terms, material, energy trace and a staging area out of it.  Host arrays
 * passed to the library are read or written during the call or, for the
 * *_async-style calls on a stream, until that stream has been synchronised.
 * Streams are hipStream_t handles passed as void* (NULL = the null stream).
 *
 * Errors.  Every call returns an hw_status; on failure nothing observable has
 * changed unless stated, and hw_last_error() returns a message for the
 * calling thread.  No call throws or aborts.
 */
#ifndef HALFWAVE_H
#define HALFWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HW_ABI_VERSION 6u

typedef enum hw_status {
    HW_OK = 0,
    HW_E_INVAL = 1,      /* bad argument, size or enum                       */
    HW_E_UNSTABLE = 2,   /* Courant number at or above the stability bound   */
    HW_E_RANGE = 3,      /* a value does not fit the storage format          */
    HW_E_NOMEM = 4,      /* arena or energy trace too small                  */
    HW_E_DEVICE = 5,     /* a HIP call failed                                */
    HW_E_NONFINITE = 6,  /* the state became inf/NaN (sticky, see below)     */
    HW_E_STATE = 7       /* call out of order (e.g. advance before upload)   */
} hw_status;

enum hw_physics { HW_ACOUSTIC2D = 0, HW_ELASTIC3D = 1, HW_ELASTIC2D = 2 };
enum hw_storage { HW_F32 = 0, HW_F16 = 1, HW_BF16 = 2 };
/* HW_COMP_TWOSUM8: the 6-operation sum with the compensation term held in
 * an 8-bit word instead of a value of the storage format: the TwoSum error t
 * of the new value s (|t| <= ulp(s)/2, ulp the spacing of s's binade) is
 * kept as q = round(t / ulp(s) * 2^7), ties to even, and read back as
 * q * ulp(s) / 2^7 -- 3 bytes of state per field and cell instead of 4.
 * Acoustic plans with fp16 or bf16 storage only. */
enum hw_comp { HW_COMP_NONE = 0, HW_COMP_FAST2SUM = 1, HW_COMP_TWOSUM = 2,
               HW_COMP_TWOSUM8 = 3 };
/* Precision of the stencil arithmetic (spatial differences, staggered
 * material, scaling by the material); the solution update is always in the
 * storage format.  HW_STENCIL_F32, the default, computes in fp32 from the
 * stored values.  HW_STENCIL_STORAGE computes every operation in the storage
 * format with the weights and the material rounded to it first (the
 * all-fp16 step of Alg. 1 read literally).  HW_STENCIL_F64 computes in fp64
 * from the stored values and the fp32 weights and material, rounding the
 * increment once into the storage format (the promoted stencil of App. B).
 * Non-default stencils are acoustic only. */
enum hw_stencil { HW_STENCIL_F32 = 0, HW_STENCIL_STORAGE = 1, HW_STENCIL_F64 = 2 };

typedef struct hw_problem {
    uint32_t abi_version;  /* must be HW_ABI_VERSION                          */
    int32_t physics;       /* enum hw_physics                                 */
    int32_t order;         /* spatial order: 2 or 4 (acoustic), 2 (elastic)   */
    int32_t storage;       /* enum hw_storage: format of fields and comps     */
    int32_t comp;          /* enum hw_comp: update of Alg. 1 or Alg. 2        */
    int32_t scale_log2;    /* fields are held multiplied by 2^scale_log2, to
                              keep them inside the storage range (Sec. 5);
                              results are returned unscaled. |.| <= 60       */
    int64_t nx, ny, nz;    /* cells per axis, >= 1; nz must be 1 for 2D       */
    double dx;             /* grid spacing, all axes, > 0                     */
    double dt;             /* time step, > 0                                  */
    int64_t trace_cap;     /* energy samples reserved in the arena, >= 0      */
    /* Point source and receivers (acoustic and 2D elastic; 0 for 3D): */
    int64_t src_cap;       /* source samples reserved in the arena, >= 0      */
    int32_t rec_cap;       /* receivers reserved, 0 .. 64                     */
    int32_t stencil;       /* enum hw_stencil (acoustic only; 0 for elastic)  */
    int64_t rec_steps;     /* receiver trace rows reserved, >= 0              */
} hw_problem;

typedef struct hw_plan hw_plan;

/* Version of the ABI the library implements (HW_ABI_VERSION). */
uint32_t hw_abi_version(void);

/* Message describing the last failure on the calling thread ("" if none). */
const char *hw_last_error(void);

/* Number of fields (3 acoustic, 9 elastic, 5 elastic2d) and material
 * arrays (2, 3, 3). */
int32_t hw_num_fields(int32_t physics);
int32_t hw_num_materials(int32_t physics);

/* Device bytes a plan for *pb needs.  Host only; works without a GPU.
 * HW_E_INVAL for an invalid problem. */
hw_status hw_footprint(const hw_problem *pb, size_t *device_bytes);

/* Stability bound on the Courant number c_eff*dt/dx for this physics and
 * order: 1/sqrt(2) (2D, order 2, acoustic or elastic), 1/(sqrt(2)*(9/8+1/24))
 * (2D, order 4), 1/sqrt(3) (3D).  Returns a negative value for invalid arguments. */
double hw_cfl_bound(int32_t physics, int32_t order);

/* Create a plan: validate *pb and carve the arena.  Host only, no HIP call.
 * arena: device pointer, 256-byte aligned, arena_bytes >= hw_footprint().
 * *out is written only on success; the plan borrows the arena. */
hw_status hw_plan_create(const hw_problem *pb, void *arena, size_t arena_bytes,
                         hw_plan **out);

/* Destroy a plan (releases host-side objects only; never frees the arena).
 * Waits for nothing: the caller must not destroy a plan with work in flight. */
void hw_plan_destroy(hw_plan *plan);

/* Upload the material: hw_num_materials() host fp64 arrays, in the material
 * order above, each of nx*ny*nz values.  Validates on the host first: all
 * values finite, rho > 0, kappa > 0 (acoustic), mu > 0 and
 * 3 lambda + 2 mu > 0 (elastic), mu > 0 and lambda + mu > 0 (elastic2d),
 * the fp32 values finite, and the Courant
 * number below hw_cfl_bound() (HW_E_INVAL / HW_E_UNSTABLE).  The Courant
 * number uses, for every cell face, the staggered buoyancy of the face times
 * the larger modulus (kappa, or lambda + 2 mu) of the two cells it joins.
 * Then copies and converts on `stream`. */
hw_status hw_set_material(hw_plan *plan, const double *const *material,
                          void *stream);

/* Upload the initial state: hw_num_fields() host fp64 arrays in the field
 * order above (a NULL entry means all zeros).  Each value times
 * 2^scale_log2 must be finite and within the storage format's largest
 * finite value (HW_E_RANGE); it is rounded to nearest-even.  2D elastic:
 * syy on rows 0 and ny-1 and vy, sxy on row ny-1 must be zero (HW_E_INVAL).
 * Compensation terms, step counter and energy trace are reset.  Async on
 * `stream`. */
hw_status hw_set_fields(hw_plan *plan, const double *const *fields,
                        void *stream);

/* Advance nsteps >= 0 leapfrog steps (Alg. 1 or 2 per the plan).  If
 * energy_every > 0, the energy is appended to the trace for every state
 * whose step count is a multiple of energy_every (including the starting
 * state, unless already recorded).  HW_E_NOMEM if the trace would overflow
 * (nothing is launched then).  Async on `stream`. */
hw_status hw_advance(hw_plan *plan, int64_t nsteps, int64_t energy_every,
                     void *stream);

/* Append the energy of the current state to the trace.  Async.  The energy
 * (fp64, of the stored state (v^{n-1/2}, p^n)):
 *   acoustic  E = dx^2/2 * sum[ p^2/kappa + vx^- vx^+ / bx + vy^- vy^+ / by ]
 *   elastic   E = dx^3/2 * sum[ v^- . v^+ / b + s_n^T C^-1 s_n + s_ij^2/mu_ij ]
 *   elastic2d E = dx^2/2 * sum_i[ sum_j h_j (vx^- vx^+ / bx + s_n^T C^-1 s_n)
 *                                + sum_{j<ny-1} (vy^- vy^+ / by + sxy^2/mu_xy) ]
 * where v^+ = v^- + b * (stencil of p or div sigma) is recomputed in fp64,
 * C = lambda 1 1^T + 2 mu I acts on the normal stresses (2D elastic: the
 * 2x2 [[l2m, lam], [lam, l2m]] with l2m = lambda + 2 mu and lam = lambda,
 * on the surface rows l2m = the plate modulus and lam = 0), h_j = 1/2 on
 * the two surface rows and 1 elsewhere; this energy is conserved exactly by
 * the scheme in exact arithmetic.  A non-finite
 * energy sets the plan's sticky HW_E_NONFINITE, reported by hw_energy_trace
 * and hw_get_fields. */
hw_status hw_record_energy(hw_plan *plan, void *stream);

/* Copy the energy trace to the host: energy[k] and step[k] (either may be
 * NULL) for k < min(cap, count); *n_out = count.  Synchronises `stream`. */
hw_status hw_energy_trace(hw_plan *plan, double *energy, int64_t *step,
                          int64_t cap, int64_t *n_out, void *stream);

/* Copy the state to the host as fp64 (exact widening, unscaled): fields and,
 * if comps is non-NULL, the compensation terms (zeros for HW_COMP_NONE),
 * both in the field order.  NULL entries are skipped.  Synchronises. */
hw_status hw_get_fields(hw_plan *plan, double *const *fields,
                        double *const *comps, void *stream);

/* Point source on the pressure (the s_p term of Eq. 1, Sec. 3; the source
 * line of Alg. 1/2).  In the plan's step n (advancing the state from step n
 * to n+1, n counted from the last hw_set_fields or the imported step), the
 * pressure right-hand side at cell (ix, iy) -- the sum of the two stencil
 * terms -- gets samples[n] added before the multiplication by kappa, for
 * 0 <= n < nsamples; the sample is rounded to fp32 like the rest of the
 * stencil arithmetic.  samples: nsamples host fp64 values (already scaled
 * by 2^scale_log2 if the plan uses a field scale).  nsamples = 0 removes the
 * source.  The sample is rounded to fp32 on the host (and to the storage
 * format inside the step when the plan's stencil is HW_STENCIL_STORAGE).
 * A plan with a source or receivers steps on its hw_plan_set_tile shape if
 * that is a two-step shape (kinds 4 and 5, which compile the same source
 * and recording code), else on kernel shape 0; a plan with a non-default
 * stencil steps on shape 0 whatever its setting (the shapes give identical
 * bits).
 * 2D elastic plans: the source acts on vy at (ix, iy+1/2), 0 <= iy <= ny-2
 * (the s^{vy} term of Eq. A1): the sample is added to the velocity
 * increment after the multiplication by the staggered buoyancy.
 * HW_E_INVAL for 3D elastic plans or a cell outside the grid,
 * HW_E_NOMEM if nsamples > src_cap.  Synchronises `stream` (the samples are
 * copied before the call returns). */
hw_status hw_set_source(hw_plan *plan, int64_t ix, int64_t iy,
                        const double *samples, int64_t nsamples, void *stream);

/* Receivers: after each step n < rec_steps the new pressure p^{n+1} and
 * velocities vx^{n+1/2}, vy^{n+1/2} (2D elastic: the five new fields) at
 * each of the n cells (ix[r], iy[r]) are recorded in fp64 (exact widening,
 * unscaled); row n of the trace
 * belongs to step n, counted as for hw_set_source.  0 <= n <= rec_cap
 * (HW_E_NOMEM), cells inside the grid (HW_E_INVAL).  n = 0 removes the
 * receivers.  Synchronises `stream`. */
hw_status hw_set_receivers(hw_plan *plan, int32_t n, const int64_t *ix,
                           const int64_t *iy, void *stream);

/* Copy the receiver trace to the host: out[(k*n + r)*m + {0, 1, 2}] =
 * (p, vx, vy) of receiver r after step k (m = 3; 2D elastic: m = 5 values
 * in the field order), for k < min(cap_rows, rows), n the receiver count;
 * *rows_out = rows recorded (min(step, rec_steps)).
 * Synchronises `stream`. */
hw_status hw_receiver_trace(hw_plan *plan, double *out, int64_t cap_rows,
                            int64_t *rows_out, void *stream);

/* Current step count of the plan. */
int64_t hw_plan_step(const hw_plan *plan);

/* Checkpoint: the state (fields, compensation terms, step count) as an
 * opaque byte blob; importing it into a plan of the same problem and
 * continuing gives bit-identical results to never having stopped.  Equal
 * states export equal blobs, whatever the arenas held before (the row
 * padding inside the blob is always zero).  The energy trace is not part of
 * the blob.  Both synchronise `stream`. */
hw_status hw_state_size(const hw_plan *plan, size_t *bytes);
hw_status hw_state_export(hw_plan *plan, void *blob, size_t bytes,
                          void *stream);
hw_status hw_state_import(hw_plan *plan, const void *blob, size_t bytes,
                          void *stream);

/* Kernel shapes the library was built with, by index.  tx by ty cells of
 * a plane per workgroup; tz planes per workgroup; kind:
 *   acoustic2d  0 = one tile per workgroup (4 wavefronts), 3 = the same
 *               with 8 wavefronts, 1 = a workgroup marches down a strip ty
 *               rows tall; 4 and 5 = two time steps per launch (4 and 8
 *               wavefronts; tz = 2): a workgroup advances its tile by two
 *               steps in one pass over memory, recomputing the cells around
 *               it that the second step needs (an odd step left over runs
 *               on shape 0);
 *   elastic3d   0 = two passes per step (velocities, then stresses), one
 *               plane per workgroup; 2 = one fused pass per step, a
 *               workgroup walks a tx by ty column through tz planes;
 *   elastic2d   1 = one fused pass per step (each thread recomputes the
 *               neighbouring new velocities its stresses read), 0 = two
 *               passes (velocities, then stresses); one tx by ty tile per
 *               workgroup.
 * hw_plan_set_tile picks one for a plan; every shape gives bit-identical
 * results.  A new plan runs shape 0; the faster shapes are picked per size
 * by the Python package's tuning table (for acoustic2d the two-step kinds
 * at every size measured).  hw_simulate and hw_simulate_noalloc run the
 * two-step 64 x 24 shape (acoustic2d), the fused 64 x 6 x 128 shape
 * (elastic3d) or shape 0 (elastic2d).  Plans with HW_COMP_TWOSUM8
 * take every kind but 1 (HW_E_INVAL);
 * in hw_batch_advance a kind-1 tile argument runs their group on shape 0.
 * Any of the output pointers may be NULL. */
int32_t hw_tile_count(int32_t physics);
hw_status hw_tile_info(int32_t physics, int32_t tile, int32_t *tx,
                       int32_t *ty, int32_t *tz, int32_t *kind);
hw_status hw_plan_set_tile(hw_plan *plan, int32_t tile);

/* Advance n plans (0 < n) by nsteps[i] steps each, batching all plans with
 * the same physics, order, storage and compensation into one launch per
 * time step that covers every tile of every such plan still running (2D
 * elastic plans: their launches per step, one plan after another, captured
 * into the same graph).  Each
 * plan's results (fields, comps, energy trace) are bit-identical to
 * hw_advance(plan, nsteps[i], energy_every) on it alone.  Plans are
 * borrowed and must be distinct.  tile >= 0 selects the kernel shape (as
 * hw_tile_info; it must exist for every plan's physics, else HW_E_INVAL),
 * -1 gives each group the shape set on its first plan.  Async. */
hw_status hw_batch_advance(hw_plan *const *plans, int32_t n,
                           const int64_t *nsteps, int64_t energy_every,
                           int32_t tile, void *stream);

/* Blocking convenience: create a plan in the arena, upload material and
 * fields, advance nsteps with the energy every energy_every steps, download
 * the fields into the same arrays (fields must be non-NULL host arrays) and
 * copy up to energy_cap energies.  *n_energy receives the trace length.
 * The plan runs the shape stated above hw_tile_count. */
hw_status hw_simulate(const hw_problem *pb, const double *const *material,
                      double *const *fields, int64_t nsteps,
                      int64_t energy_every, double *energy, int64_t energy_cap,
                      int64_t *n_energy, void *arena, size_t arena_bytes,
                      void *stream);

/* Largest device footprint (hw_footprint) hw_simulate_noalloc accepts. */
#define HW_NOALLOC_MAX_BYTES (64u << 20)

/* For callers that cannot allocate device memory (no hipMalloc, no torch
 * allocator: tight serving loops, harnesses that forbid allocation): the
 * same computation as hw_simulate, with the same arguments except the
 * arena.  The plan lives in a statically allocated device array of
 * HW_NOALLOC_MAX_BYTES bytes, one per GPU, held by the library from its
 * first use on that GPU until the process ends; the call runs on the
 * calling thread's current device (`stream` must belong to it), allocates
 * no device memory and creates no stream, event or graph (every step is
 * launched directly on `stream`).  Problems whose hw_footprint exceeds
 * HW_NOALLOC_MAX_BYTES get HW_E_NOMEM before any device work.  Everything
 * the kernels read is written by the call itself first, so a call does not
 * depend on what an earlier one left in the array.  All calls on one GPU
 * share that array: calls that overlap in time on the same GPU (from
 * several threads, or on streams that are not synchronised with each
 * other) race and give undefined results.  The call synchronises `stream`
 * before it returns, so sequential calls never overlap. */
hw_status hw_simulate_noalloc(const hw_problem *pb, const double *const *material,
                              double *const *fields, int64_t nsteps,
                              int64_t energy_every, double *energy,
                              int64_t energy_cap, int64_t *n_energy,
                              void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HALFWAVE_H */
