/*
 * ch.h -- C ABI of libch: the Cahn-Hilliard scalar update of the phase-field
 * method of Liu, Ng, Chong, Lohse & Verzicco (arXiv 2105.01865) on one
 * AMD Instinct MI355X (gfx950).
 *
 * One step advances the volume fraction C of eq-ch (sec. 2.1),
 *
 *   dC/dt + div(u C) = (1/Pe) [ -Cn^2 lap^2 C + lap psi'(C) ],
 *
 * on a uniform cell-centred mesh of spacing h with a prescribed staggered
 * face velocity (u, v, w), using
 *   - fifth-order WENO face values for the conservative advection flux
 *     (sec. 3),
 *   - the central 7-point Laplacian of psi'(C) (sec. 3),
 *   - the new biharmonic scheme of sec. 3.1 without mixed derivatives,
 *     sum_d A_d C with A_d = kappa Cn^2/h^4 (1,-4,6,-4,1)_d (eq-divbi,
 *     eq-a3d; kappa = 4 as printed for 3-D),
 *   - a low-storage third-order Runge-Kutta scheme with Crank-Nicolson on
 *     the biharmonic term in delta form (eq-re), approximately factorised
 *     (eq-fac) into three pentadiagonal line solves along x, y, z
 *     (eq-fac-1 .. eq-fac-3).
 *
 * RK3 substage k = 1, 2, 3 with gamma = (8/15, 5/12, 3/4), rho = (0, -17/60,
 * -5/12), alpha = gamma + rho:
 *   E_k   = -div(u C) + lap psi'(C) / Pe
 *   rhs   = dt (gamma_k E_k + rho_k E_{k-1}) - alpha_k dt / Pe sum_d A_d C
 *   (I + alpha_k dt/(2 Pe) A_x)(I + alpha_k dt/(2 Pe) A_y)
 *       (I + alpha_k dt/(2 Pe) A_z) dC = rhs ;   C += dC
 *
 * Memory: every field is x-fastest, C[z][y][x].  Face i along an axis is the
 * low face of cell i.  A periodic axis of n cells has n faces along it (face
 * n is face 0); a no-flux axis has n + 1 (the first and last are the walls,
 * where the normal velocity must be zero).  So u is [nz][ny][fx],
 * v is [nz][fy][nx], w is [fz][ny][nx] with f = n or n + 1.
 *
 * Precision: CH_FP64 stores and computes in double; CH_FP32 stores and
 * computes C, E and the stencils in float, while the mass is always summed
 * in double and the line-solve recurrences use double when the solve's
 * diagonal dominance is weak (solve_fp64 = CH_SOLVE_AUTO) or always
 * (CH_SOLVE_FP64).
 *
 * Streams: all work is enqueued on the state's HIP stream (default: the
 * null stream); calls return once the work is enqueued, except ch_mass,
 * ch_get_field and ch_batch_mass, which wait for it.
 *
 * Errors: every call returns a ch_status; ch_last_error() gives a
 * thread-local message for the last failure.  Handles are checked: a call on
 * a destroyed or foreign handle returns CH_EHANDLE.
 */
#ifndef CH_H
#define CH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CH_OK = 0,
    CH_EINVAL = -1,        /* invalid argument */
    CH_ENOMEM = -2,        /* device or host allocation failed */
    CH_EHIP = -3,          /* a HIP runtime call failed */
    CH_EUNSUPPORTED = -4,  /* valid request outside what the library supports */
    CH_ENONFINITE = -5,    /* NaN or Inf found by a checking call */
    CH_EHANDLE = -6        /* handle not live (destroyed or never created) */
} ch_status;

enum { CH_PERIODIC = 0, CH_NOFLUX = 1 };
enum { CH_FP64 = 0, CH_FP32 = 1 };
enum { CH_SOLVE_AUTO = 0, CH_SOLVE_FP64 = 1, CH_SOLVE_NATIVE = 2 };

/* Uniform mesh: n_x x n_y x n_z cells of width h (sec. 3: uniform h in all
 * three directions for C).  Each n is 1 (a degenerate axis: no variation,
 * no flux, the solve along it is the identity) or at least 8. */
typedef struct {
    int64_t nx, ny, nz;
    double h;
} ch_grid;

/* psi'(C) = c[0] + c[1] C + c[2] C^2 + c[3] C^3; the double well of eq-ch,
 * psi = C^2 (C-1)^2 / 4, is {0, 0.5, -1.5, 1}. */
typedef struct {
    double c[4];
} ch_psi;

/* Boundary per axis: CH_PERIODIC, or CH_NOFLUX (even reflection of C across
 * the wall and zero normal velocity on it; the paper leaves the first and
 * last operator rows to the boundary condition, after eq-a2d). */
typedef struct {
    int x, y, z;
} ch_bc;

typedef struct {
    int precision;      /* CH_FP64 (default) or CH_FP32 */
    double kappa;       /* weight of the per-direction fourth difference; 4 */
    double weno_eps;    /* WENO regularisation; 1e-6 */
    int solve_fp64;     /* CH_SOLVE_AUTO (default), CH_SOLVE_FP64, CH_SOLVE_NATIVE */
    int use_graph;      /* 1 (default): replay each step as one HIP graph */
    int x_rows;         /* rows per x-pass work-group; 0 = automatic */
    int seg_len;        /* y/z line segment per work-group; 0 = automatic */
    int waves_yz;       /* waves per y/z work-group (1..8); 0 = automatic */
    int z_chunk;        /* planes one x-pass work-group marches over; 0 = automatic */
    int x_general;      /* 1: always run the general x-pass program; 0 (default):
                           the one-row program wherever a task holds one x-line
                           (the same arithmetic; a tuning and testing knob) */
    double dt_hint;     /* > 0: plan the line-solve recurrences and launches for
                           this dt at creation (a dt the solver cannot take is
                           then reported by the create call, and a first step
                           with this dt does no planning); 0 (default): plan
                           at the first step.  Negative or non-finite:
                           CH_EINVAL. */
} ch_opts;

typedef struct ch_state ch_state;
typedef struct ch_batch ch_batch;
typedef struct ch_interp ch_interp;
typedef struct ch_poisson ch_poisson;

/* Fill *opt with the defaults above. */
void ch_default_opts(ch_opts* opt);

/* Create a single-box state.  Cn, Pe > 0 (eq-ch); psi NULL = double well;
 * bc NULL = periodic everywhere; opt NULL = defaults.  The state owns C, the
 * explicit-term history E and two line-solve buffers on the current device.
 * C starts at zero.  Errors: CH_EINVAL (bad sizes, h, Cn, Pe, kappa, eps),
 * CH_ENOMEM, CH_EHIP. */
ch_status ch_create(const ch_grid* g, double Cn, double Pe, const ch_psi* psi,
                    const ch_bc* bc, const ch_opts* opt, ch_state** out);

/* Use the given HIP stream (hipStream_t; NULL = null stream) for all work. */
ch_status ch_set_stream(ch_state* s, void* stream);

/* Copy C in / out: nx*ny*nz values in the state's precision, x fastest.
 * on_device = 1: C is device memory; 0: host memory (pinned memory copies
 * fastest).  ch_get_field always waits for the copy; ch_set_field waits when
 * C is host memory, so the host buffer may be reused on return, and only
 * enqueues a device-to-device copy.  Errors: CH_EINVAL (null pointer),
 * CH_EHIP, CH_EHANDLE. */
ch_status ch_set_field(ch_state* s, const void* C, int on_device);
ch_status ch_get_field(ch_state* s, void* C, int on_device);

/* Enqueue nsteps RK3 steps with the frozen face velocity (u, v, w): borrowed
 * device pointers in the state's precision with the shapes given above; the
 * caller keeps them alive until the stream has passed the work.  dt > 0 and
 * finite, nsteps >= 0.  Errors: CH_EINVAL, CH_EHIP, CH_EHANDLE. */
ch_status ch_step(ch_state* s, const void* u, const void* v, const void* w,
                  double dt, int nsteps);

/* Enqueue nsteps RK3 steps of the explicit 25-point scheme the paper starts
 * from (sec. 3.1, eq-disbi in three dimensions): no Crank-Nicolson and no
 * line solves, every term advanced by the low-storage RK3 (sec. 2):
 *   N_k = -div(u C) + lap psi'(C)/Pe - B(C)/Pe,
 *   B   = Cn^2/h^4 [ sum_d (1,-4,6,-4,1)_d + 2 sum_{d<e} (1,-2,1)_d (1,-2,1)_e ] C,
 *   C  += dt (gamma_k N_k + rho_k N_{k-1}),
 * the full 25-point discrete biharmonic with its mixed terms (kappa is not
 * used).  Stable only below the explicit limit, about
 * dt < 2.51 Pe h^4 / (144 Cn^2) for the biharmonic's highest mode, which is
 * what the paper's implicit scheme removes.  Same arguments, layout and
 * errors as ch_step; the state's buffers are reused (C and a solve buffer
 * trade places each substage), so a later ch_step re-plans. */
ch_status ch_step_explicit25(ch_state* s, const void* u, const void* v, const void* w,
                             double dt, int nsteps);

/* Mass h^3 sum C in double, summed in a fixed order (the quantity behind
 * the mass-loss measure of sec. 4.3.1).  Waits for the stream. */
ch_status ch_mass(ch_state* s, double* out);

/* Allocation-free mass of a field, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same fixed-order FP64 sum h^3 sum C as ch_mass
 * (the same bits for the same field), of the field C (device memory,
 * [nz][ny][nx] x-fastest, FP64 or FP32 by `precision`), written as one
 * double to out_dev (device memory) on `stream` (a hipStream_t; NULL is the
 * null stream).  It enqueues two kernels and returns without waiting; it
 * calls no allocating routine.  The partial sums live in one library-wide
 * device array of 2^20 doubles (8 MiB, held per GPU until the process
 * ends), so a field has at most 2^32 cells (CH_EINVAL beyond).  Calls that
 * overlap on one GPU (different streams, or threads) share that array and
 * race: order them on one stream.  Errors: CH_EINVAL (null pointer, an
 * extent < 1, h <= 0 or non-finite, unknown precision, too many cells),
 * CH_EHIP. */
ch_status ch_mass_field_noalloc(const void* C, int64_t nx, int64_t ny, int64_t nz, double h,
                                int precision, void* stream, double* out_dev);

/* Check the velocity: finite everywhere and zero on no-flux walls.  Waits.
 * Returns CH_OK, CH_ENONFINITE or CH_EINVAL. */
ch_status ch_check_velocity(ch_state* s, const void* u, const void* v, const void* w);

/* Free everything the state owns.  NULL is accepted. */
void ch_destroy(ch_state* s);

/* Thread-local message of the last failed call ("" if none). */
const char* ch_last_error(void);

/* ---- batched ensemble: independent boxes advanced together -------------
 * Box b has grid g[b], Cn[b], Pe[b], psi[b] (NULL = double well for all),
 * bc[b] (NULL = periodic for all); opt applies to all boxes.  Fields are
 * packed: box b's C starts at element c_off[b] of the packed array, its
 * u, v, w at u_off[b], v_off[b], w_off[b] of theirs (see
 * ch_batch_field_offsets).  One step of all boxes is one HIP graph launch. */
ch_status ch_batch_create(int nbox, const ch_grid* g, const double* Cn, const double* Pe,
                          const ch_psi* psi, const ch_bc* bc, const ch_opts* opt,
                          ch_batch** out);
/* Offsets (elements) of each box in the packed C, u, v, w arrays, and the
 * four packed lengths in totals[4]; any pointer may be NULL. */
ch_status ch_batch_field_offsets(const ch_batch* b, int64_t* c_off, int64_t* u_off,
                                 int64_t* v_off, int64_t* w_off, int64_t totals[4]);
ch_status ch_batch_set_stream(ch_batch* b, void* stream);
/* Copy the packed C (totals[0] values) in / out; on_device and waiting as
 * for ch_set_field / ch_get_field. */
ch_status ch_batch_set_field(ch_batch* b, const void* C_packed, int on_device);
ch_status ch_batch_get_field(ch_batch* b, void* C_packed, int on_device);
ch_status ch_batch_step(ch_batch* b, const void* u_packed, const void* v_packed,
                        const void* w_packed, double dt, int nsteps);
/* Per-box mass h_b^3 sum C_b into out[nbox]; waits. */
ch_status ch_batch_mass(ch_batch* b, double* out);
void ch_batch_destroy(ch_batch* b);

/* ---- multiple-resolution velocity (sec. 3.4) -----------------------------
 * The velocity lives on a coarse mesh, ncx x ncy cells uniform and periodic
 * in x and y, ncz cells between walls at z = 0 and 1 with face positions
 * zf[0..ncz] (host array, increasing, zf[0] = 0, zf[ncz] = 1); it is
 * transferred to the faces of the fine uniform mesh of `fine` (periodic x,
 * y; no-flux z) by tensor-product cubic Hermite interpolation with four
 * points per direction (slopes: chord through the two neighbours; beyond a
 * wall the tangential components continue evenly, the normal one oddly).
 * The 1-D stencils are built once at creation; the coarse mesh needs at
 * least 4 cells per axis and at most 8192 along x in single precision,
 * 4096 in double (CH_EINVAL / CH_EUNSUPPORTED otherwise).  Coarse arrays: uc, vc
 * [ncz][ncy][ncx], wc [ncz+1][ncy][ncx]; fine: u, v [nz][ny][nx],
 * w [nz+1][ny][nx]; all device memory in the given precision. */
ch_status ch_interp_create(const ch_grid* fine, int64_t ncx, int64_t ncy, int64_t ncz,
                           const double* zf, int precision, ch_interp** out);
ch_status ch_interp_set_stream(ch_interp* ip, void* stream);
ch_status ch_interp_apply(ch_interp* ip, const void* uc, const void* vc, const void* wc,
                          void* u, void* v, void* w);
void ch_interp_destroy(ch_interp* ip);

/* Solenoidal mode of the transfer (sec. 3.4: the normal velocity gradients
 * are interpolated instead of the velocity, then integrated from a 2-D
 * reference plane).  With `on` set, ch_interp_apply and ch_step_multires
 * form the coarse cell-centred gradients (u[i+1]-u[i]) ncx,
 * (v[j+1]-v[j]) ncy and (w[k+1]-w[k]) / (zf[k+1]-zf[k]), take all three to
 * the fine cell centres with one and the same interpolant (so that their
 * sum is the interpolated coarse divergence), and integrate each component
 * along its direction:  u[i] = u_ref + (1/nx) sum_{i'<i} G_x[i'] from the
 * x = 0 face (u_ref: the plain transfer on that face), v likewise from the
 * y = 0 face, w from 0 on the bottom wall; the top wall stays 0.  A coarse
 * field that is discretely divergence-free then gives a fine field that is
 * too in every cell but the last of each line, where the line's closure sum
 * is left (see ch_interp_closure).  Switching allocates (on) or frees (off)
 * one coarse field, one reference plane and small tables; it waits for the
 * handle's stream.  Switching makes step graphs captured with the old mode
 * stale (they are re-captured).  CH_ENOMEM if the buffers cannot be had. */
ch_status ch_interp_set_solenoidal(ch_interp* ip, int on);

/* Largest |closure sum| (velocity units) over the x, y and z lines of the
 * last solenoidal transfer enqueued on the handle: out[d] = max over lines
 * of |h sum G_d|, zero when the mode is off.  Waits for the stream. */
ch_status ch_interp_closure(ch_interp* ip, double out[3]);

/* Back-coupling of C (sec. 3.4): the fine cell-centred field Cf
 * [nz][ny][nx] interpolated to the coarse cell centres, Cc [ncz][ncy][ncx]
 * (the same interpolant; C continues evenly beyond the walls).  Device
 * memory in the handle's precision, on the handle's stream.  CH_EUNSUPPORTED
 * when the fine x extent is too long for the kernel's LDS rows (above 8192
 * in single precision or 4096 in double, or fewer when the y ratio is
 * large). */
ch_status ch_interp_project_c(ch_interp* ip, const void* Cf, void* Cc);

/* nsteps steps where every step first transfers the coarse velocity to the
 * fine faces (into buffers the state allocates on first use) and then
 * advances C by one RK3 step. */
ch_status ch_step_multires(ch_state* s, ch_interp* ip, const void* uc, const void* vc,
                           const void* wc, double dt, int nsteps);

/* ---- split-density pressure step (sec. 3.2: eq-poi, eq-split, eq-newpoi,
 * eq-u) --------------------------------------------------------------------
 * The pressure projection of the coupled solver on the uniform staggered
 * mesh of the CH field: P and C at the nx x ny x nz cell centres (spacing
 * h, x fastest), u / v / w on the low faces of the cells, periodic in x and
 * y; z periodic (z_walls = 0: w has nz planes) or between two walls
 * (z_walls = 1: w has nz + 1 planes, zero on both walls, dP/dz = 0 there).
 * The density is rho = rho2 + (rho1 - rho2) clamp(C, 0, 1) (rho2 <= rho1),
 * taken on a face as the mean of its two cells.  Creation makes the hipFFT
 * plans and the work arrays (three fields and a spectrum); nx, ny, nz >= 2
 * (CH_EINVAL), fewer than 2^31 cells and planes (nx ny) under 4 GiB
 * (CH_EUNSUPPORTED).  Device memory in
 * the given precision; work is enqueued on the handle's stream.
 *
 * ch_poisson_solve: P with lap P = rhs - mean(rhs) and zero mean, for the
 * 7-point Laplacian of these face differences (transforms in x and y; along
 * z a tridiagonal solve per mode between walls, the 3-D transform when
 * periodic).  rhs is not modified.
 *
 * ch_pressure_step: with P = P^l, Pold = P^{l-1} and u, v, w = u*:
 *   Phat = 2 P^l - P^{l-1};
 *   lap P^{l+1} = div[(1 - rho2/rho) grad Phat] + (rho2/dt) div u*;
 *   u^{l+1} = u* - dt [grad P^{l+1} / rho2 + (1/rho - 1/rho2) grad Phat];
 * on return P = P^{l+1}, Pold = P^l and u, v, w = u^{l+1} (the wall planes of
 * w are not written).  The new velocity is discretely divergence-free for
 * any density and pressure history.  CH_EINVAL unless 0 < rho2 <= rho1 and
 * dt > 0. */
ch_status ch_poisson_create(const ch_grid* g, int z_walls, int precision, ch_poisson** out);
ch_status ch_poisson_set_stream(ch_poisson* p, void* stream);
ch_status ch_poisson_solve(ch_poisson* p, const void* rhs, void* P);
ch_status ch_pressure_step(ch_poisson* p, const void* C, double rho1, double rho2, double dt,
                           void* u, void* v, void* w, void* P, void* Pold);
void ch_poisson_destroy(ch_poisson* p);

/* ---- launch-plan autotuning ----------------------------------------------
 * The tiles of the x pass (rows per task, planes per task) are chosen by a
 * heuristic at creation.  ch_autotune / ch_batch_autotune time `steps` RK3
 * steps (1 .. 1000, after one untimed step) of every plan in the candidate
 * set  x_rows in {auto, 1, 2, 4} x z_chunk in {auto, 4, 6, ..., 16, 20, 24}  that
 * the planner admits for dt, then the y / z segment lengths {auto, 128, 64}
 * with the fastest of those, each from the same C with the given velocity
 * (borrowed device pointers, as for ch_step), and keep the fastest as the
 * state's launch options.  C is restored before returning; the call waits
 * for the stream and allocates one copy of C for its duration.  The tuned
 * options stay fixed: a later dt for which they are not admitted fails in
 * ch_step (tune again).  out receives the chosen plan, its ms per step, the
 * automatic plan's ms per step and the number of candidates timed (the
 * automatic plan is also run once first, untimed for the choice, to warm the
 * device up). */
typedef struct {
    int x_rows, z_chunk;
    double ms_per_step, auto_ms_per_step;
    int candidates;
    int seg_len;   /* segment length of the y and z line passes */
} ch_tune;
ch_status ch_autotune(ch_state* s, const void* u, const void* v, const void* w, double dt,
                      int steps, ch_tune* out);
ch_status ch_batch_autotune(ch_batch* b, const void* u, const void* v, const void* w, double dt,
                            int steps, ch_tune* out);

/* ---- drop diagnostics (sec. 4) -------------------------------------------
 * The drops of a box for the drop-size statistics: cells with
 * C >= threshold (the paper's mid-value 1/2; compared in the state's
 * precision) joined through cell faces, across periodic boundaries but not
 * across walls.  Each drop is named by its root, the smallest linear index
 * (x fastest, [z][y][x]) of its cells, and `cells` counts its cells; its
 * volume is V = h^3 cells and its effective diameter D follows from
 * (4 pi / 3)(D/2)^3 = V.  The first min(cap, *ndrops) drops in increasing
 * root order go to the host arrays root[] and cells[]; *ndrops receives
 * the number of drops.  The labelling runs on the state's stream and the
 * call waits for it.  The first call allocates two ints per cell of the box
 * (kept until destroy).  Boxes of 2^31 cells or more: CH_EUNSUPPORTED.
 * ch_batch_drops does the same for box `box` of an ensemble. */
ch_status ch_drops(ch_state* s, double threshold, int64_t cap, int64_t* ndrops, int64_t* root,
                   int64_t* cells);
ch_status ch_batch_drops(ch_batch* b, int box, double threshold, int64_t cap, int64_t* ndrops,
                         int64_t* root, int64_t* cells);

/* ---- measurement ---------------------------------------------------------
 * With profiling on, ch_step / ch_batch_step launch kernels one by one
 * (no graph) and time each launch with HIP events on the state's stream.
 * ch_profile_read returns, for kernel class k (0 = x pass: RHS + x solve,
 * 1 = y solve, 2 = z solve + update, 3 = velocity transfer), the summed
 * milliseconds and the launch count since profiling was switched on.  It
 * waits for the stream. */
ch_status ch_profile_enable(ch_state* s, int on);
ch_status ch_profile_read(ch_state* s, int kernel, double* total_ms, int64_t* launches);
ch_status ch_batch_profile_enable(ch_batch* b, int on);
ch_status ch_batch_profile_read(ch_batch* b, int kernel, double* total_ms, int64_t* launches);

/* Launch configuration the library chose (or was given) for the state at
 * its last time step: cfg[0] = x rows per x-pass work-group, cfg[1] = y/z
 * line segment, cfg[2] = threads per y/z work-group, cfg[3..5] = warm-up
 * length of the line recurrences in substages 1..3 (first box), cfg[6] = 1
 * if the solves run in double, cfg[7] = planes an x-pass work-group marches
 * over. */
ch_status ch_get_config(const ch_state* s, int cfg[8]);

/* Which x-pass program the plan of a state (batch) runs, for reports and
 * tests (the arithmetic is the same in all): *kind = 0 the general program,
 * 1 the row program (one cell per thread, the y stencil in registers), 2 the
 * row program with several rows in some task, 3 the segmented program (x
 * lines longer than a work-group), 4 the row program in two or three
 * launches (a batch whose boxes take different row modes: one row per task,
 * several rows with per-thread row offsets, several rows of whole waves; one
 * launch per mode, each with its own work-group size).  CH_EINVAL before the
 * first plan (no step yet and no dt_hint) or on a null output. */
ch_status ch_get_x_program(const ch_state* s, int* kind);
ch_status ch_batch_get_x_program(const ch_batch* b, int* kind);

#ifdef __cplusplus
}
#endif
#endif /* CH_H */
