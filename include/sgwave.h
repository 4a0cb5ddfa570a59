/*
 * sgwave.h -- C ABI of the MI355X (gfx950) acoustic finite-difference
 * propagator: the seismic-data path of SubsurfaceGen (arXiv 2605.30541).
 *
 * Problem statement followed (Sec. 2 and App. E): a 2D velocity slice on a
 * regular grid, the grid spacing, the time step and the number of steps, a
 * source wavelet with source positions, and receiver positions go in; the
 * wavefield p(x,t) (snapshots) and/or the shot gather R p come out.  The
 * scheme is the constant-density acoustic equation (eq. "acoustic_2d"),
 * 8th order in space and 2nd order in time (Table "params"), with a free
 * surface on top (eq. "free_surface") and a Cerjan sponge on the other three
 * sides (eqs. "cerjan_pde", "cerjan_damp").  The velocity gradient of an L2
 * gather misfit is the exact adjoint of that discrete scheme.
 *
 * Conventions shared by every call
 *   - Arrays are row-major with x fastest: a velocity slice is [nz][nx], a
 *     gather is [nshot][nrows][nrec], snapshots are [nshot][snap_count][nz][nx].
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory read during the call only.
 *   - The caller owns every buffer.  The library owns only plans; it never
 *     allocates or frees device memory.  Scratch device memory is passed in as
 *     a workspace whose size the *_workspace_size calls report.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their work on it and return without waiting for the device.  Host
 *     tables are staged in pinned host memory owned by the plan (four slots
 *     used in turn) and copied to the workspace with hipMemcpyAsync; a slot
 *     is reused only after its previous copy has completed, so the host runs
 *     up to three calls on a plan ahead of the GPU without blocking.  The
 *     slots are sized at sg_plan_create for the forward tables of up to 64
 *     shots and 2 nx receivers; a call needing more grows them once (a
 *     pinned host allocation), which sg_plan_reserve does beforehand.
 *     Calls that share a workspace must be ordered on one stream.
 *   - Inputs are validated before anything is enqueued: on an error return
 *     no output and no workspace byte is touched.  No C++ exception crosses
 *     the ABI.  sg_last_error() returns a thread-local message for the last
 *     failing call on the calling thread.
 *   - Time levels are t_n = n*dt, n = 0..nt-1; the initial state is zero
 *     (App. E.2) so level 0 of every output is exactly 0.
 */
#ifndef SGWAVE_H
#define SGWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_ABI_VERSION 2

typedef int32_t sg_status;
enum {
    SG_OK = 0,
    SG_EINVAL = 1,        /* bad argument, size, pointer or position */
    SG_ECFL = 2,          /* dt above the CFL bound of App. E.3.2 */
    SG_ENOSPACE = 3,      /* workspace smaller than required */
    SG_EHIP = 4,          /* a HIP runtime call failed */
    SG_EDIVERGED = 5,     /* non-finite values found by sg_check_finite */
    SG_EUNSUPPORTED = 6   /* valid but not implemented (e.g. a tuning variant) */
};

/* sg_geometry.top */
enum { SG_TOP_FREE = 0, SG_TOP_ABSORBING = 1 };

/* sg_plan_create flags */
enum { SG_ALLOW_UNSTABLE = 1u << 0 };

/* sg_plan_warnings bits */
enum { SG_WARN_DISPERSION = 1u << 0 };

/*
 * Grid, time axis, boundary and output sampling of one velocity slice.
 *   nz, nx        physical nodes; node (iz,ix) is at z = iz*dz, x = ix*dx [m]
 *   dz, dx, dt    spacing [m] and time step [s]
 *   nt            number of time levels (nt-1 updates); >= 2
 *   nbl           sponge width in cells added left, right, bottom (and top
 *                 when top = SG_TOP_ABSORBING); 0 = rigid p = 0 just outside
 *   top           SG_TOP_FREE (p = 0 at z = 0, App. E.2) or SG_TOP_ABSORBING
 *   damp_R        target reflection coefficient R of eq. "cerjan_damp" (1e-3)
 *   vmax_hint     largest velocity [m/s] used for the CFL check
 *                 dt <= s_max h / v_max, s_max = (sqrt(2 sum|c_m|))^-1 (App. E.3.2)
 *   vmin_hint, fmax_hint   for the dispersion warning h <= v_min/(4 f_max)
 *                 (App. E.3.1); 0 skips it
 *   rec_every     gather rows keep levels n = 0, k, 2k, ... (k >= 1, App. E.3.3)
 *   snap_every, snap_count   snapshots at n = j*snap_every, j < snap_count
 *                 (snap_count 0 = none); (snap_count-1)*snap_every <= nt-1
 */
typedef struct {
    int32_t nz, nx;
    double dz, dx, dt;
    int32_t nt;
    int32_t nbl;
    int32_t top;
    double damp_R;
    double vmax_hint;
    double vmin_hint;
    double fmax_hint;
    int32_t rec_every;
    int32_t snap_every;
    int32_t snap_count;
} sg_geometry;

/*
 * Acquisition of one call (Sec. 2, App. E.5): nshot independent shots, each
 * one point source, and one receiver spread shared by every shot.
 *   src_zx    host [nshot][2] source (z, x) [m] inside the physical grid
 *   rec_zx    host [nrec][2]  receiver (z, x) [m] inside the physical grid
 *   wavelet   device [wavelet_per_shot ? nshot : 1][nt] float source time
 *             functions w(t_n)
 * Off-grid positions use bilinear weights; a point source adds
 * weight * w(t_n) / (dx dz) at its nodes into the step n -> n+1, receivers
 * sample p^n with the same weights.  A node on the free-surface row
 * carries no source (p is pinned to 0 there) and reads 0.
 */
typedef struct {
    int32_t nshot;
    const double *src_zx;
    int32_t nrec;
    const double *rec_zx;
    const float *wavelet;
    int32_t wavelet_per_shot;
} sg_shots;

/*
 * Kernel tuning of the time-stepping launches.
 *   variant      0 = library default; 1 = one launch per time step with the
 *                stencil read from global memory; 2 = LDS-tiled, time-blocked
 *                launches; 3 = column sweep: a workgroup walks a strip of
 *                tile_x columns (128 or 256, 0 = 256) from top to bottom --
 *                the whole height, or one segment of tile_z output rows
 *                (0 = whole height, else >= 8) -- advancing time_block (1..6,
 *                0 = 4) levels in a skewed pipeline, so only the x halo of
 *                4*time_block per side (and 4*time_block + 4 rows above a
 *                segment) is recomputed (forward calls with dz == dx; the
 *                gradient calls run variant 2 instead); rows_per_thread is 0
 *   tile_x, tile_z   cells (x by z) of the LDS tile one workgroup loads
 *                (variant 2), one of the built shapes 128x64, 64x128, 64x64;
 *                the output tile is that minus a halo of 4*time_block per side
 *                (under a free top the top tile row trades halo for ghost rows)
 *   time_block   time steps per launch (variant 2), 1..8; 0 = 4 for forward
 *                calls, 3 for the gradient calls (sg_forward_ckpt,
 *                sg_adjoint_gradient, sg_batch_adjoint_gradient)
 *   rows_per_thread   rows of the tile column each thread keeps in registers
 *                (variant 2): 8 or 16 for 128x64, 16 for 64x128, 8 for 64x64;
 *                0 = the first built one
 * All zeros ask for the library's default.  sg_plan_set_tuning rejects
 * shapes that are not built with SG_EUNSUPPORTED.
 */
typedef struct {
    int32_t variant;
    int32_t tile_x;
    int32_t tile_z;
    int32_t time_block;
    int32_t rows_per_thread;
} sg_tuning;

typedef struct sg_plan sg_plan;

/* ABI version of the loaded library (SG_ABI_VERSION of its header). */
int32_t sg_abi_version(void);

/* Name of a status code; never NULL. */
const char *sg_status_string(sg_status s);

/* Message of the last failing call on this thread ("" if none); never NULL. */
const char *sg_last_error(void);

/*
 * Validate a geometry and create a plan (no device work; where a device is
 * present it reserves the plan's pinned staging, see the conventions above).
 * Returns SG_EINVAL for bad sizes (among them a stored padded field, guard
 * ring included, of more than 2^29 cells: the kernels address a field with
 * 32-bit byte offsets, the FP64 gradient accumulator included), SG_ECFL when
 * dt > s_max h / vmax_hint unless flags has SG_ALLOW_UNSTABLE.  *out is NULL
 * on error.
 */
sg_status sg_plan_create(const sg_geometry *g, uint32_t flags, sg_plan **out);

/* Destroy a plan; NULL is accepted. */
sg_status sg_plan_destroy(sg_plan *p);

/* Size the plan's pinned table staging for calls of up to nshot shots and
 * nrec receivers: the forward calls, and with ckpt_every > 0 also the
 * gradient calls with that checkpoint spacing (their residual-injection
 * tables are larger).  Later calls within those sizes allocate nothing on
 * the host.  SG_EINVAL for nshot < 1, nrec < 0 or ckpt_every < 0, SG_EHIP if
 * pinned memory cannot be allocated. */
sg_status sg_plan_reserve(sg_plan *p, int32_t nshot, int32_t nrec, int32_t ckpt_every);

/* Warning bits (SG_WARN_*) raised by sg_plan_create. */
uint32_t sg_plan_warnings(const sg_plan *p);

/* Padded grid of the plan: rows and columns including the sponge. */
sg_status sg_plan_padded_shape(const sg_plan *p, int32_t *Nz, int32_t *Nx);

/* Set the tuning used by later calls on this plan (NULL = library default).
 * Returns SG_EINVAL for values outside the documented ranges. */
sg_status sg_plan_set_tuning(sg_plan *p, const sg_tuning *t);

/* Tuning the plan will use for nshot shots (after defaults are resolved). */
sg_status sg_plan_get_tuning(const sg_plan *p, int32_t nshot, sg_tuning *t);

/*
 * Autotuner: times every built tile shape with every admissible time block
 * (1..8), and the column sweep (variant 3, strips of 128 and 256 columns,
 * time blocks 2..6, whole height or segments of 160, 224 or 320 rows) where
 * dz == dx, on this call's real shape -- trial_levels (>= 8) levels of the
 * time-stepping launches for `shots` on `vp`, after one untimed pass -- and
 * keeps the fastest as the plan's tuning (also returned in *best).  Uses the
 * workspace of sg_forward (no outputs are written).  Synchronises the stream.
 */
sg_status sg_autotune(sg_plan *p, const float *vp, const sg_shots *shots, int32_t trial_levels, void *ws,
                      size_t ws_bytes, void *stream, sg_tuning *best);

/*
 * Kernel timing of the time-stepping launches.  With profiling on, later
 * calls on this plan bracket their back-to-back run of time-stepping
 * launches with a pair of HIP events on the call's stream; sg_plan_profile
 * waits for the second event and returns the elapsed time [ms] and the
 * number of launches in between for the most recent call.  Used by the
 * benchmark to price the dominant kernel (time / launches = average launch).
 */
sg_status sg_plan_set_profiling(sg_plan *p, int32_t on);
sg_status sg_plan_profile(sg_plan *p, double *kernel_ms, int32_t *launches);

/*
 * Ricker pulse of App. E.4 evaluated in double precision and rounded to
 * float: w(t_n) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = n dt - t0.
 * t0 <= 0 selects t0 = 1/f0.  `out` is host memory of nt floats.
 */
sg_status sg_ricker(double f0, double dt, int32_t nt, double t0, float *out);

/*
 * Band-limited source of App. E.4 (Table "bands"): the Ricker pulse of peak
 * frequency f0 centred at 1/f0, filtered forward and backward (zero phase) by
 * a 4th-order Butterworth band-pass with corners fmin < fmax [Hz] (bilinear
 * design with pre-warped corners; each pass starts from the filter's rest
 * state at the first sample of an odd extension of 27 samples at both ends),
 * divided by its l2 norm and scaled by sqrt((fmax - fmin) / bandwidth_ref)
 * (the paper uses 24 Hz).  Computed in double precision on the host, rounded
 * to float into `out` (host memory of nt floats).  SG_EINVAL for nt <= 27,
 * corners outside (0, Nyquist) or fmin >= fmax.
 */
sg_status sg_bandpass_ricker(double f0, double fmin, double fmax, double dt, int32_t nt, double bandwidth_ref,
                             float *out);

/* CFL time-step limit s_max h / vmax of App. E.3.2 for this stencil, with
 * h = min(dz, dx). */
double sg_cfl_dt_max(double dz, double dx, double vmax);

/* Bytes of device workspace sg_forward needs for nshot shots and nrec
 * receivers. */
sg_status sg_forward_workspace_size(const sg_plan *p, int32_t nshot, int32_t nrec, size_t *bytes);

/*
 * Forward modelling (the hot path).
 *   vp        device [nz][nx] float velocity [m/s], > 0
 *   shots     host description, see sg_shots
 *   gathers   device [nshot][ceil(nt/rec_every)][nrec] float, or NULL
 *   snaps     device [nshot][snap_count][nz][nx] float, or NULL
 *   ws        device workspace of ws_bytes >= sg_forward_workspace_size
 * Every element of the non-NULL outputs is written.  The time-stepping
 * launches of a call are recorded once into a hipGraph per (plan shape,
 * tuning, workspace, output and wavelet pointers) and replayed on later calls
 * with the same ones (positions, velocities and wavelet values may change
 * between calls: they are read from the workspace and the caller's buffers at
 * run time), unless graphs are turned off (sg_set_graphs) or the caller is
 * already capturing the stream.
 */
sg_status sg_forward(sg_plan *p, const float *vp, const sg_shots *shots,
                     float *gathers, float *snaps, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * sg_forward without a workspace argument, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid allocation).
 * The workspace is a static device array of SG_NOALLOC_SCRATCH_BYTES per
 * device, held from library load until the process ends.  Same arguments,
 * outputs and errors as sg_forward, plus SG_ENOSPACE when the call would need
 * more than that (sg_forward_workspace_size > SG_NOALLOC_SCRATCH_BYTES; e.g.
 * the 620 x 1001 slice with a 40-cell sponge fits two shots) or when the
 * plan's pinned table staging is smaller than this call's tables (it is
 * sized at sg_plan_create for 64 shots and 2 nx receivers; sg_plan_reserve
 * sizes it up).  The call allocates nothing: no device or host allocation,
 * no graph recording (its launches are enqueued directly).  Every call on a
 * device shares that device's array, which keeps the last call's contents:
 * calls that overlap on one device (another stream, another thread) race and
 * must be serialised by the caller.
 */
#define SG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sg_status sg_forward_noalloc(sg_plan *p, const float *vp, const sg_shots *shots, float *gathers, float *snaps,
                             void *stream);

/*
 * Differentiation (adjoint-state velocity gradient).
 * sg_grad_workspace_size: bytes for nshot shots and nrec receivers with
 * checkpoints every ckpt_every levels (<= 0: ceil(sqrt(nt))).  sg_forward_ckpt runs the forward
 * like sg_forward (gathers, no snapshots) and keeps checkpoints in ws;
 * sg_adjoint_gradient then consumes them:
 *   resid     device [nshot][ceil(nt/rec_every)][nrec] float, dJ/dd for any
 *             misfit J (for J = 1/2 |d - d_obs|^2 this is d - d_obs)
 *   grad      device [nz][nx] float, overwritten with dJ/dv summed over shots
 * Both calls must get the same plan, vp, shots, ckpt_every and ws.  The
 * gradient call also runs work on a second stream of the plan (created on
 * first use, default priority) that it forks from and joins back into
 * `stream` with events, so work enqueued on `stream` after the call sees the
 * finished gradient; calls on one plan must not overlap.
 */
sg_status sg_grad_workspace_size(const sg_plan *p, int32_t nshot, int32_t nrec,
                                 int32_t ckpt_every, size_t *bytes);
sg_status sg_forward_ckpt(sg_plan *p, const float *vp, const sg_shots *shots,
                          int32_t ckpt_every, float *gathers, void *ws, size_t ws_bytes,
                          void *stream);
sg_status sg_adjoint_gradient(sg_plan *p, const float *vp, const sg_shots *shots,
                              int32_t ckpt_every, const float *resid, float *grad,
                              void *ws, size_t ws_bytes, void *stream);

/*
 * Batched forward over several slices of uneven size (one item per slice,
 * all with the same dt and nt); every time block of every shot of every item
 * runs in one launch.
 */
typedef struct {
    sg_plan *plan;
    const float *vp;
    const sg_shots *shots;
    float *gathers;
    float *snaps;
} sg_batch_item;

sg_status sg_batch_workspace_size(const sg_batch_item *items, int32_t nitems, size_t *bytes);

/*
 * Runs every item as sg_forward would (same outputs), on the tiled kernel or
 * the column sweep, with one tuning for the whole batch (NULL = the first
 * item's plan tuning).
 * Each time block of the whole batch is one launch over a flattened list of
 * (item, shot, tile) work; the sequence of launches is captured once into a
 * hipGraph per (workspace, batch shape) and replayed on later calls, unless
 * the stream is already being captured by the caller (then the launches go
 * into the caller's capture).  Items must share nt.
 */
sg_status sg_batch_forward(const sg_batch_item *items, int32_t nitems, const sg_tuning *tuning,
                           void *ws, size_t ws_bytes, void *stream);

/*
 * Batched autotuner: times every built tile shape with every admissible time
 * block that tiles every item, and the column sweep (variant 3) where every
 * item has dz == dx, on the whole batch -- trial_levels (>= 8)
 * levels of the batched time-stepping launches after one untimed pass -- and
 * returns the fastest in *best, to pass to sg_batch_forward (or to
 * sg_batch_adjoint_gradient).  Uses the workspace of sg_batch_forward; no
 * output of the items is written and no plan is changed.  Synchronises the
 * stream.
 */
sg_status sg_batch_autotune(const sg_batch_item *items, int32_t nitems, int32_t trial_levels, void *ws,
                            size_t ws_bytes, void *stream, sg_tuning *best);

/*
 * Batched velocity gradients over several slices of uneven size (items share
 * dt and nt).  Shots run in waves of at most shots_per_wave shots per item
 * (<= 0: all at once), so the checkpoint and recompute store fits the
 * workspace; within a wave every time block of every shot of every item is
 * one launch.  Each wave runs the forward with checkpoints every ckpt_every
 * levels (<= 0: ceil(sqrt(nt))), then the segments backwards (recompute +
 * adjoint), and adds its shots' contribution to the item's gradient.
 *   resid  device [nshot][ceil(nt/rec_every)][nrec] float, dJ/dd of the item
 *   grad   device [nz][nx] float, overwritten with dJ/dv summed over the item's shots
 * A column-sweep tuning (variant 3) runs the forward and the recompute on the
 * sweep; the adjoint always runs the tiled kernel.  Like sg_adjoint_gradient
 * the call forks work onto the first item's plan's second stream and joins it
 * back into `stream`.
 */
typedef struct {
    sg_plan *plan;
    const float *vp;
    const sg_shots *shots;
    const float *resid;
    float *grad;
} sg_batch_grad_item;

sg_status sg_batch_grad_workspace_size(const sg_batch_grad_item *items, int32_t nitems, int32_t ckpt_every,
                                       int32_t shots_per_wave, size_t *bytes);
sg_status sg_batch_adjoint_gradient(const sg_batch_grad_item *items, int32_t nitems, int32_t ckpt_every,
                                    int32_t shots_per_wave, const sg_tuning *tuning, void *ws, size_t ws_bytes,
                                    void *stream);

/*
 * Physics residual of a stack of wavefield frames (App. F.5: the residual of
 * the discretised acoustic wave operator, used there to assess predicted
 * wavefields without the ground truth):
 *     R_t = (u_{t+1} - 2 u_t + u_{t-1}) / dt^2 - v^2 L u_t
 * with L the 8th-order Laplacian of App. E.3 and dt the spacing of the frames,
 * evaluated where the frames alone define it: frames 1..nframes-2, columns
 * 4..nx-5, rows 1..nz-5 under SG_TOP_FREE (odd mirror above the pinned row 0)
 * or rows 4..nz-5 under SG_TOP_ABSORBING.
 *   frames  device [nframes][nz][nx] float (physical grid, x fastest)
 *   vp      device [nz][nx] float velocity [m/s]
 *   res2    device [nframes] double, written: sum over the cells of R_t^2
 *   dtt2    device [nframes] double, written: sum of ((u_{t+1} - 2u_t + u_{t-1}) / dt^2)^2
 * (0 for the first and last frame).  sqrt(sum res2 / sum dtt2) is the
 * residual ratio.  FP32 stencil arithmetic; FP32 sums over the 8 rows of a
 * lane and the 16 lanes of a row, FP64 beyond, in a fixed order
 * (deterministic).  ws: sg_wave_residual_workspace_size bytes (caller-owned
 * device scratch).  SG_EINVAL for NULL pointers, non-positive sizes or
 * spacings, more than 65537 frames or frames of 2^30 cells or more;
 * SG_ENOSPACE for a short workspace.  Fewer than 3 frames, or a grid with no
 * evaluated cell, gives all-zero sums.
 */
sg_status sg_wave_residual_workspace_size(int32_t nframes, int32_t nz, int32_t nx, int32_t top, size_t *bytes);
sg_status sg_wave_residual(const float *frames, int32_t nframes, int32_t nz, int32_t nx, const float *vp, double dz,
                           double dx, double dt, int32_t top, double *res2, double *dtt2, void *ws, size_t ws_bytes,
                           void *stream);

/*
 * Velocity-model builder modules (App. B): the interbedded band of Deposit
 * (Alg. 1), the vertical warp of Squish (Alg. 2) and the listric normal
 * fault of Fault (Alg. 3), on a device volume
 * [nz][ny][nx] of floats (x fastest; a 2D slice is ny = 1), z = depth.  Squish
 * and Fault pull-sample the input through an 8-point Kaiser-windowed sinc (beta 6,
 * weights normalised to sum 1, tap indices clamped to the axis), exact at
 * integer positions.  out must not alias the input.  Stream-ordered, no
 * allocation.  SG_EINVAL for NULL pointers, non-positive sizes or spacings,
 * aliasing, or parameters outside the ranges below.
 */

/* Alg. 1 (Deposit, boundary path): an interbedded band out [t][ny][nx] of t
 * cells.  The method's random draws are inputs (device floats): thick
 * [nbeds] bed thicknesses in cells (drawn and clamped by the caller), vbed
 * [nbeds] bed velocities [m/s], eta_b [nbeds-1][ny][nx] contact noise (e.g.
 * from sg_fractal_noise2d with amplitude 1), tex_lattice [gz][gy][gx] a
 * periodic value-noise lattice with node spacings lam_z/y/x [m], tex_off
 * [nbeds] per-bed depth offsets into it [m].  Contacts H_i = thick_0 + ... +
 * thick_{i-1} (i = 1..nbeds-1) move by taper(H_i) a_B eta_b[i-1] and are
 * clamped to [0, t-1]; a voxel at depth z belongs to bed l = number of
 * contacts <= z, which starts at the deepest of them (0 for bed 0); then
 *   V = (vbar + beta z dz) + taper(z) [(vbed_l - vbar) + a_eta noise],
 * vbar the mean bed velocity, noise the quintic-fade value noise at
 * ((z - start) dz + tex_off_l, y dy, x dx), taper(z) = min(z / (f_top t), 1)
 * min((t - z) / (f_base t), 1).  beta in m/s per m, a_B in cells, a_eta in
 * m/s; nbeds in 1..129.  Placing the band under a topography is a
 * per-column vertical warp (sg_squish). */
sg_status sg_deposit(int32_t t, int32_t ny, int32_t nx, double dz, double dy, double dx, int32_t nbeds,
                     const float *thick, const float *vbed, double beta, const float *eta_b, double a_B,
                     const float *tex_lattice, int32_t gz, int32_t gy, int32_t gx, double lam_z, double lam_y,
                     double lam_x, const float *tex_off, double a_eta, double f_top, double f_base, float *out,
                     void *stream);

/* 3D simplex noise (the noise fields of Deposit, App. B: boundary surfaces
 * and texture): Perlin's simplex noise as formulated by Gustavson (2005) --
 * skew by 1/3, unskew by 1/6, the twelve cube-edge gradients chosen by the
 * corner hash perm[i + perm[j + perm[k]]] mod 12 (indices mod 256), falloff
 * (0.6 - d^2)^4, scale 32; values within about [-1, 1], 0 at lattice corners.
 * perm: device int32 [256], a permutation of 0..255 (the random draw; entries
 * are taken mod 256).  FP64 evaluation, FP32 output:
 *   out[z][y][x] = amplitude S(oz + z sz, oy + y sy, ox + x sx)
 * (coordinates in lattice cells, within 2^40).  SG_EINVAL for NULL pointers,
 * non-positive sizes, non-finite arguments or coordinates beyond 2^40. */
sg_status sg_simplex_noise3d(const int32_t *perm, int32_t nz, int32_t ny, int32_t nx, double oz, double oy, double ox,
                             double sz, double sy, double sx, double amplitude, float *out, void *stream);

/* Alg. 1 (Deposit, boundary path) with both noise fields from 3D simplex
 * noise, as the module's prose describes: contact i (mean depth H_i =
 * thick_0 + .. + thick_{i-1} cells) moves by taper(H_i) a_B S_b(H_i dz /
 * lam_bz, y dy / lam_by, x dx / lam_bx) -- the field perm_b on the plane at
 * the contact's depth -- and is clamped to [0, t-1]; the texture is
 * a_eta S_t(((z - start) dz + tex_off_l) / lam_tz, y dy / lam_ty,
 * x dx / lam_tx), the field perm_t (both perms device int32 [256]).  Bed
 * lookup, depth trend and taper as sg_deposit; lengths in metres, a_B in
 * cells, a_eta in m/s; nbeds in 1..129.  Errors as sg_deposit. */
sg_status sg_deposit_simplex(int32_t t, int32_t ny, int32_t nx, double dz, double dy, double dx, int32_t nbeds,
                             const float *thick, const float *vbed, double beta, const int32_t *perm_b,
                             double lam_bz, double lam_by, double lam_bx, double a_B, const int32_t *perm_t,
                             double lam_tz, double lam_ty, double lam_tx, const float *tex_off, double a_eta,
                             double f_top, double f_base, float *out, void *stream);

/* Deposit's sinusoidal bedform mode (the module's prose in App. B): freq
 * [t] (device float, the raw instantaneous frequency in cycles per cell) is
 * smoothed by the normalised Gaussian of sigma cells over |m| <= int(4 sigma +
 * 0.5) with reflecting ends (sigma 0: unsmoothed) and summed into the warped
 * axis W[z] = f[0] + .. + f[z-1]; with phi = 2 pi (W[z] + a_r rug[y][x])
 * (rug device float [ny][nx], the rugosity field, may be NULL when a_r = 0):
 *   out[z][y][x] = (v0 + beta z dz) + taper(z) [amp1 sin(phi)
 *                  + amp2 sin(2 phi + phase2) + a_eta S_t(z dz / lam_tz, y dy / lam_ty, x dx / lam_tx)]
 * with sg_deposit's taper and S_t the simplex field perm_t.  FP64 throughout,
 * FP32 output.  t <= 4096, sigma in [0, 255].  SG_EINVAL for NULL pointers,
 * sizes or spacings out of range, non-finite parameters. */
sg_status sg_deposit_sinusoidal(int32_t t, int32_t ny, int32_t nx, double dz, double dy, double dx, double v0,
                                double beta, const float *freq, double sigma, double amp1, double amp2,
                                double phase2, const float *rug, double a_r, const int32_t *perm_t, double lam_tz,
                                double lam_ty, double lam_tx, double a_eta, double f_top, double f_base, float *out,
                                void *stream);

/* Alg. 2, first step: the displacement field out [ny][nx] (metres, device)
 * as fractal value noise: per octave o = 0..noct-1 a periodic lattice
 * lattice[o] [gy][gx] (device floats, e.g. uniform in [-1, 1]), sampled with
 * a quintic fade at the horizontal coordinates rotated by azimuth_deg and
 * divided by the wavelengths lam_y, lam_x [m], times 2^o; octave weights
 * 2^-o; the sum divided by sum_o 2^-o and multiplied by amplitude [m], so
 * |out| <= amplitude.  noct in 1..24. */
sg_status sg_fractal_noise2d(const float *lattice, int32_t noct, int32_t gy, int32_t gx, int32_t ny, int32_t nx,
                             double dy, double dx, double lam_y, double lam_x, double azimuth_deg, double amplitude,
                             float *out, void *stream);

/* Alg. 2, second step: out(z, y, x) = v sampled at depth z + shift(y, x) / dz
 * cells (shift [ny][nx] in metres, device; rows past either end repeat the
 * edge row). */
sg_status sg_squish(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, const float *shift, float *out,
                    void *stream);

/* Alg. 3 (one fault, smooth or rough; subsidiary faults are further calls).  Positions in
 * metres are (z dz, y dy, x dx).  The cylinder axis runs along the strike
 * s = (cos a, -sin a) in (y, x); it sits at c~ = c - (R sin(dip), R cos(dip) n)
 * with n = (sin a, cos a), a = azimuth.  Each voxel, in the plane across the
 * axis (radius r, angle theta = atan2(depth offset, offset along n)), turns by
 * -chi direction w slip / R (chi = +1 where r >= R, else -1) with the taper
 * w = cos(pi/2 |r - R| / die_r) cos(pi/2 |theta - theta0| / die_theta)
 *     cos(pi/2 |along-strike offset| / die_strike)
 * inside all three extents and 0 outside; theta0 = atan2(R sin(dip),
 * R cos(dip)).  The output pulls v from src = 2p - p_forward; where src lies
 * above depth 0 or at/below nz cells it is `fill`.  radius, die_* > 0,
 * direction +1 or -1. */
typedef struct sg_fault_params {
    double cz, cy, cx;      /* fault centre [m] */
    double azimuth_deg;     /* a */
    double dip_deg;         /* dip */
    double radius;          /* R [m] */
    double slip;            /* arc length [m] */
    int32_t direction;      /* +1 or -1 */
    double die_r;           /* die-off across the fault [m] */
    double die_strike;      /* die-off along strike [m] */
    double die_theta_deg;   /* die-off in angle about the axis [deg] */
    /* Optional rough fault surface (the module perturbs the fault radius with
     * fractal noise): with rough_lattice non-NULL the surface lies at radius
     * R + rough_amplitude N(u, w), N = normalised fractal value noise as in
     * sg_fractal_noise2d (octave o: lattice o, frequency 2^o, weight 2^-o, sum
     * divided by sum_o 2^-o; |N| <= max |lattice|), at u = along-strike
     * offset / rough_lam_strike and w = R (theta - theta0) / rough_lam_dip
     * (down-dip arc length).  It moves the side test (chi) and the
     * across-fault taper; the rotation stays slip / R.  rough_lattice:
     * device floats [rough_noct][rough_gd][rough_gs] (rows down dip, columns
     * along strike), rough_noct in 1..24, rough_gd, rough_gs >= 1, at most
     * 2^26 finite values, lam > 0.  With a rough lattice the call reads the
     * lattice back once to bound the region the fault can move: it
     * synchronises `stream` (the only builder call besides sg_salt_sdt that
     * does). */
    const float *rough_lattice;
    int32_t rough_noct, rough_gd, rough_gs;
    double rough_amplitude; /* [m] */
    double rough_lam_strike, rough_lam_dip; /* [m] */
} sg_fault_params;
sg_status sg_fault(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                   const sg_fault_params *p, float fill, float *out, void *stream);

/* Faults applied one after another (a primary and its subsidiaries, App. B
 * Fault prose): out = fault[n-1](... fault[0](v)), each as sg_fault; ws a
 * second device volume [nz][ny][nx] (NULL allowed when nfaults <= 1), v, out
 * and ws pairwise disjoint.  The steps alternate between out and ws; a fault
 * whose reach is a box inside the volume costs that box plus a copy of the
 * previous fault's box (never the whole volume after the second step).
 * nfaults in 0..100000 (0 copies v).  A rough fault synchronises `stream`
 * once, as in sg_fault.  Errors as sg_fault, plus SG_EINVAL for overlapping
 * buffers or a missing ws. */
sg_status sg_fault_sequence(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                            const sg_fault_params *faults, int32_t nfaults, float fill, float *out, float *ws,
                            void *stream);

/* Subsidiary faults of a primary in simplified Riedel-shear geometry (the
 * Fault prose of App. B; App. C's fault-array setting gives R-shears at +15
 * deg, R' at +165 deg, an 85 % synthetic and 75 % hanging-wall bias and a
 * minimum-distance filter).  Host only, FP64.  Candidate k reads five
 * uniforms in [0, 1] from uniforms[5 k ..] (the random draw, host) and is:
 * synthetic (azimuth + synthetic_offset_deg) when u0 < synthetic_fraction,
 * else antithetic (+ antithetic_offset_deg); on the hanging-wall side (-n, n =
 * (sin a, cos a) in (y, x), the side the primary dips towards) when u1 <
 * hangingwall_fraction, else the footwall side (+n); centred at the primary's
 * depth, (2 u2 - 1) along_strike along the strike (cos a, -sin a) and
 * across_min + u3 (across_max - across_min) across it; a smooth copy of the
 * primary with radius, die_r and die_strike times size_scale and slip times
 * slip_min + u4 (slip_max - slip_min).  Candidates are taken in order and one
 * closer than min_distance (map view) to an accepted subsidiary is dropped.
 * out: host [ncand] (the first *nout entries are written).  Each subsidiary is
 * one more fault of a sequence.  SG_EINVAL for NULL pointers, ncand outside
 * 0..1000000, fractions outside [0, 1], negative or non-finite distances,
 * size_scale <= 0, uniforms outside [0, 1] or an invalid primary. */
typedef struct sg_riedel_config {
    double synthetic_fraction;     /* 0.85 */
    double hangingwall_fraction;   /* 0.75 */
    double synthetic_offset_deg;   /* 15 */
    double antithetic_offset_deg;  /* 165 */
    double along_strike;           /* half-length of the placement zone along strike [m] */
    double across_min, across_max; /* distance from the primary's trace across strike [m] */
    double size_scale;             /* radius and die-off lengths relative to the primary */
    double slip_min, slip_max;     /* slip relative to the primary's */
    double min_distance;           /* between subsidiary centres, map view [m] */
} sg_riedel_config;
sg_status sg_riedel_subsidiaries(const sg_fault_params *primary, const sg_riedel_config *cfg, int32_t ncand,
                                 const double *uniforms, sg_fault_params *out, int32_t *nout);

/* Alg. 3 for integer fields such as layer labels (the module resamples them
 * by nearest neighbour): the same fault and pull source as sg_fault, with
 * out(voxel) = labels at the voxel nearest the source (floor(s + 0.5) per axis
 * in cell units, y and x clamped to the volume), `fill` where the source depth
 * lies above depth 0 or at/below nz cells, the label itself outside the
 * taper.  labels and out [nz][ny][nx] int32 (device), out must not alias
 * labels.  Same argument errors as sg_fault. */
sg_status sg_fault_labels(const int32_t *labels, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                          const sg_fault_params *p, int32_t fill, int32_t *out, void *stream);

/* Labels through a sequence of faults (nearest-neighbour pulls, as
 * sg_fault_labels); buffers and errors as sg_fault_sequence. */
sg_status sg_fault_labels_sequence(const int32_t *labels, int32_t nz, int32_t ny, int32_t nx, double dz, double dy,
                                   double dx, const sg_fault_params *faults, int32_t nfaults, int32_t fill,
                                   int32_t *out, int32_t *ws, void *stream);

/* Alg. 4 (SaltSDT) on a device volume v [nz][ny][nx] (positions (z dz, y dy,
 * x dx) in metres).  Body i (host arrays): centre centres[3i..3i+2] and radii
 * radii[3i..3i+2] > 0 in metres as (z, y, x), rotation rotations[9i..9i+8]
 * row-major taking world offsets to the body frame (orthonormal: R R^T = I
 * within 1e-7 per entry); the voxel centres with
 * sum_k (u_k / r_k)^2 <= 1 (u = R (p - c)) form its raster.  phi = distance to
 * the nearest voxel outside minus distance to the nearest voxel inside
 * (exact Euclidean, metres, FP64), and K |= phi + amplitude rbar grf[i] > 0
 * with rbar the mean radius and grf [nbodies][nz][ny][nx] device floats (the
 * random field, e.g. a smoothed Gaussian).  A body covering no voxel adds
 * nothing and one covering all adds all.  K is then opened and closed with
 * the 6-neighbour cross (a voxel outside the volume counts as empty); its
 * 6-connected components of fewer than min_voxels voxels are dropped, K is
 * limited to v >= v_water and out = v_salt on K, v elsewhere.  mask_out
 * [nz][ny][nx] bytes (device, may be NULL) receives K as 0/1.  ws:
 * sg_salt_workspace_size bytes of caller-owned device scratch (256-byte
 * aligned).  nbodies in 0..4096; nz ny nx < 2^31.  Synchronises the stream
 * once: the extremes of the fields are read back to bound how far beyond its
 * ellipsoid each body can reach, and each body's distances are computed only
 * on that box (the result is the same as on the whole volume).  SG_EINVAL for
 * NULL pointers, bad sizes or non-finite or non-positive parameters, a
 * rotation that is not orthonormal and out aliasing v; SG_ENOSPACE for a short
 * workspace. */
sg_status sg_salt_workspace_size(int32_t nz, int32_t ny, int32_t nx, size_t *bytes);
sg_status sg_salt_sdt(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                      int32_t nbodies, const double *centres, const double *radii, const double *rotations,
                      const float *grf, double amplitude, float v_salt, float v_water, int64_t min_voxels,
                      float *out, uint8_t *mask_out, void *ws, size_t ws_bytes, void *stream);

/* Alg. 4, the random field xi of one salt body: white noise shaped in
 * Fourier space by sqrt(P(k)), P(k) = (1 + sum_k (k_k l_k)^2)^-p, the
 * spectrum of the paper's GRF step.  The field lives on a periodic grid of
 * grid[0] x grid[1] x grid[2] cells (the smallest powers of two >= nz, ny, nx;
 * sg_grf_workspace_size reports it), k_k is the angular wavenumber in radians
 * per cell along axis k, l_k (lz, ly, lx) the correlation lengths in cells
 * (the module takes l_k = max(r_k f_lk, 5)); the real part of the transform
 * back is cropped to [nz][ny][nx] and scaled to zero mean and unit variance
 * over the volume (the paper fixes neither).
 *   noise  device floats [grid[0]][grid[1]][grid[2]], white noise (the draw
 *          is the caller's, e.g. standard normal)
 *   out    device floats [nz][ny][nx] (for sg_salt_sdt's grf), not aliasing noise
 *   ws     device workspace of sg_grf_workspace_size bytes (two complex grids)
 * Extents 1..1024; lengths finite and >= 0 (0 leaves an axis white); p >= 0.
 * The 3D transforms are hand-written radix-2 FFTs in FP32.  Stream-ordered,
 * no allocation; SG_EINVAL / SG_ENOSPACE as usual. */
sg_status sg_grf_workspace_size(int32_t nz, int32_t ny, int32_t nx, int32_t *grid, size_t *bytes);
sg_status sg_grf(const float *noise, int32_t nz, int32_t ny, int32_t nx, double lz, double ly, double lx, double p,
                 float *out, void *ws, size_t ws_bytes, void *stream);

/* Turn the graph replay of sg_forward and sg_batch_forward on (default) or
 * off (plain stream launches); process-wide. */
sg_status sg_set_graphs(int32_t on);

/*
 * Scan `n` device floats for NaN/Inf.  Synchronises the stream; returns
 * SG_EDIVERGED if any is found (used to flag blow-ups).
 */
sg_status sg_check_finite(const float *x, size_t n, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SGWAVE_H */
