// Internal declarations shared by the host runtime (sg_runtime.cpp) and the
// HIP kernels (sg_kernels.hip: propagator and adjoint; sg_residual.hip: wave
// residual; sg_builder.hip and sg_salt.hip: model-builder modules).  Not part
// of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sgwave.h"

namespace sg {

// Shared by the C ABI files (sg_runtime.cpp, sg_static.hip).  forward_call is
// the body of sg_forward on a workspace of ws_bytes; with no_alloc it
// allocates nothing: the launches are enqueued directly (recording a graph
// allocates) and the plan's pinned staging must already hold the tables
// (SG_ENOSPACE otherwise).  report_error sets the thread-local last-error
// message and returns st.
sg_status forward_call(sg_plan *p, const float *vp, const sg_shots *shots, float *gathers, float *snaps, void *ws,
                       size_t ws_bytes, void *stream, bool no_alloc);
sg_status report_error(sg_status st, const char *msg);

// Stencil half width: the 8th-order central difference reaches 4 cells on
// each side (M = 4, App. E.3 / Table "params").
constexpr int kHalo = 4;

// Guard cells kept at zero around every stored field (rows above and below,
// columns left and right).  They let the one-step kernel read neighbours of
// any padded cell without a bounds test.
constexpr int kGuard = 4;

// Up to four bilinear nodes per source or receiver.
constexpr int kNodes = 4;

// Largest time block (sub-steps per launch) of the time-blocked kernel.
constexpr int kMaxTimeBlock = 8;

// Device-side description of one padded slice and its fields.  All offsets
// are in floats relative to a field's base; node (Iz, Ix) of the padded grid
// lives at (Iz + kGuard) * pitch + (Ix + kGuard).
struct SliceDesc {
    int32_t Nz, Nx;          // padded grid
    int32_t pitch;           // floats per stored row
    int32_t nz, nx;          // physical grid
    int32_t ztop, xleft;     // padded index of physical (0, 0)
    int32_t free_top;        // 1: row 0 pinned to 0, odd mirror above
    int32_t unit_z0, unit_z1, unit_x0, unit_x1;   // padded box [z0, z1) x [x0, x1) of updated cells with a = 1
    int32_t nshot;
    int32_t nrec;
    int32_t nrow;            // gather rows = ceil(nt / rec_every)
    int32_t rec_every;
    int32_t snap_every, snap_count;
    int32_t wavelet_stride;  // 0 if one wavelet is shared, else nt
    int64_t frame;           // floats per stored field = (Nz + 2 kGuard) * pitch
    float cz[kHalo + 1];     // c_m / dz^2
    float cx[kHalo + 1];     // c_m / dx^2
    const float *V2;         // (v dt)^2 on the padded grid, stored-field layout
    const float *W;          // W = a (v dt)^2 on updated cells, else 0 (stored-field layout)
    const float *A2;         // 2a on updated cells, else 0 (stored-field layout)
    const float *gx;         // [Nx] eta_x / (2 dt); gamma = (gx + gz) * V2
    const float *gz;         // [Nz]
    const int32_t *src_off;  // [nshot][kNodes] stored-field offsets, -1 = unused
    const int32_t *src_iz;   // [nshot][kNodes] padded row of each node (-1 << 20 = unused)
    const int32_t *src_ix;   // [nshot][kNodes] padded column
    const float *src_w;      // [nshot][kNodes] weight / (dx dz), 0 = unused
    const int32_t *rec_off;  // [nrec][kNodes] stored-field offsets, -1 = unused
    const int32_t *rec_iz;   // [nrec] padded row of the base node (weights in rec_w
    const int32_t *rec_ix;   // [nrec]   for (0,0), (0,1), (1,0), (1,1))
    const float *rec_w;      // [nrec][kNodes], 0 = unused
    const int32_t *tile_rec; // tiled path: [tiles + 1] start of each tile's entries in rec_list
    const struct RecEntry *rec_list;   // tiled path: receivers grouped by tile
    const float *wavelet;    // [nshot or 1][nt]
    float *fields;           // [nshot][kFramesPerShot][frame]
    float *gathers;          // [nshot][nrow][nrec] or null
    float *snaps;            // [nshot][snap_count][nz][nx] or null
};

// A receiver as the tiled kernel reads it: LDS index of its base node within
// the owning tile's buffer (nodes at +0, +1, +LW, +LW+1), its output column
// and the bilinear weights of those nodes.
struct RecEntry {
    int32_t lds;
    int32_t r;
    float w[kNodes];
};

// Each shot owns two pairs of fields.  The one-step kernel keeps level m in
// frame m & 1 of pair 0.  The tiled kernel reads a pair (frame 0 = level m-1,
// frame 1 = level m) and writes the other, so no workgroup overwrites a level
// another workgroup still reads as halo.
constexpr int kFramesPerShot = 4;

// Residual injection tables of the adjoint (one tiling): for tile t the cells
// tile_start[t] .. tile_start[t+1]-1 are the receiver nodes inside its loaded
// region; cell e sits at LDS index lds[e] (padded row iz[e], column ix[e]) and
// gets sum_q w[q] r[rid[q]] for q in pstart[e] .. pstart[e+1]-1.
struct InjTables {
    const int32_t *tile_start;
    const int32_t *lds;
    const int32_t *iz;
    const int32_t *ix;
    const int32_t *pstart;
    const int32_t *rid;
    const float *w;
};

// One launch of the time-blocked kernel.
struct TileArgs {
    int32_t n;          // forward: levels n-1, n are read, n+1.. computed;
                        // adjoint: mu^{n+2}, mu^{n+1} are read, mu^n, mu^{n-1}.. computed
    int32_t nsteps;     // levels advanced by this launch (<= tb)
    int32_t tb;         // time block the tiling was sized for: halo = 4 * tb
    int32_t tx, tz;     // output tile
    int32_t tz_top;     // output rows of the top tile row under a free top
    int32_t ntx, ntz;   // tiles per row / column
    int32_t in_pair, out_pair;
    float *fields;      // [nshot][kFramesPerShot][frame]
    // forward with ring != null: the second time difference D^n of the output
    // tile is stored in ring slot n - ring_lo for every level n advanced;
    // adjoint: the ring holds D^ring_lo .. D^ring_hi read by the imaging term
    float *ring;
    int32_t ring_lo, ring_hi;
    int64_t ring_shot;  // floats per shot in the ring
    // adjoint only
    const float *resid; // [nshot][nrow][nrec], dJ/dd at the recorded levels
    double *hsum;       // [nshot][frame] sum_n mu^{n+1} (p^{n+1} - 2p^n + p^{n-1}), accumulated in FP64
    int32_t nt;
    InjTables inj;
};

// One slice of a batched launch: its descriptor, its tiling and field
// pointers (launch-level fields of `t` are overwritten per launch), and the
// first logical block it owns.
struct BatchItem {
    SliceDesc s;
    TileArgs t;
    int32_t block_start;
};

// Output tiling of the time-blocked kernel for an extended (LDS) tile of
// ex x ez cells with time block tb and k rows per thread.
struct Tiling {
    int ex, ez, k, tb;
    int tx, tz, tz_top, ntx, ntz;
    bool ok;
    int sweep_nw;   // > 0: column sweep (sg_sweep.hip) over strips of 64 sweep_nw columns, ntz = 1
};
Tiling make_tiling(int Nz, int Nx, bool free_top, int ex, int ez, int k, int tb);
// Strips of ex = 64 nw loaded columns for the column-sweep kernel: output
// width ex - 8 tb; each strip cut in segments of seg_h output rows (0 = the
// whole height), one tile row per segment.
Tiling make_sweep_tiling(int Nz, int Nx, int nw, int tb, int seg_h = 0);
// Largest time block of the column-sweep kernel, and its strip widths (waves).
constexpr int kSweepMaxTimeBlock = 6;

// Instantiated shapes of the time-blocked kernel (extended tile ex x ez,
// k rows per thread); `config` indexes this list.
struct TiledShape { int ex, ez, k; };
constexpr int kTiledShapes = 4;
TiledShape tiled_shape(int config);

// Kernel launchers (sg_kernels.hip).  All return hipSuccess or the launch error.
// launch_prepare fills V2, W and A2 (needs gx and gz in place).
hipError_t launch_prepare(const SliceDesc &s, const float *vp, float dt2, hipStream_t st);
hipError_t launch_zero(float *p, size_t n, hipStream_t st);
hipError_t launch_step_naive(const SliceDesc &s, int n, hipStream_t st);
hipError_t launch_step_tiled(const SliceDesc &s, const TileArgs &t, int config, hipStream_t st);
hipError_t launch_adjoint_tiled(const SliceDesc &s, const TileArgs &t, int config, hipStream_t st);
// Column-sweep forward (sg_sweep.hip, dz == dx only): t.nsteps levels (1..6)
// over strips of 64 nw columns (nw 2 or 4); with t.ring (ring for the batched
// form) also the second time differences into the ring, as the tiled kernel's
// recompute mode.  The batched form like launch_step_tiled_batch.
hipError_t launch_sweep(const SliceDesc &s, const TileArgs &t, int nw, hipStream_t st);
hipError_t launch_sweep_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps, int in_pair,
                              int nw, hipStream_t st, bool ring = false, int ring_lo = 0);
// Batched launches: items[0..nitems) in device memory, total_blocks = sum of
// the items' blocks (items[i].block_start is the prefix sum).
hipError_t launch_step_tiled_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps,
                                   int in_pair, int config, bool iso, hipStream_t st);
hipError_t launch_ring_tiled_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps,
                                   int in_pair, int config, bool iso, int ring_lo, hipStream_t st);
hipError_t launch_adjoint_tiled_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps,
                                      int in_pair, int config, bool iso, int ring_lo, int ring_hi, hipStream_t st);
// dst[shot][0..n) = src[shot][0..n) for every shot (strides in floats)
hipError_t launch_copy(float *dst, int64_t dst_shot, const float *src, int64_t src_shot, int64_t n, int nshot,
                       hipStream_t st);
// grad[iz][ix] (+)= 2 / (dt^2 v^3) * sum over shots and over the padded cells
// whose velocity is copied from (iz, ix) of hsum
// hsum += the adjoint launches' FP32 partial sums kept in ring slots first,
// first - step, ... (nslot slots), in that order, for every shot of s.
hipError_t launch_fold_partials(const SliceDesc &s, double *hsum, const float *ring, int64_t ring_shot, int first,
                                int step, int nslot, hipStream_t st);
hipError_t launch_fold_gradient(const SliceDesc &s, const float *vp, const double *hsum,
                                int64_t shot_stride, float dt, float *grad, hipStream_t st, bool accumulate = false);
// Records level n held in frame `slot` of every shot: gather row (what & 1)
// and snapshot (what & 2) when that level is due for them.
hipError_t launch_record_slot(const SliceDesc &s, int n, int slot, hipStream_t st, int what = 3);
hipError_t launch_count_nonfinite(const float *x, size_t n, unsigned int *count, hipStream_t st);

// Fault (Alg. 3) in the form the kernel uses: grid spacings, the cylinder axis
// point c~ (metres), the unit vectors n (axis offset, across strike) and s
// (strike) in (y, x), the reference angle, the rotation for w = 1 and the
// reciprocal die-off extents.
struct FaultFrame {
    double dz, dy, dx, inv_dz, inv_dy, inv_dx;
    double cz, cy, cx;
    double n_y, n_x, s_y, s_x;
    double radius, theta0, shift, direction;
    double inv_die_r, inv_die_t, inv_die_s;
    // rough surface (rough == nullptr: smooth): radius + rough_amp * N, N the
    // noise sum times rough_inv_norm, at (along-strike offset * inv_lam_s,
    // radius (theta - theta0) * inv_lam_d); |N| <= max |lattice| (each octave
    // is a convex combination of lattice values and the weights sum to 1), so
    // rough_reach = die_r + |rough_amp| max |lattice| bounds where the noise
    // can matter
    const float *rough;      // [rough_noct][rough_gd][rough_gs], device
    int rough_noct, rough_gd, rough_gs;
    double rough_amp, rough_inv_norm, inv_lam_s, inv_lam_d, rough_reach;
};
// Deposit (Alg. 1): band size, spacings, the bed tables (device, nbeds
// entries; eta_b [nbeds-1][ny][nx]), the texture lattice [gz][gy][gx] with
// reciprocal node spacings, amplitudes and taper fractions.
struct DepositArgs {
    int t, ny, nx, nbeds, gz, gy, gx;
    double dz, dy, dx, inv_lam_z, inv_lam_y, inv_lam_x;
    double beta, a_B, a_eta, f_top, f_base;
    const float *thick, *vbed, *tex_off, *eta_b, *lattice;
    // simplex form: both noise fields from 3D simplex noise (perm tables of
    // 256 entries; lengths in metres as (z, y, x)); eta_b and lattice unused
    int simplex;
    const int32_t *perm_b, *perm_t;
    double lam_b[3], lam_t[3];
};
constexpr int kDepositMaxBeds = 129;   // contacts of a column held in LDS (128 x 64 lanes x 8 B)
hipError_t launch_deposit(const DepositArgs &A, float *out, hipStream_t st);

// Deposit's sinusoidal bedform mode.
struct DepositSinArgs {
    int t, ny, nx;
    double dz, dy, dx, v0, beta, sigma, amp1, amp2, phase2, a_r, a_eta, f_top, f_base;
    double lam_t[3];
    const float *freq, *rug;
    const int32_t *perm_t;
};
constexpr int kDepositSinMaxT = 4096;          // depths of a band (warped axis held in LDS)
constexpr double kDepositSinMaxSigma = 255.0;  // smoothing radius int(4 sigma + 0.5) <= 1020
hipError_t launch_deposit_sinusoidal(const DepositSinArgs &A, float *out, hipStream_t st);

// out[z][y][x] = amplitude S(o[0] + z s[0], o[1] + y s[1], o[2] + x s[2]),
// S the 3D simplex noise of the permutation perm[256].
hipError_t launch_simplex3d(const int32_t *perm, int nz, int ny, int nx, const double o[3], const double s[3],
                            double amplitude, float *out, hipStream_t st);
hipError_t launch_fractal_noise2d(const float *lattice, int noct, int gy, int gx, int ny, int nx, double dy,
                                  double dx, double lam_y, double lam_x, double azimuth_rad, double amplitude,
                                  float *out, hipStream_t st);
hipError_t launch_squish(const float *v, int nz, int ny, int nx, double dz, const float *shift, float *out,
                         hipStream_t st);
hipError_t launch_fault(const float *v, int nz, int ny, int nx, const FaultFrame &F, float fill, float *out,
                        hipStream_t st);
hipError_t launch_fault_labels(const int32_t *lab, int nz, int ny, int nx, const FaultFrame &F, int32_t fill,
                               int32_t *out, hipStream_t st);
// Faults F[0..n-1] applied in order: the result in out, ws a second volume
// (may be NULL when n <= 1); neither aliases v or the other.
hipError_t launch_fault_sequence(const float *v, int nz, int ny, int nx, const FaultFrame *F, int n, float fill,
                                 float *out, float *ws, hipStream_t st);
hipError_t launch_fault_labels_sequence(const int32_t *lab, int nz, int ny, int nx, const FaultFrame *F, int n,
                                        int32_t fill, int32_t *out, int32_t *ws, hipStream_t st);

// One salt body of Alg. 4: centre and radii in metres as (z, y, x); R row-major,
// taking world offsets to the body frame.
struct SaltBody {
    double c[3], r[3], R[9];
};
constexpr int kSaltMaxBodies = 4096;
size_t salt_workspace_bytes(int64_t nvoxels);
// Synchronises `st` once (to read the fields' extremes); `ws` holds
// salt_workspace_bytes(nz * ny * nx), 256-byte aligned; R orthonormal.
hipError_t launch_salt_sdt(const float *v, int nz, int ny, int nx, double dz, double dy, double dx, int nbodies,
                           const SaltBody *bodies, const float *grf, double amplitude, float v_salt, float v_water,
                           unsigned min_voxels, float *out, uint8_t *mask_out, void *ws, hipStream_t st);

// Random field of Alg. 4 (sg_grf.hip): the periodic grid (powers of two >=
// the extents, each <= 1024), the workspace (two complex grids and the
// partial sums) and the launch: noise [P0][P1][P2] -> out [nz][ny][nx].
void grf_grid(int nz, int ny, int nx, int P[3]);
size_t grf_workspace_bytes(int nz, int ny, int nx);
hipError_t launch_grf(const float *noise, int nz, int ny, int nx, double lz, double ly, double lx, double p, float *out,
                      void *ws, hipStream_t st);

// Wave-equation residual of a frame stack: c_m / dz^2 and c_m / dx^2, m = 0..4.
struct ResidualCoef {
    float cz[kHalo + 1];
    float cx[kHalo + 1];
};
// Partial sums per frame of the residual kernel (one per wave of each tile)
// for rows z0..nz-5, columns 4..nx-5.
int wave_residual_slots(int nz, int nx, int z0);
// res2/dtt2 [nframes] (device) from frames [nframes][nz][nx] and vp [nz][nx];
// partials: 2 * (nframes - 2) * wave_residual_slots doubles of scratch.
hipError_t launch_wave_residual(const float *frames, int nframes, int nz, int nx, const float *vp, double dt,
                                const ResidualCoef &cf, int z0, double *partials, double *res2, double *dtt2,
                                hipStream_t st);

}  // namespace sg
