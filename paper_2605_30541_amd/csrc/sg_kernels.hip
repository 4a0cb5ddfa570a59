// HIP kernels of the acoustic finite-difference propagator for gfx950.
//
// Scheme (SubsurfaceGen, arXiv 2605.30541; eqs. "acoustic_2d", "cerjan_pde",
// "free_surface"; App. E.3): for every padded cell,
//   p^{n+1} = 2a p^n + W (L p^n + S^n) - b p^{n-1},
//   gamma = eta v^2 dt / 2, a = 1/(1+gamma), b = (1-gamma) a, W = a (v dt)^2,
// with L the 8th-order Laplacian, p = 0 outside the padded grid, and under a
// free top row 0 pinned to 0 with the odd mirror p(-m) = -p(m) above it.
// S^n is the point-source term w(t_n) * weight / (dx dz) on bilinear nodes.
// Receivers read p^n with the same bilinear weights.
//
// Storage: a field is (Nz + 2G) rows of `pitch` floats, padded node (Iz, Ix)
// at (Iz + G) * pitch + Ix + G, G = 4 zero guard cells on every side.  Each
// shot owns two such fields; time level m lives in field m & 1, so a step
// overwrites level n-1 with level n+1 in place.
#include "sg_internal.h"

#include <atomic>
#include <type_traits>

namespace sg {

namespace {

__device__ inline float wavelet_at(const SliceDesc &s, int shot, int n)
{
    return s.wavelet[(int64_t)shot * s.wavelet_stride + n];
}

// One term pair of the 8th-order Laplacian in difference form:
//   L p = sum_{m=1..4} cz_m (p(z+m) + p(z-m) - 2p) + cx_m (p(x+m) + p(x-m) - 2p),
// the same operator as c_0 p + sum_m c_m (...) with c_0 = -2 sum_m c_m, but a
// constant field gives exactly 0 whatever the rounding of the weights, and each
// term stays small on smooth fields.  Over 10^4 steps this keeps the FP32
// round-off two orders of magnitude below the summed form.
__device__ inline float lap_pair(float acc, float cz, float cx, float zsum, float xsum, float c2)
{
    acc = fmaf(cz, zsum - c2, acc);
    return fmaf(cx, xsum - c2, acc);
}

// Leapfrog update with b = 2a - 1:
//   p^{n+1} = 2a p^n + W L p^n - b p^{n-1} = W L p^n + (2a (p^n - p^{n-1}) + p^{n-1}).
__device__ inline float leapfrog(float W, float lap, float a2, float c, float prev)
{
    return fmaf(W, lap, fmaf(a2, c - prev, prev));
}

// Records level n of one shot: gather row n / rec_every (when n is a multiple
// of rec_every) and snapshot n / snap_every (when due).  `tid`/`nthr` spread
// the receivers and the physical cells over the calling threads.
__device__ inline void record_level(const SliceDesc &s, const float *cur, int shot, int n,
                                    int tid, int nthr)
{
    if (s.gathers && n % s.rec_every == 0) {
        float *row = s.gathers + ((int64_t)shot * s.nrow + n / s.rec_every) * s.nrec;
        for (int r = tid; r < s.nrec; r += nthr) {
            float d = 0.f;
#pragma unroll
            for (int k = 0; k < kNodes; ++k) {
                int off = s.rec_off[r * kNodes + k];
                if (off >= 0) d += s.rec_w[r * kNodes + k] * cur[off];
            }
            __builtin_nontemporal_store(d, row + r);      // written once
        }
    }
    if (s.snaps && n % s.snap_every == 0 && n / s.snap_every < s.snap_count) {
        float *fr = s.snaps + ((int64_t)shot * s.snap_count + n / s.snap_every) * s.nz * s.nx;
        const int npts = s.nz * s.nx;
        for (int q = tid; q < npts; q += nthr) {
            int iz = q / s.nx, ix = q - iz * s.nx;
            __builtin_nontemporal_store(cur[(int64_t)(iz + s.ztop + kGuard) * s.pitch + ix + s.xleft + kGuard], fr + q);
        }
    }
}

// Velocity -> (v dt)^2 on the padded grid (edge replication into the sponge),
// and the update coefficients of every cell: W = a (v dt)^2 and 2a with
// a = 1 / (1 + gamma), gamma = (eta_x + eta_z) / (2 dt) (v dt)^2; both 0 on
// cells the scheme does not update (the guard cells, the pinned free-surface
// row).  The tiled kernel reads W and 2a; the one-step kernel forms them from
// (v dt)^2 with the same operations.
__global__ void __launch_bounds__(256) k_prepare(SliceDesc s, const float *vp, float dt2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s.frame) return;
    const int r = (int)(q / s.pitch), c = (int)(q - (int64_t)r * s.pitch);
    const int Iz = r - kGuard, Ix = c - kGuard;
    float out = 0.f, w = 0.f, a2 = 0.f;
    if (Iz >= 0 && Iz < s.Nz && Ix >= 0 && Ix < s.Nx) {
        int iz = min(max(Iz - s.ztop, 0), s.nz - 1);
        int ix = min(max(Ix - s.xleft, 0), s.nx - 1);
        float v = vp[(int64_t)iz * s.nx + ix];
        out = v * v * dt2;
        if (!(s.free_top && Iz == 0)) {
            const float gam = (s.gx[Ix] + s.gz[Iz]) * out;
            const float a = 1.f / (1.f + gam);
            w = a * out;
            a2 = 2.f * a;
        }
    }
    ((float *)s.V2)[q] = out;
    ((float *)s.W)[q] = w;
    ((float *)s.A2)[q] = a2;
}

__global__ void __launch_bounds__(256) k_zero(float *p, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.f;
}

// One time step n -> n+1 for every shot (blockIdx.z), one thread per padded
// cell, operands straight from global memory.  Also records level n.
__global__ void __launch_bounds__(256) k_step_naive(SliceDesc s, int n)
{
    const int Ix = blockIdx.x * 64 + threadIdx.x;
    const int Iz = blockIdx.y * 4 + threadIdx.y;
    const int shot = blockIdx.z;
    float *base = s.fields + (int64_t)shot * kFramesPerShot * s.frame;
    const float *cur = base + (n & 1) * s.frame;
    float *nxt = base + ((n + 1) & 1) * s.frame;   // level n-1 on entry

    const int tid = ((blockIdx.y * gridDim.x + blockIdx.x) * 4 + threadIdx.y) * 64 + threadIdx.x;
    const int nthr = gridDim.x * gridDim.y * 256;
    record_level(s, cur, shot, n, tid, nthr);

    if (Ix >= s.Nx || Iz >= s.Nz) return;
    if (s.free_top && Iz == 0) return;             // p = 0 on the free surface

    const int64_t i = (int64_t)(Iz + kGuard) * s.pitch + Ix + kGuard;
    const float c = cur[i], c2 = c + c, c4 = -4.f * c;
    const bool iso = s.cz[1] == s.cx[1] && s.cz[2] == s.cx[2] && s.cz[3] == s.cx[3] && s.cz[4] == s.cx[4];
    float lap = 0.f;
#pragma unroll
    for (int m = 1; m <= kHalo; ++m) {
        // above row 0 of a free top: odd mirror, p(Iz - m) = -p(m - Iz)
        const float up = (s.free_top && Iz - m < 0) ? -cur[i + (int64_t)(m - 2 * Iz) * s.pitch]
                                                    : cur[i - (int64_t)m * s.pitch];
        const float zs = cur[i + (int64_t)m * s.pitch] + up, xs = cur[i + m] + cur[i - m];
        // same expression as the tiled kernel: one weight per m when dz == dx
        lap = iso ? fmaf(s.cz[m], (zs + xs) + c4, lap) : lap_pair(lap, s.cz[m], s.cx[m], zs, xs, c2);
    }
    float amp = 0.f;
#pragma unroll
    for (int k = 0; k < kNodes; ++k)
        if (s.src_off[shot * kNodes + k] == (int32_t)i) amp += s.src_w[shot * kNodes + k];

    const float V2 = s.V2[i];
    const float gam = (s.gx[Ix] + s.gz[Iz]) * V2;
    const float a = 1.f / (1.f + gam);
    const float W = a * V2;
    float v = leapfrog(W, lap, 2.f * a, c, nxt[i]);
    if (amp != 0.f) v = fmaf(W, amp * wavelet_at(s, shot, n), v);
    nxt[i] = v;
}

// Records level n held in frame `slot` of every shot: the gather row when
// (what & 1), the snapshot when (what & 2), each only if that level is due.
__global__ void __launch_bounds__(256) k_record(SliceDesc s, int n, int slot, int what)
{
    const int shot = blockIdx.y;
    const float *cur = s.fields + ((int64_t)shot * kFramesPerShot + slot) * s.frame;
    if (!(what & 1)) s.gathers = nullptr;
    if (!(what & 2)) s.snaps = nullptr;
    record_level(s, cur, shot, n, blockIdx.x * 256 + threadIdx.x, gridDim.x * 256);
}

// Loads and stores through pointers that address global memory (device
// allocations).  Pointers read from memory (the batched item table) are not
// known to the compiler to be global, and a plain access through them would be
// a flat operation, which also holds up every LDS wait; the cast to the
// global address space makes it a global operation.
template <class T>
__device__ __forceinline__ T gload(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ void gstore(T *p, T v)
{
    *(__attribute__((address_space(1))) T *)p = v;
}
// The same at a byte offset from a base pointer.  Offsets within one stored
// field (or one ring level) stay far below 4 GiB; a 32-bit offset from a
// wave-uniform base is what the global load/store instructions take directly
// (base in scalar registers, offset in a vector register), so a row costs one
// vector add instead of 64-bit address arithmetic per array.
template <class T>
__device__ __forceinline__ T gload_at(const T *base, uint32_t byte_off)
{
    return gload((const T *)((const char *)base + byte_off));
}
template <class T>
__device__ __forceinline__ void gstore_at(T *base, uint32_t byte_off, T v)
{
    gstore((T *)((char *)base + byte_off), v);
}

// Streaming store (no reuse expected before the data leaves the caches).
// streaming load: data read once (it is not kept in the caches for reuse)
__device__ __forceinline__ float gload_nt_at(const float *base, uint32_t byte_off)
{
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) float *)((const char *)base + byte_off));
}
__device__ __forceinline__ void gstore_nt_at(float *base, uint32_t byte_off, float v)
{
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) float *)((char *)base + byte_off));
}

__device__ __forceinline__ RecEntry gload_rec(const RecEntry *p)
{
    RecEntry e;
    e.lds = gload(&p->lds);
    e.r = gload(&p->r);
#pragma unroll
    for (int j = 0; j < kNodes; ++j) e.w[j] = gload(&p->w[j]);
    return e;
}

// Maps a launch-order block index to a logical tile so that consecutive
// logical tiles (neighbours in one shot) land on the same XCD: the hardware
// deals workgroups round-robin over the 8 XCDs, each with its own L2.
__device__ inline int xcd_remap(int b, int nblocks)
{
    const int per = nblocks >> 3;
    if (b >= per * 8) return b;
    return (b & 7) * per + (b >> 3);
}

template <int K, int NWX, int NWZ>
struct TileShape {
    static constexpr int EX = 64 * NWX, EZ = K * NWZ, NTHR = 64 * NWX * NWZ;
    static constexpr int LW = EX + 2 * kHalo;    // LDS row: 4 pad cells each side
    static constexpr int LH = EZ + 2 * kHalo;
    static constexpr int LDS = LH * LW;          // floats per LDS buffer
};

// Time-blocked step (overlapped tiling).  One workgroup advances one tile of
// one shot by t.nsteps levels.  It loads the tile plus a halo of 4*tb cells
// (two levels) once, runs the sub-steps out of LDS, and writes the output tile
// (the last two levels) to the other field pair.  The level computed by
// sub-step s (1-based) is only needed on the loaded region shrunk by 4 s cells
// at every edge that is not a grid edge, so after tb sub-steps the output tile
// is exact; waves whose rows have all left that region stop computing.  Cells
// outside the padded grid are held at 0.  Under a free top the top tile row
// loads k ghost rows above row 0 and keeps rows -1..-4 equal to minus rows 1..4.
//
// Threads: 64 lanes across x (one wave covers 64 adjacent columns), waves
// stacked as NWX x NWZ; each thread owns one column and K consecutive rows,
// whose values stay in registers (z neighbours inside the column come from
// registers, only the 4 rows above and below and the x neighbours from LDS).
//
// MODE kFwd:  p^{n+1} = W L p^n + (2a (p^n - p^{n-1}) + p^{n-1}) + W S^n, with the
//             point sources S^n fused and the receivers of the tile sampled.
// MODE kRing: the same, also storing the second time difference
//             D^n = (p^{n+1} - p^n) - (p^n - p^{n-1}) of the output tile in ring
//             slot n - ring_lo (the forward recompute of the gradient; no receivers).
// MODE kAdj:  the transpose of that step map in the variable mu = W lambda,
//             the same stencil run backwards,
//               mu^k = W L mu^{k+1} + (2a (mu^{k+1} - mu^{k+2}) + mu^{k+2}) + W R^T r^k,
//             with the residual r^k of recorded levels injected at the receiver
//             nodes of the new level; alongside h += mu^{k+1} D^k for k <= nt-2,
//             D^k read from the ring (the velocity gradient is 2 / (dt^2 v^3) h:
//             the damping terms of the exact derivative cancel because eta does
//             not depend on v).  The launch's FP32 partial sum of h over its
//             levels is stored in the ring slot of its first level t.n (D^{t.n}
//             is dead once read; each output cell's slot is read and written by
//             its own thread only), and k_fold_partials adds the partials of a
//             segment to the FP64 accumulator in launch order.
enum { kFwd = 0, kRing = 1, kAdj = 2 };

template <int K, int NWX, int NWZ, int MODE, bool ISO, bool STREAM = false>
__device__ __forceinline__ void tiled_body(const SliceDesc &s, const TileArgs &t, int b, float *lds)
{
    using TS = TileShape<K, NWX, NWZ>;
    constexpr int EX = TS::EX, EZ = TS::EZ, NTHR = TS::NTHR, LW = TS::LW, NB = TS::LDS;
    constexpr bool ADJ = MODE == kAdj;
    const int tiles = t.ntx * t.ntz;
    const int shot = b / tiles;
    const int tile = b - shot * tiles;
    const int tzi = tile / t.ntx, txi = tile - tzi * t.ntx;
    const int halo = kHalo * t.tb;
    const bool top_tile = s.free_top && tzi == 0;
    int oz, oz_end, ez0;
    if (s.free_top) {
        oz = tzi == 0 ? 0 : t.tz_top + (tzi - 1) * t.tz;
        oz_end = tzi == 0 ? t.tz_top : oz + t.tz;
        ez0 = tzi == 0 ? -K : oz - halo;
    } else {
        oz = tzi * t.tz;
        oz_end = oz + t.tz;
        ez0 = oz - halo;
    }
    oz_end = min(oz_end, s.Nz);
    const int ox = txi * t.tx, ox_end = min(ox + t.tx, s.Nx), ex0 = ox - halo;

    // (the wave index stays a per-lane value: making it explicitly uniform
    // moves the row arithmetic to the scalar unit, which measured slower)
    const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
    const int lx = (w % NWX) * 64 + lane;        // local column in [0, EX)
    const int lz0 = (w / NWX) * K;               // first local row of this thread (wave-uniform)
    const int X = ex0 + lx, Z0 = ez0 + lz0;      // padded coordinates
    const bool xin = X >= 0 && X < s.Nx;
    const bool xout = X >= ox && X < ox_end;     // column inside the output tile
    // rows [k_lo, k_hi) of this thread's segment are output rows (wave-uniform)
    const int k_lo = __builtin_amdgcn_readfirstlane(min(max(oz - Z0, 0), K));
    const int k_hi = __builtin_amdgcn_readfirstlane(min(max(oz_end - Z0, 0), K));
    // segment entirely outside the grid rows, or the ghost segment of a top
    // tile (whose rows only the mirror writes)
    const int wave_x0 = ex0 + (w % NWX) * 64;
    const bool seg_dead = Z0 >= s.Nz || Z0 + K <= 0 || wave_x0 >= s.Nx || wave_x0 + 64 <= 0;
    const bool ghost_writer = top_tile && Z0 <= kHalo && Z0 + K > 1;

    const int64_t fshot = (int64_t)shot * kFramesPerShot * s.frame;
    const float *in_prev = t.fields + fshot + (int64_t)(2 * t.in_pair) * s.frame;
    const float *in_cur = in_prev + s.frame;
    float *out_prev = t.fields + fshot + (int64_t)(2 * t.out_pair) * s.frame;
    float *out_cur = out_prev + s.frame;
    // byte offset in a stored field of (row Z0 + k, column X): a uniform row
    // part rowb(k) plus the lane's column part xo4 (xc4 at the clamped column)
    auto rowb = [&](int k) { return (uint32_t)((Z0 + k + kGuard) * s.pitch) * 4u; };
    const uint32_t xo4 = (uint32_t)(X + kGuard) * 4u;
    // LDS index of this thread's row k = 0 (buffer 0); buffer 1 starts NB floats later
    const int lbase = (lz0 + kHalo) * LW + lx + kHalo;

    // ---- zero the LDS pad ring of both buffers (read only by cells whose
    // results are discarded; zero keeps every value finite)
    for (int q = threadIdx.x; q < 2 * kHalo * (LW + EZ); q += NTHR) {
        int r, c;
        if (q < 2 * kHalo * LW) {              // 4 rows on top, 4 at the bottom
            r = q / LW;
            c = q - r * LW;
            if (r >= kHalo) r += EZ;
        } else {                               // 4 columns left and right of each row
            const int q2 = q - 2 * kHalo * LW;
            r = kHalo + q2 / (2 * kHalo);
            c = q2 % (2 * kHalo);
            if (c >= kHalo) c += EX;
        }
        lds[r * LW + c] = 0.f;
        lds[NB + r * LW + c] = 0.f;
    }

    // ---- load the two input levels (registers; the newer one also to both
    // LDS buffers, so cells that are never recomputed keep their value) and
    // the coefficients W and 2a of every cell.  Cells the scheme does not
    // update (outside the padded grid, the pinned free-surface row) get
    // a2 = W = 0 and value 0, so the update keeps them 0.  A and B hold the two
    // live levels; their roles alternate every sub-step (the new level
    // overwrites the older one).  Every load is issued unconditionally from a
    // clamped, in-bounds cell (ghost rows above a free top read their mirror
    // row) and the values are selected afterwards, so the loads of all rows
    // are in flight together instead of one row after another.
    //
    // The newer level is loaded first and goes to LDS as soon as it arrives;
    // the older level and the coefficients are still in flight meanwhile.
    // Where every loaded cell has a = 1 (no sponge, no pinned row, inside the
    // grid; a box computed on the host) 2a is exactly 2 and is not loaded.
    //
    // The small tables (source nodes, this launch's wavelet samples, the
    // tile's receiver range and entries) are requested around the field loads
    // so that all of them travel together: used after the field loads, one
    // after another, they cost several dependent round trips.
    int psz[kNodes], psx[kNodes];
    float psw[kNodes];
    float pwav = 0.f;
    int32_t rbeg = 0, rend = 0;
    RecEntry prec{};
    if (!ADJ) {
#pragma unroll
        for (int j = 0; j < kNodes; ++j) {
            psz[j] = gload(s.src_iz + shot * kNodes + j);
            psx[j] = gload(s.src_ix + shot * kNodes + j);
            psw[j] = gload(s.src_w + shot * kNodes + j);
        }
        if ((int)threadIdx.x < t.nsteps) pwav = gload(s.wavelet + (int64_t)shot * s.wavelet_stride + t.n + threadIdx.x);
        if (MODE == kFwd && s.gathers) {
            rbeg = gload(s.tile_rec + tile);
            rend = gload(s.tile_rec + tile + 1);
        }
    }
    const int Xc = min(max(X, 0), s.Nx - 1);
    const bool unit_a = ez0 >= s.unit_z0 && ez0 + EZ <= s.unit_z1 && ex0 >= s.unit_x0 && ex0 + EX <= s.unit_x1;
    float A[K], B[K], a2[K], W[K];
    {
        float rc[K], rp[K], rw[K], ra[K];
        uint32_t ob[K];
        const uint32_t xc4 = (uint32_t)(Xc + kGuard) * 4u;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int Z = Z0 + k;
            const int Zr = min(Z < 0 ? -Z : Z, s.Nz - 1);
            ob[k] = (uint32_t)((Zr + kGuard) * s.pitch) * 4u + xc4;
            rc[k] = gload_at(in_cur, ob[k]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) rp[k] = gload_at(in_prev, ob[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) rw[k] = gload_at(s.W, ob[k]);
        if (unit_a) {
#pragma unroll
            for (int k = 0; k < K; ++k) ra[k] = 2.f;
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) ra[k] = gload_at(s.A2, ob[k]);
        }
        if (MODE == kFwd && rbeg + (int)threadIdx.x < rend) prec = gload_rec(s.rec_list + rbeg + threadIdx.x);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int Z = Z0 + k;
            const bool in = xin && Z >= 0 && Z < s.Nz;
            const bool ghost = top_tile && xin && Z < 0 && Z >= -kHalo;   // odd mirror of row -Z
            const float c = in ? rc[k] : (ghost ? -rc[k] : 0.f);
            A[k] = c;
            lds[lbase + k * LW] = c;
            lds[NB + lbase + k * LW] = c;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int Z = Z0 + k;
            const bool in = xin && Z >= 0 && Z < s.Nz;
            a2[k] = in ? ra[k] : 0.f;
            W[k] = in ? rw[k] : 0.f;
            B[k] = in ? rp[k] : 0.f;
        }
    }
    // the clamped column (in bounds for the output rows of any lane)
    const uint32_t xc4 = (uint32_t)(Xc + kGuard) * 4u;

    // forward: the source nodes of this shot inside the loaded region.  Each
    // thread keeps the (at most two) nodes in its own column segment: row and
    // weight; the wavelet samples of this launch go to LDS.  The receiver
    // entries of the tile: the first NTHR are copied to LDS.
    __shared__ float wav_s[kMaxTimeBlock];
    __shared__ RecEntry rec_s[MODE == kFwd ? NTHR : 1];
    bool has_src = false;
    int sk0 = -1, sk1 = -1;
    float sw0 = 0.f, sw1 = 0.f;
    if (!ADJ) {
#pragma unroll
        for (int j = 0; j < kNodes; ++j) {
            const int sz = psz[j], sx = psx[j];
            const float sw = psw[j];
            has_src |= sz >= ez0 && sz < ez0 + EZ && sx >= ex0 && sx < ex0 + EX;
            if (sx == X && sz >= Z0 && sz < Z0 + K && sw != 0.f) {
                if (sk0 < 0) {
                    sk0 = sz - Z0;
                    sw0 = sw;
                } else {
                    sk1 = sz - Z0;
                    sw1 = sw;
                }
            }
        }
        if (has_src && (int)threadIdx.x < t.nsteps) wav_s[threadIdx.x] = pwav;
        if (MODE == kFwd && rbeg + (int)threadIdx.x < rend) rec_s[threadIdx.x] = prec;
    }
    // adjoint: the residual injections W R^T r^n of this launch's levels at
    // the receiver nodes of the loaded region, summed (in a fixed order per
    // node) before the first sub-step when the tile has at most kInjE nodes
    constexpr int kInjE = ADJ ? 256 : 1;
    __shared__ float inj_a[kMaxTimeBlock * kInjE];
    __shared__ int inj_l[kInjE];
    int32_t ebeg = 0, eend = 0;
    if (ADJ) {
        ebeg = gload(t.inj.tile_start + tile);
        eend = gload(t.inj.tile_start + tile + 1);
    }
    const int E = eend - ebeg;
    const bool inj_pre = ADJ && E > 0 && E <= kInjE;
    if (inj_pre) {
        for (int q = threadIdx.x; q < (t.nsteps + 1) * E; q += NTHR) {
            const int st = q / E, e = q - st * E, eg = ebeg + e;
            if (st == t.nsteps) {
                inj_l[e] = gload(t.inj.lds + eg);
                continue;
            }
            const int n = t.n - st;
            float add = 0.f;
            if (n >= 1 && n % s.rec_every == 0) {
                const float *rrow = t.resid + ((int64_t)shot * s.nrow + n / s.rec_every) * s.nrec;
                float acc = 0.f;
                const int j1 = gload(t.inj.pstart + eg + 1);
                for (int j = gload(t.inj.pstart + eg); j < j1; ++j) acc += gload(t.inj.w + j) * gload(rrow + gload(t.inj.rid + j));
                const int iz = gload(t.inj.iz + eg), ix = gload(t.inj.ix + eg);
                const float v2 = gload(s.V2 + (int64_t)(iz + kGuard) * s.pitch + ix + kGuard);
                const float Wc = v2 / (1.f + (gload(s.gx + ix) + gload(s.gz + iz)) * v2);
                add = Wc * acc;
            }
            inj_a[st * kInjE + e] = add;
        }
    }
    // adjoint: the second time difference D^k of the forward field for the
    // imaging term (read one sub-step ahead, with streaming loads: each value
    // is read once), and the partial sums of h.  Only the output cells are
    // read and their sums stored.
    float pn[ADJ ? K : 1], hp[ADJ ? K : 1];
    const float *ringb = ADJ ? t.ring + (int64_t)shot * t.ring_shot : nullptr;
    auto ring_level = [&](int L, float(&dst)[ADJ ? K : 1]) {
        const bool h = xout && L >= t.ring_lo && L <= t.ring_hi;
        const float *rl = ringb + (int64_t)(h ? L - t.ring_lo : 0) * s.frame;
#pragma unroll
        for (int k = 0; k < K; ++k) dst[k] = (h && k >= k_lo && k < k_hi) ? gload_nt_at(rl, rowb(k) + xc4) : 0.f;
    };
    if (ADJ) {
        ring_level(t.n, pn);
#pragma unroll
        for (int k = 0; k < K; ++k) hp[k] = 0.f;
    }
    __syncthreads();

    // One sub-step.  PAR selects the roles: cur (level n forward, mu^{n+1}
    // adjoint) and old (the level before it, overwritten by the new level),
    // and the LDS buffer read (cur) and written (new).
    auto substep = [&](auto par, auto src, const int st) {
        constexpr bool PAR = decltype(par)::value;
        constexpr bool SRC = !ADJ && decltype(src)::value;   // this tile holds a source node
        float(&cur)[K] = PAR ? B : A;
        float(&old)[K] = PAR ? A : B;
        const int lc = PAR ? NB : 0, ln = PAR ? 0 : NB;
        const int n = ADJ ? t.n - st : t.n + st;

        if (MODE == kFwd && rend > rbeg && n % s.rec_every == 0) {
            // record level n: receivers whose base node is in this output tile
            float *row = s.gathers + ((int64_t)shot * s.nrow + n / s.rec_every) * s.nrec;
            const float *Lc = lds + lc;
            auto sample = [&](const RecEntry &e) {
                gstore(row + e.r, e.w[0] * Lc[e.lds] + e.w[1] * Lc[e.lds + 1] + e.w[2] * Lc[e.lds + LW] +
                                      e.w[3] * Lc[e.lds + LW + 1]);
            };
            if (rbeg + (int)threadIdx.x < rend) sample(rec_s[threadIdx.x]);
            for (int q = rbeg + NTHR + (int)threadIdx.x; q < rend; q += NTHR) sample(gload_rec(s.rec_list + q));
        }
        if (ADJ) {
            // imaging term n (needs mu^{n+1} = cur): h += mu^{n+1} D^n, then the
            // loads of D^{n-1} for the next sub-step go out, to land while this
            // sub-step computes
            if (n <= t.nt - 2) {
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k >= k_lo && k < k_hi) hp[k] = fmaf(cur[k], pn[k], hp[k]);
            }
            if (st + 1 < t.nsteps) ring_level(n - 1, pn);
        }

        // rows still needed after this sub-step (local rows [need_lo, need_hi))
        const int sdone = st + 1;
        const int need_lo = top_tile ? K : kHalo * sdone, need_hi = EZ - kHalo * sdone;
        const bool active = !seg_dead && lz0 + K > need_lo && lz0 < need_hi;
        if (active) {
            // the 4 rows above and below this thread's column segment
            float up[kHalo], dn[kHalo];
#pragma unroll
            for (int j = 0; j < kHalo; ++j) {
                up[j] = lds[lc + lbase + (j - kHalo) * LW];
                dn[j] = lds[lc + lbase + (K + j) * LW];
            }
            // x neighbours of row k: xv[m-1] = p(x+m), xv[kHalo+m-1] = p(x-m),
            // read one row ahead of the arithmetic.  The LDS byte address of
            // (row, x - 4) steps down one row per call in one register (the
            // empty asm keeps the optimiser from folding each row's offset
            // into the reads, which would cost an address add per read pair,
            // or from keeping every row's address live), so the eight reads
            // use small immediate offsets.
            int roff = (lc + lbase - kHalo) * 4;
            auto xrow = [&](float(&xv)[2 * kHalo]) {
                asm volatile("" : "+v"(roff));
                const float *rp = (const float *)((const char *)lds + roff);
#pragma unroll
                for (int m = 1; m <= kHalo; ++m) {
                    xv[m - 1] = rp[kHalo + m];
                    xv[kHalo + m - 1] = rp[kHalo - m];
                }
                roff += LW * 4;
            };
            // (the adjoint, short of registers, reads each row where it is used)
            constexpr bool kAhead = !ADJ;
            const float wav = SRC ? wav_s[st] : 0.f;
            // kRing: the ring slot of D^n (read back by the adjoint only after
            // the whole segment: streaming stores)
            float *rl_new = MODE == kRing ? t.ring + (int64_t)shot * t.ring_shot + (int64_t)(n - t.ring_lo) * s.frame
                                          : nullptr;
            float xa[2 * kHalo], xb[2 * kHalo];
            if (kAhead) xrow(xa);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!kAhead) xrow(xa);
                else if (k + 1 < K) xrow((k & 1) ? xa : xb);
                const float(&xv)[2 * kHalo] = (kAhead && (k & 1)) ? xb : xa;
                float lap = 0.f;
                if (ISO) {
                    // dz == dx: one weight per m, sum_m c_m ((z+m)+(z-m)+(x+m)+(x-m) - 4p)
                    const float c4 = -4.f * cur[k];
#pragma unroll
                    for (int m = 1; m <= kHalo; ++m) {
                        const float zp = k + m < K ? cur[k + m] : dn[k + m - K];
                        const float zm = k - m >= 0 ? cur[k - m] : up[k - m + kHalo];
                        lap = fmaf(s.cz[m], ((zp + zm) + (xv[m - 1] + xv[kHalo + m - 1])) + c4, lap);
                    }
                } else {
                    const float c2 = cur[k] + cur[k];
#pragma unroll
                    for (int m = 1; m <= kHalo; ++m) {
                        const float zp = k + m < K ? cur[k + m] : dn[k + m - K];
                        const float zm = k - m >= 0 ? cur[k - m] : up[k - m + kHalo];
                        lap = lap_pair(lap, s.cz[m], s.cx[m], zp + zm, xv[m - 1] + xv[kHalo + m - 1], c2);
                    }
                }
                float v = leapfrog(W[k], lap, a2[k], cur[k], old[k]);
                if (SRC) {
                    // p^{n+1} += W S^n at this thread's source nodes
                    if (k == sk0) v = fmaf(W[k], sw0 * wav, v);
                    if (k == sk1) v = fmaf(W[k], sw1 * wav, v);
                }
                if (MODE == kRing && k >= k_lo && k < k_hi && xout)
                    gstore_nt_at(rl_new, rowb(k) + xo4, (v - cur[k]) - (cur[k] - old[k]));   // D^n
                old[k] = v;
                lds[ln + lbase + k * LW] = v;
            }
        }

        // adjoint: the residual enters the new level in LDS, one thread per
        // node, after which the owners of those cells take their values back
        if (ADJ && eend > ebeg && n >= 1 && n % s.rec_every == 0) {
            __syncthreads();
            float *Ln = lds + ln;
            if (inj_pre) {
                for (int e = threadIdx.x; e < E; e += NTHR) Ln[inj_l[e]] += inj_a[st * kInjE + e];
            } else {
                const float *rrow = t.resid + ((int64_t)shot * s.nrow + n / s.rec_every) * s.nrec;
                for (int e = ebeg + (int)threadIdx.x; e < eend; e += NTHR) {
                    float acc = 0.f;
                    for (int q = t.inj.pstart[e]; q < t.inj.pstart[e + 1]; ++q) acc += t.inj.w[q] * rrow[t.inj.rid[q]];
                    const int iz = t.inj.iz[e], ix = t.inj.ix[e];
                    const float v2 = s.V2[(int64_t)(iz + kGuard) * s.pitch + ix + kGuard];
                    const float Wc = v2 / (1.f + (s.gx[ix] + s.gz[iz]) * v2);
                    Ln[t.inj.lds[e]] += Wc * acc;
                }
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int k = 0; k < K; ++k) old[k] = Ln[lbase + k * LW];
            }
        }
        if (active) {
            if (ghost_writer) {
                // ghost rows -1..-4 of the new level: minus rows 1..4
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int Z = Z0 + k;
                    if (Z >= 1 && Z <= kHalo) lds[ln + (-Z - ez0 + kHalo) * LW + lx + kHalo] = -old[k];
                }
            }
        }
        __syncthreads();
    };

    auto run = [&](auto src) {
        int st = 0;
        for (; st + 2 <= t.nsteps; st += 2) {
            substep(std::false_type{}, src, st);
            substep(std::true_type{}, src, st + 1);
        }
        if (st < t.nsteps) substep(std::false_type{}, src, st);
    };
    if (!ADJ && has_src)
        run(std::true_type{});
    else
        run(std::false_type{});
    // the newest level is in A after an even number of sub-steps, else in B
    const bool odd = t.nsteps & 1;

    // ---- write the output tile: the last two levels; the adjoint stores this
    // launch's partial imaging sums in the ring slot of level t.n
    float *hpart = ADJ ? t.ring + (int64_t)shot * t.ring_shot + (int64_t)(t.n - t.ring_lo) * s.frame : nullptr;
    // STREAM (a launch whose workgroups all run at once): the levels go out
    // with streaming (non-temporal) stores.  The next launch starts with cold
    // caches anyway, and the end of this one then has little dirty data left
    // to write back.
    if (xout) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k >= k_lo && k < k_hi) {
                const uint32_t ob = rowb(k) + xo4;
                const float vc = odd ? B[k] : A[k], vp = odd ? A[k] : B[k];
                if constexpr (STREAM) {
                    gstore_nt_at(out_cur, ob, vc);
                    gstore_nt_at(out_prev, ob, vp);
                } else {
                    gstore_at(out_cur, ob, vc);
                    gstore_at(out_prev, ob, vp);
                }
                if (ADJ) gstore_nt_at(hpart, ob, hp[k]);
            }
        }
    }
}

// Forward kernels ask for 4 waves per SIMD: two 512-thread workgroups share a
// CU, so one's loads and stores overlap the other's sub-steps.
#define SG_TILED_OCCUPANCY __attribute__((amdgpu_waves_per_eu(MODE == kAdj ? 1 : 4)))

template <int K, int NWX, int NWZ, int MODE, bool ISO, bool STREAM>
__global__ void __launch_bounds__(64 * NWX * NWZ) SG_TILED_OCCUPANCY k_tiled(SliceDesc s, TileArgs t)
{
    __shared__ float lds[2 * TileShape<K, NWX, NWZ>::LDS];
    tiled_body<K, NWX, NWZ, MODE, ISO, STREAM>(s, t, xcd_remap(blockIdx.x, gridDim.x), lds);
}

// Batched form: one launch covers every (slice, shot, tile) of the batch.
// Item i owns logical blocks [items[i].block_start, items[i+1].block_start);
// launch-level fields (levels, pairs) come from the arguments.
template <int K, int NWX, int NWZ, int MODE, bool ISO>
__global__ void __launch_bounds__(64 * NWX * NWZ) SG_TILED_OCCUPANCY k_tiled_batch(const BatchItem *__restrict__ items, int nitems,
                                                                 int n, int nsteps, int in_pair, int ring_lo, int ring_hi)
{
    __shared__ float lds[2 * TileShape<K, NWX, NWZ>::LDS];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    // the item owning logical block b is the last one starting at or before
    // b: its index is the count of such items minus one, found with one load
    // per lane (64 items per round) instead of a chain of dependent loads
    int it = 0;
    if (nitems > 1) {
        const int lane = threadIdx.x & 63;
        int count = 0;
        for (int base = 0; base < nitems; base += 64) {
            const int i = base + lane;
            const bool le = i < nitems && items[i].block_start <= b;
            count += __popcll(__ballot(le));
        }
        it = __builtin_amdgcn_readfirstlane(count - 1);
    }
    const SliceDesc s = items[it].s;     // local copies: plain registers, no aliasing with LDS
    TileArgs t = items[it].t;
    t.n = n;
    t.nsteps = nsteps;
    t.in_pair = in_pair;
    t.out_pair = in_pair ^ 1;
    t.ring_lo = ring_lo;
    t.ring_hi = ring_hi;
    tiled_body<K, NWX, NWZ, MODE, ISO>(s, t, b - items[it].block_start, lds);
}

__global__ void __launch_bounds__(256) k_copy(float *dst, int64_t dst_shot, const float *src, int64_t src_shot,
                                              int64_t n)
{
    const int shot = blockIdx.y;
    float *d = dst + (int64_t)shot * dst_shot;
    const float *sp = src + (int64_t)shot * src_shot;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = sp[i];
}

// Gradient on the physical grid: g(iz, ix) = 2 / (dt^2 v^3) * sum over shots
// and over the padded cells whose velocity is the copy of v(iz, ix) (the
// transpose of the edge replication into the sponge) of h = hsum.
__global__ void __launch_bounds__(256) k_fold_gradient(SliceDesc s, const float *vp, const double *hsum,
                                                       int64_t shot_stride, float dt,
                                                       float *grad, int accumulate)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s.nz * s.nx) return;
    const int iz = q / s.nx, ix = q - iz * s.nx;
    const int z_lo = iz == 0 ? 0 : iz + s.ztop, z_hi = iz == s.nz - 1 ? s.Nz - 1 : iz + s.ztop;
    const int x_lo = ix == 0 ? 0 : ix + s.xleft, x_hi = ix == s.nx - 1 ? s.Nx - 1 : ix + s.xleft;
    double acc = 0.0;
    for (int sh = 0; sh < s.nshot; ++sh) {
        const double *hs = hsum + (int64_t)sh * shot_stride;
        for (int Z = z_lo; Z <= z_hi; ++Z)
            for (int X = x_lo; X <= x_hi; ++X) {
                const int64_t i = (int64_t)(Z + kGuard) * s.pitch + X + kGuard;
                acc += hs[i];
            }
    }
    const double v = vp[q];
    const float g = (float)(2.0 / ((double)dt * dt * v * v * v) * acc);
    grad[q] = accumulate ? grad[q] + g : g;
}

// h += the FP32 partial sums of a segment's adjoint launches, in launch order
// (slots first, first - step, ...; nslot of them), per padded cell of every
// shot: the same FP64 additions, in the same order, as adding each launch's
// partial to h when the launch ends.
__global__ void __launch_bounds__(256) k_fold_partials(SliceDesc s, double *hsum, const float *ring, int64_t ring_shot,
                                                       int first, int step, int nslot)
{
    const int64_t per = (int64_t)s.Nz * s.Nx;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= per) return;
    const int shot = blockIdx.y;
    const int Z = (int)(q / s.Nx), X = (int)(q - (int64_t)Z * s.Nx);
    const int64_t i = (int64_t)(Z + kGuard) * s.pitch + X + kGuard;
    double *h = hsum + (int64_t)shot * s.frame + i;
    const float *r = ring + (int64_t)shot * ring_shot + i;
    double acc = *h;
    // eight slots' loads in flight at a time, added in order
    constexpr int kChunk = 8;
    for (int j0 = 0; j0 < nslot; j0 += kChunk) {
        float v[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c)
            v[c] = j0 + c < nslot ? r[(int64_t)(first - (j0 + c) * step) * s.frame] : 0.f;
#pragma unroll
        for (int c = 0; c < kChunk; ++c)
            if (j0 + c < nslot) acc += (double)v[c];
    }
    *h = acc;
}

__global__ void __launch_bounds__(256) k_count_nonfinite(const float *x, size_t n, unsigned int *count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    unsigned int bad = 0;
    for (; i < n; i += stride) bad += !isfinite(x[i]);
    if (bad) atomicAdd(count, bad);
}

}  // namespace

hipError_t launch_prepare(const SliceDesc &s, const float *vp, float dt2, hipStream_t st)
{
    const unsigned blocks = (unsigned)((s.frame + 255) / 256);
    hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, st, s, vp, dt2);
    return hipGetLastError();
}

hipError_t launch_zero(float *p, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_step_naive(const SliceDesc &s, int n, hipStream_t st)
{
    dim3 grid((s.Nx + 63) / 64, (s.Nz + 3) / 4, s.nshot);
    hipLaunchKernelGGL(k_step_naive, grid, dim3(64, 4), 0, st, s, n);
    return hipGetLastError();
}

hipError_t launch_record_slot(const SliceDesc &s, int n, int slot, hipStream_t st, int what)
{
    int work = s.nrec;
    if (s.snaps && s.nz * s.nx > work) work = s.nz * s.nx;
    unsigned blocks = (unsigned)((work + 255) / 256);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_record, dim3(blocks, s.nshot), dim3(256), 0, st, s, n, slot, what);
    return hipGetLastError();
}

namespace {
// (ex, ez, k) of the instantiations below; every one fits its register
// budget without spilling.
constexpr TiledShape kShapes[kTiledShapes] = {{128, 64, 8}, {64, 128, 16}, {64, 64, 8}, {128, 64, 16}};
}

TiledShape tiled_shape(int config) { return kShapes[config]; }

Tiling make_tiling(int Nz, int Nx, bool free_top, int ex, int ez, int k, int tb)
{
    Tiling T{};
    T.ex = ex;
    T.ez = ez;
    T.k = k;
    T.tb = tb;
    const int halo = kHalo * tb;
    T.tx = ex - 2 * halo;
    T.tz = ez - 2 * halo;
    T.tz_top = free_top ? ez - k - halo : T.tz;
    T.ok = T.tx >= 1 && T.tz >= 1 && T.tz_top >= 1 && k >= kHalo;
    if (!T.ok) return T;
    T.ntx = (Nx + T.tx - 1) / T.tx;
    T.ntz = free_top ? 1 + (Nz > T.tz_top ? (Nz - T.tz_top + T.tz - 1) / T.tz : 0) : (Nz + T.tz - 1) / T.tz;
    return T;
}

// Every mode is built in the isotropic form (dz == dx: the z and x weights
// are equal, one weight per m) and the general form.
template <int MODE, bool ISO>
static hipError_t launch_tiled_batch_iso(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps,
                                         int in_pair, int config, int ring_lo, int ring_hi, hipStream_t st)
{
    const dim3 g((unsigned)total_blocks);
#define SG_BATCH_LAUNCH(KK, NX, NZ, THR)                                                                    \
    hipLaunchKernelGGL((k_tiled_batch<KK, NX, NZ, MODE, ISO>), g, dim3(THR), 0, st, items, nitems, n, nsteps, \
                       in_pair, ring_lo, ring_hi)
    switch (config) {
    case 0: SG_BATCH_LAUNCH(8, 2, 8, 1024); break;
    case 1: SG_BATCH_LAUNCH(16, 1, 8, 512); break;
    case 2: SG_BATCH_LAUNCH(8, 1, 8, 512); break;
    case 3: SG_BATCH_LAUNCH(16, 2, 4, 512); break;
    default: return hipErrorInvalidValue;
    }
#undef SG_BATCH_LAUNCH
    return hipGetLastError();
}

hipError_t launch_step_tiled_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps,
                                   int in_pair, int config, bool iso, hipStream_t st)
{
    return iso ? launch_tiled_batch_iso<kFwd, true>(items, nitems, total_blocks, n, nsteps, in_pair, config, 0, 0, st)
               : launch_tiled_batch_iso<kFwd, false>(items, nitems, total_blocks, n, nsteps, in_pair, config, 0, 0, st);
}

hipError_t launch_ring_tiled_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps,
                                   int in_pair, int config, bool iso, int ring_lo, hipStream_t st)
{
    return iso ? launch_tiled_batch_iso<kRing, true>(items, nitems, total_blocks, n, nsteps, in_pair, config, ring_lo, 0, st)
               : launch_tiled_batch_iso<kRing, false>(items, nitems, total_blocks, n, nsteps, in_pair, config, ring_lo, 0, st);
}

hipError_t launch_adjoint_tiled_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps,
                                      int in_pair, int config, bool iso, int ring_lo, int ring_hi, hipStream_t st)
{
    return iso ? launch_tiled_batch_iso<kAdj, true>(items, nitems, total_blocks, n, nsteps, in_pair, config, ring_lo,
                                                    ring_hi, st)
               : launch_tiled_batch_iso<kAdj, false>(items, nitems, total_blocks, n, nsteps, in_pair, config, ring_lo,
                                                     ring_hi, st);
}

// Compute units of the current device (cached per device).
static int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

template <int MODE, bool ISO, bool STREAM>
static hipError_t launch_tiled_as(const SliceDesc &s, const TileArgs &t, int config, unsigned blocks, hipStream_t st)
{
    switch (config) {
    case 0: hipLaunchKernelGGL((k_tiled<8, 2, 8, MODE, ISO, STREAM>), dim3(blocks), dim3(1024), 0, st, s, t); break;
    case 1: hipLaunchKernelGGL((k_tiled<16, 1, 8, MODE, ISO, STREAM>), dim3(blocks), dim3(512), 0, st, s, t); break;
    case 2: hipLaunchKernelGGL((k_tiled<8, 1, 8, MODE, ISO, STREAM>), dim3(blocks), dim3(512), 0, st, s, t); break;
    case 3: hipLaunchKernelGGL((k_tiled<16, 2, 4, MODE, ISO, STREAM>), dim3(blocks), dim3(512), 0, st, s, t); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE, bool ISO>
static hipError_t launch_tiled(const SliceDesc &s, const TileArgs &t, int config, hipStream_t st)
{
    const unsigned blocks = (unsigned)(t.ntx * t.ntz * s.nshot);
    // all workgroups resident at once (one 1024-thread or two 512-thread
    // workgroups per compute unit): streaming stores for the output levels
    const bool one_round = blocks <= (unsigned)device_cus() * (config == 0 ? 1u : 2u);
    return one_round ? launch_tiled_as<MODE, ISO, true>(s, t, config, blocks, st)
                     : launch_tiled_as<MODE, ISO, false>(s, t, config, blocks, st);
}

static bool isotropic(const SliceDesc &s)
{
    for (int m = 1; m <= kHalo; ++m)
        if (s.cz[m] != s.cx[m]) return false;
    return true;
}

hipError_t launch_step_tiled(const SliceDesc &s, const TileArgs &t, int config, hipStream_t st)
{
    const bool iso = isotropic(s);
    if (t.ring) return iso ? launch_tiled<kRing, true>(s, t, config, st) : launch_tiled<kRing, false>(s, t, config, st);
    return iso ? launch_tiled<kFwd, true>(s, t, config, st) : launch_tiled<kFwd, false>(s, t, config, st);
}

hipError_t launch_adjoint_tiled(const SliceDesc &s, const TileArgs &t, int config, hipStream_t st)
{
    return isotropic(s) ? launch_tiled<kAdj, true>(s, t, config, st) : launch_tiled<kAdj, false>(s, t, config, st);
}

hipError_t launch_copy(float *dst, int64_t dst_shot, const float *src, int64_t src_shot, int64_t n, int nshot,
                       hipStream_t st)
{
    if (n <= 0 || nshot <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks, nshot), dim3(256), 0, st, dst, dst_shot, src, src_shot, n);
    return hipGetLastError();
}

hipError_t launch_fold_gradient(const SliceDesc &s, const float *vp, const double *hsum,
                                int64_t shot_stride, float dt, float *grad, hipStream_t st, bool accumulate)
{
    const unsigned blocks = (unsigned)((s.nz * s.nx + 255) / 256);
    hipLaunchKernelGGL(k_fold_gradient, dim3(blocks), dim3(256), 0, st, s, vp, hsum, shot_stride, dt, grad,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fold_partials(const SliceDesc &s, double *hsum, const float *ring, int64_t ring_shot, int first,
                                int step, int nslot, hipStream_t st)
{
    if (nslot <= 0) return hipSuccess;
    const int64_t per = (int64_t)s.Nz * s.Nx;
    hipLaunchKernelGGL(k_fold_partials, dim3((unsigned)((per + 255) / 256), (unsigned)s.nshot), dim3(256), 0, st, s,
                       hsum, ring, ring_shot, first, step, nslot);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float *x, size_t n, unsigned int *count, hipStream_t st)
{
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)blocks), dim3(256), 0, st, x, n, count);
    return hipGetLastError();
}

}  // namespace sg
