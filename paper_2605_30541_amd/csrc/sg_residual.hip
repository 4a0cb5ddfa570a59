// Residual of the discretised acoustic wave operator on a stack of wavefield
// frames (SubsurfaceGen, arXiv 2605.30541, App. F.5: the physics check applied
// to predicted wavefields), with the 8th-order Laplacian of App. E.3:
//   R_t = (u_{t+1} - 2 u_t + u_{t-1}) / dt^2 - v^2 L u_t.
//
// A workgroup owns a tile of 64 columns x 4K rows of the evaluated region and
// a run of consecutive frames.  Each thread keeps a strip of K rows of one
// column in registers, with the 4-row halo above and below, and walks through
// time: the levels t-1, t, t+1 of its strip roll through registers, so every
// frame is fetched once per run (the z-halo rows and the x-halo columns come
// from L2).  The x-neighbours of frame t go through a double-buffered LDS tile
// (one barrier per frame).  Arithmetic is FP32; R^2 and the squared second
// difference are summed in FP32 over each row of 16 lanes (K rows per lane,
// fixed DPP order), in FP64 beyond, and a second kernel adds the per-wave
// partials of every frame in a fixed order, so the sums do not depend on the
// launch or on scheduling.
// Bound: HBM, one frame read (4 B per evaluated cell) per frame.
#include "sg_internal.h"

#include <type_traits>

namespace sg {

namespace {

constexpr int kResK = 8;                 // rows per thread
constexpr int kResTileZ = 4 * kResK;     // rows per tile (4 waves)
constexpr int kResLdsW = 64 + 2 * kHalo; // LDS row length

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum of one value per lane over the wave, in a fixed order: FP32 within each
// row of 16 lanes (lane pairs, quads, half-rows, rows), then FP64 over the
// four rows as (row 0 + row 1) + (row 2 + row 3).  Wave-uniform result.
__device__ __forceinline__ double wave_total(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));  // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));  // row_mirror
    const int i = __float_as_int(v);
    const double r0 = __int_as_float(__builtin_amdgcn_readlane(i, 15));
    const double r1 = __int_as_float(__builtin_amdgcn_readlane(i, 31));
    const double r2 = __int_as_float(__builtin_amdgcn_readlane(i, 47));
    const double r3 = __int_as_float(__builtin_amdgcn_readlane(i, 63));
    return (r0 + r1) + (r2 + r3);
}

// Buffer resource over one frame: 32-bit byte offsets from a base held in
// scalar registers; a load past the end of the frame returns 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t frame_rsrc(const float *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
}
// (the load returns the 32 bits of the word; reinterpret them as a float)
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// One tile and run of frames of the residual pass per workgroup (grid: tiles
// x runs, remapped over the XCDs).
// partials[(t - 1) * slots + tile * 4 + wave][0..1] = the wave's sums of R^2
// and of the squared second difference for frame t.
//
// Three register strips rotate through the frames.  At step t strip A holds
// frame t (with its z-halo), B frame t - 1 and C frame t - 2: the step
// finishes the residual of frame t - 1 from the centre rows of A, B, C and the
// v^2 L u_{t-1} kept from the step before, then issues the loads of frame
// t + 1 into C, puts A in LDS and computes v^2 L u_t.  Loads are first used a
// full step after they are issued, and no register is copied between steps.
__global__ void __launch_bounds__(256) k_wave_residual(const float *__restrict__ frames, int nframes, int nz, int nx,
                                                       const float *__restrict__ vp, float dt2, double scale,
                                                       ResidualCoef cf, int z0, int run, double *__restrict__ partials)
{
    constexpr int K = kResK, S = K + 2 * kHalo;
    const int W = nx - 2 * kHalo;
    const int ntx = (W + 63) / 64;
    // Workgroups go to the 8 XCDs in turn; give each XCD a contiguous range
    // of (run, tile) pairs so that the halo rows and columns a tile shares
    // with its neighbours are fetched into one L2.
    const unsigned nblk = gridDim.x * gridDim.y, lin = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned per = nblk / 8, rem = nblk % 8, xcd = lin % 8;
    const unsigned logical = xcd * per + min(xcd, rem) + lin / 8;
    const int tile = (int)(logical % gridDim.x);
    const int runi = (int)(logical / gridDim.x);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ix = kHalo + (tile % ntx) * 64 + lane;
    const int zr = z0 + (tile / ntx) * kResTileZ + wv * K;  // first row of this strip
    const int zmax = nz - 1 - kHalo;                        // last evaluated row
    const bool colok = ix <= nx - 1 - kHalo;
    const int cx = min(ix, nx - 1);
    const int t0 = 1 + runi * run;
    const int t1 = min(nframes - 1, t0 + run);  // residuals of frames t0 .. t1-1
    const size_t F = (size_t)nz * nx;
    const uint32_t fbytes = (uint32_t)(4 * F);
    const int slots = gridDim.x * 4;
    const float c0 = cf.cz[0] + cf.cx[0];

    // strip rows zr-4 .. zr+K+3 as byte offsets inside a frame (rows above 0
    // are the odd mirror of rows below it; rows past the grid are clamped and
    // only feed rows that are not evaluated)
    uint32_t off[S];
    float sgn[kHalo];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int r = zr - kHalo + j;
        off[j] = 4u * (uint32_t)(min(r < 0 ? -r : r, nz - 1) * nx + cx);
        if (j < kHalo) sgn[j] = r < 0 ? -1.f : 1.f;
    }
    // x-halo columns of the tile: lanes 0..3 load column ix-4, lanes 60..63 column ix+4
    const bool halo = lane < kHalo || lane >= 64 - kHalo;
    const int hdx = lane < kHalo ? -kHalo : min(ix + kHalo, nx - 1) - cx;
    const int hcol = lane < kHalo ? lane : lane + 2 * kHalo;
    // the strip is inside the evaluated region (no masking), it reaches above row 0
    const bool whole = __all(colok) && zr + K - 1 <= zmax;
    const bool mirror = zr < kHalo;
    bool rowok[K];
    float w[K];  // (v dt)^2
    {
        const auto rv = frame_rsrc(vp, fbytes);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float v = bload(rv, off[k + kHalo]);
            w[k] = (v * v) * dt2;
            rowok[k] = colok && zr + k <= zmax;
        }
    }

    auto load_strip = [&](int t, float(&s)[S], float(&h)[K]) {
        const auto r = frame_rsrc(frames + (size_t)t * F, fbytes);
#pragma unroll
        for (int j = 0; j < S; ++j) s[j] = bload(r, off[j]);
        if (halo) {
#pragma unroll
            for (int k = 0; k < K; ++k) h[k] = bload(r, off[k + kHalo] + 4 * hdx);
        }
    };

    __shared__ float lds[2][kResTileZ][kResLdsW];
    float lap[K];
    // dt^2 R and the second difference of frame t - 1, squared and summed
    // over the strip's rows (all of them, or the evaluated ones)
    auto strip_sums = [&](auto masked, const float(&A)[S], const float(&B)[S], const float(&C)[S], float &r2,
                          float &d2) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float c = B[k + kHalo];
            const float d = (A[k + kHalo] - c) - (c - C[k + kHalo]);
            const float r = fmaf(-w[k], lap[k], d);
            if (!decltype(masked)::value || rowok[k]) {
                r2 = fmaf(r, r, r2);
                d2 = fmaf(d, d, d2);
            }
        }
    };
    auto step = [&](int t, float(&A)[S], float(&Ah)[K], const float(&B)[S], float(&C)[S], float(&Ch)[K]) {
        if (t > t0) {  // residual of frame t - 1
            float r2 = 0.f, d2 = 0.f;
            if (whole)
                strip_sums(std::false_type{}, A, B, C, r2, d2);
            else
                strip_sums(std::true_type{}, A, B, C, r2, d2);
            const double wr = wave_total(r2) * scale, wd = wave_total(d2) * scale;
            if (lane == 0) {
                double *p = partials + ((size_t)(t - 2) * slots + tile * 4 + wv) * 2;
                p[0] = wr;
                p[1] = wd;
            }
        }
        if (t < t1) {  // frame t + 1 into C; v^2 L u_t
            load_strip(t + 1, C, Ch);
            if (mirror) {
#pragma unroll
                for (int j = 0; j < kHalo; ++j) A[j] *= sgn[j];
            }
            float(*L)[kResLdsW] = lds[(t - t0) & 1] + wv * K;
#pragma unroll
            for (int k = 0; k < K; ++k) L[k][lane + kHalo] = A[k + kHalo];
            if (halo) {
#pragma unroll
                for (int k = 0; k < K; ++k) L[k][hcol] = Ah[k];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                float a = c0 * A[k + kHalo];
#pragma unroll
                for (int m = 1; m <= kHalo; ++m) {
                    a = fmaf(cf.cz[m], A[k + kHalo + m] + A[k + kHalo - m], a);
                    a = fmaf(cf.cx[m], L[k][lane + kHalo + m] + L[k][lane + kHalo - m], a);
                }
                lap[k] = a;
            }
        }
    };

    float X[S], Xh[K], Y[S], Yh[K], Z[S], Zh[K];
    {
        const auto r = frame_rsrc(frames + (size_t)(t0 - 1) * F, fbytes);
#pragma unroll
        for (int k = 0; k < K; ++k) Y[k + kHalo] = bload(r, off[k + kHalo]);
    }
    load_strip(t0, X, Xh);
    for (int t = t0;;) {
        step(t, X, Xh, Y, Z, Zh);
        if (++t > t1) break;
        step(t, Z, Zh, X, Y, Yh);
        if (++t > t1) break;
        step(t, Y, Yh, Z, X, Xh);
        if (++t > t1) break;
    }
}

// res2[t], dtt2[t] for frame t = blockIdx.x: thread k adds the partials of
// slots k, k + 256, ... in order, then a fixed tree over the threads (0 for
// the first and last frames).
__global__ void __launch_bounds__(256) k_sum_partials(const double *partials, int nframes, int slots, double *res2,
                                                      double *dtt2)
{
    const int t = blockIdx.x;
    double a = 0.0, b = 0.0;
    if (t >= 1 && t <= nframes - 2) {
        const double *p = partials + (size_t)(t - 1) * slots * 2;
        for (int k = threadIdx.x; k < slots; k += 256) {
            a += p[2 * k];
            b += p[2 * k + 1];
        }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    __shared__ double sa[4], sb[4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[wv] = a;
        sb[wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        res2[t] = (sa[0] + sa[1]) + (sa[2] + sa[3]);
        dtt2[t] = (sb[0] + sb[1]) + (sb[2] + sb[3]);
    }
}

int residual_tiles(int nz, int nx, int z0)
{
    const int W = nx - 2 * kHalo, H = nz - kHalo - z0;
    if (W <= 0 || H <= 0) return 0;
    return ((W + 63) / 64) * ((H + kResTileZ - 1) / kResTileZ);
}

}  // namespace

int wave_residual_slots(int nz, int nx, int z0)
{
    return residual_tiles(nz, nx, z0) * 4;
}

hipError_t launch_wave_residual(const float *frames, int nframes, int nz, int nx, const float *vp, double dt,
                                const ResidualCoef &cf, int z0, double *partials, double *res2, double *dtt2,
                                hipStream_t st)
{
    const int tiles = residual_tiles(nz, nx, z0);
    const int slots = tiles * 4;
    if (tiles > 0 && nframes >= 3) {
        // Split the frames into runs: each run re-reads two frames before its
        // first residual, and the grid runs in rounds of `resident` blocks, so
        // take the split with the fewest frame-steps per CU slot over all
        // rounds (ceil(blocks / resident) * (run + 2)), runs of 24 frames or
        // more.
        int dev = 0, ncu = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_wave_residual, 256, 0);
        if (e != hipSuccess) return e;
        const int64_t resident = std::max<int64_t>(1, (int64_t)ncu * per_cu);
        const int inner = nframes - 2;
        int best_run = inner;
        int64_t best = -1;
        for (int nrun = 1; nrun <= std::max(1, inner / 24); ++nrun) {
            const int run = (inner + nrun - 1) / nrun;
            const int64_t blocks = (int64_t)tiles * ((inner + run - 1) / run);
            const int64_t cost = (blocks + resident - 1) / resident * (run + 2);
            if (best < 0 || cost < best) {
                best = cost;
                best_run = run;
            }
        }
        const int nrun = (inner + best_run - 1) / best_run;
        hipLaunchKernelGGL(k_wave_residual, dim3((unsigned)tiles, (unsigned)nrun), dim3(256), 0, st, frames, nframes,
                           nz, nx, vp, (float)(dt * dt), 1.0 / (dt * dt * dt * dt), cf, z0, best_run, partials);
    }
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)nframes), dim3(256), 0, st, partials, nframes,
                       tiles > 0 && nframes >= 3 ? slots : 0, res2, dtt2);
    return hipGetLastError();
}

}  // namespace sg
