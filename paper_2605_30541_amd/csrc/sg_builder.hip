// Velocity-model builder modules of SubsurfaceGen (arXiv 2605.30541, App. B):
// the interbedded package of Deposit (Alg. 1), the fractal-noise displacement
// and vertical warp of Squish (Alg. 2) and the listric normal fault of Fault
// (Alg. 3); the last two pull the model through an 8-point Kaiser-windowed
// sinc (beta 6, weights normalised to sum 1, taps clamped to the axis).
// Volumes are [nz][ny][nx], x fastest.
//
// Deposit: one thread per (y, x) column of the band; the column's contacts in
// FP64 in LDS, the texture noise in FP64.
// Squish: one thread per (y, x) column.  The shift is constant down a column,
// so the 8 weights are computed once and the column streams through registers
// in blocks of 8 rows: one load and 8 FMAs per voxel (HBM-bound, 8 B per voxel
// read + written).
// Fault: a workgroup per brick of 4 x 4 rows of 64 voxels, four voxels per
// thread, the bricks dealt to the XCDs in groups.  The pull source is
// computed in FP64 (the frame and the angles of Alg. 3); voxels outside the
// taper are copied, the others take 8 x 8 x 8 taps (8 x 8 when ny = 1) with
// FP32 weights and sums.  The sinc weights are evaluated through identities
// (one sine per axis, the window as a polynomial), which makes them cheap next
// to the 512 taps.
#include "sg_internal.h"

#include <algorithm>
#include <cmath>

namespace sg {

namespace {

constexpr int kTaps = 8;
// four floats at any 4-byte-aligned address (one 16-byte load)
typedef float Float4u __attribute__((ext_vector_type(4), aligned(4)));
constexpr float kBeta = 6.f;
constexpr int kBrickZ = 16, kBrickY = 16, kBrickRows = kBrickZ * kBrickY;   // fault kernel
constexpr int kDepositThreads = 64;   // one wave per workgroup; its contacts fill up to 64 KB of LDS

// Normalised weights of the taps floor(s)-3 .. floor(s)+4 for the fractional
// part f = s - floor(s): tap j sits at t = f + 3 - j from the sample and
// weighs sinc(t) I0(beta sqrt(1 - (t/4)^2)) before normalisation.  Evaluated
// through identities, with one sine per axis: sin(pi t) = (-1)^(3-j) sin(pi f);
// I0(beta sqrt(u)) = sum_k (beta^2 u / 4)^k / (k!)^2, a polynomial in u
// (Horner; for beta = 6, where beta^2 u / 4 <= 9, the terms past k = 13 add
// less than 1e-10 of the sum, far below FP32 rounding); the constant factors
// 1/pi and 1/I0(beta) cancel in the normalisation.
__device__ inline void sinc_weights(float f, float (&w)[kTaps])
{
    constexpr int kTerms = 14;
    // 1 / (k!)^2, k = 0 .. 13
    constexpr float kInvFact2[kTerms] = {
        1.f, 1.f, 0.25f, 2.7777777777777778e-2f, 1.7361111111111111e-3f, 6.9444444444444444e-5f,
        1.9290123456790123e-6f, 3.9367598891408415e-8f, 6.1511873267825648e-10f, 7.5940584281266232e-12f,
        7.5940584281266232e-14f, 6.2760813455591927e-16f, 4.3583898233049949e-18f, 2.5789288895295828e-20f};
    const float q4 = 0.25f * kBeta * kBeta;
    const float s1 = sinpif(f);
    float sum = 0.f;
#pragma unroll
    for (int j = 0; j < kTaps; ++j) {
        const float t = f + 3.f - (float)j;
        // sinc(t) times pi; (-1)^(3-j) is +1 for odd j
        const float sc = t == 0.f ? 3.14159265358979f : ((j & 1) ? s1 : -s1) * __builtin_amdgcn_rcpf(t);
        const float q = q4 * fmaxf(1.f - 0.0625f * t * t, 0.f);
        float win = kInvFact2[kTerms - 1];
#pragma unroll
        for (int k = kTerms - 2; k >= 0; --k) win = fmaf(win, q, kInvFact2[k]);
        w[j] = sc * win;
        sum += w[j];
    }
    const float inv = 1.f / sum;
#pragma unroll
    for (int j = 0; j < kTaps; ++j) w[j] *= inv;
}

// Sum over octaves o of the periodic value noise of lattice o [gy][gx] at
// (u, w) 2^o (u along the columns), quintic fade, weight 2^-o (not yet divided
// by the sum of the weights).  FP64 coordinates; u, w bounded by the caller.
__device__ inline double fractal_sum(const float *lattice, int noct, int gy, int gx, double u, double w)
{
    double total = 0.0, f = 1.0;
    for (int o = 0; o < noct; ++o, f *= 2.0) {
        const double pu = u * f, pw = w * f;
        const double fu = floor(pu), fw = floor(pw);
        double tu = pu - fu, tw = pw - fw;
        tu = tu * tu * tu * (tu * (tu * 6.0 - 15.0) + 10.0);
        tw = tw * tw * tw * (tw * (tw * 6.0 - 15.0) + 10.0);
        const int64_t iu = (int64_t)fu, iw = (int64_t)fw;
        const int u0 = (int)(((iu % gx) + gx) % gx), u1 = (u0 + 1) % gx;
        const int w0 = (int)(((iw % gy) + gy) % gy), w1 = (w0 + 1) % gy;
        const float *L = lattice + (int64_t)o * gy * gx;
        const double v00 = L[w0 * gx + u0], v01 = L[w0 * gx + u1], v10 = L[w1 * gx + u0], v11 = L[w1 * gx + u1];
        total += ((v00 * (1 - tu) + v01 * tu) * (1 - tw) + (v10 * (1 - tu) + v11 * tu) * tw) / f;
    }
    return total;
}

__global__ void __launch_bounds__(256) k_fractal_noise2d(const float *lattice, int noct, int gy, int gx, int ny,
                                                          int nx, double dy, double dx, double inv_lam_y,
                                                          double inv_lam_x, double ca, double sa, double scale,
                                                          float *out)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)ny * nx) return;
    const int iy = (int)(q / nx), ix = (int)(q - (int64_t)iy * nx);
    const double Y = iy * dy, X = ix * dx;
    const double u = (X * ca + Y * sa) * inv_lam_x;
    const double w = (-X * sa + Y * ca) * inv_lam_y;
    out[q] = (float)(fractal_sum(lattice, noct, gy, gx, u, w) * scale);
}

__global__ void __launch_bounds__(256) k_squish(const float *__restrict__ v, int nz, int ny, int nx, double inv_dz,
                                                const float *__restrict__ shift, float *__restrict__ out)
{
    const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (col >= (int64_t)ny * nx) return;
    const int64_t plane = (int64_t)ny * nx;
    // sample position z + c, c = shift / dz: whole part c0, fraction f (c is
    // bounded before the integer cast; every tap index is clamped anyway)
    const double c = fmin(fmax((double)shift[col] * inv_dz, -1e9), 1e9);
    const double cf = floor(c);
    const int c0 = (int)cf;
    float w[kTaps];
    sinc_weights((float)(c - cf), w);
    const float *vc = v + col;
    // rows c0 - 3 + z .. c0 + 4 + z feed output row z; they come in blocks of
    // kChunk rows, so kChunk loads are in flight at a time, and the last 7
    // rows of a block carry over to the next (rows past either end clamped)
    constexpr int kChunk = 8;
    float buf[kChunk + kTaps - 1];
#pragma unroll
    for (int k = 0; k < kTaps - 1; ++k) buf[k] = vc[(int64_t)min(max(c0 - 3 + k, 0), nz - 1) * plane];
    for (int z0 = 0; z0 < nz; z0 += kChunk) {
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            buf[kTaps - 1 + k] = vc[(int64_t)min(max(z0 + c0 + 4 + k, 0), nz - 1) * plane];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < kTaps; ++j) acc = fmaf(w[j], buf[u + j], acc);
            if (z0 + u < nz) out[col + (int64_t)(z0 + u) * plane] = acc;
        }
#pragma unroll
        for (int k = 0; k < kTaps - 1; ++k) buf[k] = buf[kChunk + k];
    }
}

// Alg. 3's pull source of voxel (iz, iy, ix) in fractional cell indices (a
// rough surface moves the side test and the across-fault taper).
// Returns kFaultStill outside the taper (w = 0: the source is the voxel),
// kFaultFill where the source depth leaves [0, nz), else kFaultMoved.
constexpr int kFaultStill = 0, kFaultMoved = 1, kFaultFill = 2;

__device__ inline int fault_source(const FaultFrame &F, int nz, int iz, int iy, int ix, double &sz, double &sy,
                                   double &sx)
{
    const double Z = iz * F.dz, Y = iy * F.dy, X = ix * F.dx;
    const double qy = Y - F.cy, qx = X - F.cx, vv = Z - F.cz;
    const double h = qy * F.n_y + qx * F.n_x;
    const double az = qy * F.s_y + qx * F.s_x;
    const double r = sqrt(h * h + vv * vv);
    const double rho_s = fabs(az) * F.inv_die_s;
    // outside the taper along strike, or across it where the surface is
    // certainly the smooth one (the same expressions as below: the voxel
    // would be still), without the angle
    if (rho_s >= 1.0) return kFaultStill;
    if ((!F.rough || !(fabs(r - F.radius) < F.rough_reach)) && fabs(r - F.radius) * F.inv_die_r >= 1.0)
        return kFaultStill;
    const double t_old = atan2(vv, h);
    const double rho_t = fabs(t_old - F.theta0) * F.inv_die_t;
    double R = F.radius;   // where the fault surface is, at this (along strike, down dip) position
    if (F.rough && rho_t < 1.0 && rho_s < 1.0 && fabs(r - F.radius) < F.rough_reach) {
        const double u = fmin(fmax(az * F.inv_lam_s, -1e12), 1e12);
        const double w = fmin(fmax(F.radius * (t_old - F.theta0) * F.inv_lam_d, -1e12), 1e12);
        const double N = fractal_sum(F.rough, F.rough_noct, F.rough_gd, F.rough_gs, u, w) * F.rough_inv_norm;
        R = F.radius + F.rough_amp * N;
    }
    const double rho_r = fabs(r - R) * F.inv_die_r;
    if (!(rho_r < 1.0 && rho_t < 1.0 && rho_s < 1.0)) return kFaultStill;
    const double half_pi = 1.5707963267948966;
    const double wt = cos(half_pi * rho_r) * cos(half_pi * rho_t) * cos(half_pi * rho_s);
    const double chi = r >= R ? 1.0 : -1.0;
    const double dth = -chi * F.direction * wt * F.shift;
    // p_fwd - p in the (h, v) plane, exactly 0 where the rotation is 0
    const double mid = t_old + 0.5 * dth, hs = sin(0.5 * dth);
    const double dh = -2.0 * r * sin(mid) * hs, dv = 2.0 * r * cos(mid) * hs;
    sz = (Z - dv) * F.inv_dz;
    sy = (Y - dh * F.n_y) * F.inv_dy;
    sx = (X - dh * F.n_x) * F.inv_dx;
    return sz >= 0.0 && sz < (double)nz ? kFaultMoved : kFaultFill;
}

// Voxels [z0, z0 + bz) x [y0, y0 + by) x [x0, x0 + bx) of the volume.
struct VoxBox {
    int z0, y0, x0, bz, by, bx;
};

// The box is cut in bricks of kBrickZ x kBrickY rows of 256 columns, one
// workgroup per row.  Workgroups go to the 8 XCDs in turn; here all rows of a
// brick go to one XCD (the rows its voxels sample are then fetched into one
// L2) and the bricks are dealt round-robin (the moved region of a fault stays
// spread over the XCDs).  False for threads past the box.
__device__ inline bool brick_voxel(const VoxBox &B, int &iz, int &iy, int &ix)
{
    const int bx_n = (B.bx + 255) / 256, by_n = (B.by + kBrickY - 1) / kBrickY;
    const int64_t nbrick = (int64_t)bx_n * by_n * ((B.bz + kBrickZ - 1) / kBrickZ);
    const int64_t t = blockIdx.x / 8;
    const int64_t brick = (t / kBrickRows) * 8 + blockIdx.x % 8;
    if (brick >= nbrick) return false;
    const int row = (int)(t % kBrickRows);
    const int bx = (int)(brick % bx_n);
    const int64_t rest = brick / bx_n;
    const int by = (int)(rest % by_n), bz = (int)(rest / by_n);
    const int lz = bz * kBrickZ + row / kBrickY, ly = by * kBrickY + row % kBrickY, lx = bx * 256 + threadIdx.x;
    iz = B.z0 + lz;
    iy = B.y0 + ly;
    ix = B.x0 + lx;
    return lz < B.bz && ly < B.by && lx < B.bx;
}

// The taps of a moved voxel: source index origin (z0, y0, x0) = floor(s) - 3
// per axis (y and x bounded first) and the FP32 fractions of s.
struct FaultTaps {
    int z0, y0, x0;
    float fz, fy, fx;
};

__device__ inline FaultTaps fault_taps(double sz, double sy, double sx)
{
    // (bounded before the integer casts; every tap index is clamped anyway)
    const double cy = fmin(fmax(sy, -1e9), 1e9), cx = fmin(fmax(sx, -1e9), 1e9);
    const double fz = floor(sz), fy = floor(cy), fx = floor(cx);
    return FaultTaps{(int)fz - 3, (int)fy - 3, (int)fx - 3, (float)(sz - fz), (float)(cy - fy), (float)(cx - fx)};
}

// The 8 x 8 x 8 pull from memory (8 x 8 on a one-row y axis): for each z tap
// the sum over y rows of the 8-tap x sums, every index clamped to the volume.
__device__ inline float fault_pull(const float *__restrict__ v, int nz, int ny, int nx, int z0, int y0, int x0,
                                  float fz, float fy, float fx)
{
    const int64_t plane = (int64_t)ny * nx;
    float wz[kTaps], wy[kTaps], wx[kTaps];
    sinc_weights(fz, wz);
    sinc_weights(fy, wy);
    sinc_weights(fx, wx);
    int jx[kTaps];
#pragma unroll
    for (int c = 0; c < kTaps; ++c) jx[c] = min(max(x0 + c, 0), nx - 1);
    // away from the row ends the 8 x taps are consecutive: two 16-byte loads
    const bool x_inner = x0 >= 0 && x0 + kTaps <= nx;
    auto row_taps = [&](const float *row) {
        float s = 0.f;
        if (x_inner) {
            const Float4u lo = *(const Float4u *)(row + x0), hi = *(const Float4u *)(row + x0 + 4);
            s = fmaf(wx[0], lo.x, s);
            s = fmaf(wx[1], lo.y, s);
            s = fmaf(wx[2], lo.z, s);
            s = fmaf(wx[3], lo.w, s);
            s = fmaf(wx[4], hi.x, s);
            s = fmaf(wx[5], hi.y, s);
            s = fmaf(wx[6], hi.z, s);
            s = fmaf(wx[7], hi.w, s);
        } else {
#pragma unroll
            for (int c = 0; c < kTaps; ++c) s = fmaf(wx[c], row[jx[c]], s);
        }
        return s;
    };
    float acc = 0.f;
    if (x_inner && ny > 1) {
        // the row loads of half a z tap (8 16-byte loads) are issued before
        // any is used (load latency overlaps across rows); same arithmetic
        // order as row_taps
        constexpr int kHalf = kTaps / 2;
        int64_t ry[kTaps];
#pragma unroll
        for (int b = 0; b < kTaps; ++b) ry[b] = (int64_t)min(max(y0 + b, 0), ny - 1) * nx + x0;
#pragma unroll
        for (int a = 0; a < kTaps; ++a) {
            const float *pl = v + (int64_t)min(max(z0 + a, 0), nz - 1) * plane;
            float accy = 0.f;
#pragma unroll
            for (int h = 0; h < kTaps; h += kHalf) {
                Float4u lo[kHalf], hi[kHalf];
#pragma unroll
                for (int b = 0; b < kHalf; ++b) {
                    lo[b] = *(const Float4u *)(pl + ry[h + b]);
                    hi[b] = *(const Float4u *)(pl + ry[h + b] + 4);
                }
#pragma unroll
                for (int b = 0; b < kHalf; ++b) {
                    float s = 0.f;
                    s = fmaf(wx[0], lo[b].x, s);
                    s = fmaf(wx[1], lo[b].y, s);
                    s = fmaf(wx[2], lo[b].z, s);
                    s = fmaf(wx[3], lo[b].w, s);
                    s = fmaf(wx[4], hi[b].x, s);
                    s = fmaf(wx[5], hi[b].y, s);
                    s = fmaf(wx[6], hi[b].z, s);
                    s = fmaf(wx[7], hi[b].w, s);
                    accy = fmaf(wy[h + b], s, accy);
                }
            }
            acc = fmaf(wz[a], accy, acc);
        }
        return acc;
    }
#pragma unroll
    for (int a = 0; a < kTaps; ++a) {
        const int jz = min(max(z0 + a, 0), nz - 1);
        float accy = 0.f;
        if (ny == 1) {
            accy = row_taps(v + (int64_t)jz * plane);   // the y weights sum to 1 on a one-row axis
        } else {
#pragma unroll
            for (int b = 0; b < kTaps; ++b) {
                const int jy = min(max(y0 + b, 0), ny - 1);
                accy = fmaf(wy[b], row_taps(v + (int64_t)jz * plane + (int64_t)jy * nx), accy);
            }
        }
        acc = fmaf(wz[a], accy, acc);
    }
    return acc;
}

// Fault pull by bricks: a workgroup takes kSbZ x kSbY rows of 64 voxels (wave
// w takes y row w of the brick, each thread its kSbZ voxels down z, in
// columns 64 wide); each thread computes the pull
// sources of its rows first (FP64; still and filled voxels are written at
// once), keeping the taps of its moved voxels in LDS, then pulls them one
// after another.  Bricks go to the XCDs in groups of kSbGroup x kSbGroup
// bricks (y, z), so the source rows that neighbouring bricks share are
// fetched into one L2.
constexpr int kSbZ = 4, kSbY = 4, kSbPer = kSbZ * kSbY / 4, kSbGroup = 4;

struct BrickGrid {
    int nbx, ncy, ncz;   // bricks along x, brick groups along y and z
};

inline BrickGrid brick_grid(const VoxBox &B)
{
    const int nby = (B.by + kSbY - 1) / kSbY, nbz = (B.bz + kSbZ - 1) / kSbZ;
    return BrickGrid{(B.bx + 63) / 64, (nby + kSbGroup - 1) / kSbGroup, (nbz + kSbGroup - 1) / kSbGroup};
}

inline int64_t brick_blocks(const VoxBox &B)
{
    const BrickGrid g = brick_grid(B);
    const int64_t ngroup = (int64_t)g.nbx * g.ncy * g.ncz;
    return (ngroup + 7) / 8 * 8 * (kSbGroup * kSbGroup);
}

__global__ void __launch_bounds__(256) k_fault(const float *__restrict__ v, int nz, int ny, int nx, VoxBox B,
                                               BrickGrid G, FaultFrame F, float fill, float *__restrict__ out)
{
    __shared__ FaultTaps ptap[kSbPer][256];   // the taps of each thread's moved voxels
    // the group of this workgroup: consecutive blocks of one XCD (every 8th
    // block) take the kSbGroup^2 bricks of one group
    const int64_t j = blockIdx.x / 8;
    const int64_t group = (j / (kSbGroup * kSbGroup)) * 8 + blockIdx.x % 8;
    if (group >= (int64_t)G.nbx * G.ncy * G.ncz) return;
    const int r = (int)(j % (kSbGroup * kSbGroup));
    const int gbx = (int)(group % G.nbx);
    const int64_t rest = group / G.nbx;
    const int by = (int)(rest % G.ncy) * kSbGroup + r % kSbGroup, bz = (int)(rest / G.ncy) * kSbGroup + r / kSbGroup;
    if (by * kSbY >= B.by || bz * kSbZ >= B.bz) return;

    const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
    const int64_t plane = (int64_t)ny * nx;
    const int ix = B.x0 + gbx * 64 + lane;
    // row k of this thread is z offset k, y offset w in the brick
    const int iy = B.y0 + by * kSbY + w;
    auto voxel = [&](int k) { return (int64_t)(B.z0 + bz * kSbZ + k) * plane + (int64_t)iy * nx + ix; };
    if (iy >= B.y0 + B.by || ix >= B.x0 + B.bx) return;
    unsigned moved = 0;   // bit k: row k's voxel takes the pull
#pragma unroll
    for (int k = 0; k < kSbPer; ++k) {
        const int iz = B.z0 + bz * kSbZ + k;
        if (iz >= B.z0 + B.bz) continue;
        const int64_t q = voxel(k);
        double sz, sy, sx;
        const int kind = fault_source(F, nz, iz, iy, ix, sz, sy, sx);
        if (kind == kFaultStill) {   // w = 0: the source is the voxel itself
            out[q] = v[q];
        } else if (kind == kFaultFill) {
            out[q] = fill;
        } else {
            moved |= 1u << k;
            ptap[k][threadIdx.x] = fault_taps(sz, sy, sx);
        }
    }
#pragma unroll 1
    for (int k = 0; k < kSbPer; ++k)
        if (moved >> k & 1u) {
            const FaultTaps P = ptap[k][threadIdx.x];
            out[voxel(k)] = fault_pull(v, nz, ny, nx, P.z0, P.y0, P.x0, P.fz, P.fy, P.fx);
        }
}

// Alg. 3 for integer fields (e.g. layer labels): the same pull source,
// sampled at the nearest voxel (floor(s + 0.5) per axis; y and x clamped to
// the volume); `fill` where the source depth leaves [0, nz).
__global__ void __launch_bounds__(256) k_fault_labels(const int32_t *__restrict__ lab, int nz, int ny, int nx,
                                                      VoxBox B, FaultFrame F, int32_t fill,
                                                      int32_t *__restrict__ out)
{
    int iz, iy, ix;
    if (!brick_voxel(B, iz, iy, ix)) return;
    const int64_t plane = (int64_t)ny * nx;
    const int64_t q = (int64_t)iz * plane + (int64_t)iy * nx + ix;
    double sz, sy, sx;
    const int kind = fault_source(F, nz, iz, iy, ix, sz, sy, sx);
    if (kind == kFaultStill) {
        out[q] = lab[q];
        return;
    }
    if (kind == kFaultFill) {
        out[q] = fill;
        return;
    }
    const int jz = min((int)floor(sz + 0.5), nz - 1);
    const int jy = (int)fmin(fmax(floor(sy + 0.5), 0.0), (double)(ny - 1));
    const int jx = (int)fmin(fmax(floor(sx + 0.5), 0.0), (double)(nx - 1));
    out[q] = lab[(int64_t)jz * plane + (int64_t)jy * nx + jx];
}

// 3D simplex noise (Perlin's simplex noise as formulated by Gustavson,
// "Simplex noise demystified", 2005), FP64, at lattice coordinates (a, b, c):
// skew by 1/3 onto the cubic lattice, pick the tetrahedron of the cube cell
// by the order of the unskewed offsets, and add over its four corners
// (0.6 - |d|^2)^4 (g . d) where positive, g the cube-edge midpoint chosen by
// the corner's hash P[i + P[j + P[k]]] mod 12 (indices mod 256); times 32.
// P: 256 entries in 0..255 (LDS).  With the published radius 0.6 a corner's
// kernel reaches past the faces of its tetrahedron, so the field jumps
// slightly across them; which tetrahedron a point on a face takes is decided
// by IEEE operations without fusion (a sum, a division, floor, differences),
// the same decision as any IEEE evaluation of the same coordinates.
__device__ inline double simplex_corner(const int *P, int i, int j, int k, double x, double y, double z)
{
    const double w = 0.6 - (x * x + y * y + z * z);
    if (!(w > 0.0)) return 0.0;
    const int h = P[(i + P[(j + P[k & 255]) & 255]) & 255] % 12;
    double dot;
    switch (h) {
    case 0: dot = x + y; break;
    case 1: dot = -x + y; break;
    case 2: dot = x - y; break;
    case 3: dot = -x - y; break;
    case 4: dot = x + z; break;
    case 5: dot = -x + z; break;
    case 6: dot = x - z; break;
    case 7: dot = -x - z; break;
    case 8: dot = y + z; break;
    case 9: dot = -y + z; break;
    case 10: dot = y - z; break;
    default: dot = -y - z; break;
    }
    const double w2 = w * w;
    return w2 * w2 * dot;
}

__device__ inline double simplex3(const int *P, double a, double b, double c)
{
    const double s = (a + b + c) / 3.0;
    const double fi = floor(a + s), fj = floor(b + s), fk = floor(c + s);
    const double t = (fi + fj + fk) / 6.0;
    const double x0 = a - (fi - t), y0 = b - (fj - t), z0 = c - (fk - t);
    // corners 1 and 2 step along the largest, then the two largest offsets
    // (ties: the lower axis first)
    int i1, j1, k1, i2, j2, k2;
    if (x0 >= y0) {
        if (y0 >= z0) { i1 = 1; j1 = 0; k1 = 0; i2 = 1; j2 = 1; k2 = 0; }
        else if (x0 >= z0) { i1 = 1; j1 = 0; k1 = 0; i2 = 1; j2 = 0; k2 = 1; }
        else { i1 = 0; j1 = 0; k1 = 1; i2 = 1; j2 = 0; k2 = 1; }
    } else {
        if (y0 < z0) { i1 = 0; j1 = 0; k1 = 1; i2 = 0; j2 = 1; k2 = 1; }
        else if (x0 < z0) { i1 = 0; j1 = 1; k1 = 0; i2 = 0; j2 = 1; k2 = 1; }
        else { i1 = 0; j1 = 1; k1 = 0; i2 = 1; j2 = 1; k2 = 0; }
    }
    const int i = (int)(int64_t)fi & 255, j = (int)(int64_t)fj & 255, k = (int)(int64_t)fk & 255;
    double n = simplex_corner(P, i, j, k, x0, y0, z0);
    n += simplex_corner(P, i + i1, j + j1, k + k1, x0 - i1 + 1.0 / 6.0, y0 - j1 + 1.0 / 6.0, z0 - k1 + 1.0 / 6.0);
    n += simplex_corner(P, i + i2, j + j2, k + k2, x0 - i2 + 2.0 / 6.0, y0 - j2 + 2.0 / 6.0, z0 - k2 + 2.0 / 6.0);
    n += simplex_corner(P, i + 1, j + 1, k + 1, x0 - 1.0 + 0.5, y0 - 1.0 + 0.5, z0 - 1.0 + 0.5);
    return 32.0 * n;
}

// A permutation table into LDS (entries taken mod 256); all threads call it.
__device__ inline void load_perm(const int32_t *perm, int *P)
{
    for (int q = threadIdx.x; q < 256; q += blockDim.x) P[q] = perm[q] & 255;
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_simplex3d(const int32_t *__restrict__ perm, int nz, int ny, int nx,
                                                   double oz, double oy, double ox, double sz, double sy, double sx,
                                                   double amplitude, float *__restrict__ out)
{
    __shared__ int P[256];
    load_perm(perm, P);
    const int64_t n = (int64_t)nz * ny * nx;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t zy = q / nx;
        const int ix = (int)(q - zy * nx), iz = (int)(zy / ny), iy = (int)(zy - (int64_t)iz * ny);
        // o + i s rounded twice, never fused: the published noise jumps across
        // the tetrahedron faces, so the coordinates must round as specified
        double a, b, c;
        {
#pragma clang fp contract(off)
            a = oz + iz * sz;
            b = oy + iy * sy;
            c = ox + ix * sx;
        }
        out[q] = (float)(amplitude * simplex3(P, a, b, c));
    }
}

// Deposit (Alg. 1, boundary path): one thread per (y, x) column, walking down
// the band [t][ny][nx].  The contacts are the cumulative bed thicknesses
// (summed in FP64 in bed order), each moved by taper x a_B x its noise and
// clamped to the band; they are computed once per column into LDS (FP64,
// [contact][lane]), and at every depth the voxel's bed is the number of
// contacts at or above it, starting at the deepest of those; the texture is
// sampled at the depth below that start plus the bed's offset.  SIMPLEX: the
// contact noise is simplex noise (perm_b) on the plane at the contact's mean
// depth and the texture simplex noise (perm_t); else the contact noise is an
// input and the texture value noise on a lattice.
template <bool SIMPLEX>
__global__ void __launch_bounds__(kDepositThreads) k_deposit(DepositArgs A, float *__restrict__ out)
{
    extern __shared__ double hcol[];   // [nbeds - 1][kDepositThreads]
    __shared__ int Pb[SIMPLEX ? 256 : 1], Pt[SIMPLEX ? 256 : 1];
    if (SIMPLEX) {
        load_perm(A.perm_b, Pb);
        load_perm(A.perm_t, Pt);
    }
    const int64_t plane = (int64_t)A.ny * A.nx;
    const int64_t col = (int64_t)blockIdx.x * kDepositThreads + threadIdx.x;
    if (col >= plane) return;
    const int iy = (int)(col / A.nx), ix = (int)(col - (int64_t)iy * A.nx);
    const double t = A.t;
    // taper min(d / (f_top t), 1) min((t - d) / (f_base t), 1), by reciprocals
    // (no division per contact)
    const double rt = 1.0 / (A.f_top * t), rb = 1.0 / (A.f_base * t);
    auto tau = [&](double d) { return fmin(d * rt, 1.0) * fmin((t - d) * rb, 1.0); };
    double vsum = 0.0;
    for (int k = 0; k < A.nbeds; ++k) vsum += (double)A.vbed[k];
    const double vbar = vsum / A.nbeds;
    auto fade = [](double u) { return u * u * u * (u * (u * 6.0 - 15.0) + 10.0); };
    auto wrap = [](double f, int g) { const int64_t i = (int64_t)f % g; return (int)(i < 0 ? i + g : i); };
    auto L = [&](int a, int b, int c) { return (double)A.lattice[((int64_t)a * A.gy + b) * A.gx + c]; };
    double ty = 0.0, tx = 0.0, by = 0.0, bx = 0.0;
    int y0 = 0, x0 = 0, y1 = 0, x1 = 0;
    if (SIMPLEX) {
        ty = iy * A.dy / A.lam_t[1];
        tx = ix * A.dx / A.lam_t[2];
        by = iy * A.dy / A.lam_b[1];
        bx = ix * A.dx / A.lam_b[2];
    } else {
        const double py = iy * A.dy * A.inv_lam_y, px = ix * A.dx * A.inv_lam_x;
        const double fy = floor(py), fx = floor(px);
        ty = fade(py - fy);
        tx = fade(px - fx);
        y0 = wrap(fy, A.gy);
        x0 = wrap(fx, A.gx);
        y1 = (y0 + 1) % A.gy;
        x1 = (x0 + 1) % A.gx;
    }
    {
        double H = 0.0;
        for (int i = 0; i + 1 < A.nbeds; ++i) {
            H += (double)A.thick[i];
            const double eta =
                SIMPLEX ? simplex3(Pb, H * A.dz / A.lam_b[0], by, bx) : (double)A.eta_b[(int64_t)i * plane + col];
            hcol[i * kDepositThreads + threadIdx.x] = fmin(fmax(H + tau(H) * A.a_B * eta, 0.0), t - 1.0);
        }
    }
    for (int iz = 0; iz < A.t; ++iz) {
        const double z = iz;
        int bed = 0;
        double start = 0.0;
        for (int i = 0; i + 1 < A.nbeds; ++i) {
            const double h = hcol[i * kDepositThreads + threadIdx.x];
            if (h <= z) {
                ++bed;
                start = fmax(start, h);
            }
        }
        // texture at ((z - start) dz + offset, y dy, x dx)
        double eta;
        if (SIMPLEX) {
            // (z - start) dz + offset rounded twice, never fused (see k_simplex3d)
            double zt;
            {
#pragma clang fp contract(off)
                zt = ((z - start) * A.dz + (double)A.tex_off[bed]) / A.lam_t[0];
            }
            eta = simplex3(Pt, zt, ty, tx);
        } else {
            const double pz = ((z - start) * A.dz + (double)A.tex_off[bed]) * A.inv_lam_z;
            const double fz = floor(pz);
            const double tz = fade(pz - fz);
            const int z0 = wrap(fz, A.gz), z1 = (z0 + 1) % A.gz;
            eta = (1 - tz) * ((1 - ty) * ((1 - tx) * L(z0, y0, x0) + tx * L(z0, y0, x1)) +
                              ty * ((1 - tx) * L(z0, y1, x0) + tx * L(z0, y1, x1))) +
                  tz * ((1 - ty) * ((1 - tx) * L(z1, y0, x0) + tx * L(z1, y0, x1)) +
                        ty * ((1 - tx) * L(z1, y1, x0) + tx * L(z1, y1, x1)));
        }
        out[(int64_t)iz * plane + col] =
            (float)((vbar + A.beta * z * A.dz) + tau(z) * (((double)A.vbed[bed] - vbar) + A.a_eta * eta));
    }
}

// Deposit's sinusoidal mode: one thread per (y, x) column.  Each workgroup
// first builds the warped axis in LDS: the raw frequency smoothed by the
// normalised Gaussian over |m| <= int(4 sigma + 0.5) with reflecting ends,
// then its prefix sum W[z] = f[0] + .. + f[z-1] (per-thread runs, the run
// sums scanned by one thread).  Then every voxel takes
//   (v0 + beta z dz) + taper(z) [amp1 sin(phi) + amp2 sin(2 phi + phase2) + a_eta S_t]
// with phi = 2 pi (W[z] + a_r rug(y, x)), all in FP64.
constexpr int kSinThreads = 256;

__global__ void __launch_bounds__(kSinThreads) k_deposit_sin(DepositSinArgs A, float *__restrict__ out)
{
    __shared__ double W[kDepositSinMaxT];
    __shared__ double G[1024 + 1];     // Gaussian weights 0..radius (normalised)
    __shared__ double runs[kSinThreads];
    __shared__ int P[256];
    load_perm(A.perm_t, P);
    const int T = A.t;
    const int radius = A.sigma > 0.0 ? (int)(4.0 * A.sigma + 0.5) : 0;
    // weights exp(-m^2 / (2 sigma^2)), normalised by their sum over -radius..radius
    for (int m = threadIdx.x; m <= radius; m += kSinThreads)
        G[m] = radius == 0 ? 1.0 : exp(-0.5 * (double)m * (double)m / (A.sigma * A.sigma));
    __syncthreads();
    if (threadIdx.x == 0 && radius > 0) {
        double sum = G[0];
        for (int m = 1; m <= radius; ++m) sum += 2.0 * G[m];
        runs[0] = 1.0 / sum;
    }
    __syncthreads();
    const double norm = radius > 0 ? runs[0] : 1.0;
    __syncthreads();
    // smoothed frequency into W (reflect: index i maps into [0, T) by the
    // mirror about each end, period 2T)
    auto refl = [&](int i) {
        const int p2 = 2 * T;
        int r = i % p2;
        if (r < 0) r += p2;
        return r >= T ? p2 - 1 - r : r;
    };
    for (int z = threadIdx.x; z < T; z += kSinThreads) {
        double acc = G[0] * (double)A.freq[z];
        for (int m = 1; m <= radius; ++m) acc += G[m] * ((double)A.freq[refl(z - m)] + (double)A.freq[refl(z + m)]);
        W[z] = acc * norm;
    }
    __syncthreads();
    // exclusive prefix sum: thread r sums its run [r c, (r+1) c)
    const int chunk = (T + kSinThreads - 1) / kSinThreads;
    const int z0 = threadIdx.x * chunk, z1 = min(z0 + chunk, T);
    double run = 0.0;
    for (int z = z0; z < z1; ++z) run += W[z];
    runs[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int r = 0; r < kSinThreads; ++r) {
            const double v = runs[r];
            runs[r] = acc;
            acc += v;
        }
    }
    __syncthreads();
    {
        double acc = runs[threadIdx.x];
        for (int z = z0; z < z1; ++z) {
            const double f = W[z];
            W[z] = acc;
            acc += f;
        }
    }
    __syncthreads();
    const int64_t plane = (int64_t)A.ny * A.nx;
    const int64_t col = (int64_t)blockIdx.x * kSinThreads + threadIdx.x;
    if (col >= plane) return;
    const int iy = (int)(col / A.nx), ix = (int)(col - (int64_t)iy * A.nx);
    const double t = A.t;
    const double rt = 1.0 / (A.f_top * t), rb = 1.0 / (A.f_base * t);
    const double rough = A.a_r * (A.rug ? (double)A.rug[col] : 0.0);
    const double ty = iy * A.dy / A.lam_t[1], tx = ix * A.dx / A.lam_t[2];
    const double two_pi = 6.283185307179586;
    for (int iz = 0; iz < T; ++iz) {
        const double z = iz;
        const double tau = fmin(z * rt, 1.0) * fmin((t - z) * rb, 1.0);
        const double phi = two_pi * (W[iz] + rough);
        const double tex = A.a_eta != 0.0 ? A.a_eta * simplex3(P, z * A.dz / A.lam_t[0], ty, tx) : 0.0;
        out[(int64_t)iz * plane + col] =
            (float)((A.v0 + A.beta * z * A.dz) + tau * (A.amp1 * sin(phi) + A.amp2 * sin(2.0 * phi + A.phase2) + tex));
    }
}

}  // namespace

hipError_t launch_deposit(const DepositArgs &A, float *out, hipStream_t st)
{
    if (A.nbeds < 1 || A.nbeds > kDepositMaxBeds) return hipErrorInvalidValue;
    const int64_t n = (int64_t)A.ny * A.nx;
    const size_t lds = (size_t)std::max(A.nbeds - 1, 1) * kDepositThreads * sizeof(double);
    const dim3 grid((unsigned)((n + kDepositThreads - 1) / kDepositThreads));
    if (A.simplex)
        hipLaunchKernelGGL(k_deposit<true>, grid, dim3(kDepositThreads), lds, st, A, out);
    else
        hipLaunchKernelGGL(k_deposit<false>, grid, dim3(kDepositThreads), lds, st, A, out);
    return hipGetLastError();
}

hipError_t launch_deposit_sinusoidal(const DepositSinArgs &A, float *out, hipStream_t st)
{
    if (A.t < 1 || A.t > kDepositSinMaxT || !(A.sigma >= 0.0 && A.sigma <= kDepositSinMaxSigma))
        return hipErrorInvalidValue;
    const int64_t n = (int64_t)A.ny * A.nx;
    hipLaunchKernelGGL(k_deposit_sin, dim3((unsigned)((n + kSinThreads - 1) / kSinThreads)), dim3(kSinThreads), 0,
                       st, A, out);
    return hipGetLastError();
}

hipError_t launch_simplex3d(const int32_t *perm, int nz, int ny, int nx, const double o[3], const double s[3],
                            double amplitude, float *out, hipStream_t st)
{
    const int64_t n = (int64_t)nz * ny * nx;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_simplex3d, dim3((unsigned)blocks), dim3(256), 0, st, perm, nz, ny, nx, o[0], o[1], o[2],
                       s[0], s[1], s[2], amplitude, out);
    return hipGetLastError();
}

hipError_t launch_fractal_noise2d(const float *lattice, int noct, int gy, int gx, int ny, int nx, double dy,
                                  double dx, double lam_y, double lam_x, double azimuth_rad, double amplitude,
                                  float *out, hipStream_t st)
{
    double norm = 0.0, f = 1.0;
    for (int o = 0; o < noct; ++o, f *= 2.0) norm += 1.0 / f;
    const int64_t n = (int64_t)ny * nx;
    hipLaunchKernelGGL(k_fractal_noise2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lattice, noct, gy,
                       gx, ny, nx, dy, dx, 1.0 / lam_y, 1.0 / lam_x, cos(azimuth_rad), sin(azimuth_rad),
                       amplitude / norm, out);
    return hipGetLastError();
}

hipError_t launch_squish(const float *v, int nz, int ny, int nx, double dz, const float *shift, float *out,
                         hipStream_t st)
{
    const int64_t n = (int64_t)ny * nx;
    hipLaunchKernelGGL(k_squish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, nz, ny, nx, 1.0 / dz,
                       shift, out);
    return hipGetLastError();
}

namespace {

// Index range along one axis (spacing d, n voxels) covering [lo, hi] metres
// plus two voxels; false if it misses the axis.
bool axis_cover(double lo, double hi, double d, int n, int &a, int &b)
{
    const double fa = std::floor(lo / d) - 2.0, fb = std::ceil(hi / d) + 2.0;
    if (!(fb >= 0.0 && fa <= n - 1.0)) return false;
    a = fa < 0.0 ? 0 : (int)fa;
    b = fb > n - 1.0 ? n - 1 : (int)fb;
    return true;
}

// A box holding every voxel the fault can move: the cylinder shell
// |r - R| < die_r (+ |rough amplitude| max |lattice|), the angle band |theta - theta0| <
// die_theta and |along-strike offset| < die_strike, bounded in the (h, v)
// plane across strike by its corners and axis crossings, then carried to
// (z, y, x) by interval arithmetic; two voxels of margin.  Outside it every
// voxel keeps its value.  False if it misses the volume.
bool fault_box(const FaultFrame &F, int nz, int ny, int nx, VoxBox &B)
{
    const double pi = 3.14159265358979323846;
    const double die_r = 1.0 / F.inv_die_r, die_t = 1.0 / F.inv_die_t, die_s = 1.0 / F.inv_die_s;
    const double extra = F.rough ? F.rough_reach - die_r : 0.0;
    const double r_hi = F.radius + die_r + extra, r_lo = std::max(0.0, F.radius - die_r - extra);
    double h_lo, h_hi, v_lo, v_hi;
    if (die_t >= pi) {
        h_lo = v_lo = -r_hi;
        h_hi = v_hi = r_hi;
    } else {
        const double t0 = F.theta0 - die_t, t1 = F.theta0 + die_t;
        double ts[16];
        int nt = 0;
        ts[nt++] = t0;
        ts[nt++] = t1;
        for (int k = (int)std::ceil(t0 / (0.5 * pi)); k * 0.5 * pi < t1 && nt < 16; ++k) ts[nt++] = k * 0.5 * pi;
        h_lo = v_lo = 1e300;
        h_hi = v_hi = -1e300;
        for (int i = 0; i < nt; ++i)
            for (double r : {r_lo, r_hi}) {
                h_lo = std::min(h_lo, r * std::cos(ts[i]));
                h_hi = std::max(h_hi, r * std::cos(ts[i]));
                v_lo = std::min(v_lo, r * std::sin(ts[i]));
                v_hi = std::max(v_hi, r * std::sin(ts[i]));
            }
    }
    // y = cy + h n_y + az s_y, x = cx + h n_x + az s_x, az in [-die_s, die_s]
    auto span = [&](double c, double ny_, double sy_, double &lo, double &hi) {
        lo = c + std::min(h_lo * ny_, h_hi * ny_) - die_s * std::fabs(sy_);
        hi = c + std::max(h_lo * ny_, h_hi * ny_) + die_s * std::fabs(sy_);
    };
    double y_lo, y_hi, x_lo, x_hi;
    span(F.cy, F.n_y, F.s_y, y_lo, y_hi);
    span(F.cx, F.n_x, F.s_x, x_lo, x_hi);
    int za, zb, ya, yb, xa, xb;
    if (!axis_cover(F.cz + v_lo, F.cz + v_hi, F.dz, nz, za, zb) || !axis_cover(y_lo, y_hi, F.dy, ny, ya, yb) ||
        !axis_cover(x_lo, x_hi, F.dx, nx, xa, xb))
        return false;
    B = VoxBox{za, ya, xa, zb - za + 1, yb - ya + 1, xb - xa + 1};
    return true;
}

int64_t fault_blocks(const VoxBox &B)
{
    const int64_t nbrick =
        (int64_t)((B.bx + 255) / 256) * ((B.by + kBrickY - 1) / kBrickY) * ((B.bz + kBrickZ - 1) / kBrickZ);
    return (nbrick + 7) / 8 * 8 * kBrickRows;
}

// Copies the volume when the fault's box is smaller than it (the kernel then
// writes the box only); returns whether the kernel has anything to do.
template <typename T>
hipError_t fault_prologue(const T *in, int nz, int ny, int nx, const FaultFrame &F, T *out, hipStream_t st,
                          VoxBox &B, bool &run)
{
    const VoxBox whole{0, 0, 0, nz, ny, nx};
    run = fault_box(F, nz, ny, nx, B);
    const bool partial = !run || B.bz < nz || B.by < ny || B.bx < nx;
    if (!run) B = whole;
    if (partial)
        return hipMemcpyAsync(out, in, (size_t)nz * ny * nx * sizeof(T), hipMemcpyDeviceToDevice, st);
    return hipSuccess;
}

}  // namespace

hipError_t launch_fault(const float *v, int nz, int ny, int nx, const FaultFrame &F, float fill, float *out,
                        hipStream_t st)
{
    VoxBox B;
    bool run;
    hipError_t e = fault_prologue(v, nz, ny, nx, F, out, st, B, run);
    if (e != hipSuccess || !run) return e;
    const int64_t blocks = brick_blocks(B);
    if (blocks >= ((int64_t)1 << 32)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fault, dim3((unsigned)blocks), dim3(256), 0, st, v, nz, ny, nx, B, brick_grid(B), F, fill,
                       out);
    return hipGetLastError();
}

hipError_t launch_fault_labels(const int32_t *lab, int nz, int ny, int nx, const FaultFrame &F, int32_t fill,
                               int32_t *out, hipStream_t st)
{
    VoxBox B;
    bool run;
    hipError_t e = fault_prologue(lab, nz, ny, nx, F, out, st, B, run);
    if (e != hipSuccess || !run) return e;
    const int64_t blocks = fault_blocks(B);
    if (blocks >= ((int64_t)1 << 32)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fault_labels, dim3((unsigned)blocks), dim3(256), 0, st, lab, nz, ny, nx, B, F, fill, out);
    return hipGetLastError();
}

namespace {

// dst = src on the voxels of box B (rows of the box contiguous in x).
template <typename T>
__global__ void __launch_bounds__(256) k_copy_box(const T *__restrict__ src, int ny, int nx, VoxBox B,
                                                  T *__restrict__ dst)
{
    const int64_t nb = (int64_t)B.bz * B.by * B.bx;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = q / B.bx;
        const int x = (int)(q - row * B.bx), z = (int)(row / B.by), y = (int)(row - (int64_t)z * B.by);
        const int64_t o = ((int64_t)(B.z0 + z) * ny + (B.y0 + y)) * nx + (B.x0 + x);
        dst[o] = src[o];
    }
}

template <typename T>
hipError_t copy_box(const T *src, int ny, int nx, const VoxBox &B, T *dst, hipStream_t st)
{
    const int64_t nb = (int64_t)B.bz * B.by * B.bx;
    const int64_t blocks = std::min<int64_t>((nb + 255) / 256, (int64_t)1 << 20);
    hipLaunchKernelGGL(k_copy_box<T>, dim3((unsigned)blocks), dim3(256), 0, st, src, ny, nx, B, dst);
    return hipGetLastError();
}

// The faults in order, alternating between out and ws so the last lands in
// out.  Step k writes dst_k, which holds the state of step k-2 (garbage for
// k < 2); that state differs from step k-1's only on the box fault k-1
// wrote, so that box is copied over first (the whole volume for k < 2) when
// fault k does not cover the volume itself; then fault k runs on its box.
template <typename T, typename Launch>
hipError_t fault_sequence(const T *v, int nz, int ny, int nx, const FaultFrame *F, int n, T *out, T *ws,
                          hipStream_t st, Launch run_kernel)
{
    const VoxBox whole{0, 0, 0, nz, ny, nx};
    const size_t bytes = (size_t)nz * ny * nx * sizeof(T);
    if (n == 0) return hipMemcpyAsync(out, v, bytes, hipMemcpyDeviceToDevice, st);
    const T *src = v;
    VoxBox prev{};
    bool prev_run = false;
    for (int k = 0; k < n; ++k) {
        T *dst = ((n - 1 - k) % 2 == 0) ? out : ws;
        VoxBox B;
        const bool run = fault_box(F[k], nz, ny, nx, B);
        const bool partial = !run || B.bz < nz || B.by < ny || B.bx < nx;
        hipError_t e = hipSuccess;
        if (partial) {
            if (k < 2)
                e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
            else if (prev_run)
                e = copy_box(src, ny, nx, prev, dst, st);
        }
        if (e != hipSuccess) return e;
        if (run && (e = run_kernel(src, B, F[k], dst)) != hipSuccess) return e;
        prev = run ? B : whole;
        prev_run = run;
        src = dst;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_fault_sequence(const float *v, int nz, int ny, int nx, const FaultFrame *F, int n, float fill,
                                 float *out, float *ws, hipStream_t st)
{
    return fault_sequence(v, nz, ny, nx, F, n, out, ws, st,
                          [&](const float *src, const VoxBox &B, const FaultFrame &f, float *dst) {
                              const int64_t blocks = brick_blocks(B);
                              if (blocks >= ((int64_t)1 << 32)) return hipErrorInvalidValue;
                              hipLaunchKernelGGL(k_fault, dim3((unsigned)blocks), dim3(256), 0, st, src, nz, ny, nx,
                                                 B, brick_grid(B), f, fill, dst);
                              return hipGetLastError();
                          });
}

hipError_t launch_fault_labels_sequence(const int32_t *lab, int nz, int ny, int nx, const FaultFrame *F, int n,
                                        int32_t fill, int32_t *out, int32_t *ws, hipStream_t st)
{
    return fault_sequence(lab, nz, ny, nx, F, n, out, ws, st,
                          [&](const int32_t *src, const VoxBox &B, const FaultFrame &f, int32_t *dst) {
                              const int64_t blocks = fault_blocks(B);
                              if (blocks >= ((int64_t)1 << 32)) return hipErrorInvalidValue;
                              hipLaunchKernelGGL(k_fault_labels, dim3((unsigned)blocks), dim3(256), 0, st, src, nz,
                                                 ny, nx, B, f, fill, dst);
                              return hipGetLastError();
                          });
}

}  // namespace sg
