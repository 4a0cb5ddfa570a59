// SaltSDT (SubsurfaceGen, arXiv 2605.30541, App. B, Alg. 4): salt bodies from
// rotated ellipsoids whose signed distance is perturbed by a random field,
// merged, opened and closed, cleared of small components and written over
// the model below the water.  Volumes are [nz][ny][nx], x fastest.
//
// Kernels, in launch order:
//  * k_field_extremes: max(xi, 0) and max(-xi, 0) of every body's field,
//    read back once so the host can bound each body's reach (below);
//  * k_ellipsoid: the body raster on the voxel centres;
//  * k_edt_x, k_edt_envelope (z, then y): the exact squared Euclidean distance
//    to the nearest feature voxel as three separable passes.  Along x the
//    distance to the nearest feature of the row (the 1D transform of a
//    0/infinity function), one wave per row; along z and y the lower envelope
//    of parabolas in FP64, one thread per line (Felzenszwalb and
//    Huttenlocher's 1D transform; the paper names Meijster's algorithm, which
//    yields the same exact distances);
//  * k_salt_union: phi' = d_in - d_out + a rbar xi, K |= phi' > 0.  A body
//    covering no voxel gives d_out = infinity everywhere (phi' = -inf), one
//    covering all gives d_in = infinity (phi' = +inf): no special cases;
//  * k_morph x4: opening then closing with the 6-neighbour cross, a voxel
//    outside the volume counting as empty;
//  * k_cc_init, k_cc_merge, k_cc_flatten: 6-connected components by a
//    lock-free union-find (runs along x inside a wave are labelled by ballot;
//    the rest is joined by atomicMin on the roots; then every label is
//    pointed at its root), so each component ends labelled by its smallest
//    voxel index;
//  * k_cc_count, k_salt_write: component sizes and the final write.
//
// Each body is processed on boxes only.  d_out and phi' on the raster's
// bounding box widened by B = max over the volume of (a rbar xi) plus two
// voxels: outside it every voxel is outside the body and more than B from it,
// so phi' < 0 and the body adds nothing there, and inside it d_out is exact
// (every inside voxel is in the box).  d_in on the raster's bounding box plus
// two voxels: it is needed only at inside voxels (it is 0 at outside ones),
// and the nearest outside voxel of an inside voxel, clamped into that box, is
// still outside and no farther.  Decisions (inside the
// ellipsoid, phi' > 0) are taken in FP64 without fused multiply-adds, so they
// round as the plain definitions do.
#include "sg_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#pragma clang fp contract(off)

namespace sg {

namespace {

constexpr int kSaltThreads = 256;
constexpr int kRowsPerBlock = kSaltThreads / 64;
constexpr int kCountPerThread = 32;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kSaltThreads - 1) / kSaltThreads); }

__device__ inline double inf_d() { return __builtin_huge_val(); }

// Voxels [z0, z0 + bz) x [y0, y0 + by) x [x0, x0 + bx) of the volume.
struct Box {
    int z0, y0, x0, bz, by, bx;
};

inline unsigned row_blocks(const Box &b) { return (unsigned)((b.bx + kSaltThreads - 1) / kSaltThreads); }
inline dim3 box_grid(const Box &b) { return dim3((unsigned)((int64_t)b.bz * b.by * row_blocks(b))); }

// Voxel kernels launch bz * by rows of xb = ceil(bx / 256) blocks each; a
// block covers 256 consecutive voxels of one row, so the row (and z, y) comes
// from one division per block, and each wave covers 64 voxels starting at a
// multiple of 64 from x0.  Returns false for lanes past the end of the row.
__device__ inline bool box_voxel(const Box &b, int ny, int nx, unsigned xb, int &iz, int &iy, int &ix, int64_t &q)
{
    const unsigned row = blockIdx.x / xb;
    const int lx = (int)((blockIdx.x - row * xb) * kSaltThreads + threadIdx.x);
    const unsigned lz = row / (unsigned)b.by;
    iz = b.z0 + (int)lz;
    iy = b.y0 + (int)(row - lz * (unsigned)b.by);
    ix = b.x0 + lx;
    q = ((int64_t)iz * ny + iy) * nx + ix;
    return lx < b.bx;
}

__device__ inline float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// ext[2 b] = max(xi_b, 0), ext[2 b + 1] = max(-xi_b, 0) as float bits (a
// non-negative float orders as its bits); NaN values are ignored.  ext must
// start at zero.  Body b = blockIdx.y.
__global__ void __launch_bounds__(kSaltThreads) k_field_extremes(int64_t n, const float *grf, unsigned *ext)
{
    const float *xi = grf + (int64_t)blockIdx.y * n;
    float hi = 0.0f, lo = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * kSaltThreads;
    int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    if (n % 4 == 0 && ((uintptr_t)grf & 15) == 0) {   // every field 16-byte aligned: four values per load
        const float4 *x4 = (const float4 *)xi;
        for (; q < n / 4; q += stride) {
            const float4 v = x4[q];
            hi = fmaxf(hi, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
            lo = fmaxf(lo, fmaxf(fmaxf(-v.x, -v.y), fmaxf(-v.z, -v.w)));
        }
    } else {
        for (; q < n; q += stride) {
            const float v = xi[q];
            hi = fmaxf(hi, v);
            lo = fmaxf(lo, -v);
        }
    }
    hi = wave_max(hi);
    lo = wave_max(lo);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&ext[2 * blockIdx.y], __float_as_uint(hi));
        atomicMax(&ext[2 * blockIdx.y + 1], __float_as_uint(lo));
    }
}

__global__ void __launch_bounds__(kSaltThreads) k_ellipsoid(Box b, int ny, int nx, unsigned xb, double dz, double dy,
                                                            double dx, SaltBody B, uint8_t *mask)
{
    int iz, iy, ix;
    int64_t q;
    if (!box_voxel(b, ny, nx, xb, iz, iy, ix, q)) return;
    const double p0 = iz * dz - B.c[0], p1 = iy * dy - B.c[1], p2 = ix * dx - B.c[2];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double u = (B.R[3 * k] * p0 + B.R[3 * k + 1] * p1 + B.R[3 * k + 2] * p2) / B.r[k];
        s += u * u;
    }
    mask[q] = s <= 1.0;
}

// Along x, one wave per row of the box: g = (dx * distance in cells to the
// nearest voxel of the row segment whose mask equals the feature)^2, infinity
// if it has none, written in the box-local layout [y][z][x] (rows stay
// contiguous, so the transposition is free and the z pass reads short strides).  The segment is walked in blocks of 64 voxels, one per lane
// (coalesced); a ballot gives the block's feature voxels, and the nearest one
// at or below (forward walk) or at or above (backward walk) each lane comes
// from the ballot bits, or from the carry of the blocks already walked.
__global__ void __launch_bounds__(kSaltThreads) k_edt_x(Box b0, Box b1, int ny, int nx, double dx,
                                                        const uint8_t *mask, double *g0, double *g1)
{
    // blockIdx.y = the feature value: 0 (distance to outside voxels) on box b0 into g0, 1 on b1 into g1
    const uint8_t feature = (uint8_t)blockIdx.y;
    double *g = blockIdx.y ? g1 : g0;
    const Box b = blockIdx.y ? b1 : b0;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
    if (row >= (int64_t)b.bz * b.by) return;   // uniform over the wave
    const int lz = (int)(row / b.by), ly = (int)(row - (int64_t)lz * b.by);
    const uint8_t *m = mask + ((int64_t)(b.z0 + lz) * ny + (b.y0 + ly)) * nx + b.x0;
    double *gr = g + ((int64_t)ly * b.bz + lz) * b.bx;   // box-local [y][z][x]
    const int n = b.bx;
    const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1);   // bits 0..lane
    const unsigned long long from = ~0ull << lane;                                       // bits lane..63
    int carry = -1;   // last feature before the block
    for (int x0 = 0; x0 < n; x0 += 64) {
        const int x = x0 + lane;
        const unsigned long long bits = __ballot(x < n && m[x] == feature);
        const unsigned long long mb = bits & upto;
        const int last = mb ? x0 + 63 - __clzll((long long)mb) : carry;
        if (x < n) {
            const double d = dx * (double)(x - last);
            gr[x] = last < 0 ? inf_d() : d * d;
        }
        if (bits) carry = x0 + 63 - __clzll((long long)bits);
    }
    int next = -1;    // first feature after the block
    for (int x0 = (n - 1) / 64 * 64; x0 >= 0; x0 -= 64) {
        const int x = x0 + lane;
        const unsigned long long bits = __ballot(x < n && m[x] == feature);
        const unsigned long long ma = bits & from;
        const int nf = ma ? x0 + __ffsll((long long)ma) - 1 : next;
        if (x < n && nf >= 0) {
            const double d = dx * (double)(nf - x);
            const double e = d * d;
            if (e < gr[x]) gr[x] = e;
        }
        if (bits) next = x0 + __ffsll((long long)bits) - 1;
    }
}

// Buffers of the two distance transforms (feature 0 and 1) run side by side.
struct EnvPair {
    const uint8_t *skip_mask;   // with axis 1: transform 0 skips lines holding no voxel set here
    int ny, nx;                 // volume rows and columns (to index skip_mask)
    Box box[2];
    const double *f[2];
    double *g[2];
    int *v[2];
    double *zb[2];
};

// g(p) = min_q (w (p - q))^2 + f(q) along one line of the box: the lower
// envelope of the parabolas rooted at the finite samples.  Box-local layouts:
// axis 0, lines along z, one per (y, x), read [y][z][x] and write [z][y][x];
// axis 1, lines along y, one per (z, x), in [z][y][x].  Samples of a line are
// one row (bx values) apart; neighbouring lanes take neighbouring x, so the
// reads of f and writes of g are coalesced.
// blockIdx.y picks the transform and its box.  v (int) and zb (double) hold the
// envelope's roots and boundaries, in the layout of f; the top entry
// also lives in registers (vk, hk, zk), so a sample that pops nothing reads no
// stack memory, and f is read four samples ahead.
__global__ void __launch_bounds__(kSaltThreads) k_edt_envelope(int axis, double w, EnvPair P)
{
    const Box b = P.box[blockIdx.y];
    const int64_t l = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    int n;
    int64_t base, stride, obase, ostride;
    if (axis == 1) {
        // along y in [z][y][x], in place of layout
        if (l >= (int64_t)b.bz * b.bx) return;
        const int lz = (int)(l / b.bx), lx = (int)(l - (int64_t)lz * b.bx);
        n = b.by;
        base = (int64_t)lz * b.by * b.bx + lx;
        stride = b.bx;
        obase = base;
        ostride = stride;
    } else {
        // along z: read [y][z][x], write [z][y][x]
        if (l >= (int64_t)b.by * b.bx) return;
        const int ly = (int)(l / b.bx), lx = (int)(l - (int64_t)ly * b.bx);
        n = b.bz;
        base = (int64_t)ly * b.bz * b.bx + lx;
        stride = b.bx;
        obase = (int64_t)ly * b.bx + lx;
        ostride = (int64_t)b.by * b.bx;
    }
    const int t = blockIdx.y;
    if (axis == 1 && t == 0 && P.skip_mask) {
        // d_in's last pass: its values are read at inside voxels only
        const int lz = (int)(l / b.bx), lx = (int)(l - (int64_t)lz * b.bx);
        const uint8_t *m = P.skip_mask + ((int64_t)(b.z0 + lz) * P.ny + b.y0) * P.nx + b.x0 + lx;
        bool any = false;
        for (int q = 0; q < n && !any; ++q) any = m[(int64_t)q * P.nx] != 0;
        if (!any) return;
    }
    const double *f = P.f[t] + base;
    double *g = P.g[t] + obase;
    int *v = P.v[t] + base;
    double *zb = P.zb[t] + base;
    const double w2 = w * w;
    int k = -1;       // index of the last parabola of the envelope
    int vk = 0;       // its root
    double hk = 0.0;  // f(v_k) + w^2 v_k^2
    double zk = 0.0;  // where it starts
    double f0 = n > 0 ? f[0] : 0.0, f1 = n > 1 ? f[stride] : 0.0, f2 = n > 2 ? f[2 * stride] : 0.0,
           f3 = n > 3 ? f[3 * stride] : 0.0;
    for (int q = 0; q < n; ++q) {
        const double fq = f0;
        f0 = f1;
        f1 = f2;
        f2 = f3;
        f3 = q + 4 < n ? f[(int64_t)(q + 4) * stride] : 0.0;
        if (!(fq < inf_d())) continue;
        const double hq = fq + w2 * ((double)q * q);
        double s = 0.0;
        while (k >= 0) {
            // abscissa where parabola q starts to lie below parabola v_k
            s = (hq - hk) / (2.0 * w2 * (double)(q - vk));
            if (k == 0 || s > zk) break;
            --k;
            vk = v[k * stride];
            zk = zb[k * stride];
            hk = f[(int64_t)vk * stride] + w2 * ((double)vk * vk);
        }
        ++k;
        zk = k == 0 ? -inf_d() : s;
        v[k * stride] = q;
        zb[k * stride] = zk;
        vk = q;
        hk = hq;
    }
    if (k < 0) {
        for (int p = 0; p < n; ++p) g[p * ostride] = inf_d();
        return;
    }
    int j = 0;
    int vj = v[0];
    double zn = k > 0 ? zb[stride] : inf_d();   // start of parabola j + 1
    for (int p = 0; p < n; ++p) {
        while (zn < (double)p) {
            ++j;
            vj = v[j * stride];
            zn = j < k ? zb[(j + 1) * stride] : inf_d();
        }
        const double d = w * (double)(p - vj);
        g[p * ostride] = d * d + f[(int64_t)vj * stride];
    }
}

// Over box b (that of d_out); d_in is held on the inner box bi (every inside
// voxel is in it) and read at inside voxels only, d_out at outside voxels only.
// Both distance arrays are box-local [z][y][x].
__global__ void __launch_bounds__(kSaltThreads) k_salt_union(Box b, Box bi, int ny, int nx, unsigned xb,
                                                             const uint8_t *mask, const double *din2,
                                                             const double *dout2, const float *xi, double a_rbar,
                                                             uint8_t *K)
{
    int iz, iy, ix;
    int64_t q;
    if (!box_voxel(b, ny, nx, xb, iz, iy, ix, q)) return;
    // d_in - d_out with one of them exactly 0: d_in at an inside voxel (always in bi), -d_out outside
    const double phi = mask[q]
        ? sqrt(din2[((int64_t)(iz - bi.z0) * bi.by + (iy - bi.y0)) * bi.bx + (ix - bi.x0)])
        : -sqrt(dout2[((int64_t)(iz - b.z0) * b.by + (iy - b.y0)) * b.bx + (ix - b.x0)]);
    if (phi + a_rbar * (double)xi[q] > 0.0) K[q] = 1;
}

__global__ void __launch_bounds__(kSaltThreads) k_fill_u8(int64_t n, uint8_t val, uint8_t *p)
{
    const int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    if (q < n) p[q] = val;
}

__global__ void __launch_bounds__(kSaltThreads) k_fill_u32(int64_t n, unsigned val, unsigned *p)
{
    const int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    if (q < n) p[q] = val;
}

// erode (op 0): set where the voxel and its six neighbours are all set;
// dilate (op 1): set where the voxel or any neighbour is set.  A neighbour
// outside the volume counts as empty.
__global__ void __launch_bounds__(kSaltThreads) k_morph(int op, Box b, int nz, int ny, int nx, unsigned xb,
                                                        const uint8_t *in, uint8_t *out)
{
    int iz, iy, ix;
    int64_t q;
    if (!box_voxel(b, ny, nx, xb, iz, iy, ix, q)) return;
    const int64_t plane = (int64_t)ny * nx;
    const bool c = in[q];
    const bool zm = iz > 0 && in[q - plane], zp = iz < nz - 1 && in[q + plane];
    const bool ym = iy > 0 && in[q - nx], yp = iy < ny - 1 && in[q + nx];
    const bool xm = ix > 0 && in[q - 1], xp = ix < nx - 1 && in[q + 1];
    out[q] = op == 0 ? (c && zm && zp && ym && yp && xm && xp) : (c || zm || zp || ym || yp || xm || xp);
}

// k_morph on four voxels per lane (rows of a multiple of 4 voxels, so a
// 32-bit word never straddles two rows): the voxel bytes are 0 or 1, the x
// neighbours are the word shifted by one byte with the bytes of the adjacent
// words filled in, and the result is a bytewise AND (erode) or OR (dilate).
__global__ void __launch_bounds__(kSaltThreads) k_morph4(int op, int nz, int ny, int nx, unsigned xb,
                                                         const uint8_t *in, uint8_t *out)
{
    const int nw = nx / 4;   // words per row
    const unsigned row = blockIdx.x / xb;
    const int lw = (int)((blockIdx.x - row * xb) * kSaltThreads + threadIdx.x);
    if (lw >= nw) return;
    const unsigned iz = row / (unsigned)ny, iy = row - iz * (unsigned)ny;
    const int64_t q = (int64_t)row * nx + 4 * lw;      // first voxel of the word
    const int64_t wq = q / 4, wplane = (int64_t)ny * nw;
    const uint32_t *in4 = (const uint32_t *)in;
    const uint32_t c = in4[wq];
    const uint32_t zm = iz > 0 ? in4[wq - wplane] : 0u, zp = (int)iz < nz - 1 ? in4[wq + wplane] : 0u;
    const uint32_t ym = iy > 0 ? in4[wq - nw] : 0u, yp = (int)iy < ny - 1 ? in4[wq + nw] : 0u;
    const uint32_t left = lw > 0 ? in[q - 1] : 0u, right = lw < nw - 1 ? in[q + 4] : 0u;
    const uint32_t xm = (c << 8) | left, xp = (c >> 8) | (right << 24);
    ((uint32_t *)out)[wq] = op == 0 ? (c & zm & zp & ym & yp & xm & xp) : (c | zm | zp | ym | yp | xm | xp);
}

// Labels form a forest over the salt voxels: label[x] <= x, a root has
// label[r] == r, and every label names a voxel of the same component.  Labels
// only ever decrease (atomicMin), so a chain strictly decreases and find ends;
// a stale read returns an older ancestor, which is still an ancestor.
__device__ inline int find_root(const int *label, int x)
{
    for (;;) {
        const int p = label[x];
        if (p == x) return x;
        x = p;
    }
}

// Link the roots of a and b, the larger under the smaller.  atomicMin returns
// the previous value: equal to the root means linked; otherwise that root had
// been linked meanwhile and the loop continues from its (smaller) parent.
// Every retry lowers a + b, so the loop ends; no thread waits on another.
__device__ inline void unite(int *label, int a, int b)
{
    for (;;) {
        a = find_root(label, a);
        b = find_root(label, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(&label[b], a);
        if (old == b) return;
        b = old;
    }
}

// Initial forest: a salt voxel points at the first voxel of its run along x
// within its wave's 64 voxels (from the ballot); others get -1.
__global__ void __launch_bounds__(kSaltThreads) k_cc_init(Box b, int ny, int nx, unsigned xb, const uint8_t *K,
                                                          int *label)
{
    int iz, iy, ix;
    int64_t q;
    const bool valid = box_voxel(b, ny, nx, xb, iz, iy, ix, q);
    const bool set = valid && K[q];
    const unsigned long long bits = __ballot(set);
    const int lane = threadIdx.x & 63;
    const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1);
    const unsigned long long gaps = ~bits & upto;
    const int start = gaps ? 64 - __clzll((long long)gaps) : 0;   // one past the last gap at or below the lane
    if (valid) label[q] = set ? (int)(q - (lane - start)) : -1;
}

// Joins the runs: across a wave boundary along x, and along -y and -z unless
// the voxel's left neighbour and that neighbour's own -y (-z) neighbour are
// both salt, in which case the left neighbour's join (or one further left)
// already connects the two runs.
__global__ void __launch_bounds__(kSaltThreads) k_cc_merge(Box b, int ny, int nx, unsigned xb, const uint8_t *K,
                                                           int *label)
{
    int iz, iy, ix;
    int64_t q;
    if (!box_voxel(b, ny, nx, xb, iz, iy, ix, q)) return;
    if (!K[q]) return;
    const int64_t plane = (int64_t)ny * nx;
    const bool left = ix > 0 && K[q - 1];
    if (left && (threadIdx.x & 63) == 0) unite(label, (int)q, (int)(q - 1));
    if (iy > 0 && K[q - nx] && !(left && K[q - 1 - nx])) unite(label, (int)q, (int)(q - nx));
    if (iz > 0 && K[q - plane] && !(left && K[q - 1 - plane])) unite(label, (int)q, (int)(q - plane));
}

// After the merge has finished: every label becomes its root.  Only the
// thread's own entry is written, and only with an ancestor of it.
__global__ void __launch_bounds__(kSaltThreads) k_cc_flatten(int64_t n, int *label)
{
    const int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    if (q >= n) return;
    const int l = label[q];
    if (l >= 0 && l != (int)q) label[q] = find_root(label, l);
}

// Component sizes: each thread counts runs of equal labels over its
// kCountPerThread voxels and adds each run to a small table of
// (label, count) in LDS (linear probing by atomicCAS on the label slot); the
// table goes to memory with one atomic per distinct label per workgroup, and
// runs that find the table full go straight to memory.
constexpr int kCountSlots = 32;

__global__ void __launch_bounds__(kSaltThreads) k_cc_count(int64_t n, const int *label, unsigned *count)
{
    __shared__ int tl[kCountSlots];
    __shared__ unsigned tc[kCountSlots];
    if (threadIdx.x < kCountSlots) {
        tl[threadIdx.x] = -1;
        tc[threadIdx.x] = 0u;
    }
    __syncthreads();
    auto add = [&](int l, unsigned c) {
        for (int i = 0; i < kCountSlots; ++i) {
            const int slot = (l + i) & (kCountSlots - 1);
            const int old = atomicCAS(&tl[slot], -1, l);
            if (old == -1 || old == l) {
                atomicAdd(&tc[slot], c);
                return;
            }
        }
        atomicAdd(&count[l], c);
    };
    // the workgroup covers kSaltThreads * kCountPerThread consecutive voxels in
    // chunks of 4 per lane, the lanes on consecutive chunks (coalesced loads)
    const int64_t blk0 = (int64_t)blockIdx.x * kSaltThreads * kCountPerThread;
    int cur = -1;
    unsigned cnt = 0;
    auto step = [&](int l) {   // runs of equal labels (adjacency does not matter to a count)
        if (l != cur) {
            if (cur >= 0) add(cur, cnt);
            cur = l;
            cnt = 0;
        }
        ++cnt;
    };
#pragma unroll
    for (int i = 0; i < kCountPerThread / 4; ++i) {
        const int64_t q0 = blk0 + ((int64_t)i * kSaltThreads + threadIdx.x) * 4;
        if (q0 + 4 <= n) {
            const int4 w = *(const int4 *)(label + q0);
            step(w.x);
            step(w.y);
            step(w.z);
            step(w.w);
        } else {
            for (int j = 0; j < 4; ++j) step(q0 + j < n ? label[q0 + j] : -1);
        }
    }
    if (cur >= 0) add(cur, cnt);
    __syncthreads();
    if (threadIdx.x < kCountSlots && tl[threadIdx.x] >= 0) atomicAdd(&count[tl[threadIdx.x]], tc[threadIdx.x]);
}

__global__ void __launch_bounds__(kSaltThreads) k_salt_write(int64_t n, const float *v, const int *label,
                                                             const unsigned *count, unsigned min_voxels,
                                                             float v_salt, float v_water, float *out,
                                                             uint8_t *mask_out)
{
    const int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    if (q >= n) return;
    const int l = label[q];
    const float vq = v[q];
    const bool k = l >= 0 && count[l] >= min_voxels && vq >= v_water;
    out[q] = k ? v_salt : vq;
    if (mask_out) mask_out[q] = k;
}

struct SaltWorkspace {
    double *din, *dout, *f[2], *zb[2];
    int *v[2];
    uint8_t *K, *m;
    unsigned *ext;
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

SaltWorkspace carve(void *ws, int64_t n)
{
    char *p = (char *)ws;
    SaltWorkspace W{};
    double **d8[6] = {&W.din, &W.dout, &W.f[0], &W.f[1], &W.zb[0], &W.zb[1]};
    for (double **d : d8) {
        *d = (double *)p;
        p += align256(8 * (size_t)n);
    }
    for (int t = 0; t < 2; ++t) {
        W.v[t] = (int *)p;
        p += align256(4 * (size_t)n);
    }
    W.K = (uint8_t *)p;
    p += align256((size_t)n);
    W.m = (uint8_t *)p;
    p += align256((size_t)n);
    W.ext = (unsigned *)p;
    return W;
}

// Index range [lo, hi] along one axis of spacing h and n voxels covering
// centre +- reach (metres) plus two voxels; false if it misses the axis.
bool axis_range(double centre, double reach, double h, int n, int &lo, int &hi)
{
    if (!std::isfinite(reach)) {
        lo = 0;
        hi = n - 1;
        return true;
    }
    const double a = std::floor((centre - reach) / h) - 2.0, b = std::ceil((centre + reach) / h) + 2.0;
    if (b < 0.0 || a > n - 1.0) return false;
    lo = a < 0.0 ? 0 : (int)a;
    hi = b > n - 1.0 ? n - 1 : (int)b;
    return true;
}

}  // namespace

size_t salt_workspace_bytes(int64_t n)
{
    return 6 * align256(8 * (size_t)n) + 2 * align256(4 * (size_t)n) + 2 * align256((size_t)n) +
           align256(2 * sizeof(unsigned) * kSaltMaxBodies);
}

hipError_t launch_salt_sdt(const float *v, int nz, int ny, int nx, double dz, double dy, double dx, int nbodies,
                           const SaltBody *bodies, const float *grf, double amplitude, float v_salt, float v_water,
                           unsigned min_voxels, float *out, uint8_t *mask_out, void *ws, hipStream_t st)
{
    const int64_t n = (int64_t)nz * ny * nx;
    const SaltWorkspace W = carve(ws, n);
    const dim3 blk(kSaltThreads);
    const Box whole{0, 0, 0, nz, ny, nx};
    const unsigned xw = row_blocks(whole);
    hipError_t e;
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for(n)), blk, 0, st, n, (uint8_t)0, W.K);
    std::vector<unsigned> ext(2 * (size_t)nbodies, 0u);
    if (nbodies > 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(2 * nbodies)), blk, 0, st, (int64_t)2 * nbodies, 0u, W.ext);
        const unsigned per_body = std::min(blocks_for(n), 1024u);
        hipLaunchKernelGGL(k_field_extremes, dim3(per_body, nbodies), blk, 0, st, n, grf, W.ext);
        if ((e = hipMemcpyAsync(ext.data(), W.ext, ext.size() * sizeof(unsigned), hipMemcpyDeviceToHost, st)) !=
            hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    }
    for (int i = 0; i < nbodies; ++i) {
        const SaltBody &B = bodies[i];
        const double rbar = (B.r[0] + B.r[1] + B.r[2]) / 3.0;
        float hi, lo;
        std::memcpy(&hi, &ext[2 * i], sizeof hi);
        std::memcpy(&lo, &ext[2 * i + 1], sizeof lo);
        // largest a rbar xi over the volume: how far beyond the raster the body can reach
        const double reach = std::max(0.0, amplitude >= 0 ? amplitude * rbar * hi : -amplitude * rbar * lo);
        // half extent of the rotated ellipsoid along world axis j: |column j of R^T diag(r)|
        const double h[3] = {dz, dy, dx};
        const int nn[3] = {nz, ny, nx};
        // bo: the raster's box widened by the reach (where the body can add salt, and d_out is needed);
        // bi: the raster's box alone (d_in is needed only at inside voxels)
        int lo_o[3], hi_o[3], lo_n[3], hi_n[3];
        bool hit = true;
        for (int j = 0; j < 3 && hit; ++j) {
            double e2 = 0.0;
            for (int k = 0; k < 3; ++k) e2 += (B.R[3 * k + j] * B.r[k]) * (B.R[3 * k + j] * B.r[k]);
            const double ext = std::sqrt(e2) * (1.0 + 1e-6);
            hit = axis_range(B.c[j], ext, h[j], nn[j], lo_n[j], hi_n[j]) &&
                  axis_range(B.c[j], ext + reach, h[j], nn[j], lo_o[j], hi_o[j]);
        }
        if (!hit) continue;   // the raster misses the volume: the body adds nothing
        const Box bo{lo_o[0], lo_o[1], lo_o[2], hi_o[0] - lo_o[0] + 1, hi_o[1] - lo_o[1] + 1, hi_o[2] - lo_o[2] + 1};
        const Box bi{lo_n[0], lo_n[1], lo_n[2], hi_n[0] - lo_n[0] + 1, hi_n[1] - lo_n[1] + 1, hi_n[2] - lo_n[2] + 1};
        const unsigned xb = row_blocks(bo);
        hipLaunchKernelGGL(k_ellipsoid, box_grid(bo), blk, 0, st, bo, ny, nx, xb, dz, dy, dx, B, W.m);
        // d_in: distance to the nearest voxel outside (feature 0, on bi); d_out: to the nearest inside
        // (feature 1, on bo); both transforms run in the same launches (blockIdx.y), sized for bo
        const int64_t rows = (int64_t)bo.bz * bo.by;
        hipLaunchKernelGGL(k_edt_x, dim3((unsigned)((rows + kRowsPerBlock - 1) / kRowsPerBlock), 2), blk, 0, st, bi,
                           bo, ny, nx, dx, (const uint8_t *)W.m, W.din, W.dout);
        // then along z (box-local [y][z][x] -> [z][y][x]) and along y (in [z][y][x])
        const EnvPair along_z{nullptr, ny, nx, {bi, bo}, {W.din, W.dout}, {W.f[0], W.f[1]}, {W.v[0], W.v[1]},
                              {W.zb[0], W.zb[1]}};
        const EnvPair along_y{W.m, ny, nx, {bi, bo}, {W.f[0], W.f[1]}, {W.din, W.dout}, {W.v[0], W.v[1]},
                              {W.zb[0], W.zb[1]}};
        hipLaunchKernelGGL(k_edt_envelope, dim3(blocks_for((int64_t)bo.by * bo.bx), 2), blk, 0, st, 0, dz, along_z);
        hipLaunchKernelGGL(k_edt_envelope, dim3(blocks_for((int64_t)bo.bz * bo.bx), 2), blk, 0, st, 1, dy, along_y);
        hipLaunchKernelGGL(k_salt_union, box_grid(bo), blk, 0, st, bo, bi, ny, nx, xb, (const uint8_t *)W.m,
                           (const double *)W.din,
                           (const double *)W.dout, grf + (int64_t)i * n, amplitude * rbar, W.K);
    }
    // opening (erode, dilate) then closing (dilate, erode), ping-ponging K and m
    const dim3 gw = box_grid(whole);
    const int ops[4] = {0, 1, 1, 0};
    for (int i = 0; i < 4; ++i) {
        const uint8_t *src = i % 2 ? W.m : W.K;
        uint8_t *dst = i % 2 ? W.K : W.m;
        if (nx % 4 == 0) {
            const unsigned xb4 = (unsigned)((nx / 4 + kSaltThreads - 1) / kSaltThreads);
            hipLaunchKernelGGL(k_morph4, dim3((unsigned)((int64_t)nz * ny * xb4)), blk, 0, st, ops[i], nz, ny, nx,
                               xb4, src, dst);
        } else {
            hipLaunchKernelGGL(k_morph, gw, blk, 0, st, ops[i], whole, nz, ny, nx, xw, src, dst);
        }
    }
    // components: labels in d_in's storage, sizes in d_out's
    int *label = (int *)W.din;
    unsigned *count = (unsigned *)W.dout;
    hipLaunchKernelGGL(k_cc_init, gw, blk, 0, st, whole, ny, nx, xw, (const uint8_t *)W.K, label);
    hipLaunchKernelGGL(k_cc_merge, gw, blk, 0, st, whole, ny, nx, xw, (const uint8_t *)W.K, label);
    hipLaunchKernelGGL(k_cc_flatten, dim3(blocks_for(n)), blk, 0, st, n, label);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), blk, 0, st, n, 0u, count);
    hipLaunchKernelGGL(k_cc_count, dim3(blocks_for((n + kCountPerThread - 1) / kCountPerThread)), blk, 0, st, n,
                       (const int *)label, count);
    hipLaunchKernelGGL(k_salt_write, dim3(blocks_for(n)), blk, 0, st, n, v, (const int *)label,
                       (const unsigned *)count, min_voxels, v_salt, v_water, out, mask_out);
    return hipGetLastError();
}

}  // namespace sg
