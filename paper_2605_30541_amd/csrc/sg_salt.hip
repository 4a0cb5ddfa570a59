// SaltSDT (SubsurfaceGen, arXiv 2605.30541, App. B, Alg. 4): salt bodies from
// rotated ellipsoids whose signed distance is perturbed by a random field,
// merged, opened and closed, cleared of small components and written over
// the model below the water.  Volumes are [nz][ny][nx], x fastest.
//
// Kernels, in launch order:
//  * k_ellipsoid: the body raster on the voxel centres;
//  * k_edt_x, k_edt_envelope (y, then z): the exact squared Euclidean distance
//    to the nearest feature voxel as three separable passes.  Along x the
//    distance to the nearest feature of the row (the 1D transform of a
//    0/infinity function), one wave per row; along y and z the lower envelope
//    of parabolas in FP64, one thread per line (Felzenszwalb and
//    Huttenlocher's 1D transform; the paper names Meijster's algorithm, which
//    yields the same exact distances);
//  * k_salt_union: phi' = d_in - d_out + a rbar xi, K |= phi' > 0.  A body
//    covering no voxel gives d_out = infinity everywhere (phi' = -inf), one
//    covering all gives d_in = infinity (phi' = +inf): no special cases;
//  * k_morph x4: opening then closing with the 6-neighbour cross, a voxel
//    outside the volume counting as empty;
//  * k_cc_init, k_cc_merge, k_cc_flatten: 6-connected components by a
//    lock-free union-find (each salt voxel unites with its -x, -y, -z
//    neighbours by atomicMin on the roots; then every label is pointed at its
//    root), so each component ends labelled by its smallest voxel index;
//  * k_cc_count, k_salt_write: component sizes (one atomic per wave when the
//    wave's voxels share a label) and the final write.
// Decisions (inside the ellipsoid, phi' > 0) are taken in FP64 without
// fused multiply-adds, so they round as the plain definitions do.
#include "sg_internal.h"

#pragma clang fp contract(off)

namespace sg {

namespace {

constexpr int kSaltThreads = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kSaltThreads - 1) / kSaltThreads); }

__device__ inline double inf_d() { return __builtin_huge_val(); }

// Voxel kernels launch ny * nz rows of xb = ceil(nx / 256) blocks each; a
// block covers 256 consecutive voxels of one row, so the row (and z, y) comes
// from one division per block.  False for lanes past the end of the row.
__device__ inline bool row_voxel(int ny, int nx, unsigned xb, int &iz, int &iy, int &ix, int64_t &q)
{
    const unsigned row = blockIdx.x / xb;
    ix = (int)((blockIdx.x - row * xb) * kSaltThreads + threadIdx.x);
    if (ix >= nx) return false;
    iz = (int)(row / (unsigned)ny);
    iy = (int)(row - (unsigned)iz * (unsigned)ny);
    q = (int64_t)row * nx + ix;
    return true;
}

__global__ void __launch_bounds__(kSaltThreads) k_ellipsoid(int ny, int nx, unsigned xb, double dz, double dy,
                                                            double dx, SaltBody B, uint8_t *mask)
{
    int iz, iy, ix;
    int64_t q;
    if (!row_voxel(ny, nx, xb, iz, iy, ix, q)) return;
    const double p0 = iz * dz - B.c[0], p1 = iy * dy - B.c[1], p2 = ix * dx - B.c[2];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double u = (B.R[3 * k] * p0 + B.R[3 * k + 1] * p1 + B.R[3 * k + 2] * p2) / B.r[k];
        s += u * u;
    }
    mask[q] = s <= 1.0;
}

// Along x, one wave per (z, y) row: g = (dx * distance in cells to the nearest
// voxel of the row whose mask equals `feature`)^2, infinity if the row has
// none.  The row is walked in blocks of 64 voxels, one per lane (coalesced);
// a ballot gives the block's feature voxels, and the nearest one at or below
// (forward walk) or at or above (backward walk) each lane comes from the
// ballot bits, or from the carry of the blocks already walked.
constexpr int kRowsPerBlock = kSaltThreads / 64;

__global__ void __launch_bounds__(kSaltThreads) k_edt_x(int64_t rows, int nx, double dx, const uint8_t *mask,
                                                        uint8_t feature, double *g)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
    if (row >= rows) return;   // uniform over the wave
    const uint8_t *m = mask + row * nx;
    double *gr = g + row * nx;
    const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1);   // bits 0..lane
    const unsigned long long from = ~0ull << lane;                                       // bits lane..63
    int carry = -1;   // last feature before the block
    for (int x0 = 0; x0 < nx; x0 += 64) {
        const int x = x0 + lane;
        const unsigned long long b = __ballot(x < nx && m[x] == feature);
        const unsigned long long mb = b & upto;
        const int last = mb ? x0 + 63 - __clzll((long long)mb) : carry;
        if (x < nx) {
            const double d = dx * (double)(x - last);
            gr[x] = last < 0 ? inf_d() : d * d;
        }
        if (b) carry = x0 + 63 - __clzll((long long)b);
    }
    int next = -1;    // first feature after the block
    for (int x0 = (nx - 1) / 64 * 64; x0 >= 0; x0 -= 64) {
        const int x = x0 + lane;
        const unsigned long long b = __ballot(x < nx && m[x] == feature);
        const unsigned long long ma = b & from;
        const int nf = ma ? x0 + __ffsll((long long)ma) - 1 : next;
        if (x < nx && nf >= 0) {
            const double d = dx * (double)(nf - x);
            const double e = d * d;
            if (e < gr[x]) gr[x] = e;
        }
        if (b) next = x0 + __ffsll((long long)b) - 1;
    }
}

// g(p) = min_q (w (p - q))^2 + f(q) along one line: the lower envelope of the
// parabolas rooted at the finite samples.  axis 1: lines along y, one per
// (z, x); axis 0: lines along z, one per (y, x); neighbouring lanes take
// neighbouring x, so the reads of f and writes of g are coalesced.  v (int)
// and zb (double) hold the envelope's roots and boundaries, in the volume's
// own layout.
__global__ void __launch_bounds__(kSaltThreads) k_edt_envelope(int axis, int nz, int ny, int nx, double w,
                                                               const double *f, double *g, int *v, double *zb)
{
    const int64_t l = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    const int64_t plane = (int64_t)ny * nx;
    int n;
    int64_t base, stride;
    if (axis == 1) {
        if (l >= (int64_t)nz * nx) return;
        const int64_t iz = l / nx, ix = l - iz * nx;
        n = ny;
        base = iz * plane + ix;
        stride = nx;
    } else {
        if (l >= plane) return;
        n = nz;
        base = l;
        stride = plane;
    }
    const double w2 = w * w;
    int k = -1;       // index of the last parabola of the envelope
    double hk = 0.0;  // its f(v_k) + w^2 v_k^2
    int vk = 0;
    for (int q = 0; q < n; ++q) {
        const double fq = f[base + q * stride];
        if (!(fq < inf_d())) continue;
        const double hq = fq + w2 * ((double)q * q);
        double s = 0.0;
        while (k >= 0) {
            // abscissa where parabola q starts to lie below parabola v_k
            s = (hq - hk) / (2.0 * w2 * (double)(q - vk));
            if (k == 0 || s > zb[base + k * stride]) break;
            --k;
            vk = v[base + k * stride];
            hk = f[base + vk * stride] + w2 * ((double)vk * vk);
        }
        ++k;
        v[base + k * stride] = q;
        zb[base + k * stride] = k == 0 ? -inf_d() : s;
        vk = q;
        hk = hq;
    }
    if (k < 0) {
        for (int p = 0; p < n; ++p) g[base + p * stride] = inf_d();
        return;
    }
    int j = 0;
    int vj = v[base];
    for (int p = 0; p < n; ++p) {
        while (j < k && zb[base + (j + 1) * stride] < (double)p) {
            ++j;
            vj = v[base + j * stride];
        }
        const double d = w * (double)(p - vj);
        g[base + p * stride] = d * d + f[base + vj * stride];
    }
}

__global__ void __launch_bounds__(kSaltThreads) k_salt_union(int64_t n, const double *din2, const double *dout2,
                                                             const float *xi, double a_rbar, uint8_t *K)
{
    const int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    if (q >= n) return;
    const double phi = sqrt(din2[q]) - sqrt(dout2[q]);
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
__global__ void __launch_bounds__(kSaltThreads) k_morph(int op, int nz, int ny, int nx, unsigned xb,
                                                        const uint8_t *in, uint8_t *out)
{
    int iz, iy, ix;
    int64_t q;
    if (!row_voxel(ny, nx, xb, iz, iy, ix, q)) return;
    const int64_t plane = (int64_t)ny * nx;
    const bool c = in[q];
    const bool zm = iz > 0 && in[q - plane], zp = iz < nz - 1 && in[q + plane];
    const bool ym = iy > 0 && in[q - nx], yp = iy < ny - 1 && in[q + nx];
    const bool xm = ix > 0 && in[q - 1], xp = ix < nx - 1 && in[q + 1];
    out[q] = op == 0 ? (c && zm && zp && ym && yp && xm && xp) : (c || zm || zp || ym || yp || xm || xp);
}

__global__ void __launch_bounds__(kSaltThreads) k_cc_init(int64_t n, const uint8_t *K, int *label)
{
    const int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    if (q < n) label[q] = K[q] ? (int)q : -1;
}

// Labels form a forest: label[x] <= x for every salt voxel, a root has
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
// Every retry lowers a or b, so the loop ends; no thread waits on another.
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

__global__ void __launch_bounds__(kSaltThreads) k_cc_merge(int ny, int nx, unsigned xb, const uint8_t *K,
                                                           int *label)
{
    int iz, iy, ix;
    int64_t q;
    if (!row_voxel(ny, nx, xb, iz, iy, ix, q)) return;
    if (!K[q]) return;
    const int64_t plane = (int64_t)ny * nx;
    if (ix > 0 && K[q - 1]) unite(label, (int)q, (int)(q - 1));
    if (iy > 0 && K[q - nx]) unite(label, (int)q, (int)(q - nx));
    if (iz > 0 && K[q - plane]) unite(label, (int)q, (int)(q - plane));
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

__global__ void __launch_bounds__(kSaltThreads) k_cc_count(int64_t n, const int *label, unsigned *count)
{
    const int64_t q = (int64_t)blockIdx.x * kSaltThreads + threadIdx.x;
    const int l = q < n ? label[q] : -1;
    const unsigned long long set = __ballot(l >= 0);
    if (!set) return;
    const int lead = __ffsll((long long)set) - 1;
    const int l_lead = __shfl(l, lead);
    const unsigned long long same = __ballot(l == l_lead);
    if (same == set) {
        if ((int)(threadIdx.x & 63) == lead) atomicAdd(&count[l_lead], (unsigned)__popcll(set));
    } else if (l >= 0) {
        atomicAdd(&count[l], 1u);
    }
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
    double *din, *dout, *f, *zb;
    int *v;
    uint8_t *K, *m;
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

SaltWorkspace carve(void *ws, int64_t n)
{
    char *p = (char *)ws;
    SaltWorkspace W{};
    W.din = (double *)p;
    p += align256(8 * (size_t)n);
    W.dout = (double *)p;
    p += align256(8 * (size_t)n);
    W.f = (double *)p;
    p += align256(8 * (size_t)n);
    W.zb = (double *)p;
    p += align256(8 * (size_t)n);
    W.v = (int *)p;
    p += align256(4 * (size_t)n);
    W.K = (uint8_t *)p;
    p += align256((size_t)n);
    W.m = (uint8_t *)p;
    return W;
}

}  // namespace

size_t salt_workspace_bytes(int64_t n)
{
    return 4 * align256(8 * (size_t)n) + align256(4 * (size_t)n) + 2 * align256((size_t)n);
}

hipError_t launch_salt_sdt(const float *v, int nz, int ny, int nx, double dz, double dy, double dx, int nbodies,
                           const SaltBody *bodies, const float *grf, double amplitude, float v_salt, float v_water,
                           unsigned min_voxels, float *out, uint8_t *mask_out, void *ws, hipStream_t st)
{
    const int64_t plane = (int64_t)ny * nx, n = plane * nz;
    const SaltWorkspace W = carve(ws, n);
    const dim3 blk(kSaltThreads);
    const unsigned xb = (unsigned)((nx + kSaltThreads - 1) / kSaltThreads);
    const dim3 vox((unsigned)((int64_t)nz * ny * xb));
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for(n)), blk, 0, st, n, (uint8_t)0, W.K);
    for (int b = 0; b < nbodies; ++b) {
        const SaltBody &B = bodies[b];
        hipLaunchKernelGGL(k_ellipsoid, vox, blk, 0, st, ny, nx, xb, dz, dy, dx, B, W.m);
        // d_in: distance to the nearest voxel outside (feature 0); d_out: to the nearest inside (feature 1)
        for (int which = 0; which < 2; ++which) {
            double *D = which == 0 ? W.din : W.dout;
            const int64_t rows = (int64_t)nz * ny;
            hipLaunchKernelGGL(k_edt_x, dim3((unsigned)((rows + kRowsPerBlock - 1) / kRowsPerBlock)), blk, 0, st,
                               rows, nx, dx, (const uint8_t *)W.m, (uint8_t)which, D);
            hipLaunchKernelGGL(k_edt_envelope, dim3(blocks_for((int64_t)nz * nx)), blk, 0, st, 1, nz, ny, nx, dy,
                               (const double *)D, W.f, W.v, W.zb);
            hipLaunchKernelGGL(k_edt_envelope, dim3(blocks_for(plane)), blk, 0, st, 0, nz, ny, nx, dz,
                               (const double *)W.f, D, W.v, W.zb);
        }
        const double rbar = (B.r[0] + B.r[1] + B.r[2]) / 3.0;
        hipLaunchKernelGGL(k_salt_union, dim3(blocks_for(n)), blk, 0, st, n, (const double *)W.din,
                           (const double *)W.dout, grf + (int64_t)b * n, amplitude * rbar, W.K);
    }
    // opening (erode, dilate) then closing (dilate, erode), ping-ponging K and m
    hipLaunchKernelGGL(k_morph, vox, blk, 0, st, 0, nz, ny, nx, xb, (const uint8_t *)W.K, W.m);
    hipLaunchKernelGGL(k_morph, vox, blk, 0, st, 1, nz, ny, nx, xb, (const uint8_t *)W.m, W.K);
    hipLaunchKernelGGL(k_morph, vox, blk, 0, st, 1, nz, ny, nx, xb, (const uint8_t *)W.K, W.m);
    hipLaunchKernelGGL(k_morph, vox, blk, 0, st, 0, nz, ny, nx, xb, (const uint8_t *)W.m, W.K);
    // components: labels in d_in's storage, sizes in d_out's
    int *label = (int *)W.din;
    unsigned *count = (unsigned *)W.dout;
    hipLaunchKernelGGL(k_cc_init, dim3(blocks_for(n)), blk, 0, st, n, (const uint8_t *)W.K, label);
    hipLaunchKernelGGL(k_cc_merge, vox, blk, 0, st, ny, nx, xb, (const uint8_t *)W.K, label);
    hipLaunchKernelGGL(k_cc_flatten, dim3(blocks_for(n)), blk, 0, st, n, label);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), blk, 0, st, n, 0u, count);
    hipLaunchKernelGGL(k_cc_count, dim3(blocks_for(n)), blk, 0, st, n, (const int *)label, count);
    hipLaunchKernelGGL(k_salt_write, dim3(blocks_for(n)), blk, 0, st, n, v, (const int *)label,
                       (const unsigned *)count, min_voxels, v_salt, v_water, out, mask_out);
    return hipGetLastError();
}

}  // namespace sg
