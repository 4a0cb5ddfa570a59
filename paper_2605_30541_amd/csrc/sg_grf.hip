// The random field of SaltSDT (SubsurfaceGen, arXiv 2605.30541, App. B,
// Alg. 4): white noise on a periodic grid of powers of two shaped in Fourier
// space by sqrt(P(k)), P(k) = (1 + sum_k (k_k l_k)^2)^-p, cropped to the
// volume and scaled to zero mean and unit variance.
//
// A 3D transform is three rounds of [batched 1D FFTs along the contiguous
// axis, written transposed so the next axis becomes the contiguous one]:
// after three rounds the layout is [z][y][x] again with every axis
// transformed.  Each round is one kernel (k_fft_t): radix-2 Cooley-Tukey in
// LDS with twiddles from a per-workgroup table of sincospif values; neither
// direction is scaled (the final normalisation removes every constant
// factor).  The real noise enters in the first forward round and the spectral
// factor in the first inverse round, as they load their lines.
#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftLds = 1024;        // longest line (the grid is at most 1024 per axis)
constexpr int kFftRows = 4;          // lines per workgroup

// The spectral factor sqrt(P(k)) of cell (z, y, x) of the [Pz][Py][Px]
// spectrum; k in radians per cell in the FFT's frequency order
// (0, 1, .., P/2-1, -P/2, .., -1) / P.
struct Spectrum {
    int Pz, Py, Px;
    double lz, ly, lx, half_p;
};

__device__ inline float spectral_amp(const Spectrum &S, int z, int y, int x)
{
    const double two_pi = 6.283185307179586;
    const double fz = (z < (S.Pz + 1) / 2 ? z : z - S.Pz) / (double)S.Pz;
    const double fy = (y < (S.Py + 1) / 2 ? y : y - S.Py) / (double)S.Py;
    const double fx = (x < (S.Px + 1) / 2 ? x : x - S.Px) / (double)S.Px;
    const double kz = two_pi * fz * S.lz, ky = two_pi * fy * S.ly, kx = two_pi * fx * S.lx;
    // the power in FP32 (hardware log2 / exp2): the field is FP32 and is normalised afterwards
    return exp2f(-(float)S.half_p * log2f((float)(1.0 + kz * kz + ky * ky + kx * kx)));
}

// One radix-2 butterfly: (u, v) -> (u + w v, u - w v).
__device__ inline void butterfly(float2 &u, float2 &v, float2 w)
{
    const float cs = w.x, sn = w.y;
    const float2 t = make_float2(cs * v.x - sn * v.y, cs * v.y + sn * v.x);
    v = make_float2(u.x - t.x, u.y - t.y);
    u = make_float2(u.x + t.x, u.y + t.y);
}

// One round of the 3D transform in one pass: the FFT of every line of
// in[D0][D1][L] (L = 2^logL; sign -1 forward, +1 inverse), written transposed to
// out[L][D0][D1].  A workgroup takes kRows lines of one d0 and consecutive
// d1, so every output row gets kRows consecutive values from it; its lines
// sit in LDS padded (one value per 32, one per line), so the bit-reversed
// stores, the butterflies' strides and the column-wise reads of the
// transposed write spread over the banks.
// The input is `in`, or, when `real_in` is given, the real values real_in
// with zero imaginary parts; with S.Pz > 0 every input value is first
// multiplied by the spectral factor of its cell (line / S.Py, line % S.Py,
// position) (the lines are then the x lines of the [Pz][Py][Px] spectrum).
// Radix-2 Cooley-Tukey in LDS: a bit-reversed load, then two butterfly
// stages per pass (each thread does the four butterflies of two stages on
// four values it holds: the butterflies and twiddles of stage after stage),
// one last radix-2 stage when logL is odd.
template <int kRows>
__global__ void __launch_bounds__(kFftThreads) k_fft_t(const float2 *__restrict__ in, const float *__restrict__ real_in,
                                                     Spectrum S, float2 *__restrict__ out, int logL, int D0, int D1,
                                                     float sign)
{
    __shared__ float2 buf[kRows * (kFftLds + kFftLds / 32 + 1)];
    __shared__ float2 tw[kFftLds / 2];
    // position r of line ln sits at ln * LS + r + r / 32: the pad breaks the
    // bank conflicts of the bit-reversed stores and of the early stages' strides
    const int L = 1 << logL, LS = L + L / 32 + 1;
    auto at = [&](int ln, int r) { return ln * LS + r + (r >> 5); };
    for (int m = threadIdx.x; m < L / 2; m += kFftThreads) {
        float sn, cs;
        sincospif(sign * (float)m / (float)(L / 2), &sn, &cs);
        tw[m] = make_float2(cs, sn);
    }
    // consecutive blocks of work go to one XCD (the hardware deals workgroups
    // to the 8 XCDs in turn), so the partial output rows that neighbouring
    // blocks write meet in one L2
    const int nblk = (int)gridDim.x, per = nblk >> 3, bid = (int)blockIdx.x;
    const int blk = bid >= per * 8 ? bid : (bid & 7) * per + (bid >> 3);
    const int nb1 = (D1 + kRows - 1) / kRows;
    const int d0 = blk / nb1, d1s = (blk % nb1) * kRows;
    const int nl = min(kRows, D1 - d1s);
    const int tot = nl * L;
    const int64_t line0 = (int64_t)d0 * D1 + d1s;
    // load (bit-reversed within each line), eight values in flight per thread
    constexpr int kBatch = 8;
    for (int i0 = 0; i0 < tot; i0 += kFftThreads * kBatch) {
        float2 v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int i = i0 + u * kFftThreads + threadIdx.x;
            if (i < tot) v[u] = real_in ? make_float2(real_in[line0 * L + i], 0.f) : in[line0 * L + i];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int i = i0 + u * kFftThreads + threadIdx.x;
            if (i >= tot) continue;
            const int ln = i >> logL, j = i & (L - 1);
            float2 x = v[u];
            if (S.Pz > 0) {
                const int64_t line = line0 + ln;
                const float amp = spectral_amp(S, (int)(line / S.Py), (int)(line % S.Py), j);
                x = make_float2(x.x * amp, x.y * amp);
            }
            const int r = logL == 0 ? 0 : (int)(__brev((unsigned)j) >> (32 - logL));
            buf[at(ln, r)] = x;
        }
    }
    __syncthreads();
    int s = 1;
    for (; s + 1 <= logL; s += 2) {
        const int h = 1 << (s - 1);
        for (int b = threadIdx.x; b < (tot >> 2); b += kFftThreads) {
            const int ln = b >> (logL - 2);
            const int bb = b & ((L >> 2) - 1);
            const int g = bb >> (s - 1), j = bb & (h - 1);
            const int k = (g << (s + 1)) + j;
            const int i0 = at(ln, k), i1 = at(ln, k + h), i2 = at(ln, k + 2 * h), i3 = at(ln, k + 3 * h);
            float2 x0 = buf[i0], x1 = buf[i1], x2 = buf[i2], x3 = buf[i3];
            const float2 w1 = tw[j << (logL - s)];
            butterfly(x0, x1, w1);
            butterfly(x2, x3, w1);
            butterfly(x0, x2, tw[j << (logL - s - 1)]);
            butterfly(x1, x3, tw[(j + h) << (logL - s - 1)]);
            buf[i0] = x0;
            buf[i1] = x1;
            buf[i2] = x2;
            buf[i3] = x3;
        }
        __syncthreads();
    }
    if (s == logL) {
        const int half = 1 << (s - 1);
        for (int b = threadIdx.x; b < (tot >> 1); b += kFftThreads) {
            const int ln = b >> (logL - 1);
            const int bb = b & ((L >> 1) - 1);
            const int g = bb >> (s - 1), j = bb & (half - 1);
            const int k = (g << s) + j;
            const int i0 = at(ln, k), i1 = at(ln, k + half);
            float2 u = buf[i0], v = buf[i1];
            butterfly(u, v, tw[j << (logL - s)]);
            buf[i0] = u;
            buf[i1] = v;
        }
        __syncthreads();
    }
    // transposed write: position j of line ln goes to out[j][d0][d1s + ln]
    for (int q = threadIdx.x; q < tot; q += kFftThreads) {
        const int j = q / nl, ln = q - j * nl;
        out[((int64_t)j * D0 + d0) * D1 + d1s + ln] = buf[at(ln, j)];
    }
}

// out = real part cropped to [nz][ny][nx]; per-block FP64 sums of v and v^2.
__global__ void __launch_bounds__(256) k_crop_real(const float2 *a, int Py, int Px, int nz, int ny, int nx, float *out,
                                                  double *partials)
{
    const int64_t n = (int64_t)nz * ny * nx;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const int64_t zy = i / nx;
        const int y = (int)(zy % ny), z = (int)(zy / ny);
        const float v = a[((int64_t)z * Py + y) * Px + x].x;
        out[i] = v;
        s1 += v;
        s2 += (double)v * v;
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = r1[0];
        partials[2 * blockIdx.x + 1] = r2[0];
    }
}

// One workgroup: mean and 1/std from the partial sums, in a fixed order.
__global__ void __launch_bounds__(256) k_grf_stats(const double *partials, int nblocks, int64_t n, double *stats)
{
    __shared__ double r1[256], r2[256];
    double s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        s1 += partials[2 * b];
        s2 += partials[2 * b + 1];
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = r1[0] / (double)n;
        const double var = r2[0] / (double)n - mean * mean;
        stats[0] = mean;
        stats[1] = var > 0.0 ? 1.0 / sqrt(var) : 0.0;
    }
}

__global__ void __launch_bounds__(256) k_grf_normalize(float *out, int64_t n, const double *stats)
{
    const double mean = stats[0], inv = stats[1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)(((double)out[i] - mean) * inv);
}

int log2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

unsigned grid1d(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

constexpr int kStatBlocks = 2048;

// One 3D transform of a[Pz][Py][Px] (b: scratch of the same size); the
// result is in a.
hipError_t fft3(float2 *&a, float2 *&b, const int P[3], float sign, const float *real_in, const Spectrum &S0,
                hipStream_t st)
{
    int dims[3] = {P[0], P[1], P[2]};           // current layout [d0][d1][d2], d2 contiguous
    for (int r = 0; r < 3; ++r) {
        const int L = dims[2];
        // the first round takes the real input or the spectral factor (if given)
        const float *rin = r == 0 ? real_in : nullptr;
        const Spectrum S = r == 0 ? S0 : Spectrum{};
        const int64_t wgs = (int64_t)dims[0] * ((dims[1] + kFftRows - 1) / kFftRows);
        hipLaunchKernelGGL(k_fft_t<kFftRows>, dim3((unsigned)wgs), dim3(kFftThreads), 0, st, a, rin, S, b, log2i(L),
                           dims[0], dims[1], sign);
        float2 *t = a;
        a = b;
        b = t;
        const int d0 = dims[0], d1 = dims[1];
        dims[0] = L;
        dims[1] = d0;
        dims[2] = d1;
    }
    return hipGetLastError();
}

}  // namespace

void grf_grid(int nz, int ny, int nx, int P[3])
{
    const int n[3] = {nz, ny, nx};
    for (int k = 0; k < 3; ++k) P[k] = 1 << log2i(n[k]);
}

size_t grf_workspace_bytes(int nz, int ny, int nx)
{
    int P[3];
    grf_grid(nz, ny, nx, P);
    const size_t n = (size_t)P[0] * P[1] * P[2];
    return 2 * n * sizeof(float2) + (size_t)kStatBlocks * 2 * sizeof(double) + 256;
}

hipError_t launch_grf(const float *noise, int nz, int ny, int nx, double lz, double ly, double lx, double p, float *out,
                      void *ws, hipStream_t st)
{
    int P[3];
    grf_grid(nz, ny, nx, P);
    const int64_t n = (int64_t)P[0] * P[1] * P[2];
    float2 *a = (float2 *)ws, *b = a + n;
    double *partials = (double *)(b + n);
    double *stats = partials + 2 * kStatBlocks;
    // forward transform of the real noise; the inverse one takes the spectral
    // factor as it loads its first lines
    hipError_t e = fft3(a, b, P, -1.f, noise, Spectrum{}, st);
    if (e != hipSuccess) return e;
    if ((e = fft3(a, b, P, 1.f, nullptr, Spectrum{P[0], P[1], P[2], lz, ly, lx, 0.5 * p}, st)) != hipSuccess) return e;
    const int64_t m = (int64_t)nz * ny * nx;
    hipLaunchKernelGGL(k_crop_real, dim3(kStatBlocks), dim3(256), 0, st, a, P[1], P[2], nz, ny, nx, out, partials);
    hipLaunchKernelGGL(k_grf_stats, dim3(1), dim3(256), 0, st, partials, kStatBlocks, m, stats);
    hipLaunchKernelGGL(k_grf_normalize, dim3(grid1d(m)), dim3(256), 0, st, out, m, stats);
    return hipGetLastError();
}

}  // namespace sg
