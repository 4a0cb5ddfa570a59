// The random field of SaltSDT (SubsurfaceGen, arXiv 2605.30541, App. B,
// Alg. 4): white noise on a periodic grid of powers of two shaped in Fourier
// space by sqrt(P(k)), P(k) = (1 + sum_k (k_k l_k)^2)^-p, cropped to the
// volume and scaled to zero mean and unit variance.
//
// A 3D transform is three rounds of [batched 1D FFTs along the contiguous
// axis, then a 2D transpose of the (lines x length) matrix]: each round
// moves the transformed axis to the front, so after three the layout is
// [z][y][x] again with every axis transformed.  The 1D FFTs are radix-2
// Cooley-Tukey in LDS (bit-reversed load, log2 L butterfly stages, twiddles
// from a per-workgroup table of sincospif values); neither direction is
// scaled (the final normalisation removes every constant factor).  The real
// noise enters in the first forward pass and the spectral factor in the first
// inverse pass, as they load their lines.
#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftLds = 1024;        // complex values held per workgroup (one line of 1024 or several shorter)

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

// FFT of every line of length L = 2^logL (lines contiguous): sign -1 forward,
// +1 inverse.  A workgroup holds kFftLds / L lines (one when L = 1024).  The
// input is `data`, or, when `real_in` is given, the real values real_in with
// zero imaginary parts; with S.Pz > 0 every input value is first multiplied
// by the spectral factor of its cell (the lines are then the x lines of the
// [Pz][Py][Px] spectrum).  Two radix-2 stages per pass over LDS (the
// butterflies of both stages on four values a thread holds), one last
// radix-2 stage when logL is odd: the same butterflies, twiddles and order
// of operations as stage after stage.
__global__ void __launch_bounds__(kFftThreads) k_fft_lines(float2 *data, const float *real_in, Spectrum S, int logL,
                                                         int64_t nlines, float sign)
{
    __shared__ float2 buf[kFftLds];
    __shared__ float2 tw[kFftLds / 2];   // exp(sign i 2 pi m / L), m < L/2: stage s uses m = j 2^(logL-s)
    const int L = 1 << logL;
    for (int m = threadIdx.x; m < L / 2; m += kFftThreads) {
        float sn, cs;
        sincospif(sign * (float)m / (float)(L / 2), &sn, &cs);
        tw[m] = make_float2(cs, sn);
    }
    const int lpw = L >= kFftLds ? 1 : kFftLds / L;            // lines per workgroup
    const int64_t line0 = (int64_t)blockIdx.x * lpw;
    const int nl = (int)min((int64_t)lpw, nlines - line0);
    const int tot = nl * L;
    float2 *base = data + line0 * L;
    // load in bit-reversed order within each line
    for (int i = threadIdx.x; i < tot; i += kFftThreads) {
        const int ln = i >> logL, j = i & (L - 1);
        const int r = logL == 0 ? 0 : (int)(__brev((unsigned)j) >> (32 - logL));
        float2 v = real_in ? make_float2(real_in[line0 * L + i], 0.f) : base[i];
        if (S.Pz > 0) {
            const int64_t line = line0 + ln;
            const float amp = spectral_amp(S, (int)(line / S.Py), (int)(line % S.Py), j);
            v = make_float2(v.x * amp, v.y * amp);
        }
        buf[(ln << logL) + r] = v;
    }
    __syncthreads();
    int s = 1;
    for (; s + 1 <= logL; s += 2) {
        // stages s and s + 1 on the groups of four values k, k + h, k + 2h, k + 3h
        const int h = 1 << (s - 1);
        for (int b = threadIdx.x; b < (tot >> 2); b += kFftThreads) {
            const int ln = b >> (logL - 2);                     // line of this group
            const int bb = b & ((L >> 2) - 1);
            const int g = bb >> (s - 1), j = bb & (h - 1);
            const int k = (ln << logL) + (g << (s + 1)) + j;
            float2 x0 = buf[k], x1 = buf[k + h], x2 = buf[k + 2 * h], x3 = buf[k + 3 * h];
            const float2 w1 = tw[j << (logL - s)];              // exp(sign i 2 pi j / 2h)
            butterfly(x0, x1, w1);
            butterfly(x2, x3, w1);
            butterfly(x0, x2, tw[j << (logL - s - 1)]);         // exp(sign i 2 pi j / 4h)
            butterfly(x1, x3, tw[(j + h) << (logL - s - 1)]);   // exp(sign i 2 pi (j + h) / 4h)
            buf[k] = x0;
            buf[k + h] = x1;
            buf[k + 2 * h] = x2;
            buf[k + 3 * h] = x3;
        }
        __syncthreads();
    }
    if (s == logL) {   // the last stage alone
        const int half = 1 << (s - 1);
        for (int b = threadIdx.x; b < (tot >> 1); b += kFftThreads) {
            const int ln = b >> (logL - 1);                     // line of this butterfly
            const int bb = b & ((L >> 1) - 1);
            const int g = bb >> (s - 1), j = bb & (half - 1);
            const int k = (ln << logL) + (g << s) + j;
            float2 u = buf[k], v = buf[k + half];
            butterfly(u, v, tw[j << (logL - s)]);
            buf[k] = u;
            buf[k + half] = v;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < tot; i += kFftThreads) base[i] = buf[i];
}

// out[c][r] = in[r][c] for an R x C matrix of complex values (32 x 32 tiles).
__global__ void __launch_bounds__(256) k_transpose(const float2 *in, float2 *out, int64_t R, int64_t C)
{
    __shared__ float2 tile[32][33];
    const int64_t tr = (int64_t)blockIdx.x * 32, tc = (int64_t)blockIdx.y * 32;   // rows on x: up to 2^25 tiles
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;     // 32 x 8 threads
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = tr + k, c = tc + tx;
        if (r < R && c < C) tile[k][tx] = in[r * C + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = tc + k, r = tr + tx;
        if (r < R && c < C) out[c * R + r] = tile[tx][k];
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
    const int64_t n = (int64_t)P[0] * P[1] * P[2];
    int dims[3] = {P[0], P[1], P[2]};           // current layout [d0][d1][d2], d2 contiguous
    for (int r = 0; r < 3; ++r) {
        const int L = dims[2];
        const int logL = log2i(L);
        const int64_t nlines = n / L;
        const int lpw = L >= kFftLds ? 1 : kFftLds / L;
        // the first round takes the real input or the spectral factor (if given)
        const float *rin = r == 0 ? real_in : nullptr;
        const Spectrum S = r == 0 ? S0 : Spectrum{};
        if (L > 1 || rin || S.Pz > 0) {
            const int64_t wgs = (nlines + lpw - 1) / lpw;
            hipLaunchKernelGGL(k_fft_lines, dim3((unsigned)wgs), dim3(kFftThreads), 0, st, a, rin, S, logL, nlines,
                               sign);
        }
        const int64_t R = nlines, C = L;
        hipLaunchKernelGGL(k_transpose, dim3((unsigned)((R + 31) / 32), (unsigned)((C + 31) / 32)), dim3(256), 0, st,
                           a, b, R, C);
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
