// Column-sweep time blocking of the forward step (SubsurfaceGen, arXiv
// 2605.30541: eqs. "acoustic_2d", "cerjan_pde", "free_surface"; App. E.3), for
// launches with many workgroups (many shots):
//   p^{n+1} = W L p^n + (2a (p^n - p^{n-1}) + p^{n-1}) + W S^n
// on every padded cell, the same expression and operation order as the tiled
// kernel (sg_kernels.hip), so both give the same bits.
//
// A workgroup owns one strip of 64 NW columns of one shot (its output columns
// plus a halo of 4 tb on each side) and walks the whole height of the padded
// grid once per launch, advancing TB levels in a skewed pipeline: at step j it
// takes level n at row j from memory and computes level n+s at row j - 4s for
// s = 1..TB.  Level n+s at row R needs level n+s-1 at rows R-4..R+4, which
// the previous level finished at this step or before, so nothing in z is
// recomputed; only the x halo is.  Each level keeps its last 9 rows (the
// stencil's reach) in registers -- z neighbours come from there -- and in a
// 9-row LDS ring for the x neighbours of the next level.  The step loop is
// unrolled by 9 so queue and ring slots are compile-time constants.
//
// Boundaries without branches: loads are clamped into the 4-cell zero guard
// ring of the stored fields, so rows and columns outside the padded grid read
// p = 0 with W = 2a = 0 and every value computed there is exactly 0; the
// pinned free-surface row has W = 2a = 0 too and stays 0.  Under a free top
// the ghost rows -1..-4 of every level hold minus rows 1..4 (odd mirror):
// when a level produces row R in 1..4 it writes -p into the register slot of
// row -R, before any row that reads it is computed.
#include "sg_internal.h"

#include <type_traits>

namespace sg {

namespace {

constexpr int kQ = 9;   // rows of a level kept: R-4..R+4

template <class T>
__device__ __forceinline__ T gld(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ T gld_at(const T *base, uint32_t byte_off)
{
    return gld((const T *)((const char *)base + byte_off));
}
__device__ __forceinline__ void gst_at(float *base, uint32_t byte_off, float v)
{
    *(__attribute__((address_space(1))) float *)((char *)base + byte_off) = v;
}

// Register / ring slot of a row, row = j + d at a step j with j mod 9 = PH.
constexpr int slot(int d) { return ((d % kQ) + kQ) % kQ; }

__device__ inline int xcd_block(int b, int nblocks)
{
    const int per = nblocks >> 3;
    if (b >= per * 8) return b;
    return (b & 7) * per + (b >> 3);
}

// RECOMP (the forward recompute of the gradient): also stores, for every level
// n+q-1 advanced, the second time difference D = (p^{n+q} - p^{n+q-1}) -
// (p^{n+q-1} - p^{n+q-2}) of the output cells in ring slot n+q-1 - t.ring_lo
// (streaming stores: read back only by the adjoint after the segment).
template <int NW, int TB, bool RECOMP>
__device__ __forceinline__ void sweep_body(const SliceDesc &s, const TileArgs &t, int b, float *lds)
{
    constexpr int EX = 64 * NW, LW = EX + 2 * kHalo, NTHR = 64 * NW, RING = kQ * LW;
    // block b: (shot, segment, strip); a segment is the output rows
    // [zs0, zs1) of the strip (t.tz rows; one segment = the whole height)
    const int tiles = t.ntx * t.ntz;
    const int shot = b / tiles;
    const int tile = b - shot * tiles;
    const int seg = tile / t.ntx;
    const int strip = tile - seg * t.ntx;
    const int zs0 = seg * t.tz, zs1 = min(zs0 + t.tz, s.Nz);
    const int ox = strip * t.tx, ox_end = min(ox + t.tx, s.Nx), ex0 = ox - kHalo * t.tb;
    const int lx = (int)threadIdx.x;
    const int X = ex0 + lx;
    const bool xout = X >= ox && X < ox_end;
    // clamped into the guard columns (zeros): no test on columns outside the grid
    const int Xc = min(max(X, -kGuard), s.Nx + kGuard - 1);
    const uint32_t xo4 = (uint32_t)(Xc + kGuard) * 4u;
    const uint32_t xs4 = (uint32_t)(X + kGuard) * 4u;     // store column (output lanes only)
    const int pitch = s.pitch, Nz = s.Nz;
    auto rowb = [&](int R) -> uint32_t {                    // clamped into the guard rows (zeros)
        R = min(max(R, -kGuard), Nz + kGuard - 1);
        return (uint32_t)((R + kGuard) * pitch) * 4u;
    };
    const int64_t fshot = (int64_t)shot * kFramesPerShot * s.frame;
    const float *in_prev = t.fields + fshot + (int64_t)(2 * t.in_pair) * s.frame;
    const float *in_cur = in_prev + s.frame;
    float *out_prev = t.fields + fshot + (int64_t)(2 * t.out_pair) * s.frame;
    float *out_cur = out_prev + s.frame;
    const bool free_top = s.free_top != 0;

    // rows holding source nodes of this shot (the nodes themselves and the
    // wavelet samples are read only at those rows; level n+s takes w(t_{n+s-1}))
    const int32_t *nz_ = s.src_iz + shot * kNodes;
    const int32_t *nx_ = s.src_ix + shot * kNodes;
    const float *nw_ = s.src_w + shot * kNodes;
    const float *wshot = s.wavelet + (int64_t)shot * s.wavelet_stride + t.n;
    int srow_lo = 1 << 30, srow_hi = -(1 << 30);
#pragma unroll
    for (int k = 0; k < kNodes; ++k)
        if (gld(nw_ + k) != 0.f) {
            srow_lo = min(srow_lo, gld(nz_ + k));
            srow_hi = max(srow_hi, gld(nz_ + k));
        }
    // receivers of this strip (entries sorted by base row); levels n..n+TB-1 due
    int rbeg = 0, rend = 0, rrow_lo = 1 << 30, rrow_hi = -(1 << 30);
    unsigned due = 0;
    if (s.gathers) {
        rbeg = gld(s.tile_rec + tile);
        rend = gld(s.tile_rec + tile + 1);
        if (rend > rbeg) {
            rrow_lo = gld(&s.rec_list[rbeg].lds) / LW;
            rrow_hi = gld(&s.rec_list[rend - 1].lds) / LW;
        }
#pragma unroll
        for (int q = 0; q < TB; ++q)
            if ((t.n + q) % s.rec_every == 0 && q < t.nsteps) due |= 1u << q;
    }
    // steps at which some due level records a receiver row (one range test per step)
    const int rec_j0 = due && rend > rbeg ? rrow_lo + 6 : 1 << 30;
    const int rec_j1 = due && rend > rbeg ? rrow_hi + 4 * (TB - 1) + 6 : -(1 << 30);

    float Q[TB][kQ];
#pragma unroll
    for (int a = 0; a < TB; ++a)
#pragma unroll
        for (int c = 0; c < kQ; ++c) Q[a][c] = 0.f;
    // this lane's column in ring row 0 of level 0, as a byte address
    const int lane_b = (lx + kHalo) * 4;
    float *const my = lds + lx + kHalo;
    // zero the rings (pad columns included: read only by discarded halo cells)
    for (int q = threadIdx.x; q < TB * RING; q += NTHR) lds[q] = 0.f;

    // Loads run two steps ahead of their use: step j takes level n at row j,
    // level n-1 at row j-4 and W, 2a at the rows j-4q its levels compute from
    // prefetch slot j mod 3 (3 divides the unroll of 9, so slots are
    // compile-time too) and issues the loads of step j+2 into slot (j+2) mod 3.
    constexpr int kPf = 3;
    float pc[kPf], pp[kPf], pw[kPf][TB], pa[kPf][TB];
    auto issue = [&](const int slotp, const int jj) {
        pc[slotp] = gld_at(in_cur, rowb(jj) + xo4);
        pp[slotp] = gld_at(in_prev, rowb(jj - 4) + xo4);
#pragma unroll
        for (int q = 0; q < TB; ++q) {
            const uint32_t o = rowb(jj - 4 * (q + 1)) + xo4;
            pw[slotp][q] = gld_at(s.W, o);
            pa[slotp][q] = gld_at(s.A2, o);
        }
    };
    // first step: the top segment starts at row -9 (every row above 0 is a
    // guard or ghost row); a lower one TB levels of 4 rows, plus the 4 rows
    // level n+1 reads above, before its first output row, on a multiple of 9
    // (the unrolled loop's phase 0): rows computed before then are not exact,
    // and no output row reads them
    const int jf = zs0 - 4 * TB - kHalo;
    const int j0 = zs0 == 0 ? -kQ : jf - (jf % kQ + kQ) % kQ;
#pragma unroll
    for (int q = 0; q < kPf; ++q) {   // (registers of every slot defined; slot 2 is refilled at the first step)
        pc[q] = pp[q] = 0.f;
#pragma unroll
        for (int r = 0; r < TB; ++r) pw[q][r] = pa[q][r] = 0.f;
    }
    issue(0, j0);
    issue(1, j0 + 1);

    auto step = [&](auto ph, const int j) {
        constexpr int PH = decltype(ph)::value;
        constexpr int PS = PH % kPf;
        // loads of step j+2 (slot (PH+2) mod 3 was last read at step j-1)
        issue((PH + 2) % kPf, j + 2);
        // A level's ring row written at step j is read by other waves at step
        // j+4 (x neighbours of the next level) and rows written at steps j-6,
        // j-5 by the receivers; the slot it overwrites was last read at step
        // j-5.  A barrier every third step orders both.
        if (PH % 3 == 0) __syncthreads();
        // level n, row j
        const float cin = pc[PS];
        Q[0][slot(PH)] = cin;
        my[slot(PH) * LW] = cin;
        if (free_top && j >= 1 && j <= kHalo) Q[0][slot(-PH)] = -cin;
        // receivers of levels n..n+TB-1 at base row j - 4q - 6
        if (j >= rec_j0 && j <= rec_j1) {
#pragma unroll
            for (int q = 0; q < TB; ++q) {
                const int Rb = j - 4 * q - 6;
                if (((due >> q) & 1u) && Rb >= rrow_lo && Rb <= rrow_hi) {
                    const float *L0 = lds + q * RING + slot(PH - 4 * q - 6) * LW;
                    const float *L1 = lds + q * RING + slot(PH - 4 * q - 5) * LW;
                    float *row = s.gathers + ((int64_t)shot * s.nrow + (t.n + q) / s.rec_every) * s.nrec;
                    for (int e = rbeg + (int)threadIdx.x; e < rend; e += NTHR) {
                        const int code = gld(&s.rec_list[e].lds);
                        if (code / LW != Rb) continue;
                        const int c = code - Rb * LW;
                        const float w0 = gld(&s.rec_list[e].w[0]), w1 = gld(&s.rec_list[e].w[1]);
                        const float w2 = gld(&s.rec_list[e].w[2]), w3 = gld(&s.rec_list[e].w[3]);
                        row[gld(&s.rec_list[e].r)] = w0 * L0[c] + w1 * L0[c + 1] + w2 * L1[c] + w3 * L1[c + 1];
                    }
                }
            }
        }
        // levels n+1 .. n+TB at rows j-4 .. j-4TB
        float vlast = 0.f;
#pragma unroll
        for (int q = 1; q <= TB; ++q) {
            const int R = j - 4 * q;
            const float(&P)[kQ] = Q[q - 1];
            const float c = P[slot(PH - 4 * q)];
            // x neighbours of level q-1 at row R: one address register per
            // read group (the empty asm keeps the compiler from folding the
            // ring offset into every read, which costs an add per pair)
            int xa = lane_b + ((q - 1) * RING + slot(PH - 4 * q) * LW - kHalo) * 4;   // column x - 4
            asm volatile("" : "+v"(xa));
            const float *xr = (const float *)((const char *)lds + xa);
            const float c4 = -4.f * c;
            float lap = 0.f;
#pragma unroll
            for (int m = 1; m <= kHalo; ++m) {
                const float zs = P[slot(PH - 4 * q + m)] + P[slot(PH - 4 * q - m)];
                lap = fmaf(s.cz[m], (zs + (xr[kHalo + m] + xr[kHalo - m])) + c4, lap);
            }
            const float old = q == 1 ? pp[PS] : Q[q - 2][slot(PH - 4 * q)];
            const float Wq = pw[PS][q - 1];
            float v = fmaf(Wq, lap, fmaf(pa[PS][q - 1], c - old, old));
            if (R >= srow_lo && R <= srow_hi) {
                const float wq = gld(wshot + (q - 1));
#pragma unroll
                for (int k = 0; k < kNodes; ++k) {
                    const float wk = gld(nw_ + k);
                    if (gld(nz_ + k) == R && X == gld(nx_ + k) && wk != 0.f) v = fmaf(Wq, wk * wq, v);
                }
            }
            if (RECOMP && R >= zs0 && R < zs1 && xout) {
                float *rl = t.ring + (int64_t)shot * t.ring_shot + (int64_t)(t.n + q - 1 - t.ring_lo) * s.frame;
                __builtin_nontemporal_store((v - c) - (c - old),
                                            (__attribute__((address_space(1))) float *)((char *)rl +
                                                (uint32_t)((R + kGuard) * pitch) * 4u + xs4));
            }
            if (q < TB) {
                Q[q][slot(PH - 4 * q)] = v;
                my[q * RING + slot(PH - 4 * q) * LW] = v;
                if (free_top && R >= 1 && R <= kHalo) Q[q][slot(4 * q - PH)] = -v;
            } else {
                vlast = v;
            }
        }
        // output: levels n+TB and n+TB-1 at row j - 4TB
        const int R = j - 4 * TB;
        if (R >= zs0 && R < zs1 && xout) {
            const uint32_t o = (uint32_t)((R + kGuard) * pitch) * 4u + xs4;
            gst_at(out_cur, o, vlast);
            gst_at(out_prev, o, Q[TB - 1][slot(PH - 4 * TB)]);
        }
    };

    // steps j0 .. j1-1: guard rows outside [-4, Nz+4) read as the clamped
    // guard row; the last step computes level n+TB at row zs1-1, or later the
    // last receiver sample (a receiver on the segment's last two rows is read
    // 6 steps after its rows of level n+TB-1 are computed); the rings were
    // zeroed before the first step's barrier
    const int nsteps = max(zs1 + 4 * TB, rec_j1 + 1) - j0;
    const int j1 = j0 + (nsteps + kQ - 1) / kQ * kQ;
    for (int j = j0; j < j1; j += kQ) {
        step(std::integral_constant<int, 0>{}, j);
        step(std::integral_constant<int, 1>{}, j + 1);
        step(std::integral_constant<int, 2>{}, j + 2);
        step(std::integral_constant<int, 3>{}, j + 3);
        step(std::integral_constant<int, 4>{}, j + 4);
        step(std::integral_constant<int, 5>{}, j + 5);
        step(std::integral_constant<int, 6>{}, j + 6);
        step(std::integral_constant<int, 7>{}, j + 7);
        step(std::integral_constant<int, 8>{}, j + 8);
    }
}

template <int NW, int TB, bool RECOMP>
__global__ void __launch_bounds__(64 * NW) k_sweep(SliceDesc s, TileArgs t)
{
    __shared__ float lds[TB * kQ * (64 * NW + 2 * kHalo)];
    sweep_body<NW, TB, RECOMP>(s, t, xcd_block(blockIdx.x, gridDim.x), lds);
}

template <int NW, int TB, bool RECOMP>
__global__ void __launch_bounds__(64 * NW) k_sweep_batch(const BatchItem *__restrict__ items, int nitems, int n,
                                                          int in_pair, int ring_lo)
{
    __shared__ float lds[TB * kQ * (64 * NW + 2 * kHalo)];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    int it = 0;
    if (nitems > 1) {
        const int lane = threadIdx.x & 63;
        int count = 0;
        for (int base = 0; base < nitems; base += 64) {
            const int i = base + lane;
            const bool le = i < nitems && gld(&items[i].block_start) <= b;
            count += __popcll(__ballot(le));
        }
        it = __builtin_amdgcn_readfirstlane(count - 1);
    }
    const SliceDesc s = items[it].s;
    TileArgs t = items[it].t;
    t.n = n;
    t.nsteps = TB;
    t.in_pair = in_pair;
    t.out_pair = in_pair ^ 1;
    t.ring_lo = ring_lo;
    sweep_body<NW, TB, RECOMP>(s, t, b - items[it].block_start, lds);
}

template <int NW, bool RECOMP>
hipError_t launch_sweep_nw(const SliceDesc *s, const TileArgs *t, const BatchItem *items, int nitems,
                           unsigned blocks, int n, int nsteps, int in_pair, int ring_lo, hipStream_t st)
{
#define SG_SWEEP(TBV)                                                                                                \
    case TBV:                                                                                                        \
        if (items)                                                                                                   \
            hipLaunchKernelGGL((k_sweep_batch<NW, TBV, RECOMP>), dim3(blocks), dim3(64 * NW), 0, st, items, nitems, \
                               n, in_pair, ring_lo);                                                                 \
        else                                                                                                         \
            hipLaunchKernelGGL((k_sweep<NW, TBV, RECOMP>), dim3(blocks), dim3(64 * NW), 0, st, *s, *t);            \
        break
    switch (nsteps) {
        SG_SWEEP(1);
        SG_SWEEP(2);
        SG_SWEEP(3);
        SG_SWEEP(4);
        SG_SWEEP(5);
        SG_SWEEP(6);
    default: return hipErrorInvalidValue;
    }
#undef SG_SWEEP
    return hipGetLastError();
}

}  // namespace

Tiling make_sweep_tiling(int Nz, int Nx, int nw, int tb, int seg_h)
{
    Tiling T{};
    T.ex = 64 * nw;
    T.ez = Nz;
    T.k = 0;
    T.tb = tb;
    T.tx = T.ex - 2 * kHalo * tb;
    T.tz = seg_h > 0 && seg_h < Nz ? seg_h : Nz;
    T.tz_top = T.tz;          // segments are equal from the top (free top or not)
    T.sweep_nw = nw;
    T.ok = (nw == 2 || nw == 4) && tb >= 1 && tb <= kSweepMaxTimeBlock && T.tx >= 1 && seg_h >= 0;
    if (!T.ok) return T;
    T.ntx = (Nx + T.tx - 1) / T.tx;
    T.ntz = (Nz + T.tz - 1) / T.tz;
    return T;
}

hipError_t launch_sweep(const SliceDesc &s, const TileArgs &t, int nw, hipStream_t st)
{
    const unsigned blocks = (unsigned)(t.ntx * t.ntz * s.nshot);
    const bool ring = t.ring != nullptr;
    switch (nw * 2 + (ring ? 1 : 0)) {
    case 4: return launch_sweep_nw<2, false>(&s, &t, nullptr, 0, blocks, t.n, t.nsteps, t.in_pair, 0, st);
    case 5: return launch_sweep_nw<2, true>(&s, &t, nullptr, 0, blocks, t.n, t.nsteps, t.in_pair, 0, st);
    case 8: return launch_sweep_nw<4, false>(&s, &t, nullptr, 0, blocks, t.n, t.nsteps, t.in_pair, 0, st);
    case 9: return launch_sweep_nw<4, true>(&s, &t, nullptr, 0, blocks, t.n, t.nsteps, t.in_pair, 0, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_batch(const BatchItem *items, int nitems, int total_blocks, int n, int nsteps, int in_pair,
                              int nw, hipStream_t st, bool ring, int ring_lo)
{
    const unsigned b = (unsigned)total_blocks;
    switch (nw * 2 + (ring ? 1 : 0)) {
    case 4: return launch_sweep_nw<2, false>(nullptr, nullptr, items, nitems, b, n, nsteps, in_pair, 0, st);
    case 5: return launch_sweep_nw<2, true>(nullptr, nullptr, items, nitems, b, n, nsteps, in_pair, ring_lo, st);
    case 8: return launch_sweep_nw<4, false>(nullptr, nullptr, items, nitems, b, n, nsteps, in_pair, 0, st);
    case 9: return launch_sweep_nw<4, true>(nullptr, nullptr, items, nitems, b, n, nsteps, in_pair, ring_lo, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sg
