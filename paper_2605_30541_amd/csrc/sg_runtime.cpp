// Host runtime of the acoustic propagator: plan validation, coefficient
// tables, acquisition tables, workspace layout and launch orchestration behind
// the C ABI of include/sgwave.h.
#include "sgwave.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "sg_internal.h"

namespace {

thread_local std::string g_last_error;

sg_status fail(sg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define SG_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(SG_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

// Central second-derivative weights of the 8th-order stencil (M = 4):
// the unique symmetric weights exact for polynomials up to degree 9
// (Fornberg 1988, cited for a_m in App. E.3.2).
constexpr double kC8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

constexpr double kPi = 3.14159265358979323846;

// s_max = (sqrt(d sum_{m>=1} |a_m|))^-1 with d = 2 (App. E.3.2).
double cfl_smax()
{
    double s = 0.0;
    for (int m = 1; m <= 4; ++m) s += std::fabs(kC8[m]);
    return 1.0 / std::sqrt(2.0 * s);
}

// Cerjan damping of one sponge side at depth d = 1..nbl cells (eq. "cerjan_damp"),
// returned in SI units (s/m^2): the paper's eta is in the solver's km/s-ms
// units, so eta_SI = eta * 1e-3; rho = d / nbl.
double sponge_eta(int d, int nbl, double h, double R)
{
    if (d <= 0 || nbl <= 0) return 0.0;
    const double cdamp = 1.5 * std::log(1.0 / R) / nbl;
    const double rho = (double)d / nbl;
    return cdamp / h * (rho - std::sin(2.0 * kPi * rho) / (2.0 * kPi)) * 1e-3;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Pinned host staging of the per-call tables.  A call fills one slot and
// copies it into the workspace on the caller's stream; the slot's event marks
// the end of that copy.  Slots are used in turn, so a slot is waited for only
// when kStageSlots calls are still queued ahead of its last copy: the host
// runs up to kStageSlots - 1 calls ahead of the GPU without blocking.
constexpr int kStageSlots = 4;
struct StageSlot {
    void *buf = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;      // done was recorded after the last copy
};

struct sg_plan {
    sg_geometry g;
    int32_t Nz, Nx, ztop, xleft, pitch, nrow;
    int64_t frame;
    uint32_t warnings;
    sg_tuning tuning;          // zeros = library choice
    std::vector<float> gx, gz; // eta / (2 dt) per padded column / row
    StageSlot stage[kStageSlots];
    int stage_next = 0;
    std::mutex mu;
    // optional per-launch timing of the time-stepping kernels
    bool profiling = false;
    std::vector<hipEvent_t> prof_ev;
    int prof_used = 0;       // event pairs recorded by the last call
    int prof_launches = 0;   // time-stepping launches they bracket
    // gradient calls: a second stream (default priority) on which a segment's
    // partial sums are folded while the next segment runs, and its events
    hipStream_t side = nullptr;
    hipEvent_t ev_seg = nullptr, ev_fold[2] = {nullptr, nullptr};
};

namespace {

// Workspace layout of one slice with nshot shots and nrec receivers
// (byte offsets).  Everything from gx to tables_end is uploaded from the
// plan's pinned staging buffer in one copy.  With ckpt > 0 the layout also
// holds the gradient state: checkpoints (levels jC-1, jC of every shot every
// C = ckpt levels), the ring of one segment's recomputed second time
// differences D^n (C levels; two of them, used by alternate segments, so a
// segment's partial imaging sums can be folded while the next segment runs),
// the adjoint field pairs, the FP64 accumulator of the imaging sum,
// and the residual-injection tables.
struct Layout {
    size_t v2, w, a2, gx, gz, src_off, src_iz, src_ix, src_w, rec_off, rec_iz, rec_ix, rec_w, tile_rec, rec_list;
    size_t inj_tile, inj_lds, inj_iz, inj_ix, inj_pstart, inj_rid, inj_w;
    size_t tables_end, fields;
    size_t ckpt, ring, ring2, mu, hsum, total;
    int ckpt_every, nseg, ring_levels;
    int64_t inj_cap;   // capacity (cells and pairs) of the injection tables
};

// Upper bound on the tiles of one shot over every tiling the plan may use
// (the smallest output tile is 8 x 8 with a free top).
int64_t max_tiles(const sg_plan *p) { return ((int64_t)p->Nz / 8 + 2) * ((int64_t)p->Nx / 8 + 2); }

// Upper bound on the loaded regions (tiles) one grid node can fall into, over
// every built tiling: per dimension 1 + 2 ceil(halo / output tile) <= 9.
constexpr int64_t kMaxTilesPerNode = 81;

int ckpt_spacing(const sg_plan *p, int ckpt_every)
{
    return ckpt_every > 0 ? ckpt_every : (int)std::ceil(std::sqrt((double)p->g.nt));
}

Layout layout_of(const sg_plan *p, int nshot, int nrec, int ckpt = 0)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    const size_t ns = (size_t)nshot * sg::kNodes, nr = (size_t)std::max(nrec, 1);
    const size_t fr = (size_t)p->frame * sizeof(float);
    L.v2 = take(fr);
    L.w = take(fr);
    L.a2 = take(fr);
    L.gx = take((size_t)p->Nx * sizeof(float));
    L.gz = take((size_t)p->Nz * sizeof(float));
    L.src_off = take(ns * sizeof(int32_t));
    L.src_iz = take(ns * sizeof(int32_t));
    L.src_ix = take(ns * sizeof(int32_t));
    L.src_w = take(ns * sizeof(float));
    L.rec_off = take(nr * sg::kNodes * sizeof(int32_t));
    L.rec_iz = take(nr * sizeof(int32_t));
    L.rec_ix = take(nr * sizeof(int32_t));
    L.rec_w = take(nr * sg::kNodes * sizeof(float));
    L.tile_rec = take(((size_t)max_tiles(p) + 1) * sizeof(int32_t));
    L.rec_list = take(nr * sizeof(sg::RecEntry));
    if (ckpt > 0) {
        L.inj_cap = kMaxTilesPerNode * sg::kNodes * (int64_t)nr;
        const size_t cap = (size_t)L.inj_cap;
        L.inj_tile = take(((size_t)max_tiles(p) + 1) * sizeof(int32_t));
        L.inj_lds = take(cap * sizeof(int32_t));
        L.inj_iz = take(cap * sizeof(int32_t));
        L.inj_ix = take(cap * sizeof(int32_t));
        L.inj_pstart = take((cap + 1) * sizeof(int32_t));
        L.inj_rid = take(cap * sizeof(int32_t));
        L.inj_w = take(cap * sizeof(float));
    }
    L.tables_end = o;
    L.fields = take((size_t)nshot * sg::kFramesPerShot * fr);
    if (ckpt > 0) {
        L.ckpt_every = ckpt;
        L.nseg = (p->g.nt + ckpt - 1) / ckpt;
        L.ring_levels = ckpt;                     // D^n of one segment
        L.ckpt = take((size_t)nshot * L.nseg * 2 * fr);
        L.ring = take((size_t)nshot * L.ring_levels * fr);
        L.ring2 = take((size_t)nshot * L.ring_levels * fr);   // segments alternate between the two rings
        L.mu = take((size_t)nshot * sg::kFramesPerShot * fr);
        L.hsum = take((size_t)nshot * 2 * fr);     // doubles
    }
    L.total = o;
    return L;
}

// Bilinear nodes of a point at (z, x) metres, in the order (0,0), (0,1),
// (1,0), (1,1) from the base node: stored-field offsets, padded (row, col)
// and weights times `scale`.  Nodes with zero weight, and nodes on a pinned
// free-surface row, are dropped (offset -1, weight 0).  Returns false outside
// the physical grid.
constexpr int32_t kNoNode = -(1 << 20);

struct Nodes {
    int32_t base_iz, base_ix;
    int32_t off[sg::kNodes], iz[sg::kNodes], ix[sg::kNodes];
    float w[sg::kNodes];
};

bool bilinear(const sg_plan *p, double z, double x, double scale, Nodes *out)
{
    const sg_geometry &g = p->g;
    if (!std::isfinite(z) || !std::isfinite(x)) return false;
    const double fz = z / g.dz, fx = x / g.dx;
    if (!(fz >= 0.0 && fx >= 0.0 && fz <= g.nz - 1 && fx <= g.nx - 1)) return false;
    int iz = (int)std::floor(fz), ix = (int)std::floor(fx);
    iz = std::min(iz, g.nz - 1);
    ix = std::min(ix, g.nx - 1);
    const double rz = fz - iz, rx = fx - ix;
    out->base_iz = iz + p->ztop;
    out->base_ix = ix + p->xleft;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int k = 2 * a + b;
            const double wt = (a ? rz : 1.0 - rz) * (b ? rx : 1.0 - rx);
            const int Iz = iz + a + p->ztop, Ix = ix + b + p->xleft;
            out->off[k] = -1;
            out->iz[k] = kNoNode;
            out->ix[k] = kNoNode;
            out->w[k] = 0.f;
            if (wt != 0.0 && !(g.top == SG_TOP_FREE && Iz == 0)) {
                out->off[k] = (int32_t)((int64_t)(Iz + sg::kGuard) * p->pitch + Ix + sg::kGuard);
                out->iz[k] = Iz;
                out->ix[k] = Ix;
                out->w[k] = (float)(wt * scale);
            }
        }
    return true;
}

sg_status check_shots(const sg_plan *p, const sg_shots *sh)
{
    if (!sh) return fail(SG_EINVAL, "shots is NULL");
    if (sh->nshot < 1) return fail(SG_EINVAL, "nshot must be >= 1 (got %d)", sh->nshot);
    if (sh->nrec < 0) return fail(SG_EINVAL, "nrec must be >= 0");
    if (!sh->src_zx) return fail(SG_EINVAL, "src_zx is NULL");
    if (sh->nrec > 0 && !sh->rec_zx) return fail(SG_EINVAL, "rec_zx is NULL");
    if (!sh->wavelet) return fail(SG_EINVAL, "wavelet is NULL");
    Nodes nd;
    for (int i = 0; i < sh->nshot; ++i)
        if (!bilinear(p, sh->src_zx[2 * i], sh->src_zx[2 * i + 1], 1.0, &nd))
            return fail(SG_EINVAL, "source %d at (%g, %g) m is outside the physical grid", i,
                        sh->src_zx[2 * i], sh->src_zx[2 * i + 1]);
    for (int i = 0; i < sh->nrec; ++i)
        if (!bilinear(p, sh->rec_zx[2 * i], sh->rec_zx[2 * i + 1], 1.0, &nd))
            return fail(SG_EINVAL, "receiver %d at (%g, %g) m is outside the physical grid", i,
                        sh->rec_zx[2 * i], sh->rec_zx[2 * i + 1]);
    return SG_OK;
}

sg::SliceDesc describe(const sg_plan *p, const Layout &L, char *ws, const sg_shots *sh,
                       float *gathers, float *snaps)
{
    const sg_geometry &g = p->g;
    sg::SliceDesc s{};
    s.Nz = p->Nz;
    s.Nx = p->Nx;
    s.pitch = p->pitch;
    s.nz = g.nz;
    s.nx = g.nx;
    s.ztop = p->ztop;
    s.xleft = p->xleft;
    s.free_top = g.top == SG_TOP_FREE;
    // cells outside every sponge side have eta = 0 exactly, so a = 1 and 2a = 2;
    // the pinned free-surface row is not updated (2a = 0)
    s.unit_z0 = std::max(p->ztop, s.free_top ? 1 : 0);
    s.unit_z1 = p->ztop + g.nz;
    s.unit_x0 = p->xleft;
    s.unit_x1 = p->xleft + g.nx;
    s.nshot = sh->nshot;
    s.nrec = sh->nrec;
    s.nrow = p->nrow;
    s.rec_every = g.rec_every;
    s.snap_every = g.snap_every > 0 ? g.snap_every : 1;
    s.snap_count = g.snap_count;
    s.wavelet_stride = sh->wavelet_per_shot ? g.nt : 0;
    s.frame = p->frame;
    for (int m = 0; m <= sg::kHalo; ++m) {
        s.cz[m] = (float)(kC8[m] / (g.dz * g.dz));
        s.cx[m] = (float)(kC8[m] / (g.dx * g.dx));
    }
    s.V2 = (const float *)(ws + L.v2);
    s.W = (const float *)(ws + L.w);
    s.A2 = (const float *)(ws + L.a2);
    s.gx = (const float *)(ws + L.gx);
    s.gz = (const float *)(ws + L.gz);
    s.src_off = (const int32_t *)(ws + L.src_off);
    s.src_iz = (const int32_t *)(ws + L.src_iz);
    s.src_ix = (const int32_t *)(ws + L.src_ix);
    s.src_w = (const float *)(ws + L.src_w);
    s.rec_off = (const int32_t *)(ws + L.rec_off);
    s.rec_iz = (const int32_t *)(ws + L.rec_iz);
    s.rec_ix = (const int32_t *)(ws + L.rec_ix);
    s.rec_w = (const float *)(ws + L.rec_w);
    s.tile_rec = (const int32_t *)(ws + L.tile_rec);
    s.rec_list = (const sg::RecEntry *)(ws + L.rec_list);
    s.wavelet = sh->wavelet;
    s.fields = (float *)(ws + L.fields);
    s.gathers = sh->nrec > 0 ? gathers : nullptr;
    s.snaps = g.snap_count > 0 ? snaps : nullptr;
    return s;
}

// Instantiated kernel shape matching a tuning's extended tile; -1 if none.
int shape_of(const sg_tuning &t)
{
    for (int c = 0; c < sg::kTiledShapes; ++c) {
        const sg::TiledShape sh = sg::tiled_shape(c);
        if (sh.ex == t.tile_x && sh.ez == t.tile_z && (t.rows_per_thread == 0 || t.rows_per_thread == sh.k))
            return c;
    }
    return -1;
}

// Tuning of a call: the plan's setting with zeros replaced by defaults (time
// block 4 for forward calls, 3 for the gradient calls, the fastest in
// measurements of each on the field-scale workloads).
sg_tuning resolve_tuning(const sg_plan *p, int nshot, bool gradient = false)
{
    (void)nshot;
    sg_tuning t = p->tuning;
    if (t.variant == 0) t.variant = 2;
    if (t.variant == 1) {
        t.tile_x = t.tile_z = t.rows_per_thread = 0;
        t.time_block = 1;
        return t;
    }
    if (t.variant == 3) {         // column sweep: strip width, segment height (0 = whole)
        if (t.tile_x == 0) t.tile_x = 256;
        t.rows_per_thread = 0;
        if (t.time_block <= 0) t.time_block = 4;
        return t;
    }
    if (t.tile_x == 0 || t.tile_z == 0) {
        t.tile_x = 128;
        t.tile_z = 64;
    }
    if (t.time_block <= 0) t.time_block = gradient ? 3 : 4;
    const int c = shape_of(t);
    if (c >= 0) t.rows_per_thread = sg::tiled_shape(c).k;
    return t;
}

sg_status tiling_for(const sg_plan *p, const sg_tuning &t, int *config, sg::Tiling *T)
{
    if (t.variant == 3) {
        *config = -1;
        if (p->g.dz != p->g.dx) return fail(SG_EUNSUPPORTED, "the column-sweep kernel needs dz == dx");
        if (t.tile_x != 128 && t.tile_x != 256) return fail(SG_EUNSUPPORTED, "sweep strips are 128 or 256 columns");
        if (t.time_block < 1 || t.time_block > sg::kSweepMaxTimeBlock)
            return fail(SG_EINVAL, "sweep time_block must be in 1..%d", sg::kSweepMaxTimeBlock);
        if (t.tile_z != 0 && t.tile_z < 8) return fail(SG_EINVAL, "sweep segments are 0 (whole height) or >= 8 rows");
        *T = sg::make_sweep_tiling(p->Nz, p->Nx, t.tile_x / 64, t.time_block, t.tile_z);
        if (!T->ok) return fail(SG_EUNSUPPORTED, "time block %d leaves no output strip", t.time_block);
        if ((int64_t)T->ntx * T->ntz > max_tiles(p)) return fail(SG_EUNSUPPORTED, "tiling too fine");
        return SG_OK;
    }
    *config = shape_of(t);
    if (*config < 0) return fail(SG_EUNSUPPORTED, "no kernel built for a %d x %d tile", t.tile_x, t.tile_z);
    if (t.time_block < 1 || t.time_block > sg::kMaxTimeBlock)
        return fail(SG_EINVAL, "time_block must be in 1..%d", sg::kMaxTimeBlock);
    const sg::TiledShape sh = sg::tiled_shape(*config);
    *T = sg::make_tiling(p->Nz, p->Nx, p->g.top == SG_TOP_FREE, sh.ex, sh.ez, sh.k, t.time_block);
    if (!T->ok) return fail(SG_EUNSUPPORTED, "time block %d leaves no output tile in %d x %d", t.time_block,
                            sh.ex, sh.ez);
    if ((int64_t)T->ntx * T->ntz > max_tiles(p)) return fail(SG_EUNSUPPORTED, "tiling too fine");
    return SG_OK;
}

// Grows every staging slot of the plan to at least `bytes` (pinned host
// memory) and creates the slots' events.  Caller holds p->mu.
sg_status reserve_stage(sg_plan *p, size_t bytes)
{
    for (StageSlot &sl : p->stage) {
        if (!sl.done) SG_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        if (sl.bytes >= bytes) continue;
        if (sl.pending) SG_HIP(hipEventSynchronize(sl.done));
        sl.pending = false;
        if (sl.buf) SG_HIP(hipHostFree(sl.buf));
        sl.buf = nullptr;
        sl.bytes = 0;
        SG_HIP(hipHostMalloc(&sl.buf, bytes, hipHostMallocDefault));
        sl.bytes = bytes;
    }
    return SG_OK;
}

// Table bytes (staged per call) of a call with nshot shots and nrec receivers.
size_t table_bytes(const sg_plan *p, int nshot, int nrec, int ckpt)
{
    const Layout L = layout_of(p, nshot, nrec, ckpt);
    return L.tables_end - L.gx;
}

// Copy the 1D damping tables and the acquisition tables of `sh` into the
// workspace: filled in the plan's next staging slot, copied on `st`.  A slot
// smaller than the tables grows (one pinned allocation) unless `may_alloc`
// is false, which gives SG_ENOSPACE instead.  `T` (may be null) gives the
// tiling whose per-tile receiver lists are built.
sg_status upload_tables(sg_plan *p, const Layout &L, char *ws, const sg_shots *sh, const sg::Tiling *T,
                        hipStream_t st, bool may_alloc = true)
{
    const size_t bytes = L.tables_end - L.gx;
    std::lock_guard<std::mutex> lock(p->mu);
    StageSlot &slot = p->stage[p->stage_next];
    if (slot.bytes < bytes || !slot.done) {
        if (!may_alloc)
            return fail(SG_ENOSPACE, "the plan's pinned staging holds %zu bytes of tables, this call needs %zu "
                        "(sg_plan_reserve sizes it)", slot.bytes, bytes);
        sg_status rc = reserve_stage(p, bytes);
        if (rc != SG_OK) return rc;
    }
    // the copy out of this slot kStageSlots calls ago must have finished
    if (slot.pending) SG_HIP(hipEventSynchronize(slot.done));
    slot.pending = false;
    p->stage_next = (p->stage_next + 1) % kStageSlots;
    char *h = (char *)slot.buf;
    auto at = [&](size_t off) { return h + (off - L.gx); };
    std::memset(h, 0, bytes);
    std::memcpy(at(L.gx), p->gx.data(), p->gx.size() * sizeof(float));
    std::memcpy(at(L.gz), p->gz.data(), p->gz.size() * sizeof(float));
    const double inv_cell = 1.0 / (p->g.dx * p->g.dz);
    Nodes nd;
    for (int i = 0; i < sh->nshot; ++i) {
        bilinear(p, sh->src_zx[2 * i], sh->src_zx[2 * i + 1], inv_cell, &nd);
        for (int k = 0; k < sg::kNodes; ++k) {
            ((int32_t *)at(L.src_off))[i * sg::kNodes + k] = nd.off[k];
            ((int32_t *)at(L.src_iz))[i * sg::kNodes + k] = nd.iz[k];
            ((int32_t *)at(L.src_ix))[i * sg::kNodes + k] = nd.ix[k];
            ((float *)at(L.src_w))[i * sg::kNodes + k] = nd.w[k];
        }
    }
    std::vector<int32_t> rtile(std::max(sh->nrec, 0));
    for (int k = 0; k < std::max(sh->nrec, 1) * sg::kNodes; ++k) ((int32_t *)at(L.rec_off))[k] = -1;
    for (int i = 0; i < sh->nrec; ++i) {
        bilinear(p, sh->rec_zx[2 * i], sh->rec_zx[2 * i + 1], 1.0, &nd);
        for (int k = 0; k < sg::kNodes; ++k) {
            ((int32_t *)at(L.rec_off))[i * sg::kNodes + k] = nd.off[k];
            ((float *)at(L.rec_w))[i * sg::kNodes + k] = nd.w[k];
        }
        ((int32_t *)at(L.rec_iz))[i] = nd.base_iz;
        ((int32_t *)at(L.rec_ix))[i] = nd.base_ix;
        if (T) {   // tile holding the base node
            int tz;
            if (p->g.top == SG_TOP_FREE)
                tz = nd.base_iz < T->tz_top ? 0 : 1 + (nd.base_iz - T->tz_top) / T->tz;
            else
                tz = nd.base_iz / T->tz;
            rtile[i] = tz * T->ntx + nd.base_ix / T->tx;
        }
    }
    if (T) {   // receivers grouped by the tile holding their base node, with LDS indices
        const int tiles = T->ntx * T->ntz, LW = T->ex + 2 * sg::kHalo, halo = sg::kHalo * T->tb;
        const bool free_top = p->g.top == SG_TOP_FREE;
        int32_t *start = (int32_t *)at(L.tile_rec);
        sg::RecEntry *list = (sg::RecEntry *)at(L.rec_list);
        std::vector<int32_t> count(tiles + 1, 0);
        for (int i = 0; i < sh->nrec; ++i) ++count[rtile[i] + 1];
        for (int q = 0; q < tiles; ++q) count[q + 1] += count[q];
        for (int q = 0; q <= tiles; ++q) start[q] = count[q];
        for (int i = 0; i < sh->nrec; ++i) {
            const int tile = rtile[i], tzi = tile / T->ntx, txi = tile % T->ntx;
            const int ez0 = T->sweep_nw > 0 ? 0
                            : free_top ? (tzi == 0 ? -T->k : T->tz_top + (tzi - 1) * T->tz - halo)
                                       : tzi * T->tz - halo;
            const int ex0 = txi * T->tx - halo;
            sg::RecEntry &e = list[count[tile]++];
            const int32_t biz = ((const int32_t *)at(L.rec_iz))[i], bix = ((const int32_t *)at(L.rec_ix))[i];
            // tiled: index in the tile's LDS buffer; sweep: base row * LW + column in the strip's LDS row
            e.lds = T->sweep_nw > 0 ? biz * LW + (bix - ex0 + sg::kHalo)
                                    : (biz - ez0 + sg::kHalo) * LW + (bix - ex0 + sg::kHalo);
            e.r = i;
            for (int k = 0; k < sg::kNodes; ++k) e.w[k] = ((const float *)at(L.rec_w))[i * sg::kNodes + k];
        }
        if (T->sweep_nw > 0)   // the sweep reads a strip's entries by base row
            for (int q = 0; q < tiles; ++q)
                std::stable_sort(list + start[q], list + start[q + 1],
                                 [](const sg::RecEntry &a, const sg::RecEntry &b) { return a.lds < b.lds; });
    }
    if (T && L.inj_cap > 0) {
        // adjoint residual injection: receiver nodes inside each tile's loaded
        // region, grouped by cell in a fixed order
        const int tiles = T->ntx * T->ntz, LW = T->ex + 2 * sg::kHalo, halo = sg::kHalo * T->tb;
        const bool free_top = p->g.top == SG_TOP_FREE;
        std::vector<Nodes> rn(std::max(sh->nrec, 0));
        for (int i = 0; i < sh->nrec; ++i) bilinear(p, sh->rec_zx[2 * i], sh->rec_zx[2 * i + 1], 1.0, &rn[i]);
        int32_t *tstart = (int32_t *)at(L.inj_tile), *clds = (int32_t *)at(L.inj_lds);
        int32_t *ciz = (int32_t *)at(L.inj_iz), *cix = (int32_t *)at(L.inj_ix);
        int32_t *cps = (int32_t *)at(L.inj_pstart), *prid = (int32_t *)at(L.inj_rid);
        float *pw = (float *)at(L.inj_w);
        int64_t ncell = 0, npair = 0;
        std::vector<std::pair<int64_t, std::pair<int32_t, float>>> hits;
        for (int tile = 0; tile < tiles; ++tile) {
            const int tzi = tile / T->ntx, txi = tile % T->ntx;
            const int ez0 = free_top ? (tzi == 0 ? -T->k : T->tz_top + (tzi - 1) * T->tz - halo) : tzi * T->tz - halo;
            const int ex0 = txi * T->tx - halo;
            hits.clear();
            for (int r = 0; r < sh->nrec; ++r)
                for (int q = 0; q < sg::kNodes; ++q) {
                    if (rn[r].w[q] == 0.f) continue;
                    const int iz = rn[r].iz[q], ix = rn[r].ix[q];
                    if (iz >= ez0 && iz < ez0 + T->ez && ix >= ex0 && ix < ex0 + T->ex)
                        hits.push_back({(int64_t)iz * p->Nx + ix, {r, rn[r].w[q]}});
                }
            std::stable_sort(hits.begin(), hits.end(),
                             [](const auto &a, const auto &b) { return a.first < b.first; });
            tstart[tile] = (int32_t)ncell;
            for (size_t q = 0; q < hits.size(); ++q) {
                if (q == 0 || hits[q].first != hits[q - 1].first) {
                    if (ncell >= L.inj_cap) return fail(SG_EINVAL, "receiver injection tables overflow");
                    const int iz = (int)(hits[q].first / p->Nx), ix = (int)(hits[q].first % p->Nx);
                    ciz[ncell] = iz;
                    cix[ncell] = ix;
                    clds[ncell] = (iz - ez0 + sg::kHalo) * LW + (ix - ex0 + sg::kHalo);
                    cps[ncell] = (int32_t)npair;
                    ++ncell;
                }
                if (npair >= L.inj_cap) return fail(SG_EINVAL, "receiver injection tables overflow");
                prid[npair] = hits[q].second.first;
                pw[npair] = hits[q].second.second;
                ++npair;
            }
        }
        tstart[tiles] = (int32_t)ncell;
        cps[ncell] = (int32_t)npair;
    }
    SG_HIP(hipMemcpyAsync(ws + L.gx, h, bytes, hipMemcpyHostToDevice, st));
    SG_HIP(hipEventRecord(slot.done, st));
    slot.pending = true;
    return SG_OK;
}

// The plan's side stream and events for the gradient's folds (created on
// first use; default priority, no blocking of the null stream).
sg_status side_stream(sg_plan *p)
{
    if (!p->side) SG_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    if (!p->ev_seg) SG_HIP(hipEventCreateWithFlags(&p->ev_seg, hipEventDisableTiming));
    for (hipEvent_t &e : p->ev_fold)
        if (!e) SG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return SG_OK;
}

// Event pair i of the profiling buffer (created on first use).
sg_status prof_pair(sg_plan *p, int i, hipEvent_t *a, hipEvent_t *b)
{
    while ((int)p->prof_ev.size() < 2 * (i + 1)) {
        hipEvent_t e;
        SG_HIP(hipEventCreate(&e));
        p->prof_ev.push_back(e);
    }
    *a = p->prof_ev[2 * i];
    *b = p->prof_ev[2 * i + 1];
    return SG_OK;
}

sg::TileArgs tile_args(const sg::Tiling &T, float *fields, int n, int nsteps, int in_pair)
{
    sg::TileArgs a{};
    a.n = n;
    a.nsteps = nsteps;
    a.tb = T.tb;
    a.tx = T.tx;
    a.tz = T.tz;
    a.tz_top = T.tz_top;
    a.ntx = T.ntx;
    a.ntz = T.ntz;
    a.in_pair = in_pair;
    a.out_pair = in_pair ^ 1;
    a.fields = fields;
    return a;
}

// Forward launches from level n0 to level n_end on the field pairs of `s`
// (`*pair` holds levels n0-1, n0 on entry and n_end-1, n_end on return).
// Launches end at every multiple of `cut` (if > 0) so the caller can act on
// those levels through on_cut(level, pair).  With a ring, every new level is
// also stored there.  With profiling on, one event pair brackets the run.
template <class OnCut>
sg_status forward_run(sg_plan *p, const sg::SliceDesc &s, const sg_tuning &t, int config, const sg::Tiling &T,
                      int n0, int n_end, int cut, int *pair, float *ring, int ring_lo, int64_t ring_shot,
                      OnCut on_cut, hipStream_t st, int *count = nullptr)
{
    const int step = t.variant == 1 ? 1 : t.time_block;
    // the tiled kernel leaves snapshots to launch boundaries at snapshot levels
    const bool snap_cuts = t.variant >= 2 && s.snaps != nullptr;
    const int se = s.snap_every, slast = (s.snap_count - 1) * s.snap_every;
    auto snap_due = [&](int level) { return snap_cuts && level % se == 0 && level <= slast; };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (p->profiling) {
        sg_status rc = prof_pair(p, 0, &e0, &e1);
        if (rc != SG_OK) return rc;
        SG_HIP(hipEventRecord(e0, st));
    }
    if (snap_due(n0) && n0 < n_end) SG_HIP(sg::launch_record_slot(s, n0, 2 * (*pair) + 1, st, 2));
    int launches = 0;
    for (int n = n0; n < n_end; ++launches) {
        int k = std::min(step, n_end - n);
        if (cut > 0) k = std::min(k, cut - n % cut);
        if (snap_cuts && n < slast) k = std::min(k, se - n % se);
        if (t.variant == 1) {
            SG_HIP(sg::launch_step_naive(s, n, st));
            *pair = 0;
        } else {
            sg::TileArgs a = tile_args(T, s.fields, n, k, *pair);
            a.ring = ring;
            a.ring_lo = ring_lo;
            a.ring_shot = ring_shot;
            if (T.sweep_nw > 0) {
                SG_HIP(sg::launch_sweep(s, a, T.sweep_nw, st));
            } else {
                SG_HIP(sg::launch_step_tiled(s, a, config, st));
            }
            *pair ^= 1;
        }
        n += k;
        if (n < n_end && snap_due(n)) SG_HIP(sg::launch_record_slot(s, n, 2 * (*pair) + 1, st, 2));
        if (cut > 0 && n % cut == 0) {
            sg_status rc = on_cut(n, *pair);
            if (rc != SG_OK) return rc;
        }
    }
    if (p->profiling) {
        SG_HIP(hipEventRecord(e1, st));
        p->prof_used = 1;
        p->prof_launches = launches;
    }
    if (count) *count = launches;
    return SG_OK;
}

// Frame holding level m after forward_run: the one-step kernel keeps level m
// in frame m & 1; the tiled kernel keeps the newer level in frame 1 of the pair.
int level_slot(const sg_tuning &t, int m, int pair) { return t.variant == 1 ? (m & 1) : 2 * pair + 1; }

// Runs levels 0 .. nt-1 of every shot: records each level while stepping
// from it, then records the last level.

// Shared validation and set-up of the calls on one slice.  The gradient
// calls keep two tilings: T for the adjoint (always the tiled kernel) and Tf
// for the forward and its recompute (the column sweep when the plan's tuning
// asks for it, else the same as T).
struct CallSetup {
    Layout L;
    sg_tuning t;
    int config = -1;
    sg::Tiling T{};
    sg_tuning tf;
    int config_f = -1;
    sg::Tiling Tf{};
};

sg_status setup_call(sg_plan *p, const float *vp, const sg_shots *shots, void *ws, size_t ws_bytes, int ckpt,
                     bool need_tiled, CallSetup *c)
{
    if (!p) return fail(SG_EINVAL, "plan is NULL");
    if (!vp) return fail(SG_EINVAL, "vp is NULL");
    if (!ws) return fail(SG_EINVAL, "workspace is NULL");
    sg_status rc = check_shots(p, shots);
    if (rc != SG_OK) return rc;
    c->L = layout_of(p, shots->nshot, shots->nrec, ckpt);
    if (ws_bytes < c->L.total)
        return fail(SG_ENOSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, c->L.total);
    const bool gradient = need_tiled && ckpt > 0;
    c->t = resolve_tuning(p, shots->nshot, gradient);
    const bool sweep_fwd = gradient && c->t.variant == 3;
    if (sweep_fwd) c->tf = c->t;
    if (need_tiled && (c->t.variant == 1 || c->t.variant == 3)) {   // the adjoint runs on the tiled kernel
        sg_tuning keep = p->tuning;
        p->tuning = sg_tuning{};
        c->t = resolve_tuning(p, shots->nshot, gradient);
        p->tuning = keep;
    }
    if (c->t.variant >= 2 && (rc = tiling_for(p, c->t, &c->config, &c->T)) != SG_OK) return rc;
    if (sweep_fwd) {
        if ((rc = tiling_for(p, c->tf, &c->config_f, &c->Tf)) != SG_OK) return rc;
    } else {
        c->tf = c->t;
        c->config_f = c->config;
        c->Tf = c->T;
    }
    return SG_OK;
}

// Pinned staging of the per-call device headers of batched calls (item
// tables), used in turn like a plan's table slots; a slot grows (one pinned
// allocation) when a larger batch arrives.
struct Stage {
    std::mutex mu;
    StageSlot slot[kStageSlots];
    int next = 0;
};
Stage g_stage;

sg_status stage_upload(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    std::lock_guard<std::mutex> lock(g_stage.mu);
    StageSlot &sl = g_stage.slot[g_stage.next];
    g_stage.next = (g_stage.next + 1) % kStageSlots;
    if (!sl.done) SG_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    if (sl.pending) SG_HIP(hipEventSynchronize(sl.done));
    sl.pending = false;
    if (sl.bytes < bytes) {
        if (sl.buf) SG_HIP(hipHostFree(sl.buf));
        sl.buf = nullptr;
        sl.bytes = 0;
        SG_HIP(hipHostMalloc(&sl.buf, std::max(bytes, (size_t)4096), hipHostMallocDefault));
        sl.bytes = std::max(bytes, (size_t)4096);
    }
    std::memcpy(sl.buf, src, bytes);
    SG_HIP(hipMemcpyAsync(dst, sl.buf, bytes, hipMemcpyHostToDevice, st));
    SG_HIP(hipEventRecord(sl.done, st));
    sl.pending = true;
    return SG_OK;
}

// Instantiated graphs of batched time stepping, keyed by everything their
// kernel arguments depend on.
bool g_batch_graphs = true;

struct GraphKey {
    uintptr_t ws;
    int nitems, blocks, nt, tb, config;
    uint64_t sig;
    bool operator==(const GraphKey &o) const
    {
        return ws == o.ws && nitems == o.nitems && blocks == o.blocks && nt == o.nt && tb == o.tb &&
               config == o.config && sig == o.sig;
    }
};

// FNV-1a over the device pointers and sizes the record kernels receive by value.
uint64_t items_signature(const std::vector<sg::BatchItem> &hb)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    for (const auto &b : hb) mix(&b.s, sizeof(b.s));
    return h;
}

struct GraphCache {
    std::mutex mu;
    struct Entry {
        GraphKey key;
        hipGraphExec_t exec;
        hipEvent_t done;             // recorded after each launch of exec
        int aux;                     // a count the caller keeps with the graph
    };
    std::vector<Entry> entries;      // most recent last
    hipStream_t capture = nullptr;   // private stream used only to record graphs
};
GraphCache g_graphs;
constexpr size_t kGraphCacheSize = 8;

// Launches the instantiated graph for `key` on `st`, recording it with
// `enqueue` on first use; an event recorded after the launch lets an evicted
// graph be destroyed only once its last launch has finished.  *aux
// (optional) is stored with a new graph and returned with a cached one;
// `before` (optional) is recorded on `st` just before the launch.
template <class Enqueue>
sg_status graph_run(const GraphKey &key, hipStream_t st, Enqueue enqueue, int *aux = nullptr,
                    hipEvent_t before = nullptr)
{
    std::lock_guard<std::mutex> lock(g_graphs.mu);
    auto launch = [&](GraphCache::Entry &e) -> sg_status {
        if (before) SG_HIP(hipEventRecord(before, st));
        SG_HIP(hipGraphLaunch(e.exec, st));
        SG_HIP(hipEventRecord(e.done, st));
        return SG_OK;
    };
    for (size_t i = 0; i < g_graphs.entries.size(); ++i)
        if (g_graphs.entries[i].key == key) {
            auto e = g_graphs.entries[i];
            g_graphs.entries.erase(g_graphs.entries.begin() + i);
            g_graphs.entries.push_back(e);
            if (aux) *aux = e.aux;
            return launch(g_graphs.entries.back());
        }
    // record on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured); the graph is launched on `st`
    (void)st;
    if (!g_graphs.capture) SG_HIP(hipStreamCreateWithFlags(&g_graphs.capture, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    SG_HIP(hipStreamBeginCapture(g_graphs.capture, hipStreamCaptureModeThreadLocal));
    sg_status rc = enqueue(g_graphs.capture);
    hipError_t e2 = hipStreamEndCapture(g_graphs.capture, &graph);
    if (rc != SG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e2 != hipSuccess) return fail(SG_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e2));
    hipGraphExec_t exec = nullptr;
    hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(SG_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
    hipEvent_t done = nullptr;
    hipError_t e4 = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e4 != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return fail(SG_EHIP, "hipEventCreateWithFlags failed: %s", hipGetErrorString(e4));
    }
    if (g_graphs.entries.size() >= kGraphCacheSize) {
        // the oldest graph may still run on some stream: wait for its last launch
        GraphCache::Entry &old = g_graphs.entries.front();
        (void)hipEventSynchronize(old.done);
        (void)hipGraphExecDestroy(old.exec);
        (void)hipEventDestroy(old.done);
        g_graphs.entries.erase(g_graphs.entries.begin());
    }
    g_graphs.entries.push_back({key, exec, done, aux ? *aux : 0});
    return launch(g_graphs.entries.back());
}

// FNV-1a over a slice descriptor (every pointer and size its launches take by value).
uint64_t desc_signature(const sg::SliceDesc &d)
{
    uint64_t h = 1469598103934665603ull;
    const unsigned char *c = (const unsigned char *)&d;
    for (size_t i = 0; i < sizeof(d); ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

// The whole time stepping of one call (every level, then the last level's
// records).  The sequence of launches is recorded once into a hipGraph per
// (descriptor, tiling, nt) and replayed, unless graphs are off or the caller
// is capturing the stream already; plan profiling brackets the replay.
sg_status run_forward(sg_plan *p, const sg::SliceDesc &s, const sg_tuning &t, int config,
                      const sg::Tiling &T, hipStream_t st, bool use_graph = true)
{
    const int nt = p->g.nt;
    p->prof_used = 0;
    int launches = 0;
    auto enqueue = [&](hipStream_t s2) -> sg_status {
        int pair = 0;
        sg_status rc = forward_run(p, s, t, config, T, 0, nt - 1, 0, &pair, nullptr, 0, 0,
                                   [](int, int) { return SG_OK; }, s2, &launches);
        if (rc != SG_OK) return rc;
        SG_HIP(sg::launch_record_slot(s, nt - 1, level_slot(t, nt - 1, pair), s2));
        return SG_OK;
    };
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    SG_HIP(hipStreamIsCapturing(st, &cap));
    if (cap != hipStreamCaptureStatusNone || !g_batch_graphs || !use_graph) return enqueue(st);
    const bool prof = p->profiling;
    GraphKey key{(uintptr_t)s.fields, -1, t.variant >= 2 ? T.ntx * T.ntz * s.nshot : 0, nt,
                 t.variant >= 2 ? t.time_block : 0, t.variant >= 2 ? config + 16 * T.sweep_nw : -1,
                 desc_signature(s)};
    auto record = [&](hipStream_t s2) -> sg_status {
        p->profiling = false;          // the replay is bracketed instead
        sg_status rc = enqueue(s2);
        p->profiling = prof;
        return rc;
    };
    sg_status rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof && (rc = prof_pair(p, 0, &e0, &e1)) != SG_OK) return rc;
    if ((rc = graph_run(key, st, record, &launches, e0)) != SG_OK) return rc;
    if (prof) {
        SG_HIP(hipEventRecord(e1, st));
        p->prof_used = 1;
        p->prof_launches = launches;
    }
    return SG_OK;
}

// Candidate tunings of the autotuner: every built shape with every time block
// that leaves an output tile.
std::vector<sg_tuning> tuning_candidates(const sg_plan *p)
{
    static const int tbs[] = {1, 2, 3, 4, 5, 6, 8};
    std::vector<sg_tuning> out;
    for (int c = 0; c < sg::kTiledShapes; ++c) {
        const sg::TiledShape sh = sg::tiled_shape(c);
        for (int tb : tbs) {
            const sg::Tiling T = sg::make_tiling(p->Nz, p->Nx, p->g.top == SG_TOP_FREE, sh.ex, sh.ez, sh.k, tb);
            if (!T.ok || (int64_t)T.ntx * T.ntz > max_tiles(p)) continue;
            sg_tuning t{};
            t.variant = 2;
            t.tile_x = sh.ex;
            t.tile_z = sh.ez;
            t.time_block = tb;
            t.rows_per_thread = sh.k;
            out.push_back(t);
        }
    }
    // column sweep (dz == dx): strips of 128 or 256 columns
    if (p->g.dz == p->g.dx)
        for (int nw : {2, 4})
            for (int tb = 2; tb <= sg::kSweepMaxTimeBlock; ++tb)
                for (int seg : {0, 160, 224, 320}) {
                    const sg::Tiling T = sg::make_sweep_tiling(p->Nz, p->Nx, nw, tb, seg);
                    if (!T.ok || (int64_t)T.ntx * T.ntz > max_tiles(p) || (seg > 0 && T.ntz < 2)) continue;
                    sg_tuning t{};
                    t.variant = 3;
                    t.tile_x = 64 * nw;
                    t.tile_z = seg;
                    t.time_block = tb;
                    out.push_back(t);
                }
    return out;
}

// Shots [s0, s0 + cnt) of an item as their own sg_shots.
sg_shots shots_view(const sg_shots *sh, int s0, int cnt, int nt)
{
    sg_shots v = *sh;
    v.nshot = cnt;
    v.src_zx = sh->src_zx + 2 * (size_t)s0;
    if (sh->wavelet_per_shot) v.wavelet = sh->wavelet + (size_t)s0 * nt;
    return v;
}

int wave_shots(int nshot, int per_wave) { return per_wave > 0 ? std::min(nshot, per_wave) : nshot; }

}  // namespace

namespace sg {

sg_status forward_call(sg_plan *p, const float *vp, const sg_shots *shots, float *gathers, float *snaps, void *ws,
                       size_t ws_bytes, void *stream, bool no_alloc)
{
    CallSetup c;
    sg_status rc = setup_call(p, vp, shots, ws, ws_bytes, 0, false, &c);
    if (rc != SG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    if ((rc = upload_tables(p, c.L, w, shots, c.t.variant >= 2 ? &c.T : nullptr, st, !no_alloc)) != SG_OK)
        return rc;
    const sg::SliceDesc s = describe(p, c.L, w, shots, gathers, snaps);
    SG_HIP(sg::launch_prepare(s, vp, (float)(p->g.dt * p->g.dt), st));
    SG_HIP(sg::launch_zero(s.fields, (size_t)shots->nshot * sg::kFramesPerShot * p->frame, st));
    // recording and instantiating a graph allocates: without allocation the
    // launches are enqueued directly
    return run_forward(p, s, c.t, c.config, c.T, st, !no_alloc);
}

sg_status report_error(sg_status st, const char *msg) { return fail(st, "%s", msg); }

}  // namespace sg

extern "C" {

int32_t sg_abi_version(void) { return SG_ABI_VERSION; }

const char *sg_status_string(sg_status s)
{
    switch (s) {
    case SG_OK: return "SG_OK";
    case SG_EINVAL: return "SG_EINVAL";
    case SG_ECFL: return "SG_ECFL";
    case SG_ENOSPACE: return "SG_ENOSPACE";
    case SG_EHIP: return "SG_EHIP";
    case SG_EDIVERGED: return "SG_EDIVERGED";
    case SG_EUNSUPPORTED: return "SG_EUNSUPPORTED";
    default: return "SG_UNKNOWN";
    }
}

const char *sg_last_error(void) { return g_last_error.c_str(); }

double sg_cfl_dt_max(double dz, double dx, double vmax)
{
    return cfl_smax() * std::min(dz, dx) / vmax;
}

sg_status sg_plan_create(const sg_geometry *g, uint32_t flags, sg_plan **out)
{
    if (!out) return fail(SG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(SG_EINVAL, "geometry is NULL");
    if (g->nz < 1 || g->nx < 1) return fail(SG_EINVAL, "nz, nx must be >= 1 (got %d, %d)", g->nz, g->nx);
    if (!(g->dz > 0 && g->dx > 0 && g->dt > 0) || !std::isfinite(g->dz) || !std::isfinite(g->dx) ||
        !std::isfinite(g->dt))
        return fail(SG_EINVAL, "dz, dx, dt must be finite and > 0");
    if (g->nt < 2) return fail(SG_EINVAL, "nt must be >= 2 (got %d)", g->nt);
    if (g->nbl < 0) return fail(SG_EINVAL, "nbl must be >= 0");
    if (g->top != SG_TOP_FREE && g->top != SG_TOP_ABSORBING) return fail(SG_EINVAL, "bad top mode %d", g->top);
    if (g->nbl > 0 && !(g->damp_R > 0 && g->damp_R < 1)) return fail(SG_EINVAL, "damp_R must be in (0, 1)");
    if (!(g->vmax_hint > 0) || !std::isfinite(g->vmax_hint)) return fail(SG_EINVAL, "vmax_hint must be > 0");
    if (g->rec_every < 1) return fail(SG_EINVAL, "rec_every must be >= 1");
    if (g->snap_count < 0) return fail(SG_EINVAL, "snap_count must be >= 0");
    if (g->snap_count > 0) {
        if (g->snap_every < 1) return fail(SG_EINVAL, "snap_every must be >= 1");
        if ((int64_t)(g->snap_count - 1) * g->snap_every > g->nt - 1)
            return fail(SG_EINVAL, "snapshots reach beyond level nt-1");
    }
    const double dtmax = sg_cfl_dt_max(g->dz, g->dx, g->vmax_hint);
    if (g->dt > dtmax && !(flags & SG_ALLOW_UNSTABLE))
        return fail(SG_ECFL, "dt = %g s exceeds the CFL bound %g s at vmax = %g m/s", g->dt, dtmax,
                    g->vmax_hint);
    const int ztop = g->top == SG_TOP_FREE ? 0 : g->nbl;
    const int64_t Nz = (int64_t)g->nz + ztop + g->nbl, Nx = (int64_t)g->nx + 2 * g->nbl;
    const int64_t pitch = (int64_t)align_up((size_t)(Nx + 2 * sg::kGuard), 32);
    const int64_t frame = (Nz + 2 * sg::kGuard) * pitch;
    // in-field addressing uses 32-bit byte offsets, 8 bytes per cell in the
    // FP64 imaging accumulator
    if (frame > ((int64_t)1 << 29))
        return fail(SG_EINVAL, "grid too large (%lld x %lld padded; a stored field holds at most 2^29 cells)",
                    (long long)Nz, (long long)Nx);
    sg_plan *p = new (std::nothrow) sg_plan();
    if (!p) return fail(SG_EINVAL, "out of host memory");
    p->g = *g;
    if (p->g.snap_count == 0) p->g.snap_every = 0;
    p->Nz = (int32_t)Nz;
    p->Nx = (int32_t)Nx;
    p->ztop = ztop;
    p->xleft = g->nbl;
    p->pitch = (int32_t)pitch;
    p->frame = frame;
    p->nrow = (g->nt + g->rec_every - 1) / g->rec_every;
    p->warnings = 0;
    if (g->vmin_hint > 0 && g->fmax_hint > 0 && std::max(g->dz, g->dx) > g->vmin_hint / (4.0 * g->fmax_hint))
        p->warnings |= SG_WARN_DISPERSION;
    // gamma = eta v^2 dt / 2 = (eta / (2 dt)) * (v dt)^2; corners add the sides
    p->gx.assign(Nx, 0.f);
    p->gz.assign(Nz, 0.f);
    for (int Ix = 0; Ix < Nx; ++Ix) {
        const int dl = p->xleft - Ix, dr = Ix - (p->xleft + g->nx - 1);
        const double eta = sponge_eta(dl, g->nbl, g->dx, g->damp_R) + sponge_eta(dr, g->nbl, g->dx, g->damp_R);
        p->gx[Ix] = (float)(eta / (2.0 * g->dt));
    }
    for (int Iz = 0; Iz < Nz; ++Iz) {
        const int db = Iz - (ztop + g->nz - 1), dtp = ztop - Iz;
        const double eta = sponge_eta(db, g->nbl, g->dz, g->damp_R) + sponge_eta(dtp, g->nbl, g->dz, g->damp_R);
        p->gz[Iz] = (float)(eta / (2.0 * g->dt));
    }
    // pinned staging for the forward tables of up to 64 shots and two
    // receivers per column, where a device is present (without one the
    // plan is still usable for host-only calls; a later call grows it)
    if (hipHostMalloc(&p->stage[0].buf, 1, hipHostMallocDefault) == hipSuccess) {
        (void)hipHostFree(p->stage[0].buf);
        p->stage[0].buf = nullptr;
        std::lock_guard<std::mutex> lock(p->mu);
        (void)reserve_stage(p, table_bytes(p, 64, 2 * g->nx, 0));
    }
    (void)hipGetLastError();
    *out = p;
    return SG_OK;
}

sg_status sg_plan_reserve(sg_plan *p, int32_t nshot, int32_t nrec, int32_t ckpt_every)
{
    if (!p) return fail(SG_EINVAL, "plan is NULL");
    if (nshot < 1 || nrec < 0 || ckpt_every < 0)
        return fail(SG_EINVAL, "nshot must be >= 1, nrec >= 0, ckpt_every >= 0");
    const int ckpt = ckpt_every > 0 ? ckpt_spacing(p, ckpt_every) : 0;
    std::lock_guard<std::mutex> lock(p->mu);
    return reserve_stage(p, table_bytes(p, nshot, nrec, ckpt));
}

sg_status sg_plan_destroy(sg_plan *p)
{
    if (!p) return SG_OK;
    for (StageSlot &sl : p->stage) {
        if (sl.done) {
            if (sl.pending) (void)hipEventSynchronize(sl.done);
            (void)hipEventDestroy(sl.done);
        }
        if (sl.buf) (void)hipHostFree(sl.buf);
    }
    for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
    if (p->side) {
        (void)hipStreamSynchronize(p->side);
        (void)hipStreamDestroy(p->side);
    }
    for (hipEvent_t e : {p->ev_seg, p->ev_fold[0], p->ev_fold[1]})
        if (e) (void)hipEventDestroy(e);
    delete p;
    return SG_OK;
}

uint32_t sg_plan_warnings(const sg_plan *p) { return p ? p->warnings : 0u; }

sg_status sg_plan_set_profiling(sg_plan *p, int32_t on)
{
    if (!p) return fail(SG_EINVAL, "plan is NULL");
    p->profiling = on != 0;
    return SG_OK;
}

sg_status sg_plan_profile(sg_plan *p, double *kernel_ms, int32_t *launches)
{
    if (!p || !kernel_ms || !launches) return fail(SG_EINVAL, "NULL argument");
    double total = 0.0;
    if (p->prof_used > 0) SG_HIP(hipEventSynchronize(p->prof_ev[2 * p->prof_used - 1]));
    for (int i = 0; i < p->prof_used; ++i) {
        float ms = 0.f;
        SG_HIP(hipEventElapsedTime(&ms, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]));
        total += ms;
    }
    *kernel_ms = total;
    *launches = p->prof_launches;
    return SG_OK;
}

sg_status sg_plan_padded_shape(const sg_plan *p, int32_t *Nz, int32_t *Nx)
{
    if (!p || !Nz || !Nx) return fail(SG_EINVAL, "NULL argument");
    *Nz = p->Nz;
    *Nx = p->Nx;
    return SG_OK;
}

sg_status sg_plan_set_tuning(sg_plan *p, const sg_tuning *t)
{
    if (!p) return fail(SG_EINVAL, "plan is NULL");
    if (!t) {
        p->tuning = sg_tuning{};
        return SG_OK;
    }
    if (t->variant < 0 || t->variant > 3) return fail(SG_EINVAL, "variant must be 0, 1, 2 or 3");
    if (t->variant == 3) {
        if (t->tile_x != 0 && t->tile_x != 128 && t->tile_x != 256)
            return fail(SG_EUNSUPPORTED, "sweep strips are 128 or 256 columns");
        if ((t->tile_z != 0 && t->tile_z < 8) || t->rows_per_thread != 0)
            return fail(SG_EINVAL, "sweep tunings take tile_z = 0 or >= 8 (segment rows) and rows_per_thread = 0");
        if (t->time_block < 0 || t->time_block > sg::kSweepMaxTimeBlock)
            return fail(SG_EINVAL, "sweep time_block must be in 0..%d", sg::kSweepMaxTimeBlock);
        p->tuning = *t;
        return SG_OK;
    }
    if (t->time_block < 0 || t->time_block > sg::kMaxTimeBlock)
        return fail(SG_EINVAL, "time_block must be in 0..%d", sg::kMaxTimeBlock);
    if (t->tile_x < 0 || t->tile_z < 0) return fail(SG_EINVAL, "tile sizes must be >= 0");
    if (t->rows_per_thread < 0) return fail(SG_EINVAL, "rows_per_thread must be >= 0");
    if (t->variant != 1 && (t->tile_x || t->tile_z) && shape_of(*t) < 0)
        return fail(SG_EUNSUPPORTED, "no kernel built for a %d x %d tile with %d rows per thread", t->tile_x,
                    t->tile_z, t->rows_per_thread);
    p->tuning = *t;
    return SG_OK;
}

sg_status sg_plan_get_tuning(const sg_plan *p, int32_t nshot, sg_tuning *t)
{
    if (!p || !t) return fail(SG_EINVAL, "NULL argument");
    *t = resolve_tuning(p, nshot);
    return SG_OK;
}

sg_status sg_ricker(double f0, double dt, int32_t nt, double t0, float *out)
{
    if (!out || nt < 0 || !(f0 > 0) || !(dt > 0)) return fail(SG_EINVAL, "bad Ricker arguments");
    if (t0 <= 0) t0 = 1.0 / f0;
    for (int n = 0; n < nt; ++n) {
        const double tau = n * dt - t0;
        const double q = kPi * kPi * f0 * f0 * tau * tau;
        out[n] = (float)((1.0 - 2.0 * q) * std::exp(-q));
    }
    return SG_OK;
}

namespace {

// One second-order section y = (b0 + b1 z^-1 + b2 z^-2) / (1 + a1 z^-1 + a2 z^-2) x
// in transposed direct form II with state (s0, s1).
struct Biquad {
    double b0, b1, b2, a1, a2;
};

// State of a section at rest under a constant unit input: the fixed point
// s = A s + B of the transposed direct form, i.e. (I - A) s = B with
// A = [[-a1, 1], [-a2, 0]] and B = (b1 - a1 b0, b2 - a2 b0).
void biquad_rest_state(const Biquad &q, double s[2])
{
    const double r0 = q.b1 - q.a1 * q.b0, r1 = q.b2 - q.a2 * q.b0;
    // [[1 + a1, -1], [a2, 1]] s = r
    const double det = (1.0 + q.a1) + q.a2;
    s[0] = (r0 + r1) / det;
    s[1] = r1 - q.a2 * s[0];
}

// Runs the cascade over x[0..n) in place, starting every section from the
// state it holds at rest under the constant input `level` (zero-phase
// filtering starts both passes this way, so the edges see no step).
void run_cascade(const std::vector<Biquad> &secs, double level, std::vector<double> &x)
{
    std::vector<double> st(2 * secs.size());
    double scale = level;
    for (size_t i = 0; i < secs.size(); ++i) {
        biquad_rest_state(secs[i], &st[2 * i]);
        st[2 * i] *= scale;
        st[2 * i + 1] *= scale;
        const Biquad &q = secs[i];
        scale *= (q.b0 + q.b1 + q.b2) / (1.0 + q.a1 + q.a2);   // DC gain of the section
    }
    for (double &v : x) {
        double u = v;
        for (size_t i = 0; i < secs.size(); ++i) {
            const Biquad &q = secs[i];
            double &s0 = st[2 * i], &s1 = st[2 * i + 1];
            const double y = q.b0 * u + s0;
            s0 = q.b1 * u - q.a1 * y + s1;
            s1 = q.b2 * u - q.a2 * y;
            u = y;
        }
        v = u;
    }
}

}  // namespace

sg_status sg_bandpass_ricker(double f0, double fmin, double fmax, double dt, int32_t nt, double bandwidth_ref,
                             float *out)
{
    if (!out || nt < 2 || !(f0 > 0) || !(dt > 0) || !(fmin > 0) || !(fmax > fmin) || !(fmax < 0.5 / dt) ||
        !(bandwidth_ref > 0))
        return fail(SG_EINVAL, "bad band-pass wavelet arguments");
    // 4th-order Butterworth band-pass by the bilinear transform with
    // pre-warped corners (normalised to the Nyquist frequency, design rate 2)
    constexpr int N = 4;
    const double w1 = 4.0 * std::tan(kPi * (2.0 * fmin * dt) / 2.0);
    const double w2 = 4.0 * std::tan(kPi * (2.0 * fmax * dt) / 2.0);
    const double bw = w2 - w1, wo2 = w1 * w2;
    using cd = std::complex<double>;
    std::vector<cd> poles;
    for (int m = -N + 1; m < N; m += 2) {
        const cd p = -std::exp(cd(0.0, kPi * m / (2.0 * N)));   // analog low-pass prototype
        const cd pl = p * (bw / 2.0);
        const cd r = std::sqrt(pl * pl - wo2);
        poles.push_back(pl + r);                                 // low-pass -> band-pass
        poles.push_back(pl - r);
    }
    // bilinear map s -> z = (4 + s) / (4 - s); the N analog zeros at 0 map to
    // z = 1, the N at infinity to z = -1; gain k = bw^N prod(4 - 0) / prod(4 - p)
    cd gain = std::pow(bw, N) * std::pow(4.0, N);
    std::vector<cd> zp;
    for (const cd &p : poles) {
        gain /= (4.0 - p);
        zp.push_back((4.0 + p) / (4.0 - p));
    }
    // sections: one conjugate pole pair each (upper half plane members) with
    // one zero at +1 and one at -1; the gain goes to the first section
    std::vector<Biquad> secs;
    for (const cd &p : zp) {
        if (p.imag() <= 0.0) continue;
        Biquad q{1.0, 0.0, -1.0, -2.0 * p.real(), std::norm(p)};
        secs.push_back(q);
    }
    if ((int)secs.size() != N) return fail(SG_EINVAL, "band too narrow or too wide for the filter design");
    secs[0].b0 *= gain.real();
    secs[0].b2 *= gain.real();
    // zero-phase filtering of the Ricker pulse: odd extension of 3 (2 sections + 1)
    // samples at each end, forward pass from rest at the first sample, backward
    // pass from rest at the last output, extension removed
    const int pad = 3 * (2 * N + 1);
    if (nt <= pad) return fail(SG_EINVAL, "nt must exceed %d samples for the band-pass filter", pad);
    std::vector<double> w(nt);
    const double t0 = 1.0 / f0;
    for (int n = 0; n < nt; ++n) {
        const double tau = n * dt - t0;
        const double q = kPi * kPi * f0 * f0 * tau * tau;
        w[n] = (1.0 - 2.0 * q) * std::exp(-q);
    }
    std::vector<double> x(nt + 2 * pad);
    for (int i = 0; i < pad; ++i) {
        x[i] = 2.0 * w[0] - w[pad - i];
        x[pad + nt + i] = 2.0 * w[nt - 1] - w[nt - 2 - i];
    }
    for (int n = 0; n < nt; ++n) x[pad + n] = w[n];
    run_cascade(secs, x.front(), x);
    std::reverse(x.begin(), x.end());
    run_cascade(secs, x.front(), x);
    std::reverse(x.begin(), x.end());
    double norm = 0.0;
    for (int n = 0; n < nt; ++n) norm += x[pad + n] * x[pad + n];
    norm = std::sqrt(norm);
    if (!(norm > 0)) return fail(SG_EINVAL, "the band-passed pulse is zero");
    const double scale = std::sqrt((fmax - fmin) / bandwidth_ref) / norm;
    for (int n = 0; n < nt; ++n) out[n] = (float)(x[pad + n] * scale);
    return SG_OK;
}

sg_status sg_forward_workspace_size(const sg_plan *p, int32_t nshot, int32_t nrec, size_t *bytes)
{
    if (!p || !bytes) return fail(SG_EINVAL, "NULL argument");
    if (nshot < 1 || nrec < 0) return fail(SG_EINVAL, "nshot must be >= 1 and nrec >= 0");
    *bytes = layout_of(p, nshot, nrec).total;
    return SG_OK;
}

sg_status sg_forward(sg_plan *p, const float *vp, const sg_shots *shots, float *gathers,
                     float *snaps, void *ws, size_t ws_bytes, void *stream)
{
    return sg::forward_call(p, vp, shots, gathers, snaps, ws, ws_bytes, stream, false);
}

sg_status sg_check_finite(const float *x, size_t n, void *ws, size_t ws_bytes, void *stream)
{
    if (!x || !ws) return fail(SG_EINVAL, "NULL argument");
    if (ws_bytes < sizeof(unsigned int)) return fail(SG_ENOSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    unsigned int *cnt = (unsigned int *)ws;
    SG_HIP(sg::launch_zero((float *)cnt, 1, st));
    SG_HIP(sg::launch_count_nonfinite(x, n, cnt, st));
    unsigned int h = 0;
    SG_HIP(hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, st));
    SG_HIP(hipStreamSynchronize(st));
    if (h) return fail(SG_EDIVERGED, "%u non-finite values", h);
    return SG_OK;
}

sg_status sg_grad_workspace_size(const sg_plan *p, int32_t nshot, int32_t nrec, int32_t ckpt_every,
                                 size_t *bytes)
{
    if (!p || !bytes) return fail(SG_EINVAL, "NULL argument");
    if (nshot < 1 || nrec < 0) return fail(SG_EINVAL, "nshot must be >= 1 and nrec >= 0");
    *bytes = layout_of(p, nshot, nrec, ckpt_spacing(p, ckpt_every)).total;
    return SG_OK;
}

sg_status sg_forward_ckpt(sg_plan *p, const float *vp, const sg_shots *shots, int32_t ckpt_every,
                          float *gathers, void *ws, size_t ws_bytes, void *stream)
{
    if (!p) return fail(SG_EINVAL, "plan is NULL");
    const int C = ckpt_spacing(p, ckpt_every);
    CallSetup c;
    sg_status rc = setup_call(p, vp, shots, ws, ws_bytes, C, true, &c);
    if (rc != SG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    if ((rc = upload_tables(p, c.L, w, shots, &c.Tf, st)) != SG_OK) return rc;
    sg::SliceDesc s = describe(p, c.L, w, shots, gathers, nullptr);
    s.snaps = nullptr;
    SG_HIP(sg::launch_prepare(s, vp, (float)(p->g.dt * p->g.dt), st));
    const int nshot = shots->nshot, nt = p->g.nt;
    SG_HIP(sg::launch_zero(s.fields, (size_t)nshot * sg::kFramesPerShot * p->frame, st));
    float *ck = (float *)(w + c.L.ckpt);
    const int64_t ck_shot = (int64_t)c.L.nseg * 2 * p->frame;
    // checkpoint 0 holds levels -1 and 0, both zero
    SG_HIP(sg::launch_copy(ck, ck_shot, s.fields, (int64_t)sg::kFramesPerShot * p->frame, 2 * p->frame, nshot, st));
    int pair = 0;
    p->prof_used = 0;
    auto on_cut = [&](int level, int pr) -> sg_status {
        const int j = level / C;
        if (j >= c.L.nseg) return SG_OK;
        // levels level-1, level are frames 2 pr, 2 pr + 1 of the pair
        SG_HIP(sg::launch_copy(ck + (int64_t)j * 2 * p->frame, ck_shot, s.fields + (int64_t)(2 * pr) * p->frame,
                               (int64_t)sg::kFramesPerShot * p->frame, 2 * p->frame, nshot, st));
        return SG_OK;
    };
    rc = forward_run(p, s, c.tf, c.config_f, c.Tf, 0, nt - 1, C, &pair, nullptr, 0, 0, on_cut, st);
    if (rc != SG_OK) return rc;
    SG_HIP(sg::launch_record_slot(s, nt - 1, level_slot(c.tf, nt - 1, pair), st));
    return SG_OK;
}

sg_status sg_adjoint_gradient(sg_plan *p, const float *vp, const sg_shots *shots, int32_t ckpt_every,
                              const float *resid, float *grad, void *ws, size_t ws_bytes, void *stream)
{
    if (!p) return fail(SG_EINVAL, "plan is NULL");
    if (!resid || !grad) return fail(SG_EINVAL, "resid and grad must not be NULL");
    const int C = ckpt_spacing(p, ckpt_every);
    CallSetup c;
    sg_status rc = setup_call(p, vp, shots, ws, ws_bytes, C, true, &c);
    if (rc != SG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    if ((rc = upload_tables(p, c.L, w, shots, &c.T, st)) != SG_OK) return rc;
    sg::SliceDesc s = describe(p, c.L, w, shots, nullptr, nullptr);
    SG_HIP(sg::launch_prepare(s, vp, (float)(p->g.dt * p->g.dt), st));
    const int nshot = shots->nshot, nt = p->g.nt;
    const int64_t F = p->frame, fshot = (int64_t)sg::kFramesPerShot * F;
    float *ck = (float *)(w + c.L.ckpt), *rings[2] = {(float *)(w + c.L.ring), (float *)(w + c.L.ring2)};
    float *mu = (float *)(w + c.L.mu);
    double *hsum = (double *)(w + c.L.hsum);
    const int64_t ck_shot = (int64_t)c.L.nseg * 2 * F, ring_shot = (int64_t)c.L.ring_levels * F;
    SG_HIP(sg::launch_zero(mu, (size_t)nshot * fshot, st));
    SG_HIP(sg::launch_zero((float *)hsum, (size_t)nshot * 2 * F, st));

    sg::InjTables inj{};
    inj.tile_start = (const int32_t *)(w + c.L.inj_tile);
    inj.lds = (const int32_t *)(w + c.L.inj_lds);
    inj.iz = (const int32_t *)(w + c.L.inj_iz);
    inj.ix = (const int32_t *)(w + c.L.inj_ix);
    inj.pstart = (const int32_t *)(w + c.L.inj_pstart);
    inj.rid = (const int32_t *)(w + c.L.inj_rid);
    inj.w = (const float *)(w + c.L.inj_w);

    if ((rc = side_stream(p)) != SG_OK) return rc;
    bool folding[2] = {false, false};
    int mpair = 0;   // adjoint pair: frame 0 = mu^{k+2}, frame 1 = mu^{k+1}
    p->prof_used = 0;
    for (int j = c.L.nseg - 1; j >= 0; --j) {
        const int lo = j * C, hi = std::min((j + 1) * C - 1, nt - 1), last = std::min(hi + 1, nt - 1);
        // this segment's ring; the fold of the segment that used it last must be done
        float *ring = rings[j & 1];
        if (folding[j & 1]) SG_HIP(hipStreamWaitEvent(st, p->ev_fold[j & 1], 0));
        // recompute levels lo+1 .. last from checkpoint j (levels lo-1, lo),
        // storing D^lo .. D^{last-1} in the ring
        const float *ckj = ck + (int64_t)j * 2 * F;
        SG_HIP(sg::launch_copy(s.fields, fshot, ckj, ck_shot, 2 * F, nshot, st));
        int pair = 0;
        if (last > lo) {
            rc = forward_run(p, s, c.tf, c.config_f, c.Tf, lo, last, 0, &pair, ring, lo, ring_shot,
                             [](int, int) { return SG_OK; }, st);
            if (rc != SG_OK) return rc;
        }
        // adjoint steps k = hi .. lo (mu^k from mu^{k+1}, mu^{k+2}) with imaging;
        // each launch leaves its partial sums in the ring slot of its first level
        int nlaunch = 0;
        for (int k0 = hi; k0 >= lo;) {
            ++nlaunch;
            const int nsteps = std::min(c.t.time_block, k0 - lo + 1);
            sg::TileArgs a = tile_args(c.T, mu, k0, nsteps, mpair);
            a.ring = ring;
            a.ring_lo = lo;
            a.ring_hi = last - 1;
            a.ring_shot = ring_shot;
            a.resid = resid;
            a.hsum = hsum;
            a.nt = nt;
            a.inj = inj;
            SG_HIP(sg::launch_adjoint_tiled(s, a, c.config, st));
            mpair ^= 1;
            k0 -= nsteps;
        }
        // the fold runs on the side stream (in segment order) while the next
        // segment recomputes into the other ring
        SG_HIP(hipEventRecord(p->ev_seg, st));
        SG_HIP(hipStreamWaitEvent(p->side, p->ev_seg, 0));
        SG_HIP(sg::launch_fold_partials(s, hsum, ring, ring_shot, hi - lo, c.t.time_block, nlaunch, p->side));
        SG_HIP(hipEventRecord(p->ev_fold[j & 1], p->side));
        folding[j & 1] = true;
    }
    // every fold is done (they run in order on the side stream)
    SG_HIP(hipStreamWaitEvent(st, p->ev_fold[0], 0));
    SG_HIP(sg::launch_fold_gradient(s, vp, hsum, F, (float)p->g.dt, grad, st));
    return SG_OK;
}

sg_status sg_batch_workspace_size(const sg_batch_item *items, int32_t nitems, size_t *bytes)
{
    if (!items || !bytes || nitems < 1) return fail(SG_EINVAL, "bad batch arguments");
    size_t total = 0;
    for (int i = 0; i < nitems; ++i) {
        if (!items[i].plan || !items[i].shots) return fail(SG_EINVAL, "batch item %d has no plan or shots", i);
        total += align_up(layout_of(items[i].plan, items[i].shots->nshot, items[i].shots->nrec).total, 256);
    }
    total += align_up((size_t)nitems * sizeof(sg::BatchItem), 256);
    *bytes = total;
    return SG_OK;
}

namespace {

// The batched forward over the first `levels` levels.  A trial (autotuning)
// records nothing and replays no graph.
sg_status batch_forward_impl(const sg_batch_item *items, int32_t nitems, const sg_tuning *tuning, void *ws,
                             size_t ws_bytes, void *stream, int levels, bool trial)
{
    size_t need = 0;
    sg_status rc = sg_batch_workspace_size(items, nitems, &need);
    if (rc != SG_OK) return rc;
    if (!ws) return fail(SG_EINVAL, "workspace is NULL");
    if (ws_bytes < need) return fail(SG_ENOSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    const int nt = items[0].plan->g.nt;
    for (int i = 1; i < nitems; ++i)
        if (items[i].plan->g.nt != nt) return fail(SG_EINVAL, "batch items must share nt (%d vs %d)", items[i].plan->g.nt, nt);
    sg_tuning t = tuning ? *tuning : resolve_tuning(items[0].plan, items[0].shots->nshot);
    if (t.variant == 0) t = resolve_tuning(items[0].plan, items[0].shots->nshot);
    if (t.variant != 2 && t.variant != 3)
        return fail(SG_EUNSUPPORTED, "batched launches use the tiled (2) or column-sweep (3) kernel");
    if (t.time_block <= 0) t.time_block = 4;
    if (t.variant == 3 && t.tile_x == 0) t.tile_x = 256;
    // validate everything before enqueueing anything
    std::vector<CallSetup> cs(nitems);
    std::vector<size_t> base(nitems);
    size_t o = 0;
    int64_t total_blocks = 0;
    for (int i = 0; i < nitems; ++i) {
        const sg_batch_item &it = items[i];
        base[i] = o;
        o += align_up(layout_of(it.plan, it.shots->nshot, it.shots->nrec).total, 256);
        if (!it.vp) return fail(SG_EINVAL, "batch item %d: vp is NULL", i);
        if ((rc = check_shots(it.plan, it.shots)) != SG_OK) return rc;
        cs[i].L = layout_of(it.plan, it.shots->nshot, it.shots->nrec);
        cs[i].t = t;
        if ((rc = tiling_for(it.plan, t, &cs[i].config, &cs[i].T)) != SG_OK) return rc;
        total_blocks += (int64_t)cs[i].T.ntx * cs[i].T.ntz * it.shots->nshot;
    }
    if (total_blocks >= ((int64_t)1 << 31)) return fail(SG_EINVAL, "batch too large");
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    std::vector<sg::BatchItem> hb(nitems);
    int32_t start = 0;
    for (int i = 0; i < nitems; ++i) {
        const sg_batch_item &it = items[i];
        char *wi = w + base[i];
        if ((rc = upload_tables(it.plan, cs[i].L, wi, it.shots, &cs[i].T, st)) != SG_OK) return rc;
        hb[i].s = describe(it.plan, cs[i].L, wi, it.shots, trial ? nullptr : it.gathers, trial ? nullptr : it.snaps);
        SG_HIP(sg::launch_prepare(hb[i].s, it.vp, (float)(it.plan->g.dt * it.plan->g.dt), st));
        SG_HIP(sg::launch_zero(hb[i].s.fields, (size_t)it.shots->nshot * sg::kFramesPerShot * it.plan->frame, st));
        hb[i].t = tile_args(cs[i].T, hb[i].s.fields, 0, 0, 0);
        hb[i].block_start = start;
        start += cs[i].T.ntx * cs[i].T.ntz * it.shots->nshot;
    }
    sg::BatchItem *dev_items = (sg::BatchItem *)(w + o);
    if ((rc = stage_upload(dev_items, hb.data(), hb.size() * sizeof(sg::BatchItem), st)) != SG_OK) return rc;

    // the time-stepping launches (one per time block over the whole batch),
    // replayed from a captured graph unless the caller is capturing already
    const int config = cs[0].config, tb = t.time_block, sweep_nw = cs[0].T.sweep_nw;
    // the isotropic kernel form needs dz == dx on every item
    bool iso = true;
    for (int i = 0; i < nitems; ++i)
        for (int m = 1; m <= sg::kHalo; ++m) iso = iso && hb[i].s.cz[m] == hb[i].s.cx[m];
    // snapshots are copied at launch boundaries: launches are cut at every
    // snapshot level of any item
    auto snap_due = [&](int i, int level) {
        const sg::SliceDesc &d = hb[i].s;
        return d.snaps && level % d.snap_every == 0 && level / d.snap_every < d.snap_count;
    };
    auto next_cut = [&](int n) {   // smallest snapshot level > n of any item, or INT_MAX
        int best = INT32_MAX;
        for (int i = 0; i < nitems; ++i) {
            const sg::SliceDesc &d = hb[i].s;
            if (!d.snaps) continue;
            const int L = (n / d.snap_every + 1) * d.snap_every;
            if (L / d.snap_every < d.snap_count) best = std::min(best, L);
        }
        return best;
    };
    auto enqueue = [&](hipStream_t s2) -> sg_status {
        int pair = 0;
        for (int i = 0; i < nitems; ++i)
            if (snap_due(i, 0)) SG_HIP(sg::launch_record_slot(hb[i].s, 0, 1, s2, 2));
        const int nlast = std::min(levels, nt) - 1;
        for (int n = 0; n < nlast;) {
            const int k = std::min(std::min(tb, nlast - n), next_cut(n) - n);
            if (sweep_nw > 0)
                SG_HIP(sg::launch_sweep_batch(dev_items, nitems, (int)total_blocks, n, k, pair, sweep_nw, s2));
            else
                SG_HIP(sg::launch_step_tiled_batch(dev_items, nitems, (int)total_blocks, n, k, pair, config, iso, s2));
            pair ^= 1;
            n += k;
            if (n < nlast)
                for (int i = 0; i < nitems; ++i)
                    if (snap_due(i, n)) SG_HIP(sg::launch_record_slot(hb[i].s, n, 2 * pair + 1, s2, 2));
        }
        if (!trial)
            for (int i = 0; i < nitems; ++i)
                SG_HIP(sg::launch_record_slot(hb[i].s, nt - 1, 2 * pair + 1, s2));
        return SG_OK;
    };
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    SG_HIP(hipStreamIsCapturing(st, &cap));
    if (trial || cap != hipStreamCaptureStatusNone || !g_batch_graphs) return enqueue(st);
    // per-item launch arguments never change for the same workspace and batch
    // shape, so one instantiated graph per such key is replayed
    GraphKey key{(uintptr_t)ws, nitems, (int)total_blocks, nt, tb, config + 16 * sweep_nw, items_signature(hb)};
    return graph_run(key, st, enqueue);
}

}  // namespace

sg_status sg_batch_forward(const sg_batch_item *items, int32_t nitems, const sg_tuning *tuning, void *ws,
                           size_t ws_bytes, void *stream)
{
    if (!items || nitems < 1) return fail(SG_EINVAL, "bad batch arguments");
    return batch_forward_impl(items, nitems, tuning, ws, ws_bytes, stream, items[0].plan ? items[0].plan->g.nt : 0,
                              false);
}

sg_status sg_batch_autotune(const sg_batch_item *items, int32_t nitems, int32_t trial_levels, void *ws,
                            size_t ws_bytes, void *stream, sg_tuning *best)
{
    if (!items || nitems < 1 || !best) return fail(SG_EINVAL, "bad batch arguments");
    if (trial_levels < 8) return fail(SG_EINVAL, "trial_levels must be >= 8");
    for (int i = 0; i < nitems; ++i)
        if (!items[i].plan || !items[i].shots) return fail(SG_EINVAL, "batch item %d has no plan or shots", i);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    SG_HIP(hipEventCreate(&e0));
    SG_HIP(hipEventCreate(&e1));
    sg_status rc = SG_OK;
    double best_ms = 1e300;
    sg_tuning chosen{};
    for (const sg_tuning &t : tuning_candidates(items[0].plan)) {
        // a candidate must tile every item of the batch
        bool fits = true;
        for (int i = 0; i < nitems && fits; ++i) {
            int config = -1;
            sg::Tiling T{};
            fits = tiling_for(items[i].plan, t, &config, &T) == SG_OK;
        }
        if (!fits) continue;
        // one untimed pass to warm caches and code, then the timed pass
        for (int rep = 0; rep < 2 && rc == SG_OK; ++rep) {
            if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = fail(SG_EHIP, "event record failed");
            if (rc == SG_OK) rc = batch_forward_impl(items, nitems, &t, ws, ws_bytes, stream, trial_levels, true);
            if (rep == 1 && rc == SG_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(SG_EHIP, "event record failed");
        }
        if (rc != SG_OK) break;
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(SG_EHIP, "event timing failed");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            chosen = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SG_OK) return rc;
    if (best_ms == 1e300) return fail(SG_EUNSUPPORTED, "no tiling fits every item of the batch");
    *best = chosen;
    return SG_OK;
}

sg_status sg_autotune(sg_plan *p, const float *vp, const sg_shots *shots, int32_t trial_levels, void *ws,
                      size_t ws_bytes, void *stream, sg_tuning *best)
{
    if (!p || !best) return fail(SG_EINVAL, "NULL argument");
    if (trial_levels < 8) return fail(SG_EINVAL, "trial_levels must be >= 8");
    const sg_tuning keep = p->tuning;
    sg_tuning probe{};
    probe.variant = 2;
    p->tuning = probe;
    CallSetup c;
    sg_status rc = setup_call(p, vp, shots, ws, ws_bytes, 0, true, &c);
    p->tuning = keep;
    if (rc != SG_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    hipEvent_t e0, e1;
    SG_HIP(hipEventCreate(&e0));
    SG_HIP(hipEventCreate(&e1));
    const int levels = std::min(trial_levels, p->g.nt - 1);
    double best_ms = 1e300;
    sg_tuning chosen{};
    for (const sg_tuning &t : tuning_candidates(p)) {
        int config = -1;
        sg::Tiling T{};
        if (tiling_for(p, t, &config, &T) != SG_OK) continue;
        if ((rc = upload_tables(p, c.L, w, shots, &T, st)) != SG_OK) break;
        // a trial: no outputs recorded, fields zeroed, the same levels for every candidate
        sg::SliceDesc s = describe(p, c.L, w, shots, nullptr, nullptr);
        if (hipSuccess != sg::launch_prepare(s, vp, (float)(p->g.dt * p->g.dt), st) ||
            hipSuccess != sg::launch_zero(s.fields, (size_t)shots->nshot * sg::kFramesPerShot * p->frame, st)) {
            rc = fail(SG_EHIP, "autotune set-up launch failed");
            break;
        }
        int pair = 0;
        const bool prof = p->profiling;
        p->profiling = false;
        // one untimed pass to warm caches and code, then the timed pass
        for (int rep = 0; rep < 2 && rc == SG_OK; ++rep) {
            if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = fail(SG_EHIP, "event record failed");
            if (rc == SG_OK)
                rc = forward_run(p, s, t, config, T, 0, levels, 0, &pair, nullptr, 0, 0,
                                 [](int, int) { return SG_OK; }, st);
            if (rep == 1 && rc == SG_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(SG_EHIP, "event record failed");
        }
        p->profiling = prof;
        if (rc != SG_OK) break;
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(SG_EHIP, "event timing failed");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            chosen = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SG_OK) return rc;
    if (best_ms == 1e300) return fail(SG_EUNSUPPORTED, "no tiling fits this grid");
    p->tuning = chosen;
    *best = chosen;
    return SG_OK;
}


sg_status sg_batch_grad_workspace_size(const sg_batch_grad_item *items, int32_t nitems, int32_t ckpt_every,
                                       int32_t shots_per_wave, size_t *bytes)
{
    if (!items || !bytes || nitems < 1) return fail(SG_EINVAL, "bad batch arguments");
    size_t total = 0;
    for (int i = 0; i < nitems; ++i) {
        if (!items[i].plan || !items[i].shots) return fail(SG_EINVAL, "batch item %d has no plan or shots", i);
        const int S = wave_shots(items[i].shots->nshot, shots_per_wave);
        if (S < 1) return fail(SG_EINVAL, "batch item %d has no shots", i);
        total += align_up(layout_of(items[i].plan, S, items[i].shots->nrec,
                                    ckpt_spacing(items[i].plan, ckpt_every)).total, 256);
    }
    total += 4 * align_up((size_t)nitems * sizeof(sg::BatchItem), 256);   // forward / adjoint x two rings
    *bytes = total;
    return SG_OK;
}

sg_status sg_batch_adjoint_gradient(const sg_batch_grad_item *items, int32_t nitems, int32_t ckpt_every,
                                    int32_t shots_per_wave, const sg_tuning *tuning, void *ws, size_t ws_bytes,
                                    void *stream)
{
    size_t need = 0;
    sg_status rc = sg_batch_grad_workspace_size(items, nitems, ckpt_every, shots_per_wave, &need);
    if (rc != SG_OK) return rc;
    if (!ws) return fail(SG_EINVAL, "workspace is NULL");
    if (ws_bytes < need) return fail(SG_ENOSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    const int nt = items[0].plan->g.nt;
    const int C = ckpt_spacing(items[0].plan, ckpt_every);
    for (int i = 0; i < nitems; ++i) {
        if (items[i].plan->g.nt != nt) return fail(SG_EINVAL, "batch items must share nt");
        if (!items[i].vp || !items[i].resid || !items[i].grad) return fail(SG_EINVAL, "batch item %d: NULL pointer", i);
        if ((rc = check_shots(items[i].plan, items[i].shots)) != SG_OK) return rc;
    }
    sg_tuning t = tuning ? *tuning : resolve_tuning(items[0].plan, items[0].shots->nshot, true);
    // a column-sweep tuning runs the forward and its recompute; the adjoint
    // always runs the tiled kernel (with the default tiling unless a tiled
    // tuning is given)
    sg_tuning tf = t;
    const bool sweep_fwd = t.variant == 3;
    if (sweep_fwd) {
        if (tf.tile_x == 0) tf.tile_x = 256;
        if (tf.time_block <= 0) tf.time_block = 4;
    }
    if (t.variant != 2) {
        sg_plan *p0 = items[0].plan;
        sg_tuning keep = p0->tuning;
        p0->tuning = sg_tuning{};
        t = resolve_tuning(p0, items[0].shots->nshot, true);
        p0->tuning = keep;
    }
    if (!sweep_fwd) tf = t;
    std::vector<sg::Tiling> T(nitems), Tf(nitems);
    int config = -1, config_f = -1;
    for (int i = 0; i < nitems; ++i) {
        if ((rc = tiling_for(items[i].plan, t, &config, &T[i])) != SG_OK) return rc;
        if ((rc = tiling_for(items[i].plan, tf, &config_f, &Tf[i])) != SG_OK) return rc;
    }
    bool iso = true;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    int nwave = 0;
    for (int i = 0; i < nitems; ++i) {
        const int S = wave_shots(items[i].shots->nshot, shots_per_wave);
        nwave = std::max(nwave, (items[i].shots->nshot + S - 1) / S);
    }
    for (int wv = 0; wv < nwave; ++wv) {
        // the items that still have shots in this wave, and their set-up
        std::vector<int> act;
        std::vector<sg_shots> views;
        std::vector<Layout> Ls;
        std::vector<sg::BatchItem> hb, hb_adj;
        size_t o = 0;
        int32_t start = 0, start_adj = 0;
        views.reserve(nitems);
        for (int i = 0; i < nitems; ++i) {
            const sg_batch_grad_item &it = items[i];
            const int S = wave_shots(it.shots->nshot, shots_per_wave);
            const int s0 = wv * S, cnt = std::min(S, it.shots->nshot - s0);
            const size_t region = align_up(layout_of(it.plan, S, it.shots->nrec, C).total, 256);
            if (cnt <= 0) {
                o += region;
                continue;
            }
            act.push_back(i);
            views.push_back(shots_view(it.shots, s0, cnt, nt));
            const sg_shots *sv = &views.back();
            const Layout L = layout_of(it.plan, cnt, it.shots->nrec, C);
            Ls.push_back(L);
            char *wi = w + o;
            o += region;
            if ((rc = upload_tables(it.plan, L, wi, sv, &T[i], st)) != SG_OK) return rc;
            sg::BatchItem b{};
            b.s = describe(it.plan, L, wi, sv, nullptr, nullptr);
            for (int m = 1; m <= sg::kHalo; ++m) iso = iso && b.s.cz[m] == b.s.cx[m];
            SG_HIP(sg::launch_prepare(b.s, it.vp, (float)(it.plan->g.dt * it.plan->g.dt), st));
            const int64_t F = it.plan->frame;
            SG_HIP(sg::launch_zero(b.s.fields, (size_t)cnt * sg::kFramesPerShot * F, st));
            SG_HIP(sg::launch_zero((float *)(wi + L.mu), (size_t)cnt * sg::kFramesPerShot * F, st));
            SG_HIP(sg::launch_zero((float *)(wi + L.hsum), (size_t)cnt * 2 * F, st));
            b.t = tile_args(Tf[i], b.s.fields, 0, 0, 0);
            b.t.ring = (float *)(wi + L.ring);
            b.t.ring_shot = (int64_t)L.ring_levels * F;
            b.t.resid = it.resid + (size_t)s0 * it.plan->nrow * it.shots->nrec;
            b.t.hsum = (double *)(wi + L.hsum);
            b.t.nt = nt;
            b.t.inj.tile_start = (const int32_t *)(wi + L.inj_tile);
            b.t.inj.lds = (const int32_t *)(wi + L.inj_lds);
            b.t.inj.iz = (const int32_t *)(wi + L.inj_iz);
            b.t.inj.ix = (const int32_t *)(wi + L.inj_ix);
            b.t.inj.pstart = (const int32_t *)(wi + L.inj_pstart);
            b.t.inj.rid = (const int32_t *)(wi + L.inj_rid);
            b.t.inj.w = (const float *)(wi + L.inj_w);
            b.block_start = start;
            start += Tf[i].ntx * Tf[i].ntz * cnt;
            hb.push_back(b);
            // the adjoint's entry: its tiling, fields in the adjoint pair
            sg::BatchItem ba = b;
            const sg::TileArgs keep_t = b.t;
            ba.t = tile_args(T[i], (float *)(wi + L.mu), 0, 0, 0);
            ba.t.ring = keep_t.ring;
            ba.t.ring_shot = keep_t.ring_shot;
            ba.t.resid = keep_t.resid;
            ba.t.hsum = keep_t.hsum;
            ba.t.nt = keep_t.nt;
            ba.t.inj = keep_t.inj;
            ba.block_start = start_adj;
            start_adj += T[i].ntx * T[i].ntz * cnt;
            hb_adj.push_back(ba);
            // checkpoint 0: levels -1 and 0, both zero
            SG_HIP(sg::launch_copy((float *)(wi + L.ckpt), (int64_t)L.nseg * 2 * F, b.s.fields,
                                   (int64_t)sg::kFramesPerShot * F, 2 * F, cnt, st));
        }
        const int na = (int)act.size();
        // two device copies of the item table (forward fields, adjoint fields),
        // both uploaded once per wave in one copy
        // four device copies of the item table: forward and adjoint fields,
        // each with the first and with the second ring (segments alternate),
        // uploaded once per wave in one copy
        const size_t tbl = align_up((size_t)nitems * sizeof(sg::BatchItem), 256);
        sg::BatchItem *dev_fwd_r[2], *dev_adj_r[2];
        dev_fwd_r[0] = (sg::BatchItem *)(w + need - 4 * tbl);
        dev_adj_r[0] = (sg::BatchItem *)(w + need - 3 * tbl);
        dev_fwd_r[1] = (sg::BatchItem *)(w + need - 2 * tbl);
        dev_adj_r[1] = (sg::BatchItem *)(w + need - tbl);
        std::vector<sg::BatchItem> hb2 = hb, hb_adj2 = hb_adj;
        for (int q = 0; q < na; ++q) {
            float *r2 = (float *)((char *)hb[q].t.ring - Ls[q].ring + Ls[q].ring2);
            hb2[q].t.ring = r2;
            hb_adj2[q].t.ring = r2;
        }
        {
            std::vector<char> all(4 * tbl, 0);
            std::memcpy(all.data(), hb.data(), hb.size() * sizeof(sg::BatchItem));
            std::memcpy(all.data() + tbl, hb_adj.data(), hb_adj.size() * sizeof(sg::BatchItem));
            std::memcpy(all.data() + 2 * tbl, hb2.data(), hb2.size() * sizeof(sg::BatchItem));
            std::memcpy(all.data() + 3 * tbl, hb_adj2.data(), hb_adj2.size() * sizeof(sg::BatchItem));
            if ((rc = stage_upload(dev_fwd_r[0], all.data(), 4 * tbl, st)) != SG_OK) return rc;
        }
        sg::BatchItem *const dev_fwd = dev_fwd_r[0];
        auto copy_items = [&](auto dst_of, auto src_of, int64_t n) -> sg_status {
            for (int q = 0; q < na; ++q) {
                const int64_t F = items[act[q]].plan->frame;
                float *dst;
                int64_t dshot;
                const float *src;
                int64_t sshot;
                dst_of(q, F, &dst, &dshot);
                src_of(q, F, &src, &sshot);
                SG_HIP(sg::launch_copy(dst, dshot, src, sshot, n * F, views[q].nshot, st));
            }
            return SG_OK;
        };
        // forward with checkpoints (no outputs)
        int pair = 0;
        for (int n = 0; n < nt - 1;) {
            const int k = std::min(std::min(tf.time_block, nt - 1 - n), C - n % C);
            if (sweep_fwd)
                SG_HIP(sg::launch_sweep_batch(dev_fwd, na, start, n, k, pair, Tf[0].sweep_nw, st));
            else
                SG_HIP(sg::launch_step_tiled_batch(dev_fwd, na, start, n, k, pair, config, iso, st));
            pair ^= 1;
            n += k;
            if (n % C == 0 && n / C < Ls[0].nseg) {
                const int j = n / C, pr = pair;
                rc = copy_items(
                    [&](int q, int64_t F, float **d, int64_t *ds) {
                        *d = (float *)((char *)hb[q].s.fields - Ls[q].fields + Ls[q].ckpt) + (int64_t)j * 2 * F;
                        *ds = (int64_t)Ls[q].nseg * 2 * F;
                    },
                    [&](int q, int64_t F, const float **sp, int64_t *ss) {
                        *sp = hb[q].s.fields + (int64_t)(2 * pr) * F;
                        *ss = (int64_t)sg::kFramesPerShot * F;
                    },
                    2);
                if (rc != SG_OK) return rc;
            }
        }
        // segments backwards: recompute into the segment's ring, then the
        // adjoint; its partial sums are folded on the side stream while the
        // next segment runs on the other ring
        sg_plan *p0 = items[act[0]].plan;
        if ((rc = side_stream(p0)) != SG_OK) return rc;
        bool folding[2] = {false, false};
        int mpair = 0;
        const int nseg = Ls[0].nseg;
        for (int j = nseg - 1; j >= 0; --j) {
            const int lo = j * C, hi = std::min((j + 1) * C - 1, nt - 1), last = std::min(hi + 1, nt - 1);
            const int rb = j & 1;
            if (folding[rb]) SG_HIP(hipStreamWaitEvent(st, p0->ev_fold[rb], 0));
            rc = copy_items(
                [&](int q, int64_t F, float **d, int64_t *ds) {
                    *d = hb[q].s.fields;
                    *ds = (int64_t)sg::kFramesPerShot * F;
                },
                [&](int q, int64_t F, const float **sp, int64_t *ss) {
                    *sp = (const float *)((char *)hb[q].s.fields - Ls[q].fields + Ls[q].ckpt) + (int64_t)j * 2 * F;
                    *ss = (int64_t)Ls[q].nseg * 2 * F;
                },
                2);
            if (rc != SG_OK) return rc;
            int fp = 0;
            for (int n = lo; n < last;) {
                const int k = std::min(tf.time_block, last - n);
                if (sweep_fwd)
                    SG_HIP(sg::launch_sweep_batch(dev_fwd_r[rb], na, start, n, k, fp, Tf[0].sweep_nw, st, true, lo));
                else
                    SG_HIP(sg::launch_ring_tiled_batch(dev_fwd_r[rb], na, start, n, k, fp, config, iso, lo, st));
                fp ^= 1;
                n += k;
            }
            int nlaunch = 0;
            for (int k0 = hi; k0 >= lo;) {
                ++nlaunch;
                const int ns = std::min(t.time_block, k0 - lo + 1);
                SG_HIP(sg::launch_adjoint_tiled_batch(dev_adj_r[rb], na, start_adj, k0, ns, mpair, config, iso, lo,
                                                      last - 1, st));
                mpair ^= 1;
                k0 -= ns;
            }
            SG_HIP(hipEventRecord(p0->ev_seg, st));
            SG_HIP(hipStreamWaitEvent(p0->side, p0->ev_seg, 0));
            for (int q = 0; q < na; ++q) {
                const sg::BatchItem &ba = rb ? hb_adj2[q] : hb_adj[q];
                SG_HIP(sg::launch_fold_partials(ba.s, ba.t.hsum, ba.t.ring, ba.t.ring_shot, hi - lo, t.time_block,
                                                nlaunch, p0->side));
            }
            SG_HIP(hipEventRecord(p0->ev_fold[rb], p0->side));
            folding[rb] = true;
        }
        // every fold of this wave is done (in order on the side stream)
        SG_HIP(hipStreamWaitEvent(st, p0->ev_fold[0], 0));
        for (int q = 0; q < na; ++q) {
            const sg_batch_grad_item &it = items[act[q]];
            SG_HIP(sg::launch_fold_gradient(hb[q].s, it.vp, hb[q].t.hsum, it.plan->frame,
                                            (float)it.plan->g.dt, it.grad, st, wv > 0));
        }
    }
    return SG_OK;
}

namespace {
sg_status residual_args(int32_t nframes, int32_t nz, int32_t nx, int32_t top, int *z0, size_t *bytes)
{
    if (nframes < 1 || nz < 1 || nx < 1) return fail(SG_EINVAL, "nframes, nz and nx must be >= 1");
    if (nframes > 65537) return fail(SG_EINVAL, "at most 65537 frames per call");
    if ((int64_t)nz * nx >= ((int64_t)1 << 30)) return fail(SG_EINVAL, "frame of %d x %d cells is too large", nz, nx);
    if (top != SG_TOP_FREE && top != SG_TOP_ABSORBING) return fail(SG_EINVAL, "top must be SG_TOP_FREE or SG_TOP_ABSORBING");
    *z0 = top == SG_TOP_FREE ? 1 : 4;
    const int nb = sg::wave_residual_slots(nz, nx, *z0);
    *bytes = align_up((size_t)std::max(nframes - 2, 0) * nb * 2 * sizeof(double), 256);
    if (*bytes == 0) *bytes = 256;
    return SG_OK;
}
}  // namespace

sg_status sg_wave_residual_workspace_size(int32_t nframes, int32_t nz, int32_t nx, int32_t top, size_t *bytes)
{
    if (!bytes) return fail(SG_EINVAL, "NULL argument");
    int z0 = 0;
    return residual_args(nframes, nz, nx, top, &z0, bytes);
}

sg_status sg_wave_residual(const float *frames, int32_t nframes, int32_t nz, int32_t nx, const float *vp, double dz,
                           double dx, double dt, int32_t top, double *res2, double *dtt2, void *ws, size_t ws_bytes,
                           void *stream)
{
    if (!frames || !vp || !res2 || !dtt2 || !ws) return fail(SG_EINVAL, "NULL argument");
    if (!(dz > 0) || !(dx > 0) || !(dt > 0) || !std::isfinite(dz) || !std::isfinite(dx) || !std::isfinite(dt))
        return fail(SG_EINVAL, "dz, dx and dt must be finite and > 0");
    int z0 = 0;
    size_t need = 0;
    sg_status rc = residual_args(nframes, nz, nx, top, &z0, &need);
    if (rc != SG_OK) return rc;
    if (ws_bytes < need) return fail(SG_ENOSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    sg::ResidualCoef cf{};
    for (int m = 0; m <= sg::kHalo; ++m) {
        cf.cz[m] = (float)(kC8[m] / (dz * dz));
        cf.cx[m] = (float)(kC8[m] / (dx * dx));
    }
    SG_HIP(sg::launch_wave_residual(frames, nframes, nz, nx, vp, dt, cf, z0, (double *)ws, res2, dtt2,
                                    (hipStream_t)stream));
    return SG_OK;
}

namespace {
bool positive_finite(double x) { return std::isfinite(x) && x > 0; }
sg_status volume_args(const void *v, int32_t nz, int32_t ny, int32_t nx, const void *out)
{
    if (!v || !out) return fail(SG_EINVAL, "NULL argument");
    if (nz < 1 || ny < 1 || nx < 1) return fail(SG_EINVAL, "nz, ny and nx must be >= 1");
    if ((int64_t)nz * ny * nx >= ((int64_t)1 << 40)) return fail(SG_EINVAL, "volume too large");
    if (v == out) return fail(SG_EINVAL, "out must not alias the input volume (pull sampling reads neighbours)");
    return SG_OK;
}
}  // namespace

sg_status sg_fractal_noise2d(const float *lattice, int32_t noct, int32_t gy, int32_t gx, int32_t ny, int32_t nx,
                             double dy, double dx, double lam_y, double lam_x, double azimuth_deg, double amplitude,
                             float *out, void *stream)
{
    if (!lattice || !out) return fail(SG_EINVAL, "NULL argument");
    if (noct < 1 || noct > 24) return fail(SG_EINVAL, "noct must be in 1..24");
    if (gy < 1 || gx < 1 || ny < 1 || nx < 1) return fail(SG_EINVAL, "lattice and grid sizes must be >= 1");
    if ((int64_t)ny * nx >= ((int64_t)1 << 40)) return fail(SG_EINVAL, "grid too large");
    if (!positive_finite(dy) || !positive_finite(dx) || !positive_finite(lam_y) || !positive_finite(lam_x))
        return fail(SG_EINVAL, "spacings and wavelengths must be finite and > 0");
    if (!std::isfinite(azimuth_deg) || !std::isfinite(amplitude))
        return fail(SG_EINVAL, "azimuth and amplitude must be finite");
    SG_HIP(sg::launch_fractal_noise2d(lattice, noct, gy, gx, ny, nx, dy, dx, lam_y, lam_x, azimuth_deg * kPi / 180.0,
                                      amplitude, out, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_deposit(int32_t t, int32_t ny, int32_t nx, double dz, double dy, double dx, int32_t nbeds,
                     const float *thick, const float *vbed, double beta, const float *eta_b, double a_B,
                     const float *tex_lattice, int32_t gz, int32_t gy, int32_t gx, double lam_z, double lam_y,
                     double lam_x, const float *tex_off, double a_eta, double f_top, double f_base, float *out,
                     void *stream)
{
    if (!thick || !vbed || !tex_lattice || !tex_off || !out || (nbeds > 1 && !eta_b))
        return fail(SG_EINVAL, "NULL argument");
    if (t < 1 || ny < 1 || nx < 1 || nbeds < 1 || gz < 1 || gy < 1 || gx < 1)
        return fail(SG_EINVAL, "sizes must be >= 1");
    if (nbeds > sg::kDepositMaxBeds) return fail(SG_EINVAL, "at most %d beds per band", sg::kDepositMaxBeds);
    if ((int64_t)t * ny * nx >= ((int64_t)1 << 40)) return fail(SG_EINVAL, "band too large");
    if (!positive_finite(dz) || !positive_finite(dy) || !positive_finite(dx) || !positive_finite(lam_z) ||
        !positive_finite(lam_y) || !positive_finite(lam_x) || !positive_finite(f_top) || !positive_finite(f_base))
        return fail(SG_EINVAL, "spacings, noise wavelengths and taper fractions must be finite and > 0");
    if (!std::isfinite(beta) || !std::isfinite(a_B) || !std::isfinite(a_eta))
        return fail(SG_EINVAL, "beta, a_B and a_eta must be finite");
    sg::DepositArgs A{};
    A.t = t;
    A.ny = ny;
    A.nx = nx;
    A.nbeds = nbeds;
    A.gz = gz;
    A.gy = gy;
    A.gx = gx;
    A.dz = dz;
    A.dy = dy;
    A.dx = dx;
    A.inv_lam_z = 1.0 / lam_z;
    A.inv_lam_y = 1.0 / lam_y;
    A.inv_lam_x = 1.0 / lam_x;
    A.beta = beta;
    A.a_B = a_B;
    A.a_eta = a_eta;
    A.f_top = f_top;
    A.f_base = f_base;
    A.thick = thick;
    A.vbed = vbed;
    A.tex_off = tex_off;
    A.eta_b = eta_b;
    A.lattice = tex_lattice;
    SG_HIP(sg::launch_deposit(A, out, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_deposit_simplex(int32_t t, int32_t ny, int32_t nx, double dz, double dy, double dx, int32_t nbeds,
                             const float *thick, const float *vbed, double beta, const int32_t *perm_b,
                             double lam_bz, double lam_by, double lam_bx, double a_B, const int32_t *perm_t,
                             double lam_tz, double lam_ty, double lam_tx, const float *tex_off, double a_eta,
                             double f_top, double f_base, float *out, void *stream)
{
    if (!thick || !vbed || !perm_b || !perm_t || !tex_off || !out) return fail(SG_EINVAL, "NULL argument");
    if (t < 1 || ny < 1 || nx < 1 || nbeds < 1) return fail(SG_EINVAL, "sizes must be >= 1");
    if (nbeds > sg::kDepositMaxBeds) return fail(SG_EINVAL, "at most %d beds per band", sg::kDepositMaxBeds);
    if ((int64_t)t * ny * nx >= ((int64_t)1 << 40)) return fail(SG_EINVAL, "band too large");
    for (double v : {dz, dy, dx, lam_bz, lam_by, lam_bx, lam_tz, lam_ty, lam_tx, f_top, f_base})
        if (!positive_finite(v))
            return fail(SG_EINVAL, "spacings, noise wavelengths and taper fractions must be finite and > 0");
    if (!std::isfinite(beta) || !std::isfinite(a_B) || !std::isfinite(a_eta))
        return fail(SG_EINVAL, "beta, a_B and a_eta must be finite");
    sg::DepositArgs A{};
    A.t = t;
    A.ny = ny;
    A.nx = nx;
    A.nbeds = nbeds;
    A.dz = dz;
    A.dy = dy;
    A.dx = dx;
    A.beta = beta;
    A.a_B = a_B;
    A.a_eta = a_eta;
    A.f_top = f_top;
    A.f_base = f_base;
    A.thick = thick;
    A.vbed = vbed;
    A.tex_off = tex_off;
    A.simplex = 1;
    A.perm_b = perm_b;
    A.perm_t = perm_t;
    A.lam_b[0] = lam_bz;
    A.lam_b[1] = lam_by;
    A.lam_b[2] = lam_bx;
    A.lam_t[0] = lam_tz;
    A.lam_t[1] = lam_ty;
    A.lam_t[2] = lam_tx;
    SG_HIP(sg::launch_deposit(A, out, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_deposit_sinusoidal(int32_t t, int32_t ny, int32_t nx, double dz, double dy, double dx, double v0,
                                double beta, const float *freq, double sigma, double amp1, double amp2,
                                double phase2, const float *rug, double a_r, const int32_t *perm_t, double lam_tz,
                                double lam_ty, double lam_tx, double a_eta, double f_top, double f_base, float *out,
                                void *stream)
{
    if (!freq || !perm_t || !out || (a_r != 0.0 && !rug)) return fail(SG_EINVAL, "NULL argument");
    if (t < 1 || ny < 1 || nx < 1) return fail(SG_EINVAL, "sizes must be >= 1");
    if (t > sg::kDepositSinMaxT) return fail(SG_EINVAL, "at most %d cells per band", sg::kDepositSinMaxT);
    if ((int64_t)t * ny * nx >= ((int64_t)1 << 40)) return fail(SG_EINVAL, "band too large");
    for (double v : {dz, dy, dx, lam_tz, lam_ty, lam_tx, f_top, f_base})
        if (!positive_finite(v))
            return fail(SG_EINVAL, "spacings, noise wavelengths and taper fractions must be finite and > 0");
    if (!(sigma >= 0.0 && sigma <= sg::kDepositSinMaxSigma))
        return fail(SG_EINVAL, "sigma must be in [0, %g] cells", sg::kDepositSinMaxSigma);
    for (double v : {v0, beta, amp1, amp2, phase2, a_r, a_eta})
        if (!std::isfinite(v)) return fail(SG_EINVAL, "v0, beta, amplitudes, phase and a_r must be finite");
    sg::DepositSinArgs A{};
    A.t = t;
    A.ny = ny;
    A.nx = nx;
    A.dz = dz;
    A.dy = dy;
    A.dx = dx;
    A.v0 = v0;
    A.beta = beta;
    A.sigma = sigma;
    A.amp1 = amp1;
    A.amp2 = amp2;
    A.phase2 = phase2;
    A.a_r = a_r;
    A.a_eta = a_eta;
    A.f_top = f_top;
    A.f_base = f_base;
    A.lam_t[0] = lam_tz;
    A.lam_t[1] = lam_ty;
    A.lam_t[2] = lam_tx;
    A.freq = freq;
    A.rug = a_r != 0.0 ? rug : nullptr;
    A.perm_t = perm_t;
    SG_HIP(sg::launch_deposit_sinusoidal(A, out, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_simplex_noise3d(const int32_t *perm, int32_t nz, int32_t ny, int32_t nx, double oz, double oy, double ox,
                             double sz, double sy, double sx, double amplitude, float *out, void *stream)
{
    if (!perm || !out) return fail(SG_EINVAL, "NULL argument");
    if (nz < 1 || ny < 1 || nx < 1) return fail(SG_EINVAL, "sizes must be >= 1");
    if ((int64_t)nz * ny * nx >= ((int64_t)1 << 40)) return fail(SG_EINVAL, "volume too large");
    for (double v : {oz, oy, ox, sz, sy, sx, amplitude})
        if (!std::isfinite(v)) return fail(SG_EINVAL, "origin, steps and amplitude must be finite");
    // lattice coordinates stay within +-2^40 (integer cell indices exact)
    const double lim = 1099511627776.0;
    for (auto [o, st, n] : {std::tuple<double, double, int>{oz, sz, nz}, {oy, sy, ny}, {ox, sx, nx}})
        if (std::fabs(o) + std::fabs(st) * (n - 1) >= lim) return fail(SG_EINVAL, "coordinates beyond 2^40 cells");
    const double o[3] = {oz, oy, ox}, st[3] = {sz, sy, sx};
    SG_HIP(sg::launch_simplex3d(perm, nz, ny, nx, o, st, amplitude, out, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_squish(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, const float *shift, float *out,
                    void *stream)
{
    sg_status rc = volume_args(v, nz, ny, nx, out);
    if (rc != SG_OK) return rc;
    if (!shift) return fail(SG_EINVAL, "NULL argument");
    if (!positive_finite(dz)) return fail(SG_EINVAL, "dz must be finite and > 0");
    SG_HIP(sg::launch_squish(v, nz, ny, nx, dz, shift, out, (hipStream_t)stream));
    return SG_OK;
}

namespace {
// Validates the fault parameters and spacings and builds the device frame.
sg_status fault_frame(const sg_fault_params *p, double dz, double dy, double dx, sg::FaultFrame &F, hipStream_t st)
{
    if (!p) return fail(SG_EINVAL, "NULL argument");
    if (!positive_finite(dz) || !positive_finite(dy) || !positive_finite(dx))
        return fail(SG_EINVAL, "dz, dy and dx must be finite and > 0");
    if (!std::isfinite(p->cz) || !std::isfinite(p->cy) || !std::isfinite(p->cx) || !std::isfinite(p->azimuth_deg) ||
        !std::isfinite(p->dip_deg) || !std::isfinite(p->slip))
        return fail(SG_EINVAL, "fault centre, azimuth, dip and slip must be finite");
    if (!positive_finite(p->radius) || !positive_finite(p->die_r) || !positive_finite(p->die_strike) ||
        !positive_finite(p->die_theta_deg))
        return fail(SG_EINVAL, "radius and die-off extents must be finite and > 0");
    if (p->direction != 1 && p->direction != -1) return fail(SG_EINVAL, "direction must be +1 or -1");
    const double a = p->azimuth_deg * kPi / 180.0, th = p->dip_deg * kPi / 180.0, R = p->radius;
    F = sg::FaultFrame{};
    F.dz = dz;
    F.dy = dy;
    F.dx = dx;
    F.inv_dz = 1.0 / dz;
    F.inv_dy = 1.0 / dy;
    F.inv_dx = 1.0 / dx;
    F.n_y = std::sin(a);    // horizontal offset of the axis from the centre
    F.n_x = std::cos(a);
    F.s_y = std::cos(a);    // strike, along the axis
    F.s_x = -std::sin(a);
    const double dlt_z = R * std::sin(th), dlt_az = R * std::cos(th);
    F.cz = p->cz - dlt_z;
    F.cy = p->cy - dlt_az * F.n_y;
    F.cx = p->cx - dlt_az * F.n_x;
    F.radius = R;
    F.theta0 = std::atan2(dlt_z, dlt_az);
    F.shift = p->slip / R;  // s / (2 pi R) of a full turn, in radians
    F.direction = p->direction;
    F.inv_die_r = 1.0 / p->die_r;
    F.inv_die_t = 1.0 / (p->die_theta_deg * kPi / 180.0);
    F.inv_die_s = 1.0 / p->die_strike;
    if (p->rough_lattice) {
        if (p->rough_noct < 1 || p->rough_noct > 24) return fail(SG_EINVAL, "rough_noct must be in 1..24");
        if (p->rough_gd < 1 || p->rough_gs < 1) return fail(SG_EINVAL, "rough lattice sizes must be >= 1");
        if (!std::isfinite(p->rough_amplitude)) return fail(SG_EINVAL, "rough_amplitude must be finite");
        if (!positive_finite(p->rough_lam_strike) || !positive_finite(p->rough_lam_dip))
            return fail(SG_EINVAL, "rough wavelengths must be finite and > 0");
        double norm = 0.0, f = 1.0;
        for (int o = 0; o < p->rough_noct; ++o, f *= 2.0) norm += 1.0 / f;
        F.rough = p->rough_lattice;
        F.rough_noct = p->rough_noct;
        F.rough_gd = p->rough_gd;
        F.rough_gs = p->rough_gs;
        F.rough_amp = p->rough_amplitude;
        F.rough_inv_norm = 1.0 / norm;
        F.inv_lam_s = 1.0 / p->rough_lam_strike;
        F.inv_lam_d = 1.0 / p->rough_lam_dip;
        // the noise never exceeds the lattice's largest |value|: read it once
        // (stream-ordered after the caller's work, then synchronised) to bound
        // the region a rough fault can move
        const size_t nl = (size_t)p->rough_noct * p->rough_gd * p->rough_gs;
        if (nl > ((size_t)1 << 26)) return fail(SG_EINVAL, "rough lattice larger than 2^26 values");
        std::vector<float> lat(nl);
        SG_HIP(hipMemcpyAsync(lat.data(), p->rough_lattice, nl * sizeof(float), hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
        double amax = 0.0;
        for (float x : lat) {
            if (!std::isfinite(x)) return fail(SG_EINVAL, "rough lattice holds a non-finite value");
            amax = std::max(amax, (double)std::fabs(x));
        }
        F.rough_reach = p->die_r + std::fabs(p->rough_amplitude) * amax;
    }
    return SG_OK;
}
}  // namespace

sg_status sg_fault(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                   const sg_fault_params *p, float fill, float *out, void *stream)
{
    sg_status rc = volume_args(v, nz, ny, nx, out);
    if (rc != SG_OK) return rc;
    sg::FaultFrame F;
    if ((rc = fault_frame(p, dz, dy, dx, F, (hipStream_t)stream)) != SG_OK) return rc;
    SG_HIP(sg::launch_fault(v, nz, ny, nx, F, fill, out, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_fault_labels(const int32_t *labels, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                          const sg_fault_params *p, int32_t fill, int32_t *out, void *stream)
{
    sg_status rc = volume_args(labels, nz, ny, nx, out);
    if (rc != SG_OK) return rc;
    sg::FaultFrame F;
    if ((rc = fault_frame(p, dz, dy, dx, F, (hipStream_t)stream)) != SG_OK) return rc;
    SG_HIP(sg::launch_fault_labels(labels, nz, ny, nx, F, fill, out, (hipStream_t)stream));
    return SG_OK;
}

extern "C++" {
namespace {
bool overlap(const void *a, const void *b, size_t bytes)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

template <typename T, typename Launch>
sg_status fault_sequence_call(const T *v, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                              const sg_fault_params *faults, int32_t nfaults, T *out, T *ws, hipStream_t st,
                              Launch launch)
{
    sg_status rc = volume_args(v, nz, ny, nx, out);
    if (rc != SG_OK) return rc;
    if (nfaults < 0 || nfaults > 100000) return fail(SG_EINVAL, "nfaults must be in 0..100000");
    if (nfaults > 0 && !faults) return fail(SG_EINVAL, "NULL argument");
    if (nfaults > 1 && !ws) return fail(SG_EINVAL, "ws is required for two or more faults");
    const size_t bytes = (size_t)nz * ny * nx * sizeof(T);
    if (overlap(v, out, bytes) || (nfaults > 1 && (overlap(v, ws, bytes) || overlap(out, ws, bytes))))
        return fail(SG_EINVAL, "v, out and ws must not overlap");
    std::vector<sg::FaultFrame> F((size_t)nfaults);
    for (int32_t k = 0; k < nfaults; ++k)
        if ((rc = fault_frame(&faults[k], dz, dy, dx, F[(size_t)k], st)) != SG_OK) return rc;
    SG_HIP(launch(F.data()));
    return SG_OK;
}
}  // namespace
}  // extern "C++"

sg_status sg_fault_sequence(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                            const sg_fault_params *faults, int32_t nfaults, float fill, float *out, float *ws,
                            void *stream)
{
    const hipStream_t st = (hipStream_t)stream;
    return fault_sequence_call(v, nz, ny, nx, dz, dy, dx, faults, nfaults, out, ws, st,
                               [&](const sg::FaultFrame *F) {
                                   return sg::launch_fault_sequence(v, nz, ny, nx, F, nfaults, fill, out, ws, st);
                               });
}

sg_status sg_fault_labels_sequence(const int32_t *labels, int32_t nz, int32_t ny, int32_t nx, double dz, double dy,
                                   double dx, const sg_fault_params *faults, int32_t nfaults, int32_t fill,
                                   int32_t *out, int32_t *ws, void *stream)
{
    const hipStream_t st = (hipStream_t)stream;
    return fault_sequence_call(labels, nz, ny, nx, dz, dy, dx, faults, nfaults, out, ws, st,
                               [&](const sg::FaultFrame *F) {
                                   return sg::launch_fault_labels_sequence(labels, nz, ny, nx, F, nfaults, fill, out,
                                                                           ws, st);
                               });
}

sg_status sg_riedel_subsidiaries(const sg_fault_params *primary, const sg_riedel_config *cfg, int32_t ncand,
                                 const double *uniforms, sg_fault_params *out, int32_t *nout)
{
    if (!primary || !cfg || !nout || (ncand > 0 && (!uniforms || !out))) return fail(SG_EINVAL, "NULL argument");
    if (ncand < 0 || ncand > 1000000) return fail(SG_EINVAL, "ncand must be in 0..1000000");
    const sg_riedel_config &c = *cfg;
    if (!(c.synthetic_fraction >= 0.0 && c.synthetic_fraction <= 1.0) ||
        !(c.hangingwall_fraction >= 0.0 && c.hangingwall_fraction <= 1.0))
        return fail(SG_EINVAL, "fractions must be in [0, 1]");
    for (double x : {c.synthetic_offset_deg, c.antithetic_offset_deg})
        if (!std::isfinite(x)) return fail(SG_EINVAL, "angle offsets must be finite");
    for (double x : {c.along_strike, c.across_min, c.across_max, c.min_distance, c.slip_min, c.slip_max})
        if (!(x >= 0.0 && std::isfinite(x))) return fail(SG_EINVAL, "distances and slip fractions must be finite and >= 0");
    if (c.across_max < c.across_min || c.slip_max < c.slip_min)
        return fail(SG_EINVAL, "across_max >= across_min and slip_max >= slip_min required");
    if (!positive_finite(c.size_scale)) return fail(SG_EINVAL, "size_scale must be finite and > 0");
    const sg_fault_params &p = *primary;
    for (double x : {p.cz, p.cy, p.cx, p.azimuth_deg, p.dip_deg, p.slip})
        if (!std::isfinite(x)) return fail(SG_EINVAL, "fault centre, azimuth, dip and slip must be finite");
    for (double x : {p.radius, p.die_r, p.die_strike, p.die_theta_deg})
        if (!positive_finite(x)) return fail(SG_EINVAL, "radius and die-off extents must be finite and > 0");
    for (int64_t i = 0; i < (int64_t)ncand * 5; ++i)
        if (!(uniforms[i] >= 0.0 && uniforms[i] <= 1.0)) return fail(SG_EINVAL, "uniforms must be in [0, 1]");
    const double deg = 3.14159265358979323846 / 180.0;
    const double a = p.azimuth_deg * deg;
    const double n_y = std::sin(a), n_x = std::cos(a), s_y = std::cos(a), s_x = -std::sin(a);
    int32_t m = 0;
    for (int32_t k = 0; k < ncand; ++k) {
        const double *u = uniforms + (size_t)k * 5;
        const bool synthetic = u[0] < c.synthetic_fraction;
        const double side = u[1] < c.hangingwall_fraction ? -1.0 : 1.0;   // hanging wall: -n
        const double along = (2.0 * u[2] - 1.0) * c.along_strike;
        const double across = c.across_min + u[3] * (c.across_max - c.across_min);
        const double cy = p.cy + along * s_y + side * across * n_y;
        const double cx = p.cx + along * s_x + side * across * n_x;
        bool keep = true;
        if (c.min_distance > 0.0)
            for (int32_t q = 0; q < m && keep; ++q)
                keep = !(std::hypot(cy - out[q].cy, cx - out[q].cx) < c.min_distance);
        if (!keep) continue;
        sg_fault_params f = p;
        f.cy = cy;
        f.cx = cx;
        f.azimuth_deg = p.azimuth_deg + (synthetic ? c.synthetic_offset_deg : c.antithetic_offset_deg);
        f.radius = p.radius * c.size_scale;
        f.die_r = p.die_r * c.size_scale;
        f.die_strike = p.die_strike * c.size_scale;
        f.slip = p.slip * (c.slip_min + u[4] * (c.slip_max - c.slip_min));
        f.rough_lattice = nullptr;
        f.rough_noct = f.rough_gd = f.rough_gs = 0;
        f.rough_amplitude = f.rough_lam_strike = f.rough_lam_dip = 0.0;
        out[m++] = f;
    }
    *nout = m;
    return SG_OK;
}

namespace {
sg_status salt_size_args(int32_t nz, int32_t ny, int32_t nx)
{
    if (nz < 1 || ny < 1 || nx < 1) return fail(SG_EINVAL, "nz, ny and nx must be >= 1");
    if ((int64_t)nz * ny * nx > (int64_t)INT32_MAX) return fail(SG_EINVAL, "volume too large (at most 2^31 - 1 voxels)");
    return SG_OK;
}
}  // namespace

sg_status sg_salt_workspace_size(int32_t nz, int32_t ny, int32_t nx, size_t *bytes)
{
    if (!bytes) return fail(SG_EINVAL, "NULL argument");
    sg_status rc = salt_size_args(nz, ny, nx);
    if (rc != SG_OK) return rc;
    *bytes = sg::salt_workspace_bytes((int64_t)nz * ny * nx);
    return SG_OK;
}

sg_status sg_salt_sdt(const float *v, int32_t nz, int32_t ny, int32_t nx, double dz, double dy, double dx,
                      int32_t nbodies, const double *centres, const double *radii, const double *rotations,
                      const float *grf, double amplitude, float v_salt, float v_water, int64_t min_voxels,
                      float *out, uint8_t *mask_out, void *ws, size_t ws_bytes, void *stream)
{
    if (!v || !out || !ws) return fail(SG_EINVAL, "NULL argument");
    if (v == out) return fail(SG_EINVAL, "out must not alias the input volume");
    sg_status rc = salt_size_args(nz, ny, nx);
    if (rc != SG_OK) return rc;
    if (nbodies < 0 || nbodies > sg::kSaltMaxBodies)
        return fail(SG_EINVAL, "nbodies must be in 0..%d", sg::kSaltMaxBodies);
    if (nbodies > 0 && (!centres || !radii || !rotations || !grf)) return fail(SG_EINVAL, "NULL body argument");
    if (!positive_finite(dz) || !positive_finite(dy) || !positive_finite(dx))
        return fail(SG_EINVAL, "dz, dy and dx must be finite and > 0");
    if (!std::isfinite(amplitude) || !std::isfinite(v_salt) || !std::isfinite(v_water))
        return fail(SG_EINVAL, "amplitude, v_salt and v_water must be finite");
    if (min_voxels < 0 || min_voxels > (int64_t)UINT32_MAX) return fail(SG_EINVAL, "min_voxels out of range");
    if ((uintptr_t)ws % 256) return fail(SG_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = sg::salt_workspace_bytes((int64_t)nz * ny * nx);
    if (ws_bytes < need) return fail(SG_ENOSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    std::vector<sg::SaltBody> B(nbodies);
    for (int i = 0; i < nbodies; ++i) {
        for (int k = 0; k < 3; ++k) {
            B[i].c[k] = centres[3 * i + k];
            B[i].r[k] = radii[3 * i + k];
            if (!std::isfinite(B[i].c[k])) return fail(SG_EINVAL, "body %d: centre must be finite", i);
            if (!positive_finite(B[i].r[k])) return fail(SG_EINVAL, "body %d: radii must be finite and > 0", i);
        }
        for (int k = 0; k < 9; ++k) {
            B[i].R[k] = rotations[9 * i + k];
            if (!std::isfinite(B[i].R[k])) return fail(SG_EINVAL, "body %d: rotation must be finite", i);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double d = 0.0;
                for (int k = 0; k < 3; ++k) d += B[i].R[3 * a + k] * B[i].R[3 * b + k];
                if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-7)
                    return fail(SG_EINVAL, "body %d: rotation must be orthonormal (R R^T = I within 1e-7)", i);
            }
    }
    SG_HIP(sg::launch_salt_sdt(v, nz, ny, nx, dz, dy, dx, nbodies, B.data(), grf, amplitude, v_salt, v_water,
                               (unsigned)min_voxels, out, mask_out, ws, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_grf_workspace_size(int32_t nz, int32_t ny, int32_t nx, int32_t *grid, size_t *bytes)
{
    if (!bytes) return fail(SG_EINVAL, "NULL argument");
    if (nz < 1 || ny < 1 || nx < 1 || nz > 1024 || ny > 1024 || nx > 1024)
        return fail(SG_EINVAL, "extents must be in 1..1024 (got %d x %d x %d)", nz, ny, nx);
    int P[3];
    sg::grf_grid(nz, ny, nx, P);
    if (grid)
        for (int k = 0; k < 3; ++k) grid[k] = P[k];
    *bytes = sg::grf_workspace_bytes(nz, ny, nx);
    return SG_OK;
}

sg_status sg_grf(const float *noise, int32_t nz, int32_t ny, int32_t nx, double lz, double ly, double lx, double p,
                 float *out, void *ws, size_t ws_bytes, void *stream)
{
    size_t need = 0;
    sg_status rc = sg_grf_workspace_size(nz, ny, nx, nullptr, &need);
    if (rc != SG_OK) return rc;
    if (!noise || !out || !ws) return fail(SG_EINVAL, "NULL argument");
    if (!(std::isfinite(lz) && std::isfinite(ly) && std::isfinite(lx) && lz >= 0 && ly >= 0 && lx >= 0))
        return fail(SG_EINVAL, "correlation lengths must be finite and >= 0");
    if (!std::isfinite(p) || p < 0) return fail(SG_EINVAL, "p must be finite and >= 0");
    if (ws_bytes < need) return fail(SG_ENOSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    if ((const void *)out == (const void *)noise) return fail(SG_EINVAL, "out must not alias noise");
    SG_HIP(sg::launch_grf(noise, nz, ny, nx, lz, ly, lx, p, out, ws, (hipStream_t)stream));
    return SG_OK;
}

sg_status sg_set_graphs(int32_t on)
{
    g_batch_graphs = on != 0;
    return SG_OK;
}

}  // extern "C"
