/*
 * fdo.c -- FP64 CPU oracle of the discrete 2D acoustic scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product library never links
 * or calls it.  It shares no code, header, table or helper with the HIP path.
 *
 * What it computes (SubsurfaceGen, arXiv 2605.30541):
 *   - the constant-density acoustic wave equation with a source term
 *     (Sec. 2, eq. "acoustic"; App. E.2, eq. "acoustic_2d"),
 *   - zero initial conditions (App. E.2, "Initial conditions"),
 *   - a free surface p(x,0,t)=0 at the top (App. E.2, eq. "free_surface"),
 *   - a Cerjan sponge on the other sides: the PDE gains eta * dp/dt with
 *     eta = c_damp/h [rho - sin(2 pi rho)/(2 pi)], c_damp = 1.5 ln(1/R)/n_bl
 *     (App. E.2, eqs. "cerjan_pde" and "cerjan_damp"),
 *   - an 8th-order (M = 4) central difference in space and a 2nd-order
 *     leapfrog in time (App. E.3 and Table "params"),
 *   - point sources (Ricker pulses, Sec. 2 and App. E.4) and the receiver
 *     sampling operator R that produces shot gathers (Sec. 2),
 *   - wavefield snapshots (Sec. 4, App. E.5).
 * The adjoint and the velocity gradient are not in the paper; they are the
 * exact transpose / derivative of the discrete forward map above (the FWI
 * use the introduction motivates), written in the Lagrange-multiplier form.
 *
 * Readings of points the paper leaves open (units of eta, ghost rows of the
 * free surface, rho discretisation, corners, velocity inside the sponge,
 * source scaling and time level, time discretisation of eta p_t) are listed
 * in the design notes; each is marked "reading" below.
 *
 * Everything is double precision.  OpenMP only splits the per-cell loops
 * over rows; every cell's arithmetic is the same sequence as a serial run.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FDO_PI 3.14159265358979323846

typedef struct {
    int32_t nz, nx;     /* physical nodes; node (iz,ix) sits at z=iz*dz, x=ix*dx */
    double dz, dx;      /* grid spacing [m] */
    double dt;          /* time step [s] */
    int32_t nt;         /* number of time levels t_n = n*dt, n = 0..nt-1 */
    int32_t nbl;        /* sponge width in cells (0 = rigid p=0 just outside) */
    int32_t top_free;   /* 1 = free surface at z=0, 0 = sponge on top as well */
    double R;           /* target reflection coefficient of the sponge */
} fdo_geom;

/* 8th-order central second-derivative weights c_0..c_4 (Fornberg 1988, which
 * App. E.3.2 cites for the coefficients a_m). */
static const double C8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0,
                             8.0 / 315.0, -1.0 / 560.0};

/* Padded model: physical grid plus the sponge. */
typedef struct {
    int Nz, Nx;     /* padded size */
    int ztop;       /* padded row of physical row 0 (0 with a free top) */
    int xleft;      /* padded column of physical column 0 (= nbl) */
    int free_top;
    double dz, dx, dt;
    double *v, *eta, *a, *b, *W;
} fdo_model;

static void model_free(fdo_model *m)
{
    free(m->v); free(m->eta); free(m->a); free(m->b); free(m->W);
    memset(m, 0, sizeof(*m));
}

/* Cerjan profile of one side at depth d = 1..nbl cells into the sponge,
 * in SI units (s/m^2).  Reading: rho = d/nbl, and the eta of the paper is in
 * the km/s - ms unit system of its solver, so eta_SI = eta * 1e-3. */
static double sponge_eta(int d, int nbl, double h, double R)
{
    if (d <= 0 || nbl <= 0) return 0.0;
    double cdamp = 1.5 * log(1.0 / R) / (double)nbl;
    double rho = (double)d / (double)nbl;
    return cdamp / h * (rho - sin(2.0 * FDO_PI * rho) / (2.0 * FDO_PI)) * 1e-3;
}

static int model_build(const fdo_geom *g, const double *v_phys, fdo_model *m)
{
    memset(m, 0, sizeof(*m));
    m->free_top = g->top_free ? 1 : 0;
    m->ztop = m->free_top ? 0 : g->nbl;
    m->xleft = g->nbl;
    m->Nz = g->nz + m->ztop + g->nbl;
    m->Nx = g->nx + 2 * g->nbl;
    m->dz = g->dz; m->dx = g->dx; m->dt = g->dt;
    size_t n = (size_t)m->Nz * m->Nx;
    m->v = malloc(n * sizeof(double));
    m->eta = malloc(n * sizeof(double));
    m->a = malloc(n * sizeof(double));
    m->b = malloc(n * sizeof(double));
    m->W = malloc(n * sizeof(double));
    if (!m->v || !m->eta || !m->a || !m->b || !m->W) { model_free(m); return -1; }
    for (int Iz = 0; Iz < m->Nz; ++Iz) {
        for (int Ix = 0; Ix < m->Nx; ++Ix) {
            /* reading: velocity in the sponge is the nearest physical edge value */
            int iz = Iz - m->ztop, ix = Ix - m->xleft;
            if (iz < 0) iz = 0;
            if (iz > g->nz - 1) iz = g->nz - 1;
            if (ix < 0) ix = 0;
            if (ix > g->nx - 1) ix = g->nx - 1;
            double vel = v_phys[(size_t)iz * g->nx + ix];
            /* depth into each sponge side; reading: corners add the sides */
            int dl = m->xleft - Ix;                     /* left   */
            int dr = Ix - (m->xleft + g->nx - 1);       /* right  */
            int db = Iz - (m->ztop + g->nz - 1);        /* bottom */
            int dtp = m->ztop - Iz;                     /* top (absorbing mode only) */
            double eta = sponge_eta(dl, g->nbl, g->dx, g->R)
                       + sponge_eta(dr, g->nbl, g->dx, g->R)
                       + sponge_eta(db, g->nbl, g->dz, g->R)
                       + sponge_eta(dtp, g->nbl, g->dz, g->R);
            /* centred eta*dp/dt: (1+gamma) p^{n+1} = 2p^n - (1-gamma) p^{n-1} + v^2 dt^2 (...) */
            double gam = eta * vel * vel * g->dt / 2.0;
            size_t k = (size_t)Iz * m->Nx + Ix;
            m->v[k] = vel;
            m->eta[k] = eta;
            m->a[k] = 1.0 / (1.0 + gam);
            m->b[k] = (1.0 - gam) / (1.0 + gam);
            m->W[k] = m->a[k] * g->dt * g->dt * vel * vel;
        }
    }
    return 0;
}

/* Field value at padded (Iz,Ix).  Outside the padded grid the field is 0
 * (rigid).  With a free top, row 0 is z=0 where p=0, and rows above are the
 * odd mirror p(-m) = -p(m) (reading of the sign-flipped reflection). */
static inline double at(const fdo_model *m, const double *p, int Iz, int Ix)
{
    if (Ix < 0 || Ix >= m->Nx || Iz >= m->Nz) return 0.0;
    if (Iz < 0) {
        if (!m->free_top) return 0.0;
        Iz = -Iz;
        if (Iz >= m->Nz) return 0.0;
        return -p[(size_t)Iz * m->Nx + Ix];
    }
    return p[(size_t)Iz * m->Nx + Ix];
}

/* out = L p, the 8th-order Laplacian d2/dz2 + d2/dx2 (App. E.3). */
static void laplacian(const fdo_model *m, const double *p, double *out)
{
    const double iz2 = 1.0 / (m->dz * m->dz), ix2 = 1.0 / (m->dx * m->dx);
    #pragma omp parallel for schedule(static)
    for (int Iz = 0; Iz < m->Nz; ++Iz) {
        for (int Ix = 0; Ix < m->Nx; ++Ix) {
            double c = at(m, p, Iz, Ix);
            double dzz = C8[0] * c, dxx = C8[0] * c;
            for (int s = 1; s <= 4; ++s) {
                dzz += C8[s] * (at(m, p, Iz + s, Ix) + at(m, p, Iz - s, Ix));
                dxx += C8[s] * (at(m, p, Iz, Ix + s) + at(m, p, Iz, Ix - s));
            }
            out[(size_t)Iz * m->Nx + Ix] = dzz * iz2 + dxx * ix2;
        }
    }
}

/* Bilinear spreading / sampling weights of a point at (z,x) metres from the
 * physical origin.  Writes up to 4 padded node indices and weights; nodes with
 * zero weight are dropped.  Returns the count, or -1 outside the physical
 * domain.  Reading: a point source becomes w/(dx dz) at the nodes with these
 * weights, and receivers sample with the same weights (R and its transpose). */
static int bilinear(const fdo_model *m, int nz, int nx, double z, double x,
                    size_t node[4], double wt[4])
{
    double fz = z / m->dz, fx = x / m->dx;
    if (!(fz >= 0.0 && fx >= 0.0 && fz <= (double)(nz - 1) && fx <= (double)(nx - 1)))
        return -1;
    int iz = (int)floor(fz), ix = (int)floor(fx);
    if (iz > nz - 1) iz = nz - 1;
    if (ix > nx - 1) ix = nx - 1;
    double rz = fz - iz, rx = fx - ix;
    int cnt = 0;
    for (int dzi = 0; dzi < 2; ++dzi) {
        for (int dxi = 0; dxi < 2; ++dxi) {
            double w = (dzi ? rz : 1.0 - rz) * (dxi ? rx : 1.0 - rx);
            if (w == 0.0) continue;
            node[cnt] = (size_t)(iz + dzi + m->ztop) * m->Nx + (ix + dxi + m->xleft);
            wt[cnt] = w;
            ++cnt;
        }
    }
    return cnt;
}

typedef struct {
    int cnt;
    size_t node[4];
    double wt[4];
} fdo_point;

static int points_build(const fdo_model *m, const fdo_geom *g, int n, const double *zx,
                        fdo_point *out)
{
    for (int i = 0; i < n; ++i) {
        out[i].cnt = bilinear(m, g->nz, g->nx, zx[2 * i], zx[2 * i + 1], out[i].node, out[i].wt);
        if (out[i].cnt < 0) return -1;
    }
    return 0;
}

/* S^n on the padded grid: sum over the shot's point sources of
 * weight * w_j(t_n) / (dx dz).  `s` must be zeroed on entry. */
static void source_grid(const fdo_model *m, int nsrc, const fdo_point *src,
                        const double *wavelets, int nt, int n, double *s)
{
    const double inv_cell = 1.0 / (m->dx * m->dz);
    for (int j = 0; j < nsrc; ++j)
        for (int q = 0; q < src[j].cnt; ++q)
            s[src[j].node[q]] += src[j].wt[q] * wavelets[(size_t)j * nt + n] * inv_cell;
}

/* One leapfrog step: p_next = 2a p + W (L p + S) - b p_prev; row 0 pinned to 0
 * under a free surface.  `lap` and `s` are caller scratch (s zeroed here). */
static void step(const fdo_model *m, const double *p_prev, const double *p,
                 double *p_next, double *lap, double *s, int nsrc,
                 const fdo_point *src, const double *wavelets, int nt, int n)
{
    size_t N = (size_t)m->Nz * m->Nx;
    laplacian(m, p, lap);
    memset(s, 0, N * sizeof(double));
    source_grid(m, nsrc, src, wavelets, nt, n, s);
    #pragma omp parallel for schedule(static)
    for (int Iz = 0; Iz < m->Nz; ++Iz) {
        for (int Ix = 0; Ix < m->Nx; ++Ix) {
            size_t k = (size_t)Iz * m->Nx + Ix;
            if (m->free_top && Iz == 0) { p_next[k] = 0.0; continue; }
            p_next[k] = 2.0 * m->a[k] * p[k] + m->W[k] * (lap[k] + s[k]) - m->b[k] * p_prev[k];
        }
    }
}

static double sample(const fdo_point *r, const double *p)
{
    double d = 0.0;
    for (int q = 0; q < r->cnt; ++q) d += r->wt[q] * p[r->node[q]];
    return d;
}

/* ------------------------------------------------------------------------ */
/* Public entry points (called from Python through ctypes).                  */
/* Return codes: 0 ok, -1 out of memory, -2 bad argument / position.         */
/* ------------------------------------------------------------------------ */

int fdo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Padded coefficient arrays (for tests): each output is Nz*Nx, may be NULL. */
int fdo_model_arrays(const fdo_geom *g, const double *v, int32_t *NzNx,
                     double *vpad, double *eta, double *a, double *b, double *W)
{
    fdo_model m;
    if (model_build(g, v, &m)) return -1;
    size_t N = (size_t)m.Nz * m.Nx;
    if (NzNx) { NzNx[0] = m.Nz; NzNx[1] = m.Nx; }
    if (vpad) memcpy(vpad, m.v, N * sizeof(double));
    if (eta) memcpy(eta, m.eta, N * sizeof(double));
    if (a) memcpy(a, m.a, N * sizeof(double));
    if (b) memcpy(b, m.b, N * sizeof(double));
    if (W) memcpy(W, m.W, N * sizeof(double));
    model_free(&m);
    return 0;
}

/* L p on the padded grid (for tests). */
int fdo_apply_laplacian(const fdo_geom *g, const double *v, const double *p, double *out)
{
    fdo_model m;
    if (model_build(g, v, &m)) return -1;
    laplacian(&m, p, out);
    model_free(&m);
    return 0;
}

/*
 * Forward modelling of nshot independent shots.
 *   v         [nz][nx]                physical velocity [m/s]
 *   src_zx    [nshot][nsrc][2]        point-source positions (z, x) [m]
 *   wavelets  [nshot][nsrc][nt]       source time functions w(t_n)
 *   rec_zx    [nrec][2]               receivers, shared by every shot
 *   gathers   [nshot][ceil(nt/rec_every)][nrec]   d^n_r at n = 0, k, 2k, ... (may be NULL)
 *   snaps     [nshot][snap_count][nz][nx]        p^n at n = j*snap_every (may be NULL)
 */
int fdo_forward(const fdo_geom *g, const double *v, int nshot, int nsrc,
                const double *src_zx, const double *wavelets, int nrec,
                const double *rec_zx, int rec_every, double *gathers,
                int snap_every, int snap_count, double *snaps)
{
    if (g->nz < 1 || g->nx < 1 || g->nt < 1 || nshot < 0 || nsrc < 0 || nrec < 0 ||
        rec_every < 1 || (snaps && (snap_every < 1 || snap_count < 0 ||
                                    (snap_count > 0 && (long)(snap_count - 1) * snap_every > g->nt - 1))))
        return -2;
    fdo_model m;
    if (model_build(g, v, &m)) return -1;
    size_t N = (size_t)m.Nz * m.Nx;
    int nrow = (g->nt + rec_every - 1) / rec_every;
    double *buf = calloc(5 * N, sizeof(double));
    fdo_point *src = malloc((size_t)(nsrc > 0 ? nsrc : 1) * sizeof(fdo_point));
    fdo_point *rec = malloc((size_t)(nrec > 0 ? nrec : 1) * sizeof(fdo_point));
    int rc = 0;
    if (!buf || !src || !rec) { rc = -1; goto done; }
    if (points_build(&m, g, nrec, rec_zx, rec)) { rc = -2; goto done; }
    for (int sh = 0; sh < nshot; ++sh) {
        if (points_build(&m, g, nsrc, src_zx + (size_t)sh * nsrc * 2, src)) { rc = -2; goto done; }
        const double *wl = wavelets + (size_t)sh * nsrc * g->nt;
        double *pm = buf, *p0 = buf + N, *pn = buf + 2 * N, *lap = buf + 3 * N, *s = buf + 4 * N;
        memset(pm, 0, N * sizeof(double));   /* p^{-1} = 0 */
        memset(p0, 0, N * sizeof(double));   /* p^{0}  = 0 */
        for (int n = 0; n < g->nt; ++n) {
            /* p0 holds level n here */
            if (gathers && n % rec_every == 0) {
                double *row = gathers + ((size_t)sh * nrow + n / rec_every) * nrec;
                for (int r = 0; r < nrec; ++r) row[r] = sample(&rec[r], p0);
            }
            if (snaps && n % snap_every == 0 && n / snap_every < snap_count) {
                double *fr = snaps + ((size_t)sh * snap_count + n / snap_every) * g->nz * g->nx;
                for (int iz = 0; iz < g->nz; ++iz)
                    memcpy(fr + (size_t)iz * g->nx, p0 + (size_t)(iz + m.ztop) * m.Nx + m.xleft,
                           g->nx * sizeof(double));
            }
            if (n == g->nt - 1) break;
            step(&m, pm, p0, pn, lap, s, nsrc, src, wl, g->nt, n);
            double *t = pm; pm = p0; p0 = pn; pn = t;
        }
    }
done:
    free(buf); free(src); free(rec);
    model_free(&m);
    return rc;
}

/*
 * Gradient of J = 1/2 sum_shots sum_{recorded n} sum_r (d^n_r - d^{obs,n}_r)^2
 * with respect to the physical velocity, given the residual r = d - d_obs
 * (any dJ/dd works: the result is linear in it).
 *   resid      [nshot][ceil(nt/rec_every)][nrec]
 *   grad       [nz][nx]              overwritten with the sum over shots
 *   wl_grad    [nshot][nsrc][nt]     dJ/dw (may be NULL)
 *   ckpt       checkpoint spacing for the forward recompute (<=0: sqrt(nt))
 *
 * Adjoint (transpose of the step map, Lagrange multipliers lambda^k of the
 * equation that defines p^k, k = 1..nt-1):
 *   lambda^k = 2a lambda^{k+1} + L(W lambda^{k+1}) - b lambda^{k+2} + R^T r^k,
 *   lambda^{nt} = lambda^{nt+1} = 0; with a free top, row 0 carries no unknown
 *   so lambda is 0 there, and L keeps its odd-mirror rule (it is symmetric on
 *   rows >= 1).
 * Gradient on the padded grid (a, b, W depend on v through gamma):
 *   g = sum_{n=0}^{nt-2} lambda^{n+1} [2 a_v p^n + W_v (L p^n + S^n) - b_v p^{n-1}],
 *   gamma_v = eta v dt, a_v = -a^2 gamma_v, b_v = -2 a^2 gamma_v,
 *   W_v = dt^2 (2 v a + v^2 a_v).
 * Then each sponge cell's g is added to the physical cell its velocity was
 * copied from (transpose of the edge replication).
 */
int fdo_gradient(const fdo_geom *g, const double *v, int nshot, int nsrc,
                 const double *src_zx, const double *wavelets, int nrec,
                 const double *rec_zx, int rec_every, const double *resid,
                 double *grad, double *wl_grad, int ckpt)
{
    if (g->nz < 1 || g->nx < 1 || g->nt < 2 || nshot < 0 || nsrc < 0 || nrec < 0 || rec_every < 1)
        return -2;
    fdo_model m;
    if (model_build(g, v, &m)) return -1;
    const int nt = g->nt;
    if (ckpt <= 0) ckpt = (int)ceil(sqrt((double)nt));
    const int nseg = (nt - 1 + ckpt - 1) / ckpt;       /* segments (j*C, min((j+1)C, nt-1)] */
    const size_t N = (size_t)m.Nz * m.Nx;
    const int nrow = (nt + rec_every - 1) / rec_every;
    const double inv_cell = 1.0 / (m.dx * m.dz);
    /* checkpoints: levels (jC-1, jC) for j = 0..nseg-1 */
    double *cp = malloc((size_t)2 * nseg * N * sizeof(double));
    double *seg = malloc((size_t)(ckpt + 1) * N * sizeof(double));
    double *work = calloc(8 * N, sizeof(double));
    double *gpad = calloc(N, sizeof(double));
    double *av = malloc(N * sizeof(double)), *bv = malloc(N * sizeof(double)), *Wv = malloc(N * sizeof(double));
    fdo_point *src = malloc((size_t)(nsrc > 0 ? nsrc : 1) * sizeof(fdo_point));
    fdo_point *rec = malloc((size_t)(nrec > 0 ? nrec : 1) * sizeof(fdo_point));
    int rc = 0;
    if (!cp || !seg || !work || !gpad || !av || !bv || !Wv || !src || !rec) { rc = -1; goto done; }
    if (points_build(&m, g, nrec, rec_zx, rec)) { rc = -2; goto done; }
    for (size_t k = 0; k < N; ++k) {
        double gv = m.eta[k] * m.v[k] * g->dt;
        av[k] = -m.a[k] * m.a[k] * gv;
        bv[k] = -2.0 * m.a[k] * m.a[k] * gv;
        Wv[k] = g->dt * g->dt * (2.0 * m.v[k] * m.a[k] + m.v[k] * m.v[k] * av[k]);
    }
    if (wl_grad) memset(wl_grad, 0, (size_t)nshot * nsrc * nt * sizeof(double));

    for (int sh = 0; sh < nshot; ++sh) {
        if (points_build(&m, g, nsrc, src_zx + (size_t)sh * nsrc * 2, src)) { rc = -2; goto done; }
        const double *wl = wavelets + (size_t)sh * nsrc * nt;
        const double *rs = resid + (size_t)sh * nrow * nrec;
        double *lap = work, *s = work + N, *pm = work + 2 * N, *p0 = work + 3 * N, *pn = work + 4 * N;
        double *l1 = work + 5 * N, *l2 = work + 6 * N, *l0 = work + 7 * N;   /* lambda^{k+1}, ^{k+2}, ^k */

        /* forward sweep, keeping (p^{jC-1}, p^{jC}) */
        memset(pm, 0, N * sizeof(double));
        memset(p0, 0, N * sizeof(double));
        for (int n = 0; n < nt - 1; ++n) {
            if (n % ckpt == 0) {
                int j = n / ckpt;
                memcpy(cp + (size_t)(2 * j) * N, pm, N * sizeof(double));
                memcpy(cp + (size_t)(2 * j + 1) * N, p0, N * sizeof(double));
            }
            step(&m, pm, p0, pn, lap, s, nsrc, src, wl, nt, n);
            double *t = pm; pm = p0; p0 = pn; pn = t;
        }

        memset(l1, 0, N * sizeof(double));
        memset(l2, 0, N * sizeof(double));
        for (int j = nseg - 1; j >= 0; --j) {
            int lo = j * ckpt, hi = (j + 1) * ckpt;
            if (hi > nt - 1) hi = nt - 1;
            /* seg[i] = p^{lo-1+i}, i = 0..hi-lo */
            memcpy(seg, cp + (size_t)(2 * j) * N, N * sizeof(double));
            memcpy(seg + N, cp + (size_t)(2 * j + 1) * N, N * sizeof(double));
            for (int n = lo; n < hi - 1; ++n)
                step(&m, seg + (size_t)(n - lo) * N, seg + (size_t)(n - lo + 1) * N,
                     seg + (size_t)(n - lo + 2) * N, lap, s, nsrc, src, wl, nt, n);
            for (int k = hi; k >= lo + 1; --k) {
                /* lambda^k from lambda^{k+1} (l1) and lambda^{k+2} (l2) */
                for (size_t q = 0; q < N; ++q) s[q] = m.W[q] * l1[q];
                laplacian(&m, s, lap);
                #pragma omp parallel for schedule(static)
                for (int Iz = 0; Iz < m.Nz; ++Iz)
                    for (int Ix = 0; Ix < m.Nx; ++Ix) {
                        size_t q = (size_t)Iz * m.Nx + Ix;
                        l0[q] = 2.0 * m.a[q] * l1[q] + lap[q] - m.b[q] * l2[q];
                    }
                if (k % rec_every == 0) {
                    const double *rr = rs + (size_t)(k / rec_every) * nrec;
                    for (int r = 0; r < nrec; ++r)
                        for (int q = 0; q < rec[r].cnt; ++q)
                            l0[rec[r].node[q]] += rec[r].wt[q] * rr[r];
                }
                if (m.free_top) memset(l0, 0, (size_t)m.Nx * sizeof(double));

                /* term n = k-1: needs p^{k-1} = seg[k-lo], p^{k-2} = seg[k-1-lo] */
                const double *pk1 = seg + (size_t)(k - lo) * N;
                const double *pk2 = seg + (size_t)(k - 1 - lo) * N;
                laplacian(&m, pk1, lap);
                memset(s, 0, N * sizeof(double));
                source_grid(&m, nsrc, src, wl, nt, k - 1, s);
                #pragma omp parallel for schedule(static)
                for (int Iz = 0; Iz < m.Nz; ++Iz)
                    for (int Ix = 0; Ix < m.Nx; ++Ix) {
                        size_t q = (size_t)Iz * m.Nx + Ix;
                        gpad[q] += l0[q] * (2.0 * av[q] * pk1[q] + Wv[q] * (lap[q] + s[q])
                                            - bv[q] * pk2[q]);
                    }
                if (wl_grad) {
                    for (int jj = 0; jj < nsrc; ++jj) {
                        double acc = 0.0;
                        for (int q = 0; q < src[jj].cnt; ++q)
                            acc += src[jj].wt[q] * m.W[src[jj].node[q]] * l0[src[jj].node[q]] * inv_cell;
                        wl_grad[((size_t)sh * nsrc + jj) * nt + (k - 1)] = acc;
                    }
                }
                double *t = l2; l2 = l1; l1 = l0; l0 = t;
            }
        }
    }

    /* fold the padded gradient onto the physical cells */
    memset(grad, 0, (size_t)g->nz * g->nx * sizeof(double));
    for (int Iz = 0; Iz < m.Nz; ++Iz)
        for (int Ix = 0; Ix < m.Nx; ++Ix) {
            int iz = Iz - m.ztop, ix = Ix - m.xleft;
            if (iz < 0) iz = 0;
            if (iz > g->nz - 1) iz = g->nz - 1;
            if (ix < 0) ix = 0;
            if (ix > g->nx - 1) ix = g->nx - 1;
            grad[(size_t)iz * g->nx + ix] += gpad[(size_t)Iz * m.Nx + Ix];
        }
done:
    free(cp); free(seg); free(work); free(gpad); free(av); free(bv); free(Wv);
    free(src); free(rec);
    model_free(&m);
    return rc;
}
