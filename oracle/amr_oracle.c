/*
 * FP64 reference of the multi-level (octree block) lattice-Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY (built into liblbm_oracle.so; never linked by the
 * product library and sharing no source with it).
 *
 * Paper Sec. 2.2: the LBM runs on the cubic leaf blocks of an octree, with
 * the finest grid near the tree surface, a moderate one in the wake and
 * coarse blocks elsewhere; the coarse/fine coupling itself is delegated to
 * the authors' earlier work.  Readings taken here (listed in the design
 * notes, the same ones the product implements independently):
 *
 *  Levels l = 0 (coarsest) .. L-1 (finest); a level-l cell spans h_l =
 *  2^(L-1-l) finest cells and advances with time step h_l (acoustic
 *  scaling: the same lattice velocity everywhere); nu_l = nu_finest / h_l.
 *
 *  Refinement: level 0 holds every block of its box.  A block of level l-1
 *  that exists is refined into 8 level-l blocks when some branch axis segment
 *  meets its box grown by R + band[l] on every side, or when
 *  the block box overlaps the wake box [x0, x1 + wake[l]] x [y0 - band[l],
 *  y1 + band[l]] x [z0 - band[l], z1 + band[l]] ((x0..z1) = tree bounding
 *  box, wake[l] > 0 only).  Then, from fine to coarse, every block that is
 *  refined must have all 26 neighbours existing at its level; a missing
 *  neighbour forces the refinement of its parent.  Refined level-0 blocks
 *  may not touch the box faces.
 *
 *  Cell classes per level: active (block exists, not refined), band
 *  (refined, Chebyshev distance <= 2 to an active cell), deep (refined,
 *  farther), ghost (level >= 1: no block, distance 1 to an existing cell).
 *  Collision and streaming run on active, band and ghost cells (solid cells
 *  excluded); values streamed from outside that set are undefined (NaN here)
 *  and land only in band or ghost cells, which are overwritten before their
 *  next collision.
 *
 *  Transfer quantities of a cell: density, velocity and the strain-rate
 *  tensor in finest time units, D = S / h_l, with the lattice strain rate
 *  from the pre-collision non-equilibrium second-order central moments
 *  N = kappa_2 - rho/3 I:  S = -3/(2 rho) (omega1 dev N + omega2 tr(N)/3 I).
 *  Rebuilding at level t inverts this with t's rates and step (kappa_2 =
 *  rho/3 I + N), every cumulant above the second order set to zero.
 *
 *  Schedule of one coarse step, coarse first:
 *    advance(l): M0 = transfer quantities of level l (pre-collision, time T);
 *                step level l;
 *                if l < L-1:  ghosts of l+1 <- trilinear(M0);       advance(l+1)
 *                             M1 = transfer quantities of level l (T+1)
 *                             ghosts of l+1 <- trilinear((M0+M1)/2); advance(l+1)
 *                             band of l <- restriction of level l+1
 *  Trilinear prolongation of a fine ghost g: coarse parent P = g >> 1 and,
 *  per axis, P + s with s = +1 for an odd fine index and -1 for an even one,
 *  weights 3/4 and 1/4.  Restriction of a band cell X: children 2X + {0,1}^3
 *  (solid children skipped), mean density, mass-weighted velocity, mean D; a
 *  band cell with no fluid child lies inside the wall and takes the fluid at
 *  rest (rho = 1, u = 0, D = 0).
 *
 * Populations: f[l][i * N_l + cell], cell = x + nx_l (y + ny_l z).
 */
#include <math.h>
#include <stdint.h>

#define OR_MAX_LEVELS 8
#include <stdlib.h>
#include <string.h>

/* from lbm_oracle.c */
double or_weight(int i);
void or_equilibrium(double rho, const double *u, double *f);
void or_chimera_forward(const double *f, const double *u, double *k);
void or_chimera_inverse(const double *k, const double *u, double *f);
void or_central_from_cumulants(const double *c, double *k);
void or_collide(const double *fin, double *fout, double omega1, double omega2, double omega_high, int galilean,
                const double *force);

#define Q 27
enum { C_NONE = 0, C_ACTIVE = 1, C_BAND = 2, C_DEEP = 3, C_GHOST = 4 };

typedef struct {
    int L, B, nx, ny, nz, periodic_x, galilean;
    double u_in, nu_f;
    int lnx[OR_MAX_LEVELS], lny[OR_MAX_LEVELS], lnz[OR_MAX_LEVELS];
    int nbx[OR_MAX_LEVELS], nby[OR_MAX_LEVELS], nbz[OR_MAX_LEVELS];
    uint8_t *bmap[OR_MAX_LEVELS]; /* 0 none, 1 leaf, 2 refined, 3 ghost storage */
    uint8_t *cls[OR_MAX_LEVELS];
    double omega[OR_MAX_LEVELS];
    double *f[OR_MAX_LEVELS], *t[OR_MAX_LEVELS];
    double *m0[OR_MAX_LEVELS], *m1[OR_MAX_LEVELS];
    uint8_t *solid;   /* finest box, may be NULL */
    int n_links;
    int64_t *lcell;
    int8_t *ldir;
    double *lq;
    int32_t *lbr;
    int64_t *lstart;  /* per finest cell: first link index (links sorted by cell) */
    int n_branch;
    int64_t steps[OR_MAX_LEVELS], finest_steps;
    double *force_log;  /* 3 per finest step, capacity log_cap */
    double *branch_force; /* 3 * n_branch, last finest step */
    int64_t log_cap, log_n;
    int error;
    const double *inlet; /* optional inlet fluctuation planes: plane k (3 per level-0 inlet cell, y fastest)
                            holds u' of the ghost plane at the time of level-0 step k */
    int64_t inlet_n;
} or_amr;

static int cxo(int i) { return i % 3 - 1; }
static int cyo(int i) { return (i / 3) % 3 - 1; }
static int czo(int i) { return i / 9 - 1; }

static int64_t lidx(const or_amr *a, int l, int x, int y, int z)
{
    return (int64_t)x + (int64_t)a->lnx[l] * ((int64_t)y + (int64_t)a->lny[l] * z);
}

static int64_t bidx(const or_amr *a, int l, int bx, int by, int bz)
{
    return (int64_t)bx + (int64_t)a->nbx[l] * ((int64_t)by + (int64_t)a->nby[l] * bz);
}

/* does the segment p0 -> p1 meet the closed box [lo, hi]?  (slab test) */
static int seg_meets_box(const double *p0, const double *p1, const double *lo, const double *hi)
{
    double t0 = 0.0, t1 = 1.0;
    for (int k = 0; k < 3; k++) {
        double d = p1[k] - p0[k];
        if (d == 0.0) {
            if (p0[k] < lo[k] || p0[k] > hi[k])
                return 0;
            continue;
        }
        double ta = (lo[k] - p0[k]) / d, tb = (hi[k] - p0[k]) / d;
        if (ta > tb) {
            double s = ta;
            ta = tb;
            tb = s;
        }
        if (ta > t0)
            t0 = ta;
        if (tb < t1)
            t1 = tb;
        if (t0 > t1)
            return 0;
    }
    return 1;
}

/* refines block b of level l (creating it first through its ancestors when
 * it does not exist); its children at level l+1 come into existence */
static int refine_block(or_amr *a, int l, int bx, int by, int bz)
{
    uint8_t *m = &a->bmap[l][bidx(a, l, bx, by, bz)];
    if (*m == 0) {
        if (l == 0)
            return -1;
        if (refine_block(a, l - 1, bx / 2, by / 2, bz / 2) != 0)
            return -1;
    }
    *m = 2;
    for (int s = 0; s < 8; s++) {
        uint8_t *cm = &a->bmap[l + 1][bidx(a, l + 1, 2 * bx + (s & 1), 2 * by + ((s >> 1) & 1), 2 * bz + (s >> 2))];
        if (*cm == 0)
            *cm = 1;
    }
    return 0;
}

/* block maps of every level from the branches (rows of 10 doubles) */
static int build_maps(or_amr *a, const double *br, int n, const int *band, const int *wake)
{
    double tb[6] = {1e300, -1e300, 1e300, -1e300, 1e300, -1e300};
    for (int i = 0; i < n; i++) {
        const double *r = br + 10 * i;
        double rad = 0.5 * r[6];
        for (int k = 0; k < 3; k++) {
            double lo = (r[k] < r[3 + k] ? r[k] : r[3 + k]) - rad;
            double hi = (r[k] > r[3 + k] ? r[k] : r[3 + k]) + rad;
            if (lo < tb[2 * k])
                tb[2 * k] = lo;
            if (hi > tb[2 * k + 1])
                tb[2 * k + 1] = hi;
        }
    }
    for (int l = 0; l < a->L; l++)
        a->bmap[l] = (uint8_t *)calloc((size_t)a->nbx[l] * a->nby[l] * a->nbz[l], 1);
    memset(a->bmap[0], 1, (size_t)a->nbx[0] * a->nby[0] * a->nbz[0]);
    /* coarse to fine: mark refinement of existing blocks, create children */
    for (int l = 1; l < a->L; l++) {
        int pl = l - 1;
        double bf = (double)a->B * (double)(1 << (a->L - 1 - pl)); /* finest cells per level-pl block */
        for (int bz = 0; bz < a->nbz[pl]; bz++)
            for (int by = 0; by < a->nby[pl]; by++)
                for (int bx = 0; bx < a->nbx[pl]; bx++) {
                    uint8_t *m = &a->bmap[pl][bidx(a, pl, bx, by, bz)];
                    if (*m == 0)
                        continue;
                    int refine = 0;
                    for (int i = 0; i < n && !refine; i++) {
                        const double *r = br + 10 * i;
                        double e = 0.5 * r[6] + band[l];
                        double lo[3] = {bx * bf - e, by * bf - e, bz * bf - e};
                        double hi[3] = {(bx + 1) * bf + e, (by + 1) * bf + e, (bz + 1) * bf + e};
                        if (seg_meets_box(r, r + 3, lo, hi))
                            refine = 1;
                    }
                    if (!refine && wake[l] > 0) {
                        double lo[3] = {bx * bf, by * bf, bz * bf};
                        double w0[3] = {tb[0], tb[2] - band[l], tb[4] - band[l]};
                        double w1[3] = {tb[1] + wake[l], tb[3] + band[l], tb[5] + band[l]};
                        refine = 1;
                        for (int k = 0; k < 3; k++)
                            if (!(lo[k] < w1[k] && lo[k] + bf > w0[k]))
                                refine = 0;
                    }
                    if (refine)
                        *m = 2;
                }
        /* children of refined blocks exist */
        for (int bz = 0; bz < a->nbz[l]; bz++)
            for (int by = 0; by < a->nby[l]; by++)
                for (int bx = 0; bx < a->nbx[l]; bx++)
                    if (a->bmap[pl][bidx(a, pl, bx / 2, by / 2, bz / 2)] == 2)
                        a->bmap[l][bidx(a, l, bx, by, bz)] = 1;
    }
    /* closure, fine to coarse, until stable: a refined block needs its 26
     * neighbours at its own level; a missing one gets its parent refined */
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int l = a->L - 2; l >= 1; l--)
            for (int bz = 0; bz < a->nbz[l]; bz++)
                for (int by = 0; by < a->nby[l]; by++)
                    for (int bx = 0; bx < a->nbx[l]; bx++) {
                        if (a->bmap[l][bidx(a, l, bx, by, bz)] != 2)
                            continue;
                        for (int k = 0; k < 27; k++) {
                            int x = bx + cxo(k), y = by + cyo(k), z = bz + czo(k);
                            if (x < 0 || y < 0 || z < 0 || x >= a->nbx[l] || y >= a->nby[l] || z >= a->nbz[l])
                                return -1;
                            if (a->bmap[l][bidx(a, l, x, y, z)] != 0)
                                continue;
                            if (refine_block(a, l - 1, x / 2, y / 2, z / 2) != 0)
                                return -1;
                            changed = 1;
                        }
                    }
    }
    /* refined level-0 blocks keep all 26 neighbours inside the box */
    for (int l = 0; l < a->L - 1; l++)
        for (int bz = 0; bz < a->nbz[l]; bz++)
            for (int by = 0; by < a->nby[l]; by++)
                for (int bx = 0; bx < a->nbx[l]; bx++)
                    if (a->bmap[l][bidx(a, l, bx, by, bz)] == 2)
                        if (bx < 1 || by < 1 || bz < 1 || bx >= a->nbx[l] - 1 || by >= a->nby[l] - 1 ||
                            bz >= a->nbz[l] - 1)
                            return -1;
    /* ghost storage blocks of the finer levels */
    for (int l = 1; l < a->L; l++)
        for (int bz = 0; bz < a->nbz[l]; bz++)
            for (int by = 0; by < a->nby[l]; by++)
                for (int bx = 0; bx < a->nbx[l]; bx++) {
                    if (a->bmap[l][bidx(a, l, bx, by, bz)] != 0)
                        continue;
                    for (int k = 0; k < 27; k++) {
                        int x = bx + cxo(k), y = by + cyo(k), z = bz + czo(k);
                        if (x < 0 || y < 0 || z < 0 || x >= a->nbx[l] || y >= a->nby[l] || z >= a->nbz[l])
                            continue;
                        uint8_t v = a->bmap[l][bidx(a, l, x, y, z)];
                        if (v == 1 || v == 2) {
                            a->bmap[l][bidx(a, l, bx, by, bz)] = 3;
                            break;
                        }
                    }
                }
    return 0;
}

static int exists_cell(const or_amr *a, int l, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= a->lnx[l] || y >= a->lny[l] || z >= a->lnz[l])
        return 0;
    uint8_t v = a->bmap[l][bidx(a, l, x / a->B, y / a->B, z / a->B)];
    return v == 1 || v == 2;
}

static int active_cell(const or_amr *a, int l, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= a->lnx[l] || y >= a->lny[l] || z >= a->lnz[l])
        return 0;
    return a->bmap[l][bidx(a, l, x / a->B, y / a->B, z / a->B)] == 1;
}

static void classify(or_amr *a)
{
    for (int l = 0; l < a->L; l++) {
        int64_t N = (int64_t)a->lnx[l] * a->lny[l] * a->lnz[l];
        a->cls[l] = (uint8_t *)calloc((size_t)N, 1);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < a->lnz[l]; z++)
            for (int y = 0; y < a->lny[l]; y++)
                for (int x = 0; x < a->lnx[l]; x++) {
                    uint8_t v = a->bmap[l][bidx(a, l, x / a->B, y / a->B, z / a->B)];
                    uint8_t c = C_NONE;
                    if (v == 1)
                        c = C_ACTIVE;
                    else if (v == 2) {
                        c = C_DEEP;
                        for (int dz = -2; dz <= 2 && c == C_DEEP; dz++)
                            for (int dy = -2; dy <= 2 && c == C_DEEP; dy++)
                                for (int dx = -2; dx <= 2 && c == C_DEEP; dx++)
                                    if (active_cell(a, l, x + dx, y + dy, z + dz))
                                        c = C_BAND;
                    } else if (l >= 1) {
                        for (int k = 0; k < 27 && c == C_NONE; k++)
                            if (exists_cell(a, l, x + cxo(k), y + cyo(k), z + czo(k)))
                                c = C_GHOST;
                    }
                    a->cls[l][lidx(a, l, x, y, z)] = c;
                }
    }
}

/* ---- transfer quantities ----------------------------------------------- */

/* (rho, ux, uy, uz, Dxx, Dyy, Dzz, Dxy, Dxz, Dyz) of pre-collision populations */
void or_cell_transfer(const double *f, double omega1, double dt, double *out)
{
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; i++) {
        rho += f[i];
        j[0] += cxo(i) * f[i];
        j[1] += cyo(i) * f[i];
        j[2] += czo(i) * f[i];
    }
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho}, k[Q];
    or_chimera_forward(f, u, k);
    double N[6] = {k[2] - rho / 3.0, k[6] - rho / 3.0, k[18] - rho / 3.0, k[4], k[10], k[12]};
    double tr = N[0] + N[1] + N[2];
    double omega2 = 1.0;
    double S[6];
    for (int a = 0; a < 3; a++)
        S[a] = -1.5 / rho * (omega1 * (N[a] - tr / 3.0) + omega2 * tr / 3.0);
    for (int a = 3; a < 6; a++)
        S[a] = -1.5 / rho * omega1 * N[a];
    out[0] = rho;
    out[1] = u[0];
    out[2] = u[1];
    out[3] = u[2];
    for (int a = 0; a < 6; a++)
        out[4 + a] = S[a] / dt;
}

/* pre-collision populations of a level with rate omega1 and step dt */
void or_cell_rebuild(const double *in, double omega1, double dt, double *f)
{
    double rho = in[0], u[3] = {in[1], in[2], in[3]}, S[6];
    for (int a = 0; a < 6; a++)
        S[a] = in[4 + a] * dt;
    double trs = S[0] + S[1] + S[2], omega2 = 1.0, N[6];
    for (int a = 0; a < 3; a++)
        N[a] = -2.0 * rho / 3.0 * ((S[a] - trs / 3.0) / omega1 + trs / 3.0 / omega2);
    for (int a = 3; a < 6; a++)
        N[a] = -2.0 * rho / 3.0 * S[a] / omega1;
    double c[Q], k[Q];
    memset(c, 0, sizeof c);
    c[0] = rho;
    c[2] = rho / 3.0 + N[0];
    c[6] = rho / 3.0 + N[1];
    c[18] = rho / 3.0 + N[2];
    c[4] = N[3];
    c[10] = N[4];
    c[12] = N[5];
    or_central_from_cumulants(c, k);
    or_chimera_inverse(k, u, f);
}

static double level_dt(const or_amr *a, int l) { return (double)(1 << (a->L - 1 - l)); }

static void level_transfer(or_amr *a, int l, double *m)
{
    int64_t N = (int64_t)a->lnx[l] * a->lny[l] * a->lnz[l];
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; c++) {
        uint8_t k = a->cls[l][c];
        if (k == C_NONE || k == C_DEEP) {
            for (int v = 0; v < 10; v++)
                m[10 * c + v] = NAN;
            continue;
        }
        double f[Q];
        for (int i = 0; i < Q; i++)
            f[i] = a->f[l][i * N + c];
        or_cell_transfer(f, a->omega[l], level_dt(a, l), m + 10 * c);
    }
}

static void prolong(or_amr *a, int l, const double *m0, const double *m1)
{
    int f = l + 1;
    int64_t Nf = (int64_t)a->lnx[f] * a->lny[f] * a->lnz[f];
#pragma omp parallel for schedule(static)
    for (int z = 0; z < a->lnz[f]; z++)
        for (int y = 0; y < a->lny[f]; y++)
            for (int x = 0; x < a->lnx[f]; x++) {
                int64_t c = lidx(a, f, x, y, z);
                if (a->cls[f][c] != C_GHOST)
                    continue;
                int P[3] = {x >> 1, y >> 1, z >> 1}, s[3] = {(x & 1) ? 1 : -1, (y & 1) ? 1 : -1, (z & 1) ? 1 : -1};
                double v[10] = {0};
                for (int q = 0; q < 8; q++) {
                    int o[3] = {q & 1, (q >> 1) & 1, q >> 2};
                    double w = 1.0;
                    int p[3];
                    for (int k = 0; k < 3; k++) {
                        w *= o[k] ? 0.25 : 0.75;
                        p[k] = P[k] + o[k] * s[k];
                    }
                    int64_t pc = lidx(a, l, p[0], p[1], p[2]);
                    for (int t = 0; t < 10; t++) {
                        double val = m1 ? 0.5 * (m0[10 * pc + t] + m1[10 * pc + t]) : m0[10 * pc + t];
                        v[t] += w * val;
                    }
                }
                double fp[Q];
                or_cell_rebuild(v, a->omega[f], level_dt(a, f), fp);
                for (int i = 0; i < Q; i++)
                    a->f[f][i * Nf + c] = fp[i];
            }
}

static void restrict_band(or_amr *a, int l)
{
    int f = l + 1;
    int64_t N = (int64_t)a->lnx[l] * a->lny[l] * a->lnz[l];
    int64_t Nf = (int64_t)a->lnx[f] * a->lny[f] * a->lnz[f];
    int finest = f == a->L - 1;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < a->lnz[l]; z++)
        for (int y = 0; y < a->lny[l]; y++)
            for (int x = 0; x < a->lnx[l]; x++) {
                int64_t c = lidx(a, l, x, y, z);
                if (a->cls[l][c] != C_BAND)
                    continue;
                double rho = 0, mom[3] = {0, 0, 0}, D[6] = {0}, cnt = 0;
                for (int q = 0; q < 8; q++) {
                    int64_t fc = lidx(a, f, 2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2));
                    if (finest && a->solid && a->solid[fc])
                        continue;
                    double fv[Q], t[10];
                    for (int i = 0; i < Q; i++)
                        fv[i] = a->f[f][i * Nf + fc];
                    or_cell_transfer(fv, a->omega[f], level_dt(a, f), t);
                    rho += t[0];
                    for (int k = 0; k < 3; k++)
                        mom[k] += t[0] * t[1 + k];
                    for (int k = 0; k < 6; k++)
                        D[k] += t[4 + k];
                    cnt += 1.0;
                }
                /* a band cell whose children are all solid lies inside the
                 * wall: the fluid at rest (rho = 1, u = 0, D = 0) */
                double v[10] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                if (cnt > 0.0) {
                    v[0] = rho / cnt;
                    for (int k = 0; k < 3; k++)
                        v[1 + k] = mom[k] / rho;
                    for (int k = 0; k < 6; k++)
                        v[4 + k] = D[k] / cnt;
                }
                double fp[Q];
                or_cell_rebuild(v, a->omega[l], level_dt(a, l), fp);
                for (int i = 0; i < Q; i++)
                    a->f[l][i * N + c] = fp[i];
            }
}

/* ---- one step of one level (two arrays, collide then pull) --------------- */

static int in_set(uint8_t k) { return k == C_ACTIVE || k == C_BAND || k == C_GHOST; }

static int find_link(const or_amr *a, int64_t cell, int dir)
{
    for (int64_t s = a->lstart[cell]; s < a->lstart[cell + 1]; s++)
        if (a->ldir[s] == dir)
            return (int)s;
    return -1;
}

static void level_step(or_amr *a, int l)
{
    const int nx = a->lnx[l], ny = a->lny[l], nz = a->lnz[l];
    const int64_t N = (int64_t)nx * ny * nz;
    const int finest = l == a->L - 1;
    const uint8_t *sol = finest ? a->solid : NULL;
    double *fs = a->t[l];
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; c++) {
        double in[Q], out[Q];
        if (!in_set(a->cls[l][c]) || (sol && sol[c]))
            continue;
        for (int i = 0; i < Q; i++)
            in[i] = a->f[l][i * N + c];
        or_collide(in, out, a->omega[l], 1.0, 1.0, a->galilean, NULL);
        for (int i = 0; i < Q; i++)
            fs[i * N + c] = out[i];
    }
    double *fz = (double *)calloc((size_t)nz * 3, sizeof(double));
    double *fbz = (finest && a->n_branch > 0) ? (double *)calloc((size_t)nz * 3 * a->n_branch, sizeof(double)) : NULL;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t c = lidx(a, l, x, y, z);
                if (!in_set(a->cls[l][c]) || (sol && sol[c]))
                    continue;
                for (int i = 0; i < Q; i++) {
                    int sx = x - cxo(i), sy = y - cyo(i), sz = z - czo(i);
                    double val;
                    if (l == 0) {
                        sy = (sy + ny) % ny;
                        sz = (sz + nz) % nz;
                        if (a->periodic_x)
                            sx = (sx + nx) % nx;
                    }
                    if (l == 0 && sx < 0) {
                        double feq[Q], ug[3] = {a->u_in, 0, 0};
                        if (a->inlet && a->steps[0] < a->inlet_n) {
                            const double *du = a->inlet + 3 * ((size_t)a->steps[0] * ny * nz + (size_t)sy + (size_t)ny * sz);
                            ug[0] += du[0];
                            ug[1] += du[1];
                            ug[2] += du[2];
                        }
                        or_equilibrium(1.0, ug, feq);
                        val = feq[i];
                    } else if (l == 0 && sx >= nx) {
                        val = fs[i * N + lidx(a, l, nx - 1, sy, sz)];
                    } else if (sx < 0 || sy < 0 || sz < 0 || sx >= nx || sy >= ny || sz >= nz) {
                        val = NAN;
                    } else {
                        int64_t s = lidx(a, l, sx, sy, sz);
                        if (sol && sol[s]) {
                            int j = Q - 1 - i;
                            int lk = find_link(a, c, j);
                            double q = lk >= 0 ? a->lq[lk] : 0.5;
                            if (lk < 0)
                                a->error = 1;
                            if (q < 0.5) {
                                int ux = x - cxo(j), uy = y - cyo(j), uz = z - czo(j);
                                int64_t uc = lidx(a, l, ux, uy, uz);
                                int ok = ux >= 0 && uy >= 0 && uz >= 0 && ux < nx && uy < ny && uz < nz && !sol[uc] &&
                                         in_set(a->cls[l][uc]);
                                val = ok ? 2.0 * q * fs[j * N + c] + (1.0 - 2.0 * q) * fs[j * N + uc] : fs[j * N + c];
                            } else {
                                val = fs[j * N + c] / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * fs[i * N + c];
                            }
                            double mom = fs[j * N + c] + val - 2.0 * or_weight(j); /* gauge pressure */
                            fz[3 * z + 0] += cxo(j) * mom;
                            fz[3 * z + 1] += cyo(j) * mom;
                            fz[3 * z + 2] += czo(j) * mom;
                            if (fbz && lk >= 0 && a->lbr[lk] >= 0 && a->lbr[lk] < a->n_branch) {
                                double *tt = fbz + ((int64_t)z * a->n_branch + a->lbr[lk]) * 3;
                                tt[0] += cxo(j) * mom;
                                tt[1] += cyo(j) * mom;
                                tt[2] += czo(j) * mom;
                            }
                        } else if (in_set(a->cls[l][s])) {
                            val = fs[i * N + s];
                        } else {
                            val = NAN;
                        }
                    }
                    a->f[l][i * N + c] = val;
                }
            }
    if (finest) {
        double F[3] = {0, 0, 0};
        for (int z = 0; z < nz; z++)
            for (int k = 0; k < 3; k++)
                F[k] += fz[3 * z + k];
        if (a->log_n < a->log_cap) {
            for (int k = 0; k < 3; k++)
                a->force_log[3 * a->log_n + k] = F[k];
            a->log_n++;
        }
        if (a->branch_force) {
            memset(a->branch_force, 0, sizeof(double) * 3 * (size_t)a->n_branch);
            for (int z = 0; z < nz; z++)
                for (int b = 0; b < a->n_branch; b++)
                    for (int k = 0; k < 3; k++)
                        a->branch_force[3 * b + k] += fbz[((int64_t)z * a->n_branch + b) * 3 + k];
        }
        a->finest_steps++;
    }
    free(fz);
    free(fbz);
    a->steps[l]++;
}

static void advance(or_amr *a, int l)
{
    if (l < a->L - 1)
        level_transfer(a, l, a->m0[l]);
    level_step(a, l);
    if (l < a->L - 1) {
        prolong(a, l, a->m0[l], NULL);
        advance(a, l + 1);
        level_transfer(a, l, a->m1[l]);
        prolong(a, l, a->m0[l], a->m1[l]);
        advance(a, l + 1);
        restrict_band(a, l);
    }
}

/* ---- API ------------------------------------------------------------------ */

/* Creates the multi-level state (L = 1 .. OR_MAX_LEVELS).  branches: n rows
 * of 10 doubles; band/wake: L ints each (index = level).  solid/links
 * describe the finest box (solid
 * may be NULL for a grid without a body).  Returns NULL on an invalid
 * refinement. */
or_amr *or_amr_create(int L, int B, int nx, int ny, int nz, double u_in, double nu_f, int galilean,
                      int periodic_x, const double *br, int n, const int *band, const int *wake,
                      const uint8_t *solid, int n_links, const int64_t *lcell, const int8_t *ldir,
                      const double *lq, const int32_t *lbr, int n_branch)
{
    if (L < 1 || L > OR_MAX_LEVELS)
        return NULL;
    or_amr *a = (or_amr *)calloc(1, sizeof(or_amr));
    a->L = L;
    a->B = B;
    a->nx = nx;
    a->ny = ny;
    a->nz = nz;
    a->u_in = u_in;
    a->nu_f = nu_f;
    a->galilean = galilean;
    a->periodic_x = periodic_x;
    for (int l = 0; l < L; l++) {
        int h = 1 << (L - 1 - l);
        a->lnx[l] = nx / h;
        a->lny[l] = ny / h;
        a->lnz[l] = nz / h;
        a->nbx[l] = a->lnx[l] / B;
        a->nby[l] = a->lny[l] / B;
        a->nbz[l] = a->lnz[l] / B;
        a->omega[l] = 1.0 / (3.0 * nu_f / h + 0.5);
    }
    if (build_maps(a, br, n, band, wake) != 0) {
        a->error = 2;
        return a;
    }
    classify(a);
    int64_t Nf = (int64_t)nx * ny * nz;
    if (solid) {
        a->solid = (uint8_t *)malloc((size_t)Nf);
        memcpy(a->solid, solid, (size_t)Nf);
    }
    a->n_links = n_links;
    a->lcell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_links + 1));
    a->ldir = (int8_t *)malloc((size_t)(n_links + 1));
    a->lq = (double *)malloc(sizeof(double) * (size_t)(n_links + 1));
    a->lbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_links + 1));
    if (n_links) {
        memcpy(a->lcell, lcell, sizeof(int64_t) * n_links);
        memcpy(a->ldir, ldir, (size_t)n_links);
        memcpy(a->lq, lq, sizeof(double) * n_links);
        memcpy(a->lbr, lbr, sizeof(int32_t) * n_links);
    }
    /* links are given in (cell, direction) order */
    a->lstart = (int64_t *)calloc((size_t)Nf + 1, sizeof(int64_t));
    for (int k = 0; k < n_links; k++)
        a->lstart[lcell[k] + 1]++;
    for (int64_t c = 0; c < Nf; c++)
        a->lstart[c + 1] += a->lstart[c];
    a->n_branch = n_branch;
    a->branch_force = n_branch > 0 ? (double *)calloc(3 * (size_t)n_branch, sizeof(double)) : NULL;
    a->log_cap = 1 << 20;
    a->force_log = (double *)calloc(3 * (size_t)a->log_cap, sizeof(double));
    for (int l = 0; l < L; l++) {
        int64_t N = (int64_t)a->lnx[l] * a->lny[l] * a->lnz[l];
        a->f[l] = (double *)malloc(sizeof(double) * Q * (size_t)N);
        a->t[l] = (double *)malloc(sizeof(double) * Q * (size_t)N);
        a->m0[l] = (double *)malloc(sizeof(double) * 10 * (size_t)N);
        a->m1[l] = (double *)malloc(sizeof(double) * 10 * (size_t)N);
        double feq[Q], ug[3] = {u_in, 0, 0};
        or_equilibrium(1.0, ug, feq);
        for (int64_t c = 0; c < N; c++) {
            int sol = (l == L - 1 && a->solid && a->solid[c]);
            for (int i = 0; i < Q; i++)
                a->f[l][i * N + c] = sol ? or_weight(i) : feq[i];
        }
        for (int64_t i = 0; i < Q * N; i++)
            a->t[l][i] = NAN;
    }
    return a;
}

int or_amr_error(const or_amr *a) { return a->error; }

void or_amr_destroy(or_amr *a)
{
    if (!a)
        return;
    for (int l = 0; l < a->L; l++) {
        free(a->bmap[l]);
        free(a->cls[l]);
        free(a->f[l]);
        free(a->t[l]);
        free(a->m0[l]);
        free(a->m1[l]);
    }
    free(a->solid);
    free(a->lcell);
    free(a->ldir);
    free(a->lq);
    free(a->lbr);
    free(a->lstart);
    free(a->branch_force);
    free(a->force_log);
    free(a);
}

void or_amr_level_shape(const or_amr *a, int l, int *out6)
{
    out6[0] = a->lnx[l];
    out6[1] = a->lny[l];
    out6[2] = a->lnz[l];
    out6[3] = a->nbx[l];
    out6[4] = a->nby[l];
    out6[5] = a->nbz[l];
}

void or_amr_block_map(const or_amr *a, int l, uint8_t *out)
{
    memcpy(out, a->bmap[l], (size_t)a->nbx[l] * a->nby[l] * a->nbz[l]);
}

void or_amr_classes(const or_amr *a, int l, uint8_t *out)
{
    memcpy(out, a->cls[l], (size_t)a->lnx[l] * a->lny[l] * a->lnz[l]);
}

void or_amr_get_f(const or_amr *a, int l, double *out)
{
    memcpy(out, a->f[l], sizeof(double) * Q * (size_t)a->lnx[l] * a->lny[l] * a->lnz[l]);
}

void or_amr_set_f(or_amr *a, int l, const double *in)
{
    memcpy(a->f[l], in, sizeof(double) * Q * (size_t)a->lnx[l] * a->lny[l] * a->lnz[l]);
}

/* Inlet ghost-plane fluctuations of level-0 steps 0 .. n-1 (Sec. 4.2 inflow
 * turbulence); steps beyond n use the uniform inflow.  The array must outlive
 * the stepping. */
void or_amr_set_inlet(or_amr *a, const double *planes, int64_t n)
{
    a->inlet = planes;
    a->inlet_n = planes ? n : 0;
}

void or_amr_step(or_amr *a, int n_coarse)
{
    for (int s = 0; s < n_coarse; s++)
        advance(a, 0);
}

int64_t or_amr_force_log(const or_amr *a, double *out, int64_t cap)
{
    int64_t m = a->log_n < cap ? a->log_n : cap;
    memcpy(out, a->force_log, sizeof(double) * 3 * (size_t)m);
    return a->log_n;
}

void or_amr_branch_force(const or_amr *a, double *out)
{
    if (a->branch_force)
        memcpy(out, a->branch_force, sizeof(double) * 3 * (size_t)a->n_branch);
}

/* Block maps of every level without the state (the refinement rule of
 * or_amr_create alone), for boxes too large to hold as dense FP64 levels.
 * maps[l] receives level l's map (nbx_l * nby_l * nbz_l values, 0 none,
 * 1 leaf, 2 refined, 3 ghost storage).  Returns 0, or -1 when a refined
 * region comes too close to the box faces. */
int or_amr_maps(int L, int B, int nx, int ny, int nz, const double *br, int n, const int *band, const int *wake,
                uint8_t *const *maps)
{
    if (L < 1 || L > OR_MAX_LEVELS)
        return -1;
    or_amr a;
    memset(&a, 0, sizeof a);
    a.L = L;
    a.B = B;
    for (int l = 0; l < L; l++) {
        int h = 1 << (L - 1 - l);
        a.lnx[l] = nx / h;
        a.lny[l] = ny / h;
        a.lnz[l] = nz / h;
        a.nbx[l] = a.lnx[l] / B;
        a.nby[l] = a.lny[l] / B;
        a.nbz[l] = a.lnz[l] / B;
    }
    int rc = build_maps(&a, br, n, band, wake);
    for (int l = 0; l < L; l++) {
        if (rc == 0 && maps[l])
            memcpy(maps[l], a.bmap[l], (size_t)a.nbx[l] * a.nby[l] * a.nbz[l]);
        free(a.bmap[l]);
    }
    return rc;
}

/* The coupling steps alone, for pinning them on prescribed fields: the
 * prolongation of level l's present populations (read as pre-collision
 * state at time T) into the ghost cells of level l + 1, and the restriction
 * of level l + 1's present populations into the band cells of level l. */
void or_amr_prolong_only(or_amr *a, int l)
{
    level_transfer(a, l, a->m0[l]);
    prolong(a, l, a->m0[l], NULL);
}

void or_amr_restrict_only(or_amr *a, int l) { restrict_band(a, l); }
