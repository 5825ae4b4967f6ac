/*
 * FP64 reference ("oracle") for the D3Q27 cumulant lattice-Boltzmann step of
 * "Drag Crisis in Fractal Trees Revealed by Simulation and Theory".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is built into liblbm_oracle.so, which is
 * loaded only by the test-suite, by the smoke check and by the CPU-baseline leg
 * of the benchmark.  The product library never links, loads or calls it, and
 * the two share no source, header, table or helper.
 *
 * What it follows (paper Sec. 2.2 and Sec. 3):
 *   - D3Q27 velocity set with the cumulant collision the paper adopts (it cites
 *     Geier et al. 2015; the relations below are written out from the
 *     definition of multivariate cumulants of the normalised distribution).
 *   - fully explicit collide-then-stream update (no pressure solve), written
 *     here as two arrays with pull streaming;
 *   - second-order interpolated bounce-back (Bouzidi et al. 2001, linear form)
 *     on the tree surface;
 *   - momentum-exchange force (Wen et al. 2014) summed over the surface and per
 *     branch, feeding C_D of Eq. (7).  Each link contributes
 *     c_j (f*_j + f_opp(j)(t+1) - 2 w_j): the resting state's share sums to zero
 *     over the closed tree (links in directions j and -j pair up on every
 *     lattice line) and is left out so that a branch, whose surface is open
 *     where it joins its parent, carries gauge rather than absolute pressure.
 *
 * Readings where the paper is silent (listed with the rest in the design notes):
 *   relaxation: omega1 from the viscosity, omega2 (bulk) a parameter (1 by
 *   default), one rate omega_high for every cumulant of order >= 3 (1 by
 *   default: those cumulants are reset to zero); Galilean-correction terms of
 *   the second-order relaxation optional.  Boundaries of the box: equilibrium
 *   inlet ghost plane at x = -1, zero-gradient outlet ghost plane at x = nx that
 *   copies the post-collision state of the plane x = nx-1, periodic in y and z
 *   (optionally periodic in x for closed-form tests).  A body force (tests only)
 *   shifts the velocity by F/(2 rho) and flips the first-order central moments.
 *
 * Population index: i = (cx+1) + 3(cy+1) + 9(cz+1), opposite(i) = 26 - i.
 * Arrays of populations are structure-of-arrays: f[i*N + cell] with
 * cell = x + nx*(y + ny*z).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 27

static int cxof(int i) { return i % 3 - 1; }
static int cyof(int i) { return (i / 3) % 3 - 1; }
static int czof(int i) { return i / 9 - 1; }

/* lattice weight: product of the 1D weights 1/6, 2/3, 1/6 */
/* threads of the oracle's parallel loops (for timing it at a given count) */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

double or_weight(int i)
{
    static const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    return w1[i % 3] * w1[(i / 3) % 3] * w1[i / 9];
}

/* Product-form equilibrium: rho * e(cx,ux) e(cy,uy) e(cz,uz) with
 * e(0,a) = 2/3 - a^2 and e(+-1,a) = (1/3 + a^2 +- a)/2.  Its central moments
 * factorise (second order rho/3 on the diagonal), so every cumulant above the
 * second order vanishes. */
void or_equilibrium(double rho, const double *u, double *f)
{
    double e[3][3];
    for (int a = 0; a < 3; a++) {
        double v = u[a];
        e[a][0] = 0.5 * (1.0 / 3.0 + v * v - v);
        e[a][1] = 2.0 / 3.0 - v * v;
        e[a][2] = 0.5 * (1.0 / 3.0 + v * v + v);
    }
    for (int i = 0; i < Q; i++)
        f[i] = rho * e[0][i % 3] * e[1][(i / 3) % 3] * e[2][i / 9];
}

/* Central moments straight from their definition:
 * k[a + 3b + 9g] = sum_i f_i (cx-ux)^a (cy-uy)^b (cz-uz)^g. */
void or_central_moments_direct(const double *f, const double *u, double *k)
{
    for (int g = 0; g < 3; g++)
        for (int b = 0; b < 3; b++)
            for (int a = 0; a < 3; a++) {
                double s = 0.0;
                for (int i = 0; i < Q; i++) {
                    double dx = cxof(i) - u[0], dy = cyof(i) - u[1], dz = czof(i) - u[2];
                    s += f[i] * pow(dx, a) * pow(dy, b) * pow(dz, g);
                }
                k[a + 3 * b + 9 * g] = s;
            }
}

/* One-dimensional central-moment transform of a triple (f-, f0, f+) at
 * velocity a (the factorised "chimera" form of the definition above). */
static void chim_fwd(double *p0, double *p1, double *p2, double a)
{
    double fm = *p0, f0 = *p1, fp = *p2;
    double k0 = fm + f0 + fp;
    double k1 = (fp - fm) - a * k0;
    double k2 = (fp + fm) - 2.0 * a * (fp - fm) + a * a * k0;
    *p0 = k0;
    *p1 = k1;
    *p2 = k2;
}

/* Inverse of chim_fwd. */
static void chim_inv(double *p0, double *p1, double *p2, double a)
{
    double k0 = *p0, k1 = *p1, k2 = *p2;
    double d = k1 + a * k0;                 /* f+ - f- */
    double s = k2 + 2.0 * a * d - a * a * k0; /* f+ + f- */
    *p0 = 0.5 * (s - d);
    *p1 = k0 - s;
    *p2 = 0.5 * (s + d);
}

/* populations -> central moments: z pass, then y, then x */
void or_chimera_forward(const double *f, const double *u, double *k)
{
    double m[Q];
    memcpy(m, f, sizeof m);
    for (int b = 0; b < 9; b++)
        chim_fwd(&m[b], &m[b + 9], &m[b + 18], u[2]);
    for (int g = 0; g < 3; g++)
        for (int a = 0; a < 3; a++)
            chim_fwd(&m[a + 9 * g], &m[a + 3 + 9 * g], &m[a + 6 + 9 * g], u[1]);
    for (int r = 0; r < 9; r++)
        chim_fwd(&m[3 * r], &m[3 * r + 1], &m[3 * r + 2], u[0]);
    memcpy(k, m, sizeof m);
}

/* central moments -> populations: x pass, then y, then z */
void or_chimera_inverse(const double *k, const double *u, double *f)
{
    double m[Q];
    memcpy(m, k, sizeof m);
    for (int r = 0; r < 9; r++)
        chim_inv(&m[3 * r], &m[3 * r + 1], &m[3 * r + 2], u[0]);
    for (int g = 0; g < 3; g++)
        for (int a = 0; a < 3; a++)
            chim_inv(&m[a + 9 * g], &m[a + 3 + 9 * g], &m[a + 6 + 9 * g], u[1]);
    for (int b = 0; b < 9; b++)
        chim_inv(&m[b], &m[b + 9], &m[b + 18], u[2]);
    memcpy(f, m, sizeof m);
}

#define K(a, b, g) k[(a) + 3 * (b) + 9 * (g)]
#define C(a, b, g) c[(a) + 3 * (b) + 9 * (g)]

/* Central moments (about the fluid velocity, first moments taken as zero)
 * -> density-weighted cumulants C = rho * cumulant(f / rho).  Orders 0-3 equal
 * the central moments; orders 4-6 subtract the products over the set
 * partitions of the index multiset (moment-cumulant formula). */
void or_cumulants_from_central(const double *k, double *c)
{
    double r = K(0, 0, 0), ir = 1.0 / r, ir2 = ir * ir;
    memcpy(c, k, Q * sizeof(double));
    /* order 4 */
    C(2, 1, 1) = K(2, 1, 1) - (K(2, 0, 0) * K(0, 1, 1) + 2.0 * K(1, 1, 0) * K(1, 0, 1)) * ir;
    C(1, 2, 1) = K(1, 2, 1) - (K(0, 2, 0) * K(1, 0, 1) + 2.0 * K(1, 1, 0) * K(0, 1, 1)) * ir;
    C(1, 1, 2) = K(1, 1, 2) - (K(0, 0, 2) * K(1, 1, 0) + 2.0 * K(1, 0, 1) * K(0, 1, 1)) * ir;
    C(2, 2, 0) = K(2, 2, 0) - (K(2, 0, 0) * K(0, 2, 0) + 2.0 * K(1, 1, 0) * K(1, 1, 0)) * ir;
    C(2, 0, 2) = K(2, 0, 2) - (K(2, 0, 0) * K(0, 0, 2) + 2.0 * K(1, 0, 1) * K(1, 0, 1)) * ir;
    C(0, 2, 2) = K(0, 2, 2) - (K(0, 2, 0) * K(0, 0, 2) + 2.0 * K(0, 1, 1) * K(0, 1, 1)) * ir;
    /* order 5 */
    C(2, 2, 1) = K(2, 2, 1) - (K(2, 0, 0) * K(0, 2, 1) + K(0, 2, 0) * K(2, 0, 1)
                               + 4.0 * K(1, 1, 0) * K(1, 1, 1)
                               + 2.0 * (K(1, 0, 1) * K(1, 2, 0) + K(0, 1, 1) * K(2, 1, 0))) * ir;
    C(2, 1, 2) = K(2, 1, 2) - (K(2, 0, 0) * K(0, 1, 2) + K(0, 0, 2) * K(2, 1, 0)
                               + 4.0 * K(1, 0, 1) * K(1, 1, 1)
                               + 2.0 * (K(1, 1, 0) * K(1, 0, 2) + K(0, 1, 1) * K(2, 0, 1))) * ir;
    C(1, 2, 2) = K(1, 2, 2) - (K(0, 0, 2) * K(1, 2, 0) + K(0, 2, 0) * K(1, 0, 2)
                               + 4.0 * K(0, 1, 1) * K(1, 1, 1)
                               + 2.0 * (K(1, 0, 1) * K(0, 2, 1) + K(1, 1, 0) * K(0, 1, 2))) * ir;
    /* order 6: 15 pair|quadruple, 10 triple|triple, 15 pair|pair|pair partitions */
    double p24 = K(2, 0, 0) * K(0, 2, 2) + K(0, 2, 0) * K(2, 0, 2) + K(0, 0, 2) * K(2, 2, 0)
                 + 4.0 * (K(1, 1, 0) * K(1, 1, 2) + K(1, 0, 1) * K(1, 2, 1) + K(0, 1, 1) * K(2, 1, 1));
    double p33 = 2.0 * (K(2, 1, 0) * K(0, 1, 2) + K(2, 0, 1) * K(0, 2, 1) + K(1, 2, 0) * K(1, 0, 2))
                 + 4.0 * K(1, 1, 1) * K(1, 1, 1);
    double p222 = K(2, 0, 0) * K(0, 2, 0) * K(0, 0, 2)
                  + 2.0 * (K(2, 0, 0) * K(0, 1, 1) * K(0, 1, 1) + K(0, 2, 0) * K(1, 0, 1) * K(1, 0, 1)
                           + K(0, 0, 2) * K(1, 1, 0) * K(1, 1, 0))
                  + 8.0 * K(1, 1, 0) * K(1, 0, 1) * K(0, 1, 1);
    C(2, 2, 2) = K(2, 2, 2) - (p24 + p33) * ir + 2.0 * p222 * ir2;
}

/* Inverse of or_cumulants_from_central (orders 4, 5, 6 solved in turn). */
void or_central_from_cumulants(const double *c, double *k)
{
    double r = C(0, 0, 0), ir = 1.0 / r, ir2 = ir * ir;
    memcpy(k, c, Q * sizeof(double));
    K(2, 1, 1) = C(2, 1, 1) + (K(2, 0, 0) * K(0, 1, 1) + 2.0 * K(1, 1, 0) * K(1, 0, 1)) * ir;
    K(1, 2, 1) = C(1, 2, 1) + (K(0, 2, 0) * K(1, 0, 1) + 2.0 * K(1, 1, 0) * K(0, 1, 1)) * ir;
    K(1, 1, 2) = C(1, 1, 2) + (K(0, 0, 2) * K(1, 1, 0) + 2.0 * K(1, 0, 1) * K(0, 1, 1)) * ir;
    K(2, 2, 0) = C(2, 2, 0) + (K(2, 0, 0) * K(0, 2, 0) + 2.0 * K(1, 1, 0) * K(1, 1, 0)) * ir;
    K(2, 0, 2) = C(2, 0, 2) + (K(2, 0, 0) * K(0, 0, 2) + 2.0 * K(1, 0, 1) * K(1, 0, 1)) * ir;
    K(0, 2, 2) = C(0, 2, 2) + (K(0, 2, 0) * K(0, 0, 2) + 2.0 * K(0, 1, 1) * K(0, 1, 1)) * ir;
    K(2, 2, 1) = C(2, 2, 1) + (K(2, 0, 0) * K(0, 2, 1) + K(0, 2, 0) * K(2, 0, 1)
                               + 4.0 * K(1, 1, 0) * K(1, 1, 1)
                               + 2.0 * (K(1, 0, 1) * K(1, 2, 0) + K(0, 1, 1) * K(2, 1, 0))) * ir;
    K(2, 1, 2) = C(2, 1, 2) + (K(2, 0, 0) * K(0, 1, 2) + K(0, 0, 2) * K(2, 1, 0)
                               + 4.0 * K(1, 0, 1) * K(1, 1, 1)
                               + 2.0 * (K(1, 1, 0) * K(1, 0, 2) + K(0, 1, 1) * K(2, 0, 1))) * ir;
    K(1, 2, 2) = C(1, 2, 2) + (K(0, 0, 2) * K(1, 2, 0) + K(0, 2, 0) * K(1, 0, 2)
                               + 4.0 * K(0, 1, 1) * K(1, 1, 1)
                               + 2.0 * (K(1, 0, 1) * K(0, 2, 1) + K(1, 1, 0) * K(0, 1, 2))) * ir;
    double p24 = K(2, 0, 0) * K(0, 2, 2) + K(0, 2, 0) * K(2, 0, 2) + K(0, 0, 2) * K(2, 2, 0)
                 + 4.0 * (K(1, 1, 0) * K(1, 1, 2) + K(1, 0, 1) * K(1, 2, 1) + K(0, 1, 1) * K(2, 1, 1));
    double p33 = 2.0 * (K(2, 1, 0) * K(0, 1, 2) + K(2, 0, 1) * K(0, 2, 1) + K(1, 2, 0) * K(1, 0, 2))
                 + 4.0 * K(1, 1, 1) * K(1, 1, 1);
    double p222 = K(2, 0, 0) * K(0, 2, 0) * K(0, 0, 2)
                  + 2.0 * (K(2, 0, 0) * K(0, 1, 1) * K(0, 1, 1) + K(0, 2, 0) * K(1, 0, 1) * K(1, 0, 1)
                           + K(0, 0, 2) * K(1, 1, 0) * K(1, 1, 0))
                  + 8.0 * K(1, 1, 0) * K(1, 0, 1) * K(0, 1, 1);
    K(2, 2, 2) = C(2, 2, 2) + (p24 + p33) * ir - 2.0 * p222 * ir2;
}

/* Relaxation of the cumulants (in place).  Second order: shear rate omega1 on
 * the deviatoric part, bulk rate omega2 on the trace, with the optional
 * Galilean-correction terms built from the velocity-gradient estimates
 * D_xu, D_yv, D_zw that the non-equilibrium second-order cumulants give.
 * Orders 3 to 6 relax towards zero at omega_high. */
void or_relax_cumulants(double *c, const double *u, double omega1, double omega2,
                        double omega_high, int galilean)
{
    double rho = C(0, 0, 0);
    double c200 = C(2, 0, 0), c020 = C(0, 2, 0), c002 = C(0, 0, 2);
    double mxy = c200 - c020, mxz = c200 - c002, axx = c200 + c020 + c002;
    double dxu = -omega1 / (2.0 * rho) * (2.0 * c200 - c020 - c002) - omega2 / (2.0 * rho) * (axx - rho);
    double dyv = dxu + 3.0 * omega1 / (2.0 * rho) * mxy;
    double dzw = dxu + 3.0 * omega1 / (2.0 * rho) * mxz;
    double ux2 = u[0] * u[0], uy2 = u[1] * u[1], uz2 = u[2] * u[2];
    double g = galilean ? 1.0 : 0.0;
    double mxy_s = (1.0 - omega1) * mxy - g * 3.0 * rho * (1.0 - 0.5 * omega1) * (ux2 * dxu - uy2 * dyv);
    double mxz_s = (1.0 - omega1) * mxz - g * 3.0 * rho * (1.0 - 0.5 * omega1) * (ux2 * dxu - uz2 * dzw);
    double a_s = rho + (1.0 - omega2) * (axx - rho)
                 - g * 3.0 * rho * (1.0 - 0.5 * omega2) * (ux2 * dxu + uy2 * dyv + uz2 * dzw);
    C(2, 0, 0) = (mxy_s + mxz_s + a_s) / 3.0;
    C(0, 2, 0) = (a_s - 2.0 * mxy_s + mxz_s) / 3.0;
    C(0, 0, 2) = (a_s + mxy_s - 2.0 * mxz_s) / 3.0;
    C(1, 1, 0) *= (1.0 - omega1);
    C(1, 0, 1) *= (1.0 - omega1);
    C(0, 1, 1) *= (1.0 - omega1);
    for (int g3 = 0; g3 < 3; g3++)
        for (int b = 0; b < 3; b++)
            for (int a = 0; a < 3; a++)
                if (a + b + g3 >= 3)
                    C(a, b, g3) *= (1.0 - omega_high);
}

/* Full cumulant collision of one cell.  force may be NULL. */
void or_collide(const double *fin, double *fout, double omega1, double omega2,
                double omega_high, int galilean, const double *force)
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; i++) {
        rho += fin[i];
        j[0] += cxof(i) * fin[i];
        j[1] += cyof(i) * fin[i];
        j[2] += czof(i) * fin[i];
    }
    double u[3];
    for (int a = 0; a < 3; a++)
        u[a] = (j[a] + (force ? 0.5 * force[a] : 0.0)) / rho;
    double k[Q], c[Q];
    or_chimera_forward(fin, u, k);
    double k1[3] = {K(1, 0, 0), K(0, 1, 0), K(0, 0, 1)};
    or_cumulants_from_central(k, c);
    or_relax_cumulants(c, u, omega1, omega2, omega_high, galilean);
    or_central_from_cumulants(c, k);
    /* momentum: first-order central moments flip sign (zero without force) */
    K(1, 0, 0) = -k1[0];
    K(0, 1, 0) = -k1[1];
    K(0, 0, 1) = -k1[2];
    or_chimera_inverse(k, u, fout);
}

/* ------------------------------------------------------------------------ */
/* uniform grid step                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nx, ny, nz;
    int periodic_x;        /* 1: periodic in x (closed-form tests); 0: inlet/outlet */
    double omega1, omega2, omega_high;
    int galilean;
    double u_in;           /* inlet speed along +x */
    double force[3];       /* body force per cell (tests only) */
    const double *inlet_u; /* optional: velocity fluctuation of the inlet ghost plane, 3*ny*nz, or NULL */
    int lateral_inflow;    /* 1: the y and z faces are inflow faces (ghosts hold f_eq(1, u_in e_x),
                              Sec. 2.3); 0: periodic in y and z */
} or_params;

static inline int64_t cidx(const or_params *p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}

static inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

/* Link lookup: links grouped per fluid cell (compressed rows). */
typedef struct {
    int64_t *start;  /* N+1 */
    int32_t *order;  /* link ids grouped by cell */
} or_link_index;

static void build_link_index(int64_t ncell, int n_links, const int64_t *link_cell, or_link_index *ix)
{
    ix->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    ix->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_links > 0 ? n_links : 1));
    for (int l = 0; l < n_links; l++)
        ix->start[link_cell[l] + 1]++;
    for (int64_t c = 0; c < ncell; c++)
        ix->start[c + 1] += ix->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, ix->start, sizeof(int64_t) * (size_t)ncell);
    for (int l = 0; l < n_links; l++)
        ix->order[fill[link_cell[l]]++] = l;
    free(fill);
}

static int find_link(const or_link_index *ix, const int8_t *link_dir, int64_t cell, int dir)
{
    for (int64_t s = ix->start[cell]; s < ix->start[cell + 1]; s++)
        if (link_dir[ix->order[s]] == dir)
            return ix->order[s];
    return -1;
}

/*
 * One time step f_in -> f_out (both 27*N, SoA).
 * Links: (link_cell, link_dir, link_q, link_branch); link_dir is the direction
 * pointing from the fluid cell into the solid.  Forces on the solid from the
 * momentum exchange of this step are written to force_total[3] and, when
 * force_branch != NULL, to force_branch[3*b].  Returns the number of missing
 * links found (cells next to solid without a link: 0 when the table is whole).
 */
int or_step(const or_params *p, const double *f_in, double *f_out, const uint8_t *solid,
            int n_links, const int64_t *link_cell, const int8_t *link_dir, const double *link_q,
            const int32_t *link_branch, int n_branch, double *force_total, double *force_branch)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const int64_t N = (int64_t)nx * ny * nz;
    double *fs = (double *)malloc(sizeof(double) * (size_t)N * Q);
    const double *F = (p->force[0] != 0.0 || p->force[1] != 0.0 || p->force[2] != 0.0) ? p->force : NULL;

    /* collision */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t c = cidx(p, x, y, z);
                double a[Q], b[Q];
                for (int i = 0; i < Q; i++)
                    a[i] = f_in[i * N + c];
                if (solid && solid[c]) {
                    for (int i = 0; i < Q; i++)
                        b[i] = a[i];
                } else {
                    or_collide(a, b, p->omega1, p->omega2, p->omega_high, p->galilean, F);
                }
                for (int i = 0; i < Q; i++)
                    fs[i * N + c] = b[i];
            }

    or_link_index ix;
    build_link_index(N, n_links, link_cell, &ix);

    double *fz = (double *)calloc((size_t)nz * 3, sizeof(double));
    double *fbz = (force_branch && n_branch > 0) ? (double *)calloc((size_t)nz * 3 * n_branch, sizeof(double)) : NULL;
    int missing = 0;

    /* pull streaming with boundary rules */
#pragma omp parallel for schedule(static) reduction(+ : missing)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t c = cidx(p, x, y, z);
                if (solid && solid[c]) {
                    for (int i = 0; i < Q; i++)
                        f_out[i * N + c] = or_weight(i);
                    continue;
                }
                for (int i = 0; i < Q; i++) {
                    int sx = x - cxof(i), sy = wrap(y - cyof(i), ny), sz = wrap(z - czof(i), nz);
                    double val;
                    if (p->periodic_x)
                        sx = wrap(sx, nx);
                    const int lat = p->lateral_inflow && (y - cyof(i) < 0 || y - cyof(i) >= ny ||
                                                          z - czof(i) < 0 || z - czof(i) >= nz);
                    if (lat) {
                        /* a lateral or vertical inflow face: the ghost holds the
                         * equilibrium of the undisturbed inflow */
                        double ug[3] = {p->u_in, 0.0, 0.0}, feq[Q];
                        or_equilibrium(1.0, ug, feq);
                        val = feq[i];
                    } else if (sx < 0) {
                        double ug[3] = {p->u_in, 0.0, 0.0}, feq[Q];
                        if (p->inlet_u) {
                            const double *du = p->inlet_u + 3 * ((int64_t)sy + (int64_t)ny * sz);
                            ug[0] += du[0];
                            ug[1] += du[1];
                            ug[2] += du[2];
                        }
                        or_equilibrium(1.0, ug, feq);
                        val = feq[i];
                    } else if (sx >= nx) {
                        val = fs[i * N + cidx(p, nx - 1, sy, sz)];
                    } else {
                        int64_t s = cidx(p, sx, sy, sz);
                        if (solid && solid[s]) {
                            /* interpolated bounce-back over link (c, j = opposite(i)) */
                            int j = Q - 1 - i;
                            int l = find_link(&ix, link_dir, c, j);
                            double q = 0.5;
                            if (l < 0)
                                missing++;
                            else
                                q = link_q[l];
                            if (q < 0.5) {
                                int ux = x - cxof(j), uy = wrap(y - cyof(j), ny), uz = wrap(z - czof(j), nz);
                                int ok = 1;
                                if (p->periodic_x)
                                    ux = wrap(ux, nx);
                                if (ux < 0 || ux >= nx)
                                    ok = 0;
                                else if (solid[cidx(p, ux, uy, uz)])
                                    ok = 0;
                                if (ok)
                                    val = 2.0 * q * fs[j * N + c] + (1.0 - 2.0 * q) * fs[j * N + cidx(p, ux, uy, uz)];
                                else
                                    val = fs[j * N + c];
                            } else {
                                val = fs[j * N + c] / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * fs[i * N + c];
                            }
                            /* gauge pressure: the resting state's share 2 w_j drops out
                             * of the total over a closed surface and is removed so that
                             * per-branch sums over open surfaces are meaningful */
                            double mom = fs[j * N + c] + val - 2.0 * or_weight(j);
                            fz[3 * z + 0] += cxof(j) * mom;
                            fz[3 * z + 1] += cyof(j) * mom;
                            fz[3 * z + 2] += czof(j) * mom;
                            if (fbz && l >= 0) {
                                int br = link_branch[l];
                                if (br >= 0 && br < n_branch) {
                                    double *t = fbz + ((int64_t)z * n_branch + br) * 3;
                                    t[0] += cxof(j) * mom;
                                    t[1] += cyof(j) * mom;
                                    t[2] += czof(j) * mom;
                                }
                            }
                        } else {
                            val = fs[i * N + s];
                        }
                    }
                    f_out[i * N + c] = val;
                }
            }

    /* deterministic reduction: z-slab partials added in z order */
    if (force_total) {
        force_total[0] = force_total[1] = force_total[2] = 0.0;
        for (int z = 0; z < nz; z++)
            for (int a = 0; a < 3; a++)
                force_total[a] += fz[3 * z + a];
    }
    if (force_branch && n_branch > 0) {
        memset(force_branch, 0, sizeof(double) * 3 * (size_t)n_branch);
        for (int z = 0; z < nz; z++)
            for (int b = 0; b < n_branch; b++)
                for (int a = 0; a < 3; a++)
                    force_branch[3 * b + a] += fbz[((int64_t)z * n_branch + b) * 3 + a];
    }
    free(fz);
    free(fbz);
    free(ix.start);
    free(ix.order);
    free(fs);
    return missing;
}

/* Macroscopic fields: rho and u = (sum f c + F/2) / rho per cell. */
void or_fields(const double *f, int64_t N, const double *force, double *rho, double *u)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; c++) {
        double r = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
        for (int i = 0; i < Q; i++) {
            double v = f[i * N + c];
            r += v;
            j0 += cxof(i) * v;
            j1 += cyof(i) * v;
            j2 += czof(i) * v;
        }
        rho[c] = r;
        u[3 * c + 0] = (j0 + (force ? 0.5 * force[0] : 0.0)) / r;
        u[3 * c + 1] = (j1 + (force ? 0.5 * force[1] : 0.0)) / r;
        u[3 * c + 2] = (j2 + (force ? 0.5 * force[2] : 0.0)) / r;
    }
}

/* Equilibrium initial state: f_eq(1, (u0,0,0)) in fluid, weights in solid. */
void or_init(int64_t N, const uint8_t *solid, double u0, double *f)
{
    double feq[Q], u[3] = {u0, 0.0, 0.0};
    or_equilibrium(1.0, u, feq);
    for (int64_t c = 0; c < N; c++)
        for (int i = 0; i < Q; i++)
            f[i * N + c] = (solid && solid[c]) ? or_weight(i) : feq[i];
}
