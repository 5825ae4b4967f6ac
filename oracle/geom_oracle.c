/*
 * FP64 reference geometry: L-system fractal trees, voxelisation, boundary
 * links with their wall distance q, frontal area.
 *
 * TEST INFRASTRUCTURE ONLY (built into liblbm_oracle.so; never linked by the
 * product library and sharing no source with it).
 *
 * Follows paper Sec. 2.1: the parametric L-system of Eq. (1) read by a turtle
 * with frame (H, L, U), H x L = U (Table 1 symbols: "+" rotates about U, "/"
 * about H, "[" / "]" push and pop the state, "!(w)" sets the diameter, "F(s)"
 * draws a cylinder of length s).  Each tree is rescaled to a given height with
 * its proportions kept, and its centre of mass placed at a given point
 * (Sec. 2.3 puts it at (8H, 8H, 8H) of a 32H x 16H x 16H box).
 *
 * Readings: the turtle starts at the origin with H = +z, L = +y, U = -x;
 * "+(a)": H' = H cos a + L sin a, L' = -H sin a + L cos a; "/(p)":
 * L' = L cos p + U sin p, U' = -L sin p + U cos p.  Child j of a node applies
 * roll(pre_roll[j]), pitch(pitch[j] + jitter draw), roll(post_roll[j]) and then
 * draws F(s * len_ratio[j]) with diameter w * wid_ratio[j].  "order" counts the
 * child generations below the trunk.  Jitter draws come from SplitMix64 (Steele,
 * Lea and Flood 2014), one per child in depth-first pre-order; the draw is the
 * top 53 bits scaled to [0,1), jitter angle = jitter * (2 xi - 1) degrees.
 * The solid is the union of the finite cylinders and of a sphere of the
 * branch diameter at each branch end; a cell is solid when its centre
 * (integer + 1/2) lies strictly inside.  Height = highest branch end above
 * the trunk base; centre of mass = volume-weighted over the cylinders.
 *
 * Branch record (10 doubles): p0[3], p1[3], diameter, generation, parent, id.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int m;                /* children per node (<= 4) */
    int order;            /* child generations below the trunk */
    double s0, w0;        /* trunk length and diameter */
    double len_ratio[4], wid_ratio[4];
    double pre_roll[4], pitch[4], post_roll[4]; /* degrees */
    double jitter;        /* +- degrees on the pitch, 0 = none */
    uint64_t seed;
} or_tree_params;

static uint64_t sm64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double or_splitmix_uniform(uint64_t *state) { return (double)(sm64_next(state) >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
    double P[3], H[3], L[3], U[3];
} turtle;

static void rot_pitch(turtle *t, double deg)
{
    double a = deg * M_PI / 180.0, ca = cos(a), sa = sin(a);
    for (int k = 0; k < 3; k++) {
        double h = t->H[k], l = t->L[k];
        t->H[k] = h * ca + l * sa;
        t->L[k] = -h * sa + l * ca;
    }
}

static void rot_roll(turtle *t, double deg)
{
    double a = deg * M_PI / 180.0, ca = cos(a), sa = sin(a);
    for (int k = 0; k < 3; k++) {
        double l = t->L[k], u = t->U[k];
        t->L[k] = l * ca + u * sa;
        t->U[k] = -l * sa + u * ca;
    }
}

typedef struct {
    const or_tree_params *p;
    double *out;
    int cap, n;
    uint64_t rng;
} gen_ctx;

static void grow(gen_ctx *g, turtle t, double s, double w, int gen, int parent)
{
    int id = g->n++;
    if (id < g->cap) {
        double *b = g->out + 10 * id;
        for (int k = 0; k < 3; k++) {
            b[k] = t.P[k];
            b[3 + k] = t.P[k] + s * t.H[k];
        }
        b[6] = w;
        b[7] = gen;
        b[8] = parent;
        b[9] = id;
    }
    for (int k = 0; k < 3; k++)
        t.P[k] += s * t.H[k];
    if (gen >= g->p->order)
        return;
    for (int j = 0; j < g->p->m; j++) {
        turtle c = t;
        double jit = 0.0;
        if (g->p->jitter != 0.0)
            jit = g->p->jitter * (2.0 * or_splitmix_uniform(&g->rng) - 1.0);
        rot_roll(&c, g->p->pre_roll[j]);
        rot_pitch(&c, g->p->pitch[j] + jit);
        rot_roll(&c, g->p->post_roll[j]);
        grow(g, c, s * g->p->len_ratio[j], w * g->p->wid_ratio[j], gen + 1, id);
    }
}

/* Generates the raw tree (trunk base at the origin).  Returns the number of
 * branches (records beyond cap are counted, not written). */
int or_tree_generate(const or_tree_params *p, double *out, int cap)
{
    gen_ctx g = {p, out, cap, 0, p->seed};
    turtle t = {{0, 0, 0}, {0, 0, 1}, {0, 1, 0}, {-1, 0, 0}};
    grow(&g, t, p->s0, p->w0, 0, -1);
    return g.n;
}

/* Height of the tree: highest branch end point above the trunk base. */
double or_tree_height(const double *b, int n)
{
    double base = b[2], top = b[2];
    for (int i = 0; i < n; i++) {
        const double *r = b + 10 * i;
        if (r[2] > top)
            top = r[2];
        if (r[5] > top)
            top = r[5];
    }
    return top - base;
}

/* Scales the tree (about the trunk base) to height target_h when > 0, then
 * translates it so the cylinder-volume centre of mass sits at com[3]. */
void or_tree_place(double *b, int n, double target_h, const double *com)
{
    double s = target_h > 0.0 ? target_h / or_tree_height(b, n) : 1.0;
    double o[3] = {b[0], b[1], b[2]};
    for (int i = 0; i < n; i++) {
        double *r = b + 10 * i;
        for (int k = 0; k < 3; k++) {
            r[k] = o[k] + s * (r[k] - o[k]);
            r[3 + k] = o[k] + s * (r[3 + k] - o[k]);
        }
        r[6] *= s;
    }
    double vs = 0.0, m[3] = {0, 0, 0};
    for (int i = 0; i < n; i++) {
        double *r = b + 10 * i;
        double dx = r[3] - r[0], dy = r[4] - r[1], dz = r[5] - r[2];
        double len = sqrt(dx * dx + dy * dy + dz * dz);
        double v = M_PI * 0.25 * r[6] * r[6] * len;
        vs += v;
        for (int k = 0; k < 3; k++)
            m[k] += v * 0.5 * (r[k] + r[3 + k]);
    }
    for (int k = 0; k < 3; k++)
        m[k] = com[k] - m[k] / vs;
    for (int i = 0; i < n; i++) {
        double *r = b + 10 * i;
        for (int k = 0; k < 3; k++) {
            r[k] += m[k];
            r[3 + k] += m[k];
        }
    }
}

/* point strictly inside branch i (cylinder or end sphere) */
static int inside_branch(const double *r, const double *pt)
{
    double a[3] = {r[3] - r[0], r[4] - r[1], r[5] - r[2]};
    double len2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    double R = 0.5 * r[6], R2 = R * R;
    double v[3] = {pt[0] - r[0], pt[1] - r[1], pt[2] - r[2]};
    double e[3] = {pt[0] - r[3], pt[1] - r[4], pt[2] - r[5]};
    if (e[0] * e[0] + e[1] * e[1] + e[2] * e[2] < R2)
        return 1;
    double t = (v[0] * a[0] + v[1] * a[1] + v[2] * a[2]);
    if (t <= 0.0 || t >= len2)
        return 0;
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double d2 = vv - t * t / len2;
    return d2 < R2;
}

/* Brute force: every cell centre against every branch. */
void or_voxelize(const double *b, int n, int nx, int ny, int nz, uint8_t *solid)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                double pt[3] = {x + 0.5, y + 0.5, z + 0.5};
                uint8_t s = 0;
                for (int i = 0; i < n && !s; i++)
                    s = (uint8_t)inside_branch(b + 10 * i, pt);
                solid[(int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z)] = s;
            }
}

/* Entry parameter of the ray o + t d into branch i (open interval of inside
 * points); returns +inf when the ray never enters. */
static double entry_branch(const double *r, const double *o, const double *d)
{
    double best = INFINITY;
    /* end sphere */
    {
        double R = 0.5 * r[6];
        double w[3] = {o[0] - r[3], o[1] - r[4], o[2] - r[5]};
        double A = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double B = 2.0 * (w[0] * d[0] + w[1] * d[1] + w[2] * d[2]);
        double Cc = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] - R * R;
        double disc = B * B - 4.0 * A * Cc;
        if (disc > 0.0) {
            double sq = sqrt(disc);
            double t0 = (-B - sq) / (2.0 * A), t1 = (-B + sq) / (2.0 * A);
            if (t1 > 0.0)
                best = t0 > 0.0 ? t0 : 0.0;
        }
    }
    /* finite cylinder: axial slab intersected with the infinite cylinder */
    {
        double a[3] = {r[3] - r[0], r[4] - r[1], r[5] - r[2]};
        double len = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        for (int k = 0; k < 3; k++)
            a[k] /= len;
        double R = 0.5 * r[6];
        double w[3] = {o[0] - r[0], o[1] - r[1], o[2] - r[2]};
        double wa = w[0] * a[0] + w[1] * a[1] + w[2] * a[2];
        double da = d[0] * a[0] + d[1] * a[1] + d[2] * a[2];
        double lo = -INFINITY, hi = INFINITY;
        if (da != 0.0) {
            double t0 = (0.0 - wa) / da, t1 = (len - wa) / da;
            lo = t0 < t1 ? t0 : t1;
            hi = t0 < t1 ? t1 : t0;
        } else if (!(wa > 0.0 && wa < len)) {
            lo = INFINITY;
            hi = -INFINITY;
        }
        double r0[3], r1[3];
        for (int k = 0; k < 3; k++) {
            r0[k] = w[k] - wa * a[k];
            r1[k] = d[k] - da * a[k];
        }
        double A = r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2];
        double B = 2.0 * (r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2]);
        double Cc = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2] - R * R;
        double clo, chi;
        if (A == 0.0) {
            clo = Cc < 0.0 ? -INFINITY : INFINITY;
            chi = Cc < 0.0 ? INFINITY : -INFINITY;
        } else {
            double disc = B * B - 4.0 * A * Cc;
            if (disc > 0.0) {
                double sq = sqrt(disc);
                clo = (-B - sq) / (2.0 * A);
                chi = (-B + sq) / (2.0 * A);
            } else {
                clo = INFINITY;
                chi = -INFINITY;
            }
        }
        double L0 = lo > clo ? lo : clo, H0 = hi < chi ? hi : chi;
        if (L0 < H0 && H0 > 0.0) {
            double t = L0 > 0.0 ? L0 : 0.0;
            if (t < best)
                best = t;
        }
    }
    return best;
}

/*
 * Boundary links of the fluid next to the tree: every fluid cell x and
 * direction i (0..26, i = (cx+1) + 3(cy+1) + 9(cz+1)) with x + c_i solid, in
 * order of (cell index, direction).  Neighbours wrap periodically in y and z;
 * neighbours outside the box in x are not solid.  q = first entry parameter of
 * the segment x -> x + c_i into the union of the branch shapes (clamped to
 * (0, 1]); the branch is the one whose shape is entered first (lowest id on a
 * tie).  Arrays are written up to cap entries; returns the number of links.
 */
int64_t or_links(const double *b, int n, int nx, int ny, int nz, const uint8_t *solid, int64_t cap,
                 int64_t *lcell, int8_t *ldir, double *lq, int32_t *lbranch)
{
    int64_t cnt = 0;
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t c = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
                if (solid[c])
                    continue;
                for (int i = 0; i < 27; i++) {
                    int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
                    if (i == 13)
                        continue;
                    int sx = x + cx, sy = (y + cy + ny) % ny, sz = (z + cz + nz) % nz;
                    if (sx < 0 || sx >= nx)
                        continue;
                    if (!solid[(int64_t)sx + (int64_t)nx * ((int64_t)sy + (int64_t)ny * sz)])
                        continue;
                    double o[3] = {x + 0.5, y + 0.5, z + 0.5}, d[3] = {cx, cy, cz};
                    double best = INFINITY;
                    int bb = -1;
                    for (int k = 0; k < n; k++) {
                        double t = entry_branch(b + 10 * k, o, d);
                        if (t < best) {
                            best = t;
                            bb = k;
                        }
                    }
                    if (!(best <= 1.0))
                        best = 1.0;
                    if (best <= 0.0)
                        best = 1e-12;
                    if (cnt < cap) {
                        lcell[cnt] = c;
                        ldir[cnt] = (int8_t)i;
                        lq[cnt] = best;
                        lbranch[cnt] = bb >= 0 ? (int32_t)b[10 * bb + 9] : -1;
                    }
                    cnt++;
                }
            }
    return cnt;
}

/* Frontal area: number of (y, z) columns holding at least one solid cell. */
int64_t or_area_x(const uint8_t *solid, int nx, int ny, int nz)
{
    int64_t a = 0;
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++) {
            int any = 0;
            for (int x = 0; x < nx && !any; x++)
                any = solid[(int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z)];
            a += any;
        }
    return a;
}
