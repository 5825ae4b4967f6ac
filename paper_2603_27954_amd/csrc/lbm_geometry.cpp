// Host geometry for liblbmtree: L-system trees (paper Sec. 2.1, Eq. (1),
// Table 1), placement (Sec. 2.3), voxelisation of the union of branch shapes,
// boundary links with their wall distance q (interpolated bounce-back,
// Sec. 2.2) and the frontal area A_x of Eq. (7).
//
// Turtle conventions: start at the origin with heading H = +z, left L = +y,
// up U = H x L = -x.  Pitch "+(a)" turns H towards L about U; roll "/(p)"
// turns L towards U about H.  Child j of an apex rolls by pre_roll[j], pitches
// by pitch[j] (plus a jitter draw), rolls by post_roll[j] and draws
// F(s len_ratio[j]) with diameter w wid_ratio[j].  Jitter draws come from
// SplitMix64 (Steele, Lea & Flood 2014), one per child, in depth-first
// pre-order of the children.
#include "lbm_geometry.h"
#include "lbm_random.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace lbm {

namespace {

struct V3 {
    double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

struct Frame {
    V3 pos, head, left, up;
};

Frame pitch(Frame f, double deg)
{
    const double r = deg * (M_PI / 180.0), c = std::cos(r), s = std::sin(r);
    const V3 h = f.head, l = f.left;
    f.head = c * h + s * l;
    f.left = c * l - s * h;
    return f;
}

Frame roll(Frame f, double deg)
{
    const double r = deg * (M_PI / 180.0), c = std::cos(r), s = std::sin(r);
    const V3 l = f.left, u = f.up;
    f.left = c * l + s * u;
    f.up = c * u - s * l;
    return f;
}

}  // namespace

int tree_generate(const lbm_tree_params &p, std::vector<lbm_branch> &out)
{
    struct Pending {
        Frame parent_end;  // frame at the end of the parent branch
        double s, w;       // parent's length and diameter
        int gen, parent, child;
    };
    out.clear();
    SplitMix64 rng{p.seed};
    std::vector<Pending> stack;
    // trunk
    {
        Frame f{{0, 0, 0}, {0, 0, 1}, {0, 1, 0}, {-1, 0, 0}};
        lbm_branch b{};
        const V3 e = f.pos + p.s0 * f.head;
        b.p0[0] = f.pos.x, b.p0[1] = f.pos.y, b.p0[2] = f.pos.z;
        b.p1[0] = e.x, b.p1[1] = e.y, b.p1[2] = e.z;
        b.diameter = p.w0;
        b.generation = 0;
        b.parent = -1;
        b.id = 0;
        out.push_back(b);
        f.pos = e;
        if (p.order > 0)
            for (int j = p.m - 1; j >= 0; --j)
                stack.push_back({f, p.s0, p.w0, 1, 0, j});
    }
    while (!stack.empty()) {
        const Pending pe = stack.back();
        stack.pop_back();
        const int j = pe.child;
        const double jit = p.jitter != 0.0 ? p.jitter * (2.0 * rng.uniform() - 1.0) : 0.0;
        Frame f = roll(pe.parent_end, p.pre_roll[j]);
        f = pitch(f, p.pitch[j] + jit);
        f = roll(f, p.post_roll[j]);
        const double s = pe.s * p.len_ratio[j], w = pe.w * p.wid_ratio[j];
        const V3 e = f.pos + s * f.head;
        lbm_branch b{};
        b.p0[0] = f.pos.x, b.p0[1] = f.pos.y, b.p0[2] = f.pos.z;
        b.p1[0] = e.x, b.p1[1] = e.y, b.p1[2] = e.z;
        b.diameter = w;
        b.generation = pe.gen;
        b.parent = pe.parent;
        b.id = (int32_t)out.size();
        out.push_back(b);
        f.pos = e;
        if (pe.gen < p.order)
            for (int c = p.m - 1; c >= 0; --c)
                stack.push_back({f, s, w, pe.gen + 1, b.id, c});
    }
    return (int)out.size();
}

double tree_height(const lbm_branch *b, int n)
{
    double top = b[0].p0[2];
    for (int i = 0; i < n; ++i)
        top = std::max(top, std::max(b[i].p0[2], b[i].p1[2]));
    return top - b[0].p0[2];
}

void tree_place(lbm_branch *b, int n, double target_h, const double com[3])
{
    const double h = tree_height(b, n);
    const double sc = (target_h > 0.0 && h > 0.0) ? target_h / h : 1.0;
    const double o[3] = {b[0].p0[0], b[0].p0[1], b[0].p0[2]};
    double vol = 0.0, m[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            b[i].p0[a] = o[a] + sc * (b[i].p0[a] - o[a]);
            b[i].p1[a] = o[a] + sc * (b[i].p1[a] - o[a]);
        }
        b[i].diameter *= sc;
        const double dx = b[i].p1[0] - b[i].p0[0], dy = b[i].p1[1] - b[i].p0[1], dz = b[i].p1[2] - b[i].p0[2];
        const double v = 0.25 * M_PI * b[i].diameter * b[i].diameter * std::sqrt(dx * dx + dy * dy + dz * dz);
        vol += v;
        for (int a = 0; a < 3; ++a)
            m[a] += v * 0.5 * (b[i].p0[a] + b[i].p1[a]);
    }
    for (int a = 0; a < 3; ++a) {
        const double shift = com[a] - m[a] / vol;
        for (int i = 0; i < n; ++i) {
            b[i].p0[a] += shift;
            b[i].p1[a] += shift;
        }
    }
}

// ---------------------------------------------------------------------------
// shapes
// ---------------------------------------------------------------------------

namespace {

struct Shape {
    V3 p0, p1, axis;   // axis: unit vector p0 -> p1
    double len, r, r2;
    int id;
    double lo[3], hi[3];  // bounding box
};

Shape make_shape(const lbm_branch &b)
{
    Shape s;
    s.p0 = {b.p0[0], b.p0[1], b.p0[2]};
    s.p1 = {b.p1[0], b.p1[1], b.p1[2]};
    const V3 d = s.p1 - s.p0;
    s.len = std::sqrt(dot(d, d));
    s.axis = (1.0 / s.len) * d;
    s.r = 0.5 * b.diameter;
    s.r2 = s.r * s.r;
    s.id = b.id;
    const double p0[3] = {s.p0.x, s.p0.y, s.p0.z}, p1[3] = {s.p1.x, s.p1.y, s.p1.z};
    for (int a = 0; a < 3; ++a) {
        s.lo[a] = std::min(p0[a], p1[a]) - s.r;
        s.hi[a] = std::max(p0[a], p1[a]) + s.r;
    }
    return s;
}

// strictly inside the cylinder (open axial range) or the end sphere
bool inside(const Shape &s, V3 pt)
{
    const V3 e = pt - s.p1;
    if (dot(e, e) < s.r2)
        return true;
    const V3 v = pt - s.p0;
    const double along = dot(v, s.axis);
    if (!(along > 0.0 && along < s.len))
        return false;
    const V3 perp = v - along * s.axis;
    return dot(perp, perp) < s.r2;
}

// first parameter t >= 0 at which o + t d is inside the shape (inf if never)
double entry(const Shape &s, V3 o, V3 d)
{
    double best = std::numeric_limits<double>::infinity();
    // sphere
    {
        const V3 w = o - s.p1;
        const double A = dot(d, d), Bh = dot(w, d), C = dot(w, w) - s.r2;
        const double disc = Bh * Bh - A * C;
        if (disc > 0.0) {
            const double sq = std::sqrt(disc);
            const double t0 = (-Bh - sq) / A, t1 = (-Bh + sq) / A;
            if (t1 > 0.0)
                best = std::max(t0, 0.0);
        }
    }
    // cylinder: slab along the axis intersected with the radial interval
    {
        const V3 w = o - s.p0;
        const double wa = dot(w, s.axis), da = dot(d, s.axis);
        double lo, hi;
        if (da != 0.0) {
            const double ta = -wa / da, tb = (s.len - wa) / da;
            lo = std::min(ta, tb);
            hi = std::max(ta, tb);
        } else if (wa > 0.0 && wa < s.len) {
            lo = -std::numeric_limits<double>::infinity();
            hi = std::numeric_limits<double>::infinity();
        } else {
            return best;
        }
        const V3 r0 = w - wa * s.axis, r1 = d - da * s.axis;
        const double A = dot(r1, r1), Bh = dot(r0, r1), C = dot(r0, r0) - s.r2;
        double clo, chi;
        if (A == 0.0) {
            if (C >= 0.0)
                return best;
            clo = -std::numeric_limits<double>::infinity();
            chi = std::numeric_limits<double>::infinity();
        } else {
            const double disc = Bh * Bh - A * C;
            if (disc <= 0.0)
                return best;
            const double sq = std::sqrt(disc);
            clo = (-Bh - sq) / A;
            chi = (-Bh + sq) / A;
        }
        const double a = std::max(lo, clo), b = std::min(hi, chi);
        if (a < b && b > 0.0)
            best = std::min(best, std::max(a, 0.0));
    }
    return best;
}

}  // namespace

// Exact extent of branch i along axis a: the cylinder's end discs reach
// r sqrt(1 - axis_a^2) beyond the axis ends, the end sphere r beyond p1.
static void branch_extent(const Shape &s, int a, double *lo, double *hi)
{
    const double p0[3] = {s.p0.x, s.p0.y, s.p0.z}, p1[3] = {s.p1.x, s.p1.y, s.p1.z};
    const double ax[3] = {s.axis.x, s.axis.y, s.axis.z};
    const double disc = s.r * std::sqrt(std::max(0.0, 1.0 - ax[a] * ax[a]));
    *lo = std::min(std::min(p0[a], p1[a]) - disc, p1[a] - s.r);
    *hi = std::max(std::max(p0[a], p1[a]) + disc, p1[a] + s.r);
}

bool spans_y(const lbm_branch &b, int ny, double margin)
{
    const double r = 0.5 * b.diameter;
    return b.p0[0] == b.p1[0] && b.p0[2] == b.p1[2] && std::min(b.p0[1], b.p1[1]) <= -r - margin &&
           std::max(b.p0[1], b.p1[1]) >= ny + r + margin;
}

bool tree_fits_box(const lbm_branch *b, int n, int nx, int ny, int nz, double margin, bool y_spans_ok)
{
    const double ext[3] = {(double)nx, (double)ny, (double)nz};
    for (int i = 0; i < n; ++i) {
        const Shape s = make_shape(b[i]);
        const bool span = y_spans_ok && spans_y(b[i], ny, margin);
        for (int a = 0; a < 3; ++a) {
            if (a == 1 && span)
                continue;
            double lo, hi;
            branch_extent(s, a, &lo, &hi);
            if (lo < margin || hi > ext[a] - margin)
                return false;
        }
    }
    return true;
}

int64_t SolidMask::count() const
{
    int64_t c = 0;
    for (uint8_t v : m)
        c += v != 0;
    return c;
}

void SolidMask::expand(uint8_t *dense) const
{
    std::memset(dense, 0, (size_t)nx * ny * nz);
    for (int z = 0; z < s[2]; ++z)
        for (int y = 0; y < s[1]; ++y)
            std::memcpy(dense + (size_t)o[0] + (size_t)nx * ((size_t)(o[1] + y) + (size_t)ny * (o[2] + z)),
                        m.data() + (size_t)s[0] * ((size_t)y + (size_t)s[1] * z), (size_t)s[0]);
}

void voxelize(const lbm_branch *b, int n, int nx, int ny, int nz, SolidMask &solid)
{
    solid = SolidMask{};
    solid.nx = nx;
    solid.ny = ny;
    solid.nz = nz;
    const int ext[3] = {nx, ny, nz};
    std::vector<Shape> shapes;
    int blo[3] = {ext[0], ext[1], ext[2]}, bhi[3] = {-1, -1, -1};
    for (int i = 0; i < n; ++i) {
        shapes.push_back(make_shape(b[i]));
        for (int a = 0; a < 3; ++a) {
            blo[a] = std::min(blo[a], std::max(0, (int)std::floor(shapes.back().lo[a] - 0.5)));
            bhi[a] = std::max(bhi[a], std::min(ext[a] - 1, (int)std::ceil(shapes.back().hi[a] - 0.5)));
        }
    }
    if (n == 0 || blo[0] > bhi[0] || blo[1] > bhi[1] || blo[2] > bhi[2])
        return;
    for (int a = 0; a < 3; ++a) {
        solid.o[a] = blo[a];
        solid.s[a] = bhi[a] - blo[a] + 1;
    }
    solid.m.assign((size_t)solid.s[0] * solid.s[1] * solid.s[2], 0);
    for (const Shape &sh : shapes) {
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::max(0, (int)std::floor(sh.lo[a] - 0.5));
            hi[a] = std::min(ext[a] - 1, (int)std::ceil(sh.hi[a] - 0.5));
        }
#pragma omp parallel for schedule(static)
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    uint8_t &c = solid.m[(size_t)(x - solid.o[0]) +
                                         (size_t)solid.s[0] * ((size_t)(y - solid.o[1]) + (size_t)solid.s[1] * (z - solid.o[2]))];
                    if (!c && inside(sh, {x + 0.5, y + 0.5, z + 0.5}))
                        c = 1;
                }
    }
}

int64_t build_links(const lbm_branch *b, int n, const SolidMask &solid, std::vector<HostLink> &links)
{
    const int nx = solid.nx, ny = solid.ny, nz = solid.nz;
    std::vector<Shape> shapes;
    shapes.reserve(n);
    for (int i = 0; i < n; ++i)
        shapes.push_back(make_shape(b[i]));
    links.clear();
    // only cells within two cells of the tree's bounding box can have links
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    {
        const int ext[3] = {nx, ny, nz};
        for (const Shape &sh : shapes)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], std::max(0, (int)std::floor(sh.lo[a]) - 2));
                hi[a] = std::max(hi[a], std::min(ext[a] - 1, (int)std::ceil(sh.hi[a]) + 2));
            }
    }
    if (n == 0 || lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2])
        return 0;
    // bins of 16 cells over that region listing the shapes whose box reaches
    // into them
    const int BS = 16;
    const int gx = (hi[0] - lo[0]) / BS + 1, gy = (hi[1] - lo[1]) / BS + 1, gz = (hi[2] - lo[2]) / BS + 1;
    std::vector<std::vector<int>> bins((size_t)gx * gy * gz);
    for (int i = 0; i < n; ++i) {
        int blo[3], bhi[3];
        const int g[3] = {gx, gy, gz};
        for (int a = 0; a < 3; ++a) {
            blo[a] = std::max(0, (int)std::floor((shapes[i].lo[a] - 2.0 - lo[a]) / BS));
            bhi[a] = std::min(g[a] - 1, (int)std::floor((shapes[i].hi[a] + 2.0 - lo[a]) / BS));
        }
        for (int z = blo[2]; z <= bhi[2]; ++z)
            for (int y = blo[1]; y <= bhi[1]; ++y)
                for (int x = blo[0]; x <= bhi[0]; ++x)
                    bins[(size_t)x + (size_t)gx * ((size_t)y + (size_t)gy * z)].push_back(i);
    }
    // cells with a solid cell among their 26 neighbours (y and z wrapped as
    // below), marked from the solid cells: only those can hold links
    const int rx = hi[0] - lo[0] + 1, ry = hi[1] - lo[1] + 1, rz = hi[2] - lo[2] + 1;
    std::vector<uint8_t> near((size_t)rx * ry * rz, 0);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < solid.s[2]; ++z)
        for (int y = 0; y < solid.s[1]; ++y)
            for (int x = 0; x < solid.s[0]; ++x) {
                if (!solid.m[(size_t)x + (size_t)solid.s[0] * ((size_t)y + (size_t)solid.s[1] * z)])
                    continue;
                const int X = solid.o[0] + x, Y = solid.o[1] + y, Z = solid.o[2] + z;
                for (int k = 0; k < 27; ++k) {
                    const int fx = X + k % 3 - 1, fy = (Y + (k / 3) % 3 - 1 + ny) % ny, fz = (Z + k / 9 - 1 + nz) % nz;
                    if (fx < lo[0] || fx > hi[0] || fy < lo[1] || fy > hi[1] || fz < lo[2] || fz > hi[2])
                        continue;
                    // neighbouring slices are marked by several threads: atomic byte stores
                    __atomic_store_n(&near[(size_t)(fx - lo[0]) + (size_t)rx * ((size_t)(fy - lo[1]) + (size_t)ry * (fz - lo[2]))],
                                     (uint8_t)1, __ATOMIC_RELAXED);
                }
            }
    // links per z-slice in parallel, joined in slice order: (cell, direction)
    // order as a serial sweep gives
    std::vector<std::vector<HostLink>> per_z((size_t)rz);
#pragma omp parallel for schedule(dynamic, 4)
    for (int z = lo[2]; z <= hi[2]; ++z) {
        std::vector<HostLink> &out = per_z[(size_t)(z - lo[2])];
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                if (!near[(size_t)(x - lo[0]) + (size_t)rx * ((size_t)(y - lo[1]) + (size_t)ry * (z - lo[2]))])
                    continue;
                const int64_t c = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
                if (solid(x, y, z))
                    continue;
                for (int i = 0; i < 27; ++i) {
                    if (i == 13)
                        continue;
                    const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
                    const int sx = x + cx;
                    if (sx < 0 || sx >= nx)
                        continue;
                    const int sy = (y + cy + ny) % ny, sz = (z + cz + nz) % nz;
                    if (!solid(sx, sy, sz))
                        continue;
                    HostLink L;
                    L.cell = c;
                    L.dir = (int8_t)i;
                    const V3 o{x + 0.5, y + 0.5, z + 0.5}, d{(double)cx, (double)cy, (double)cz};
                    double best = std::numeric_limits<double>::infinity();
                    int bid = -1;
                    const V3 mid = o + 0.5 * d;
                    const int bxi = std::min(gx - 1, std::max(0, (int)std::floor((mid.x - lo[0]) / BS)));
                    const int byi = std::min(gy - 1, std::max(0, (int)std::floor((mid.y - lo[1]) / BS)));
                    const int bzi = std::min(gz - 1, std::max(0, (int)std::floor((mid.z - lo[2]) / BS)));
                    for (int si : bins[(size_t)bxi + (size_t)gx * ((size_t)byi + (size_t)gy * bzi)]) {
                        const double t = entry(shapes[si], o, d);
                        if (t < best || (t == best && shapes[si].id < bid)) {
                            best = t;
                            bid = shapes[si].id;
                        }
                    }
                    if (!(best <= 1.0))
                        best = 1.0;
                    if (best <= 0.0)
                        best = 1e-12;
                    L.q = best;
                    L.branch = bid;
                    // upstream neighbour x - c_i fluid and inside the box
                    const int ux = x - cx;
                    L.up_fluid = (ux >= 0 && ux < nx) && !solid(ux, (y - cy + ny) % ny, (z - cz + nz) % nz);
                    out.push_back(L);
                }
            }
    }
    for (const std::vector<HostLink> &v : per_z)
        links.insert(links.end(), v.begin(), v.end());
    return (int64_t)links.size();
}

void branch_wall_normal(const lbm_branch &b, const double x[3], double n[3])
{
    const Shape s = make_shape(b);
    const V3 p{x[0], x[1], x[2]};
    const V3 rel = p - s.p0;
    const double along = dot(rel, s.axis);  // distance along the axis from p0
    double best = 1e300;
    V3 nb{0.0, 0.0, 1.0};
    // side of the cylinder
    const V3 radial = rel - along * s.axis;
    const double rr = std::sqrt(dot(radial, radial));
    if (along >= 0.0 && along <= s.len && rr > 0.0) {
        best = std::fabs(rr - s.r);
        nb = (1.0 / rr) * radial;
    }
    // sphere at the end
    const V3 sp = p - s.p1;
    const double rs = std::sqrt(dot(sp, sp));
    if (rs > 0.0 && std::fabs(rs - s.r) < best) {
        best = std::fabs(rs - s.r);
        nb = (1.0 / rs) * sp;
    }
    // base disc at p0
    if (rr <= s.r && std::fabs(along) < best) {
        best = std::fabs(along);
        nb = -1.0 * s.axis;
    }
    n[0] = nb.x;
    n[1] = nb.y;
    n[2] = nb.z;
}

int64_t frontal_area(const SolidMask &solid)
{
    int64_t a = 0;
    for (int z = 0; z < solid.s[2]; ++z)
        for (int y = 0; y < solid.s[1]; ++y) {
            const uint8_t *row = solid.m.data() + (size_t)solid.s[0] * ((size_t)y + (size_t)solid.s[1] * z);
            a += std::any_of(row, row + solid.s[0], [](uint8_t v) { return v != 0; }) ? 1 : 0;
        }
    return a;
}

}  // namespace lbm
