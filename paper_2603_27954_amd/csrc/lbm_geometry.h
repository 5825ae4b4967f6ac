// Host geometry of liblbmtree (trees, voxels, links).  Internal.
#pragma once
#include <stdint.h>

#include <vector>

#include "../../include/lbmtree.h"

namespace lbm {

struct HostLink {
    int64_t cell;   // finest-box cell index of the fluid cell x_f
    int8_t dir;     // direction from x_f into the solid
    double q;       // wall distance fraction along the link, (0, 1]
    int32_t branch; // branch entered first
    bool up_fluid;  // x_f - c_dir is fluid and inside the box
};

// Solid cells of the finest box.  Only the box bounding the tree's solid
// (clipped to the finest box) is stored: every cell outside it is fluid, so a
// finest box of any size costs the tree's own extent.
struct SolidMask {
    int nx = 0, ny = 0, nz = 0;  // finest box
    int o[3] = {0, 0, 0};        // first stored cell
    int s[3] = {0, 0, 0};        // stored extent (zero: no solid)
    std::vector<uint8_t> m;      // x fastest over the stored box
    bool operator()(int x, int y, int z) const
    {
        x -= o[0];
        y -= o[1];
        z -= o[2];
        if ((unsigned)x >= (unsigned)s[0] || (unsigned)y >= (unsigned)s[1] || (unsigned)z >= (unsigned)s[2])
            return false;
        return m[(size_t)x + (size_t)s[0] * ((size_t)y + (size_t)s[1] * z)] != 0;
    }
    // by finest-box cell index x + nx (y + ny z)
    bool cell(int64_t c) const
    {
        return (*this)((int)(c % nx), (int)((c / nx) % ny), (int)(c / ((int64_t)nx * ny)));
    }
    int64_t count() const;
    // the whole finest box, x fastest (nx * ny * nz bytes)
    void expand(uint8_t *dense) const;
};

int tree_generate(const lbm_tree_params &p, std::vector<lbm_branch> &out);
double tree_height(const lbm_branch *b, int n);
void tree_place(lbm_branch *b, int n, double target_h, const double com[3]);
// A branch parallel to y whose axis runs past both y faces by its radius plus
// margin: within the box it is the same at every y, so a periodic y wrap keeps
// it whole (an infinitely long cylinder).
bool spans_y(const lbm_branch &b, int ny, double margin);
// every branch at least margin inside the box; with y_spans_ok, branches that
// span y are exempt from the y test
bool tree_fits_box(const lbm_branch *b, int n, int nx, int ny, int nz, double margin, bool y_spans_ok = false);
void voxelize(const lbm_branch *b, int n, int nx, int ny, int nz, SolidMask &solid);
int64_t build_links(const lbm_branch *b, int n, const SolidMask &solid, std::vector<HostLink> &links);
int64_t frontal_area(const SolidMask &solid);
// Outward unit normal of one branch's solid (cylinder p0 -> p1 of diameter D
// and a sphere of diameter D at p1) at a point x of its surface: the normal
// of the nearest of the cylinder side, the end sphere and the base disc.
void branch_wall_normal(const lbm_branch &b, const double x[3], double n[3]);

}  // namespace lbm
