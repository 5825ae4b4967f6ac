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

int tree_generate(const lbm_tree_params &p, std::vector<lbm_branch> &out);
double tree_height(const lbm_branch *b, int n);
void tree_place(lbm_branch *b, int n, double target_h, const double com[3]);
bool tree_fits_box(const lbm_branch *b, int n, int nx, int ny, int nz, double margin);
void voxelize(const lbm_branch *b, int n, int nx, int ny, int nz, std::vector<uint8_t> &solid);
int64_t build_links(const lbm_branch *b, int n, int nx, int ny, int nz, const std::vector<uint8_t> &solid,
                    std::vector<HostLink> &links);
int64_t frontal_area(const std::vector<uint8_t> &solid, int nx, int ny, int nz);
// Outward unit normal of one branch's solid (cylinder p0 -> p1 of diameter D
// and a sphere of diameter D at p1) at a point x of its surface: the normal
// of the nearest of the cylinder side, the end sphere and the base disc.
void branch_wall_normal(const lbm_branch &b, const double x[3], double n[3]);

}  // namespace lbm
