/*
 * lbmtree — D3Q27 cumulant lattice-Boltzmann drag of L-system fractal trees
 * on MI355X (gfx950).  C ABI of liblbmtree.so.
 *
 * The method is the one of "Drag Crisis in Fractal Trees Revealed by
 * Simulation and Theory":
 *   - tree geometry: parametric L-system of Eq. (1) read by a turtle (Sec. 2.1,
 *     Table 1), rescaled to a height and placed by its centre of mass (Sec. 2.3);
 *   - flow: D3Q27 cumulant collision with fully explicit collide-and-stream on
 *     an octree of cubic leaf blocks, finest near the tree surface, moderate in
 *     the wake, coarse elsewhere (Sec. 2.2);
 *   - wall: second-order interpolated bounce-back (Sec. 2.2, Bouzidi et al.);
 *   - force: momentum exchange summed over the tree surface (Sec. 2.2) and the
 *     drag coefficient C_D = F_D / (rho U^2 A_x / 2) of Eq. (7).
 *
 * Conventions (all functions):
 *   - every call returns an lbm_status; no exception or signal crosses the ABI;
 *     on error lbm_last_error() returns a message (per grid, or per thread when
 *     the grid handle is NULL);
 *   - lengths are in cells of the finest level, velocities in lattice units of
 *     the finest level (the same on every level: acoustic scaling);
 *   - population index i = (cx+1) + 3(cy+1) + 9(cz+1) over c in {-1,0,1}^3,
 *     opposite direction 26 - i;
 *   - dense per-level arrays use cell = x + nx_l*(y + ny_l*z) over the level's
 *     whole box (nx_l = nx >> (levels-1-l), likewise y, z); SoA for populations
 *     (f[i*N + cell]);
 *   - all host pointers are owned by the caller, read or written only during
 *     the call; device memory is allocated and owned by the library, except
 *     the populations when the caller binds its own (lbm_bind_memory);
 *   - one grid handle is used by one host thread at a time.
 */
#ifndef LBMTREE_H
#define LBMTREE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_grid lbm_grid; /* opaque */

typedef enum {
    LBM_OK = 0,
    LBM_E_INVALID = -1,  /* bad argument or description; nothing was changed */
    LBM_E_NOMEM = -2,    /* device or host allocation failed */
    LBM_E_DEVICE = -3,   /* a HIP call failed (message names it) */
    LBM_E_UNSTABLE = -4, /* NaN / density outside [0.5, 1.5] detected */
    LBM_E_STATE = -5     /* call out of order (e.g. step before set_geometry) */
} lbm_status;

typedef enum {
    LBM_FP32 = 0,     /* populations stored as FP32 deviations f_i - w_i */
    LBM_FP16_DEV = 1, /* stored as FP16 deviations f_i - w_i, FP32 arithmetic */
    LBM_BF16_DEV = 2  /* stored as BF16 deviations f_i - w_i, FP32 arithmetic */
} lbm_storage;

/* flags of lbm_grid_desc.flags */
#define LBM_F_NO_GALILEAN 1u /* drop the Galilean-correction terms of the second-order relaxation */
#define LBM_F_GRAPH 2u       /* replay each coarse step from a captured HIP graph */
#define LBM_F_PERSISTENT 4u  /* run each coarse step as one persistent launch over its phase list;
                                currently disabled: lbm_create_grid rejects it with LBM_E_INVALID */
#define LBM_F_AUTOTUNE 8u    /* time the tile candidates at set_geometry and keep the fastest */
#define LBM_F_FRICTION 16u   /* with every force sample, also integrate the wall shear stress over the
                                tree surface (friction force, Sec. 3 Eq. (8)); lbm_drag then reports
                                C_F and C_P = C_D - C_F (Eq. (9)) */

/* One cylinder of the tree (Sec. 2.1: the tree is an assembly of cylinders).
 * The solid is the union of the cylinders and of a sphere of the same
 * diameter at each p1. */
typedef struct {
    double p0[3], p1[3]; /* axis start and end, finest cells */
    double diameter;     /* finest cells */
    int32_t generation;  /* trunk 0 */
    int32_t parent;      /* -1 for the trunk */
    int32_t id;          /* 0 .. n-1, unique */
} lbm_branch;

/* Turtle parameters of Eq. (1) with up to four children per apex.  Child j
 * applies a roll by pre_roll[j] about H, a pitch by pitch[j] (+ jitter) about
 * U and a roll by post_roll[j] about H, then draws F(s * len_ratio[j]) with
 * diameter w * wid_ratio[j].  order = number of child generations below the
 * trunk.  jitter > 0 draws one uniform angle in [-jitter, jitter] degrees per
 * child, in depth-first pre-order, from SplitMix64 seeded with seed. */
typedef struct {
    int32_t m, order;
    double s0, w0;
    double len_ratio[4], wid_ratio[4];
    double pre_roll[4], pitch[4], post_roll[4];
    double jitter;
    uint64_t seed;
} lbm_tree_params;

/* Levels of the octree grid: 1 (uniform) .. LBM_MAX_LEVELS; per-level arrays
 * below hold LBM_MAX_LEVELS entries, of which the first `levels` are used. */
#define LBM_MAX_LEVELS 8

typedef struct {
    int32_t nx, ny, nz;   /* finest-level cells; multiples of block_edge << (levels-1) */
    int32_t block_edge;   /* 8 or 16 */
    int32_t levels;       /* 1 (uniform) .. LBM_MAX_LEVELS */
    double u_in;          /* inflow speed along +x, lattice units; Mach sqrt(3) u_in < 0.3 */
    double re_h;          /* Re_H = u_in H / nu_finest, H = tree height; used when nu <= 0 */
    double nu;            /* finest-level lattice viscosity; > 0 overrides re_h */
    int32_t storage;      /* lbm_storage */
    int32_t periodic_yz;  /* 1: periodic lateral (y) and vertical (z) faces; 0: inflow faces there, ghosts
                             holding f_eq(1, u_in e_x) (Sec. 2.3: inflow conditions on every boundary but
                             the outlet) */
    double turb_intensity; /* inlet I_u (0 = uniform inflow); synthesis as lbm_inflow_modes */
    double turb_length;    /* longitudinal integral length of the inflow turbulence, finest cells */
    uint64_t turb_seed;
    int32_t turb_modes;    /* number of random Fourier modes (0 -> 200) */
    int32_t drag_every;    /* finest sub-steps between force samples (>= 1) */
    uint32_t flags;        /* LBM_F_* */
    int32_t device;        /* HIP device ordinal */
    void *stream;          /* hipStream_t to run on; NULL = the library's own stream */
} lbm_grid_desc;

/* Refinement bands (Sec. 2.2: finest near the surface, moderate in the wake).
 * For level l = 1 .. levels-1, a leaf block of level l-1 is refined when it
 * lies within band[l] finest cells of a branch surface or inside the wake box
 * that extends wake[l] finest cells downstream of the tree's bounding box
 * (laterally padded by band[l]).  Refinement is then closed so that every
 * refined block has all 26 neighbours at its own level.  Ignored when
 * levels == 1. */
typedef struct {
    int32_t band[LBM_MAX_LEVELS];
    int32_t wake[LBM_MAX_LEVELS];
} lbm_refine_desc;

typedef struct {
    double force[3];   /* FP64 mean force on the tree over the samples since the last lbm_drag */
    double cd;         /* C_D = force[0] / (0.5 * u_in^2 * area_x), Eq. (7), rho0 = 1 */
    double area_x;     /* frontal area: finest (y,z) columns holding a solid cell */
    double height;     /* tree height H, finest cells */
    double mass;       /* sum of rho * cell volume (finest units) over all active cells */
    int64_t samples;   /* force samples averaged */
    int64_t step;      /* coarse steps done */
    double friction[3]; /* FP64 mean friction force over the same samples (LBM_F_FRICTION; else 0) */
    double cf, cp;      /* C_F = friction[0] / (0.5 u_in^2 area_x) (Eq. (8)), C_P = C_D - C_F (Eq. (9)) */
} lbm_drag_result;

typedef struct {
    int32_t levels, block_edge, storage;
    int64_t blocks[LBM_MAX_LEVELS];        /* allocated blocks per level (active + covered + ghost) */
    int64_t active_cells[LBM_MAX_LEVELS];  /* leaf fluid + solid cells per level */
    int64_t updated_cells[LBM_MAX_LEVELS]; /* leaf fluid cells per level: the cell updates one level sub-step counts */
    int64_t links;
    int32_t branches;
    double omega1[LBM_MAX_LEVELS];
    double height, area_x, nu_finest;
    size_t device_bytes;
    int32_t tile_cells;       /* cells per work-group of the block-level collide kernel */
    int32_t threads;          /* work-group size of the block-level collide kernel */
    int32_t occ_even, occ_odd;/* resident-wave caps per SIMD of the collide kernel (0 = none) */
    int32_t persist_wgs;      /* work-groups of the persistent launch (all resident) */
    int32_t persist_graph;    /* 1: the persistent launch replays from a captured graph */
    int64_t collided_cells[LBM_MAX_LEVELS];/* cells collided per level sub-step (leaf + band + ghost, solid excluded) */
    int32_t xcd_group;        /* consecutive collide tiles per XCD run (1 = plain dispatch order) */
    int32_t wall_clock_khz;   /* the device's constant real-time clock (hipDeviceAttributeWallClockRate) */
    uint64_t persist_wait_ticks; /* time limit of one wait of the persistent launch, in ticks of that clock */
} lbm_info;

/* ---- lifecycle ------------------------------------------------------------ */

/* The problem statement of Sec. 2.3: the inflow speed u_in (uniform at x = 0,
 * or with the turbulence of Sec. 4.2), Re_H = u_in H / nu, the box and the
 * refinement levels of the octree of Sec. 2.2.  Validates d on the host
 * (sizes, Mach, levels, storage) and creates a grid bound to d->device.  No
 * device memory is allocated yet. */
lbm_status lbm_create_grid(const lbm_grid_desc *d, lbm_grid **out);

/* The tree geometry (Sec. 2.1, an assembly of cylinders) and the grid around
 * it (Sec. 2.2: finest blocks near the surface, a moderately refined wake,
 * coarse blocks elsewhere).  Voxelises the branches (copied), builds boundary
 * links with their wall distances q for the interpolated bounce-back, the
 * block grid and its refinement (refine may be NULL when levels == 1), uploads
 * everything and initialises f = f_eq(1, u_in) in fluid (Sec. 2.3).
 * Fails with LBM_E_INVALID when a branch or refined region comes within one
 * block of the box faces (two cells on one level).  One exception, on one
 * level with periodic y and z faces: a branch parallel to y whose axis runs
 * past both y faces by its radius plus two cells is the same at every y of
 * the box, so the periodic wrap makes it an infinitely long cylinder (the
 * single-cylinder runs behind the C_f table of lbm_analytic_split).
 * device_bytes_out (may be NULL) receives the device
 * memory the library allocated (memory bound with lbm_bind_memory excluded). */
lbm_status lbm_set_geometry(lbm_grid *g, const lbm_branch *b, int32_t n_b,
                            const lbm_refine_desc *refine, size_t *device_bytes_out);

/* Places the populations of every level in caller-owned device memory (for
 * example a torch tensor) instead of memory the library allocates, so that a
 * framework above the library keeps the largest buffer.  Call between
 * lbm_create_grid and lbm_set_geometry (LBM_E_STATE otherwise).  device_ptr:
 * device memory of the grid's device, 256-byte aligned (LBM_E_INVALID
 * otherwise); bytes: its size, at least lbm_plan_levels' pop_bytes for the
 * same description (checked by lbm_set_geometry, LBM_E_INVALID when short).
 * The caller keeps the memory alive until lbm_destroy_grid; the library never
 * frees it and owns its contents (populations as deviations, per level 27
 * direction arrays) while the grid lives.  The rest of the grid (tables,
 * links, sums) stays library-allocated. */
lbm_status lbm_bind_memory(lbm_grid *g, void *device_ptr, size_t bytes);

/* The time marching of Sec. 2.2: cumulant collision and streaming on every
 * level, sub-cycled (a level-l sub-step is 2^(levels-1-l) finest steps), with
 * the coarse/fine coupling, the interpolated bounce-back at the tree surface
 * and the momentum-exchange force sampled every drag_every finest steps.
 * Advances n coarse steps (2^(levels-1) finest sub-steps each),
 * asynchronously on the grid's stream. */
lbm_status lbm_step(lbm_grid *g, int32_t n_coarse_steps);

/* The drag of Sec. 2.2 (momentum exchange over the tree surface) and Eq. (7)
 * (C_D = F_x / (rho U^2 A_x / 2), A_x the frontal area).  Synchronises,
 * returns the mean force over the samples taken since the
 * previous lbm_drag (then restarts the mean), C_D, mass; per_branch (3*n_b
 * doubles, may be NULL) receives the mean force per branch id.  Returns
 * LBM_E_UNSTABLE when the run has produced NaN or a density outside
 * [0.5, 1.5]. */
lbm_status lbm_drag(lbm_grid *g, lbm_drag_result *out, double *per_branch);

/* lbm_drag, and per_branch_friction (3*n_b doubles, may be NULL) receives the
 * mean friction force per branch id (Sec. 3: the wall shear stress integrated
 * over the branch's surface).  Friction is sampled only with LBM_F_FRICTION
 * (LBM_E_STATE otherwise when per_branch_friction is given).  The shear stress
 * of a surface cell is the deviatoric stress -(1 - omega1/2) dev(N) of its
 * pre-collision non-equilibrium second-order central moments N; each axis face
 * between a fluid cell x_f and a solid neighbour x_f + e_k carries the stress
 * extrapolated along e_k from x_f and x_f - e_k to the wall point x_f + q e_k,
 * its traction on the branch's analytic outward normal n with the normal part
 * removed, and the weight |n_k|. */
lbm_status lbm_drag_split(lbm_grid *g, lbm_drag_result *out, double *per_branch, double *per_branch_friction);

/* The drag history of Sec. 2.2 / Eq. (7) sample by sample: copies out up to
 * cap force samples (3 doubles each, FP64, oldest first) of the ring of the
 * last 65536 samples; *n receives the count copied. */
lbm_status lbm_drag_series(lbm_grid *g, double *out, int64_t cap, int64_t *n);

void lbm_destroy_grid(lbm_grid *g);
const char *lbm_last_error(const lbm_grid *g);
lbm_status lbm_get_info(const lbm_grid *g, lbm_info *out);

/* ---- geometry helpers (host only) ------------------------------------------ */

/* The L-system of Eq. (1) read by the turtle of Table 1 (Sec. 2.1): writes up
 * to cap branches of the tree of p (trunk base at the origin, heading +z, left
 * +y); *n receives the full count. */
lbm_status lbm_tree_generate(const lbm_tree_params *p, lbm_branch *out, int32_t cap, int32_t *n);

/* The placement of Sec. 2.3 (tree height H, centre of mass at a given point):
 * scales about the trunk base to height target_h (when > 0) and translates so
 * the cylinder-volume centre of mass is at com.  *height_out (may be NULL)
 * receives the final height. */
lbm_status lbm_tree_place(lbm_branch *b, int32_t n, double target_h, const double com[3],
                          double *height_out);

/* ---- state access for tests and checkpoints (synchronous) ------------------ */

/* Dense FP64 populations of level l over its box, f[i*N + cell].  Cells the
 * level does not hold read as NaN and are ignored on write. */
lbm_status lbm_get_populations(lbm_grid *g, int32_t level, double *f);
lbm_status lbm_set_populations(lbm_grid *g, int32_t level, const double *f);

/* FP64 populations of n listed cells of level l, given as indices over the
 * level's box (x + nx_l (y + ny_l z)): f[i*n + k] for cell cells[k] (host
 * arrays).  Same values as lbm_get_populations at those cells, without the
 * dense box (for grids whose finest box is too large to copy whole); cells the
 * level does not hold, or out of range, read as NaN.  At most 2^26 cells per
 * call. */
lbm_status lbm_get_cells(lbm_grid *g, int32_t level, int64_t n, const int64_t *cells, double *f);

/* Dense density and velocity (u[3*cell + a]) of level l; NaN where not held. */
lbm_status lbm_get_fields(lbm_grid *g, int32_t level, double *rho, double *u);

/* Finest-level solid mask (uint8 over the finest box) and the link table in
 * (cell, direction) order: cell index over the finest box, direction pointing
 * into the solid, q, branch id.  The library itself holds the mask only over
 * the box bounding the tree; lbm_get_solid writes the whole finest box
 * (nx * ny * nz bytes, caller-owned), so it suits boxes that fit host memory. */
lbm_status lbm_get_solid(lbm_grid *g, uint8_t *solid);
lbm_status lbm_get_links(lbm_grid *g, int64_t cap, int64_t *cell, int8_t *dir, double *q,
                         int32_t *branch, int64_t *n);

/* Block map of level l over its block lattice (nbx_l * nby_l * nbz_l int8,
 * caller-owned): 0 none, 1 leaf, 2 refined (covered by level l+1), 3 ghost
 * storage.  The library holds each level above 0 only over the blocks around
 * its refined region and writes zeros elsewhere. */
lbm_status lbm_get_block_map(lbm_grid *g, int32_t level, int8_t *map);

/* ---- learned per-branch drag surrogate ---------------------------------------
 * A network stands in for the branch-wise drag-coefficient lookup of the
 * analytic model (paper Sec. 2.4, Eq. (2)): 5 inputs (log10 Re_D, inclination
 * alpha in degrees, generation, inflow intensity I_u, midpoint height / H) ->
 * 64 ReLU -> 64 ReLU -> 1 output, the branch force coefficient
 * F_x / ((rho U^2 / 2) L D).  Parameters, 4609 floats, packed as W1 (64 x 5,
 * row-major, out x in), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1).
 * Weights are used in BF16 (rounded to nearest even from an FP32 master copy),
 * biases in FP32, accumulation in FP32; inference runs on the matrix cores
 * with BF16 operands.  Features are standardised with x_mean / x_std inside
 * the network and the output is y_mean + y_std * (network output).  The loss
 * is the mean square error on standardised targets; the optimiser is Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).  All array arguments
 * named x, t, y are device pointers (rows of 5 floats for x); host arrays are
 * said so.  One handle per host thread; calls are ordered on the handle's
 * stream and return after their work completed. */
typedef struct lbm_mlp lbm_mlp;

/* He-uniform hidden weights, Glorot-uniform output weights and zero biases
 * drawn from SplitMix64(seed); stream NULL -> the handle owns one. */
lbm_status lbm_mlp_create(uint64_t seed, int32_t device, void *stream, lbm_mlp **out);
void lbm_mlp_destroy(lbm_mlp *m);
/* FP32 master parameters to / from host arrays of 4609 floats; setting them
 * also resets the optimiser state. */
lbm_status lbm_mlp_get_params(lbm_mlp *m, float *params);
lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *params);
/* feature and target standardisation (host arrays of 5; scales > 0) */
lbm_status lbm_mlp_set_scaling(lbm_mlp *m, const float *x_mean, const float *x_std, float y_mean, float y_std);
/* gradient (host, 4609) and loss (host, may be NULL) of the mean-square loss
 * over n samples x (n x 5) with raw targets t (n); deterministic */
lbm_status lbm_mlp_grad(lbm_mlp *m, const float *x, const float *t, int64_t n, float *grad, float *loss);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * gradient of lbm_mlp_grad with the same kernels, whose per-chunk partial
 * sums live in a static device workspace of the library instead of a buffer
 * the handle allocates.  x, t: device arrays (n x 5, n); grad (4609 floats)
 * and loss (1 float, may be NULL): DEVICE outputs.  n <= 32768 samples, else
 * LBM_E_INVALID.  Allocates nothing and does not synchronise: the work is
 * enqueued on the handle's stream and the outputs are valid once that stream
 * has reached this point.  The workspace (18.9 MB per device, resolved by
 * lbm_mlp_create and held until the process ends) is shared by every handle on
 * the device and keeps the last call's contents: two calls on one device that
 * overlap in time (different streams or threads) race on it and must be
 * ordered by the caller. */
lbm_status lbm_mlp_grad_noalloc(lbm_mlp *m, const float *x, const float *t, int64_t n, float *grad, float *loss);
/* one Adam step with a host gradient (4609) */
lbm_status lbm_mlp_adam_step(lbm_mlp *m, const float *grad, float lr);
/* epochs over n samples in shuffled mini-batches (Fisher-Yates from
 * SplitMix64(seed + epoch)); learning rate lr for the first 70 % of the
 * epochs, lr / 10 after; loss_per_epoch (host, epochs floats, may be NULL)
 * receives the full-data loss after each epoch */
lbm_status lbm_mlp_train(lbm_mlp *m, const float *x, const float *t, int64_t n, int32_t epochs, int32_t batch,
                         float lr, uint64_t seed, float *loss_per_epoch);
/* y (n floats, output units) of n rows of raw features x */
lbm_status lbm_mlp_predict(lbm_mlp *m, const float *x, int64_t n, float *y);

/* ---- branch-wise drag sums over many trees -------------------------------
 * Host-only batch of seeded trees from base: tree i has seed seed0 + i and
 * order orders[i] (orders may be NULL: base->order), is scaled to unit height
 * (lbm_tree_place) and yields one record of 10 floats per branch: log10(D/H),
 * alpha (angle to +x, degrees), generation, midpoint height above the trunk
 * base / H, L D / H^2, then the axis projected on the (y, z) plane and the
 * radius (y0, z0, y1, z1, D/2, units of H).  tree_start (n_trees + 1) gets the
 * branch offsets; with rec == NULL only tree_start is filled (sizing).
 * Trees are generated in parallel (OpenMP). */
lbm_status lbm_tree_batch(const lbm_tree_params *base, uint64_t seed0, int32_t n_trees, const int32_t *orders,
                          int64_t cap, float *rec, int64_t *tree_start);

/* Frontal area A_x / H^2 of each tree of a batch (device arrays): the union of
 * the branches' projected capsules (segment plus radius), rasterised on pixels
 * of edge h (units of H; 1/256 in the sweeps) anchored at the tree's lower
 * (y, z) bound; a pixel counts when its centre lies within a capsule (-1 when a
 * tree spans more than 640 pixels).  Ordered on stream; returns when done. */
lbm_status lbm_frontal_area(const float *rec, const int64_t *tree_start, int32_t n_trees, double h, float *area,
                            void *stream);

typedef struct {
    const float *rec;           /* device: branch records of lbm_tree_batch */
    const int64_t *tree_start;  /* device: n_trees + 1 offsets */
    int32_t n_trees;
    const double *re_h;         /* host: Re_H values (1 .. 32) */
    int32_t n_re;
    double intensity;           /* inflow I_u in [0, 0.2]: network input and cylinder curve */
    double re_d_lo, re_d_hi;    /* surrogate: branch Re_D range of its training data */
    const float *area;          /* device: A_x / H^2 per tree */
    float *cd;                  /* device: n_trees x n_re drag coefficients (row per tree) */
} lbm_sweep_desc;

/* C_D of every tree at every Re_H from the surrogate (Eqs. (2), (4) with the
 * network's branch force coefficient y_b in place of C_d sin^3(alpha)):
 * C_D = sum_b y_b L_b D_b / A_x.  Outside [re_d_lo, re_d_hi] the network is
 * evaluated at the clamped Re_D and scaled by the cylinder curve's ratio
 * C_d(Re_D) / C_d(Re_D,clamped).  The cylinder curve is the analytic model's
 * (a synthetic stand-in for the measurements the paper fits): a subcritical
 * 1 + 10 Re^(-2/3) blended into a post-critical 0.25 + 0.35 / (1 + exp(-(ln Re -
 * ln(20 Re_cr)) / 0.8)) by 1 / (1 + exp((ln Re - ln Re_cr) / 0.12)), Re_cr =
 * 2.7e5 for uniform inflow and 1.4e4 at I_u = 8 % (log-linear in between).
 * Matrix cores, one wave per tree. */
lbm_status lbm_surrogate_sweep(lbm_mlp *m, const lbm_sweep_desc *d);
/* The analytic model of Eqs. (2) and (4), C_D = sum_b C_d(Re_b) L_b D_b
 * sin^3(alpha_b) / A_x, on the same inputs (re_d_lo / re_d_hi unused). */
lbm_status lbm_analytic_sweep(const lbm_sweep_desc *d, void *stream);

/* Friction coefficient C_f(Re_D) of a cylinder normal to the flow, as a table
 * (Sec. 2.4: the paper takes it from its own LBM runs of single cylinders and
 * prints no values).  Between consecutive nodes C_f follows the power law
 * through them (linear in log10 Re_D against ln C_f); below the first node and
 * above the last the end segments' power laws continue. */
typedef struct {
    const double *lg_re;  /* host: n nodes of log10 Re_D, strictly increasing */
    const double *cf;     /* host: n values of C_f, finite and > 0 */
    int32_t n;            /* 2 .. 32 */
} lbm_cf_table;

/* The friction / pressure split of the analytic model, Eqs. (3), (5), (6):
 * d->cd receives C_D-est as lbm_analytic_sweep does, cf (device, n_trees x
 * n_re floats, row per tree) C_F-est = sum_b C_f(Re_b) L_b D_b sin^3(alpha_b)
 * / A_x with C_f from t, and cp (device, same shape; may be NULL) C_P-est =
 * C_D-est - C_F-est.  One pass over the branch records for all three.
 * LBM_E_INVALID for a bad description or table (nothing launched); ordered on
 * stream, returns when done. */
lbm_status lbm_analytic_split(const lbm_sweep_desc *d, const lbm_cf_table *t, float *cf, float *cp, void *stream);

/* Host-only surrogate features of a tree's branches at Re_H (rows of 5 floats
 * in feat): log10(Re_H D / H), the angle alpha between the branch axis and the
 * flow (+x) in degrees, the generation, the inflow intensity, and the height
 * of the branch midpoint above the trunk base over H (H as lbm_tree_place
 * measures it).  ld (may be NULL) receives L D per branch. */
lbm_status lbm_branch_features(const lbm_branch *b, int32_t n, double re_h, double intensity, float *feat,
                               double *ld);

/* Host-only mode set of the synthetic turbulent inflow that lbm_set_geometry
 * builds from turb_seed / turb_modes / turb_intensity / turb_length (inlet grid
 * spacing dx = 2^(levels-1) finest cells).  Random Fourier modes with a von
 * Karman spectrum (the paper, Sec. 4.2, fixes only the intensity I_u =
 * u'_rms / U_inf): u'(x, t) = 2 sum_n amp_n sigma_n cos(k_n . (x - u_in t e_x)
 * + psi_n).  out: 8 * n_modes doubles, blocks kx, ky, kz, sigma_x, sigma_y,
 * sigma_z, psi, amp; *k_e (may be NULL) the calibrated spectrum peak
 * parameter. */
lbm_status lbm_inflow_modes(uint64_t seed, int32_t n_modes, double intensity, double length, double u_in,
                            double dx, double *out, double *k_e);

/* Host-only plan of a grid: the validation of lbm_create_grid and
 * lbm_set_geometry, the voxelisation and the block grid of every level, as
 * lbm_set_geometry would build them, without touching a device.  For sizing a
 * run against device memory before allocating it. */
typedef struct {
    int32_t levels, block_edge;
    int32_t lattice[LBM_MAX_LEVELS][3]; /* blocks along x, y, z of each level's box */
    int64_t blocks[LBM_MAX_LEVELS];            /* blocks held per level (leaf + refined + ghost storage) */
    int64_t leaf_cells[LBM_MAX_LEVELS];        /* leaf cells per level (solid included) */
    int64_t collided_cells[LBM_MAX_LEVELS];    /* cells collided per level sub-step (leaf + band + ghost) */
    int64_t updated_cells[LBM_MAX_LEVELS];     /* leaf fluid cells per level (what MLUPS counts) */
    int64_t work_blocks[LBM_MAX_LEVELS];       /* blocks (dense: 256-cell tiles) holding cells to collide */
    int64_t work_tiles[LBM_MAX_LEVELS];        /* of those, B^2-cell z-slices holding cells to collide */
    int64_t links, solid_cells;
    int64_t pop_bytes;            /* population storage of every level in d->storage: the size
                                     lbm_bind_memory needs */
} lbm_plan;

/* maps may be NULL; otherwise maps[l] (may be NULL) receives level l's block
 * map (lattice[l] product int8, values as lbm_get_block_map; pass NULL for
 * lattices too large for host memory: the plan itself does not need them).  Errors as
 * lbm_create_grid and lbm_set_geometry (LBM_E_INVALID), the message in
 * lbm_last_error(NULL). */
lbm_status lbm_plan_levels(const lbm_grid_desc *d, const lbm_branch *b, int32_t n_b,
                           const lbm_refine_desc *refine, lbm_plan *out, int8_t *const *maps);

/* FP64 mass sum over active cells (synchronous). */
lbm_status lbm_mass(lbm_grid *g, double *mass);

/* Per-kernel timing with HIP events recorded on the grid's stream around each
 * collide launch and each bounce-back launch.  lbm_timing_enable(g, 1) clears
 * the totals and starts recording, (g, 0) stops.  lbm_timing_read synchronises
 * and returns total milliseconds and launch counts (any pointer may be NULL). */
lbm_status lbm_timing_enable(lbm_grid *g, int32_t enable);
lbm_status lbm_timing_read(lbm_grid *g, double *collide_ms, int64_t *collide_launches, double *links_ms,
                           int64_t *links_launches);

/* Picks the collide kernels' launch shapes (block tile and threads, an
 * occupancy cap per parity, the XCD run length) by timing coarse steps of each
 * candidate on this grid, then restores the populations, the force
 * accumulators and the step counters.  Appends the choice to the text file
 * cache_path (may be NULL), one line per grid key; a later call with a key
 * already in the file takes the shapes from it without timing.  Allocates a
 * device copy of every level for the duration of the call (LBM_E_NOMEM when
 * that fails, the grid unchanged); LBM_E_DEVICE when a copy of the state
 * fails; LBM_E_STATE before lbm_set_geometry.  Synchronous. */
lbm_status lbm_autotune(lbm_grid *g, const char *cache_path);

/* Checkpoint of populations, step counters, force accumulators and the
 * force-sample ring, taken after an even number of steps on every level
 * (LBM_E_STATE otherwise; synchronous).  lbm_load restores it into a grid set
 * up with the same description and geometry (LBM_E_INVALID when the file does
 * not match): the run then continues bit for bit as if it had not stopped. */
lbm_status lbm_save(lbm_grid *g, const char *path);
lbm_status lbm_load(lbm_grid *g, const char *path);

/* Host-only geometry of a uniform box: solid mask (uint8 over nx*ny*nz, may be
 * NULL), up to cap links in (cell, direction) order (any array may be NULL),
 * *n_links the full count, *area_x the frontal area.  The same routines feed
 * lbm_set_geometry; no device is touched. */
lbm_status lbm_geometry_build(const lbm_branch *b, int32_t n_b, int32_t nx, int32_t ny, int32_t nz,
                              uint8_t *solid, int64_t cap, int64_t *cell, int8_t *dir, double *q,
                              int32_t *branch, int64_t *n_links, double *area_x);

/* ---- persistent coarse step: phase lists and the protocol model ------------
 * The persistent form (LBM_F_PERSISTENT) runs one coarse step as one launch
 * over a recorded list of phases (collide of one level sub-step, bounce-back,
 * force sums, coarse/fine transfer, in the order of the coarse-first
 * recursion of Sec. 2.2).  Work-groups claim chunks of a phase's items from a
 * counter, count each finished chunk, and start a phase once the previous
 * phase is complete; the last work-group to leave clears the counters. */
typedef struct {
    int32_t kind;   /* 0 collide, 1 bounce-back links, 2 link-piece sums, 3 branch totals,
                       4 transfer records at T+1, 5 prolongation, 6 restriction */
    int32_t step;   /* coarse step of the recording (0-based) */
    int32_t items;  /* work items (one work-group each) */
    int32_t chunk;  /* items per claim for the given work-group count */
    int32_t chunks; /* claims of the phase */
} lbm_phase_info;

/* Host only: the phase lists of coarse_steps consecutive coarse steps of the
 * grid d would run in the persistent form (planned as lbm_set_geometry plans
 * it, without a device), chunked for a launch of `groups` work-groups.  Up to
 * cap entries go to out; *n receives the full count.  Errors as
 * lbm_plan_levels; turbulent inflow is not available in this form
 * (LBM_E_INVALID). */
lbm_status lbm_plan_phases(const lbm_grid_desc *d, const lbm_branch *b, int32_t n_b, const lbm_refine_desc *refine,
                           int32_t groups, int32_t coarse_steps, lbm_phase_info *out, int32_t cap, int32_t *n);

typedef struct {
    int64_t chunks_run;        /* chunk executions */
    int64_t chunks_missed;     /* chunks never run */
    int64_t chunks_repeated;   /* chunks run more than once */
    int64_t order_violations;  /* chunks started before the previous phase was complete */
    int64_t waits_given_up;    /* waits that gave up (abort flag or time limit) */
    int32_t abandoned;         /* the abort flag is set at the end */
    int32_t counters_zero;     /* every counter is zero at the end */
    double seconds;            /* wall time of the launch */
} lbm_persist_model_result;

/* Host only: one launch of the persistent kernel's work-distribution protocol
 * (the same code the kernel runs), with `groups` work-groups run by `threads`
 * host threads (each work-group to its end before a thread takes the next:
 * groups > threads models a launch larger than the device holds at once).
 * chunks: n_phases claim counts (lbm_phase_info.chunks).  ctr (2 n_phases + 1
 * words) and *abort_flag are the launch's counters and flag, read at the start
 * (zero for a clean launch) and written back at the end.  A wait gives up
 * after wait_s seconds.  stuck_phase >= 0 makes every chunk of that phase take
 * 3 wait_s (a hung work item); -1 for none. */
lbm_status lbm_persist_model(const int32_t *chunks, int32_t n_phases, int32_t groups, int32_t threads,
                             uint32_t *ctr, uint32_t *abort_flag, double wait_s, int32_t stuck_phase,
                             lbm_persist_model_result *out);

/* ---- host probe (tests) ------------------------------------------------------ */

/* Runs the FP32 cumulant collision of the kernels on the host for one cell:
 * f_in, f_out are 27 full populations (FP64 in and out, rounded to FP32
 * deviations inside), omega1 / omega2 the shear and bulk rates, galilean 0/1
 * for the correction terms.  No device is touched. */
lbm_status lbm_collide_cell_host(const double *f_in, double *f_out, double omega1, double omega2, int galilean);

#ifdef __cplusplus
}
#endif
#endif
