// fsl_kernels.h -- device state shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsl {

// Everything a kernel needs, passed by value.  Per-cell arrays are dense
// over the whole lattice (cell = x + nx*(y + ny*z)); PDF arrays are
// row-interleaved structures of arrays (see pdf_index).
struct Dev {
    int nx, ny, nz, N;
    int nbx, rows;            // dense grid: x-blocks of 256 cells per (y, z) row
    int xcd_map;              // 1: rows are interleaved over the 8 XCDs
    int bulk_blocks;          // workgroups of the dense pass (0: one per row segment, at most 2048)
    void *pdf[2];             // storage type depends on the precision form
    double *mq;               // interface: mass m; liquid: m minus own outgoing PDFs
    double *phi;              // interface fill level m / rho*
    double *rho;              // interface post-collision density
    double *share;            // excess-mass share of a cell converted this step
    double *poolc;            // per-cell excess mass that found no receiver
    void *geom;               // interface normal (xyz) and curvature (w): double4 or float4
    uint32_t *mark;           // conversion marks, epoch << 8 | bits
    uint8_t *est;             // learned estimator: outcome per interface cell (0 none)
    int32_t *owner;           // owning sphere of a solid cell, -1 otherwise
    uint8_t *flags;           // cell type (2 bits) | near-solid bit
    uint32_t *smask;          // bit j: the source x - c_j is solid or beyond a wall
    int32_t *bbslot;          // moving-wall record of a cell with sphere links: k >= 0 compact
                              // record k, k <= -2 full record -k-2, -1 none
    void *bbterm;             // compact records, 8 Real values each: the rigid velocities of
                              // the first two spheres at the cell centre (3 + 3), the mask of the
                              // links into the second sphere (uint32 bits), unused
    void *bbfull;             // full records of cells next to three or more spheres (every
                              // cell in the FP16-storage form): the moving-wall term of each
                              // direction, 32 Real values each
    int32_t *rcell;           // cell of each record: compact record k at rcell[k], full record
                              // f at rcell[N - 1 - f]
    int rec_compact;          // 1: compact records where they suffice (FP64, FP32 storage)
    int img_check;            // 1: some sphere nearly spans the periodic box, so a link
                              // midpoint and its cell centre may see different images
    int32_t *list[2];         // interface cells, current / next step
    int32_t *lnew;            // cells that become interface cells this step
    int32_t *cnt;             // [0],[1] list lengths, [2] lnew length, [3] highest fluid z,
                              // [4] compact and [5] full bounce-back records
    unsigned long long *stats;  // conversion counters
    const double *sph;        // spheres: X[3], r, U[3], Omega[3]
    double *partial;          // reduction partials
    double *wd;               // watchdog: per-block partials of the step kernels, the
                              // result of the last check and the running pool total
    double omega, gx, gy, gz, sigma, rho_gas, eps, tie;
    int rule_iso;
    int variants;             // VAR_* bits
};

// Momentum-exchange link lists.  Sphere q owns the entry slot
// [offs[q], offs[q+1]) of ent, cnt[q] entries of it in use (cell index,
// mask of the cell's links into the sphere).  dirty[q] is set where a remap
// may have changed the list, box[6q .. 6q+5] is the bounding box the list
// was last filled from, flag[0] is set when a list outgrows its slot.
struct MemLists {
    int32_t *offs, *cnt, *dirty, *box;
    int *flag;
    int2 *ent;
};

// variants: flux modifiers between interface cells and normal-weighted
// excess mass (Thuerey 2007), curvature from corner normals (Brackbill et al.
// 1992), Galilean correction of the cumulant collision (Geier et al. 2015)
constexpr int VAR_FLUX_MODIFIERS = 1, VAR_NORMAL_EXCESS = 2, VAR_CSF_CURVATURE = 4, VAR_GALILEAN = 8;

// Element of f_i of cell c = x + nx*r (row r = y + ny*z): the 27 direction
// sub-rows of a row follow one another, f_i(x, r) at (27 r + i) nx + x.
// Loads along x stay coalesced, and the 27 pulls of a wavefront (from nine
// rows) and its 27 stores (into its own row) fall into a few pages instead
// of 54 arrays a whole lattice apart, which would thrash the address
// translation caches on large lattices.
__host__ __device__ __forceinline__ size_t pdf_index(int nx, int i, int c)
{
    const int r = c / nx;
    return (size_t)(27 * (size_t)r + (size_t)i) * (size_t)nx + (size_t)(c - r * nx);
}
__host__ __device__ __forceinline__ size_t pdf_index(int nx, int i, int r, int x)
{
    return (size_t)(27 * (size_t)r + (size_t)i) * (size_t)nx + (size_t)x;
}

constexpr int BULK_THREADS = 256;
constexpr int BULK_MAX_BLOCKS = 2048;
constexpr int LIST_THREADS = 256;
constexpr int RED_BLOCKS = 1024;

// watchdog area (doubles): 4 per block of the dense and of the interface
// kernel (mass, lowest and highest density, cells outside [0.5, 1.5]), then
// the combined result (mass, lowest, highest, outside) and the pool total
constexpr int WD_BULK = 0;
constexpr int WD_IFACE = 4 * BULK_MAX_BLOCKS;
constexpr int WD_OUT = WD_IFACE + 4 * 2048;
constexpr int WD_POOL = WD_OUT + 4;
constexpr int WD_POOL_SNAP = WD_OUT + 5;  // the pool total before this step's conversions
constexpr int WD_SIZE = WD_OUT + 8;
constexpr double WD_RHO_MIN = 0.5, WD_RHO_MAX = 1.5;

}  // namespace fsl
