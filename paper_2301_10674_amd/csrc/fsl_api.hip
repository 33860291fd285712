// fsl_api.hip -- host runtime of the free-surface LBM library: workspace
// layout, lattice set-up (initial state, sphere mapping), step sequencing,
// reductions, read-back and the C-ABI declared in include/fsl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fsl.h"
#include "fsl_device.h"
#include "fsl_kernels.h"
#include "fsl_mlp.h"

namespace fsl {
template <class S>
void launch_step(const Dev &d, int p, uint32_t epoch, int list_blocks, int watch, hipStream_t st,
                 hipEvent_t ev0, hipEvent_t ev1, const float *mlpP, const uint16_t *mlpPk);
template <class R>
void launch_geom(const Dev &d, int which, int list_blocks, hipStream_t st);
void launch_watch_final(const Dev &d, int list_blocks, hipStream_t st);
void launch_setup_links(const Dev &d, int from_slots, int c0, int c1, hipStream_t st);
void launch_kinds_list(const Dev &d, const int32_t *list, const int *count, int bound, hipStream_t st);
void launch_mem_count(const Dev &d, int nsph, int32_t *counts, hipStream_t st);
void launch_mem_fill(const Dev &d, int nsph, const MemLists &ml, int only_changed, hipStream_t st);
template <class S>
void launch_mem(const Dev &d, int p, int nsph, const MemLists &ml, double *out, hipStream_t st);
template <class R>
void launch_bb_terms(const Dev &d, int nrec, hipStream_t st);
}  // namespace fsl

using namespace fsl;

static thread_local std::string g_err = "no error";

static FslStatus fail(FslStatus s, const std::string &msg)
{
    g_err = msg;
    return s;
}

namespace fsl {
// the error text of the other entry points of the library (particles)
FslStatus set_error(FslStatus s, const std::string &msg) { return fail(s, msg); }
}  // namespace fsl

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(FSL_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct FslLattice {
    FslParams P;
    Dev d;
    hipStream_t st;
    int parity = 0;           // PDFs of the current state are in pdf[parity]
    int64_t steps = 0;
    uint32_t epoch = 0;       // epoch of the last step's marks
    int list_blocks = 64;
    int nsph = 0;
    bool geometry_set = false;
    std::vector<double> sph_host;
    double *sph_dev = nullptr;     // sphere table (10 per sphere), one force evaluation
                                   // (6 per sphere), a staging table (10 per sphere), a flag
    bool sph_host_stale = false;   // the table was last written from device arrays
    void *bb_dev = nullptr;   // moving-wall bounce-back records
    size_t bb_cap = 0;
    void *mem_dev = nullptr;  // momentum exchange: the link lists (ml points into it)
    void *move_dev = nullptr; // moving spheres: new owner map, round types and densities, counter
    size_t mem_cap = 0;
    MemLists ml{};
    bool mem_stale = true;    // link lists must be rebuilt before the next force evaluation
    bool mem_moved = false;   // spheres moved since the lists were last brought up to date
    bool own_stale = true;    // the remap's owner map is not the current one
    int own_zlo = 0, own_zhi = -1;  // rows the spheres reached at the last remap (widened by two)
    float *mlpP = nullptr;    // learned estimator: FP32 weights
    uint16_t *mlpPk = nullptr;  //   and their packed BF16 copies
    void *read_buf = nullptr; // device staging of fields read to the host
    size_t read_cap = 0;
    bool timing = false;
    double mass_ref = 0.0;    // watchdog: total mass after set-up (fsl_total_mass)
    bool mass_fast = false;   // the last call was fsl_step: its mass partials are current
    int nrec = 0;             // bounce-back records (compact + full) of the current geometry
    double watch_last[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t ev_used = 0;
};

static FslStatus set_mass_ref(FslLattice *L);

// ---------------------------------------------------------------- workspace
static size_t store_bytes(int prec) { return prec == FSL_FP64 ? 8 : (prec == FSL_FP32 ? 4 : 2); }

static_assert(FSL_VAR_FLUX_MODIFIERS == VAR_FLUX_MODIFIERS && FSL_VAR_NORMAL_EXCESS == VAR_NORMAL_EXCESS &&
                  FSL_VAR_CSF_CURVATURE == VAR_CSF_CURVATURE && FSL_VAR_GALILEAN == VAR_GALILEAN,
              "variant bits of the header and the kernels differ");

static bool params_ok(const FslParams *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return false; }
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) { why = "each lattice extent must be >= 3"; return false; }
    // per-cell arrays of 8-byte values are addressed with 32-bit byte offsets
    if ((double)p->nx * p->ny * p->nz * 8.0 >= 4294967296.0) { why = "lattice too large"; return false; }
    if (p->grid_blocks != 0 && (p->grid_blocks < 8 || p->grid_blocks > 2048)) {
        why = "grid_blocks must be 0 or lie in [8, 2048]";
        return false;
    }
    if (p->precision < 0 || p->precision > 2) { why = "unknown precision"; return false; }
    if (!(p->omega > 0.0 && p->omega < 2.0)) { why = "omega must lie in (0, 2)"; return false; }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->accel[a])) { why = "non-finite acceleration"; return false; }
    if (!std::isfinite(p->sigma) || p->sigma < 0.0) { why = "sigma must be finite and >= 0"; return false; }
    if (!(p->rho_gas > 0.0) || !std::isfinite(p->rho_gas)) { why = "rho_gas must be > 0"; return false; }
    if (!(p->conv_eps >= 0.0 && p->conv_eps < 1.0)) { why = "conv_eps must lie in [0, 1)"; return false; }
    if (!(p->normal_tie >= 0.0)) { why = "normal_tie must be >= 0"; return false; }
    if (p->normals != 0 && p->normals != 1) { why = "normals must be 0 or 1"; return false; }
    if (p->check_every < 0) { why = "check_every must be >= 0"; return false; }
    if (p->variants & ~(FSL_VAR_FLUX_MODIFIERS | FSL_VAR_NORMAL_EXCESS | FSL_VAR_CSF_CURVATURE | FSL_VAR_GALILEAN)) {
        why = "unknown variant bits";
        return false;
    }
    if ((p->variants & FSL_VAR_CSF_CURVATURE) && p->normals != 0) {
        why = "the corner-normal curvature variant needs the finite-difference estimator (normals = 0)";
        return false;
    }
    return true;
}

struct Layout {
    size_t pdf[2], mq, phi, rho, share, poolc, geom, mark, est, owner, flags, smask, bbslot, list0, list1,
        lnew, rcell, cnt, stats, partial, total;
};

static Layout layout(const FslParams *p)
{
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const size_t s = store_bytes(p->precision);
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L.pdf[0] = take(27 * N * s);
    L.pdf[1] = take(27 * N * s);
    L.mq = take(8 * N);
    L.phi = take(8 * N);
    L.rho = take(8 * N);
    L.share = take(8 * N);
    L.poolc = take(8 * N);
    L.geom = take((p->precision == FSL_FP64 ? 32 : 16) * N);
    L.mark = take(4 * N);
    L.est = take(N);
    L.owner = take(4 * N);
    L.flags = take(N + 4);
    L.smask = take(4 * N);
    L.bbslot = take(4 * N);
    L.list0 = take(4 * N);
    L.list1 = take(4 * N);
    L.lnew = take(4 * N);
    L.rcell = take(4 * N);
    L.cnt = take(64);
    L.stats = take(8 * 16);
    L.partial = take(8 * (5 * RED_BLOCKS + 8 + WD_SIZE));
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- set-up kernels
template <class S>
__global__ void k_init(Dev d, const double *fill, const double *rho, const double *vel)
{
    using R = typename Real<S>::type;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.N) return;
    const double fl = fill[c];
    const uint8_t ty = fl >= 1.0 ? T_LIQ : (fl <= 0.0 ? T_GAS : T_IF);
    d.flags[c] = ty;
    d.owner[c] = -1;
    d.mark[c] = 0;
    d.est[c] = 0;
    d.share[c] = 0.0;
    d.poolc[c] = 0.0;
    const double cl = fl < 0.0 ? 0.0 : (fl > 1.0 ? 1.0 : fl);
    d.mq[c] = ty == T_GAS ? 0.0 : cl * rho[c];
    R u[3] = {R(0), R(0), R(0)};
    if (vel)
        for (int a = 0; a < 3; ++a) u[a] = R(vel[(size_t)a * d.N + c]);
    R e[27];
    feq_dev<R>(R(rho[c] - 1.0), u[0], u[1], u[2], e);
    // both buffers: cells that never stream (solid, gas) keep finite values
    S *pdf0 = (S *)d.pdf[0], *pdf1 = (S *)d.pdf[1];
    for (int i = 0; i < 27; ++i) {
        const S v = to_store<S, R>(e[i]);
        pdf0[pdf_index(d.nx, i, c)] = v;
        pdf1[pdf_index(d.nx, i, c)] = v;
    }
}

__device__ static int nbr(const Dev &d, int c, int i)
{
    const int x = c % d.nx, y = (c / d.nx) % d.ny, z = c / (d.nx * d.ny);
    const int zz = z + cz(i);
    if (zz < 0 || zz >= d.nz) return -1;
    const int xx = (x + cx(i) + d.nx) % d.nx, yy = (y + cy(i) + d.ny) % d.ny;
    return xx + d.nx * (yy + d.ny * zz);
}

// a liquid cell next to a gas cell becomes an interface cell
__global__ void k_closure(Dev d)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.N || (d.flags[c] & T_MASK) != T_LIQ) return;
    for (int i = 0; i < 27; ++i) {
        if (i == REST) continue;
        const int y = nbr(d, c, i);
        if (y >= 0 && (d.flags[y] & T_MASK) == T_GAS) {
            d.flags[c] = (uint8_t)((d.flags[c] & ~T_MASK) | T_IF);
            return;
        }
    }
}

// liquid cells: switch between the mass m and the stored form m - own outgoing
template <class S>
__device__ void liquid_form_cell(const Dev &d, int p, int to_q, int c)
{
    if ((d.flags[c] & T_MASK) != T_LIQ) return;
    const S *pdf = (const S *)d.pdf[p];
    // the neighbour x + c_i is solid or beyond a wall where the solid-link
    // mask has bit opp(i); the 26 loads are issued together
    const uint32_t sm = d.smask[c];
    double fluid = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if (i == REST) continue;
        const double v = (double)ld(pdf + pdf_index(d.nx, i, c));
        if (!((sm >> opp(i)) & 1u)) fluid += v;
    }
    d.mq[c] = to_q ? d.mq[c] - fluid : d.mq[c] + fluid;
}

template <class S>
__global__ void k_liquid_form(Dev d, int p, int to_q)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < d.N) liquid_form_cell<S>(d, p, to_q, c);
}

// sphere -> solid cells; owner = lowest covering sphere index
__global__ __launch_bounds__(256) void k_map(Dev d, int nsph, int32_t *own)
{
    // Cells whose centre lies inside sphere q (the rule in inside()).  The
    // box rows (y, z) are walked over the x-run where the centre can be
    // inside (widened by a cell against rounding), 256 rows at a time: each
    // thread takes a row, a prefix over the rows numbers the cells of the
    // runs, and the threads then test those cells.
    __shared__ int s_end[256], s_x0[256];
    const int q = blockIdx.x;
    if (q >= nsph) return;
    const double *s = d.sph + 10 * q;
    const double r = s[3];
    const int x0 = (int)floor(s[0] - r) - 1, x1 = (int)floor(s[0] + r) + 1;
    const int y0 = (int)floor(s[1] - r) - 1, y1 = (int)floor(s[1] + r) + 1;
    const int z0 = max((int)floor(s[2] - r) - 1, 0), z1 = min((int)floor(s[2] + r) + 1, d.nz - 1);
    const int wx = x1 - x0 + 1, wy = y1 - y0 + 1, wz = z1 - z0 + 1;
    if (wz <= 0) return;
    const int t = (int)threadIdx.x, lane = __lane_id();
    auto inside = [&](int xx, int yy, int z) {
        const int x = ((xx % d.nx) + d.nx) % d.nx, y = ((yy % d.ny) + d.ny) % d.ny;
        // same rounding as written: no contraction into fused multiply-adds
        double dx = (x + 0.5) - s[0];
        if (dx > 0.5 * d.nx) dx -= d.nx; else if (dx < -0.5 * d.nx) dx += d.nx;
        double dy = (y + 0.5) - s[1];
        if (dy > 0.5 * d.ny) dy -= d.ny; else if (dy < -0.5 * d.ny) dy += d.ny;
        const double dz = (z + 0.5) - s[2];
        const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        if (r2 <= __dmul_rn(r, r)) atomicMin(&own[x + d.nx * (y + d.ny * z)], q);
    };
    if (2 * wx >= d.nx || 2 * wy >= d.ny) {
        // the box reaches half a period: a cell's nearest image need not be
        // its box position, so every box cell is tested
        const int total = wx * wy * wz;
        for (int k = t; k < total; k += blockDim.x)
            inside(x0 + k % wx, y0 + (k / wx) % wy, z0 + k / (wx * wy));
        return;
    }
    const int nrow = wy * wz;
    for (int r0 = 0; r0 < nrow; r0 += 256) {
        const int row = r0 + t;
        int a = 0, n = 0;
        if (row < nrow) {
            const double ey = (y0 + row % wy + 0.5) - s[1], ez = (z0 + row / wy + 0.5) - s[2];
            const double h = r * r - ey * ey - ez * ez;
            if (h >= -1e-9 * (r * r + 1.0)) {
                const double w = sqrt(fmax(h, 0.0)) + 1.0;
                a = max((int)floor(s[0] - w - 0.5) - x0, 0);
                const int e = min((int)ceil(s[0] + w - 0.5) - x0, wx - 1);
                n = max(e - a + 1, 0);
            }
        }
        int inc = n;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(inc, o);
            if (lane >= o) inc += v;
        }
        s_end[t] = inc;
        __syncthreads();
        int wbase = 0;
        for (int w = 0; w < (t >> 6); ++w) wbase += s_end[64 * w + 63];
        const int total = s_end[63] + s_end[127] + s_end[191] + s_end[255];
        __syncthreads();
        s_end[t] = wbase + inc;
        s_x0[t] = a;
        __syncthreads();
        for (int k = t; k < total; k += 256) {
            int lo = 0, hi = 255;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_end[mid] > k) hi = mid;
                else lo = mid + 1;
            }
            const int rr = r0 + lo;
            inside(x0 + s_x0[lo] + (k - (lo ? s_end[lo - 1] : 0)), y0 + rr % wy, z0 + rr / wy);
        }
        __syncthreads();
    }
}

// no owner for cells c0 .. c1 - 1
__global__ void k_owner_reset(int32_t *own, int c0, int c1)
{
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c < c1) own[c] = INT_MAX;
}

// cells inside spheres become solid (their mass leaves the system)
__global__ void k_apply_solid(Dev d)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.N) return;
    if (d.owner[c] == INT_MAX) {
        d.owner[c] = -1;
    } else {
        d.flags[c] = T_SOLID;
        d.mq[c] = 0.0;
    }
}

// ---------------------------------------------------------------- moving spheres
// Flag bits used only while the lattice is remapped: an uncovered cell not
// typed yet, and one typed in an earlier round.
constexpr uint8_t F_OPEN = 8, F_NEWC = 16;

// Appends c0 + k for every set bit k of bits (ascending) to list, in thread
// order over a block of 256: one atomic per block, so that long lists built
// by many blocks do not queue on the counter.  Every thread of the block
// calls it.
__device__ void block_append_bits(int32_t *list, int32_t *counter, uint32_t bits, int32_t c0)
{
    __shared__ int s_w[4], s_base;
    const int n = __popcll((unsigned long long)bits);
    const int lane = __lane_id(), w = (int)threadIdx.x >> 6;
    int inc = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    int off = 0, total = 0;
    for (int k = 0; k < 4; ++k) {
        if (k == w) off = total;
        total += s_w[k];
    }
    if (threadIdx.x == 0) s_base = total ? atomicAdd(counter, total) : 0;
    __syncthreads();
    int pos = s_base + off + inc - n;
    while (bits) {
        const int k = __ffsll((unsigned long long)bits) - 1;
        bits &= bits - 1u;
        list[pos++] = c0 + k;
    }
}

// cells whose owner changes with the new map (INT_MAX: no sphere), appended
// to a list in cell order within a block (one atomic per block of 4096
// cells: the counter is the bottleneck when many blocks append); count =
// list length.  Sixteen cells per thread (both maps are 256-byte aligned),
// the groups w0 .. w1 - 1 of four cells.
__global__ __launch_bounds__(256) void k_owner_changes(Dev d, const int32_t *own, int *count, int32_t *list,
                                                       int w0, int w1)
{
    const int g = w0 + 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t bits = 0u;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int w = g + h;
        int a[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX}, b[4] = {-1, -1, -1, -1};
        if (w >= w1) {
            // past the range: no cells (the block still appends together)
        } else if (4 * w + 3 < d.N) {
            const int4 va = ((const int4 *)own)[w], vb = ((const int4 *)d.owner)[w];
            a[0] = va.x, a[1] = va.y, a[2] = va.z, a[3] = va.w;
            b[0] = vb.x, b[1] = vb.y, b[2] = vb.z, b[3] = vb.w;
        } else {
            for (int k = 0; k < 4 && 4 * w + k < d.N; ++k) {
                a[k] = own[4 * w + k];
                b[k] = d.owner[4 * w + k];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if ((a[k] == INT_MAX ? -1 : a[k]) != b[k]) bits |= 1u << (4 * h + k);
    }
    block_append_bits(list, count, bits, 4 * g);
}

// The listed cells and their 26 neighbours get mark 1 (repeats store the
// same value).
__global__ __launch_bounds__(256) void k_mark_list(Dev d, const int32_t *list, int n, uint32_t *mark)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * 27) return;
    const int y = nbr(d, list[t / 27], (int)(t % 27));
    if (y >= 0) mark[y] = 1u;
}

// The marked cells of the groups w0 .. w1 - 1 of four cells, appended to out
// in cell order within a block (count): the lists the remap's per-cell
// passes walk then read neighbouring cells from neighbouring lanes.
__global__ __launch_bounds__(256) void k_marked_cells(const uint32_t *mark, int N, int32_t *out, int *count, int w0,
                                                      int w1)
{
    // sixteen cells per thread, as k_owner_changes
    const int g = w0 + 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t bits = 0u;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int w = g + h;
        if (w >= w1) continue;
        if (4 * w + 3 < N) {
            const uint4 v = ((const uint4 *)mark)[w];
            bits |= ((v.x ? 1u : 0u) | (v.y ? 2u : 0u) | (v.z ? 4u : 0u) | (v.w ? 8u : 0u)) << (4 * h);
        } else {
            for (int k = 0; k < 4 && 4 * w + k < N; ++k)
                if (mark[4 * w + k]) bits |= 1u << (4 * h + k);
        }
    }
    block_append_bits(out, count, bits, 4 * g);
}

// clear the marks of the cells in list[0 .. *count)
__global__ void k_unmark_list(const int32_t *list, const int *count, uint32_t *mark)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < *count) mark[list[t]] = 0u;
}

// covered fluid cells turn solid, their mass (m form) into the pool;
// uncovered cells are marked open (over the changed cells)
__global__ void k_cover(Dev d, const int32_t *own, const int32_t *list, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int c = list[t];
    const uint8_t ty = d.flags[c] & T_MASK;
    if (own[c] != INT_MAX && ty != T_SOLID) {
        if (ty == T_LIQ || ty == T_IF) d.poolc[c] += d.mq[c];
        d.flags[c] = T_SOLID;
        d.mq[c] = 0.0;
        d.phi[c] = 0.0;
    } else if (own[c] == INT_MAX && ty == T_SOLID) {
        d.flags[c] = T_SOLID | F_OPEN;
    }
}

// One round of typing uncovered cells: an open cell with neighbours typed
// before this round becomes liquid (liquid/interface neighbours, no gas),
// interface (both) or gas (gas only); rn = mean density of its
// liquid/interface neighbours (their rn when they were typed in an earlier
// round).  tn = 0xFF: not typed this round.
template <class S>
__global__ __launch_bounds__(256) void k_uncover_round(Dev d, int p, const int32_t *list, int n, uint8_t *tn,
                                                       double *rn, int *typed)
{
    // 32 lanes per listed cell: lane k < 26 looks at neighbour k
    __shared__ int s_n[4];
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
    const int k = (int)threadIdx.x & 31;
    int did = 0;
    int c = -1;
    if (t < n) c = list[t];
    const bool open = c >= 0 && (d.flags[c] & F_OPEN);
    int nfl = 0, ngas = 0;
    double rs = 0.0;
    if (open && k < 26) {
        const int i = k < REST ? k : k + 1;
        const int y = nbr(d, c, i);
        if (y >= 0) {
            const uint8_t fy = d.flags[y];
            const uint8_t ty = fy & T_MASK;
            if (!(fy & F_OPEN)) {
                if (ty == T_LIQ || ty == T_IF) {
                    nfl = 1;
                    if (fy & F_NEWC) {
                        rs = rn[y];
                    } else {
                        const S *pdf = (const S *)d.pdf[p];
                        double r = 0.0;
                        for (int q = 0; q < 27; ++q) r += (double)ld(pdf + pdf_index(d.nx, q, y));
                        rs = 1.0 + r;
                    }
                } else if (ty == T_GAS) {
                    ngas = 1;
                }
            }
        }
    }
    // sums over the 32 lanes of the cell, in a fixed order
    for (int o = 16; o > 0; o >>= 1) {
        nfl += __shfl_xor(nfl, o);
        ngas += __shfl_xor(ngas, o);
        rs += __shfl_xor(rs, o);
    }
    if (open && k == 0) {
        if (nfl + ngas > 0) {
            tn[c] = nfl > 0 ? (ngas > 0 ? T_IF : T_LIQ) : T_GAS;
            rn[c] = nfl > 0 ? rs / nfl : 1.0;
            did = 1;
        } else {
            tn[c] = 0xFF;
        }
    }
    for (int o = 32; o > 0; o >>= 1) did += __shfl_xor(did, o);
    if (__lane_id() == 0) s_n[threadIdx.x >> 6] = did;
    __syncthreads();
    if (threadIdx.x == 0 && s_n[0] + s_n[1] + s_n[2] + s_n[3]) atomicAdd(typed, s_n[0] + s_n[1] + s_n[2] + s_n[3]);
}

__global__ void k_uncover_apply(Dev d, const int32_t *list, int n, const uint8_t *tn)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int c = list[t];
    if ((d.flags[c] & F_OPEN) && tn[c] != 0xFF) d.flags[c] = (uint8_t)(tn[c] | F_NEWC);
}

// uncovered cells: gas if no round reached them; liquid and interface cells
// at f^eq(rn, u), u the rigid velocity of the sphere that covered them (old
// owner, new table) at the cell centre; liquid mass (m form) from the pool
template <class S>
__global__ void k_uncover_finish(Dev d, int p, const int32_t *list, int n, const double *rn)
{
    using R = typename Real<S>::type;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int c = list[t];
    const uint8_t f = d.flags[c];
    if (!(f & (F_OPEN | F_NEWC))) return;
    const uint8_t ty = (f & F_OPEN) ? T_GAS : (f & T_MASK);
    d.flags[c] = ty;
    d.mq[c] = 0.0;
    d.phi[c] = 0.0;
    if (ty == T_GAS) return;
    const double *s = d.sph + 10 * d.owner[c];
    const int x = c % d.nx, y = (c / d.nx) % d.ny, z = c / (d.nx * d.ny);
    double rx = (x + 0.5) - s[0];
    if (rx > 0.5 * d.nx) rx -= d.nx; else if (rx < -0.5 * d.nx) rx += d.nx;
    double ry = (y + 0.5) - s[1];
    if (ry > 0.5 * d.ny) ry -= d.ny; else if (ry < -0.5 * d.ny) ry += d.ny;
    const double rz = (z + 0.5) - s[2];
    const double u[3] = {s[4] + (s[8] * rz - s[9] * ry), s[5] + (s[9] * rx - s[7] * rz),
                         s[6] + (s[7] * ry - s[8] * rx)};
    R e[27];
    feq_dev<R>(R(rn[c] - 1.0), R(u[0]), R(u[1]), R(u[2]), e);
    S *pdf = (S *)d.pdf[p];
    for (int i = 0; i < 27; ++i) pdf[pdf_index(d.nx, i, c)] = to_store<S, R>(e[i]);
    if (ty == T_LIQ) {
        d.mq[c] = rn[c];
        d.poolc[c] -= rn[c];
    } else {
        d.rho[c] = rn[c];
    }
}

// Closure of the surface after the uncovering rounds: a cell typed liquid in
// the same round as a neighbour typed gas (or never reached, which becomes
// gas) would border gas; it is an interface cell of fill 0 instead.
__global__ void k_uncover_closure(Dev d, const int32_t *list, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int c = list[t];
    const uint8_t f = d.flags[c];
    if (!(f & F_NEWC) || (f & T_MASK) != T_LIQ) return;
    for (int i = 0; i < 27; ++i) {
        if (i == REST) continue;
        const int y = nbr(d, c, i);
        if (y < 0) continue;
        const uint8_t fy = d.flags[y];
        if ((fy & F_OPEN) || (fy & T_MASK) == T_GAS) {
            d.flags[c] = (uint8_t)(T_IF | F_NEWC);
            return;
        }
    }
}

__global__ void k_owner_commit(Dev d, const int32_t *own, const int32_t *list, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int c = list[t];
    d.owner[c] = own[c] == INT_MAX ? -1 : own[c];
}

// solid-link mask and near-solid bit of cell c
__device__ void near_solid_cell(const Dev &d, int c)
{
    uint32_t m = 0;
    for (int j = 0; j < 27; ++j) {
        if (j == REST) continue;
        const int y = nbr(d, c, opp(j));
        if (y < 0 || (d.flags[y] & T_MASK) == T_SOLID) m |= 1u << j;
    }
    d.smask[c] = m;
    d.flags[c] = (uint8_t)((d.flags[c] & ~F_NEAR_SOLID) | (m ? F_NEAR_SOLID : 0));
}

// Momentum-exchange lists a remap may change: a cell's links into spheres
// change only when the cell or a neighbour changes owner, so only the
// changed cells and their neighbours change entries, and only in the lists
// of the old and the new owners of their neighbours (marked before the new
// owners are committed).
__device__ void mem_dirty_cell(const Dev &d, const int32_t *own, int c, int32_t *dirty)
{
    // a cell solid before and after has no links
    if (d.owner[c] >= 0 && own[c] != INT_MAX) return;
    int qo[27], qn[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) {
        const int y = nbr(d, c, j);
        qo[j] = y >= 0 ? d.owner[y] : -1;
        qn[j] = y >= 0 ? own[y] : INT_MAX;
    }
#pragma unroll
    for (int j = 0; j < 27; ++j) {
        if (qo[j] >= 0) dirty[qo[j]] = 1;
        if (qn[j] != INT_MAX) dirty[qn[j]] = 1;
    }
}

// The remap's passes over the changed cells and their neighbours
// (list[0 .. *count)): before the cover, their link lists marked (dirty,
// when the lists are live) and their liquid mass back to m; after the new
// owners are committed, their solid-link masks and the stored liquid form.
template <class S>
__global__ void k_before_cover(Dev d, int p, const int32_t *list, const int *count, const int32_t *own,
                               int32_t *dirty)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= *count) return;
    const int c = list[t];
    if (dirty) mem_dirty_cell(d, own, c, dirty);
    liquid_form_cell<S>(d, p, 0, c);
}

template <class S>
__global__ void k_after_commit(Dev d, int p, const int32_t *list, const int *count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= *count) return;
    const int c = list[t];
    near_solid_cell(d, c);
    liquid_form_cell<S>(d, p, 1, c);
}

// zero n bytes (16 per thread; n a multiple of 16)
__global__ void k_zero_bytes(uint4 *p, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_zero_int(int *v)
{
    if (threadIdx.x == 0) *v = 0;
}

// solid-link mask (bit j: the source x - c_j of direction j is solid or
// beyond a z wall) and the near-solid flag bit
__global__ void k_near_solid(Dev d)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.N) return;
    uint32_t m = 0;
    for (int j = 0; j < 27; ++j) {
        if (j == REST) continue;
        const int y = nbr(d, c, opp(j));
        if (y < 0 || (d.flags[y] & T_MASK) == T_SOLID) m |= 1u << j;
    }
    d.smask[c] = m;
    d.flags[c] = (uint8_t)((d.flags[c] & T_MASK) | (m ? F_NEAR_SOLID : 0));
}

// interface cells: density of the stored PDFs and fill level
template <class S>
__global__ void k_refresh_if(Dev d, int p)
{
    // the interface list of the current state (rebuilt just before)
    const int n = d.cnt[p];
    const int32_t *list = d.list[p];
    const S *pdf = (const S *)d.pdf[p];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int c = list[t];
        double s = 0.0;
        for (int i = 0; i < 27; ++i) s += (double)ld(pdf + pdf_index(d.nx, i, c));
        d.rho[c] = 1.0 + s;
        d.phi[c] = d.mq[c] / d.rho[c];
    }
}

// the interface cells in cell order, sixteen flag bytes per thread (the flag
// array is 256-byte aligned; bytes past N are never appended)
__global__ void k_build_list(Dev d, int which)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (16 * w + 15 < d.N) {
        v = ((const uint4 *)d.flags)[w];
    } else if (16 * w < d.N) {
        uint32_t b[4] = {0u, 0u, 0u, 0u};
        for (int k = 0; 16 * w + k < d.N; ++k) b[k >> 2] |= (uint32_t)d.flags[16 * w + k] << (8 * (k & 3));
        v = make_uint4(b[0], b[1], b[2], b[3]);
    }
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
    uint32_t bits = 0u;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (((u[k >> 2] >> (8 * (k & 3))) & T_MASK) == T_IF) bits |= 1u << k;
    list_append_bits(d.list[which], &d.cnt[which], bits, 16 * w);
}

__global__ void k_zero_counts(Dev d, int stats)
{
    if (threadIdx.x < 6) d.cnt[threadIdx.x] = 0;
    if (stats && threadIdx.x < 16) d.stats[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------- reductions
// total mass, fixed order: block partials, then one block over the partials
// sum of v over a block of 256 threads in a fixed order (butterflies within
// each wavefront, then the four wavefronts in order); the result in thread 0
__device__ __forceinline__ double block_sum256(double v)
{
    __shared__ double s_w[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

// Exact total mass, in a fixed order: per block, the interface masses, the
// liquid masses (stored m minus own outgoing, plus the outgoing PDFs over
// the links that do not end in a solid or beyond a wall: the solid-link
// mask of the opposite direction) and the per-cell pool; one block sums the
// block partials.
template <class S>
__global__ __launch_bounds__(256) void k_mass_partial(Dev d, int p)
{
    const S *pdf = (const S *)d.pdf[p];
    const int nx = d.nx;
    double acc = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d.N; c += gridDim.x * blockDim.x) {
        const uint8_t ty = d.flags[c] & T_MASK;
        double m = d.poolc[c];
        if (ty == T_IF) {
            m += d.mq[c];
        } else if (ty == T_LIQ) {
            const int row = c / nx;
            const S *f = pdf + pdf_index(nx, 0, row, c - row * nx);
            const uint32_t sm = d.smask[c];
            double out = 0.0;
            for (int i = 0; i < 27; ++i)
                if (i != REST && !((sm >> opp(i)) & 1u)) out += (double)ld(f + (size_t)i * nx);
            m += d.mq[c] + out;
        }
        acc += m;
    }
    acc = block_sum256(acc);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_sum_partials(Dev d, int n, int out_slot)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += d.partial[i];
    acc = block_sum256(acc);
    if (threadIdx.x == 0) d.partial[out_slot] = acc;
}

__global__ __launch_bounds__(256) void k_pool_partial(Dev d)
{
    // two cells per load (the array is 256-byte aligned); an odd last cell
    // goes to the first thread
    double acc = 0.0;
    const int n2 = d.N >> 1;
    const double2 *p2 = (const double2 *)d.poolc;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n2; c += gridDim.x * blockDim.x) {
        const double2 v = p2[c];
        acc += v.x + v.y;
    }
    if ((d.N & 1) && blockIdx.x == 0 && threadIdx.x == 0) acc += d.poolc[d.N - 1];
    acc = block_sum256(acc);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = acc;
}

// bulk velocity: per-block partial sums of fill * u (3 components) and of
// the fill over liquid (fill 1) and interface cells, stored after the
// mass partials; u = (j* - rho g / 2) / rho as in the read-back
template <class S>
__global__ __launch_bounds__(256) void k_bulkvel_partial(Dev d, int p)
{
    __shared__ double sh[4][256];
    const S *pdf = (const S *)d.pdf[p];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d.N; c += gridDim.x * blockDim.x) {
        const uint8_t ty = d.flags[c] & T_MASK;
        if (ty != T_LIQ && ty != T_IF) continue;
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 27; ++i) {
            const double v = (double)ld(pdf + pdf_index(d.nx, i, c));
            r += v;
            j[0] += cx(i) * v;
            j[1] += cy(i) * v;
            j[2] += cz(i) * v;
        }
        r += 1.0;
        const double g[3] = {d.gx, d.gy, d.gz};
        const double w = ty == T_LIQ ? 1.0 : d.phi[c];
        for (int a = 0; a < 3; ++a) acc[a] += w * ((j[a] - 0.5 * r * g[a]) / r);
        acc[3] += w;
    }
    for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) d.partial[RED_BLOCKS + 8 + threadIdx.x * RED_BLOCKS + blockIdx.x] = sh[threadIdx.x][0];
}

// the four sums over the block partials, fixed order; u to partial[RED_BLOCKS + 1 .. 3]
__global__ __launch_bounds__(256) void k_bulkvel_final(Dev d)
{
    __shared__ double sh[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < RED_BLOCKS; i += blockDim.x)
        for (int a = 0; a < 4; ++a) acc[a] += d.partial[RED_BLOCKS + 8 + a * RED_BLOCKS + i];
    for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) d.partial[RED_BLOCKS + 1 + threadIdx.x] = sh[3][0] > 0.0 ? sh[threadIdx.x][0] / sh[3][0] : 0.0;
}

// bed profile: phi_b[z * nx + x] = solid cells of the column (x, z) over ny
__global__ void k_phib(Dev d, double *phi)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.nx * d.nz) return;
    const int x = t % d.nx, z = t / d.nx;
    int n = 0;
    for (int y = 0; y < d.ny; ++y) n += (d.flags[x + d.nx * (y + d.ny * z)] & T_MASK) == T_SOLID;
    phi[t] = (double)n / (double)d.ny;
}

// bed height: the uppermost z at which phi_b crosses the threshold, linear
// between cell centres z + 1/2; 0 without solid cells above it, nz when the
// top cell is at or above it
__global__ void k_hb(Dev d, const double *phi, double thr, double *h)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= d.nx) return;
    const int nx = d.nx, nz = d.nz;
    int k = -1;
    for (int z = nz - 1; z >= 0; --z)
        if (phi[z * nx + x] >= thr) {
            k = z;
            break;
        }
    double v;
    if (k < 0) v = 0.0;
    else if (k == nz - 1) v = (double)nz;
    else {
        const double a = phi[k * nx + x], b = phi[(k + 1) * nx + x];
        v = (k + 0.5) + (a - thr) / (a - b);
    }
    h[x] = v;
}

// ---------------------------------------------------------------- read-back
template <class S, class R4>
__global__ void k_read(Dev d, int p, int field, void *out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.N) return;
    const size_t N = (size_t)d.N;
    const uint8_t ty = d.flags[c] & T_MASK;
    const bool fluid = ty == T_LIQ || ty == T_IF;
    const S *pdf = (const S *)d.pdf[p];
    switch (field) {
    case FSL_FIELD_TYPE: ((uint8_t *)out)[c] = ty; break;
    case FSL_FIELD_MASS: {
        double m = 0.0;
        if (ty == T_IF) m = d.mq[c];
        if (ty == T_LIQ) {
            double fl = 0.0;
            for (int i = 0; i < 27; ++i) {
                if (i == REST) continue;
                const int y = nbr(d, c, i);
                if (y >= 0 && (d.flags[y] & T_MASK) != T_SOLID) fl += (double)ld(pdf + pdf_index(d.nx, i, c));
            }
            m = d.mq[c] + fl;
        }
        ((double *)out)[c] = m;
        break;
    }
    case FSL_FIELD_FILL: ((double *)out)[c] = ty == T_IF ? d.phi[c] : (ty == T_LIQ ? 1.0 : 0.0); break;
    case FSL_FIELD_ESTIMATOR: ((uint8_t *)out)[c] = ty == T_IF ? d.est[c] : (uint8_t)0; break;
    case FSL_FIELD_RHO:
    case FSL_FIELD_VEL: {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        if (fluid)
            for (int i = 0; i < 27; ++i) {
                const double v = (double)ld(pdf + pdf_index(d.nx, i, c));
                r += v;
                j[0] += cx(i) * v;
                j[1] += cy(i) * v;
                j[2] += cz(i) * v;
            }
        r += 1.0;
        if (field == FSL_FIELD_RHO) {
            ((double *)out)[c] = fluid ? r : 0.0;
        } else {
            const double g[3] = {d.gx, d.gy, d.gz};
            for (int a = 0; a < 3; ++a)
                ((double *)out)[(size_t)a * N + c] = fluid ? (j[a] - 0.5 * r * g[a]) / r : 0.0;
        }
        break;
    }
    case FSL_FIELD_PDF:
        for (int i = 0; i < 27; ++i)
            ((double *)out)[(size_t)i * N + c] = fluid ? wgt(i) + (double)ld(pdf + pdf_index(d.nx, i, c)) : 0.0;
        break;
    case FSL_FIELD_NORMAL: {
        const R4 g = ((const R4 *)d.geom)[c];
        const bool itf = ty == T_IF;
        ((double *)out)[c] = itf ? (double)g.x : 0.0;
        ((double *)out)[N + c] = itf ? (double)g.y : 0.0;
        ((double *)out)[2 * N + c] = itf ? (double)g.z : 0.0;
        break;
    }
    case FSL_FIELD_CURV: {
        const R4 g = ((const R4 *)d.geom)[c];
        ((double *)out)[c] = ty == T_IF ? (double)g.w : 0.0;
        break;
    }
    case FSL_FIELD_OWNER: ((int32_t *)out)[c] = d.owner[c]; break;
    default: break;
    }
}

// ---------------------------------------------------------------- dispatch
static int blocks_for(int n) { return (n + 255) / 256; }

template <class S>
static void run_setup(FslLattice *L, const double *fill, const double *rho, const double *vel)
{
    const Dev &d = L->d;
    k_init<S><<<blocks_for(d.N), 256, 0, L->st>>>(d, fill, rho, vel);
    k_closure<<<blocks_for(d.N), 256, 0, L->st>>>(d);
}

// all liquid cells, or those in list[0 .. *count) (at most `bound` of them)
template <class S>
static void run_liquid_form(FslLattice *L, int to_q)
{
    k_liquid_form<S><<<blocks_for(L->d.N), 256, 0, L->st>>>(L->d, L->parity, to_q);
}

template <class S>
static void run_before_cover(FslLattice *L, const int32_t *list, const int *count, int64_t bound, const int32_t *own,
                             int32_t *dirty)
{
    if (bound > 0)
        k_before_cover<S><<<(int)((bound + 255) / 256), 256, 0, L->st>>>(L->d, L->parity, list, count, own, dirty);
}

template <class S>
static void run_after_commit(FslLattice *L, const int32_t *list, const int *count, int64_t bound)
{
    if (bound > 0) k_after_commit<S><<<(int)((bound + 255) / 256), 256, 0, L->st>>>(L->d, L->parity, list, count);
}

template <class S> static void run_refresh(FslLattice *L)
{
    k_refresh_if<S><<<std::max(1, std::min(blocks_for(L->d.N), 1024)), 256, 0, L->st>>>(L->d, L->parity);
}

template <class S> static void run_mass(FslLattice *L)
{
    k_mass_partial<S><<<RED_BLOCKS, 256, 0, L->st>>>(L->d, L->parity);
    k_sum_partials<<<1, 256, 0, L->st>>>(L->d, RED_BLOCKS, RED_BLOCKS);
}

template <class S> static void run_bulkvel(FslLattice *L)
{
    k_bulkvel_partial<S><<<RED_BLOCKS, 256, 0, L->st>>>(L->d, L->parity);
    k_bulkvel_final<<<1, 256, 0, L->st>>>(L->d);
}

template <class S> static void run_read(FslLattice *L, int field, void *out)
{
    using R = typename Real<S>::type;
    using R4 = typename std::conditional<sizeof(R) == 8, double4, float4>::type;
    k_read<S, R4><<<blocks_for(L->d.N), 256, 0, L->st>>>(L->d, L->parity, field, out);
}

#define DISPATCH(L, fn, ...)                                         \
    do {                                                             \
        switch ((L)->P.precision) {                                  \
        case FSL_FP64: fn<double>(__VA_ARGS__); break;               \
        case FSL_FP32: fn<float>(__VA_ARGS__); break;                \
        default: fn<_Float16>(__VA_ARGS__); break;                   \
        }                                                            \
    } while (0)

static void run_bb_terms(FslLattice *L)
{
    if (!L->d.bbterm || L->nrec == 0) return;
    if (L->P.precision == FSL_FP64)
        launch_bb_terms<double>(L->d, L->nrec, L->st);
    else
        launch_bb_terms<float>(L->d, L->nrec, L->st);
}

template <class S>
static void run_mem(FslLattice *L, double *out)
{
    launch_mem<S>(L->d, L->parity, L->nsph, L->ml, out, L->st);
}

// Per-sphere lists of the cells that can link into each sphere (for the
// momentum exchange), built from scratch: count on the device, slots on the
// host (a quarter and 16 entries more than the count, room for the lists to
// grow as the spheres move), fill.
static FslStatus build_mem_lists(FslLattice *L)
{
    Dev &d = L->d;
    const int n = L->nsph;
    if (n == 0 || !d.sph) return FSL_OK;
    // the per-sphere counts use the new-cell list as scratch (free between steps; n <= N)
    launch_mem_count(d, n, d.lnew, L->st);
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> offs((size_t)n + 1, 0);
    HIP_TRY(hipMemcpyAsync(offs.data() + 1, d.lnew, (size_t)n * 4, hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    int64_t total = 0;
    for (int q = 0; q < n; ++q) {
        const int64_t c = offs[q + 1];
        total += c + c / 4 + 16;
        if (total > INT32_MAX) return fail(FSL_ERR_NOMEM, "too many momentum-exchange entries");
        offs[q + 1] = (int32_t)total;
    }
    // slot offsets, counts, marks, boxes (6 per sphere), flag, entries
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_cnt = al(((size_t)n + 1) * 4), o_dirty = o_cnt + al((size_t)n * 4),
                 o_box = o_dirty + al((size_t)n * 4), o_flag = o_box + al((size_t)n * 24), o_ent = o_flag + 256;
    const size_t need = o_ent + (size_t)total * 8;
    if (need > L->mem_cap) {
        if (L->mem_dev) HIP_TRY(hipFree(L->mem_dev));
        L->mem_dev = nullptr;
        L->mem_cap = 0;
        L->ml = MemLists{};
        HIP_TRY(hipMalloc(&L->mem_dev, need + need / 8));
        L->mem_cap = need + need / 8;
    }
    char *base = (char *)L->mem_dev;
    L->ml.offs = (int32_t *)base;
    L->ml.cnt = (int32_t *)(base + o_cnt);
    L->ml.dirty = (int32_t *)(base + o_dirty);
    L->ml.box = (int32_t *)(base + o_box);
    L->ml.flag = (int *)(base + o_flag);
    L->ml.ent = (int2 *)(base + o_ent);
    HIP_TRY(hipMemcpyAsync(L->ml.offs, offs.data(), offs.size() * 4, hipMemcpyHostToDevice, L->st));
    k_zero_int<<<1, 64, 0, L->st>>>(L->ml.flag);
    launch_mem_fill(d, n, L->ml, 0, L->st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(L->st));
    return FSL_OK;
}

template <class S>
static void run_uncover_round(FslLattice *L, const int32_t *list, int n, uint8_t *tn, double *rn, int *typed)
{
    k_uncover_round<S><<<(int)(((int64_t)n * 32 + 255) / 256), 256, 0, L->st>>>(L->d, L->parity, list, n, tn, rn, typed);
}

template <class S>
static void run_uncover_finish(FslLattice *L, const int32_t *list, int n, const double *rn)
{
    k_uncover_finish<S><<<(n + 255) / 256, 256, 0, L->st>>>(L->d, L->parity, list, n, rn);
}

// rebuild everything derived from the cell types: solid-link masks,
// bounce-back records, the highest fluid row, the interface list and the
// interface geometry
// near_done: the solid-link masks are current; kinds_done: the slot array
// holds every cell's record kind (a remap re-encoded the cells it changed);
// rec_c0 .. rec_c1 - 1: the only cells that can hold records (rec_c1 < 0:
// any cell)
static FslStatus finalize(FslLattice *L, bool reset_stats = true, bool near_done = false, bool kinds_done = false,
                          int rec_c0 = 0, int rec_c1 = -1)
{
    Dev &d = L->d;
    L->mass_fast = false;
    if (!near_done) k_near_solid<<<blocks_for(d.N), 256, 0, L->st>>>(d);
    k_zero_counts<<<1, 64, 0, L->st>>>(d, reset_stats ? 1 : 0);
    k_build_list<<<blocks_for((d.N + 15) / 16), 256, 0, L->st>>>(d, L->parity);
    // density and fill level of the listed interface cells
    DISPATCH(L, run_refresh, L);
    // running pool total of the watchdog, exact after every rebuild
    k_pool_partial<<<RED_BLOCKS, 256, 0, L->st>>>(d);
    k_sum_partials<<<1, 256, 0, L->st>>>(d, RED_BLOCKS, (int)(d.wd - d.partial) + WD_POOL);
    launch_setup_links(d, kinds_done ? 1 : 0, rec_c0, rec_c1, L->st);
    // the geometry of the rebuilt list, with the estimator the steps use
    const bool learned = L->P.normals == 1 && L->mlpP;
    if (L->P.precision == FSL_FP64) {
        if (learned) launch_geom_mlp<double>(d, L->parity, L->list_blocks, L->mlpP, L->mlpPk, L->st);
        else launch_geom<double>(d, L->parity, L->list_blocks, L->st);
    } else {
        if (learned) launch_geom_mlp<float>(d, L->parity, L->list_blocks, L->mlpP, L->mlpPk, L->st);
        else launch_geom<float>(d, L->parity, L->list_blocks, L->st);
    }
    HIP_TRY(hipGetLastError());
    int32_t nrec[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(nrec, d.cnt + 4, 8, hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    d.bbterm = nullptr;
    d.bbfull = nullptr;
    L->nrec = nrec[0] + nrec[1];
    if (nrec[0] > 0 || nrec[1] > 0) {
        // compact records, then the full ones, in one allocation (kept and
        // reused while large enough: moving spheres rebuild it often)
        const size_t rs = L->P.precision == FSL_FP64 ? 8 : 4;
        const size_t hb = ((size_t)nrec[0] * 8 * rs + 255) & ~(size_t)255;
        const size_t need = hb + (size_t)nrec[1] * 32 * rs;
        if (need > L->bb_cap) {
            if (L->bb_dev) HIP_TRY(hipFree(L->bb_dev));
            L->bb_dev = nullptr;
            L->bb_cap = 0;
            HIP_TRY(hipMalloc(&L->bb_dev, need + need / 8));
            L->bb_cap = need + need / 8;
        }
        d.bbterm = L->bb_dev;
        d.bbfull = (char *)L->bb_dev + hb;
        run_bb_terms(L);
        HIP_TRY(hipGetLastError());
    }
    // the momentum-exchange link lists follow on the next force evaluation
    L->mem_stale = true;
    return FSL_OK;
}

// bring the host copy of the sphere table up to date after moves from
// device arrays
static FslStatus sync_sph_host(FslLattice *L)
{
    if (!L->sph_host_stale) return FSL_OK;
    HIP_TRY(hipMemcpyAsync(L->sph_host.data(), L->sph_dev, L->sph_host.size() * 8, hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    L->sph_host_stale = false;
    return FSL_OK;
}

// New centres and velocities from device arrays into the staging table
// (radii kept); flag = 1 for a non-finite value.  One thread per sphere.
__global__ void k_sph_stage(const double *table, double *stage, int n, const double *centre, const double *vel,
                            const double *angvel, double nx, double ny, int *flag)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double t[10];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        const double c = centre[3 * q + a], v = vel ? vel[3 * q + a] : 0.0, w = angvel ? angvel[3 * q + a] : 0.0;
        ok = ok && isfinite(c) && isfinite(v) && isfinite(w);
        t[a] = c;
        t[4 + a] = v;
        t[7 + a] = w;
    }
    if (!ok) {
        atomicOr(flag, 1);
        return;
    }
    t[0] -= nx * floor(t[0] / nx);
    t[1] -= ny * floor(t[1] / ny);
    t[3] = table[10 * q + 3];
    for (int k = 0; k < 10; ++k) stage[10 * q + k] = t[k];
    // the rows the spheres reach, widened by two (flag[1], flag[2])
    atomicMin(flag + 1, (int)fmax(floor(t[2] - t[3]) - 2.0, -2147483648.0));
    atomicMax(flag + 2, (int)fmin(floor(t[2] + t[3]) + 2.0, 2147483647.0));
}

__global__ void k_stage_init(int *flag)
{
    if (threadIdx.x == 0) {
        flag[0] = 0;
        flag[1] = INT_MAX;
        flag[2] = INT_MIN;
    }
}

static bool finite_all(const float *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// device buffers of a standalone estimator call, freed on scope exit
struct DevBufs {
    std::vector<void *> p;
    ~DevBufs()
    {
        for (void *q : p) (void)hipFree(q);
    }
    template <class T> hipError_t get(T **out, size_t n)
    {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, n * sizeof(T) + 16);
        if (e == hipSuccess) p.push_back(q);
        *out = (T *)q;
        return e;
    }
};

static const int MLP_GPW = 1;  // groups of 16 samples per wavefront

// ---------------------------------------------------------------- no-allocation gradient
// Device scratch of fsl_estimator_grad_device: the packed BF16 weights, then
// the partial gradients and losses of at most GRAD_DEVICE_WAVES wavefronts.
// A file-scope device array: each GPU the library runs on holds one copy for
// the life of the process.  Host code uses the address that
// hipGetSymbolAddress returns for the current device, never the array's
// name (which on the host is only a stand-in for the symbol).
constexpr int GRAD_DEVICE_WAVES = 256;
constexpr int64_t GRAD_DEVICE_MAX_SAMPLES = (int64_t)1 << 24;
constexpr size_t SCRATCH_PK = ((size_t)MLP_PACK_SIZE * 2 + 255) & ~(size_t)255;
constexpr size_t SCRATCH_PART = ((size_t)GRAD_DEVICE_WAVES * MLP_NPARAM * 4 + 255) & ~(size_t)255;
constexpr size_t SCRATCH_BYTES = SCRATCH_PK + SCRATCH_PART + (size_t)GRAD_DEVICE_WAVES * 4;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::atomic<unsigned char *> g_scratch[64];

// address of this device's scratch, looked up once per device
static FslStatus device_scratch(unsigned char **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(FSL_ERR_DEVICE, "device index beyond 64");
    unsigned char *p = g_scratch[dev].load();
    if (!p) {
        void *q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q)
            return fail(FSL_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        p = (unsigned char *)q;
        g_scratch[dev].store(p);
    }
    *out = p;
    return FSL_OK;
}

// ---------------------------------------------------------------- C-ABI
extern "C" {

size_t fsl_workspace_bytes(const FslParams *params)
{
    std::string why;
    if (!params_ok(params, why)) {
        g_err = why;
        return 0;
    }
    return layout(params).total;
}

FslStatus fsl_create_lattice(const FslParams *params, void *ws, size_t bytes, void *hip_stream,
                             const double *fill, const double *rho, const double *vel,
                             FslLattice **out)
{
    std::string why;
    if (!out) return fail(FSL_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!params_ok(params, why)) return fail(FSL_ERR_ARG, why);
    if (!ws || !fill || !rho) return fail(FSL_ERR_ARG, "workspace, fill and rho are required");
    const Layout lay = layout(params);
    if (bytes < lay.total) return fail(FSL_ERR_NOMEM, "workspace smaller than fsl_workspace_bytes()");
    if (((uintptr_t)ws & 255) != 0) return fail(FSL_ERR_ARG, "workspace must be 256-byte aligned");
    const size_t N = (size_t)params->nx * params->ny * params->nz;
    for (size_t c = 0; c < N; ++c) {
        if (!std::isfinite(fill[c]) || !std::isfinite(rho[c]) || !(rho[c] > 0.0))
            return fail(FSL_ERR_ARG, "fill and rho must be finite, rho > 0");
        if (vel)
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(vel[a * N + c])) return fail(FSL_ERR_ARG, "non-finite velocity");
    }

    FslLattice *L = new FslLattice();
    L->P = *params;
    L->st = (hipStream_t)hip_stream;
    char *base = (char *)ws;
    Dev &d = L->d;
    d.nx = params->nx;
    d.ny = params->ny;
    d.nz = params->nz;
    d.N = (int)N;
    d.nbx = (d.nx + BULK_THREADS - 1) / BULK_THREADS;
    d.rows = d.ny * d.nz;
    d.xcd_map = (d.rows % 8) == 0;
    d.bulk_blocks = params->grid_blocks;
    d.pdf[0] = base + lay.pdf[0];
    d.pdf[1] = base + lay.pdf[1];
    d.mq = (double *)(base + lay.mq);
    d.phi = (double *)(base + lay.phi);
    d.rho = (double *)(base + lay.rho);
    d.share = (double *)(base + lay.share);
    d.poolc = (double *)(base + lay.poolc);
    d.geom = base + lay.geom;
    d.mark = (uint32_t *)(base + lay.mark);
    d.est = (uint8_t *)(base + lay.est);
    d.owner = (int32_t *)(base + lay.owner);
    d.flags = (uint8_t *)(base + lay.flags);
    d.smask = (uint32_t *)(base + lay.smask);
    d.bbslot = (int32_t *)(base + lay.bbslot);
    d.bbterm = nullptr;
    d.bbfull = nullptr;
    d.rec_compact = params->precision != FSL_FP16_STORE;
    d.img_check = 0;
    d.list[0] = (int32_t *)(base + lay.list0);
    d.list[1] = (int32_t *)(base + lay.list1);
    d.lnew = (int32_t *)(base + lay.lnew);
    d.rcell = (int32_t *)(base + lay.rcell);
    d.cnt = (int32_t *)(base + lay.cnt);
    d.stats = (unsigned long long *)(base + lay.stats);
    d.partial = (double *)(base + lay.partial);
    d.wd = d.partial + 5 * RED_BLOCKS + 8;
    d.sph = nullptr;
    d.omega = params->omega;
    d.gx = params->accel[0];
    d.gy = params->accel[1];
    d.gz = params->accel[2];
    d.sigma = params->sigma;
    d.rho_gas = params->rho_gas;
    d.eps = params->conv_eps;
    d.tie = params->normal_tie;
    d.rule_iso = params->rule_isolated;
    d.variants = params->variants;
    L->list_blocks = params->grid_blocks ? params->grid_blocks
                                         : (int)std::min<size_t>(2048, std::max<size_t>(64, N / 4096));

    // stage the host inputs
    double *tmp = nullptr;
    const size_t nin = N * (vel ? 5 : 2);
    hipError_t e = hipMalloc(&tmp, nin * sizeof(double));
    if (e != hipSuccess) {
        delete L;
        return fail(FSL_ERR_NOMEM, "staging buffer for the initial state");
    }
    e = hipMemcpyAsync(tmp, fill, N * 8, hipMemcpyHostToDevice, L->st);
    if (e == hipSuccess) e = hipMemcpyAsync(tmp + N, rho, N * 8, hipMemcpyHostToDevice, L->st);
    if (e == hipSuccess && vel) e = hipMemcpyAsync(tmp + 2 * N, vel, 3 * N * 8, hipMemcpyHostToDevice, L->st);
    if (e == hipSuccess) {
        DISPATCH(L, run_setup, L, tmp, tmp + N, vel ? tmp + 2 * N : nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        d.sph = nullptr;
        // m -> stored liquid form, then everything derived from the types
        k_near_solid<<<blocks_for(d.N), 256, 0, L->st>>>(d);
        DISPATCH(L, run_liquid_form, L, 1);
        if (finalize(L) != FSL_OK) e = hipErrorUnknown;
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(L->st);
    (void)hipFree(tmp);
    if (e != hipSuccess) {
        delete L;
        return fail(FSL_ERR_DEVICE, std::string("initialisation: ") + hipGetErrorString(e));
    }
    FslStatus r = set_mass_ref(L);
    if (r != FSL_OK) {
        delete L;
        return r;
    }
    *out = L;
    return FSL_OK;
}

FslStatus fsl_set_particles(FslLattice *L, int32_t n, const double *centre, const double *radius,
                            const double *vel, const double *angvel)
{
    if (!L) return fail(FSL_ERR_ARG, "lattice is NULL");
    if (n < 0 || (n > 0 && (!centre || !radius))) return fail(FSL_ERR_ARG, "bad sphere arrays");
    const int nx = L->P.nx, ny = L->P.ny;
    std::vector<double> t((size_t)std::max(n, 1) * 10, 0.0);
    for (int q = 0; q < n; ++q) {
        double *s = &t[10 * (size_t)q];
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(centre[3 * q + a])) return fail(FSL_ERR_ARG, "non-finite centre");
        if (!(radius[q] > 0.0) || !(2.0 * radius[q] < std::min(nx, ny)))
            return fail(FSL_ERR_ARG, "radius must satisfy 0 < r < min(nx, ny)/2");
        s[0] = centre[3 * q] - nx * std::floor(centre[3 * q] / nx);
        s[1] = centre[3 * q + 1] - ny * std::floor(centre[3 * q + 1] / ny);
        s[2] = centre[3 * q + 2];
        s[3] = radius[q];
        for (int a = 0; a < 3; ++a) {
            s[4 + a] = vel ? vel[3 * q + a] : 0.0;
            s[7 + a] = angvel ? angvel[3 * q + a] : 0.0;
            if (!std::isfinite(s[4 + a]) || !std::isfinite(s[7 + a]))
                return fail(FSL_ERR_ARG, "non-finite sphere velocity");
        }
    }
    if (L->geometry_set) {
        FslStatus hs = sync_sph_host(L);
        if (hs != FSL_OK) return hs;
        // the geometry is mapped once; later calls may only change velocities
        bool same = n == L->nsph;
        for (int q = 0; same && q < n; ++q)
            for (int a = 0; a < 4; ++a) same = same && t[10 * q + a] == L->sph_host[10 * q + a];
        if (!same) return fail(FSL_ERR_STATE, "sphere geometry is already mapped; only velocities may change");
        L->sph_host = t;
        if (n > 0) {
            HIP_TRY(hipMemcpyAsync(L->sph_dev, t.data(), t.size() * 8, hipMemcpyHostToDevice, L->st));
            run_bb_terms(L);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipStreamSynchronize(L->st));
        return FSL_OK;
    }
    if (L->steps > 0) return fail(FSL_ERR_STATE, "spheres must be mapped before the first step");
    // the sphere table, room for one force/torque evaluation (6 per sphere),
    // a staging table for moves from device arrays and its flag
    HIP_TRY(hipMalloc(&L->sph_dev, 2 * t.size() * 8 + (size_t)std::max(n, 1) * 6 * 8 + 64));
    HIP_TRY(hipMemcpyAsync(L->sph_dev, t.data(), t.size() * 8, hipMemcpyHostToDevice, L->st));
    L->sph_host = t;
    L->nsph = n;
    L->geometry_set = true;
    Dev &d = L->d;
    d.sph = L->sph_dev;
    // a cell next to a sphere lies within r + 1.5 of its centre; its link
    // midpoints and its centre can only see different periodic images when
    // that reaches half a period
    d.img_check = 0;
    for (int q = 0; q < n; ++q)
        if (2.0 * (t[10 * (size_t)q + 3] + 2.0) >= (double)std::min(nx, ny)) d.img_check = 1;
    // liquid cells back to m, re-map, then the stored form with the new solids
    DISPATCH(L, run_liquid_form, L, 0);
    k_owner_reset<<<blocks_for(d.N), 256, 0, L->st>>>(d.owner, 0, d.N);
    L->own_stale = true;
    if (n > 0) k_map<<<n, 256, 0, L->st>>>(d, n, d.owner);
    k_apply_solid<<<blocks_for(d.N), 256, 0, L->st>>>(d);
    k_near_solid<<<blocks_for(d.N), 256, 0, L->st>>>(d);
    DISPATCH(L, run_liquid_form, L, 1);
    FslStatus r = finalize(L);
    if (r != FSL_OK) return r;
    // mass inside the new solids has left: a new reference for the watchdog
    return set_mass_ref(L);
}

FslStatus fsl_particle_forces(FslLattice *L, double *out, int32_t out_on_device)
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (L->nsph == 0) return FSL_OK;
    if (!out) return fail(FSL_ERR_ARG, "out is NULL");
    // the lists: rebuilt after set-up, else refilled for the spheres that
    // moved their box or were marked by a remap; a list that outgrew its
    // slot is only found after the sums, which are then redone
    bool refill = false;
    if (L->mem_stale) {
        FslStatus r = build_mem_lists(L);
        if (r != FSL_OK) return r;
        L->mem_stale = false;
    } else if (L->mem_moved) {
        k_zero_int<<<1, 64, 0, L->st>>>(L->ml.flag);
        launch_mem_fill(L->d, L->nsph, L->ml, 1, L->st);
        refill = true;
    }
    L->mem_moved = false;
    if (!L->mem_dev) return fail(FSL_ERR_STATE, "sphere link lists missing");
    double *buf = out_on_device ? out : L->sph_dev + (size_t)L->nsph * 10;
    for (int pass = 0; pass < 2; ++pass) {
        DISPATCH(L, run_mem, L, buf);
        HIP_TRY(hipGetLastError());
        if (!out_on_device)
            HIP_TRY(hipMemcpyAsync(out, buf, (size_t)L->nsph * 6 * 8, hipMemcpyDeviceToHost, L->st));
        int outgrown = 0;
        if (refill) HIP_TRY(hipMemcpyAsync(&outgrown, L->ml.flag, 4, hipMemcpyDeviceToHost, L->st));
        HIP_TRY(hipStreamSynchronize(L->st));
        if (!outgrown) break;
        FslStatus r = build_mem_lists(L);
        if (r != FSL_OK) return r;
        refill = false;
    }
    return FSL_OK;
}

// The spheres of the lattice move to the state in the device table: remap
// owners, cover and uncover cells, rebuild what follows from the cell types.
// zlo .. zhi: the rows the spheres reach at their new positions, widened by
// two.  Between remaps the remap's own owner map (own) holds the current
// owners, none outside the rows the spheres reached, so only the rows the
// spheres reach before or after the move are cleared and compared.
static FslStatus remap(FslLattice *L, int zlo, int zhi)
{
    const int n = L->nsph;
    Dev &d = L->d;
    const size_t N = (size_t)d.N;
    const int nz = L->P.nz, plane = L->P.nx * L->P.ny;
    zlo = std::max(zlo, 0);
    zhi = std::min(zhi, nz - 1);
    int slo = zlo, shi = zhi;
    if (L->own_stale) {
        slo = 0;
        shi = nz - 1;
    } else {
        slo = std::min(slo, L->own_zlo);
        shi = std::max(shi, L->own_zhi);
    }
    L->own_stale = true;
    const int c0 = slo * plane, c1 = shi >= slo ? (shi + 1) * plane : c0;
    // scratch, each part 256-byte aligned: densities (8 B), new owners
    // (4 B), changed cells (4 B), marks (4 B), the marked cells (4 B) and
    // round types (1 B) per cell, two counters; marks start zero and are
    // cleared again after use
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_own = al(N * 8), o_chg = o_own + al(N * 4), o_mark = o_chg + al(N * 4),
                 o_mlist = o_mark + al(N * 4), o_tn = o_mlist + al(N * 4), o_cnt = o_tn + al(N);
    if (!L->move_dev) {
        HIP_TRY(hipMalloc(&L->move_dev, o_cnt + 64));
        const size_t z16 = al(N * 4) / 16;
        k_zero_bytes<<<(int)((z16 + 255) / 256), 256, 0, L->st>>>((uint4 *)((char *)L->move_dev + o_mark), z16);
    }
    char *mv = (char *)L->move_dev;
    double *rn = (double *)mv;
    int32_t *own = (int32_t *)(mv + o_own);
    int32_t *chg = (int32_t *)(mv + o_chg);
    uint32_t *mark = (uint32_t *)(mv + o_mark);
    int32_t *mlist = (int32_t *)(mv + o_mlist);
    uint8_t *tn = (uint8_t *)(mv + o_tn);
    int *counter = (int *)(mv + o_cnt);
    int *mcount = counter + 4;
    if (c1 > c0) k_owner_reset<<<blocks_for(c1 - c0), 256, 0, L->st>>>(own, c0, c1);
    k_map<<<n, 256, 0, L->st>>>(d, n, own);
    k_zero_int<<<1, 64, 0, L->st>>>(counter);
    const int w0 = c0 / 4, w1 = (c1 + 3) / 4;
    if (w1 > w0) k_owner_changes<<<blocks_for((w1 - w0 + 3) / 4), 256, 0, L->st>>>(d, own, counter, chg, w0, w1);
    HIP_TRY(hipGetLastError());
    int nch = 0;
    HIP_TRY(hipMemcpyAsync(&nch, counter, 4, hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    // live momentum-exchange lists are refilled where they may have changed
    const bool lists_live = L->mem_dev && !L->mem_stale;
    L->mem_moved = true;
    if (nch == 0) {
        // no cell changes owner: only the moving-wall records follow the spheres
        run_bb_terms(L);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(L->st));
        L->own_stale = false;
        L->own_zlo = zlo;
        L->own_zhi = zhi;
        return FSL_OK;
    }
    const int gch = (nch + 255) / 256, gmk = (int)(((int64_t)nch * 27 + 255) / 256);
    const int64_t nmax = std::min<int64_t>((int64_t)nch * 27, (int64_t)N);
    // only the changed cells and their neighbours change type or solid
    // neighbours: listed once each
    k_zero_int<<<1, 64, 0, L->st>>>(mcount);
    // (the changed cells lie in the rows of the spheres before or after the
    // move, their neighbours in the rows scanned for changes, widened by two)
    k_mark_list<<<gmk, 256, 0, L->st>>>(d, chg, nch, mark);
    k_marked_cells<<<blocks_for((w1 - w0 + 3) / 4), 256, 0, L->st>>>(mark, d.N, mlist, mcount, w0, w1);
    const int gml = (int)((nmax + 255) / 256);
    DISPATCH(L, run_before_cover, L, mlist, mcount, nmax, own, lists_live ? L->ml.dirty : nullptr);
    k_cover<<<gch, 256, 0, L->st>>>(d, own, chg, nch);
    // rounds in pairs between checks by the host: a round that types no
    // cell changes nothing (its apply finds no typed cell), so the second
    // of a pair may run idle
    for (int round = 0;; round += 2) {
        if (round > nch + 1) return fail(FSL_ERR_DEVICE, "uncovered cells: rounds do not end");
        k_zero_int<<<1, 64, 0, L->st>>>(counter);
        k_zero_int<<<1, 64, 0, L->st>>>(counter + 1);
        for (int k = 0; k < 2; ++k) {
            DISPATCH(L, run_uncover_round, L, chg, nch, tn, rn, counter + k);
            k_uncover_apply<<<gch, 256, 0, L->st>>>(d, chg, nch, tn);
        }
        HIP_TRY(hipGetLastError());
        int typed[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(typed, counter, 8, hipMemcpyDeviceToHost, L->st));
        HIP_TRY(hipStreamSynchronize(L->st));
        if (typed[0] == 0 || typed[1] == 0) break;
    }
    k_uncover_closure<<<gch, 256, 0, L->st>>>(d, chg, nch);
    DISPATCH(L, run_uncover_finish, L, chg, nch, rn);
    k_owner_commit<<<gch, 256, 0, L->st>>>(d, own, chg, nch);
    DISPATCH(L, run_after_commit, L, mlist, mcount, nmax);
    // record kinds: only the listed cells can change theirs, unless a sphere
    // nearly spans the periodic box (kinds then depend on sphere positions)
    const bool kinds_done = !d.img_check;
    if (kinds_done) launch_kinds_list(d, mlist, mcount, (int)nmax, L->st);
    k_unmark_list<<<gml, 256, 0, L->st>>>(mlist, mcount, mark);
    HIP_TRY(hipGetLastError());
    // records lie next to spheres: in the rows scanned for owner changes
    FslStatus r = finalize(L, false, true, kinds_done, c0, c1);
    if (r != FSL_OK) return r;
    L->mem_stale = !lists_live;
    HIP_TRY(hipStreamSynchronize(L->st));
    L->own_stale = false;
    L->own_zlo = zlo;
    L->own_zhi = zhi;
    return FSL_OK;
}

FslStatus fsl_move_particles(FslLattice *L, const double *centre, const double *vel, const double *angvel)
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (!L->geometry_set || L->nsph == 0) return fail(FSL_ERR_STATE, "no spheres are mapped");
    if (!centre) return fail(FSL_ERR_ARG, "centre is NULL");
    FslStatus hs = sync_sph_host(L);
    if (hs != FSL_OK) return hs;
    const int n = L->nsph, nx = L->P.nx, ny = L->P.ny;
    std::vector<double> t = L->sph_host;
    for (int q = 0; q < n; ++q) {
        double *sp = &t[10 * (size_t)q];
        for (int a = 0; a < 3; ++a) {
            const double v = vel ? vel[3 * q + a] : 0.0, w = angvel ? angvel[3 * q + a] : 0.0;
            if (!std::isfinite(centre[3 * q + a]) || !std::isfinite(v) || !std::isfinite(w))
                return fail(FSL_ERR_ARG, "non-finite sphere centre or velocity");
            sp[4 + a] = v;
            sp[7 + a] = w;
        }
        sp[0] = centre[3 * q] - nx * std::floor(centre[3 * q] / nx);
        sp[1] = centre[3 * q + 1] - ny * std::floor(centre[3 * q + 1] / ny);
        sp[2] = centre[3 * q + 2];
    }
    HIP_TRY(hipMemcpyAsync(L->sph_dev, t.data(), (size_t)n * 10 * 8, hipMemcpyHostToDevice, L->st));
    L->sph_host = t;
    int zlo = INT_MAX, zhi = INT_MIN;
    for (int q = 0; q < n; ++q) {
        const double z = t[10 * (size_t)q + 2], r = t[10 * (size_t)q + 3];
        zlo = std::min(zlo, (int)std::max(std::floor(z - r) - 2.0, -2147483648.0));
        zhi = std::max(zhi, (int)std::min(std::floor(z + r) + 2.0, 2147483647.0));
    }
    return remap(L, zlo, zhi);
}

FslStatus fsl_move_particles_device(FslLattice *L, const double *centre, const double *vel, const double *angvel)
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (!L->geometry_set || L->nsph == 0) return fail(FSL_ERR_STATE, "no spheres are mapped");
    if (!centre) return fail(FSL_ERR_ARG, "centre is NULL");
    const int n = L->nsph;
    const size_t tsz = L->sph_host.size();
    double *stage = L->sph_dev + tsz + (size_t)std::max(n, 1) * 6;
    int *flag = (int *)(stage + tsz);
    k_stage_init<<<1, 64, 0, L->st>>>(flag);
    k_sph_stage<<<(n + 255) / 256, 256, 0, L->st>>>(L->sph_dev, stage, n, centre, vel, angvel, (double)L->P.nx,
                                                     (double)L->P.ny, flag);
    HIP_TRY(hipGetLastError());
    int fl[3] = {0, 0, 0};   // non-finite input, lowest and highest row reached
    HIP_TRY(hipMemcpyAsync(fl, flag, 12, hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    if (fl[0]) return fail(FSL_ERR_ARG, "non-finite sphere centre or velocity");
    HIP_TRY(hipMemcpyAsync(L->sph_dev, stage, (size_t)n * 10 * 8, hipMemcpyDeviceToDevice, L->st));
    L->sph_host_stale = true;
    return remap(L, fl[1], fl[2]);
}

// reference mass of the watchdog: the exact total after set-up
static FslStatus set_mass_ref(FslLattice *L)
{
    DISPATCH(L, run_mass, L);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&L->mass_ref, L->d.partial + RED_BLOCKS, 8, hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    return FSL_OK;
}

// Watchdog after a step that wrote its partials: the total mass must be
// finite and within a relative 1e-10 of the reference, and every fluid
// cell's density within [0.5, 1.5].
static FslStatus check_watch(FslLattice *L)
{
    double w[4];
    HIP_TRY(hipMemcpyAsync(w, L->d.wd + WD_OUT, sizeof(w), hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    double *o = L->watch_last;
    o[0] = w[0];
    o[1] = L->mass_ref;
    o[2] = w[1];
    o[3] = w[2];
    o[4] = w[3];
    char msg[200];
    if (!std::isfinite(w[0])) {
        snprintf(msg, sizeof(msg), "watchdog at step %lld: total mass is not finite", (long long)L->steps);
        return fail(FSL_ERR_UNSTABLE, msg);
    }
    if (w[3] > 0.0) {
        snprintf(msg, sizeof(msg), "watchdog at step %lld: %.0f fluid cells with density outside [%.1f, %.1f] "
                 "(range %.6g .. %.6g)", (long long)L->steps, w[3], WD_RHO_MIN, WD_RHO_MAX, w[1], w[2]);
        return fail(FSL_ERR_UNSTABLE, msg);
    }
    const double drift = std::fabs(w[0] - L->mass_ref) / std::max(std::fabs(L->mass_ref), 1e-300);
    if (!(drift <= 1e-10)) {
        snprintf(msg, sizeof(msg), "watchdog at step %lld: total mass %.17g drifted from %.17g (relative %.3g > 1e-10)",
                 (long long)L->steps, w[0], L->mass_ref, drift);
        return fail(FSL_ERR_UNSTABLE, msg);
    }
    return FSL_OK;
}

FslStatus fsl_step(FslLattice *L, int32_t nsteps)
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (nsteps < 0) return fail(FSL_ERR_ARG, "nsteps < 0");
    for (int s = 0; s < nsteps; ++s) {
        uint32_t ep = L->epoch + 1;
        if (ep >= (1u << 24)) {
            // epoch stamps wrap: clear every mark before reusing small epochs
            HIP_TRY(hipMemsetAsync(L->d.mark, 0, (size_t)L->d.N * 4, L->st));
            ep = 1;
        }
        L->epoch = ep;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (L->timing) {
            if (L->ev_used == L->events.size()) {
                hipEvent_t a, b;
                HIP_TRY(hipEventCreate(&a));
                HIP_TRY(hipEventCreate(&b));
                L->events.push_back({a, b});
            }
            e0 = L->events[L->ev_used].first;
            e1 = L->events[L->ev_used].second;
            ++L->ev_used;
        }
        const bool learned = L->P.normals == 1 && L->mlpP;
        const float *mP = learned ? L->mlpP : nullptr;
        const uint16_t *mK = learned ? L->mlpPk : nullptr;
        const int watch = L->P.check_every > 0 && (L->steps + 1) % L->P.check_every == 0;
        const int lb = L->list_blocks;
        switch (L->P.precision) {
        case FSL_FP64: launch_step<double>(L->d, L->parity, ep, lb, watch, L->st, e0, e1, mP, mK); break;
        case FSL_FP32: launch_step<float>(L->d, L->parity, ep, lb, watch, L->st, e0, e1, mP, mK); break;
        default: launch_step<_Float16>(L->d, L->parity, ep, lb, watch, L->st, e0, e1, mP, mK); break;
        }
        L->parity ^= 1;
        ++L->steps;
        L->mass_fast = true;
        if (watch) {
            FslStatus r = check_watch(L);
            if (r != FSL_OK) return r;
        }
    }
    HIP_TRY(hipGetLastError());
    return FSL_OK;
}

FslStatus fsl_read_fields(FslLattice *L, uint32_t mask, void *const *dst, int32_t on_device)
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (!dst) return fail(FSL_ERR_ARG, "dst is NULL");
    const size_t N = (size_t)L->d.N;
    for (int f = 0; f < FSL_NFIELDS; ++f) {
        if (!(mask & (1u << f))) continue;
        if (!dst[f]) return fail(FSL_ERR_ARG, "destination of a selected field is NULL");
        size_t bytes = N * 8;
        if (f == FSL_FIELD_TYPE || f == FSL_FIELD_ESTIMATOR) bytes = N;
        if (f == FSL_FIELD_OWNER) bytes = N * 4;
        if (f == FSL_FIELD_VEL || f == FSL_FIELD_NORMAL) bytes = 3 * N * 8;
        if (f == FSL_FIELD_PDF) bytes = 27 * N * 8;
        if ((f == FSL_FIELD_NORMAL || f == FSL_FIELD_CURV) && !(L->P.normals == 1 && L->mlpP)) {
            // the plain estimator evaluates the geometry inside the step;
            // evaluate it here for the current interface list
            if (L->P.precision == FSL_FP64)
                launch_geom<double>(L->d, L->parity, L->list_blocks, L->st);
            else
                launch_geom<float>(L->d, L->parity, L->list_blocks, L->st);
        }
        // host output is staged on the device: in a buffer kept by the
        // lattice for fields up to three doubles per cell, in a temporary
        // one for the PDFs
        void *buf = dst[f];
        bool temp = false;
        if (!on_device) {
            if (bytes <= 3 * N * 8) {
                if (L->read_cap < bytes) {
                    if (L->read_buf) HIP_TRY(hipFree(L->read_buf));
                    L->read_buf = nullptr;
                    L->read_cap = 0;
                    HIP_TRY(hipMalloc(&L->read_buf, 3 * N * 8));
                    L->read_cap = 3 * N * 8;
                }
                buf = L->read_buf;
            } else {
                HIP_TRY(hipMalloc(&buf, bytes));
                temp = true;
            }
        }
        DISPATCH(L, run_read, L, f, buf);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && !on_device) {
            e = hipMemcpyAsync(dst[f], buf, bytes, hipMemcpyDeviceToHost, L->st);
            if (e == hipSuccess) e = hipStreamSynchronize(L->st);
        }
        if (temp) (void)hipFree(buf);
        if (e != hipSuccess) return fail(FSL_ERR_DEVICE, std::string("read_fields: ") + hipGetErrorString(e));
    }
    HIP_TRY(hipStreamSynchronize(L->st));
    return FSL_OK;
}

FslStatus fsl_total_mass(FslLattice *L, double *mass)
{
    if (!L || !mass) return fail(FSL_ERR_ARG, "NULL argument");
    if (L->mass_fast) {
        // right after steps: the last step's block partials (liquid mass
        // after streaming, interface mass after the flux) and the pool
        // before its conversions, which only move mass
        launch_watch_final(L->d, L->list_blocks, L->st);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(mass, L->d.wd + WD_OUT, 8, hipMemcpyDeviceToHost, L->st));
    } else {
        DISPATCH(L, run_mass, L);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(mass, L->d.partial + RED_BLOCKS, 8, hipMemcpyDeviceToHost, L->st));
    }
    HIP_TRY(hipStreamSynchronize(L->st));
    return FSL_OK;
}

FslStatus fsl_watchdog(FslLattice *L, double out[5])
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (!out) return fail(FSL_ERR_ARG, "out is NULL");
    for (int k = 0; k < 5; ++k) out[k] = L->watch_last[k];
    return FSL_OK;
}

FslStatus fsl_set_accel(FslLattice *L, const double accel[3])
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (!accel) return fail(FSL_ERR_ARG, "accel is NULL");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(accel[a])) return fail(FSL_ERR_ARG, "non-finite acceleration");
    for (int a = 0; a < 3; ++a) L->P.accel[a] = accel[a];
    L->d.gx = accel[0];
    L->d.gy = accel[1];
    L->d.gz = accel[2];
    return FSL_OK;
}

FslStatus fsl_bulk_velocity(FslLattice *L, double u[3])
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (!u) return fail(FSL_ERR_ARG, "u is NULL");
    DISPATCH(L, run_bulkvel, L);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(u, L->d.partial + RED_BLOCKS + 1, 24, hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    return FSL_OK;
}

FslStatus fsl_bed_profile(FslLattice *L, double *phi_b, double *h_b, int32_t out_on_device)
{
    if (!L) return fail(FSL_ERR_STATE, "lattice is NULL");
    if (!phi_b || !h_b) return fail(FSL_ERR_ARG, "NULL output");
    const Dev &d = L->d;
    const size_t nxz = (size_t)d.nx * d.nz;
    // host output is staged in the per-step excess-share array (free between
    // steps; nx*nz + nx <= N since ny >= 3)
    double *dphi = out_on_device ? phi_b : d.share;
    double *dh = out_on_device ? h_b : d.share + nxz;
    k_phib<<<(int)((nxz + 255) / 256), 256, 0, L->st>>>(d, dphi);
    k_hb<<<(d.nx + 255) / 256, 256, 0, L->st>>>(d, dphi, 0.3, dh);
    HIP_TRY(hipGetLastError());
    if (!out_on_device) {
        HIP_TRY(hipMemcpyAsync(phi_b, dphi, nxz * 8, hipMemcpyDeviceToHost, L->st));
        HIP_TRY(hipMemcpyAsync(h_b, dh, (size_t)d.nx * 8, hipMemcpyDeviceToHost, L->st));
    }
    HIP_TRY(hipStreamSynchronize(L->st));
    return FSL_OK;
}

FslStatus fsl_counters(FslLattice *L, int64_t out[8])
{
    if (!L || !out) return fail(FSL_ERR_ARG, "NULL argument");
    unsigned long long h[8];
    HIP_TRY(hipMemcpyAsync(h, L->d.stats, sizeof(h), hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    for (int i = 0; i < 8; ++i) out[i] = (int64_t)h[i];
    out[7] = 0;
    return FSL_OK;
}

FslStatus fsl_info(FslLattice *L, int64_t *steps, int64_t *interface_cells)
{
    if (!L) return fail(FSL_ERR_ARG, "NULL argument");
    int32_t c[3];
    HIP_TRY(hipMemcpyAsync(c, L->d.cnt, sizeof(c), hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    if (steps) *steps = L->steps;
    if (interface_cells) *interface_cells = c[L->parity];
    return FSL_OK;
}

FslStatus fsl_timing(FslLattice *L, int32_t enable)
{
    if (!L) return fail(FSL_ERR_ARG, "NULL argument");
    L->timing = enable != 0;
    if (enable) L->ev_used = 0;
    return FSL_OK;
}

FslStatus fsl_timing_read(FslLattice *L, double *ms_total, int64_t *launches)
{
    if (!L) return fail(FSL_ERR_ARG, "NULL argument");
    HIP_TRY(hipStreamSynchronize(L->st));
    double tot = 0.0;
    for (size_t i = 0; i < L->ev_used; ++i) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, L->events[i].first, L->events[i].second));
        tot += ms;
    }
    if (ms_total) *ms_total = tot;
    if (launches) *launches = (int64_t)L->ev_used;
    return FSL_OK;
}

FslStatus fsl_estimator_stats(FslLattice *L, int64_t *learned, int64_t *fallback)
{
    if (!L) return fail(FSL_ERR_ARG, "NULL argument");
    unsigned long long h[2];
    HIP_TRY(hipMemcpyAsync(h, L->d.stats + 8, sizeof(h), hipMemcpyDeviceToHost, L->st));
    HIP_TRY(hipStreamSynchronize(L->st));
    if (learned) *learned = (int64_t)h[0];
    if (fallback) *fallback = (int64_t)h[1];
    return FSL_OK;
}

FslStatus fsl_set_estimator(FslLattice *L, const float *weights)
{
    if (!L || !weights) return fail(FSL_ERR_ARG, "NULL argument");
    if (!finite_all(weights, MLP_NPARAM)) return fail(FSL_ERR_ARG, "non-finite estimator weights");
    if (!L->mlpP) {
        HIP_TRY(hipMalloc(&L->mlpP, MLP_NPARAM * sizeof(float)));
        HIP_TRY(hipMalloc(&L->mlpPk, MLP_PACK_SIZE * sizeof(uint16_t)));
    }
    HIP_TRY(hipMemcpyAsync(L->mlpP, weights, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, L->st));
    mlp_pack(L->mlpP, L->mlpPk, L->st);
    if (L->P.normals == 1) {
        // geometry of the current interface cells with the estimator
        if (L->P.precision == FSL_FP64)
            launch_geom_mlp<double>(L->d, L->parity, L->list_blocks, L->mlpP, L->mlpPk, L->st);
        else
            launch_geom_mlp<float>(L->d, L->parity, L->list_blocks, L->mlpP, L->mlpPk, L->st);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(L->st));
    return FSL_OK;
}

FslStatus fsl_estimator_grad(const float *weights, const float *x, const float *y, int64_t n,
                             float *grad_out, double *loss_out, void *hip_stream)
{
    if (!weights || !x || !y || !grad_out || n <= 0 || n > (1 << 30)) return fail(FSL_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    DevBufs B;
    float *P, *X, *T, *part, *ploss, *g, *loss;
    uint16_t *pk;
    int32_t *idx;
    const int nw = (int)((n + 16 * MLP_GPW - 1) / (16 * MLP_GPW));
    HIP_TRY(B.get(&P, MLP_NPARAM));
    HIP_TRY(B.get(&pk, MLP_PACK_SIZE));
    HIP_TRY(B.get(&X, (size_t)n * 27));
    HIP_TRY(B.get(&T, (size_t)n * 4));
    HIP_TRY(B.get(&idx, (size_t)n));
    HIP_TRY(B.get(&part, (size_t)nw * MLP_NPARAM));
    HIP_TRY(B.get(&ploss, (size_t)nw));
    HIP_TRY(B.get(&g, MLP_NPARAM));
    HIP_TRY(B.get(&loss, 1));
    std::vector<int32_t> id((size_t)n);
    for (int64_t i = 0; i < n; ++i) id[i] = (int32_t)i;
    HIP_TRY(hipMemcpyAsync(P, weights, MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(X, x, (size_t)n * 27 * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(T, y, (size_t)n * 16, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(idx, id.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
    mlp_pack(P, pk, st);
    mlp_grad(X, T, idx, (int)n, 1.0f / (float)n, P, pk, MLP_GPW, part, ploss, nw, g, loss, st);
    HIP_TRY(hipGetLastError());
    float lh = 0.f;
    HIP_TRY(hipMemcpyAsync(grad_out, g, MLP_NPARAM * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&lh, loss, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (loss_out) *loss_out = lh;
    return FSL_OK;
}

FslStatus fsl_estimator_grad_device(const float *weights, const float *x, const float *y, int64_t n,
                                    float *grad, float *loss, void *hip_stream)
{
    if (!weights || !x || !y || !grad || !loss) return fail(FSL_ERR_ARG, "NULL argument");
    if (n <= 0 || n > GRAD_DEVICE_MAX_SAMPLES) return fail(FSL_ERR_ARG, "n must lie in [1, 2^24]");
    unsigned char *sp = nullptr;
    FslStatus r = device_scratch(&sp);
    if (r != FSL_OK) return r;
    hipStream_t st = (hipStream_t)hip_stream;
    uint16_t *pk = (uint16_t *)sp;
    float *part = (float *)(sp + SCRATCH_PK);
    float *ploss = (float *)(sp + SCRATCH_PK + SCRATCH_PART);
    // groups of 16 samples per wavefront so that at most GRAD_DEVICE_WAVES
    // partials are written; every partial slot used is written in full, so
    // nothing in the scratch has to start at zero
    const int gpw = (int)((n + 16 * GRAD_DEVICE_WAVES - 1) / (16 * GRAD_DEVICE_WAVES));
    const int nw = (int)((n + 16 * (int64_t)gpw - 1) / (16 * (int64_t)gpw));
    mlp_pack(weights, pk, st);
    mlp_grad(x, y, nullptr, (int)n, 1.0f / (float)n, weights, pk, gpw, part, ploss, nw, grad, loss, st);
    HIP_TRY(hipGetLastError());
    return FSL_OK;
}

FslStatus fsl_estimator_train(const float *x, const float *y, int64_t n, const FslTrainParams *tp,
                              float *weights, float *epoch_loss, void *hip_stream)
{
    if (!x || !y || !tp || !weights || n <= 0 || n > (1 << 30)) return fail(FSL_ERR_ARG, "bad argument");
    if (tp->epochs <= 0 || tp->batch < 16 || !(tp->lr > 0.0)) return fail(FSL_ERR_ARG, "bad training parameters");
    if (!finite_all(weights, MLP_NPARAM)) return fail(FSL_ERR_ARG, "non-finite initial weights");
    hipStream_t st = (hipStream_t)hip_stream;
    const int batch = (int)std::min<int64_t>(tp->batch, n);
    const int nbat = (int)((n + batch - 1) / batch);
    const int nw = (batch + 16 * MLP_GPW - 1) / (16 * MLP_GPW);
    DevBufs B;
    float *P, *M, *V, *X, *T, *part, *ploss, *losses;
    uint16_t *pk;
    int32_t *idx;
    HIP_TRY(B.get(&P, MLP_NPARAM));
    HIP_TRY(B.get(&M, MLP_NPARAM));
    HIP_TRY(B.get(&V, MLP_NPARAM));
    HIP_TRY(B.get(&pk, MLP_PACK_SIZE));
    HIP_TRY(B.get(&X, (size_t)n * 27));
    HIP_TRY(B.get(&T, (size_t)n * 4));
    HIP_TRY(B.get(&idx, (size_t)n));
    HIP_TRY(B.get(&part, (size_t)nw * MLP_NPARAM));
    HIP_TRY(B.get(&ploss, (size_t)nw));
    HIP_TRY(B.get(&losses, (size_t)nbat));
    HIP_TRY(hipMemsetAsync(M, 0, MLP_NPARAM * 4, st));
    HIP_TRY(hipMemsetAsync(V, 0, MLP_NPARAM * 4, st));
    HIP_TRY(hipMemcpyAsync(P, weights, MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(X, x, (size_t)n * 27 * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(T, y, (size_t)n * 16, hipMemcpyHostToDevice, st));
    mlp_pack(P, pk, st);
    // per-epoch shuffles from a seeded 64-bit linear congruential generator
    std::vector<int32_t> perm((size_t)n);
    std::vector<float> hl((size_t)nbat);
    uint64_t rs = tp->seed * 6364136223846793005ull + 1442695040888963407ull;
    int64_t t = 0;
    for (int ep = 0; ep < tp->epochs; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
        for (int64_t i = n - 1; i > 0; --i) {
            rs = rs * 6364136223846793005ull + 1442695040888963407ull;
            const int64_t j = (int64_t)((rs >> 33) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        HIP_TRY(hipMemcpyAsync(idx, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
        for (int b = 0; b < nbat; ++b) {
            const int nb = (int)std::min<int64_t>(batch, n - (int64_t)b * batch);
            ++t;
            const float c1 = (float)(1.0 - std::pow(tp->beta1, (double)t));
            const float c2 = (float)(1.0 - std::pow(tp->beta2, (double)t));
            mlp_train_step(X, T, idx + (size_t)b * batch, nb, 1.0f / (float)nb, P, M, V, pk, MLP_GPW, part, ploss,
                           (nb + 16 * MLP_GPW - 1) / (16 * MLP_GPW), (float)tp->lr, (float)tp->beta1,
                           (float)tp->beta2, (float)tp->eps, c1, c2, losses + b, st);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(hl.data(), losses, (size_t)nbat * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (epoch_loss) {
            double s = 0.0;
            for (int b = 0; b < nbat; ++b) s += hl[b];
            epoch_loss[ep] = (float)(s / nbat);
        }
    }
    HIP_TRY(hipMemcpyAsync(weights, P, MLP_NPARAM * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return FSL_OK;
}

FslStatus fsl_estimator_infer(const float *weights, const float *x, int64_t n, float *y, void *hip_stream)
{
    if (!weights || !x || !y || n <= 0 || n > (1 << 30)) return fail(FSL_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    DevBufs B;
    float *P, *X, *Y;
    uint16_t *pk;
    HIP_TRY(B.get(&P, MLP_NPARAM));
    HIP_TRY(B.get(&pk, MLP_PACK_SIZE));
    HIP_TRY(B.get(&X, (size_t)n * 27));
    HIP_TRY(B.get(&Y, (size_t)n * 4));
    HIP_TRY(hipMemcpyAsync(P, weights, MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(X, x, (size_t)n * 27 * 4, hipMemcpyHostToDevice, st));
    mlp_pack(P, pk, st);
    mlp_infer(X, (int)n, P, pk, Y, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(y, Y, (size_t)n * 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return FSL_OK;
}

FslStatus fsl_estimator_stencils(const double *params, int64_t n, int32_t ss, float *x, void *hip_stream)
{
    if (!params || !x || n <= 0 || n > (1 << 26) || ss < 1 || ss > 64)
        return fail(FSL_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    DevBufs B;
    double *P;
    float *X;
    HIP_TRY(B.get(&P, (size_t)n * 16));
    HIP_TRY(B.get(&X, (size_t)n * 27));
    HIP_TRY(hipMemcpyAsync(P, params, (size_t)n * 16 * 8, hipMemcpyHostToDevice, st));
    stencil_fill(P, (int)n, ss, X, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(x, X, (size_t)n * 27 * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return FSL_OK;
}

FslStatus fsl_fd_geometry(const float *x, int64_t n, float *y, void *hip_stream)
{
    if (!x || !y || n <= 0 || n > (1 << 30)) return fail(FSL_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    DevBufs B;
    float *X, *Y;
    HIP_TRY(B.get(&X, (size_t)n * 27));
    HIP_TRY(B.get(&Y, (size_t)n * 4));
    HIP_TRY(hipMemcpyAsync(X, x, (size_t)n * 27 * 4, hipMemcpyHostToDevice, st));
    fd_stencils(X, (int)n, Y, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(y, Y, (size_t)n * 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return FSL_OK;
}

const char *fsl_last_error(void) { return g_err.c_str(); }

void fsl_destroy(FslLattice *L)
{
    if (!L) return;
    (void)hipStreamSynchronize(L->st);
    for (auto &p : L->events) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (L->sph_dev) (void)hipFree(L->sph_dev);
    if (L->bb_dev) (void)hipFree(L->bb_dev);
    if (L->mem_dev) (void)hipFree(L->mem_dev);
    if (L->move_dev) (void)hipFree(L->move_dev);
    if (L->mlpP) (void)hipFree(L->mlpP);
    if (L->mlpPk) (void)hipFree(L->mlpPk);
    if (L->read_buf) (void)hipFree(L->read_buf);
    delete L;
}

}  // extern "C"
