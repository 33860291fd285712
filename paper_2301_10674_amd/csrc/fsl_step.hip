// fsl_step.hip -- the kernels of one free-surface LBM time step on gfx950.
//
// Per step (Section 2.1 fluid model; readings of the cited free-surface
// method as listed in the design notes):
//   k_bulk    dense over the liquid rows: pull streaming, bounce-back next
//             to walls and spheres, mass bookkeeping, cumulant collision,
//             store.  This is the HBM-bound hot kernel.
//   k_classes (flux-modifier variant only) interface list: the class of
//             each interface cell from its neighbours' types.
//   k_iface   interface list: the same plus the interface normal and
//             curvature (finite differences on the fill stencil),
//             reconstruction of PDFs from the gas side, the fill-weighted
//             mass flux and the conversion marks.
//   k_conv1   interface list: cancel emptyings next to fillings, mark the
//             cells that become interface cells (list lnew).
//   k_conv23  lnew: initialise the new interface cells; interface list:
//             excess mass of converted cells.
//   k_conv4   interface list + lnew: commit cell types, gather excess mass,
//             refresh fill levels, build the next interface list.
//   k_geom_mlp (learned estimator only) next interface list: normal and
//             curvature from the network, finite differences as fallback.
//   k_geom    normal and curvature of the list, for set-up and reads.
#include "fsl_device.h"
#include "fsl_kernels.h"
#include "fsl_mlp.h"

namespace fsl {

// ---------------------------------------------------------------- indexing
struct Cell {
    int x, y, z;
};

__device__ __forceinline__ Cell cell_xyz(const Dev &d, int c)
{
    Cell r;
    r.x = c % d.nx;
    int t = c / d.nx;
    r.y = t % d.ny;
    r.z = t / d.ny;
    return r;
}

// neighbour x + c_i (periodic x, y); -1 beyond the z walls
__device__ __forceinline__ int nb_of(const Dev &d, const Cell &p, int i)
{
    int z = p.z + cz(i);
    if (z < 0 || z >= d.nz) return -1;
    int x = cx(i) == 1 ? wrap_p(p.x, d.nx) : (cx(i) == -1 ? wrap_m(p.x, d.nx) : p.x);
    int y = cy(i) == 1 ? wrap_p(p.y, d.ny) : (cy(i) == -1 ? wrap_m(p.y, d.ny) : p.y);
    return x + d.nx * (y + d.ny * z);
}

__device__ __forceinline__ double min_image(double v, int n)
{
    if (v > 0.5 * n) v -= n;
    else if (v < -0.5 * n) v += n;
    return v;
}

// Owners of the sources x - c_j of the solid links j of cell p (mask sm):
// qo[j] for the links of the returned mask, whose sources lie inside the
// lattice.  The loads do not depend on each other and are all issued before
// any is used (masked-off links load the cell's own entry).
__device__ __forceinline__ uint32_t link_owners(const Dev &d, const Cell &p, int c, uint32_t sm, int (&qo)[27])
{
    uint32_t vm = 0u;
#pragma unroll
    for (int j = 0; j < 27; ++j) {
        const int s = j != REST ? nb_of(d, p, opp(j)) : -1;
        const bool on = ((sm >> j) & 1u) && s >= 0;
        qo[j] = d.owner[on ? s : c];
        vm |= on ? 1u << j : 0u;
    }
    return vm;
}

// Moving-wall bounce-back term 6 w_j (c_j . u_w) for the link from fluid
// cell p along -c_j into the solid cell s (Ladd; wall density 1).
template <class R>
__device__ __forceinline__ R bb_term(const Dev &d, int s, int j, const Cell &p)
{
    const double *sp = d.sph + 10 * d.owner[s];
    double rx = min_image((p.x + 0.5 - 0.5 * cx(j)) - sp[0], d.nx);
    double ry = min_image((p.y + 0.5 - 0.5 * cy(j)) - sp[1], d.ny);
    double rz = (p.z + 0.5 - 0.5 * cz(j)) - sp[2];
    double ux = sp[4] + (sp[8] * rz - sp[9] * ry);
    double uy = sp[5] + (sp[9] * rx - sp[7] * rz);
    double uz = sp[6] + (sp[7] * ry - sp[8] * rx);
    return R(6.0 * wgt(j) * (cx(j) * ux + cy(j) * uy + cz(j) * uz));
}

// Rigid-body velocity of sphere q at the centre of cell p.  The wall term of
// a link from p into q, taken at the link midpoint p - c_j/2, equals
// 6 w_j (c_j . V) with this V, since c_j . (Omega x c_j) = 0.
__device__ __forceinline__ void rigid_velocity(const Dev &d, int q, const Cell &p, double V[3])
{
    const double *sp = d.sph + 10 * q;
    const double rx = min_image((p.x + 0.5) - sp[0], d.nx);
    const double ry = min_image((p.y + 0.5) - sp[1], d.ny);
    const double rz = (p.z + 0.5) - sp[2];
    V[0] = sp[4] + (sp[8] * rz - sp[9] * ry);
    V[1] = sp[5] + (sp[9] * rx - sp[7] * rz);
    V[2] = sp[6] + (sp[7] * ry - sp[8] * rx);
}

// Does the periodic image of sphere q nearest to the link midpoint of
// direction j equal the one nearest to the cell centre?  (Only on lattices
// barely wider than a sphere can they differ; such cells keep per-link terms.)
__device__ __forceinline__ bool same_image(const Dev &d, int q, const Cell &p, int j)
{
    const double *sp = d.sph + 10 * q;
    const double mx = min_image((p.x + 0.5 - 0.5 * cx(j)) - sp[0], d.nx);
    const double my = min_image((p.y + 0.5 - 0.5 * cy(j)) - sp[1], d.ny);
    const double cxm = min_image((p.x + 0.5) - sp[0], d.nx) - 0.5 * cx(j);
    const double cym = min_image((p.y + 0.5) - sp[1], d.ny) - 0.5 * cy(j);
    // images differ by a whole period (>= 3 cells); rounding differs by far less
    return fabs(mx - cxm) < 0.25 && fabs(my - cym) < 0.25;
}

// A cell's moving-wall record (bbslot k; one uint4 array per Real type):
// NU = 28 Real values in u.  k >= 0: compact record (first 8 values);
// k <= -2: full record.  Nothing is loaded for k == -1.
template <class R>
__device__ __forceinline__ void load_record(const Dev &d, int k, uint4 (&u)[28 * sizeof(R) / 16])
{
    constexpr int NF = 28 * (int)sizeof(R) / 16, NH = 8 * (int)sizeof(R) / 16;
#pragma unroll
    for (int i = 0; i < NF; ++i) u[i] = make_uint4(0u, 0u, 0u, 0u);
    if (k >= 0) {
        const uint4 *hp = (const uint4 *)((const R *)d.bbterm + (size_t)k * 8);
#pragma unroll
        for (int i = 0; i < NH; ++i) u[i] = hp[i];
    } else if (k <= -2) {
        const uint4 *fp = (const uint4 *)((const R *)d.bbfull + (size_t)(-k - 2) * 32);
#pragma unroll
        for (int i = 0; i < NF; ++i) u[i] = fp[i];
    }
}

// Moving-wall term of link j from a loaded record; zero for k == -1 and for
// links the caller does not treat as sphere links.
template <class R>
__device__ __forceinline__ R record_term(const R (&r)[28], int k, int j)
{
    if (k <= -2) return r[j];
    uint32_t m2;
    __builtin_memcpy(&m2, &r[6], 4);
    const bool two = (m2 >> j) & 1u;
    const R vx = two ? r[3] : r[0], vy = two ? r[4] : r[1], vz = two ? r[5] : r[2];
    R cu = R(0);
    if (cx(j)) cu += cx(j) > 0 ? vx : -vx;
    if (cy(j)) cu += cy(j) > 0 ? vy : -vy;
    if (cz(j)) cu += cz(j) > 0 ? vz : -vz;
    return R(6.0 * wgt(j)) * cu;
}

// ---------------------------------------------------------------- dense step
// load / store of direction i at 32-bit element offset e from a per-direction
// base that is uniform over the wavefront (scalar base + one vector offset)
template <class S>
__device__ __forceinline__ typename Real<S>::type ld_at(const S *base, uint32_t e)
{
    return ld((const S *)((const char *)base + e * (uint32_t)sizeof(S)));
}
template <class S>
__device__ __forceinline__ void st_at(S *base, uint32_t e, S v)
{
    // non-temporal: the new PDFs stream out and are not read again in this
    // pass, so they should not displace lines the pulls still use
    __builtin_nontemporal_store(v, (S *)((char *)base + e * (uint32_t)sizeof(S)));
}
// Row streams of the dense kernel through buffer descriptors: one
// descriptor per row block (its 27 direction sub-rows, 27 nx values; the
// hardware returns 0 for loads and drops stores beyond it), the direction's
// sub-row offset i nx in the scalar offset register and the lane's x in the
// vector one, so that a load or store costs no vector address arithmetic.
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int BUF_WORD3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)
constexpr int BUF_NT = 2;              // cache policy: non-temporal (the new PDFs stream out)
template <class S>
__device__ __forceinline__ Rsrc row_rsrc(const S *pdf, int nx, int row)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)(pdf + pdf_index(nx, 0, row, 0)), 0,
                                             27 * nx * (int)sizeof(S), BUF_WORD3);
}
__device__ __forceinline__ float bload(const float *, Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double bload(const double *, Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, (u32x2)__builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ float bload(const _Float16 *, Rsrc r, uint32_t voff, uint32_t soff)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float v, Rsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, BUF_NT);
}
__device__ __forceinline__ void bstore(double v, Rsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, BUF_NT);
}
__device__ __forceinline__ void bstore(_Float16 v, Rsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, BUF_NT);
}

// Ties a loaded value to this point (an empty asm statement that reads and
// writes the register; no instruction is emitted).  Placed after all loads
// of a stage, it keeps the compiler from sinking a load into the branch of
// a select that consumes it, which would serialise the loads.
template <class T>
__device__ __forceinline__ void keep(T &v)
{
    asm volatile("" : "+v"(v));
}

// plain load of element e of a per-cell array (element offsets fit in 32
// bits: the lattice is limited to 2^32 / 8 cells)
template <class T>
__device__ __forceinline__ T at(const T *base, uint32_t e)
{
    return *(const T *)((const char *)base + e * (uint32_t)sizeof(T));
}

// one liquid cell of the dense step.  Every load of the cell is issued
// before any arithmetic so that a wavefront keeps all of its streams in
// flight; fl is the cell's flag byte (liquid).
// NEAR: the wavefront holds a cell next to a solid or a wall (the other
// lanes run the same code with an empty solid mask); without it the code
// has no bounce-back part at all.
// What one liquid cell of the dense step reads: the pulled PDFs, the stored
// mass, and next to solids the bounce-back values, the solid-link mask and
// the moving-wall record.
template <class S, bool NEAR>
struct BulkIn {
    using R = typename Real<S>::type;
    R f[27];
    double mq0;
    R fb[NEAR ? 27 : 1];
    uint4 rv[NEAR ? 28 * sizeof(R) / 16 : 1];
    uint32_t solid;
    int slot;
};

// The loads of one liquid cell of the dense step, all issued before any
// arithmetic so that a wavefront keeps its streams in flight; fl is the
// cell's flag byte (liquid).  NEAR: the wavefront holds a cell next to a
// solid or a wall (the other lanes run the same code with an empty solid
// mask); without it the code has no bounce-back part at all.
template <class S, bool NEAR>
__device__ __forceinline__ void bulk_loads(const Dev &d, const S *__restrict__ src, int x, int row, uint8_t fl,
                                           BulkIn<S, NEAR> &in)
{
    using R = typename Real<S>::type;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    // the row is the same over the wavefront: its PDF addresses are scalar
    row = __builtin_amdgcn_readfirstlane(row);
    const int y = row % ny, z = row / ny;
    const int c = x + nx * row;
    const bool near = NEAR && (fl & F_NEAR_SOLID) != 0;

    // bookkeeping loads first: the record slot gates a second round of loads
    in.mq0 = d.mq[c];
    in.solid = 0;
    in.slot = -1;
    if (near) {
        in.solid = d.smask[c];
        in.slot = d.bbslot[c];
    }

    // Source x - c_i: its row (scalar; periodic in y, z clamped -- the wall
    // layers are near-solid cells whose wall links are replaced) and its x
    // (per lane; periodic).  One descriptor per source row (index b + 3 c
    // for the row y + 1 - b, z + 1 - c) and the byte offset of each source x
    // per lane; the direction selects the sub-row through the scalar offset.
    const int ryp = y == ny - 1 ? 1 - ny : 1, rym = y == 0 ? ny - 1 : -1;
    const int rzp = z == nz - 1 ? 0 : ny, rzm = z == 0 ? 0 : -ny;
    const int xp = x == nx - 1 ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
    Rsrc rs[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if constexpr (sizeof(S) == 8) break;
        const int b = k % 3, cc = k / 3;
        rs[k] = row_rsrc(src, nx, row + (b == 0 ? ryp : (b == 2 ? rym : 0)) + (cc == 0 ? rzp : (cc == 2 ? rzm : 0)));
    }
    const uint32_t vx[3] = {(uint32_t)(xp * (int)sizeof(S)), (uint32_t)(x * (int)sizeof(S)),
                            (uint32_t)(xm * (int)sizeof(S))};
    const uint32_t sub = (uint32_t)(nx * (int)sizeof(S));  // bytes of one direction sub-row
    // (FP64 keeps plain loads from scalar row bases: with its 64-bit values
    // the descriptors' registers would cost it one of its two wavefronts
    // per SIMD)
    constexpr bool BUF = sizeof(S) < 8;
    auto pull = [&](int i) -> R {
        if constexpr (BUF) return bload(src, rs[i / 3], vx[i % 3], (uint32_t)i * sub);
        const int b = (i / 3) % 3, cc = i / 9;
        const int sr = row + (b == 0 ? ryp : (b == 2 ? rym : 0)) + (cc == 0 ? rzp : (cc == 2 ? rzm : 0));
        return ld_at(src + pdf_index(nx, 0, sr, 0), (uint32_t)(i * nx) + vx[i % 3] / (uint32_t)sizeof(S));
    };
#pragma unroll
    for (int i = 0; i < 27; ++i) in.f[i] = pull(i);

    if constexpr (NEAR) {
        // links whose source is solid or beyond a wall bounce back: the
        // cell's own post-collision value of the opposite direction, plus the
        // precomputed moving-wall term of sphere links (zero for wall links).
        // In FP32 only the lanes whose link is solid load it (fewer bytes;
        // the FP16 and FP64 forms run slower with the per-link masks).
#pragma unroll
        for (int j = 0; j < 27; ++j) in.fb[j] = R(0);
        if (near) {
#pragma unroll
            for (int j = 0; j < 27; ++j)
                if (j != REST && (sizeof(S) != 4 || ((in.solid >> j) & 1u)))
                    in.fb[j] = BUF ? bload(src, rs[4], vx[1], (uint32_t)opp(j) * sub)
                                   : ld_at(src + pdf_index(nx, 0, row, 0), (uint32_t)(opp(j) * nx + x));
        }
        load_record<R>(d, in.slot, in.rv);
    }
}

// The update of one liquid cell from its loads: bounce-back, mass
// bookkeeping, collision and the stores.
template <class S, bool NEAR, bool GC>
__device__ __forceinline__ void bulk_update(const Dev &d, S *__restrict__ dst, int x, int row,
                                            BulkIn<S, NEAR> &in, Watch &wd)
{
    using R = typename Real<S>::type;
    const int nx = d.nx, nz = d.nz;
    row = __builtin_amdgcn_readfirstlane(row);
    const int z = row / d.ny;
    const int c = x + nx * row;
    R *f = in.f;
    const uint32_t solid = NEAR ? in.solid : 0u;
    // incoming mass over the non-solid links; links beyond a z wall (the
    // bottom and top rows, uniform over the wavefront) carry no wall term
    double in_sum = 0.0;
    if constexpr (NEAR) {
        R rec[28];
        __builtin_memcpy(rec, in.rv, sizeof(in.rv));
        const int slot = in.slot;
#pragma unroll
        for (int j = 0; j < 27; ++j) {
            if (j == REST) continue;
            const bool sj = (solid >> j) & 1u;
            in_sum += sj ? 0.0 : (double)f[j];
            const bool wall = (z == 0 && j / 9 == 2) || (z == nz - 1 && j / 9 == 0);
            // FP16 storage keeps full records: its dense pass is bound by ALU
            // work rather than by the record bytes
            const R tm = sizeof(S) > 2 ? (wall ? R(0) : record_term<R>(rec, slot, j)) : rec[j];
            f[j] = sj ? in.fb[j] + tm : f[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < 27; ++j)
            if (j != REST) in_sum += (double)f[j];
    }

    using E = typename Eq<S>::type;
    E fo[27];
    double rho;
    collide<R, E, GC>(f, R(d.omega), R(d.gx), R(d.gy), R(d.gz), fo, rho);

    constexpr bool BUF = sizeof(S) < 8;
    const uint32_t sub = (uint32_t)(nx * (int)sizeof(S)), vx = (uint32_t)(x * (int)sizeof(S));
    double out_sum = 0.0;
    Rsrc rd;
    if constexpr (BUF) rd = row_rsrc(dst, nx, row);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const S v = to_store<S, E>(fo[i]);
        if constexpr (BUF) bstore(v, rd, vx, (uint32_t)i * sub);
        else st_at(dst + pdf_index(nx, 0, row, 0), (uint32_t)(i * nx + x), v);
        if (i != REST) out_sum += ((solid >> opp(i)) & 1u) ? 0.0 : (double)ld(&v);
    }
    // liquid cells keep m - own outgoing: m' = (m - out) + in over non-solid links
    const double m = in.mq0 + in_sum;
    d.mq[c] = m - out_sum;
    wd.add(m, rho);
}

// one liquid cell of the dense step: its loads, then its update
template <class S, bool NEAR, bool GC>
__device__ __forceinline__ void bulk_cell(const Dev &d, const S *__restrict__ src, S *__restrict__ dst,
                                          int x, int row, uint8_t fl, Watch &wd)
{
    BulkIn<S, NEAR> in;
    bulk_loads<S, NEAR>(d, src, x, row, fl, in);
    __builtin_amdgcn_sched_barrier(0);
    bulk_update<S, NEAR, GC>(d, dst, x, row, in, wd);
}

// Dense part over the rows (y, z) up to the highest fluid row; each block
// walks over 256-cell row segments, loading the flag byte of its next
// segment before it works on the current one.  With xcd_map, hardware
// block b runs on XCD b % 8 and takes whole rows k, k+8, k+16, ... of that
// XCD, so the segments of one row (which share cache lines at their edges)
// meet in one L2 while the liquid/gas split in z stays balanced over the
// XCDs.
template <class S, bool GC>
__device__ __forceinline__ void dense_rows(const Dev &d, const S *__restrict__ src, S *__restrict__ dst,
                                           int b, int nblocks, Watch &wd)
{
    const int rowmax = (d.cnt[3] + 1) * d.ny;
    const int tx = (int)threadIdx.x;
    const int nx = d.nx, nbx = d.nbx;
    int s, step, k;
    if (d.xcd_map) {
        k = b & 7;
        s = b >> 3;
        step = nblocks >> 3;
    } else {
        k = 0;
        s = b;
        step = nblocks;
    }
    const int rmul = d.xcd_map ? 8 : 1;
    // segment s -> (row, x); out-of-range lanes read as interface cells
    // (nothing to do).  Each pass takes the segments s and s + step.
    auto seg = [&](int sg, int &row, int &x, uint8_t &fl) {
        row = k + rmul * (sg / nbx);
        x = (sg % nbx) * BULK_THREADS + tx;
        fl = (row < rowmax && x < nx) ? d.flags[x + nx * row] : (uint8_t)T_IF;
    };
    int rowa, xa, rowb, xb;
    uint8_t fla, flb;
    seg(s, rowa, xa, fla);
    seg(s + step, rowb, xb, flb);
    while (rowa < rowmax) {
        s += 2 * step;
        int rowc, xc, rowd, xd;
        uint8_t flc, fld;
        seg(s, rowc, xc, flc);
        seg(s + step, rowd, xd, fld);
        const bool la = (fla & T_MASK) == T_LIQ, lb = (flb & T_MASK) == T_LIQ;
        if (__ballot((la && (fla & F_NEAR_SOLID)) || (lb && (flb & F_NEAR_SOLID))) != 0) {
            if (la) bulk_cell<S, true, GC>(d, src, dst, xa, rowa, fla, wd);
            if (lb) bulk_cell<S, true, GC>(d, src, dst, xb, rowb, flb, wd);
        } else if (__ballot(la || lb) != 0) {
            // (issuing both cells' loads before either update gains nothing
            // measurable here and costs the FP16 form a wavefront per SIMD)
            if (la) bulk_cell<S, false, GC>(d, src, dst, xa, rowa, fla, wd);
            if (lb) bulk_cell<S, false, GC>(d, src, dst, xb, rowb, flb, wd);
        }
        rowa = rowc;
        xa = xc;
        fla = flc;
        rowb = rowd;
        xb = xd;
        flb = fld;
    }
}

// four values of a record in one 16-byte store (FP32) or two (FP64): the
// records are 256-byte aligned, 8 or 32 values apart
__device__ __forceinline__ void store4(float *dst, float a, float b, float c, float e)
{
    *(float4 *)dst = make_float4(a, b, c, e);
}
__device__ __forceinline__ void store4(double *dst, double a, double b, double c, double e)
{
    ((double2 *)dst)[0] = make_double2(a, b);
    ((double2 *)dst)[1] = make_double2(c, e);
}

// moving-wall records of every cell that has sphere links (one thread per
// record, through the record-cell list)
template <class R>
__global__ void k_bb_terms(Dev d, int nrec)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrec) return;
    const int nc = d.cnt[4];
    const int c = t < nc ? d.rcell[t] : d.rcell[d.N - 1 - (t - nc)];
    const int slot = d.bbslot[c];
    const Cell pc = cell_xyz(d, c);
    const uint32_t sm = d.smask[c];
    if (slot <= -2) {
        R *rec = (R *)d.bbfull + (size_t)(-slot - 2) * 32;
        for (int j0 = 0; j0 < 32; j0 += 4) {
            R t[4] = {R(0), R(0), R(0), R(0)};
            for (int k = 0; k < 4; ++k) {
                const int j = j0 + k;
                if (j < 27 && j != REST && ((sm >> j) & 1u)) {
                    const int s = nb_of(d, pc, opp(j));
                    if (s >= 0) t[k] = bb_term<R>(d, s, j, pc);
                }
            }
            store4(rec + j0, t[0], t[1], t[2], t[3]);
        }
        return;
    }
    // compact: the (at most two) spheres in link order
    int q1 = -1, q2 = -1;
    uint32_t m2 = 0;
    for (int j = 0; j < 27; ++j) {
        if (j == REST || !((sm >> j) & 1u)) continue;
        const int s = nb_of(d, pc, opp(j));
        if (s < 0) continue;
        const int q = d.owner[s];
        if (q1 < 0 || q == q1) {
            q1 = q;
        } else {
            q2 = q;
            m2 |= 1u << j;
        }
    }
    double V1[3] = {0.0, 0.0, 0.0}, V2[3] = {0.0, 0.0, 0.0};
    if (q1 >= 0) rigid_velocity(d, q1, pc, V1);
    if (q2 >= 0) rigid_velocity(d, q2, pc, V2);
    R *h = (R *)d.bbterm + (size_t)slot * 8;
    R mbits = R(0);
    __builtin_memcpy(&mbits, &m2, 4);
    store4(h, R(V1[0]), R(V1[1]), R(V1[2]), R(V2[0]));
    store4(h + 4, R(V2[1]), R(V2[2]), mbits, R(0));
}

// ---------------------------------------------------------------- momentum exchange
// Force and torque on the spheres, Galilean-invariant momentum exchange for
// the streaming of the next step: each liquid or interface cell x with a
// link j whose source x - c_j belongs to sphere q sends f*_{opp j}(x)
// towards the wall and receives f_j = f*_{opp j} + 6 w_j c_j.u_w; q gains
// (c_{opp j} - u_w) f*_{opp j} - (c_j - u_w) f_j and the torque r x F, r the
// link midpoint's offset from the centre (u_w the rigid velocity there).
//
// Per sphere, the cells that can link into it are listed once per geometry
// (entries: cell index and the mask of its links into that sphere), in the
// fixed order of a walk over the sphere's bounding box widened by two cells
// (at most one period per axis).  The evaluation sums each sphere's entries
// in FP64 in a fixed order and reduces over a fixed tree: the result does
// not depend on scheduling.
struct SphereBox {
    int x0, y0, z0, ex, ey, ez;
};

__device__ __forceinline__ SphereBox sphere_box(const Dev &d, int q)
{
    const double *sp = d.sph + 10 * q;
    const double X = sp[0], Y = sp[1], Z = sp[2], rad = sp[3];
    SphereBox b;
    b.x0 = (int)floor(X - rad) - 2;
    b.y0 = (int)floor(Y - rad) - 2;
    b.ex = min((int)floor(X + rad) + 2 - b.x0 + 1, d.nx);
    b.ey = min((int)floor(Y + rad) + 2 - b.y0 + 1, d.ny);
    b.z0 = max((int)floor(Z - rad) - 2, 0);
    b.ez = max(min((int)floor(Z + rad) + 2, d.nz - 1) - b.z0 + 1, 0);
    return b;
}

// cell k of the walk over box b, and the mask of its links into sphere q
__device__ __forceinline__ uint32_t box_links(const Dev &d, const SphereBox &b, int q, int k, int &c)
{
    const int x = ((b.x0 + k % b.ex) % d.nx + d.nx) % d.nx;
    const int y = ((b.y0 + (k / b.ex) % b.ey) % d.ny + d.ny) % d.ny;
    const int z = b.z0 + k / (b.ex * b.ey);
    c = x + d.nx * (y + d.ny * z);
    if ((d.flags[c] & T_MASK) == T_SOLID) return 0u;
    const uint32_t sm = d.smask[c];
    uint32_t m = 0u;
    if (sm == 0u) return 0u;
    const Cell pc{x, y, z};
    int qo[27];
    const uint32_t vm = link_owners(d, pc, c, sm, qo);
#pragma unroll
    for (int j = 0; j < 27; ++j)
        if (((vm >> j) & 1u) && qo[j] == q) m |= 1u << j;
    return m;
}

// The walk over the cells of box b that can link into sphere q, in box
// order (z, then y, then x ascending from the box origin), one cell per
// thread and call of visit(m, c) (the mask of the cell's links into q and
// the cell; m = 0 for idle threads).  Every thread makes the same calls, so
// visit may synchronise the block.  A link into q starts within sqrt(3) of
// a cell centre at most r from the sphere's centre, so only cells centred
// within r + 1.75 can hold one, and cells centred within r - 0.5 are solid:
// per box row the walk takes the one or two x-runs of that shell.  Where
// the sphere nearly spans a periodic axis (the box's offsets may then not
// be the nearest image) it walks the whole box.
template <class Visit>
__device__ __forceinline__ void sphere_walk(const Dev &d, const SphereBox &b, int q, Visit &&visit)
{
    __shared__ int s_end[256], s_lo0[256], s_n0[256], s_lo1[256];
    const double *sp = d.sph + 10 * q;
    const double X = sp[0], Y = sp[1], Z = sp[2], rad = sp[3];
    const int t = (int)threadIdx.x;
    if (!(2.0 * (rad + 4.0) < (double)d.nx && 2.0 * (rad + 4.0) < (double)d.ny)) {
        const int ncell = b.ex * b.ey * b.ez;
        for (int k0 = 0; k0 < ncell; k0 += 256) {
            const int k = k0 + t;
            int c = 0;
            const uint32_t m = k < ncell ? box_links(d, b, q, k, c) : 0u;
            visit(m, c);
        }
        return;
    }
    const double ro = rad + 1.75, ri = rad - 0.5;
    const int nrow = b.ey * b.ez;
    for (int r0 = 0; r0 < nrow; r0 += 256) {
        // this thread's row of the chunk: its runs [lo0, lo0 + n0) and
        // [lo1, lo1 + n) - n0 (x offsets in the box)
        const int row = r0 + t;
        int lo0 = 0, n0 = 0, lo1 = 0, n = 0;
        if (row < nrow) {
            const double dy = (double)(b.y0 + row % b.ey) + 0.5 - Y, dz = (double)(b.z0 + row / b.ey) + 0.5 - Z;
            const double ho = ro * ro - dy * dy - dz * dz;
            if (ho >= 0.0) {
                const double wo = sqrt(ho);
                const int a = max((int)ceil(X - wo - 0.5) - b.x0, 0);
                const int e = min((int)floor(X + wo - 0.5) - b.x0, b.ex - 1);
                const double hi = ri * ri - dy * dy - dz * dz;
                int ia = e + 1, ie = e;
                if (ri > 0.0 && hi > 0.0) {
                    const double wi = sqrt(hi);
                    ia = max((int)ceil(X - wi - 0.5) - b.x0, a);
                    ie = min((int)floor(X + wi - 0.5) - b.x0, e);
                }
                if (a <= e) {
                    if (ia <= ie) {
                        lo0 = a;
                        n0 = ia - a;
                        lo1 = ie + 1;
                        n = n0 + (e - ie);
                    } else {
                        lo0 = a;
                        n0 = e - a + 1;
                        n = n0;
                    }
                }
            }
        }
        // inclusive prefix of the run lengths over the chunk's rows
        int inc = n;
        const int lane = __lane_id();
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
        s_lo0[t] = lo0;
        s_n0[t] = n0;
        s_lo1[t] = lo1;
        __syncthreads();
        for (int k0 = 0; k0 < total; k0 += 256) {
            const int k = k0 + t;
            uint32_t m = 0u;
            int c = 0;
            if (k < total) {
                // the row holding shell cell k: the first with s_end > k
                int lo = 0, hi = 255;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_end[mid] > k) hi = mid;
                    else lo = mid + 1;
                }
                const int j = k - (lo ? s_end[lo - 1] : 0);
                const int xi = j < s_n0[lo] ? s_lo0[lo] + j : s_lo1[lo] + (j - s_n0[lo]);
                m = box_links(d, b, q, xi + b.ex * (r0 + lo), c);
            }
            visit(m, c);
        }
        __syncthreads();
    }
}

// entries per sphere (one block per sphere)
__global__ __launch_bounds__(256) void k_mem_count(Dev d, int32_t *counts)
{
    __shared__ int s_cnt[4];
    const int q = blockIdx.x;
    const SphereBox b = sphere_box(d, q);
    int n = 0;
    sphere_walk(d, b, q, [&](uint32_t m, int) { n += m != 0u; });
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    if (__lane_id() == 0) s_cnt[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) counts[q] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

// The entries of sphere q in walk order into its slot, their number and the
// box they were taken from (one block per sphere).  With only_changed a
// sphere keeps its list when no remap marked it and its box is the same: a
// list depends only on the solid cells, solid-link masks and owners inside
// the box, which a remap changes only at the cells it marks.
__global__ __launch_bounds__(256) void k_mem_fill(Dev d, MemLists ml, int only_changed)
{
    __shared__ int s_cnt[4];
    const int q = blockIdx.x;
    const SphereBox b = sphere_box(d, q);
    int32_t *bx = ml.box + 6 * q;
    if (only_changed && ml.dirty[q] == 0 && bx[0] == b.x0 && bx[1] == b.y0 && bx[2] == b.z0 && bx[3] == b.ex &&
        bx[4] == b.ey && bx[5] == b.ez)
        return;
    const int start = ml.offs[q], cap = ml.offs[q + 1] - start;
    int base = 0;
    const int w = (int)threadIdx.x >> 6, lane = __lane_id();
    sphere_walk(d, b, q, [&](uint32_t m, int c) {
        const uint64_t bal = __ballot(m != 0u);
        if (lane == 0) s_cnt[w] = (int)__popcll(bal);
        __syncthreads();
        int pos = base;
        for (int i = 0; i < w; ++i) pos += s_cnt[i];
        pos += (int)__popcll(bal & ((1ull << lane) - 1ull));
        if (m != 0u && pos < cap) ml.ent[start + pos] = make_int2(c, (int)m);
        base += s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        __syncthreads();
    });
    // every thread has read dirty[q] and the box above
    __syncthreads();
    if (threadIdx.x == 0) {
        ml.cnt[q] = base;
        if (base > cap) ml.flag[0] = 1;
        bx[0] = b.x0;
        bx[1] = b.y0;
        bx[2] = b.z0;
        bx[3] = b.ex;
        bx[4] = b.ey;
        bx[5] = b.ez;
        ml.dirty[q] = 0;
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_mem(Dev d, int p, MemLists ml, double *out)
{
    __shared__ double sh[6][256];
    const int q = blockIdx.x;
    const double *sp = d.sph + 10 * q;
    const double X = sp[0], Y = sp[1], Z = sp[2];
    const int nx = d.nx, ny = d.ny;
    const S *pdf = (const S *)d.pdf[p];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int e0 = ml.offs[q], e1 = e0 + min(ml.cnt[q], ml.offs[q + 1] - e0);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
        const int2 en = ml.ent[e];
        const int c = en.x;
        const uint8_t ty = d.flags[c] & T_MASK;
        if (ty != T_LIQ && ty != T_IF) continue;
        const uint32_t m = (uint32_t)en.y;
        const int x = c % nx, y = (c / nx) % ny, z = c / (nx * ny);
        for (int j = 0; j < 27; ++j) {
            if (!((m >> j) & 1u)) continue;
            const double rx = min_image((x + 0.5 - 0.5 * cx(j)) - X, nx);
            const double ry = min_image((y + 0.5 - 0.5 * cy(j)) - Y, ny);
            const double rz = (z + 0.5 - 0.5 * cz(j)) - Z;
            const double ux = sp[4] + (sp[8] * rz - sp[9] * ry);
            const double uy = sp[5] + (sp[9] * rx - sp[7] * rz);
            const double uz = sp[6] + (sp[7] * ry - sp[8] * rx);
            const double fout = wgt(opp(j)) + (double)ld(pdf + pdf_index(nx, opp(j), c));
            const double fin = fout + 6.0 * wgt(j) * (cx(j) * ux + cy(j) * uy + cz(j) * uz);
            const double Fx = (-cx(j) - ux) * fout - (cx(j) - ux) * fin;
            const double Fy = (-cy(j) - uy) * fout - (cy(j) - uy) * fin;
            const double Fz = (-cz(j) - uz) * fout - (cz(j) - uz) * fin;
            acc[0] += Fx;
            acc[1] += Fy;
            acc[2] += Fz;
            acc[3] += ry * Fz - rz * Fy;
            acc[4] += rz * Fx - rx * Fz;
            acc[5] += rx * Fy - ry * Fx;
        }
    }
    for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[6 * (size_t)q + threadIdx.x] = sh[threadIdx.x][0];
}

void launch_mem_count(const Dev &d, int nsph, int32_t *counts, hipStream_t st)
{
    if (nsph > 0) k_mem_count<<<nsph, 256, 0, st>>>(d, counts);
}

void launch_mem_fill(const Dev &d, int nsph, const MemLists &ml, int only_changed, hipStream_t st)
{
    if (nsph > 0) k_mem_fill<<<nsph, 256, 0, st>>>(d, ml, only_changed);
}

template <class S>
void launch_mem(const Dev &d, int p, int nsph, const MemLists &ml, double *out, hipStream_t st)
{
    if (nsph > 0) k_mem<S><<<nsph, 256, 0, st>>>(d, p, ml, out);
}
template void launch_mem<double>(const Dev &, int, int, const MemLists &, double *, hipStream_t);
template void launch_mem<float>(const Dev &, int, int, const MemLists &, double *, hipStream_t);
template void launch_mem<_Float16>(const Dev &, int, int, const MemLists &, double *, hipStream_t);

constexpr int SLOT_THREADS = 1024, SLOT_CELLS = 4 * SLOT_THREADS;  // four cells per thread

// record kind of cell c with solid-link mask sm: 0 none, 1 compact, 2 full
__device__ __forceinline__ uint32_t slot_kind(const Dev &d, int c, uint32_t sm)
{
    if (sm == 0 || (d.flags[c] & T_MASK) == T_SOLID) return 0u;
    const Cell pc = cell_xyz(d, c);
    int q1 = -1, q2 = -1;
    bool more = false;
    for (int j = 0; j < 27; ++j) {
        if (j == REST || !((sm >> j) & 1u)) continue;
        const int s = nb_of(d, pc, opp(j));
        if (s < 0) continue;
        const int q = d.owner[s];
        if (q1 < 0 || q == q1) q1 = q;
        else if (q2 < 0 || q == q2) q2 = q;
        else more = true;
        if (d.img_check && !same_image(d, q, pc, j)) more = true;
    }
    if (q1 < 0) return 0u;
    return (more || !d.rec_compact) ? 2u : 1u;
}

// exclusive prefix over the block's threads (in thread order) of a and b,
// and the block totals
__device__ __forceinline__ void slot_scan(int a, int b, int &ea, int &eb, int &ta, int &tb)
{
    __shared__ int s_a[SLOT_THREADS / 64], s_b[SLOT_THREADS / 64];
    const int lane = __lane_id(), w = (int)threadIdx.x >> 6;
    int ia = a, ib = b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int ya = __shfl_up(ia, o), yb = __shfl_up(ib, o);
        if (lane >= o) {
            ia += ya;
            ib += yb;
        }
    }
    if (lane == 63) {
        s_a[w] = ia;
        s_b[w] = ib;
    }
    __syncthreads();
    int oa = 0, ob = 0;
    ta = 0;
    tb = 0;
    for (int k = 0; k < SLOT_THREADS / 64; ++k) {
        if (k == w) {
            oa = ta;
            ob = tb;
        }
        ta += s_a[k];
        tb += s_b[k];
    }
    ea = oa + ia - a;
    eb = ob + ib - b;
    __syncthreads();
}

// Cells with links into spheres get a record: compact when the links reach
// at most two spheres, full otherwise.  Three passes without contended
// atomics, numbering the records in cell order: each cell's kind and the
// per-block counts; exclusive prefix sums of the counts; slots from the
// kinds (compact records count up from 0, full ones from -2 down).
// With from_slots the kinds are read from the slot array instead, where a
// remap has re-encoded the cells whose kind may have changed (k_kinds_list).
__global__ __launch_bounds__(SLOT_THREADS) void k_slot_kinds(Dev d, uint8_t *kind, int32_t *bc, int32_t *bf,
                                                             int from_slots, int b0)
{
    const int t = (b0 + (int)blockIdx.x) * blockDim.x + threadIdx.x, c0 = 4 * t;
    // smask, or with from_slots the slot of each of the four cells
    uint32_t sm[4] = {0u, 0u, 0u, 0u};
    const uint32_t *src = from_slots ? (const uint32_t *)d.bbslot : d.smask;
    if (c0 + 3 < d.N) {
        const uint4 v = ((const uint4 *)src)[t];
        sm[0] = v.x, sm[1] = v.y, sm[2] = v.z, sm[3] = v.w;
    } else {
        for (int k = 0; k < 4 && c0 + k < d.N; ++k) sm[k] = src[c0 + k];
    }
    uint32_t packed = 0u;
    int nc = 0, nf = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t kd;
        if (from_slots) {
            const int sl = (int)sm[k];
            kd = c0 + k >= d.N ? 0u : (sl >= 0 ? 1u : (sl <= -2 ? 2u : 0u));
        } else {
            kd = sm[k] ? slot_kind(d, c0 + k, sm[k]) : 0u;
        }
        packed |= kd << (8 * k);
        nc += kd == 1u;
        nf += kd == 2u;
    }
    if (c0 + 3 < d.N) {
        ((uint32_t *)kind)[t] = packed;
    } else {
        for (int k = 0; k < 4 && c0 + k < d.N; ++k) kind[c0 + k] = (uint8_t)(packed >> (8 * k));
    }
    int ec, ef, tc, tf;
    slot_scan(nc, nf, ec, ef, tc, tf);
    if (threadIdx.x == 0) {
        bc[blockIdx.x] = tc;
        bf[blockIdx.x] = tf;
    }
}

// exclusive prefix sum of n counts in place (one block); the total to *total
__global__ __launch_bounds__(1024) void k_scan_counts(int32_t *v, int n, int32_t *total)
{
    __shared__ int s_w[16];
    __shared__ int s_carry;
    const int lane = __lane_id(), w = (int)threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int x = i < n ? v[i] : 0;
        int sc = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(sc, o);
            if (lane >= o) sc += y;
        }
        if (lane == 63) s_w[w] = sc;
        __syncthreads();
        int off = s_carry;
        for (int k = 0; k < w; ++k) off += s_w[k];
        if (i < n) v[i] = off + sc - x;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = off + sc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = s_carry;
}

// The kinds of the cells in list[0 .. *count) into their slot entries
// (0, -2 or -1 for compact, full or none): after a remap the only cells
// whose kind can change are the changed cells and their neighbours, and
// every other cell's slot entry still encodes its kind.
__global__ void k_kinds_list(Dev d, const int32_t *list, const int *count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= *count) return;
    const int c = list[t];
    const uint32_t sm = d.smask[c];
    const uint32_t kd = sm ? slot_kind(d, c, sm) : 0u;
    d.bbslot[c] = kd == 1u ? 0 : (kd == 2u ? -2 : -1);
}

__global__ __launch_bounds__(SLOT_THREADS) void k_slot_write(Dev d, const uint8_t *kind, const int32_t *bc,
                                                             const int32_t *bf, int b0)
{
    const int t = (b0 + (int)blockIdx.x) * blockDim.x + threadIdx.x, c0 = 4 * t;
    uint32_t packed = 0u;
    if (c0 + 3 < d.N) {
        packed = ((const uint32_t *)kind)[t];
    } else {
        for (int k = 0; k < 4 && c0 + k < d.N; ++k) packed |= (uint32_t)kind[c0 + k] << (8 * k);
    }
    int nc = 0, nf = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nc += ((packed >> (8 * k)) & 255u) == 1u;
        nf += ((packed >> (8 * k)) & 255u) == 2u;
    }
    int oc, of, tc, tf;
    slot_scan(nc, nf, oc, of, tc, tf);
    oc += bc[blockIdx.x];
    of += bf[blockIdx.x];
    int slot[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t kd = (packed >> (8 * k)) & 255u;
        slot[k] = -1;
        if (kd == 1u) {
            slot[k] = oc++;
            d.rcell[slot[k]] = c0 + k;
        } else if (kd == 2u) {
            slot[k] = -2 - of;
            d.rcell[d.N - 1 - of] = c0 + k;
            ++of;
        }
    }
    if (c0 + 3 < d.N) {
        ((int4 *)d.bbslot)[t] = make_int4(slot[0], slot[1], slot[2], slot[3]);
    } else {
        for (int k = 0; k < 4 && c0 + k < d.N; ++k) d.bbslot[c0 + k] = slot[k];
    }
}

// highest z that holds a liquid or interface cell
// (grid-stride; a maximum per block, then one atomic per block)
__global__ __launch_bounds__(256) void k_zmax(Dev d)
{
    __shared__ int s_max[4];
    // sixteen flag bytes per load (the flag array is 256-byte aligned); a
    // byte is liquid or interface when its two type bits differ
    const int nw = d.N >> 4;
    const uint4 *f4 = (const uint4 *)d.flags;
    int last = -1;   // highest fluid cell seen by this thread
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
        const uint4 v = f4[w];
        const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t t = (u[k] ^ (u[k] >> 1)) & 0x01010101u;
            if (t) last = 16 * w + 4 * k + (31 - __clz(t)) / 8;
        }
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < (d.N & 15)) {
        const int c = 16 * nw + (int)threadIdx.x;
        const uint8_t ty = d.flags[c] & T_MASK;
        if (ty == T_LIQ || ty == T_IF) last = max(last, c);
    }
    int zm = last >= 0 ? last / (d.nx * d.ny) : -1;
    for (int o = 32; o > 0; o >>= 1) zm = max(zm, __shfl_xor(zm, o));
    if (__lane_id() == 0) s_max[threadIdx.x >> 6] = zm;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int m = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
        if (m >= 0) atomicMax(&d.cnt[3], m);
    }
}

// ---------------------------------------------------------------- interface
// One interface cell: pull streaming with bounce-back at solid links and
// reconstruction of the links from the gas side (and of the links that
// point against the normal), the fill-weighted mass flux, collision, and
// the conversion marks.  GI: the normal and curvature are evaluated here
// from the fill stencil (finite differences); otherwise they are read from
// the geometry array (learned estimator).
// flux-modifier rank of an interface cell from its flag byte: 0 may only
// lose mass to other interface cells, 2 may only gain, 1 both (every cell
// when the variant is off, since the class bits are then never set)
__device__ __forceinline__ uint32_t fm_rank(uint32_t f)
{
    return 1u + ((f >> 6) & 1u) - ((f >> 5) & 1u);
}

template <class S, bool GI, bool GC>
__device__ __forceinline__ void iface_cell(const Dev &d, const S *__restrict__ src, S *__restrict__ dst,
                                           int c, uint32_t epoch)
{
    using R = typename Real<S>::type;
    using R4 = typename std::conditional<sizeof(R) == 8, double4, float4>::type;
    using Et = typename Eq<S>::type;
    const int nx = d.nx, ny = d.ny, nz = d.nz, nxy = nx * ny;
    const int x = c % nx, row = c / nx, y = row % ny, z = row / ny;
    // neighbour x + c_i = c + OX[cx+1] + OY[cy+1] + OZ[cz+1] (periodic in x
    // and y); -1 beyond the z walls
    const int OX[3] = {x == 0 ? nx - 1 : -1, 0, x == nx - 1 ? 1 - nx : 1};
    const int OY[3] = {y == 0 ? (ny - 1) * nx : -nx, 0, y == ny - 1 ? (1 - ny) * nx : nx};
    const int OZ[3] = {-nxy, 0, nxy};
    const bool WZ[3] = {z == 0, false, z == nz - 1};
    auto nb = [&](int i) { return WZ[i / 9] ? -1 : c + OX[i % 3] + OY[(i / 3) % 3] + OZ[i / 9]; };
    // PDF element of direction k at the neighbour x + c_i (the cell itself
    // beyond a z wall)
    const int RY[3] = {y == 0 ? ny - 1 : -1, 0, y == ny - 1 ? 1 - ny : 1};
    const int RZ[3] = {-ny, 0, ny};
    auto pdf_nb = [&](int k, int i) {
        return WZ[i / 9] ? pdf_index(nx, k, row, x)
                         : pdf_index(nx, k, row + RY[(i / 3) % 3] + RZ[i / 9], x + OX[i % 3]);
    };

    // stage 1: neighbour types (walls count as solid, 2 bits each) and the
    // fill stencil (liquid 1, gas 0, interface clamped fill, solid the centre)
    const double phic = d.phi[c];
    const int slot = d.bbslot[c];
    const double phicl = fmin(fmax(phic, 0.0), 1.0);
    uint32_t fl[27];
    double ph[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int n = nb(i);
        const uint32_t a = (uint32_t)(n < 0 ? c : n);
        fl[i] = at(d.flags, a);
        ph[i] = at(d.phi, a);
    }
    // stage 2 loads follow at once (they depend on nothing loaded above) and
    // arrive while the geometry is evaluated: the cell's own post-collision
    // PDFs and the pulled ones
    R own[27], pulled[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        own[i] = ld(src + pdf_index(nx, i, row, x));
        // source of incoming i is x - c_i = neighbour opp(i)
        pulled[i] = ld(src + pdf_nb(i, opp(i)));
    }
    double mq0 = d.mq[c];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        keep(fl[i]);
        keep(ph[i]);
    }
    // moving-wall terms of the links into spheres (zero for walls); the
    // record slot has arrived with the stencil
    uint4 rv[28 * sizeof(R) / 16];
    load_record<R>(d, slot, rv);
    R rec[28];
    __builtin_memcpy(rec, rv, sizeof(rv));
    uint64_t tyb = 0, rkb = 0;
    double sv[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const uint32_t t = nb(i) < 0 ? (uint32_t)T_SOLID : (fl[i] & T_MASK);
        const double pv = fmin(fmax(ph[i], 0.0), 1.0);
        tyb |= (uint64_t)t << (2 * i);
        rkb |= (uint64_t)fm_rank(fl[i]) << (2 * i);
        // liquid 1, gas 0, interface its clamped fill, solid or wall the
        // centre's, as a sum of the cases (arithmetic, not a branch chain)
        sv[i] = i == REST ? phicl
                          : (double)(t == T_LIQ) + (double)(t == T_IF) * pv + (double)(t == T_SOLID) * phicl;
    }
    auto ty = [&](int i) { return (uint32_t)(tyb >> (2 * i)) & 3u; };
    auto rk = [&](int i) { return (uint32_t)(rkb >> (2 * i)) & 3u; };
    double4 gn;
    if constexpr (GI) {
        gn = fd_geometry(sv);
        if (d.variants & VAR_CSF_CURVATURE) gn.w = csf_curvature(sv);
    } else {
        const R4 g = ((const R4 *)d.geom)[c];
        gn = make_double4((double)g.x, (double)g.y, (double)g.z, (double)g.w);
    }
    __builtin_amdgcn_sched_barrier(0);

    // stage 2 values
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        keep(own[i]);
        keep(pulled[i]);
    }
    keep(mq0);

    // mass flux from the stored PDFs: s_i (f*_{-i}(x+c_i) - f*_i(x)); with
    // the flux modifiers, between interface cells of different ranks only
    // the term that moves mass from the lower to the higher rank is kept
    // Written with selects only (no per-lane branches), like the
    // reconstruction below: see the note at the mass store.
    double dm = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if (i == REST) continue;
        const uint32_t t = ty(i);
        const bool flows = (t == T_LIQ) | (t == T_IF), itf = t == T_IF;
        const double sw = itf ? 0.5 * (phicl + sv[i]) : 1.0;
        // a single kept term is a whole PDF: the stored deviations get their
        // weight back (w_{-i} = w_i), which the difference of two terms cancels
        const bool lower = itf & (rk(REST) < rk(i)), higher = itf & (rk(REST) > rk(i));
        const double in0 = (double)pulled[opp(i)], out0 = (double)own[i];
        const double in = lower ? 0.0 : (higher ? in0 + wgt(i) : in0);
        const double out = higher ? 0.0 : (lower ? out0 + wgt(i) : out0);
        dm += flows ? sw * (in - out) : 0.0;
    }
    // The new mass is stored here and read back for the conversion marks
    // below, so that no mass value has to stay in registers through the
    // reconstruction and the collision.  Builds of this kernel whose flux
    // and reconstruction compiled to per-lane branches handed a value live
    // across them to only one side of a branch (the other lanes summed a
    // stale register); the loops are now written with selects and the mass
    // is not carried.  The read-back is a fresh load of the cell's own, just
    // written entry (an empty asm with a memory clobber keeps the compiler
    // from forwarding the stored value).
    d.mq[c] = mq0 + dm;
    __builtin_amdgcn_sched_barrier(0);

    // stage 3: the collision    // gas-side equilibrium at rho_gas + 6 sigma kappa and the cell's own
    // post-collision velocity (formed like the collision's equilibrium
    // part, in FP64 unless the storage is FP16)
    double drho_o = 0.0, jxo = 0.0, jyo = 0.0, jzo = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const double v = (double)own[i];
        drho_o += v;
        jxo += cx(i) * v;
        jyo += cy(i) * v;
        jzo += cz(i) * v;
    }
    const double irho_o = 1.0 / (1.0 + drho_o);
    Et ef[3][3];
    psi_dev<Et>(Et(jxo * irho_o), Et(jyo * irho_o), Et(jzo * irho_o), ef);
    const Et drg = Et(d.rho_gas - 1.0 + 6.0 * d.sigma * gn.w);

    // incoming PDFs, by pairs (j, opp j) that share the sum of the two
    // gas-side equilibria.  Every candidate -- bounce-back, reconstruction,
    // streamed value -- is formed for every link and one is selected (the
    // equilibria are tied to registers first, so the compiler cannot move
    // them into per-lane branches).
    Et G[REST];
#pragma unroll
    for (int j = 0; j < REST; ++j) {
        G[j] = feq_dev_one<Et>(drg, ef, j) + feq_dev_one<Et>(drg, ef, opp(j));
        keep(G[j]);
    }
    R f[27];
    f[REST] = own[REST];
#pragma unroll
    for (int j = 0; j < REST; ++j) {
        const int sj = opp(j);
        const double nc = gn.x * cx(j) + gn.y * cy(j) + gn.z * cz(j);  // n . c_j = -(n . c_sj)
        const uint32_t tj = ty(j), tsj = ty(sj);
        // incoming j comes from neighbour sj, incoming sj from neighbour j
        const bool rj = (tsj == T_GAS) | (nc < -d.tie);
        const bool rsj = (tj == T_GAS) | (-nc < -d.tie);
        // wall links (no neighbour) carry no wall term
        const R tmj = sizeof(S) == 2 ? rec[j] : (nb(sj) < 0 ? R(0) : record_term<R>(rec, slot, j));
        const R tmsj = sizeof(S) == 2 ? rec[sj] : (nb(j) < 0 ? R(0) : record_term<R>(rec, slot, sj));
        const R bj = own[sj] + tmj, bsj = own[j] + tmsj;
        const R gj = R(G[j] - Et(own[sj])), gsj = R(G[j] - Et(own[j]));
        f[j] = tsj == T_SOLID ? bj : (rj ? gj : pulled[j]);
        f[sj] = tj == T_SOLID ? bsj : (rsj ? gsj : pulled[sj]);
    }

    Et fo[27];
    double rho_in;
    collide<R, Et, GC>(f, R(d.omega), R(d.gx), R(d.gy), R(d.gz), fo, rho_in);

    double rs = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const S v = to_store<S, Et>(fo[i]);
        __builtin_nontemporal_store(v, dst + pdf_index(nx, i, row, x));
        rs += (double)ld(&v);
    }
    const double rho = 1.0 + rs;
    asm volatile("" ::: "memory");
    const double m = d.mq[c];
    d.rho[c] = rho;

    uint32_t bits = 0;
    if (m > (1.0 + d.eps) * rho) {
        bits = MK_TO_LIQ;
    } else if (m < -d.eps * rho) {
        bits = MK_TO_GAS;
    } else if (d.rule_iso) {
        bool has_gas = false, has_liq = false;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (i == REST || nb(i) < 0) continue;
            has_gas |= ty(i) == T_GAS;
            has_liq |= ty(i) == T_LIQ;
        }
        if (!has_gas && has_liq) bits = MK_TO_LIQ | MK_ISO;
        else if (!has_liq && has_gas) bits = MK_TO_GAS | MK_ISO;
    }
    d.mark[c] = (epoch << 8) | bits;
    if constexpr (GI) {
        // the normal-weighted excess of a converting cell needs its normal
        if ((d.variants & VAR_NORMAL_EXCESS) && (bits & (MK_TO_LIQ | MK_TO_GAS))) {
            R4 g;
            g.x = R(gn.x);
            g.y = R(gn.y);
            g.z = R(gn.z);
            g.w = R(gn.w);
            ((R4 *)d.geom)[c] = g;
        }
    }
}

// Flux-modifier classes of the interface cells from the cell types at the
// start of the step (Thuerey 2007): F_CLS_LOSE with gas but no liquid
// neighbours, F_CLS_GAIN with liquid but no gas neighbours.  Only the class
// bits of the cell's own flag byte change, so concurrent readers of its type
// are unaffected.
__global__ __launch_bounds__(LIST_THREADS) void k_classes(Dev d, int p)
{
    const int32_t *list = d.list[p];
    const int count = d.cnt[p];
    const int nx = d.nx, ny = d.ny, nz = d.nz, nxy = nx * ny;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
        const int c = list[t];
        const int x = c % nx, row = c / nx, y = row % ny, z = row / ny;
        const int OX[3] = {x == 0 ? nx - 1 : -1, 0, x == nx - 1 ? 1 - nx : 1};
        const int OY[3] = {y == 0 ? (ny - 1) * nx : -nx, 0, y == ny - 1 ? (1 - ny) * nx : nx};
        const int OZ[3] = {z == 0 ? 0 : -nxy, 0, z == nz - 1 ? 0 : nxy};
        const bool WZ[3] = {z == 0, false, z == nz - 1};
        // every neighbour's flag byte at once (beyond a wall: the cell's own,
        // ignored below)
        uint32_t f[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) f[i] = at(d.flags, (uint32_t)(c + OX[i % 3] + OY[(i / 3) % 3] + OZ[i / 9]));
        bool g = false, q = false;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (i == REST || WZ[i / 9]) continue;
            const uint32_t ty = f[i] & T_MASK;
            g |= ty == T_GAS;
            q |= ty == T_LIQ;
        }
        const uint8_t cls = (g && !q) ? F_CLS_LOSE : ((q && !g) ? F_CLS_GAIN : 0);
        d.flags[c] = (uint8_t)((f[REST] & ~(F_CLS_LOSE | F_CLS_GAIN)) | cls);
    }
}

// Interface list of the step (one cell per thread).  Block 0 starts the
// next list and the new-cell list empty.  GC: with the Galilean correction
// of the collision (a compile-time flag, as in the dense kernel, so that the
// instance without it keeps its own code).
// The interface kernel keeps no watchdog accumulators: values kept live
// across its whole loop (five more registers) made the compiler's register
// allocation hand the cell's mass to only one side of a divergent branch;
// k_conv1 takes the interface partial from the stored mass and density.
template <class S, bool GI, bool GC>
__global__ __launch_bounds__(LIST_THREADS) void k_iface(Dev d, int p, uint32_t epoch)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.cnt[p ^ 1] = 0;
        d.cnt[2] = 0;
    }
    const S *__restrict__ src = (const S *)d.pdf[p];
    S *__restrict__ dst = (S *)d.pdf[p ^ 1];
    const int32_t *list = d.list[p];
    const int count = d.cnt[p];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x)
        iface_cell<S, GI, GC>(d, src, dst, list[t], epoch);
}

// Dense stream-collide over the liquid rows; GC: with the Galilean
// correction of the collision.  Each block writes its partial of the
// watchdog and of the global mass (liquid mass after streaming, density
// range) to wd[WD_BULK + 4 block].
template <class S, bool GC>
__global__ __launch_bounds__(BULK_THREADS) void k_bulk(Dev d, int p)
{
    Watch wd;
    dense_rows<S, GC>(d, (const S *)d.pdf[p], (S *)d.pdf[p ^ 1], (int)blockIdx.x, (int)gridDim.x, wd);
    block_watch<BULK_THREADS>(wd, d.wd + WD_BULK + 4 * blockIdx.x);
}

// Watchdog result of a step: the partials of the nb dense and ni interface
// blocks summed in a fixed order, plus the pool; wd[WD_OUT ..] = total mass,
// lowest and highest density, cells outside [0.5, 1.5].  The mass is the
// liquid and interface mass before the step's conversions, which only move
// mass between cells and the pool, so it equals the total after the step to
// rounding.
__global__ __launch_bounds__(256) void k_watch_final(Dev d, int nb, int ni)
{
    Watch w;
    for (int i = (int)threadIdx.x; i < nb + ni; i += 256) {
        const double *q = d.wd + (i < nb ? WD_BULK + 4 * i : WD_IFACE + 4 * (i - nb));
        w.mass += q[0];
        w.rmin = fminf(w.rmin, (float)q[1]);
        w.rmax = fmaxf(w.rmax, (float)q[2]);
        w.bad += (int)q[3];
    }
    block_watch<256>(w, d.wd + WD_OUT);
    __syncthreads();
    if (threadIdx.x == 0) d.wd[WD_OUT] += d.wd[WD_POOL_SNAP];
}

// ---------------------------------------------------------------- conversion
__device__ __forceinline__ void push_new(const Dev &d, int c, uint32_t epoch, unsigned long long stat)
{
    const uint32_t old = atomicMax(&d.mark[c], (epoch << 8) | MK_NEW);
    if ((old >> 8) != epoch) {
        const int k = atomicAdd(&d.cnt[2], 1);
        d.lnew[k] = c;
        atomicAdd(&d.stats[stat], 1ull);
    }
}

// Each block also writes the watchdog and global-mass partial of its
// interface cells (mass after the flux, density) to wd[WD_IFACE + 4 block],
// and block 0 keeps the pool total before this step's conversions.
__global__ __launch_bounds__(LIST_THREADS) void k_conv1(Dev d, int p, uint32_t epoch)
{
    const int32_t *list = d.list[p];
    const int count = d.cnt[p];
    Watch wd;
    if (blockIdx.x == 0 && threadIdx.x == 0) d.wd[WD_POOL_SNAP] = d.wd[WD_POOL];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
        const int c = list[t];
        wd.add(d.mq[c], d.rho[c]);
        const uint32_t mk = mark_bits(d.mark[c], epoch);
        if (!(mk & (MK_TO_LIQ | MK_TO_GAS))) continue;
        const Cell pc = cell_xyz(d, c);
        if (mk & MK_TO_LIQ) {
            atomicAdd(&d.stats[(mk & MK_ISO) ? 2 : 0], 1ull);
            for (int i = 0; i < 27; ++i) {
                if (i == REST) continue;
                const int y = nb_of(d, pc, i);
                if (y >= 0 && (d.flags[y] & T_MASK) == T_GAS) push_new(d, y, epoch, 5);
            }
        } else {
            bool near_fill = false;
            for (int i = 0; i < 27 && !near_fill; ++i) {
                if (i == REST) continue;
                const int y = nb_of(d, pc, i);
                if (y >= 0 && (mark_bits(d.mark[y], epoch) & MK_TO_LIQ)) near_fill = true;
            }
            if (near_fill) {
                atomicAdd(&d.stats[4], 1ull);
                continue;
            }
            atomicOr(&d.mark[c], MK_EMPTY);
            atomicAdd(&d.stats[(mk & MK_ISO) ? 3 : 1], 1ull);
            for (int i = 0; i < 27; ++i) {
                if (i == REST) continue;
                const int y = nb_of(d, pc, i);
                if (y >= 0 && (d.flags[y] & T_MASK) == T_LIQ) push_new(d, y, epoch, 6);
            }
        }
    }
    block_watch<LIST_THREADS>(wd, d.wd + WD_IFACE + 4 * blockIdx.x);
}

// sum of a cell's stored deviations over all directions (all) and over the
// outgoing directions whose target is not solid, rest excluded (fluid)
template <class S>
__device__ __forceinline__ void stored_sums(const Dev &d, const S *pdf, int c, const Cell &pc,
                                            double &all, double &fluid)
{
    all = 0.0;
    fluid = 0.0;
    for (int i = 0; i < 27; ++i) {
        const double v = (double)ld(pdf + pdf_index(d.nx, i, c));
        all += v;
        if (i == REST) continue;
        const int y = nb_of(d, pc, i);
        if (y >= 0 && (d.flags[y] & T_MASK) != T_SOLID) fluid += v;
    }
}

// a cell that becomes an interface cell this step
template <class S>
__device__ __forceinline__ void conv2_cell(const Dev &d, int p, uint32_t epoch, int c)
{
    S *pdf = (S *)d.pdf[p ^ 1];
    {
        const Cell pc = cell_xyz(d, c);
        if ((d.flags[c] & T_MASK) == T_GAS) {
            // equilibrium at the mean density and velocity of the liquid and
            // old interface neighbours that are not marked for emptying
            double rs = 0.0, us[3] = {0.0, 0.0, 0.0};
            int n = 0;
            for (int i = 0; i < 27; ++i) {
                if (i == REST) continue;
                const int y = nb_of(d, pc, i);
                if (y < 0) continue;
                const uint8_t ty = d.flags[y] & T_MASK;
                if (ty != T_LIQ && ty != T_IF) continue;
                if (mark_bits(d.mark[y], epoch) & MK_TO_GAS) continue;
                double r = 0.0, j[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < 27; ++k) {
                    const double v = (double)ld(pdf + pdf_index(d.nx, k, y));
                    r += v;
                    j[0] += cx(k) * v;
                    j[1] += cy(k) * v;
                    j[2] += cz(k) * v;
                }
                r += 1.0;
                rs += r;
                for (int a = 0; a < 3; ++a) us[a] += j[a] / r;
                ++n;
            }
            using Et = typename Eq<S>::type;
            const double rb = rs / n;
            Et e[27];
            feq_dev<Et>(Et(rb - 1.0), Et(us[0] / n), Et(us[1] / n), Et(us[2] / n), e);
            double sum = 0.0;
            for (int i = 0; i < 27; ++i) {
                const S v = to_store<S, Et>(e[i]);
                pdf[pdf_index(d.nx, i, c)] = v;
                sum += (double)ld(&v);
            }
            d.mq[c] = 0.0;
            d.rho[c] = 1.0 + sum;
        } else {
            // liquid -> interface keeps its PDFs and mass
            double all, fluid;
            stored_sums(d, (const S *)pdf, c, pc, all, fluid);
            d.mq[c] = d.mq[c] + fluid;
            d.rho[c] = 1.0 + all;
        }
    }
}

__device__ __forceinline__ bool interface_after(const Dev &d, int y, uint32_t epoch)
{
    const uint32_t mk = mark_bits(d.mark[y], epoch);
    if (mk & MK_NEW) return true;
    return (d.flags[y] & T_MASK) == T_IF && !(mk & (MK_TO_LIQ | MK_EMPTY));
}

// weight of the link c_i from a converted cell with normal n (liquid to gas)
// when the excess is shared by normal weights: along n for a filled cell,
// against it for an emptied one; projections up to the normal tie are zero
__device__ __forceinline__ double excess_weight(const double (&n)[3], int i, bool filled, double tie)
{
    double nc = n[0] * cx(i) + n[1] * cy(i) + n[2] * cz(i);
    if (!filled) nc = -nc;
    return nc > tie ? nc : 0.0;
}

template <class S>
__device__ __forceinline__ void load_normal(const Dev &d, int c, double (&n)[3])
{
    using R = typename Real<S>::type;
    using R4 = typename std::conditional<sizeof(R) == 8, double4, float4>::type;
    const R4 g = ((const R4 *)d.geom)[c];
    n[0] = (double)g.x;
    n[1] = (double)g.y;
    n[2] = (double)g.z;
}

// excess mass of an interface cell that fills or empties this step
template <class S>
__device__ __forceinline__ void conv3_cell(const Dev &d, int p, uint32_t epoch, int c)
{
    const S *pdf = (const S *)d.pdf[p ^ 1];
    {
        const uint32_t mk = mark_bits(d.mark[c], epoch);
        const bool filled = mk & MK_TO_LIQ, emptied = mk & MK_EMPTY;
        if (!filled && !emptied) return;
        const Cell pc = cell_xyz(d, c);
        double e;
        if (filled) {
            e = d.mq[c] - d.rho[c];
            double all, fluid;
            stored_sums(d, pdf, c, pc, all, fluid);
            d.mq[c] = d.rho[c] - fluid;  // liquid form: m minus own outgoing
        } else {
            e = d.mq[c];
            d.mq[c] = 0.0;
        }
        const bool weighted = (d.variants & VAR_NORMAL_EXCESS) != 0;
        double n[3] = {0.0, 0.0, 0.0};
        if (weighted) load_normal<S>(d, c, n);
        int recv = 0;
        double wsum = 0.0;
        for (int i = 0; i < 27; ++i) {
            if (i == REST) continue;
            const int y = nb_of(d, pc, i);
            if (y >= 0 && interface_after(d, y, epoch)) {
                ++recv;
                if (weighted) wsum += excess_weight(n, i, filled, d.tie);
            }
        }
        if (wsum > 0.0) {
            // the receiver along c_i takes share * weight of c_i
            d.share[c] = e / wsum;
            atomicOr(&d.mark[c], MK_WEIGHTED);
        } else if (recv > 0) {
            d.share[c] = e / recv;
        } else {
            d.share[c] = 0.0;
            d.poolc[c] += e;
            atomicAdd(d.wd + WD_POOL, e);  // running pool total (watchdog)
        }
    }
}

// The new interface cells (lnew) and the converted cells of the interface
// list touch disjoint cells, so both run in one launch.
template <class S>
__global__ __launch_bounds__(LIST_THREADS) void k_conv23(Dev d, int p, uint32_t epoch)
{
    const int nnew = d.cnt[2], ncur = d.cnt[p];
    const int n = nnew > ncur ? nnew : ncur;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        if (t < nnew) conv2_cell<S>(d, p, epoch, d.lnew[t]);
        if (t < ncur) conv3_cell<S>(d, p, epoch, d.list[p][t]);
    }
}

// Block-aggregated append of `value` to list[] when pred holds: one atomic
// per workgroup.  Every thread of the block must call it (uniform control).
__device__ __forceinline__ void block_append(int32_t *list, int32_t *counter, bool pred, int32_t value)
{
    __shared__ int s_cnt[LIST_THREADS / 64];
    __shared__ int s_base;
    const uint64_t m = __ballot(pred);
    const int w = (int)threadIdx.x >> 6, lane = __lane_id();
    if (lane == 0) s_cnt[w] = (int)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
#pragma unroll
        for (int k = 0; k < LIST_THREADS / 64; ++k) tot += s_cnt[k];
        s_base = tot ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    int base = s_base;
    for (int k = 0; k < w; ++k) base += s_cnt[k];
    if (pred) list[base + (int)__popcll(m & ((1ull << lane) - 1ull))] = value;
    __syncthreads();
}

template <class S>
__global__ __launch_bounds__(LIST_THREADS) void k_conv4(Dev d, int p, uint32_t epoch)
{
    const int32_t *list = d.list[p];
    const int ncur = d.cnt[p];
    const int total = ncur + d.cnt[2];
    const int nxy = d.nx * d.ny;
    // block-uniform trip count: every thread reaches the block-wide append
    for (int t0 = blockIdx.x * LIST_THREADS; t0 < total; t0 += gridDim.x * LIST_THREADS) {
        const int t = t0 + (int)threadIdx.x;
        int c = 0;
        bool kept = false;
        int newz = -1;
        if (t < ncur) {
            c = list[t];
            const uint32_t mk = mark_bits(d.mark[c], epoch);
            kept = true;
            if (mk & (MK_TO_LIQ | MK_EMPTY)) {
                d.flags[c] = (uint8_t)((d.flags[c] & ~T_MASK) | ((mk & MK_TO_LIQ) ? T_LIQ : T_GAS));
                kept = false;
            }
        } else if (t < total) {
            c = d.lnew[t - ncur];
            d.flags[c] = (uint8_t)((d.flags[c] & ~T_MASK) | T_IF);
            newz = c / nxy;
            kept = true;
        }
        // highest fluid row: one atomic per wavefront
        int zw = newz;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) zw = max(zw, __shfl_xor(zw, o));
        if (__lane_id() == 0 && zw >= 0) atomicMax(&d.cnt[3], zw);
        if (kept) {
            const Cell pc = cell_xyz(d, c);
            double mq0 = d.mq[c], rho0 = d.rho[c];
            int nb[27];
            uint32_t mk[27];
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                nb[i] = i == REST ? -1 : nb_of(d, pc, i);
                mk[i] = at(d.mark, (uint32_t)(nb[i] < 0 ? c : nb[i]));
            }
#pragma unroll
            for (int i = 0; i < 27; ++i) keep(mk[i]);
            keep(mq0);
            keep(rho0);
            // seen from the converted neighbour y = c + c_i, this cell lies
            // along -c_i
            double add = 0.0;
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                if (nb[i] < 0) continue;
                const uint32_t b = mark_bits(mk[i], epoch);
                if (!(b & (MK_TO_LIQ | MK_EMPTY))) continue;
                double s = d.share[nb[i]];
                if (b & MK_WEIGHTED) {
                    double n[3];
                    load_normal<S>(d, nb[i], n);
                    s *= excess_weight(n, opp(i), (b & MK_TO_LIQ) != 0, d.tie);
                }
                add += s;
            }
            const double m = mq0 + add;
            d.mq[c] = m;
            d.phi[c] = m / rho0;
        }
        block_append(d.list[p ^ 1], &d.cnt[p ^ 1], kept, c);
    }
}

// ---------------------------------------------------------------- geometry
template <class R>
__device__ __forceinline__ R stencil_value(const Dev &d, int y, R centre)
{
    if (y < 0) return centre;
    switch (d.flags[y] & T_MASK) {
    case T_LIQ: return R(1);
    case T_GAS: return R(0);
    case T_IF: {
        double v = d.phi[y];
        return R(v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v));
    }
    default: return centre;
    }
}

// Normal and curvature of each interface cell from its fill stencil
// (finite differences, evaluated in FP64 for every storage form), stored as R.
template <class R>
__global__ __launch_bounds__(LIST_THREADS) void k_geom(Dev d, int which)
{
    using R4 = typename std::conditional<sizeof(R) == 8, double4, float4>::type;
    const int32_t *list = d.list[which];
    const int count = d.cnt[which];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
        const int c = list[t];
        const Cell pc = cell_xyz(d, c);
        const double pv = d.phi[c];
        const double centre = pv < 0.0 ? 0.0 : (pv > 1.0 ? 1.0 : pv);
        double s[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) s[i] = i == REST ? centre : stencil_value<double>(d, nb_of(d, pc, i), centre);
        double4 o = fd_geometry(s);
        if (d.variants & VAR_CSF_CURVATURE) o.w = csf_curvature(s);
        R4 out;
        out.x = R(o.x);
        out.y = R(o.y);
        out.z = R(o.z);
        out.w = R(o.w);
        ((R4 *)d.geom)[c] = out;
    }
}

// ---------------------------------------------------------------- launchers
// workgroups of the persistent dense kernel
static int bulk_grid(const Dev &d)
{
    int gb = d.bulk_blocks > 0 ? d.bulk_blocks : d.nbx * d.rows;
    if (gb > BULK_MAX_BLOCKS) gb = BULK_MAX_BLOCKS;
    if (d.xcd_map) gb &= ~7;
    return gb;
}

// the watchdog result (and global mass) of the last step from its partials
void launch_watch_final(const Dev &d, int list_blocks, hipStream_t st)
{
    k_watch_final<<<1, 256, 0, st>>>(d, bulk_grid(d), list_blocks);
}

template <class S>
void launch_step(const Dev &d, int p, uint32_t epoch, int list_blocks, int watch, hipStream_t st,
                 hipEvent_t ev0, hipEvent_t ev1, const float *mlpP, const uint16_t *mlpPk)
{
    using R = typename Real<S>::type;
    const int gb = bulk_grid(d);
    const bool gc = (d.variants & VAR_GALILEAN) != 0;
    if (ev0) (void)hipEventRecord(ev0, st);
    if (gc)
        k_bulk<S, true><<<gb, BULK_THREADS, 0, st>>>(d, p);
    else
        k_bulk<S, false><<<gb, BULK_THREADS, 0, st>>>(d, p);
    if (ev1) (void)hipEventRecord(ev1, st);
    if (d.variants & VAR_FLUX_MODIFIERS) k_classes<<<list_blocks, LIST_THREADS, 0, st>>>(d, p);
    if (mlpP) {
        if (gc) k_iface<S, false, true><<<list_blocks, LIST_THREADS, 0, st>>>(d, p, epoch);
        else k_iface<S, false, false><<<list_blocks, LIST_THREADS, 0, st>>>(d, p, epoch);
    } else {
        if (gc) k_iface<S, true, true><<<list_blocks, LIST_THREADS, 0, st>>>(d, p, epoch);
        else k_iface<S, true, false><<<list_blocks, LIST_THREADS, 0, st>>>(d, p, epoch);
    }
    k_conv1<<<list_blocks, LIST_THREADS, 0, st>>>(d, p, epoch);
    // the watchdog result is complete before the conversions touch the pool
    if (watch) k_watch_final<<<1, 256, 0, st>>>(d, gb, list_blocks);
    k_conv23<S><<<list_blocks, LIST_THREADS, 0, st>>>(d, p, epoch);
    k_conv4<S><<<list_blocks, LIST_THREADS, 0, st>>>(d, p, epoch);
    if (mlpP) launch_geom_mlp<R>(d, p ^ 1, list_blocks, mlpP, mlpPk, st);
}

#define FSL_STEP_INST(S)                                                                          \
    template void launch_step<S>(const Dev &, int, uint32_t, int, int, hipStream_t, hipEvent_t, hipEvent_t, \
                                 const float *, const uint16_t *);
FSL_STEP_INST(double)
FSL_STEP_INST(float)
FSL_STEP_INST(_Float16)

template <class R>
void launch_geom(const Dev &d, int which, int list_blocks, hipStream_t st)
{
    k_geom<R><<<list_blocks, LIST_THREADS, 0, st>>>(d, which);
}
template void launch_geom<double>(const Dev &, int, int, hipStream_t);
template void launch_geom<float>(const Dev &, int, int, hipStream_t);

// record slots and the highest fluid row.  Scratch: the per-cell kinds in
// the excess-share array and the per-block counts in the new-cell list
// (both free between steps; 2 * blocks <= N).  Only the cells c0 .. c1 - 1
// can hold records (c1 < 0: all): outside them every cell keeps slot -1.
void launch_setup_links(const Dev &d, int from_slots, int c0, int c1, hipStream_t st)
{
    const int b = (d.N + 255) / 256;
    const int bs = (d.N + SLOT_CELLS - 1) / SLOT_CELLS;
    const int b0 = c1 < 0 ? 0 : c0 / SLOT_CELLS, b1 = c1 < 0 ? bs : std::min((c1 + SLOT_CELLS - 1) / SLOT_CELLS, bs);
    uint8_t *kind = (uint8_t *)d.share;
    int32_t *bc = d.lnew, *bf = d.lnew + bs;
    if (b1 > b0) {
        k_slot_kinds<<<b1 - b0, SLOT_THREADS, 0, st>>>(d, kind, bc + b0, bf + b0, from_slots, b0);
        k_scan_counts<<<1, 1024, 0, st>>>(bc + b0, b1 - b0, d.cnt + 4);
        k_scan_counts<<<1, 1024, 0, st>>>(bf + b0, b1 - b0, d.cnt + 5);
        k_slot_write<<<b1 - b0, SLOT_THREADS, 0, st>>>(d, kind, bc + b0, bf + b0, b0);
    }
    k_zmax<<<b < 1024 ? b : 1024, 256, 0, st>>>(d);
}

void launch_kinds_list(const Dev &d, const int32_t *list, const int *count, int bound, hipStream_t st)
{
    if (bound > 0) k_kinds_list<<<(bound + 255) / 256, 256, 0, st>>>(d, list, count);
}

template <class R>
void launch_bb_terms(const Dev &d, int nrec, hipStream_t st)
{
    k_bb_terms<R><<<(nrec + 255) / 256, 256, 0, st>>>(d, nrec);
}
template void launch_bb_terms<double>(const Dev &, int, hipStream_t);
template void launch_bb_terms<float>(const Dev &, int, hipStream_t);

}  // namespace fsl
