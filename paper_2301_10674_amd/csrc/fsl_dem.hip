// fsl_dem.hip -- particle motion on the GPU: rigid spheres under the
// hydrodynamic load, gravity, collisions and lubrication, sub-stepped within
// one lattice step (Section 2.2: Newton-Euler equations per particle, a
// discrete element method parameterised by e_dry, T_c, nu_p and mu_p, and
// lubrication corrections for gaps the lattice does not resolve).
//
// Model (the readings of the cited coupling paper, which is not available):
// linear spring-dashpot normal force with k_n = m_eff (pi^2 + ln^2 e)/T_c^2
// and gamma_n = -2 m_eff ln(e)/T_c; tangential spring on the accumulated
// tangential displacement plus dashpot, k_t = kappa k_n and gamma_t =
// sqrt(kappa) gamma_n with Mindlin's kappa = 2(1-nu)/(2-nu), capped by
// Coulomb friction mu |F_n|; forces act at the middle of the overlap;
// Brenner's leading-order normal lubrication force -6 pi mu R_eff^2 u_n
// (1/s - 1/s_c) and the leading tangential one -6 pi mu R_t ln(s_c/s) v_t,
// R_t = 4 r1 r2 (2 r1^2 + r1 r2 + 2 r2^2) / (15 (r1 + r2)^3) (Jeffrey and
// Onishi; 8 r/15 against a wall, Goldman, Cox and Brenner), for gaps
// 0 < s < s_c (s >= s_min); walls z = 0 and z = nz as bodies of infinite
// radius and mass; symplectic Euler per sub-step.
//
// Layout: one wavefront per sphere for the lists, one lane per (sphere,
// list slot) for the forces.  Each call first rebuilds every sphere's
// partner list (spheres within r_i + r_j + s_c + skin, in index order, at
// most DEM_MAXN) and carries the tangential displacements of the pairs that
// stay over; then each sub-step reads the state of the previous one and
// writes the next (double buffer).  A pair's force is evaluated by both of
// its spheres in the same canonical order (lower index first), so the two
// copies of its tangential displacement stay identical and the forces are
// exactly opposite.  Floating-point contraction is off in the force code:
// every sum and product rounds as written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "fsl.h"

namespace fsl {
FslStatus set_error(FslStatus s, const std::string &msg);
}
using fsl::set_error;

namespace {

constexpr int DEM_MAXN = 32;       // partners per sphere
constexpr int DEM_THREADS = 256;
constexpr double PI = 3.14159265358979323846;

struct DemDev {
    int n;
    double Lx, Ly, Lz;
    double kn_num, kn_den;   // k_n = m_eff * kn_num / kn_den
    double lne, tc;          // gamma_n = -2 m_eff lne / tc
    double kappa, skappa;    // k_t / k_n and its square root
    double mu, visc, lub_cut, lub_min, h, skin;
    double ax, ay, az;
    const double *r, *m, *inertia;
    const uint8_t *fixed;
    double *x[2], *v[2], *w[2];   // 3 per sphere
    double *x0;                   // positions when the lists were built
    int32_t *nb[2], *cnt[2];      // partner lists (DEM_MAXN per sphere), counts
    double *xi[2];                // tangential displacement per list slot (3)
    double *wxi;                  // bottom and top wall displacement (6 per sphere)
    const double *hydro;          // 6 per sphere or null
    int32_t *err;                 // bit 0: list overflow, bit 1: moved beyond the skin
    // bins for the partner search (nbx = 0: every sphere tests every other):
    // nbx x nby x nbz boxes of at least the largest reach, periodic in x
    // and y; per bin its first entry and count in bin_idx (sphere indices)
    int nbx, nby, nbz;
    double wbx, wby, wbz;
    int32_t *bin_cnt, *bin_start, *bin_cur, *bin_idx;
};

__device__ __forceinline__ double min_image(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

// Rebuild the partner lists: one wavefront per sphere tests 64 candidates
// at a time and appends the hits in index order (ballot + prefix count);
// each hit lane carries over the tangential displacement its pair had in
// the sphere's old list.
__global__ __launch_bounds__(DEM_THREADS) void k_dem_list(DemDev D, int s, int cur)
{
    const int i = (int)((blockIdx.x * DEM_THREADS + threadIdx.x) >> 6);
    const int lane = (int)(threadIdx.x & 63);
    if (i >= D.n) return;   // the whole wavefront shares i
    const int nxt = cur ^ 1;
    const double xi0 = D.x[s][3 * i], xi1 = D.x[s][3 * i + 1], xi2 = D.x[s][3 * i + 2];
    const double ri = D.r[i];
    const double reach = D.lub_cut + D.skin;
    const int co = D.cnt[cur][i];
    int c = 0;
    for (int base = 0; base < D.n; base += 64) {
        const int j = base + lane;
        bool hit = false;
        if (j < D.n && j != i) {
            const double dx = min_image(D.x[s][3 * j] - xi0, D.Lx);
            const double dy = min_image(D.x[s][3 * j + 1] - xi1, D.Ly);
            const double dz = D.x[s][3 * j + 2] - xi2;
            const double lim = ri + D.r[j] + reach;
            hit = dx * dx + dy * dy + dz * dz < lim * lim;
        }
        const uint64_t m = __ballot(hit);
        if (hit) {
            const int pos = c + (int)__popcll(m & ((1ull << lane) - 1ull));
            if (pos < DEM_MAXN) {
                const size_t slot = (size_t)i * DEM_MAXN + pos;
                D.nb[nxt][slot] = j;
                double a = 0.0, b = 0.0, e = 0.0;
                for (int q = 0; q < co; ++q)
                    if (D.nb[cur][(size_t)i * DEM_MAXN + q] == j) {
                        const size_t o = 3 * ((size_t)i * DEM_MAXN + q);
                        a = D.xi[cur][o];
                        b = D.xi[cur][o + 1];
                        e = D.xi[cur][o + 2];
                        break;
                    }
                D.xi[nxt][3 * slot] = a;
                D.xi[nxt][3 * slot + 1] = b;
                D.xi[nxt][3 * slot + 2] = e;
            }
        }
        c += (int)__popcll(m);
    }
    if (lane == 0) {
        if (c > DEM_MAXN) atomicOr(D.err, 1);
        D.cnt[nxt][i] = min(c, DEM_MAXN);
        D.x0[3 * i] = xi0;
        D.x0[3 * i + 1] = xi1;
        D.x0[3 * i + 2] = xi2;
    }
}

// bin of sphere i (x and y wrapped into the box, z clamped to the bins)
__device__ __forceinline__ int dem_bin(const DemDev &D, int s, int i)
{
    const double x = D.x[s][3 * i], y = D.x[s][3 * i + 1], z = D.x[s][3 * i + 2];
    const int bx = min(max((int)floor((x - D.Lx * floor(x / D.Lx)) / D.wbx), 0), D.nbx - 1);
    const int by = min(max((int)floor((y - D.Ly * floor(y / D.Ly)) / D.wby), 0), D.nby - 1);
    const int bz = min(max((int)floor(z / D.wbz), 0), D.nbz - 1);
    return bx + D.nbx * (by + D.nby * bz);
}

__global__ void k_bin_zero(DemDev D)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < D.nbx * D.nby * D.nbz) D.bin_cnt[b] = 0;
}

__global__ void k_bin_count(DemDev D, int s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < D.n) atomicAdd(&D.bin_cnt[dem_bin(D, s, i)], 1);
}

// exclusive prefix of the bin counts (one block of 1024), also as cursors
__global__ __launch_bounds__(1024) void k_bin_scan(DemDev D)
{
    __shared__ int s_w[16];
    __shared__ int s_carry;
    const int nbins = D.nbx * D.nby * D.nbz;
    const int lane = __lane_id(), w = (int)threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < nbins; base += 1024) {
        const int b = base + (int)threadIdx.x;
        const int x = b < nbins ? D.bin_cnt[b] : 0;
        int sc = x;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(sc, o);
            if (lane >= o) sc += y;
        }
        if (lane == 63) s_w[w] = sc;
        __syncthreads();
        int off = s_carry;
        for (int k = 0; k < w; ++k) off += s_w[k];
        if (b < nbins) {
            D.bin_start[b] = off + sc - x;
            D.bin_cur[b] = off + sc - x;
        }
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = off + sc;
        __syncthreads();
    }
}

__global__ void k_bin_fill(DemDev D, int s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < D.n) D.bin_idx[atomicAdd(&D.bin_cur[dem_bin(D, s, i)], 1)] = i;
}

// The partner lists as k_dem_list builds them, candidates taken from the
// 27 bins around the sphere's (bins are at least as wide as any reach, at
// least three per periodic axis, so the 27 are distinct).  A bin's spheres
// come in no particular order: the hits are gathered in LDS and each takes
// the position of its rank by index, so the lists are identical.
constexpr int DEM_HITS = 64;   // hits kept per sphere (more than DEM_MAXN: overflow is reported)

__global__ __launch_bounds__(DEM_THREADS) void k_dem_list_bins(DemDev D, int s, int cur)
{
    __shared__ int s_hit[DEM_THREADS / 64][DEM_HITS];
    const int wv = (int)threadIdx.x >> 6;
    const int i = (int)((blockIdx.x * DEM_THREADS + threadIdx.x) >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const bool active = i < D.n;   // the whole wavefront shares i; every one reaches the barrier
    const int nxt = cur ^ 1;
    int c = 0, co = 0;
    double xi0 = 0.0, xi1 = 0.0, xi2 = 0.0;
    if (active) {
        xi0 = D.x[s][3 * i];
        xi1 = D.x[s][3 * i + 1];
        xi2 = D.x[s][3 * i + 2];
        const double ri = D.r[i];
        const double reach = D.lub_cut + D.skin;
        co = D.cnt[cur][i];
        const int b = dem_bin(D, s, i);
        const int bx = b % D.nbx, by = (b / D.nbx) % D.nby, bz = b / (D.nbx * D.nby);
        for (int k = 0; k < 27; ++k) {
            const int zz = bz + k / 9 - 1;
            if (zz < 0 || zz >= D.nbz) continue;
            const int xx = (bx + k % 3 - 1 + D.nbx) % D.nbx, yy = (by + (k / 3) % 3 - 1 + D.nby) % D.nby;
            const int bb = xx + D.nbx * (yy + D.nby * zz);
            const int b0 = D.bin_start[bb], nbn = D.bin_cnt[bb];
            for (int base = 0; base < nbn; base += 64) {
                int j = -1;
                bool hit = false;
                if (base + lane < nbn) {
                    j = D.bin_idx[b0 + base + lane];
                    if (j != i) {
                        const double dx = min_image(D.x[s][3 * j] - xi0, D.Lx);
                        const double dy = min_image(D.x[s][3 * j + 1] - xi1, D.Ly);
                        const double dz = D.x[s][3 * j + 2] - xi2;
                        const double lim = ri + D.r[j] + reach;
                        hit = dx * dx + dy * dy + dz * dz < lim * lim;
                    }
                }
                const uint64_t m = __ballot(hit);
                if (hit) {
                    const int pos = c + (int)__popcll(m & ((1ull << lane) - 1ull));
                    if (pos < DEM_HITS) s_hit[wv][pos] = j;
                }
                c += (int)__popcll(m);
            }
        }
    }
    __syncthreads();   // the hits are in LDS
    if (!active) return;
    const int nh = min(c, DEM_HITS);
    if (lane < nh) {
        const int j = s_hit[wv][lane];
        int pos = 0;
        for (int q = 0; q < nh; ++q) pos += s_hit[wv][q] < j;
        if (pos < DEM_MAXN) {
            const size_t slot = (size_t)i * DEM_MAXN + pos;
            D.nb[nxt][slot] = j;
            double a = 0.0, bq = 0.0, e = 0.0;
            for (int q = 0; q < co; ++q)
                if (D.nb[cur][(size_t)i * DEM_MAXN + q] == j) {
                    const size_t o = 3 * ((size_t)i * DEM_MAXN + q);
                    a = D.xi[cur][o];
                    bq = D.xi[cur][o + 1];
                    e = D.xi[cur][o + 2];
                    break;
                }
            D.xi[nxt][3 * slot] = a;
            D.xi[nxt][3 * slot + 1] = bq;
            D.xi[nxt][3 * slot + 2] = e;
        }
    }
    if (lane == 0) {
        if (c > DEM_MAXN) atomicOr(D.err, 1);
        D.cnt[nxt][i] = min(c, DEM_MAXN);
        D.x0[3 * i] = xi0;
        D.x0[3 * i + 1] = xi1;
        D.x0[3 * i + 2] = xi2;
    }
}

#pragma clang fp contract(off)

__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Force F on body a (tangential part Ft) from body b: contact (delta > 0,
// xi updated) or lubrication (gap -delta below the cut-off).
__device__ void pair_force(const DemDev &D, const double n[3], double delta, const double vrel[3],
                           double ucen, double meff, double reff, double rt, double *xi, double F[3],
                           double Ft[3])
{
    F[0] = F[1] = F[2] = 0.0;
    Ft[0] = Ft[1] = Ft[2] = 0.0;
    if (delta > 0.0) {
        const double kn = meff * D.kn_num / D.kn_den;
        const double gn = -2.0 * meff * D.lne / D.tc;
        const double kt = D.kappa * kn, gt = D.skappa * gn;
        const double un = dot3(vrel, n);
        const double fn = kn * delta + gn * un;
        double vt[3];
        for (int d = 0; d < 3; ++d) vt[d] = vrel[d] - un * n[d];
        const double xn = dot3(xi, n);
        for (int d = 0; d < 3; ++d) xi[d] -= xn * n[d];
        for (int d = 0; d < 3; ++d) Ft[d] = -kt * xi[d] - gt * vt[d];
        const double ft = sqrt(dot3(Ft, Ft)), lim = D.mu * fabs(fn);
        if (ft > lim) {
            for (int d = 0; d < 3; ++d) {
                Ft[d] = lim * Ft[d] / ft;
                xi[d] = -(Ft[d] + gt * vt[d]) / kt;
            }
        }
        for (int d = 0; d < 3; ++d) xi[d] += D.h * vt[d];
        for (int d = 0; d < 3; ++d) F[d] = -fn * n[d] + Ft[d];
    } else if (D.lub_cut > 0.0 && -delta < D.lub_cut) {
        double s = -delta;
        if (s < D.lub_min) s = D.lub_min;
        const double f = -6.0 * PI * D.visc * reff * reff * ucen * (1.0 / s - 1.0 / D.lub_cut);
        const double un = dot3(vrel, n);
        const double g = -6.0 * PI * D.visc * rt * log(D.lub_cut / s);
        for (int d = 0; d < 3; ++d) {
            Ft[d] = g * (vrel[d] - un * n[d]);
            F[d] = f * n[d] + Ft[d];
        }
    }
}

// One sub-step: state s -> s ^ 1 with the lists of parity l.  A sphere
// owns DEM_MAXN consecutive lanes, one per list slot: each lane evaluates
// its pair (and updates that slot's tangential displacement); the sphere's
// first lane then adds the pair forces in list (= partner index) order to
// the external load, adds the walls and integrates.
constexpr int DEM_PER_BLOCK = DEM_THREADS / DEM_MAXN;

__global__ __launch_bounds__(DEM_THREADS) void k_dem_sub(DemDev D, int s, int l)
{
    __shared__ double sf[DEM_PER_BLOCK][DEM_MAXN][6];
    __shared__ uint8_t act[DEM_PER_BLOCK][DEM_MAXN];
    const int q = (int)threadIdx.x / DEM_MAXN, k = (int)threadIdx.x % DEM_MAXN;
    const int i = blockIdx.x * DEM_PER_BLOCK + q;
    const bool live = i < D.n;
    const double *X = D.x[s], *V = D.v[s], *Wv = D.w[s];
    const int cn = live ? D.cnt[l][i] : 0;
    bool used = false;
    if (k < cn) {
        const int j = D.nb[l][i * DEM_MAXN + k];
        double *xi = &D.xi[l][3 * (i * DEM_MAXN + k)];
        const int a = i < j ? i : j, b = i < j ? j : i;
        double dv[3];
        dv[0] = min_image(X[3 * b] - X[3 * a], D.Lx);
        dv[1] = min_image(X[3 * b + 1] - X[3 * a + 1], D.Ly);
        dv[2] = X[3 * b + 2] - X[3 * a + 2];
        const double dist = sqrt(dot3(dv, dv));
        const double ra = D.r[a], rb = D.r[b];
        const double delta = ra + rb - dist;
        if (delta <= -D.lub_cut || dist == 0.0) {
            xi[0] = xi[1] = xi[2] = 0.0;
        } else if (!(D.fixed[a] && D.fixed[b])) {
            const double nv[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
            double meff;
            if (D.fixed[a]) meff = D.m[b];
            else if (D.fixed[b]) meff = D.m[a];
            else meff = D.m[a] * D.m[b] / (D.m[a] + D.m[b]);
            const double reff = ra * rb / (ra + rb);
            const double rt = 4.0 * ra * rb * (2.0 * ra * ra + ra * rb + 2.0 * rb * rb) /
                              (15.0 * (ra + rb) * (ra + rb) * (ra + rb));
            const double la = ra - 0.5 * delta, lb = rb - 0.5 * delta;
            const double arm_a[3] = {la * nv[0], la * nv[1], la * nv[2]};
            const double arm_b[3] = {-lb * nv[0], -lb * nv[1], -lb * nv[2]};
            double wa[3], wb[3];
            cross3(&Wv[3 * a], arm_a, wa);
            cross3(&Wv[3 * b], arm_b, wb);
            double vrel[3], vc[3];
            for (int d = 0; d < 3; ++d) {
                vc[d] = V[3 * a + d] - V[3 * b + d];
                vrel[d] = (V[3 * a + d] + wa[d]) - (V[3 * b + d] + wb[d]);
            }
            const double ucen = dot3(vc, nv);
            if (delta <= 0.0) xi[0] = xi[1] = xi[2] = 0.0;
            double f[3], ft[3], t[3];
            pair_force(D, nv, delta, vrel, ucen, meff, reff, rt, delta > 0.0 ? xi : nullptr, f, ft);
            if (i == a) {
                cross3(arm_a, ft, t);
            } else {
                // b takes the opposite force (adding -f rounds as subtracting f)
                const double ftb[3] = {-ft[0], -ft[1], -ft[2]};
                cross3(arm_b, ftb, t);
                for (int d = 0; d < 3; ++d) f[d] = -f[d];
            }
            for (int d = 0; d < 3; ++d) {
                sf[q][k][d] = f[d];
                sf[q][k][3 + d] = t[d];
            }
            used = true;
        }
    }
    act[q][k] = used ? 1 : 0;
    __syncthreads();
    if (!live || k != 0) return;

    double F[3], T[3];
    const double mi = D.m[i];
    const double acc[3] = {D.ax, D.ay, D.az};
    for (int d = 0; d < 3; ++d) {
        F[d] = (D.hydro ? D.hydro[6 * i + d] : 0.0) + mi * acc[d];
        T[d] = D.hydro ? D.hydro[6 * i + 3 + d] : 0.0;
    }
    for (int kk = 0; kk < cn; ++kk) {
        if (!act[q][kk]) continue;
        for (int d = 0; d < 3; ++d) {
            F[d] += sf[q][kk][d];
            T[d] += sf[q][kk][3 + d];
        }
    }
    const bool fx = D.fixed[i] != 0;
    if (!fx) {
        for (int kw = 0; kw < 2; ++kw) {
            const double gap = kw == 0 ? X[3 * i + 2] : D.Lz - X[3 * i + 2];
            const double delta = D.r[i] - gap;
            double *xi = &D.wxi[6 * i + 3 * kw];
            if (delta <= -D.lub_cut) {
                xi[0] = xi[1] = xi[2] = 0.0;
                continue;
            }
            const double nv[3] = {0.0, 0.0, kw == 0 ? -1.0 : 1.0};
            const double la = D.r[i] - 0.5 * delta;
            const double arm[3] = {la * nv[0], la * nv[1], la * nv[2]};
            double wa[3];
            cross3(&Wv[3 * i], arm, wa);
            double vrel[3];
            for (int d = 0; d < 3; ++d) vrel[d] = V[3 * i + d] + wa[d];
            const double ucen = V[3 * i + 2] * nv[2];
            if (delta <= 0.0) xi[0] = xi[1] = xi[2] = 0.0;
            double f[3], ft[3], t[3];
            pair_force(D, nv, delta, vrel, ucen, mi, D.r[i], 8.0 * D.r[i] / 15.0, delta > 0.0 ? xi : nullptr, f,
                       ft);
            cross3(arm, ft, t);
            for (int d = 0; d < 3; ++d) {
                F[d] += f[d];
                T[d] += t[d];
            }
        }
    }
    double *Xo = D.x[s ^ 1], *Vo = D.v[s ^ 1], *Wo = D.w[s ^ 1];
    for (int d = 0; d < 3; ++d) {
        double v = V[3 * i + d], w = Wv[3 * i + d], x = X[3 * i + d];
        if (!fx) {
            v += D.h * F[d] / mi;
            w += D.h * T[d] / D.inertia[i];
            x += D.h * v;
        }
        Vo[3 * i + d] = v;
        Wo[3 * i + d] = w;
        Xo[3 * i + d] = x;
    }
    if (!fx) {
        Xo[3 * i] -= D.Lx * floor(Xo[3 * i] / D.Lx);
        Xo[3 * i + 1] -= D.Ly * floor(Xo[3 * i + 1] / D.Ly);
    }
}

#pragma clang fp contract(on)

// every sphere must stay within half the skin of where its list was built
__global__ __launch_bounds__(DEM_THREADS) void k_dem_check(DemDev D, int s)
{
    const int i = blockIdx.x * DEM_THREADS + threadIdx.x;
    if (i >= D.n) return;
    const double dx = min_image(D.x[s][3 * i] - D.x0[3 * i], D.Lx);
    const double dy = min_image(D.x[s][3 * i + 1] - D.x0[3 * i + 1], D.Ly);
    const double dz = D.x[s][3 * i + 2] - D.x0[3 * i + 2];
    if (!(dx * dx + dy * dy + dz * dz <= 0.25 * D.skin * D.skin)) atomicOr(D.err, 2);
}

// Bedload transport rate of Eq. (1), sum_i u_x,i V_i / (Lx Ly): one block;
// each thread sums a strided share in index order, then a fixed tree.
__global__ __launch_bounds__(DEM_THREADS) void k_dem_bedload(DemDev D, int s, double *out)
{
    __shared__ double part[DEM_THREADS];
    double q = 0.0;
    for (int i = (int)threadIdx.x; i < D.n; i += DEM_THREADS) {
        const double r = D.r[i];
        q += D.v[s][3 * i] * ((4.0 / 3.0) * PI * r * r * r);
    }
    part[threadIdx.x] = q;
    __syncthreads();
    for (int w = DEM_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / (D.Lx * D.Ly);
}

}  // namespace

struct FslDem {
    FslDemParams P;
    DemDev d;
    hipStream_t st = nullptr;
    void *mem = nullptr;
    int s = 0;          // state parity
    int l = 0;          // list parity
    double *hbuf = nullptr;   // device copy of a host hydrodynamic load
    void *bins = nullptr;     // bin counts, starts, cursors and sphere indices
};

#define DEM_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_error(FSL_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static int dem_blocks(int n) { return (n + DEM_THREADS - 1) / DEM_THREADS; }

extern "C" {

FslStatus fsl_dem_create(const FslDemParams *p, void *hip_stream, int32_t n, const double *centre,
                         const double *radius, const double *vel, const double *angvel,
                         const uint8_t *fixed, FslDem **out)
{
    if (!out) return set_error(FSL_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return set_error(FSL_ERR_ARG, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return set_error(FSL_ERR_ARG, "box extents must be >= 1");
    if (!(p->density > 0.0) || !(p->restitution > 0.0 && p->restitution <= 1.0) ||
        !(p->collision_time > 0.0) || !(p->poisson >= 0.0 && p->poisson < 0.5) || !(p->friction >= 0.0) ||
        !(p->viscosity >= 0.0) || !(p->lub_cut >= 0.0) || !(p->lub_min > 0.0) || !(p->dt > 0.0) ||
        p->substeps < 1 || !(p->skin > 0.0) || !std::isfinite(p->accel[0]) || !std::isfinite(p->accel[1]) ||
        !std::isfinite(p->accel[2]))
        return set_error(FSL_ERR_ARG, "invalid particle parameters");
    if (n < 1 || !centre || !radius) return set_error(FSL_ERR_ARG, "need n >= 1, centre and radius");
    for (int32_t i = 0; i < n; ++i) {
        if (!(radius[i] > 0.0) || !std::isfinite(radius[i])) return set_error(FSL_ERR_ARG, "radius must be > 0");
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(centre[3 * i + d]) || (vel && !std::isfinite(vel[3 * i + d])) ||
                (angvel && !std::isfinite(angvel[3 * i + d])))
                return set_error(FSL_ERR_ARG, "non-finite particle state");
        }
    }
    FslDem *D = new FslDem();
    D->P = *p;
    D->st = (hipStream_t)hip_stream;
    DemDev &d = D->d;
    d.n = n;
    d.Lx = p->nx;
    d.Ly = p->ny;
    d.Lz = p->nz;
    // the constants are formed exactly as the oracle forms them
    const double lne = std::log(p->restitution);
    d.kn_num = PI * PI + lne * lne;
    d.kn_den = p->collision_time * p->collision_time;
    d.lne = lne;
    d.tc = p->collision_time;
    d.kappa = 2.0 * (1.0 - p->poisson) / (2.0 - p->poisson);
    d.skappa = std::sqrt(d.kappa);
    d.mu = p->friction;
    d.visc = p->viscosity;
    d.lub_cut = p->lub_cut;
    d.lub_min = p->lub_min;
    d.h = p->dt / p->substeps;
    d.skin = p->skin;
    d.ax = p->accel[0];
    d.ay = p->accel[1];
    d.az = p->accel[2];
    d.hydro = nullptr;

    // one allocation.  Doubles per sphere: r, m, I (3), x/v/w double
    // buffers (18), list-build positions (3), displacement per list slot x2
    // (6 DEM_MAXN), wall displacements (6), staged hydrodynamic load (6);
    // int32 per sphere: lists x2 (2 DEM_MAXN) and counts x2 (2), plus the
    // error word; u8 per sphere: fixed flags
    const size_t N = (size_t)n;
    const size_t nd = N * (36 + 6 * DEM_MAXN);
    const size_t ni = N * (2 * DEM_MAXN + 2) + 1;
    const size_t bytes = nd * 8 + ni * 4 + N + 64;
    hipError_t e = hipMalloc(&D->mem, bytes);
    if (e != hipSuccess) {
        delete D;
        return set_error(FSL_ERR_NOMEM, "particle state");
    }
    double *dev = (double *)D->mem;
    d.r = dev;
    d.m = dev + N;
    d.inertia = dev + 2 * N;
    d.x[0] = dev + 3 * N;
    d.x[1] = dev + 6 * N;
    d.v[0] = dev + 9 * N;
    d.v[1] = dev + 12 * N;
    d.w[0] = dev + 15 * N;
    d.w[1] = dev + 18 * N;
    d.x0 = dev + 21 * N;
    d.xi[0] = dev + 24 * N;
    d.xi[1] = dev + (24 + 3 * DEM_MAXN) * N;
    d.wxi = dev + (24 + 6 * DEM_MAXN) * N;
    D->hbuf = dev + (30 + 6 * DEM_MAXN) * N;
    int32_t *ip = (int32_t *)(dev + nd);
    d.nb[0] = ip;
    d.nb[1] = ip + N * DEM_MAXN;
    d.cnt[0] = ip + 2 * N * DEM_MAXN;
    d.cnt[1] = ip + 2 * N * DEM_MAXN + N;
    d.err = ip + 2 * N * DEM_MAXN + 2 * N;
    d.fixed = (const uint8_t *)(ip + ni);
    // the masses are formed exactly as the oracle forms them
    std::vector<double> stage(nd, 0.0);
    for (size_t i = 0; i < N; ++i) {
        const double ri = radius[i];
        stage[i] = ri;
        stage[N + i] = p->density * (4.0 / 3.0) * PI * ri * ri * ri;
        stage[2 * N + i] = 0.4 * stage[N + i] * ri * ri;
        for (int k = 0; k < 3; ++k) {
            stage[3 * N + 3 * i + k] = centre[3 * i + k];
            stage[9 * N + 3 * i + k] = vel ? vel[3 * i + k] : 0.0;
            stage[15 * N + 3 * i + k] = angvel ? angvel[3 * i + k] : 0.0;
        }
    }
    std::vector<uint8_t> fx(N, 0);
    if (fixed)
        for (size_t i = 0; i < N; ++i) fx[i] = fixed[i] ? 1 : 0;
    const std::vector<int32_t> zi(ni, 0);
    e = hipMemcpyAsync(D->mem, stage.data(), nd * 8, hipMemcpyHostToDevice, D->st);
    if (e == hipSuccess) e = hipMemcpyAsync(ip, zi.data(), ni * 4, hipMemcpyHostToDevice, D->st);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)d.fixed, fx.data(), N, hipMemcpyHostToDevice, D->st);
    if (e == hipSuccess) e = hipStreamSynchronize(D->st);
    if (e != hipSuccess) {
        (void)hipFree(D->mem);
        delete D;
        return set_error(FSL_ERR_DEVICE, std::string("particle state upload: ") + hipGetErrorString(e));
    }
    // bins for the partner search on large sets: at least as wide as the
    // largest reach 2 r_max + lub_cut + skin, at least three per periodic
    // axis, and not many more bins than spheres (below a few thousand
    // spheres testing every pair is as fast as the five binning launches)
    d.nbx = 0;
    double rmax = 0.0;
    for (size_t i = 0; i < N; ++i) rmax = std::max(rmax, radius[i]);
    double hb = 2.0 * rmax + p->lub_cut + p->skin;
    if (n >= 4096) {
        for (;;) {
            const int bx = (int)std::floor(d.Lx / hb), by = (int)std::floor(d.Ly / hb);
            const int bz = std::max(1, (int)std::floor(d.Lz / hb));
            if (bx < 3 || by < 3) break;
            if ((double)bx * by * bz <= 4.0 * n + 64.0) {
                d.nbx = bx;
                d.nby = by;
                d.nbz = bz;
                break;
            }
            hb *= 1.25;
        }
    }
    if (d.nbx > 0) {
        d.wbx = d.Lx / d.nbx;
        d.wby = d.Ly / d.nby;
        d.wbz = d.Lz / d.nbz;
        const size_t nbins = (size_t)d.nbx * d.nby * d.nbz;
        if (hipMalloc(&D->bins, (3 * nbins + N) * 4) != hipSuccess) {
            (void)hipFree(D->mem);
            delete D;
            return set_error(FSL_ERR_NOMEM, "particle bins");
        }
        d.bin_cnt = (int32_t *)D->bins;
        d.bin_start = d.bin_cnt + nbins;
        d.bin_cur = d.bin_start + nbins;
        d.bin_idx = d.bin_cur + nbins;
    }
    *out = D;
    return FSL_OK;
}

FslStatus fsl_dem_step(FslDem *D, const double *hydro, int32_t hydro_on_device, int32_t nsteps)
{
    if (!D) return set_error(FSL_ERR_STATE, "particle state is NULL");
    if (nsteps < 0) return set_error(FSL_ERR_ARG, "nsteps < 0");
    const int n = D->d.n;
    if (hydro && !hydro_on_device)
        DEM_TRY(hipMemcpyAsync(D->hbuf, hydro, (size_t)n * 6 * sizeof(double), hipMemcpyHostToDevice, D->st));
    DemDev d = D->d;
    d.hydro = hydro ? (hydro_on_device ? hydro : D->hbuf) : nullptr;
    const int nb = dem_blocks(n);
    const int lb = (n + DEM_THREADS / 64 - 1) / (DEM_THREADS / 64);
    for (int t = 0; t < nsteps; ++t) {
        if (d.nbx > 0) {
            const int nbins = d.nbx * d.nby * d.nbz;
            k_bin_zero<<<(nbins + 255) / 256, 256, 0, D->st>>>(d);
            k_bin_count<<<nb, DEM_THREADS, 0, D->st>>>(d, D->s);
            k_bin_scan<<<1, 1024, 0, D->st>>>(d);
            k_bin_fill<<<nb, DEM_THREADS, 0, D->st>>>(d, D->s);
            k_dem_list_bins<<<lb, DEM_THREADS, 0, D->st>>>(d, D->s, D->l);
        } else {
            k_dem_list<<<lb, DEM_THREADS, 0, D->st>>>(d, D->s, D->l);
        }
        D->l ^= 1;
        for (int k = 0; k < D->P.substeps; ++k) {
            k_dem_sub<<<(n + DEM_PER_BLOCK - 1) / DEM_PER_BLOCK, DEM_THREADS, 0, D->st>>>(d, D->s, D->l);
            D->s ^= 1;
        }
        k_dem_check<<<nb, DEM_THREADS, 0, D->st>>>(d, D->s);
    }
    int32_t err = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&err, d.err, 4, hipMemcpyDeviceToHost, D->st);
    if (e == hipSuccess) e = hipStreamSynchronize(D->st);
    if (e != hipSuccess) return set_error(FSL_ERR_DEVICE, std::string("particle step: ") + hipGetErrorString(e));
    if (err & 1) return set_error(FSL_ERR_NOMEM, "a sphere has more than 32 partners within reach");
    if (err & 2) return set_error(FSL_ERR_UNSTABLE, "a sphere moved more than half the skin in one step");
    return FSL_OK;
}

FslStatus fsl_dem_read(FslDem *D, double *centre, double *vel, double *angvel, int32_t out_on_device)
{
    if (!D) return set_error(FSL_ERR_STATE, "particle state is NULL");
    const size_t b = (size_t)D->d.n * 3 * sizeof(double);
    const hipMemcpyKind k = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (centre) DEM_TRY(hipMemcpyAsync(centre, D->d.x[D->s], b, k, D->st));
    if (vel) DEM_TRY(hipMemcpyAsync(vel, D->d.v[D->s], b, k, D->st));
    if (angvel) DEM_TRY(hipMemcpyAsync(angvel, D->d.w[D->s], b, k, D->st));
    DEM_TRY(hipStreamSynchronize(D->st));
    return FSL_OK;
}

FslStatus fsl_dem_bedload(FslDem *D, double *qb)
{
    if (!D) return set_error(FSL_ERR_STATE, "particle state is NULL");
    if (!qb) return set_error(FSL_ERR_ARG, "qb is NULL");
    // the staging area of host hydrodynamic loads holds the result
    k_dem_bedload<<<1, DEM_THREADS, 0, D->st>>>(D->d, D->s, D->hbuf);
    DEM_TRY(hipGetLastError());
    DEM_TRY(hipMemcpyAsync(qb, D->hbuf, sizeof(double), hipMemcpyDeviceToHost, D->st));
    DEM_TRY(hipStreamSynchronize(D->st));
    return FSL_OK;
}

void fsl_dem_destroy(FslDem *D)
{
    if (!D) return;
    if (D->mem) {
        (void)hipStreamSynchronize(D->st);
        (void)hipFree(D->mem);
    }
    if (D->bins) (void)hipFree(D->bins);
    delete D;
}

}  // extern "C"
