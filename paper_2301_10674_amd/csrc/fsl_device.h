// fsl_device.h -- device-side building blocks of the free-surface LBM step
// on gfx950: D3Q27 constants, PDF storage formats, the cumulant collision
// written on deviations from the rest weights, the product equilibrium, and
// small wavefront helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fsl {

// ---------------------------------------------------------------- lattice
// Direction i = (cx+1) + 3(cy+1) + 9(cz+1); rest = 13; opposite = 26 - i.
__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int opp(int i) { return 26 - i; }
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wgt(int i) { return w1(cx(i)) * w1(cy(i)) * w1(cz(i)); }
__host__ __device__ constexpr int MI(int a, int b, int c) { return a + 3 * b + 9 * c; }
constexpr int REST = 13;

// cell types (low two bits of the flag byte) and static flag bits
enum : uint8_t { T_GAS = 0, T_LIQ = 1, T_IF = 2, T_SOLID = 3, T_MASK = 3, F_NEAR_SOLID = 4,
                 // flux-modifier class of an interface cell (set only when that
                 // variant is on): gas but no liquid neighbours / liquid but no gas
                 F_CLS_LOSE = 32, F_CLS_GAIN = 64 };
// conversion marks (low byte of the epoch-stamped mark word)
enum : uint32_t { MK_TO_LIQ = 1, MK_TO_GAS = 2, MK_EMPTY = 4, MK_NEW = 8, MK_ISO = 16,
                  MK_WEIGHTED = 32 /* excess shared by normal weights */ };

__device__ __forceinline__ uint32_t mark_bits(uint32_t mk, uint32_t epoch)
{
    return (mk >> 8) == epoch ? (mk & 0xffu) : 0u;
}

// ---------------------------------------------------------------- storage
// PDFs are stored as deviations d_i = f_i - w_i in S; the collision runs in
// Real<S>::type.
template <class S> struct Real { using type = float; };
template <> struct Real<double> { using type = double; };
// type of the equilibrium part and of the final sum of the collision: the
// equilibrium shift D (nested products of O(u) terms, size ~1e-3) decides the
// FP32 form's accuracy, so it is formed in FP64 there; with FP16 storage the
// rounding of the stored values dominates and FP32 suffices
template <class S> struct Eq { using type = double; };
template <> struct Eq<_Float16> { using type = float; };

template <class S> __device__ __forceinline__ typename Real<S>::type ld(const S *p)
{
    return (typename Real<S>::type)(*p);
}
__device__ __forceinline__ float ld(const _Float16 *p) { return (float)(*p); }

template <class S, class R> __device__ __forceinline__ S to_store(R v) { return (S)v; }

// ---------------------------------------------------------------- equilibrium
// Deviation of the product-form equilibrium from the rest weights,
// D_i(u) = prod_d psi(c_d, u_d) - w_i with psi(0,u) = 2/3 - u^2 and
// psi(+-1,u) = (1/3 + u^2 +- u)/2, written as nested differences so that no
// O(1) quantity is subtracted.
template <class R>
__device__ __forceinline__ void product_dev(R ux, R uy, R uz, R D[27])
{
    const R u[3] = {ux, uy, uz};
    R e[3][3], w[3];
    w[0] = R(1.0 / 6.0);
    w[1] = R(2.0 / 3.0);
    w[2] = R(1.0 / 6.0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R uu = u[d] * u[d];
        e[d][0] = R(0.5) * (uu - u[d]);
        e[d][1] = -uu;
        e[d][2] = R(0.5) * (uu + u[d]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                R d2 = e[0][a] * (w[b] + e[1][b]) + w[a] * e[1][b];
                D[MI(a, b, c)] = d2 * (w[c] + e[2][c]) + (w[a] * w[b]) * e[2][c];
            }
}

// One entry of feq_dev below, from the 1D factors of product_dev:
// e[d][k] = psi(k-1, u_d) - w1(k-1).  Same arithmetic as the full table.
template <class R>
__device__ __forceinline__ void psi_dev(R ux, R uy, R uz, R e[3][3])
{
    const R u[3] = {ux, uy, uz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R uu = u[d] * u[d];
        e[d][0] = R(0.5) * (uu - u[d]);
        e[d][1] = -uu;
        e[d][2] = R(0.5) * (uu + u[d]);
    }
}
template <class R>
__device__ __forceinline__ R feq_dev_one(R drho, const R e[3][3], int i)
{
    const R w[3] = {R(1.0 / 6.0), R(2.0 / 3.0), R(1.0 / 6.0)};
    const int a = i % 3, b = (i / 3) % 3, c = i / 9;
    R d2 = e[0][a] * (w[b] + e[1][b]) + w[a] * e[1][b];
    R D = d2 * (w[c] + e[2][c]) + (w[a] * w[b]) * e[2][c];
    return drho * (R(wgt(i)) + D) + D;
}

// f^eq(rho, u) - w  with rho = 1 + drho
template <class R>
__device__ __forceinline__ void feq_dev(R drho, R ux, R uy, R uz, R out[27])
{
    R D[27];
    product_dev(ux, uy, uz, D);
#pragma unroll
    for (int i = 0; i < 27; ++i) out[i] = drho * (R(wgt(i)) + D[i]) + D[i];
}

// ---------------------------------------------------------------- collision
// One 1D inverse chimera step: central moments (k0,k1,k2) about u ->
// values at velocities -1, 0, +1:
//   f0 = (1 - u^2) k0 - 2u k1 - k2,
//   f-/+ = ((u^2 -/+ u) k0 + (2u -/+ 1) k1 + k2) / 2.
// The coefficients depend on u only and are formed once per pass.
template <class R>
struct Chimera {
    R a0, a1, m0, m1, p0, p1;
    __device__ __forceinline__ explicit Chimera(R u)
    {
        const R uu = u * u;
        a0 = R(1) - uu;
        a1 = R(-2) * u;
        m0 = R(0.5) * (uu - u);
        m1 = u - R(0.5);
        p0 = R(0.5) * (uu + u);
        p1 = u + R(0.5);
    }
    __device__ __forceinline__ void apply(R &a, R &b, R &c) const
    {
        const R k0 = a, k1 = b, k2 = c, h = R(0.5) * k2;
        a = m0 * k0 + (m1 * k1 + h);
        b = a0 * k0 + (a1 * k1 - k2);
        c = p0 * k0 + (p1 * k1 + h);
    }
};

// Cumulant collision (Geier et al. 2015, as chosen in Section 2.1: shear
// rate omega, bulk and all higher-order rates 1) on PDF deviations
// d_i = f_i - w_i, in place.  g is the body acceleration: the velocity is
// shifted by F/(2 rho) and the first-order central moments leave the
// collision as +F/(2 rho) = g/2.  GC adds the Galilean-invariance
// correction of the same paper (a variant): the lattice lacks the cubic
// velocity moments, which puts 3 u_a^2 d_a u_a into the normal stresses;
// the relaxed diagonal second-order cumulants lose 3 (1 - w/2) u_a^2 d_a u_a
// (w = omega for the deviator, 1 for the trace), with the strain rates
// d_a u_a read from the cell's non-equilibrium second-order cumulants.
//
// With every higher-order rate equal to 1 the post-collision cumulants of
// order >= 3 vanish, so the post-collision central moments are the Gaussian
// (Isserlis) moments of the relaxed second-order cumulant tensor K*; only
// rho, the momentum and the second moments of the input matter.  Everything
// is carried as a deviation from the rest state (rho = 1, u = 0, K = I/3) so
// FP32 keeps the small quantities exact enough.
template <class R, class E, bool GC = false>
__device__ __forceinline__ void collide(const R d[27], R omega, R gx, R gy, R gz, E out[27], double &rho_out)
{
    // Raw moments of the deviations, passes x, y, z of (sum, odd, even), in
    // M = FP64 with FP64 and FP32 storage: the non-equilibrium second
    // moments are small differences of O(1e-3) sums, which FP32 would
    // resolve only to a few times the FP32 storage rounding (FP64 adds issue
    // at the unpacked FP32 rate).  With FP16 storage its own rounding is far
    // coarser and the moments are taken in FP32.
    using M = E;
    M m[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) m[i] = (M)d[i];
    auto pass = [&](int i0, int i1, int i2) {
        const M vm = m[i0], v0 = m[i1], vp = m[i2], s = vp + vm;
        m[i0] = s + v0;
        m[i1] = vp - vm;
        m[i2] = s;
    };
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) pass(MI(0, b, c), MI(1, b, c), MI(2, b, c));
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) pass(MI(a, 0, c), MI(a, 1, c), MI(a, 2, c));
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) pass(MI(a, b, 0), MI(a, b, 1), MI(a, b, 2));
    const M drho_d = m[MI(0, 0, 0)];
    const M rho_d = M(1) + drho_d;
    rho_out = (double)rho_d;
    const M irho_d = M(1) / rho_d;
    const M jxd = m[MI(1, 0, 0)], jyd = m[MI(0, 1, 0)], jzd = m[MI(0, 0, 1)];
    const M uxd = (jxd + M(0.5) * rho_d * (M)gx) * irho_d;
    const M uyd = (jyd + M(0.5) * rho_d * (M)gy) * irho_d;
    const M uzd = (jzd + M(0.5) * rho_d * (M)gz) * irho_d;
    const M dtr = drho_d * irho_d * M(1.0 / 3.0);
    // second-order central moments minus I/3
    const R Kxx = R((m[MI(2, 0, 0)] - M(2) * uxd * jxd) * irho_d + uxd * uxd - dtr);
    const R Kyy = R((m[MI(0, 2, 0)] - M(2) * uyd * jyd) * irho_d + uyd * uyd - dtr);
    const R Kzz = R((m[MI(0, 0, 2)] - M(2) * uzd * jzd) * irho_d + uzd * uzd - dtr);
    const R Kxy = R((m[MI(1, 1, 0)] - uxd * jyd - uyd * jxd) * irho_d + uxd * uyd);
    const R Kxz = R((m[MI(1, 0, 1)] - uxd * jzd - uzd * jxd) * irho_d + uxd * uzd);
    const R Kyz = R((m[MI(0, 1, 1)] - uyd * jzd - uzd * jyd) * irho_d + uyd * uzd);
    const R ux = R(uxd), uy = R(uyd), uz = R(uzd);
    const R third = R(1.0 / 3.0);
    // relaxation: deviator with omega, trace to equilibrium
    const R om1 = R(1) - omega;
    const R tr3 = (Kxx + Kyy + Kzz) * third;
    R ax = om1 * (Kxx - tr3), ay = om1 * (Kyy - tr3), az = om1 * (Kzz - tr3);
    if constexpr (GC) {
        // first-order non-equilibrium K = -(2/(3 w)) x strain rate, solved
        // for the normal strain rates from the deviator (w = omega) and the
        // trace (w = 1); the correction enters as a source with (1 - w/2)
        const R hw = R(0.5) * omega, trn = Kxx + Kyy + Kzz;
        const R ex = ux * ux * (-hw * (R(2) * Kxx - Kyy - Kzz) - R(0.5) * trn);
        const R ey = uy * uy * (-hw * (R(2) * Kyy - Kxx - Kzz) - R(0.5) * trn);
        const R ez = uz * uz * (-hw * (R(2) * Kzz - Kxx - Kyy) - R(0.5) * trn);
        const R es = ex + ey + ez, cw = R(3) - R(3) * hw;
        // deviator part: -cw (e_a - es/3); trace part: -(3/2) es over 3 axes
        ax -= cw * (ex - es * third) + R(0.5) * es;
        ay -= cw * (ey - es * third) + R(0.5) * es;
        az -= cw * (ez - es * third) + R(0.5) * es;
    }
    const R bxy = om1 * Kxy, bxz = om1 * Kxz, byz = om1 * Kyz;
    // post-collision central moments minus their rest values
    R k[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) k[i] = R(0);
    k[MI(1, 0, 0)] = R(0.5) * gx;
    k[MI(0, 1, 0)] = R(0.5) * gy;
    k[MI(0, 0, 1)] = R(0.5) * gz;
    k[MI(2, 0, 0)] = ax;
    k[MI(0, 2, 0)] = ay;
    k[MI(0, 0, 2)] = az;
    k[MI(1, 1, 0)] = bxy;
    k[MI(1, 0, 1)] = bxz;
    k[MI(0, 1, 1)] = byz;
    const R sx = third + ax, sy = third + ay, sz = third + az;
    k[MI(2, 2, 0)] = (ax + ay) * third + ax * ay + R(2) * bxy * bxy;
    k[MI(2, 0, 2)] = (ax + az) * third + ax * az + R(2) * bxz * bxz;
    k[MI(0, 2, 2)] = (ay + az) * third + ay * az + R(2) * byz * byz;
    k[MI(2, 1, 1)] = sx * byz + R(2) * bxy * bxz;
    k[MI(1, 2, 1)] = sy * bxz + R(2) * bxy * byz;
    k[MI(1, 1, 2)] = sz * bxy + R(2) * bxz * byz;
    k[MI(2, 2, 2)] = (ax + ay + az) * R(1.0 / 9.0) + (ax * ay + ay * az + ax * az) * third
                     + ax * ay * az
                     + R(2) * (sx * byz * byz + sy * bxz * bxz + sz * bxy * bxy)
                     + R(8) * bxy * bxz * byz;
    // back to velocity space about u (linear, so applied to the deviations)
    const Chimera<R> chx(ux), chy(uy), chz(uz);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) chx.apply(k[MI(0, b, c)], k[MI(1, b, c)], k[MI(2, b, c)]);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) chy.apply(k[MI(a, 0, c)], k[MI(a, 1, c)], k[MI(a, 2, c)]);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) chz.apply(k[MI(a, b, 0)], k[MI(a, b, 1)], k[MI(a, b, 2)]);
    // rest state about u is the product equilibrium: f* = rho (w + D + G)
    E D[27];
    product_dev(E(uxd), E(uyd), E(uzd), D);
    const E dre = E(drho_d), re = E(rho_d);
#pragma unroll
    for (int i = 0; i < 27; ++i) out[i] = dre * (E(wgt(i)) + D[i]) + D[i] + re * E(k[i]);
}

// ---------------------------------------------------------------- geometry
// Finite-difference interface geometry of a 3x3x3 fill stencil s (index
// MI(a,b,c) = offset (a-1,b-1,c-1)), Section 2.2: Parker-Youngs normal
// (gradient of the fill level with weights 1-2-1 across, pointing from
// liquid to gas) and mean curvature -(tr H - h.H.h) / (2 |g|) from the
// central-difference Hessian H.  Returns (nx, ny, nz, kappa); all zero where
// the gradient vanishes.  FP64: the normal decides which links are
// reconstructed, so the decision is taken at the fill level's precision.
__device__ __forceinline__ double4 fd_geometry(const double s[27])
{
    const double W[3] = {1.0, 2.0, 1.0};
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double w = W[p] * W[q];
            gx += w * (s[MI(2, p, q)] - s[MI(0, p, q)]);
            gy += w * (s[MI(p, 2, q)] - s[MI(p, 0, q)]);
            gz += w * (s[MI(p, q, 2)] - s[MI(p, q, 0)]);
        }
    gx /= 32.0;
    gy /= 32.0;
    gz /= 32.0;
    const double gn = sqrt(gx * gx + gy * gy + gz * gz);
    double4 o = make_double4(0.0, 0.0, 0.0, 0.0);
    if (gn < 1e-12) return o;
    const double hx = gx / gn, hy = gy / gn, hz = gz / gn;
    const double c0 = s[MI(1, 1, 1)];
    const double Hxx = s[MI(2, 1, 1)] - 2.0 * c0 + s[MI(0, 1, 1)];
    const double Hyy = s[MI(1, 2, 1)] - 2.0 * c0 + s[MI(1, 0, 1)];
    const double Hzz = s[MI(1, 1, 2)] - 2.0 * c0 + s[MI(1, 1, 0)];
    const double Hxy = 0.25 * (s[MI(2, 2, 1)] - s[MI(2, 0, 1)] - s[MI(0, 2, 1)] + s[MI(0, 0, 1)]);
    const double Hxz = 0.25 * (s[MI(2, 1, 2)] - s[MI(2, 1, 0)] - s[MI(0, 1, 2)] + s[MI(0, 1, 0)]);
    const double Hyz = 0.25 * (s[MI(1, 2, 2)] - s[MI(1, 2, 0)] - s[MI(1, 0, 2)] + s[MI(1, 0, 0)]);
    const double tr = Hxx + Hyy + Hzz;
    const double gHg = hx * hx * Hxx + hy * hy * Hyy + hz * hz * Hzz + 2.0 * (hx * hy * Hxy + hx * hz * Hxz + hy * hz * Hyz);
    o.x = -hx;
    o.y = -hy;
    o.z = -hz;
    o.w = -(tr - gHg) / (2.0 * gn);
    return o;
}

// Curvature as half the divergence of the unit normal (Brackbill et al.
// 1992): normals -grad/|grad| at the 8 cell corners from the 2x2x2 cells
// around each corner, divergence from the differences between the four
// corners on either side.  Corner gradients below 0.01 give the shortened
// normal -grad/0.01, which keeps the curvature continuous where a corner's
// gradient vanishes.  The free-surface variant that replaces the Hessian
// curvature above.
__device__ __forceinline__ double csf_curvature(const double s[27])
{
    double div = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // offsets 0 or the corner's side (-1 or +1), as stencil indices
                const int X = 2 * a, Y = 2 * b, Z = 2 * c;
                double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int py = p ? Y : 1, qz = q ? Z : 1, px = p ? X : 1, qy = q ? Y : 1;
                        gx += s[MI(X, py, qz)] - s[MI(1, py, qz)];
                        gy += s[MI(px, Y, qz)] - s[MI(px, 1, qz)];
                        gz += s[MI(px, qy, Z)] - s[MI(px, qy, 1)];
                    }
                gx *= 0.25 * (2 * a - 1);
                gy *= 0.25 * (2 * b - 1);
                gz *= 0.25 * (2 * c - 1);
                const double gn = sqrt(gx * gx + gy * gy + gz * gz);
                const double gd = gn > 1e-2 ? gn : 1e-2;
                const double nx = -gx / gd, ny = -gy / gd, nz = -gz / gd;
                div += 0.25 * (2 * a - 1) * nx;
                div += 0.25 * (2 * b - 1) * ny;
                div += 0.25 * (2 * c - 1) * nz;
            }
    return 0.5 * div;
}

// ---------------------------------------------------------------- watchdog
// Per-thread accumulation of the watchdog quantities of the step kernels:
// the FP64 mass of the cells a thread updates, their density range, and the
// number of cells whose density is outside [0.5, 1.5] or not a number.
struct Watch {
    double mass = 0.0;
    float rmin = 3.0e38f, rmax = -3.0e38f;
    int bad = 0;
    __device__ __forceinline__ void add(double m, double rho)
    {
        mass += m;
        const float r = (float)rho;
        rmin = fminf(rmin, r);
        rmax = fmaxf(rmax, r);
        bad += !(rho >= 0.5 && rho <= 1.5);
    }
};

// Reduce a block's Watch values (every thread of the block calls this, in
// uniform control flow) in a fixed order -- butterflies within each
// wavefront, then the wavefronts in order -- and let thread 0 write 4
// doubles: mass, lowest density, highest density, cells out of range.
template <int NT>
__device__ __forceinline__ void block_watch(Watch w, double *out)
{
    __shared__ double s_m[NT / 64];
    __shared__ float s_lo[NT / 64], s_hi[NT / 64];
    __shared__ int s_bad[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        w.mass += __shfl_xor(w.mass, o);
        w.rmin = fminf(w.rmin, __shfl_xor(w.rmin, o));
        w.rmax = fmaxf(w.rmax, __shfl_xor(w.rmax, o));
        w.bad += __shfl_xor(w.bad, o);
    }
    const int wv = (int)threadIdx.x >> 6;
    if (__lane_id() == 0) {
        s_m[wv] = w.mass;
        s_lo[wv] = w.rmin;
        s_hi[wv] = w.rmax;
        s_bad[wv] = w.bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        float lo = 3.0e38f, hi = -3.0e38f;
        int bad = 0;
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) {
            m += s_m[k];
            lo = fminf(lo, s_lo[k]);
            hi = fmaxf(hi, s_hi[k]);
            bad += s_bad[k];
        }
        out[0] = m;
        out[1] = (double)lo;
        out[2] = (double)hi;
        out[3] = (double)bad;
    }
}

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int wrap_m(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrap_p(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// Wave-aggregated append of `value` to list[] when pred holds: one atomic
// per wavefront.  Call with every active lane of the wave.
__device__ __forceinline__ void list_append(int32_t *list, int32_t *counter, bool pred, int32_t value)
{
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) list[base + (int)__popcll(mask & ((1ull << lane) - 1ull))] = value;
}

// Appends c0 + k for every set bit k of bits (ascending) to list: lanes hold
// consecutive cell groups, so the list gets the wavefront's cells in cell
// order (the list kernels' loads stay coalesced); one atomic per wavefront.
__device__ __forceinline__ void list_append_bits(int32_t *list, int32_t *counter, uint32_t bits, int32_t c0)
{
    const int n = __popcll((unsigned long long)bits);
    const int lane = __lane_id();
    int inc = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
    }
    const int total = __shfl(inc, 63);
    if (total == 0) return;
    int base = 0;
    if (lane == 63) base = atomicAdd(counter, total);
    base = __shfl(base, 63);
    int pos = base + inc - n;
    while (bits) {
        const int k = __ffsll((unsigned long long)bits) - 1;
        bits &= bits - 1u;
        list[pos++] = c0 + k;
    }
}

}  // namespace fsl
