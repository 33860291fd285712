// fsl_mlp.hip -- the learned interface estimator on gfx950: a 27 -> 64 ->
// 64 -> 4 perceptron (tanh hidden layers) from the 3x3x3 fill stencil of an
// interface cell to the correction of its finite-difference normal (outputs
// 0..2) and of 4 x its mean curvature (output 3).  BF16 weights and
// activations on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32
// accumulation), FP32 master weights, Adam.  The kernels train and evaluate
// the network on whatever targets they are given; the lattice kernel adds
// its outputs to the finite-difference estimate.
//
// Layout of the flat FP32 parameter vector (6212 floats):
//   W1[64][27], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]
//
// Matrix-core conventions (16x16x16 tile, lane l = r + 16 q):
//   A (M x K): lane holds A[r][4q .. 4q+3]
//   B (K x N): lane holds B[4q .. 4q+3][r]
//   C (M x N): lane holds C[4q .. 4q+3][r]
// Every layer is computed transposed, Z^T = W H^T, with samples along N: the
// C tile of one layer (lane: sample r, features 4q..4q+3) is then exactly
// the B operand of the next layer's K block, so activations never leave the
// registers in the forward and backward passes.  Only the weight gradients
// (a contraction over samples) need the activations transposed, via LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsl_device.h"
#include "fsl_kernels.h"
#include "fsl_mlp.h"

namespace fsl {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// FP32 -> BF16 bits, round to nearest even
__host__ __device__ __forceinline__ uint16_t bf16_bits(float x)
{
    uint32_t u;
    __builtin_memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// tanh(x) = 1 - 2 / (e^{2x} + 1) with the hardware base-2 exponential and
// reciprocal: no branches, saturates to +-1 (e^{2x} -> inf or 0), absolute
// error ~1e-7 -- far below the BF16 rounding of the activations.
__device__ __forceinline__ float act_tanh(float x)
{
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);  // e^{2x}
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ __forceinline__ v4s pack4(float a, float b, float c, float d)
{
    v4s v;
    v[0] = (short)bf16_bits(a);
    v[1] = (short)bf16_bits(b);
    v[2] = (short)bf16_bits(c);
    v[3] = (short)bf16_bits(d);
    return v;
}

// 4 consecutive bf16 of a row-major bf16 matrix (8-byte aligned)
__device__ __forceinline__ v4s ld4(const uint16_t *m)
{
    return *(const v4s *)m;
}

// ---------------------------------------------------------------- packing
// Packed BF16 copies of the weights, each laid out as the A operand it feeds:
//   W1p [64][32] (inputs padded), W2p [64][64], W3p [16][64] (outputs padded),
//   W2t [64][64] = W2^T, W3t [64][16] = W3^T (padded)
__global__ void k_mlp_pack(const float *P, uint16_t *pk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_PACK_SIZE) return;
    float v = 0.f;
    if (i < MLP_W2P) {                         // W1p
        const int m = i / 32, k = i % 32;
        v = k < 27 ? P[MLP_OFF_W1 + m * 27 + k] : 0.f;
    } else if (i < MLP_W3P) {                  // W2p
        const int t = i - MLP_W2P;
        v = P[MLP_OFF_W2 + t];
    } else if (i < MLP_W2T) {                  // W3p
        const int t = i - MLP_W3P, m = t / 64, k = t % 64;
        v = m < 4 ? P[MLP_OFF_W3 + m * 64 + k] : 0.f;
    } else if (i < MLP_W3T) {                  // W2t[m][k] = W2[k][m]
        const int t = i - MLP_W2T, m = t / 64, k = t % 64;
        v = P[MLP_OFF_W2 + k * 64 + m];
    } else {                                   // W3t[m][k] = W3[k][m]
        const int t = i - MLP_W3T, m = t / 16, k = t % 16;
        v = k < 4 ? P[MLP_OFF_W3 + k * 64 + m] : 0.f;
    }
    pk[i] = bf16_bits(v);
}

// ---------------------------------------------------------------- forward
struct Fwd {
    float h1[4][4], h2[4][4];  // [tile][j]: sample r, feature 16 t + 4 q + j
    v4s h1b[4], h2b[4];
    float y[4];                // lane q == 0: outputs 0..3 of sample r
};

// forward pass of 16 samples; xb[kt]: B operand of the inputs (K block kt)
__device__ __forceinline__ void mlp_forward16(const uint16_t *sW, const float *P, const v4s xb[2], Fwd &F)
{
    const int l = __lane_id(), r = l & 15, q = l >> 4;
    const uint16_t *W1p = sW, *W2p = sW + MLP_W2P, *W3p = sW + MLP_W3P;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) acc = mfma(ld4(W1p + (16 * mt + r) * 32 + 16 * kt + 4 * q), xb[kt], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) F.h1[mt][j] = act_tanh(acc[j] + P[MLP_OFF_B1 + 16 * mt + 4 * q + j]);
        F.h1b[mt] = pack4(F.h1[mt][0], F.h1[mt][1], F.h1[mt][2], F.h1[mt][3]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) acc = mfma(ld4(W2p + (16 * mt + r) * 64 + 16 * kt + 4 * q), F.h1b[kt], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) F.h2[mt][j] = act_tanh(acc[j] + P[MLP_OFF_B2 + 16 * mt + 4 * q + j]);
        F.h2b[mt] = pack4(F.h2[mt][0], F.h2[mt][1], F.h2[mt][2], F.h2[mt][3]);
    }
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) acc = mfma(ld4(W3p + r * 64 + 16 * kt + 4 * q), F.h2b[kt], acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) F.y[j] = q == 0 ? acc[j] + P[MLP_OFF_B3 + j] : 0.f;
}

// stage the first n packed weights (n a multiple of 8) of one workgroup in
// LDS: 16-byte loads, eight per thread in flight before they are stored
template <int N>
__device__ __forceinline__ void load_weights(uint16_t *sW, const uint16_t *pk)
{
    static_assert(N % 8 == 0, "16-byte chunks");
    constexpr int NV = N / 8;
    const uint4 *s = (const uint4 *)pk;
    uint4 *d = (uint4 *)sW;
    for (int i0 = 0; i0 < NV; i0 += 8 * (int)blockDim.x) {
        // every lane loads (the index clamped in range), so that the eight
        // values stay in registers
        uint4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = i0 + k * (int)blockDim.x + (int)threadIdx.x;
            v[k] = s[i < NV ? i : 0];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = i0 + k * (int)blockDim.x + (int)threadIdx.x;
            if (i < NV) d[i] = v[k];
        }
    }
}

// ---------------------------------------------------------------- training
// Loss gradient of a batch: each single-wave workgroup takes groups of 16
// samples (sample ids idx[...]), accumulates the weight gradients of its
// groups in matrix-core accumulators and writes one partial gradient; the
// partials are summed in a fixed order by k_mlp_reduce.
__global__ __launch_bounds__(64) void k_mlp_grad(const float *X, const float *T, const int32_t *idx,
                                                 int nbatch, float inv_n, const float *P,
                                                 const uint16_t *pk, int groups_per_wave,
                                                 float *partial, float *partial_loss)
{
    __shared__ __attribute__((aligned(16))) uint16_t sW[MLP_PACK_SIZE];
    __shared__ __attribute__((aligned(16))) uint16_t sX[32 * 16], sH1[64 * 16], sH2[64 * 16],
        sD1[64 * 16], sD2[64 * 16], sDY[16 * 16];
    load_weights<MLP_PACK_SIZE>(sW, pk);
    __syncthreads();
    const uint16_t *W2t = sW + MLP_W2T, *W3t = sW + MLP_W3T;
    const int l = __lane_id(), r = l & 15, q = l >> 4;

    v4f gW1[4][2], gW2[4][4], gW3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW3[a] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < 2; ++b) gW1[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < 4; ++b) gW2[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    float gb1[4][4] = {}, gb2[4][4] = {}, gb3[4] = {}, loss = 0.f;

    for (int g = 0; g < groups_per_wave; ++g) {
        const int s = (blockIdx.x * groups_per_wave + g) * 16 + r;
        const bool valid = s < nbatch;
        const int sid = valid ? (idx ? idx[s] : s) : 0;  // no id list: samples in order
        // inputs: clamp(phi) - 1/2, features 16 kt + 4 q + j
        v4s xb[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * kt + 4 * q + j;
                float x = (valid && k < 27) ? X[(size_t)sid * 27 + k] : 0.5f;
                x = fminf(fmaxf(x, 0.f), 1.f) - 0.5f;
                v[j] = (valid && k < 27) ? x : 0.f;
                sX[k * 16 + r] = bf16_bits(v[j]);
            }
            xb[kt] = pack4(v[0], v[1], v[2], v[3]);
        }
        Fwd F;
        mlp_forward16(sW, P, xb, F);
        // output gradient (lanes q == 0 own sample r's four outputs)
        float dy[4] = {0.f, 0.f, 0.f, 0.f};
        if (q == 0 && valid) {
            // loss |y[0..2] - n*|^2 + (y[3] - 4 kappa*)^2
            const float *t = T + (size_t)sid * 4;
            float e[4];
            for (int a = 0; a < 3; ++a) e[a] = F.y[a] - t[a];
            e[3] = F.y[3] - 4.f * t[3];
            for (int a = 0; a < 4; ++a) dy[a] = 2.f * e[a] * inv_n;
            loss += e[0] * e[0] + e[1] * e[1] + e[2] * e[2] + e[3] * e[3];
        }
        const v4s dyb = pack4(dy[0], dy[1], dy[2], dy[3]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sDY[(4 * q + j) * 16 + r] = bf16_bits(dy[j]);
            gb3[j] += dy[j];
        }
        // dH2^T = W3^T dY^T, dZ2 = dH2 (1 - H2^2)
        v4s d2b[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(ld4(W3t + (16 * mt + r) * 16 + 4 * q), dyb, acc);
            float dz[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dz[j] = valid ? acc[j] * (1.f - F.h2[mt][j] * F.h2[mt][j]) : 0.f;
                gb2[mt][j] += dz[j];
                sD2[(16 * mt + 4 * q + j) * 16 + r] = bf16_bits(dz[j]);
                sH1[(16 * mt + 4 * q + j) * 16 + r] = bf16_bits(valid ? F.h1[mt][j] : 0.f);
                sH2[(16 * mt + 4 * q + j) * 16 + r] = bf16_bits(valid ? F.h2[mt][j] : 0.f);
            }
            d2b[mt] = pack4(dz[0], dz[1], dz[2], dz[3]);
        }
        // dH1^T = W2^T dZ2^T, dZ1 = dH1 (1 - H1^2)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) acc = mfma(ld4(W2t + (16 * mt + r) * 64 + 16 * kt + 4 * q), d2b[kt], acc);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float dz = valid ? acc[j] * (1.f - F.h1[mt][j] * F.h1[mt][j]) : 0.f;
                gb1[mt][j] += dz;
                sD1[(16 * mt + 4 * q + j) * 16 + r] = bf16_bits(dz);
            }
        }
        __syncthreads();
        // weight gradients, contracted over the 16 samples of the group:
        // dW = dZ^T H with A rows = output features, B rows = input features
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const v4s a1 = ld4(sD1 + (16 * mt + r) * 16 + 4 * q);
            const v4s a2 = ld4(sD2 + (16 * mt + r) * 16 + 4 * q);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) gW1[mt][nt] = mfma(a1, ld4(sX + (16 * nt + r) * 16 + 4 * q), gW1[mt][nt]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) gW2[mt][nt] = mfma(a2, ld4(sH1 + (16 * nt + r) * 16 + 4 * q), gW2[mt][nt]);
        }
        const v4s a3 = ld4(sDY + r * 16 + 4 * q);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) gW3[nt] = mfma(a3, ld4(sH2 + (16 * nt + r) * 16 + 4 * q), gW3[nt]);
        __syncthreads();
    }

    // bias sums over the 16 samples held by lanes r = 0..15 of each q
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                gb1[a][j] += __shfl_xor(gb1[a][j], off);
                gb2[a][j] += __shfl_xor(gb2[a][j], off);
            }
#pragma unroll
        for (int j = 0; j < 4; ++j) gb3[j] += __shfl_xor(gb3[j], off);
        loss += __shfl_xor(loss, off);
    }
    float *out = partial + (size_t)blockIdx.x * MLP_NPARAM;
    // C layout: lane holds rows 4q + j (output feature), column r (input feature)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 16 * mt + 4 * q + j;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int k = 16 * nt + r;
                if (k < 27) out[MLP_OFF_W1 + m * 27 + k] = gW1[mt][nt][j];
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) out[MLP_OFF_W2 + m * 64 + 16 * nt + r] = gW2[mt][nt][j];
            if (r == 0) {
                out[MLP_OFF_B1 + m] = gb1[mt][j];
                out[MLP_OFF_B2 + m] = gb2[mt][j];
            }
        }
    }
    if (q == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) out[MLP_OFF_W3 + j * 64 + 16 * nt + r] = gW3[nt][j];
        if (r == 0) {
            for (int j = 0; j < 4; ++j) out[MLP_OFF_B3 + j] = gb3[j];
            partial_loss[blockIdx.x] = loss * inv_n;
        }
    }
}

// grad[i] = sum over waves of partial[w][i], fixed order
__global__ void k_mlp_reduce(const float *partial, const float *partial_loss, int nwaves, float *grad,
                             float *loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_NPARAM) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += partial[(size_t)w * MLP_NPARAM + i];
        grad[i] = s;
    }
    if (i == 0) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += partial_loss[w];
        *loss = s;
    }
}

// One training update per parameter: sum the per-wave partial gradients in a
// fixed order, apply Adam (Kingma & Ba 2015) to the FP32 master weight and refresh its BF16
// copies in the packed operands (the padding entries stay as packed at the
// start); thread 0 also sums the batch loss.
__global__ void k_mlp_update(const float *partial, const float *partial_loss, int nwaves, float *P, float *m,
                             float *v, float lr, float b1, float b2, float eps, float c1, float c2,
                             uint16_t *pk, float *loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += partial_loss[w];
        *loss = s;
    }
    if (i >= MLP_NPARAM) return;
    float gi = 0.f;
    for (int w = 0; w < nwaves; ++w) gi += partial[(size_t)w * MLP_NPARAM + i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    P[i] = pi;
    const uint16_t h = bf16_bits(pi);
    if (i < MLP_OFF_B1) {
        const int t = i - MLP_OFF_W1;
        pk[(t / 27) * 32 + t % 27] = h;
    } else if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) {
        const int t = i - MLP_OFF_W2;
        pk[MLP_W2P + t] = h;
        pk[MLP_W2T + (t % 64) * 64 + t / 64] = h;
    } else if (i >= MLP_OFF_W3 && i < MLP_OFF_B3) {
        const int t = i - MLP_OFF_W3;
        pk[MLP_W3P + (t / 64) * 64 + t % 64] = h;
        pk[MLP_W3T + (t % 64) * 16 + t / 64] = h;
    }
}

// ---------------------------------------------------------------- inference
// batch inference: 16 samples per wave iteration
__global__ __launch_bounds__(64) void k_mlp_infer(const float *X, int n, const float *P, const uint16_t *pk,
                                                  float *Y)
{
    __shared__ __attribute__((aligned(16))) uint16_t sW[MLP_PACK_SIZE];
    load_weights<MLP_W2T>(sW, pk);  // forward weights only
    __syncthreads();
    const int l = __lane_id(), r = l & 15, q = l >> 4;
    for (int g = blockIdx.x; g * 16 < n; g += gridDim.x) {
        const int s = g * 16 + r;
        const bool valid = s < n;
        v4s xb[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * kt + 4 * q + j;
                const float x = (valid && k < 27) ? X[(size_t)s * 27 + k] : 0.5f;
                v[j] = (valid && k < 27) ? fminf(fmaxf(x, 0.f), 1.f) - 0.5f : 0.f;
            }
            xb[kt] = pack4(v[0], v[1], v[2], v[3]);
        }
        Fwd F;
        mlp_forward16(sW, P, xb, F);
        if (q == 0 && valid)
            for (int j = 0; j < 4; ++j) Y[(size_t)s * 4 + j] = F.y[j];
    }
}

// ---------------------------------------------------------------- lattice
__device__ __forceinline__ int nb_cell(const Dev &d, int x, int y, int z, int i)
{
    const int zz = z + cz(i);
    if (zz < 0 || zz >= d.nz) return -1;
    const int xx = cx(i) == 1 ? wrap_p(x, d.nx) : (cx(i) == -1 ? wrap_m(x, d.nx) : x);
    const int yy = cy(i) == 1 ? wrap_p(y, d.ny) : (cy(i) == -1 ? wrap_m(y, d.ny) : y);
    return xx + d.nx * (yy + d.ny * zz);
}

// Ties a loaded value to this point so that the loads of a stage are issued
// together (empty asm statement on the register; no instruction).
template <class T>
__device__ __forceinline__ void keep_reg(T &v)
{
    asm volatile("" : "+v"(v));
}

// Per-cell outcome of the learned estimator (read back as a field): the
// corrected estimate was used, or finite differences were kept because of a
// solid or wall neighbour, |n_raw| outside [0.5, 2], an angle to the finite-
// difference normal above 30 degrees, or |kappa| > 0.5 (first rule that holds).
enum : uint8_t { EST_NETWORK = 1, EST_SOLID = 2, EST_LENGTH = 3, EST_ANGLE = 4, EST_KAPPA = 5 };

// Interface normal and curvature with the learned estimator: per group of 16
// interface cells, the four lanes of a cell (lane = cell + 16 q) gather
// entries q, q+4, ... of its fill stencil (liquid 1, gas 0, interface
// clamp(m/rho), wall/solid = centre), lanes q == 0 compute the finite-
// difference estimate (n_fd, k_fd) and the wavefront runs the network, whose
// outputs y correct it: n_raw = n_fd + y[0..2], kappa = k_fd + y[3] / 4.
// The corrected estimate replaces the finite-difference one unless a stencil
// cell is solid, |n_raw| lies outside [0.5, 2], the two normals differ by
// more than 30 degrees, or |kappa| > 0.5.  Counters are aggregated per
// wavefront.
template <class R>
__global__ __launch_bounds__(64) void k_geom_mlp(Dev d, int which, const float *P, const uint16_t *pk)
{
    using R4 = typename std::conditional<sizeof(R) == 8, double4, float4>::type;
    __shared__ __attribute__((aligned(16))) uint16_t sW[MLP_W2T];
    __shared__ double sS[16][28];
    load_weights<MLP_W2T>(sW, pk);
    __syncthreads();
    const int32_t *list = d.list[which];
    const int count = d.cnt[which];
    const int l = __lane_id(), r = l & 15, q = l >> 4;
    unsigned long long used = 0, fell = 0;
    for (int g = blockIdx.x; g * 16 < count; g += gridDim.x) {
        const int t = g * 16 + r;
        const bool valid = t < count;
        const int c = valid ? list[t] : 0;
        const int x = c % d.nx, y = (c / d.nx) % d.ny, z = c / (d.nx * d.ny);
        // entries k = q + 4 m of the stencil, all loads issued together
        uint32_t fl[7];
        double ph[7];
        double pc = d.phi[c];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const int k = q + 4 * m;
            const int yc = k < 27 ? nb_cell(d, x, y, z, k) : -1;
            const uint32_t a = (uint32_t)(yc < 0 ? c : yc);
            fl[m] = yc < 0 ? (uint32_t)T_SOLID : (uint32_t)d.flags[a];
            ph[m] = d.phi[a];
        }
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            keep_reg(fl[m]);
            keep_reg(ph[m]);
        }
        keep_reg(pc);
        const double centre = pc < 0.0 ? 0.0 : (pc > 1.0 ? 1.0 : pc);
        bool solid = false;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const int k = q + 4 * m;
            if (k >= 27) continue;
            const uint32_t ty = fl[m] & T_MASK;
            const double pv = ph[m] < 0.0 ? 0.0 : (ph[m] > 1.0 ? 1.0 : ph[m]);
            solid |= k != REST && ty == T_SOLID;
            sS[r][k] = k == REST ? centre
                                 : (ty == T_LIQ ? 1.0 : (ty == T_GAS ? 0.0 : (ty == T_IF ? pv : centre)));
        }
        const uint64_t sb = __ballot(solid);
        const bool any_solid = ((sb >> r) | (sb >> (r + 16)) | (sb >> (r + 32)) | (sb >> (r + 48))) & 1ull;
        __syncthreads();
        double4 fd = make_double4(0.0, 0.0, 0.0, 0.0);
        if (q == 0) {
            double st[27];
#pragma unroll
            for (int i = 0; i < 27; ++i) st[i] = sS[r][i];
            fd = fd_geometry(st);
        }
        v4s xb[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * kt + 4 * q + j;
                v[j] = (valid && k < 27) ? (float)sS[r][k] - 0.5f : 0.f;
            }
            xb[kt] = pack4(v[0], v[1], v[2], v[3]);
        }
        Fwd F;
        mlp_forward16(sW, P, xb, F);
        __syncthreads();
        bool use = false;
        if (q == 0 && valid) {
            R4 out;
            out.x = R(fd.x);
            out.y = R(fd.y);
            out.z = R(fd.z);
            out.w = R(fd.w);
            // the network corrects the finite-difference estimate; the first
            // rule that fails keeps finite differences (codes 2..5)
            const double nx = fd.x + (double)F.y[0], ny = fd.y + (double)F.y[1], nz = fd.z + (double)F.y[2];
            const double rn = sqrt(nx * nx + ny * ny + nz * nz);
            const double kap = fd.w + 0.25 * (double)F.y[3];
            uint8_t rule = EST_NETWORK;
            if (any_solid) {
                rule = EST_SOLID;
            } else if (!(rn >= 0.5 && rn <= 2.0)) {
                rule = EST_LENGTH;
            } else {
                // cosine of the angle between n_raw and the unit (or zero) n_fd
                const double cosang = (fd.x * nx + fd.y * ny + fd.z * nz) / rn;
                if (!(cosang >= 0.8660254037844386)) rule = EST_ANGLE;
                else if (!(fabs(kap) <= 0.5)) rule = EST_KAPPA;
            }
            use = rule == EST_NETWORK;
            d.est[c] = rule;
            if (use) {
                out.x = R(nx / rn);
                out.y = R(ny / rn);
                out.z = R(nz / rn);
                out.w = R(kap);
            }
            ((R4 *)d.geom)[c] = out;
        }
        used += __popcll(__ballot(q == 0 && valid && use));
        fell += __popcll(__ballot(q == 0 && valid && !use));
    }
    if (l == 0) {
        if (used) atomicAdd(&d.stats[8], used);
        if (fell) atomicAdd(&d.stats[9], fell);
    }
}

// finite-difference geometry of stencils given as fill levels [n][27]
__global__ __launch_bounds__(256) void k_fd_stencils(const float *X, int n, float *Y)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        double s[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const double v = (double)X[(size_t)t * 27 + i];
            s[i] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
        }
        const double4 g = fd_geometry(s);
        float4 o;
        o.x = (float)g.x;
        o.y = (float)g.y;
        o.z = (float)g.z;
        o.w = (float)g.w;
        ((float4 *)Y)[t] = o;
    }
}

// Fill levels of analytic stencils by supersampling: one wavefront per
// (stencil, cell); each cell is sampled on ss^3 points (i + 1/2)/ss - 1/2
// per axis around its offset (a-1, b-1, c-1), entry a + 3b + 9c.  Shape
// parameters per stencil, 16 doubles: [0] kind (0 sphere, 1 sinusoidal
// sheet), [1] 1 to count the outside (a bubble), sphere: [2..4] centre X,
// [5] radius R -- inside if |p - X|^2 <= R^2; sheet: [2..4] e1, [5..7] e3,
// [8] A, [9] k, [10] psi, [11] s -- inside if p.e3 < A sin(k p.e1 + psi) + s.
// The inside tests round each product and sum on its own (no fused
// multiply-add), in the order written.
__global__ __launch_bounds__(256) void k_stencil_fill(const double *P, int n, int ss, float *X)
{
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = __lane_id();
    if (g >= n * 27) return;
    const int s = g / 27, k = g % 27;
    const double *q = P + (size_t)16 * s;
    const double ox = (double)(k % 3 - 1), oy = (double)((k / 3) % 3 - 1), oz = (double)(k / 9 - 1);
    const int np = ss * ss * ss;
    const double inv = 1.0 / (double)ss;
    int count = 0;
    for (int t = lane; t < np; t += 64) {
        const int i = t / (ss * ss), j = (t / ss) % ss, l = t % ss;
        const double px = __dadd_rn(ox, __dsub_rn(__dmul_rn((double)i + 0.5, inv), 0.5));
        const double py = __dadd_rn(oy, __dsub_rn(__dmul_rn((double)j + 0.5, inv), 0.5));
        const double pz = __dadd_rn(oz, __dsub_rn(__dmul_rn((double)l + 0.5, inv), 0.5));
        bool in;
        if (q[0] == 0.0) {
            const double dx = __dsub_rn(px, q[2]), dy = __dsub_rn(py, q[3]), dz = __dsub_rn(pz, q[4]);
            const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            in = r2 <= __dmul_rn(q[5], q[5]);
        } else {
            const double u = __dadd_rn(__dadd_rn(__dmul_rn(px, q[2]), __dmul_rn(py, q[3])), __dmul_rn(pz, q[4]));
            const double w = __dadd_rn(__dadd_rn(__dmul_rn(px, q[5]), __dmul_rn(py, q[6])), __dmul_rn(pz, q[7]));
            const double h = __dadd_rn(__dmul_rn(q[8], sin(__dadd_rn(__dmul_rn(q[9], u), q[10]))), q[11]);
            in = w < h;
        }
        count += in ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) count += __shfl_xor(count, o);
    if (lane == 0) {
        const float phi = (float)((double)count / (double)np);
        X[(size_t)s * 27 + k] = q[1] != 0.0 ? 1.0f - phi : phi;
    }
}

// ---------------------------------------------------------------- launchers
void stencil_fill(const double *P, int n, int ss, float *X, hipStream_t st)
{
    const int64_t waves = (int64_t)n * 27;
    k_stencil_fill<<<(int)((waves + 3) / 4), 256, 0, st>>>(P, n, ss, X);
}

void fd_stencils(const float *X, int n, float *Y, hipStream_t st)
{
    int blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_fd_stencils<<<blocks, 256, 0, st>>>(X, n, Y);
}

void mlp_pack(const float *P, uint16_t *pk, hipStream_t st)
{
    k_mlp_pack<<<(MLP_PACK_SIZE + 255) / 256, 256, 0, st>>>(P, pk);
}

void mlp_grad(const float *X, const float *T, const int32_t *idx, int nbatch, float inv_n, const float *P,
              const uint16_t *pk, int groups_per_wave, float *partial, float *partial_loss, int nwaves,
              float *grad, float *loss, hipStream_t st)
{
    k_mlp_grad<<<nwaves, 64, 0, st>>>(X, T, idx, nbatch, inv_n, P, pk, groups_per_wave, partial, partial_loss);
    k_mlp_reduce<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(partial, partial_loss, nwaves, grad, loss);
}

void mlp_train_step(const float *X, const float *T, const int32_t *idx, int nbatch, float inv_n, float *P,
                    float *m, float *v, uint16_t *pk, int groups_per_wave, float *partial, float *partial_loss,
                    int nwaves, float lr, float b1, float b2, float eps, float c1, float c2, float *loss,
                    hipStream_t st)
{
    k_mlp_grad<<<nwaves, 64, 0, st>>>(X, T, idx, nbatch, inv_n, P, pk, groups_per_wave, partial, partial_loss);
    k_mlp_update<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(partial, partial_loss, nwaves, P, m, v, lr, b1, b2,
                                                          eps, c1, c2, pk, loss);
}

void mlp_infer(const float *X, int n, const float *P, const uint16_t *pk, float *Y, hipStream_t st)
{
    int blocks = (n + 15) / 16;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_mlp_infer<<<blocks, 64, 0, st>>>(X, n, P, pk, Y);
}

template <class R>
void launch_geom_mlp(const Dev &d, int which, int blocks, const float *P, const uint16_t *pk, hipStream_t st)
{
    k_geom_mlp<R><<<blocks, 64, 0, st>>>(d, which, P, pk);
}
template void launch_geom_mlp<double>(const Dev &, int, int, const float *, const uint16_t *, hipStream_t);
template void launch_geom_mlp<float>(const Dev &, int, int, const float *, const uint16_t *, hipStream_t);

}  // namespace fsl
