// Learned hoppings: radial descriptor (Eq. (2)), per-bond MLP on bf16 MFMA,
// training (forward, backward, AdamW) and the fused learned assembly of H.
//
// Model: per unordered bond {i, j} the input is x = [f_0..f_7(r_ij) || v_i + v_j]
// (16 values, symmetric in i and j) with v_i = sum_j f(r_ij) over the descriptor
// cutoff and f_k(r) = (T_k(2 (r/rc - 1)^2 - 1) + 1)/2 * f_c(r),
// f_c(r) = (1 + cos(pi r / rc))/2; standardised per feature by fixed
// (shift, scale); MLP 16 -> 32 -> tanh -> 32 -> tanh -> 1; hopping
// t_ij = t_plain(r_ij) (1 + y_ij).  Parameters (FP32, 1633): W1 [32][16], b1 [32],
// W2 [32][32], b2 [32], W3 [32], b3.
//
// MFMA layout (v_mfma_f32_16x16x16_bf16, one wavefront, lane l, n = l % 16,
// q = l / 16): A[m][k] is held at lane m + 16 (k / 4), element k % 4; B[k][n]
// at lane n + 16 (k / 4), element k % 4; D[m][n] at lane n + 16 (m / 4),
// element m % 4.  The K = 32 products take one v_mfma_f32_16x16x32_bf16
// (mfma32) on the two K = 16 halves.  Activations are kept transposed (hidden x bonds): a tile of
// 16 bonds sits on n, so the D registers of one layer (hidden 16 m + 4 q + i)
// are exactly the B operand of the next layer's K-block m, with no shuffle.
// The weight-gradient products (sums over bonds) need bonds on K and go
// through an LDS transpose.  Every product uses bfloat16 operands (round to
// nearest even); sums are FP32 inside a wavefront and FP64 across wavefronts,
// in a fixed order.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdint>
#include <vector>

#include "builder.hpp"
#include "common.hpp"
#include "nlist.hpp"

namespace tbk {

namespace {

constexpr int kNR = 8;            // radial functions
constexpr int kNI = 16;           // MLP inputs
constexpr int kNH = 32;           // hidden width
constexpr int kNP = 1633;         // parameters
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 544, kOffB2 = 1568, kOffW3 = 1600, kOffB3 = 1632;
constexpr int kWaves = 4;         // wavefronts per block of the MLP kernels

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// double -> bfloat16 bits, one rounding (nearest even at the 8th significant bit).
__device__ __forceinline__ uint16_t d2bf(double x) {
    if (!(fabs(x) >= 0x1p-126) || !isfinite(x)) return f2bf((float)x);   // zero, subnormal range, inf, nan
    uint64_t u = (uint64_t)__double_as_longlong(x);
    u += (1ull << 44) - 1ull + ((u >> 45) & 1ull);
    u &= ~((1ull << 45) - 1ull);
    return (uint16_t)(__float_as_uint((float)__longlong_as_double((long long)u)) >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ float rbf(float x) { return bf2f(f2bf(x)); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

// The K = 32 products in one CDNA4 v_mfma_f32_16x16x32_bf16: lane n + 16 q holds
// K elements 8 q .. 8 q + 7 of A row n and of B column n.  The two K = 16 halves a
// lane already holds (elements 4 q .. 4 q + 3 of each half) are concatenated, so
// K element 8 q + j is index 4 q + j of the first half (j < 4) or of the second
// half (j >= 4) on both operands: the same 32 products as two chained K = 16 MFMAs.
__device__ __forceinline__ f32x4 mfma32(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c) {
    const s16x8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const s16x8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 r;
    r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
    return r;
}

// Chebyshev radial functions f_k(r), k < nk (recurrence for T_k).
__device__ __forceinline__ void radial(double r, double rc, int nk, double *f) {
    const double u = r / rc - 1.0;
    const double x = 2.0 * u * u - 1.0;
    const double c = r < rc ? 0.5 * (1.0 + cos(M_PI * r / rc)) : 0.0;
    double tm = 1.0, tn = x;
    for (int k = 0; k < nk; ++k) {
        double tk;
        if (k == 0) tk = 1.0;
        else if (k == 1) tk = x;
        else { const double tp = 2.0 * x * tn - tm; tm = tn; tn = tp; tk = tp; }
        f[k] = 0.5 * (tk + 1.0) * c;
    }
}

// ------------------------------------------------------------------------
// Descriptor, bonds, features, synthetic targets
// ------------------------------------------------------------------------

// Bond descriptor of Eq. (2): C_n(r) = sum_k c[n][k] f_k(r) with the
// coefficients c [nk][nk] of the bond's species pair, or f itself (c = NULL).
__device__ __forceinline__ void bond_basis(double r, double rc, int nk, const double *__restrict__ c, double *C) {
    double f[16];
    radial(r, rc, nk, f);
    for (int a = 0; a < nk; ++a) {
        if (!c) { C[a] = f[a]; continue; }
        double s = 0.0;
        for (int k = 0; k < nk; ++k) s += c[a * nk + k] * f[k];
        C[a] = s;
    }
}

// Coefficients of the species pair (s_i, s_j): cnk [ns][ns][nk][nk], or NULL.
__device__ __forceinline__ const double *pair_cnk(const double *__restrict__ cnk, const int32_t *__restrict__ species,
                                                  int32_t ns, int nk, int32_t i, int32_t j) {
    return cnk ? cnk + ((int64_t)species[i] * ns + species[j]) * nk * nk : nullptr;
}

__global__ void k_descriptor(CellList cl, const double *__restrict__ pos, int64_t n, double rc, int32_t nk,
                             const int32_t *__restrict__ species, int32_t ns, const double *__restrict__ cnk,
                             double *__restrict__ v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[16];
    for (int k = 0; k < nk; ++k) acc[k] = 0.0;
    for_each_neighbor(cl, pos, (int32_t)i, rc, [&](int32_t j, double r, double, double, double) {
        double f[16];
        bond_basis(r, rc, nk, pair_cnk(cnk, species, ns, nk, (int32_t)i, j), f);
        for (int k = 0; k < nk; ++k) acc[k] += f[k];
    });
    for (int k = 0; k < nk; ++k) v[i * nk + k] = acc[k];
}

// The same for a compile-time basis size (the workloads' 8 functions): the per-bond
// basis and the sums stay in registers instead of per-thread scratch memory.
template <int NK>
__global__ void k_descriptor_nk(CellList cl, const double *__restrict__ pos, int64_t n, double rc,
                                const int32_t *__restrict__ species, int32_t ns, const double *__restrict__ cnk,
                                double *__restrict__ v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) acc[k] = 0.0;
    for_each_neighbor(cl, pos, (int32_t)i, rc, [&](int32_t j, double r, double, double, double) {
        const double u = r / rc - 1.0;
        const double x = 2.0 * u * u - 1.0;
        const double c = r < rc ? 0.5 * (1.0 + cos(M_PI * r / rc)) : 0.0;
        double f[NK];
        double tm = 1.0, tn = x;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            double tk;
            if (k == 0) tk = 1.0;
            else if (k == 1) tk = x;
            else { const double tp = 2.0 * x * tn - tm; tm = tn; tn = tp; tk = tp; }
            f[k] = 0.5 * (tk + 1.0) * c;
        }
        const double *cp = pair_cnk(cnk, species, ns, NK, (int32_t)i, j);
        if (cp) {
#pragma unroll
            for (int a = 0; a < NK; ++a) {
                double sa = 0.0;
#pragma unroll
                for (int k = 0; k < NK; ++k) sa += cp[a * NK + k] * f[k];
                acc[a] += sa;
            }
        } else {
#pragma unroll
            for (int k = 0; k < NK; ++k) acc[k] += f[k];
        }
    });
#pragma unroll
    for (int k = 0; k < NK; ++k) v[i * NK + k] = acc[k];
}

__global__ void k_bond_count(CellList cl, const double *__restrict__ pos, int64_t n, double rc,
                             int64_t *__restrict__ cnt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t c = 0;
    for_each_neighbor(cl, pos, (int32_t)i, rc, [&](int32_t j, double, double, double, double) { c += (j > i); });
    cnt[i] = c;
}

// Bonds (i, j > i) of atom i at off[i], sorted by j.
__global__ void k_bond_fill(CellList cl, const double *__restrict__ pos, int64_t n, double rc,
                            const int64_t *__restrict__ off, int32_t *__restrict__ bi, int32_t *__restrict__ bj,
                            double *__restrict__ br) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = off[i];
    int64_t c = 0;
    for_each_neighbor(cl, pos, (int32_t)i, rc, [&](int32_t j, double r, double, double, double) {
        if (j > i) { bi[o + c] = (int32_t)i; bj[o + c] = j; br[o + c] = r; ++c; }
    });
    for (int64_t a = 1; a < c; ++a) {
        const int32_t jj = bj[o + a];
        const double rr = br[o + a];
        int64_t b = a - 1;
        while (b >= 0 && bj[o + b] > jj) { bj[o + b + 1] = bj[o + b]; br[o + b + 1] = br[o + b]; --b; }
        bj[o + b + 1] = jj;
        br[o + b + 1] = rr;
    }
}

struct FeatNorm {
    double shift[2 * kNR];
    double inv_scale[2 * kNR];
};

// Standardised bond feature k of bond (i, j, r) in double.
__device__ __forceinline__ void bond_features(double r, const double *__restrict__ vi, const double *__restrict__ vj,
                                              double rc, const FeatNorm &fn, double *x,
                                              const double *__restrict__ c = nullptr) {
    bond_basis(r, rc, kNR, c, x);
    for (int k = 0; k < kNR; ++k) x[kNR + k] = vi[k] + vj[k];
    for (int k = 0; k < kNI; ++k) x[k] = (x[k] - fn.shift[k]) * fn.inv_scale[k];
}

__global__ void k_bond_features(int64_t nb, const int32_t *__restrict__ bi, const int32_t *__restrict__ bj,
                                const double *__restrict__ br, const double *__restrict__ v, double rc, FeatNorm fn,
                                const int32_t *__restrict__ species, int32_t ns, const double *__restrict__ cnk,
                                uint16_t *__restrict__ X) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double x[kNI];
    bond_features(br[b], v + (int64_t)bi[b] * kNR, v + (int64_t)bj[b] * kNR, rc, fn, x,
                  pair_cnk(cnk, species, ns, kNR, bi[b], bj[b]));
    for (int k = 0; k < kNI; ++k) X[b * kNI + k] = d2bf(x[k]);
}

// Onsite-network inputs: X[i] = bf16([(v_i - shift) / scale || 0 x 8]).
__global__ void k_node_features(int64_t n, const double *__restrict__ v, FeatNorm fn, uint16_t *__restrict__ X) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < kNR; ++k) X[i * kNI + k] = d2bf((v[i * kNR + k] - fn.shift[k]) / fn.inv_scale[k]);
    for (int k = kNR; k < kNI; ++k) X[i * kNI + k] = 0;
}

// Per-block partial sums of each standardisation-free feature and its square
// (for the fixed feature shift/scale taken from training data): part[block][2][16].
__global__ __launch_bounds__(256) void k_feature_moments(int64_t nb, const int32_t *__restrict__ bi, const int32_t *__restrict__ bj,
                                  const double *__restrict__ br, const double *__restrict__ v, double rc,
                                  double *__restrict__ part) {
    __shared__ double red[2 * kNI][256];
    double x[kNI];
    double s1[kNI], s2[kNI];
    for (int k = 0; k < kNI; ++k) { s1[k] = 0.0; s2[k] = 0.0; }
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        radial(br[b], rc, kNR, x);
        for (int k = 0; k < kNR; ++k) x[kNR + k] = v[(int64_t)bi[b] * kNR + k] + v[(int64_t)bj[b] * kNR + k];
        for (int k = 0; k < kNI; ++k) { s1[k] += x[k]; s2[k] += x[k] * x[k]; }
    }
    for (int k = 0; k < kNI; ++k) { red[k][threadIdx.x] = s1[k]; red[kNI + k][threadIdx.x] = s2[k]; }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 2 * kNI; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if ((int)threadIdx.x < 2 * kNI) part[blockIdx.x * 2 * kNI + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_coord_target(int64_t nb, const int32_t *__restrict__ bi, const int32_t *__restrict__ bj,
                               const double *__restrict__ v, int32_t nk, double kappa, double z0,
                               float *__restrict__ y) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    y[b] = (float)(kappa * (v[(int64_t)bi[b] * nk] + v[(int64_t)bj[b] * nk] - 2.0 * z0));
}

// ------------------------------------------------------------------------
// MLP on one wavefront: 16 bonds per tile
// ------------------------------------------------------------------------

// Per-lane copies of the weights in MFMA operand layout.
struct WaveWeights {
    bf16x4 A1[2];        // W1[16 m + n][4 q + i]
    bf16x4 A2[2][2];     // W2[16 mo + n][16 kb + 4 q + i]
    bf16x4 A2T[2][2];    // W2[16 hb + 4 q + i][16 ko + n]      (W2 transposed)
    float b1[2][4], b2[2][4];  // b[16 m + 4 q + i]
    float w3[2][4];            // bf16(W3[16 m + 4 q + i])
    float b3;
};

__device__ __forceinline__ void load_weights(const float *__restrict__ P, WaveWeights &w) {
    const int l = threadIdx.x & 63, n = l & 15, q = l >> 4;
    for (int m = 0; m < 2; ++m) {
        const float *r1 = P + kOffW1 + (16 * m + n) * kNI + 4 * q;
        w.A1[m] = pack4(r1[0], r1[1], r1[2], r1[3]);
        for (int kb = 0; kb < 2; ++kb) {
            const float *r2 = P + kOffW2 + (16 * m + n) * kNH + 16 * kb + 4 * q;
            w.A2[m][kb] = pack4(r2[0], r2[1], r2[2], r2[3]);
            // transposed: element i = W2[16 kb + 4 q + i][16 m + n]
            const float *c2 = P + kOffW2 + (16 * kb + 4 * q) * kNH + 16 * m + n;
            w.A2T[m][kb] = pack4(c2[0], c2[kNH], c2[2 * kNH], c2[3 * kNH]);
        }
        for (int i = 0; i < 4; ++i) {
            w.b1[m][i] = P[kOffB1 + 16 * m + 4 * q + i];
            w.b2[m][i] = P[kOffB2 + 16 * m + 4 * q + i];
            w.w3[m][i] = rbf(P[kOffW3 + 16 * m + 4 * q + i]);
        }
    }
    w.b3 = P[kOffB3];
}

struct TileAct {
    f32x4 h1[2], h2[2];   // post-tanh activations, hidden 16 m + 4 q + i, bond n
    float y;              // output of bond n (all four q lanes)
};

// Forward pass of the 16 bonds whose features (bf16, 4 per lane) are xq.
__device__ __forceinline__ void mlp_tile_forward(const WaveWeights &w, bf16x4 xq, TileAct &a) {
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    bf16x4 hb[2];
    for (int m = 0; m < 2; ++m) {
        f32x4 z = mfma16(w.A1[m], xq, zero);
        for (int i = 0; i < 4; ++i) a.h1[m][i] = tanhf(z[i] + w.b1[m][i]);
        hb[m] = pack4(a.h1[m][0], a.h1[m][1], a.h1[m][2], a.h1[m][3]);
    }
    float part = 0.f;
    for (int mo = 0; mo < 2; ++mo) {
        const f32x4 z = mfma32(w.A2[mo][0], w.A2[mo][1], hb[0], hb[1], zero);
        for (int i = 0; i < 4; ++i) {
            a.h2[mo][i] = tanhf(z[i] + w.b2[mo][i]);
            part += w.w3[mo][i] * rbf(a.h2[mo][i]);
        }
    }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    a.y = part + w.b3;
}

// Order in which a minibatch takes the bonds of the training set, in chunks of 16
// consecutive bonds (one MFMA tile, so a tile's feature loads stay contiguous):
// position i = first + b lies in chunk c = i / 16, which takes stored chunk
// (mul c + add) mod n_chunks, a bijection of the n_chunks = n_total / 16 whole
// chunks when gcd(mul, n_chunks) = 1; the last n_total % 16 bonds keep their
// positions.  mul = 1, add = 0 is the stored order.
struct BondOrder {
    int64_t n_total, first, mul, add;
    __device__ __forceinline__ int64_t map(int64_t b) const {
        const int64_t i = first + b;
        const int64_t n_chunks = n_total >> 4;
        const int64_t c = i >> 4;
        if ((mul == 1 && add == 0) || c >= n_chunks) return i;
        const uint64_t pc = (uint64_t)(((unsigned __int128)mul * (uint64_t)c + (uint64_t)add) % (uint64_t)n_chunks);
        return (int64_t)(pc << 4) + (i & 15);
    }
};

// Features of bond tile t for this lane: X[16 t + n][4 q .. 4 q + 3]; zero past nb.
__device__ __forceinline__ bf16x4 load_x(const uint16_t *__restrict__ X, int64_t nb, int64_t b) {
    const int q = (threadIdx.x & 63) >> 4;
    bf16x4 r = {0, 0, 0, 0};
    if (b < nb) {
        const uint2 raw = *reinterpret_cast<const uint2 *>(X + b * kNI + 4 * q);
        r[0] = (short)(raw.x & 0xffff); r[1] = (short)(raw.x >> 16);
        r[2] = (short)(raw.y & 0xffff); r[3] = (short)(raw.y >> 16);
    }
    return r;
}

__global__ __launch_bounds__(64 * kWaves) void k_mlp_forward(int64_t nb, const uint16_t *__restrict__ X,
                                                             const float *__restrict__ P, float *__restrict__ y) {
    WaveWeights w;
    load_weights(P, w);
    const int l = threadIdx.x & 63, n = l & 15, q = l >> 4;
    const int64_t wave = blockIdx.x * (int64_t)kWaves + (threadIdx.x >> 6);
    const int64_t nwave = (int64_t)gridDim.x * kWaves;
    const int64_t ntile = (nb + 15) / 16;
    for (int64_t t = wave; t < ntile; t += nwave) {
        const int64_t b = 16 * t + n;
        TileAct a;
        mlp_tile_forward(w, load_x(X, nb, b), a);
        if (q == 0 && b < nb) y[b] = a.y;
    }
}

// Loss sum_b w_b (y_b - y*_b)^2 / B and its gradient: each wavefront writes its
// FP32 partial gradient (parameter layout) and FP64 partial loss.
__global__ __launch_bounds__(64 * kWaves) void k_mlp_grad(int64_t nb, const uint16_t *__restrict__ X,
                                                          const float *__restrict__ target,
                                                          const float *__restrict__ weight,
                                                          const float *__restrict__ P, float inv_b,
                                                          BondOrder order, float *__restrict__ gpart,
                                                          double *__restrict__ lpart) {
    __shared__ uint16_t s_d2[kWaves][16][kNH];
    __shared__ uint16_t s_h1[kWaves][16][kNH];
    __shared__ uint16_t s_d1[kWaves][16][kNH];
    __shared__ uint16_t s_x[kWaves][16][kNI];
    WaveWeights w;
    load_weights(P, w);
    const int wv = threadIdx.x >> 6;
    const int l = threadIdx.x & 63, n = l & 15, q = l >> 4;
    const int64_t wave = blockIdx.x * (int64_t)kWaves + wv;
    const int64_t nwave = (int64_t)gridDim.x * kWaves;
    const int64_t ntile = (nb + 15) / 16;
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    f32x4 gW1[2] = {zero, zero};                 // (h = 16 mh + 4 q + i, f = n)
    f32x4 gW2[2][2] = {{zero, zero}, {zero, zero}};  // (h = 16 mh + 4 q + i, k = 16 nk + n)
    float gb1[2][4] = {}, gb2[2][4] = {}, gw3[2][4] = {};
    float gb3 = 0.f;
    double loss = 0.0;
    for (int64_t t = wave; t < ntile; t += nwave) {
        const int64_t b = 16 * t + n;
        const bool ok = b < nb;
        const int64_t src = ok ? order.map(b) : 0;   // the training-set bond at minibatch position b
        const bf16x4 xq = load_x(X, order.n_total, ok ? src : order.n_total);
        TileAct a;
        mlp_tile_forward(w, xq, a);
        const float wb = ok ? (weight ? weight[src] : 1.f) : 0.f;
        const float diff = ok ? a.y - target[src] : 0.f;
        if (q == 0) loss += (double)wb * (double)diff * (double)diff;
        const float dy = 2.f * wb * diff * inv_b;
        if (q == 0) gb3 += dy;
        const float dyb = rbf(dy);
        // output and second layer deltas
        f32x4 d2[2];
        bf16x4 d2b[2];
        for (int m = 0; m < 2; ++m) {
            for (int i = 0; i < 4; ++i) {
                gw3[m][i] += dyb * rbf(a.h2[m][i]);
                d2[m][i] = w.w3[m][i] * dyb * (1.f - a.h2[m][i] * a.h2[m][i]);
                gb2[m][i] += d2[m][i];
            }
            d2b[m] = pack4(d2[m][0], d2[m][1], d2[m][2], d2[m][3]);
        }
        // first layer deltas: d1 = (W2^T d2) * (1 - h1^2)
        f32x4 d1[2];
        for (int ko = 0; ko < 2; ++ko) {
            const f32x4 z = mfma32(w.A2T[ko][0], w.A2T[ko][1], d2b[0], d2b[1], zero);
            for (int i = 0; i < 4; ++i) {
                d1[ko][i] = z[i] * (1.f - a.h1[ko][i] * a.h1[ko][i]);
                gb1[ko][i] += d1[ko][i];
            }
        }
        // bonds onto K through LDS: [bond][hidden] bf16
        for (int m = 0; m < 2; ++m)
            for (int i = 0; i < 4; ++i) {
                s_d2[wv][n][16 * m + 4 * q + i] = (uint16_t)d2b[m][i];
                s_h1[wv][n][16 * m + 4 * q + i] = f2bf(a.h1[m][i]);
                s_d1[wv][n][16 * m + 4 * q + i] = f2bf(d1[m][i]);
            }
        for (int i = 0; i < 4; ++i) s_x[wv][n][4 * q + i] = (uint16_t)xq[i];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        for (int mh = 0; mh < 2; ++mh) {
            bf16x4 ad2, ad1;
            for (int i = 0; i < 4; ++i) {
                ad2[i] = (short)s_d2[wv][4 * q + i][16 * mh + n];
                ad1[i] = (short)s_d1[wv][4 * q + i][16 * mh + n];
            }
            for (int nk = 0; nk < 2; ++nk) {
                bf16x4 bh;
                for (int i = 0; i < 4; ++i) bh[i] = (short)s_h1[wv][4 * q + i][16 * nk + n];
                gW2[mh][nk] = mfma16(ad2, bh, gW2[mh][nk]);
            }
            bf16x4 bx;
            for (int i = 0; i < 4; ++i) bx[i] = (short)s_x[wv][4 * q + i][n];
            gW1[mh] = mfma16(ad1, bx, gW1[mh]);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // sums over the 16 bonds of a lane group (lanes with equal q)
    for (int m = 0; m < 2; ++m)
        for (int i = 0; i < 4; ++i)
            for (int off = 1; off < 16; off <<= 1) {
                gb1[m][i] += __shfl_xor(gb1[m][i], off);
                gb2[m][i] += __shfl_xor(gb2[m][i], off);
                gw3[m][i] += __shfl_xor(gw3[m][i], off);
            }
    for (int off = 1; off < 64; off <<= 1) {
        gb3 += __shfl_xor(gb3, off);
        loss += __shfl_xor(loss, off);
    }
    float *G = gpart + wave * kNP;
    for (int m = 0; m < 2; ++m)
        for (int i = 0; i < 4; ++i) {
            const int h = 16 * m + 4 * q + i;
            G[kOffW1 + h * kNI + n] = gW1[m][i];
            G[kOffW2 + h * kNH + n] = gW2[m][0][i];
            G[kOffW2 + h * kNH + 16 + n] = gW2[m][1][i];
            if (n == 0) {
                G[kOffB1 + h] = gb1[m][i];
                G[kOffB2 + h] = gb2[m][i];
                G[kOffW3 + h] = gw3[m][i];
            }
        }
    if (l == 0) {
        G[kOffB3] = gb3;
        lpart[wave] = loss * (double)inv_b;
    }
}

// grad[p] = sum over the wavefront partials (FP64), loss likewise.  A block
// serves kRedParams parameters with kRedSplit threads each: thread k of a
// parameter sums waves k, k + kRedSplit, ... in order and the kRedSplit sums are
// added in order (a fixed order: deterministic).  With `adam` the block then
// applies the AdamW update of tbk_adamw_step to its parameters (the training
// loop's fused step; t-dependent factors c1, c2 precomputed on the host).
constexpr int kRedParams = 64, kRedSplit = 4;

struct AdamArgs {
    float *p, *m, *v;
    float lr, b1, b2, eps, wd, c1, c2;
};

template <bool ADAM>
__global__ __launch_bounds__(kRedParams * kRedSplit) void k_grad_reduce(int64_t nwave, const float *__restrict__ gpart,
                                                                       const double *__restrict__ lpart,
                                                                       float *__restrict__ grad,
                                                                       double *__restrict__ loss, AdamArgs ad) {
    __shared__ double red[kRedSplit][kRedParams];
    const int pl = threadIdx.x % kRedParams, k = threadIdx.x / kRedParams;
    const int p = blockIdx.x * kRedParams + pl;
    double s = 0.0;
    if (p < kNP)
        for (int64_t wv = k; wv < nwave; wv += kRedSplit) s += (double)gpart[wv * kNP + p];
    red[k][pl] = s;
    __syncthreads();
    if (k == 0 && p < kNP) {
        double g = red[0][pl];
        for (int j = 1; j < kRedSplit; ++j) g += red[j][pl];
        const float gf = (float)g;
        if (grad) grad[p] = gf;
        if constexpr (ADAM) {
            const float mi = ad.b1 * ad.m[p] + (1.f - ad.b1) * gf;
            const float vi = ad.b2 * ad.v[p] + (1.f - ad.b2) * gf * gf;
            ad.m[p] = mi;
            ad.v[p] = vi;
            const float mh = mi / ad.c1, vh = vi / ad.c2;
            ad.p[p] -= ad.lr * (mh / (sqrtf(vh) + ad.eps) + ad.wd * ad.p[p]);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        double l = 0.0;
        for (int64_t wv = 0; wv < nwave; ++wv) l += lpart[wv];
        *loss = l;
    }
}

// One AdamW step with decoupled weight decay (FP32 state).
__global__ void k_adamw(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1, float c2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
}

// ------------------------------------------------------------------------
// Fused learned assembly: bond tiles -> features -> MLP -> both H entries
// ------------------------------------------------------------------------

struct HopModel {
    double r0, beta;
    int32_t n_species;
    const double *t_pair;     // device [n_species^2]
};

template <class V>
__device__ __forceinline__ void set_entry(const int64_t *__restrict__ ptr, int32_t *__restrict__ col,
                                          V *__restrict__ val, int32_t log2_slice, int64_t row, int32_t c, double t) {
    const int64_t smask = ((int64_t)1 << log2_slice) - 1;
    const int64_t s = row >> log2_slice;
    const int64_t base = ptr[s] + (row & smask);
    const int w = (int)((ptr[s + 1] - ptr[s]) >> log2_slice);
    for (int k = 0; k < w; ++k)
        if (col[base + ((int64_t)k << log2_slice)] == c) { val[base + ((int64_t)k << log2_slice)] = (V)t; return; }
}

template <class V>
__global__ __launch_bounds__(64 * kWaves) void k_learned_values(
    int64_t nb, const int32_t *__restrict__ bi, const int32_t *__restrict__ bj, const double *__restrict__ br,
    const double *__restrict__ v, const int32_t *__restrict__ species, const int32_t *__restrict__ iperm,
    double rc_desc, FeatNorm fn, const float *__restrict__ P, HopModel hm, const int64_t *__restrict__ ptr,
    int32_t *__restrict__ col, V *__restrict__ val, int32_t log2_slice, float *__restrict__ y_out) {
    WaveWeights w;
    load_weights(P, w);
    const int l = threadIdx.x & 63, n = l & 15, q = l >> 4;
    const int64_t wave = blockIdx.x * (int64_t)kWaves + (threadIdx.x >> 6);
    const int64_t nwave = (int64_t)gridDim.x * kWaves;
    const int64_t ntile = (nb + 15) / 16;
    for (int64_t t = wave; t < ntile; t += nwave) {
        const int64_t b = 16 * t + n;
        const bool ok = b < nb;
        const int64_t bc = ok ? b : nb - 1;
        const int32_t i = bi[bc], j = bj[bc];
        const double r = br[bc];
        double x[kNI];
        bond_features(r, v + (int64_t)i * kNR, v + (int64_t)j * kNR, rc_desc, fn, x);
        bf16x4 xq = {0, 0, 0, 0};
        if (ok)
            for (int k = 0; k < 4; ++k) xq[k] = (short)d2bf(x[4 * q + k]);
        TileAct a;
        mlp_tile_forward(w, xq, a);
        if (ok && q == 0) {
            const double tp = hm.t_pair[species[i] * hm.n_species + species[j]] * exp(-hm.beta * (r / hm.r0 - 1.0));
            const double tl = tp * (1.0 + (double)a.y);
            const int64_t ri = iperm[i], rj = iperm[j];
            set_entry<V>(ptr, col, val, log2_slice, ri, (int32_t)rj, tl);
            set_entry<V>(ptr, col, val, log2_slice, rj, (int32_t)ri, tl);
            if (y_out) y_out[b] = a.y;
        }
    }
}

// Row Gershgorin bounds from the stored values, per segment.
template <class V>
__global__ void k_row_bounds(int64_t n, const int64_t *__restrict__ ptr, const V *__restrict__ val,
                             const V *__restrict__ onsite, const int32_t *__restrict__ perm,
                             const int32_t *__restrict__ seg_of, int32_t log2_slice, int64_t *__restrict__ keys) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    int32_t sg = -1;
    if (r < n) {
        const int64_t smask = ((int64_t)1 << log2_slice) - 1;
        const int64_t s = r >> log2_slice;
        const int64_t base = ptr[s] + (r & smask);
        const int w = (int)((ptr[s + 1] - ptr[s]) >> log2_slice);
        double asum = 0.0;
        for (int k = 0; k < w; ++k) asum += fabs((double)val[base + ((int64_t)k << log2_slice)]);
        const double e = (double)onsite[r];
        lo = e - asum;
        hi = e + asum;
        sg = seg_of[perm[r]];
    }
    block_segment_bounds(lo, hi, sg, keys);
}

int mlp_grid(int64_t nb) {
    const int64_t tiles = (nb + 15) / 16;
    // about 2 tiles per wavefront: a minibatch of 2048 bonds spreads over 16 workgroups
    // (its tiles' latency chains run side by side; the per-wave partials stay small)
    const int64_t want = (tiles + kWaves * 2 - 1) / (kWaves * 2);
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, 1024));
}

tbk_status check_model(const tbk_mlp_model *mdl) {
    TBK_CHECK(mdl != nullptr && mdl->params && mdl->shift && mdl->scale, TBK_ERR_INVALID_ARG, "model is NULL");
    TBK_CHECK(mdl->c_nk == nullptr, TBK_ERR_UNSUPPORTED,
              "descriptor coefficients per species pair are taken by the Slater-Koster builder only");
    TBK_CHECK(mdl->n_radial == kNR, TBK_ERR_UNSUPPORTED, "the bond MLP takes %d radial functions", kNR);
    TBK_CHECK(std::isfinite(mdl->r_cut) && mdl->r_cut > 0, TBK_ERR_INVALID_ARG, "descriptor cutoff must be positive");
    for (int k = 0; k < kNI; ++k) {
        TBK_CHECK(std::isfinite(mdl->shift[k]) && std::isfinite(mdl->scale[k]), TBK_ERR_NOT_FINITE,
                  "feature normalisation %d is not finite", k);
        TBK_CHECK(mdl->scale[k] != 0.0, TBK_ERR_INVALID_ARG, "feature scale %d is zero", k);
    }
    return TBK_OK;
}

FeatNorm make_norm(const double *shift, const double *scale) {
    FeatNorm fn{};
    for (int k = 0; k < kNI; ++k) { fn.shift[k] = shift[k]; fn.inv_scale[k] = 1.0 / scale[k]; }
    return fn;
}

}  // namespace

// Descriptor of every atom: cell list at the descriptor cutoff, then sums.
static tbk_status descriptor_impl(const double *pos, int64_t n, int32_t nseg, const int64_t *seg_atoms,
                                  const double *boxes, const int32_t periodic[3], double rc, int32_t nk, double *v,
                                  hipStream_t s, const int32_t *species = nullptr, int32_t ns = 1,
                                  const double *cnk_dev = nullptr) {
    TBK_CHECK(nk >= 1 && nk <= 16, TBK_ERR_INVALID_ARG, "n_radial = %d outside [1, 16]", nk);
    TBK_CHECK(std::isfinite(rc) && rc > 0, TBK_ERR_INVALID_ARG, "descriptor cutoff must be positive");
    TBK_CHECK(v != nullptr, TBK_ERR_INVALID_ARG, "v is NULL");
    CellListOwner cells;
    // with coefficients per species pair the cell list also validates the species indices
    tbk_status st = cells.build(pos, cnk_dev ? species : nullptr, cnk_dev ? ns : 1, n, nseg, seg_atoms, boxes,
                                periodic, rc, s);
    if (st != TBK_OK) return st;
    if (nk == 8)
        k_descriptor_nk<8><<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(cells.view, pos, n, rc, species, ns, cnk_dev,
                                                                      v);
    else
        k_descriptor<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(cells.view, pos, n, rc, nk, species, ns, cnk_dev, v);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

// Unique bonds (i < j) within rc, ordered by (i, j); bonds written only when
// cap suffices; returns the count in *nb.
// Bonds i < j within rc over a built cell list: per-atom counts, their offsets,
// then (bi, bj, br) ordered by (i, j).  *nb = the number of bonds; they are
// written only when *nb <= cap.
static tbk_status bonds_on_cells(const CellList &cl, const double *pos, int64_t n, double rc, int64_t cap,
                                 int32_t *bi, int32_t *bj, double *br, int64_t *nb, hipStream_t s) {
    DevBuf cnt, off, tmp;
    TBK_HIP(cnt.alloc(sizeof(int64_t) * (n + 1), s));
    TBK_HIP(off.alloc(sizeof(int64_t) * (n + 1), s));
    TBK_HIP(hipMemsetAsync(cnt.as<int64_t>() + n, 0, sizeof(int64_t), s));
    const unsigned g = (unsigned)ceil_div(n, 256);
    k_bond_count<<<g, 256, 0, s>>>(cl, pos, n, rc, cnt.as<int64_t>());
    TBK_HIP(hipGetLastError());
    size_t tb = 0;
    TBK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt.as<int64_t>(), off.as<int64_t>(), (int)(n + 1), s));
    TBK_HIP(tmp.alloc(tb, s));
    TBK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.as<void>(), tb, cnt.as<int64_t>(), off.as<int64_t>(), (int)(n + 1), s));
    int64_t total = 0;
    TBK_HIP(hipMemcpyAsync(&total, off.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    *nb = total;
    if (total > cap) return TBK_OK;
    TBK_CHECK(total == 0 || (bi && bj && br), TBK_ERR_INVALID_ARG, "bond arrays are NULL");
    if (total > 0) {
        k_bond_fill<<<g, 256, 0, s>>>(cl, pos, n, rc, off.as<int64_t>(), bi, bj, br);
        TBK_HIP(hipGetLastError());
    }
    return TBK_OK;
}

static tbk_status bonds_impl(const double *pos, int64_t n, int32_t nseg, const int64_t *seg_atoms, const double *boxes,
                             const int32_t periodic[3], double rc, int64_t cap, int32_t *bi, int32_t *bj, double *br,
                             int64_t *nb, hipStream_t s) {
    CellListOwner cells;
    tbk_status st = cells.build(pos, nullptr, 1, n, nseg, seg_atoms, boxes, periodic, rc, s);
    if (st != TBK_OK) return st;
    st = bonds_on_cells(cells.view, pos, n, rc, cap, bi, bj, br, nb, s);
    if (st != TBK_OK) return st;
    TBK_HIP(hipStreamSynchronize(s));
    return TBK_OK;
}

}  // namespace tbk

using namespace tbk;

extern "C" tbk_status tbk_node_features(int64_t n, const double *v, int32_t n_radial, const double *shift,
                                        const double *scale, uint16_t *X, void *stream) {
    clear_error();
    TBK_CHECK(n_radial == kNR, TBK_ERR_UNSUPPORTED, "features need %d radial functions", kNR);
    TBK_CHECK(n >= 0 && shift && scale, TBK_ERR_INVALID_ARG, "bad arguments");
    FeatNorm fn{};
    for (int k = 0; k < kNR; ++k) {
        TBK_CHECK(scale[k] != 0.0 && std::isfinite(scale[k]) && std::isfinite(shift[k]), TBK_ERR_INVALID_ARG,
                  "node feature %d: shift/scale invalid", k);
        fn.shift[k] = shift[k];
        fn.inv_scale[k] = scale[k];        // this kernel divides by the scale itself
    }
    if (n == 0) return TBK_OK;
    TBK_CHECK(v && X, TBK_ERR_INVALID_ARG, "NULL array");
    hipStream_t s = as_stream(stream);
    k_node_features<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, v, fn, X);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status tbk_descriptor(const double *pos, int32_t n_seg, const int64_t *seg_atoms, const double *boxes,
                                     const int32_t periodic[3], double r_cut, int32_t n_radial, double *v,
                                     void *stream) {
    clear_error();
    TBK_CHECK(seg_atoms && n_seg >= 1, TBK_ERR_INVALID_ARG, "bad segment table");
    return descriptor_impl(pos, seg_atoms[n_seg], n_seg, seg_atoms, boxes, periodic, r_cut, n_radial, v,
                           as_stream(stream));
}

extern "C" tbk_status tbk_bonds(const double *pos, int32_t n_seg, const int64_t *seg_atoms, const double *boxes,
                                const int32_t periodic[3], double r_cut, int64_t cap, int32_t *bi, int32_t *bj,
                                double *br, int64_t *n_bonds, void *stream) {
    clear_error();
    TBK_CHECK(seg_atoms && n_seg >= 1 && n_bonds, TBK_ERR_INVALID_ARG, "bad arguments");
    TBK_CHECK(std::isfinite(r_cut) && r_cut > 0, TBK_ERR_INVALID_ARG, "r_cut must be positive");
    tbk_status st = bonds_impl(pos, seg_atoms[n_seg], n_seg, seg_atoms, boxes, periodic, r_cut, cap, bi, bj, br,
                               n_bonds, as_stream(stream));
    if (st != TBK_OK) return st;
    TBK_CHECK(*n_bonds <= cap, TBK_ERR_BUFFER_TOO_SMALL, "%lld bonds, capacity %lld", (long long)*n_bonds,
              (long long)cap);
    return TBK_OK;
}

extern "C" tbk_status tbk_bond_features(int64_t nb, const int32_t *bi, const int32_t *bj, const double *br,
                                        const double *v, int32_t n_radial, double r_cut, const double *shift,
                                        const double *scale, uint16_t *X, void *stream) {
    clear_error();
    TBK_CHECK(n_radial == kNR, TBK_ERR_UNSUPPORTED, "features need %d radial functions", kNR);
    TBK_CHECK(nb >= 0 && shift && scale, TBK_ERR_INVALID_ARG, "bad arguments");
    for (int k = 0; k < kNI; ++k) TBK_CHECK(scale[k] != 0.0 && std::isfinite(scale[k]) && std::isfinite(shift[k]),
                                             TBK_ERR_INVALID_ARG, "bad feature normalisation %d", k);
    if (nb == 0) return TBK_OK;
    TBK_CHECK(bi && bj && br && v && X, TBK_ERR_INVALID_ARG, "NULL array");
    hipStream_t s = as_stream(stream);
    k_bond_features<<<(unsigned)ceil_div(nb, 256), 256, 0, s>>>(nb, bi, bj, br, v, r_cut, make_norm(shift, scale),
                                                                 nullptr, 1, nullptr, X);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

namespace tbk {
namespace {

// Coefficients per species pair: host [ns][ns][nk][nk], finite, symmetric in the pair.
tbk_status check_cnk(int32_t ns, int32_t nk, const double *cnk) {
    TBK_CHECK(ns >= 1 && ns <= 16, TBK_ERR_INVALID_ARG, "n_species = %d outside [1, 16]", ns);
    TBK_CHECK(cnk != nullptr, TBK_ERR_INVALID_ARG, "c_nk is NULL");
    const int64_t blk = (int64_t)nk * nk;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int64_t q = 0; q < blk; ++q) {
                const double x = cnk[(a * ns + b) * blk + q];
                TBK_CHECK(std::isfinite(x), TBK_ERR_NOT_FINITE, "c_nk[%d][%d] is not finite", a, b);
                TBK_CHECK(x == cnk[(b * ns + a) * blk + q], TBK_ERR_INVALID_ARG,
                          "c_nk[%d][%d] differs from c_nk[%d][%d] (must be symmetric in the pair)", a, b, b, a);
            }
    return TBK_OK;
}

}  // namespace
}  // namespace tbk

extern "C" tbk_status tbk_descriptor_species(const double *pos, const int32_t *species, int32_t n_seg,
                                             const int64_t *seg_atoms, const double *boxes,
                                             const int32_t periodic[3], double r_cut, int32_t n_radial,
                                             int32_t n_species, const double *c_nk, double *v, void *stream) {
    clear_error();
    TBK_CHECK(seg_atoms && n_seg >= 1 && species, TBK_ERR_INVALID_ARG, "bad segment table or species");
    TBK_CHECK(n_radial >= 1 && n_radial <= 16, TBK_ERR_INVALID_ARG, "n_radial = %d outside [1, 16]", n_radial);
    tbk_status st = check_cnk(n_species, n_radial, c_nk);
    if (st != TBK_OK) return st;
    hipStream_t s = as_stream(stream);
    const size_t bytes = sizeof(double) * n_species * n_species * n_radial * n_radial;
    DevBuf c;
    TBK_HIP(c.alloc(bytes, s));
    TBK_HIP(hipMemcpyAsync(c.as<double>(), c_nk, bytes, hipMemcpyHostToDevice, s));
    st = descriptor_impl(pos, seg_atoms[n_seg], n_seg, seg_atoms, boxes, periodic, r_cut, n_radial, v, s, species,
                         n_species, c.as<double>());
    if (st != TBK_OK) return st;
    TBK_HIP(hipStreamSynchronize(s));      // the caller's c_nk must outlive the transfer
    return TBK_OK;
}

extern "C" tbk_status tbk_bond_features_species(int64_t nb, const int32_t *bi, const int32_t *bj, const double *br,
                                                const int32_t *species, const double *v, int32_t n_radial,
                                                double r_cut, int32_t n_species, const double *c_nk,
                                                const double *shift, const double *scale, uint16_t *X,
                                                void *stream) {
    clear_error();
    TBK_CHECK(n_radial == kNR, TBK_ERR_UNSUPPORTED, "features need %d radial functions", kNR);
    TBK_CHECK(nb >= 0 && shift && scale && species, TBK_ERR_INVALID_ARG, "bad arguments");
    for (int k = 0; k < kNI; ++k) TBK_CHECK(scale[k] != 0.0 && std::isfinite(scale[k]) && std::isfinite(shift[k]),
                                             TBK_ERR_INVALID_ARG, "bad feature normalisation %d", k);
    tbk_status st = check_cnk(n_species, kNR, c_nk);
    if (st != TBK_OK) return st;
    if (nb == 0) return TBK_OK;
    TBK_CHECK(bi && bj && br && v && X, TBK_ERR_INVALID_ARG, "NULL array");
    hipStream_t s = as_stream(stream);
    const size_t bytes = sizeof(double) * n_species * n_species * kNR * kNR;
    DevBuf c;
    TBK_HIP(c.alloc(bytes, s));
    TBK_HIP(hipMemcpyAsync(c.as<double>(), c_nk, bytes, hipMemcpyHostToDevice, s));
    k_bond_features<<<(unsigned)ceil_div(nb, 256), 256, 0, s>>>(nb, bi, bj, br, v, r_cut, make_norm(shift, scale),
                                                                 species, n_species, c.as<double>(), X);
    TBK_HIP(hipGetLastError());
    TBK_HIP(hipStreamSynchronize(s));      // the caller's c_nk must outlive the transfer
    return TBK_OK;
}

extern "C" tbk_status tbk_feature_moments(int64_t nb, const int32_t *bi, const int32_t *bj, const double *br,
                                          const double *v, int32_t n_radial, double r_cut, double *mean,
                                          double *stddev, void *stream) {
    clear_error();
    TBK_CHECK(n_radial == kNR, TBK_ERR_UNSUPPORTED, "features need %d radial functions", kNR);
    TBK_CHECK(nb >= 1 && bi && bj && br && v && mean && stddev, TBK_ERR_INVALID_ARG, "bad arguments");
    hipStream_t s = as_stream(stream);
    const int G = (int)std::min<int64_t>(256, ceil_div(nb, 256));
    DevBuf part;
    TBK_HIP(part.alloc(sizeof(double) * G * 2 * kNI, s));
    k_feature_moments<<<G, 256, 0, s>>>(nb, bi, bj, br, v, r_cut, part.as<double>());
    TBK_HIP(hipGetLastError());
    std::vector<double> hp((size_t)G * 2 * kNI);
    TBK_HIP(hipMemcpyAsync(hp.data(), part.as<double>(), sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < kNI; ++k) {
        double a = 0.0, b2 = 0.0;
        for (int g = 0; g < G; ++g) { a += hp[(size_t)g * 2 * kNI + k]; b2 += hp[(size_t)g * 2 * kNI + kNI + k]; }
        const double mu = a / (double)nb;
        mean[k] = mu;
        stddev[k] = std::sqrt(std::max(b2 / (double)nb - mu * mu, 0.0));
    }
    return TBK_OK;
}

extern "C" tbk_status tbk_coordination_target(int64_t nb, const int32_t *bi, const int32_t *bj, const double *v,
                                              int32_t n_radial, double kappa, double z0, float *y, void *stream) {
    clear_error();
    TBK_CHECK(nb >= 0 && n_radial >= 1, TBK_ERR_INVALID_ARG, "bad arguments");
    if (nb == 0) return TBK_OK;
    TBK_CHECK(bi && bj && v && y, TBK_ERR_INVALID_ARG, "NULL array");
    hipStream_t s = as_stream(stream);
    k_coord_target<<<(unsigned)ceil_div(nb, 256), 256, 0, s>>>(nb, bi, bj, v, n_radial, kappa, z0, y);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status tbk_mlp_forward(int64_t nb, const uint16_t *X, const float *params, float *y, void *stream) {
    clear_error();
    TBK_CHECK(nb >= 0, TBK_ERR_INVALID_ARG, "nb < 0");
    if (nb == 0) return TBK_OK;
    TBK_CHECK(X && params && y, TBK_ERR_INVALID_ARG, "NULL array");
    hipStream_t s = as_stream(stream);
    k_mlp_forward<<<mlp_grid(nb), 64 * kWaves, 0, s>>>(nb, X, params, y);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status tbk_mlp_workspace_size(int64_t nb, int64_t *bytes) {
    clear_error();
    TBK_CHECK(nb >= 1 && bytes, TBK_ERR_INVALID_ARG, "bad arguments");
    const int64_t nwave = (int64_t)mlp_grid(nb) * kWaves;
    *bytes = ((nwave * kNP * 4 + 255) / 256) * 256 + ((nwave * 8 + 255) / 256) * 256;
    return TBK_OK;
}

static tbk_status loss_grad_impl(int64_t nb, const uint16_t *X, const float *target, const float *weight,
                                 const float *params, float *grad, double *loss, void *work, int64_t work_bytes,
                                 hipStream_t s, BondOrder order, const AdamArgs *adam = nullptr) {
    int64_t need = 0;
    tbk_status st = tbk_mlp_workspace_size(nb, &need);
    if (st != TBK_OK) return st;
    TBK_CHECK(work_bytes >= need, TBK_ERR_BUFFER_TOO_SMALL, "work has %lld bytes, needs %lld", (long long)work_bytes,
              (long long)need);
    TBK_CHECK(X && target && params && grad && work, TBK_ERR_INVALID_ARG, "NULL array");
    const int G = mlp_grid(nb);
    const int64_t nwave = (int64_t)G * kWaves;
    float *gpart = static_cast<float *>(work);
    double *lpart = reinterpret_cast<double *>(static_cast<char *>(work) + ((nwave * kNP * 4 + 255) / 256) * 256);
    k_mlp_grad<<<G, 64 * kWaves, 0, s>>>(nb, X, target, weight, params, 1.0f / (float)nb, order, gpart, lpart);
    TBK_HIP(hipGetLastError());
    const unsigned rb = (kNP + kRedParams - 1) / kRedParams;
    if (adam)
        k_grad_reduce<true><<<rb, kRedParams * kRedSplit, 0, s>>>(nwave, gpart, lpart, grad, loss, *adam);
    else
        k_grad_reduce<false><<<rb, kRedParams * kRedSplit, 0, s>>>(nwave, gpart, lpart, grad, loss, AdamArgs{});
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status tbk_mlp_loss_grad(int64_t nb, const uint16_t *X, const float *target, const float *weight,
                                        const float *params, float *grad, double *loss, void *work,
                                        int64_t work_bytes, void *stream) {
    clear_error();
    TBK_CHECK(nb >= 1, TBK_ERR_INVALID_ARG, "nb must be positive");
    return loss_grad_impl(nb, X, target, weight, params, grad, loss, work, work_bytes, as_stream(stream),
                          BondOrder{nb, 0, 1, 0});
}

extern "C" tbk_status tbk_adamw_step(int64_t n, float *p, const float *g, float *m, float *v, int64_t t, double lr,
                                     double beta1, double beta2, double eps, double wd, void *stream) {
    clear_error();
    TBK_CHECK(n >= 0 && t >= 1, TBK_ERR_INVALID_ARG, "bad n or step count");
    TBK_CHECK(lr >= 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && wd >= 0,
              TBK_ERR_INVALID_ARG, "bad AdamW hyper-parameters");
    if (n == 0) return TBK_OK;
    TBK_CHECK(p && g && m && v, TBK_ERR_INVALID_ARG, "NULL array");
    const double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
    hipStream_t s = as_stream(stream);
    k_adamw<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(n, p, g, m, v, (float)lr, (float)beta1, (float)beta2,
                                                      (float)eps, (float)wd, (float)c1, (float)c2);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

// SplitMix64 output k of `seed` (Steele, Lea & Flood 2014): the epoch's shuffle.
static uint64_t mix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) { const uint64_t t = a % b; a = b; b = t; }
    return a;
}

// Bond order of one epoch: in order without a seed; otherwise the 16-bond chunks
// go through an affine bijection c -> (mul c + add) mod n_chunks with mul coprime
// to n_chunks taken from the middle half of [1, n_chunks), so consecutive chunks of
// a minibatch land far apart in the stored (structure-major) order.
static BondOrder epoch_order(int64_t nb, uint64_t seed, int e) {
    const uint64_t n = (uint64_t)(nb >> 4);
    if (seed == 0 || n < 3) return BondOrder{nb, 0, 1, 0};
    uint64_t mul = n / 4 + mix64(seed, 2 * (uint64_t)e) % (n / 2 + 1);
    while (mul <= 1 || gcd64(mul, n) != 1) mul = mul + 1 < n ? mul + 1 : 2;
    return BondOrder{nb, 0, (int64_t)mul, (int64_t)(mix64(seed, 2 * (uint64_t)e + 1) % n)};
}

extern "C" tbk_status tbk_mlp_train(int64_t nb, const uint16_t *X, const float *target, const float *weight,
                                    float *params, float *m, float *v, int64_t *step, int32_t epochs, int64_t batch,
                                    uint64_t shuffle_seed, double lr, double beta1, double beta2, double eps,
                                    double wd, double *loss_history, void *work, int64_t work_bytes,
                                    void *stream) {
    clear_error();
    TBK_CHECK(nb >= 1 && epochs >= 1 && batch >= 1 && step && loss_history, TBK_ERR_INVALID_ARG, "bad arguments");
    TBK_CHECK(params && m && v, TBK_ERR_INVALID_ARG, "NULL array");
    TBK_CHECK(*step >= 0, TBK_ERR_INVALID_ARG, "step count %lld < 0", (long long)*step);
    TBK_CHECK(lr >= 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && wd >= 0,
              TBK_ERR_INVALID_ARG, "bad AdamW hyper-parameters");
    hipStream_t s = as_stream(stream);
    const int64_t bsz = std::min(batch, nb);
    int64_t need = 0;
    tbk_status st = tbk_mlp_workspace_size(bsz, &need);
    if (st != TBK_OK) return st;
    const int64_t extra = 256 + ((int64_t)kNP * 4 + 255) / 256 * 256;
    TBK_CHECK(work_bytes >= need + extra, TBK_ERR_BUFFER_TOO_SMALL, "work has %lld bytes, needs %lld",
              (long long)work_bytes, (long long)(need + extra));
    char *w = static_cast<char *>(work);
    double *dloss = reinterpret_cast<double *>(w);
    float *grad = reinterpret_cast<float *>(w + 256);
    void *gw = w + extra;
    const int64_t nbatch = (nb + bsz - 1) / bsz;
    std::vector<double> hl(nbatch);
    DevBuf losses;
    TBK_HIP(losses.alloc(sizeof(double) * nbatch, s));
    for (int e = 0; e < epochs; ++e) {
        BondOrder order = epoch_order(nb, shuffle_seed, e);
        for (int64_t bt = 0; bt < nbatch; ++bt) {
            const int64_t b0 = bt * bsz, cnt = std::min(bsz, nb - b0);
            order.first = b0;
            *step += 1;
            // the AdamW update of tbk_adamw_step, fused into the gradient reduction
            const AdamArgs ad{params, m, v, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)wd,
                              (float)(1.0 - std::pow(beta1, (double)*step)),
                              (float)(1.0 - std::pow(beta2, (double)*step))};
            st = loss_grad_impl(cnt, X, target, weight, params, grad, losses.as<double>() + bt, gw,
                                work_bytes - extra, s, order, &ad);
            if (st != TBK_OK) return st;
        }
        TBK_HIP(hipMemcpyAsync(hl.data(), losses.as<double>(), sizeof(double) * nbatch, hipMemcpyDeviceToHost, s));
        TBK_HIP(hipStreamSynchronize(s));
        double sum = 0.0, cntw = 0.0;
        for (int64_t bt = 0; bt < nbatch; ++bt) {
            const double c = (double)std::min(bsz, nb - bt * bsz);
            sum += hl[bt] * c;
            cntw += c;
        }
        loss_history[e] = sum / cntw;
    }
    (void)dloss;
    return TBK_OK;
}

extern "C" tbk_status tb_build_hamiltonian_learned(const double *pos, const int32_t *species, int32_t n_seg,
                                                   const int64_t *seg_atoms, const double *boxes,
                                                   const int32_t periodic[3], const tbk_tb_params *p,
                                                   const tbk_mlp_model *model, tbk_ham *h, double *spec_bounds,
                                                   float *bond_y, int64_t bond_cap, int64_t *n_bonds,
                                                   void *stream) {
    clear_error();
    TBK_CHECK(seg_atoms && n_seg >= 1, TBK_ERR_INVALID_ARG, "bad segment table");
    TBK_CHECK(h != nullptr && spec_bounds != nullptr, TBK_ERR_INVALID_ARG, "h or bounds is NULL");
    TBK_CHECK(h->fmt == TBK_SELL_F32 || h->fmt == TBK_SELL_F64, TBK_ERR_INVALID_ARG, "learned assembly needs SELL");
    tbk_status st = check_model(model);
    if (st != TBK_OK) return st;
    TBK_CHECK(p != nullptr && p->n_species <= 16, TBK_ERR_INVALID_ARG, "bad hopping model");
    hipStream_t s = as_stream(stream);
    const int64_t n = seg_atoms[n_seg];
    // 1. pattern and plain values (also validates all structure inputs)
    HamPlan plan;
    st = plan.run(pos, species, n, n_seg, seg_atoms, boxes, periodic, p, h->fmt, h->slice, s);
    if (st != TBK_OK) return st;
    std::vector<double> tmpb(2 * (size_t)n_seg);
    st = plan.fill(pos, species, n, p, h, tmpb.data(), s);
    if (st != TBK_OK) return st;
    // 2. descriptors and the hop bonds
    DevBuf v, bi, bj, br;
    TBK_HIP(v.alloc(sizeof(double) * n * kNR, s));
    st = descriptor_impl(pos, n, n_seg, seg_atoms, boxes, periodic, model->r_cut, kNR, v.as<double>(), s);
    if (st != TBK_OK) return st;
    const int64_t nb = plan.n_bonds;
    TBK_HIP(bi.alloc(sizeof(int32_t) * std::max<int64_t>(nb, 1), s));
    TBK_HIP(bj.alloc(sizeof(int32_t) * std::max<int64_t>(nb, 1), s));
    TBK_HIP(br.alloc(sizeof(double) * std::max<int64_t>(nb, 1), s));
    int64_t nb2 = 0;
    // the hop bonds over the Hamiltonian's own cell list (same cutoff)
    st = bonds_on_cells(plan.cells.view, pos, n, p->r_cut, nb, bi.as<int32_t>(), bj.as<int32_t>(), br.as<double>(),
                        &nb2, s);
    if (st != TBK_OK) return st;
    TBK_CHECK(nb2 == nb, TBK_ERR_DEVICE, "bond count mismatch (%lld vs %lld)", (long long)nb2, (long long)nb);
    if (n_bonds) *n_bonds = nb;
    TBK_CHECK(bond_y == nullptr || bond_cap >= nb, TBK_ERR_BUFFER_TOO_SMALL, "bond_y holds %lld, needs %lld",
              (long long)bond_cap, (long long)nb);
    // 3. fused features -> MLP -> both entries of each bond
    HopModel hm{};
    hm.r0 = p->r0;
    hm.beta = p->beta;
    hm.n_species = p->n_species;
    DevBuf tp;
    TBK_HIP(tp.alloc(sizeof(double) * p->n_species * p->n_species, s));
    TBK_HIP(hipMemcpyAsync(tp.as<double>(), p->t_pair, sizeof(double) * p->n_species * p->n_species,
                           hipMemcpyHostToDevice, s));
    hm.t_pair = tp.as<double>();
    const FeatNorm fn = make_norm(model->shift, model->scale);
    int l2 = 0;
    while ((1 << l2) < plan.slice) ++l2;
    if (nb > 0) {
        if (h->fmt == TBK_SELL_F32)
            k_learned_values<float><<<mlp_grid(nb), 64 * kWaves, 0, s>>>(
                nb, bi.as<int32_t>(), bj.as<int32_t>(), br.as<double>(), v.as<double>(), species,
                plan.iperm.as<int32_t>(), model->r_cut, fn, model->params, hm, h->ptr, h->col,
                static_cast<float *>(h->val), l2, bond_y);
        else
            k_learned_values<double><<<mlp_grid(nb), 64 * kWaves, 0, s>>>(
                nb, bi.as<int32_t>(), bj.as<int32_t>(), br.as<double>(), v.as<double>(), species,
                plan.iperm.as<int32_t>(), model->r_cut, fn, model->params, hm, h->ptr, h->col,
                static_cast<double *>(h->val), l2, bond_y);
        TBK_HIP(hipGetLastError());
    }
    // 4. bounds of the learned H
    DevBuf keys;
    st = init_bound_keys(keys, n_seg, s);
    if (st != TBK_OK) return st;
    const unsigned gr = (unsigned)ceil_div(n, kBlock);
    if (h->fmt == TBK_SELL_F32)
        k_row_bounds<float><<<gr, kBlock, 0, s>>>(n, h->ptr, static_cast<const float *>(h->val),
                                                  static_cast<const float *>(h->onsite), h->perm,
                                                  plan.cells.view.seg_of, l2, keys.as<int64_t>());
    else
        k_row_bounds<double><<<gr, kBlock, 0, s>>>(n, h->ptr, static_cast<const double *>(h->val),
                                                   static_cast<const double *>(h->onsite), h->perm,
                                                   plan.cells.view.seg_of, l2, keys.as<int64_t>());
    TBK_HIP(hipGetLastError());
    plan.vkeys.release();    // the plain values' range no longer describes the learned ones
    return plan.finish(keys, n, p, h, spec_bounds, s);
}
