// Device-side building blocks shared by the kernels: the counter-based
// Gaussian generator for Omega and thin wrappers over the gfx950 matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rh {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup for every streaming kernel
// LDS per workgroup on gfx950 and the room kept for a kernel's static
// __shared__ arrays on top of a dynamic request (checked on the host).
constexpr size_t kLdsLimit = 160 * 1024;
constexpr size_t kStaticLdsMargin = 12 * 1024;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of
// (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key bumped by the Weyl increments after each round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform in (0,1): ((x >> 9) + 0.5) * 2^-23 = (2m+1) 2^-24, exact in binary32.
__device__ __forceinline__ float uniform01f(uint32_t x) {
    return (static_cast<float>(x >> 9) + 0.5f) * 0x1p-23f;
}

// Box-Muller on two uniforms: (r cos 2 pi u1, r sin 2 pi u1), r = sqrt(-2 ln u0).
// The FP32 form uses the hardware sine/cosine, whose argument is in
// revolutions, so 2 pi u1 is never rounded.
__device__ __forceinline__ void box_muller(float u0, float u1, float& z0, float& z1) {
    const float r = sqrtf(-2.0f * logf(u0));
    z0 = r * __builtin_amdgcn_cosf(u1);
    z1 = r * __builtin_amdgcn_sinf(u1);
}
__device__ __forceinline__ void box_muller(double u0, double u1, double& z0, double& z1) {
    const double r = sqrt(-2.0 * log(u0));
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// The four normals of quad q: Omega at linear indices e = 4q .. 4q+3 of the
// (seed, mode, tag) stream.  T selects the precision of the Box-Muller
// transform (the uniforms are identical in both).
template <typename T>
__device__ __forceinline__ void normals4(uint64_t q, uint32_t mode, uint32_t tag, uint64_t seed,
                                         T z[4]) {
    uint32_t c0 = static_cast<uint32_t>(q), c1 = static_cast<uint32_t>(q >> 32);
    uint32_t c2 = mode, c3 = tag;
    philox4x32_10(c0, c1, c2, c3, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    box_muller(static_cast<T>(uniform01f(c0)), static_cast<T>(uniform01f(c1)), z[0], z[1]);
    box_muller(static_cast<T>(uniform01f(c2)), static_cast<T>(uniform01f(c3)), z[2], z[3]);
}

// Omega entry for column j of the unfolding of an (L, I, T) view and sketch
// column k.  The generator row is the cyclic position c = t + T l of
// j = l + L t (the modes after n come first), so for L = 1 it is j itself.
template <typename V>
__device__ __forceinline__ V omega_entry(uint64_t seed, uint32_t mode, uint32_t tag, int64_t j,
                                         int k, int64_t L, int64_t T, int64_t J) {
    const int64_t t = j / L, l = j - t * L;
    const uint64_t e = static_cast<uint64_t>(k) * static_cast<uint64_t>(J) +
                       static_cast<uint64_t>(t + T * l);
    V z[4];
    normals4<V>(e >> 2, mode, tag, seed, z);
    return z[e & 3];
}

// ---------------------------------------------------------------------------
// 16x16x4 matrix-core step, D = A B + C, for float and double.
// Operand layout (one wave): lane = m + 16 k holds A[m][k] and B[k][m].
// Accumulator element r of lane l is D[row(l / 16, r)][l % 16] with
// row = 4 (l / 16) + r for the f32 instruction and row = 4 r + l / 16 for
// the f64 one (measured lane layouts of v_mfma_f32_16x16x4_f32 and
// v_mfma_f64_16x16x4_f64 on gfx950).
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
template <>
struct Mma<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int quad, int r) { return 4 * quad + r; }
};
template <>
struct Mma<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int quad, int r) { return 4 * r + quad; }
};

template <typename V>
__device__ __forceinline__ V zero4() {
    V v;
    v[0] = 0; v[1] = 0; v[2] = 0; v[3] = 0;
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

}  // namespace rh
