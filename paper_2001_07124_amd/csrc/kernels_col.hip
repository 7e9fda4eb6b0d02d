// Streaming passes over a contiguous unfolding (L = 1) of an FP32 tensor on
// the gfx950 bf16 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// S = S_(n) is I x J with column j at src + j I.  A wave owns blocks of 32
// consecutive columns and keeps a whole block (I <= 32 NCH rows) in
// registers.  Lane (c = l % 16, g = l / 16) loads, for column half h2 and
// 32-row chunk h, rows 32 h + 8 g .. 32 h + 8 g + 7 of column 16 h2 + c with
// two 16-byte buffer loads.  Rows past I belong to the next column (or, past
// the end of the tensor, read as zero through the buffer's range check); they
// only meet zero rows of M or land in rows of Y that are dropped, and the
// sum of squares masks them.
//
// Rounded to bf16, the loaded registers are the A operand of Z = S^T M
// (m = column, k = row) as they stand.  Y += S W needs A = S (m = row,
// k = column): each wave writes its block column-major into LDS and reads it
// back with ds_read_b64_tr_b16, which hands lane (i, g) the columns
// 4g .. 4g+3 of a 16-column half for row i.  The two halves form the k
// operand in the order {4g .. 4g+3, 16+4g .. 16+4g+3}; the B operand W
// (Omega in the sketch, Z in the power step) is built in the same order,
// which is how Z's accumulators already sit in the lanes.
//
// Precision: in the sketch the tensor and Omega are rounded to bf16.  M (Q
// or the factor) and Z are always split into hi + lo bf16, because rounding
// the small operand would bias the captured energy ||M^T S||^2 at first
// order.  With SPLIT (CT_BF16X3) the tensor is split as well in Z = S^T M
// (hi*lo + lo*hi + hi*hi, about 16 bits); without it (CT_BF16X2) it is
// rounded, which on the 200^4 workload moves the relative error by a few
// 1e-4.  The power step's Y += S Z takes the rounded tensor against split Z.
// The Gram Z^T Z takes hi*hi + hi*lo + lo*hi.  Accumulation is FP32.
//
// FP8 sketch (VAR in the sketch): the block and Omega enter the
// v_mfma_f32_16x16x32_fp8_fp8 matrix cores as OCP e4m3 (3 mantissa bits).
// Each 32-column block is scaled by a power of two s that brings its largest
// magnitude into [128, 256) (exact), the accumulators are multiplied by s
// before the block's products and by 1/s after (both exact), so Y is the
// unscaled sum; Omega (|z| < 6) needs no scale.  The bf16 tile of the block
// holds one fp8 code per 16-bit slot so that the same transposing LDS read
// serves both precisions.
//
// Outputs of the mode-n product are written with non-temporal stores: they
// are read back only by the next pass, after far more traffic than the
// caches hold, and streaming them past the caches costs the reads less.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

constexpr int kColThreads = 256;            // 4 independent waves per workgroup
constexpr int kColWaves = kColThreads / kWave;

__device__ __forceinline__ f32x4 mma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 to_bf16x8(f32x4 a, f32x4 b) {
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        r[e] = static_cast<__bf16>(a[e]);
        r[e + 4] = static_cast<__bf16>(b[e]);
    }
    return r;
}

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split8(f32x4 a, f32x4 b, bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const __bf16 ha = static_cast<__bf16>(a[e]), hb = static_cast<__bf16>(b[e]);
        hi[e] = ha;
        hi[e + 4] = hb;
        lo[e] = static_cast<__bf16>(a[e] - static_cast<float>(ha));
        lo[e + 4] = static_cast<__bf16>(b[e] - static_cast<float>(hb));
    }
}

// Uniform (2m + 1) 2^-24 from the top 23 bits of x: the float 1 + m 2^-23
// assembled by a funnel shift, minus (1 - 2^-24); exact.
__device__ __forceinline__ float uniform01_bits(uint32_t x) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0x1.fffffep-1f;
}

// Rows 16 rt .. 16 rt + 15 of the column-major block tile (column pitch rowp
// bf16), columns 16 h2 .. 16 h2 + 15: lane (i, g) receives S(16 rt + i,
// 16 h2 + 4 g .. 16 h2 + 4 g + 3).
__device__ __forceinline__ s16x4 tile_tr(const __bf16* tile, int rowp, int h2, int rt, int lane) {
    const int s = lane & 15, G = lane >> 4;
    const __bf16* p = tile + (16 * h2 + 4 * G + (s >> 2)) * rowp + 16 * rt + 4 * (s & 3);
    return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p));
}

__device__ __forceinline__ bf16x8 cat_bf(s16x4 a, s16x4 b) {
    s16x8 v;
    v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
    v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ f32x4 mma32_fp8(long a, long b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// Eight floats as e4m3 codes, in order, packed into 64 bits.
__device__ __forceinline__ long to_fp8x8(f32x4 a, f32x4 b) {
    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a[0], a[1], 0, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(a[2], a[3], lo, true);
    int hi = __builtin_amdgcn_cvt_pk_fp8_f32(b[0], b[1], 0, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(b[2], b[3], hi, true);
    return static_cast<long>((static_cast<unsigned long>(static_cast<unsigned>(hi)) << 32) |
                             static_cast<unsigned>(lo));
}

// Eight floats scaled by s as e4m3 codes, one per 16-bit slot (low byte).
__device__ __forceinline__ bf16x8 to_fp8_slots(f32x4 a, f32x4 b, float s) {
    const long c = to_fp8x8(a * s, b * s);
    s16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = static_cast<short>((c >> (8 * e)) & 0xff);
    return __builtin_bit_cast(bf16x8, v);
}

// The low bytes of the eight 16-bit slots of a transposed tile read (the
// same k order as cat_bf).
__device__ __forceinline__ long cat_fp8(s16x4 a, s16x4 b) {
    unsigned long v = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v |= static_cast<unsigned long>(static_cast<unsigned short>(a[e]) & 0xff) << (8 * e);
        v |= static_cast<unsigned long>(static_cast<unsigned short>(b[e]) & 0xff) << (8 * (e + 4));
    }
    return static_cast<long>(v);
}

// One 64-bit product a * b of 32-bit words as a single v_mad_u64_u32 (the
// compiler otherwise issues v_mul_lo_u32 and v_mul_hi_u32).
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t b) {
    uint64_t r, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "s"(a), "v"(b));
    return r;
}

// Philox4x32-10 (see device_common.hpp) with the wide products above.
__device__ __forceinline__ void philox_wide(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = mul_wide(0xD2511F53u, c0);
        const uint64_t p1 = mul_wide(0xCD9E8D57u, c2);
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The four normals of counter quad q (same definition as normals4), with the
// hardware log2 / sqrt / sine / cosine: the values are rounded to bf16 next.
__device__ __forceinline__ void normals4_w(uint64_t q, uint32_t mode, uint32_t tag, uint64_t seed,
                                           float z[4]) {
    uint32_t c0 = static_cast<uint32_t>(q), c1 = static_cast<uint32_t>(q >> 32);
    uint32_t c2 = mode, c3 = tag;
    philox_wide(c0, c1, c2, c3, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const float u0 = uniform01_bits(c0), u1 = uniform01_bits(c1);
    const float u2 = uniform01_bits(c2), u3 = uniform01_bits(c3);
    const float r0 = __builtin_amdgcn_sqrtf(-1.38629436f * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_amdgcn_sqrtf(-1.38629436f * __builtin_amdgcn_logf(u2));
    z[0] = r0 * __builtin_amdgcn_cosf(u1);
    z[1] = r0 * __builtin_amdgcn_sinf(u1);
    z[2] = r1 * __builtin_amdgcn_cosf(u3);
    z[3] = r1 * __builtin_amdgcn_sinf(u3);
}

// Omega at linear indices e0 .. e0 + 3; `aligned` when e0 % 4 == 0.
__device__ __forceinline__ f32x4 omega4_w(uint64_t e0, uint32_t mode, uint32_t tag, uint64_t seed,
                                          bool aligned) {
    float z[4];
    normals4_w(e0 >> 2, mode, tag, seed, z);
    f32x4 w;
    w[0] = z[0]; w[1] = z[1]; w[2] = z[2]; w[3] = z[3];
    if (!aligned) {
        float z2[4];
        normals4_w((e0 >> 2) + 1, mode, tag, seed, z2);
        const int off = static_cast<int>(e0 & 3);
        // w[e] = (z ++ z2)[off + e], by selects (no indexed registers)
        f32x4 v;
        v[0] = off == 0 ? z[0] : off == 1 ? z[1] : off == 2 ? z[2] : z[3];
        v[1] = off == 0 ? z[1] : off == 1 ? z[2] : off == 2 ? z[3] : z2[0];
        v[2] = off == 0 ? z[2] : off == 1 ? z[3] : off == 2 ? z2[0] : z2[1];
        v[3] = off == 0 ? z[3] : off == 1 ? z2[0] : off == 2 ? z2[1] : z2[2];
        w = v;
    }
    return w;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const float* src, int64_t blk,
                                                             int64_t nblocks, int I, int64_t J) {
    // an empty range for a block past the end: its loads return zeros
    const int64_t b = blk < nblocks ? blk : nblocks - 1;
    const float* base = src + b * 32 * static_cast<int64_t>(I);
    int64_t rem = (J - b * 32) * static_cast<int64_t>(I) * 4;
    if (blk >= nblocks) rem = 0;
    const int nrec = rem > 0x7ffff000 ? 0x7ffff000 : static_cast<int>(rem);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), static_cast<short>(0), nrec,
                                             0x00020000);
}

// FLAG: the sum of squares (sketch) or the Gram Z^T Z (mode-n product).
// VAR: in the power step and the mode-n product (SPLIT), the tensor also
// enters Z = S^T M split (hi*lo + lo*hi + hi*hi) instead of rounded (hi*lo +
// hi*hi); in the sketch (FP8), e4m3 inputs instead of bf16.
template <int OP, int NCH, int NB, bool FLAG, bool VAR>
__device__ __forceinline__ void col_body(const ColGeom& g, const StreamArgs& a, int bidx, int nwg) {
    constexpr bool SPLIT = VAR && OP != OP_SKETCH;
    constexpr bool FP8 = VAR && OP == OP_SKETCH;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RT = 2 * NCH;                 // 16-row tiles of Y
    constexpr bool SS = (OP == OP_SKETCH) && FLAG;
    constexpr bool GRAM = (OP == OP_TTM) && FLAG;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int c16 = lane & 15, grp = lane >> 4;
    const int I = static_cast<int>(g.I), K = g.K;
    const int64_t J = g.J;
    const int rowp = g.rowp;

    // M fragments (B operand of Z = S^T M), fragment (h, nb): lane (n, g)
    // holds M(32 h + 8 g + e, 16 nb + n), e = 0..7, split hi / lo.
    bf16x8* mfr = reinterpret_cast<bf16x8*>(smem);
    __bf16* tile = reinterpret_cast<__bf16*>(smem + g.mfr_bytes) +
                   static_cast<size_t>(wave) * 32 * rowp;
    if (OP != OP_SKETCH) {
        // M (I x K, column-major) staged in LDS past the fragments with 16-byte
        // loads, then the fragments built from LDS
        const float* __restrict__ mg = static_cast<const float*>(a.mat);
        float* ms = reinterpret_cast<float*>(smem + g.mfr_bytes);
        if (mg) {
            const int n = I * K;
            if ((reinterpret_cast<uintptr_t>(mg) & 15) == 0) {
                for (int e = 4 * tid; e + 3 < n; e += 4 * kColThreads)
                    *reinterpret_cast<f32x4*>(ms + e) = *reinterpret_cast<const f32x4*>(mg + e);
                for (int e = (n & ~3) + tid; e < n; e += kColThreads) ms[e] = mg[e];
            } else {
                for (int e = tid; e < n; e += kColThreads) ms[e] = mg[e];
            }
            __syncthreads();
        }
        const float* m = mg ? ms : nullptr;
        for (int idx = tid; idx < NCH * NB * 64; idx += kColThreads) {
            const int ln = idx & 63, hn = idx >> 6;
            const int h = hn / NB, nb = hn - h * NB;
            const int r = 16 * nb + (ln & 15), gq = ln >> 4;
            f32x4 v0, v1;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = 32 * h + 8 * gq + e;
                float x = 0.0f;
                if (i < I && r < K) x = m ? m[static_cast<int64_t>(r) * I + i] : (i == r ? 1.0f : 0.0f);
                if (e < 4) v0[e] = x; else v1[e - 4] = x;
            }
            bf16x8 hi, lo;
            split8(v0, v1, hi, lo);
            mfr[(hn * 2 + 0) * 64 + ln] = hi;
            mfr[(hn * 2 + 1) * 64 + ln] = lo;
        }
        __syncthreads();
    }

    constexpr int AR = (OP == OP_TTM) ? 1 : RT;     // Y accumulators (sketch, power)
    constexpr int AN = (OP == OP_TTM) ? 1 : NB;
    constexpr int GN = GRAM ? NB : 1;               // Gram accumulators
    f32x4 acc[AR][AN];
    f32x4 accg[GN][GN];
#pragma unroll
    for (int f = 0; f < AR; ++f)
#pragma unroll
        for (int nb = 0; nb < AN; ++nb) acc[f][nb] = zero4<f32x4>();
#pragma unroll
    for (int f = 0; f < GN; ++f)
#pragma unroll
        for (int nb = 0; nb < GN; ++nb) accg[f][nb] = zero4<f32x4>();
    double ss = 0.0;

    const float* __restrict__ src = static_cast<const float*>(a.src);
    const int64_t wid = static_cast<int64_t>(bidx) * kColWaves + wave;
    const int64_t nw = static_cast<int64_t>(nwg) * kColWaves;
    const bool jal = (J & 3) == 0;
    const int voff = (c16 * I + 8 * grp) * 4;       // bytes: column c16 of half 0, row 8 grp
    const int half1 = 16 * I * 4;                   // bytes to column half 1
    // Omega linear index of (row j0 + 4 grp, column 16 nb + c16), less j0
    uint64_t eb[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
        eb[nb] = static_cast<uint64_t>(16 * nb + c16) * static_cast<uint64_t>(J) + 4 * grp;

    // PD blocks in flight per wave: the loop alternates between the register
    // sets F0 and F1 (PD = 2), each refilled chunk by chunk with the block
    // PD nw ahead.  The sketch and the power step, whose Y accumulators need
    // the registers, keep one block in flight (the power step spills with
    // two), as do the largest tiles.
    constexpr int PD = (OP != OP_TTM || NCH * NB > 24) ? 1 : 2;
    // The power step reads the M fragments of chunk h + 1 while chunk h is
    // multiplied (the projection, measured, does better without).
    constexpr bool MPF = OP == OP_POWER;
    f32x4 F0[NCH][2][2], F1[NCH][2][2];
    // The first loads of a register set, chunk 0 first: the loop body consumes
    // the chunks in that order, and with the order pinned (no reordering across
    // the scheduling barriers) the wait before chunk h covers only the loads
    // issued before it.  Otherwise the waits at the top of the loop, which
    // also cover entry from here, drain every load in flight.
    auto issue = [&](f32x4 (&Fb)[NCH][2][2], int64_t blk) {
        const __amdgpu_buffer_rsrc_t rs = block_rsrc(src, blk, g.nblocks, I, J);
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    Fb[h][h2][q] = __builtin_bit_cast(
                        f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 128 * h + 16 * q,
                                                                     h2 ? half1 : 0, 0));
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // mode-n product output staging (TTM): 32 x 16 NB floats per wave
    float* stage = reinterpret_cast<float*>(smem + g.mfr_bytes) + static_cast<size_t>(wave) * 32 * 16 * NB;

    // Omega rows j .. j + 3 and j + 16 .. j + 19 of column k (linear index e0
    // of the first): the Gaussian stream, or the structured matrix
    auto omega8 = [&](uint64_t e0, int64_t j, int k, f32x4& w0, f32x4& w1) {
        if (a.kr.nq) {
            float t0[4], t1[4];
            kr_entry4<float>(a.kr, j, k, t0);
            kr_entry4<float>(a.kr, j + 16, k, t1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                w0[e] = t0[e];
                w1[e] = t1[e];
            }
        } else {
            w0 = omega4_w(e0, a.mode, a.tag, a.seed, jal);
            w1 = omega4_w(e0 + 16, a.mode, a.tag, a.seed, jal);
        }
    };
    auto body = [&](f32x4 (&Fb)[NCH][2][2], int64_t blk) {
        const int64_t j0 = blk * 32;
        const __amdgpu_buffer_rsrc_t rn = block_rsrc(src, blk + PD * nw, g.nblocks, I, J);
        f32x4 Z[2][NB];
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) Z[h2][nb] = zero4<f32x4>();
        float part = 0.0f;
        bf16x8 mcu[MPF ? NB : 1][2], mnx[MPF ? NB : 1][2];
        if constexpr (MPF) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                mcu[nb][0] = mfr[(nb * 2 + 0) * 64 + lane];
                mcu[nb][1] = mfr[(nb * 2 + 1) * 64 + lane];
            }
        }

        // FP8: the power-of-two scale of the block (largest magnitude to [128, 256))
        float fscale = 1.0f, finv = 1.0f;
        if constexpr (FP8) {
            float mx = 0.0f;
#pragma unroll
            for (int h = 0; h < NCH; ++h)
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) mx = fmaxf(mx, fabsf(Fb[h][h2][q][e]));
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
            if (mx > 0.0f) {
                int ex = 8 - __builtin_amdgcn_frexp_expf(mx);
                ex = ex > 64 ? 64 : ex;
                fscale = __builtin_amdgcn_ldexpf(1.0f, ex);
                finv = __builtin_amdgcn_ldexpf(1.0f, -ex);
            }
        }
        // chunk by chunk: round to bf16, stage for the transpose, refill the
        // chunk's registers with the block 2 nw ahead, and Z = S^T M
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
            if (SS) {
                const int hv = I - 32 * h;          // valid rows of the chunk (uniform)
                if (hv >= 32) {
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                        for (int q = 0; q < 2; ++q)
#pragma unroll
                            for (int e = 0; e < 4; ++e) part = fmaf(Fb[h][h2][q][e], Fb[h][h2][q][e], part);
                } else if (hv > 0) {
                    const int lim = hv - 8 * grp;
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                        for (int q = 0; q < 2; ++q)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const float v = (4 * q + e < lim) ? Fb[h][h2][q][e] : 0.0f;
                                part = fmaf(v, v, part);
                            }
                }
            }
            bf16x8 D0, D1, L0, L1;
            if constexpr (SPLIT) {
                split8(Fb[h][0][0], Fb[h][0][1], D0, L0);
                split8(Fb[h][1][0], Fb[h][1][1], D1, L1);
            } else if constexpr (FP8) {
                D0 = to_fp8_slots(Fb[h][0][0], Fb[h][0][1], fscale);
                D1 = to_fp8_slots(Fb[h][1][0], Fb[h][1][1], fscale);
            } else {
                D0 = to_bf16x8(Fb[h][0][0], Fb[h][0][1]);
                D1 = to_bf16x8(Fb[h][1][0], Fb[h][1][1]);
            }
            if (OP != OP_TTM) {
                *reinterpret_cast<bf16x8*>(tile + c16 * rowp + 32 * h + 8 * grp) = D0;
                *reinterpret_cast<bf16x8*>(tile + (16 + c16) * rowp + 32 * h + 8 * grp) = D1;
            }
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    Fb[h][h2][q] = __builtin_bit_cast(
                        f32x4, __builtin_amdgcn_raw_buffer_load_b128(rn, voff + 128 * h + 16 * q,
                                                                     h2 ? half1 : 0, 0));
            if (OP != OP_SKETCH) {
                if constexpr (MPF) {
                    if (h + 1 < NCH) {
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) {
                            mnx[nb][0] = mfr[(((h + 1) * NB + nb) * 2 + 0) * 64 + lane];
                            mnx[nb][1] = mfr[(((h + 1) * NB + nb) * 2 + 1) * 64 + lane];
                        }
                    }
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    bf16x8 mhi, mlo;
                    if constexpr (MPF) {
                        mhi = mcu[nb][0];
                        mlo = mcu[nb][1];
                    } else {
                        mhi = mfr[((h * NB + nb) * 2 + 0) * 64 + lane];
                        mlo = mfr[((h * NB + nb) * 2 + 1) * 64 + lane];
                    }
                    if (SPLIT) {
                        Z[0][nb] = mma32(L0, mhi, Z[0][nb]);
                        Z[1][nb] = mma32(L1, mhi, Z[1][nb]);
                    }
                    Z[0][nb] = mma32(D0, mlo, Z[0][nb]);
                    Z[1][nb] = mma32(D1, mlo, Z[1][nb]);
                    Z[0][nb] = mma32(D0, mhi, Z[0][nb]);
                    Z[1][nb] = mma32(D1, mhi, Z[1][nb]);
                }
                if constexpr (MPF) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        mcu[nb][0] = mnx[nb][0];
                        mcu[nb][1] = mnx[nb][1];
                    }
                }
            }
        }
        if (SS) ss += static_cast<double>(part);

        // ---- Y += S_blk W, W = Omega (sketch) or Z (power step)
        if constexpr (FP8) {
            long W8[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const uint64_t e0 = eb[nb] + static_cast<uint64_t>(j0);
                f32x4 w0, w1;
                omega8(e0, j0 + 4 * grp, 16 * nb + c16, w0, w1);
                W8[nb] = to_fp8x8(w0, w1);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const long A8 = cat_fp8(tile_tr(tile, rowp, 0, rt, lane), tile_tr(tile, rowp, 1, rt, lane));
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[rt][nb] = mma32_fp8(A8, W8[nb], acc[rt][nb] * fscale) * finv;
            }
        } else if (OP != OP_TTM) {
            bf16x8 Whi[NB], Wlo[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                if (OP == OP_SKETCH) {
                    const uint64_t e0 = eb[nb] + static_cast<uint64_t>(j0);
                    f32x4 w0, w1;
                    omega8(e0, j0 + 4 * grp, 16 * nb + c16, w0, w1);
                    Whi[nb] = to_bf16x8(w0, w1);
                } else {
                    split8(Z[0][nb], Z[1][nb], Whi[nb], Wlo[nb]);
                }
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const bf16x8 A = cat_bf(tile_tr(tile, rowp, 0, rt, lane), tile_tr(tile, rowp, 1, rt, lane));
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    if (OP == OP_POWER) acc[rt][nb] = mma32(A, Wlo[nb], acc[rt][nb]);
                    acc[rt][nb] = mma32(A, Whi[nb], acc[rt][nb]);
                }
            }
        }

        // ---- mode-n product output and its Gram
        if (OP == OP_TTM) {
            float* __restrict__ out = static_cast<float*>(a.out);
            const bool full = j0 + 32 <= J;
            if (a.out_t) {
                // rotated layout out[r * J + j]: four consecutive j per lane
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        const int r = 16 * nb + c16;
                        const int64_t jj = j0 + 16 * h2 + 4 * grp;
                        if (r < K) {
                            float* o = out + static_cast<int64_t>(r) * J + jj;
                            if (jal && full) {
                                __builtin_nontemporal_store(Z[h2][nb], reinterpret_cast<f32x4*>(o));
                            } else {
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    if (jj + e < J) __builtin_nontemporal_store(Z[h2][nb][e], o + e);
                            }
                        }
                    }
            } else {
                // out[j * K + r]: the block's 32 K values are contiguous; stage
                // them in LDS and write 16-byte pieces
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        const int r = 16 * nb + c16;
                        if (r < K) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) stage[(16 * h2 + 4 * grp + e) * K + r] = Z[h2][nb][e];
                        }
                    }
                const int64_t nval = (full ? 32 : (J > j0 ? J - j0 : 0)) * static_cast<int64_t>(K);
                float* ob = out + j0 * static_cast<int64_t>(K);
                const int n4 = static_cast<int>(nval >> 2);
                for (int t = lane; t < n4; t += kWave)
                    __builtin_nontemporal_store(*reinterpret_cast<const f32x4*>(stage + 4 * t),
                                                reinterpret_cast<f32x4*>(ob + 4 * t));
                for (int t = 4 * n4 + lane; t < nval; t += kWave) __builtin_nontemporal_store(stage[t], ob + t);
            }
            if (GRAM) {
                bf16x8 Ghi[NB], Glo[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) split8(Z[0][nb], Z[1][nb], Ghi[nb], Glo[nb]);
#pragma unroll
                for (int n1 = 0; n1 < NB; ++n1)
#pragma unroll
                    for (int n2 = 0; n2 < NB; ++n2) {
                        accg[n1][n2] = mma32(Glo[n1], Ghi[n2], accg[n1][n2]);
                        accg[n1][n2] = mma32(Ghi[n1], Glo[n2], accg[n1][n2]);
                        accg[n1][n2] = mma32(Ghi[n1], Ghi[n2], accg[n1][n2]);
                    }
            }
        }
    };

    issue(F0, wid);
    if (PD == 2) {
        issue(F1, wid + nw);
        for (int64_t blk = wid; blk < g.nblocks; blk += 2 * nw) {
            body(F0, blk);
            if (blk + nw < g.nblocks) body(F1, blk + nw);
        }
    } else {
        for (int64_t blk = wid; blk < g.nblocks; blk += nw) body(F0, blk);
    }

    // ---- cross-wave reduction (fixed order) and the per-workgroup partials
    __syncthreads();
    float* red = reinterpret_cast<float*>(smem);
    const size_t gidx = static_cast<size_t>(bidx);
    const int I_pad = 32 * NCH, K_pad = 16 * NB;
    if (OP != OP_TTM && g.red3) {
        // waves 1..3 store their accumulators (16-byte pieces) in regions
        // 0..2; wave 0 adds them in wave order, ((a0 + a1) + a2) + a3, and
        // writes the partial from registers
        const int region = K_pad * I_pad;
        if (wave > 0) {
            float* rw = red + (wave - 1) * region;
#pragma unroll
            for (int rt = 0; rt < AR; ++rt)
#pragma unroll
                for (int nb = 0; nb < AN; ++nb)
                    *reinterpret_cast<f32x4*>(rw + (16 * nb + c16) * I_pad + 16 * rt + 4 * grp) = acc[rt][nb];
        }
        __syncthreads();
        if (wave == 0) {
            float* __restrict__ py = static_cast<float*>(a.part_y) + gidx * K_pad * I_pad;
#pragma unroll
            for (int rt = 0; rt < AR; ++rt)
#pragma unroll
                for (int nb = 0; nb < AN; ++nb) {
                    const int off = (16 * nb + c16) * I_pad + 16 * rt + 4 * grp;
                    f32x4 v = acc[rt][nb];
#pragma unroll
                    for (int w = 0; w < kColWaves - 1; ++w) {
                        const f32x4 o = *reinterpret_cast<const f32x4*>(red + w * region + off);
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] += o[e];
                    }
                    *reinterpret_cast<f32x4*>(py + off) = v;
                }
        }
        __syncthreads();
    } else if (OP != OP_TTM) {
        for (int w = 0; w < kColWaves; ++w) {
            if (wave == w) {
#pragma unroll
                for (int rt = 0; rt < AR; ++rt)
#pragma unroll
                    for (int nb = 0; nb < AN; ++nb)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int idx = (16 * nb + c16) * I_pad + 16 * rt + 4 * grp + e;
                            red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[rt][nb][e];
                        }
            }
            __syncthreads();
        }
        float* __restrict__ py = static_cast<float*>(a.part_y) + gidx * K_pad * I_pad;
        for (int e = tid; e < K_pad * I_pad; e += kColThreads) py[e] = red[e];
    }
    if (GRAM) {
        for (int w = 0; w < kColWaves; ++w) {
            if (wave == w) {
#pragma unroll
                for (int n1 = 0; n1 < GN; ++n1)
#pragma unroll
                    for (int n2 = 0; n2 < GN; ++n2)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int idx = (16 * n2 + c16) * K_pad + 16 * n1 + 4 * grp + e;
                            red[idx] = (w == 0 ? 0.0f : red[idx]) + accg[n1][n2][e];
                        }
            }
            __syncthreads();
        }
        float* __restrict__ pg = static_cast<float*>(a.part_g) + gidx * K_pad * K_pad;
        for (int e = tid; e < K_pad * K_pad; e += kColThreads) pg[e] = red[e];
    }
    if (SS) {
        __shared__ double rs[kColWaves];
        ss = wave_sum(ss);
        if (lane == 0) rs[wave] = ss;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kColWaves; ++w) s += rs[w];
            a.part_ss[gidx] = s;
        }
    }
}

template <int OP, int NCH, int NB, bool FLAG, bool VAR>
__global__ __launch_bounds__(kColThreads, 1) void k_col(ColGeom g, StreamArgs a) {
    col_body<OP, NCH, NB, FLAG, VAR>(g, a, blockIdx.x, gridDim.x);
}

// Many problems: job blockIdx.y on workgroups 0 .. units - 1 of grid x (the
// job read in place: uniform, scalar loads).
template <int OP, int NCH, int NB, bool FLAG, bool VAR>
__global__ __launch_bounds__(kColThreads, 1) void k_col_batch(const ColJob* __restrict__ jobs) {
    const ColJob& j = jobs[blockIdx.y];
    if (static_cast<int>(blockIdx.x) >= j.units) return;
    col_body<OP, NCH, NB, FLAG, VAR>(j.g, j.a, blockIdx.x, j.units);
}

// ---------------------------------------------------------------------------
// Planning and dispatch: (32-row chunks, 16-column operand blocks) shapes,
// exact ones first; a shape runs on the smallest instantiation that covers it.
// ---------------------------------------------------------------------------
static const int kColShapes[][2] = {{7, 3}, {2, 2}, {1, 2}, {2, 4}, {4, 2}, {4, 4}, {8, 2}, {8, 4}};
constexpr int kNumColShapes = 8;

// The batched instantiations: generic shapes only (a shape runs every
// geometry it covers, its rows and operand columns padded to 32 NCH and
// 16 NB).  Every row-chunk count up to eight with two operand blocks, and
// three or four operand blocks at 4, 6 and 8 chunks: on the 512-tensor
// workload (extents 32..256, K 9..37) 8.1 ms against 8.9 with 8 shapes and
// 9.7 with 5 (2, 4 and 8 chunks), the padding's work being the difference.
static const int kColBatchShapes[][2] = {{2, 2}, {4, 2}, {8, 2}, {4, 4}, {8, 4}, {3, 2}, {6, 2}, {6, 4},
                                         {5, 2}, {7, 2}, {4, 3}, {6, 3}, {8, 3}};
constexpr int kNumColBatchShapes = 13;

static bool plan_col_in(int op, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu,
                        const int (*shapes)[2], int nshapes, ColGeom* g) {
    if (L != 1 || I < 1 || I > 256 || T < 1 || K < 1 || K > 64) return false;
    if (op == OP_SKETCH ? (ct != CT_BF16 && ct != CT_FP8) : (ct != CT_BF16X2 && ct != CT_BF16X3))
        return false;
    g->split = (op != OP_SKETCH && ct == CT_BF16X3) ? 1 : 0;
    g->fp8 = (op == OP_SKETCH && ct == CT_FP8) ? 1 : 0;
    const int nch = static_cast<int>((I + 31) / 32), nb = (K + 15) / 16;
    int var = -1, best = 1 << 30;
    for (int v = 0; v < nshapes; ++v) {
        const int c = shapes[v][0], b = shapes[v][1];
        if (c >= nch && b >= nb && c * b < best) {
            best = c * b;
            var = v;
        }
    }
    if (var < 0) return false;
    const int NCH = shapes[var][0], NB = shapes[var][1];
    g->I = I;
    g->J = T;
    g->K = K;
    g->nch = NCH;
    g->nb = NB;
    g->variant = var;
    g->rowp = 32 * NCH + 8;
    g->mfr_bytes = (op != OP_SKETCH) ? static_cast<size_t>(NCH) * NB * 2 * 64 * 16 : 0;
    // per wave: the bf16 block tile (sketch, power step) or the 32 x K output
    // staging of the mode-n product
    const size_t tiles = (op != OP_TTM) ? static_cast<size_t>(kColWaves) * 32 * g->rowp * 2
                                        : static_cast<size_t>(kColWaves) * 32 * 16 * NB * 4;
    size_t lds = g->mfr_bytes + tiles;
    // M staged past the fragments at the start
    if (op != OP_SKETCH && g->mfr_bytes + static_cast<size_t>(I) * K * 4 > lds)
        lds = g->mfr_bytes + static_cast<size_t>(I) * K * 4;
    const size_t red = (op != OP_TTM) ? static_cast<size_t>(32 * NCH) * 16 * NB * 4
                                      : static_cast<size_t>(16 * NB) * 16 * NB * 4;
    if (red > lds) lds = red;
    if (lds + kStaticLdsMargin > kLdsLimit) return false;
    g->red3 = 0;
    if (op != OP_TTM) {
        const size_t l3 = 3 * red > lds ? 3 * red : lds;
        if (l3 + kStaticLdsMargin <= kLdsLimit) {
            lds = l3;
            g->red3 = 1;
        }
    }
    g->lds_bytes = lds;
    g->nblocks = (T + 31) / 32;
    const int64_t wgs = (g->nblocks + kColWaves - 1) / kColWaves;
    const int64_t cap = num_cu > 0 ? num_cu : 256;
    g->grid = static_cast<int>(wgs < cap ? wgs : cap);
    g->I_pad = 32 * NCH;
    g->K_pad = 16 * NB;
    return true;
}

bool plan_col(int op, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu, ColGeom* g) {
    return plan_col_in(op, ct, L, I, T, K, num_cu, kColShapes, kNumColShapes, g);
}

bool plan_col_batch(int op, int ct, int64_t I, int64_t T, int K, ColGeom* g) {
    // the sketch on e4m3 and the split-free (BF16X2) passes have no batched
    // instantiation
    if (op == OP_SKETCH ? ct != CT_BF16 : ct != CT_BF16X3) return false;
    return plan_col_in(op, ct, 1, I, T, K, 256, kColBatchShapes, kNumColBatchShapes, g);
}

template <int OP, int NCH, int NB, bool VAR>
static hipError_t launch_col_s(const ColGeom& g, const StreamArgs& a, hipStream_t s) {
    const bool flag = (OP == OP_SKETCH) ? a.part_ss != nullptr : (OP == OP_TTM && a.part_g != nullptr);
    if (flag)
        hipLaunchKernelGGL((k_col<OP, NCH, NB, true, VAR>), dim3(g.grid), dim3(kColThreads),
                           g.lds_bytes, s, g, a);
    else
        hipLaunchKernelGGL((k_col<OP, NCH, NB, false, VAR>), dim3(g.grid), dim3(kColThreads),
                           g.lds_bytes, s, g, a);
    return hipGetLastError();
}

template <int OP, int NCH, int NB>
static hipError_t launch_col_t(const ColGeom& g, const StreamArgs& a, hipStream_t s) {
    if constexpr (OP != OP_SKETCH) {
        if (g.split) return launch_col_s<OP, NCH, NB, true>(g, a, s);
    } else {
        if (g.fp8) return launch_col_s<OP, NCH, NB, true>(g, a, s);
    }
    return launch_col_s<OP, NCH, NB, false>(g, a, s);
}

template <int OP>
static hipError_t launch_col_op(const ColGeom& g, const StreamArgs& a, hipStream_t s) {
    switch (g.variant) {
        case 0: return launch_col_t<OP, 7, 3>(g, a, s);
        case 1: return launch_col_t<OP, 2, 2>(g, a, s);
        case 2: return launch_col_t<OP, 1, 2>(g, a, s);
        case 3: return launch_col_t<OP, 2, 4>(g, a, s);
        case 4: return launch_col_t<OP, 4, 2>(g, a, s);
        case 5: return launch_col_t<OP, 4, 4>(g, a, s);
        case 6: return launch_col_t<OP, 8, 2>(g, a, s);
        default: return launch_col_t<OP, 8, 4>(g, a, s);
    }
}

hipError_t launch_col(int op, const ColGeom& g, const StreamArgs& a, hipStream_t s) {
    if (op == OP_SKETCH) return launch_col_op<OP_SKETCH>(g, a, s);
    if (op == OP_POWER) return launch_col_op<OP_POWER>(g, a, s);
    return launch_col_op<OP_TTM>(g, a, s);
}

template <int OP, int NCH, int NB, bool FLAG, bool VAR>
static hipError_t launch_col_batch_t(const ColJob* jobs, int njobs, int max_units, size_t lds,
                                     hipStream_t s) {
    hipLaunchKernelGGL((k_col_batch<OP, NCH, NB, FLAG, VAR>), dim3(max_units, njobs), dim3(kColThreads),
                       lds, s, jobs);
    return hipGetLastError();
}

// (op, flag) of the batched kinds: sketch with or without the sum of squares
// (bf16), the power step (split), the mode-n product with or without its
// Gram (split)
template <int OP, bool FLAG, bool VAR>
static hipError_t launch_col_batch_k(int shape, const ColJob* jobs, int njobs, int max_units,
                                     size_t lds, hipStream_t s) {
    switch (shape) {
        case 0: return launch_col_batch_t<OP, 2, 2, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 1: return launch_col_batch_t<OP, 4, 2, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 2: return launch_col_batch_t<OP, 8, 2, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 3: return launch_col_batch_t<OP, 4, 4, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 4: return launch_col_batch_t<OP, 8, 4, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 5: return launch_col_batch_t<OP, 3, 2, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 6: return launch_col_batch_t<OP, 6, 2, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 7: return launch_col_batch_t<OP, 6, 4, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 8: return launch_col_batch_t<OP, 5, 2, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 9: return launch_col_batch_t<OP, 7, 2, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 10: return launch_col_batch_t<OP, 4, 3, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 11: return launch_col_batch_t<OP, 6, 3, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        case 12: return launch_col_batch_t<OP, 8, 3, FLAG, VAR>(jobs, njobs, max_units, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_col_batch(int op, int shape, bool flag, const ColJob* jobs, int njobs, int max_units,
                            size_t lds, hipStream_t s) {
    if (njobs < 1 || max_units < 1 || lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    if (op == OP_SKETCH)
        return flag ? launch_col_batch_k<OP_SKETCH, true, false>(shape, jobs, njobs, max_units, lds, s)
                    : launch_col_batch_k<OP_SKETCH, false, false>(shape, jobs, njobs, max_units, lds, s);
    if (op == OP_POWER) return launch_col_batch_k<OP_POWER, false, true>(shape, jobs, njobs, max_units, lds, s);
    return flag ? launch_col_batch_k<OP_TTM, true, true>(shape, jobs, njobs, max_units, lds, s)
                : launch_col_batch_k<OP_TTM, false, true>(shape, jobs, njobs, max_units, lds, s);
}

}  // namespace rh
