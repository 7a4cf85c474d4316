// GHASH multiplication (SP 800-38D section 6.3) on the device, shared by the
// single-buffer GCM kernels and the batch kernels: products by a fixed
// multiplier M through 4-bit tables in LDS, the builds of those tables (by a
// workgroup or by one wave), a product of two arbitrary elements by one wave,
// and one AES encryption from the row-0 round table.
//
// Multiplication by a fixed element M uses 4-bit tables: for each of the 32
// nibble positions of a block, the 16 products (nibble value at that
// position) * M, 16 bytes each (8 KiB per multiplier).  A product is 32
// 16-byte LDS reads XORed together.  A table of 256 bytes covers every LDS
// bank once, so the 64 lanes of a read never conflict (equal values are
// broadcast).
#pragma once

#include <hip/hip_runtime.h>

#include "cipher_core.h"
#include "gf128.h"

namespace aesgpu {
namespace {

constexpr uint32_t kTabBytes = 8192;   // one multiplier's nibble tables
constexpr uint32_t kVecBytes = 2048;   // M * x^e for e < 128, while building them

__device__ __forceinline__ u32x4 lds_load16(const uint32_t *lds, uint32_t off) {
    return *reinterpret_cast<const u32x4 *>(reinterpret_cast<const char *>(lds) + off);
}

__device__ __forceinline__ void lds_store16(uint32_t *lds, uint32_t off, u32x4 v) {
    *reinterpret_cast<u32x4 *>(reinterpret_cast<char *>(lds) + off) = v;
}

// y = x * M for the multiplier whose tables start at byte offset `tab` (a
// multiple of 256 below 16 MiB).  Position p = 8c + m is bits 4m .. 4m+3 of
// word c (byte 4c + m/2 of the block); entry (p, v) sits at tab + 256 p +
// 16 v: the position's offset rides in the read's immediate field, and the
// address register is 16 v in byte 0 and tab in bytes 1 and 2, put together
// by one byte permute from the word's nibbles masked in place (high nibbles:
// x & 0xF0F0F0F0; low ones: (x << 4) & 0xF0F0F0F0).
__device__ __forceinline__ void mul_tab(const uint32_t *lds, uint32_t tab, const uint32_t (&x)[4],
                                        uint32_t (&y)[4]) {
    uint32_t acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; c++) {
        uint32_t xc = x[c];
        // an empty step the compiler cannot see through: this word's eight
        // addresses and reads are formed here rather than all 32 up front,
        // which would need 128 more registers
        asm volatile("" : "+v"(xc) :: "memory");
        const uint32_t xh = xc & 0xF0F0F0F0u;           // high nibble of every byte, times 16
        const uint32_t xl = (xc << 4) & 0xF0F0F0F0u;    // low nibble of every byte, times 16
#pragma unroll
        for (int b = 0; b < 4; b++) {
            // byte 0: byte b of the masked word; bytes 1, 2: tab's; byte 3: 0
            const uint32_t sel = 0x0C020104u + uint32_t(b);
            const uint32_t alo = __builtin_amdgcn_perm(xl, tab, sel);
            const uint32_t ahi = __builtin_amdgcn_perm(xh, tab, sel);
            const u32x4 t0 = lds_load16(lds, alo + uint32_t(8 * c + 2 * b) * 256u);
            const u32x4 t1 = lds_load16(lds, ahi + uint32_t(8 * c + 2 * b + 1) * 256u);
            acc[0] = xor3(acc[0], t0.x, t1.x);
            acc[1] = xor3(acc[1], t0.y, t1.y);
            acc[2] = xor3(acc[2], t0.z, t1.z);
            acc[3] = xor3(acc[3], t0.w, t1.w);
        }
    }
    // and the product is complete here: no XOR of it is deferred past this
    // point (which would keep all 32 reads alive)
    asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]));
#pragma unroll
    for (int c = 0; c < 4; c++)
        y[c] = acc[c];
}

// Builds the tables of the multipliers src(k) (four words each, a block in
// memory order), k < count, at byte offsets dst + k * kTabBytes, using
// count * kVecBytes of scratch at `vec`.
// Every thread of the workgroup takes part; starts and ends with a barrier
// (the tables may overwrite LDS that other waves were reading).
template <typename Src>
__device__ __forceinline__ void build_tables(uint32_t *lds, uint32_t dst, uint32_t vec, int count, Src src) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < uint32_t(count) * 128u; i += blockDim.x) {
        const uint32_t k = i >> 7, e = i & 127u;
        const uint32_t *m = src(int(k));
        const uint32_t w[4] = {m[0], m[1], m[2], m[3]};
        uint64_t lo, hi;
        to_poly(w, lo, hi);
        mulx_pow(lo, hi, e);
        uint32_t r[4];
        from_poly(lo, hi, r);
        lds_store16(lds, vec + (k * 128u + e) * 16u, vec4(r[0], r[1], r[2], r[3]));
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < uint32_t(count) * 512u; i += blockDim.x) {
        const uint32_t k = i >> 9, p = (i >> 4) & 31u, v = i & 15u;
        const uint32_t byte = 4u * (p >> 3) + ((p & 7u) >> 1), half = p & 1u;
        u32x4 acc = vec4(0, 0, 0, 0);
#pragma unroll
        for (uint32_t t = 0; t < 4; t++) {
            if ((v >> t) & 1u) {
                // bit 4*half + t of the byte is the coefficient of x^(8*byte + 7 - 4*half - t)
                const uint32_t e = 8u * byte + 7u - 4u * half - t;
                acc ^= lds_load16(lds, vec + (k * 128u + e) * 16u);
            }
        }
        lds_store16(lds, dst + k * kTabBytes + p * 256u + v * 16u, acc);
    }
    __syncthreads();
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int mask) {
    const int lo = __shfl_xor(int(uint32_t(v)), mask, 64);
    const int hi = __shfl_xor(int(uint32_t(v >> 32)), mask, 64);
    return uint64_t(uint32_t(lo)) | (uint64_t(uint32_t(hi)) << 32);
}

// x * y in the arithmetic form, x and y the same in every lane of the wave:
// lane l adds x_(2l) y x^(2l) and x_(2l+1) y x^(2l+1), then the wave XORs
// its 64 partial sums.
__device__ void mul_wave(uint64_t xlo, uint64_t xhi, uint64_t ylo, uint64_t yhi, uint64_t &rlo,
                         uint64_t &rhi) {
    const uint32_t e = 2u * (threadIdx.x & 63u);
    uint64_t vlo = ylo, vhi = yhi;
    mulx_pow(vlo, vhi, e);
    const uint64_t bits = e < 64 ? xlo >> e : xhi >> (e - 64);
    uint64_t alo = (bits & 1) ? vlo : 0, ahi = (bits & 1) ? vhi : 0;
    mulx_small(vlo, vhi, 1);
    if (bits & 2) {
        alo ^= vlo;
        ahi ^= vhi;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        alo ^= shfl_xor64(alo, off);
        ahi ^= shfl_xor64(ahi, off);
    }
    rlo = alo;
    rhi = ahi;
}

// One AES encryption (every lane its own input), the row-0 round table
// at t0 (LDS or global memory; the other rows are its rotations).
template <int NR>
__device__ __forceinline__ void encrypt_one(const uint32_t *t0, const uint32_t *rk, uint32_t (&s)[4]) {
    auto T = [&](int t, uint32_t w, int k) { return rotl(t0[(w >> (8 * k)) & 255u], 8 * t); };
    uint32_t a0 = s[0] ^ rk[0], a1 = s[1] ^ rk[1], a2 = s[2] ^ rk[2], a3 = s[3] ^ rk[3];
#pragma unroll
    for (int r = 1; r < NR; r++) {
        const uint32_t b0 = T(0, a0, 0) ^ T(1, a1, 1) ^ T(2, a2, 2) ^ T(3, a3, 3) ^ rk[4 * r];
        const uint32_t b1 = T(0, a1, 0) ^ T(1, a2, 1) ^ T(2, a3, 2) ^ T(3, a0, 3) ^ rk[4 * r + 1];
        const uint32_t b2 = T(0, a2, 0) ^ T(1, a3, 1) ^ T(2, a0, 2) ^ T(3, a1, 3) ^ rk[4 * r + 2];
        const uint32_t b3 = T(0, a3, 0) ^ T(1, a0, 1) ^ T(2, a1, 2) ^ T(3, a2, 3) ^ rk[4 * r + 3];
        a0 = b0;
        a1 = b1;
        a2 = b2;
        a3 = b3;
    }
    // last round: S[x] is byte 1 of T0[x]
    auto S = [&](uint32_t w, int k) { return (t0[(w >> (8 * k)) & 255u] >> 8) & 255u; };
    s[0] = (S(a0, 0) | (S(a1, 1) << 8) | (S(a2, 2) << 16) | (S(a3, 3) << 24)) ^ rk[4 * NR];
    s[1] = (S(a1, 0) | (S(a2, 1) << 8) | (S(a3, 2) << 16) | (S(a0, 3) << 24)) ^ rk[4 * NR + 1];
    s[2] = (S(a2, 0) | (S(a3, 1) << 8) | (S(a0, 2) << 16) | (S(a1, 3) << 24)) ^ rk[4 * NR + 2];
    s[3] = (S(a3, 0) | (S(a0, 1) << 8) | (S(a1, 2) << 16) | (S(a2, 3) << 24)) ^ rk[4 * NR + 3];
}


// One wave builds the table of multiplier m (the same four words in every
// lane) at byte offset dst, which belongs to this wave alone.  Lane l fills
// the 8 entries (p, v) of position p = l / 2 with bit 3 of v equal to l & 1:
// bit t of nibble value v at position p (4c + h/2 ... see mul_tab) is the
// coefficient of x^(e + 3 - t), e = 8 * byte + 4 - 4 * half, so the lane
// forms M x^e .. M x^(e+3) itself (a shift by e and three by one) and its
// entries as sums of those, in memory form (the conversion is linear).  No
// LDS is read; the fences only keep the compiler from moving table reads
// above the writes (a wave's LDS accesses complete in order).
__device__ __forceinline__ void build_table_wave(uint32_t *lds, uint32_t dst, const uint32_t (&m)[4]) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t p = lane >> 1, hb = lane & 1u;
    const uint32_t byte = 4u * (p >> 3) + ((p & 7u) >> 1), half = p & 1u;
    uint64_t lo, hi;
    to_poly(m, lo, hi);
    mulx_pow(lo, hi, 8u * byte + 4u - 4u * half);
    uint32_t vk[4][4];   // M x^(e + k), memory form
#pragma unroll
    for (int k = 0; k < 4; k++) {
        from_poly(lo, hi, vk[k]);
        mulx_small(lo, hi, 1);
    }
    // v = 8 hb + j: bit 3 (t = 3) takes M x^e, bit 2 M x^(e+1), bit 1 M x^(e+2), bit 0 M x^(e+3)
    uint32_t base[4];
#pragma unroll
    for (int c = 0; c < 4; c++)
        base[c] = hb ? vk[0][c] : 0u;
#pragma unroll
    for (uint32_t j = 0; j < 8; j++) {
        uint32_t e[4];
#pragma unroll
        for (int c = 0; c < 4; c++)
            e[c] = base[c] ^ ((j & 1u) ? vk[3][c] : 0u) ^ ((j & 2u) ? vk[2][c] : 0u) ^ ((j & 4u) ? vk[1][c] : 0u);
        lds_store16(lds, dst + p * 256u + (8u * hb + j) * 16u, vec4(e[0], e[1], e[2], e[3]));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace
}  // namespace aesgpu
