// GF(2^128) modulo x^128 + x^7 + x^2 + x + 1 on the device, for the XTS
// tweak (IEEE 1619) and GHASH (SP 800-38D section 6.3).
//
// Arithmetic form: a 128-bit little-endian integer whose bit i is the
// coefficient of x^i, held as two 64-bit halves (lo = bits 0..63).  This is
// XTS's own byte order; GCM's blocks store coefficient x^i in bit 7 - (i mod
// 8) of byte i / 8, so a GCM block becomes this form by reversing the bits
// of every byte (to_poly / from_poly).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace aesgpu {
namespace {

// v * x^b for 0 <= b < 64: a shift, and the bits that leave the top
// (o * x^128) folded back as o * (x^7 + x^2 + x + 1).
__device__ __forceinline__ void mulx_small(uint64_t &lo, uint64_t &hi, uint32_t b) {
    const uint32_t bb = b & 63u;
    const uint64_t o = bb ? hi >> (64 - bb) : 0;
    hi = bb ? (hi << bb) | (lo >> (64 - bb)) : hi;
    lo = lo << bb;
    // o has at most 63 bits, so o * (x^7 + x^2 + x + 1) stays below x^71
    lo ^= o ^ (o << 1) ^ (o << 2) ^ (o << 7);
    hi ^= (o >> 63) ^ (o >> 62) ^ (o >> 57);
}

// v * x^64.
__device__ __forceinline__ void mulx64(uint64_t &lo, uint64_t &hi) {
    const uint64_t o = hi;
    hi = lo ^ (o >> 63) ^ (o >> 62) ^ (o >> 57);
    lo = o ^ (o << 1) ^ (o << 2) ^ (o << 7);
}

// v * x^e for 0 <= e < 256.
__device__ __forceinline__ void mulx_pow(uint64_t &lo, uint64_t &hi, uint32_t e) {
    mulx_small(lo, hi, e & 63u);
    for (uint32_t q = e >> 6; q > 0; q--)
        mulx64(lo, hi);
}

// v * v.  Squaring is linear over GF(2): coefficient i moves to 2i (the bits
// spread out with zeros between them), and the upper 128 bits of the
// 255-bit result fold back through x^128 = x^7 + x^2 + x + 1.
__device__ __forceinline__ uint64_t spread32(uint32_t w) {
    uint64_t x = w;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ __forceinline__ void gf_square(uint64_t &lo, uint64_t &hi) {
    const uint64_t w0 = spread32(uint32_t(lo)), w1 = spread32(uint32_t(lo >> 32));
    const uint64_t a0 = spread32(uint32_t(hi)), a1 = spread32(uint32_t(hi >> 32));
    // (a1:a0) * (x^7 + x^2 + x + 1): its bits above x^127 (at most 7 of
    // them, o) fold back once more
    const uint64_t o = (a1 >> 63) ^ (a1 >> 62) ^ (a1 >> 57);
    lo = w0 ^ a0 ^ (a0 << 1) ^ (a0 << 2) ^ (a0 << 7) ^ o ^ (o << 1) ^ (o << 2) ^ (o << 7);
    hi = w1 ^ a1 ^ ((a1 << 1) | (a0 >> 63)) ^ ((a1 << 2) | (a0 >> 62)) ^ ((a1 << 7) | (a0 >> 57));
}

// A GCM block given as four little-endian words (bytes 0..15 in memory
// order) to the arithmetic form, and back: the bits of each byte reversed.
__device__ __forceinline__ uint32_t rev_bits_in_bytes(uint32_t w) {
    return __builtin_bitreverse32(__builtin_bswap32(w));
}

__device__ __forceinline__ void to_poly(const uint32_t (&w)[4], uint64_t &lo, uint64_t &hi) {
    lo = uint64_t(rev_bits_in_bytes(w[0])) | (uint64_t(rev_bits_in_bytes(w[1])) << 32);
    hi = uint64_t(rev_bits_in_bytes(w[2])) | (uint64_t(rev_bits_in_bytes(w[3])) << 32);
}

__device__ __forceinline__ void from_poly(uint64_t lo, uint64_t hi, uint32_t (&w)[4]) {
    w[0] = rev_bits_in_bytes(uint32_t(lo));
    w[1] = rev_bits_in_bytes(uint32_t(lo >> 32));
    w[2] = rev_bits_in_bytes(uint32_t(hi));
    w[3] = rev_bits_in_bytes(uint32_t(hi >> 32));
}

}  // namespace
}  // namespace aesgpu
