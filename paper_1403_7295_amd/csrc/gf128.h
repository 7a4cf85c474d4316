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
