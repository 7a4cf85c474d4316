// Bitsliced AES for gfx950: the comparison variant of the table kernels.
//
// Each lane carries 32 blocks at once as 128 bit-planes: plane 32c + 8r + k
// holds, in its bit t, bit k of row r, column c of block t (column c is the
// little-endian word c of the block).  SubBytes is then a Boolean circuit
// applied to eight planes at a time, ShiftRows is a renaming of planes,
// MixColumns is XOR algebra on planes and AddRoundKey XORs each plane with
// all-zeros or all-ones.  No table and no data-dependent address is used, so
// the kernel needs no LDS and runs in constant time; the price is many more
// VALU operations per block than a table lookup costs.
//
// S-box circuit: Boyar and Peralta, "A depth-16 circuit for the AES S-box"
// (the published straight-line program: a linear top layer, a non-linear
// middle layer with 32 AND gates, and a linear bottom layer), restated here.
// Inputs u0..u7 are the byte's bits from most to least significant; so are
// the outputs.
//
// Blocks reach the bit-plane form by 32x32 bit-matrix transposes (the
// classic five-stage swap network), four per 32 blocks in and out.
// Encryption only (ECB and CTR); there is no inverse circuit here.
#include <hip/hip_runtime.h>

#include "cipher_core.h"
#include "internal.h"

namespace aesgpu {
namespace {

__device__ __forceinline__ void sbox_circuit(uint32_t &b7, uint32_t &b6, uint32_t &b5, uint32_t &b4,
                                             uint32_t &b3, uint32_t &b2, uint32_t &b1, uint32_t &b0) {
    const uint32_t U0 = b7, U1 = b6, U2 = b5, U3 = b4, U4 = b3, U5 = b2, U6 = b1, U7 = b0;
    // top linear layer
    const uint32_t T1 = U0 ^ U3, T2 = U0 ^ U5, T3 = U0 ^ U6, T4 = U3 ^ U5, T5 = U4 ^ U6;
    const uint32_t T6 = T1 ^ T5, T7 = U1 ^ U2, T8 = U7 ^ T6, T9 = U7 ^ T7, T10 = T6 ^ T7;
    const uint32_t T11 = U1 ^ U5, T12 = U2 ^ U5, T13 = T3 ^ T4, T14 = T6 ^ T11, T15 = T5 ^ T11;
    const uint32_t T16 = T5 ^ T12, T17 = T9 ^ T16, T18 = U3 ^ U7, T19 = T7 ^ T18, T20 = T1 ^ T19;
    const uint32_t T21 = U6 ^ U7, T22 = T7 ^ T21, T23 = T2 ^ T22, T24 = T2 ^ T10, T25 = T20 ^ T17;
    const uint32_t T26 = T3 ^ T16, T27 = T1 ^ T12;
    // non-linear middle layer
    const uint32_t M1 = T13 & T6, M2 = T23 & T8, M3 = T14 ^ M1, M4 = T19 & U7, M5 = M4 ^ M1;
    const uint32_t M6 = T3 & T16, M7 = T22 & T9, M8 = T26 ^ M6, M9 = T20 & T17, M10 = M9 ^ M6;
    const uint32_t M11 = T1 & T15, M12 = T4 & T27, M13 = M12 ^ M11, M14 = T2 & T10, M15 = M14 ^ M11;
    const uint32_t M16 = M3 ^ M2, M17 = M5 ^ T24, M18 = M8 ^ M7, M19 = M10 ^ M15, M20 = M16 ^ M13;
    const uint32_t M21 = M17 ^ M15, M22 = M18 ^ M13, M23 = M19 ^ T25, M24 = M22 ^ M23, M25 = M22 & M20;
    const uint32_t M26 = M21 ^ M25, M27 = M20 ^ M21, M28 = M23 ^ M25, M29 = M28 & M27, M30 = M26 & M24;
    const uint32_t M31 = M20 & M23, M32 = M27 & M31, M33 = M27 ^ M25, M34 = M21 & M22, M35 = M24 & M34;
    const uint32_t M36 = M24 ^ M25, M37 = M21 ^ M29, M38 = M32 ^ M33, M39 = M23 ^ M30, M40 = M35 ^ M36;
    const uint32_t M41 = M38 ^ M40, M42 = M37 ^ M39, M43 = M37 ^ M38, M44 = M39 ^ M40, M45 = M42 ^ M41;
    const uint32_t M46 = M44 & T6, M47 = M40 & T8, M48 = M39 & U7, M49 = M43 & T16, M50 = M38 & T9;
    const uint32_t M51 = M37 & T17, M52 = M42 & T15, M53 = M45 & T27, M54 = M41 & T10, M55 = M44 & T13;
    const uint32_t M56 = M40 & T23, M57 = M39 & T19, M58 = M43 & T3, M59 = M38 & T22, M60 = M37 & T20;
    const uint32_t M61 = M42 & T1, M62 = M45 & T4, M63 = M41 & T2;
    // bottom linear layer
    const uint32_t L0 = M61 ^ M62, L1 = M50 ^ M56, L2 = M46 ^ M48, L3 = M47 ^ M55, L4 = M54 ^ M58;
    const uint32_t L5 = M49 ^ M61, L6 = M62 ^ L5, L7 = M46 ^ L3, L8 = M51 ^ M59, L9 = M52 ^ M53;
    const uint32_t L10 = M53 ^ L4, L11 = M60 ^ L2, L12 = M48 ^ M51, L13 = M50 ^ L0, L14 = M52 ^ M61;
    const uint32_t L15 = M55 ^ L1, L16 = M56 ^ L0, L17 = M57 ^ L1, L18 = M58 ^ L8, L19 = M63 ^ L4;
    const uint32_t L20 = L0 ^ L1, L21 = L1 ^ L7, L22 = L3 ^ L12, L23 = L18 ^ L2, L24 = L15 ^ L9;
    const uint32_t L25 = L6 ^ L10, L26 = L7 ^ L9, L27 = L8 ^ L10, L28 = L11 ^ L14, L29 = L11 ^ L17;
    b7 = L6 ^ L24;
    b6 = ~(L16 ^ L26);
    b5 = ~(L19 ^ L28);
    b4 = L6 ^ L21;
    b3 = L20 ^ L22;
    b2 = L25 ^ L29;
    b1 = ~(L13 ^ L27);
    b0 = ~(L6 ^ L23);
}

// Transpose the 32x32 bit matrix a[row] (bit t of a[r] <-> bit r of a[t]).
__device__ __forceinline__ void transpose32(uint32_t (&a)[32]) {
    constexpr uint32_t masks[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int s = 0; s < 5; s++) {
        const int j = 16 >> s;
        const uint32_t m = masks[s];
#pragma unroll
        for (int k = 0; k < 32; k++) {
            if (k & j)
                continue;
            // swap the high j bits of the low half-rows with the low j bits of the high ones
            const uint32_t t = ((a[k] >> j) ^ a[k + j]) & m;
            a[k + j] ^= t;
            a[k] ^= t << j;
        }
    }
#pragma unroll
    for (int k = 0; k < 32; k++)
        asm volatile("" : "+v"(a[k]));
}

// Plane index of bit k of row r, column c.
__device__ __forceinline__ constexpr int P(int c, int r, int k) { return 32 * c + 8 * r + k; }

__device__ __forceinline__ void add_round_key(uint32_t (&st)[128], const uint32_t *rk) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const uint32_t w = rk[c];
#pragma unroll
        for (int b = 0; b < 32; b++)
            st[32 * c + b] ^= 0u - ((w >> b) & 1u);
    }
}

__device__ __forceinline__ void sub_bytes(uint32_t (&st)[128]) {
#pragma unroll
    for (int c = 0; c < 4; c++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            sbox_circuit(st[P(c, r, 7)], st[P(c, r, 6)], st[P(c, r, 5)], st[P(c, r, 4)], st[P(c, r, 3)],
                         st[P(c, r, 2)], st[P(c, r, 1)], st[P(c, r, 0)]);
            asm volatile("" : "+v"(st[P(c, r, 7)]), "+v"(st[P(c, r, 6)]), "+v"(st[P(c, r, 5)]), "+v"(st[P(c, r, 4)]),
                              "+v"(st[P(c, r, 3)]), "+v"(st[P(c, r, 2)]), "+v"(st[P(c, r, 1)]), "+v"(st[P(c, r, 0)]));
        }
}

// ShiftRows and MixColumns, in place.  Output column c takes row r from
// input column c + r; each input byte feeds exactly one output column, so
// output column c is written over the 32 planes it was computed from, and a
// final renaming of rows 1..3 restores the plane order (the compiler turns it
// into register moves, not memory traffic).
template <bool MIX>
__device__ __forceinline__ void shift_mix(uint32_t (&st)[128]) {
    if (MIX) {
#pragma unroll
        for (int c = 0; c < 4; c++) {
            uint32_t s[8];
#pragma unroll
            for (int k = 0; k < 8; k++)
                s[k] = st[P(c, 0, k)] ^ st[P((c + 1) & 3, 1, k)] ^ st[P((c + 2) & 3, 2, k)] ^
                       st[P((c + 3) & 3, 3, k)];
            uint32_t o[4][8];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                // out_r = a_r ^ s ^ xtime(a_r ^ a_{r+1}), s = a_0 ^ a_1 ^ a_2 ^ a_3;
                // xtime shifts up one bit and reduces by 0x1b (bits 0, 1, 3, 4)
                uint32_t t[8];
#pragma unroll
                for (int k = 0; k < 8; k++)
                    t[k] = st[P((c + r) & 3, r, k)] ^ st[P((c + r + 1) & 3, (r + 1) & 3, k)];
                const uint32_t x[8] = {t[7], t[0] ^ t[7], t[1], t[2] ^ t[7], t[3] ^ t[7], t[4], t[5], t[6]};
#pragma unroll
                for (int k = 0; k < 8; k++)
                    o[r][k] = st[P((c + r) & 3, r, k)] ^ s[k] ^ x[k];
            }
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    st[P((c + r) & 3, r, k)] = o[r][k];
                    asm volatile("" : "+v"(st[P((c + r) & 3, r, k)]));
                }
        }
    }
    // ShiftRows as a renaming: row r of column c now comes from column c + r
#pragma unroll
    for (int r = 1; r < 4; r++)
#pragma unroll
        for (int k = 0; k < 8; k++) {
            uint32_t v[4];
#pragma unroll
            for (int c = 0; c < 4; c++)
                v[c] = st[P((c + r) & 3, r, k)];
#pragma unroll
            for (int c = 0; c < 4; c++)
                st[P(c, r, k)] = v[c];
        }
}

// Encrypts the 32 blocks held as planes.
template <int NR>
__device__ __forceinline__ void encrypt_planes(uint32_t (&st)[128], const uint32_t *rk) {
    add_round_key(st, rk);
#pragma unroll 1
    for (int r = 1; r < NR; r++) {
        sub_bytes(st);
        shift_mix<true>(st);
        add_round_key(st, rk + 4 * r);
    }
    sub_bytes(st);
    shift_mix<false>(st);
    add_round_key(st, rk + 4 * NR);
}

// Every wave takes 2048 consecutive blocks per step: lane l holds blocks
// base + 64 t + l for t = 0..31.  Two waves per SIMD (256 registers each):
// the 128-plane state plus one S-box circuit's or one MixColumns column's
// temporaries.  Left to itself the compiler interleaves the 16 circuits of a
// round and spills; the empty asm statements after each circuit, each
// column and each transpose make it finish one before the next, and the
// store phase recomputes the block addresses (else the load phase's are kept
// live across the rounds), so nothing spills; the second wave hides the
// other's memory waits and fills the issue slots its scalar instructions
// leave.
template <int NR, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bitslice_kernel(const CipherArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t nfull = a.nbytes >> 4;
    const uint32_t tail = uint32_t(a.nbytes & 15u);
    const uint64_t nblk = nfull + (tail ? 1 : 0);
    const uint64_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint64_t nwaves = uint64_t(gridDim.x) * (blockDim.x >> 6);
    for (uint64_t base = wave * 2048u; base < nblk; base += nwaves * 2048u) {
        uint32_t st[128];
        if (MODE == MODE_ECB) {
            // one 16-byte load per block; word w of block t goes to st[32w + t],
            // then each word position is transposed in place
#pragma unroll
            for (int t = 0; t < 32; t++) {
                const uint64_t j = base + 64u * t + lane;
                u32x4 x = vec4(0, 0, 0, 0);
                if (j < nfull)
                    x = load16(a.in + 16 * j);
                st[t] = x.x;
                st[32 + t] = x.y;
                st[64 + t] = x.z;
                st[96 + t] = x.w;
            }
#pragma unroll
            for (int w = 0; w < 4; w++)
                transpose32(*reinterpret_cast<uint32_t(*)[32]>(st + 32 * w));
        } else {
            // counter blocks: words 0..2 are the nonce in every block (planes
            // of all zeros or all ones); only word 3 needs a transpose
#pragma unroll
            for (int w = 0; w < 3; w++)
#pragma unroll
                for (int b = 0; b < 32; b++)
                    st[32 * w + b] = 0u - ((a.ctr[w] >> b) & 1u);
            uint32_t col[32];
#pragma unroll
            for (int t = 0; t < 32; t++)
                col[t] = bswap(a.ctr[3] + uint32_t(base) + 64u * t + lane);
            transpose32(col);
#pragma unroll
            for (int b = 0; b < 32; b++)
                st[96 + b] = col[b];
        }
        encrypt_planes<NR>(st, a.rk);
        // back to blocks, word position by word position
#pragma unroll
        for (int w = 0; w < 4; w++)
            transpose32(*reinterpret_cast<uint32_t(*)[32]>(st + 32 * w));
        // the block addresses again from an opaque copy of the base, so the
        // compiler does not keep the load phase's ones live across the rounds
        uint64_t sbase = base;
        asm volatile("" : "+s"(sbase));
#pragma unroll
        for (int t = 0; t < 32; t++) {
            const uint64_t j = sbase + 64u * t + lane;
            u32x4 o = vec4(st[t], st[32 + t], st[64 + t], st[96 + t]);
            if (MODE == MODE_CTR) {
                if (j < nfull) {
                    const u32x4 x = load16(a.in + 16 * j);
                    o = vec4(o.x ^ x.x, o.y ^ x.y, o.z ^ x.z, o.w ^ x.w);
                } else if (j == nfull && tail) {
                    const u32x4 x = load_tail(a.in + 16 * j, tail);
                    store_tail(a.out + 16 * j, vec4(o.x ^ x.x, o.y ^ x.y, o.z ^ x.z, o.w ^ x.w), tail);
                }
            }
            if (j < nfull)
                store16(a.out + 16 * j, o);
        }
    }
}

}  // namespace

hipError_t launch_bitslice(int nr, int mode, int grid, const CipherArgs &a, hipStream_t stream) {
    void (*fn)(const CipherArgs);
    if (mode == MODE_CTR)
        fn = nr == 10 ? bitslice_kernel<10, MODE_CTR> : nr == 12 ? bitslice_kernel<12, MODE_CTR>
                                                                 : bitslice_kernel<14, MODE_CTR>;
    else
        fn = nr == 10 ? bitslice_kernel<10, MODE_ECB> : nr == 12 ? bitslice_kernel<12, MODE_ECB>
                                                                 : bitslice_kernel<14, MODE_ECB>;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace aesgpu
