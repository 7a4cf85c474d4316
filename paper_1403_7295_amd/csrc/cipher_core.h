// Device-side building blocks shared by the buffer kernels and the batch
// kernels: LDS table staging, table lookups, the AES rounds, 16-byte loads
// and stores, and the loop that carries a range of blocks through the cipher.
//
// One thread carries BPT independent 16-byte blocks through all rounds; a
// wave's 64 lanes hold 64 consecutive blocks per slot, so every global load
// and store is one 16-byte-per-lane, fully coalesced access (1 KiB per wave).
// The grid is persistent: a fixed number of workgroups sweeps the buffer, so
// the round tables are staged into LDS once per workgroup and not once per
// tile.
//
// A full round (SubBytes, ShiftRows, MixColumns, AddRoundKey; FIPS-197
// sections 5.1.1 - 5.1.4) is computed per output column c as
//     T0[s_c.b0] ^ T1[s_{c+1}.b1] ^ T2[s_{c+2}.b2] ^ T3[s_{c+3}.b3] ^ k_c
// where s_c is column c as a little-endian word (row r in byte r) and Ti is
// the table of row i: the column that MixColumns makes of S[x] placed in
// row i (so T_i is T0 rotated left by 8i bits).  Decryption uses the
// equivalent inverse cipher (FIPS-197 section 5.3.5): the same shape with
// the inverse tables, ShiftRows taken the other way (s_{c-r}) and the
// decryption key schedule.
//
// LDS layout.  A lookup by a random byte from 64 lanes would pile onto a few
// LDS banks, so every table entry is stored once per bank: the copy a lane
// reads always sits in that lane's own bank, and no two lanes of a
// half-wave ever collide.  The byte address of entry x is built by ONE
// v_perm_b32 from the state word (which supplies x as byte 1 of the
// address) and a per-lane constant (which supplies the copy offset in byte 0
// and the table bank in byte 2):
//   layout T4X32: four tables, 32 copies;  addr = pair<<16 | x<<8 | (t&1)<<7 | (lane&31)<<2
//   layout T2X64: two tables (T0, T1), 64 copies; addr = t<<16 | x<<8 | lane<<2,
//                 and T2, T3 are T0, T1 rotated by 16 bits.
//   layout T1X64: T0 alone, 64 copies;  addr = x<<8 | lane<<2, and T1, T2, T3
//                 are T0 rotated by 8, 16, 24 bits (three rotations per
//                 column): 64 KiB, so two 1024-thread workgroups fit on a
//                 compute unit.
//   layout T4X1:  four tables, one copy each (4 KiB, no replication):
//                 addr = t<<10 | x<<2; lanes collide on banks whenever their
//                 bytes agree modulo the bank count.
// T4X32 and T2X64 use 128 KiB.  Decryption adds the inverse S-box for the
// last round (32 copies, 32 KiB) after the round tables: at 0x20000 (a
// decryption workgroup then uses all 160 KiB), 0x10000 for T1X64 and 0x1000
// for T4X1.
// The last encryption round reads S[x] out of the round tables (byte 2 of
// T0[x] and byte 3 of T1[x] are S[x]) and assembles the column with two
// v_perm_b32.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace aesgpu {

// te0 | td0 | isw, 256 words each, uploaded from the host tables once per
// device.  Each translation unit that includes this header has its own copy
// and uploads it with upload_base_tables().
static __device__ uint32_t g_base[768];

namespace {

constexpr uint32_t kInvSboxWords = 8192;      // 32 KiB: inverse S-box, 32 copies

// Words of round tables, and the byte address of the inverse S-box after them.
template <int LAYOUT>
constexpr uint32_t table_words() {
    return LAYOUT == LAYOUT_T1X64 ? 16384u : LAYOUT == LAYOUT_T4X1 ? 1024u : 32768u;
}
template <int LAYOUT>
constexpr uint32_t inv_sbox_addr() { return table_words<LAYOUT>() * 4u; }

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // a ^ b ^ c in one VALU op
}

__device__ __forceinline__ uint32_t rotl(uint32_t x, int n) {
    return n == 0 ? x : (x << n) | (x >> (32 - n));
}

__device__ __forceinline__ uint32_t bswap(uint32_t x) {
    return __builtin_amdgcn_perm(0u, x, 0x00010203u);
}

// Byte address of a table entry: byte 0 and byte 2 from the lane constant,
// byte 1 = byte K of the state word, byte 3 = 0.
template <int K>
__device__ __forceinline__ uint32_t entry_addr(uint32_t w, uint32_t lane_const) {
    return __builtin_amdgcn_perm(w, lane_const, 0x0C010400u | (uint32_t(K) << 8));
}

__device__ __forceinline__ uint32_t lds_word(const uint32_t *lds, uint32_t byte_addr) {
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(lds) + byte_addr);
}

struct LaneConsts {
    uint32_t t[4];   // per physical table
    uint32_t isb;    // inverse S-box (address is built shifted left by one)
};

template <int LAYOUT>
__device__ __forceinline__ LaneConsts lane_consts(uint32_t lane) {
    LaneConsts c;
    if (LAYOUT == LAYOUT_T4X32) {
        for (int t = 0; t < 4; t++)
            c.t[t] = ((lane & 31u) << 2) | (uint32_t(t & 1) << 7) | (uint32_t(t >> 1) << 8);
    } else if (LAYOUT == LAYOUT_T2X64) {
        for (int t = 0; t < 4; t++)
            c.t[t] = (lane << 2) | (uint32_t(t & 1) << 8);
    } else if (LAYOUT == LAYOUT_T1X64) {
        for (int t = 0; t < 4; t++)
            c.t[t] = lane << 2;
    } else {
        for (int t = 0; t < 4; t++)
            c.t[t] = uint32_t(t) << 10;   // the table's base address
    }
    // inverse S-box, 32 copies after the round tables: the address is built
    // as (x<<8 | (lane&31)<<3 | base<<1) and halved, giving
    // base | x<<7 | (lane&31)<<2 (base<<1 sits in byte 2 for the 64 and 128
    // KiB layouts; for T4X1 the table's base is added after halving)
    constexpr uint32_t base = inv_sbox_addr<LAYOUT>();
    c.isb = ((lane & 31u) << 3) | (LAYOUT == LAYOUT_T4X1 ? 0u : (base >> 15) << 8);
    return c;
}

// Byte address of entry (byte K of w) of physical table T in the unreplicated layout.
template <int K>
__device__ __forceinline__ uint32_t flat_addr(uint32_t w, uint32_t table_base) {
    return table_base | (((w >> (8 * K)) & 255u) << 2);
}

// Logical table T (0..3) looked up with byte K of w.
template <int LAYOUT, int T, int K>
__device__ __forceinline__ uint32_t tl(const uint32_t *lds, const LaneConsts &lc, uint32_t w) {
    if (LAYOUT == LAYOUT_T4X32) {
        return lds_word(lds, entry_addr<K>(w, lc.t[T]));
    } else if (LAYOUT == LAYOUT_T2X64) {
        uint32_t v = lds_word(lds, entry_addr<K>(w, lc.t[T & 1]));
        return (T >> 1) ? rotl(v, 16) : v;
    } else if (LAYOUT == LAYOUT_T1X64) {
        return rotl(lds_word(lds, entry_addr<K>(w, lc.t[0])), 8 * T);
    } else {
        return lds_word(lds, flat_addr<K>(w, lc.t[T]));
    }
}

// The entry of the row-0 table (T0, or Td0 in the decryption layouts)
// looked up with byte K of w, unrotated; T1 is its rotation by 8 bits.
template <int LAYOUT, int K>
__device__ __forceinline__ uint32_t t0_entry(const uint32_t *lds, const LaneConsts &lc, uint32_t w) {
    return LAYOUT == LAYOUT_T4X1 ? lds_word(lds, flat_addr<K>(w, lc.t[0])) : lds_word(lds, entry_addr<K>(w, lc.t[0]));
}
template <int LAYOUT, int K>
__device__ __forceinline__ uint32_t t1_entry(const uint32_t *lds, const LaneConsts &lc, uint32_t w) {
    return LAYOUT == LAYOUT_T4X1 ? lds_word(lds, flat_addr<K>(w, lc.t[1])) : lds_word(lds, entry_addr<K>(w, lc.t[1]));
}

template <int LAYOUT, int K>
__device__ __forceinline__ uint32_t inv_sbox_word(const uint32_t *lds, const LaneConsts &lc, uint32_t w) {
    if (LAYOUT == LAYOUT_T4X1)
        return lds_word(lds, inv_sbox_addr<LAYOUT>() + (entry_addr<K>(w, lc.isb) >> 1));
    return lds_word(lds, entry_addr<K>(w, lc.isb) >> 1);
}

// One full round for one output column: the four bytes come from columns
// a, b, c, d (already ShiftRows-selected by the caller).
template <int LAYOUT>
__device__ __forceinline__ uint32_t round_col(const uint32_t *lds, const LaneConsts &lc, uint32_t a,
                                              uint32_t b, uint32_t c, uint32_t d, uint32_t k) {
    if (LAYOUT == LAYOUT_T4X32 || LAYOUT == LAYOUT_T1X64 || LAYOUT == LAYOUT_T4X1) {
        return xor3(tl<LAYOUT, 0, 0>(lds, lc, a), tl<LAYOUT, 1, 1>(lds, lc, b),
                    xor3(tl<LAYOUT, 2, 2>(lds, lc, c), tl<LAYOUT, 3, 3>(lds, lc, d), k));
    } else {
        // T2 ^ T3 = rotl16(T0' ^ T1'): one rotation per column
        uint32_t hi = lds_word(lds, entry_addr<2>(c, lc.t[0])) ^ lds_word(lds, entry_addr<3>(d, lc.t[1]));
        return xor3(tl<LAYOUT, 0, 0>(lds, lc, a), tl<LAYOUT, 1, 1>(lds, lc, b), k) ^ rotl(hi, 16);
    }
}

// Last encryption round for one column: S[a.b0] | S[b.b1]<<8 | S[c.b2]<<16 | S[d.b3]<<24, ^ k.
template <int LAYOUT>
__device__ __forceinline__ uint32_t final_enc_col(const uint32_t *lds, const LaneConsts &lc, uint32_t a,
                                                  uint32_t b, uint32_t c, uint32_t d, uint32_t k) {
    // physical tables 0 and 1 are T0 and T1 (T1X64: table 0 is T0 for all)
    uint32_t ea = t0_entry<LAYOUT, 0>(lds, lc, a);
    uint32_t eb = t1_entry<LAYOUT, 1>(lds, lc, b);
    uint32_t ec = t0_entry<LAYOUT, 2>(lds, lc, c);
    uint32_t ed = t1_entry<LAYOUT, 3>(lds, lc, d);
    if (LAYOUT == LAYOUT_T1X64) {
        // S from byte 2 of every T0 entry
        uint32_t lo = __builtin_amdgcn_perm(ea, eb, 0x0C0C0206u);
        uint32_t hi = __builtin_amdgcn_perm(ec, ed, 0x02060C0Cu);
        return xor3(lo, hi, k);
    }
    uint32_t lo = __builtin_amdgcn_perm(ea, eb, 0x0C0C0306u);  // S from byte 2 of T0, byte 3 of T1
    uint32_t hi = __builtin_amdgcn_perm(ec, ed, 0x03060C0Cu);
    return xor3(lo, hi, k);
}

template <int LAYOUT>
__device__ __forceinline__ uint32_t final_dec_col(const uint32_t *lds, const LaneConsts &lc, uint32_t a,
                                                  uint32_t b, uint32_t c, uint32_t d, uint32_t k) {
    uint32_t ea = inv_sbox_word<LAYOUT, 0>(lds, lc, a);
    uint32_t eb = inv_sbox_word<LAYOUT, 1>(lds, lc, b);
    uint32_t ec = inv_sbox_word<LAYOUT, 2>(lds, lc, c);
    uint32_t ed = inv_sbox_word<LAYOUT, 3>(lds, lc, d);
    uint32_t lo = __builtin_amdgcn_perm(ea, eb, 0x0C0C0104u);
    uint32_t hi = __builtin_amdgcn_perm(ec, ed, 0x03060C0Cu);
    return xor3(lo, hi, k);
}

template <int NR, int DIR, int LAYOUT, int BPT>
__device__ __forceinline__ void rounds(uint32_t (&s)[BPT][4], const uint32_t *lds, const LaneConsts &lc,
                                       const uint32_t *rk, int first_round) {
#pragma unroll
    for (int r = 1; r < NR; r++) {
        if (r < first_round)
            continue;
        const uint32_t k0 = rk[4 * r], k1 = rk[4 * r + 1], k2 = rk[4 * r + 2], k3 = rk[4 * r + 3];
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint32_t a0 = s[i][0], a1 = s[i][1], a2 = s[i][2], a3 = s[i][3];
            if (DIR == DIR_ENC) {
                s[i][0] = round_col<LAYOUT>(lds, lc, a0, a1, a2, a3, k0);
                s[i][1] = round_col<LAYOUT>(lds, lc, a1, a2, a3, a0, k1);
                s[i][2] = round_col<LAYOUT>(lds, lc, a2, a3, a0, a1, k2);
                s[i][3] = round_col<LAYOUT>(lds, lc, a3, a0, a1, a2, k3);
            } else {
                s[i][0] = round_col<LAYOUT>(lds, lc, a0, a3, a2, a1, k0);
                s[i][1] = round_col<LAYOUT>(lds, lc, a1, a0, a3, a2, k1);
                s[i][2] = round_col<LAYOUT>(lds, lc, a2, a1, a0, a3, k2);
                s[i][3] = round_col<LAYOUT>(lds, lc, a3, a2, a1, a0, k3);
            }
        }
    }
    const uint32_t k0 = rk[4 * NR], k1 = rk[4 * NR + 1], k2 = rk[4 * NR + 2], k3 = rk[4 * NR + 3];
#pragma unroll
    for (int i = 0; i < BPT; i++) {
        const uint32_t a0 = s[i][0], a1 = s[i][1], a2 = s[i][2], a3 = s[i][3];
        if (DIR == DIR_ENC) {
            s[i][0] = final_enc_col<LAYOUT>(lds, lc, a0, a1, a2, a3, k0);
            s[i][1] = final_enc_col<LAYOUT>(lds, lc, a1, a2, a3, a0, k1);
            s[i][2] = final_enc_col<LAYOUT>(lds, lc, a2, a3, a0, a1, k2);
            s[i][3] = final_enc_col<LAYOUT>(lds, lc, a3, a0, a1, a2, k3);
        } else {
            s[i][0] = final_dec_col<LAYOUT>(lds, lc, a0, a3, a2, a1, k0);
            s[i][1] = final_dec_col<LAYOUT>(lds, lc, a1, a0, a3, a2, k1);
            s[i][2] = final_dec_col<LAYOUT>(lds, lc, a2, a1, a0, a3, k2);
            s[i][3] = final_dec_col<LAYOUT>(lds, lc, a3, a2, a1, a0, k3);
        }
    }
}

// One AES encryption with the round table read from the base table in
// global memory (through the vector L1), for the few blocks a kernel
// encrypts outside its LDS tables: XTS tweaks while the LDS holds the
// inverse tables, GCM's hash key and pre-counter block.
template <int NR>
__device__ __forceinline__ void encrypt_global(const uint32_t *rk, uint32_t (&s)[4]) {
    const uint32_t *te0 = g_base;
    auto T = [&](int t, uint32_t w, int k) { return rotl(te0[(w >> (8 * k)) & 255u], 8 * t); };
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
    // last round: S[x] is byte 1 of te0[x]
    auto S = [&](uint32_t w, int k) { return (te0[(w >> (8 * k)) & 255u] >> 8) & 255u; };
    s[0] = (S(a0, 0) | (S(a1, 1) << 8) | (S(a2, 2) << 16) | (S(a3, 3) << 24)) ^ rk[4 * NR];
    s[1] = (S(a1, 0) | (S(a2, 1) << 8) | (S(a3, 2) << 16) | (S(a0, 3) << 24)) ^ rk[4 * NR + 1];
    s[2] = (S(a2, 0) | (S(a3, 1) << 8) | (S(a0, 2) << 16) | (S(a1, 3) << 24)) ^ rk[4 * NR + 2];
    s[3] = (S(a3, 0) | (S(a0, 1) << 8) | (S(a1, 2) << 16) | (S(a2, 3) << 24)) ^ rk[4 * NR + 3];
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 vec4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    u32x4 v;
    v.x = a; v.y = b; v.z = c; v.w = d;
    return v;
}

// Fills the LDS tables from the 1 KiB base tables.  Words i..i+3 of a table
// are copies of the same entry in neighbouring banks (the copy index is the
// low bits of i), so every thread writes four of them with one 16-byte store.
template <int LAYOUT, int DIR>
__device__ __forceinline__ void stage_tables(uint32_t *lds) {
    const uint32_t *base = g_base + (DIR == DIR_ENC ? 0 : 256);
    for (uint32_t i = 4 * threadIdx.x; i < table_words<LAYOUT>(); i += 4 * blockDim.x) {
        // word index i = table<<14 | x<<6 | copy (T2X64),
        //                pair<<14 | x<<6 | (t&1)<<5 | copy (T4X32),
        //                x<<6 | copy (T1X64), table<<8 | x (T4X1)
        uint32_t x, t;
        if (LAYOUT == LAYOUT_T4X1) {
            x = i & 255u;
            t = i >> 8;
            *reinterpret_cast<u32x4 *>(lds + i) = vec4(rotl(base[x], 8 * int(t)), rotl(base[x + 1], 8 * int(t)),
                                                        rotl(base[x + 2], 8 * int(t)), rotl(base[x + 3], 8 * int(t)));
            continue;
        }
        x = (i >> 6) & 255u;
        t = LAYOUT == LAYOUT_T4X32 ? (((i >> 14) << 1) | ((i >> 5) & 1u)) : LAYOUT == LAYOUT_T2X64 ? (i >> 14) : 0u;
        const uint32_t v = rotl(base[x], 8 * int(t));
        *reinterpret_cast<u32x4 *>(lds + i) = vec4(v, v, v, v);
    }
    if (DIR == DIR_DEC) {
        for (uint32_t i = 4 * threadIdx.x; i < kInvSboxWords; i += 4 * blockDim.x) {
            const uint32_t v = g_base[512 + (i >> 5)];
            *reinterpret_cast<u32x4 *>(lds + (inv_sbox_addr<LAYOUT>() >> 2) + i) = vec4(v, v, v, v);
        }
    }
}

// Streaming 16-byte accesses: every byte is touched exactly once, so they are
// marked non-temporal to keep them from evicting the (reused) table lines.
__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
}

__device__ __forceinline__ void store16(uint8_t *p, u32x4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
}

// The partial final block of a CTR message, one byte at a time.
__device__ __forceinline__ u32x4 load_tail(const uint8_t *p, uint32_t n) {
    uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
    for (uint32_t b = 0; b < 16; b++)
        if (b < n)
            w[b >> 2] |= uint32_t(p[b]) << (8 * (b & 3));
    return vec4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ void store_tail(uint8_t *p, u32x4 v, uint32_t n) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (uint32_t b = 0; b < 16; b++)
        if (b < n)
            p[b] = uint8_t(w[b >> 2] >> (8 * (b & 3)));
}

// min(v, 64 * BPT) for a 64-bit v, written on 32-bit halves (the scalar unit
// has no 64-bit less-than).
template <int BPT>
__device__ __forceinline__ uint32_t clamp_step(uint64_t v) {
    const uint32_t hi = uint32_t(v >> 32), lo = uint32_t(v);
    return (hi != 0 || lo > 64u * BPT) ? 64u * BPT : lo;
}

// Carries blocks j = base + 64*i + lane (i < BPT) through the cipher for
// every wave-uniform base in [begin, end) stepping by `step`; only blocks
// below `limit` exist.  Blocks are 16-byte units of a message of `nbytes`
// bytes at `in` / `out`; in CTR a final partial block is read and written
// byte by byte.  `rk` points at the round keys in the order the rounds use
// them (wave-uniform, so they are read into scalar registers); `ctr` holds
// the nonce words 0..2 and the initial counter value c0.
template <int NR, int MODE, int DIR, int LAYOUT, int BPT>
__device__ __forceinline__ void process_blocks(const uint32_t *lds, const LaneConsts &lc,
                                               const uint32_t *rk, const uint32_t *ctr,
                                               const uint8_t *in, uint8_t *out, uint64_t nbytes,
                                               uint64_t begin, uint64_t limit, uint64_t step) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t nfull = nbytes >> 4;
    const uint32_t tail = uint32_t(nbytes & 15u);
    // The loop below assumes `step` >= 64 * BPT: each step is a private
    // range of at most 64 * BPT blocks for the wave.

    // CTR: after the first AddRoundKey, columns 0..2 of every counter block
    // are the same (the nonce), so 12 of round 1's 16 lookups are the same
    // for every block; they are summed once here.
    uint32_t pre0 = 0, pre1 = 0, pre2 = 0, pre3 = 0;
    if (MODE == MODE_CTR) {
        const uint32_t u0 = ctr[0] ^ rk[0], u1 = ctr[1] ^ rk[1], u2 = ctr[2] ^ rk[2];
        pre0 = tl<LAYOUT, 0, 0>(lds, lc, u0) ^ tl<LAYOUT, 1, 1>(lds, lc, u1) ^ tl<LAYOUT, 2, 2>(lds, lc, u2) ^ rk[4];
        pre1 = tl<LAYOUT, 0, 0>(lds, lc, u1) ^ tl<LAYOUT, 1, 1>(lds, lc, u2) ^ tl<LAYOUT, 3, 3>(lds, lc, u0) ^ rk[5];
        pre2 = tl<LAYOUT, 0, 0>(lds, lc, u2) ^ tl<LAYOUT, 2, 2>(lds, lc, u0) ^ tl<LAYOUT, 3, 3>(lds, lc, u1) ^ rk[6];
        pre3 = tl<LAYOUT, 1, 1>(lds, lc, u0) ^ tl<LAYOUT, 2, 2>(lds, lc, u1) ^ tl<LAYOUT, 3, 3>(lds, lc, u2) ^ rk[7];
    }
    const uint32_t c0 = MODE == MODE_CTR ? ctr[3] : 0u;

    for (uint64_t base = begin; base < limit; base += step) {
        // Wave-uniform per step: pointers to block `base` and how many blocks
        // from there exist (whole ones, and the index of a partial tail), so
        // every lane works with a 32-bit offset from a scalar base address.
        const uint8_t *inb = in + 16 * base;
        uint8_t *outb = out + 16 * base;
        const uint64_t room = limit - base;
        const uint64_t whole = nfull > base ? min(nfull, limit) - base : 0;
        const uint32_t nwhole = clamp_step<BPT>(whole);
        const uint32_t tail_at = (MODE == MODE_CTR && tail && nfull >= base && nfull - base < room &&
                                  clamp_step<BPT>(nfull - base) == uint32_t(nfull - base) &&
                                  uint32_t(nfull - base) < 64u * BPT)
                                     ? uint32_t(nfull - base) : 0xFFFFFFFFu;
        uint32_t s[BPT][4];
        u32x4 x[BPT];
        const uint32_t cstep = c0 + uint32_t(base);   // CTR: counter value of block `base`
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint32_t jj = uint32_t(i) * 64u + lane;
            x[i] = vec4(0, 0, 0, 0);
            if (jj < nwhole)
                x[i] = load16(inb + 16u * jj);
            else if (MODE == MODE_CTR && jj == tail_at)
                x[i] = load_tail(inb + 16u * jj, tail);
            if (MODE == MODE_ECB || MODE == MODE_CBC) {
                s[i][0] = x[i].x ^ rk[0];
                s[i][1] = x[i].y ^ rk[1];
                s[i][2] = x[i].z ^ rk[2];
                s[i][3] = x[i].w ^ rk[3];
            }
        }
        if (MODE == MODE_ECB || MODE == MODE_CBC) {
            rounds<NR, DIR, LAYOUT, BPT>(s, lds, lc, rk, 1);
        } else if (((cstep & 255u) + 64u * BPT) <= 256u) {
            // All counters of this step share bytes 0..2 (the top 24 bits of
            // c0 + j): columns 1..3 after round 1 are the same for every
            // block, and so are 12 of round 2's 16 lookups.  Those 15
            // lookups are done once for the step; each block needs one
            // lookup in round 1 and four in round 2.
            const uint32_t g3 = bswap(cstep) ^ rk[3];
            const uint32_t t1 = pre1 ^ tl<LAYOUT, 2, 2>(lds, lc, g3);
            const uint32_t t2 = pre2 ^ tl<LAYOUT, 1, 1>(lds, lc, g3);
            const uint32_t t3 = pre3 ^ tl<LAYOUT, 0, 0>(lds, lc, g3);
            const uint32_t q0 = tl<LAYOUT, 1, 1>(lds, lc, t1) ^ tl<LAYOUT, 2, 2>(lds, lc, t2) ^ tl<LAYOUT, 3, 3>(lds, lc, t3) ^ rk[8];
            const uint32_t q1 = tl<LAYOUT, 0, 0>(lds, lc, t1) ^ tl<LAYOUT, 1, 1>(lds, lc, t2) ^ tl<LAYOUT, 2, 2>(lds, lc, t3) ^ rk[9];
            const uint32_t q2 = tl<LAYOUT, 0, 0>(lds, lc, t2) ^ tl<LAYOUT, 1, 1>(lds, lc, t3) ^ tl<LAYOUT, 3, 3>(lds, lc, t1) ^ rk[10];
            const uint32_t q3 = tl<LAYOUT, 0, 0>(lds, lc, t3) ^ tl<LAYOUT, 2, 2>(lds, lc, t1) ^ tl<LAYOUT, 3, 3>(lds, lc, t2) ^ rk[11];
#pragma unroll
            for (int i = 0; i < BPT; i++) {
                const uint32_t v3 = bswap(cstep + uint32_t(i) * 64u + lane) ^ rk[3];
                const uint32_t t0 = pre0 ^ tl<LAYOUT, 3, 3>(lds, lc, v3);
                s[i][0] = q0 ^ tl<LAYOUT, 0, 0>(lds, lc, t0);
                s[i][1] = q1 ^ tl<LAYOUT, 3, 3>(lds, lc, t0);
                s[i][2] = q2 ^ tl<LAYOUT, 2, 2>(lds, lc, t0);
                s[i][3] = q3 ^ tl<LAYOUT, 1, 1>(lds, lc, t0);
            }
            rounds<NR, DIR, LAYOUT, BPT>(s, lds, lc, rk, 3);
        } else if (BPT == 4) {
            // The step's 256 counters cross one multiple of 256: the blocks
            // before it share their top 24 bits (A), the others the next
            // value (B, mod 2^24).  The 15 shared lookups are done for both,
            // and each block takes its own set: 30 lookups for the step
            // instead of 15 per block.
            auto shared = [&](uint32_t g3, uint32_t (&q)[4]) __attribute__((always_inline)) {
                const uint32_t t1 = pre1 ^ tl<LAYOUT, 2, 2>(lds, lc, g3);
                const uint32_t t2 = pre2 ^ tl<LAYOUT, 1, 1>(lds, lc, g3);
                const uint32_t t3 = pre3 ^ tl<LAYOUT, 0, 0>(lds, lc, g3);
                q[0] = tl<LAYOUT, 1, 1>(lds, lc, t1) ^ tl<LAYOUT, 2, 2>(lds, lc, t2) ^ tl<LAYOUT, 3, 3>(lds, lc, t3) ^ rk[8];
                q[1] = tl<LAYOUT, 0, 0>(lds, lc, t1) ^ tl<LAYOUT, 1, 1>(lds, lc, t2) ^ tl<LAYOUT, 2, 2>(lds, lc, t3) ^ rk[9];
                q[2] = tl<LAYOUT, 0, 0>(lds, lc, t2) ^ tl<LAYOUT, 1, 1>(lds, lc, t3) ^ tl<LAYOUT, 3, 3>(lds, lc, t1) ^ rk[10];
                q[3] = tl<LAYOUT, 0, 0>(lds, lc, t3) ^ tl<LAYOUT, 2, 2>(lds, lc, t1) ^ tl<LAYOUT, 3, 3>(lds, lc, t2) ^ rk[11];
            };
            uint32_t qa[4], qb[4];
            shared(bswap(cstep) ^ rk[3], qa);
            shared(bswap(cstep + 256u) ^ rk[3], qb);
            const uint32_t lo = cstep & 255u;
#pragma unroll
            for (int i = 0; i < BPT; i++) {
                const uint32_t jj = uint32_t(i) * 64u + lane;
                const bool b = lo + jj >= 256u;
                const uint32_t v3 = bswap(cstep + jj) ^ rk[3];
                const uint32_t t0 = pre0 ^ tl<LAYOUT, 3, 3>(lds, lc, v3);
                s[i][0] = (b ? qb[0] : qa[0]) ^ tl<LAYOUT, 0, 0>(lds, lc, t0);
                s[i][1] = (b ? qb[1] : qa[1]) ^ tl<LAYOUT, 3, 3>(lds, lc, t0);
                s[i][2] = (b ? qb[2] : qa[2]) ^ tl<LAYOUT, 2, 2>(lds, lc, t0);
                s[i][3] = (b ? qb[3] : qa[3]) ^ tl<LAYOUT, 1, 1>(lds, lc, t0);
            }
            rounds<NR, DIR, LAYOUT, BPT>(s, lds, lc, rk, 3);
        } else {
            // counter block j: nonce || big-endian (c0 + j) mod 2^32;
            // round 1 needs only the four lookups on column 3.
#pragma unroll
            for (int i = 0; i < BPT; i++) {
                const uint32_t v3 = bswap(cstep + uint32_t(i) * 64u + lane) ^ rk[3];
                s[i][0] = pre0 ^ tl<LAYOUT, 3, 3>(lds, lc, v3);
                s[i][1] = pre1 ^ tl<LAYOUT, 2, 2>(lds, lc, v3);
                s[i][2] = pre2 ^ tl<LAYOUT, 1, 1>(lds, lc, v3);
                s[i][3] = pre3 ^ tl<LAYOUT, 0, 0>(lds, lc, v3);
            }
            rounds<NR, DIR, LAYOUT, BPT>(s, lds, lc, rk, 2);
        }
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint32_t jj = uint32_t(i) * 64u + lane;
            u32x4 o;
            if (MODE == MODE_ECB) {
                o = vec4(s[i][0], s[i][1], s[i][2], s[i][3]);
            } else if (MODE == MODE_CBC) {
                // CBC decryption: P_j = InvCipher(C_j) ^ C_{j-1}, C_{-1} = IV.
                // C_{j-1} is the neighbouring lane's input, moved one lane up
                // by a DPP wave shift (a VALU op: no second read of the data,
                // no LDS); lane 0 takes lane 63 of the previous slot, or for
                // the first slot the block before the step (the IV before
                // block 0), one wave-uniform load.
                u32x4 f;
                if (i == 0) {
                    f = vec4(ctr[0], ctr[1], ctr[2], ctr[3]);
                    if (base > 0)
                        f = load16(inb - 16);
                } else {
                    f = vec4(__builtin_amdgcn_readlane(x[i - 1].x, 63), __builtin_amdgcn_readlane(x[i - 1].y, 63),
                             __builtin_amdgcn_readlane(x[i - 1].z, 63), __builtin_amdgcn_readlane(x[i - 1].w, 63));
                }
                constexpr int kWaveShr1 = 0x138;   // lane l reads lane l - 1; lane 0 keeps `old`
                const u32x4 p = vec4(__builtin_amdgcn_update_dpp(f.x, x[i].x, kWaveShr1, 0xf, 0xf, false),
                                     __builtin_amdgcn_update_dpp(f.y, x[i].y, kWaveShr1, 0xf, 0xf, false),
                                     __builtin_amdgcn_update_dpp(f.z, x[i].z, kWaveShr1, 0xf, 0xf, false),
                                     __builtin_amdgcn_update_dpp(f.w, x[i].w, kWaveShr1, 0xf, 0xf, false));
                o = vec4(s[i][0] ^ p.x, s[i][1] ^ p.y, s[i][2] ^ p.z, s[i][3] ^ p.w);
            } else
                o = vec4(s[i][0] ^ x[i].x, s[i][1] ^ x[i].y, s[i][2] ^ x[i].z, s[i][3] ^ x[i].w);
            if (jj < nwhole)
                store16(outb + 16u * jj, o);
            else if (MODE == MODE_CTR && jj == tail_at)
                store_tail(outb + 16u * jj, o, tail);
        }
    }
}

// CBC encryption (SP 800-38A section 6.2): each block depends on the
// previous ciphertext, so a message is one chain.  The chain is serial but
// the plaintext is not: blocks are read a group of kCbcGroup ahead, so a
// group's loads are in flight while the previous group is enciphered and
// neither the read latency nor the completion of the last store stalls a
// block.
constexpr int kCbcGroup = 4;

// CBC encryption of one message by a quad of four lanes (lanes 4q .. 4q+3
// of a wave, all four active together): lane j of the quad holds column j
// of the state, looks up the four bytes of its own column (byte r in table
// r) and the round's output column i gathers table r's entry from lane
// i + r of the quad, a quad permute inside the XOR (DPP), so the sixteen
// lookups of a round are spread over four lanes instead of waiting in one.
// rk_col[r] is round key word 4r + j (this lane's column of round key r);
// iv_col is word j of the IV.  Plaintext words are read a group of
// kCbcGroup blocks ahead, as in the one-lane form.
// quad_perm controls: lane i of every quad reads lane i + 1, i + 2, i + 3 (mod 4)
constexpr int kQuadNext1 = 0x39, kQuadNext2 = 0x4E, kQuadNext3 = 0x93;
template <int QUAD_PERM>
__device__ __forceinline__ uint32_t quad_from(uint32_t v) {
    return uint32_t(__builtin_amdgcn_mov_dpp(int(v), QUAD_PERM, 0xF, 0xF, false));
}

template <int NR, int LAYOUT>
__device__ __forceinline__ void cbc_encrypt_quad(const uint32_t *lds, const LaneConsts &lc,
                                                 const uint32_t (&rk_col)[NR + 1], uint32_t iv_col,
                                                 const uint8_t *in, uint8_t *out, uint64_t nblocks) {
    const uint32_t j = threadIdx.x & 3u;
    uint32_t c = iv_col;
    uint32_t cur[kCbcGroup];
#pragma unroll
    for (int i = 0; i < kCbcGroup; i++)
        cur[i] = uint64_t(i) < nblocks ? *reinterpret_cast<const uint32_t *>(in + 16 * i + 4 * j) : 0u;
    for (uint64_t g = 0; g < nblocks; g += kCbcGroup) {
        uint32_t nxt[kCbcGroup];
#pragma unroll
        for (int i = 0; i < kCbcGroup; i++) {
            const uint64_t b = g + kCbcGroup + i;
            nxt[i] = b < nblocks ? *reinterpret_cast<const uint32_t *>(in + 16 * b + 4 * j) : 0u;
        }
#pragma unroll
        for (int i = 0; i < kCbcGroup; i++) {
            if (g + i < nblocks) {
                uint32_t s = cur[i] ^ c ^ rk_col[0];
#pragma unroll
                for (int r = 1; r < NR; r++) {
                    const uint32_t u0 = tl<LAYOUT, 0, 0>(lds, lc, s), u1 = tl<LAYOUT, 1, 1>(lds, lc, s);
                    const uint32_t u2 = tl<LAYOUT, 2, 2>(lds, lc, s), u3 = tl<LAYOUT, 3, 3>(lds, lc, s);
                    s = (((u0 ^ rk_col[r]) ^ quad_from<kQuadNext1>(u1)) ^ quad_from<kQuadNext2>(u2)) ^
                        quad_from<kQuadNext3>(u3);
                }
                // last round: S of byte r in byte r of the output column (T3
                // holds S in byte 0, T0 in bytes 1 and 2, T1 in byte 3)
                const uint32_t f0 = tl<LAYOUT, 3, 0>(lds, lc, s) & 0x000000FFu;
                const uint32_t f1 = tl<LAYOUT, 0, 1>(lds, lc, s) & 0x0000FF00u;
                const uint32_t f2 = tl<LAYOUT, 0, 2>(lds, lc, s) & 0x00FF0000u;
                const uint32_t f3 = tl<LAYOUT, 1, 3>(lds, lc, s) & 0xFF000000u;
                c = (((f0 ^ rk_col[NR]) ^ quad_from<kQuadNext1>(f1)) ^ quad_from<kQuadNext2>(f2)) ^
                    quad_from<kQuadNext3>(f3);
                *reinterpret_cast<uint32_t *>(out + 16 * (g + i) + 4 * j) = c;
            }
        }
#pragma unroll
        for (int i = 0; i < kCbcGroup; i++)
            cur[i] = nxt[i];
    }
}

template <int DIR, int LAYOUT = LAYOUT_T4X32>
constexpr uint32_t lds_words() {
    return DIR == DIR_DEC ? table_words<LAYOUT>() + kInvSboxWords : table_words<LAYOUT>();
}

}  // namespace

// Copies the host-built base tables into this translation unit's g_base on
// the current device.
static inline hipError_t upload_base_tables(const HostTables &t) {
    uint32_t words[768];
    for (int i = 0; i < 256; i++) {
        words[i] = t.te0[i];
        words[256 + i] = t.td0[i];
        words[512 + i] = t.isw[i];
    }
    return hipMemcpyToSymbol(HIP_SYMBOL(g_base), words, sizeof(words), 0, hipMemcpyHostToDevice);
}

}  // namespace aesgpu
