// AES-GCM (NIST SP 800-38D) for gfx950: CTR encryption fused with the GHASH
// authenticator in one pass over the data.
//
// Definitions (SP 800-38D sections 6 and 7).  H = Cipher_K(0^128).  The
// pre-counter block J0 is IV || 0^31 || 1 for a 96-bit IV and otherwise
// GHASH_H of the zero-padded IV followed by its bit length.  Ciphertext
// block j is P_j XOR Cipher_K(J0 + 1 + j), the count in the last 32 bits.
// The tag is Cipher_K(J0) XOR S, where S is GHASH_H over the sequence
// X_1 .. X_m = A (zero-padded) || C (zero-padded) || [len(A)]_64 [len(C)]_64,
// i.e. S = sum_i X_i * H^(m - i + 1) in GF(2^128).
//
// Evaluation order.  Number the sequence from its end, r = m - i, so that
// S = H * sum_r X_r * H^r: r = 0 is the length block, r = 1 .. nC the
// ciphertext blocks (block j at r = nC - j), then the additional data.
// The first `head` = (nC + 1) mod 64 positions (the length block and the
// last head - 1 ciphertext blocks) are left to the last kernel, so that the
// bulk's positions start at r = head, where every group of 64 positions
// covers 64 ciphertext blocks starting on a 1 KiB boundary: a wave's 16-byte
// stores then write whole 128-byte lines, none shared with another wave.
// The bulk's positions p = r - head are cut into chunks of 256 (64 lanes x
// 4 slots); wave w of NW takes chunks w, w + NW, w + 2 NW, ... from the last
// to the first, so every (lane, slot) stream is a Horner evaluation with the
// same multiplier G = H^(256 NW):  W <- W * G + X.  At the end a stream at
// offset s in its wave's first chunk needs the factor H^(s + 256 w); the
// streams are folded with factors H^64 (slots), H^1 .. H^32 (lanes, a
// tree), H^256 .. H^2048 (the 16 waves of a workgroup) and H^(4096 b)
// (workgroups, in the last kernel), giving B = sum_(r >= head) X_r H^(r -
// head).  The last kernel encrypts the head's blocks, adds them in, S = H *
// (sum_(r < head) X_r H^r + H^head * B).  Every factor is a power H^(2^t),
// computed once by the first kernel.
//
// Multiplication by a fixed element M uses 4-bit tables in LDS: for each of
// the 32 nibble positions of a block, the 16 products (nibble value at that
// position) * M, 16 bytes each (8 KiB per multiplier).  A product is 32
// 16-byte LDS reads XORed together.  A table of 256 bytes covers every LDS
// bank once, so the 64 lanes of a read never conflict (equal values are
// broadcast).  The bulk kernel keeps the AES encryption tables (128 KiB) and
// G's table; after its loop the AES tables' space holds the folding tables.
#include <hip/hip_runtime.h>

#include "cipher_core.h"
#include "gf128.h"
#include "ghash_core.h"
#include "internal.h"

namespace aesgpu {
namespace {

// LDS of the bulk kernel: G's tables at 0, the AES encryption tables at
// kAesBase (128 KiB), scratch for building G's tables after them.  After the
// loop: eleven folding tables from 0, their scratch, the wave partials.
constexpr uint32_t kGTab = 0;
constexpr uint32_t kAesBase = 0x2000;
constexpr uint32_t kGVec = kAesBase + 0x20000;
constexpr uint32_t kFoldTabs = 11;
constexpr uint32_t kFoldVec = kFoldTabs * kTabBytes;
constexpr uint32_t kWavePartials = kFoldVec + kFoldTabs * kVecBytes;

// One wave: H, J0, Cipher_K(J0) and the powers H^(2^t) that this launch's
// folding needs (t <= 12 + grid_log2).
template <int NR>
__global__ __launch_bounds__(64) void gcm_setup_kernel(const GcmArgs a) {
    __shared__ uint32_t t0[256];
    for (uint32_t i = threadIdx.x; i < 256; i += 64)
        t0[i] = g_base[i];
    __syncthreads();
    uint32_t h[4] = {0, 0, 0, 0};
    encrypt_one<NR>(t0, a.rk, h);
    uint64_t hlo, hhi;
    to_poly(h, hlo, hhi);
    uint32_t j0[4];
    if (a.iv_bytes == 12) {
        for (int c = 0; c < 3; c++)
            j0[c] = uint32_t(a.iv[4 * c]) | (uint32_t(a.iv[4 * c + 1]) << 8) |
                    (uint32_t(a.iv[4 * c + 2]) << 16) | (uint32_t(a.iv[4 * c + 3]) << 24);
        j0[3] = 0x01000000u;   // 0^31 || 1, big-endian
    } else {
        // GHASH_H(IV || 0^(s+64) || [len(IV)]_64)
        uint64_t ylo = 0, yhi = 0;
        const uint32_t nblk = (a.iv_bytes + 15u) / 16u;
        for (uint32_t b = 0; b <= nblk; b++) {
            uint32_t x[4] = {0, 0, 0, 0};
            if (b < nblk) {
                for (uint32_t i = 0; i < 16; i++)
                    if (16u * b + i < a.iv_bytes)
                        x[i >> 2] |= uint32_t(a.iv[16u * b + i]) << (8 * (i & 3));
            } else {
                const uint64_t bits = 8ull * a.iv_bytes;
                x[2] = __builtin_bswap32(uint32_t(bits >> 32));
                x[3] = __builtin_bswap32(uint32_t(bits));
            }
            uint64_t xlo, xhi;
            to_poly(x, xlo, xhi);
            mul_wave(ylo ^ xlo, yhi ^ xhi, hlo, hhi, ylo, yhi);
        }
        from_poly(ylo, yhi, j0);
    }
    uint32_t ej0[4] = {j0[0], j0[1], j0[2], j0[3]};
    encrypt_one<NR>(t0, a.rk, ej0);
    const bool writer = threadIdx.x == 0;
    uint64_t plo = hlo, phi = hhi;
    const int tmax = 12 + int(a.grid_log2);
    for (int t = 0; t <= tmax; t++) {
        if (writer) {
            uint32_t w[4];
            from_poly(plo, phi, w);
            for (int c = 0; c < 4; c++)
                a.ws->powers[t][c] = w[c];
        }
        gf_square(plo, phi);
    }
    if (writer)
        for (int c = 0; c < 4; c++) {
            a.ws->j0[c] = j0[c];
            a.ws->ej0[c] = ej0[c];
        }
}

template <int NR, bool DEC, int BPT>
__global__ __launch_bounds__(1024) void gcm_kernel(const GcmArgs a) {
    static_assert(BPT == 4, "a chunk is 64 lanes x 4 slots = 256 positions");
    __shared__ uint32_t lds[40960];   // 160 KiB
    uint32_t *aes = lds + kAesBase / 4;
    stage_tables<LAYOUT_T4X32, DIR_ENC>(aes);
    // G = H^(256 * 16 * gridDim.x), gridDim.x = 2^grid_log2
    const int gpow = 12 + int(a.grid_log2);
    build_tables(lds, kGTab, kGVec, 1, [&](int) { return a.ws->powers[gpow]; });

    const uint32_t lane = threadIdx.x & 63u;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(lane);
    const uint64_t nC = (a.nbytes + 15) >> 4, nA = (a.aad_bytes + 15) >> 4;
    // positions r < head belong to the last kernel (head <= nC + 1)
    const uint64_t head = (nC + 1) & 63u;
    const uint64_t nchunks = (nC + nA + 1 - head + 255) >> 8;
    const uint64_t cwhole = a.nbytes >> 4, awhole = a.aad_bytes >> 4;
    const uint32_t ctail = uint32_t(a.nbytes & 15u), atail = uint32_t(a.aad_bytes & 15u);
    const uint64_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint64_t nwaves = uint64_t(gridDim.x) * (blockDim.x >> 6);
    // counter blocks: J0's first 12 bytes, then the 32-bit count of J0 plus 1 + j
    const uint32_t n0 = a.ws->j0[0] ^ a.rk[0], n1 = a.ws->j0[1] ^ a.rk[1], n2 = a.ws->j0[2] ^ a.rk[2];
    const uint32_t c1 = __builtin_bswap32(a.ws->j0[3]) + 1u;
    // [len(A)]_64 || [len(C)]_64 in bits, big-endian
    const uint64_t abits = 8 * a.aad_bytes, cbits = 8 * a.nbytes;
    const uint32_t len[4] = {__builtin_bswap32(uint32_t(abits >> 32)), __builtin_bswap32(uint32_t(abits)),
                             __builtin_bswap32(uint32_t(cbits >> 32)), __builtin_bswap32(uint32_t(cbits))};
    // bytes of a partial last ciphertext block that enter GHASH
    uint32_t tmask[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int keep = int(ctail) - 4 * c;
        tmask[c] = keep >= 4 ? ~0u : keep <= 0 ? 0u : (1u << (8 * keep)) - 1u;
    }

    uint32_t W[BPT][4];
#pragma unroll
    for (int i = 0; i < BPT; i++)
        W[i][0] = W[i][1] = W[i][2] = W[i][3] = 0;
    // A chunk of 256 positions that are all whole ciphertext blocks: every
    // chunk but the one holding the length block and a partial block, and
    // those holding additional data.
    // Round 1 of a counter block: columns 0..2 are J0's first twelve bytes
    // after AddRoundKey, the same for every block, so 12 of its 16 lookups
    // are summed once here; a block adds the four on column 3.
    const uint32_t pre0 = tl<LAYOUT_T4X32, 0, 0>(aes, lc, n0) ^ tl<LAYOUT_T4X32, 1, 1>(aes, lc, n1) ^
                          tl<LAYOUT_T4X32, 2, 2>(aes, lc, n2) ^ a.rk[4];
    const uint32_t pre1 = tl<LAYOUT_T4X32, 0, 0>(aes, lc, n1) ^ tl<LAYOUT_T4X32, 1, 1>(aes, lc, n2) ^
                          tl<LAYOUT_T4X32, 3, 3>(aes, lc, n0) ^ a.rk[5];
    const uint32_t pre2 = tl<LAYOUT_T4X32, 0, 0>(aes, lc, n2) ^ tl<LAYOUT_T4X32, 2, 2>(aes, lc, n0) ^
                          tl<LAYOUT_T4X32, 3, 3>(aes, lc, n1) ^ a.rk[6];
    const uint32_t pre3 = tl<LAYOUT_T4X32, 1, 1>(aes, lc, n0) ^ tl<LAYOUT_T4X32, 2, 2>(aes, lc, n1) ^
                          tl<LAYOUT_T4X32, 3, 3>(aes, lc, n2) ^ a.rk[7];
    auto fast_chunk = [&](uint64_t q) __attribute__((always_inline)) {
        uint32_t s[BPT][4], x[BPT][4];
        // all four slots' loads first, ahead of the per-slot branches below
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            // position r = head + 256q + 64i + lane is block j = nC - r; the
            // slot's 64 blocks start at block nC - head - 256q - 64i - 63, a
            // multiple of 64
            const uint64_t top = nC - head - 256 * q - 64u * uint32_t(i) - 63;
            const u32x4 v = load16(a.in + 16 * top + 16u * (63u - lane));
            x[i][0] = v.x;
            x[i][1] = v.y;
            x[i][2] = v.z;
            x[i][3] = v.w;
        }
        // rounds 1 and 2.  The chunk's blocks are 256 consecutive ones, from
        // `low` = nC - head - 256q - 255 (slot 3's first) up; their counters
        // cross at most one multiple of 256, so they have at most two values
        // of their top 24 bits (A below it, B from it on).  After round 1
        // columns 1..3 depend only on those bits, and so do 12 of round 2's
        // lookups: 15 lookups for each of A and B per chunk, and five per
        // block.
        const uint32_t cb = c1 + uint32_t(nC - head - 256 * q - 255);
        auto shared = [&](uint32_t g3, uint32_t (&qv)[4]) __attribute__((always_inline)) {
            const uint32_t t1 = pre1 ^ tl<LAYOUT_T4X32, 2, 2>(aes, lc, g3);
            const uint32_t t2 = pre2 ^ tl<LAYOUT_T4X32, 1, 1>(aes, lc, g3);
            const uint32_t t3 = pre3 ^ tl<LAYOUT_T4X32, 0, 0>(aes, lc, g3);
            qv[0] = xor3(tl<LAYOUT_T4X32, 1, 1>(aes, lc, t1), tl<LAYOUT_T4X32, 2, 2>(aes, lc, t2),
                         tl<LAYOUT_T4X32, 3, 3>(aes, lc, t3)) ^ a.rk[8];
            qv[1] = xor3(tl<LAYOUT_T4X32, 0, 0>(aes, lc, t1), tl<LAYOUT_T4X32, 1, 1>(aes, lc, t2),
                         tl<LAYOUT_T4X32, 2, 2>(aes, lc, t3)) ^ a.rk[9];
            qv[2] = xor3(tl<LAYOUT_T4X32, 0, 0>(aes, lc, t2), tl<LAYOUT_T4X32, 1, 1>(aes, lc, t3),
                         tl<LAYOUT_T4X32, 3, 3>(aes, lc, t1)) ^ a.rk[10];
            qv[3] = xor3(tl<LAYOUT_T4X32, 0, 0>(aes, lc, t3), tl<LAYOUT_T4X32, 2, 2>(aes, lc, t1),
                         tl<LAYOUT_T4X32, 3, 3>(aes, lc, t2)) ^ a.rk[11];
        };
        uint32_t qa[4], qb[4];
        shared(__builtin_bswap32(cb) ^ a.rk[3], qa);
        shared(__builtin_bswap32(cb + 256u) ^ a.rk[3], qb);
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            // lane l of slot i: block top + 63 - l, the (64 (3 - i) + 63 - l)-th of the chunk
            const uint32_t jj = 64u * uint32_t(BPT - 1 - i) + (63u - lane);
            const bool b = (cb & 255u) + jj >= 256u;
            const uint32_t v3 = __builtin_bswap32(cb + jj) ^ a.rk[3];
            const uint32_t t0 = pre0 ^ tl<LAYOUT_T4X32, 3, 3>(aes, lc, v3);
            s[i][0] = (b ? qb[0] : qa[0]) ^ tl<LAYOUT_T4X32, 0, 0>(aes, lc, t0);
            s[i][1] = (b ? qb[1] : qa[1]) ^ tl<LAYOUT_T4X32, 3, 3>(aes, lc, t0);
            s[i][2] = (b ? qb[2] : qa[2]) ^ tl<LAYOUT_T4X32, 2, 2>(aes, lc, t0);
            s[i][3] = (b ? qb[3] : qa[3]) ^ tl<LAYOUT_T4X32, 1, 1>(aes, lc, t0);
        }
        rounds<NR, DIR_ENC, LAYOUT_T4X32, BPT>(s, aes, lc, a.rk, 3);
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint64_t top = nC - head - 256 * q - 64u * uint32_t(i) - 63;
            const uint32_t o[4] = {x[i][0] ^ s[i][0], x[i][1] ^ s[i][1], x[i][2] ^ s[i][2], x[i][3] ^ s[i][3]};
            store16(a.out + 16 * top + 16u * (63u - lane), vec4(o[0], o[1], o[2], o[3]));
            uint32_t g[4];
            mul_tab(lds, kGTab, W[i], g);
#pragma unroll
            for (int c = 0; c < 4; c++)
                W[i][c] = g[c] ^ (DEC ? x[i][c] : o[c]);
        }
    };
    // Any other chunk, one slot of 64 positions at a time: the length block,
    // ciphertext blocks (whole or the partial last one), additional data, or
    // nothing past the start of the sequence.
    // A chunk of 256 positions that are all whole blocks of additional data:
    // only the hash (GMAC over long additional data runs here).
    auto aad_chunk = [&](uint64_t q) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            // position r is additional-data block k = nC + nA - r; the slot's
            // 64 blocks end at block nC + nA - head - 256q - 64i
            const uint64_t top = nC + nA - head - 256 * q - 64u * uint32_t(i) - 63;
            const u32x4 v = load16(a.aad + 16 * top + 16u * (63u - lane));
            uint32_t g[4];
            mul_tab(lds, kGTab, W[i], g);
            W[i][0] = g[0] ^ v.x;
            W[i][1] = g[1] ^ v.y;
            W[i][2] = g[2] ^ v.z;
            W[i][3] = g[3] ^ v.w;
        }
    };
    auto slow_chunk = [&](uint64_t q) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint64_t r = head + 256 * q + 64u * uint32_t(i) + lane;
            const bool is_c = r >= 1 && r <= nC;
            const uint64_t j = nC - r;
            u32x4 v = vec4(0, 0, 0, 0);
            if (r == 0) {
                v = vec4(len[0], len[1], len[2], len[3]);
            } else if (is_c) {
                v = j < cwhole ? load16(a.in + 16 * j) : load_tail(a.in + 16 * j, ctail);
            } else if (r <= nC + nA) {
                const uint64_t k = nC + nA - r;
                v = k < awhole ? load16(a.aad + 16 * k) : load_tail(a.aad + 16 * k, atail);
            }
            uint32_t x[4] = {v.x, v.y, v.z, v.w};
            uint32_t s[1][4] = {{n0, n1, n2, __builtin_bswap32(c1 + uint32_t(j)) ^ a.rk[3]}};
            rounds<NR, DIR_ENC, LAYOUT_T4X32, 1>(s, aes, lc, a.rk, 1);
            if (is_c) {
                const uint32_t o[4] = {x[0] ^ s[0][0], x[1] ^ s[0][1], x[2] ^ s[0][2], x[3] ^ s[0][3]};
                const bool whole = j < cwhole;
                if (whole)
                    store16(a.out + 16 * j, vec4(o[0], o[1], o[2], o[3]));
                else
                    store_tail(a.out + 16 * j, vec4(o[0], o[1], o[2], o[3]), ctail);
                if (!DEC)
#pragma unroll
                    for (int c = 0; c < 4; c++)
                        x[c] = whole ? o[c] : o[c] & tmask[c];
            }
            uint32_t g[4];
            mul_tab(lds, kGTab, W[i], g);
#pragma unroll
            for (int c = 0; c < 4; c++)
                W[i][c] = g[c] ^ x[c];
            asm volatile("" ::: "memory");   // one slot's work at a time
        }
    };
    if (wave < nchunks) {
        uint64_t q = wave + nwaves * ((nchunks - 1 - wave) / nwaves);
        for (;;) {
            // fast: all 256 positions whole ciphertext blocks (r >= 2 leaves
            // out the length block and a partial last block)
            const uint64_t rq = head + 256 * q;
            if (rq >= 2 && rq + 255 <= nC)
                fast_chunk(q);
            else if (rq > nC && rq + 255 <= nC + nA && nC + nA - rq < awhole)
                aad_chunk(q);
            else
                slow_chunk(q);
            if (q < nwaves)
                break;
            q -= nwaves;
        }
    }

    // fold: tables 0..6 hold H^1 .. H^64, tables 7..10 hold H^256 .. H^2048
    build_tables(lds, 0, kFoldVec, int(kFoldTabs), [&](int k) { return a.ws->powers[k < 7 ? k : k + 1]; });
    uint32_t u[4] = {W[BPT - 1][0], W[BPT - 1][1], W[BPT - 1][2], W[BPT - 1][3]};
#pragma unroll
    for (int i = BPT - 2; i >= 0; i--) {
        mul_tab(lds, 6 * kTabBytes, u, u);
#pragma unroll
        for (int c = 0; c < 4; c++)
            u[c] ^= W[i][c];
    }
#pragma unroll
    for (int k = 0; k < 6; k++) {
        uint32_t v[4];
#pragma unroll
        for (int c = 0; c < 4; c++)
            v[c] = uint32_t(__shfl_down(int(u[c]), 1u << k, 64));
        mul_tab(lds, uint32_t(k) * kTabBytes, v, v);
#pragma unroll
        for (int c = 0; c < 4; c++)
            u[c] ^= v[c];
    }
    const uint32_t wv = threadIdx.x >> 6;
    if (lane == 0)
        lds_store16(lds, kWavePartials + 16u * wv, vec4(u[0], u[1], u[2], u[3]));
    __syncthreads();
    if (wv == 0) {
        const u32x4 p = lane < 16 ? lds_load16(lds, kWavePartials + 16u * lane) : vec4(0, 0, 0, 0);
        uint32_t y[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint32_t v[4];
#pragma unroll
            for (int c = 0; c < 4; c++)
                v[c] = uint32_t(__shfl_down(int(y[c]), 1u << k, 64));
            mul_tab(lds, uint32_t(7 + k) * kTabBytes, v, v);
#pragma unroll
            for (int c = 0; c < 4; c++)
                y[c] ^= v[c];
        }
        if (lane == 0)
            for (int c = 0; c < 4; c++)
                a.ws->partials[blockIdx.x][c] = y[c];
    }
}

// One workgroup: folds the workgroups' partial sums with the factors
// H^(4096 b) into B, then one wave encrypts the head's ciphertext blocks
// (the last head - 1 blocks, r = 1 .. head - 1), adds the head's positions
// as sum_(r < head) X_r H^r (a tree over lanes, lane r holding X_r) to
// H^head * B, multiplies by H and forms (or checks) the tag.
template <int NR, bool DEC>
__global__ __launch_bounds__(1024) void gcm_final_kernel(const GcmArgs a) {
    constexpr uint32_t kMaxTabs = 14, kParts = kMaxTabs * kTabBytes + kMaxTabs * kVecBytes;
    __shared__ uint32_t lds[(kParts + kGcmMaxGrid * 16) / 4];
    // tables 0 .. lg-1 hold H^4096 .. H^(4096 * 2^(lg-1)), tables lg .. lg+5
    // hold H, H^2, .. H^32
    const int lg = int(a.grid_log2);
    build_tables(lds, 0, uint32_t(lg + 6) * kTabBytes, lg + 6,
                 [&](int k) { return a.ws->powers[k < lg ? 12 + k : k - lg]; });
    const uint32_t t = threadIdx.x, grid = 1u << a.grid_log2;
    if (t < kGcmMaxGrid) {
        u32x4 p = vec4(0, 0, 0, 0);
        if (t < grid)
            p = vec4(a.ws->partials[t][0], a.ws->partials[t][1], a.ws->partials[t][2], a.ws->partials[t][3]);
        lds_store16(lds, kParts + 16u * t, p);
    }
    __syncthreads();
    for (uint32_t k = 0, d = 1; d < grid; k++, d <<= 1) {
        if ((t & (2 * d - 1)) == 0 && t + d < grid) {
            const u32x4 o = lds_load16(lds, kParts + 16u * (t + d));
            uint32_t v[4] = {o.x, o.y, o.z, o.w};
            mul_tab(lds, k * kTabBytes, v, v);
            const u32x4 m = lds_load16(lds, kParts + 16u * t);
            lds_store16(lds, kParts + 16u * t, vec4(m.x ^ v[0], m.y ^ v[1], m.z ^ v[2], m.w ^ v[3]));
        }
        __syncthreads();
    }
    if (t >= 64)
        return;
    const uint32_t hpow = uint32_t(lg) * kTabBytes;   // table of H^(2^k) is hpow + k * kTabBytes
    const uint64_t nC = (a.nbytes + 15) >> 4, cwhole = a.nbytes >> 4;
    const uint32_t head = uint32_t((nC + 1) & 63u), ctail = uint32_t(a.nbytes & 15u);
    // lane r < head holds X_r: r = 0 the length block, else ciphertext block
    // j = nC - r, encrypted here with counter count(J0) + 1 + j
    uint32_t x[4] = {0, 0, 0, 0};
    if (t == 0 && head > 0) {
        const uint64_t abits = 8 * a.aad_bytes, cbits = 8 * a.nbytes;
        x[0] = __builtin_bswap32(uint32_t(abits >> 32));
        x[1] = __builtin_bswap32(uint32_t(abits));
        x[2] = __builtin_bswap32(uint32_t(cbits >> 32));
        x[3] = __builtin_bswap32(uint32_t(cbits));
    } else if (t < head) {
        const uint64_t j = nC - t;
        uint32_t ks[4] = {a.ws->j0[0], a.ws->j0[1], a.ws->j0[2],
                          __builtin_bswap32(__builtin_bswap32(a.ws->j0[3]) + 1u + uint32_t(j))};
        encrypt_global<NR>(a.rk, ks);
        const bool whole = j < cwhole;
        const u32x4 v = whole ? load16(a.in + 16 * j) : load_tail(a.in + 16 * j, ctail);
        const u32x4 o = vec4(v.x ^ ks[0], v.y ^ ks[1], v.z ^ ks[2], v.w ^ ks[3]);
        if (whole)
            store16(a.out + 16 * j, o);
        else
            store_tail(a.out + 16 * j, o, ctail);
        const u32x4 c = DEC ? v : o;
        x[0] = c.x;
        x[1] = c.y;
        x[2] = c.z;
        x[3] = c.w;
        if (!whole) {
            // only the tail's bytes enter GHASH
#pragma unroll
            for (int w = 0; w < 4; w++) {
                const int keep = int(ctail) - 4 * w;
                x[w] &= keep >= 4 ? ~0u : keep <= 0 ? 0u : (1u << (8 * keep)) - 1u;
            }
        }
    }
    // sum_r X_r H^r over the lanes: lane l adds lane l + 2^k's sum times H^(2^k)
#pragma unroll
    for (int k = 0; k < 6; k++) {
        uint32_t v[4];
#pragma unroll
        for (int c = 0; c < 4; c++)
            v[c] = uint32_t(__shfl_down(int(x[c]), 1u << k, 64));
        mul_tab(lds, hpow + uint32_t(k) * kTabBytes, v, v);
#pragma unroll
        for (int c = 0; c < 4; c++)
            x[c] ^= v[c];
    }
    // B * H^head, then the sum times H
    const u32x4 o = lds_load16(lds, kParts);
    uint32_t sum[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
    for (int k = 0; k < 6; k++)
        if ((head >> k) & 1u)
            mul_tab(lds, hpow + uint32_t(k) * kTabBytes, sum, sum);
#pragma unroll
    for (int c = 0; c < 4; c++)
        sum[c] ^= x[c];
    mul_tab(lds, hpow, sum, sum);
    if (t == 0) {
        uint8_t tag[16];
        for (int b = 0; b < 16; b++)
            tag[b] = uint8_t((sum[b >> 2] ^ a.ws->ej0[b >> 2]) >> (8 * (b & 3)));
        if (DEC) {
            uint32_t diff = 0;
            for (uint32_t b = 0; b < a.tag_bytes; b++)
                diff |= uint32_t(tag[b] ^ a.tag_in[b]);
            *a.ok = diff == 0 ? 1 : 0;
        } else {
            for (int b = 0; b < 16; b++)
                a.tag_out[b] = tag[b];
        }
    }
}

}  // namespace

hipError_t upload_tables_gcm(const HostTables &t) { return upload_base_tables(t); }

hipError_t launch_gcm(int nr, const GcmArgs &a, hipStream_t stream) {
    void (*setup)(const GcmArgs) = nr == 10 ? gcm_setup_kernel<10> : nr == 12 ? gcm_setup_kernel<12>
                                                                              : gcm_setup_kernel<14>;
    void (*bulk)(const GcmArgs);
    if (a.decrypt)
        bulk = nr == 10 ? gcm_kernel<10, true, 4> : nr == 12 ? gcm_kernel<12, true, 4> : gcm_kernel<14, true, 4>;
    else
        bulk = nr == 10 ? gcm_kernel<10, false, 4> : nr == 12 ? gcm_kernel<12, false, 4>
                                                              : gcm_kernel<14, false, 4>;
    hipLaunchKernelGGL(setup, dim3(1), dim3(64), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(bulk, dim3(1u << a.grid_log2), dim3(1024), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    void (*fin)(const GcmArgs);
    if (a.decrypt)
        fin = nr == 10 ? gcm_final_kernel<10, true> : nr == 12 ? gcm_final_kernel<12, true>
                                                               : gcm_final_kernel<14, true>;
    else
        fin = nr == 10 ? gcm_final_kernel<10, false> : nr == 12 ? gcm_final_kernel<12, false>
                                                                : gcm_final_kernel<14, false>;
    hipLaunchKernelGGL(fin, dim3(1), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

}  // namespace aesgpu
