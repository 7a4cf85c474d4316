// Batches of independent messages (each with its own key, length, mode and
// direction) in one launch sequence:
//
//   prep_kernel     one lane per message: checks the descriptor, runs Key
//                   Expansion (FIPS-197 section 5.2) plus the
//                   equivalent-inverse schedule (section 5.3.5) for
//                   decryption and the tweak key's schedule for XTS, and
//                   adds up per chunk of 256 messages what the plan needs.
//   plan_kernel     one lane per message: puts the messages in three lists,
//                   forward (ECB encryption, CTR, XTS encryption: the
//                   encryption tables), inverse (ECB, CBC and XTS
//                   decryption: the inverse ones) and serial (CBC
//                   encryption), each message with the work of the list
//                   before it.  It also zeroes the counters, so the sequence
//                   can be replayed from a graph without any memset.
//   batch_kernel    persistent, one per list: the list's work is cut into
//                   equal shares, one per wave and round, each covering parts
//                   of one or more messages; a wave runs its shares (for
//                   long lists, the second half of them taken off a counter)
//                   with every message's round keys in scalar registers and
//                   the same block loop as the single-buffer kernels.
//   gcm_fused_kernel  GCM messages of at least kFusedMinPositions GHASH
//                   positions (one kernel per key size): counter mode and
//                   GHASH in one pass over each piece of kFusedPiece
//                   positions, one workgroup per piece, as the single-buffer
//                   GCM kernel does over a whole buffer.
//   ghash_kernel    GCM messages only: GHASH (SP 800-38D section 6.4) over
//                   each message's additional data, ciphertext and lengths,
//                   cut into pieces of kGhashPiece positions, one wave per
//                   piece with its own multiplier table in LDS; a piece's
//                   sum, times the power of H its position calls for, is
//                   XORed into the message's sum (GHASH is linear).
//   gcm_tag_kernel  one lane per GCM message: the tag Cipher_K(J0) XOR the
//                   sum, written (encryption) or compared (decryption).
//
// This is the paper's method (cut the data into one chunk per processor and
// process the chunks in parallel, Section IV) applied across messages, with
// the processors being the GPU's waves.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "aesgpu.h"
#include "cipher_core.h"
#include "ghash_core.h"
#include "internal.h"
#include "xts_core.h"

namespace aesgpu {
namespace {

// Workgroup size of the prep and plan kernels, one lane per message of a
// chunk: four waves, so that their workgroups fit beside a cipher kernel's
// 16 waves on a compute unit (the request loop runs several batches at once).
constexpr int kPlanThreads = kBatchChunk;

__device__ __forceinline__ int desc_nr(const aes_msg_desc &d) { return 10 + 2 * int(d.keybits_code); }

__device__ __forceinline__ uint32_t le32(const uint8_t *p) {
    return uint32_t(p[0]) | (uint32_t(p[1]) << 8) | (uint32_t(p[2]) << 16) | (uint32_t(p[3]) << 24);
}

// XTS messages carry in ctr0: bytes 0..7 the tweak value of the first data
// unit, 8..11 the slot of the tweak key, 12..15 the data-unit size in bytes
// (all little-endian).
__device__ __forceinline__ uint64_t xts_first_unit(const aes_msg_desc &d) {
    return uint64_t(le32(d.ctr0)) | (uint64_t(le32(d.ctr0 + 4)) << 32);
}
__device__ __forceinline__ uint32_t xts_key2(const aes_msg_desc &d) { return le32(d.ctr0 + 8); }
__device__ __forceinline__ uint32_t xts_unit_bytes(const aes_msg_desc &d) { return le32(d.ctr0 + 12); }
__device__ __forceinline__ uint32_t xts_unit_shift(const aes_msg_desc &d) {
    return 31u - __builtin_clz(xts_unit_bytes(d) >> 4);   // log2 of the blocks per unit
}

__device__ __forceinline__ bool ranges_overlap(uintptr_t a, uint64_t na, uintptr_t b, uint64_t nb) {
    return na && nb && a < b + nb && b < a + na;
}

// The GCM fields of message m (SP 800-38D limits; every range inside its
// buffer; the additional data and the tag clear of the message's output,
// which is written before they are read).
__device__ __forceinline__ bool gcm_valid(const aes_msg_desc &d, uint32_t m, const BatchKArgs &a) {
    if (!a.gcm)
        return false;
    const aes_gcm_desc g = a.gcm[m];
    if (d.nbytes > (uint64_t(1) << 36) - 32 || g.aad_bytes > (uint64_t(1) << 36) || (g.aad_off & 15u))
        return false;
    if (g.aad_bytes > a.in_bytes || g.aad_off > a.in_bytes - g.aad_bytes)
        return false;
    const uint64_t tb = d.decrypt ? g.tag_bytes : 16u;
    if (d.decrypt && !(tb == 4 || tb == 8 || (tb >= 12 && tb <= 16)))
        return false;
    const uint64_t tbuf = d.decrypt ? a.in_bytes : a.out_bytes;
    if (tb > tbuf || g.tag_off > tbuf - tb)
        return false;
    const uintptr_t out = reinterpret_cast<uintptr_t>(a.out_base) + d.out_off;
    const uintptr_t aad = reinterpret_cast<uintptr_t>(a.in_base) + g.aad_off;
    const uintptr_t tag = reinterpret_cast<uintptr_t>(d.decrypt ? a.in_base : a.out_base) + g.tag_off;
    return !ranges_overlap(aad, g.aad_bytes, out, d.nbytes) && !ranges_overlap(tag, tb, out, d.nbytes);
}

// Same test as the host applies to a single-buffer call, plus bounds.
__device__ __forceinline__ bool desc_valid(const aes_msg_desc &d, uint32_t m, const BatchKArgs &a) {
    if (d.keybits_code > 2 || d.mode > AES_MODE_GCM || d.decrypt > 1)
        return false;
    if ((d.mode == AES_MODE_ECB || d.mode == AES_MODE_CBC || d.mode == AES_MODE_XTS) && (d.nbytes & 15u))
        return false;
    if (d.mode == AES_MODE_GCM && !gcm_valid(d, m, a))
        return false;
    if (d.mode == AES_MODE_XTS) {
        const uint32_t u = xts_unit_bytes(d);
        if (u < 16 || u > 4096 || (u & (u - 1)) != 0 || xts_key2(d) >= uint32_t(a.nkeys))
            return false;
    }
    // Input and output are the same bytes or disjoint (waves of one message
    // would race otherwise); for CBC decryption disjoint, as it reads block
    // j-1 of the input after other waves may have written their outputs.
    const uintptr_t ip = reinterpret_cast<uintptr_t>(a.in_base) + d.in_off;
    const uintptr_t op = reinterpret_cast<uintptr_t>(a.out_base) + d.out_off;
    const bool overlap = d.nbytes && ip < op + d.nbytes && op < ip + d.nbytes;
    if (overlap && (ip != op || (d.mode == AES_MODE_CBC && d.decrypt)))
        return false;
    // a CTR message's 32-bit counter must not repeat a block within it
    if (d.mode == AES_MODE_CTR && d.nbytes > kCtrMaxBytes)
        return false;
    // a CBC encryption runs on one lane; its block count must fit the list item
    if (d.mode == AES_MODE_CBC && !d.decrypt && (d.nbytes >> 4) >= 0xFFFFFFFFull)
        return false;
    if ((d.in_off | d.out_off) & 15u)
        return false;
    if (d.key_idx >= uint32_t(a.nkeys))
        return false;
    if (d.nbytes > a.in_bytes || d.in_off > a.in_bytes - d.nbytes)
        return false;
    if (d.nbytes > a.out_bytes || d.out_off > a.out_bytes - d.nbytes)
        return false;
    return true;
}

// Forward list (encryption tables): ECB encrypt, CTR, XTS encrypt, GCM (its
// CTR part, either direction).  Inverse list (decryption tables): ECB, CBC
// and XTS decrypt.  Serial list: CBC encrypt.
__device__ __forceinline__ int desc_class(const aes_msg_desc &d) {
    if (d.mode == AES_MODE_CBC)
        return d.decrypt ? 1 : 2;
    return ((d.mode == AES_MODE_ECB || d.mode == AES_MODE_XTS) && d.decrypt) ? 1 : 0;
}

// Where a wave's share of a message may start or end: multiples of
// split_blocks blocks; for XTS, of whole data units (the tweak work starts
// at a unit), as many units as fit in split_blocks, at least one.
__device__ __forceinline__ uint64_t split_step(const aes_msg_desc &d, uint32_t split_blocks) {
    if (d.mode != AES_MODE_XTS)
        return split_blocks;
    const uint32_t ushift = xts_unit_shift(d);
    const uint64_t units = split_blocks >> ushift;
    return (units ? units : 1) << ushift;
}

// Work of one block in cost units, for splitting a list evenly: the rounds
// (their table lookups dominate) plus a share for loads, stores and the
// initial key addition.
__device__ __forceinline__ uint64_t block_cost(const aes_msg_desc &d) { return uint64_t(desc_nr(d)) + 2; }

__device__ __forceinline__ uint32_t batch_count(const BatchKArgs &a) {
    int n = a.d_nmsg ? *a.d_nmsg : a.nmsg;
    if (n < 0)
        n = 0;
    if (n > a.max_msgs)
        n = a.max_msgs;
    return uint32_t(n);
}

// The S-box and the inverse round table, read from a copy of the base tables
// in LDS: tab[0 .. 255] is the encryption round table for row 0, whose byte
// 1 is S[x]; tab[256 .. 511] the decryption one.
__device__ __forceinline__ uint32_t sbox(const uint32_t *tab, uint32_t x) { return (tab[x & 255u] >> 8) & 255u; }

__device__ __forceinline__ uint32_t sub_word(const uint32_t *tab, uint32_t w) {
    return sbox(tab, w) | (sbox(tab, w >> 8) << 8) | (sbox(tab, w >> 16) << 16) | (sbox(tab, w >> 24) << 24);
}

// InvMixColumns of a column word, through the inverse round table:
// td0[S[b]] is InvMixColumns of the column (b, 0, 0, 0).
__device__ __forceinline__ uint32_t inv_mix_column(const uint32_t *tab, uint32_t w) {
    return tab[256 + sbox(tab, w)] ^ rotl(tab[256 + sbox(tab, w >> 8)], 8) ^
           rotl(tab[256 + sbox(tab, w >> 16)], 16) ^ rotl(tab[256 + sbox(tab, w >> 24)], 24);
}

// Key Expansion (FIPS-197 section 5.2) of the Nk-word key at `key`, fully
// unrolled: each word w[i], i = 0 .. 4Nr+3, is handed to emit(i, w[i]) as
// soon as it exists (only the last Nk words are needed to go on).
template <int NK, typename Emit>
__device__ __forceinline__ void expand_key(const uint8_t *key, const uint32_t *tab, Emit emit) {
    uint32_t w[4 * (NK + 7)];
#pragma unroll
    for (int i = 0; i < NK; i++) {
        w[i] = le32(key + 4 * i);
        emit(i, w[i]);
    }
    uint32_t rcon = 1;
#pragma unroll
    for (int i = NK; i < 4 * (NK + 7); i++) {
        uint32_t t = w[i - 1];
        if (i % NK == 0) {
            t = sub_word(tab, rotl(t, 24)) ^ rcon;  // RotWord is a right rotation of a little-endian word
            rcon = ((rcon << 1) ^ ((rcon & 0x80u) ? 0x1bu : 0u)) & 0xffu;
        } else if (NK > 6 && i % NK == 4) {
            t = sub_word(tab, t);
        }
        w[i] = w[i - NK] ^ t;
        emit(i, w[i]);
    }
}

// One message's key slot: the encryption schedule at 0; for the inverse
// list the equivalent-inverse schedule (section 5.3.5) at kKeySlotWords / 2,
// whose round r is InvMixColumns of encryption round Nr - r (rounds 0 and Nr
// swapped, unmixed); for XTS the tweak key's encryption schedule in the half
// the data key's direction leaves free.  A lane expands its message's key
// into registers and stores each round key as one 16-byte write (the slot
// is 512-byte aligned): each lane writes a slot of its own, so word-sized
// stores would each touch a different cache line for every lane.
template <int NK>
__device__ __forceinline__ void store_schedule(uint32_t *dst, const uint32_t (&w)[4 * (NK + 7)]) {
#pragma unroll
    for (int r = 0; r <= NK + 6; r++)
        reinterpret_cast<u32x4 *>(dst)[r] = vec4(w[4 * r], w[4 * r + 1], w[4 * r + 2], w[4 * r + 3]);
}

template <int NK>
__device__ __forceinline__ void expand_message_keys(const BatchKArgs &a, const aes_msg_desc &d, uint32_t *slot,
                                                    const uint32_t *tab) {
    constexpr int NR = NK + 6;
    uint32_t w[4 * (NR + 1)];
    expand_key<NK>(a.keys + size_t(d.key_idx) * 32, tab, [&](int i, uint32_t v) { w[i] = v; });
    store_schedule<NK>(slot, w);
    if (desc_class(d) == 1) {
        u32x4 *dk = reinterpret_cast<u32x4 *>(slot + kKeySlotWords / 2);
        dk[0] = vec4(w[4 * NR], w[4 * NR + 1], w[4 * NR + 2], w[4 * NR + 3]);
#pragma unroll
        for (int r = 1; r < NR; r++) {
            const int e = 4 * (NR - r);
            dk[r] = vec4(inv_mix_column(tab, w[e]), inv_mix_column(tab, w[e + 1]), inv_mix_column(tab, w[e + 2]),
                         inv_mix_column(tab, w[e + 3]));
        }
        dk[NR] = vec4(w[0], w[1], w[2], w[3]);
    }
    if (d.mode == AES_MODE_XTS) {
        uint32_t w2[4 * (NR + 1)];
        expand_key<NK>(a.keys + size_t(xts_key2(d)) * 32, tab, [&](int i, uint32_t v) { w2[i] = v; });
        store_schedule<NK>(slot + (d.decrypt ? 0 : kKeySlotWords / 2), w2);
        // the encrypted tweak of the message's first unit, so that a
        // one-unit message's wave need not run it on one lane
        const uint64_t u = xts_first_unit(d);
        uint32_t t[4] = {uint32_t(u), uint32_t(u >> 32), 0u, 0u};
        encrypt_one<NR>(tab, w2, t);
        reinterpret_cast<u32x4 *>(slot)[kXtsSlotTweak / 4] = vec4(t[0], t[1], t[2], t[3]);
    }
    if (d.mode == AES_MODE_GCM) {
        // H = Cipher_K(0^128); J0 = IV || 0^31 || 1 (a 96-bit IV) and
        // Cipher_K(J0); the message's GHASH sum starts at zero
        uint32_t h[4] = {0, 0, 0, 0};
        encrypt_one<NR>(tab, w, h);
        uint32_t e[4] = {le32(d.ctr0), le32(d.ctr0 + 4), le32(d.ctr0 + 8), 0x01000000u};
        encrypt_one<NR>(tab, w, e);
        u32x4 *g = reinterpret_cast<u32x4 *>(slot);
        g[kGcmSlotH / 4] = vec4(h[0], h[1], h[2], h[3]);
        g[kGcmSlotEJ0 / 4] = vec4(e[0], e[1], e[2], e[3]);
        g[kGcmSlotSum / 4] = vec4(0, 0, 0, 0);
        // H^(kGhashPiece * 2^t): the factors of the GHASH pieces' positions
        uint64_t lo, hi;
        to_poly(h, lo, hi);
        for (int t = 0; t < kGhashPieceLog2; t++)
            gf_square(lo, hi);
        for (int t = 0; t < kGcmSlotPowers; t++) {
            uint32_t pw[4];
            from_poly(lo, hi, pw);
            g[kGcmSlotPow / 4 + t] = vec4(pw[0], pw[1], pw[2], pw[3]);
            gf_square(lo, hi);
        }
    }
}

// Exclusive prefix sums over the workgroup's kPlanThreads threads of N
// counters at once: scans within each wave by lane shifts, then the wave
// totals through LDS.  total[] gets the workgroup sums.
template <int N>
__device__ __forceinline__ void block_exclusive_scan(uint64_t (&v)[N], uint64_t (*wsum)[kPlanThreads / 64],
                                                     uint64_t (&total)[N]) {
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint64_t x[N];
#pragma unroll
    for (int k = 0; k < N; k++)
        x[k] = v[k];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int k = 0; k < N; k++) {
            const uint64_t y = __shfl_up(x[k], d, 64);
            if (lane >= uint32_t(d))
                x[k] += y;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < N; k++)
            wsum[k][wave] = x[k];
    }
    __syncthreads();
    // lane l of every group of NW lanes reads wave l's total; butterfly sums
    // give the total of the waves before this one and of all of them
    constexpr int NW = kPlanThreads / 64;
    static_assert(NW >= 1 && NW <= 64 && (NW & (NW - 1)) == 0, "a power-of-two number of waves");
    const uint32_t lw = lane & uint32_t(NW - 1);
#pragma unroll
    for (int k = 0; k < N; k++) {
        const uint64_t s = wsum[k][lw];
        uint64_t before = lw < wave ? s : 0, sum = s;
#pragma unroll
        for (int o = 1; o < NW; o <<= 1) {
            before += __shfl_xor(before, o, NW);
            sum += __shfl_xor(sum, o, NW);
        }
        v[k] = before + x[k] - v[k];
        total[k] = sum;
    }
}

// items in lists 0, 1, 2; cost of lists 0, 1; rejected; GCM messages hashed
// in pieces; their GHASH pieces; the short ones among them (at most
// kLaneGhashMaxPositions positions: one piece each); GCM messages encrypted
// and hashed in one pass, per key size (9 .. 11), and their pieces (12 .. 14)
constexpr int kPlanCounters = kBatchChunkCounters;
constexpr int kFusedMsgs = 9, kFusedPieces = 12;

// GHASH positions of a GCM message: its additional data, its ciphertext
// and the length block, 16 bytes each.
__device__ __forceinline__ uint64_t ghash_positions(const aes_msg_desc &d, const aes_gcm_desc &g) {
    return ((g.aad_bytes + 15) >> 4) + ((d.nbytes + 15) >> 4) + 1;
}

// floor(a b / c) without overflow (messages may overlap, so a list's cost is
// not bounded by the memory size).
__device__ __forceinline__ uint64_t mul_div_floor(uint64_t a, uint64_t b, uint64_t c) {
    return uint64_t((unsigned __int128)a * b / c);
}


// One message's contribution to the plan's counters (all zero past the
// batch's end).  fused: a GCM message of the fused list, in no other list.
__device__ __forceinline__ void message_counts(const BatchKArgs &a, uint32_t m, uint32_t n, bool &valid, int &k,
                                               bool &fused, uint64_t (&c)[kPlanCounters]) {
    for (int j = 0; j < kPlanCounters; j++)
        c[j] = 0;
    valid = false;
    fused = false;
    k = 0;
    if (m >= n)
        return;
    const aes_msg_desc d = a.desc[m];
    if (!desc_valid(d, m, a)) {
        c[5] = 1;
        return;
    }
    valid = true;
    k = desc_class(d);
    if (d.mode == AES_MODE_GCM) {
        const uint64_t npos = ghash_positions(d, a.gcm[m]);
        fused = a.fuse_gcm && npos >= kFusedMinPositions;
        if (fused) {
            const uint64_t pieces = (npos + kFusedPiece - 1) / kFusedPiece;
#pragma unroll
            for (int j = 0; j < 3; j++) {
                c[kFusedMsgs + j] = d.keybits_code == uint32_t(j) ? 1 : 0;
                c[kFusedPieces + j] = d.keybits_code == uint32_t(j) ? pieces : 0;
            }
            return;
        }
        c[6] = 1;
        c[7] = (npos + kGhashPiece - 1) / kGhashPiece;
        c[8] = npos <= kLaneGhashMaxPositions ? 1 : 0;
    }
    const uint64_t cost = ((d.nbytes + 15) >> 4) * block_cost(d);
    // (selects, not indexed stores: keeps c[] in registers)
    c[0] = k == 0 ? 1 : 0;
    c[1] = k == 1 ? 1 : 0;
    c[2] = k == 2 ? 1 : 0;
    c[3] = k == 0 ? cost : 0;
    c[4] = k == 1 ? cost : 0;
}

// Whether the batch hashes its short GCM messages one per lane: when there
// are enough of them that a wave per message would cost more (each wave
// builds seven multiplier tables and folds its lanes for a few Horner steps)
// than one pass of the longest allowed message through a lane.
__device__ __forceinline__ bool lane_ghash(const uint64_t (&total)[kPlanCounters]) {
    return total[8] >= kLaneGhashMinMessages;
}

// The GHASH counts of the header: messages and pieces hashed by waves, and
// messages hashed by lanes.
__device__ __forceinline__ void gcm_header(BatchHeader *h, const uint64_t (&total)[kPlanCounters]) {
    const uint64_t short_msgs = lane_ghash(total) ? total[8] : 0;
    h->ngcm = uint32_t(total[6] - short_msgs);
    h->gcm_pieces = total[7] - short_msgs;
    h->nlane = uint32_t(short_msgs);
    for (int j = 0; j < 3; j++) {
        h->nfused[j] = uint32_t(total[kFusedMsgs + j]);
        h->fused_pieces[j] = total[kFusedPieces + j];
        h->next_fused[j] = 0;
    }
}

// The GHASH list's item of GCM message m: its pieces, and the pieces of the
// GCM messages before it (c: the message's exclusive prefix of the counters),
// or, for a short message when the batch hashes those per lane, its place at
// the back of the list.
__device__ __forceinline__ void gcm_item(const BatchKArgs &a, uint32_t m, const uint64_t (&before)[kPlanCounters],
                                         const uint64_t (&c)[kPlanCounters], const uint64_t (&total)[kPlanCounters],
                                         bool lanes) {
    const aes_msg_desc d = a.desc[m];
    if (d.mode != AES_MODE_GCM)
        return;
    const uint64_t npos = ghash_positions(d, a.gcm[m]);
    if (a.fuse_gcm && npos >= kFusedMinPositions) {
        // after the messages of the smaller key sizes
        const int j = int(d.keybits_code);
        const uint64_t off = (j > 0 ? total[kFusedMsgs] : 0) + (j > 1 ? total[kFusedMsgs + 1] : 0);
        BatchItem it;
        it.msg = m;
        it.count = uint32_t((npos + kFusedPiece - 1) / kFusedPiece);
        it.start = before[kFusedPieces + j] + c[kFusedPieces + j];
        a.items[size_t(4) * a.max_msgs + off + before[kFusedMsgs + j] + c[kFusedMsgs + j]] = it;
        return;
    }
    const uint64_t short_before = lanes ? before[8] + c[8] : 0;
    BatchItem it;
    it.msg = m;
    if (lanes && npos <= kLaneGhashMaxPositions) {
        it.count = 1;
        it.start = 0;
        a.items[size_t(3) * a.max_msgs + (size_t(a.max_msgs) - 1 - short_before)] = it;
        return;
    }
    it.count = uint32_t((npos + kGhashPiece - 1) / kGhashPiece);
    it.start = before[7] + c[7] - short_before;   // a short message is one piece
    a.items[size_t(3) * a.max_msgs + (before[6] + c[6] - short_before)] = it;
}

// The first launch of a batch, one message per thread, kPlanThreads messages
// per workgroup (a chunk): Key Expansion, and the chunk's counters for the
// plan (items and cost per list, rejected descriptors).
__global__ __launch_bounds__(kPlanThreads) void prep_kernel(const BatchKArgs a) {
    __shared__ uint32_t tab[512];
    __shared__ uint64_t wsum[kPlanCounters][kPlanThreads / 64];
    for (uint32_t i = threadIdx.x; i < 512; i += kPlanThreads)
        tab[i] = g_base[i];
    const uint32_t n = batch_count(a);
    const uint32_t m = blockIdx.x * kPlanThreads + threadIdx.x;
    bool valid, fused;
    int k;
    uint64_t c[kPlanCounters], total[kPlanCounters];
    message_counts(a, m, n, valid, k, fused, c);
    (void)fused;
    if (m < n && !valid && a.reject_flags)
        a.reject_flags[m] = 1;
    block_exclusive_scan<kPlanCounters>(c, wsum, total);   // its barrier also covers tab[]
    if (threadIdx.x == 0) {
        for (int j = 0; j < kPlanCounters; j++)
            a.chunk_totals[size_t(blockIdx.x) * kPlanCounters + j] = total[j];
    }
    if (!valid)
        return;
    const aes_msg_desc d = a.desc[m];
    uint32_t *slot = a.keytab + size_t(m) * kKeySlotWords;
    if (d.keybits_code == 0)
        expand_message_keys<4>(a, d, slot, tab);
    else if (d.keybits_code == 1)
        expand_message_keys<6>(a, d, slot, tab);
    else
        expand_message_keys<8>(a, d, slot, tab);
}

// Both launches in one, for batches of at most one chunk (a single
// workgroup): Key Expansion, the scan of the messages' counters, the list
// items and the header.
__global__ __launch_bounds__(kPlanThreads) void prep_plan_kernel(const BatchKArgs a) {
    __shared__ uint32_t tab[512];
    __shared__ uint64_t wsum[kPlanCounters][kPlanThreads / 64];
    for (uint32_t i = threadIdx.x; i < 512; i += kPlanThreads)
        tab[i] = g_base[i];
    const uint32_t n = min(batch_count(a), uint32_t(kPlanThreads));
    const uint32_t m = threadIdx.x;
    bool valid, fused;
    int k;
    uint64_t c[kPlanCounters], total[kPlanCounters];
    message_counts(a, m, n, valid, k, fused, c);
    if (m < n && !valid && a.reject_flags)
        a.reject_flags[m] = 1;
    block_exclusive_scan<kPlanCounters>(c, wsum, total);   // its barrier also covers tab[]
    if (m == 0) {
        BatchHeader *h = a.header;
        for (int j = 0; j < 3; j++) {
            h->nitems[j] = uint32_t(total[j]);
            h->next[j] = 0;
        }
        h->cost[0] = total[3];
        h->cost[1] = total[4];
        h->rejected = uint32_t(total[5]);
        gcm_header(h, total);
    }
    if (!valid)
        return;
    const aes_msg_desc d = a.desc[m];
    if (!fused) {
        BatchItem it;
        it.msg = m;
        it.count = k == 2 ? uint32_t((d.nbytes + 15) >> 4) : 0u;
        it.start = k == 0 ? c[3] : k == 1 ? c[4] : 0;
        a.items[size_t(k) * a.max_msgs + (k == 0 ? c[0] : k == 1 ? c[1] : c[2])] = it;
    }
    const uint64_t zero[kPlanCounters] = {};
    gcm_item(a, m, zero, c, total, lane_ghash(total));
    uint32_t *slot = a.keytab + size_t(m) * kKeySlotWords;
    if (d.keybits_code == 0)
        expand_message_keys<4>(a, d, slot, tab);
    else if (d.keybits_code == 1)
        expand_message_keys<6>(a, d, slot, tab);
    else
        expand_message_keys<8>(a, d, slot, tab);
}

// The second launch, same chunks: each workgroup adds up the counters of the
// chunks before it, scans its own messages and writes their list items in
// message order, each with the cost of the list before it (its start).
// Workgroup 0 also writes the header and zeroes the counters, so the whole
// sequence can be replayed from a graph without any memset.
__global__ __launch_bounds__(kPlanThreads) void plan_kernel(const BatchKArgs a) {
    __shared__ uint64_t wsum[kPlanCounters][kPlanThreads / 64];
    const uint32_t n = batch_count(a);
    const uint32_t chunks = gridDim.x;
    // counters of the chunks before this one, and of all of them
    uint64_t before[kPlanCounters], all[kPlanCounters];
    for (int j = 0; j < kPlanCounters; j++)
        before[j] = all[j] = 0;
    for (uint32_t ch = threadIdx.x; ch < chunks; ch += kPlanThreads) {
        for (int j = 0; j < kPlanCounters; j++) {
            const uint64_t v = a.chunk_totals[size_t(ch) * kPlanCounters + j];
            before[j] += ch < blockIdx.x ? v : 0;
            all[j] += v;
        }
    }
    uint64_t base[kPlanCounters], sum_all[kPlanCounters];
    block_exclusive_scan<kPlanCounters>(before, wsum, base);
    __syncthreads();   // wsum is used again
    block_exclusive_scan<kPlanCounters>(all, wsum, sum_all);
    __syncthreads();
    const uint32_t m = blockIdx.x * kPlanThreads + threadIdx.x;
    bool valid, fused;
    int k;
    uint64_t c[kPlanCounters], chunk_total[kPlanCounters];
    message_counts(a, m, n, valid, k, fused, c);
    block_exclusive_scan<kPlanCounters>(c, wsum, chunk_total);   // c: the messages before m in the chunk
    if (valid) {
        const aes_msg_desc d = a.desc[m];
        if (!fused) {
            BatchItem it;
            it.msg = m;
            it.count = k == 2 ? uint32_t((d.nbytes + 15) >> 4) : 0u;   // desc_valid keeps a serial message below 2^32 blocks
            it.start = k == 0 ? base[3] + c[3] : k == 1 ? base[4] + c[4] : 0;
            const uint64_t i = k == 0 ? base[0] + c[0] : k == 1 ? base[1] + c[1] : base[2] + c[2];
            a.items[size_t(k) * a.max_msgs + i] = it;
        }
        gcm_item(a, m, base, c, sum_all, lane_ghash(sum_all));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        BatchHeader *h = a.header;
        for (int j = 0; j < 3; j++) {
            h->nitems[j] = uint32_t(sum_all[j]);
            h->next[j] = 0;
        }
        h->cost[0] = sum_all[3];
        h->cost[1] = sum_all[4];
        h->rejected = uint32_t(sum_all[5]);
        gcm_header(h, sum_all);
    }
}

__device__ __forceinline__ uint32_t uniform32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    return uint64_t(uniform32(uint32_t(x))) | (uint64_t(uniform32(uint32_t(x >> 32))) << 32);
}

// A message's round keys into scalar registers: one coalesced load (lane j
// reads word j) and a lane read per word, instead of one load per word.
template <int NR>
__device__ __forceinline__ void load_round_keys(const uint32_t *rkp, uint32_t (&rk)[4 * (NR + 1)]) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t v = lane < 4u * (NR + 1) ? rkp[lane] : 0u;
#pragma unroll
    for (int i = 0; i < 4 * (NR + 1); i++)
        rk[i] = uint32_t(__builtin_amdgcn_readlane(int(v), i));
}

// Blocks [first, end) of message `msg` through the buffer kernels' block loop.
template <int NR, int MODE, int DIR, int BPT>
__device__ __forceinline__ void run_range(const uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a,
                                          const aes_msg_desc &d, uint32_t msg, uint64_t first, uint64_t end) {
    // The round keys are the same for the whole wave: read them once per
    // range and keep them in scalar registers.  (The compiler cannot use
    // scalar loads here: the kernel also stores to memory that it cannot
    // prove distinct from the key table.)
    const uint32_t *rkp = a.keytab + size_t(msg) * kKeySlotWords + (DIR == DIR_DEC ? kKeySlotWords / 2 : 0);
    uint32_t rk[4 * (NR + 1)];
    load_round_keys<NR>(rkp, rk);
    uint32_t ctr[4] = {0, 0, 0, 0};
    if (MODE == MODE_CBC) {
        for (int i = 0; i < 4; i++)
            ctr[i] = le32(d.ctr0 + 4 * i);
    }
    if (MODE == MODE_CTR) {
        for (int i = 0; i < 3; i++)
            ctr[i] = le32(d.ctr0 + 4 * i);
        // GCM: the first data block's counter is J0 + 1 = IV || 0^31 || 2
        ctr[3] = d.mode == AES_MODE_GCM ? 2u
                                        : (uint32_t(d.ctr0[12]) << 24) | (uint32_t(d.ctr0[13]) << 16) |
                                              (uint32_t(d.ctr0[14]) << 8) | uint32_t(d.ctr0[15]);
    }
    const uint8_t *in = static_cast<const uint8_t *>(a.in_base) + d.in_off;
    uint8_t *out = static_cast<uint8_t *>(a.out_base) + d.out_off;
    process_blocks<NR, MODE, DIR, LAYOUT_T4X32, BPT>(lds, lc, rk, ctr, in, out, d.nbytes, first, end, 64u * BPT);
}

// Blocks [first, end) of an XTS message, first at a unit boundary (the split
// keeps both ends on unit multiples, or end at the message's end): groups of
// up to 64 data units, one tweak per lane.
template <int NR, int DIR, int BPT>
__device__ __forceinline__ void run_xts_range(const uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a,
                                              const aes_msg_desc &d, uint32_t msg, uint64_t first, uint64_t end) {
    const uint32_t *slot = a.keytab + size_t(msg) * kKeySlotWords;
    const uint32_t *rkp = slot + (DIR == DIR_DEC ? kKeySlotWords / 2 : 0);
    uint32_t rk[4 * (NR + 1)];
    load_round_keys<NR>(rkp, rk);
    const uint32_t *rk2 = slot + (DIR == DIR_DEC ? 0 : kKeySlotWords / 2);   // read once per group
    const uint8_t *in = static_cast<const uint8_t *>(a.in_base) + d.in_off;
    uint8_t *out = static_cast<uint8_t *>(a.out_base) + d.out_off;
    const uint32_t ushift = xts_unit_shift(d);
    const uint64_t group = uint64_t(64) << ushift;
    const uint64_t first_unit = xts_first_unit(d);
    for (uint64_t gb0 = first; gb0 < end; gb0 += group)
        xts_group<NR, DIR, BPT>(lds, lc, rk, rk2, in, out, gb0, min(end, gb0 + group),
                                first_unit + (gb0 >> ushift), ushift, slot + kXtsSlotTweak, first_unit);
}

// The serial list (CBC encryption): one message per quad of four lanes,
// each lane carrying one column of the state (cbc_encrypt_quad), each
// message with its own round keys (a lane holds its column of every round
// key).  Wave w takes messages 16w .. 16w+15 first; only when there are
// more than 16 per wave are the rest handed out 16 at a time from a
// counter.  These run before the wave's parallel share, so the long serial
// chains start early.
template <int NR>
__device__ __forceinline__ void serial_message(const uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a,
                                               const BatchItem &item) {
    const uint32_t j = threadIdx.x & 3u;
    const aes_msg_desc d = a.desc[item.msg];
    const uint32_t *rkp = a.keytab + size_t(item.msg) * kKeySlotWords;
    uint32_t rk[NR + 1];
#pragma unroll
    for (int r = 0; r <= NR; r++)
        rk[r] = rkp[4 * r + j];
    const uint8_t *in = static_cast<const uint8_t *>(a.in_base) + d.in_off;
    uint8_t *out = static_cast<uint8_t *>(a.out_base) + d.out_off;
    // word j of the IV, read from the descriptor in memory (indexing the
    // local copy by the lane's column would put that copy in scratch)
    const uint32_t iv = le32(a.desc[item.msg].ctr0 + 4 * j);
    cbc_encrypt_quad<NR, LAYOUT_T4X32>(lds, lc, rk, iv, in, out, item.count);
}

__device__ __forceinline__ void run_serial(const uint32_t *lds, const BatchKArgs &a, uint32_t n, uint32_t wave,
                                           uint32_t nwaves) {
    const uint32_t lane = threadIdx.x & 63u;
    const BatchItem *list = a.items + size_t(2) * a.max_msgs;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(lane);
    constexpr uint32_t kPerWave = 16;   // quads per wave
    const uint64_t statics = uint64_t(nwaves) * kPerWave;
    uint64_t t0 = uint64_t(wave) * kPerWave;
    while (t0 < n) {
        const uint64_t t = t0 + (lane >> 2);
        // the four lanes of a quad take the same message, so they are active together
        if (t < n) {
            const BatchItem item = list[t];
            const int nr = desc_nr(a.desc[item.msg]);
            if (nr == 10)
                serial_message<10>(lds, lc, a, item);
            else if (nr == 12)
                serial_message<12>(lds, lc, a, item);
            else
                serial_message<14>(lds, lc, a, item);
        }
        if (n <= statics)
            break;
        uint64_t c = 0;
        if (lane == 0)
            c = atomicAdd(reinterpret_cast<unsigned long long *>(&a.header->next[2]), uint64_t(kPerWave));
        t0 = statics + uniform64(c);
    }
}

// Block index of message item `start` (its first cost unit) at which a share
// boundary x falls: the blocks whose cost units begin before x, rounded up to
// the split step, within [0, nblk].  Both neighbours of a boundary evaluate
// it the same way, so the shares partition every message exactly.
__device__ __forceinline__ uint64_t split_point(uint64_t x, uint64_t start, uint64_t unit, uint64_t step,
                                                uint64_t nblk) {
    if (x <= start)
        return 0;
    // unit is block_cost: Nr + 2, so 12, 14 or 16 for a valid descriptor; step
    // is mostly a power of two: constant divisors and masks instead of a
    // general 64-bit division
    const uint64_t v = x - start + unit - 1;
    uint64_t b = unit == 12 ? v / 12 : unit == 14 ? v / 14 : v / 16;
    if ((step & (step - 1)) == 0) {
        b = (b + step - 1) & ~(step - 1);
    } else {
        b = (b + step - 1) / step * step;
    }
    return b < nblk ? b : nblk;
}

// The item holding cost unit x: the last item whose start is <= x (items
// are in order of start; the first starts at 0).  A 64-way search: each step
// every lane tests one of 64 evenly spaced items and the ballot narrows the
// range to the gap between two of them.
__device__ __forceinline__ uint32_t find_item(const BatchItem *list, uint32_t n, uint64_t x) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t span = hi - lo;
        const uint32_t p = lo + uint32_t((uint64_t(lane) * span) >> 6);
        // the starts do not decrease, so the lanes that pass are 0 .. L
        const uint64_t pass = __ballot(list[p].start <= x);
        const int L = 63 - __builtin_clzll(pass);
        const uint32_t nlo = uint32_t(__builtin_amdgcn_readlane(int(p), L));
        hi = L == 63 ? hi : uint32_t(__builtin_amdgcn_readlane(int(p), L + 1));
        lo = nlo;
    }
    return lo;
}

// Cost units per share, roughly: a list larger than one share per wave is
// cut into rounds of nwaves shares, wave w taking share w of every round, so
// that at any time all waves work in the same region (a few hundred MiB)
// instead of each streaming through its own part of the whole batch.
constexpr uint64_t kShareCost = 4096 * 16;
// A list of at least this many rounds (some milliseconds of work) hands out
// the shares of its second half of rounds from a counter instead: over a
// long kernel the waves drift apart in speed, and the waves that are ahead
// take the rest.  Shorter lists are split statically only, without atomics.
constexpr uint64_t kDynamicMinRounds = 8;

// Blocks per thread of XTS pieces: four in the forward kernel (4 KiB one-unit
// sector messages: 1 step of 256 blocks instead of 2 of 128, 853-858 ->
// 881 GB/s); two in the inverse kernel, where the tweak work's registers
// on top of four blocks per thread spill.
template <int CLASS>
constexpr int kXtsBpt = CLASS == 0 ? 4 : 2;

// Share s of S over a list of total cost C: the cost units
// [s C / S, (s+1) C / S), from the item holding its start through the one
// holding its end.
template <int CLASS, int BPT>
__device__ __forceinline__ void run_share(const uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a,
                                          const BatchItem *list, uint32_t n, uint64_t C, uint64_t s, uint64_t S) {
    const uint64_t lo = mul_div_floor(s, C, S), hi = mul_div_floor(s + 1, C, S);
    if (lo < hi) {
        for (uint32_t i = uniform32(find_item(list, n, lo)); i < n; i++) {
            const uint64_t start = uniform64(list[i].start);
            if (start >= hi)
                break;
            const uint32_t msg = uniform32(list[i].msg);
            const aes_msg_desc d = a.desc[msg];
            const uint64_t nblk = (d.nbytes + 15) >> 4, unit = block_cost(d), step = split_step(d, a.split_blocks);
            const uint64_t first = uniform64(split_point(lo, start, unit, step, nblk));
            const uint64_t end = uniform64(split_point(hi, start, unit, step, nblk));
            if (first >= end)
                continue;
            const int nr = desc_nr(d);
            if (d.mode == AES_MODE_XTS) {
                constexpr int XDIR = CLASS == 0 ? DIR_ENC : DIR_DEC;
                if (nr == 10) run_xts_range<10, XDIR, kXtsBpt<CLASS>>(lds, lc, a, d, msg, first, end);
                else if (nr == 12) run_xts_range<12, XDIR, kXtsBpt<CLASS>>(lds, lc, a, d, msg, first, end);
                else run_xts_range<14, XDIR, kXtsBpt<CLASS>>(lds, lc, a, d, msg, first, end);
            } else if (CLASS == 1 && d.mode == AES_MODE_CBC) {
                if (nr == 10) run_range<10, MODE_CBC, DIR_DEC, BPT>(lds, lc, a, d, msg, first, end);
                else if (nr == 12) run_range<12, MODE_CBC, DIR_DEC, BPT>(lds, lc, a, d, msg, first, end);
                else run_range<14, MODE_CBC, DIR_DEC, BPT>(lds, lc, a, d, msg, first, end);
            } else if (CLASS == 1) {
                if (nr == 10) run_range<10, MODE_ECB, DIR_DEC, BPT>(lds, lc, a, d, msg, first, end);
                else if (nr == 12) run_range<12, MODE_ECB, DIR_DEC, BPT>(lds, lc, a, d, msg, first, end);
                else run_range<14, MODE_ECB, DIR_DEC, BPT>(lds, lc, a, d, msg, first, end);
            } else if (d.mode == AES_MODE_ECB) {
                if (nr == 10) run_range<10, MODE_ECB, DIR_ENC, BPT>(lds, lc, a, d, msg, first, end);
                else if (nr == 12) run_range<12, MODE_ECB, DIR_ENC, BPT>(lds, lc, a, d, msg, first, end);
                else run_range<14, MODE_ECB, DIR_ENC, BPT>(lds, lc, a, d, msg, first, end);
            } else {
                if (nr == 10) run_range<10, MODE_CTR, DIR_ENC, BPT>(lds, lc, a, d, msg, first, end);
                else if (nr == 12) run_range<12, MODE_CTR, DIR_ENC, BPT>(lds, lc, a, d, msg, first, end);
                else run_range<14, MODE_CTR, DIR_ENC, BPT>(lds, lc, a, d, msg, first, end);
            }
        }
    }
}

// A wave's part of the forward (CLASS 0) or inverse (CLASS 1) list: share w
// of every static round, then (long lists only) shares of the remaining
// rounds taken off the list's counter until none is left.
template <int CLASS, int BPT>
__device__ __forceinline__ void run_shares(const uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a,
                                           uint32_t n, uint32_t wave, uint32_t nwaves) {
    const uint64_t C = a.header->cost[CLASS];
    if (C == 0)
        return;
    const uint64_t per_round = uint64_t(nwaves) * kShareCost;
    const uint64_t rounds = max<uint64_t>(1, (C + per_round - 1) / per_round);
    const uint64_t dynamic = rounds >= kDynamicMinRounds ? rounds / 2 : 0;
    const uint64_t S = rounds * nwaves, S_static = (rounds - dynamic) * nwaves;
    const BatchItem *list = a.items + size_t(CLASS) * a.max_msgs;
    for (uint64_t s = wave; s < S_static; s += nwaves)
        run_share<CLASS, BPT>(lds, lc, a, list, n, C, s, S);
    if (dynamic == 0)
        return;
    const uint32_t lane = threadIdx.x & 63u;
    for (;;) {
        uint64_t c = 0;
        if (lane == 0)
            c = atomicAdd(reinterpret_cast<unsigned long long *>(&a.header->next[CLASS]), 1ull);
        const uint64_t s = S_static + uniform64(c);
        if (s >= S)
            break;
        run_share<CLASS, BPT>(lds, lc, a, list, n, C, s, S);
    }
}

// One per list: CLASS 0 runs the serial list and then its shares of the
// forward list with the encryption tables, CLASS 1 its shares of the inverse
// list with the decryption tables.  Persistent: one workgroup per compute
// unit, every wave with its own shares.
template <int CLASS, int BPT>
__global__ __launch_bounds__(kBatchWavesPerGroup * 64) void batch_kernel(const BatchKArgs a) {
    constexpr int DIR = CLASS == 0 ? DIR_ENC : DIR_DEC;
    const uint32_t n = a.header->nitems[CLASS];
    const uint32_t nserial = CLASS == 0 ? a.header->nitems[2] : 0u;
    if (n == 0 && nserial == 0)
        return;
    __shared__ uint32_t lds[lds_words<DIR>()];
    stage_tables<LAYOUT_T4X32, DIR>(lds);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(lane);
    const uint32_t wave = blockIdx.x * kBatchWavesPerGroup + uniform32(threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * kBatchWavesPerGroup;
    if (CLASS == 0 && nserial)
        run_serial(lds, a, nserial, wave, nwaves);
    if (n)
        run_shares<CLASS, BPT>(lds, lc, a, n, wave, nwaves);
}

// ---- GCM: GHASH pieces and tags ----------------------------------------------
// LDS of the GHASH kernel: per wave, one multiplier's table (16 waves x
// 8 KiB = 128 KiB per workgroup, one workgroup per compute unit like the
// cipher kernels: 4,096 waves, which the usual piece counts divide evenly).
constexpr uint32_t kGhashWaveBytes = kTabBytes;
constexpr int kGhashWavesPerGroup = kBatchWavesPerGroup;

__device__ __forceinline__ u32x4 load16_masked(const uint8_t *p, bool whole, uint32_t tail) {
    return whole ? load16(p) : load_tail(p, tail);
}

// GHASH position r of a GCM message, numbered from the end of the hashed
// sequence (so that the sum is H * sum_r X_r H^r): r = 0 the length block,
// 1 .. nC ciphertext block nC - r, nC + 1 .. nC + nA additional-data block
// nC + nA - r; partial blocks zero-padded.  `ct` points at the ciphertext
// (the input when decrypting, the output when encrypting).
__device__ __forceinline__ u32x4 ghash_block(uint64_t r, uint64_t nC, uint64_t nA, const uint8_t *ct, uint64_t cbytes,
                                             const uint8_t *aad, uint64_t abytes) {
    if (r == 0) {
        const uint64_t abits = 8 * abytes, cbits = 8 * cbytes;
        return vec4(__builtin_bswap32(uint32_t(abits >> 32)), __builtin_bswap32(uint32_t(abits)),
                    __builtin_bswap32(uint32_t(cbits >> 32)), __builtin_bswap32(uint32_t(cbits)));
    }
    if (r <= nC) {
        const uint64_t j = nC - r;
        return load16_masked(ct + 16 * j, j < (cbytes >> 4), uint32_t(cbytes & 15u));
    }
    const uint64_t k = nC + nA - r;
    return load16_masked(aad + 16 * k, k < (abytes >> 4), uint32_t(abytes & 15u));
}

// One wave: piece `piece` of GCM message `msg`, positions [p_lo, p_hi), as
// sum_(r in piece) X_r H^(r + 1), XORed into the message's sum.  Lane l
// takes positions p_lo + 64q + l, Horner over q from the top with the
// multiplier G = H^64 (one table); the lanes are folded with H, H^2, ..,
// H^32 (a tree, each level's table built in the same space); the result is
// multiplied by H and by H^(p_lo) = product of the stored powers
// H^(kGhashPiece 2^t) over the set bits t of the piece index (products by
// the whole wave).
__device__ __forceinline__ void ghash_piece(uint32_t *lds, uint32_t tab, const BatchKArgs &a,
                                            uint32_t msg, uint64_t piece) {
    const uint32_t lane = threadIdx.x & 63u;
    const aes_msg_desc d = a.desc[msg];
    const aes_gcm_desc g = a.gcm[msg];
    const uint64_t nC = (d.nbytes + 15) >> 4, nA = (g.aad_bytes + 15) >> 4;
    const uint64_t npos = nC + nA + 1;
    const uint64_t p_lo = piece * kGhashPiece;
    const uint64_t p_hi = min(npos, p_lo + kGhashPiece);
    const uint8_t *ct = d.decrypt ? static_cast<const uint8_t *>(a.in_base) + d.in_off
                                  : static_cast<const uint8_t *>(a.out_base) + d.out_off;
    const uint8_t *aad = static_cast<const uint8_t *>(a.in_base) + g.aad_off;
    uint32_t *slot = a.keytab + size_t(msg) * kKeySlotWords;
    const uint32_t h[4] = {uniform32(slot[kGcmSlotH]), uniform32(slot[kGcmSlotH + 1]), uniform32(slot[kGcmSlotH + 2]),
                           uniform32(slot[kGcmSlotH + 3])};
    uint64_t hlo, hhi;
    to_poly(h, hlo, hhi);
    uint64_t glo = hlo, ghi = hhi;
    for (int t = 0; t < 6; t++)
        gf_square(glo, ghi);
    uint32_t gw[4];
    from_poly(glo, ghi, gw);
    build_table_wave(lds, tab, gw);
    // X_r for the Horner steps, kPrefetch steps ahead: every lane loads 16
    // bytes from an address that is always valid (a whole block of the
    // message, else its key slot) and picks the value when the step comes,
    // so the loads' latency is not waited out step by step; the length block
    // and the partial last blocks are formed once
    const uint64_t cbytes = d.nbytes, abytes = g.aad_bytes, nCw = cbytes >> 4, nAw = abytes >> 4;
    const bool has_ctail = (cbytes & 15u) != 0, has_atail = (abytes & 15u) != 0;
    const u32x4 ctail = has_ctail ? load_tail(ct + 16 * nCw, uint32_t(cbytes & 15u)) : vec4(0, 0, 0, 0);
    const u32x4 atail = has_atail ? load_tail(aad + 16 * nAw, uint32_t(abytes & 15u)) : vec4(0, 0, 0, 0);
    const u32x4 lenblk = ghash_block(0, nC, nA, ct, cbytes, aad, abytes);
    const uint8_t *dummy = reinterpret_cast<const uint8_t *>(slot);
    auto load_at = [&](uint64_t q) -> u32x4 {
        const uint64_t r = p_lo + 64 * q + lane, j = nC - r, k = nC + nA - r;
        const uint8_t *p = (r >= 1 && r <= nC && j < nCw) ? ct + 16 * j
                         : (r > nC && r < p_hi && k < nAw) ? aad + 16 * k : dummy;
        return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    };
    auto pick = [&](uint64_t q, u32x4 v) -> u32x4 {
        const uint64_t r = p_lo + 64 * q + lane;
        const bool is_len = r == 0, is_ct = r == 1 && has_ctail, is_at = r == nC + 1 && has_atail;
        const bool out = r >= p_hi;
        auto sel = [&](uint32_t vw, uint32_t lw, uint32_t cw, uint32_t aw) {
            const uint32_t x = is_len ? lw : is_ct ? cw : is_at ? aw : vw;
            return out ? 0u : x;
        };
        return vec4(sel(v.x, lenblk.x, ctail.x, atail.x), sel(v.y, lenblk.y, ctail.y, atail.y),
                    sel(v.z, lenblk.z, ctail.z, atail.z), sel(v.w, lenblk.w, ctail.w, atail.w));
    };
    // the stored powers H^(kGhashPiece 2^t) for the piece's factor below,
    // one vector load for all of them (lane t holds power t) issued here, so
    // that its latency passes during the hashing
    const u32x4 pows = *reinterpret_cast<const u32x4 *>(
        slot + kGcmSlotPow + 4 * (lane < uint32_t(kGcmSlotPowers) ? lane : 0u));
    constexpr int kPrefetch = 2;
    uint32_t w[4] = {0, 0, 0, 0};
    if (p_lo >= 2 && p_lo + kGhashPiece <= nC + 1) {
        // a whole piece of whole ciphertext blocks (neither the length block
        // nor a partial last block, no additional data): step s (q = 63 - s)
        // reads the 1 KiB at p0 + 1024 s, no position tests
        constexpr uint32_t kSteps = uint32_t(kGhashPiece >> 6);
        constexpr uint32_t kAhead = uint32_t(kPrefetch);
        const uint8_t *p0 = ct + 16 * (nC - p_lo - (kGhashPiece - 64) - lane);
        auto ld = [&](uint32_t s) {
            return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p0 + 1024u * s));
        };
        u32x4 v[kAhead];
#pragma unroll
        for (uint32_t i = 0; i < kAhead; i++)
            v[i] = ld(i);
        for (uint32_t s = 0; s < kSteps; s++) {
            const u32x4 vn = ld(min(s + kAhead, kSteps - 1));   // always a block of the piece
            uint32_t t[4];
            mul_tab(lds, tab, w, t);
            w[0] = t[0] ^ v[0].x;
            w[1] = t[1] ^ v[0].y;
            w[2] = t[2] ^ v[0].z;
            w[3] = t[3] ^ v[0].w;
#pragma unroll
            for (uint32_t i = 0; i + 1 < kAhead; i++)
                v[i] = v[i + 1];
            v[kAhead - 1] = vn;
        }
    } else {
        const uint64_t steps = (p_hi - p_lo + 63) >> 6;
        u32x4 v[kPrefetch];
#pragma unroll
        for (int i = 0; i < kPrefetch; i++)
            v[i] = steps > uint64_t(i) ? load_at(steps - 1 - i) : vec4(0, 0, 0, 0);
        for (uint64_t q = steps; q-- > 0;) {
            const u32x4 vn = q >= uint64_t(kPrefetch) ? load_at(q - kPrefetch) : vec4(0, 0, 0, 0);
            uint32_t t[4];
            mul_tab(lds, tab, w, t);
            const u32x4 x = pick(q, v[0]);
            w[0] = t[0] ^ x.x;
            w[1] = t[1] ^ x.y;
            w[2] = t[2] ^ x.z;
            w[3] = t[3] ^ x.w;
#pragma unroll
            for (int i = 0; i + 1 < kPrefetch; i++)
                v[i] = v[i + 1];
            v[kPrefetch - 1] = vn;
        }
    }
    // sum_l w_l H^l over the lanes
    uint64_t plo = hlo, phi = hhi;
    for (int k = 0; k < 6; k++) {
        uint32_t pw[4];
        from_poly(plo, phi, pw);
        build_table_wave(lds, tab, pw);
        uint32_t v[4];
#pragma unroll
        for (int c = 0; c < 4; c++)
            v[c] = uint32_t(__shfl_down(int(w[c]), 1u << k, 64));
        mul_tab(lds, tab, v, v);
#pragma unroll
        for (int c = 0; c < 4; c++)
            w[c] ^= v[c];
        gf_square(plo, phi);
    }
    // times H^(p_lo + 1): lane 0's sum, the same in every lane
    const uint32_t s0[4] = {uniform32(w[0]), uniform32(w[1]), uniform32(w[2]), uniform32(w[3])};
    uint64_t rlo, rhi, blo = 0, bhi = 0;
    to_poly(s0, rlo, rhi);
    mul_wave(rlo, rhi, hlo, hhi, rlo, rhi);
    for (int t = 0; (piece >> t) != 0; t++) {
        if (t < kGcmSlotPowers) {
            const uint32_t pw[4] = {uint32_t(__builtin_amdgcn_readlane(int(pows.x), t)),
                                    uint32_t(__builtin_amdgcn_readlane(int(pows.y), t)),
                                    uint32_t(__builtin_amdgcn_readlane(int(pows.z), t)),
                                    uint32_t(__builtin_amdgcn_readlane(int(pows.w), t))};
            to_poly(pw, blo, bhi);
        } else {
            gf_square(blo, bhi);   // beyond the stored powers (messages over 2^(12+13) blocks)
        }
        if ((piece >> t) & 1)
            mul_wave(rlo, rhi, blo, bhi, rlo, rhi);
    }
    uint32_t res[4];
    from_poly(rlo, rhi, res);
    if (lane == 0) {
        // two 64-bit atomics (the sum sits at an 8-byte aligned offset of the
        // 512-byte slot): the pieces of one message all XOR into the same line
        unsigned long long *sum = reinterpret_cast<unsigned long long *>(slot + kGcmSlotSum);
        atomicXor(sum, (unsigned long long)res[0] | ((unsigned long long)res[1] << 32));
        atomicXor(sum + 1, (unsigned long long)res[2] | ((unsigned long long)res[3] << 32));
    }
}

// Persistent: wave w of NW takes pieces w, w + NW, w + 2 NW, ... of the
// GHASH list (every GCM message's pieces, in message order).
__global__ __launch_bounds__(kGhashWavesPerGroup * 64) void ghash_kernel(const BatchKArgs a) {
    const uint32_t n = a.header->ngcm;
    const uint64_t npieces = a.header->gcm_pieces;
    if (n == 0)
        return;
    __shared__ uint32_t lds[kGhashWavesPerGroup * kGhashWaveBytes / 4];
    const uint32_t wv = uniform32(threadIdx.x >> 6);
    const uint32_t tab = wv * kGhashWaveBytes;
    const uint64_t wave = uint64_t(blockIdx.x) * kGhashWavesPerGroup + wv;
    const uint64_t nwaves = uint64_t(gridDim.x) * kGhashWavesPerGroup;
    const BatchItem *list = a.items + size_t(3) * a.max_msgs;
    for (uint64_t p = wave; p < npieces; p += nwaves) {
        const uint32_t i = uniform32(find_item(list, n, p));
        const uint32_t msg = uniform32(list[i].msg);
        ghash_piece(lds, tab, a, msg, p - uniform64(list[i].start));
    }
}

// ---- GHASH of short messages, four lanes per message -----------------------
// For batches of many short GCM messages (lane_ghash) the four lanes of a
// quad hash one message whole, in four interleaved Horner chains: lane p of
// the quad takes the positions r = 4s + p, Z_p <- Z_p G ^ X_(4s+p) for s from
// the top down, with G = H^4, so that Z_p = sum_s X_(4s+p) G^s; the sum over
// all r of X_r H^(r+1) is then H (Z_0 ^ H (Z_1 ^ H (Z_2 ^ H Z_3))), which every
// lane of the quad forms from the four Z_p (the first one writes it).
// Products go through 4-bit tables of the lane's own copy of the multiplier M
// in arithmetic form (gf128.h): T[v] = v M for the 16 nibble values v, 256
// bytes per lane, 16 KiB per wave, so that ten waves fit on a compute unit
// and cover each other's latencies.  Entry v of lane l sits at byte
// v * 1024 + l * 16, so the 16-byte reads of any 16 neighbouring lanes fall
// on 16 different bank groups, whatever entries they read.  A product Y M is
// the sum over the 32 nibbles of Y, nibble 8q + c (bits 4c .. 4c+3 of word
// q), of T[nibble] x^(32q + 4c): the word shift is where the entry is added
// (an accumulator per nibble position c, seven words long), the shifts by 4c
// are applied once per product, and the 256-bit sum is reduced modulo
// x^128 + x^7 + x^2 + x + 1.
constexpr uint32_t kLaneEntryStride = 64u * 16u;             // one entry of every lane
constexpr uint32_t kLaneTabBytes = 16u * kLaneEntryStride;   // 16 KiB per wave
constexpr uint32_t kLaneMsgsPerWave = 16;                    // a quad of lanes each

// The lane's table of the multiplier (lo, hi), at byte offset `base` =
// 16 * lane.
__device__ __forceinline__ void lane_build(uint32_t *lds, uint32_t base, uint64_t lo, uint64_t hi) {
    uint32_t p[4][4];   // M x^t for t < 4
#pragma unroll
    for (int t = 0; t < 4; t++) {
        p[t][0] = uint32_t(lo);
        p[t][1] = uint32_t(lo >> 32);
        p[t][2] = uint32_t(hi);
        p[t][3] = uint32_t(hi >> 32);
        mulx_small(lo, hi, 1);
    }
#pragma unroll
    for (uint32_t v = 0; v < 16; v++) {
        uint32_t e[4] = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if ((v >> t) & 1u) {
#pragma unroll
                for (int c = 0; c < 4; c++)
                    e[c] ^= p[t][c];
            }
        }
        lds_store16(lds, base + v * kLaneEntryStride, vec4(e[0], e[1], e[2], e[3]));
    }
}

// Byte offset of the entry for the nibble at bits s .. s+3 of y (s is a
// constant once the callers' loops are unrolled).
__device__ __forceinline__ uint32_t lane_entry(uint32_t y, int s, uint32_t base) {
    constexpr int kPos = 10;   // log2(kLaneEntryStride)
    const uint32_t shifted = s <= kPos ? y << (kPos - s) : y >> (s - kPos);
    return (shifted & (15u << kPos)) | base;
}

// z = y M through the lane's table (both in arithmetic form).
__device__ __forceinline__ void lane_mul(const uint32_t *lds, uint32_t base, const uint32_t (&y)[4],
                                         uint32_t (&z)[4]) {
    // acc[c][w]: word w of sum_q entry(nibble 8q + c) x^(32q), from the
    // words w - q of the entries
    uint32_t acc[8][7];
#pragma unroll
    for (int c = 0; c < 8; c++) {
        u32x4 e[4];
#pragma unroll
        for (int q = 0; q < 4; q++)
            e[q] = lds_load16(lds, lane_entry(y[q], 4 * c, base));
        acc[c][0] = e[0].x;
        acc[c][1] = e[0].y ^ e[1].x;
        acc[c][2] = xor3(e[0].z, e[1].y, e[2].x);
        acc[c][3] = xor3(e[0].w, e[1].z, e[2].y) ^ e[3].x;
        acc[c][4] = xor3(e[1].w, e[2].z, e[3].y);
        acc[c][5] = e[2].w ^ e[3].z;
        acc[c][6] = e[3].w;
    }
    // s = sum_c acc[c] x^(4c), 256 bits: per word the eight shifted terms
    uint32_t s[8];
#pragma unroll
    for (int w = 0; w < 8; w++) {
        uint32_t t[8];
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const uint32_t hiw = w < 7 ? acc[c][w] : 0u, low = w > 0 ? acc[c][w - 1] : 0u;
            t[c] = c == 0 ? hiw : __builtin_amdgcn_alignbit(hiw, low, uint32_t(32 - 4 * c));   // (hiw:low) >> (32 - 4c)
        }
        s[w] = xor3(xor3(xor3(t[0], t[1], t[2]), t[3], t[4]), t[5], t[6]) ^ t[7];
    }
    // s mod P: the upper half U folds back as U (1 + x + x^2 + x^7); the at
    // most 7 bits that leaves above x^127 (o) fold back once more
    const uint32_t u[4] = {s[4], s[5], s[6], s[7]};
    uint32_t s1[4], s2[4], s7[4];
    s1[0] = u[0] << 1;
    s2[0] = u[0] << 2;
    s7[0] = u[0] << 7;
#pragma unroll
    for (int j = 1; j < 4; j++) {
        s1[j] = __builtin_amdgcn_alignbit(u[j], u[j - 1], 31u);
        s2[j] = __builtin_amdgcn_alignbit(u[j], u[j - 1], 30u);
        s7[j] = __builtin_amdgcn_alignbit(u[j], u[j - 1], 25u);
    }
    const uint32_t o = xor3(u[3] >> 31, u[3] >> 30, u[3] >> 25);
#pragma unroll
    for (int j = 0; j < 4; j++)
        z[j] = xor3(xor3(s[j], u[j], s1[j]), s2[j], s7[j]);
    z[0] ^= xor3(o, o << 1, o << 2) ^ (o << 7);
}

// One wave per workgroup, kLaneMsgsPerWave messages per wave: workgroup g
// takes messages 16g .. 16g + 15 from the back of the GHASH list, a quad of
// lanes each.
__global__ __launch_bounds__(64) void ghash_lane_kernel(const BatchKArgs a) {
    const uint32_t n = a.header->nlane;
    const uint32_t first = blockIdx.x * kLaneMsgsPerWave;
    if (first >= n)
        return;
    __shared__ uint32_t lds[kLaneTabBytes / 4];
    const uint32_t lane = threadIdx.x, chain = lane & 3u;
    const uint32_t base = lane * 16u;
    const BatchItem *list = a.items + size_t(3) * a.max_msgs;
    const uint32_t i = first + (lane >> 2);
    const bool on = i < n;
    uint32_t msg = 0;
    uint64_t nC = 0, nA = 0, cbytes = 0, abytes = 0;
    const uint8_t *ct = nullptr, *aad = nullptr;
    uint32_t h[4] = {0, 0, 0, 0};
    if (on) {
        msg = list[size_t(a.max_msgs) - 1 - i].msg;
        const aes_msg_desc d = a.desc[msg];
        const aes_gcm_desc gd = a.gcm[msg];
        cbytes = d.nbytes;
        abytes = gd.aad_bytes;
        nC = (cbytes + 15) >> 4;
        nA = (abytes + 15) >> 4;
        ct = d.decrypt ? static_cast<const uint8_t *>(a.in_base) + d.in_off
                       : static_cast<const uint8_t *>(a.out_base) + d.out_off;
        aad = static_cast<const uint8_t *>(a.in_base) + gd.aad_off;
        const uint32_t *slot = a.keytab + size_t(msg) * kKeySlotWords;
#pragma unroll
        for (int c = 0; c < 4; c++)
            h[c] = slot[kGcmSlotH + c];
    }
    uint64_t hlo, hhi;
    to_poly(h, hlo, hhi);
    uint64_t glo = hlo, ghi = hhi;   // G = H^4
    gf_square(glo, ghi);
    gf_square(glo, ghi);
    lane_build(lds, base, glo, ghi);
    // a wave's LDS accesses complete in order; the fences only keep the
    // compiler from moving the table reads above the writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // steps of the longest message of the wave; a shorter one keeps Z_p = 0
    // (and X = 0) until its own top position
    const uint32_t npos = on ? uint32_t(nC + nA + 1) : 0u;
    uint32_t top = npos;
#pragma unroll
    for (int off = 32; off >= 4; off >>= 1)
        top = max(top, uint32_t(__shfl_xor(int(top), off, 64)));
    const uint32_t steps = uniform32((top + 3) / 4);
    // X_r of this lane's message, zero from its top position on.  The partial
    // last blocks of the ciphertext (position 1) and of the additional data
    // (position nC + 1) are read here, zero-padded; in the loop every lane
    // loads 16 bytes from an address that is always valid (a whole block of
    // its message, else its own key slot) and picks the value one step
    // later, so no load waits where it is issued.  Plain (cached) loads: the
    // four lanes of a quad read 64 neighbouring bytes.
    const uint64_t nCw = cbytes >> 4, nAw = abytes >> 4;
    const u32x4 ctail = (cbytes & 15u) ? load_tail(ct + 16 * nCw, uint32_t(cbytes & 15u)) : vec4(0, 0, 0, 0);
    const u32x4 atail = (abytes & 15u) ? load_tail(aad + 16 * nAw, uint32_t(abytes & 15u)) : vec4(0, 0, 0, 0);
    const u32x4 lenblk = ghash_block(0, nC, nA, ct, cbytes, aad, abytes);
    const uint8_t *dummy = reinterpret_cast<const uint8_t *>(a.keytab + size_t(msg) * kKeySlotWords);
    auto load_at = [&](uint32_t r) -> u32x4 {
        const uint64_t j = nC - r, k = nC + nA - r;
        const uint8_t *p = (r >= 1 && r <= nC && j < nCw) ? ct + 16 * j
                         : (r > nC && r < npos && k < nAw) ? aad + 16 * k : dummy;
        return *reinterpret_cast<const u32x4 *>(p);
    };
    auto pick = [&](uint32_t r, u32x4 v) -> u32x4 {
        if (r >= npos)
            return vec4(0, 0, 0, 0);
        if (r == 0)
            return lenblk;
        if (r == 1 && (cbytes & 15u))
            return ctail;
        if (r == nC + 1 && (abytes & 15u))
            return atail;
        return v;
    };
    uint32_t z[4] = {0, 0, 0, 0};
    u32x4 v = load_at(steps ? 4 * (steps - 1) + chain : 0);
    for (uint32_t st = steps; st-- > 0;) {
        const u32x4 vn = load_at(st ? 4 * (st - 1) + chain : 0);   // one step ahead
        uint32_t t[4];
        lane_mul(lds, base, z, t);
        const u32x4 x = pick(4 * st + chain, v);
        z[0] = t[0] ^ rev_bits_in_bytes(x.x);
        z[1] = t[1] ^ rev_bits_in_bytes(x.y);
        z[2] = t[2] ^ rev_bits_in_bytes(x.z);
        z[3] = t[3] ^ rev_bits_in_bytes(x.w);
        v = vn;
    }
    // H (Z_0 ^ H (Z_1 ^ H (Z_2 ^ H Z_3))) with the table of H, in every lane
    // of the quad
    uint32_t zq[4][4];
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int c = 0; c < 4; c++)
            zq[p][c] = uint32_t(__shfl(int(z[c]), int((lane & ~3u) | uint32_t(p)), 64));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    lane_build(lds, base, hlo, hhi);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t w[4] = {zq[3][0], zq[3][1], zq[3][2], zq[3][3]};
#pragma unroll
    for (int p = 2; p >= -1; p--) {
        uint32_t t[4];
        lane_mul(lds, base, w, t);
#pragma unroll
        for (int c = 0; c < 4; c++)
            w[c] = p >= 0 ? t[c] ^ zq[p][c] : t[c];
    }
    if (on && chain == 0) {
        uint32_t *slot = a.keytab + size_t(msg) * kKeySlotWords;
#pragma unroll
        for (int c = 0; c < 4; c++)
            slot[kGcmSlotSum + c] = rev_bits_in_bytes(w[c]);
    }
}

// ---- GCM: large messages encrypted and hashed in one pass -----------------
// A GCM message of at least kFusedMinPositions GHASH positions is cut into
// pieces of kFusedPiece positions (numbered from the end as in ghash_block:
// piece f holds r = kFusedPiece f .. kFusedPiece (f + 1) - 1), and one
// workgroup takes a piece whole, with the AES tables and the table of
// G = H^256 in LDS.  Wave w takes the 4,096 positions from
// p_lo + 4,096 w up, 256 at a time from the top down: four slots of 64
// lanes, a Horner chain W_i <- W_i G ^ X_r per slot and lane.  A step of 256
// whole ciphertext blocks is a counter-mode chunk as in the single-buffer
// kernel (load, encrypt, store, hash the ciphertext); any other step goes
// one slot at a time (the length block, partial blocks, additional data,
// positions past the end).  After the loop the AES tables' space holds the
// eleven folding tables: the slots with H^64, the lanes with H, H^2 .. H^32,
// the waves with H^4096 .. H^32768; the workgroup's sum times H^(p_lo + 1)
// is XORed into the message's sum (GHASH is linear), and the AES tables are
// staged again for the next piece.
constexpr uint32_t kFusedAesBytes = 128u * 1024u;
constexpr uint32_t kFusedGTab = kFusedAesBytes;              // G's table, after the AES tables
constexpr uint32_t kFusedPartials = kFusedGTab + kTabBytes;  // the waves' sums
constexpr uint32_t kFusedLdsWords = (kFusedPartials + 16u * kBatchWavesPerGroup) / 4u;
constexpr int kFusedFoldTabs = 11;
constexpr uint64_t kFusedWavePositions = kFusedPiece / kBatchWavesPerGroup;
constexpr int kFusedWaveSteps = int(kFusedWavePositions / 256);
static_assert(kFusedFoldTabs * kTabBytes <= kFusedAesBytes, "the folding tables fit the AES tables' space");
static_assert(kFusedWavePositions == 4096, "the waves' folding tables are H^4096 .. H^32768");

// Piece `piece` of fused GCM message `msg`, by the whole workgroup; the AES
// tables are staged, and G's table is built here when build_g.  Ends with a
// barrier (the next piece stages the tables again).
template <int NR>
__device__ __forceinline__ void fused_piece(uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a, uint32_t msg,
                                            uint64_t piece, bool build_g) {
    const uint32_t lane = threadIdx.x & 63u, wv = uniform32(threadIdx.x >> 6);
    // the message's fields, the same in every lane: kept in scalar registers
    const aes_msg_desc &d = a.desc[msg];
    const aes_gcm_desc &g = a.gcm[msg];
    const bool dec = uniform32(d.decrypt) != 0;
    const uint64_t cbytes = uniform64(d.nbytes), abytes = uniform64(g.aad_bytes);
    const uint64_t nC = (cbytes + 15) >> 4, nA = (abytes + 15) >> 4, npos = nC + nA + 1;
    const uint64_t nCw = cbytes >> 4, nAw = abytes >> 4;
    const uint32_t ctail = uint32_t(cbytes & 15u), atail = uint32_t(abytes & 15u);
    const uint8_t *in = static_cast<const uint8_t *>(a.in_base) + uniform64(d.in_off);
    uint8_t *out = static_cast<uint8_t *>(a.out_base) + uniform64(d.out_off);
    const uint8_t *aad = static_cast<const uint8_t *>(a.in_base) + uniform64(g.aad_off);
    uint32_t *slot = a.keytab + size_t(msg) * kKeySlotWords;
    uint32_t rk[4 * (NR + 1)];
    load_round_keys<NR>(slot, rk);
    const uint32_t h[4] = {uniform32(slot[kGcmSlotH]), uniform32(slot[kGcmSlotH + 1]), uniform32(slot[kGcmSlotH + 2]),
                           uniform32(slot[kGcmSlotH + 3])};
    uint64_t hlo, hhi;
    to_poly(h, hlo, hhi);
    const u32x4 pows = *reinterpret_cast<const u32x4 *>(
        slot + kGcmSlotPow + 4 * (lane < uint32_t(kGcmSlotPowers) ? lane : 0u));
    if (build_g && wv == 0) {
        uint64_t glo = hlo, ghi = hhi;
        for (int t = 0; t < 8; t++)
            gf_square(glo, ghi);
        uint32_t gw[4];
        from_poly(glo, ghi, gw);
        build_table_wave(lds, kFusedGTab, gw);
    }
    __syncthreads();   // the AES tables (staged by the caller) and G's

    // counter blocks: IV || BE32(2 + j) for ciphertext block j (J0 + 1 + j)
    const uint32_t n0 = uniform32(le32(d.ctr0)) ^ rk[0], n1 = uniform32(le32(d.ctr0 + 4)) ^ rk[1],
                   n2 = uniform32(le32(d.ctr0 + 8)) ^ rk[2];
    const uint32_t pre0 = tl<LAYOUT_T4X32, 0, 0>(lds, lc, n0) ^ tl<LAYOUT_T4X32, 1, 1>(lds, lc, n1) ^
                          tl<LAYOUT_T4X32, 2, 2>(lds, lc, n2) ^ rk[4];
    const uint32_t pre1 = tl<LAYOUT_T4X32, 0, 0>(lds, lc, n1) ^ tl<LAYOUT_T4X32, 1, 1>(lds, lc, n2) ^
                          tl<LAYOUT_T4X32, 3, 3>(lds, lc, n0) ^ rk[5];
    const uint32_t pre2 = tl<LAYOUT_T4X32, 0, 0>(lds, lc, n2) ^ tl<LAYOUT_T4X32, 2, 2>(lds, lc, n0) ^
                          tl<LAYOUT_T4X32, 3, 3>(lds, lc, n1) ^ rk[6];
    const uint32_t pre3 = tl<LAYOUT_T4X32, 1, 1>(lds, lc, n0) ^ tl<LAYOUT_T4X32, 2, 2>(lds, lc, n1) ^
                          tl<LAYOUT_T4X32, 3, 3>(lds, lc, n2) ^ rk[7];
    const uint64_t abits = 8 * abytes, cbits = 8 * cbytes;
    const u32x4 lenblk = vec4(__builtin_bswap32(uint32_t(abits >> 32)), __builtin_bswap32(uint32_t(abits)),
                              __builtin_bswap32(uint32_t(cbits >> 32)), __builtin_bswap32(uint32_t(cbits)));
    uint32_t tmask[4];   // bytes of a partial last ciphertext block that enter GHASH
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int keep = int(ctail) - 4 * c;
        tmask[c] = keep >= 4 ? ~0u : keep <= 0 ? 0u : (1u << (8 * keep)) - 1u;
    }

    uint32_t W[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
        W[i][0] = W[i][1] = W[i][2] = W[i][3] = 0;
    // Steps of 256 whole ciphertext blocks: the blocks from `low` up, slot i
    // lane l taking block low + 64 (3 - i) + 63 - l (position rq + 64 i + l).
    auto fast_step = [&](uint64_t rq) __attribute__((always_inline)) {
        const uint64_t low = nC - rq - 255;
        uint32_t x[4][4], s[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const u32x4 v = load16(in + 16 * (low + 64u * uint32_t(3 - i) + (63u - lane)));
            x[i][0] = v.x;
            x[i][1] = v.y;
            x[i][2] = v.z;
            x[i][3] = v.w;
        }
        // rounds 1 and 2: the 256 counters have at most two values of their
        // top 24 bits (A below a multiple of 256, B from it on); the 15
        // lookups that depend only on those bits are done for both
        const uint32_t cb = 2u + uint32_t(low);
        auto shared = [&](uint32_t g3, uint32_t (&qv)[4]) __attribute__((always_inline)) {
            const uint32_t t1 = pre1 ^ tl<LAYOUT_T4X32, 2, 2>(lds, lc, g3);
            const uint32_t t2 = pre2 ^ tl<LAYOUT_T4X32, 1, 1>(lds, lc, g3);
            const uint32_t t3 = pre3 ^ tl<LAYOUT_T4X32, 0, 0>(lds, lc, g3);
            qv[0] = xor3(tl<LAYOUT_T4X32, 1, 1>(lds, lc, t1), tl<LAYOUT_T4X32, 2, 2>(lds, lc, t2),
                         tl<LAYOUT_T4X32, 3, 3>(lds, lc, t3)) ^ rk[8];
            qv[1] = xor3(tl<LAYOUT_T4X32, 0, 0>(lds, lc, t1), tl<LAYOUT_T4X32, 1, 1>(lds, lc, t2),
                         tl<LAYOUT_T4X32, 2, 2>(lds, lc, t3)) ^ rk[9];
            qv[2] = xor3(tl<LAYOUT_T4X32, 0, 0>(lds, lc, t2), tl<LAYOUT_T4X32, 1, 1>(lds, lc, t3),
                         tl<LAYOUT_T4X32, 3, 3>(lds, lc, t1)) ^ rk[10];
            qv[3] = xor3(tl<LAYOUT_T4X32, 0, 0>(lds, lc, t3), tl<LAYOUT_T4X32, 2, 2>(lds, lc, t1),
                         tl<LAYOUT_T4X32, 3, 3>(lds, lc, t2)) ^ rk[11];
        };
        uint32_t qa[4], qb[4];
        shared(__builtin_bswap32(cb) ^ rk[3], qa);
        shared(__builtin_bswap32(cb + 256u) ^ rk[3], qb);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t jj = 64u * uint32_t(3 - i) + (63u - lane);
            const bool b = (cb & 255u) + jj >= 256u;
            const uint32_t v3 = __builtin_bswap32(cb + jj) ^ rk[3];
            const uint32_t t0 = pre0 ^ tl<LAYOUT_T4X32, 3, 3>(lds, lc, v3);
            s[i][0] = (b ? qb[0] : qa[0]) ^ tl<LAYOUT_T4X32, 0, 0>(lds, lc, t0);
            s[i][1] = (b ? qb[1] : qa[1]) ^ tl<LAYOUT_T4X32, 3, 3>(lds, lc, t0);
            s[i][2] = (b ? qb[2] : qa[2]) ^ tl<LAYOUT_T4X32, 2, 2>(lds, lc, t0);
            s[i][3] = (b ? qb[3] : qa[3]) ^ tl<LAYOUT_T4X32, 1, 1>(lds, lc, t0);
        }
        rounds<NR, DIR_ENC, LAYOUT_T4X32, 4>(s, lds, lc, rk, 3);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t o[4] = {x[i][0] ^ s[i][0], x[i][1] ^ s[i][1], x[i][2] ^ s[i][2], x[i][3] ^ s[i][3]};
            store16(out + 16 * (low + 64u * uint32_t(3 - i) + (63u - lane)), vec4(o[0], o[1], o[2], o[3]));
            uint32_t t[4];
            mul_tab(lds, kFusedGTab, W[i], t);
#pragma unroll
            for (int c = 0; c < 4; c++)
                W[i][c] = t[c] ^ (dec ? x[i][c] : o[c]);
        }
    };
    // Any other step, one slot at a time.
    auto slow_step = [&](uint64_t rq) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint64_t r = rq + 64u * uint32_t(i) + lane;
            const bool is_c = r >= 1 && r <= nC;
            const uint64_t j = nC - r;
            u32x4 v = vec4(0, 0, 0, 0);
            if (r == 0) {
                v = lenblk;
            } else if (is_c) {
                v = j < nCw ? load16(in + 16 * j) : load_tail(in + 16 * j, ctail);
            } else if (r < npos) {
                const uint64_t k = nC + nA - r;
                v = k < nAw ? load16(aad + 16 * k) : load_tail(aad + 16 * k, atail);
            }
            uint32_t x[4] = {v.x, v.y, v.z, v.w};
            uint32_t st[1][4] = {{n0, n1, n2, __builtin_bswap32(2u + uint32_t(j)) ^ rk[3]}};
            rounds<NR, DIR_ENC, LAYOUT_T4X32, 1>(st, lds, lc, rk, 1);
            if (is_c) {
                const uint32_t o[4] = {x[0] ^ st[0][0], x[1] ^ st[0][1], x[2] ^ st[0][2], x[3] ^ st[0][3]};
                const bool whole = j < nCw;
                if (whole)
                    store16(out + 16 * j, vec4(o[0], o[1], o[2], o[3]));
                else
                    store_tail(out + 16 * j, vec4(o[0], o[1], o[2], o[3]), ctail);
                if (!dec)
#pragma unroll
                    for (int c = 0; c < 4; c++)
                        x[c] = whole ? o[c] : o[c] & tmask[c];
            }
            uint32_t t[4];
            mul_tab(lds, kFusedGTab, W[i], t);
#pragma unroll
            for (int c = 0; c < 4; c++)
                W[i][c] = t[c] ^ x[c];
            asm volatile("" ::: "memory");   // one slot's work at a time
        }
    };
    const uint64_t p_lo = piece * kFusedPiece;
    const uint64_t w_lo = p_lo + uint64_t(wv) * kFusedWavePositions;
    for (int st = kFusedWaveSteps - 1; st >= 0; st--) {
        const uint64_t rq = w_lo + 256u * uint32_t(st);
        if (rq >= npos)
            continue;   // past the end: the chains are still zero
        if (rq >= 2 && rq + 255 <= nC)
            fast_step(rq);
        else
            slow_step(rq);
    }

    // fold: tables k < 6 hold H^(2^k), table 6 H^64, tables 7 .. 10 H^(4096 2^(k-7))
    __syncthreads();   // every wave is done with the AES tables
    if (wv < uint32_t(kFusedFoldTabs)) {
        const int e = wv < 7 ? int(wv) : int(wv) + 5;
        uint64_t lo = hlo, hi = hhi;
        for (int t = 0; t < e; t++)
            gf_square(lo, hi);
        uint32_t mw[4];
        from_poly(lo, hi, mw);
        build_table_wave(lds, wv * kTabBytes, mw);
    }
    __syncthreads();
    uint32_t u[4] = {W[3][0], W[3][1], W[3][2], W[3][3]};
#pragma unroll
    for (int i = 2; i >= 0; i--) {
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
    if (lane == 0)
        lds_store16(lds, kFusedPartials + 16u * wv, vec4(u[0], u[1], u[2], u[3]));
    __syncthreads();
    if (wv == 0) {
        const u32x4 pv = lane < uint32_t(kBatchWavesPerGroup) ? lds_load16(lds, kFusedPartials + 16u * lane)
                                                              : vec4(0, 0, 0, 0);
        uint32_t y[4] = {pv.x, pv.y, pv.z, pv.w};
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
        // times H^(p_lo + 1): H, times the stored powers H^(4096 2^t) over
        // the set bits t of p_lo / 4096 (= 16 piece)
        const uint32_t s0[4] = {uniform32(y[0]), uniform32(y[1]), uniform32(y[2]), uniform32(y[3])};
        uint64_t rlo, rhi, blo = 0, bhi = 0;
        to_poly(s0, rlo, rhi);
        mul_wave(rlo, rhi, hlo, hhi, rlo, rhi);
        const uint64_t idx = p_lo >> kGhashPieceLog2;
        for (int t = 0; (idx >> t) != 0; t++) {
            if (t < kGcmSlotPowers) {
                const uint32_t pw[4] = {uint32_t(__builtin_amdgcn_readlane(int(pows.x), t)),
                                        uint32_t(__builtin_amdgcn_readlane(int(pows.y), t)),
                                        uint32_t(__builtin_amdgcn_readlane(int(pows.z), t)),
                                        uint32_t(__builtin_amdgcn_readlane(int(pows.w), t))};
                to_poly(pw, blo, bhi);
            } else {
                gf_square(blo, bhi);
            }
            if ((idx >> t) & 1)
                mul_wave(rlo, rhi, blo, bhi, rlo, rhi);
        }
        uint32_t res[4];
        from_poly(rlo, rhi, res);
        if (lane == 0) {
            unsigned long long *sum = reinterpret_cast<unsigned long long *>(slot + kGcmSlotSum);
            atomicXor(sum, (unsigned long long)res[0] | ((unsigned long long)res[1] << 32));
            atomicXor(sum + 1, (unsigned long long)res[2] | ((unsigned long long)res[3] << 32));
        }
    }
    __syncthreads();   // the folding tables are read until here
}

// Persistent, one kernel per key size (one instantiation of the piece each,
// which keeps its registers within four waves per SIMD): every workgroup
// takes the pieces of that key size's messages off a counter, one at a time,
// until none is left.
template <int NR>
__global__ __launch_bounds__(kBatchWavesPerGroup * 64) void gcm_fused_kernel(const BatchKArgs a) {
    constexpr int J = (NR - 10) / 2;
    const uint32_t n = a.header->nfused[J];
    if (n == 0)
        return;
    const uint64_t total = a.header->fused_pieces[J];
    __shared__ uint32_t lds[kFusedLdsWords];
    __shared__ uint64_t next_piece;
    const uint32_t lane = threadIdx.x & 63u;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(lane);
    const uint32_t off = (J > 0 ? a.header->nfused[0] : 0u) + (J > 1 ? a.header->nfused[1] : 0u);
    const BatchItem *list = a.items + size_t(4) * a.max_msgs + off;
    uint32_t have_g = 0xFFFFFFFFu;   // the message whose G table is in LDS
    for (;;) {
        if (threadIdx.x == 0)
            next_piece = atomicAdd(reinterpret_cast<unsigned long long *>(&a.header->next_fused[J]), 1ull);
        __syncthreads();
        const uint64_t p = next_piece;
        if (p >= total)
            break;
        stage_tables<LAYOUT_T4X32, DIR_ENC>(lds);
        const uint32_t i = uniform32(find_item(list, n, p));
        const uint32_t msg = uniform32(list[i].msg);
        const uint64_t piece = p - uniform64(list[i].start);
        const bool build_g = msg != have_g;
        have_g = msg;
        fused_piece<NR>(lds, lc, a, msg, piece, build_g);
    }
}

// One lane per message: every GCM message's tag, Cipher_K(J0) XOR its GHASH
// sum, written after its output (encryption) or compared with the expected
// one (decryption); the verdict goes to the message's aes_gcm_desc.
__global__ __launch_bounds__(256) void gcm_tag_kernel(const BatchKArgs a) {
    const uint32_t n = batch_count(a);
    const uint32_t m = blockIdx.x * 256u + threadIdx.x;
    if (m >= n || !a.gcm)
        return;
    const aes_msg_desc d = a.desc[m];
    if (d.mode != AES_MODE_GCM)
        return;
    if (!desc_valid(d, m, a)) {
        a.gcm[m].ok = 0;
        return;
    }
    const aes_gcm_desc g = a.gcm[m];
    const uint32_t *slot = a.keytab + size_t(m) * kKeySlotWords;
    uint8_t tag[16];
#pragma unroll
    for (int b = 0; b < 16; b++)
        tag[b] = uint8_t((slot[kGcmSlotSum + b / 4] ^ slot[kGcmSlotEJ0 + b / 4]) >> (8 * (b & 3)));
    if (!d.decrypt) {
        uint8_t *t = static_cast<uint8_t *>(a.out_base) + g.tag_off;
#pragma unroll
        for (int b = 0; b < 16; b++)
            t[b] = tag[b];
        a.gcm[m].ok = 1;
    } else {
        const uint8_t *t = static_cast<const uint8_t *>(a.in_base) + g.tag_off;
        uint32_t diff = 0;
        for (uint32_t b = 0; b < g.tag_bytes; b++)
            diff |= uint32_t(tag[b] ^ t[b]);
        a.gcm[m].ok = diff == 0 ? 1 : 0;
    }
}

// ---- synthetic payloads for the request loop ------------------------------
// The payload of a request is the SplitMix64 stream of its seed: word i =
// mix64(seed + (i + 1) * 0x9E3779B97F4A7C15), stored little-endian (Steele,
// Lea and Flood 2014; mix64 is that generator's published output function).
__device__ __forceinline__ uint64_t splitmix_word(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Chunks of kFillChunk bytes, numbered across the batch's messages; every
// workgroup fills whole chunks, rounding each message up to 16 bytes (the
// arena rounds every buffer up to 256).
__global__ __launch_bounds__(256) void fill_kernel(const FillKArgs a) {
    const uint32_t n = uint32_t(*a.d_nmsg);
    const uint64_t nchunks = *a.d_nchunks;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        // the message holding chunk c: the last one whose first chunk is <= c
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (a.fd[mid].chunk_first <= c)
                lo = mid;
            else
                hi = mid;
        }
        const FillDesc d = a.fd[lo];
        const uint64_t start = (c - d.chunk_first) * kFillChunk;
        const uint64_t padded = (d.nbytes + 15) & ~uint64_t(15);
        const uint64_t end = min(start + kFillChunk, padded);
        for (uint64_t b = start + 16u * threadIdx.x; b < end; b += 16u * blockDim.x) {
            const uint64_t w0 = splitmix_word(d.seed, b >> 3), w1 = splitmix_word(d.seed, (b >> 3) + 1);
            store16(a.base + d.off + b, vec4(uint32_t(w0), uint32_t(w0 >> 32), uint32_t(w1), uint32_t(w1 >> 32)));
        }
    }
}

// A small copy from pinned host memory (16 bytes per lane and step).
__global__ __launch_bounds__(256) void stage_kernel(const u32x4 *src, u32x4 *dst, uint64_t n16) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += uint64_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

hipError_t upload_tables_batch(const HostTables &t) { return upload_base_tables(t); }

// The workspace of aes_batch_run_noalloc, for callers that cannot allocate:
// a file-scope device array, held by every device the library runs on until
// the process ends.  Host code never passes the array's name to a kernel or
// copy (in host code it is only a stand-in for the symbol): its device
// address is looked up per device at the device's set-up and kept here.
namespace {
__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];
constexpr int kScratchDevices = 64;
void *g_scratch_ptr[kScratchDevices];
}  // namespace

hipError_t init_batch_scratch(int dev) {
    if (dev < 0 || dev >= kScratchDevices)
        return hipErrorInvalidDevice;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    g_scratch_ptr[dev] = ptr;
    return hipSuccess;
}

void *batch_scratch(int dev) { return dev >= 0 && dev < kScratchDevices ? g_scratch_ptr[dev] : nullptr; }

hipError_t launch_stage(const void *host_dev, void *dev, uint64_t nbytes, hipStream_t stream) {
    const uint64_t n16 = nbytes / 16;
    const uint64_t grid = std::min<uint64_t>(std::max<uint64_t>((n16 + 255) / 256, 1), 64);
    hipLaunchKernelGGL(stage_kernel, dim3(uint32_t(grid)), dim3(256), 0, stream,
                       static_cast<const u32x4 *>(host_dev), static_cast<u32x4 *>(dev), n16);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchKArgs &args, int grid, hipStream_t stream, unsigned lists, int max_count) {
    if (grid < 1 || grid * kBatchWavesPerGroup > kBatchMaxWaves)
        return hipErrorInvalidConfiguration;
    BatchKArgs a = args;
    a.fuse_gcm = (lists & 16u) ? 1u : 0u;
    hipError_t e;
    if (uint64_t(max_count) <= uint64_t(kPlanThreads)) {
        hipLaunchKernelGGL(prep_plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, a);
        e = hipGetLastError();
    } else {
        const int chunks = (a.max_msgs + kPlanThreads - 1) / kPlanThreads;
        hipLaunchKernelGGL(prep_kernel, dim3(chunks), dim3(kPlanThreads), 0, stream, a);
        e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(plan_kernel, dim3(chunks), dim3(kPlanThreads), 0, stream, a);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess || !(lists & 15u))
        return e;
    using BatchFn = void (*)(const BatchKArgs);
    // the forward kernel also runs the serial list
    if (lists & 5u) {
        BatchFn fwd = a.bpt == 2 ? batch_kernel<0, 2> : batch_kernel<0, 4>;
        hipLaunchKernelGGL(fwd, dim3(grid), dim3(kBatchWavesPerGroup * 64), 0, stream, a);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (lists & 2u) {
        BatchFn inv = a.bpt == 2 ? batch_kernel<1, 2> : batch_kernel<1, 4>;
        hipLaunchKernelGGL(inv, dim3(grid), dim3(kBatchWavesPerGroup * 64), 0, stream, a);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    // GCM: the hash reads the ciphertext the forward kernel has written
    if (lists & 8u) {
        if (lists & 16u) {
            for (BatchFn fused : {gcm_fused_kernel<10>, gcm_fused_kernel<12>, gcm_fused_kernel<14>}) {
                hipLaunchKernelGGL(fused, dim3(grid), dim3(kBatchWavesPerGroup * 64), 0, stream, a);
                e = hipGetLastError();
                if (e != hipSuccess)
                    return e;
            }
        }
        hipLaunchKernelGGL(ghash_kernel, dim3(grid), dim3(kGhashWavesPerGroup * 64), 0, stream, a);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        if (uint64_t(max_count) >= kLaneGhashMinMessages) {
            // one wave per workgroup, kLaneMsgsPerWave messages per wave
            const int64_t lane_groups = (int64_t(max_count) + kLaneMsgsPerWave - 1) / kLaneMsgsPerWave;
            hipLaunchKernelGGL(ghash_lane_kernel, dim3(unsigned(lane_groups)), dim3(64), 0, stream, a);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        const int groups = (std::max(max_count, 1) + 255) / 256;
        hipLaunchKernelGGL(gcm_tag_kernel, dim3(groups), dim3(256), 0, stream, a);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_fill(const FillKArgs &a, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace aesgpu
