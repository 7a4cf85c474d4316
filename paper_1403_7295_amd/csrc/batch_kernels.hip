// Batches of independent messages (each with its own key, length, mode and
// direction) in one launch sequence:
//
//   keyexp_kernel   one lane per message: Key Expansion on the device
//                   (FIPS-197 section 5.2), plus the equivalent-inverse
//                   schedule (section 5.3.5) for decryption and the tweak
//                   key's schedule for XTS.
//   plan_kernel     one workgroup: checks every descriptor, cuts each message
//                   into tiles of at most T blocks (a tile never spans two
//                   messages; an XTS tile is whole groups of 64 data units),
//                   and lays the tiles out in three lists: forward (ECB
//                   encryption, CTR, XTS encryption: the encryption tables),
//                   inverse (ECB, CBC and XTS decryption: the inverse ones)
//                   and serial (CBC encryption, one message per tile).
//                   It also zeroes the two tile counters, so the sequence can
//                   be replayed from a graph without any memset.
//   batch_kernel    persistent, one per list: every wave takes the next tile
//                   off its list's counter, reads that message's round keys
//                   into scalar registers and runs the same block loop as the
//                   single-buffer kernels, until the list is empty.
//
// This is the paper's method (cut the data into chunks, process the chunks
// in parallel, Section IV) applied per message, with the chunk size chosen
// for the GPU rather than by the number of cores.
#include <hip/hip_runtime.h>

#include "aesgpu.h"
#include "cipher_core.h"
#include "internal.h"
#include "xts_core.h"

namespace aesgpu {
namespace {

constexpr int kPlanThreads = 1024;

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

// Same test as the host applies to a single-buffer call, plus bounds.
__device__ __forceinline__ bool desc_valid(const aes_msg_desc &d, const BatchKArgs &a) {
    if (d.keybits_code > 2 || d.mode > AES_MODE_XTS || d.decrypt > 1)
        return false;
    if ((d.mode == AES_MODE_ECB || d.mode == AES_MODE_CBC || d.mode == AES_MODE_XTS) && (d.nbytes & 15u))
        return false;
    if (d.mode == AES_MODE_XTS) {
        const uint32_t u = xts_unit_bytes(d);
        if (u < 16 || u > 4096 || (u & (u - 1)) != 0 || xts_key2(d) >= uint32_t(a.nkeys))
            return false;
    }
    // CBC decryption reads block j-1 of the input after other waves may have
    // written their outputs: input and output must not share bytes
    if (d.mode == AES_MODE_CBC && d.decrypt && a.in_base == a.out_base && d.nbytes &&
        d.in_off < d.out_off + d.nbytes && d.out_off < d.in_off + d.nbytes)
        return false;
    // a CBC encryption is one serial tile; its block count must fit the tile
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

// Forward list (encryption tables): ECB encrypt, CTR, XTS encrypt.  Inverse
// list (decryption tables): ECB, CBC and XTS decrypt.  Serial list: CBC
// encrypt.
__device__ __forceinline__ int desc_class(const aes_msg_desc &d) {
    if (d.mode == AES_MODE_CBC)
        return d.decrypt ? 1 : 2;
    return ((d.mode == AES_MODE_ECB || d.mode == AES_MODE_XTS) && d.decrypt) ? 1 : 0;
}

// Blocks per XTS tile: whole groups of 64 data units (the unit of the tweak
// work), as many as fit in the tile size, at least one.
__device__ __forceinline__ uint64_t xts_tile_blocks(const aes_msg_desc &d, uint32_t tile_blocks) {
    const uint64_t group = uint64_t(64) << xts_unit_shift(d);
    const uint64_t g = tile_blocks / group;
    return (g ? g : 1) * group;
}

__device__ __forceinline__ uint32_t batch_count(const BatchKArgs &a) {
    int n = a.d_nmsg ? *a.d_nmsg : a.nmsg;
    if (n < 0)
        n = 0;
    if (n > a.max_msgs)
        n = a.max_msgs;
    return uint32_t(n);
}

__device__ __forceinline__ uint32_t sbox(uint32_t x) { return (g_base[x & 255u] >> 8) & 255u; }

__device__ __forceinline__ uint32_t sub_word(uint32_t w) {
    return sbox(w) | (sbox(w >> 8) << 8) | (sbox(w >> 16) << 16) | (sbox(w >> 24) << 24);
}

// InvMixColumns of a column word, through the inverse round table:
// td0[S[b]] is InvMixColumns of the column (b, 0, 0, 0).
__device__ __forceinline__ uint32_t inv_mix_column(uint32_t w) {
    return g_base[256 + sbox(w)] ^ rotl(g_base[256 + sbox(w >> 8)], 8) ^
           rotl(g_base[256 + sbox(w >> 16)], 16) ^ rotl(g_base[256 + sbox(w >> 24)], 24);
}

// Key Expansion (FIPS-197 section 5.2) of the key at `key` into w[0 .. 4Nr+3].
__device__ void expand_key_words(const uint8_t *key, int nk, int nr, uint32_t *w) {
    uint32_t prev = 0;
    for (int i = 0; i < nk; i++) {
        prev = uint32_t(key[4 * i]) | (uint32_t(key[4 * i + 1]) << 8) | (uint32_t(key[4 * i + 2]) << 16) |
               (uint32_t(key[4 * i + 3]) << 24);
        w[i] = prev;
    }
    uint32_t rcon = 1;
    for (int i = nk; i < 4 * (nr + 1); i++) {
        uint32_t t = prev;
        if (i % nk == 0) {
            t = sub_word(rotl(t, 24)) ^ rcon;  // RotWord is a right rotation of a little-endian word
            rcon = ((rcon << 1) ^ ((rcon & 0x80u) ? 0x1bu : 0u)) & 0xffu;
        } else if (nk > 6 && i % nk == 4) {
            t = sub_word(t);
        }
        prev = w[i - nk] ^ t;
        w[i] = prev;
    }
}

__global__ __launch_bounds__(256) void keyexp_kernel(const BatchKArgs a) {
    const uint32_t n = batch_count(a);
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n)
        return;
    const aes_msg_desc d = a.desc[m];
    if (!desc_valid(d, a))
        return;
    const int nk = 4 + 2 * int(d.keybits_code), nr = nk + 6;
    uint32_t *w = a.keytab + size_t(m) * kKeySlotWords;
    expand_key_words(a.keys + size_t(d.key_idx) * 32, nk, nr, w);
    if (desc_class(d) == 1) {
        uint32_t *dk = w + kKeySlotWords / 2;
        for (int c = 0; c < 4; c++) {
            dk[c] = w[4 * nr + c];
            dk[4 * nr + c] = w[c];
        }
        for (int r = 1; r < nr; r++)
            for (int c = 0; c < 4; c++)
                dk[4 * r + c] = inv_mix_column(w[4 * (nr - r) + c]);
    }
    // XTS: the tweak key's encryption schedule in the half of the slot the
    // data key's direction leaves free
    if (d.mode == AES_MODE_XTS)
        expand_key_words(a.keys + size_t(xts_key2(d)) * 32, nk, nr, w + (d.decrypt ? 0 : kKeySlotWords / 2));
}

__device__ __forceinline__ uint64_t tiles_of(const aes_msg_desc &d, uint32_t tile_blocks) {
    const uint64_t nblk = (d.nbytes + 15) >> 4;
    if (desc_class(d) == 2)
        return nblk ? 1 : 0;
    const uint64_t step = d.mode == AES_MODE_XTS ? xts_tile_blocks(d, tile_blocks) : tile_blocks;
    return (nblk + step - 1) / step;
}

__global__ __launch_bounds__(kPlanThreads) void plan_kernel(const BatchKArgs a) {
    __shared__ uint64_t cnt[3][kPlanThreads];
    __shared__ uint64_t base[3];
    __shared__ uint32_t bad[kPlanThreads];
    const uint32_t n = batch_count(a);
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (n + kPlanThreads - 1) / kPlanThreads;
    const uint32_t m0 = min(n, tid * per), m1 = min(n, m0 + per);
    uint64_t c[3] = {0, 0, 0};
    uint32_t rejected = 0;
    for (uint32_t m = m0; m < m1; m++) {
        const aes_msg_desc d = a.desc[m];
        if (!desc_valid(d, a)) {
            rejected++;
            continue;
        }
        c[desc_class(d)] += tiles_of(d, a.tile_blocks);
    }
    cnt[0][tid] = c[0];
    cnt[1][tid] = c[1];
    cnt[2][tid] = c[2];
    bad[tid] = rejected;
    __syncthreads();
    if (tid < 3) {
        // exclusive scan of one class's per-thread counts (1024 adds)
        uint64_t run = 0;
        for (int t = 0; t < kPlanThreads; t++) {
            const uint64_t v = cnt[tid][t];
            cnt[tid][t] = run;
            run += v;
        }
        base[tid] = run;
    }
    __syncthreads();
    bool fits[3];
    for (int k = 0; k < 3; k++)
        fits[k] = base[k] <= a.tile_capacity;
    uint64_t off[3] = {cnt[0][tid], cnt[1][tid], cnt[2][tid]};
    for (uint32_t m = m0; m < m1; m++) {
        const aes_msg_desc d = a.desc[m];
        if (!desc_valid(d, a))
            continue;
        const int k = desc_class(d);
        if (!fits[k])
            continue;
        const uint64_t nblk = (d.nbytes + 15) >> 4;
        BatchTile *list = a.tiles + size_t(k) * a.tile_capacity;
        // a serial message is one tile; XTS tiles are whole groups of units
        const uint64_t step = k == 2 ? nblk : d.mode == AES_MODE_XTS ? xts_tile_blocks(d, a.tile_blocks)
                                                                     : uint64_t(a.tile_blocks);
        for (uint64_t first = 0; first < nblk; first += step) {
            BatchTile t;
            t.msg = m;
            t.count = uint32_t(min<uint64_t>(step, nblk - first));
            t.first = first;
            list[off[k]++] = t;
        }
    }
    if (tid == 0) {
        uint32_t r = 0;
        for (int t = 0; t < kPlanThreads; t++)
            r += bad[t];
        BatchHeader *h = a.header;
        for (int k = 0; k < 3; k++) {
            h->ntiles[k] = fits[k] ? uint32_t(base[k]) : 0u;
            h->next[k] = 0;
        }
        h->rejected = r;
        h->overflow = (fits[0] && fits[1] && fits[2]) ? 0u : 1u;
    }
}

template <int NR, int MODE, int DIR, int BPT>
__device__ __forceinline__ void run_tile(const uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a,
                                         const aes_msg_desc &d, const BatchTile &t) {
    // The round keys are the same for the whole wave: read them once per
    // tile and keep them in scalar registers.  (The compiler cannot use
    // scalar loads itself here: the kernel also stores to memory that it
    // cannot prove distinct from the key table.)
    const uint32_t *rkp = a.keytab + size_t(t.msg) * kKeySlotWords + (DIR == DIR_DEC ? kKeySlotWords / 2 : 0);
    uint32_t rk[4 * (NR + 1)];
#pragma unroll
    for (int i = 0; i < 4 * (NR + 1); i++)
        rk[i] = __builtin_amdgcn_readfirstlane(rkp[i]);
    uint32_t ctr[4] = {0, 0, 0, 0};
    if (MODE == MODE_CBC) {
        for (int i = 0; i < 4; i++)
            ctr[i] = uint32_t(d.ctr0[4 * i]) | (uint32_t(d.ctr0[4 * i + 1]) << 8) |
                     (uint32_t(d.ctr0[4 * i + 2]) << 16) | (uint32_t(d.ctr0[4 * i + 3]) << 24);
    }
    if (MODE == MODE_CTR) {
        for (int i = 0; i < 3; i++)
            ctr[i] = uint32_t(d.ctr0[4 * i]) | (uint32_t(d.ctr0[4 * i + 1]) << 8) |
                     (uint32_t(d.ctr0[4 * i + 2]) << 16) | (uint32_t(d.ctr0[4 * i + 3]) << 24);
        ctr[3] = (uint32_t(d.ctr0[12]) << 24) | (uint32_t(d.ctr0[13]) << 16) | (uint32_t(d.ctr0[14]) << 8) |
                 uint32_t(d.ctr0[15]);
    }
    const uint8_t *in = static_cast<const uint8_t *>(a.in_base) + d.in_off;
    uint8_t *out = static_cast<uint8_t *>(a.out_base) + d.out_off;
    process_blocks<NR, MODE, DIR, LAYOUT_T4X32, BPT>(lds, lc, rk, ctr, in, out, d.nbytes, t.first,
                                                     t.first + t.count, 64u * BPT);
}

// An XTS tile: whole groups of 64 data units starting at a unit boundary.
template <int NR, int DIR, int BPT>
__device__ __forceinline__ void run_xts_tile(const uint32_t *lds, const LaneConsts &lc, const BatchKArgs &a,
                                             const aes_msg_desc &d, const BatchTile &t) {
    const uint32_t *slot = a.keytab + size_t(t.msg) * kKeySlotWords;
    const uint32_t *rkp = slot + (DIR == DIR_DEC ? kKeySlotWords / 2 : 0);
    uint32_t rk[4 * (NR + 1)];
#pragma unroll
    for (int i = 0; i < 4 * (NR + 1); i++)
        rk[i] = __builtin_amdgcn_readfirstlane(rkp[i]);
    const uint32_t *rk2 = slot + (DIR == DIR_DEC ? 0 : kKeySlotWords / 2);   // read once per group
    const uint8_t *in = static_cast<const uint8_t *>(a.in_base) + d.in_off;
    uint8_t *out = static_cast<uint8_t *>(a.out_base) + d.out_off;
    const uint32_t ushift = xts_unit_shift(d);
    const uint64_t group = uint64_t(64) << ushift, end = t.first + t.count;
    const uint64_t first_unit = xts_first_unit(d);
    for (uint64_t gb0 = t.first; gb0 < end; gb0 += group)
        xts_group<NR, DIR, BPT>(lds, lc, rk, rk2, in, out, gb0, min(end, gb0 + group),
                                first_unit + (gb0 >> ushift), ushift);
}

// The serial list (CBC encryption): every wave takes 64 messages at a time,
// one per lane, and each lane encrypts its message block after block with its
// own round keys.  These run first, so the long serial chains start early and
// the parallel tiles fill in around them.
__device__ __forceinline__ void run_serial_tiles(const uint32_t *lds, const BatchKArgs &a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n = a.header->ntiles[2];
    const BatchTile *list = a.tiles + size_t(2) * a.tile_capacity;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(lane);
    for (;;) {
        uint32_t t0 = 0;
        if (lane == 0)
            t0 = atomicAdd(&a.header->next[2], 64u);
        t0 = __builtin_amdgcn_readfirstlane(t0);
        if (t0 >= n)
            break;
        const uint32_t t = t0 + lane;
        if (t >= n)
            continue;
        const BatchTile tile = list[t];
        const aes_msg_desc d = a.desc[tile.msg];
        const uint32_t *rkp = a.keytab + size_t(tile.msg) * kKeySlotWords;
        uint32_t iv[4];
        for (int i = 0; i < 4; i++)
            iv[i] = uint32_t(d.ctr0[4 * i]) | (uint32_t(d.ctr0[4 * i + 1]) << 8) |
                    (uint32_t(d.ctr0[4 * i + 2]) << 16) | (uint32_t(d.ctr0[4 * i + 3]) << 24);
        const uint8_t *in = static_cast<const uint8_t *>(a.in_base) + d.in_off;
        uint8_t *out = static_cast<uint8_t *>(a.out_base) + d.out_off;
        const int nr = desc_nr(d);
        uint32_t rk[60];
        if (nr == 10) {
#pragma unroll
            for (int i = 0; i < 44; i++)
                rk[i] = rkp[i];
            cbc_encrypt_serial<10, LAYOUT_T4X32>(lds, lc, rk, iv, in, out, tile.count);
        } else if (nr == 12) {
#pragma unroll
            for (int i = 0; i < 52; i++)
                rk[i] = rkp[i];
            cbc_encrypt_serial<12, LAYOUT_T4X32>(lds, lc, rk, iv, in, out, tile.count);
        } else {
#pragma unroll
            for (int i = 0; i < 60; i++)
                rk[i] = rkp[i];
            cbc_encrypt_serial<14, LAYOUT_T4X32>(lds, lc, rk, iv, in, out, tile.count);
        }
    }
}

template <int CLASS, int BPT>
__global__ __launch_bounds__(1024) void batch_kernel(const BatchKArgs a) {
    constexpr int DIR = CLASS == 0 ? DIR_ENC : DIR_DEC;
    const uint32_t ntiles = a.header->ntiles[CLASS];
    if (ntiles == 0 && (CLASS != 0 || a.header->ntiles[2] == 0))
        return;
    __shared__ uint32_t lds[lds_words<DIR>()];
    stage_tables<LAYOUT_T4X32, DIR>(lds);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(lane);
    if (CLASS == 0)
        run_serial_tiles(lds, a);
    const BatchTile *list = a.tiles + size_t(CLASS) * a.tile_capacity;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0)
            t = atomicAdd(&a.header->next[CLASS], 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntiles)
            break;
        const BatchTile tile = list[t];
        const aes_msg_desc d = a.desc[tile.msg];
        const int nr = desc_nr(d);
        if (d.mode == AES_MODE_XTS) {
            constexpr int XDIR = CLASS == 0 ? DIR_ENC : DIR_DEC;
            if (nr == 10) run_xts_tile<10, XDIR, BPT>(lds, lc, a, d, tile);
            else if (nr == 12) run_xts_tile<12, XDIR, BPT>(lds, lc, a, d, tile);
            else run_xts_tile<14, XDIR, BPT>(lds, lc, a, d, tile);
        } else if (CLASS == 1 && d.mode == AES_MODE_CBC) {
            if (nr == 10) run_tile<10, MODE_CBC, DIR_DEC, BPT>(lds, lc, a, d, tile);
            else if (nr == 12) run_tile<12, MODE_CBC, DIR_DEC, BPT>(lds, lc, a, d, tile);
            else run_tile<14, MODE_CBC, DIR_DEC, BPT>(lds, lc, a, d, tile);
        } else if (CLASS == 1) {
            if (nr == 10) run_tile<10, MODE_ECB, DIR_DEC, BPT>(lds, lc, a, d, tile);
            else if (nr == 12) run_tile<12, MODE_ECB, DIR_DEC, BPT>(lds, lc, a, d, tile);
            else run_tile<14, MODE_ECB, DIR_DEC, BPT>(lds, lc, a, d, tile);
        } else if (d.mode == AES_MODE_ECB) {
            if (nr == 10) run_tile<10, MODE_ECB, DIR_ENC, BPT>(lds, lc, a, d, tile);
            else if (nr == 12) run_tile<12, MODE_ECB, DIR_ENC, BPT>(lds, lc, a, d, tile);
            else run_tile<14, MODE_ECB, DIR_ENC, BPT>(lds, lc, a, d, tile);
        } else {
            if (nr == 10) run_tile<10, MODE_CTR, DIR_ENC, BPT>(lds, lc, a, d, tile);
            else if (nr == 12) run_tile<12, MODE_CTR, DIR_ENC, BPT>(lds, lc, a, d, tile);
            else run_tile<14, MODE_CTR, DIR_ENC, BPT>(lds, lc, a, d, tile);
        }
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

}  // namespace

hipError_t upload_tables_batch(const HostTables &t) { return upload_base_tables(t); }

hipError_t launch_batch(const BatchKArgs &a, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(keyexp_kernel, dim3((a.max_msgs + 255) / 256), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((batch_kernel<0, 2>), dim3(grid), dim3(1024), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((batch_kernel<1, 2>), dim3(grid), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_fill(const FillKArgs &a, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace aesgpu
