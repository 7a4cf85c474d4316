// Declarations shared by the library's own translation units (not public).
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime_api.h>

#include "aesgpu.h"

namespace aesgpu {

// ---- host arithmetic (tables.cpp) ----------------------------------------
struct HostTables {
    uint8_t sbox[256];
    uint8_t inv_sbox[256];
    uint32_t te0[256];  // encryption round table for row 0 (column word)
    uint32_t td0[256];  // decryption round table for row 0
    uint32_t isw[256];  // inverse S-box value repeated in all four bytes
};
const HostTables &host_tables();

// Key schedule as little-endian column words; returns Nr or -1.
int expand_key_host(const uint8_t *key, int keybits, uint32_t *w);
uint32_t inv_mix_column_word(uint32_t col);
// Equivalent-inverse-cipher schedule, in the order the rounds use it.
void decryption_schedule(const uint32_t *w, int nr, uint32_t *dk);

// CTR: at most 2^32 blocks per message or buffer, so that the 32-bit
// counter (incremented modulo 2^32 without a carry into the nonce) never
// repeats a keystream block within it.
constexpr uint64_t kCtrMaxBytes = uint64_t(1) << 36;

// ---- kernels (aes_kernels.hip) --------------------------------------------
enum Mode { MODE_ECB = 0, MODE_CTR = 1, MODE_CBC = 2 };
enum Dir { DIR_ENC = 0, DIR_DEC = 1 };
// Table layouts in LDS (2 is the bitsliced kernel, which has no tables).
enum Layout { LAYOUT_T4X32 = 0, LAYOUT_T2X64 = 1, LAYOUT_T1X64 = 3, LAYOUT_T4X1 = 4 };

// Everything one launch of a buffer kernel needs; passed by value, so the
// round keys and counter land in scalar registers.
struct CipherArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t nbytes;
    uint32_t rk[60];   // round keys in the order the rounds use them
    uint32_t ctr[4];   // CTR: nonce words 0..2 (little-endian), ctr[3] = c0;
                       // CBC: the IV as four little-endian words
};

struct LaunchCfg {
    int layout;
    int bpt;
    int wg;
    int grid;
};

// Uploads the base tables to the current device (once per device).
hipError_t upload_tables(const HostTables &t);

hipError_t launch_cipher(int nr, int mode, int dir, const LaunchCfg &cfg, const CipherArgs &a,
                         hipStream_t stream);
// Workgroups of `wg` threads of that buffer kernel that fit on one compute
// unit at once (its LDS array and registers), as the runtime reports it.
int cipher_groups_per_cu(int nr, int mode, int dir, int layout, int bpt, int wg);
hipError_t launch_copy(const void *in, void *out, uint64_t nbytes, int grid, hipStream_t stream);
// The LDS gather calibration kernel (lds_gather.hip): grid workgroups of 16 waves.
using LdsGatherStat = aes_lds_gather_stat;
constexpr int kLdsGatherWavesPerGroup = 16;
uint32_t lds_gather_reads_per_round();
// layout: LAYOUT_T4X32 or LAYOUT_T1X64; grid = compute units x lds_gather_groups_per_cu(layout)
int lds_gather_groups_per_cu(int layout);
hipError_t launch_lds_gather(LdsGatherStat *out, uint32_t rounds, int layout, int grid, hipStream_t stream);
// CBC encryption is serial: one lane walks the whole buffer.
hipError_t launch_cbc_encrypt(int nr, const CipherArgs &a, hipStream_t stream);
// The bitsliced comparison kernel (bitslice.hip): encryption only.
constexpr int LAYOUT_BITSLICED = 2;
hipError_t launch_bitslice(int nr, int mode, int grid, const CipherArgs &a, hipStream_t stream);

// ---- XTS (xts.hip) ------------------------------------------------------------
struct XtsArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t nbytes;       // a multiple of 16
    uint64_t first_unit;   // tweak value of the first data unit
    uint32_t unit_shift;   // log2 of the blocks per data unit, 0..8
    uint32_t rk1[60];      // data key, in the order the rounds use it (direction's schedule)
    uint32_t rk2[60];      // tweak key, encryption schedule
};
hipError_t upload_tables_xts(const HostTables &t);
hipError_t launch_xts(int nr, int dir, int grid, const XtsArgs &a, hipStream_t stream);

// ---- GCM (gcm.hip) --------------------------------------------------------------
constexpr int kGcmPowers = 32;
constexpr int kGcmMaxGrid = 256;
// The caller's device workspace for one GCM call.  Blocks are stored as four
// little-endian words (bytes in memory order).
struct GcmWork {
    uint32_t powers[kGcmPowers][4];     // H^(2^t)
    uint32_t j0[4];                     // pre-counter block
    uint32_t ej0[4];                    // Cipher_K(J0)
    uint32_t pad[56];
    uint32_t partials[kGcmMaxGrid][4];  // one hash partial per workgroup
};
static_assert(sizeof(GcmWork) <= 8192, "GCM workspace");
constexpr size_t kGcmWorkspaceBytes = 8192;

struct GcmArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t nbytes;
    const uint8_t *aad;
    uint64_t aad_bytes;
    GcmWork *ws;
    uint8_t *tag_out;        // encryption: the 16-byte tag
    const uint8_t *tag_in;   // decryption: the expected tag (tag_bytes bytes)
    int *ok;                 // decryption: 1 if authentic, else 0
    uint32_t tag_bytes;
    uint32_t iv_bytes;       // 1 .. 256
    uint32_t grid_log2;      // the bulk kernel runs 2^grid_log2 workgroups of 1024
    uint32_t decrypt;
    uint32_t rk[60];         // encryption schedule
    uint8_t iv[256];
};
hipError_t upload_tables_gcm(const HostTables &t);
hipError_t launch_gcm(int nr, const GcmArgs &a, hipStream_t stream);

// ---- batches (batch_kernels.hip) -------------------------------------------
// Workspace = header | key schedules (max_msgs slots) | items[3][max_msgs] |
// chunk totals (the plan's counters per chunk of messages).
struct BatchHeader {
    uint32_t nitems[3];   // messages in the forward list (ECB encrypt, CTR, XTS encrypt,
                          // GCM), the inverse list (ECB, CBC and XTS decrypt) and the
                          // serial list (CBC encrypt)
    uint32_t rejected;    // messages whose descriptor failed the checks
    uint64_t next[3];     // forward and inverse lists: next share handed out from the
                          // counter; serial list: next message
    uint64_t cost[2];     // work of the forward and inverse lists, in cost units
    uint32_t ngcm;        // GCM messages hashed in pieces (the GHASH list)
    uint32_t pad0;
    uint64_t gcm_pieces;  // GHASH pieces of all of them
    uint32_t nlane;       // GCM messages hashed one per lane (the back of the GHASH list)
    uint32_t nfused[3];       // GCM messages encrypted and hashed in one pass (the fused
                              // list), per key size (128, 192, 256 bits)
    uint64_t fused_pieces[3];  // their pieces, per key size
    uint64_t next_fused[3];   // next piece of each key size handed out from the counter
    uint32_t pad[30];
};
static_assert(sizeof(BatchHeader) == 256, "header is one 256-byte line");

// One message in a list.  Forward and inverse lists: start = the cost units of
// the messages before it in the list.  Serial list: count = its blocks.
// GHASH list: start = the pieces of the messages before it, count = its own;
// the messages hashed one per lane fill the same array from its end (entry
// max_msgs - 1 - i is the i-th of them).  Fused list: the 128-bit keys'
// messages, then the 192-bit and the 256-bit ones, start = the pieces of the
// messages before it with the same key size.
struct BatchItem {
    uint32_t msg;     // message index
    uint32_t count;
    uint64_t start;
};

// encryption schedule at 0, decryption schedule at 64; an XTS message keeps
// its tweak key's encryption schedule in the half its direction leaves free;
// a GCM message keeps H = Cipher_K(0), Cipher_K(J0), its GHASH sum and the
// powers H^(kGhashPiece * 2^t), t < kGcmSlotPowers, there
constexpr int kKeySlotWords = 128;
// an XTS message keeps the encrypted tweak of its first data unit in the four
// words after the schedule in the first half (a schedule has at most 60)
constexpr int kXtsSlotTweak = 60;
constexpr int kGcmSlotH = 64, kGcmSlotEJ0 = 68, kGcmSlotSum = 72, kGcmSlotPow = 76, kGcmSlotPowers = 13;
static_assert(kGcmSlotPow + 4 * kGcmSlotPowers <= kKeySlotWords, "GCM powers fit the key slot");
// GHASH positions (16-byte blocks of additional data, ciphertext and the
// length block) per piece: one wave hashes one piece
constexpr int kGhashPieceLog2 = 12;
constexpr uint64_t kGhashPiece = uint64_t(1) << kGhashPieceLog2;
// A batch with at least kLaneGhashMinMessages GCM messages of at most
// kLaneGhashMaxPositions positions hashes each of those in one lane (whole
// Horner recurrence, per-lane tables) instead of a wave per piece.
constexpr uint64_t kLaneGhashMaxPositions = 512;
constexpr uint64_t kLaneGhashMinMessages = 32768;
// GCM messages of at least kFusedMinPositions positions are encrypted and
// hashed in one pass (the fused list) in pieces of kFusedPiece positions, one
// workgroup per piece, instead of a counter-mode pass and a hash pass that
// reads the ciphertext again.
constexpr int kFusedPieceLog2 = 16;
constexpr uint64_t kFusedPiece = uint64_t(1) << kFusedPieceLog2;
constexpr uint64_t kFusedMinPositions = 2 * kFusedPiece;
// A wave's share of a message starts and ends on a multiple of this many
// blocks by default (four steps of the block loop, 64 lanes x 2 blocks; the
// best of 128 .. 1024 over batch sizes from one message to gigabytes).  The
// largest allowed keeps the rounding well below a share (thousands of blocks).
constexpr int kDefaultSplitBlocks = 512;
constexpr int kMaxSplitBlocks = 1024;
// The cipher kernels run at most this many waves (256 workgroups of 16).
constexpr int kBatchMaxWaves = 4096;
constexpr int kBatchWavesPerGroup = 16;
// Messages per chunk of the plan (one workgroup of the prep and plan
// kernels), and the plan's counters per chunk.
constexpr int kBatchChunk = 256;
constexpr int kBatchChunkCounters = 15;
constexpr int kBatchLists = 5;   // forward, inverse, serial, GHASH, fused GCM

struct BatchKArgs {
    const aes_msg_desc *desc;
    int nmsg;
    const int *d_nmsg;
    int max_msgs;
    const uint8_t *keys;
    int nkeys;
    const void *in_base;
    uint64_t in_bytes;
    void *out_base;
    uint64_t out_bytes;
    BatchHeader *header;
    uint32_t *keytab;
    BatchItem *items;        // kBatchLists lists of max_msgs entries
    uint64_t *chunk_totals;  // the plan's counters per chunk of messages
    uint32_t split_blocks;   // a share starts and ends on a multiple of this
    uint32_t bpt;            // blocks per lane in the parallel lists: 2 or 4
    uint8_t *reject_flags;   // NULL, or one byte per message, set to 1 for each
                             // message the descriptor check refuses (the
                             // caller clears them; the request loop points
                             // this at pinned host memory)
    aes_gcm_desc *gcm;       // NULL, or the GCM fields per message
    uint32_t fuse_gcm;       // 1: GCM messages of at least kFusedMinPositions positions go to
                             // the fused list (set by launch_batch from its lists argument)
};

// Synthetic payloads of the request loop (batch_kernels.hip).
constexpr uint64_t kFillChunk = 65536;
struct FillDesc {
    uint64_t off;          // byte offset of the payload in the arena
    uint64_t nbytes;
    uint64_t seed;         // SplitMix64 seed
    uint64_t chunk_first;  // index of the message's first fill chunk in the batch
};
struct FillKArgs {
    const FillDesc *fd;
    const int *d_nmsg;
    const uint64_t *d_nchunks;
    uint8_t *base;
};
hipError_t launch_fill(const FillKArgs &a, int grid, hipStream_t stream);
// Copies nbytes (a multiple of 16, both pointers 16-byte aligned) from pinned
// host memory, read through its device address, to device memory, as a
// kernel on `stream` (the request loop's descriptors for the kernels after
// it on the same stream).
hipError_t launch_stage(const void *host_dev, void *dev, uint64_t nbytes, hipStream_t stream);

hipError_t upload_tables_batch(const HostTables &t);

// Workspace bytes for batches of up to max_msgs messages: header, one key
// slot and one list entry per message in each of the lists, the plan's
// counters per chunk of messages.
constexpr size_t batch_layout(int max_msgs) {
    return sizeof(BatchHeader) + size_t(max_msgs) * kKeySlotWords * 4 +
           size_t(kBatchLists) * size_t(max_msgs) * sizeof(BatchItem) +
           (size_t(max_msgs) + kBatchChunk - 1) / kBatchChunk * kBatchChunkCounters * sizeof(uint64_t);
}
// The library-held batch workspace of aes_batch_run_noalloc
// (batch_kernels.hip): one per device, for batches of up to
// AES_BATCH_NOALLOC_MAX_MSGS messages.  init_batch_scratch looks up its
// address on the current device (once per device, at the device's set-up);
// batch_scratch returns it (NULL before that).
constexpr size_t kNoAllocScratchBytes = batch_layout(AES_BATCH_NOALLOC_MAX_MSGS);
hipError_t init_batch_scratch(int dev);
void *batch_scratch(int dev);
// lists: bit k set if list k may hold messages (bit 0 forward, 1 inverse, 2
// serial, 3 GCM: the GHASH and tag kernels, 4 the fused list: GCM messages
// of at least kFusedMinPositions positions are encrypted and hashed in one
// pass, else in the forward and GHASH lists); a kernel whose lists are all
// known to be empty is not launched.  max_count: a bound on the message count known to the caller
// (at most max_msgs); up to one chunk, Key Expansion and the plan run as one
// launch.  Key Expansion and the plan always run.
hipError_t launch_batch(const BatchKArgs &a, int grid, hipStream_t stream, unsigned lists, int max_count);

}  // namespace aesgpu
