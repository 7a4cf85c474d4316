/*
 * aesgpu: AES (FIPS-197) encryption and decryption of large device-resident
 * buffers on AMD Instinct MI355X (gfx950), in ECB and CTR mode, and in the
 * modes after the paper's: CBC, XTS and GCM.
 *
 * The operation is the one the paper (Barnes, Fernando, Mettananda, Ragel,
 * "Improving the Throughput of the AES Algorithm with Multicore Processors")
 * parallelises: a buffer is cut into independent 16-byte blocks and each
 * block goes through Key Expansion's round keys, an initial AddRoundKey,
 * Nr - 1 rounds of SubBytes, ShiftRows, MixColumns and AddRoundKey, and a
 * final round without MixColumns (Section III-A).  The arithmetic of each
 * step is that of FIPS-197 (sections 5.1 - 5.3); CTR is NIST SP 800-38A
 * section 6.5 with a 32-bit big-endian counter in bytes 12..15 of the
 * counter block.
 *
 * Conventions for every call:
 *   - Every function returns an aes_status; none throws or aborts.  On a
 *     non-zero status, aes_last_error() holds a message (per thread).
 *   - Buffers are owned by the caller.  The library never allocates device
 *     memory on these paths; it only launches kernels.
 *   - Calls are asynchronous with respect to the host: they return once the
 *     kernel is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream).  Host-side arguments (round keys, counter block) are read
 *     before the call returns and may be freed at once.  Device buffers must
 *     stay valid until the stream has run the kernel.
 *   - Arguments are validated on the host before anything is enqueued; a
 *     launch failure reports AES_E_DEVICE.
 *   - Only gfx950 devices are supported; any other device gives
 *     AES_E_DEVICE.
 */
#ifndef AESGPU_H
#define AESGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AES_OK = 0,
    AES_E_NULL = 1,     /* a required pointer is NULL (ctr0 in CTR mode too) */
    AES_E_KEYBITS = 2,  /* key size not 128, 192 or 256                      */
    AES_E_NR = 3,       /* Nr not 10, 12 or 14                               */
    AES_E_LENGTH = 4,   /* ECB length not a multiple of 16, or size too big  */
    AES_E_ALIGN = 5,    /* device pointer not 16-byte aligned                */
    AES_E_OVERLAP = 6,  /* in and out overlap without being identical        */
    AES_E_MODE = 7,     /* unknown mode                                      */
    AES_E_DEVICE = 8,   /* no usable gfx950 device, or a HIP call failed     */
    AES_E_ARG = 9,      /* any other invalid argument                        */
    AES_E_BUDGET = 10   /* a served request larger than the admission budget */
} aes_status;

/* ECB and CTR: every block independent.  CBC (SP 800-38A section 6.2, one of
 * the modes after the paper's): decryption is block-parallel (each block
 * needs the previous ciphertext block); encryption is serial by definition
 * and runs on one lane per message.  XTS (IEEE 1619) and GCM (SP 800-38D)
 * are modes of batch descriptors (GCM also of served requests); single
 * buffers use aes_xts_* / aes_gcm_* (aes_encrypt with AES_MODE_XTS or
 * AES_MODE_GCM is AES_E_MODE). */
typedef enum { AES_MODE_ECB = 0, AES_MODE_CTR = 1, AES_MODE_CBC = 2, AES_MODE_XTS = 3,
               AES_MODE_GCM = 4 } aes_mode;

/*
 * Key Expansion (FIPS-197 section 5.2; the paper's first step,
 * Section III-A).
 *   key        host pointer to keybits/8 bytes.
 *   keybits    128, 192 or 256.
 *   roundkeys  host pointer to at least 16*(Nr+1) bytes (176, 208 or 240),
 *              receives the words w[0] .. w[4Nr+3] of the key schedule, each
 *              word as its 4 bytes in the standard's order, so that bytes
 *              16r .. 16r+15 are exactly the bytes XORed into state bytes
 *              0..15 by AddRoundKey in round r.
 *   Nr         host pointer; receives 10, 12 or 14.
 * Runs on the host only.  Errors: AES_E_NULL, AES_E_KEYBITS.
 */
int aes_expand_key(const uint8_t *key, int keybits, uint8_t *roundkeys, int *Nr);

/*
 * Encrypt nbytes of `in` into `out` (the cipher of FIPS-197 section 5.1,
 * applied to every 16-byte block; the paper's Section III-A step list).
 *   in, out    device pointers, 16-byte aligned.  in == out (in place) is
 *              allowed; any other overlap is AES_E_OVERLAP.
 *   nbytes     ECB and CBC: a multiple of 16.  CTR: any length up to 2^36
 *              bytes (2^32 blocks: beyond that the 32-bit counter would
 *              repeat a keystream block within the call; AES_E_LENGTH); a
 *              final partial block uses the leading bytes of its keystream
 *              block.  nbytes == 0 returns AES_OK and enqueues nothing.
 *   roundkeys  host pointer to the 16*(Nr+1)-byte ENCRYPTION schedule as
 *              written by aes_expand_key.
 *   Nr         10, 12 or 14.
 *   mode       AES_MODE_ECB, AES_MODE_CTR or AES_MODE_CBC.
 *   ctr0       CTR: host pointer to the 16-byte initial counter block; block
 *              j uses bytes 0..11 of ctr0 followed by (c0 + j) mod 2^32 in
 *              big-endian order, c0 being the big-endian value of
 *              ctr0[12..15] (no carry into bytes 0..11).  CBC: host pointer
 *              to the 16-byte initialization vector.  ECB: ignored, may be
 *              NULL.
 *   stream     hipStream_t to enqueue on, or NULL.
 */
int aes_encrypt(const void *in, void *out, size_t nbytes,
                const uint8_t *roundkeys, int Nr, int mode,
                const uint8_t *ctr0, void *stream);

/*
 * Decrypt: the inverse cipher (FIPS-197 section 5.3), computed in the
 * equivalent-inverse-cipher form of section 5.3.5.  Same arguments as
 * aes_encrypt; `roundkeys` is still the ENCRYPTION schedule (the decryption
 * schedule is derived inside).  For CTR, decryption is the same operation
 * as encryption.  CBC decryption cannot run in place (in == out gives
 * AES_E_OVERLAP): block j needs ciphertext block j-1 after other workgroups
 * may have written their outputs.
 */
int aes_decrypt(const void *in, void *out, size_t nbytes,
                const uint8_t *roundkeys, int Nr, int mode,
                const uint8_t *ctr0, void *stream);

/*
 * XTS-AES (IEEE 1619; NIST SP 800-38E), the storage mode after the paper's
 * (its motivating use is encrypting stored files).  The buffer is a run of
 * data units ("sectors") of unit_bytes each; unit u has the tweak value
 * i = first_unit + u (mod 2^64), taken as a 16-byte little-endian number.
 * Block j of a unit (j counted from 0 within the unit) is
 *     C_j = Cipher_K1(P_j ^ T_j) ^ T_j,  T_j = Cipher_K2(i) * alpha^j,
 * the product in GF(2^128) modulo x^128 + x^7 + x^2 + x + 1 with the
 * standard's little-endian bit order (alpha = x).  Decryption uses
 * InvCipher_K1 with the same T_j.
 *   in, out          device pointers, 16-byte aligned; in == out allowed,
 *                    any other overlap is AES_E_OVERLAP.
 *   nbytes           a multiple of 16 (no ciphertext stealing); the last
 *                    unit may be shorter than unit_bytes.  0 enqueues
 *                    nothing.
 *   roundkeys1/2     host pointers to the ENCRYPTION schedules of the data
 *                    key K1 and the tweak key K2 (aes_expand_key output),
 *                    both with Nr rounds (the standard names AES-128 and
 *                    AES-256; Nr = 12 is accepted and computed the same way).
 *   unit_bytes       a power of two from 16 to 4096.
 *   first_unit       tweak value of the buffer's first unit.
 *   stream           hipStream_t or NULL.
 * Errors: AES_E_NULL, AES_E_NR, AES_E_LENGTH (nbytes), AES_E_ARG
 * (unit_bytes), AES_E_ALIGN, AES_E_OVERLAP, AES_E_DEVICE.
 */
int aes_xts_encrypt(const void *in, void *out, size_t nbytes,
                    const uint8_t *roundkeys1, const uint8_t *roundkeys2, int Nr,
                    size_t unit_bytes, uint64_t first_unit, void *stream);
int aes_xts_decrypt(const void *in, void *out, size_t nbytes,
                    const uint8_t *roundkeys1, const uint8_t *roundkeys2, int Nr,
                    size_t unit_bytes, uint64_t first_unit, void *stream);

/*
 * AES-GCM (NIST SP 800-38D), authenticated encryption after the paper's
 * modes: CTR encryption with the counter starting one past the pre-counter
 * block J0, and the tag Cipher_K(J0) XOR GHASH_H(A || C || lengths) with
 * H = Cipher_K(0^128) (sections 6.3 - 6.5, 7.1, 7.2).  One pass over the
 * data: each ciphertext block is hashed in the kernel that produces it.
 *   in, out          device pointers, 16-byte aligned, nbytes of them (any
 *                    length up to 2^36 - 32 bytes; 0 is GMAC, a tag over
 *                    the additional data alone).  in == out allowed.
 *   aad, aad_bytes   additional authenticated data: device pointer, 16-byte
 *                    aligned (NULL only when aad_bytes == 0), up to 2^36
 *                    bytes; must not overlap out.
 *   roundkeys, Nr    host pointer to the encryption schedule
 *                    (aes_expand_key output); 10, 12 or 14.
 *   iv, iv_bytes     host pointer to the IV, 1 .. 256 bytes (12 is the
 *                    standard's recommended length; others go through
 *                    GHASH to form J0).
 *   workspace        device memory of at least aes_gcm_workspace_size()
 *                    bytes, 256-byte aligned, private to the call until the
 *                    stream has run it (calls in flight at once need their
 *                    own).
 *   stream           hipStream_t or NULL.
 * Encryption writes the full 16-byte tag to device memory at `tag` (callers
 * that use a shorter tag keep its leading bytes).  Decryption recomputes the
 * tag over `in` and compares its first tag_bytes (4, 8 or 12 .. 16) with the
 * device buffer `tag`, writing 1 (authentic) or 0 to the device int `*ok`.
 * The plaintext is written in either case: a caller must not release it
 * unless *ok is 1.
 * Errors: AES_E_NULL, AES_E_NR, AES_E_LENGTH, AES_E_ALIGN, AES_E_OVERLAP,
 * AES_E_ARG (iv_bytes, tag_bytes), AES_E_DEVICE.
 */
int aes_gcm_workspace_size(size_t *bytes);
int aes_gcm_encrypt(const void *in, void *out, size_t nbytes,
                    const void *aad, size_t aad_bytes,
                    const uint8_t *roundkeys, int Nr,
                    const uint8_t *iv, size_t iv_bytes, void *tag,
                    void *workspace, size_t workspace_bytes, void *stream);
int aes_gcm_decrypt(const void *in, void *out, size_t nbytes,
                    const void *aad, size_t aad_bytes,
                    const uint8_t *roundkeys, int Nr,
                    const uint8_t *iv, size_t iv_bytes,
                    const void *tag, size_t tag_bytes, int *ok,
                    void *workspace, size_t workspace_bytes, void *stream);

/* Message for the last non-zero status returned on this thread. */
const char *aes_last_error(void);

/*
 * Launch configuration of the buffer kernels (ECB and CTR).  Exposed so
 * that a tuner can sweep it and tests can show the result does not depend
 * on it.  All fields 0 mean "the library's choice".
 *   layout            0 = four round tables, 32 copies each, in LDS
 *                         (128 KiB);
 *                     1 = two round tables, 64 copies each (the other two
 *                         are rotations of them; 128 KiB);
 *                     2 = bitsliced: no tables, 32 blocks per lane as 128
 *                         bit-planes, S-box as a Boolean circuit (constant
 *                         time; encryption only: ECB decryption with this
 *                         layout returns AES_E_ARG);
 *                     3 = one round table, 64 copies (the other three are
 *                         its rotations; 64 KiB, so two 1024-thread
 *                         workgroups share a compute unit);
 *                     4 = four round tables, one copy each (4 KiB, with
 *                         LDS bank conflicts).
 *                     Decryption adds a 32 KiB inverse S-box to each.
 *   blocks_per_thread 1, 2 or 4 16-byte blocks in flight per thread (table
 *                     layouts; the bitsliced layout always carries 32).
 *   wg_size           256, 512 or 1024 threads per workgroup (table layouts;
 *                     the bitsliced layout uses 256).
 *   grid              workgroups launched (each loops over the buffer); 0 =
 *                     as many as fit on every compute unit at once (their
 *                     LDS and registers; two per compute unit for the
 *                     bitsliced layout, two waves per SIMD), fewer for small
 *                     buffers.
 */
typedef struct {
    int layout;
    int blocks_per_thread;
    int wg_size;
    int grid;
} aes_launch;

/* Set (cfg != NULL) or clear (cfg == NULL) the launch configuration used by
 * later aes_encrypt / aes_decrypt calls from every thread.  Errors:
 * AES_E_ARG for values outside the lists above. */
int aes_set_launch(const aes_launch *cfg);

/*
 * Tuned launch configurations.  An entry applies to calls with its mode,
 * direction and Nr whose length is at least min_bytes; among matching
 * entries the one with the largest min_bytes wins.  A configuration set with
 * aes_set_launch overrides the table.  aes_set_tuned replaces the whole
 * table (n = 0 clears it); at most 256 entries.  Errors: AES_E_ARG for an
 * entry with values outside the aes_launch lists, or the bitsliced layout
 * for ECB decryption.
 */
typedef struct {
    int mode;          /* AES_MODE_ECB or AES_MODE_CTR */
    int decrypt;       /* 0 or 1 */
    int Nr;            /* 10, 12 or 14 */
    uint64_t min_bytes;
    aes_launch cfg;
} aes_tuned_entry;

int aes_set_tuned(const aes_tuned_entry *entries, int n);

/* The configuration the next call with these arguments would use. */
int aes_get_launch(size_t nbytes, int mode, int decrypt, int Nr, aes_launch *cfg);

/*
 * Measurement helper (not part of the cipher): copies nbytes (a multiple of
 * 16) from `in` to `out` with the same 16-byte-per-lane loads and stores and
 * the same persistent grid as the cipher kernels.  Its run time is the HBM
 * ceiling the cipher is compared with, and its hardware counters calibrate
 * byte counts.  Errors as for aes_encrypt.
 */
int aes_copy(const void *in, void *out, size_t nbytes, void *stream);

/*
 * Measurement helper (not part of the cipher): the LDS lookup rate the table
 * kernels are compared with.  Launches the cipher's shape (one 1024-thread
 * workgroup per compute unit, 128 KiB of LDS) with every lane reading 32-bit
 * words from its own LDS bank, 16 reads per round for `rounds` rounds, and no
 * global memory traffic.  Each wave writes one record to `out` (device
 * memory, caller-owned): the cycle-counter delta (s_memtime) and the
 * constant-rate clock ticks (s_memrealtime) its loop took, and a fold of the
 * words it read.  Lookups per launch = waves x 64 x 16 x rounds, waves =
 * compute units x 16; *waves receives that count and *tick_khz the rate of
 * the constant-rate clock (hipDeviceAttributeWallClockRate), both set before
 * the size check.  out_bytes must hold waves records.
 * Errors: AES_E_NULL, AES_E_ARG (rounds < 1), AES_E_LENGTH (out_bytes too
 * small), AES_E_DEVICE.
 */
typedef struct {
    uint64_t cycles;    /* cycle-counter delta of the wave's loop       */
    uint64_t ticks;     /* constant-rate clock ticks of the same loop    */
    uint32_t fold;      /* XOR of every word the wave read               */
    uint32_t pad;
} aes_lds_gather_stat;

int aes_lds_gather(aes_lds_gather_stat *out, size_t out_bytes, int rounds, int *waves, int *tick_khz,
                   void *stream);

/* The same calibration over another table layout, in its launch shape:
 * layout 0 as aes_lds_gather; layout 3 (one table x 64 copies, 64 KiB) with
 * as many workgroups per compute unit as fit (two), each lane reading copy
 * `lane` of the one table.  *waves = workgroups x 16.  Errors as
 * aes_lds_gather, and AES_E_ARG for another layout. */
int aes_lds_gather_layout(aes_lds_gather_stat *out, size_t out_bytes, int rounds, int layout, int *waves,
                          int *tick_khz, void *stream);


/* ---------------------------------------------------------------------- */
/* Batches: many independent messages, each with its own key, length and  */
/* mode, in one launch sequence.                                           */
/* ---------------------------------------------------------------------- */

/*
 * One message of a batch (48 bytes, device-resident array).  The message is
 * nbytes bytes at in_base + in_off, written to out_base + out_off; both
 * offsets are multiples of 16.  Its key is the first 16/24/32 bytes of the
 * 32-byte slot key_idx of the key array.  ECB and CBC messages are whole
 * blocks; CTR messages may end in a partial block and hold at most 2^36
 * bytes (as for aes_encrypt).  ctr0 is the initial
 * counter block (CTR) or the IV (CBC) exactly as for aes_encrypt.  Input
 * and output are the same bytes or disjoint (CBC decryption: disjoint), else
 * the message is rejected; a CBC encryption runs serially on one lane.  XTS messages (whole blocks, as
 * aes_xts_encrypt) use key_idx for the data key and ctr0 for the rest, all
 * little-endian: bytes 0..7 the tweak value of the message's first data
 * unit, 8..11 the key slot of the tweak key (same key size), 12..15 the
 * data-unit size in bytes (a power of two, 16 .. 4096).  GCM messages
 * (any length up to 2^36 - 32 bytes) carry their 96-bit IV in ctr0[0..11]
 * (J0 = IV || 0^31 || 1; ctr0[12..15] are ignored) and the rest in the
 * batch's aes_gcm_desc array.
 */
typedef struct {
    uint64_t in_off;
    uint64_t out_off;
    uint64_t nbytes;
    uint32_t key_idx;
    uint8_t keybits_code;  /* 0 = 128, 1 = 192, 2 = 256 */
    uint8_t mode;          /* AES_MODE_ECB, _CTR, _CBC or _XTS */
    uint8_t decrypt;       /* 0 = encrypt, 1 = decrypt */
    uint8_t reserved;
    uint8_t ctr0[16];
} aes_msg_desc;

/*
 * The GCM part of batch message m (SP 800-38D): element m of an array
 * parallel to the descriptors, 32 bytes each, device memory owned by the
 * caller.  Entries of messages of other modes are not read.
 *   aad_off, aad_bytes  the additional authenticated data: aad_bytes (up to
 *                       2^36) at in_base + aad_off, a multiple of 16; it
 *                       must not overlap the message's output.
 *   tag_off             encryption: the 16-byte tag is written at
 *                       out_base + tag_off; decryption: the expected tag is
 *                       read from in_base + tag_off.  Inside the buffer, and
 *                       not overlapping the message's output.
 *   tag_bytes           decryption: how many leading tag bytes to compare
 *                       (4, 8 or 12 .. 16); encryption: ignored.
 *   ok                  written by the device after the batch: encryption 1;
 *                       decryption 1 if the tag matches, else 0; 0 for a
 *                       refused descriptor.  A decryption writes the
 *                       plaintext whatever the verdict: a caller must not
 *                       release it unless ok is 1.
 */
typedef struct {
    uint64_t aad_off;
    uint64_t aad_bytes;
    uint64_t tag_off;
    uint32_t tag_bytes;
    int32_t ok;
} aes_gcm_desc;

/*
 * A batch.  Every pointer is a device pointer owned by the caller.
 *   desc, nmsg       the messages.  If d_nmsg is not NULL the count is read
 *                    from that device int at run time instead (it must stay
 *                    <= max_msgs), so a captured graph can be replayed with a
 *                    different number of messages.
 *   keys, nkeys      raw keys, 32-byte slots.
 *   in_base/in_bytes, out_base/out_bytes   the buffers messages live in; a
 *                    message that does not fit inside them is rejected.
 *   workspace        256-byte aligned scratch of workspace_bytes, sized by
 *                    aes_batch_workspace_size for max_msgs.  It holds the
 *                    expanded key schedules, the work lists and the split.
 *   tile_blocks      granularity of the split, 1 .. 1024: a wave's part of a
 *                    message starts and ends on a multiple of this many
 *                    16-byte blocks (XTS: of whole data units), or at the
 *                    message's end; 0 = library choice (512).
 *   gcm              the GCM fields of the messages (aes_gcm_desc, one per
 *                    message slot, at least max_msgs of them), or NULL if
 *                    the batch has no GCM message (a GCM descriptor is then
 *                    refused).
 *   blocks_per_thread  16-byte blocks each lane carries through the rounds
 *                    at once in the parallel lists, 2 or 4; 0 = library
 *                    choice (4).  (XTS pieces always carry 2.)
 *   gcm_two_pass     0: GCM messages of at least 131,072 GHASH blocks are
 *                    encrypted and hashed in one pass (the kernels for it
 *                    are launched whenever gcm is set); nonzero: every GCM
 *                    message takes the counter-mode pass and the hash pass,
 *                    and those kernels are not launched (a caller that
 *                    knows its batches hold no such message saves their
 *                    launches; the results are the same either way).
 * The sequence is: on-device Key Expansion for every message (FIPS-197
 * section 5.2; the decryption schedule of section 5.3.5 where needed) and a
 * plan that puts the messages in lists (encryption tables, inverse tables,
 * serial CBC encryption, and for GCM the hash lists) and splits each parallel list into equal
 * shares of work, one per wave, by cost (blocks times rounds): the paper's
 * chunking into one piece per processor, Section IV-A, across messages; then
 * persistent kernels, one workgroup per compute unit, in which every wave
 * runs its share.  GCM messages run their CTR part (from J0 + 1) in the
 * forward list; then their GHASH (section 6.4) over the additional data,
 * the ciphertext and the lengths is cut into pieces of up to 4,096 blocks,
 * one wave per piece (the pieces' sums are added by linearity), and a last
 * kernel forms or checks each tag.  GCM messages of at least 131,072 GHASH
 * blocks (about 2 MiB) are encrypted and hashed in one pass instead, one
 * workgroup per piece of 65,536 blocks.  A message with an invalid descriptor (bad key code or
 * mode, ECB length not a multiple of 16, misaligned offset, outside the
 * buffers, input and output partly overlapping, key_idx >= nkeys) is
 * skipped and counted (aes_batch_query).
 */
typedef struct {
    const aes_msg_desc *desc;
    int nmsg;
    const int *d_nmsg;
    const uint8_t *keys;
    int nkeys;
    const void *in_base;
    uint64_t in_bytes;
    void *out_base;
    uint64_t out_bytes;
    void *workspace;
    size_t workspace_bytes;
    int max_msgs;
    int tile_blocks;
    aes_gcm_desc *gcm;
    int blocks_per_thread;
    int gcm_two_pass;
} aes_batch;

/* Workspace bytes for batches of up to max_msgs messages (any lengths).
 * Host only. */
int aes_batch_workspace_size(int max_msgs, size_t *bytes);

/* The same figure under the name of the batched call's planning step: the
 * workspace a batch of nmsg messages needs.  The size depends on the count
 * only (one key-schedule slot and one list entry per message), so d_desc is
 * not read and may be NULL; it is in the signature so that a caller that
 * plans from its descriptor table passes it unchanged.  Host only.
 * Errors: AES_E_NULL (workspace_bytes), AES_E_ARG (nmsg < 1). */
int aes_batch_plan(const aes_msg_desc *d_desc, int nmsg, size_t *workspace_bytes);

/* Enqueue the whole batch on `stream`.  Errors are found on the host from
 * the aes_batch fields; descriptor contents are checked on the device. */
int aes_batch_run(const aes_batch *b, void *stream);

/*
 * aes_batch_run for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The batch's workspace is not the caller's: it is a buffer the library
 * holds in device memory for the life of the process, one per device
 * (AES_BATCH_NOALLOC_MAX_MSGS messages' worth, about 9.3 MiB), set up with
 * the device's other state on the first call.  The call allocates nothing;
 * the caller still passes descriptors, keys, input and output as for
 * aes_batch_run, with b->workspace NULL and b->workspace_bytes 0.
 * Every call on a device shares that device's buffer and leaves its
 * contents behind for the next (the batch sequence rewrites everything it
 * reads, so nothing has to start cleared): calls whose batches may run at
 * the same time on one device (different streams, or another thread's)
 * race and give wrong results; calls queued on one stream do not.
 * aes_batch_query does not apply (the counts live in the shared buffer).
 * Errors: as aes_batch_run; AES_E_ARG if b->workspace or workspace_bytes is
 * set, AES_E_LENGTH if b->max_msgs > AES_BATCH_NOALLOC_MAX_MSGS.
 */
#define AES_BATCH_NOALLOC_MAX_MSGS 16384
int aes_batch_run_noalloc(const aes_batch *b, void *stream);

/* After the stream has run the batch: messages planned (accepted into the
 * lists) and messages rejected by the device-side checks.  Synchronous
 * (waits for `stream`). */
int aes_batch_query(const aes_batch *b, void *stream, uint64_t *planned, uint64_t *rejected);

/* The same sequence captured once as a HIP graph for repeated launches on
 * any stream.  Descriptors, keys and (through d_nmsg) the message count may
 * be rewritten between launches; the pointers and sizes in *b may not. */
int aes_batch_graph_create(const aes_batch *b, void **graph);
int aes_batch_graph_launch(void *graph, void *stream);
int aes_batch_graph_destroy(void *graph);

/* ---------------------------------------------------------------------- */
/* Serving: a request loop with admission by HBM budget and continuous     */
/* batching over several streams.                                         */
/* ---------------------------------------------------------------------- */

/*
 * One request.  It arrives arrival_s seconds after the run starts.  Its
 * payload is nbytes bytes of the SplitMix64 stream with seed payload_seed
 * (word i = mix64(seed + (i+1) * 0x9E3779B97F4A7C15), bytes little-endian),
 * written on the device when the request is launched: the synthetic stand-in
 * for data arriving over the network.  Key, mode, direction and counter are
 * as in aes_msg_desc (modes ECB, CTR, CBC and GCM).  A GCM request (96-bit
 * IV in ctr0[0..11], no additional data) has 16 more payload bytes (the
 * next 16 of its stream, after the data rounded up to 16 bytes): the
 * expected tag when decrypting; when encrypting, its tag is written at the
 * same place after its output.  Each GCM buffer counts 16 more bytes
 * against the budget.
 */
typedef struct {
    double arrival_s;
    uint64_t nbytes;
    uint64_t payload_seed;
    uint32_t key_idx;
    uint8_t keybits_code;
    uint8_t mode;
    uint8_t decrypt;
    uint8_t reserved;
    uint8_t ctr0[16];
} aes_request;

/*
 * streams          batches in flight at once (1..16), one HIP stream each.
 * budget_bytes     admission budget: the input and output buffers of all
 *                  requests admitted and not yet finished (each rounded up to
 *                  256 bytes) never exceed it.  It is also the size of the
 *                  device arena they are carved from.  A request that alone
 *                  exceeds it is rejected (status AES_E_BUDGET), never queued.
 * max_batch_msgs   requests per launch (1..65536).
 * tile_blocks      as for aes_batch (0 = library choice).
 * blocks_per_thread  as for aes_batch (0 = library choice).
 * timeout_s        the run fails with AES_E_DEVICE if nothing completes for
 *                  this long while work is in flight (0 = 60 s).
 * simulate_gbps    > 0: no device is touched; every launch is taken to finish
 *                  after its bytes at this rate plus 20 us, so the admission
 *                  and batching logic can run without a GPU.  d_keys and
 *                  d_scratch are then ignored and may be NULL.
 */
typedef struct {
    int streams;
    uint64_t budget_bytes;
    int max_batch_msgs;
    int tile_blocks;
    int blocks_per_thread;
    double timeout_s;
    double simulate_gbps;
} aes_serve_cfg;

typedef struct {
    double latency_s;   /* completion seen by the loop minus arrival */
    double admit_s;     /* admission time minus arrival (queueing for budget) */
    uint64_t in_off;    /* input and output location in the arena */
    uint64_t out_off;
    int status;         /* AES_OK; AES_E_BUDGET if larger than the budget;
                           AES_E_ARG if the device-side descriptor check
                           refused it (the host checks make this unexpected) */
    int launch;         /* sequence number of the launch it ran in */
    int overwritten;    /* 1 if a later request of the same call was given
                           arena memory that overlaps this request's output
                           (its bytes at out_off are then no longer its
                           result), else 0 */
    int authentic;      /* GCM: 1 if the tag was written (encryption) or
                           matched (decryption), else 0; other modes: -1 */
} aes_request_result;

typedef struct {
    double span_s;            /* first arrival to last completion */
    uint64_t bytes_done;      /* payload bytes of completed requests */
    int completed;
    int rejected;
    int launches;
    int max_inflight_reqs;    /* most requests admitted at once */
    uint64_t max_inflight_bytes;
    double fill_device_s;     /* summed over launches, from HIP events on each
                                 launch's stream: device time of the payload
                                 fill (with the descriptor upload) ... */
    double cipher_device_s;   /* ... and of the batch sequence (0 when
                                 simulating; launches on other streams may
                                 overlap either span) */
} aes_serve_stats;

/* Device scratch bytes aes_serve_run needs for cfg (the arena plus per-stream
 * descriptor tables and batch workspaces).  Host only. */
int aes_serve_scratch_size(const aes_serve_cfg *cfg, size_t *bytes);

/*
 * Run the requests (sorted by arrival_s) to completion on the current
 * device.  The loop, on one host thread: finish launches whose events have
 * completed (their requests' latencies are taken then and their memory
 * returns to the budget); admit arrived requests in arrival order while the
 * budget has room; when a stream is free, launch everything admitted and not
 * yet launched as one batch (payload fill, Key Expansion, the plan,
 * persistent cipher kernels) on it.  Batches on different streams overlap on
 * the device.  results[i] describes reqs[i].  d_scratch (256-byte aligned)
 * holds aes_serve_scratch_size(cfg) bytes.  A request's arena memory goes
 * back to the budget when its launch finishes, so a later request may be
 * carved from it: a result is readable at out_off from its completion until
 * that happens, and after the call returns exactly for the results whose
 * `overwritten` is 0 (until the next call on the same scratch).  Every
 * request is checked before anything runs: key slot < nkeys (nkeys >= 1),
 * key size, mode (ECB, CTR or CBC), direction, ECB/CBC lengths in whole
 * blocks and CTR lengths up to 2^36 bytes; a failure returns AES_E_ARG or
 * AES_E_LENGTH for the whole call.
 */
int aes_serve_run(const aes_request *reqs, int nreq, const uint8_t *d_keys, int nkeys,
                  void *d_scratch, size_t scratch_bytes, const aes_serve_cfg *cfg,
                  aes_request_result *results, aes_serve_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* AESGPU_H */
