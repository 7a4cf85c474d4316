// The C ABI of libaesgpu (declared in include/aesgpu.h): argument checks,
// per-device set-up, the launch-configuration choice, and the host halves of
// the key schedule.  No call here allocates device memory.
#include "aesgpu.h"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace {

using namespace aesgpu;

thread_local std::string g_error;

int fail(int status, const std::string &msg) {
    g_error = msg;
    return status;
}

constexpr int kMaxDevices = 64;

struct DeviceState {
    int status = AES_E_DEVICE;
    std::string error;
    int cus = 0;
};

std::once_flag g_once[kMaxDevices];
DeviceState g_dev[kMaxDevices];

void init_device(int dev) {
    DeviceState &d = g_dev[dev];
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        d.error = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
        return;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        d.error = std::string("aesgpu is built for gfx950 only; device is ") + prop.gcnArchName;
        return;
    }
    if (prop.sharedMemPerBlock < 160 * 1024) {
        d.error = "device offers less than 160 KiB of LDS per workgroup";
        return;
    }
    e = upload_tables(host_tables());
    if (e == hipSuccess)
        e = upload_tables_batch(host_tables());
    if (e == hipSuccess)
        e = init_batch_scratch(dev);
    if (e == hipSuccess)
        e = upload_tables_xts(host_tables());
    if (e == hipSuccess)
        e = upload_tables_gcm(host_tables());
    if (e != hipSuccess) {
        d.error = std::string("table upload: ") + hipGetErrorString(e);
        return;
    }
    d.cus = prop.multiProcessorCount;
    d.status = AES_OK;
}

// Checks the current device and initialises it once; returns its state.
const DeviceState *current_device(int *status) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *status = fail(AES_E_DEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
        return nullptr;
    }
    std::call_once(g_once[dev], init_device, dev);
    if (g_dev[dev].status != AES_OK) {
        *status = fail(AES_E_DEVICE, g_dev[dev].error);
        return nullptr;
    }
    *status = AES_OK;
    return &g_dev[dev];
}

// Launch-configuration override (0 = library choice).
std::mutex g_launch_mu;
aes_launch g_launch = {0, 0, 0, 0};
bool g_launch_set = false;

bool valid_launch(const aes_launch &c) {
    return (c.layout == LAYOUT_T4X32 || c.layout == LAYOUT_T2X64 || c.layout == LAYOUT_BITSLICED ||
            c.layout == LAYOUT_T1X64 || c.layout == LAYOUT_T4X1) &&
           (c.blocks_per_thread == 0 || c.blocks_per_thread == 1 || c.blocks_per_thread == 2 ||
            c.blocks_per_thread == 4) &&
           (c.wg_size == 0 || c.wg_size == 256 || c.wg_size == 512 || c.wg_size == 1024) &&
           c.grid >= 0;
}

std::vector<aes_tuned_entry> g_tuned;  // guarded by g_launch_mu

// mode and decrypt pick the tuned entry (AES_MODE_ECB or _CTR); kmode is the
// kernel that will run (MODE_ECB, MODE_CTR or MODE_CBC), whose occupancy sets
// the default grid.
LaunchCfg choose_launch(const DeviceState &d, uint64_t nbytes, int mode, int decrypt, int nr, int kmode) {
    aes_launch o;
    bool set;
    {
        std::lock_guard<std::mutex> lk(g_launch_mu);
        o = g_launch;
        set = g_launch_set;
        if (!set) {
            const aes_tuned_entry *best = nullptr;
            for (const aes_tuned_entry &e : g_tuned)
                if (e.mode == mode && e.decrypt == decrypt && e.Nr == nr && e.min_bytes <= nbytes &&
                    (!best || e.min_bytes > best->min_bytes))
                    best = &e;
            if (best) {
                o = best->cfg;
                set = true;
            }
        }
    }
    LaunchCfg c;
    c.layout = set ? o.layout : LAYOUT_T4X32;
    c.bpt = set && o.blocks_per_thread ? o.blocks_per_thread : 2;
    c.wg = set && o.wg_size ? o.wg_size : 1024;
    if (c.layout == LAYOUT_BITSLICED) {
        // 256-thread workgroups, two per CU (two waves per SIMD); each lane
        // carries 32 blocks
        c.bpt = 32;
        c.wg = 256;
        uint64_t grid = set && o.grid ? uint64_t(o.grid) : 2 * uint64_t(d.cus);
        const uint64_t useful = ((nbytes + 15) / 16 + 256 * 32 - 1) / (256 * 32);
        if (!(set && o.grid) && useful < grid)
            grid = useful;
        c.grid = int(grid < 1 ? 1 : grid > 0x7fffffff ? 0x7fffffff : grid);
        return c;
    }
    // A persistent grid of as many workgroups as fit on every compute unit
    // at once (the 128 KiB table layouts: one; the 64 KiB one: two of 1024
    // threads) sweeps the buffer.  Small buffers get only as many workgroups
    // as they can keep busy.
    const uint64_t per_cu = uint64_t(cipher_groups_per_cu(nr, kmode, decrypt ? DIR_DEC : DIR_ENC, c.layout, c.bpt, c.wg));
    uint64_t grid = set && o.grid ? uint64_t(o.grid) : uint64_t(d.cus) * per_cu;
    const uint64_t nblk = (nbytes + 15) / 16;
    const uint64_t per_wg = uint64_t(c.wg) * c.bpt;
    const uint64_t useful = (nblk + per_wg - 1) / per_wg;
    if (!(set && o.grid) && useful < grid)
        grid = useful;
    if (grid < 1)
        grid = 1;
    if (grid > 0x7fffffff)
        grid = 0x7fffffff;
    c.grid = int(grid);
    return c;
}

int check_buffers(const void *in, void *out, size_t nbytes) {
    if (!in || !out)
        return fail(AES_E_NULL, "in and out must not be NULL");
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u)
        return fail(AES_E_ALIGN, "in and out must be 16-byte aligned");
    const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
    if (a != b && a < b + nbytes && b < a + nbytes)
        return fail(AES_E_OVERLAP, "in and out overlap without being the same buffer");
    return AES_OK;
}

int crypt(int decrypt, const void *in, void *out, size_t nbytes, const uint8_t *roundkeys, int Nr,
          int mode, const uint8_t *ctr0, void *stream) {
    if (Nr != 10 && Nr != 12 && Nr != 14)
        return fail(AES_E_NR, "Nr must be 10, 12 or 14");
    if (mode != AES_MODE_ECB && mode != AES_MODE_CTR && mode != AES_MODE_CBC)
        return fail(AES_E_MODE, "mode must be AES_MODE_ECB, AES_MODE_CTR or AES_MODE_CBC");
    if (!roundkeys)
        return fail(AES_E_NULL, "roundkeys must not be NULL");
    if (mode == AES_MODE_CTR && !ctr0)
        return fail(AES_E_NULL, "CTR needs the initial counter block ctr0");
    if (mode == AES_MODE_CBC && !ctr0)
        return fail(AES_E_NULL, "CBC needs the initialization vector in ctr0");
    if ((mode == AES_MODE_ECB || mode == AES_MODE_CBC) && nbytes % 16 != 0)
        return fail(AES_E_LENGTH, "ECB and CBC lengths must be a multiple of 16 bytes");
    if (mode == AES_MODE_CTR && nbytes > kCtrMaxBytes)
        return fail(AES_E_LENGTH, "CTR is limited to 2^36 bytes per call (the 32-bit counter would repeat)");
    if (nbytes == 0)
        return AES_OK;
    int st = check_buffers(in, out, nbytes);
    if (st != AES_OK)
        return st;
    if (mode == AES_MODE_CBC && decrypt && in == out)
        return fail(AES_E_OVERLAP, "CBC decryption cannot run in place (block j needs ciphertext j-1)");
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;

    CipherArgs a;
    std::memset(&a, 0, sizeof(a));
    a.in = static_cast<const uint8_t *>(in);
    a.out = static_cast<uint8_t *>(out);
    a.nbytes = nbytes;
    uint32_t w[60];
    const int nwords = 4 * (Nr + 1);
    for (int i = 0; i < nwords; i++)
        std::memcpy(&w[i], roundkeys + 4 * i, 4);  // bytes in order = little-endian column word
    const bool dec_cipher = decrypt && mode != AES_MODE_CTR;
    if (dec_cipher)
        decryption_schedule(w, Nr, a.rk);
    else
        std::memcpy(a.rk, w, 4 * nwords);
    if (mode == AES_MODE_CTR) {
        std::memcpy(a.ctr, ctr0, 12);
        a.ctr[3] = (uint32_t(ctr0[12]) << 24) | (uint32_t(ctr0[13]) << 16) |
                   (uint32_t(ctr0[14]) << 8) | uint32_t(ctr0[15]);
    } else if (mode == AES_MODE_CBC) {
        std::memcpy(a.ctr, ctr0, 16);   // the IV as little-endian words
    }
    hipError_t e;
    if (mode == AES_MODE_CBC && !decrypt) {
        // each block depends on the previous ciphertext: one lane, serially
        e = launch_cbc_encrypt(Nr, a, static_cast<hipStream_t>(stream));
        if (e != hipSuccess)
            return fail(AES_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        return AES_OK;
    }
    // CBC decryption has the shape of ECB decryption and shares its tuning
    const int kmode = mode == AES_MODE_CTR ? MODE_CTR : mode == AES_MODE_CBC ? MODE_CBC : MODE_ECB;
    const LaunchCfg cfg = choose_launch(*d, nbytes, mode == AES_MODE_CBC ? AES_MODE_ECB : mode, dec_cipher, Nr, kmode);
    if (cfg.layout == LAYOUT_BITSLICED) {
        if (dec_cipher)
            return fail(AES_E_ARG, "the bitsliced kernel encrypts only (ECB encrypt, CTR)");
        e = launch_bitslice(Nr, mode == AES_MODE_CTR ? MODE_CTR : MODE_ECB, cfg.grid, a,
                            static_cast<hipStream_t>(stream));
        if (e != hipSuccess)
            return fail(AES_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        return AES_OK;
    }
    e = launch_cipher(Nr, kmode, dec_cipher ? DIR_DEC : DIR_ENC, cfg, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return AES_OK;
}

int xts_crypt(int decrypt, const void *in, void *out, size_t nbytes, const uint8_t *rk1, const uint8_t *rk2,
              int Nr, size_t unit_bytes, uint64_t first_unit, void *stream) {
    if (Nr != 10 && Nr != 12 && Nr != 14)
        return fail(AES_E_NR, "Nr must be 10, 12 or 14");
    if (!rk1 || !rk2)
        return fail(AES_E_NULL, "roundkeys1 and roundkeys2 must not be NULL");
    if (unit_bytes < 16 || unit_bytes > 4096 || (unit_bytes & (unit_bytes - 1)) != 0)
        return fail(AES_E_ARG, "unit_bytes must be a power of two from 16 to 4096");
    if (nbytes % 16 != 0)
        return fail(AES_E_LENGTH, "XTS length must be a multiple of 16 bytes (no ciphertext stealing)");
    if (nbytes == 0)
        return AES_OK;
    int st = check_buffers(in, out, nbytes);
    if (st != AES_OK)
        return st;
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;

    XtsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.in = static_cast<const uint8_t *>(in);
    a.out = static_cast<uint8_t *>(out);
    a.nbytes = nbytes;
    a.first_unit = first_unit;
    uint32_t shift = 0;
    while ((uint64_t(16) << shift) < unit_bytes)
        shift++;
    a.unit_shift = shift;
    uint32_t w[60];
    const int nwords = 4 * (Nr + 1);
    for (int i = 0; i < nwords; i++)
        std::memcpy(&w[i], rk1 + 4 * i, 4);
    if (decrypt)
        decryption_schedule(w, Nr, a.rk1);
    else
        std::memcpy(a.rk1, w, 4 * nwords);
    for (int i = 0; i < nwords; i++)
        std::memcpy(&a.rk2[i], rk2 + 4 * i, 4);
    // one 1024-thread workgroup per CU, fewer if the buffer has fewer
    // groups of 64 units than the grid has waves
    const uint64_t nunits = ((nbytes >> 4) + (uint64_t(1) << shift) - 1) >> shift;
    const uint64_t groups = (nunits + 63) / 64;
    const int grid = int(std::min<uint64_t>(uint64_t(d->cus), (groups + 15) / 16));
    hipError_t e = launch_xts(Nr, decrypt ? DIR_DEC : DIR_ENC, grid, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return AES_OK;
}

int gcm_crypt(int decrypt, const void *in, void *out, size_t nbytes, const void *aad, size_t aad_bytes,
              const uint8_t *roundkeys, int Nr, const uint8_t *iv, size_t iv_bytes, void *tag, const void *tag_in,
              size_t tag_bytes, int *ok, void *workspace, size_t workspace_bytes, void *stream) {
    if (Nr != 10 && Nr != 12 && Nr != 14)
        return fail(AES_E_NR, "Nr must be 10, 12 or 14");
    if (!roundkeys || !iv || !workspace)
        return fail(AES_E_NULL, "roundkeys, iv and workspace must not be NULL");
    if (decrypt ? (!tag_in || !ok) : !tag)
        return fail(AES_E_NULL, decrypt ? "tag and ok must not be NULL" : "tag must not be NULL");
    if (iv_bytes < 1 || iv_bytes > 256)
        return fail(AES_E_ARG, "iv_bytes must be 1 .. 256");
    if (decrypt && !(tag_bytes == 4 || tag_bytes == 8 || (tag_bytes >= 12 && tag_bytes <= 16)))
        return fail(AES_E_ARG, "tag_bytes must be 4, 8 or 12 .. 16");
    if (nbytes > (uint64_t(1) << 36) - 32)
        return fail(AES_E_LENGTH, "GCM plaintext is limited to 2^36 - 32 bytes");
    if (aad_bytes > (uint64_t(1) << 36))
        return fail(AES_E_LENGTH, "additional data is limited to 2^36 bytes");
    if (aad_bytes && !aad)
        return fail(AES_E_NULL, "aad must not be NULL when aad_bytes > 0");
    if (reinterpret_cast<uintptr_t>(aad) & 15u)
        return fail(AES_E_ALIGN, "aad must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u)
        return fail(AES_E_ALIGN, "workspace must be 256-byte aligned");
    if (workspace_bytes < kGcmWorkspaceBytes)
        return fail(AES_E_LENGTH, "workspace smaller than aes_gcm_workspace_size reports");
    int st;
    if (nbytes) {
        st = check_buffers(in, out, nbytes);
        if (st != AES_OK)
            return st;
        const uintptr_t o = reinterpret_cast<uintptr_t>(out), ad = reinterpret_cast<uintptr_t>(aad);
        if (aad_bytes && ad < o + nbytes && o < ad + aad_bytes)
            return fail(AES_E_OVERLAP, "aad must not overlap out");
    }
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;

    GcmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.in = static_cast<const uint8_t *>(in);
    a.out = static_cast<uint8_t *>(out);
    a.nbytes = nbytes;
    a.aad = static_cast<const uint8_t *>(aad);
    a.aad_bytes = aad_bytes;
    a.ws = static_cast<GcmWork *>(workspace);
    a.tag_out = static_cast<uint8_t *>(tag);
    a.tag_in = static_cast<const uint8_t *>(tag_in);
    a.ok = ok;
    a.tag_bytes = uint32_t(tag_bytes);
    a.iv_bytes = uint32_t(iv_bytes);
    a.decrypt = uint32_t(decrypt);
    for (int i = 0; i < 4 * (Nr + 1); i++)
        std::memcpy(&a.rk[i], roundkeys + 4 * i, 4);
    std::memcpy(a.iv, iv, iv_bytes);
    // one chunk of 256 hash positions per wave, 16 waves per workgroup; the
    // workgroup count is a power of two (the folding factors are H^(2^t))
    const uint64_t positions = (nbytes + 15) / 16 + (aad_bytes + 15) / 16 + 1;
    const uint64_t wgs = (positions + 4095) / 4096;
    uint32_t lg = 0;
    while ((uint64_t(1) << lg) < wgs && (2 << lg) <= std::min(d->cus, kGcmMaxGrid))
        lg++;
    a.grid_log2 = lg;
    hipError_t e = launch_gcm(Nr, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return AES_OK;
}

// Cipher-kernel workgroups for a batch launch on this device.
int batch_grid(const DeviceState &d) { return std::min(d.cus, kBatchMaxWaves / kBatchWavesPerGroup); }

// The lists a batch may use (launch_batch's mask): without GCM fields the
// three cipher lists; with them also the GCM kernels, and the one-pass GCM
// list unless the caller asked for two passes throughout.
unsigned batch_lists(const aes_batch &b, const BatchKArgs &a) {
    if (!a.gcm)
        return 7u;
    return b.gcm_two_pass ? 15u : 31u;
}

int batch_args(const aes_batch *b, BatchKArgs *a) {
    if (!b)
        return fail(AES_E_NULL, "batch must not be NULL");
    if (!b->desc || !b->keys || !b->in_base || !b->out_base || !b->workspace)
        return fail(AES_E_NULL, "desc, keys, in_base, out_base and workspace must not be NULL");
    if (b->max_msgs < 1 || b->nmsg < 0 || b->nmsg > b->max_msgs || b->nkeys < 1)
        return fail(AES_E_ARG, "need 1 <= max_msgs, 0 <= nmsg <= max_msgs and nkeys >= 1");
    if (b->tile_blocks < 0 || b->tile_blocks > kMaxSplitBlocks)
        return fail(AES_E_ARG, "tile_blocks must be 0 .. " + std::to_string(kMaxSplitBlocks));
    if (b->blocks_per_thread != 0 && b->blocks_per_thread != 2 && b->blocks_per_thread != 4)
        return fail(AES_E_ARG, "blocks_per_thread must be 0, 2 or 4");
    if ((reinterpret_cast<uintptr_t>(b->in_base) | reinterpret_cast<uintptr_t>(b->out_base)) & 15u)
        return fail(AES_E_ALIGN, "in_base and out_base must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(b->workspace) & 255u)
        return fail(AES_E_ALIGN, "workspace must be 256-byte aligned");
    if (b->workspace_bytes < batch_layout(b->max_msgs))
        return fail(AES_E_LENGTH, "workspace smaller than aes_batch_workspace_size reports");
    char *ws = static_cast<char *>(b->workspace);
    a->desc = b->desc;
    a->nmsg = b->nmsg;
    a->d_nmsg = b->d_nmsg;
    a->max_msgs = b->max_msgs;
    a->keys = b->keys;
    a->nkeys = b->nkeys;
    a->in_base = b->in_base;
    a->in_bytes = b->in_bytes;
    a->out_base = b->out_base;
    a->out_bytes = b->out_bytes;
    const size_t items_off = sizeof(BatchHeader) + size_t(b->max_msgs) * kKeySlotWords * 4;
    a->header = reinterpret_cast<BatchHeader *>(ws);
    a->keytab = reinterpret_cast<uint32_t *>(ws + sizeof(BatchHeader));
    a->items = reinterpret_cast<BatchItem *>(ws + items_off);
    a->chunk_totals =
        reinterpret_cast<uint64_t *>(ws + items_off + size_t(kBatchLists) * size_t(b->max_msgs) * sizeof(BatchItem));
    a->split_blocks = uint32_t(b->tile_blocks ? b->tile_blocks : kDefaultSplitBlocks);
    a->bpt = uint32_t(b->blocks_per_thread ? b->blocks_per_thread : 4);
    a->reject_flags = nullptr;
    a->gcm = b->gcm;
    if (reinterpret_cast<uintptr_t>(b->gcm) & 7u)
        return fail(AES_E_ALIGN, "gcm must be 8-byte aligned");
    return AES_OK;
}

}  // namespace

// Helpers the request loop (serve.cpp) shares with this file.
namespace aesgpu {
int serve_fail(int status, const std::string &msg) { return fail(status, msg); }
int serve_device(int *cus, int *batch_grid_out) {
    int st;
    const DeviceState *d = current_device(&st);
    if (d) {
        *cus = d->cus;
        *batch_grid_out = batch_grid(*d);
    }
    return st;
}
size_t serve_batch_layout(int max_msgs) { return batch_layout(max_msgs); }
int serve_batch_args(const aes_batch *b, BatchKArgs *a) { return batch_args(b, a); }
}  // namespace aesgpu

extern "C" {

int aes_expand_key(const uint8_t *key, int keybits, uint8_t *roundkeys, int *Nr) {
    if (!key || !roundkeys || !Nr)
        return fail(AES_E_NULL, "key, roundkeys and Nr must not be NULL");
    uint32_t w[60];
    const int nr = expand_key_host(key, keybits, w);
    if (nr < 0)
        return fail(AES_E_KEYBITS, "keybits must be 128, 192 or 256");
    for (int i = 0; i < 4 * (nr + 1); i++)
        std::memcpy(roundkeys + 4 * i, &w[i], 4);
    *Nr = nr;
    return AES_OK;
}

int aes_encrypt(const void *in, void *out, size_t nbytes, const uint8_t *roundkeys, int Nr, int mode,
                const uint8_t *ctr0, void *stream) {
    return crypt(0, in, out, nbytes, roundkeys, Nr, mode, ctr0, stream);
}

int aes_decrypt(const void *in, void *out, size_t nbytes, const uint8_t *roundkeys, int Nr, int mode,
                const uint8_t *ctr0, void *stream) {
    return crypt(1, in, out, nbytes, roundkeys, Nr, mode, ctr0, stream);
}

int aes_xts_encrypt(const void *in, void *out, size_t nbytes, const uint8_t *roundkeys1,
                    const uint8_t *roundkeys2, int Nr, size_t unit_bytes, uint64_t first_unit, void *stream) {
    return xts_crypt(0, in, out, nbytes, roundkeys1, roundkeys2, Nr, unit_bytes, first_unit, stream);
}

int aes_xts_decrypt(const void *in, void *out, size_t nbytes, const uint8_t *roundkeys1,
                    const uint8_t *roundkeys2, int Nr, size_t unit_bytes, uint64_t first_unit, void *stream) {
    return xts_crypt(1, in, out, nbytes, roundkeys1, roundkeys2, Nr, unit_bytes, first_unit, stream);
}

int aes_gcm_workspace_size(size_t *bytes) {
    if (!bytes)
        return fail(AES_E_NULL, "bytes must not be NULL");
    *bytes = kGcmWorkspaceBytes;
    return AES_OK;
}

int aes_gcm_encrypt(const void *in, void *out, size_t nbytes, const void *aad, size_t aad_bytes,
                    const uint8_t *roundkeys, int Nr, const uint8_t *iv, size_t iv_bytes, void *tag,
                    void *workspace, size_t workspace_bytes, void *stream) {
    return gcm_crypt(0, in, out, nbytes, aad, aad_bytes, roundkeys, Nr, iv, iv_bytes, tag, nullptr, 16, nullptr,
                     workspace, workspace_bytes, stream);
}

int aes_gcm_decrypt(const void *in, void *out, size_t nbytes, const void *aad, size_t aad_bytes,
                    const uint8_t *roundkeys, int Nr, const uint8_t *iv, size_t iv_bytes, const void *tag,
                    size_t tag_bytes, int *ok, void *workspace, size_t workspace_bytes, void *stream) {
    return gcm_crypt(1, in, out, nbytes, aad, aad_bytes, roundkeys, Nr, iv, iv_bytes, nullptr, tag, tag_bytes, ok,
                     workspace, workspace_bytes, stream);
}

const char *aes_last_error(void) { return g_error.c_str(); }

int aes_set_launch(const aes_launch *cfg) {
    std::lock_guard<std::mutex> lk(g_launch_mu);
    if (!cfg) {
        g_launch_set = false;
        g_launch = aes_launch{0, 0, 0, 0};
        return AES_OK;
    }
    if (!valid_launch(*cfg))
        return fail(AES_E_ARG, "launch configuration out of range");
    g_launch = *cfg;
    g_launch_set = true;
    return AES_OK;
}

int aes_set_tuned(const aes_tuned_entry *entries, int n) {
    if (n < 0 || n > 256 || (n > 0 && !entries))
        return fail(AES_E_ARG, "0 <= n <= 256 entries, entries not NULL");
    for (int i = 0; i < n; i++) {
        const aes_tuned_entry &e = entries[i];
        if ((e.mode != AES_MODE_ECB && e.mode != AES_MODE_CTR) || (e.decrypt != 0 && e.decrypt != 1) ||
            (e.Nr != 10 && e.Nr != 12 && e.Nr != 14) || !valid_launch(e.cfg))
            return fail(AES_E_ARG, "tuned entry " + std::to_string(i) + " out of range");
        if (e.cfg.layout == LAYOUT_BITSLICED && e.mode == AES_MODE_ECB && e.decrypt)
            return fail(AES_E_ARG, "tuned entry " + std::to_string(i) + ": bitsliced layout cannot decrypt ECB");
    }
    std::lock_guard<std::mutex> lk(g_launch_mu);
    g_tuned.assign(entries, entries + n);
    return AES_OK;
}

int aes_get_launch(size_t nbytes, int mode, int decrypt, int Nr, aes_launch *cfg) {
    if (!cfg)
        return fail(AES_E_NULL, "cfg must not be NULL");
    int st;
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;
    const LaunchCfg c = choose_launch(*d, nbytes, mode, decrypt && mode == AES_MODE_ECB, Nr,
                                      mode == AES_MODE_CTR ? MODE_CTR : MODE_ECB);
    cfg->layout = c.layout;
    cfg->blocks_per_thread = c.bpt;
    cfg->wg_size = c.wg;
    cfg->grid = c.grid;
    return AES_OK;
}

int aes_copy(const void *in, void *out, size_t nbytes, void *stream) {
    if (nbytes % 16 != 0)
        return fail(AES_E_LENGTH, "copy length must be a multiple of 16 bytes");
    if (nbytes == 0)
        return AES_OK;
    int st = check_buffers(in, out, nbytes);
    if (st != AES_OK)
        return st;
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;
    hipError_t e = launch_copy(in, out, nbytes, d->cus, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return AES_OK;
}

int aes_lds_gather(aes_lds_gather_stat *out, size_t out_bytes, int rounds, int *waves, int *tick_khz,
                   void *stream) {
    return aes_lds_gather_layout(out, out_bytes, rounds, LAYOUT_T4X32, waves, tick_khz, stream);
}

int aes_lds_gather_layout(aes_lds_gather_stat *out, size_t out_bytes, int rounds, int layout, int *waves,
                          int *tick_khz, void *stream) {
    if (!out || !waves || !tick_khz)
        return fail(AES_E_NULL, "out, waves and tick_khz must not be NULL");
    if (rounds < 1)
        return fail(AES_E_ARG, "need rounds >= 1");
    if (layout != LAYOUT_T4X32 && layout != LAYOUT_T1X64)
        return fail(AES_E_ARG, "layout must be 0 (four tables x 32 copies) or 3 (one table x 64 copies)");
    int st = AES_OK;
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;
    int dev = 0;
    hipError_t a = hipGetDevice(&dev);
    if (a == hipSuccess)
        a = hipDeviceGetAttribute(tick_khz, hipDeviceAttributeWallClockRate, dev);
    if (a != hipSuccess)
        return fail(AES_E_DEVICE, std::string("wall clock rate: ") + hipGetErrorString(a));
    const int grid = d->cus * lds_gather_groups_per_cu(layout);
    const int nw = grid * kLdsGatherWavesPerGroup;
    *waves = nw;
    if (out_bytes < size_t(nw) * sizeof(aes_lds_gather_stat))
        return fail(AES_E_LENGTH, "out must hold one record per wave (" + std::to_string(nw) + " waves)");
    hipError_t e = launch_lds_gather(out, uint32_t(rounds), layout, grid, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return AES_OK;
}

int aes_batch_workspace_size(int max_msgs, size_t *bytes) {
    if (!bytes)
        return fail(AES_E_NULL, "bytes must not be NULL");
    if (max_msgs < 1)
        return fail(AES_E_ARG, "need max_msgs >= 1");
    *bytes = batch_layout(max_msgs);
    return AES_OK;
}

int aes_batch_plan(const aes_msg_desc *d_desc, int nmsg, size_t *workspace_bytes) {
    (void)d_desc;   // the workspace depends on the message count only
    if (!workspace_bytes)
        return fail(AES_E_NULL, "workspace_bytes must not be NULL");
    if (nmsg < 1)
        return fail(AES_E_ARG, "need nmsg >= 1");
    *workspace_bytes = batch_layout(nmsg);
    return AES_OK;
}

int aes_batch_run(const aes_batch *b, void *stream) {
    BatchKArgs a;
    int st = batch_args(b, &a);
    if (st != AES_OK)
        return st;
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;
    // without a device-side count the host knows how many messages there are
    // the GHASH and tag kernels only if the batch can hold GCM messages
    hipError_t e = launch_batch(a, batch_grid(*d), static_cast<hipStream_t>(stream), batch_lists(*b, a),
                                a.d_nmsg ? a.max_msgs : a.nmsg);
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    return AES_OK;
}

int aes_batch_run_noalloc(const aes_batch *b, void *stream) {
    if (!b)
        return fail(AES_E_NULL, "batch must not be NULL");
    if (b->workspace || b->workspace_bytes)
        return fail(AES_E_ARG, "the no-allocation call uses the library's own workspace: "
                               "workspace must be NULL and workspace_bytes 0");
    if (b->max_msgs > AES_BATCH_NOALLOC_MAX_MSGS)
        return fail(AES_E_LENGTH, "max_msgs is limited to " + std::to_string(AES_BATCH_NOALLOC_MAX_MSGS) +
                                      " without a caller-supplied workspace");
    int st;
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    aes_batch w = *b;
    w.workspace = batch_scratch(dev);   // the array's device address, looked up at set-up
    w.workspace_bytes = kNoAllocScratchBytes;
    if (!w.workspace)
        return fail(AES_E_DEVICE, "the library's batch workspace has no address on this device");
    BatchKArgs a;
    st = batch_args(&w, &a);
    if (st != AES_OK)
        return st;
    e = launch_batch(a, batch_grid(*d), static_cast<hipStream_t>(stream), batch_lists(*b, a),
                     a.d_nmsg ? a.max_msgs : a.nmsg);
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    return AES_OK;
}

int aes_batch_query(const aes_batch *b, void *stream, uint64_t *planned, uint64_t *rejected) {
    BatchKArgs a;
    int st = batch_args(b, &a);
    if (st != AES_OK)
        return st;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    BatchHeader h;
    if (e == hipSuccess)
        e = hipMemcpy(&h, a.header, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("batch query: ") + hipGetErrorString(e));
    if (planned)
        *planned = uint64_t(h.nitems[0]) + h.nitems[1] + h.nitems[2] + h.nfused[0] + h.nfused[1] + h.nfused[2];
    if (rejected)
        *rejected = h.rejected;
    return AES_OK;
}

int aes_batch_graph_create(const aes_batch *b, void **graph) {
    if (!graph)
        return fail(AES_E_NULL, "graph must not be NULL");
    BatchKArgs a;
    int st = batch_args(b, &a);
    if (st != AES_OK)
        return st;
    const DeviceState *d = current_device(&st);
    if (!d)
        return st;
    hipStream_t s = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // the count may change per replay
        hipError_t le = launch_batch(a, batch_grid(*d), s, batch_lists(*b, a), a.max_msgs);
        e = hipStreamEndCapture(s, &g);
        if (le != hipSuccess)
            e = le;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (g)
        (void)hipGraphDestroy(g);
    if (s)
        (void)hipStreamDestroy(s);
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    *graph = x;
    return AES_OK;
}

int aes_batch_graph_launch(void *graph, void *stream) {
    if (!graph)
        return fail(AES_E_NULL, "graph must not be NULL");
    hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(graph), static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
    return AES_OK;
}

int aes_batch_graph_destroy(void *graph) {
    if (!graph)
        return AES_OK;
    hipError_t e = hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph));
    if (e != hipSuccess)
        return fail(AES_E_DEVICE, std::string("graph destroy: ") + hipGetErrorString(e));
    return AES_OK;
}

}  // extern "C"
