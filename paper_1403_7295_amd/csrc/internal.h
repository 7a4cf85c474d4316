// Declarations shared by the library's own translation units (not public).
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime_api.h>

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

// ---- kernels (aes_kernels.hip) --------------------------------------------
enum Mode { MODE_ECB = 0, MODE_CTR = 1 };
enum Dir { DIR_ENC = 0, DIR_DEC = 1 };
enum Layout { LAYOUT_T4X32 = 0, LAYOUT_T2X64 = 1 };

// Everything one launch of a buffer kernel needs; passed by value, so the
// round keys and counter land in scalar registers.
struct CipherArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t nbytes;
    uint32_t rk[60];   // round keys in the order the rounds use them
    uint32_t ctr[4];   // CTR: nonce words 0..2 (little-endian), ctr[3] = c0
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
hipError_t launch_copy(const void *in, void *out, uint64_t nbytes, int grid, hipStream_t stream);

}  // namespace aesgpu
