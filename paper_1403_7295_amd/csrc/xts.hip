// XTS-AES (IEEE 1619; NIST SP 800-38E) for gfx950: a buffer of data units
// (sectors), unit u with tweak value first_unit + u.  Block j of a unit is
//     C_j = Cipher_K1(P_j ^ T_j) ^ T_j,   T_j = Cipher_K2(i) * alpha^j
// in GF(2^128) with x^128 + x^7 + x^2 + x + 1 (decryption uses InvCipher_K1).
// Units are powers of two from 16 bytes to 4 KiB, so within a unit j < 256.
//
// Work: each wave takes groups of 64 consecutive units.  Lane l encrypts the
// tweak of unit 64g + l (one AES per lane per group: through the LDS round
// tables when encrypting; when decrypting the LDS holds the inverse tables,
// so the tweak's forward rounds read the 1 KiB base table from global
// memory), then the wave runs through the group's blocks 64 x BPT at a time
// like the ECB kernels.  A block fetches its unit's tweak from the owning
// lane (ds_bpermute; a scalar readlane when units span 64 blocks or more, so
// a slot of 64 blocks lies in one unit) and multiplies it by alpha^j: one
// shift by j mod 64 with reduction, then up to three shifts by 64.
#include <hip/hip_runtime.h>

#include "cipher_core.h"
#include "gf128.h"
#include "internal.h"

namespace aesgpu {
namespace {

template <int NR, int DIR, int BPT>
__global__ __launch_bounds__(1024) void xts_kernel(const XtsArgs a) {
    __shared__ uint32_t lds[lds_words<DIR>()];
    stage_tables<LAYOUT_T4X32, DIR>(lds);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(lane);
    const uint64_t nblk = a.nbytes >> 4;
    const uint32_t ushift = a.unit_shift;                 // log2(blocks per unit), 0..8
    const uint64_t nunits = (nblk + (uint64_t(1) << ushift) - 1) >> ushift;
    const uint64_t ngroups = (nunits + 63) >> 6;
    const uint64_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint64_t nwaves = uint64_t(gridDim.x) * (blockDim.x >> 6);
    for (uint64_t g = wave; g < ngroups; g += nwaves) {
        // the tweak of unit 64g + lane: Cipher_K2 of the unit number, little-endian
        const uint64_t unit = a.first_unit + 64 * g + lane;
        uint32_t tw[4] = {uint32_t(unit), uint32_t(unit >> 32), 0u, 0u};
        if (DIR == DIR_ENC) {
            uint32_t t1[1][4] = {{tw[0] ^ a.rk2[0], tw[1] ^ a.rk2[1], a.rk2[2], a.rk2[3]}};
            rounds<NR, DIR_ENC, LAYOUT_T4X32, 1>(t1, lds, lc, a.rk2, 1);
#pragma unroll
            for (int c = 0; c < 4; c++)
                tw[c] = t1[0][c];
        } else {
            encrypt_global<NR>(a.rk2, tw);
        }
        const uint64_t gb0 = (64 * g) << ushift;           // first block of the group
        const uint64_t gb1 = min(nblk, (64 * (g + 1)) << ushift);
        for (uint64_t base = gb0; base < gb1; base += 64u * BPT) {
            const uint32_t nwhole = uint32_t(min<uint64_t>(gb1 - base, 64u * BPT));
            const uint8_t *inb = a.in + 16 * base;
            uint8_t *outb = a.out + 16 * base;
            uint32_t s[BPT][4];
            uint64_t tlo[BPT], thi[BPT];
#pragma unroll
            for (int i = 0; i < BPT; i++) {
                const uint32_t jj = uint32_t(i) * 64u + lane;
                const uint64_t k = base - gb0 + jj;            // block index within the group
                const uint32_t src = uint32_t(k >> ushift) & 63u;
                const uint32_t j = uint32_t(k) & ((1u << ushift) - 1u);
                uint32_t w0, w1, w2, w3;
                if (ushift >= 6) {
                    // 64-aligned slot inside one unit: src is the same on every lane
                    const int us = __builtin_amdgcn_readfirstlane(int(src));
                    w0 = __builtin_amdgcn_readlane(int(tw[0]), us);
                    w1 = __builtin_amdgcn_readlane(int(tw[1]), us);
                    w2 = __builtin_amdgcn_readlane(int(tw[2]), us);
                    w3 = __builtin_amdgcn_readlane(int(tw[3]), us);
                } else {
                    // all lanes take part in the permutes
                    w0 = __builtin_amdgcn_ds_bpermute(int(src << 2), int(tw[0]));
                    w1 = __builtin_amdgcn_ds_bpermute(int(src << 2), int(tw[1]));
                    w2 = __builtin_amdgcn_ds_bpermute(int(src << 2), int(tw[2]));
                    w3 = __builtin_amdgcn_ds_bpermute(int(src << 2), int(tw[3]));
                }
                uint64_t lo = uint64_t(w0) | (uint64_t(w1) << 32), hi = uint64_t(w2) | (uint64_t(w3) << 32);
                mulx_pow(lo, hi, j);
                tlo[i] = lo;
                thi[i] = hi;
                u32x4 x = vec4(0, 0, 0, 0);
                if (jj < nwhole)
                    x = load16(inb + 16u * jj);
                s[i][0] = x.x ^ uint32_t(lo) ^ a.rk1[0];
                s[i][1] = x.y ^ uint32_t(lo >> 32) ^ a.rk1[1];
                s[i][2] = x.z ^ uint32_t(hi) ^ a.rk1[2];
                s[i][3] = x.w ^ uint32_t(hi >> 32) ^ a.rk1[3];
            }
            rounds<NR, DIR, LAYOUT_T4X32, BPT>(s, lds, lc, a.rk1, 1);
#pragma unroll
            for (int i = 0; i < BPT; i++) {
                const uint32_t jj = uint32_t(i) * 64u + lane;
                if (jj < nwhole)
                    store16(outb + 16u * jj,
                            vec4(s[i][0] ^ uint32_t(tlo[i]), s[i][1] ^ uint32_t(tlo[i] >> 32),
                                 s[i][2] ^ uint32_t(thi[i]), s[i][3] ^ uint32_t(thi[i] >> 32)));
            }
        }
    }
}

}  // namespace

hipError_t upload_tables_xts(const HostTables &t) { return upload_base_tables(t); }

hipError_t launch_xts(int nr, int dir, int grid, const XtsArgs &a, hipStream_t stream) {
    void (*fn)(const XtsArgs);
    if (dir == DIR_ENC)
        fn = nr == 10 ? xts_kernel<10, DIR_ENC, 4> : nr == 12 ? xts_kernel<12, DIR_ENC, 4> : xts_kernel<14, DIR_ENC, 4>;
    else
        fn = nr == 10 ? xts_kernel<10, DIR_DEC, 4> : nr == 12 ? xts_kernel<12, DIR_DEC, 4> : xts_kernel<14, DIR_DEC, 4>;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

}  // namespace aesgpu
