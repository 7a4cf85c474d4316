// XTS-AES (IEEE 1619; NIST SP 800-38E) on one group of at most 64
// consecutive data units, by one wave; shared by the buffer kernel and the
// batch kernel.  Block j of a unit is
//     C_j = Cipher_K1(P_j ^ T_j) ^ T_j,   T_j = Cipher_K2(i) * alpha^j
// in GF(2^128) with x^128 + x^7 + x^2 + x + 1 (decryption uses InvCipher_K1).
// Units are powers of two from 16 bytes to 4 KiB, so within a unit j < 256.
//
// Lane l encrypts the tweak of the group's unit l (one AES per lane per
// group: through the LDS round tables when encrypting; when decrypting the
// LDS holds the inverse tables, so the tweak's forward rounds read the 1 KiB
// base table from global memory), then the wave runs through the group's
// blocks 64 x BPT at a time.  A block fetches its unit's tweak from the
// owning lane (ds_bpermute; a scalar readlane when units span 64 blocks or
// more, so a slot of 64 blocks lies in one unit) and multiplies it by
// alpha^j: one shift by j mod 64 with reduction, then up to three shifts by
// 64.
#pragma once

#include <hip/hip_runtime.h>

#include "cipher_core.h"
#include "gf128.h"
#include "internal.h"

namespace aesgpu {
namespace {

// Blocks [gb0, gb1) of the buffer at in/out (gb0 is the first block of a
// unit, the range covers at most 64 units of 2^ushift blocks); unit0 is the
// tweak value of the unit starting at gb0.  rk1: the data key in the order
// the rounds use it (wave-uniform); rk2: the tweak key's encryption schedule.
// known, if not NULL, holds the encrypted tweak of unit known_unit, which
// the lane owning that unit loads instead of computing it.
template <int NR, int DIR, int BPT>
__device__ __forceinline__ void xts_group(const uint32_t *lds, const LaneConsts &lc, const uint32_t *rk1,
                                          const uint32_t *rk2, const uint8_t *in, uint8_t *out, uint64_t gb0,
                                          uint64_t gb1, uint64_t unit0, uint32_t ushift,
                                          const uint32_t *known = nullptr, uint64_t known_unit = 0) {
    const uint32_t lane = threadIdx.x & 63u;
    // the tweak of unit unit0 + lane: Cipher_K2 of the unit number, little-endian;
    // only lanes that own one of the group's units compute it (a batch of
    // one-unit messages has one per group, and inactive lanes cost the LDS
    // and the vector memory path nothing); the others' tweaks are never used
    const uint64_t unit = unit0 + lane;
    const uint32_t units = uint32_t((gb1 - gb0 + (uint64_t(1) << ushift) - 1) >> ushift);
    uint32_t tw[4] = {uint32_t(unit), uint32_t(unit >> 32), 0u, 0u};
    if (known && lane < units && unit == known_unit) {
#pragma unroll
        for (int c = 0; c < 4; c++)
            tw[c] = known[c];
    } else if (lane < units) {
        if (DIR == DIR_ENC) {
            uint32_t t1[1][4] = {{tw[0] ^ rk2[0], tw[1] ^ rk2[1], rk2[2], rk2[3]}};
            rounds<NR, DIR_ENC, LAYOUT_T4X32, 1>(t1, lds, lc, rk2, 1);
#pragma unroll
            for (int c = 0; c < 4; c++)
                tw[c] = t1[0][c];
        } else {
            encrypt_global<NR>(rk2, tw);
        }
    }
    // when a unit spans at least 64 x BPT blocks, a lane's BPT blocks of a
    // step (64 apart, the step starting on a multiple of 64 x BPT inside the
    // unit) all lie in one unit, and each tweak is the previous one times
    // alpha^64: one shift by 64 with reduction instead of a shift by j
    constexpr uint32_t kLogBpt = BPT == 1 ? 0u : BPT == 2 ? 1u : BPT == 4 ? 2u : 3u;
    const bool one_unit = ushift >= 6u + kLogBpt;
    for (uint64_t base = gb0; base < gb1; base += 64u * BPT) {
        const uint32_t nwhole = uint32_t(min<uint64_t>(gb1 - base, 64u * BPT));
        const uint8_t *inb = in + 16 * base;
        uint8_t *outb = out + 16 * base;
        uint32_t s[BPT][4];
        uint64_t tlo[BPT], thi[BPT];
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint32_t jj = uint32_t(i) * 64u + lane;
            uint64_t lo, hi;
            if (i > 0 && one_unit) {
                lo = tlo[i - 1];
                hi = thi[i - 1];
                mulx64(lo, hi);
                tlo[i] = lo;
                thi[i] = hi;
                u32x4 x = vec4(0, 0, 0, 0);
                if (jj < nwhole)
                    x = load16(inb + 16u * jj);
                s[i][0] = x.x ^ uint32_t(lo) ^ rk1[0];
                s[i][1] = x.y ^ uint32_t(lo >> 32) ^ rk1[1];
                s[i][2] = x.z ^ uint32_t(hi) ^ rk1[2];
                s[i][3] = x.w ^ uint32_t(hi >> 32) ^ rk1[3];
                continue;
            }
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
            lo = uint64_t(w0) | (uint64_t(w1) << 32);
            hi = uint64_t(w2) | (uint64_t(w3) << 32);
            mulx_pow(lo, hi, j);
            tlo[i] = lo;
            thi[i] = hi;
            u32x4 x = vec4(0, 0, 0, 0);
            if (jj < nwhole)
                x = load16(inb + 16u * jj);
            s[i][0] = x.x ^ uint32_t(lo) ^ rk1[0];
            s[i][1] = x.y ^ uint32_t(lo >> 32) ^ rk1[1];
            s[i][2] = x.z ^ uint32_t(hi) ^ rk1[2];
            s[i][3] = x.w ^ uint32_t(hi >> 32) ^ rk1[3];
        }
        rounds<NR, DIR, LAYOUT_T4X32, BPT>(s, lds, lc, rk1, 1);
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

}  // namespace
}  // namespace aesgpu
