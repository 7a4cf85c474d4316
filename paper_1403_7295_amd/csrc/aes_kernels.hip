// AES buffer kernels for gfx950 (MI355X): ECB encryption, ECB decryption and
// CTR over one buffer, for Nr = 10, 12, 14, plus the plain copy kernel the
// measurements are calibrated with.  The round code is in cipher_core.h.
//
// The grid is persistent: a fixed number of workgroups (as many as fit on
// every compute unit at once: one for the 128 KiB table layouts, two for the
// 64 KiB one) sweeps the buffer, so the tables are staged into LDS once per
// workgroup, not once per tile.
// Lane l of a wave owns blocks base + 64*i + l, so every 16-byte load and
// store instruction of a wave covers 1 KiB of contiguous memory.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "cipher_core.h"
#include "internal.h"

namespace aesgpu {
namespace {

template <int NR, int MODE, int DIR, int LAYOUT, int BPT>
__global__ __launch_bounds__(1024) void cipher_kernel(const CipherArgs a) {
    __shared__ uint32_t lds[lds_words<DIR, LAYOUT>()];
    stage_tables<LAYOUT, DIR>(lds);
    __syncthreads();

    const LaneConsts lc = lane_consts<LAYOUT>(threadIdx.x & 63u);
    const uint64_t nblk = (a.nbytes + 15) >> 4;
    // the wave index is the same in all 64 lanes; saying so lets the block
    // loop keep its base address in scalar registers
    const uint64_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint64_t sweep = uint64_t(gridDim.x) * blockDim.x * BPT;  // blocks per pass of the grid
    process_blocks<NR, MODE, DIR, LAYOUT, BPT>(lds, lc, a.rk, a.ctr, a.in, a.out, a.nbytes,
                                               wave * 64u * BPT, nblk, sweep);
}

// CBC encryption of one buffer: inherently serial, so the first quad of
// lanes does all of it (one column of the state each) after the workgroup
// has staged the tables.
template <int NR>
__global__ __launch_bounds__(256) void cbc_encrypt_kernel(const CipherArgs a) {
    __shared__ uint32_t lds[lds_words<DIR_ENC>()];
    stage_tables<LAYOUT_T4X32, DIR_ENC>(lds);
    __syncthreads();
    if (threadIdx.x >= 4)
        return;
    const uint32_t j = threadIdx.x;
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(j);
    // this lane's column of every round key, and of the IV
    uint32_t rk[NR + 1];
#pragma unroll
    for (int r = 0; r <= NR; r++)
        rk[r] = j == 0 ? a.rk[4 * r] : j == 1 ? a.rk[4 * r + 1] : j == 2 ? a.rk[4 * r + 2] : a.rk[4 * r + 3];
    const uint32_t iv = j == 0 ? a.ctr[0] : j == 1 ? a.ctr[1] : j == 2 ? a.ctr[2] : a.ctr[3];
    cbc_encrypt_quad<NR, LAYOUT_T4X32>(lds, lc, rk, iv, a.in, a.out, a.nbytes >> 4);
}

template <int BPT>
__global__ __launch_bounds__(1024) void copy_kernel(const uint8_t *in, uint8_t *out, uint64_t n16) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t sweep = uint64_t(gridDim.x) * blockDim.x * BPT;
    for (uint64_t base = wave * 64u * BPT; base < n16; base += sweep) {
        u32x4 x[BPT];
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint64_t j = base + uint64_t(i) * 64u + lane;
            if (j < n16)
                x[i] = load16(in + 16 * j);
        }
#pragma unroll
        for (int i = 0; i < BPT; i++) {
            const uint64_t j = base + uint64_t(i) * 64u + lane;
            if (j < n16)
                store16(out + 16 * j, x[i]);
        }
    }
}

using KernelFn = void (*)(const CipherArgs);

template <int NR, int MODE, int DIR, int LAYOUT>
KernelFn pick_bpt(int bi) {
    return bi == 0 ? cipher_kernel<NR, MODE, DIR, LAYOUT, 1>
         : bi == 1 ? cipher_kernel<NR, MODE, DIR, LAYOUT, 2>
                   : cipher_kernel<NR, MODE, DIR, LAYOUT, 4>;
}

template <int NR, int MODE, int DIR>
KernelFn pick_layout(int layout, int bi) {
    return layout == LAYOUT_T4X32 ? pick_bpt<NR, MODE, DIR, LAYOUT_T4X32>(bi)
         : layout == LAYOUT_T2X64 ? pick_bpt<NR, MODE, DIR, LAYOUT_T2X64>(bi)
         : layout == LAYOUT_T1X64 ? pick_bpt<NR, MODE, DIR, LAYOUT_T1X64>(bi)
                                  : pick_bpt<NR, MODE, DIR, LAYOUT_T4X1>(bi);
}

template <int NR>
KernelFn pick_op(int mode, int dir, int layout, int bi) {
    if (mode == MODE_CTR)
        return pick_layout<NR, MODE_CTR, DIR_ENC>(layout, bi);
    if (mode == MODE_CBC)   // decryption only: CBC encryption is serial
        return pick_layout<NR, MODE_CBC, DIR_DEC>(layout, bi);
    return dir == DIR_ENC ? pick_layout<NR, MODE_ECB, DIR_ENC>(layout, bi)
                          : pick_layout<NR, MODE_ECB, DIR_DEC>(layout, bi);
}

KernelFn cipher_fn(int nr, int mode, int dir, int layout, int bpt) {
    const int bi = bpt == 1 ? 0 : bpt == 2 ? 1 : 2;
    return nr == 10 ? pick_op<10>(mode, dir, layout, bi)
         : nr == 12 ? pick_op<12>(mode, dir, layout, bi)
                    : pick_op<14>(mode, dir, layout, bi);
}

}  // namespace

hipError_t upload_tables(const HostTables &t) { return upload_base_tables(t); }

int cipher_groups_per_cu(int nr, int mode, int dir, int layout, int bpt, int wg) {
    // what the kernel's LDS array and registers allow, asked of the runtime
    // once per kernel and workgroup size
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> known;
    const void *fn = reinterpret_cast<const void *>(cipher_fn(nr, mode, dir, layout, bpt));
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find({fn, wg});
    if (it != known.end())
        return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, wg, 0) != hipSuccess || n < 1)
        n = 1;
    known[{fn, wg}] = n;
    return n;
}

hipError_t launch_cipher(int nr, int mode, int dir, const LaunchCfg &cfg, const CipherArgs &a,
                         hipStream_t stream) {
    KernelFn fn = cipher_fn(nr, mode, dir, cfg.layout, cfg.bpt);
    hipLaunchKernelGGL(fn, dim3(cfg.grid), dim3(cfg.wg), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_cbc_encrypt(int nr, const CipherArgs &a, hipStream_t stream) {
    void (*fn)(const CipherArgs) = nr == 10 ? cbc_encrypt_kernel<10> : nr == 12 ? cbc_encrypt_kernel<12>
                                                                               : cbc_encrypt_kernel<14>;
    hipLaunchKernelGGL(fn, dim3(1), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_copy(const void *in, void *out, uint64_t nbytes, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(copy_kernel<4>, dim3(grid), dim3(1024), 0, stream,
                       static_cast<const uint8_t *>(in), static_cast<uint8_t *>(out), nbytes >> 4);
    return hipGetLastError();
}

}  // namespace aesgpu
