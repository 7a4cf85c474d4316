// LDS gather calibration kernel (not part of the cipher).  It issues the
// table kernels' kind of LDS access, 32-bit reads in which every lane reads
// its own bank, as fast as the LDS accepts them, with no global memory
// traffic and almost no VALU work, and so measures the lookup rate the
// cipher's issue roofline is compared with on the device at hand.
//
// Launch shape as the cipher: 1024-thread workgroups, 16 waves each, as many
// per compute unit as fit.  The LDS array is laid out as one of the cipher's
// table layouts: four round tables of 256 entries x 32 copies (copy = lane &
// 31, 128 KiB, one workgroup per CU), or one table x 64 copies at a 256-byte
// stride (copy = lane, 64 KiB, two workgroups per CU).  Per round each lane
// takes four words, one per column as the cipher has, and looks byte K of
// each up in table K (or in the one table): 16 reads, each address built by
// one v_perm_b32 from the word and a per-lane constant, the 16 words folded
// by three-input XORs.  That is the cipher's lookup instruction
// stream; what it leaves out is global memory, the round keys, and the
// dependence of a round's addresses on the previous round's reads: the
// words advance by a constant each round instead, so the loop measures what
// the LDS accepts rather than how well the cipher hides its latency.
//
// Each wave also reads the cycle counter (s_memtime) and the constant-rate
// wall clock (s_memrealtime) around its loop; the host reports the ratio of
// the two deltas as the counter's rate.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace aesgpu {
namespace {

constexpr uint32_t kGatherReads = 16;      // reads per lane per round

// words of the LDS array: 128 KiB (four tables x 32 copies) or 64 KiB (one table x 64 copies)
template <int LAYOUT>
constexpr uint32_t gather_words() { return LAYOUT == LAYOUT_T1X64 ? 16384u : 32768u; }

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

template <int LAYOUT>
__global__ __launch_bounds__(1024) void lds_gather_kernel(LdsGatherStat *out, uint32_t rounds) {
    __shared__ uint32_t lds[gather_words<LAYOUT>()];
    for (uint32_t i = threadIdx.x; i < gather_words<LAYOUT>(); i += blockDim.x)
        lds[i] = i * 0x9E3779B1u;
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63u;
    const char *bytes = reinterpret_cast<const char *>(lds);
    // four tables: byte 0 the copy (lane & 31) and table bit 0, byte 1 table
    // bit 1 (to address bit 16); one table: byte 0 the copy (lane)
    uint32_t lc[4];
#pragma unroll
    for (uint32_t t = 0; t < 4; t++)
        lc[t] = LAYOUT == LAYOUT_T1X64 ? (lane << 2) : ((lane & 31u) << 2) | ((t & 1u) << 7) | ((t >> 1) << 8);
    uint32_t w[4];
#pragma unroll
    for (uint32_t c = 0; c < 4; c++)
        w[c] = (lane + 64u * c + 1u) * 0x9E3779B1u ^ blockIdx.x;
    uint32_t acc0 = lane, acc1 = 0u;
    const uint64_t c0 = __builtin_amdgcn_s_memtime();
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t r = 0; r < rounds; r++) {
        uint32_t v[kGatherReads];
#pragma unroll
        for (uint32_t c = 0; c < 4; c++) {
            w[c] += 0x3B5D7F91u + c;
            // address = table bit 1 << 16 | byte K of the word << 8 | copy and table bit 0
            v[4 * c + 0] = *reinterpret_cast<const uint32_t *>(bytes + __builtin_amdgcn_perm(w[c], lc[0], 0x0C010400u));
            v[4 * c + 1] = *reinterpret_cast<const uint32_t *>(bytes + __builtin_amdgcn_perm(w[c], lc[1], 0x0C010500u));
            v[4 * c + 2] = *reinterpret_cast<const uint32_t *>(bytes + __builtin_amdgcn_perm(w[c], lc[2], 0x0C010600u));
            v[4 * c + 3] = *reinterpret_cast<const uint32_t *>(bytes + __builtin_amdgcn_perm(w[c], lc[3], 0x0C010700u));
        }
#pragma unroll
        for (uint32_t k = 0; k < kGatherReads; k += 4) {
            acc0 = xor3(acc0, v[k], v[k + 1]);
            acc1 = xor3(acc1, v[k + 2], v[k + 3]);
        }
    }
    const uint64_t c1 = __builtin_amdgcn_s_memtime();
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    // fold the accumulator over the wave so one lane can write the wave's record
    uint32_t x = acc0 ^ acc1;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        x ^= __shfl_xor(x, s);
    if (lane == 0) {
        const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
        LdsGatherStat st;
        st.cycles = c1 - c0;
        st.ticks = t1 - t0;
        st.fold = x;
        st.pad = 0;
        out[wave] = st;
    }
}

}  // namespace

uint32_t lds_gather_reads_per_round() { return kGatherReads; }

int lds_gather_groups_per_cu(int layout) {
    int n = 0;
    const void *fn = layout == LAYOUT_T1X64 ? reinterpret_cast<const void *>(lds_gather_kernel<LAYOUT_T1X64>)
                                            : reinterpret_cast<const void *>(lds_gather_kernel<LAYOUT_T4X32>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 1024, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

hipError_t launch_lds_gather(LdsGatherStat *out, uint32_t rounds, int layout, int grid, hipStream_t stream) {
    if (layout == LAYOUT_T1X64)
        hipLaunchKernelGGL(lds_gather_kernel<LAYOUT_T1X64>, dim3(grid), dim3(1024), 0, stream, out, rounds);
    else
        hipLaunchKernelGGL(lds_gather_kernel<LAYOUT_T4X32>, dim3(grid), dim3(1024), 0, stream, out, rounds);
    return hipGetLastError();
}

}  // namespace aesgpu
