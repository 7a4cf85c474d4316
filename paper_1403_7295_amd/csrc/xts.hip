// XTS-AES (IEEE 1619; NIST SP 800-38E) for gfx950 over a buffer of data
// units (sectors), unit u with tweak value first_unit + u.  Each wave takes
// groups of 64 consecutive units (xts_core.h does one group).
#include <hip/hip_runtime.h>

#include <cstddef>

#include "cipher_core.h"
#include "internal.h"
#include "xts_core.h"

namespace aesgpu {
namespace {

// The tweak key's schedule where the kernel's argument (an XtsArgs, the
// only one, at the start of the argument segment) holds it.
__device__ __forceinline__ const uint32_t *kernarg_rk2() {
    const char *seg = (const char *)__builtin_amdgcn_kernarg_segment_ptr();
    return reinterpret_cast<const uint32_t *>(seg + offsetof(XtsArgs, rk2));
}

template <int NR, int DIR, int BPT>
__global__ __launch_bounds__(1024) void xts_kernel(const XtsArgs a) {
    __shared__ uint32_t lds[lds_words<DIR>()];
    // the tweak key's schedule (encryption; decryption's tables fill the LDS)
    __shared__ uint32_t tkey[DIR == DIR_ENC ? 4 * (NR + 1) : 1];
    stage_tables<LAYOUT_T4X32, DIR>(lds);
    if (DIR == DIR_ENC && threadIdx.x < uint32_t(4 * (NR + 1)))
        tkey[threadIdx.x] = a.rk2[threadIdx.x];
    __syncthreads();
    const LaneConsts lc = lane_consts<LAYOUT_T4X32>(threadIdx.x & 63u);
    const uint64_t nblk = a.nbytes >> 4;
    const uint32_t ushift = a.unit_shift;                 // log2(blocks per unit), 0..8
    const uint64_t nunits = (nblk + (uint64_t(1) << ushift) - 1) >> ushift;
    const uint64_t ngroups = (nunits + 63) >> 6;
    const uint64_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint64_t nwaves = uint64_t(gridDim.x) * (blockDim.x >> 6);
    for (uint64_t g = wave; g < ngroups; g += nwaves) {
        const uint64_t gb0 = (64 * g) << ushift;           // first block of the group
        const uint64_t gb1 = min(nblk, (64 * (g + 1)) << ushift);
        // the tweak key is read where the group uses it, from LDS (encryption)
        // or the kernel arguments (decryption), through a pointer the
        // compiler cannot see through, so that it does not hoist the reads:
        // held in scalar registers for the whole kernel beside the data key,
        // it made the compiler spill data-key words that the rounds then
        // read back one by one
        const uint32_t *rk2 = DIR == DIR_ENC ? tkey : kernarg_rk2();
        asm volatile("" : "+s"(rk2));
        xts_group<NR, DIR, BPT>(lds, lc, a.rk1, rk2, a.in, a.out, gb0, gb1, a.first_unit + 64 * g, ushift);
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
