// Verification kernel: exact verification (Section 3.2) of the start
// positions a filter kernel deferred to a device buffer. The filter kernels
// keep only a few waves per compute unit for their own candidates, and a
// verification is a chain of dependent loads (text words, then the probe
// table, then the pattern words), so plans that pass many windows verify here
// instead, with every wave of a full-occupancy grid in flight.
#include <hip/hip_runtime.h>

#include "mag_internal.hpp"
#include "scan_common.hpp"
#include "verify.hpp"

namespace mag {
namespace {

constexpr int kVerifyThreads = 256;
constexpr uint32_t kVerifyFound = 256;   // found keys buffered per wave

// The waves are spread evenly over the buffer's segments; each takes 64
// consecutive starts of its segment per step, one per lane. Loop bounds are
// wave-uniform, so every lane reaches the collective output reservation.
// Found keys collect in a per-wave LDS buffer (patterns of equal length).
// The finishing kernel clears the segment counters afterwards.
__global__ __launch_bounds__(kVerifyThreads) void k_verify(VerifyArgs a) {
    __shared__ uint64_t s_found[(kVerifyThreads / 64) * kVerifyFound];
    __shared__ uint64_t s_wg[3 * (kVerifyThreads / 64)];
    uint64_t *fbuf = s_found + (threadIdx.x >> 6) * kVerifyFound;
    uint32_t fbn = 0;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * kVerifyThreads + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * kVerifyThreads) >> 6;
    const uint64_t per = waves >= kPendingSegments ? waves / kPendingSegments : 1;   // waves per segment
    for (uint64_t w = wave; w < per * kPendingSegments; w += waves) {
        const uint32_t seg = (uint32_t)(w % kPendingSegments);
        const uint64_t sub = w / kPendingSegments;
        const uint64_t count = a.seg_count[seg];
        const uint64_t total = count < a.seg_cap ? count : a.seg_cap;
        const uint64_t *src = a.pending + (uint64_t)seg * a.seg_cap;
        for (uint64_t c = sub * 64; c < total; c += per * 64) {
            const uint64_t i = c + lane;
            const bool active = i < total;
            const uint64_t i0 = active ? src[i] : 0ull;
            if (a.var) verify_wave(a, i0, active);
            else fbn = emit_found_buffered(a, i0, active ? find_pattern(a, i0) : 0u, fbuf, fbn, kVerifyFound);
        }
    }
    // the kernel's only argument is `a`, at the start of the argument segment
    const VerifyArgs *va = (const VerifyArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    dev::workgroup_out<kVerifyThreads / 64>(va, fbuf, fbn, 0, 0, nullptr, s_wg);
}

}  // namespace

mag_status launch_verify(const VerifyArgs &v, hipStream_t stream) {
    static int grid = 0;
    if (!grid) {
        int dev = 0, ncu = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_verify, kVerifyThreads, 0);
        if (e != hipSuccess) return hip_fail(e, "occupancy query (verify)");
        if (ncu < 1 || occ < 1) return fail(MAG_E_UNSUPPORTED, "verification kernel does not fit");
        grid = ncu * occ;
    }
    hipLaunchKernelGGL(k_verify, dim3((uint32_t)grid), dim3(kVerifyThreads), 0, stream, v);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "verification launch");
    return MAG_OK;
}

}  // namespace mag
