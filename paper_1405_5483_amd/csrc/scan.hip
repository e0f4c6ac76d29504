// MAG scan kernel for gfx950: the sampled Shift-Or filter over superimposed
// q-gram classes (Sections 3.1-3.2) with fused exact verification.
//
// Work decomposition. Sample x is the text q-gram at byte x*k*q. A workgroup
// owns a tile of consecutive samples; each lane owns S consecutive samples of
// the tile and warms its state up on the m'-1 samples before them, so every
// window (x, j) is evaluated by exactly one lane. Window (x, j) stands for the
// q start positions i0 = (x-m'+1)kq - jq - s (s < q); every start position
// maps to exactly one (x, j, s), so each position is verified at most once and
// no de-duplication is needed.
//
// Per tile: the text bytes the tile reads (samples, warm-up and every
// verification window) are staged into LDS with 128-bit buffer loads
// (range-checked, so any text alignment is fine); the alphabet map and, when it
// fits, the mask table live in LDS for the whole kernel. Candidate windows are
// compacted per wavefront with a ballot + mbcnt prefix into an LDS queue and
// verified 64 at a time, one per lane: a hash of the window's first 16 bytes
// probes an open-addressing table of the distinct patterns, a fingerprint hit
// is confirmed by a full word compare, and every id of the matching pattern is
// emitted as a 64-bit key (pos << idbits | id).
#include <hip/hip_runtime.h>

#include "mag_internal.hpp"

namespace mag {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kQueue = 128;          // per-wave candidate queue entries
constexpr uint32_t kBufferWord3 = 0x00020000u;   // raw 32-bit buffer resource (gfx9)

struct ScanArgs {
    const uint8_t *tbase;      // text pointer rounded down to 16 bytes
    uint64_t delta;            // text - tbase
    uint64_t n, X, ntiles;
    uint32_t q, k, kq, mprime, W, sp, m, mw, hw;
    uint32_t S, tile_samples, tile_lds, table_vec;
    uint32_t slot_shift, slot_mask, idbits, lastmask;
    const uint8_t *mu;
    const void *table;
    const uint64_t *slots;
    const uint32_t *pwords, *idstart, *ids;
    uint64_t *keys;
    uint64_t cap;
    uint64_t *counters;
};

__device__ __forceinline__ uint32_t lds_word(const uint32_t *s32, uint32_t o) {
    const uint32_t lo = s32[o >> 2];
    const uint32_t hi = s32[(o >> 2) + 1];
    return __builtin_amdgcn_alignbyte(hi, lo, o & 3);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Verifies start position i0 (0 <= i0 <= n-m) whose bytes are staged in LDS at
// offset o, and emits every (i0, id) occurrence.
__device__ void verify_start(const ScanArgs &a, const uint32_t *s32, uint32_t o, uint64_t i0) {
    uint32_t hv[kHashWords];
#pragma unroll
    for (int t = 0; t < kHashWords; ++t) {
        uint32_t w = 0;
        if (t < (int)a.hw) {
            w = lds_word(s32, o + 4 * t);
            if (t == (int)a.mw - 1) w &= a.lastmask;
        }
        hv[t] = w;
    }
    const uint32_t h = window_hash(hv, (int)a.hw);
    uint32_t slot = h >> a.slot_shift;
    for (;;) {
        const uint64_t e = a.slots[slot];
        if (e == 0) return;
        if ((uint32_t)(e >> 32) == h) {
            const uint32_t u = (uint32_t)e - 1u;
            const uint32_t *pw = a.pwords + (size_t)u * a.mw;
            bool eq = true;
            for (uint32_t t = 0; t < a.mw; ++t) {
                uint32_t w = lds_word(s32, o + 4 * t);
                if (t == a.mw - 1) w &= a.lastmask;
                if (w != pw[t]) { eq = false; break; }
            }
            if (eq) {
                const uint32_t b = a.idstart[u], c = a.idstart[u + 1] - b;
                const uint64_t base = atomicAdd((unsigned long long *)&a.counters[0],
                                                (unsigned long long)c);
                for (uint32_t t = 0; t < c; ++t)
                    if (base + t < a.cap)
                        a.keys[base + t] = (i0 << a.idbits) | (uint64_t)a.ids[b + t];
                return;     // distinct patterns: at most one can be equal
            }
        }
        slot = (slot + 1) & a.slot_mask;
    }
}

// All q start positions of window (x, j).
__device__ __forceinline__ uint32_t verify_window(const ScanArgs &a, const uint32_t *s32,
                                                  int64_t obase, int64_t x, uint32_t j) {
    uint32_t nv = 0;
    const int64_t top = (x - (int64_t)a.mprime + 1) * a.kq - (int64_t)j * a.q;
    const int64_t last = (int64_t)a.n - (int64_t)a.m;
    for (uint32_t s = 0; s < a.q; ++s) {
        const int64_t i0 = top - s;
        if (i0 < 0 || i0 > last) continue;
        ++nv;
        verify_start(a, s32, (uint32_t)(obase + i0), (uint64_t)i0);
    }
    return nv;
}

template <typename DT, typename ET, bool TLDS>
__global__ __launch_bounds__(kThreads) void k_scan(ScanArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t *s_mu = smem;
    uint32_t *s_queue = reinterpret_cast<uint32_t *>(smem + 256);
    uint8_t *s_text = smem + 256 + kWaves * kQueue * 4;
    ET *s_tab = reinterpret_cast<ET *>(s_text + a.tile_lds);
    const uint32_t *s32 = reinterpret_cast<const uint32_t *>(s_text);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s_mu[tid] = a.mu[tid];
    if (TLDS) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.table);
        uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
        for (uint32_t v = tid; v < a.table_vec; v += kThreads) dst[v] = src[v];
    }
    const ET *g_tab = reinterpret_cast<const ET *>(a.table);

    uint32_t *queue = s_queue + wave * kQueue;
    uint32_t qn = 0;
    uint64_t ncand = 0, nver = 0;
    const uint32_t kmask = a.k >= 32 ? 0xFFFFFFFFu : ((1u << a.k) - 1u);
    const uint32_t topshift = a.W - a.k;
    const uint32_t sp = a.sp, q = a.q;

    for (uint64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const int64_t X0 = (int64_t)tile * a.tile_samples;
        int64_t b0 = (X0 - (int64_t)a.mprime) * a.kq + 1;
        if (b0 < 0) b0 = 0;
        int64_t b1 = (X0 + (int64_t)a.tile_samples - (int64_t)a.mprime) * a.kq + a.m;
        if (b1 > (int64_t)a.n) b1 = (int64_t)a.n;
        if (b1 < b0) b1 = b0;
        const uint64_t pa0 = (a.delta + (uint64_t)b0) & ~15ull;
        const uint64_t pa1 = (a.delta + (uint64_t)b1 + 15) & ~15ull;
        const uint32_t nvec = (uint32_t)((pa1 - pa0) >> 4);
        __syncthreads();    // the previous tile is fully consumed
        {
            __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.tbase + pa0), (short)0, (int)(pa1 - pa0), (int)kBufferWord3);
            uint4 *dst = reinterpret_cast<uint4 *>(s_text);
            for (uint32_t v = tid; v < nvec; v += kThreads) {
                auto val = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(v * 16), 0, 0);
                dst[v] = make_uint4(val[0], val[1], val[2], val[3]);
            }
        }
        __syncthreads();

        const int64_t obase = (int64_t)a.delta - (int64_t)pa0;   // LDS offset of text byte 0
        const int64_t xs = X0 + (int64_t)tid * a.S;
        DT D = ~(DT)0;
        for (int i = -(int)(a.mprime - 1); i < (int)a.S; ++i) {
            const int64_t x = xs + i;
            const bool valid = x >= 0 && x < (int64_t)a.X;
            uint32_t c = 0;
            if (valid) {
                const uint32_t o = (uint32_t)(obase + x * (int64_t)a.kq);
                const uint32_t lo = lds_word(s32, o);
                const uint32_t hi = q > 4 ? lds_word(s32, o + 4) : 0u;
                uint32_t g = 0;
#pragma unroll
                for (int t = kMaxQ - 1; t >= 0; --t) {
                    if (t < (int)q) {
                        const uint32_t byte = (t < 4 ? (lo >> (8 * t)) : (hi >> (8 * (t - 4)))) & 0xFFu;
                        g = g * sp + s_mu[byte];
                    }
                }
                const ET e = TLDS ? s_tab[g] : g_tab[g];
                D = (D << a.k) | (DT)e;
                if (i >= 0) c = (uint32_t)((~D) >> topshift) & kmask;
            }
            uint64_t any = __ballot(c != 0);
            while (any) {
                const bool has = c != 0;
                if (has) {
                    const uint32_t j = __builtin_ctz(c);
                    c &= c - 1u;
                    queue[qn + lanes_below(any)] = ((uint32_t)(x - X0) << 5) | j;
                }
                const uint32_t cnt = (uint32_t)__popcll(any);
                qn += cnt;
                ncand += cnt;
                if (qn >= 64) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    const uint32_t e = queue[qn - 64 + lane];
                    __builtin_amdgcn_wave_barrier();
                    qn -= 64;
                    nver += verify_window(a, s32, obase, X0 + (int64_t)(e >> 5), e & 31u);
                }
                any = __ballot(c != 0);
            }
        }
        if (qn) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if ((uint32_t)lane < qn) {
                const uint32_t e = queue[lane];
                nver += verify_window(a, s32, obase, X0 + (int64_t)(e >> 5), e & 31u);
            }
            __builtin_amdgcn_wave_barrier();
            qn = 0;
        }
    }
    if (lane == 0 && ncand) atomicAdd((unsigned long long *)&a.counters[1], (unsigned long long)ncand);
    // wave sum of verifications
    unsigned long long nv = nver;
    for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off);
    nver = nv;
    if (lane == 0 && nver) atomicAdd((unsigned long long *)&a.counters[2], (unsigned long long)nver);
}

template <typename DT, typename ET, bool TLDS>
mag_status launch_one(const ScanArgs &a, size_t shmem, hipStream_t stream) {
    auto fn = k_scan<DT, ET, TLDS>;
    static int configured_bytes = 0;    // per instantiation
    if ((int)shmem > configured_bytes) {
        // not every runtime needs the opt-in; a real LDS overflow fails the launch below
        (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shmem);
        (void)hipGetLastError();
        configured_bytes = (int)shmem;
    }
    int dev = 0, ncu = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kThreads, shmem);
    if (e != hipSuccess) return hip_fail(e, "occupancy query (scan)");
    if (occ < 1) return fail(MAG_E_UNSUPPORTED, "scan kernel does not fit on a compute unit");
    uint64_t grid = (uint64_t)ncu * (uint64_t)occ;
    if (grid > a.ntiles) grid = a.ntiles;
    if (grid == 0) return MAG_OK;
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kThreads), shmem, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "scan launch");
    return MAG_OK;
}

uint32_t pick_samples_per_lane(uint32_t kq, uint32_t mprime) {
    // enough samples per lane to amortise the m'-1 warm-up steps, a tile of
    // roughly 8-32 KiB, and a lane stride (S*kq bytes) that is an odd number of
    // 32-bit words when possible so lanes hit distinct LDS banks
    uint32_t S = 64 / kq;
    S = S < 8 ? 8 : S;
    const uint32_t warm = 4 * (mprime > 0 ? mprime - 1 : 0);
    if (S < warm) S = warm;
    while ((uint64_t)kThreads * S * kq > 32768 && S > 4) --S;
    for (uint32_t c = S; c < S + 8; ++c)
        if (((uint64_t)c * kq) % 8 == 4 && (uint64_t)kThreads * c * kq <= 32768) return c;
    return S;
}

}  // namespace

mag_status launch_scan(const mag_plan *p, const ScanLaunch &s, hipStream_t stream) {
    if (s.n < p->q || p->r == 0) return MAG_OK;
    ScanArgs a{};
    const uintptr_t t = reinterpret_cast<uintptr_t>(s.text);
    a.tbase = reinterpret_cast<const uint8_t *>(t & ~(uintptr_t)15);
    a.delta = t & 15;
    a.n = s.n;
    a.q = p->q;
    a.k = p->k;
    a.kq = p->k * p->q;
    a.mprime = p->mprime;
    a.W = p->W;
    a.sp = p->sigma_prime;
    a.m = p->m;
    a.mw = p->mw;
    a.hw = p->mw < (uint32_t)kHashWords ? p->mw : (uint32_t)kHashWords;
    a.X = (s.n - p->q) / a.kq + 1;
    a.S = pick_samples_per_lane(a.kq, a.mprime);
    a.tile_samples = kThreads * a.S;
    a.ntiles = (a.X + a.tile_samples - 1) / a.tile_samples;
    // staged bytes: at most tile_samples*kq + m - 1 plus 30 bytes of 16-byte
    // alignment; word reads run up to 7 bytes past the last staged byte
    a.tile_lds = (uint32_t)(((uint64_t)a.tile_samples * a.kq + a.m + 64) & ~15ull);
    a.slot_shift = 32 - p->slot_bits;
    a.slot_mask = (uint32_t)((1ull << p->slot_bits) - 1);
    a.idbits = (uint32_t)s.idbits;
    a.lastmask = (p->m & 3) ? ((1u << (8 * (p->m & 3))) - 1u) : 0xFFFFFFFFu;
    a.mu = p->dev.mu;
    a.table = p->dev.table;
    a.slots = p->dev.slots;
    a.pwords = p->dev.pwords;
    a.idstart = p->dev.idstart;
    a.ids = p->dev.ids;
    a.keys = s.keys;
    a.cap = s.cap;
    a.counters = s.counters;

    const uint64_t tbytes = p->table.size();
    const bool tlds = tbytes <= 64 * 1024;
    a.table_vec = (uint32_t)((tbytes + 15) / 16);
    const size_t shmem = 256 + (size_t)kWaves * kQueue * 4 + a.tile_lds +
                         (tlds ? (size_t)a.table_vec * 16 : 0);
    const bool wide = p->W > 32 || p->k >= 32;
    switch (p->esz) {
        case 1:
            if (wide) return tlds ? launch_one<uint64_t, uint8_t, true>(a, shmem, stream)
                                  : launch_one<uint64_t, uint8_t, false>(a, shmem, stream);
            return tlds ? launch_one<uint32_t, uint8_t, true>(a, shmem, stream)
                        : launch_one<uint32_t, uint8_t, false>(a, shmem, stream);
        case 2:
            return tlds ? launch_one<uint32_t, uint16_t, true>(a, shmem, stream)
                        : launch_one<uint32_t, uint16_t, false>(a, shmem, stream);
        case 4:
            if (wide) return tlds ? launch_one<uint64_t, uint32_t, true>(a, shmem, stream)
                                  : launch_one<uint64_t, uint32_t, false>(a, shmem, stream);
            return tlds ? launch_one<uint32_t, uint32_t, true>(a, shmem, stream)
                        : launch_one<uint32_t, uint32_t, false>(a, shmem, stream);
        default:
            return tlds ? launch_one<uint64_t, uint64_t, true>(a, shmem, stream)
                        : launch_one<uint64_t, uint64_t, false>(a, shmem, stream);
    }
}

}  // namespace mag
