// mc_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// precision traits, the Philox4x32-10 generator, the trial-move formulas and
// the device-wide wait / publish primitives.
//
// Paper: Liang, Xing, Li, arXiv:1602.05716.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcdev {

constexpr int kGroup = 64;   // movers per group = lanes of one wavefront
constexpr int kRing = 1024;  // group records kept per chain
constexpr int kMaxBand = 4;  // largest look-ahead band, in groups
constexpr int kDaMaxBand = 3;  // ... of chains on the delayed-acceptance kernel
constexpr int kMaxBandPerIon = 3;  // ... of float chains with per-ion diameters
constexpr int kMaxBandWide = 3;    // ... of float chains on eight waves per workgroup
constexpr int kMaxBandWidePerIon = 2;  // ... and per-ion diameters

// Per-group record published by the workgroup that decided the group; one
// 16-byte transaction, so the tag and the accept mask are read together.
struct GroupRec {
    uint32_t tag;    // (stream index + 1) mod 2^32 of the group held in this slot
    uint32_t spare;
    uint64_t acc;    // accept mask of the group's 64 trials
};

// Status words shared by every workgroup of a launch.
struct Ctl {
    int* abort;              // set to a nonzero mc_status on a fatal device condition
    uint64_t timeout_ticks;  // limit of one wait, in wall_clock64() ticks
};

// --------------------------------------------------------------------------
// Precision traits.  The float path keeps positions in float4 {x, y, z, q}
// (the paper's X_dev layout, Sec. 3.1) and evaluates pair terms with the
// hardware reciprocal square root; the double path uses correctly rounded
// sqrt and division so that every pair term equals the textbook value.
// --------------------------------------------------------------------------
template <typename T> struct Prec;

template <> struct Prec<float> {
    using T4 = float4;
    static __device__ __forceinline__ float rinv(float d2) { return __builtin_amdgcn_rsqf(d2); }
    // d2 = dx^2 + dy^2 + dz^2 with fused multiply-adds
    static __device__ __forceinline__ float norm2(float dx, float dy, float dz) {
        return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    }
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    // operands are never NaN here: one v_min instruction
    static __device__ __forceinline__ float min(float a, float b) { return __builtin_fminf(a, b); }
    // fused multiply-add where the product is exact (a multiplier of 0 or 1)
    static __device__ __forceinline__ float fma_exact(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

template <> struct Prec<double> {
    using T4 = double4;
    static __device__ __forceinline__ double rinv(double d2) { return 1.0 / __builtin_sqrt(d2); }
    // left-to-right sum of three rounded squares, no fused multiply-add
    static __device__ __forceinline__ double norm2(double dx, double dy, double dz) {
        return dx * dx + dy * dy + dz * dz;
    }
    // the double path keeps the textbook rounding: product, then sum
    static __device__ __forceinline__ double fma(double a, double b, double c) { return a * b + c; }
    static __device__ __forceinline__ double min(double a, double b) { return __builtin_fmin(a, b); }
    // fused multiply-add where the product is exact (a multiplier of 0 or 1):
    // the same result as the separately rounded form
    static __device__ __forceinline__ double fma_exact(double a, double b, double c) { return __builtin_fma(a, b, c); }
};

template <typename T>
__device__ __forceinline__ typename Prec<T>::T4 mk4(T x, T y, T z, T w) {
    typename Prec<T>::T4 v;
    v.x = x; v.y = y; v.z = z; v.w = w;
    return v;
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products; the key is bumped by the Weyl constants between
// rounds.  One block per trial move: counter (i, sweep, chain, tag), key
// (seed low word, seed high word).
// --------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a0 = 0xD2511F53u * c.x, h0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t a1 = 0xCD9E8D57u * c.z, h1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(h1 ^ c.y ^ k0, a1, h0 ^ c.w ^ k1, a0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint4 move_words(uint64_t seed, uint32_t chain, uint32_t sweep,
                                            uint32_t ion, uint32_t tag = 0u) {
    return philox4x32_10(make_uint4(ion, sweep, chain, tag), (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Trial coordinate x + D (u - 1/2) (Sec. 3.2, Algorithm 1), every step rounded
// in the working precision (build with contraction off).
__device__ __forceinline__ float trial_coord(float x, uint32_t w, float D) {
    float u = (float)(w >> 8) * 0x1p-24f;
    float t = u - 0.5f;
    t = D * t;
    return x + t;
}
__device__ __forceinline__ double trial_coord(double x, uint32_t w, double D) {
    double u = (double)w * 0x1p-32;
    double t = u - 0.5;
    t = D * t;
    return x + t;
}

__device__ __forceinline__ double accept_uniform(uint32_t w) { return (double)w * 0x1p-32; }

// --------------------------------------------------------------------------
// Device-wide communication without cache maintenance.  Everything one
// workgroup publishes for others (versioned positions, group records) is
// written and read with agent-coherent 16-byte accesses (the sc1 cache
// policy: coherent across the separate L2 caches of the 8 XCDs), so no L2
// write-back or invalidate is ever needed.  Every published record carries
// its own validity tag, so readers need no separate flag.
// --------------------------------------------------------------------------
constexpr int kCoherent = 16;  // buffer-instruction cache policy: sc1

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}

using u32x4 = __attribute__((ext_vector_type(4))) unsigned int;

__device__ __forceinline__ float4 coherent_load(__amdgpu_buffer_rsrc_t r, uint32_t idx, float4*) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 16u, 0, kCoherent));
}
__device__ __forceinline__ double4 coherent_load(__amdgpu_buffer_rsrc_t r, uint32_t idx, double4*) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, idx * 32u, 0, kCoherent);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, idx * 32u + 16u, 0, kCoherent);
    const double2 lo = __builtin_bit_cast(double2, a), hi = __builtin_bit_cast(double2, b);
    return make_double4(lo.x, lo.y, hi.x, hi.y);
}
__device__ __forceinline__ void coherent_store(__amdgpu_buffer_rsrc_t r, uint32_t idx, float4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, idx * 16u, 0, kCoherent);
}
__device__ __forceinline__ void coherent_store(__amdgpu_buffer_rsrc_t r, uint32_t idx, double4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, make_double2(v.x, v.y)), r,
                                           idx * 32u, 0, kCoherent);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, make_double2(v.z, v.w)), r,
                                           idx * 32u + 16u, 0, kCoherent);
}
__device__ __forceinline__ GroupRec load_rec(__amdgpu_buffer_rsrc_t r, uint32_t slot) {
    return __builtin_bit_cast(GroupRec, __builtin_amdgcn_raw_buffer_load_b128(r, slot * 16u, 0, kCoherent));
}
__device__ __forceinline__ void store_rec(__amdgpu_buffer_rsrc_t r, uint32_t slot, GroupRec v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, slot * 16u, 0, kCoherent);
}

// Compiler-level barrier: no memory access moves across it.
__device__ __forceinline__ void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// Waits until every memory access this wave has issued is complete.
__device__ __forceinline__ void drain_memory() {
    compiler_fence();
    __builtin_amdgcn_s_waitcnt(0);
    compiler_fence();
}

__device__ __forceinline__ bool abort_raised(const Ctl& ctl) {
    return __hip_atomic_load(ctl.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ __forceinline__ void raise_timeout(const Ctl& ctl) {
    int expected = 0;
    __hip_atomic_compare_exchange_strong(ctl.abort, &expected, -7 /* MC_E_TIMEOUT */, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bookkeeping of one bounded wait.  The clock is read on every poll; the
// abort flag -- a single word that every waiting wave of the launch would
// otherwise read on every poll -- on every 32nd only.
struct PollGuard {
    uint64_t t0;
    uint32_t k;
    __device__ __forceinline__ PollGuard() : t0(wall_clock64()), k(0) {}
    // true when the wait has to end: abort raised elsewhere, or time-out here
    __device__ __forceinline__ bool stop(const Ctl& ctl) {
        if ((++k & 31u) == 0u && abort_raised(ctl)) return true;
        if (wall_clock64() - t0 > ctl.timeout_ticks) {
            raise_timeout(ctl);
            return true;
        }
        return false;
    }
};

// Waits for the record of group gp and returns it.  A record only carries the
// group's accept mask (positions carry their own version tags).  Readers are
// at most a few groups behind the newest publication, far fewer than the
// ring holds; a slot found already reused raises MC_E_STATE.
__device__ __forceinline__ GroupRec wait_rec(__amdgpu_buffer_rsrc_t rr, int64_t gp, const Ctl& ctl) {
    const uint32_t slot = (uint32_t)(gp & (kRing - 1));
    const uint32_t want = (uint32_t)(gp + 1);
    PollGuard pg;
    for (;;) {
        const GroupRec r = load_rec(rr, slot);
        const int32_t ahead = (int32_t)(r.tag - want);
        if (ahead == 0) {
            compiler_fence();
            return r;
        }
        if (ahead > 0) {
            // the slot was reused before this reader got to it: report, never guess
            int expected = 0;
            __hip_atomic_compare_exchange_strong(ctl.abort, &expected, -8 /* MC_E_STATE */,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            return r;
        }
        if (pg.stop(ctl)) return r;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Orders this wave's LDS accesses for other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace mcdev
