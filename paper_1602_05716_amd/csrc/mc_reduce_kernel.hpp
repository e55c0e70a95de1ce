// mc_reduce_kernel.hpp -- the per-move parallel-reduction scheme, the GPU
// comparison code of the paper's benchmark (Liang, Xing, Li,
// arXiv:1602.05716, Sec. 4), written for gfx950.
//
// One launch per trial move.  Thread j of the grid evaluates the pair term of
// partner j with the mover (the mover's own thread idles); each workgroup
// reduces its terms (wavefront butterfly, then its four waves through LDS)
// into one partial; the last workgroup to arrive -- a device-wide arrival
// counter -- sums every partial in workgroup order, takes the decision and
// updates the chain.  The scheme reads the whole state once per move and
// pays a launch per move: it is the baseline that the sequential-sweep
// kernel is measured against, not a production path.
//
// It works on the sweep kernel's chain state and leaves it as that kernel
// would: the position of trial (s, i) goes to slot pos[s & 1][i] tagged with
// the sweep index, the group records carry each group's accept mask, the
// padding ions are carried forward at the end of every sweep, and the trace,
// counters and per-group energy changes are filled in the same way.  The two
// schemes can therefore take turns on one chain.
#pragma once

#include "mc_sweep_kernel.hpp"

namespace mcdev {

constexpr int kReduceThreads = 256;  // threads per workgroup of the per-move launch

// Partial of one workgroup for one move, one 16-byte agent-coherent record;
// the tag (move serial + 1) tells the deciding workgroup that it is current.
struct ReducePart {
    double s;      // sum of the workgroup's pair terms
    uint32_t ov;   // nonzero: a partner overlaps the trial position
    uint32_t tag;
};

// State that lives across the launches of one mc_sweep_reduction call.
struct ReduceCtl {
    unsigned int arrived;  // workgroups of the current move done with their partial
    unsigned int pad;
    uint64_t gmask;        // accept bits of the current group so far
    double gde;            // sum of the accepted energy changes of the current group so far
};

__device__ __forceinline__ void raise_state(const Ctl& ctl) {
    int expected = 0;
    __hip_atomic_compare_exchange_strong(ctl.abort, &expected, -8 /* MC_E_STATE */, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Position of ion idx from the image of the given parity, which must carry
// version ver (the launches before this one wrote it).
template <typename T>
__device__ __forceinline__ typename PosIO<T>::Rec load_pos(__amdgpu_buffer_rsrc_t r, uint32_t idx);
template <>
__device__ __forceinline__ PosIO<float>::Rec load_pos<float>(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
    return PosIO<float>::load(r, idx);
}
template <>
__device__ __forceinline__ PosIO<double>::Rec load_pos<double>(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
    const PosIO<double>::Hi h = PosIO<double>::load_hi(r, idx);
    const PosIO<double>::Lo l = PosIO<double>::load_lo(r, idx);
    return PosIO<double>::Rec{l.x, l.y, h.z, h.ver, 0u};
}

// Sum over the workgroup in a fixed order: butterfly inside each wave, then
// the waves' sums in wave order.  Every thread gets the result.
__device__ __forceinline__ double block_sum(double v, bool ov, bool* ov_out, double* lds_s, uint32_t* lds_ov) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int W = kReduceThreads / 64;
    v = wave_sum(v);
    const uint64_t b = __ballot(ov);
    __syncthreads();  // a previous call's reads of the LDS slots are done
    if (lane == 0) {
        lds_s[wave] = v;
        lds_ov[wave] = b != 0ull ? 1u : 0u;
    }
    __syncthreads();
    double s = 0.0;
    uint32_t o = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        s += lds_s[w];
        o |= lds_ov[w];
    }
    *ov_out = o != 0;
    return s;
}

// Trial move (s, ion) of the chain.  Grid: ceil(npad / 256) workgroups of
// 256 threads.  s0: first sweep of the current launch sequence (indexes the
// per-group energy changes).
template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
reduce_move_kernel(const ChainDesc* __restrict__ chains, ReducePart* __restrict__ parts, ReduceCtl* rctl,
                   uint32_t s, int32_t ion, uint32_t s0, Ctl ctl)
{
    using IO = PosIO<T>;
    __shared__ double lds_s[kReduceThreads / 64];
    __shared__ uint32_t lds_ov[kReduceThreads / 64];
    __shared__ int lds_last;
    const ChainDesc& cd = chains[0];
    const int n = cd.n, npad = cd.npad, nb = cd.nb;
    const uint32_t nblk = gridDim.x;
    const __amdgpu_buffer_rsrc_t pos_r = make_rsrc(cd.pos, (uint32_t)(2u * npad * IO::kBytes));
    const __amdgpu_buffer_rsrc_t part_r = make_rsrc(parts, (uint32_t)(nblk * sizeof(ReducePart)));
    const T* __restrict__ charge = (const T*)cd.charge;
    const T* __restrict__ half = (const T*)cd.half;
    const uint32_t cur = s & 1u, prev = (s - 1u) & 1u;
    const uint32_t tag = (uint32_t)((uint64_t)s * (uint64_t)n + (uint64_t)ion) + 1u;

    // the mover: old position (result of its trial in sweep s - 1) and the
    // trial position of Algorithm 1
    const auto xr = load_pos<T>(pos_r, prev * npad + ion);
    const T xi = xr.x, yi = xr.y, zi = xr.z, qi = charge[ion], hi = half[ion];
    const T D = (T)cd.D;
    const uint4 wd = move_words(cd.seed, cd.chain_id, s, (uint32_t)ion);
    const T txi = trial_coord(xi, wd.x, D), tyi = trial_coord(yi, wd.y, D), tzi = trial_coord(zi, wd.z, D);

    // partner j: final position for j < ion (this sweep), previous one for j > ion
    const int j = blockIdx.x * kReduceThreads + threadIdx.x;
    double term = 0.0;
    bool ov = false;
    bool stale = xr.ver != s - 1u;
    if (j < npad && j != ion) {
        const uint32_t par = j < ion ? cur : prev, want = j < ion ? s : s - 1u;
        const auto pr = load_pos<T>(pos_r, par * npad + j);
        stale |= pr.ver != want;
        const T qj = charge[j], hj = half[j];
        const T d2o = Prec<T>::norm2(pr.x - xi, pr.y - yi, pr.z - zi);
        const T d2t = Prec<T>::norm2(pr.x - txi, pr.y - tyi, pr.z - tzi);
        term = (double)(qj * (Prec<T>::rinv(d2t) - Prec<T>::rinv(d2o)));
        const T s_ij = hi + hj;
        ov = d2t < s_ij * s_ij;
    }
    if (__ballot(stale) != 0ull && (threadIdx.x & 63) == 0) raise_state(ctl);

    bool bov = false;
    const double bs = block_sum(term, ov, &bov, lds_s, lds_ov);
    if (threadIdx.x == 0) {
        const ReducePart p{bs, bov ? 1u : 0u, tag};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, p), part_r, blockIdx.x * 16u, 0, kCoherent);
        drain_memory();  // the partial is out before the arrival is counted
        const unsigned int before =
            __hip_atomic_fetch_add(&rctl->arrived, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lds_last = before == nblk - 1u ? 1 : 0;
    }
    __syncthreads();
    if (!lds_last) return;

    // ---- the last workgroup: every partial, in workgroup order
    double acc = 0.0;
    bool aov = false;
    for (uint32_t b = threadIdx.x; b < nblk; b += kReduceThreads) {
        ReducePart p = __builtin_bit_cast(ReducePart, __builtin_amdgcn_raw_buffer_load_b128(part_r, b * 16u, 0, kCoherent));
        if (p.tag != tag) {
            PollGuard pg;
            while (p.tag != tag && !pg.stop(ctl)) {
                __builtin_amdgcn_s_sleep(1);
                p = __builtin_bit_cast(ReducePart, __builtin_amdgcn_raw_buffer_load_b128(part_r, b * 16u, 0, kCoherent));
            }
        }
        acc += p.s;
        aov |= p.ov != 0u;
    }
    bool tov = false;
    const double S = block_sum(acc, aov, &tov, lds_s, lds_ov);

    const int b = ion / kGroup, lane = ion % kGroup;
    if (threadIdx.x == 0) {
        // hard wall (Sec. 5.2), overlap (Sec. 3.3), Metropolis test
        const double a = cd.wall_a[ion];
        const double X = (double)txi, Y = (double)tyi, Z = (double)tzi;
        const bool wall = X * X + Y * Y + Z * Z > a * a;
        const double thr = -log(accept_uniform(wd.w));
        const double dE = cd.lB * (double)qi * S;
        const bool dec = !wall && !tov && (dE <= 0.0 || dE < thr);
        __hip_atomic_store(&rctl->arrived, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (dec)
            IO::store(pos_r, cur * npad + ion, txi, tyi, tzi, s);
        else
            IO::store(pos_r, cur * npad + ion, xi, yi, zi, s);
        const int64_t mv = (int64_t)s * n + ion;
        if (mv < cd.trace_cap) {
            cd.trace_acc[mv] = (uint8_t)dec;
            cd.trace_de[mv] = dE;
        }
        unsigned long long* st = cd.stats;
        st[0] += 1ull;
        st[1] += dec ? 1ull : 0ull;
        st[2] += wall ? 1ull : 0ull;
        st[3] += (!wall && tov) ? 1ull : 0ull;
        st[4] += (!wall && !tov && !dec) ? 1ull : 0ull;
        uint64_t gm = lane == 0 ? 0ull : rctl->gmask;
        double gde = lane == 0 ? 0.0 : rctl->gde;
        gm |= (uint64_t)dec << lane;
        gde += dec ? dE : 0.0;
        rctl->gmask = gm;
        rctl->gde = gde;
        if (lane == kGroup - 1 || ion == n - 1) {
            // the group is decided (padding lanes never accept)
            const int64_t g = (int64_t)s * nb + b;
            const __amdgpu_buffer_rsrc_t rec_r = make_rsrc(cd.rec, (uint32_t)(kRing * sizeof(GroupRec)));
            store_rec(rec_r, (uint32_t)(g & (kRing - 1)), GroupRec{(uint32_t)(g + 1), 0u, gm});
            cd.de_group[(int64_t)(s - s0) * nb + b] = gde;
        }
    }
    if (ion == n - 1) {
        // end of the sweep: the padding ions keep their positions
        const int k = n + (int)threadIdx.x;
        if (k < npad) {
            const auto pr = load_pos<T>(pos_r, prev * npad + k);
            IO::store(pos_r, cur * npad + k, pr.x, pr.y, pr.z, s);
        }
    }
}

}  // namespace mcdev
