// mc_sweep_kernel.hpp -- the persistent sequential-sweep kernel for gfx950.
//
// Method (Liang, Xing, Li, arXiv:1602.05716): sequential-update Metropolis
// Monte Carlo with the exact energy change of every trial (Sec. 2, Eq.
// (Delta E_ij)), hard-core overlap indicator (Sec. 3.3) and spherical hard
// wall (Sec. 5.2).  The kernel keeps the chain resident on the device for a
// whole mc_sweep call; there is no host round trip between trials.
//
// Decomposition (our own design for CDNA4; the paper's Sec. 3.2-3.7 scheme is
// prior art):
//   * Ions are cut into groups of 64 = one wavefront; group b of sweep s has
//     stream index g = s*B + b, and the trials form one sequence over g.
//   * Each target group g is served by one workgroup of M waves.  Lane i of
//     every wave is mover i of the group; wave w takes a 64/M-ion slice of
//     every partner group.  This is the paper's "brush" (Sec. 3.4) turned so
//     that the partner index is uniform across the wave.
//   * By Eq. (Delta E_ij) the term of partner j is final as soon as j's own
//     latest trial is decided.  Partner groups decided more than `band`
//     groups before g are summed directly with their published positions, in
//     stream order, as they get decided (this is the upper/lower triangle
//     split of Sec. 2 applied continuously across sweep boundaries).
//   * For the last `band` groups and for the mover's own group, both possible
//     outcomes of partner j are evaluated ahead of time (old position and
//     trial position), so that once j's accept bit is known only a select and
//     an add remain on the critical path.
//   * Inside the own group the accept bits are found by iterating the
//     sequential rule a_i = f_i(a_0..a_{i-1}) to its fixed point (Jacobi
//     sweeps over the wave); the fixed point is unique and equals the
//     sequential outcome, reached in at most 64 iterations, usually two.
//   * The deciding wave writes the group's new positions in place (double
//     buffered by sweep parity), its accept mask and the running energy, and
//     advances the chain's front counter with release semantics.
#pragma once

#include "mc_device.hpp"

namespace mcdev {

// Description of one chain inside a sweep launch (device memory).
struct ChainDesc {
    int32_t n;           // ions
    int32_t nb;          // groups of 64 (last one padded with inert ions)
    int32_t band;        // look-ahead band in groups, 0..min(kMaxBand, nb-1)
    int32_t wg_count;    // workgroups serving this chain
    int32_t wg_first;    // first workgroup index of this chain in the grid
    uint32_t chain_id;   // Philox counter word 2
    uint64_t seed;       // Philox key
    double lB;           // Bjerrum length
    double D;            // trial cube side
    double half_uniform; // sigma/2 when every ion has the same diameter
    void* pos;           // T4[2][npad]: positions by sweep parity, w = charge
    void* half;          // T[npad]: sigma_i / 2
    const double* wall_a;// double[npad]: R - sigma_i / 2
    GroupRec* rec;       // [kRing]
    uint64_t* front;     // groups decided (stream index of the next group)
    unsigned long long* stats;  // [8] counters, see mc_host
    double* e_series;    // [capacity] running energy after each sweep (global sweep index)
    int64_t e_capacity;
    uint8_t* trace_acc;  // [trace_cap]
    double* trace_de;    // [trace_cap]
    int64_t trace_cap;   // moves traced from the start of the chain
};

template <typename T, int M>
struct SweepShared {
    using T4 = typename Prec<T>::T4;
    static constexpr int P = kGroup / M;
    T4 st_old[M][P];         // partner slice: position (old position for the band)
    T4 st_new[M][P];         // partner slice: trial position (band / own group)
    T st_half[M][P];
    double part_s[M][kGroup];        // per-wave partial sums
    uint64_t part_ov[M];             // per-wave overlap ballots
    uint32_t part_ovo[M][kGroup];    // own group: overlap with old positions (slice bits)
    uint32_t part_ovt[M][kGroup];    // own group: overlap with trial positions (slice bits)
    T c_own[kGroup][kGroup];         // own group corrections [partner j][mover i]
};

template <typename T, int M, bool UNIFORM_SIGMA>
__global__ void __launch_bounds__(64 * M)
sweep_kernel(const ChainDesc* __restrict__ chains, const int32_t* __restrict__ wg_chain,
             uint32_t s0, int32_t n_sweeps, Ctl ctl)
{
    using T4 = typename Prec<T>::T4;
    constexpr int P = kGroup / M;
    __shared__ SweepShared<T, M> sh;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const ChainDesc& cd = chains[wg_chain[blockIdx.x]];
    const int k_wg = (int)blockIdx.x - cd.wg_first;

    const int n = cd.n, nb = cd.nb, band = cd.band;
    const int npad = nb * kGroup;
    T4* __restrict__ pos = (T4*)cd.pos;
    const T* __restrict__ half = (const T*)cd.half;
    const T D = (T)cd.D;
    const double lB = cd.lB;
    const T hu = (T)cd.half_uniform;
    const int64_t g_begin = (int64_t)s0 * nb;
    const int64_t g_end = g_begin + (int64_t)n_sweeps * nb;
    int64_t known = -1;  // largest front value this wave has observed

    for (int64_t g = g_begin + k_wg; g < g_end; g += cd.wg_count) {
        const int64_t s = g / nb;
        const int b = (int)(g - s * nb);
        const int ion = b * kGroup + lane;
        const bool valid = ion < n;

        // ---- the movers: old position (result of the group's previous trial) and trial
        wait_front(cd.front, g - nb + 1, known, ctl);
        const T4 xo = pos[(size_t)((s - 1) & 1) * npad + ion];
        const uint4 wd = move_words(cd.seed, cd.chain_id, (uint32_t)s, (uint32_t)ion);
        const T xi = xo.x, yi = xo.y, zi = xo.z, qi = xo.w;
        const T txi = trial_coord(xi, wd.x, D), tyi = trial_coord(yi, wd.y, D),
                tzi = trial_coord(zi, wd.z, D);
        const T hi = UNIFORM_SIGMA ? hu : half[ion];
        bool wall;
        {
            const double a = cd.wall_a[ion];
            const double X = (double)txi, Y = (double)tyi, Z = (double)tzi;
            const double r2 = X * X + Y * Y + Z * Z;
            wall = r2 > a * a;
        }
        const double u3 = accept_uniform(wd.w);

        double S = 0.0;     // sum_j q_j (1/|x~_i - x_j| - 1/|x_i - x_j|)
        bool ov = false;    // overlap with a partner whose position is final

        // ---- own group: both outcomes of every partner j != i
        T c_own[P];
        uint32_t ovo_own = 0, ovt_own = 0;
        {
            if (lane >= wave * P && lane < wave * P + P) {
                const int m = lane - wave * P;
                sh.st_old[wave][m] = xo;
                sh.st_new[wave][m] = mk4<T>(txi, tyi, tzi, qi);
                sh.st_half[wave][m] = hi;
            }
            wave_lds_sync();
            T sf = 0;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int j = wave * P + m;
                const T4 po = sh.st_old[wave][m];
                const T4 pt = sh.st_new[wave][m];
                const T hj = UNIFORM_SIGMA ? hu : sh.st_half[wave][m];
                const T s_ij = hi + hj;
                const T d2o = Prec<T>::norm2(po.x - xi, po.y - yi, po.z - zi);
                const T d2ot = Prec<T>::norm2(po.x - txi, po.y - tyi, po.z - tzi);
                const T d2t = Prec<T>::norm2(pt.x - xi, pt.y - yi, pt.z - zi);
                const T d2tt = Prec<T>::norm2(pt.x - txi, pt.y - tyi, pt.z - tzi);
                const T o = po.w * (Prec<T>::rinv(d2ot) - Prec<T>::rinv(d2o));
                const T t = pt.w * (Prec<T>::rinv(d2tt) - Prec<T>::rinv(d2t));
                const bool oo = d2ot < s_ij * s_ij, ot = d2tt < s_ij * s_ij;
                if (j > lane) {
                    sf += o;
                    ov |= oo;
                    c_own[m] = 0;
                } else if (j < lane) {
                    sf += o;
                    c_own[m] = t - o;
                    ovo_own |= (uint32_t)oo << m;
                    ovt_own |= (uint32_t)ot << m;
                } else {
                    c_own[m] = 0;
                }
            }
            S += (double)sf;
        }

        // ---- band groups g-1..g-band: both outcomes, evaluated ahead of their decisions
        T c_band[kMaxBand][P];
        uint32_t ovo_band[kMaxBand], ovt_band[kMaxBand];
#pragma unroll
        for (int kb = 0; kb < kMaxBand; ++kb) {
            ovo_band[kb] = 0;
            ovt_band[kb] = 0;
            if (kb < band) {
                const int64_t gp = g - 1 - kb;
                const int64_t sp = floor_div(gp, nb);
                const int bp = (int)(gp - sp * nb);
                // old position of j = result of its trial one sweep before (front >= g-nb+1 covers it)
                if (lane < P) {
                    const int j = bp * kGroup + wave * P + lane;
                    const T4 po = pos[(size_t)((sp - 1) & 1) * npad + j];
                    const uint4 wj = move_words(cd.seed, cd.chain_id, (uint32_t)sp, (uint32_t)j);
                    sh.st_old[wave][lane] = po;
                    sh.st_new[wave][lane] = mk4<T>(trial_coord(po.x, wj.x, D), trial_coord(po.y, wj.y, D),
                                                    trial_coord(po.z, wj.z, D), po.w);
                    if (!UNIFORM_SIGMA) sh.st_half[wave][lane] = half[j];
                }
                wave_lds_sync();
                T sf = 0;
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const T4 po = sh.st_old[wave][m];
                    const T4 pt = sh.st_new[wave][m];
                    const T hj = UNIFORM_SIGMA ? hu : sh.st_half[wave][m];
                    const T s_ij = hi + hj;
                    const T d2o = Prec<T>::norm2(po.x - xi, po.y - yi, po.z - zi);
                    const T d2ot = Prec<T>::norm2(po.x - txi, po.y - tyi, po.z - tzi);
                    const T d2t = Prec<T>::norm2(pt.x - xi, pt.y - yi, pt.z - zi);
                    const T d2tt = Prec<T>::norm2(pt.x - txi, pt.y - tyi, pt.z - tzi);
                    const T o = po.w * (Prec<T>::rinv(d2ot) - Prec<T>::rinv(d2o));
                    const T t = pt.w * (Prec<T>::rinv(d2tt) - Prec<T>::rinv(d2t));
                    sf += o;
                    c_band[kb][m] = t - o;
                    ovo_band[kb] |= (uint32_t)(d2ot < s_ij * s_ij) << m;
                    ovt_band[kb] |= (uint32_t)(d2tt < s_ij * s_ij) << m;
                }
                S += (double)sf;
                wave_lds_sync();
            }
        }

        // ---- decided partner groups g-nb+1 .. g-band-1, in stream order
        int64_t sp = (b + 1 < nb) ? s - 1 : s;   // sweep and group of g-nb+1
        int bp = (b + 1 < nb) ? b + 1 : 0;
        for (int64_t gp = g - nb + 1; gp <= g - band - 1; ++gp) {
            wait_front(cd.front, gp + 1, known, ctl);
            if (lane < P) {
                const int j = bp * kGroup + wave * P + lane;
                sh.st_old[wave][lane] = pos[(size_t)(sp & 1) * npad + j];
                if (!UNIFORM_SIGMA) sh.st_half[wave][lane] = half[j];
            }
            wave_lds_sync();
            T sf = 0;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const T4 p = sh.st_old[wave][m];
                const T hj = UNIFORM_SIGMA ? hu : sh.st_half[wave][m];
                const T s_ij = hi + hj;
                const T d2 = Prec<T>::norm2(p.x - xi, p.y - yi, p.z - zi);
                const T d2t = Prec<T>::norm2(p.x - txi, p.y - tyi, p.z - tzi);
                sf = Prec<T>::fma(p.w, Prec<T>::rinv(d2t) - Prec<T>::rinv(d2), sf);
                ov |= d2t < s_ij * s_ij;
            }
            S += (double)sf;
            wave_lds_sync();
            if (++bp == nb) {
                bp = 0;
                ++sp;
            }
        }

        // ---- apply the band groups' decisions as they arrive (oldest first)
        double e_prev = 0.0;
#pragma unroll
        for (int kb = kMaxBand - 1; kb >= 0; --kb) {
            if (kb < band) {
                const int64_t gp = g - 1 - kb;
                wait_front(cd.front, gp + 1, known, ctl);
                const uint64_t acc = cd.rec[(size_t)(gp & (kRing - 1))].acc;
                const uint32_t a = (uint32_t)(acc >> (wave * P)) & (uint32_t)((1ull << P) - 1);
                T cf = 0;
#pragma unroll
                for (int m = 0; m < P; ++m)
                    if ((a >> m) & 1u) cf += c_band[kb][m];
                S += (double)cf;
                ov |= (((a & ovt_band[kb]) | (~a & ovo_band[kb])) != 0u);
            }
        }

        // ---- combine the waves
        sh.part_s[wave][lane] = S;
        {
            const uint64_t ob = __ballot(ov);
            if (lane == 0) sh.part_ov[wave] = ob;
        }
        sh.part_ovo[wave][lane] = ovo_own;
        sh.part_ovt[wave][lane] = ovt_own;
#pragma unroll
        for (int m = 0; m < P; ++m) sh.c_own[wave * P + m][lane] = c_own[m];
        __syncthreads();

        if (wave == 0) {
            double St = 0.0;
            uint64_t ovo = 0, ovt = 0;
            bool ovb = false;
#pragma unroll
            for (int w = 0; w < M; ++w) {
                St += sh.part_s[w][lane];
                ovb |= ((sh.part_ov[w] >> lane) & 1ull) != 0;
                ovo |= (uint64_t)sh.part_ovo[w][lane] << (w * P);
                ovt |= (uint64_t)sh.part_ovt[w][lane] << (w * P);
            }
            wait_front(cd.front, g, known, ctl);  // group g-1 decided: running energy
            e_prev = cd.rec[(size_t)((g - 1) & (kRing - 1))].e_run;

            // Sequential decisions inside the group by fixed-point iteration.
            const double lq = lB * (double)qi;
            uint64_t acc = 0;
            double dE = 0.0;
            bool dec = false;
            int it = 0;
            for (;;) {
                T own = 0;
                uint64_t bits = acc;
                while (bits) {
                    const int j = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    own += sh.c_own[j][lane];
                }
                const bool ovown = ((acc & ovt) | (~acc & ovo)) != 0;
                dE = lq * (St + (double)own);
                dec = valid && !wall && !ovb && !ovown && (dE <= 0.0 || u3 < exp(-dE));
                const uint64_t nacc = __ballot(dec);
                ++it;
                if (nacc == acc || it > kGroup + 1) { acc = nacc; break; }
                acc = nacc;
            }

            // in-place update (double buffered by sweep parity)
            pos[(size_t)(s & 1) * npad + ion] = dec ? mk4<T>(txi, tyi, tzi, qi) : xo;
            const double de_acc = __shfl(wave_sum(dec ? dE : 0.0), 0, 64);
            const double e_new = e_prev + de_acc;
            if (valid) {
                const int64_t mv = s * (int64_t)n + ion;
                if (mv < cd.trace_cap) {
                    cd.trace_acc[mv] = (uint8_t)dec;
                    cd.trace_de[mv] = dE;
                }
            }
            const uint64_t m_wall = __ballot(valid && wall);
            const uint64_t m_ov = __ballot(valid && !wall && (ovb || ((acc & ovt) | (~acc & ovo)) != 0));
            const uint64_t m_valid = __ballot(valid);
            if (lane == 0) {
                atomicAdd(&cd.stats[0], (unsigned long long)__popcll(m_valid));
                atomicAdd(&cd.stats[1], (unsigned long long)__popcll(acc));
                atomicAdd(&cd.stats[2], (unsigned long long)__popcll(m_wall));
                atomicAdd(&cd.stats[3], (unsigned long long)__popcll(m_ov));
                atomicAdd(&cd.stats[4], (unsigned long long)(__popcll(m_valid) - __popcll(acc) -
                                                             __popcll(m_wall) - __popcll(m_ov)));
                atomicAdd(&cd.stats[5], (unsigned long long)it);
                if (b == nb - 1 && s < cd.e_capacity) cd.e_series[s] = e_new;
                GroupRec& r = cd.rec[(size_t)(g & (kRing - 1))];
                r.acc = acc;
                r.e_run = e_new;
                r.tag = g + 1;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                __hip_atomic_store(cd.front, (uint64_t)(g + 1), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

}  // namespace mcdev
