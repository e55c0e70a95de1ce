// mc_aux_kernels.hpp -- double-precision total-energy re-sum and pair
// correlation (g(r)) kernels for gfx950.
//
// Paper: Liang, Xing, Li, arXiv:1602.05716.  Sec. 3.3: energy sums in double
// precision; Sec. 5.2: the total energy is monitored, and the pair
// correlation functions are measured on ions away from the wall.
#pragma once

#include "mc_sweep_kernel.hpp"

namespace mcdev {

// Small device-side record of the energy bookkeeping.
struct EnergyAux {
    double e_resum;      // last re-summed total energy
    double drift_last;   // running minus re-summed energy at the last re-sum
    double drift_max;    // largest |drift| seen
    unsigned long long n_resum;
};

// Work item of a batched auxiliary launch: chain index and the block's index
// inside that chain.
struct BlockItem {
    int32_t chain;
    int32_t part;
};

// Positions are read as {x, y, z, *} records (the fourth word is the sweep
// version tag of the sweep kernel) from the image of the given parity, and
// charges from their own array.  E = l_B sum_{i<j} q_i q_j / r_ij, every term
// formed exactly as (q_i q_j) / sqrt(d2) in double.  Block p of a chain
// handles the row groups p and nb-1-p (so every block does nb+1 tiles); wave
// w of the block takes the tiles t = row + w, row + w + 4, ...  The chain's
// e_partial[p] receives the block's sum.
template <typename T>
__global__ void __launch_bounds__(256)
energy_partial_kernel(const ChainDesc* __restrict__ chains, const BlockItem* __restrict__ items, int parity)
{
    using T4 = typename Prec<T>::T4;
    __shared__ double st[4][kGroup][4];
    __shared__ double wsum[4];
    const BlockItem it = items[blockIdx.x];
    const ChainDesc& cd = chains[it.chain];
    const int nb = cd.nb;
    const T4* __restrict__ pos = (const T4*)cd.pos + (size_t)parity * nb * kGroup;
    const T* __restrict__ charge = (const T*)cd.charge;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = it.part;
    double acc = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        const int row = pass == 0 ? p : nb - 1 - p;
        if (pass == 1 && row == p) break;
        const int i = row * kGroup + lane;
        const T4 xi4 = pos[i];
        const double xi = (double)xi4.x, yi = (double)xi4.y, zi = (double)xi4.z, qi = (double)charge[i];
        double e = 0.0;
        for (int t = row + wave; t < nb; t += 4) {
            const T4 pj = pos[t * kGroup + lane];
            st[wave][lane][0] = (double)pj.x;
            st[wave][lane][1] = (double)pj.y;
            st[wave][lane][2] = (double)pj.z;
            st[wave][lane][3] = (double)charge[t * kGroup + lane];
            wave_lds_sync();
            for (int m = 0; m < kGroup; ++m) {
                const int j = t * kGroup + m;
                const double dx = xi - st[wave][m][0];
                const double dy = yi - st[wave][m][1];
                const double dz = zi - st[wave][m][2];
                const double d2 = dx * dx + dy * dy + dz * dz;
                const double term = (qi * st[wave][m][3]) / __builtin_sqrt(d2);
                if (j > i) e += term;
            }
            wave_lds_sync();
        }
        acc += e;
    }
    const double ws = __shfl(wave_sum(acc), 0, 64);
    if (lane == 0) wsum[wave] = ws;
    __syncthreads();
    if (threadIdx.x == 0) cd.e_partial[p] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// One block per chain: sums the chain's partials in a fixed order, records
// the drift of the running energy and, when `reset` is set, makes the re-sum
// the new running energy.
__global__ void energy_finalize_kernel(const ChainDesc* __restrict__ chains, int reset, int record_drift)
{
    if (threadIdx.x != 0) return;
    const ChainDesc& cd = chains[blockIdx.x];
    EnergyAux* aux = (EnergyAux*)cd.aux;
    const int nparts = (cd.nb + 1) / 2;
    double e = 0.0;
    for (int k = 0; k < nparts; ++k) e += cd.e_partial[k];
    e *= cd.lB;
    aux->e_resum = e;
    if (record_drift) {
        const double d = *cd.e_state - e;
        aux->drift_last = d;
        const double ad = d < 0 ? -d : d;
        if (ad > aux->drift_max) aux->drift_max = ad;
        aux->n_resum += 1;
    }
    if (reset) *cd.e_state = e;
}

// Pair counts for g_ab(r): centre i needs |x_i| <= R - rmax (the wall
// exclusion of Sec. 5.2), neighbours are all j != i; bin k = floor(r / dr)
// for r < rmax.  Distances and bins are formed in double exactly as written
// (no fused multiply-add), so the integer counts do not depend on the
// kernel's tiling.  One block of 4 waves per group of 64 centres of a chain;
// each wave takes every 4th partner tile; counts go to an LDS histogram
// first.
template <typename T>
__global__ void __launch_bounds__(256)
rdf_kernel(const ChainDesc* __restrict__ chains, const BlockItem* __restrict__ items, int parity,
           double rmax, double dr, int bins)
{
    using T4 = typename Prec<T>::T4;
    extern __shared__ unsigned int hist[];   // [ntypes*ntypes*bins]
    __shared__ double st[4][kGroup][3];
    __shared__ int stt[4][kGroup];
    const BlockItem item = items[blockIdx.x];
    const ChainDesc& cd = chains[item.chain];
    const int n = cd.n, nb = cd.nb, ntypes = cd.ntypes;
    const T4* __restrict__ pos = (const T4*)cd.pos + (size_t)parity * nb * kGroup;
    const int32_t* __restrict__ type = cd.type;
    const double rc = cd.rdf_rc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nh = ntypes * ntypes * bins;
    for (int k = threadIdx.x; k < nh; k += blockDim.x) hist[k] = 0u;
    __syncthreads();

    const int row = item.part;
    const int i = row * kGroup + lane;
    const T4 xi4 = pos[i];
    const double xi = (double)xi4.x, yi = (double)xi4.y, zi = (double)xi4.z;
    const double r2i = xi * xi + yi * yi + zi * zi;
    const bool centre = i < n && rc >= 0.0 && !(r2i > rc * rc);
    const int ti = i < n ? type[i] : 0;
    const double rmax2 = rmax * rmax * (1.0 + 1e-12);
    if (wave == 0) {
        const unsigned long long cm = __ballot(centre);
        if (cm) {
            // centres of this block by type
            for (int a = 0; a < ntypes; ++a) {
                const unsigned long long ca = __ballot(centre && ti == a);
                if (lane == 0 && ca) atomicAdd(&cd.rdf_centres[a], (unsigned long long)__popcll(ca));
            }
        }
    }
    for (int t = wave; t < nb; t += 4) {
        const int jj = t * kGroup + lane;
        const T4 pj = pos[jj];
        st[wave][lane][0] = (double)pj.x;
        st[wave][lane][1] = (double)pj.y;
        st[wave][lane][2] = (double)pj.z;
        stt[wave][lane] = jj < n ? type[jj] : -1;
        wave_lds_sync();
        if (centre) {
            for (int m = 0; m < kGroup; ++m) {
                const int j = t * kGroup + m;
                const int tj = stt[wave][m];
                if (j == i || tj < 0) continue;
                const double dx = xi - st[wave][m][0];
                const double dy = yi - st[wave][m][1];
                const double dz = zi - st[wave][m][2];
                const double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 < rmax2) {
                    const double r = __builtin_sqrt(d2);
                    if (r < rmax) {
                        const int k = (int)__builtin_floor(r / dr);
                        if (k < bins) atomicAdd(&hist[(ti * ntypes + tj) * bins + k], 1u);
                    }
                }
            }
        }
        wave_lds_sync();
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nh; k += blockDim.x)
        if (hist[k]) atomicAdd(&cd.rdf_counts[k], (unsigned long long)hist[k]);
}

}  // namespace mcdev
