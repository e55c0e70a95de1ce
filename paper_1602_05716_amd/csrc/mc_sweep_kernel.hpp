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
//     every partner group.  This is
//     the paper's "brush" (Sec. 3.4) turned so that the partner index is
//     uniform across the wave.
//   * By Eq. (Delta E_ij) the term of partner j is final as soon as j's own
//     latest trial is decided.  Partner groups decided more than `band`
//     groups before g are summed directly with their published positions, in
//     stream order, as they get decided (the upper/lower triangle split of
//     Sec. 2 applied continuously across sweep boundaries).
//   * For the last `band` groups and for the mover's own group, both possible
//     outcomes of partner j are evaluated at the start of the target's work
//     (old position and trial position), so that once j's accept bit is
//     known only a select and an add remain.
//   * The newest band groups' candidates (g-1, g-2) and the own group's go to
//     LDS for the chain step as soon as they are computed.  The older band
//     groups' accept masks are published before the compute waves finish;
//     each wave folds its slice of their candidates from the mask, then hands
//     over its partial sum and moves on to its next target.
//   * Wave 0 then decides the group: if the threshold lies outside the
//     interval spanned by the unknown corrections for every lane, at once.
//     Otherwise it solves the group's own accept bits, the fixed point of the
//     sequential rule a_i = f_i(a_0..a_{i-1}) (Jacobi sweeps over the wave;
//     the system is lower triangular, so the fixed point is unique, equals
//     the sequential outcome and is reached from any start), for a guess of
//     the pending band groups' masks (all rejected), while wave 1 sums the
//     older pending groups' masked rows as their masks arrive.  Each true
//     correction then costs one evaluation when the guess was right, a few
//     more iterations (updating the row sum by the flipped bits) when not.
//   * Publication: the accept mask goes out at once in the group record; the
//     new positions are written in place, double buffered by sweep parity,
//     each 16-byte record carrying the sweep index of the trial that produced
//     it in its fourth word, so a reader validates every record it loads and
//     no device-wide counter or cache flush is needed (agent-coherent
//     accesses only).
#pragma once

#include <type_traits>

#include "mc_device.hpp"

namespace mcdev {

// Delayed-acceptance surrogate: sizes of the network and of its input.
constexpr int kDaBins = 64;               // bins of each neighbour histogram
constexpr int kDaIn = 2 * kDaBins;        // like- and unlike-charge histograms
constexpr int kDaHid = 128;               // hidden units of both hidden layers
constexpr int kDaParams = kDaIn * kDaHid + kDaHid + kDaHid * kDaHid + kDaHid + kDaHid + 1;

// Device state of a chain's delayed-acceptance stage and its drift monitor.
struct DAState {
    int32_t active;          // 1: two-stage test for moves without a conflict
    int32_t window;          // monitor window in sweeps (launches end on its multiples)
    int64_t fallback_sweep;  // sweep at which the monitor switched to the plain test, -1 = never
    double ref_rate;         // stage-2 rejection rate of stage-1 passes at training time (< 0: no monitor)
    double delta;            // switch to the plain test when a window's rate exceeds ref_rate + delta
    unsigned long long win_pass0, win_rej0;  // counters at the start of the window
    double last_rate;        // rate of the last complete window
    int64_t min_count;       // windows with fewer stage-1 passes are not judged
};

// Description of one chain inside a sweep launch (device memory).
struct ChainDesc {
    int32_t n;           // ions
    int32_t nb;          // groups of 64 (last one padded with inert ions)
    int32_t band;        // look-ahead band in groups, 0..min(kMaxBand, nb-1)
    int32_t wg_count;    // workgroups serving this chain
    int32_t npad;        // nb * 64
    uint32_t chain_id;   // Philox counter word 2
    uint64_t seed;       // Philox key
    double lB;           // Bjerrum length
    double D;            // trial cube side
    double half_uniform; // sigma/2 when every ion has the same diameter
    void* pos;           // versioned positions by sweep parity (see PosIO)
    void* charge;        // T[npad]: q_i
    void* half;          // T[npad]: sigma_i / 2
    const double* wall_a;// double[npad]: R - sigma_i / 2
    GroupRec* rec;       // [kRing]
    unsigned long long* stats;  // [7] counters: moves, accepted, wall, overlap, Metropolis rejections, iterations, early groups
    double* de_group;    // [launch groups] energy change of each group of the launch
    uint8_t* trace_acc;  // [trace_cap]
    double* trace_de;    // [trace_cap]
    int64_t trace_cap;   // moves traced from the start of the chain
    unsigned long long* clk;  // [2] wall clock at the launch start and when the
                              // chain's last group of the launch was published
    // energy bookkeeping and g(r) (auxiliary kernels)
    double* e_partial;   // [(nb + 1) / 2] re-sum partials
    void* aux;           // EnergyAux
    double* e_state;     // running energy
    double* sweep_tot;   // [max sweeps per launch] scratch of the scan
    double* e_series;    // [e_capacity] running energy after each sweep
    int64_t e_capacity;
    const int32_t* type; // [npad] species index, -1 for padding
    int32_t ntypes;
    int32_t pad0;
    double rdf_rc;       // centres need |x| <= rdf_rc
    unsigned long long* rdf_counts;   // [ntypes * ntypes * bins]
    unsigned long long* rdf_centres;  // [ntypes]
    // delayed acceptance (kernels with DA = true only)
    const float* da_w;   // [kDaParams] network parameters (bfloat16 values held in float)
    const uint16_t* da_w1b;  // [128 x 128] W1 as bfloat16, transposed (row = hidden unit)
    const uint16_t* da_w2b;  // [128 x 128] W2 as bfloat16, transposed
    DAState* da;         // monitor state
    double da_rc;        // histogram range
    double da_dr;        // histogram bin width da_rc / 64
    uint32_t* log_feat;  // [log_cap][64] packed byte histograms of logged moves
    double* log_de;      // [log_cap] exact dE
    double* log_deh;     // [log_cap] surrogate dEh (0 when not evaluated)
    uint8_t* log_flags;  // [log_cap] bit0 wall, 1 overlap, 2 conflict, 3 stage-1 reject,
                         //           4 stage-2 reject, 5 accepted, 7 written
    int64_t log_cap;     // moves logged from the start of the chain
};

// A position record is {x, y, z, version}: version = sweep index (mod 2^32)
// of the trial that produced the position; slot pos[s & 1][i] holds the
// result of trial (s, i).  Float path: one 16-byte record.  Double path: two
// 16-byte halves {x, y}, {z, version}; the writer drains the first half
// before storing the second and the reader validates the second half before
// loading the first.
// Pause between two polls of a global-memory slot: the shortest sleep, or
// about 0.85 us (32 x 64 clocks) for a patient reader.
__device__ __forceinline__ void poll_pause(bool patient) {
    if (patient)
        __builtin_amdgcn_s_sleep(32);
    else
        __builtin_amdgcn_s_sleep(1);
}

template <typename T> struct PosIO;

template <> struct PosIO<float> {
    struct Rec { float x, y, z; uint32_t ver; };
    static constexpr uint32_t kBytes = 16;
    static __device__ __forceinline__ Rec load(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
        return __builtin_bit_cast(Rec, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 16u, 0, kCoherent));
    }
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t idx, float x, float y,
                                                 float z, uint32_t ver) {
        Rec v{x, y, z, ver};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, idx * 16u, 0, kCoherent);
    }
    // loads slot idx until its version is `ver` (all lanes with `active`);
    // a patient reader (one whose result is not needed for several groups)
    // polls about once a microsecond instead of back to back
    static __device__ __forceinline__ Rec load_valid(__amdgpu_buffer_rsrc_t r, uint32_t idx, uint32_t ver,
                                                     bool active, const Ctl& ctl, bool patient = false) {
        Rec v{0.f, 0.f, 0.f, ver};
        if (active) v = load(r, idx);
        if (__ballot(active && v.ver != ver) == 0ull) return v;
        PollGuard pg;
        for (;;) {
            poll_pause(patient);
            if (active && v.ver != ver) v = load(r, idx);
            if (__ballot(active && v.ver != ver) == 0ull) break;
            if (pg.stop(ctl)) break;
        }
        return v;
    }
};

template <> struct PosIO<double> {
    struct Rec { double x, y, z; uint32_t ver, pad; };
    struct Lo { double x, y; };
    struct Hi { double z; uint32_t ver, pad; };
    static constexpr uint32_t kBytes = 32;
    static __device__ __forceinline__ Hi load_hi(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
        return __builtin_bit_cast(Hi, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 32u + 16u, 0, kCoherent));
    }
    static __device__ __forceinline__ Lo load_lo(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
        return __builtin_bit_cast(Lo, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 32u, 0, kCoherent));
    }
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t idx, double x, double y,
                                                 double z, uint32_t ver) {
        Lo lo{x, y};
        Hi hi{z, ver, 0u};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, lo), r, idx * 32u, 0, kCoherent);
        drain_memory();
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, hi), r, idx * 32u + 16u, 0, kCoherent);
    }
    static __device__ __forceinline__ Rec load_valid(__amdgpu_buffer_rsrc_t r, uint32_t idx, uint32_t ver,
                                                     bool active, const Ctl& ctl, bool patient = false) {
        Hi h{0.0, ver, 0u};
        if (active) h = load_hi(r, idx);
        if (__ballot(active && h.ver != ver) != 0ull) {
            PollGuard pg;
            for (;;) {
                poll_pause(patient);
                if (active && h.ver != ver) h = load_hi(r, idx);
                if (__ballot(active && h.ver != ver) == 0ull) break;
                if (pg.stop(ctl)) break;
            }
        }
        drain_memory();  // the high half is validated before the low half is read
        Lo l{0.0, 0.0};
        if (active) l = load_lo(r, idx);
        return Rec{l.x, l.y, h.z, h.ver, 0u};
    }
};

// Bit masks over one wave's slice of a partner group.
template <int P> struct SliceBits;
template <> struct SliceBits<8> { using type = uint8_t; };
template <> struct SliceBits<16> { using type = uint16_t; };

// Band groups with both-outcome candidates: up to kMaxBand (kDaMaxBand in
// the delayed-acceptance kernels, whose network would otherwise spill).
// The newest kChainSlots of them (g-1, g-2[, g-3]) go to the chain step
// through LDS; the accept masks of the older ones are out before the compute
// waves finish, and each wave resolves its own slice of their candidates
// itself.  (The four-wave float kernels keep two slots: a third would no
// longer let two workgroups share a CU's LDS.  The double kernels run one workgroup
// per CU and take three.  The delayed-acceptance kernels, whose LDS also
// holds the neighbour histograms and the network, take one.)
template <bool DA> constexpr int kBandSlots = DA ? kDaMaxBand : kMaxBand;
// ... and of the float kernels that hold fewer band groups in registers: the
// one for per-ion diameters, whose extra per-partner work leaves no room for
// a fourth (it would spill, and a spilling persistent kernel runs one
// workgroup per CU), and the eight-wave ones, which fit 128 registers so
// that two workgroups (sixteen waves) share a CU.
template <typename T, int M, bool UNIFORM_SIGMA, bool DA>
constexpr int kChainBand = DA ? kBandSlots<DA>
                              : sizeof(T) != 4 ? kMaxBand
                              : M == 8 ? (UNIFORM_SIGMA ? kMaxBandWide : kMaxBandWidePerIon)
                                       : (UNIFORM_SIGMA ? kMaxBand : kMaxBandPerIon);
// LDS chain slots; the eight-wave float kernels take one, which brings their
// LDS to 47.8 KB for two workgroups per CU.
template <typename T, int M, bool DA>
constexpr int kChainSlots = DA ? 1 : (sizeof(T) == 4 ? (M == 8 ? 1 : 2) : 3);
// Partners per wave in a tile of a decided partner group.  The eight-wave
// float kernels take 64: wave w takes every eighth decided group (w, w + 8,
// ... after the oldest) whole, so that a tile's fixed costs (its load and
// version check, the LDS staging and its waits, the double accumulation) fall
// on 64 pair terms a lane instead of 8, and every lane loads.  Measured 12-14 %
// faster where the pair terms bound (N >= 65536); with four waves, 32-partner
// slices were slower (the last decided tile lengthens the hand-off that the
// decision chain waits for).  The other kernels split every group over all
// their waves.
template <typename T, int M, bool DA>
constexpr int kDecidedSlice = (sizeof(T) == 4 && M == 8 && !DA) ? 64 : kGroup / M;
// A compute wave waiting for a partner group more than this many groups
// before its target polls patiently: the chain publishes about one group
// every two microseconds, far slower than a tile takes to compute.
constexpr int kPatientDistance = 6;

template <typename T, int M, bool DA = false>
struct SweepShared {
    using T4 = typename Prec<T>::T4;
    static constexpr int P = kGroup / M;
    static constexpr int PD = kDecidedSlice<T, M, DA>;
    static constexpr int KB = kBandSlots<DA>;
    static constexpr int LC = kChainSlots<T, M, DA>;
    using SB = typename SliceBits<P>::type;
    // per compute wave: staging of the current partner slice {x, y, z, q}
    // (a decided tile of PD > P partners continues in st_old2 / st_half2)
    T4 st_old[M][P];
    T4 st_new[M][P];
    T st_half[M][P];
    // hand-off from the compute waves to the chain wave (one target at a time)
    double part_s[M][kGroup];   // partial sums over each wave's partners
    uint64_t part_ov[M];        // overlap ballots over final partners
    T part_pn[M][2][kGroup];    // per wave: sums of the positive / negative
                                // corrections still unknown (groups g-1..g-LC, own group)
    // overlap bits per mover i, one 64-bit word over the partners j in which
    // wave w fills the slice of its own partners (bits w P .. w P + P - 1)
    static_assert(sizeof(SB) * M == 8, "the waves' slices tile a 64-bit word");
    alignas(8) SB ovo_own[kGroup][M];    // own group, j < i: overlap with j's old position
    alignas(8) SB ovt_own[kGroup][M];    //                   overlap with j's trial position
    alignas(8) SB ovo_b[LC][kGroup][M];  // group g-1-kb: overlap with j's old / trial position
    alignas(8) SB ovt_b[LC][kGroup][M];
    // corrections, one padded row per mover i (16-byte reads of 4 partners
    // are free of bank conflicts)
    static constexpr int CS = kGroup + (sizeof(T) == 4 ? 4 : 2);
    T c_own[kGroup][CS];           // own group [mover i][partner j]
    T c_b[LC][kGroup][CS];         // group g-1-kb [mover i][partner j]
    T fac[kGroup];                 // chain wave: 0/1 factors of a row sum's mask
    int ready;                  // compute waves done filling the hand-off for the current target
    int consumed;               // local target index + 1 the chain wave last released
    // the helper wave's part of the chain step: band corrections of groups
    // g-LC..g-2 (summed oldest first), their overlap ballot, its factor row,
    // and the local target index + 1 it last finished
    double h_corr[LC > 1 ? kGroup : 1];
    uint64_t h_ov;
    T fac_h[LC > 1 ? kGroup : 1];
    int h_done;
    // delayed acceptance: per mover, byte histograms of neighbour distances at
    // the old position (bytes 0..127) and at the trial position (128..255),
    // each like-charged bins 0..63 then unlike-charged; conflict ballots of
    // the waves; the surrogate's dEh; partial sums of the network's last layer
    uint32_t hist[DA ? kGroup : 1][DA ? 65 : 1];   // rows padded to 65 words (bank-conflict free)
    uint64_t part_conf[DA ? M : 1];
    double deh[DA ? kGroup : 1];
    float part_out[DA ? M : 1][2][DA ? kGroup : 1];
    // the network's two matrices, transposed ([hidden unit][input]), as
    // bfloat16, rows padded to 132 values (8-byte reads free of bank
    // conflicts); loaded once per launch
    static constexpr bool kWtsLds = DA && sizeof(T) == 4;  // (the double kernel reads them from memory)
    uint16_t wts[kWtsLds ? 2 * kDaHid : 1][kWtsLds ? kDaIn + 4 : 1];
    // bfloat16 hidden activations [mover][position][unit] of the network, in
    // the space of c_own and c_b (free between the chain wave's release and
    // the next hand-off)
    __device__ uint16_t* h1() { return reinterpret_cast<uint16_t*>(&c_own[0][0]); }
    // placed last, so that the fields above keep their offsets
    T4 st_old2[M][PD > P ? PD - P : 1];
    T st_half2[M][PD > P ? PD - P : 1];
};

// The 64-bit word of overlap bits that the waves' slices tile.
template <typename SB, int M>
__device__ __forceinline__ uint64_t slice_word(const SB (&w)[M]) {
    uint64_t v;
    __builtin_memcpy(&v, &w[0], sizeof(v));
    return v;
}

// Bounded LDS wait used between the compute waves and the chain wave.
__device__ __forceinline__ void wait_lds_at_least(int* flag, int want, const Ctl& ctl) {
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < want) {
        PollGuard pg;
        for (;;) {
            __builtin_amdgcn_s_sleep(1);
            if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= want) break;
            if (pg.stop(ctl)) break;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// sum_j [bit j of mask] row[j] over the 64 partners, branch free.  The
// (wave-uniform) mask is spread over the lanes as 0/1 factors in LDS, one
// per partner, written lane-parallel; every lane then reads the factors as
// broadcasts beside its own row and multiply-adds: one vector instruction
// per partner (fma(1, v, a) rounds exactly as a + v, and fma(0, v, a) = a).
// 16-byte loads; fixed order, four independent accumulators: deterministic.
// Only the chain wave calls it, on its own factor row.
template <typename T>
__device__ __forceinline__ T masked_row_sum(const T* __restrict__ row, T* fac, uint64_t mask) {
    constexpr int V = 16 / (int)sizeof(T);  // values per 16-byte read
    typedef T VT __attribute__((ext_vector_type(V)));
    const int lane = threadIdx.x & 63;
    wave_lds_sync();  // the previous call's factor reads come first
    fac[lane] = (T)(uint32_t)((mask >> lane) & 1ull);
    wave_lds_sync();
    T a[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < kGroup; j += V) {
        const VT v = *reinterpret_cast<const VT*>(row + j);
        const VT f = *reinterpret_cast<const VT*>(fac + j);
#pragma unroll
        for (int k = 0; k < V; ++k) a[(j + k) & 3] = Prec<T>::fma_exact(f[k], v[k], a[(j + k) & 3]);
    }
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// The row sum of mask `to` from that of mask `from` (at most kFewFlips bits
// apart): for every bit that differs, in ascending order (a fixed order:
// deterministic), adds the entry if the bit is set in `to` and subtracts it
// otherwise.  Cheaper than a full masked_row_sum for a few flips: a scalar
// bit scan and one LDS read per flip, the reads issued before the first add.
constexpr int kFewFlips = 4;
template <typename T>
__device__ __forceinline__ T row_sum_update(const T* __restrict__ row, T own, uint64_t from, uint64_t to) {
    uint64_t f = from ^ to;
    T v[kFewFlips];
    bool up[kFewFlips];
#pragma unroll
    for (int q = 0; q < kFewFlips; ++q) {
        v[q] = 0;
        up[q] = true;
        if (f) {
            const int j = __builtin_ctzll(f);
            f &= f - 1;
            v[q] = row[j];
            up[q] = ((to >> j) & 1ull) != 0;
        }
    }
#pragma unroll
    for (int q = 0; q < kFewFlips; ++q) own = up[q] ? own + v[q] : own - v[q];
    return own;
}

// Publishes group g: its accept mask in the group record, then the new
// positions (trial position if accepted, old one otherwise), each tagged with
// the sweep index.
template <typename T>
__device__ __forceinline__ void publish_group(__amdgpu_buffer_rsrc_t rec_r, __amdgpu_buffer_rsrc_t pos_r,
                                              int64_t g, int64_t s, int npad, int ion, uint64_t acc,
                                              bool dec, T xi, T yi, T zi, T txi, T tyi, T tzi) {
    using IO = PosIO<T>;
    if ((threadIdx.x & 63) == 0) {
        GroupRec r;
        r.tag = (uint32_t)(g + 1);
        r.spare = 0;
        r.acc = acc;
        store_rec(rec_r, (uint32_t)(g & (kRing - 1)), r);
    }
    if (dec)
        IO::store(pos_r, (uint32_t)((s & 1) * npad + ion), txi, tyi, tzi, (uint32_t)s);
    else
        IO::store(pos_r, (uint32_t)((s & 1) * npad + ion), xi, yi, zi, (uint32_t)s);
}

// The sequential part of target group g, run by wave 0 after its own share
// of the pair terms: combine the waves' hand-off, decide the group (from the
// bounds, or after the band groups' accept masks by fixed-point iteration)
// and publish.
// Per-mover inputs of the chain step that do not depend on the other moves,
// formed at the start of the target's work, long before its decisions are
// due: the hard-wall test of the trial position (Sec. 5.2), the Metropolis
// threshold -log(u3) (u3 < exp(-dE) is evaluated as dE < -log(u3); the two
// forms can only disagree within rounding of the threshold itself, and
// dE <= 0 always accepts), and l_B q_i.
struct MoverInputs {
    bool wall;
    double thr;
    double lq;
};

template <typename T>
__device__ __forceinline__ MoverInputs mover_inputs(const ChainDesc& cd, int ion, T qi, T txi, T tyi, T tzi,
                                                    uint32_t w3) {
    MoverInputs mi;
    const double a = cd.wall_a[ion];
    const double X = (double)txi, Y = (double)tyi, Z = (double)tzi;
    int wall = (X * X + Y * Y + Z * Z > a * a) ? 1 : 0;
    double thr = -log(accept_uniform(w3));
    double lq = cd.lB * (double)qi;
    // evaluated here, not sunk to their first use behind the hand-off wait
    asm volatile("" : "+v"(wall), "+v"(thr), "+v"(lq));
    mi.wall = wall != 0;
    mi.thr = thr;
    mi.lq = lq;
    return mi;
}

// Counters of one workgroup, added to the chain's stats at the end.
struct WgCounters {
    unsigned long long moves = 0, acc = 0, wall = 0, ov = 0, iters = 0, early = 0;
    unsigned long long da_moves = 0, conflicts = 0, s1_rej = 0, s2_rej = 0, s1_pass = 0;
};

// The helper wave's part of the chain step of target g (wave 1, after its
// own hand-off): once every wave's candidates are in, the band corrections
// of groups g-LC..g-2 as their accept masks arrive, oldest first, for the
// chain wave -- which meanwhile solves the own group's fixed point.
template <typename T, int M, bool DA>
__device__ __forceinline__ void band_helper(SweepShared<T, M, DA>& sh, __amdgpu_buffer_rsrc_t rec_r, int64_t g,
                                            int t, int band, const Ctl& ctl) {
    constexpr int LC = SweepShared<T, M, DA>::LC;
    const int lane = threadIdx.x & 63;
    wait_lds_at_least(&sh.ready, M, ctl);
    double corr = 0.0;
    bool ov = false;
#pragma unroll
    for (int kb = LC - 1; kb >= 1; --kb) {
        if (kb < band) {
            const GroupRec r = wait_rec(rec_r, g - 1 - kb, ctl);
            corr += (double)masked_row_sum<T>(sh.c_b[kb][lane], sh.fac_h, r.acc);
            const uint64_t ovo = slice_word(sh.ovo_b[kb][lane]), ovt = slice_word(sh.ovt_b[kb][lane]);
            ov |= ((r.acc & ovt) | (~r.acc & ovo)) != 0;
        }
    }
    sh.h_corr[lane] = corr;
    const uint64_t ob = __ballot(ov);
    if (lane == 0) sh.h_ov = ob;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) __hip_atomic_store(&sh.h_done, t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

#ifdef MC_TIMELINE
constexpr int kTlSlots = 32;  // diagnostic build: stamps per group in the dE trace buffer
#endif

template <typename T, int M, bool DA>
__device__ __forceinline__ void chain_step(SweepShared<T, M, DA>& sh, const ChainDesc& cd,
                                           __amdgpu_buffer_rsrc_t pos_r, __amdgpu_buffer_rsrc_t rec_r,
                                           int64_t g_begin, int64_t g, int t,
                                           T xi, T yi, T zi, T txi, T tyi, T tzi, const MoverInputs& mi, bool da_active,
                                           const Ctl& ctl, WgCounters& ctr)
{
    const int lane = threadIdx.x & 63;
    const int n = cd.n, nb = cd.nb, band = cd.band;
    const int npad = nb * kGroup;
    const int64_t s = g / nb;
    const int b = (int)(g - s * nb);
    const int ion = b * kGroup + lane;
    const bool valid = ion < n;
    const bool wall = mi.wall;
    const double thr = mi.thr;

#ifdef MC_TIMELINE
    // diagnostic build only: per-group wall-clock stamps in the dE trace buffer
    uint64_t tl0 = wall_clock64(), tl1 = 0, tl2 = 0, tl3 = 0, tl4 = 0, tl5 = 0, tl6 = 0, tlA = 0, tlB = 0, tlC = 0;
    uint64_t tlE = 0, tlR = 0, tlN = 0, tlN1 = 0;  // early check done, first row sum done, row sums (in the first solve)
#endif
    // the waves' partial sums
    wait_lds_at_least(&sh.ready, M, ctl);
#ifdef MC_TIMELINE
    tl1 = wall_clock64();
#endif
    double St = 0.0;
    constexpr int LC = SweepShared<T, M, DA>::LC;
    uint64_t ovo = 0, ovt = 0, ovob[LC], ovtb[LC];
    bool ovb = false;
    T cp = 0, cn = 0;
#pragma unroll
    for (int w = 0; w < M; ++w) {
        cp += sh.part_pn[w][0][lane];
        cn += sh.part_pn[w][1][lane];
        St += sh.part_s[w][lane];
        ovb |= ((sh.part_ov[w] >> lane) & 1ull) != 0;
    }
    ovo = slice_word(sh.ovo_own[lane]);
    ovt = slice_word(sh.ovt_own[lane]);
#pragma unroll
    for (int kb = 0; kb < LC; ++kb) {
        ovob[kb] = slice_word(sh.ovo_b[kb][lane]);
        ovtb[kb] = slice_word(sh.ovt_b[kb][lane]);
    }

#ifdef MC_TIMELINE
    tlA = wall_clock64();
#endif
    // Delayed acceptance (two-stage rule): a move without a conflict passes
    // stage 1 when dEh <= 0 or u3 < exp(-dEh), i.e. dEh < thr, and is then
    // accepted when dE - dEh <= 0 or u2 < exp(-(dE - dEh)), i.e. when
    // dE <= dEh or dE < dEh - log(u2).  The plain rule is the special case
    // shift = 0, thr_eff = thr; a stage-1 rejection sets both to -inf.
    double shift = 0.0, thr_eff = thr, deh = 0.0;
    bool conflict = false, da_lane = false, s1_rej = false;
    if constexpr (DA) {
        uint64_t cm = 0;
#pragma unroll
        for (int w = 0; w < M; ++w) cm |= sh.part_conf[w];
        conflict = ((cm >> lane) & 1ull) != 0;
        if (da_active && valid && !conflict) {
            da_lane = true;
            deh = sh.deh[lane];
            if (deh <= 0.0 || deh < thr) {
                const uint4 w2 = move_words(cd.seed, cd.chain_id, (uint32_t)s, (uint32_t)ion, 2u);
                shift = deh;
                thr_eff = deh - log(accept_uniform(w2.x));
            } else {
                s1_rej = true;
                shift = thr_eff = -1.0e300;
            }
        }
    }

    // ---- decisions.  dE = lB q (St + sum_kb corr_{g-1-kb} + own): the band
    // corrections and the own-group term stay unknown until the accept bits
    // of groups g-band..g-1 and of this group are known, but they are bounded
    // by the sums of their negative and positive candidate terms.  When the
    // threshold lies outside every lane's interval (with a margin far larger
    // than the rounding of these sums) and no hard-core overlap can flip, the
    // group's decisions are certain and are published before the band
    // groups' accept masks have even arrived; the exact dE follows.
    // Otherwise: solve the sequential rule's fixed point for a guess of the
    // pending masks, then correct it as the true masks arrive (below).
    __builtin_amdgcn_s_setprio(3);
    const double lq = mi.lq;
    const bool can = valid && !wall && !ovb;
    uint64_t acc = 0;
    double dE = 0.0;
    bool dec = false;
    int it = 0;
    bool early = false;
    {
        const double lo = St + (double)cn;
        const double hi = St + (double)cp;
        const double e_lo = lq >= 0 ? lq * lo : lq * hi;
        const double e_hi = lq >= 0 ? lq * hi : lq * lo;
        const double span = (double)(cp - cn);
        const double margin = fabs(lq) * (1e-4 * span + 1e-9 * (fabs(St) + 1.0)) + 1e-12;
        uint64_t ov_sure = 0, ov_flip = ovo ^ ovt;
#pragma unroll
        for (int kb = 0; kb < LC; ++kb) {
            ov_sure |= ovob[kb] & ovtb[kb];
            ov_flip |= ovob[kb] ^ ovtb[kb];
        }
        const bool reject_sure = !can || s1_rej || ov_sure != 0 || (ovo & ovt) != 0;
        const bool accept_sure = !reject_sure && ov_flip == 0 && e_hi < thr_eff - margin;
        const bool sure = reject_sure || accept_sure || (ov_flip == 0 && e_lo >= thr_eff + margin);
        if (__ballot(!sure) == 0ull) {
            early = true;
            acc = __ballot(accept_sure);
            dec = accept_sure;
            publish_group<T>(rec_r, pos_r, g, s, npad, ion, acc, dec, xi, yi, zi, txi, tyi, tzi);
#ifdef MC_TIMELINE
            tl3 = wall_clock64();
#endif
        }
    }
#ifdef MC_TIMELINE
    tlB = tlE = wall_clock64();
#endif
    // One evaluation of the sequential rule inside the group given an accept
    // mask `a` of the own group (row sum `own`): the decisions every lane
    // would take.  Lane i depends on lanes j < i only (the system is lower
    // triangular), so the iteration a <- rule(a) reaches the one fixed point
    // from any start within kGroup + 1 evaluations, and a mask that the rule
    // reproduces is that fixed point.
    auto rule = [&](double Sx, bool canx, uint64_t a, T own) {
        const bool ovown = ((a & ovt) | (~a & ovo)) != 0;
        dE = lq * (Sx + (double)own);
        dec = canx && !ovown && (dE <= shift || dE < thr_eff);
        return __ballot(dec);
    };
    // iterates from mask a (row sum own) to the fixed point; a step that
    // flips few bits updates the row sum by them instead of summing the row
    auto solve = [&](double Sx, bool canx, uint64_t a, T own) {
        uint64_t na = rule(Sx, canx, a, own);
        ++it;
        while (na != a && it <= kGroup + 2) {
            if (__popcll(na ^ a) <= kFewFlips)
                own = row_sum_update<T>(sh.c_own[lane], own, a, na);
            else
                own = masked_row_sum<T>(sh.c_own[lane], sh.fac, na);
#ifdef MC_TIMELINE
            if (tlN++ == 0) tlR = wall_clock64();
#endif
            a = na;
            na = rule(Sx, canx, a, own);
            ++it;
        }
        acc = na;
        return own;
    };
    double corr = 0.0;  // band corrections of groups g-LC..g-1, oldest first
#ifdef MC_TIMELINE
    tlC = wall_clock64();
#endif
    // groups g-LC..g-2 come from the helper wave: their sum, in the same
    // order, and the overlap ballot
    auto helper_part = [&]() {
        wait_lds_at_least(&sh.h_done, t + 1, ctl);
        corr = sh.h_corr[lane];
        ovb |= ((sh.h_ov >> lane) & 1ull) != 0;
    };
    // group g-1's correction, added to corr once its mask arrives
    auto g1_part = [&]() {
        const GroupRec r = wait_rec(rec_r, g - 1, ctl);
#ifdef MC_TIMELINE
        tl2 = wall_clock64();
#endif
        corr += (double)masked_row_sum<T>(sh.c_b[0][lane], sh.fac, r.acc);
        ovb |= ((r.acc & ovtb[0]) | (~r.acc & ovob[0])) != 0;
    };
    if (early) {
        if (LC > 1 && band >= 2) helper_part();
        if (band >= 1) g1_part();
        // exact energy change of the (already decided) trials
        const T own = acc ? masked_row_sum<T>(sh.c_own[lane], sh.fac, acc) : (T)0;
        dE = lq * ((St + corr) + (double)own);
        it = 1;
    } else {
        // While the accept masks of the chain band groups are on their way,
        // the fixed point is solved for a guess of them (every move
        // rejected).  As the true corrections come in (the helper's, then
        // g-1's) one evaluation confirms the solution, or the iteration goes
        // on from it.
        uint64_t pend = 0;  // overlaps with old positions of pending groups (rejected guess)
#pragma unroll
        for (int kb = 0; kb < LC; ++kb)
            if (kb < band) pend |= ovob[kb];
        T own = solve(St, valid && !wall && !ovb && pend == 0, 0, (T)0);
        if (LC > 1 && band >= 2) {
#ifdef MC_TIMELINE
            tlC = wall_clock64();  // end of the first solve
            tlN1 = tlN;
#endif
            helper_part();
#ifdef MC_TIMELINE
            tlB = wall_clock64();  // helper's part in
#endif
            pend = ovob[0];
            it = 0;
            own = solve(St + corr, valid && !wall && !ovb && pend == 0, acc, own);
        }
        if (band >= 1) {
#ifdef MC_TIMELINE
            tl6 = wall_clock64();
#endif
            g1_part();
#ifdef MC_TIMELINE
            tl4 = wall_clock64();
#endif
            it = 0;
            own = solve(St + corr, valid && !wall && !ovb, acc, own);
        }
#ifdef MC_TIMELINE
        if (band < 1) tl2 = tl4 = tl6 = wall_clock64();
        tl5 = wall_clock64();
#endif
        (void)own;
        publish_group<T>(rec_r, pos_r, g, s, npad, ion, acc, dec, xi, yi, zi, txi, tyi, tzi);
#ifdef MC_TIMELINE
        tl3 = wall_clock64();
#endif
    }
    const uint64_t m_ov = __ballot(valid && !wall && (ovb || ((acc & ovt) | (~acc & ovo)) != 0));

    // ---- release the hand-off buffer
    if (lane == 0) {
        __hip_atomic_store(&sh.ready, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __hip_atomic_store(&sh.consumed, t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    __builtin_amdgcn_s_setprio(0);
#ifdef MC_TIMELINE
    if (lane == 0 && kTlSlots * (g + 1) <= cd.trace_cap) {
        uint64_t* tl = (uint64_t*)cd.trace_de + kTlSlots * g;
        tl[0] = tl0;
        tl[1] = tl1;
        tl[2] = tl2;
        tl[3] = tl3;
        {
            tl[4] = tl4;
            tl[5] = tl5;
            tl[6] = tl6;
            tl[7] = (uint64_t)it;
            tl[8] = tlA;
            tl[9] = tlB;
            tl[10] = tlC;
            tl[29] = tlE;
            tl[30] = tlR;
            tl[31] = tlN1;
        }
    }
#endif

    const double de_group = __shfl(wave_sum(dec ? dE : 0.0), 0, 64);
#ifndef MC_TIMELINE
    if (valid) {
#else
    if (false) {
#endif
        const int64_t mv = s * (int64_t)n + ion;
        if (mv < cd.trace_cap) {
            cd.trace_acc[mv] = (uint8_t)dec;
            cd.trace_de[mv] = dE;
        }
    }
    if (lane == 0) cd.de_group[g - g_begin] = de_group;
    const uint64_t m_wall = __ballot(valid && wall);
    const uint64_t m_valid = __ballot(valid);
    ctr.moves += __popcll(m_valid);
    ctr.acc += __popcll(acc);
    ctr.wall += __popcll(m_wall);
    ctr.ov += __popcll(m_ov);
    ctr.iters += it;
    ctr.early += early ? 1 : 0;
    if constexpr (DA) {
        const bool ov_final = ((m_ov >> lane) & 1ull) != 0;
        const bool passed = da_lane && !s1_rej && !wall && !ov_final;
        ctr.da_moves += __popcll(__ballot(da_lane));
        ctr.conflicts += __popcll(__ballot(valid && conflict));
        ctr.s1_rej += __popcll(__ballot(s1_rej));
        ctr.s1_pass += __popcll(__ballot(passed));
        ctr.s2_rej += __popcll(__ballot(passed && !dec));
        const int64_t mv = s * (int64_t)n + ion;
        if (valid && mv < cd.log_cap) {
            cd.log_de[mv] = dE;
            cd.log_deh[mv] = deh;
            cd.log_flags[mv] = (uint8_t)(0x80u | (uint32_t)wall | ((uint32_t)ov_final << 1) |
                                         ((uint32_t)conflict << 2) | ((uint32_t)s1_rej << 3) |
                                         ((uint32_t)(passed && !dec) << 4) | ((uint32_t)dec << 5));
        }
    }
}

// Occupancy asked of the compiler (waves per SIMD): two workgroups per CU.
// (the delayed-acceptance kernels take one wave per SIMD: their register use
// would otherwise spill; they run one workgroup per CU)
template <typename T, int M, bool DA = false>
constexpr int kWavesPerEU = DA ? 1 : (sizeof(T) == 4 ? (M == 8 ? 4 : 2) : 1);

// Squared distance in double, summed in the order x, y, z with no fused
// multiply-add: the neighbour-histogram bins and the conflict rule of the
// delayed-acceptance stage are decided on this value.
__device__ __forceinline__ double d2_exact(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return dx * dx + dy * dy + dz * dz;
}

// Adds a neighbour at squared distance d2 to byte bin (pos, like/unlike, k)
// of mover `lane`'s histogram (four byte counters per LDS word).
template <typename SH>
__device__ __forceinline__ void da_hist_add(SH& sh, const ChainDesc& cd, int lane, int pos, bool unlike, double d2) {
    if (!(d2 < cd.da_rc * cd.da_rc)) return;
    const int k = (int)__builtin_floor(__builtin_sqrt(d2) / cd.da_dr);
    if (k >= kDaBins) return;
    const int byte = pos * kDaIn + (unlike ? kDaBins : 0) + k;
    atomicAdd(&sh.hist[lane][byte >> 2], 1u << (8 * (byte & 3)));
}

__device__ __forceinline__ float bf16_round(float v) {
    uint32_t b = __builtin_bit_cast(uint32_t, v);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return __builtin_bit_cast(float, b & 0xFFFF0000u);
}

// Delayed-acceptance stage of one target group, run by all 4 waves between
// the chain wave's release of the hand-off buffer and the next hand-off:
// logs the movers' histograms, evaluates the network eps at both positions
// of every mover and leaves dEh = l_B (eps(trial) - eps(old)) in sh.deh, then
// clears the histograms.  Both hidden layers run on the matrix cores as
// [128 rows x 128] x [128 x 128] bfloat16 products with float sums
// (v_mfma_f32_32x32x8bf16_1k): row r = 64 * position + mover, wave w takes
// rows 32 w .. 32 w + 31 and all four 32-column tiles (the matrices are
// read from LDS, where the kernel put them at its start); lane l holds
// A[l % 32][4 (l / 32) + v], B[4 (l / 32) + v][l % 32] and
// D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].  Hidden activations are
// rounded to bfloat16.
typedef short da_bf16x4 __attribute__((ext_vector_type(4)));
typedef float da_f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short bf16_bits(float v) {
    return (short)(__builtin_bit_cast(uint32_t, bf16_round(v)) >> 16);
}

template <typename T, int M>
__device__ __forceinline__ void da_network(SweepShared<T, M, true>& sh, const ChainDesc& cd, int wave, int lane,
                                           bool da_on, int64_t mv, bool valid, int64_t g) {
#ifdef MC_TIMELINE
    // diagnostic build only: stamps of the network phase after the chain stamps
    uint64_t* tln = (uint64_t*)cd.trace_de + kTlSlots * g + 11;
    const bool stamp = wave == 0 && lane == 0 && kTlSlots * (g + 1) <= cd.trace_cap;
    if (stamp) tln[0] = wall_clock64();
#else
    (void)g;
#endif
    static_assert(M == 4, "the network phase assumes 4 waves");
    constexpr int WW = 64 / M;        // histogram words logged and cleared per wave
    constexpr int H1S = 2 * kDaHid + 2;  // row stride in bfloat16 values (odd word stride)
    static_assert(sizeof(sh.c_own) + sizeof(sh.c_b) >= sizeof(uint16_t) * kGroup * H1S,
                  "hidden activations must fit in the candidate space");
    __syncthreads();  // every histogram add of this target is done
#ifdef MC_TIMELINE
    if (stamp) tln[1] = wall_clock64();
#endif
    if (valid && mv < cd.log_cap) {
        uint32_t* dst = cd.log_feat + mv * 64;
#pragma unroll
        for (int k = 0; k < WW; ++k) dst[wave * WW + k] = sh.hist[lane][wave * WW + k];
    }
    uint16_t* h1 = sh.h1();
    float* outs = &sh.part_out[0][0][0];  // [128] network outputs by row
    // biases and the last layer are read through a buffer resource: its loads
    // wait on the vector-memory counter only, so the LDS traffic of this
    // phase never waits for them (generic-pointer loads count on both)
    const __amdgpu_buffer_rsrc_t wr = make_rsrc((void*)cd.da_w, (uint32_t)(sizeof(float) * kDaParams));
    auto wload = [&](int k) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(wr, (uint32_t)(4 * k), 0, 0));
    };
    constexpr int oB1 = kDaIn * kDaHid, oB2 = oB1 + kDaHid + kDaHid * kDaHid, oW3 = oB2 + kDaHid;
    // B fragment (4 consecutive inputs k of hidden unit `unit`) of layer `layer`
    const __amdgpu_buffer_rsrc_t wbr = make_rsrc((void*)cd.da_w1b, (uint32_t)(4u * kDaIn * kDaHid));
    auto bfrag = [&](int layer, int unit, int k) -> uint2 {
        if constexpr (SweepShared<T, M, true>::kWtsLds)
            return *reinterpret_cast<const uint2*>(&sh.wts[layer * kDaHid + unit][k]);
        else
            return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(
                                                 wbr, (uint32_t)(2 * ((layer * kDaHid + unit) * kDaIn + k)), 0, 0));
    };
    // this lane's A row
    const int arow = wave * 32 + (lane & 31);
    const int amover = arow & 63, apos = arow >> 6;
    const int kq = (lane >> 5) * 4;
    // B fragments of a layer: the transposed bfloat16 matrix gives each lane
    // its four consecutive k of column 32 t + l % 32 in one 8-byte load; all
    // 64 loads of a layer are issued before its products
    const int bcol = lane & 31;
    if (da_on) {
        da_f32x16 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
#pragma unroll 2
        for (int j = 0; j < kDaIn / 8; ++j) {
            const uint32_t w = sh.hist[amover][apos * 32 + (8 * j + kq) / 4];
            da_bf16x4 a;
#pragma unroll
            for (int v = 0; v < 4; ++v) a[v] = bf16_bits((float)((w >> (8 * v)) & 0xFFu));
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint2 bv = bfrag(0, 32 * t + bcol, 8 * j + kq);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, __builtin_bit_cast(da_bf16x4, bv), acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = 32 * t + (lane & 31);
            const float bias = wload(oB1 + col);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = wave * 32 + 8 * (i / 4) + 4 * (lane >> 5) + (i % 4);
                const float z = acc[t][i] + bias;
                h1[(r & 63) * H1S + (r >> 6) * kDaHid + col] = (uint16_t)bf16_bits(z > 0.f ? z : 0.f);
            }
        }
    }
    __syncthreads();  // first hidden layer complete
#ifdef MC_TIMELINE
    if (stamp) tln[2] = wall_clock64();
#endif
#pragma unroll
    for (int k = 0; k < WW; ++k) sh.hist[lane][wave * WW + k] = 0u;
    if (da_on) {
        da_f32x16 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
        const uint16_t* arow_h = h1 + amover * H1S + apos * kDaHid;
#pragma unroll 2
        for (int j = 0; j < kDaHid / 8; ++j) {
            const uint32_t lo = *reinterpret_cast<const uint32_t*>(arow_h + 8 * j + kq);
            const uint32_t hi = *reinterpret_cast<const uint32_t*>(arow_h + 8 * j + kq + 2);
            uint2 av;
            av.x = lo;
            av.y = hi;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint2 bv = bfrag(1, 32 * t + bcol, 8 * j + kq);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(da_bf16x4, av),
                                                                  __builtin_bit_cast(da_bf16x4, bv), acc[t], 0, 0, 0);
            }
        }
        // last layer: sum over the columns of bf16(relu(Z2 + b2)) w3
        float part[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) part[i] = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = 32 * t + (lane & 31);
            const float bias = wload(oB2 + col), wc = wload(oW3 + col);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float z = acc[t][i] + bias;
                part[i] = __builtin_fmaf(bf16_round(z > 0.f ? z : 0.f), wc, part[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
#pragma unroll
            for (int d = 1; d < 32; d <<= 1) part[i] += __shfl_xor(part[i], d, 64);
        }
        if ((lane & 31) == 0) {
#pragma unroll
            for (int i = 0; i < 16; ++i) outs[wave * 32 + 8 * (i / 4) + 4 * (lane >> 5) + (i % 4)] = part[i];
        }
    }
    __syncthreads();  // outputs complete; the candidate space is free again
#ifdef MC_TIMELINE
    if (stamp) tln[3] = wall_clock64();
#endif
    if (da_on && wave == 0) {
        const float b3 = wload(kDaParams - 1);
        const float o0 = b3 + outs[lane], o1 = b3 + outs[64 + lane];
        sh.deh[lane] = cd.lB * ((double)o1 - (double)o0);
    }
}

// One workgroup's share of one chain for sweeps s0 .. s0 + n_sweeps - 1:
// the targets g = k_wg (mod the chain's workgroup count).
template <typename T, int M, bool UNIFORM_SIGMA, bool DA>
__device__ __forceinline__ void sweep_chain(SweepShared<T, M, DA>& sh, const ChainDesc& cd, const int k_wg,
                                            uint32_t s0, int32_t n_sweeps, const Ctl& ctl)
{
    using T4 = typename Prec<T>::T4;
    using IO = PosIO<T>;
    constexpr int P = kGroup / M;
    constexpr int KB = kChainBand<T, M, UNIFORM_SIGMA, DA>;
    constexpr int LC = SweepShared<T, M, DA>::LC;
    static_assert(KB >= LC, "the chain step's band slots are band groups");
    using SB = typename SliceBits<P>::type;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int nb = cd.nb, band = cd.band;
    const int npad = nb * kGroup;
    const __amdgpu_buffer_rsrc_t pos_r = make_rsrc(cd.pos, (uint32_t)(2u * npad * IO::kBytes));
    const __amdgpu_buffer_rsrc_t rec_r = make_rsrc(cd.rec, (uint32_t)(kRing * sizeof(GroupRec)));
    const T* __restrict__ charge = (const T*)cd.charge;
    const T* __restrict__ half = (const T*)cd.half;
    const T D = (T)cd.D;
    const T hu = (T)cd.half_uniform;
    const int64_t g_begin = (int64_t)s0 * nb;
    const int64_t g_end = g_begin + (int64_t)n_sweeps * nb;

    if (threadIdx.x == 0) {
        // one store each (a merged 64-bit store of zeros has kept a register
        // pair live through the whole kernel)
        __hip_atomic_store(&sh.ready, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(&sh.consumed, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(&sh.h_done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k_wg == 0) cd.clk[0] = wall_clock64();
    }
    if constexpr (DA) {
        static_assert(sizeof(sh.hist) == sizeof(uint32_t) * kGroup * 65, "histogram rows");
        for (int k = threadIdx.x; k < kGroup * 65; k += 64 * M) (&sh.hist[0][0])[k] = 0u;
    }
    // the delayed-acceptance switch is constant during a launch (the drift
    // monitor changes it between launches)
    const bool da_on = DA && cd.da != nullptr && cd.da->active != 0 && cd.da_w != nullptr;
    if constexpr (SweepShared<T, M, DA>::kWtsLds) {
        if (da_on) {
            static_assert(kDaIn == kDaHid, "both matrices are 128 x 128");
            for (int k = threadIdx.x; k < 2 * kDaHid * kDaIn / 4; k += 64 * M) {
                const int row = k / (kDaIn / 4), c4 = k % (kDaIn / 4);  // row of the two stacked matrices
                const uint16_t* src = row < kDaHid ? cd.da_w1b + row * kDaIn : cd.da_w2b + (row - kDaHid) * kDaIn;
                *reinterpret_cast<uint2*>(&sh.wts[row][4 * c4]) = *reinterpret_cast<const uint2*>(src + 4 * c4);
            }
        }
    }
    __syncthreads();

    WgCounters ctr;
    {
        int t = 0;
        for (int64_t g = g_begin + k_wg; g < g_end; g += cd.wg_count, ++t) {
            const int64_t s = g / nb;
            const int b = (int)(g - s * nb);
            const int ion = b * kGroup + lane;

            // the movers: old position = result of the group's previous trial
            const auto xr = IO::load_valid(pos_r, (uint32_t)(((s - 1) & 1) * npad + ion), (uint32_t)(s - 1),
                                           true, ctl);
            const T xi = xr.x, yi = xr.y, zi = xr.z, qi = charge[ion];
            const uint4 wd = move_words(cd.seed, cd.chain_id, (uint32_t)s, (uint32_t)ion);
            const T txi = trial_coord(xi, wd.x, D), tyi = trial_coord(yi, wd.y, D),
                    tzi = trial_coord(zi, wd.z, D);
            const T hi = UNIFORM_SIGMA ? hu : half[ion];
            MoverInputs mi{};
            if (wave == 0) mi = mover_inputs(cd, ion, qi, txi, tyi, tzi, wd.w);

#ifdef MC_TIMELINE
            if (!DA && wave == 0 && lane == 0 && kTlSlots * (g + 1) <= cd.trace_cap)
                ((uint64_t*)cd.trace_de)[kTlSlots * g + 11] = wall_clock64();
#endif
            double S = 0.0;     // sum_j q_j (1/|x~_i - x_j| - 1/|x_i - x_j|)
            bool ov = false;    // overlap with a partner whose position is final
            bool conf = false;  // delayed acceptance: a pending partner is near (conflict rule)

            // ---- own group: both outcomes of every partner j != i
            T c_own[P];
            SB ovo_own = 0, ovt_own = 0;
            {
                if (lane >= wave * P && lane < wave * P + P) {
                    const int m = lane - wave * P;
                    sh.st_old[wave][m] = mk4<T>(xi, yi, zi, qi);
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
                    const T tt = pt.w * (Prec<T>::rinv(d2tt) - Prec<T>::rinv(d2t));
                    const bool oo = d2ot < s_ij * s_ij, ot = d2tt < s_ij * s_ij;
                    if (j > lane) {
                        sf += o;
                        ov |= oo;
                        c_own[m] = 0;
                    } else if (j < lane) {
                        sf += o;
                        c_own[m] = tt - o;
                        ovo_own |= (SB)((SB)oo << m);
                        ovt_own |= (SB)((SB)ot << m);
                    } else {
                        c_own[m] = 0;
                    }
                    if constexpr (DA) {
                        if (j > lane) {  // not moved yet: its current position counts
                            const double qq = (double)po.w * (double)qi;
                            if (qq != 0.0) {
                                da_hist_add(sh, cd, lane, 0, qq < 0.0, d2_exact(xi, yi, zi, po.x, po.y, po.z));
                                da_hist_add(sh, cd, lane, 1, qq < 0.0, d2_exact(txi, tyi, tzi, po.x, po.y, po.z));
                            }
                        } else if (j < lane) {  // decision pending: conflict rule
                            const double rc2 = cd.da_rc * cd.da_rc;
                            conf |= d2_exact(xi, yi, zi, po.x, po.y, po.z) < rc2 ||
                                    d2_exact(xi, yi, zi, pt.x, pt.y, pt.z) < rc2 ||
                                    d2_exact(txi, tyi, tzi, po.x, po.y, po.z) < rc2 ||
                                    d2_exact(txi, tyi, tzi, pt.x, pt.y, pt.z) < rc2;
                        }
                    }
                }
                S += (double)sf;
                wave_lds_sync();
            }

            // ---- band groups g-1..g-band: both outcomes, evaluated ahead of their decisions
            T c_band[KB][P];
            SB ovo_band[KB], ovt_band[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                ovo_band[kb] = 0;
                ovt_band[kb] = 0;
#pragma unroll
                for (int m = 0; m < P; ++m) c_band[kb][m] = 0;
                if (kb < band) {
                    const int64_t gp = g - 1 - kb;
                    const int64_t sp = floor_div(gp, nb);
                    const int bp = (int)(gp - sp * nb);
                    // old position of j = result of its trial one sweep before
                    const int j = bp * kGroup + wave * P + (lane < P ? lane : 0);
                    const auto pr = IO::load_valid(pos_r, (uint32_t)(((sp - 1) & 1) * npad + j),
                                                   (uint32_t)(sp - 1), lane < P, ctl);
                    if (lane < P) {
                        const T qj = charge[j];
                        const uint4 wj = move_words(cd.seed, cd.chain_id, (uint32_t)sp, (uint32_t)j);
                        sh.st_old[wave][lane] = mk4<T>(pr.x, pr.y, pr.z, qj);
                        sh.st_new[wave][lane] = mk4<T>(trial_coord((T)pr.x, wj.x, D), trial_coord((T)pr.y, wj.y, D),
                                                        trial_coord((T)pr.z, wj.z, D), qj);
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
                        const T tt = pt.w * (Prec<T>::rinv(d2tt) - Prec<T>::rinv(d2t));
                        sf += o;
                        c_band[kb][m] = tt - o;
                        ovo_band[kb] |= (SB)((SB)(d2ot < s_ij * s_ij) << m);
                        ovt_band[kb] |= (SB)((SB)(d2tt < s_ij * s_ij) << m);
                        if constexpr (DA) {
                            if (gp >= 0) {  // decision pending: conflict rule
                                const double rc2 = cd.da_rc * cd.da_rc;
                                conf |= d2_exact(xi, yi, zi, po.x, po.y, po.z) < rc2 ||
                                        d2_exact(xi, yi, zi, pt.x, pt.y, pt.z) < rc2 ||
                                        d2_exact(txi, tyi, tzi, po.x, po.y, po.z) < rc2 ||
                                        d2_exact(txi, tyi, tzi, pt.x, pt.y, pt.z) < rc2;
                            } else {
                                // before the chain's first group: nothing moved, the
                                // ion sits at its starting position, which counts
                                const double qq = (double)po.w * (double)qi;
                                if (qq != 0.0) {
                                    da_hist_add(sh, cd, lane, 0, qq < 0.0, d2_exact(xi, yi, zi, po.x, po.y, po.z));
                                    da_hist_add(sh, cd, lane, 1, qq < 0.0, d2_exact(txi, tyi, tzi, po.x, po.y, po.z));
                                }
                            }
                        }
                    }
                    S += (double)sf;
                    wave_lds_sync();
                }
            }

            // the candidates of group g-1 and of the own group for the chain
            // wave: overlap slices, the sums of their positive and negative
            // parts (bounds of the corrections still unknown) and the rows
            auto hand_off_candidates = [&]() {
                sh.ovo_own[lane][wave] = ovo_own;
                sh.ovt_own[lane][wave] = ovt_own;
#pragma unroll
                for (int kb = 0; kb < LC; ++kb) {
                    sh.ovo_b[kb][lane][wave] = ovo_band[kb];
                    sh.ovt_b[kb][lane][wave] = ovt_band[kb];
                }
                T cp = 0, cn = 0;
#pragma unroll
                for (int m = 0; m < P; ++m) {
#pragma unroll
                    for (int kb = 0; kb < LC; ++kb) {
                        cp += c_band[kb][m] > 0 ? c_band[kb][m] : (T)0;
                        cn += c_band[kb][m] < 0 ? c_band[kb][m] : (T)0;
                    }
                    cp += c_own[m] > 0 ? c_own[m] : (T)0;
                    cn += c_own[m] < 0 ? c_own[m] : (T)0;
                }
                sh.part_pn[wave][0][lane] = cp;
                sh.part_pn[wave][1][lane] = cn;
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    sh.c_own[lane][wave * P + m] = c_own[m];
#pragma unroll
                    for (int kb = 0; kb < LC; ++kb)
                        sh.c_b[kb][lane][wave * P + m] = c_band[kb][m];  // zero beyond the band
                }
            };
            if constexpr (!DA) {
                // complete from here on: handed off now, off the critical
                // path, once the chain wave has released the previous target
                // (the delayed-acceptance kernels reuse this LDS for the
                // network and hand off at the end)
                wait_lds_at_least(&sh.consumed, t, ctl);
                hand_off_candidates();
            }

            // ---- decided partner groups g-nb+1 .. g-band-1, in stream order.  The next
            // tile is loaded speculatively while this one is computed (float path); a
            // record whose version is not the expected one yet is loaded again.
            // A round of tiles covers KD decided groups, each shared by M / KD
            // waves with PD partners a wave: KD = 1 in most kernels (every
            // wave a P-partner slice of every group), KD = 8 in the eight-wave
            // float kernels (every wave one group whole).
            {
                constexpr int PD = kDecidedSlice<T, M, DA>;
                constexpr int KD = PD / P;
                static_assert(KD * P == PD && M % KD == 0 && (!DA || KD == 1), "decided tiles");
                const int64_t g_last = g - band - 1;
                int64_t sp = (b + 1 < nb) ? s - 1 : s;   // sweep and group of g-nb+1
                int bp = (b + 1 < nb) ? b + 1 : 0;
                const int dphase = wave / (M / KD);      // this wave's first group: g-nb+1+dphase
                for (int k = 0; k < dphase; ++k)
                    if (++bp == nb) {
                        bp = 0;
                        ++sp;
                    }
                const int jl = (wave % (M / KD)) * PD + (lane < PD ? lane : 0);
                typename IO::Rec nxt{};
                bool have_next = false;
                // uniform diameters: overlap with any of these partners iff the
                // smallest trial distance is below the contact distance
                T d2t_min = (T)3.0e38;
                // a working-precision squared distance below this bound may be
                // below rc^2 exactly (the bound is a relative 1e-5 above it)
                const T rc2_wide = (T)(cd.da_rc * cd.da_rc * (1.0 + 1e-5));
                for (int64_t gp = g - nb + 1 + dphase; gp <= g_last; gp += KD) {
                    const int j = bp * kGroup + jl;
                    typename IO::Rec cur;
                    if (have_next && __ballot(lane < PD && nxt.ver != (uint32_t)sp) == 0ull)
                        cur = nxt;
                    else
                        cur = IO::load_valid(pos_r, (uint32_t)((sp & 1) * npad + j), (uint32_t)sp, lane < PD, ctl,
                                             g - gp > kPatientDistance);
#ifdef MC_TIMELINE
                    if (!DA && gp + KD > g_last && lane == 0 && kTlSlots * (g + 1) <= cd.trace_cap)
                        ((uint64_t*)cd.trace_de)[kTlSlots * g + (wave == 0 ? 14 : 24 + wave)] = wall_clock64();
#endif
                    // per-ion diameters: a slice whose partners all have one
                    // diameter (every slice but those at a species boundary)
                    // takes the running-minimum contact test of the uniform case
                    T hj0 = (T)0;
                    bool slice_uniform = true;
                    if (lane < PD) {
                        const bool lo = PD == P || lane < P;
                        const int ls = lo ? lane : lane - P;
                        (lo ? sh.st_old[wave] : sh.st_old2[wave])[ls] = mk4<T>(cur.x, cur.y, cur.z, charge[j]);
                        if (!UNIFORM_SIGMA) {
                            hj0 = half[j];
                            (lo ? sh.st_half[wave] : sh.st_half2[wave])[ls] = hj0;
                        }
                    }
                    if constexpr (!UNIFORM_SIGMA && !DA) {
                        const T hjl = hj0;
                        hj0 = __shfl(hjl, 0, 64);
                        slice_uniform = __ballot(lane < PD && hjl != hj0) == 0ull;
                    }
                    wave_lds_sync();
                    int bn = bp;
                    int64_t sn = sp;
                    for (int k = 0; k < KD; ++k)
                        if (++bn == nb) {
                            bn = 0;
                            ++sn;
                        }
                    have_next = false;
                    if constexpr (sizeof(T) == 4) {
                        if (gp + KD <= g_last) {
                            if (lane < PD) nxt = IO::load(pos_r, (uint32_t)((sn & 1) * npad + bn * kGroup + jl));
                            have_next = true;
                        }
                    }
                    T sf = 0;
                    uint32_t nearm = 0;  // delayed acceptance: partners possibly within rc
                    if constexpr (UNIFORM_SIGMA || DA) {
                        // P partners at a time (a loop, not unrolled, so that a
                        // round needs the registers of one P-partner slice)
#pragma nounroll
                        for (int c = 0; c < KD; ++c)
#pragma unroll
                        for (int mm = 0; mm < P; ++mm) {
                            const int m = c * P + mm;
                            const T4 p = c == 0 ? sh.st_old[wave][mm] : sh.st_old2[wave][(c - 1) * P + mm];
                            const T hj = UNIFORM_SIGMA ? hu
                                         : c == 0 ? sh.st_half[wave][mm] : sh.st_half2[wave][(c - 1) * P + mm];
                            const T s_ij = hi + hj;
                            const T d2 = Prec<T>::norm2(p.x - xi, p.y - yi, p.z - zi);
                            const T d2t = Prec<T>::norm2(p.x - txi, p.y - tyi, p.z - tzi);
                            sf = Prec<T>::fma(p.w, Prec<T>::rinv(d2t) - Prec<T>::rinv(d2), sf);
                            if (UNIFORM_SIGMA)
                                d2t_min = Prec<T>::min(d2t, d2t_min);
                            else
                                ov |= d2t < s_ij * s_ij;
                            if constexpr (DA) nearm |= (uint32_t)(Prec<T>::min(d2, d2t) < rc2_wide) << m;
                        }
                    } else {
                        // per-ion diameters: the contact test per pair, or as a
                        // running minimum of the trial distances for a slice
                        // with one diameter -- exact: min_j d2t_j < s^2 iff some
                        // d2t_j < s^2, with the one s = hi + hj the per-pair
                        // test forms for every partner of the slice
                        auto slice_terms = [&](auto per_pair_c) {
                            constexpr bool PER_PAIR = decltype(per_pair_c)::value;
                            T tmin = (T)3.0e38;
#pragma nounroll
                            for (int c = 0; c < KD; ++c)
#pragma unroll
                            for (int mm = 0; mm < P; ++mm) {
                                const T4 p = c == 0 ? sh.st_old[wave][mm] : sh.st_old2[wave][(c - 1) * P + mm];
                                const T d2 = Prec<T>::norm2(p.x - xi, p.y - yi, p.z - zi);
                                const T d2t = Prec<T>::norm2(p.x - txi, p.y - tyi, p.z - tzi);
                                sf = Prec<T>::fma(p.w, Prec<T>::rinv(d2t) - Prec<T>::rinv(d2), sf);
                                if constexpr (PER_PAIR) {
                                    const T s_ij = hi + (c == 0 ? sh.st_half[wave][mm]
                                                                : sh.st_half2[wave][(c - 1) * P + mm]);
                                    ov |= d2t < s_ij * s_ij;
                                } else {
                                    tmin = Prec<T>::min(d2t, tmin);
                                }
                            }
                            if constexpr (!PER_PAIR) {
                                const T s_ij = hi + hj0;
                                ov |= tmin < s_ij * s_ij;
                            }
                        };
                        if (slice_uniform)
                            slice_terms(std::false_type{});
                        else
                            slice_terms(std::true_type{});
                    }
                    if constexpr (DA) {
                        // rare: bin the near partners with exact double distances
                        if (__ballot(nearm != 0u) != 0ull) {
                            while (nearm) {
                                const int m = __builtin_ctz(nearm);
                                nearm &= nearm - 1u;
                                const T4 p = sh.st_old[wave][m];
                                const double qq = (double)p.w * (double)qi;
                                if (qq != 0.0) {
                                    da_hist_add(sh, cd, lane, 0, qq < 0.0, d2_exact(xi, yi, zi, p.x, p.y, p.z));
                                    da_hist_add(sh, cd, lane, 1, qq < 0.0, d2_exact(txi, tyi, tzi, p.x, p.y, p.z));
                                }
                            }
                        }
                    }
                    S += (double)sf;
                    wave_lds_sync();
                    bp = bn;
                    sp = sn;
                }
                if (UNIFORM_SIGMA) ov |= d2t_min < (hu + hu) * (hu + hu);
            }
#ifdef MC_TIMELINE
            if (!DA && wave == 0 && lane == 0 && kTlSlots * (g + 1) <= cd.trace_cap)
                ((uint64_t*)cd.trace_de)[kTlSlots * g + 12] = wall_clock64();
#endif

            // ---- delayed acceptance: the features are complete after the
            // last partner tile, so the network runs here, while the older
            // band groups' accept masks are still on their way
            if constexpr (DA) {
                wait_lds_at_least(&sh.consumed, t, ctl);
                const uint64_t cb = __ballot(conf);
                if (lane == 0) sh.part_conf[wave] = cb;
                da_network<T, M>(sh, cd, wave, lane, da_on, s * (int64_t)cd.n + ion, ion < cd.n, g);
            }

            // ---- band groups older than the chain step's: their accept
            // masks are out by now (published about one group after the last
            // partner tile); this wave's slice of their candidates becomes final
            GroupRec rb[KB];
#pragma unroll
            for (int kb = LC; kb < KB; ++kb)  // all loads in flight at once
                if (kb < band) rb[kb] = load_rec(rec_r, (uint32_t)((g - 1 - kb) & (kRing - 1)));
#pragma unroll
            for (int kb = KB - 1; kb >= LC; --kb) {
                if (kb < band) {
                    const GroupRec r = rb[kb].tag == (uint32_t)(g - kb) ? rb[kb] : wait_rec(rec_r, g - 1 - kb, ctl);
                    const uint32_t a = (uint32_t)(r.acc >> (wave * P));
                    T sf = 0;
                    SB hit = 0;
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const bool am = ((a >> m) & 1u) != 0;
                        sf += am ? c_band[kb][m] : (T)0;
                        hit |= am ? (ovt_band[kb] & (SB)(1u << m)) : (ovo_band[kb] & (SB)(1u << m));
                    }
                    S += (double)sf;
                    ov |= hit != 0;
                }
            }

#ifdef MC_TIMELINE
            if (!DA && lane == 0 && kTlSlots * (g + 1) <= cd.trace_cap)
                ((uint64_t*)cd.trace_de)[kTlSlots * g + (wave == 0 ? 13 : 20 + wave)] = wall_clock64();
#endif
            // ---- hand off to the chain wave once it has released the previous target
            if constexpr (DA) hand_off_candidates();
            sh.part_s[wave][lane] = S;
            {
                const uint64_t ob = __ballot(ov);
                if (lane == 0) sh.part_ov[wave] = ob;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0)
                __hip_atomic_fetch_add(&sh.ready, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#ifdef MC_TIMELINE
            if (!DA && lane == 0 && wave < 4 && kTlSlots * (g + 1) <= cd.trace_cap)
                ((uint64_t*)cd.trace_de)[kTlSlots * g + 16 + wave] = wall_clock64();
#endif

            // ---- wave 1 helps with the older chain band groups, wave 0
            // finishes the group: decisions and publication
            if constexpr (LC > 1) {
                if (wave == 1 && band >= 2) {
                    band_helper<T, M, DA>(sh, rec_r, g, t, band, ctl);
#ifdef MC_TIMELINE
                    if (lane == 0 && kTlSlots * (g + 1) <= cd.trace_cap)
                        ((uint64_t*)cd.trace_de)[kTlSlots * g + 28] = wall_clock64();
#endif
                }
            }
            if (wave == 0) {
                chain_step<T, M, DA>(sh, cd, pos_r, rec_r, g_begin, g, t, xi, yi, zi, txi, tyi, tzi, mi, da_on,
                                     ctl, ctr);
                if (g == g_end - 1 && lane == 0) cd.clk[1] = wall_clock64();
            }
        }
    }
    if (wave == 0 && lane == 0 && ctr.moves) {
        atomicAdd(&cd.stats[0], ctr.moves);
        atomicAdd(&cd.stats[1], ctr.acc);
        atomicAdd(&cd.stats[2], ctr.wall);
        atomicAdd(&cd.stats[3], ctr.ov);
        atomicAdd(&cd.stats[4], ctr.moves - ctr.acc - ctr.wall - ctr.ov);
        atomicAdd(&cd.stats[5], ctr.iters);
        atomicAdd(&cd.stats[6], ctr.early);
        if constexpr (DA) {
            atomicAdd(&cd.stats[7], ctr.da_moves);
            atomicAdd(&cd.stats[8], ctr.conflicts);
            atomicAdd(&cd.stats[9], ctr.s1_rej);
            atomicAdd(&cd.stats[10], ctr.s1_pass);
            atomicAdd(&cd.stats[11], ctr.s2_rej);
        }
    }
    __syncthreads();  // every wave is done with this chain's LDS state
}

// The sweep launch.  Workgroup w runs its items (chain, index of the
// workgroup among the chain's) one after another: a chain served by several
// workgroups is their only item; chains served by one workgroup alone may
// share it (a chain never waits on a workgroup busy with another chain).
template <typename T, int M, bool UNIFORM_SIGMA, bool DA = false>
__global__ void __launch_bounds__(64 * M)
__attribute__((amdgpu_waves_per_eu(kWavesPerEU<T, M, DA>)))
sweep_kernel(const ChainDesc* __restrict__ chains, const int2* __restrict__ wg_range,
             const int2* __restrict__ items, uint32_t s0, int32_t n_sweeps, Ctl ctl)
{
    __shared__ SweepShared<T, M, DA> sh;
    const int2 r = wg_range[blockIdx.x];
    for (int q = r.x; q < r.y; ++q) {
        const int2 it = items[q];
        sweep_chain<T, M, UNIFORM_SIGMA, DA>(sh, chains[it.x], it.y, s0, n_sweeps, ctl);
    }
}

// Running energy after each sweep of a launch, one block per chain:
// per-sweep totals of the group energy changes (each summed in group order),
// then a serial prefix from the previous running energy.  Deterministic.
__global__ void __launch_bounds__(256)
energy_scan_kernel(const ChainDesc* __restrict__ chains, int32_t n_sweeps, int64_t s0)
{
    const ChainDesc& cd = chains[blockIdx.x];
    const int nb = cd.nb;
    for (int s = threadIdx.x; s < n_sweeps; s += blockDim.x) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += cd.de_group[(int64_t)s * nb + b];
        cd.sweep_tot[s] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = *cd.e_state;
        for (int s = 0; s < n_sweeps; ++s) {
            e += cd.sweep_tot[s];
            if (s0 + s < cd.e_capacity) cd.e_series[s0 + s] = e;
        }
        *cd.e_state = e;
        // delayed-acceptance drift monitor: at the end of each window, the
        // stage-2 rejection rate of stage-1 passes against its training-time
        // value; above ref_rate + delta the chain falls back to the plain
        // test for good (from the next launch, i.e. the next window)
        DAState* da = cd.da;
        const int64_t s_end = s0 + n_sweeps;
        if (da != nullptr && da->window > 0 && s_end % da->window == 0) {
            const unsigned long long pass = cd.stats[10], rej = cd.stats[11];
            const unsigned long long dp = pass - da->win_pass0, dr = rej - da->win_rej0;
            if (dp > 0) da->last_rate = (double)dr / (double)dp;
            if (da->active && da->ref_rate >= 0.0 && (int64_t)dp >= da->min_count &&
                da->last_rate > da->ref_rate + da->delta) {
                da->active = 0;
                da->fallback_sweep = s_end;
            }
            da->win_pass0 = pass;
            da->win_rej0 = rej;
        }
    }
}

}  // namespace mcdev
