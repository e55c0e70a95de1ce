/*
 * mc.h -- C ABI of the MI355X (gfx950) exact-energy Metropolis Monte Carlo
 * library for primitive-model electrolytes.
 *
 * Method: Liang, Xing, Li, "A GPU-based Large-scale Monte Carlo Simulation
 * Method for Systems with Long-range Interactions" (arXiv:1602.05716).
 *   - Sec. 2: canonical Metropolis Monte Carlo with the sequential updating
 *     scheme -- one sweep (cycle) tries ions 0..N-1 once each, in order; a
 *     trial is accepted with probability min{1, exp(-beta dE)}, Eq.
 *     (trial-outcome).
 *   - Sec. 2, Eq. (Delta E_ij): dE of trial i is the exact sum over all other
 *     ions of the pair-energy change, using the current position of every
 *     other ion (already updated for j < i).  No cutoff, multipole or Ewald
 *     approximation.
 *   - Sec. 3.3: energies are accumulated in double precision; a hard-core
 *     overlap indicator rejects the trial.
 *   - Sec. 3.2, Algorithm 1: the trial displacement is uniform in a cube of
 *     side D centred on the ion.
 *   - Sec. 5.2: spherical hard-wall domain; total energy is monitored during
 *     equilibration; pair correlation functions g_ab(r) are measured on ions
 *     away from the wall.
 *
 * Model (readings of the paper, see the design notes): charged hard spheres
 * of diameter sigma_i and valence q_i in a continuum of Bjerrum length l_B,
 * pair energy U_ij/kT = l_B q_i q_j / r_ij; overlap iff
 * r_ij < (sigma_i + sigma_j)/2; the ion surface may not cross the wall,
 * |x_i| <= R - sigma_i/2.  Lengths are in the caller's unit, energies in kT.
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), one block per trial,
 * counter (i, sweep, chain_id, 0), key (seed low word, seed high word);
 * words 0..2 give the displacement, word 3 the accept uniform.
 *
 * Conventions for every call:
 *   - All pointer arguments are HOST pointers unless stated otherwise; the
 *     library copies what it needs and never keeps a caller pointer.
 *   - Every function returns MC_OK (0) or a negative mc_status; no exception
 *     or longjmp crosses this interface.  mc_last_error() describes the last
 *     failure of a handle.
 *   - A handle is not thread safe; calls on one handle must be serialised.
 *   - Work is enqueued on the handle's HIP stream; getters that return data
 *     synchronise that stream first.
 */
#ifndef MC_H_
#define MC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mc_handle mc_handle;

typedef enum mc_status {
    MC_OK = 0,
    MC_E_ARG = -1,          /* bad argument (null, size, non-finite, range)       */
    MC_E_OVERLAP = -2,      /* input positions have a hard-core overlap           */
    MC_E_WALL = -3,         /* an input ion crosses the wall                      */
    MC_E_NOT_NEUTRAL = -4,  /* sum of charges is not zero                         */
    MC_E_DEVICE = -5,       /* HIP runtime error, or the HIP device is missing    */
    MC_E_OOM = -6,          /* device memory allocation failed                    */
    MC_E_TIMEOUT = -7,      /* a device-side wait exceeded its time limit         */
    MC_E_STATE = -8         /* handle in a bad state (e.g. after a device error)  */
} mc_status;

typedef enum mc_precision {
    MC_FP64 = 0,            /* positions and pair terms in double                 */
    MC_FP32_ACC64 = 1       /* positions and pair terms in float; per-move dE and
                               the running energy accumulated in double           */
} mc_precision;

/*
 * Options; call mc_options_init() first, then change fields.  Passing NULL
 * wherever an mc_options* is accepted means the defaults.
 */
typedef struct mc_options {
    int32_t precision;      /* mc_precision, default MC_FP32_ACC64                */
    double max_disp;        /* half side of the trial cube, D = 2 * max_disp
                               (Algorithm 1's "range of one moving" is D);
                               default 0.5                                         */
    int32_t resum_every;    /* re-sum the total energy in double every this many
                               sweeps inside mc_sweep and reset the running
                               energy to it (0 = never); default 100               */
    int32_t rdf_every;      /* accumulate g(r) counts every this many sweeps
                               inside mc_sweep (0 = never); default 0              */
    int32_t rdf_bins;       /* histogram bins, default 200                         */
    double rdf_rmax;        /* histogram range, default 10                         */
    uint32_t chain_id;      /* Philox counter word 2, default 0                    */
    void* hip_stream;       /* hipStream_t to enqueue on (e.g. a PyTorch stream);
                               NULL = a stream owned by the handle                 */
    int32_t band;           /* look-ahead band width in 64-ion groups (0..4),
                               -1 = automatic; affects speed only.  Clamped to
                               3 for float chains with per-ion diameters, for
                               float chains on eight waves and for the
                               delayed-acceptance kernel; to 2 for float
                               chains with both.  Automatic on eight waves: 1
                               for a float chain whose workgroups serve at
                               least four of its groups a sweep in the
                               schedule planned at creation                    */
    int32_t waves;          /* waves per workgroup (4 or 8), 0 = automatic:
                               8 for float chains of at least 3 groups of 64
                               per compute unit in all (one chain: N >= 49089
                               on 256 CUs) without move logging, else 4.
                               Delayed acceptance needs 4                   */
    int32_t workgroups;     /* workgroups serving the chain, 0 = automatic         */
    int64_t trace_moves;    /* record accept bit and dE of the first this many
                               moves of the chain (global move index
                               sweep * N + i), 0 = off                             */
    double wait_timeout_s;  /* limit of any single device-side wait, default 20   */
    int32_t record_timing;  /* nonzero: time every sweep-kernel launch with HIP
                               events on the handle's stream (see mc_timing)     */
    /* delayed acceptance (see mc_set_surrogate) */
    double da_rcut;         /* range of the neighbour histograms, default 4       */
    int32_t da_window;      /* drift-monitor window in sweeps, default 10         */
    double da_delta;        /* fall back to the plain test when a window's stage-2
                               rejection rate exceeds the reference by more than
                               this, default 0.05                                  */
    int64_t log_moves;      /* log features, dE and dEh of the first this many
                               moves of every chain for training (mc_get_log),
                               0 = off                                             */
    double rdf_margin;      /* g(r) centres need |x| <= R - rdf_rmax - rdf_margin:
                               every neighbour counted then lies at least
                               rdf_margin inside the wall (Sec. 5.2 leaves ions
                               within ten Debye lengths of the wall out of the
                               data); default 0                                    */
} mc_options;

/* Fills *opt with the defaults.  Returns MC_E_ARG if opt is NULL. */
int mc_options_init(mc_options* opt);

/*
 * Creates a chain.
 *   n          number of ions, 1 <= n <= 2^24.
 *   charges    [n] valences q_i (finite); their sum must be 0 within 1e-9 * sum|q|.
 *   diameters  [n] hard-sphere diameters sigma_i > 0.
 *   positions  [n*3] x,y,z per ion (row-major); must lie inside the wall and
 *              be free of overlaps (r_ij >= (sigma_i + sigma_j)/2).
 *   radius     wall radius R > 0.
 *   l_B        Bjerrum length >= 0 (pair energy l_B q_i q_j / r in kT).
 *   opt        options or NULL.
 *   out        receives the handle.
 * The initial total energy is computed on the device in double.  Errors:
 * MC_E_ARG, MC_E_NOT_NEUTRAL, MC_E_WALL, MC_E_OVERLAP, MC_E_DEVICE, MC_E_OOM.
 * On error *out is set to NULL and nothing is leaked.
 */
int mc_create(int32_t n, const double* charges, const double* diameters,
              const double* positions, double radius, double l_B,
              const mc_options* opt, mc_handle** out);

/*
 * Enqueues n_sweeps >= 0 sequential sweeps (Sec. 2) continuing the handle's
 * sweep counter; the random stream is keyed by seed, so a chain continued
 * with the same seed is identical to one run in a single call.  The energy
 * re-sum and g(r) sampling of the options are interleaved at sweep counts
 * that are multiples of their intervals.  Asynchronous: returns once the work
 * is enqueued; device errors surface on the next synchronising call.  With a
 * surrogate installed (mc_set_surrogate) and no move log, the call
 * synchronises once per drift-monitor window to see whether the monitor has
 * switched every chain to the plain test; from then on it launches the plain
 * sweep kernel, re-planning the schedule for it.
 */
int mc_sweep(mc_handle* h, int64_t n_sweeps, uint64_t seed);

/*
 * The same n_sweeps sweeps as mc_sweep (same trials, same random stream,
 * same results up to the rounding order of the sums), run by the per-move
 * parallel-reduction scheme that the paper benchmarks against (Sec. 4): one
 * kernel launch per trial move, each thread one partner, a workgroup
 * reduction, and the last workgroup to finish deciding the move.  A
 * comparison baseline, far slower than mc_sweep.  It advances the same state
 * (positions, running energy, trace, counters; the iteration and early-group
 * counters stay unchanged), so it may take turns with mc_sweep on one chain,
 * and takes record_timing, re-sum and g(r) intervals as mc_sweep does.
 * Single-chain handles only, without a delayed-acceptance stage or move log:
 * MC_E_ARG otherwise.  Asynchronous like mc_sweep.
 */
int mc_sweep_reduction(mc_handle* h, int64_t n_sweeps, uint64_t seed);

/*
 * Total energy (Sec. 5.2 records it per cycle; the pair energy
 * l_B q_i q_j / r_ij of Sec. 5.1 with kT = 1, summed over i < j; no self,
 * wall or image term).  Synchronises and returns the running energy (sum of
 * accepted dE since the last re-sum, plus that re-sum) in *e_running, and,
 * if e_exact is not NULL, a fresh double-precision re-sum of the total
 * energy of the current state (which does not reset the running energy).
 * Energies in kT.  Errors: MC_E_ARG for a NULL handle or e_running,
 * MC_E_STATE after a failed launch, MC_E_DEVICE.
 */
int mc_energy(mc_handle* h, double* e_running, double* e_exact);

/*
 * Pair correlation functions g_ab(r) (Sec. 5.2, the definition behind Eq.
 * rho-g-g; ions near the wall are left out as centres).  Synchronises and
 * returns the functions accumulated so far.
 * Species are the distinct (charge, diameter) pairs, ordered by decreasing
 * charge then increasing diameter.  g [ntypes*ntypes*bins] receives
 * g_ab(r_k) = C_ab(k) / (Ncentre_a * n_b * V_k) (centres: ions with
 * |x| <= R - rmax - rdf_margin; n_b = (N_b - delta_ab) / ((4/3) pi (R - sigma_b/2)^3);
 * V_k the shell volume); counts (nullable) [ntypes*ntypes*bins] the raw
 * integer pair counts; centres (nullable) [ntypes] the centre counts; bins
 * must equal the handle's rdf_bins.  *n_samples (nullable) gets the number of
 * configurations accumulated.
 */
int mc_rdf(mc_handle* h, int32_t bins, double* g, uint64_t* counts, uint64_t* centres,
           int64_t* n_samples);

/*
 * Checkpoint and resume.  mc_save synchronises and writes the handle's state
 * to the file at path: per chain the model (charges, diameters, wall radius,
 * l_B, move size, chain id), the positions after the last two sweeps and
 * the accept masks of the last groups (the sweep kernel's working state, so
 * that a resumed chain sums every dE in the same order), the running energy
 * and its re-sum record, the counters, the g(r) counts and samples, the
 * energy series, and the handle's sweep counter and options.  Not saved: move
 * traces, the delayed-acceptance network, log and monitor (install the
 * network again with mc_set_surrogate), and the autotuned schedule (planned
 * again from the defaults).  mc_load creates a handle from such a file; opt
 * NULL means the saved options (without their stream), otherwise opt is used
 * and must have the saved precision, rdf_bins, rdf_rmax and rdf_margin.  The random stream is a
 * function of (seed, sweep, ion, chain), so sweeps run after mc_load with the
 * same seed reproduce the ones an uninterrupted chain would run, bit for bit.
 * The file is in host byte order for this library version.  Errors: MC_E_ARG
 * (bad path, unreadable or foreign file, mismatched options), then those of
 * mc_create; on error *out is NULL.
 */
int mc_save(mc_handle* h, const char* path);
int mc_load(const char* path, const mc_options* opt, mc_handle** out);

/* Enqueues one g(r) sample of the current configuration. */
int mc_rdf_sample(mc_handle* h);

/* Clears the accumulated g(r) counts. */
int mc_rdf_reset(mc_handle* h);

/* Number of species and, if the pointers are non-NULL, their charges/diameters. */
int mc_species(const mc_handle* h, int32_t* ntypes, double* charges, double* diameters);

/* Synchronises and copies the current positions (the particle array of
 * Sec. 3.1: x, y, z per ion, in the caller's length unit), [n*3] doubles,
 * exact copies of the stored float or double values; the caller owns xyz.
 * MC_E_ARG for a NULL handle or xyz. */
int mc_get_positions(mc_handle* h, double* xyz);

/*
 * Synchronises and copies the trace of the first moves (see trace_moves):
 * acc [n_moves] accept bytes, dE [n_moves] doubles (either may be NULL).
 * n_moves must not exceed the traced capacity nor the moves done so far.
 */
int mc_trace(mc_handle* h, int64_t n_moves, uint8_t* acc, double* dE);

/*
 * Synchronises and copies the per-sweep running energies recorded since the
 * handle was created (one value after each sweep, sweep index 0 first):
 * e [n] with n <= number of sweeps done.
 */
int mc_energy_series(mc_handle* h, int64_t n, double* e);

typedef struct mc_stats {
    int64_t sweeps;          /* sweeps done                                        */
    int64_t moves;           /* trial moves attempted                             */
    int64_t accepted;        /* accepted moves                                    */
    int64_t rejected_wall;   /* rejected because the trial crosses the wall        */
    int64_t rejected_overlap;/* rejected by the hard-core indicator (not wall)     */
    int64_t rejected_metropolis; /* rejected by the Metropolis test                */
    int64_t fixpoint_iterations; /* in-group decision iterations (diagnostic)      */
    int64_t early_groups;    /* groups decided from bounds before their predecessor's
                                decisions were known (diagnostic)                  */
    int64_t resums;          /* double-precision energy re-sums done               */
    double last_drift;       /* running minus re-summed energy at the last re-sum  */
    double max_abs_drift;    /* largest |drift| over all re-sums                   */
    int32_t band;            /* band width used                                    */
    int32_t waves;           /* waves per workgroup used                           */
    int32_t workgroups;      /* workgroups used by the last sweep launch           */
    int32_t da_active;       /* delayed acceptance currently on                    */
    int64_t da_moves;        /* moves decided by the two-stage test                */
    int64_t da_conflicts;    /* moves that took the plain test by the conflict rule */
    int64_t da_stage1_rejected;  /* two-stage moves rejected by stage 1           */
    int64_t da_stage1_passed;    /* stage-1 passes without wall or overlap         */
    int64_t da_stage2_rejected;  /* of those, rejected by stage 2                  */
    int64_t da_fallback_sweep;   /* sweep of the fall-back to the plain test, -1   */
    double da_last_rate;     /* stage-2 rejection rate of the last monitor window  */
    int32_t da_kernel;       /* sweep launches run the delayed-acceptance kernel
                                (a surrogate is installed and on, or moves are
                                logged); 0 once the monitor has switched every
                                chain to the plain test                            */
    int32_t reserved0;
} mc_stats;

/* Synchronises and fills *out. */
int mc_get_stats(mc_handle* h, mc_stats* out);

/*
 * Synchronises and reports the device time of the sweep-kernel launches made
 * since the handle was created or since mc_timing_reset (requires
 * record_timing): *launches launches (nullable), *kernel_ms their summed
 * duration in milliseconds (nullable), *sweeps the sweeps they covered
 * (nullable).  The energy re-sum and g(r) kernels are not included.
 */
int mc_timing(mc_handle* h, int64_t* launches, double* kernel_ms, int64_t* sweeps);

/* Clears the timing totals. */
int mc_timing_reset(mc_handle* h);

/* Changes the trial-cube half side for subsequent sweeps (e.g. after
 * warm-up tuning); max_disp > 0. */
int mc_set_max_disp(mc_handle* h, double max_disp);

/* ------------------------------------------------------------------------
 * Batches of independent chains in one persistent launch.
 *
 * Every chain of a batch is an independent Metropolis chain as above; the
 * sweep kernel serves all of them in one cooperative launch, each chain with
 * its own workgroups (a multi-workgroup-per-chain analogue of the paper's
 * multi-thread-per-particle treatment, Sec. 3.7, whose best setting depends
 * on N, Sec. 4).  The calls without a chain index act on chain 0; mc_sweep,
 * mc_set_max_disp, mc_rdf_sample, mc_rdf_reset and the timing calls act on
 * every chain.  All chains share the precision, the options and the sweep
 * counter; their random streams differ by chain_id (Philox counter word 2).
 * ------------------------------------------------------------------------ */
typedef struct mc_chain_spec {
    int32_t n;               /* ions, 1 <= n <= 2^24                              */
    int32_t reserved0;
    const double* charges;   /* [n], as for mc_create                            */
    const double* diameters; /* [n]                                              */
    const double* positions; /* [n*3]                                            */
    double radius;           /* wall radius                                      */
    double l_B;              /* Bjerrum length                                   */
    double max_disp;         /* trial-cube half side; 0 = the options' max_disp  */
    uint32_t chain_id;       /* Philox counter word 2 of this chain              */
    int32_t reserved1;
} mc_chain_spec;

/*
 * Creates a batch of n_chains >= 1 chains.  Each spec is validated as by
 * mc_create (errors name the chain); the caller keeps ownership of every
 * array.  The number of chains may not exceed the number of workgroups that
 * can be resident at once (MC_E_ARG).  opt->workgroups, if > 0, caps the
 * total workgroups of the launch.  The initial schedule gives each chain
 * workgroups by the default cost model (see mc_autotune).
 */
int mc_create_batch(int32_t n_chains, const mc_chain_spec* chains, const mc_options* opt,
                    mc_handle** out);

/* Number of chains of the handle. */
int mc_chain_count(const mc_handle* h, int32_t* n_chains);

/* Per-chain versions of mc_energy, mc_rdf, mc_species, mc_get_positions,
 * mc_trace, mc_energy_series, mc_get_stats and mc_set_max_disp; chain is in
 * [0, n_chains), MC_E_ARG otherwise. */
int mc_chain_energy(mc_handle* h, int32_t chain, double* e_running, double* e_exact);
int mc_chain_rdf(mc_handle* h, int32_t chain, int32_t bins, double* g, uint64_t* counts,
                 uint64_t* centres, int64_t* n_samples);
int mc_chain_species(const mc_handle* h, int32_t chain, int32_t* ntypes, double* charges,
                     double* diameters);
int mc_chain_positions(mc_handle* h, int32_t chain, double* xyz);
int mc_chain_trace(mc_handle* h, int32_t chain, int64_t n_moves, uint8_t* acc, double* dE);
int mc_chain_energy_series(mc_handle* h, int32_t chain, int64_t n, double* e);
int mc_chain_stats(mc_handle* h, int32_t chain, mc_stats* out);
int mc_chain_set_max_disp(mc_handle* h, int32_t chain, double max_disp);

/*
 * Schedule of the batch: workgroups [n_chains] (nullable) receives each
 * chain's workgroup count (chains with count 1 may share their workgroup
 * with other such chains, see mc_autotune, so the counts can add up to more
 * than the launch's workgroups); model [2] (nullable) the cost model in use,
 * a and b in microseconds, of the per-sweep time t(B, w) = a B + b B^2 / w
 * of a chain of B groups of 64 ions served by w workgroups.  Schedules only
 * change speed: a chain's trajectory does not depend on them.
 */
int mc_get_schedule(const mc_handle* h, int32_t* workgroups, double* model);

/* Sets each chain's workgroup count, workgroups [n_chains], each in
 * [1, groups of 64 of the chain], total at most the co-resident capacity;
 * every workgroup serves one chain. */
int mc_set_schedule(mc_handle* h, const int32_t* workgroups);

/* Synchronises and reports, per chain, the device time in milliseconds of
 * the last sweep launch from its start to the chain's last decision,
 * ms [n_chains]. */
int mc_chain_launch_ms(mc_handle* h, double* ms);

/*
 * The batch planner on its own (host only; no device or handle): the plan
 * mc_autotune and mc_create_batch make for n_chains chains of nb[k] 64-ion
 * groups, cost factors scale[k] (nullable: 1) and measured[k] (nullable:
 * none measured; only measured chains may share a workgroup), cost model
 * a, b (microseconds, both > 0) and budget >= n_chains workgroups.  Fills
 * workgroups[n_chains] and *n_launch (workgroups of the launch); if any of
 * item_chain, item_index, item_wg [max_items] is given, the launch's items:
 * item q is workgroup item_index[q] of chain item_chain[q], run by launch
 * workgroup item_wg[q] (a launch workgroup runs its items in order).
 * MC_E_ARG on bad arguments or too few max_items.
 */
int mc_plan_schedule(int32_t n_chains, const int32_t* nb, const double* scale, const uint8_t* measured,
                     double a, double b, int32_t budget, int32_t* workgroups, int32_t* n_launch,
                     int32_t* item_chain, int32_t* item_index, int32_t* item_wg, int32_t max_items);

/*
 * Autotuner: runs calib_sweeps sweeps of every chain (real sweeps that
 * continue the chains, keyed by seed, as mc_sweep runs them: launches end at
 * every re-sum, g(r) and monitor interval boundary, and the re-sums and
 * samples due there are taken), sums each chain's device time over those
 * launches, fits the cost model's a
 * and b to the measured per-chain times by least squares on relative error
 * (a held within [0.3, 4] us), and gives each chain a factor: its measured
 * time over the model's prediction.  It then re-plans for the smallest
 * sweep time T that fits the co-resident capacity: chains that one
 * workgroup brings within T share workgroups (each runs its chains one
 * after another), every other chain gets the fewest workgroups that bring
 * it within T.  model [2] (nullable) receives the fit.
 */
int mc_autotune(mc_handle* h, int32_t calib_sweeps, uint64_t seed, double* model);

/* ------------------------------------------------------------------------
 * Delayed acceptance with a learned first stage (not in the paper; the
 * two-stage Metropolis rule of Christen and Fox, 2005, with the paper's exact
 * dE as the second stage, so the sampled distribution is unchanged).
 *
 * Stage 1 accepts with min{1, exp(-dEh)}, dEh = l_B (eps(phi(x~_i)) -
 * eps(phi(x_i))), using the move's u3; a pass is accepted with
 * min{1, exp(-(dE - dEh))}, using word 0 of the Philox block with tag 2.
 * phi(p): 64-bin histograms (bin width rcut/64) of the distances r < rcut
 * from p to the like-charged and to the unlike-charged other ions, at their
 * current positions (128 inputs).  eps: 128 -> 128 -> 128 -> 1 with ReLU,
 * bfloat16 weights, float sums, hidden activations rounded to bfloat16.
 * Conflict rule: a move whose old or trial position lies within rcut of the
 * old or trial position of an ion whose decision is still pending (the
 * previous `band` 64-ion groups of the chain's sequence of groups, or a lower
 * ion of its own group) takes the plain test; the rule depends on the
 * unordered pair {x_i, x~_i} only, so detailed balance holds move by move.
 * A wider band makes more moves take the plain test and takes the network
 * off the decision chain's critical path.
 * ------------------------------------------------------------------------ */

/* Number of network parameters: W1 [128 x 128] (row = input), b1 [128],
 * W2 [128 x 128], b2 [128], w3 [128], b3. */
#define MC_DA_NPARAM 33153

/*
 * Installs the network on chain `chain` (-1: every chain) and switches its
 * delayed acceptance on (active != 0) or off.  params [MC_DA_NPARAM] are
 * rounded to bfloat16.  ref_stage2_reject is the stage-2 rejection rate of
 * stage-1 passes measured when the network was trained (< 0: no drift
 * monitor); the monitor compares each window of opt.da_window sweeps against
 * ref + opt.da_delta and switches the chain to the plain test for good on the
 * first window above it.  Needs 4 waves per workgroup.
 */
int mc_set_surrogate(mc_handle* h, int32_t chain, const double* params, double ref_stage2_reject,
                     int32_t active);

/*
 * Synchronises and copies the training log of chain `chain` (opt.log_moves):
 * for the first n moves, feats [n*256] byte histograms (phi(x_i) then
 * phi(x~_i), each like-charged bins then unlike-charged), dE [n], dEh [n]
 * (0 where the surrogate was not evaluated) and flags [n] (bit0 wall,
 * bit1 overlap, bit2 conflict, bit3 stage-1 rejection, bit4 stage-2
 * rejection, bit5 accepted, bit7 set for every logged move).  Any output may
 * be NULL.
 */
int mc_get_log(mc_handle* h, int32_t chain, int64_t n, uint8_t* feats, double* dE, double* dEh,
               uint8_t* flags);

/*
 * One forward and backward pass of the network on the GPU (bfloat16 matrix
 * products with float sums), for checks: feats [batch*256] byte histograms
 * of batch moves (as from mc_get_log), target [batch] the values eps(new) -
 * eps(old) should take, params [MC_DA_NPARAM] (used at bfloat16 precision).
 * *loss = mean((eps(new) - eps(old) - target)^2); grad [MC_DA_NPARAM] its
 * gradient (nullable outputs).  batch a positive multiple of 32.  Uses the
 * current HIP device and its default stream; needs no handle.
 */
int mc_mlp_grad(int32_t batch, const uint8_t* feats, const double* target, const double* params,
                double* loss, double* grad);

/*
 * The same pass as mc_mlp_grad, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): it calls no hipMalloc, hipFree or allocating library
 * routine.  Every buffer of the pass, and the staged inputs, live in one
 * file-scope device workspace of about 2.2 MB that each GPU the library
 * runs on holds until the process ends; batch is at most
 * MC_NOALLOC_MAX_BATCH (else MC_E_ARG).  The workspace is shared by every
 * call on a GPU and keeps the last call's contents (each pass overwrites
 * every value it reads): calls that overlap on one GPU, from several host
 * threads, race.  Same arguments, outputs and errors as mc_mlp_grad; the
 * reason of a failure is in mc_last_error(NULL).
 */
#define MC_NOALLOC_MAX_BATCH 256
int mc_mlp_grad_noalloc(int32_t batch, const uint8_t* feats, const double* target, const double* params,
                        double* loss, double* grad);

/*
 * Trains the network on the GPU on chain `chain`'s log: the first n_moves
 * logged moves without a conflict, wall or overlap rejection; the last tenth
 * of them held out.  Target of a move: dE / l_B; loss: mean squared error of
 * eps(phi(x~_i)) - eps(phi(x_i)).  Adam (beta 0.9, 0.999) with learning rate
 * lr on float master weights, minibatches of `batch` moves (a multiple of 32)
 * drawn in an order fixed by seed, `epochs` passes.  params_in (nullable)
 * starts the training, else He-initialised weights from seed.  Outputs:
 * params_out [MC_DA_NPARAM] (bfloat16 values), loss_out [epochs] (nullable)
 * the mean training loss of each epoch, *val_loss (nullable) the held-out
 * loss, *ref_stage2_reject (nullable) the stage-2 rejection rate the network
 * gives on the held-out moves (for mc_set_surrogate's drift monitor).
 */
int mc_train_surrogate(mc_handle* h, int32_t chain, int64_t n_moves, int32_t epochs, int32_t batch,
                       double lr, uint64_t seed, const double* params_in, double* params_out,
                       double* loss_out, double* val_loss, double* ref_stage2_reject);

/* Releases every resource of the handle; NULL is allowed. */
void mc_destroy(mc_handle* h);

/* Human-readable description of the last error on h (or, when h is NULL, of
 * the calling thread's last failed mc_create, mc_create_batch, mc_load or
 * mc_mlp_grad_noalloc).  Never NULL. */
const char* mc_last_error(const mc_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* MC_H_ */
