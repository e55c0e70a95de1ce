/*
 * mc_oracle.c -- plain, slow, sequential CPU oracle for exact-energy
 * Metropolis Monte Carlo of the primitive-model electrolyte.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the only thing the two have in
 * common is the published definition of the Philox4x32-10 generator, which
 * each side implements on its own.
 *
 * Everything is IEEE double (except the explicitly float trial formula of the
 * FP32 state replay), evaluated in source order; build with
 * -O2 -ffp-contract=off so that no multiply-add is fused.
 *
 * Paper: Liang, Xing, Li, "A GPU-based Large-scale Monte Carlo Simulation
 * Method for Systems with Long-range Interactions" (arXiv:1602.05716).
 *   - Sec. 2 "Concurrency": a Monte Carlo step is selection, trial, and
 *     acceptance with probability min{1, exp(-beta dE)}, Eq. (trial-outcome);
 *     the sequential updating scheme tries particles 0..N-1 in ascending
 *     order, each exactly once per cycle (sweep).
 *   - Sec. 2, Eq. (Delta E_ij): the energy change of step i is the sum over
 *     j != i of U(x~_i - x_j) - U(x_i - x_j), where x_j is the *current*
 *     position of j (already updated for j < i).
 *   - Sec. 3.3 "Energy computation": energy sums are double precision; a
 *     hard-core overlap is tracked as a separate indicator and rejects the
 *     trial.
 *   - Sec. 3.2, Algorithm 1: the trial displacement is (u - 0.5) * D per
 *     Cartesian component, D being the move range (cube side).
 *   - Sec. 3.5, Algorithm 4: the trial is accepted when the fourth uniform is
 *     below exp(-lambda * dE'), lambda the Bjerrum length and dE' the
 *     Coulomb sum in units of e^2/(4 pi eps); here dE already carries the
 *     Bjerrum length, so the test reads u3 < exp(-dE) with dE in kT.
 *   - Sec. 5.2: spherical simulation domain with a hard wall.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes): the ion surface may not cross the wall (|x| <= R - sigma/2);
 * additive hard-sphere diameters, overlap iff r < (sigma_i + sigma_j)/2;
 * random numbers come from Philox4x32-10 with counter (i, sweep, chain, tag)
 * and key (seed low word, seed high word) instead of the host-side ran4;
 * dE <= 0 accepts without evaluating exp().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as defined by Salmon, Moraes, Dror and Shaw, "Parallel      */
/* random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64   */
/* multiplications; between rounds the two key words are bumped by the Weyl   */
/* constants.                                                                  */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The four words of move (ion i, sweep s) of chain c with tag t. */
static void move_words(uint64_t seed, uint32_t chain, uint32_t sweep, uint32_t i,
                       uint32_t tag, uint32_t w[4])
{
    uint32_t ctr[4] = {i, sweep, chain, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, w);
}

void orc_move_words(uint64_t seed, uint32_t chain, uint32_t sweep, uint32_t i,
                    uint32_t tag, uint32_t w[4])
{
    move_words(seed, chain, sweep, i, tag, w);
}

/* ------------------------------------------------------------------------ */
/* Pair energy and the energy change of one trial move.                       */
/* ------------------------------------------------------------------------ */

/* Squared distance, summed left to right with no fused multiply-add. */
/* Threads the partner sum may use: 1, or the OpenMP build's thread count. */
int32_t orc_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

static double dist2(const double* a, const double* b)
{
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    double dz = a[2] - b[2];
    return dx * dx + dy * dy + dz * dz;
}

/*
 * Total Coulomb energy in kT: E = l_B * sum_{i<j} q_i q_j / r_ij (Sec. 5.1,
 * the bare pair potential; beta e^2 / (4 pi eps) = l_B).  No self term, no
 * wall energy, no image charges.  Order: i ascending, j ascending.
 */
double orc_total_energy(int32_t n, const double* xyz, const double* q, double lB)
{
    double e = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            e += q[i] * q[j] / sqrt(dist2(xyz + 3 * i, xyz + 3 * j));
    return lB * e;
}

/*
 * Energy change of moving ion i from xyz[i] to xt (Eq. Delta E_ij summed
 * over j != i, with the positions currently held in xyz), in kT, plus the
 * hard-core overlap indicator of Sec. 3.3 evaluated at the trial position.
 * The sum runs over j in ascending order and is never cut short: the
 * indicator is carried alongside the sum, as in the GPU scheme of Sec. 3.3.
 */
double orc_delta_energy(int32_t n, const double* xyz, const double* q,
                        const double* sigma, int32_t i, const double* xt,
                        double lB, int32_t* overlap)
{
    const double* xi = xyz + 3 * i;
    double s = 0.0;
    int ov = 0;
    /* the OpenMP build (timing only; it sums in another order) splits the
       partners over the host's threads; the oracle proper ignores this */
#pragma omp parallel for schedule(static) reduction(+ : s) reduction(| : ov) if (n >= 4096)
    for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const double* xj = xyz + 3 * j;
        double d2t = dist2(xt, xj);
        double d2 = dist2(xi, xj);
        double sij = 0.5 * (sigma[i] + sigma[j]);
        if (d2t < sij * sij) ov = 1;
        s += q[j] * (1.0 / sqrt(d2t) - 1.0 / sqrt(d2));
    }
    if (overlap) *overlap = ov;
    return lB * q[i] * s;
}

/* Hard wall (Sec. 5.2, reading: the ion surface stays inside radius R). */
static int outside_wall(const double* x, double R, double sigma)
{
    double a = R - 0.5 * sigma;
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    return r2 > a * a;
}

int32_t orc_outside_wall(const double* x, double R, double sigma)
{
    return outside_wall(x, R, sigma);
}

/*
 * Contact margin of a trial position: min over j != i of r~_ij / sigma_ij - 1
 * (negative when the trial overlaps an ion).  Not part of the chain: the
 * parity tests use it to tell a decision taken at contact, within float
 * rounding of sigma_ij, from a wrong one.
 */
static double contact_margin(int32_t n, const double* xyz, const double* sigma, int32_t i,
                             const double* xt)
{
    double m = INFINITY;
    for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double contact = 0.5 * (sigma[i] + sigma[j]);
        if (!(contact > 0.0)) continue;
        double g = sqrt(dist2(xt, xyz + 3 * j)) / contact - 1.0;
        if (g < m) m = g;
    }
    return m;
}

/* Metropolis test, Eq. (trial-outcome) with Algorithm 4's uniform. */
static int metropolis(double dE, double u3)
{
    return dE <= 0.0 || u3 < exp(-dE);
}

/* Trial position in double: x~ = x + D (u - 1/2), u = w 2^-32 (Algorithm 1). */
static void trial_f64(const double* x, const uint32_t w[4], double D, double* xt)
{
    for (int k = 0; k < 3; ++k) {
        double u = (double)w[k] * 0x1p-32;
        double t = u - 0.5;
        t = D * t;
        xt[k] = x[k] + t;
    }
}

void orc_trial_f64(const double* x, const uint32_t w[4], double D, double* xt)
{
    trial_f64(x, w, D, xt);
}

/*
 * n_sweeps sequential sweeps starting at sweep index sweep0 (Sec. 2,
 * sequential updating scheme).  xyz and *e_run are updated in place.  For the
 * first out_cap moves the accept bit and dE are written to acc_out/de_out
 * (either may be NULL); flags_out (nullable) receives bit0 = wall,
 * bit1 = overlap for those moves.  e_series (nullable) receives the running
 * energy after each sweep.  Returns the number of accepted moves.
 */
int64_t orc_sweeps_f64(int32_t n, double* xyz, const double* q, const double* sigma,
                       double R, double lB, double D, uint64_t seed, uint32_t chain,
                       uint32_t sweep0, int32_t n_sweeps, double* e_run,
                       uint8_t* acc_out, double* de_out, uint8_t* flags_out,
                       int64_t out_cap, double* e_series)
{
    int64_t accepted = 0, m = 0;
    for (int32_t s = 0; s < n_sweeps; ++s) {
        uint32_t sweep = sweep0 + (uint32_t)s;
        for (int32_t i = 0; i < n; ++i, ++m) {
            uint32_t w[4];
            move_words(seed, chain, sweep, (uint32_t)i, 0u, w);
            double xt[3];
            trial_f64(xyz + 3 * i, w, D, xt);
            int wall = outside_wall(xt, R, sigma[i]);
            int ov = 0;
            double dE = orc_delta_energy(n, xyz, q, sigma, i, xt, lB, &ov);
            double u3 = (double)w[3] * 0x1p-32;
            int acc = !wall && !ov && metropolis(dE, u3);
            if (acc) {
                xyz[3 * i + 0] = xt[0];
                xyz[3 * i + 1] = xt[1];
                xyz[3 * i + 2] = xt[2];
                *e_run += dE;
                ++accepted;
            }
            if (m < out_cap) {
                if (acc_out) acc_out[m] = (uint8_t)acc;
                if (de_out) de_out[m] = dE;
                if (flags_out) flags_out[m] = (uint8_t)(wall | (ov << 1));
            }
        }
        if (e_series) e_series[s] = *e_run;
    }
    return accepted;
}

/*
 * FP32-state replay.  The state is a float array (the paper keeps positions
 * in float4, Sec. 3.1) and the trial position is formed in float:
 * u = (w >> 8) 2^-24, t = u - 1/2, t = D t, x~ = x + t, each step rounded to
 * float.  The trajectory follows the decisions in acc_given (one byte per
 * move, e.g. produced by another implementation), so that every move is
 * evaluated on exactly the state that implementation saw.  For each move the
 * exact double dE over that float state, the wall/overlap flags, the accept
 * uniform u3 = w3 2^-32 and this oracle's own decision are returned.
 * Returns the number of moves where acc_given differs from the oracle's own
 * decision.
 */
int64_t orc_replay_f32(int32_t n, float* xyz, const double* q, const double* sigma,
                       double R, double lB, float D, uint64_t seed, uint32_t chain,
                       uint32_t sweep0, int64_t n_moves, const uint8_t* acc_given,
                       const uint8_t* eval_mask, double* de_out, double* u3_out,
                       uint8_t* flags_out, uint8_t* own_out, double* margin_out)
{
    double* xd = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!xd) return -1;
    for (int64_t k = 0; k < 3 * (int64_t)n; ++k) xd[k] = (double)xyz[k];
    int64_t mismatches = 0;
    for (int64_t m = 0; m < n_moves; ++m) {
        int32_t i = (int32_t)(m % n);
        uint32_t sweep = sweep0 + (uint32_t)(m / n);
        uint32_t w[4];
        move_words(seed, chain, sweep, (uint32_t)i, 0u, w);
        float xtf[3];
        for (int k = 0; k < 3; ++k) {
            float u = (float)(w[k] >> 8) * 0x1p-24f;
            float t = u - 0.5f;
            t = D * t;
            xtf[k] = xyz[3 * i + k] + t;
        }
        double xt[3] = {(double)xtf[0], (double)xtf[1], (double)xtf[2]};
        int wall = outside_wall(xt, R, sigma[i]);
        int ov = 0;
        double u3 = (double)w[3] * 0x1p-32;
        int evaluate = !eval_mask || eval_mask[m] || !acc_given;
        double dE = 0.0;
        int own = 0;
        if (evaluate) {
            dE = orc_delta_energy(n, xd, q, sigma, i, xt, lB, &ov);
            own = !wall && !ov && metropolis(dE, u3);
            if (margin_out) margin_out[m] = contact_margin(n, xd, sigma, i, xt);
        }
        int acc = acc_given ? (int)acc_given[m] : own;
        if (evaluate && acc != own) ++mismatches;
        if (de_out) de_out[m] = dE;
        if (u3_out) u3_out[m] = u3;
        if (flags_out) flags_out[m] = (uint8_t)(wall | (ov << 1));
        if (own_out) own_out[m] = (uint8_t)own;
        if (acc) {
            for (int k = 0; k < 3; ++k) {
                xyz[3 * i + k] = xtf[k];
                xd[3 * i + k] = xt[k];
            }
        }
    }
    free(xd);
    return mismatches;
}

/*
 * Radial distribution counts (Sec. 5.2): centres are the ions whose centre
 * lies within R - r_max of the origin (so that every shell up to r_max is
 * inside the domain -- the reading of "ions near the boundary are not used
 * for data collection"); neighbours are all other ions.  Ordered pairs.
 * Bin k = floor(r / dr), dr = r_max / bins, pairs with r >= r_max dropped.
 * counts[(ti * ntypes + tj) * bins + k] and centres[ti] are incremented.
 */
void orc_rdf_counts(int32_t n, const double* xyz, const int32_t* type, int32_t ntypes,
                    double R, double rmax, int32_t bins, uint64_t* counts,
                    uint64_t* centres)
{
    double dr = rmax / (double)bins;
    double rc = R - rmax;
    for (int32_t i = 0; i < n; ++i) {
        const double* xi = xyz + 3 * i;
        double r2i = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        if (rc < 0.0 || r2i > rc * rc) continue;
        centres[type[i]] += 1;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r = sqrt(dist2(xi, xyz + 3 * j));
            if (r >= rmax) continue;
            int32_t k = (int32_t)floor(r / dr);
            if (k >= bins) continue;
            counts[((int64_t)type[i] * ntypes + type[j]) * bins + k] += 1;
        }
    }
}

/* ======================================================================== */
/* Delayed acceptance with a learned first stage (not in the paper).          */
/*                                                                            */
/* Two-stage Metropolis (Christen and Fox, J. Comput. Graph. Stat. 14, 2005): */
/* stage 1 accepts with min{1, exp(-dEh)}, dEh an inexpensive estimate of dE; */
/* a stage-1 pass is then accepted with min{1, exp(-(dE - dEh))}.  With dEh   */
/* antisymmetric in the move the product of the two keeps detailed balance.  */
/* Here dEh = l_B (eps(phi(x~_i)) - eps(phi(x_i))): eps is a small MLP and    */
/* phi the neighbour-distance histograms of a position, built from the        */
/* current positions of all other ions.                                       */
/*                                                                            */
/* Readings (listed in the design notes):                                     */
/*  - phi(p): 64 bins of width rc/64 over r = |p - x_j| < rc, j != i, one      */
/*    histogram for like-charged j (q_i q_j > 0), one for unlike-charged j    */
/*    (q_i q_j < 0); r from the squared distance summed in double with no     */
/*    fused multiply-add, bin = floor(r / (rc / 64)).                          */
/*  - eps: 128 -> 128 -> 128 -> 1, ReLU, weights held at bfloat16 values;     */
/*    each hidden activation is rounded to bfloat16 (round to nearest even)    */
/*    before it feeds the next layer.                                         */
/*  - stage 1 uses the move's accept uniform u3 (Philox word 3, tag 0);       */
/*    stage 2 uses word 0 of the Philox block with tag 2.                     */
/*  - conflict rule: ion i's move uses the plain Metropolis test instead when */
/*    an ion j with a pending decision -- an ion of the `band` 64-ion groups  */
/*    before i's group in the chain's sequence of groups, or of i's own group */
/*    with j < i -- has its old or its trial position within rc of x_i or     */
/*    x~_i.  The rule is symmetric in the move (it depends on the unordered   */
/*    pair {x_i, x~_i}), so every move still satisfies detailed balance; for  */
/*    all other moves phi is final when it is evaluated.  Groups before the   */
/*    chain's first group do not exist.                                       */
/* ======================================================================== */
#define DA_BINS 64
#define DA_IN (2 * DA_BINS)
#define DA_HID 128
#define DA_NPARAM (DA_IN * DA_HID + DA_HID + DA_HID * DA_HID + DA_HID + DA_HID + 1)

int32_t orc_da_nparam(void) { return DA_NPARAM; }

/* Round to the nearest bfloat16 (ties to even), through float. */
static double bf16_round(double v)
{
    float f = (float)v;
    uint32_t b;
    memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    b &= 0xFFFF0000u;
    memcpy(&f, &b, 4);
    return (double)f;
}

double orc_bf16_round(double v) { return bf16_round(v); }

/* phi(p) for ion i: out[0..63] like-charged, out[64..127] unlike-charged. */
void orc_da_features(int32_t n, const double* xyz, const double* q, int32_t i,
                     const double* p, double rc, int32_t* out)
{
    double dr = rc / (double)DA_BINS;
    for (int k = 0; k < DA_IN; ++k) out[k] = 0;
    for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double qq = q[i] * q[j];
        if (qq == 0.0) continue;
        double d2 = dist2(p, xyz + 3 * j);
        if (!(d2 < rc * rc)) continue;
        int32_t k = (int32_t)floor(sqrt(d2) / dr);
        if (k >= DA_BINS) continue;
        out[(qq > 0.0 ? 0 : DA_BINS) + k] += 1;
    }
}

/*
 * eps(phi) with params = [W1 (128 x 128, row = input), b1 (128),
 * W2 (128 x 128, row = input), b2 (128), w3 (128), b3]; sums in double.
 */
double orc_mlp_eps(const double* params, const int32_t* feat)
{
    const double* W1 = params;
    const double* b1 = W1 + DA_IN * DA_HID;
    const double* W2 = b1 + DA_HID;
    const double* b2 = W2 + DA_HID * DA_HID;
    const double* w3 = b2 + DA_HID;
    const double b3 = w3[DA_HID];
    double h1[DA_HID], h2[DA_HID];
    for (int h = 0; h < DA_HID; ++h) {
        double z = b1[h];
        for (int k = 0; k < DA_IN; ++k) z += (double)feat[k] * W1[k * DA_HID + h];
        h1[h] = bf16_round(z > 0.0 ? z : 0.0);
    }
    for (int h = 0; h < DA_HID; ++h) {
        double z = b2[h];
        for (int k = 0; k < DA_HID; ++k) z += h1[k] * W2[k * DA_HID + h];
        h2[h] = bf16_round(z > 0.0 ? z : 0.0);
    }
    double out = b3;
    for (int k = 0; k < DA_HID; ++k) out += h2[k] * w3[k];
    return out;
}

static int within(const double* a, const double* b, double rc)
{
    return dist2(a, b) < rc * rc;
}

/*
 * DA chain over n_moves moves (move m = ion m % n of sweep sweep0 + m / n)
 * in the chain's own sequence of 64-ion groups.  f32 != 0: the state is
 * float (xyz holds float values) and trials are formed in float as in
 * orc_replay_f32; otherwise as in orc_sweeps_f64.  With acc_given the
 * trajectory follows the given decisions (a replay); otherwise this
 * oracle's own decisions.  da_on == 0 gives the plain test for every move.
 * Per move (first out_cap moves; outputs nullable): dE, dEh (0 for conflict
 * moves), flags (bit0 wall, bit1 overlap, bit2 conflict, bit3 stage-1
 * rejection, bit4 stage-2 rejection -- of the oracle's own evaluation),
 * own decision, features [256] (phi(x_i), phi(x~_i); conflict moves too),
 * u3 and u2.  eval_mask (nullable) limits the evaluation to marked moves
 * (replays only).  *e_run accumulates accepted dE.  snap_out (nullable)
 * receives the positions after every completed sweep of the run,
 * [n_moves / n][n][3]; margin_out (nullable) the contact margin of every
 * evaluated trial.  Returns the number of
 * evaluated moves whose given decision differs from the oracle's, or -1 if
 * a DA run with band > 0 does not start at sweep 0 (the pending trials of
 * the previous sweep are not known; with DA off the conflict flags of the
 * first band groups are then only indicative), -2 on allocation failure.
 */
int64_t orc_da_run(int32_t n, double* xyz, const double* q, const double* sigma,
                   double R, double lB, double D, uint64_t seed, uint32_t chain,
                   uint32_t sweep0, int64_t n_moves, int32_t f32, const double* params,
                   double rc, int32_t band, int32_t da_on, const uint8_t* acc_given,
                   const uint8_t* eval_mask, int64_t out_cap, double* de_out,
                   double* deh_out, uint8_t* flags_out, uint8_t* own_out,
                   int32_t* feat_out, double* u3_out, double* u2_out, double* e_run,
                   double* snap_out, double* margin_out)
{
    if (band > 0 && sweep0 != 0 && da_on) return -1;
    const int32_t group = 64;
    const int32_t nb = (n + group - 1) / group;
    /* latest old and trial position of every ion */
    double* old = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* tri = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!old || !tri) {
        free(old);
        free(tri);
        return -2;
    }
    /* before its first move in this run an ion's pending positions are its current one */
    memcpy(old, xyz, sizeof(double) * 3 * (size_t)n);
    memcpy(tri, xyz, sizeof(double) * 3 * (size_t)n);
    int64_t mismatches = 0;
    for (int64_t m = 0; m < n_moves; ++m) {
        int32_t i = (int32_t)(m % n);
        uint32_t sweep = sweep0 + (uint32_t)(m / n);
        uint32_t w[4], w2[4];
        move_words(seed, chain, sweep, (uint32_t)i, 0u, w);
        move_words(seed, chain, sweep, (uint32_t)i, 2u, w2);
        double xt[3];
        if (f32) {
            float Df = (float)D;
            for (int k = 0; k < 3; ++k) {
                float u = (float)(w[k] >> 8) * 0x1p-24f;
                float t = u - 0.5f;
                t = Df * t;
                xt[k] = (double)((float)xyz[3 * i + k] + t);
            }
        } else {
            trial_f64(xyz + 3 * i, w, D, xt);
        }
        const double* xi = xyz + 3 * i;
        double u3 = (double)w[3] * 0x1p-32;
        double u2 = (double)w2[0] * 0x1p-32;
        int evaluate = !acc_given || !eval_mask || eval_mask[m];
        int own = 0, flags = 0;
        double dE = 0.0, deh = 0.0;
        int32_t fo[DA_IN], fn[DA_IN];
        if (evaluate) {
            int wall = outside_wall(xt, R, sigma[i]);
            int ov = 0;
            dE = orc_delta_energy(n, xyz, q, sigma, i, xt, lB, &ov);
            if (margin_out && m < out_cap) margin_out[m] = contact_margin(n, xyz, sigma, i, xt);
            /* conflict: pending ions near x_i or x~_i in either of their positions */
            int conflict = 0;
            int64_t g = (int64_t)sweep * nb + i / group;
            for (int64_t gp = g - band; gp <= g && !conflict; ++gp) {
                if (gp < 0) continue;
                int32_t bp = (int32_t)(gp % nb);
                int32_t j0 = bp * group, j1 = j0 + group < n ? j0 + group : n;
                if (gp == g) j1 = i;  /* own group: j < i */
                for (int32_t j = j0; j < j1 && !conflict; ++j)
                    conflict = within(xi, old + 3 * j, rc) || within(xi, tri + 3 * j, rc) ||
                               within(xt, old + 3 * j, rc) || within(xt, tri + 3 * j, rc);
            }
            orc_da_features(n, xyz, q, i, xi, rc, fo);
            orc_da_features(n, xyz, q, i, xt, rc, fn);
            int s1 = 1, s2 = 1;
            if (da_on && !conflict) {
                deh = lB * (orc_mlp_eps(params, fn) - orc_mlp_eps(params, fo));
                s1 = metropolis(deh, u3);
                s2 = metropolis(dE - deh, u2);
                own = !wall && !ov && s1 && s2;
            } else {
                own = !wall && !ov && metropolis(dE, u3);
            }
            flags = wall | (ov << 1) | (conflict << 2) | ((!s1) << 3) | ((s1 && !s2) << 4);
        }
        int acc = acc_given ? (int)acc_given[m] : own;
        if (evaluate && acc != own) ++mismatches;
        if (m < out_cap) {
            if (de_out) de_out[m] = dE;
            if (deh_out) deh_out[m] = deh;
            if (flags_out) flags_out[m] = (uint8_t)flags;
            if (own_out) own_out[m] = (uint8_t)own;
            if (u3_out) u3_out[m] = u3;
            if (u2_out) u2_out[m] = u2;
            if (feat_out && evaluate)
                for (int k = 0; k < DA_IN; ++k) {
                    feat_out[m * 2 * DA_IN + k] = fo[k];
                    feat_out[m * 2 * DA_IN + DA_IN + k] = fn[k];
                }
        }
        for (int k = 0; k < 3; ++k) {
            old[3 * i + k] = xi[k];
            tri[3 * i + k] = xt[k];
        }
        if (acc) {
            if (e_run) *e_run += dE;
            for (int k = 0; k < 3; ++k) xyz[3 * i + k] = xt[k];
        }
        if (snap_out && i == n - 1)
            memcpy(snap_out + (size_t)(m / n) * 3 * (size_t)n, xyz, sizeof(double) * 3 * (size_t)n);
    }
    free(old);
    free(tri);
    return mismatches;
}
