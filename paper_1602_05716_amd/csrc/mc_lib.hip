// mc_lib.hip -- host runtime behind include/mc.h (C ABI) and the kernel
// instantiations for gfx950.
//
// Paper: Liang, Xing, Li, arXiv:1602.05716 (see include/mc.h for the
// passages each entry point follows).  A handle holds one or more
// independent chains; the host never touches a chain between trials:
// mc_sweep enqueues one persistent cooperative launch per stretch of sweeps
// that serves every chain of the handle, interleaved with the
// double-precision energy re-sum and g(r) sampling kernels, all on the
// handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <queue>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/mc.h"
#include "mc_aux_kernels.hpp"
#include "mc_internal.hpp"
#include "mc_reduce_kernel.hpp"
#include "mc_sweep_kernel.hpp"

using namespace mcdev;

namespace {

thread_local std::string g_create_error = "no error";

// Stats slots written by the sweep kernel.
enum { ST_MOVES = 0, ST_ACC, ST_WALL, ST_OVERLAP, ST_METRO, ST_ITERS, ST_EARLY,
       ST_DA_MOVES, ST_DA_CONFLICTS, ST_DA_S1REJ, ST_DA_S1PASS, ST_DA_S2REJ, ST_N };

constexpr int64_t kMaxLaunchSweeps = 4096;
static_assert(kDaParams == MC_DA_NPARAM, "network size differs from the header");
// Default cost model of a chain (microseconds): per-sweep time
// t(nb, w) = a nb + b nb^2 / w for nb groups of 64 served by w workgroups
// (a: one group's decision step; b: one 64 x 64 partner tile of a workgroup
// sharing its CU).  The autotuner keeps a within [kModelAMin, kModelAMax]:
// per-chain times from one shared launch cannot always tell the two terms
// apart, and a latency term far outside what a group's step costs misleads
// the schedule.
constexpr double kModelA = 1.2, kModelB = 1.3;
constexpr double kModelAMin = 0.3, kModelAMax = 4.0;

struct DeviceInfo {
    int device = -1;
    int cus = 0;
    double wall_clock_hz = 1e8;
    size_t lds_per_block = 0;
};

bool device_info(DeviceInfo& di, std::string& err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "no HIP device";
        return false;
    }
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
        err = "hipGetDeviceProperties failed";
        return false;
    }
    di.device = dev;
    di.cus = p.multiProcessorCount;
    di.lds_per_block = p.sharedMemPerBlock;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        di.wall_clock_hz = 1000.0 * khz;
    return true;
}

using SweepFn = void (*)(const ChainDesc*, const int2*, const int2*, uint32_t, int32_t, Ctl);

template <typename T, int M, bool U, bool DA = false>
SweepFn sweep_fn() {
    return sweep_kernel<T, M, U, DA>;
}

// The delayed-acceptance kernels exist for 4 waves per workgroup.
SweepFn pick_sweep(bool fp64, int waves, bool uniform, bool da = false) {
    if (da) {
        if (fp64) return uniform ? sweep_fn<double, 4, true, true>() : sweep_fn<double, 4, false, true>();
        return uniform ? sweep_fn<float, 4, true, true>() : sweep_fn<float, 4, false, true>();
    }
    if (fp64) {
        if (waves == 8) return uniform ? sweep_fn<double, 8, true>() : sweep_fn<double, 8, false>();
        return uniform ? sweep_fn<double, 4, true>() : sweep_fn<double, 4, false>();
    }
    if (waves == 8) return uniform ? sweep_fn<float, 8, true>() : sweep_fn<float, 8, false>();
    return uniform ? sweep_fn<float, 4, true>() : sweep_fn<float, 4, false>();
}

// One independent chain of a handle: host copy of its model and schedule,
// and its device buffers (carved from the handle's arena, except the two
// that grow).
struct Chain {
    int32_t n = 0, nb = 0, npad = 0;
    double R = 0, lB = 0, D = 1.0;
    bool uniform_sigma = true;
    double sigma0 = 1.0;
    uint32_t chain_id = 0;
    int band = 0;
    // the cost model's factor for this chain: its measured time in the last
    // calibration over the model's prediction (1 until measured)
    double cost_scale = 1.0;
    bool measured = false;
    int wg = 1;
    std::vector<std::pair<double, double>> species;  // (charge, diameter)
    std::vector<int64_t> n_of_type;
    std::vector<int32_t> type;
    // device memory
    void* pos = nullptr;          // versioned records [2][npad]
    void* half = nullptr;         // T[npad]
    void* charge = nullptr;       // T[npad]
    double* wall_a = nullptr;     // [npad]
    int32_t* d_type = nullptr;    // [npad]
    GroupRec* rec = nullptr;      // [kRing]
    unsigned long long* stats = nullptr;  // [ST_N]
    unsigned long long* clk = nullptr;    // [2]
    double* e_partial = nullptr;  // [(nb + 1) / 2]
    EnergyAux* aux = nullptr;
    double* e_state = nullptr;
    double* sweep_tot = nullptr;  // [kMaxLaunchSweeps]
    unsigned long long* rdf_counts = nullptr;
    unsigned long long* rdf_centres = nullptr;
    uint8_t* trace_acc = nullptr;
    double* trace_de = nullptr;
    int64_t trace_cap = 0;
    double* e_series = nullptr;   // grows
    int64_t e_capacity = 0;
    double* de_group = nullptr;   // grows: [n_sweeps * nb] of one launch
    int64_t de_capacity = 0;
    // delayed acceptance
    DAState* da = nullptr;        // arena
    float* da_w = nullptr;        // [kDaParams], own allocation once installed
    uint16_t* da_wb = nullptr;    // [2][128 x 128] bfloat16 W1 and W2
    uint32_t* log_feat = nullptr; // [log_cap][64], own allocation
    double* log_de = nullptr;
    double* log_deh = nullptr;
    uint8_t* log_flags = nullptr;
    int64_t log_cap = 0;
    ChainDesc desc{};
};

}  // namespace

struct mc_handle {
    std::vector<Chain> chains;
    bool fp64 = false;
    bool uniform_sigma = true;
    int waves = 4;
    int cap = 1;                  // co-resident workgroups of the sweep kernel
    int cap_da = 0;               // ... of the delayed-acceptance kernel (0: not available)
    int wg_total = 1;             // workgroups of the sweep launch
    int wg_budget = 1;            // workgroups the schedule may use
    double model_a = kModelA, model_b = kModelB;
    bool da_kernel = false;       // sweep launches use the delayed-acceptance kernel
    int da_window = 0;            // monitor window of the installed surrogates (0: none)
    int64_t da_checked = -1;      // sweep count at the last look at the chains' DAState
    mc_options opt{};
    DeviceInfo dev;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool failed = false;
    int64_t sweeps = 0;
    int64_t rdf_samples = 0;
    std::string err = "no error";
    // device memory shared by the chains
    void* arena = nullptr;
    int* abort_flag = nullptr;
    ChainDesc* d_desc = nullptr;
    int2* d_wgmap = nullptr;      // [cap + chains] items (chain, index among the chain's workgroups)
    int2* d_wgrange = nullptr;    // [cap] per workgroup: its items [begin, end)
    BlockItem* d_eitems = nullptr;   // energy re-sum blocks
    int n_eitems = 0;
    BlockItem* d_ritems = nullptr;   // g(r) blocks
    int n_ritems = 0;
    size_t rdf_lds = 0;
    // sweep-kernel timing (record_timing)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    std::vector<int64_t> ev_sweeps;
    int64_t t_launches = 0, t_sweeps = 0;
    double t_ms = 0.0;
    int64_t last_launch_sweeps = 0;
    // per-move parallel-reduction scheme (allocated on first use)
    ReducePart* d_rparts = nullptr;  // [r_blocks]
    ReduceCtl* d_rctl = nullptr;
    int r_blocks = 0;
};

namespace {

int fail(mc_handle* h, int code, const std::string& msg) {
    if (h) {
        h->err = msg;
        if (code == MC_E_DEVICE || code == MC_E_TIMEOUT || (code == MC_E_STATE && !h->failed)) h->failed = true;
    } else {
        g_create_error = msg;
    }
    return code;
}

#define HIPCHECK(h, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((h), e_ == hipErrorOutOfMemory ? MC_E_OOM : MC_E_DEVICE,          \
                        std::string(#call) + ": " + hipGetErrorString(e_));                \
    } while (0)

template <typename P>
int dalloc(mc_handle* h, P** p, size_t bytes) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
    if (e != hipSuccess) return fail(h, MC_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    *p = (P*)v;
    return MC_OK;
}

void drop_events(mc_handle* h) {
    for (auto& e : h->ev_pending) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    h->ev_pending.clear();
    h->ev_sweeps.clear();
}

void free_all(mc_handle* h) {
    drop_events(h);
    for (Chain& c : h->chains) {
        void* own[] = {c.e_series, c.de_group, c.da_w, c.da_wb, c.log_feat, c.log_de, c.log_deh, c.log_flags};
        for (void* b : own)
            if (b) (void)hipFree(b);
        c.e_series = c.de_group = nullptr;
        c.da_w = nullptr;
        c.da_wb = nullptr;
        c.log_feat = nullptr;
        c.log_de = c.log_deh = nullptr;
        c.log_flags = nullptr;
    }
    if (h->arena) (void)hipFree(h->arena);
    h->arena = nullptr;
    if (h->d_rparts) (void)hipFree(h->d_rparts);
    if (h->d_rctl) (void)hipFree(h->d_rctl);
    h->d_rparts = nullptr;
    h->d_rctl = nullptr;
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    h->stream = nullptr;
}

// Checks the device abort word and the stream; marks the handle failed on error.
int sync_check(mc_handle* h) {
    if (h->failed) return fail(h, MC_E_STATE, "handle is in a failed state: " + h->err);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, MC_E_DEVICE, std::string("stream: ") + hipGetErrorString(e));
    int ab = 0;
    HIPCHECK(h, hipMemcpy(&ab, h->abort_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (ab != 0) {
        return fail(h, ab == MC_E_TIMEOUT ? MC_E_TIMEOUT : ab == MC_E_STATE ? MC_E_STATE : MC_E_DEVICE,
                    ab == MC_E_TIMEOUT ? "a device-side wait timed out (chain state is invalid)"
                    : ab == MC_E_STATE ? "a group record or position was not the one expected (chain state is invalid)"
                                       : "device reported an error");
    }
    return MC_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

// Uniform-grid overlap check of the input, O(n) for bounded density.
bool find_overlap(int n, const double* x, const double* sigma, double smax, int* a, int* b) {
    const double cell = smax > 0 ? smax : 1.0;
    std::unordered_map<int64_t, std::vector<int>> grid;
    grid.reserve(n * 2);
    auto key = [](int64_t i, int64_t j, int64_t k) {
        return ((i + (1 << 20)) << 42) ^ ((j + (1 << 20)) << 21) ^ (k + (1 << 20));
    };
    for (int i = 0; i < n; ++i) {
        int64_t ci = (int64_t)std::floor(x[3 * i] / cell), cj = (int64_t)std::floor(x[3 * i + 1] / cell),
                ck = (int64_t)std::floor(x[3 * i + 2] / cell);
        for (int64_t di = -1; di <= 1; ++di)
            for (int64_t dj = -1; dj <= 1; ++dj)
                for (int64_t dk = -1; dk <= 1; ++dk) {
                    auto it = grid.find(key(ci + di, cj + dj, ck + dk));
                    if (it == grid.end()) continue;
                    for (int j : it->second) {
                        double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1],
                               dz = x[3 * i + 2] - x[3 * j + 2];
                        double d2 = dx * dx + dy * dy + dz * dz;
                        double s = 0.5 * (sigma[i] + sigma[j]);
                        if (d2 < s * s) {
                            *a = j;
                            *b = i;
                            return true;
                        }
                    }
                }
        grid[key(ci, cj, ck)].push_back(i);
    }
    return false;
}

// Host-side validation of one chain's inputs (before any device work).
// check_overlap false: the positions come from a chain's own state (a
// checkpoint), whose float overlap test may round a contact either way.
int validate_chain(const mc_chain_spec& sp, const mc_options& opt, const std::string& who,
                   bool check_overlap = true) {
    const int32_t n = sp.n;
    if (n < 1 || n > (1 << 24)) return fail(nullptr, MC_E_ARG, who + "n out of range [1, 2^24]");
    if (!sp.charges || !sp.diameters || !sp.positions) return fail(nullptr, MC_E_ARG, who + "null input array");
    if (!is_finite(sp.radius) || sp.radius <= 0) return fail(nullptr, MC_E_ARG, who + "radius must be finite and > 0");
    if (!is_finite(sp.l_B) || sp.l_B < 0) return fail(nullptr, MC_E_ARG, who + "l_B must be finite and >= 0");
    if (!is_finite(sp.max_disp) || sp.max_disp < 0)
        return fail(nullptr, MC_E_ARG, who + "max_disp must be >= 0 (0 = the options' value)");
    double qsum = 0, qabs = 0, smax = 0;
    for (int i = 0; i < n; ++i) {
        if (!is_finite(sp.charges[i]) || !is_finite(sp.diameters[i]) || sp.diameters[i] <= 0)
            return fail(nullptr, MC_E_ARG, who + "charges must be finite and diameters finite and > 0");
        for (int k = 0; k < 3; ++k)
            if (!is_finite(sp.positions[3 * i + k])) return fail(nullptr, MC_E_ARG, who + "non-finite position");
        qsum += sp.charges[i];
        qabs += std::fabs(sp.charges[i]);
        smax = std::max(smax, sp.diameters[i]);
    }
    if (std::fabs(qsum) > 1e-9 * std::max(qabs, 1.0))
        return fail(nullptr, MC_E_NOT_NEUTRAL, who + "sum of charges is not zero");
    for (int i = 0; i < n; ++i) {
        const double* x = sp.positions + 3 * i;
        const double a = sp.radius - 0.5 * sp.diameters[i];
        if (a < 0 || x[0] * x[0] + x[1] * x[1] + x[2] * x[2] > a * a)
            return fail(nullptr, MC_E_WALL, who + "ion " + std::to_string(i) + " crosses the wall");
    }
    int oa = -1, ob = -1;
    if (check_overlap && find_overlap(n, sp.positions, sp.diameters, smax, &oa, &ob))
        return fail(nullptr, MC_E_OVERLAP,
                    who + "ions " + std::to_string(oa) + " and " + std::to_string(ob) + " overlap");
    // species: distinct (q, sigma)
    std::vector<std::pair<double, double>> sp_list;
    for (int i = 0; i < n; ++i) {
        auto key = std::make_pair(sp.charges[i], sp.diameters[i]);
        if (std::find(sp_list.begin(), sp_list.end(), key) == sp_list.end()) {
            sp_list.push_back(key);
            if (sp_list.size() > 8) return fail(nullptr, MC_E_ARG, who + "more than 8 species");
        }
    }
    if (sizeof(unsigned int) * sp_list.size() * sp_list.size() * (size_t)opt.rdf_bins > 48 * 1024)
        return fail(nullptr, MC_E_ARG, who + "species^2 * rdf_bins histogram does not fit in 48 KiB of LDS");
    return MC_OK;
}

// Fills the host side of a chain from its (validated) spec.
void setup_chain(Chain& c, const mc_chain_spec& sp, const mc_options& opt) {
    const int32_t n = sp.n;
    c.n = n;
    c.nb = (n + kGroup - 1) / kGroup;
    c.npad = c.nb * kGroup;
    c.R = sp.radius;
    c.lB = sp.l_B;
    c.D = 2.0 * (sp.max_disp > 0 ? sp.max_disp : opt.max_disp);
    c.chain_id = sp.chain_id;
    c.sigma0 = sp.diameters[0];
    c.uniform_sigma = true;
    for (int i = 1; i < n; ++i)
        if (sp.diameters[i] != sp.diameters[0]) c.uniform_sigma = false;
    // species: decreasing charge, then increasing diameter
    c.species.clear();
    for (int i = 0; i < n; ++i) {
        auto key = std::make_pair(sp.charges[i], sp.diameters[i]);
        if (std::find(c.species.begin(), c.species.end(), key) == c.species.end()) c.species.push_back(key);
    }
    std::sort(c.species.begin(), c.species.end(), [](const auto& a, const auto& b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
    });
    c.type.assign(c.npad, -1);
    c.n_of_type.assign(c.species.size(), 0);
    for (int i = 0; i < n; ++i) {
        auto it = std::find(c.species.begin(), c.species.end(), std::make_pair(sp.charges[i], sp.diameters[i]));
        c.type[i] = (int32_t)(it - c.species.begin());
        c.n_of_type[c.type[i]] += 1;
    }
    c.band = opt.band >= 0 ? opt.band : kMaxBand;
    c.band = std::min(c.band, std::min(kMaxBand, c.nb - 1));
    c.trace_cap = opt.trace_moves;
}

// Sub-allocation of one device arena (256-byte aligned pieces).
struct ArenaPlan {
    size_t size = 0;
    std::vector<std::pair<void**, size_t>> items;  // (where the pointer goes, offset)
    template <typename P>
    void add(P** where, size_t bytes) {
        size = (size + 255) & ~(size_t)255;
        items.emplace_back((void**)where, size);
        size += bytes ? bytes : 16;
    }
    void assign(void* base) {
        for (auto& it : items) *it.first = (char*)base + it.second;
    }
};


// A workgroup's items: (chain, index of the workgroup among the chain's).
using WgLists = std::vector<std::vector<int2>>;

// Grid order: workgroups sorted by their work (sum of nb^2 / w over their
// items), the heaviest half placed in order and the lightest half after it
// in reverse, so that grid positions i and i + W/2 pair heavy with light.
void order_grid(std::vector<std::pair<double, std::vector<int2>>>& per, WgLists& lists) {
    std::stable_sort(per.begin(), per.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    const int W = (int)per.size(), half = (W + 1) / 2;
    lists.assign(W, {});
    for (int q = 0; q < W; ++q) lists[q < half ? q : W - 1 - (q - half)] = std::move(per[q].second);
}
// What the planner needs of each chain.
struct PlanChain {
    int nb;           // groups of 64
    double scale;     // measured cost factor (1 until measured)
    bool measured;
};

double plan_cost(const PlanChain& c, double a, double b, int w) {
    return c.scale * (a * c.nb + b * (double)c.nb * c.nb / std::max(1, w));
}

// Workgroups per chain and the grid, on the cost model, for a target sweep
// time T.  A chain whose cost was measured (autotuner) and that one
// workgroup brings within T shares a workgroup with others: first fit by
// decreasing time, the workgroup running them one after another.  Every
// other chain gets the fewest workgroups that bring it within T (at most one
// per group).  T is the smallest value (bisection) whose plan fits the
// budget; workgroups left over go, one at a time, to the multi-workgroup
// chain predicted to finish last.  Host only.
void plan_lists(const std::vector<PlanChain>& ch, double ma, double mb, int budget, std::vector<int>& wg,
                WgLists& lists) {
    const int nc = (int)ch.size();
    auto cost = [&](int k, int w) { return plan_cost(ch[k], ma, mb, w); };
    std::vector<int> order(nc);
    for (int k = 0; k < nc; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x, 1) > cost(y, 1); });
    std::vector<double> bin_t;
    std::vector<std::vector<int2>> bin_items;
    auto plan = [&](double T, std::vector<int>& w) {
        w.assign(nc, 0);
        bin_t.clear();
        bin_items.clear();
        int used = 0;
        for (int k : order) {
            const double t1 = cost(k, 1);
            if (t1 > T || !ch[k].measured) {
                int need = ch[k].nb;
                for (int ww = 1; ww <= ch[k].nb; ++ww)
                    if (cost(k, ww) <= T) {
                        need = ww;
                        break;
                    }
                w[k] = need;
                used += need;
            } else {
                size_t q = 0;
                while (q < bin_t.size() && bin_t[q] + t1 > T) ++q;
                if (q == bin_t.size()) {
                    bin_t.push_back(0.0);
                    bin_items.emplace_back();
                }
                bin_t[q] += t1;
                bin_items[q].push_back(make_int2(k, 0));
                w[k] = 1;
            }
        }
        return used + (int)bin_t.size();
    };
    double lo = 0.0, hi = 0.0;
    for (int k = 0; k < nc; ++k) hi = std::max(hi, cost(k, 1));
    for (int it = 0; it < 50; ++it) {
        const double mid = 0.5 * (lo + hi);
        std::vector<int> w;
        if (plan(mid, w) <= budget)
            hi = mid;
        else
            lo = mid;
    }
    int used = plan(hi, wg);
    std::vector<char> packed(nc, 0);
    for (const auto& bi : bin_items)
        for (const int2& it : bi) packed[it.x] = 1;
    using Item = std::pair<double, int>;
    std::priority_queue<Item> pq;
    for (int k = 0; k < nc; ++k)
        if (!packed[k] && wg[k] < ch[k].nb) pq.emplace(cost(k, wg[k]), k);
    while (used < budget && !pq.empty()) {
        const int k = pq.top().second;
        pq.pop();
        wg[k] += 1;
        used += 1;
        if (wg[k] < ch[k].nb) pq.emplace(cost(k, wg[k]), k);
    }
    std::vector<std::pair<double, std::vector<int2>>> per;
    for (int k = 0; k < nc; ++k) {
        if (packed[k]) continue;
        const double work = (double)ch[k].nb * ch[k].nb / wg[k];
        for (int j = 0; j < wg[k]; ++j) per.emplace_back(work, std::vector<int2>{make_int2(k, j)});
    }
    for (size_t q = 0; q < bin_items.size(); ++q) {
        double work = 0.0;
        for (const int2& it : bin_items[q]) work += (double)ch[it.x].nb * ch[it.x].nb;
        per.emplace_back(work, bin_items[q]);
    }
    order_grid(per, lists);
}

void plan_schedule(mc_handle* h, std::vector<int>& wg, WgLists& lists) {
    std::vector<PlanChain> ch;
    for (const Chain& c : h->chains) ch.push_back(PlanChain{c.nb, c.cost_scale, c.measured});
    const int budget = h->da_kernel ? std::min(h->wg_budget, h->cap_da) : h->wg_budget;
    plan_lists(ch, h->model_a, h->model_b, budget, wg, lists);
}

// Fills every chain's descriptor from the host state.
void fill_desc(mc_handle* h) {
    for (Chain& c : h->chains) {
        ChainDesc& d = c.desc;
        d.n = c.n;
        d.nb = c.nb;
        d.band = c.band;
        d.wg_count = c.wg;
        d.npad = c.npad;
        d.chain_id = c.chain_id;
        d.lB = c.lB;
        d.D = c.D;
        d.half_uniform = 0.5 * c.sigma0;
        d.pos = c.pos;
        d.charge = c.charge;
        d.half = c.half;
        d.wall_a = c.wall_a;
        d.rec = c.rec;
        d.stats = c.stats;
        d.de_group = c.de_group;
        d.trace_acc = c.trace_acc;
        d.trace_de = c.trace_de;
        d.trace_cap = c.trace_cap;
        d.clk = c.clk;
        d.e_partial = c.e_partial;
        d.aux = c.aux;
        d.e_state = c.e_state;
        d.sweep_tot = c.sweep_tot;
        d.e_series = c.e_series;
        d.e_capacity = c.e_capacity;
        d.type = c.d_type;
        d.ntypes = (int32_t)c.species.size();
        d.rdf_rc = c.R - h->opt.rdf_rmax - h->opt.rdf_margin;
        d.rdf_counts = c.rdf_counts;
        d.rdf_centres = c.rdf_centres;
        d.da_w = c.da_w;
        d.da_w1b = c.da_wb;
        d.da_w2b = c.da_wb ? c.da_wb + kDaIn * kDaHid : nullptr;
        d.da = c.da;
        d.da_rc = h->opt.da_rcut;
        d.da_dr = h->opt.da_rcut / (double)kDaBins;
        d.log_feat = c.log_feat;
        d.log_de = c.log_de;
        d.log_deh = c.log_deh;
        d.log_flags = c.log_flags;
        d.log_cap = c.log_cap;
    }
}

// The descriptors are read by running kernels: drain the stream, then copy.
int upload_desc(mc_handle* h) {
    fill_desc(h);
    std::vector<ChainDesc> v;
    v.reserve(h->chains.size());
    for (const Chain& c : h->chains) v.push_back(c.desc);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(h->d_desc, v.data(), sizeof(ChainDesc) * v.size(), hipMemcpyHostToDevice));
    return MC_OK;
}

// Applies a workgroup count per chain: new grid map and descriptors.
int apply_schedule(mc_handle* h, const std::vector<int>& wg, const WgLists& lists) {
    std::vector<int2> items, range;
    for (const auto& l : lists) {
        range.push_back(make_int2((int)items.size(), (int)(items.size() + l.size())));
        items.insert(items.end(), l.begin(), l.end());
    }
    if (range.empty() || (int)range.size() > h->cap || items.size() > (size_t)h->cap + h->chains.size())
        return fail(h, MC_E_STATE, "schedule does not fit the launch");
    for (size_t k = 0; k < h->chains.size(); ++k) h->chains[k].wg = wg[k];
    h->wg_total = (int)range.size();
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(h->d_wgmap, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
    HIPCHECK(h, hipMemcpy(h->d_wgrange, range.data(), sizeof(int2) * range.size(), hipMemcpyHostToDevice));
    return upload_desc(h);
}

int grow_buffer(mc_handle* h, double** buf, int64_t* capacity, int64_t need, bool keep) {
    if (need <= *capacity) return MC_OK;
    const int64_t cap = std::max<int64_t>(need, std::max<int64_t>(1024, 2 * *capacity));
    double* nb = nullptr;
    int rc = dalloc(h, &nb, sizeof(double) * cap);
    if (rc) return rc;
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    if (*buf) {
        if (keep) HIPCHECK(h, hipMemcpy(nb, *buf, sizeof(double) * *capacity, hipMemcpyDeviceToDevice));
        (void)hipFree(*buf);
    }
    *buf = nb;
    *capacity = cap;
    return MC_OK;
}

int launch_energy(mc_handle* h, int reset, int record_drift) {
    const int parity = (int)((h->sweeps - 1) & 1);
    if (h->fp64)
        hipLaunchKernelGGL(energy_partial_kernel<double>, dim3(h->n_eitems), dim3(256), 0, h->stream,
                           h->d_desc, h->d_eitems, parity);
    else
        hipLaunchKernelGGL(energy_partial_kernel<float>, dim3(h->n_eitems), dim3(256), 0, h->stream,
                           h->d_desc, h->d_eitems, parity);
    HIPCHECK(h, hipGetLastError());
    hipLaunchKernelGGL(energy_finalize_kernel, dim3((unsigned)h->chains.size()), dim3(64), 0, h->stream,
                       h->d_desc, reset, record_drift);
    HIPCHECK(h, hipGetLastError());
    return MC_OK;
}

int launch_rdf(mc_handle* h) {
    const int bins = h->opt.rdf_bins;
    const double rmax = h->opt.rdf_rmax;
    const double dr = rmax / (double)bins;
    const int parity = (int)((h->sweeps - 1) & 1);
    if (h->fp64)
        hipLaunchKernelGGL(rdf_kernel<double>, dim3(h->n_ritems), dim3(256), h->rdf_lds, h->stream, h->d_desc,
                           h->d_ritems, parity, rmax, dr, bins);
    else
        hipLaunchKernelGGL(rdf_kernel<float>, dim3(h->n_ritems), dim3(256), h->rdf_lds, h->stream, h->d_desc,
                           h->d_ritems, parity, rmax, dr, bins);
    HIPCHECK(h, hipGetLastError());
    h->rdf_samples += 1;
    return MC_OK;
}

// Buffers sized for a launch of n_sweeps sweeps and descriptors carrying the seed.
int prepare_launch(mc_handle* h, int64_t n_sweeps, uint64_t seed) {
    bool changed = false;
    for (Chain& c : h->chains) {
        const int64_t s_cap = c.e_capacity, d_cap = c.de_capacity;
        int rc = grow_buffer(h, &c.e_series, &c.e_capacity, h->sweeps + n_sweeps, true);
        if (!rc) rc = grow_buffer(h, &c.de_group, &c.de_capacity, n_sweeps * (int64_t)c.nb, false);
        if (rc) return rc;
        changed |= s_cap != c.e_capacity || d_cap != c.de_capacity;
    }
    bool reseed = false;
    for (Chain& c : h->chains) reseed |= c.desc.seed != seed;
    if (changed || reseed) {
        for (Chain& c : h->chains) c.desc.seed = seed;
        int rc = upload_desc(h);
        if (rc) return rc;
    }
    return MC_OK;
}

// Running energies of the launch's sweeps, then the host's sweep count.
int finish_launch(mc_handle* h, int64_t n_sweeps) {
    hipLaunchKernelGGL(energy_scan_kernel, dim3((unsigned)h->chains.size()), dim3(256), 0, h->stream, h->d_desc,
                       (int32_t)n_sweeps, (int64_t)h->sweeps);
    HIPCHECK(h, hipGetLastError());
    h->sweeps += n_sweeps;
    h->last_launch_sweeps = n_sweeps;
    return MC_OK;
}

int launch_sweeps(mc_handle* h, int64_t n_sweeps, uint64_t seed) {
    if (n_sweeps <= 0) return MC_OK;
    if (n_sweeps > kMaxLaunchSweeps) {
        int rc = launch_sweeps(h, kMaxLaunchSweeps, seed);
        if (rc) return rc;
        return launch_sweeps(h, n_sweeps - kMaxLaunchSweeps, seed);
    }
    int rc = prepare_launch(h, n_sweeps, seed);
    if (rc) return rc;
    SweepFn fn = pick_sweep(h->fp64, h->waves, h->uniform_sigma, h->da_kernel);
    Ctl ctl;
    ctl.abort = h->abort_flag;
    ctl.timeout_ticks = (uint64_t)(h->opt.wait_timeout_s * h->dev.wall_clock_hz);
    uint32_t s0 = (uint32_t)h->sweeps;
    int32_t ns = (int32_t)n_sweeps;
    const ChainDesc* dd = h->d_desc;
    const int2* wr = h->d_wgrange;
    const int2* wm = h->d_wgmap;
    void* args[] = {(void*)&dd, (void*)&wr, (void*)&wm, (void*)&s0, (void*)&ns, (void*)&ctl};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->opt.record_timing) {
        HIPCHECK(h, hipEventCreate(&e0));
        HIPCHECK(h, hipEventCreate(&e1));
        HIPCHECK(h, hipEventRecord(e0, h->stream));
    }
    HIPCHECK(h, hipLaunchCooperativeKernel((const void*)fn, dim3(h->wg_total), dim3(64 * h->waves), args, 0,
                                           h->stream));
    if (h->opt.record_timing) {
        HIPCHECK(h, hipEventRecord(e1, h->stream));
        h->ev_pending.emplace_back(e0, e1);
        h->ev_sweeps.push_back(n_sweeps);
    }
    return finish_launch(h, n_sweeps);
}

// The per-move parallel-reduction scheme: one launch per trial move, on the
// state of the single chain of the handle.
int launch_reduction(mc_handle* h, int64_t n_sweeps, uint64_t seed) {
    if (n_sweeps <= 0) return MC_OK;
    if (n_sweeps > kMaxLaunchSweeps) {
        int rc = launch_reduction(h, kMaxLaunchSweeps, seed);
        if (rc) return rc;
        return launch_reduction(h, n_sweeps - kMaxLaunchSweeps, seed);
    }
    int rc = prepare_launch(h, n_sweeps, seed);
    if (rc) return rc;
    const Chain& c = h->chains[0];
    const int nblk = (c.npad + kReduceThreads - 1) / kReduceThreads;
    if (nblk > h->r_blocks) {
        if (h->d_rparts) HIPCHECK(h, hipFree(h->d_rparts));
        h->d_rparts = nullptr;
        h->r_blocks = 0;
        if ((rc = dalloc(h, &h->d_rparts, sizeof(ReducePart) * nblk))) return rc;
        HIPCHECK(h, hipMemsetAsync(h->d_rparts, 0, sizeof(ReducePart) * nblk, h->stream));
        h->r_blocks = nblk;
    }
    if (!h->d_rctl) {
        if ((rc = dalloc(h, &h->d_rctl, sizeof(ReduceCtl)))) return rc;
        HIPCHECK(h, hipMemsetAsync(h->d_rctl, 0, sizeof(ReduceCtl), h->stream));
    }
    Ctl ctl;
    ctl.abort = h->abort_flag;
    ctl.timeout_ticks = (uint64_t)(h->opt.wait_timeout_s * h->dev.wall_clock_hz);
    const uint32_t s0 = (uint32_t)h->sweeps;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->opt.record_timing) {
        HIPCHECK(h, hipEventCreate(&e0));
        HIPCHECK(h, hipEventCreate(&e1));
        HIPCHECK(h, hipEventRecord(e0, h->stream));
    }
    for (int64_t k = 0; k < n_sweeps; ++k) {
        const uint32_t s = s0 + (uint32_t)k;
        for (int32_t i = 0; i < c.n; ++i) {
            if (h->fp64)
                hipLaunchKernelGGL(reduce_move_kernel<double>, dim3(nblk), dim3(kReduceThreads), 0, h->stream,
                                   h->d_desc, h->d_rparts, h->d_rctl, s, i, s0, ctl);
            else
                hipLaunchKernelGGL(reduce_move_kernel<float>, dim3(nblk), dim3(kReduceThreads), 0, h->stream,
                                   h->d_desc, h->d_rparts, h->d_rctl, s, i, s0, ctl);
        }
        HIPCHECK(h, hipGetLastError());
    }
    if (h->opt.record_timing) {
        HIPCHECK(h, hipEventRecord(e1, h->stream));
        h->ev_pending.emplace_back(e0, e1);
        h->ev_sweeps.push_back(n_sweeps);
    }
    return finish_launch(h, n_sweeps);
}

using LaunchFn = int (*)(mc_handle*, int64_t, uint64_t);

// After the drift monitor has switched every chain of the handle to the plain
// test, the delayed-acceptance kernel (one wave per SIMD, histograms and
// conflict tests) has nothing left to do: later launches use the plain sweep
// kernel on a schedule planned for it.  Looked at once per monitor window,
// before the next launch (a stream synchronisation); the chains' bands are
// kept, and a move log keeps the delayed-acceptance kernel (it fills the
// log).
int leave_da_kernel_if_off(mc_handle* h) {
    if (!h->da_kernel || h->opt.log_moves > 0 || h->da_window <= 0 || h->da_checked == h->sweeps ||
        h->sweeps % h->da_window != 0)
        return MC_OK;
    h->da_checked = h->sweeps;
    int rc = sync_check(h);
    if (rc) return rc;
    for (Chain& c : h->chains) {
        int32_t active = 0;
        HIPCHECK(h, hipMemcpy(&active, &c.da->active, sizeof(active), hipMemcpyDeviceToHost));
        if (active) return MC_OK;
    }
    h->da_kernel = false;
    std::vector<int> wg;
    WgLists lists;
    plan_schedule(h, wg, lists);
    return apply_schedule(h, wg, lists);
}

int last_launch_ms(mc_handle* h, std::vector<double>& ms);

// n_sweeps sweeps in launches that end at every re-sum, g(r) and monitor
// interval boundary, with the re-sums and samples due there.  With
// chain_ms the device time of every chain is summed over the launches.
int sweep_all(mc_handle* h, int64_t n_sweeps, uint64_t seed, LaunchFn launch = launch_sweeps,
              std::vector<double>* chain_ms = nullptr) {
    if (n_sweeps < 0 || h->sweeps + n_sweeps > (int64_t)UINT32_MAX)
        return fail(h, MC_E_ARG, "n_sweeps out of range");
    if (chain_ms) chain_ms->assign(h->chains.size(), 0.0);
    int64_t left = n_sweeps;
    while (left > 0) {
        int rc = leave_da_kernel_if_off(h);
        if (rc) return rc;
        int64_t step = left;
        const int re = h->opt.resum_every, rd = h->opt.rdf_every;
        if (re > 0) step = std::min<int64_t>(step, re - h->sweeps % re);
        if (rd > 0) step = std::min<int64_t>(step, rd - h->sweeps % rd);
        const int dw = h->da_window;  // the drift monitor judges at window ends
        if (dw > 0) step = std::min<int64_t>(step, dw - h->sweeps % dw);
        if ((rc = launch(h, step, seed))) return rc;
        if (chain_ms) {
            std::vector<double> ms;
            if ((rc = last_launch_ms(h, ms))) return rc;
            for (size_t k = 0; k < ms.size(); ++k) (*chain_ms)[k] += ms[k];
        }
        left -= step;
        if (re > 0 && h->sweeps % re == 0 && (rc = launch_energy(h, 1, 1))) return rc;
        if (rd > 0 && h->sweeps % rd == 0 && (rc = launch_rdf(h))) return rc;
    }
    return MC_OK;
}

// Builds a handle from validated chain specs.
int create_handle(int32_t n_chains, const mc_chain_spec* specs, const mc_options& opt, mc_handle** out) {
    mc_handle* h = new (std::nothrow) mc_handle();
    if (!h) return fail(nullptr, MC_E_OOM, "host allocation failed");
    std::string derr;
    if (!device_info(h->dev, derr)) {
        delete h;
        return fail(nullptr, MC_E_DEVICE, derr);
    }
    h->opt = opt;
    h->fp64 = opt.precision == MC_FP64;
    h->waves = opt.waves ? opt.waves : 4;
    h->chains.resize(n_chains);
    h->uniform_sigma = true;
    for (int k = 0; k < n_chains; ++k) {
        setup_chain(h->chains[k], specs[k], opt);
        h->uniform_sigma = h->uniform_sigma && h->chains[k].uniform_sigma;
    }
    // Automatic waves per workgroup: eight for float chains of at least three
    // groups per CU in all (measured, for one chain and for the 256-chain
    // ensemble: from there on the workgroups serve several targets a sweep,
    // the launch is bound by the pair terms rather than by the decision
    // chain, and sixteen waves per CU, each taking whole decided groups, are
    // the faster), four otherwise and when moves are logged (the
    // delayed-acceptance kernels have four waves).
    int64_t groups = 0;
    for (const Chain& c : h->chains) groups += c.nb;
    if (opt.waves == 0 && !h->fp64 && opt.log_moves == 0 && groups >= 3 * h->dev.cus)
        h->waves = 8;
    // the float kernels for per-ion diameters and with eight waves hold
    // fewer band groups
    if (!h->fp64) {
        const int cap = h->waves == 8 ? (h->uniform_sigma ? kMaxBandWide : kMaxBandWidePerIon)
                                      : (h->uniform_sigma ? kMaxBand : kMaxBandPerIon);
        for (Chain& c : h->chains) c.band = std::min(c.band, cap);
    }

    int rc = MC_OK;
    auto bail = [&](int code) {
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        std::string m = h->err;
        free_all(h);
        delete h;
        g_create_error = m;
        return code;
    };
    if (opt.hip_stream) {
        h->stream = (hipStream_t)opt.hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
            h->err = "hipStreamCreate failed";
            return bail(MC_E_DEVICE);
        }
        h->own_stream = true;
    }

    // co-residency of the sweep kernel: every workgroup of the cooperative
    // grid must be resident at once
    SweepFn fn = pick_sweep(h->fp64, h->waves, h->uniform_sigma);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, 64 * h->waves, 0) != hipSuccess ||
        per_cu < 1) {
        h->err = "occupancy query failed for the sweep kernel";
        return bail(MC_E_DEVICE);
    }
    // The occupancy query has been seen to over-promise for workgroups with
    // more than 64 KiB of LDS: such kernels get one workgroup per CU.
    // Kernels that spill to scratch have been seen to run fewer workgroups at
    // once than the query reports: they also get one workgroup per CU.
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, (const void*)fn) == hipSuccess &&
        (fa.sharedSizeBytes > 64 * 1024 || fa.localSizeBytes > 0))
        per_cu = 1;
    h->cap = per_cu * h->dev.cus;
    if (h->waves == 4) {
        // co-residency of the delayed-acceptance kernel (schedules are re-planned
        // for it when it is switched on)
        SweepFn fd = pick_sweep(h->fp64, 4, h->uniform_sigma, true);
        int pd = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pd, (const void*)fd, 256, 0) != hipSuccess || pd < 1) {
            h->err = "occupancy query failed for the delayed-acceptance kernel";
            return bail(MC_E_DEVICE);
        }
        if (hipFuncGetAttributes(&fa, (const void*)fd) == hipSuccess &&
            (fa.sharedSizeBytes > 64 * 1024 || fa.localSizeBytes > 0))
            pd = 1;
        h->cap_da = pd * h->dev.cus;
    }
    if (n_chains > h->cap || (opt.log_moves > 0 && n_chains > h->cap_da)) {
        h->err = "more chains (" + std::to_string(n_chains) + ") than co-resident workgroups (" +
                 std::to_string(h->cap) + ")";
        return bail(MC_E_ARG);
    }
    h->wg_budget = opt.workgroups > 0 ? std::max(n_chains, std::min(opt.workgroups, h->cap)) : h->cap;

    // device memory: one arena for the fixed-size buffers
    const size_t t4 = h->fp64 ? sizeof(double4) : sizeof(float4);
    const size_t t1 = h->fp64 ? sizeof(double) : sizeof(float);
    ArenaPlan plan;
    plan.add(&h->abort_flag, sizeof(int));
    plan.add(&h->d_desc, sizeof(ChainDesc) * n_chains);
    plan.add(&h->d_wgmap, sizeof(int2) * (h->cap + n_chains));
    plan.add(&h->d_wgrange, sizeof(int2) * h->cap);
    int n_e = 0, n_r = 0;
    size_t max_hist = 0;
    for (Chain& c : h->chains) {
        n_e += (c.nb + 1) / 2;
        n_r += c.nb;
        const size_t nt = c.species.size();
        max_hist = std::max(max_hist, nt * nt * (size_t)opt.rdf_bins);
    }
    h->n_eitems = n_e;
    h->n_ritems = n_r;
    h->rdf_lds = sizeof(unsigned int) * max_hist;
    plan.add(&h->d_eitems, sizeof(BlockItem) * n_e);
    plan.add(&h->d_ritems, sizeof(BlockItem) * n_r);
    for (Chain& c : h->chains) {
        const size_t nt = c.species.size();
        plan.add(&c.pos, 2 * t4 * c.npad);
        plan.add(&c.half, t1 * c.npad);
        plan.add(&c.charge, t1 * c.npad);
        plan.add(&c.wall_a, sizeof(double) * c.npad);
        plan.add(&c.d_type, sizeof(int32_t) * c.npad);
        plan.add(&c.rec, sizeof(GroupRec) * kRing);
        plan.add(&c.stats, sizeof(unsigned long long) * ST_N);
        plan.add(&c.clk, sizeof(unsigned long long) * 2);
        plan.add(&c.e_partial, sizeof(double) * ((c.nb + 1) / 2));
        plan.add(&c.aux, sizeof(EnergyAux));
        plan.add(&c.e_state, sizeof(double));
        plan.add(&c.sweep_tot, sizeof(double) * kMaxLaunchSweeps);
        plan.add(&c.rdf_counts, sizeof(unsigned long long) * nt * nt * opt.rdf_bins);
        plan.add(&c.rdf_centres, sizeof(unsigned long long) * nt);
        plan.add(&c.da, sizeof(DAState));
        if (c.trace_cap > 0) {
            plan.add(&c.trace_acc, (size_t)c.trace_cap);
            plan.add(&c.trace_de, sizeof(double) * c.trace_cap);
        }
    }
    if ((rc = dalloc(h, &h->arena, plan.size))) return bail(rc);
    plan.assign(h->arena);
    // zero everything once (the handle's stream is non-blocking: drain it
    // before the synchronous uploads below)
    if (hipMemsetAsync(h->arena, 0, plan.size, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        h->err = "clearing device memory failed";
        return bail(MC_E_DEVICE);
    }

    // host images and uploads, chain by chain
    std::vector<BlockItem> eitems, ritems;
    for (int k = 0; k < n_chains; ++k) {
        Chain& c = h->chains[k];
        const mc_chain_spec& sp = specs[k];
        for (int p = 0; p < (c.nb + 1) / 2; ++p) eitems.push_back(BlockItem{k, p});
        for (int r = 0; r < c.nb; ++r) ritems.push_back(BlockItem{k, r});
        // positions carry the version tag of the sweep that produced them;
        // the initial state is the result of virtual sweeps -2 (parity 0)
        // and -1 (parity 1)
        std::vector<char> hpos(2 * t4 * c.npad), hhalf(t1 * c.npad), hq(t1 * c.npad);
        std::vector<double> hwall(c.npad, 0.0);
        for (int i = 0; i < c.npad; ++i) {
            double x, y, z, qq, hh;
            if (i < c.n) {
                x = sp.positions[3 * i];
                y = sp.positions[3 * i + 1];
                z = sp.positions[3 * i + 2];
                qq = sp.charges[i];
                hh = 0.5 * sp.diameters[i];
                hwall[i] = c.R - 0.5 * sp.diameters[i];
            } else {
                // inert padding ion: no charge, no size, far from everything and from each other
                x = 1.0e6 * (double)(i - c.n + 1);
                y = -2.0e6;
                z = 3.0e6;
                qq = 0.0;
                hh = 0.0;
            }
            for (int par = 0; par < 2; ++par) {
                const uint32_t ver = par == 0 ? 0xFFFFFFFEu : 0xFFFFFFFFu;
                char* dst = &hpos[t4 * ((size_t)par * c.npad + i)];
                if (h->fp64) {
                    struct { double x, y, z; uint32_t ver, pad; } r{x, y, z, ver, 0u};
                    std::memcpy(dst, &r, t4);
                } else {
                    struct { float x, y, z; uint32_t ver; } r{(float)x, (float)y, (float)z, ver};
                    std::memcpy(dst, &r, t4);
                }
            }
            if (h->fp64) {
                std::memcpy(&hhalf[t1 * i], &hh, t1);
                std::memcpy(&hq[t1 * i], &qq, t1);
            } else {
                float hf = (float)hh, qf = (float)qq;
                std::memcpy(&hhalf[t1 * i], &hf, t1);
                std::memcpy(&hq[t1 * i], &qf, t1);
            }
        }
        std::vector<GroupRec> hrec(kRing);
        for (int q = 0; q < kRing; ++q) {
            const int64_t g = (int64_t)q - kRing;  // virtual groups -kRing..-1: decided, nothing accepted
            hrec[(size_t)(g & (kRing - 1))] = GroupRec{(uint32_t)(g + 1), 0u, 0ull};
        }
        hipError_t e = hipSuccess;
        if ((e = hipMemcpy(c.pos, hpos.data(), hpos.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.half, hhalf.data(), hhalf.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.charge, hq.data(), hq.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.wall_a, hwall.data(), sizeof(double) * c.npad, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.d_type, c.type.data(), sizeof(int32_t) * c.npad, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.rec, hrec.data(), sizeof(GroupRec) * kRing, hipMemcpyHostToDevice)) != hipSuccess) {
            h->err = std::string("upload failed: ") + hipGetErrorString(e);
            return bail(MC_E_DEVICE);
        }
        if (c.trace_cap) {
            std::vector<uint8_t> ff((size_t)c.trace_cap, 0xFF);
            if ((e = hipMemcpy(c.trace_acc, ff.data(), ff.size(), hipMemcpyHostToDevice)) != hipSuccess) {
                h->err = std::string("upload failed: ") + hipGetErrorString(e);
                return bail(MC_E_DEVICE);
            }
        }
    }
    {
        hipError_t e = hipSuccess;
        if ((e = hipMemcpy(h->d_eitems, eitems.data(), sizeof(BlockItem) * eitems.size(), hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(h->d_ritems, ritems.data(), sizeof(BlockItem) * ritems.size(), hipMemcpyHostToDevice)) !=
                hipSuccess) {
            h->err = std::string("upload failed: ") + hipGetErrorString(e);
            return bail(MC_E_DEVICE);
        }
    }
    for (Chain& c : h->chains) {
        if ((rc = grow_buffer(h, &c.e_series, &c.e_capacity, 1024, false))) return bail(rc);
        DAState z{};
        z.fallback_sweep = -1;
        z.ref_rate = -1.0;
        z.last_rate = -1.0;
        z.min_count = 64;
        if (hipMemcpy(c.da, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) {
            h->err = "upload failed";
            return bail(MC_E_DEVICE);
        }
        if (opt.log_moves > 0) {
            c.log_cap = opt.log_moves;
            if ((rc = dalloc(h, &c.log_feat, sizeof(uint32_t) * 64 * (size_t)c.log_cap)) ||
                (rc = dalloc(h, &c.log_de, sizeof(double) * c.log_cap)) ||
                (rc = dalloc(h, &c.log_deh, sizeof(double) * c.log_cap)) ||
                (rc = dalloc(h, &c.log_flags, (size_t)c.log_cap)))
                return bail(rc);
            if (hipMemset(c.log_flags, 0, (size_t)c.log_cap) != hipSuccess) {
                h->err = "clearing the log failed";
                return bail(MC_E_DEVICE);
            }
        }
    }
    if (opt.log_moves > 0) {
        // logging runs the delayed-acceptance kernel (features)
        h->da_kernel = true;
        for (Chain& c : h->chains) c.band = std::min(c.band, kDaMaxBand);
    }
    std::vector<int> wg;
    WgLists lists;
    plan_schedule(h, wg, lists);
    if ((rc = apply_schedule(h, wg, lists))) return bail(rc);
    // An automatic band on the eight-wave float kernels: 1 for a chain whose
    // workgroups each serve at least four of its groups a sweep in the
    // schedule planned here (the pair terms bound such a chain, and the band
    // tiles, which evaluate both outcomes of every partner, are extra work;
    // measured 8 % faster on the 256-chain ensemble), the wider band
    // otherwise (it hides the decision chain).  Fixed here: later schedules
    // (the autotuner's) leave a chain's arithmetic, and so its trajectory,
    // unchanged.
    if (opt.band < 0 && h->waves == 8 && !h->fp64) {
        bool narrowed = false;
        for (Chain& c : h->chains)
            if (c.band > 1 && c.nb >= 4 * c.wg) {
                c.band = 1;
                narrowed = true;
            }
        if (narrowed && (rc = upload_desc(h))) return bail(rc);
    }
    // initial energy: re-sum into the running energy
    if ((rc = launch_energy(h, 1, 0))) return bail(rc);
    if ((rc = sync_check(h))) return bail(rc);
    *out = h;
    return MC_OK;
}

int check_options(const mc_options& opt) {
    if (opt.precision != MC_FP64 && opt.precision != MC_FP32_ACC64)
        return fail(nullptr, MC_E_ARG, "unknown precision");
    if (!is_finite(opt.max_disp) || opt.max_disp <= 0) return fail(nullptr, MC_E_ARG, "max_disp must be > 0");
    if (opt.resum_every < 0 || opt.rdf_every < 0) return fail(nullptr, MC_E_ARG, "negative interval");
    if (opt.rdf_bins < 1 || opt.rdf_bins > 4096 || !is_finite(opt.rdf_rmax) || opt.rdf_rmax <= 0)
        return fail(nullptr, MC_E_ARG, "rdf_bins must be in [1, 4096] and rdf_rmax > 0");
    if (!is_finite(opt.rdf_margin) || opt.rdf_margin < 0)
        return fail(nullptr, MC_E_ARG, "rdf_margin must be finite and >= 0");
    if (opt.band < -1 || opt.band > kMaxBand) return fail(nullptr, MC_E_ARG, "band out of range");
    if (opt.waves != 0 && opt.waves != 4 && opt.waves != 8) return fail(nullptr, MC_E_ARG, "waves must be 0, 4 or 8");
    if (opt.workgroups < 0 || opt.trace_moves < 0) return fail(nullptr, MC_E_ARG, "negative count");
    if (!is_finite(opt.wait_timeout_s) || opt.wait_timeout_s <= 0) return fail(nullptr, MC_E_ARG, "bad wait_timeout_s");
    if (!is_finite(opt.da_rcut) || opt.da_rcut <= 0 || opt.da_window < 0 || !is_finite(opt.da_delta) ||
        opt.da_delta < 0 || opt.log_moves < 0)
        return fail(nullptr, MC_E_ARG, "bad delayed-acceptance options");
    if (opt.log_moves > 0 && opt.waves == 8)
        return fail(nullptr, MC_E_ARG, "move logging needs 4 waves per workgroup");
    return MC_OK;
}

Chain* get_chain(mc_handle* h, int32_t c) {
    if (!h || c < 0 || c >= (int32_t)h->chains.size()) return nullptr;
    return &h->chains[c];
}

int chain_energy(mc_handle* h, int32_t ci, double* e_running, double* e_exact) {
    Chain* c = get_chain(h, ci);
    if (!c || !e_running) return h ? fail(h, MC_E_ARG, "bad chain index or null output") : MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    HIPCHECK(h, hipMemcpy(e_running, c->e_state, sizeof(double), hipMemcpyDeviceToHost));
    if (e_exact) {
        if ((rc = launch_energy(h, 0, 0))) return rc;
        if ((rc = sync_check(h))) return rc;
        EnergyAux a;
        HIPCHECK(h, hipMemcpy(&a, c->aux, sizeof(EnergyAux), hipMemcpyDeviceToHost));
        *e_exact = a.e_resum;
    }
    return MC_OK;
}

int chain_rdf(mc_handle* h, int32_t ci, int32_t bins, double* g, uint64_t* counts, uint64_t* centres,
              int64_t* n_samples) {
    Chain* c = get_chain(h, ci);
    if (!c) return h ? fail(h, MC_E_ARG, "bad chain index") : MC_E_ARG;
    if (bins != h->opt.rdf_bins) return fail(h, MC_E_ARG, "bins differs from the handle's rdf_bins");
    int rc = sync_check(h);
    if (rc) return rc;
    const size_t nt = c->species.size();
    const size_t nh = nt * nt * (size_t)bins;
    std::vector<unsigned long long> cnt(nh), ce(nt);
    HIPCHECK(h, hipMemcpy(cnt.data(), c->rdf_counts, sizeof(unsigned long long) * nh, hipMemcpyDeviceToHost));
    HIPCHECK(h, hipMemcpy(ce.data(), c->rdf_centres, sizeof(unsigned long long) * nt, hipMemcpyDeviceToHost));
    if (counts)
        for (size_t k = 0; k < nh; ++k) counts[k] = cnt[k];
    if (centres)
        for (size_t k = 0; k < nt; ++k) centres[k] = ce[k];
    if (n_samples) *n_samples = h->rdf_samples;
    if (g) {
        const double rmax = h->opt.rdf_rmax, dr = rmax / (double)bins;
        const double pi = 3.14159265358979323846;
        for (size_t a = 0; a < nt; ++a)
            for (size_t b = 0; b < nt; ++b) {
                const double rb = c->R - 0.5 * c->species[b].second;
                const double vb = 4.0 / 3.0 * pi * rb * rb * rb;
                const double nbd = (double)(c->n_of_type[b] - (a == b ? 1 : 0)) / vb;
                for (int k = 0; k < bins; ++k) {
                    const double r0 = k * dr, r1 = (k + 1) * dr;
                    const double vk = 4.0 / 3.0 * pi * (r1 * r1 * r1 - r0 * r0 * r0);
                    const double den = (double)ce[a] * nbd * vk;
                    g[(a * nt + b) * bins + k] = den > 0 ? (double)cnt[(a * nt + b) * bins + k] / den : 0.0;
                }
            }
    }
    return MC_OK;
}

int chain_species(const mc_handle* h, int32_t ci, int32_t* ntypes, double* q, double* s) {
    if (!h || ci < 0 || ci >= (int32_t)h->chains.size()) return MC_E_ARG;
    const Chain& c = h->chains[ci];
    if (ntypes) *ntypes = (int32_t)c.species.size();
    for (size_t k = 0; k < c.species.size(); ++k) {
        if (q) q[k] = c.species[k].first;
        if (s) s[k] = c.species[k].second;
    }
    return MC_OK;
}

int chain_positions(mc_handle* h, int32_t ci, double* xyz) {
    Chain* c = get_chain(h, ci);
    if (!c || !xyz) return h ? fail(h, MC_E_ARG, "bad chain index or null output") : MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    const int parity = (int)((h->sweeps - 1) & 1);
    if (h->fp64) {
        std::vector<double4> v(c->n);
        HIPCHECK(h, hipMemcpy(v.data(), (double4*)c->pos + (size_t)parity * c->npad, sizeof(double4) * c->n,
                              hipMemcpyDeviceToHost));
        for (int i = 0; i < c->n; ++i) {
            xyz[3 * i] = v[i].x;
            xyz[3 * i + 1] = v[i].y;
            xyz[3 * i + 2] = v[i].z;
        }
    } else {
        std::vector<float4> v(c->n);
        HIPCHECK(h, hipMemcpy(v.data(), (float4*)c->pos + (size_t)parity * c->npad, sizeof(float4) * c->n,
                              hipMemcpyDeviceToHost));
        for (int i = 0; i < c->n; ++i) {
            xyz[3 * i] = v[i].x;
            xyz[3 * i + 1] = v[i].y;
            xyz[3 * i + 2] = v[i].z;
        }
    }
    return MC_OK;
}

int chain_trace(mc_handle* h, int32_t ci, int64_t n_moves, uint8_t* acc, double* dE) {
    Chain* c = get_chain(h, ci);
    if (!c) return h ? fail(h, MC_E_ARG, "bad chain index") : MC_E_ARG;
    if (n_moves < 0 || n_moves > c->trace_cap || n_moves > h->sweeps * (int64_t)c->n)
        return fail(h, MC_E_ARG, "n_moves exceeds the traced moves");
    int rc = sync_check(h);
    if (rc) return rc;
    if (acc && n_moves) HIPCHECK(h, hipMemcpy(acc, c->trace_acc, (size_t)n_moves, hipMemcpyDeviceToHost));
    if (dE && n_moves) HIPCHECK(h, hipMemcpy(dE, c->trace_de, sizeof(double) * n_moves, hipMemcpyDeviceToHost));
    return MC_OK;
}

int chain_energy_series(mc_handle* h, int32_t ci, int64_t n, double* e) {
    Chain* c = get_chain(h, ci);
    if (!c) return h ? fail(h, MC_E_ARG, "bad chain index") : MC_E_ARG;
    if (n < 0 || n > h->sweeps || (n && !e)) return fail(h, MC_E_ARG, "n exceeds the sweeps done");
    int rc = sync_check(h);
    if (rc) return rc;
    if (n) HIPCHECK(h, hipMemcpy(e, c->e_series, sizeof(double) * n, hipMemcpyDeviceToHost));
    return MC_OK;
}

int chain_stats(mc_handle* h, int32_t ci, mc_stats* out) {
    Chain* c = get_chain(h, ci);
    if (!c || !out) return h ? fail(h, MC_E_ARG, "bad chain index or null output") : MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    unsigned long long st[ST_N];
    EnergyAux a;
    HIPCHECK(h, hipMemcpy(st, c->stats, sizeof(st), hipMemcpyDeviceToHost));
    HIPCHECK(h, hipMemcpy(&a, c->aux, sizeof(a), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->sweeps = h->sweeps;
    out->moves = (int64_t)st[ST_MOVES];
    out->accepted = (int64_t)st[ST_ACC];
    out->rejected_wall = (int64_t)st[ST_WALL];
    out->rejected_overlap = (int64_t)st[ST_OVERLAP];
    out->rejected_metropolis = (int64_t)st[ST_METRO];
    out->fixpoint_iterations = (int64_t)st[ST_ITERS];
    out->early_groups = (int64_t)st[ST_EARLY];
    out->resums = (int64_t)a.n_resum;
    out->last_drift = a.drift_last;
    out->max_abs_drift = a.drift_max;
    out->band = c->band;
    out->waves = h->waves;
    out->workgroups = c->wg;
    DAState ds;
    HIPCHECK(h, hipMemcpy(&ds, c->da, sizeof(ds), hipMemcpyDeviceToHost));
    out->da_active = ds.active && c->da_w != nullptr ? 1 : 0;
    out->da_moves = (int64_t)st[ST_DA_MOVES];
    out->da_conflicts = (int64_t)st[ST_DA_CONFLICTS];
    out->da_stage1_rejected = (int64_t)st[ST_DA_S1REJ];
    out->da_stage1_passed = (int64_t)st[ST_DA_S1PASS];
    out->da_stage2_rejected = (int64_t)st[ST_DA_S2REJ];
    out->da_fallback_sweep = ds.fallback_sweep;
    out->da_last_rate = ds.last_rate;
    out->da_kernel = h->da_kernel ? 1 : 0;
    return MC_OK;
}

int chain_set_max_disp(mc_handle* h, int32_t ci, double max_disp) {
    Chain* c = get_chain(h, ci);
    if (!c) return h ? fail(h, MC_E_ARG, "bad chain index") : MC_E_ARG;
    if (!is_finite(max_disp) || max_disp <= 0) return fail(h, MC_E_ARG, "max_disp must be > 0");
    c->D = 2.0 * max_disp;
    return upload_desc(h);
}

// Device time of the last sweep launch for every chain, in milliseconds, from
// the chain clocks (launch start to the chain's last published group).
int last_launch_ms(mc_handle* h, std::vector<double>& ms) {
    int rc = sync_check(h);
    if (rc) return rc;
    ms.assign(h->chains.size(), 0.0);
    for (size_t k = 0; k < h->chains.size(); ++k) {
        unsigned long long clk[2];
        HIPCHECK(h, hipMemcpy(clk, h->chains[k].clk, sizeof(clk), hipMemcpyDeviceToHost));
        ms[k] = clk[1] > clk[0] ? 1e3 * (double)(clk[1] - clk[0]) / h->dev.wall_clock_hz : 0.0;
    }
    return MC_OK;
}

}  // namespace

int mc_internal_log(mc_handle* h, int32_t chain, MCLogView* out) {
    Chain* c = get_chain(h, chain);
    if (!c || !out) return h ? fail(h, MC_E_ARG, "bad chain index") : MC_E_ARG;
    if (c->log_cap == 0) return fail(h, MC_E_ARG, "the chain has no move log (log_moves)");
    int rc = sync_check(h);
    if (rc) return rc;
    out->feat = c->log_feat;
    out->de = c->log_de;
    out->flags = c->log_flags;
    out->cap = c->log_cap;
    out->lB = c->lB;
    out->stream = h->stream;
    return MC_OK;
}

int mc_internal_fail(mc_handle* h, int code, const char* msg) { return fail(h, code, msg); }

void mc_internal_note_error(const char* msg) { g_create_error = msg ? msg : "unknown error"; }

namespace {

// ---- checkpoints --------------------------------------------------------
// File layout (host byte order): magic "MCCKPT01", then int32 version,
// n_chains, sizeof(mc_options), ST_N; int64 sweeps, rdf_samples; the options
// (hip_stream zeroed); per chain: int32 n, species, rdf_bins, chain_id;
// double R, l_B, max_disp, running energy; EnergyAux; uint64 stats[ST_N];
// double charges[n], diameters[n], positions[3n] (after the last sweep),
// previous[3n] (after the one before); uint64 accept masks of the last kRing
// groups (oldest first); uint64 counts[nt*nt*bins], centres[nt]; int64 m;
// double energy_series[m].
constexpr char kCkptMagic[8] = {'M', 'C', 'C', 'K', 'P', 'T', '0', '1'};
constexpr int32_t kCkptVersion = 1;

struct CkptChain {
    int32_t n = 0, nt = 0, bins = 0;
    uint32_t chain_id = 0;
    double R = 0, lB = 0, max_disp = 0, e_run = 0;
    EnergyAux aux{};
    unsigned long long stats[ST_N] = {};
    std::vector<double> q, sigma, xyz, prev, series;
    std::vector<uint64_t> masks;  // [kRing], oldest group first
    std::vector<unsigned long long> counts, centres;
};

struct File {
    FILE* f = nullptr;
    explicit File(FILE* x) : f(x) {}
    ~File() {
        if (f) fclose(f);
    }
    template <typename T> bool put(const T* v, size_t k) { return fwrite(v, sizeof(T), k, f) == k; }
    template <typename T> bool get(T* v, size_t k) { return fread(v, sizeof(T), k, f) == k; }
};

// Positions [n][3] of the image of the given parity.
int read_image(mc_handle* h, const Chain& c, int parity, double* xyz) {
    if (h->fp64) {
        std::vector<double4> v(c.n);
        HIPCHECK(h, hipMemcpy(v.data(), (double4*)c.pos + (size_t)parity * c.npad, sizeof(double4) * c.n,
                              hipMemcpyDeviceToHost));
        for (int i = 0; i < c.n; ++i) {
            xyz[3 * i] = v[i].x;
            xyz[3 * i + 1] = v[i].y;
            xyz[3 * i + 2] = v[i].z;
        }
    } else {
        std::vector<float4> v(c.n);
        HIPCHECK(h, hipMemcpy(v.data(), (float4*)c.pos + (size_t)parity * c.npad, sizeof(float4) * c.n,
                              hipMemcpyDeviceToHost));
        for (int i = 0; i < c.n; ++i) {
            xyz[3 * i] = v[i].x;
            xyz[3 * i + 1] = v[i].y;
            xyz[3 * i + 2] = v[i].z;
        }
    }
    return MC_OK;
}

// Writes both position images and the group-record ring as a finished sweep
// s0 - 1 leaves them: the image of sweep s0 - 1 holds xyz, that of sweep
// s0 - 2 holds prev, and the last kRing groups before sweep s0 are decided
// with the accept masks given (oldest first; all rejected when masks is
// NULL).  Every reader then sees the state exactly as the sweep kernel
// wrote it.
int write_start(mc_handle* h, Chain& c, const double* xyz, const double* prev, const uint64_t* masks,
                int64_t s0) {
    const size_t t4 = h->fp64 ? sizeof(double4) : sizeof(float4);
    std::vector<char> img(2 * t4 * c.npad);
    HIPCHECK(h, hipMemcpy(img.data(), c.pos, img.size(), hipMemcpyDeviceToHost));
    for (int par = 0; par < 2; ++par) {
        // parity (s0 - 1) & 1 holds sweep s0 - 1, the other one sweep s0 - 2
        const bool last = par == ((s0 - 1) & 1);
        const uint32_t ver = (uint32_t)(last ? s0 - 1 : s0 - 2);
        const double* src = last ? xyz : prev;
        for (int i = 0; i < c.npad; ++i) {
            char* dst = &img[t4 * ((size_t)par * c.npad + i)];
            if (h->fp64) {
                struct { double x, y, z; uint32_t ver, pad; } r;
                std::memcpy(&r, dst, t4);
                if (i < c.n) {
                    r.x = src[3 * i];
                    r.y = src[3 * i + 1];
                    r.z = src[3 * i + 2];
                }
                r.ver = ver;
                std::memcpy(dst, &r, t4);
            } else {
                struct { float x, y, z; uint32_t ver; } r;
                std::memcpy(&r, dst, t4);
                if (i < c.n) {
                    r.x = (float)src[3 * i];
                    r.y = (float)src[3 * i + 1];
                    r.z = (float)src[3 * i + 2];
                }
                r.ver = ver;
                std::memcpy(dst, &r, t4);
            }
        }
    }
    HIPCHECK(h, hipMemcpy(c.pos, img.data(), img.size(), hipMemcpyHostToDevice));
    std::vector<GroupRec> ring(kRing);
    const int64_t g0 = s0 * (int64_t)c.nb;
    for (int q = 0; q < kRing; ++q) {
        const int64_t g = g0 - kRing + q;
        ring[(size_t)(g & (kRing - 1))] = GroupRec{(uint32_t)(g + 1), 0u, masks ? masks[q] : 0ull};
    }
    HIPCHECK(h, hipMemcpy(c.rec, ring.data(), sizeof(GroupRec) * kRing, hipMemcpyHostToDevice));
    return MC_OK;
}

}  // namespace

extern "C" {

int mc_options_init(mc_options* o) {
    if (!o) return MC_E_ARG;
    std::memset(o, 0, sizeof(*o));
    o->precision = MC_FP32_ACC64;
    o->max_disp = 0.5;
    o->resum_every = 100;
    o->rdf_every = 0;
    o->rdf_bins = 200;
    o->rdf_rmax = 10.0;
    o->rdf_margin = 0.0;
    o->chain_id = 0;
    o->hip_stream = nullptr;
    o->band = -1;
    o->waves = 0;
    o->workgroups = 0;
    o->trace_moves = 0;
    o->wait_timeout_s = 20.0;
    o->da_rcut = 4.0;
    o->da_window = 10;
    o->da_delta = 0.05;
    o->log_moves = 0;
    return MC_OK;
}

int mc_create(int32_t n, const double* charges, const double* diameters, const double* positions,
              double radius, double l_B, const mc_options* opt_in, mc_handle** out) {
    if (!out) return fail(nullptr, MC_E_ARG, "out is NULL");
    *out = nullptr;
    mc_options opt;
    mc_options_init(&opt);
    if (opt_in) opt = *opt_in;
    int rc = check_options(opt);
    if (rc) return rc;
    mc_chain_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.n = n;
    sp.charges = charges;
    sp.diameters = diameters;
    sp.positions = positions;
    sp.radius = radius;
    sp.l_B = l_B;
    sp.max_disp = opt.max_disp;
    sp.chain_id = opt.chain_id;
    if ((rc = validate_chain(sp, opt, ""))) return rc;
    return create_handle(1, &sp, opt, out);
}

int mc_create_batch(int32_t n_chains, const mc_chain_spec* chains, const mc_options* opt_in, mc_handle** out) {
    if (!out) return fail(nullptr, MC_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_chains < 1 || !chains) return fail(nullptr, MC_E_ARG, "need n_chains >= 1 and a chain array");
    mc_options opt;
    mc_options_init(&opt);
    if (opt_in) opt = *opt_in;
    int rc = check_options(opt);
    if (rc) return rc;
    for (int k = 0; k < n_chains; ++k)
        if ((rc = validate_chain(chains[k], opt, "chain " + std::to_string(k) + ": "))) return rc;
    return create_handle(n_chains, chains, opt, out);
}

int mc_save(mc_handle* h, const char* path) {
    if (!h) return MC_E_ARG;
    if (!path) return fail(h, MC_E_ARG, "path is NULL");
    int rc = sync_check(h);
    if (rc) return rc;
    std::vector<CkptChain> cs(h->chains.size());
    for (size_t k = 0; k < h->chains.size(); ++k) {
        Chain& c = h->chains[k];
        CkptChain& o = cs[k];
        o.n = c.n;
        o.nt = (int32_t)c.species.size();
        o.bins = h->opt.rdf_bins;
        o.chain_id = c.chain_id;
        o.R = c.R;
        o.lB = c.lB;
        o.max_disp = 0.5 * c.D;
        o.q.resize(c.n);
        o.sigma.resize(c.n);
        for (int i = 0; i < c.n; ++i) {
            o.q[i] = c.species[(size_t)c.type[i]].first;
            o.sigma[i] = c.species[(size_t)c.type[i]].second;
        }
        o.xyz.resize(3 * (size_t)c.n);
        o.prev.resize(3 * (size_t)c.n);
        if ((rc = read_image(h, c, (int)((h->sweeps - 1) & 1), o.xyz.data())) ||
            (rc = read_image(h, c, (int)(h->sweeps & 1), o.prev.data())))
            return rc;
        std::vector<GroupRec> ring(kRing);
        HIPCHECK(h, hipMemcpy(ring.data(), c.rec, sizeof(GroupRec) * kRing, hipMemcpyDeviceToHost));
        o.masks.resize(kRing);
        const int64_t g0 = h->sweeps * (int64_t)c.nb;
        for (int q = 0; q < kRing; ++q) {
            const int64_t g = g0 - kRing + q;
            const GroupRec& r = ring[(size_t)(g & (kRing - 1))];
            if (r.tag != (uint32_t)(g + 1)) return fail(h, MC_E_STATE, "group record ring out of step");
            o.masks[q] = r.acc;
        }
        HIPCHECK(h, hipMemcpy(&o.e_run, c.e_state, sizeof(double), hipMemcpyDeviceToHost));
        HIPCHECK(h, hipMemcpy(&o.aux, c.aux, sizeof(EnergyAux), hipMemcpyDeviceToHost));
        HIPCHECK(h, hipMemcpy(o.stats, c.stats, sizeof(o.stats), hipMemcpyDeviceToHost));
        o.counts.resize((size_t)o.nt * o.nt * o.bins);
        o.centres.resize((size_t)o.nt);
        HIPCHECK(h, hipMemcpy(o.counts.data(), c.rdf_counts, sizeof(unsigned long long) * o.counts.size(),
                              hipMemcpyDeviceToHost));
        HIPCHECK(h, hipMemcpy(o.centres.data(), c.rdf_centres, sizeof(unsigned long long) * o.centres.size(),
                              hipMemcpyDeviceToHost));
        o.series.resize((size_t)std::min<int64_t>(h->sweeps, c.e_capacity));
        if (!o.series.empty())
            HIPCHECK(h, hipMemcpy(o.series.data(), c.e_series, sizeof(double) * o.series.size(),
                                  hipMemcpyDeviceToHost));
    }
    File f(fopen(path, "wb"));
    if (!f.f) return fail(h, MC_E_ARG, std::string("cannot open ") + path + " for writing");
    mc_options opt = h->opt;
    opt.hip_stream = nullptr;
    const int32_t hdr[4] = {kCkptVersion, (int32_t)cs.size(), (int32_t)sizeof(mc_options), (int32_t)ST_N};
    const int64_t cnt[2] = {h->sweeps, h->rdf_samples};
    bool ok = f.put(kCkptMagic, 8) && f.put(hdr, 4) && f.put(cnt, 2) && f.put(&opt, 1);
    for (const CkptChain& o : cs) {
        const int32_t ci[4] = {o.n, o.nt, o.bins, (int32_t)o.chain_id};
        const double cd[4] = {o.R, o.lB, o.max_disp, o.e_run};
        const int64_t m = (int64_t)o.series.size();
        ok = ok && f.put(ci, 4) && f.put(cd, 4) && f.put(&o.aux, 1) && f.put(o.stats, ST_N) &&
             f.put(o.q.data(), o.q.size()) && f.put(o.sigma.data(), o.sigma.size()) &&
             f.put(o.xyz.data(), o.xyz.size()) && f.put(o.prev.data(), o.prev.size()) &&
             f.put(o.masks.data(), o.masks.size()) && f.put(o.counts.data(), o.counts.size()) &&
             f.put(o.centres.data(), o.centres.size()) && f.put(&m, 1) &&
             (m == 0 || f.put(o.series.data(), o.series.size()));
    }
    if (!ok || fflush(f.f) != 0) return fail(h, MC_E_ARG, std::string("writing ") + path + " failed");
    return MC_OK;
}

int mc_load(const char* path, const mc_options* opt_in, mc_handle** out) {
    if (!out) return fail(nullptr, MC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!path) return fail(nullptr, MC_E_ARG, "path is NULL");
    File f(fopen(path, "rb"));
    if (!f.f) return fail(nullptr, MC_E_ARG, std::string("cannot open ") + path);
    const std::string bad = std::string(path) + " is not a checkpoint of this library version";
    char magic[8];
    int32_t hdr[4];
    int64_t cnt[2];
    mc_options saved;
    if (!f.get(magic, 8) || std::memcmp(magic, kCkptMagic, 8) != 0 || !f.get(hdr, 4) || hdr[0] != kCkptVersion ||
        hdr[1] < 1 || hdr[2] != (int32_t)sizeof(mc_options) || hdr[3] != (int32_t)ST_N || !f.get(cnt, 2) ||
        cnt[0] < 0 || cnt[0] > (int64_t)UINT32_MAX || cnt[1] < 0 || !f.get(&saved, 1))
        return fail(nullptr, MC_E_ARG, bad);
    saved.hip_stream = nullptr;
    mc_options opt = saved;
    if (opt_in) {
        opt = *opt_in;
        // the restored g(r) counts belong to the saved histogram and centre rule
        if (opt.precision != saved.precision || opt.rdf_bins != saved.rdf_bins ||
            opt.rdf_rmax != saved.rdf_rmax || opt.rdf_margin != saved.rdf_margin)
            return fail(nullptr, MC_E_ARG,
                        "precision, rdf_bins, rdf_rmax and rdf_margin must be those of the checkpoint");
    }
    int rc = check_options(opt);
    if (rc) return rc;
    std::vector<CkptChain> cs((size_t)hdr[1]);
    for (CkptChain& o : cs) {
        int32_t ci[4];
        double cd[4];
        if (!f.get(ci, 4) || !f.get(cd, 4) || ci[0] < 1 || ci[0] > (1 << 24) || ci[1] < 1 || ci[1] > 8 ||
            ci[2] != saved.rdf_bins)
            return fail(nullptr, MC_E_ARG, bad);
        o.n = ci[0];
        o.nt = ci[1];
        o.bins = ci[2];
        o.chain_id = (uint32_t)ci[3];
        o.R = cd[0];
        o.lB = cd[1];
        o.max_disp = cd[2];
        o.e_run = cd[3];
        o.q.resize(o.n);
        o.sigma.resize(o.n);
        o.xyz.resize(3 * (size_t)o.n);
        o.prev.resize(3 * (size_t)o.n);
        o.masks.resize(kRing);
        o.counts.resize((size_t)o.nt * o.nt * o.bins);
        o.centres.resize((size_t)o.nt);
        int64_t m = 0;
        if (!f.get(&o.aux, 1) || !f.get(o.stats, ST_N) || !f.get(o.q.data(), o.q.size()) ||
            !f.get(o.sigma.data(), o.sigma.size()) || !f.get(o.xyz.data(), o.xyz.size()) ||
            !f.get(o.prev.data(), o.prev.size()) || !f.get(o.masks.data(), o.masks.size()) ||
            !f.get(o.counts.data(), o.counts.size()) || !f.get(o.centres.data(), o.centres.size()) ||
            !f.get(&m, 1) || m < 0 || m > cnt[0])
            return fail(nullptr, MC_E_ARG, bad);
        o.series.resize((size_t)m);
        if (m > 0 && !f.get(o.series.data(), o.series.size())) return fail(nullptr, MC_E_ARG, bad);
    }
    std::vector<mc_chain_spec> specs(cs.size());
    for (size_t k = 0; k < cs.size(); ++k) {
        mc_chain_spec& sp = specs[k];
        std::memset(&sp, 0, sizeof(sp));
        sp.n = cs[k].n;
        sp.charges = cs[k].q.data();
        sp.diameters = cs[k].sigma.data();
        sp.positions = cs[k].xyz.data();
        sp.radius = cs[k].R;
        sp.l_B = cs[k].lB;
        sp.max_disp = cs[k].max_disp;
        sp.chain_id = cs[k].chain_id;
        if ((rc = validate_chain(sp, opt, "chain " + std::to_string(k) + ": ", false))) return rc;
    }
    mc_handle* h = nullptr;
    if ((rc = create_handle((int32_t)specs.size(), specs.data(), opt, &h))) return rc;
    auto bail = [&](int code) {
        g_create_error = h->err;
        mc_destroy(h);
        return code;
    };
    h->sweeps = cnt[0];
    h->rdf_samples = cnt[1];
    for (size_t k = 0; k < cs.size(); ++k) {
        Chain& c = h->chains[k];
        const CkptChain& o = cs[k];
        if (c.species.size() != (size_t)o.nt) {
            h->err = bad;
            return bail(MC_E_ARG);
        }
        for (double v : o.prev)
            if (!is_finite(v)) {
                h->err = bad;
                return bail(MC_E_ARG);
            }
        if ((rc = write_start(h, c, o.xyz.data(), o.prev.data(), o.masks.data(), h->sweeps))) return bail(rc);
        if ((rc = grow_buffer(h, &c.e_series, &c.e_capacity, std::max<int64_t>(1024, h->sweeps), true)))
            return bail(rc);
        hipError_t e = hipSuccess;
        if ((e = hipMemcpy(c.e_state, &o.e_run, sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.aux, &o.aux, sizeof(EnergyAux), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.stats, o.stats, sizeof(o.stats), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.rdf_counts, o.counts.data(), sizeof(unsigned long long) * o.counts.size(),
                           hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c.rdf_centres, o.centres.data(), sizeof(unsigned long long) * o.centres.size(),
                           hipMemcpyHostToDevice)) != hipSuccess ||
            (!o.series.empty() && (e = hipMemcpy(c.e_series, o.series.data(), sizeof(double) * o.series.size(),
                                                 hipMemcpyHostToDevice)) != hipSuccess)) {
            h->err = std::string("upload failed: ") + hipGetErrorString(e);
            return bail(MC_E_DEVICE);
        }
    }
    if ((rc = upload_desc(h))) return bail(rc);
    if ((rc = sync_check(h))) return bail(rc);
    *out = h;
    return MC_OK;
}

int mc_sweep(mc_handle* h, int64_t n_sweeps, uint64_t seed) {
    if (!h) return MC_E_ARG;
    if (h->failed) return fail(h, MC_E_STATE, "handle is in a failed state: " + h->err);
    return sweep_all(h, n_sweeps, seed);
}

int mc_sweep_reduction(mc_handle* h, int64_t n_sweeps, uint64_t seed) {
    if (!h) return MC_E_ARG;
    if (h->failed) return fail(h, MC_E_STATE, "handle is in a failed state: " + h->err);
    if (h->chains.size() != 1) return fail(h, MC_E_ARG, "the per-move reduction scheme takes a single-chain handle");
    if (h->da_kernel)
        return fail(h, MC_E_ARG, "the per-move reduction scheme has no delayed-acceptance stage or move log");
    return sweep_all(h, n_sweeps, seed, launch_reduction);
}

int mc_energy(mc_handle* h, double* e_running, double* e_exact) { return chain_energy(h, 0, e_running, e_exact); }

int mc_rdf_sample(mc_handle* h) {
    if (!h) return MC_E_ARG;
    if (h->failed) return fail(h, MC_E_STATE, "handle is in a failed state: " + h->err);
    return launch_rdf(h);
}

int mc_rdf_reset(mc_handle* h) {
    if (!h) return MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    for (Chain& c : h->chains) {
        const size_t nt = c.species.size();
        std::vector<unsigned long long> z(nt * nt * (size_t)h->opt.rdf_bins, 0ull);
        HIPCHECK(h, hipMemcpy(c.rdf_counts, z.data(), sizeof(unsigned long long) * z.size(), hipMemcpyHostToDevice));
        HIPCHECK(h, hipMemcpy(c.rdf_centres, z.data(), sizeof(unsigned long long) * nt, hipMemcpyHostToDevice));
    }
    h->rdf_samples = 0;
    return sync_check(h);
}

int mc_rdf(mc_handle* h, int32_t bins, double* g, uint64_t* counts, uint64_t* centres, int64_t* n_samples) {
    return chain_rdf(h, 0, bins, g, counts, centres, n_samples);
}

int mc_species(const mc_handle* h, int32_t* ntypes, double* q, double* s) { return chain_species(h, 0, ntypes, q, s); }

int mc_get_positions(mc_handle* h, double* xyz) { return chain_positions(h, 0, xyz); }

int mc_trace(mc_handle* h, int64_t n_moves, uint8_t* acc, double* dE) { return chain_trace(h, 0, n_moves, acc, dE); }

int mc_energy_series(mc_handle* h, int64_t n, double* e) { return chain_energy_series(h, 0, n, e); }

int mc_get_stats(mc_handle* h, mc_stats* out) { return chain_stats(h, 0, out); }

int mc_timing(mc_handle* h, int64_t* launches, double* kernel_ms, int64_t* sweeps) {
    if (!h) return MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    for (size_t k = 0; k < h->ev_pending.size(); ++k) {
        float ms = 0.f;
        HIPCHECK(h, hipEventElapsedTime(&ms, h->ev_pending[k].first, h->ev_pending[k].second));
        h->t_ms += ms;
        h->t_launches += 1;
        h->t_sweeps += h->ev_sweeps[k];
    }
    drop_events(h);
    if (launches) *launches = h->t_launches;
    if (kernel_ms) *kernel_ms = h->t_ms;
    if (sweeps) *sweeps = h->t_sweeps;
    return MC_OK;
}

int mc_timing_reset(mc_handle* h) {
    if (!h) return MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    drop_events(h);
    h->t_ms = 0.0;
    h->t_launches = h->t_sweeps = 0;
    return MC_OK;
}

int mc_set_max_disp(mc_handle* h, double max_disp) {
    if (!h) return MC_E_ARG;
    if (!is_finite(max_disp) || max_disp <= 0) return fail(h, MC_E_ARG, "max_disp must be > 0");
    for (Chain& c : h->chains) c.D = 2.0 * max_disp;
    return upload_desc(h);
}

int mc_chain_count(const mc_handle* h, int32_t* n_chains) {
    if (!h || !n_chains) return MC_E_ARG;
    *n_chains = (int32_t)h->chains.size();
    return MC_OK;
}

int mc_chain_energy(mc_handle* h, int32_t chain, double* e_running, double* e_exact) {
    return chain_energy(h, chain, e_running, e_exact);
}

int mc_chain_rdf(mc_handle* h, int32_t chain, int32_t bins, double* g, uint64_t* counts, uint64_t* centres,
                 int64_t* n_samples) {
    return chain_rdf(h, chain, bins, g, counts, centres, n_samples);
}

int mc_chain_species(const mc_handle* h, int32_t chain, int32_t* ntypes, double* charges, double* diameters) {
    return chain_species(h, chain, ntypes, charges, diameters);
}

int mc_chain_positions(mc_handle* h, int32_t chain, double* xyz) { return chain_positions(h, chain, xyz); }

int mc_chain_trace(mc_handle* h, int32_t chain, int64_t n_moves, uint8_t* acc, double* dE) {
    return chain_trace(h, chain, n_moves, acc, dE);
}

int mc_chain_energy_series(mc_handle* h, int32_t chain, int64_t n, double* e) {
    return chain_energy_series(h, chain, n, e);
}

int mc_chain_stats(mc_handle* h, int32_t chain, mc_stats* out) { return chain_stats(h, chain, out); }

int mc_chain_set_max_disp(mc_handle* h, int32_t chain, double max_disp) {
    return chain_set_max_disp(h, chain, max_disp);
}

int mc_get_schedule(const mc_handle* h, int32_t* workgroups, double* model) {
    if (!h) return MC_E_ARG;
    if (workgroups)
        for (size_t k = 0; k < h->chains.size(); ++k) workgroups[k] = h->chains[k].wg;
    if (model) {
        model[0] = h->model_a;
        model[1] = h->model_b;
    }
    return MC_OK;
}

int mc_set_schedule(mc_handle* h, const int32_t* workgroups) {
    if (!h || !workgroups) return h ? fail(h, MC_E_ARG, "null workgroups") : MC_E_ARG;
    int total = 0;
    for (size_t k = 0; k < h->chains.size(); ++k) {
        if (workgroups[k] < 1 || workgroups[k] > h->chains[k].nb)
            return fail(h, MC_E_ARG, "chain " + std::to_string(k) + ": workgroups must be in [1, groups of 64]");
        total += workgroups[k];
    }
    const int cap_now = h->da_kernel ? h->cap_da : h->cap;
    if (total > cap_now)
        return fail(h, MC_E_ARG, "total workgroups exceed the co-resident capacity " + std::to_string(cap_now));
    int rc = sync_check(h);
    if (rc) return rc;
    std::vector<int> wg(workgroups, workgroups + h->chains.size());
    std::vector<std::pair<double, std::vector<int2>>> per;
    for (size_t k = 0; k < h->chains.size(); ++k)
        for (int j = 0; j < wg[k]; ++j)
            per.emplace_back((double)h->chains[k].nb * h->chains[k].nb / wg[k], std::vector<int2>{make_int2((int)k, j)});
    WgLists lists;
    order_grid(per, lists);
    return apply_schedule(h, wg, lists);
}

int mc_plan_schedule(int32_t n_chains, const int32_t* nb, const double* scale, const uint8_t* measured,
                     double a, double b, int32_t budget, int32_t* workgroups, int32_t* n_launch,
                     int32_t* item_chain, int32_t* item_index, int32_t* item_wg, int32_t max_items) {
    if (n_chains < 1 || !nb || !workgroups || !n_launch || budget < n_chains || !(a > 0) || !(b > 0) ||
        !is_finite(a) || !is_finite(b))
        return MC_E_ARG;
    std::vector<PlanChain> ch(n_chains);
    for (int k = 0; k < n_chains; ++k) {
        if (nb[k] < 1) return MC_E_ARG;
        const double sc = scale ? scale[k] : 1.0;
        if (!(sc > 0) || !is_finite(sc)) return MC_E_ARG;
        ch[k] = PlanChain{nb[k], sc, measured ? measured[k] != 0 : false};
    }
    std::vector<int> wg;
    WgLists lists;
    plan_lists(ch, a, b, budget, wg, lists);
    size_t items = 0;
    for (const auto& l : lists) items += l.size();
    if (items > (size_t)std::max(0, max_items) && (item_chain || item_index || item_wg)) return MC_E_ARG;
    for (int k = 0; k < n_chains; ++k) workgroups[k] = wg[k];
    *n_launch = (int32_t)lists.size();
    size_t q = 0;
    for (size_t w = 0; w < lists.size(); ++w)
        for (const int2& it : lists[w]) {
            if (item_chain) item_chain[q] = it.x;
            if (item_index) item_index[q] = it.y;
            if (item_wg) item_wg[q] = (int32_t)w;
            ++q;
        }
    return MC_OK;
}

int mc_chain_launch_ms(mc_handle* h, double* ms) {
    if (!h || !ms) return h ? fail(h, MC_E_ARG, "null output") : MC_E_ARG;
    std::vector<double> v;
    int rc = last_launch_ms(h, v);
    if (rc) return rc;
    for (size_t k = 0; k < v.size(); ++k) ms[k] = v[k];
    return MC_OK;
}

int mc_autotune(mc_handle* h, int32_t calib_sweeps, uint64_t seed, double* model) {
    if (!h) return MC_E_ARG;
    if (calib_sweeps < 1 || calib_sweeps > kMaxLaunchSweeps)
        return fail(h, MC_E_ARG, "calib_sweeps must be in [1, 4096]");
    if (h->failed) return fail(h, MC_E_STATE, "handle is in a failed state: " + h->err);
    // calibration sweeps (real sweeps of every chain, with the re-sums, g(r)
    // samples and monitor checks that fall due) on the current schedule
    std::vector<double> ms;
    int rc = sweep_all(h, calib_sweeps, seed, launch_sweeps, &ms);
    if (rc) return rc;
    // least squares, relative error: t_c / S = a nb_c + b nb_c^2 / w_c (microseconds)
    double s11 = 0, s12 = 0, s22 = 0, r1 = 0, r2 = 0;
    int used = 0;
    for (size_t k = 0; k < h->chains.size(); ++k) {
        const Chain& c = h->chains[k];
        const double t = 1e3 * ms[k] / calib_sweeps;
        if (!(t > 0)) continue;
        const double x1 = c.nb / t, x2 = (double)c.nb * c.nb / c.wg / t;  // weight 1/t
        s11 += x1 * x1;
        s12 += x1 * x2;
        s22 += x2 * x2;
        r1 += x1;
        r2 += x2;
        ++used;
    }
    double a = h->model_a, b = h->model_b;
    const double det = s11 * s22 - s12 * s12;
    if (used >= 2 && det > 1e-12 * s11 * s22) {
        a = (r1 * s22 - r2 * s12) / det;
        b = (s11 * r2 - s12 * r1) / det;
    }
    if (used >= 1 && s22 > 0 && !(a >= kModelAMin && a <= kModelAMax)) {
        // latency term out of range: hold it at the bound (or the default)
        // and refit the work term alone
        a = (a > kModelAMax) ? kModelAMax : (a < kModelAMin ? kModelAMin : kModelA);
        b = (r2 - a * s12) / s22;
    }
    if (!(a > 0) || !(b > 0)) {
        // degenerate fit (e.g. one chain): one-parameter fits, keeping the model's ratio
        double num = 0, den = 0;
        for (size_t k = 0; k < h->chains.size(); ++k) {
            const Chain& c = h->chains[k];
            const double t = 1e3 * ms[k] / calib_sweeps;
            if (!(t > 0)) continue;
            const double f = (h->model_a * c.nb + h->model_b * (double)c.nb * c.nb / c.wg) / t;
            num += f;
            den += f * f;
        }
        const double scale = den > 0 ? num / den : 1.0;
        a = h->model_a * scale;
        b = h->model_b * scale;
    }
    h->model_a = a;
    h->model_b = b;
    // per-chain factors: what the two-term model misses for one chain
    // (sharing a CU, short chains' fixed costs) it measured here
    for (size_t k = 0; k < h->chains.size(); ++k) {
        Chain& c = h->chains[k];
        const double t = 1e3 * ms[k] / calib_sweeps;
        c.cost_scale = 1.0;
        const double pred = a * c.nb + b * (double)c.nb * c.nb / c.wg;
        if (t > 0 && pred > 0) {
            c.cost_scale = std::min(4.0, std::max(0.25, t / pred));
            c.measured = true;
        }
    }
    if (model) {
        model[0] = a;
        model[1] = b;
    }
    std::vector<int> wg;
    WgLists lists;
    plan_schedule(h, wg, lists);
    return apply_schedule(h, wg, lists);
}

int mc_set_surrogate(mc_handle* h, int32_t chain, const double* params, double ref_stage2_reject,
                     int32_t active) {
    if (!h) return MC_E_ARG;
    if (!params) return fail(h, MC_E_ARG, "params is NULL");
    if (chain < -1 || chain >= (int32_t)h->chains.size()) return fail(h, MC_E_ARG, "bad chain index");
    if (h->waves != 4) return fail(h, MC_E_ARG, "delayed acceptance needs 4 waves per workgroup");
    if (!is_finite(ref_stage2_reject)) return fail(h, MC_E_ARG, "ref_stage2_reject must be finite");
    std::vector<float> w(kDaParams);
    std::vector<uint16_t> wb(2 * kDaIn * kDaHid);
    for (int k = 0; k < kDaParams; ++k) {
        if (!is_finite(params[k])) return fail(h, MC_E_ARG, "non-finite network parameter");
        float f = (float)params[k];
        uint32_t b;
        std::memcpy(&b, &f, 4);
        b += 0x7FFFu + ((b >> 16) & 1u);
        b &= 0xFFFF0000u;
        std::memcpy(&f, &b, 4);
        w[k] = f;
        // bfloat16 copies of the two hidden layers' matrices, transposed
        // ([hidden unit][input]) for the kernel's 8-byte operand loads
        const int oW2 = kDaIn * kDaHid + kDaHid;
        if (k < kDaIn * kDaHid) {
            const int in = k / kDaHid, hu = k % kDaHid;
            wb[hu * kDaIn + in] = (uint16_t)(b >> 16);
        } else if (k >= oW2 && k < oW2 + kDaHid * kDaHid) {
            const int in = (k - oW2) / kDaHid, hu = (k - oW2) % kDaHid;
            wb[kDaIn * kDaHid + hu * kDaHid + in] = (uint16_t)(b >> 16);
        }
    }
    int rc = sync_check(h);
    if (rc) return rc;
    for (int32_t k = 0; k < (int32_t)h->chains.size(); ++k) {
        if (chain >= 0 && k != chain) continue;
        Chain& c = h->chains[k];
        if (!c.da_w && (rc = dalloc(h, &c.da_w, sizeof(float) * kDaParams))) return rc;
        if (!c.da_wb && (rc = dalloc(h, &c.da_wb, sizeof(uint16_t) * wb.size()))) return rc;
        HIPCHECK(h, hipMemcpy(c.da_w, w.data(), sizeof(float) * kDaParams, hipMemcpyHostToDevice));
        HIPCHECK(h, hipMemcpy(c.da_wb, wb.data(), sizeof(uint16_t) * wb.size(), hipMemcpyHostToDevice));
        unsigned long long st[ST_N];
        HIPCHECK(h, hipMemcpy(st, c.stats, sizeof(st), hipMemcpyDeviceToHost));
        DAState ds;
        HIPCHECK(h, hipMemcpy(&ds, c.da, sizeof(ds), hipMemcpyDeviceToHost));
        ds.active = active ? 1 : 0;
        ds.window = h->opt.da_window;
        ds.fallback_sweep = -1;
        ds.ref_rate = ref_stage2_reject;
        ds.delta = h->opt.da_delta;
        ds.win_pass0 = st[ST_DA_S1PASS];
        ds.win_rej0 = st[ST_DA_S2REJ];
        ds.last_rate = -1.0;
        ds.min_count = 64;
        HIPCHECK(h, hipMemcpy(c.da, &ds, sizeof(ds), hipMemcpyHostToDevice));
        c.band = std::min(c.band, kDaMaxBand);
    }
    h->da_window = h->opt.da_window;
    if (!h->da_kernel) {
        if ((int)h->chains.size() > h->cap_da)
            return fail(h, MC_E_ARG, "more chains than co-resident workgroups of the delayed-acceptance kernel");
        h->da_kernel = true;
        std::vector<int> wg;
        WgLists lists;
        plan_schedule(h, wg, lists);
        return apply_schedule(h, wg, lists);
    }
    return upload_desc(h);
}

int mc_get_log(mc_handle* h, int32_t chain, int64_t n, uint8_t* feats, double* dE, double* dEh, uint8_t* flags) {
    Chain* c = get_chain(h, chain);
    if (!c) return h ? fail(h, MC_E_ARG, "bad chain index") : MC_E_ARG;
    if (n < 0 || n > c->log_cap) return fail(h, MC_E_ARG, "n exceeds the log capacity");
    int rc = sync_check(h);
    if (rc) return rc;
    if (n == 0) return MC_OK;
    if (feats) HIPCHECK(h, hipMemcpy(feats, c->log_feat, sizeof(uint32_t) * 64 * (size_t)n, hipMemcpyDeviceToHost));
    if (dE) HIPCHECK(h, hipMemcpy(dE, c->log_de, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (dEh) HIPCHECK(h, hipMemcpy(dEh, c->log_deh, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (flags) HIPCHECK(h, hipMemcpy(flags, c->log_flags, (size_t)n, hipMemcpyDeviceToHost));
    return MC_OK;
}

void mc_destroy(mc_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
}

const char* mc_last_error(const mc_handle* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
