// mc_lib.hip -- host runtime behind include/mc.h (C ABI) and the kernel
// instantiations for gfx950.
//
// Paper: Liang, Xing, Li, arXiv:1602.05716 (see include/mc.h for the
// passages each entry point follows).  The host never touches the chain
// between trials: mc_sweep enqueues one persistent cooperative launch per
// stretch of sweeps, interleaved with the double-precision energy re-sum and
// g(r) sampling kernels, all on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/mc.h"
#include "mc_aux_kernels.hpp"
#include "mc_sweep_kernel.hpp"

using namespace mcdev;

namespace {

thread_local std::string g_create_error = "no error";

// Stats slots written by the sweep kernel.
enum { ST_MOVES = 0, ST_ACC, ST_WALL, ST_OVERLAP, ST_METRO, ST_ITERS, ST_EARLY, ST_N };

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

using SweepFn = void (*)(const ChainDesc*, const int32_t*, uint32_t, int32_t, Ctl);

template <typename T, int M, bool U>
SweepFn sweep_fn() {
    return sweep_kernel<T, M, U>;
}

SweepFn pick_sweep(bool fp64, int waves, bool uniform) {
    if (fp64) {
        if (waves == 8) return uniform ? sweep_fn<double, 8, true>() : sweep_fn<double, 8, false>();
        return uniform ? sweep_fn<double, 4, true>() : sweep_fn<double, 4, false>();
    }
    if (waves == 8) return uniform ? sweep_fn<float, 8, true>() : sweep_fn<float, 8, false>();
    return uniform ? sweep_fn<float, 4, true>() : sweep_fn<float, 4, false>();
}

}  // namespace

struct mc_handle {
    // model
    int32_t n = 0, nb = 0, npad = 0;
    bool fp64 = false;
    double R = 0, lB = 0, D = 1.0;
    bool uniform_sigma = true;
    std::vector<double> q, sigma;
    std::vector<int32_t> type;
    std::vector<std::pair<double, double>> species;  // (charge, diameter)
    std::vector<int64_t> n_of_type;
    // options
    mc_options opt{};
    int band = 0, waves = 4, wg = 1;
    // runtime
    DeviceInfo dev;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool failed = false;
    int64_t sweeps = 0;
    int64_t rdf_samples = 0;
    std::string err = "no error";
    // device memory
    void* pos = nullptr;          // T4[2][npad]
    void* half = nullptr;         // T[npad]
    void* charge = nullptr;       // T[npad]
    double* wall_a = nullptr;     // [npad]
    int32_t* d_type = nullptr;    // [npad]
    GroupRec* rec = nullptr;      // [kRing]
    unsigned long long* stats = nullptr;  // [ST_N]
    int* abort_flag = nullptr;
    double* e_series = nullptr;
    int64_t e_capacity = 0;
    uint8_t* trace_acc = nullptr;
    double* trace_de = nullptr;
    int64_t trace_cap = 0;
    double* e_partial = nullptr;  // [nb]
    EnergyAux* aux = nullptr;
    double* e_state = nullptr;    // running energy
    double* de_group = nullptr;   // [de_capacity] group energy changes of one launch
    double* sweep_tot = nullptr;  // [max_launch_sweeps]
    int64_t de_capacity = 0;
    unsigned long long* rdf_counts = nullptr;
    unsigned long long* rdf_centres = nullptr;
    ChainDesc* d_desc = nullptr;
    int32_t* d_wgmap = nullptr;
    int32_t wgmap_len = 0;
    // host staging
    ChainDesc desc{};
    // sweep-kernel timing (record_timing)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    std::vector<int64_t> ev_sweeps;
    int64_t t_launches = 0, t_sweeps = 0;
    double t_ms = 0.0;
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
    void* bufs[] = {h->pos, h->half, h->charge, h->wall_a, h->d_type, h->rec, h->stats,
                    h->abort_flag, h->e_series, h->trace_acc, h->trace_de, h->e_partial, h->aux,
                    h->e_state, h->de_group, h->sweep_tot, h->rdf_counts, h->rdf_centres,
                    h->d_desc, h->d_wgmap};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
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
                    : ab == MC_E_STATE ? "a group record was reused before it was read (chain state is invalid)"
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

// The descriptor is read by running kernels: drain the stream, then copy.
int upload_desc(mc_handle* h) {
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(h->d_desc, &h->desc, sizeof(ChainDesc), hipMemcpyHostToDevice));
    return MC_OK;
}

int ensure_series(mc_handle* h, int64_t need) {
    if (need <= h->e_capacity) return MC_OK;
    int64_t cap = std::max<int64_t>(need, std::max<int64_t>(1024, 2 * h->e_capacity));
    double* nb = nullptr;
    int rc = dalloc(h, &nb, sizeof(double) * cap);
    if (rc) return rc;
    if (h->e_series) {
        HIPCHECK(h, hipMemcpyAsync(nb, h->e_series, sizeof(double) * h->e_capacity,
                                   hipMemcpyDeviceToDevice, h->stream));
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        (void)hipFree(h->e_series);
    }
    h->e_series = nb;
    h->e_capacity = cap;
    return MC_OK;
}

int launch_energy(mc_handle* h, int reset, int record_drift) {
    const int nparts = (h->nb + 1) / 2;
    const int parity = (int)((h->sweeps - 1) & 1);
    const size_t t4 = h->fp64 ? sizeof(double4) : sizeof(float4);
    const void* p = (const char*)h->pos + (size_t)parity * h->npad * t4;
    if (h->fp64)
        hipLaunchKernelGGL(energy_partial_kernel<double>, dim3(nparts), dim3(256), 0, h->stream,
                           (const double4*)p, (const double*)h->charge, h->nb, h->e_partial);
    else
        hipLaunchKernelGGL(energy_partial_kernel<float>, dim3(nparts), dim3(256), 0, h->stream,
                           (const float4*)p, (const float*)h->charge, h->nb, h->e_partial);
    HIPCHECK(h, hipGetLastError());
    hipLaunchKernelGGL(energy_finalize_kernel, dim3(1), dim3(64), 0, h->stream, h->e_partial, nparts,
                       h->lB, h->e_state, h->aux, reset, record_drift);
    HIPCHECK(h, hipGetLastError());
    return MC_OK;
}

int launch_rdf(mc_handle* h) {
    const int nt = (int)h->species.size();
    const int bins = h->opt.rdf_bins;
    const double rmax = h->opt.rdf_rmax;
    const double dr = rmax / (double)bins;
    const double rc = h->R - rmax;
    const size_t lds = sizeof(unsigned int) * (size_t)nt * nt * bins;
    const int parity = (int)((h->sweeps - 1) & 1);
    const size_t t4 = h->fp64 ? sizeof(double4) : sizeof(float4);
    const void* p = (const char*)h->pos + (size_t)parity * h->npad * t4;
    if (h->fp64)
        hipLaunchKernelGGL(rdf_kernel<double>, dim3(h->nb), dim3(256), lds, h->stream, (const double4*)p,
                           h->d_type, h->n, h->nb, nt, rc, rmax, dr, bins, h->rdf_counts, h->rdf_centres);
    else
        hipLaunchKernelGGL(rdf_kernel<float>, dim3(h->nb), dim3(256), lds, h->stream, (const float4*)p,
                           h->d_type, h->n, h->nb, nt, rc, rmax, dr, bins, h->rdf_counts, h->rdf_centres);
    HIPCHECK(h, hipGetLastError());
    h->rdf_samples += 1;
    return MC_OK;
}

constexpr int64_t kMaxLaunchSweeps = 4096;

int launch_sweeps(mc_handle* h, int64_t n_sweeps, uint64_t seed) {
    if (n_sweeps <= 0) return MC_OK;
    if (n_sweeps > kMaxLaunchSweeps) {
        int rc = launch_sweeps(h, kMaxLaunchSweeps, seed);
        if (rc) return rc;
        return launch_sweeps(h, n_sweeps - kMaxLaunchSweeps, seed);
    }
    int rc = ensure_series(h, h->sweeps + n_sweeps);
    if (rc) return rc;
    const int64_t ngroups = n_sweeps * (int64_t)h->nb;
    if (ngroups > h->de_capacity) {
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        if (h->de_group) (void)hipFree(h->de_group);
        h->de_group = nullptr;
        h->de_capacity = 0;
        if ((rc = dalloc(h, &h->de_group, sizeof(double) * ngroups))) return rc;
        h->de_capacity = ngroups;
        h->desc.de_group = h->de_group;
        if ((rc = upload_desc(h))) return rc;
    }
    if (h->desc.seed != seed) {
        h->desc.seed = seed;
        if ((rc = upload_desc(h))) return rc;
    }
    SweepFn fn = pick_sweep(h->fp64, h->waves, h->uniform_sigma);
    Ctl ctl;
    ctl.abort = h->abort_flag;
    ctl.timeout_ticks = (uint64_t)(h->opt.wait_timeout_s * h->dev.wall_clock_hz);
    uint32_t s0 = (uint32_t)h->sweeps;
    int32_t ns = (int32_t)n_sweeps;
    const ChainDesc* dd = h->d_desc;
    const int32_t* wm = h->d_wgmap;
    void* args[] = {(void*)&dd, (void*)&wm, (void*)&s0, (void*)&ns, (void*)&ctl};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->opt.record_timing) {
        HIPCHECK(h, hipEventCreate(&e0));
        HIPCHECK(h, hipEventCreate(&e1));
        HIPCHECK(h, hipEventRecord(e0, h->stream));
    }
    HIPCHECK(h, hipLaunchCooperativeKernel((const void*)fn, dim3(h->wg), dim3(64 * h->waves), args, 0,
                                           h->stream));
    if (h->opt.record_timing) {
        HIPCHECK(h, hipEventRecord(e1, h->stream));
        h->ev_pending.emplace_back(e0, e1);
        h->ev_sweeps.push_back(n_sweeps);
    }
    hipLaunchKernelGGL(energy_scan_kernel, dim3(1), dim3(256), 0, h->stream, h->de_group, h->nb,
                       (int32_t)n_sweeps, (int64_t)h->sweeps, h->sweep_tot, h->e_state, h->e_series,
                       h->e_capacity);
    HIPCHECK(h, hipGetLastError());
    h->sweeps += n_sweeps;
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
    o->chain_id = 0;
    o->hip_stream = nullptr;
    o->band = -1;
    o->waves = 0;
    o->workgroups = 0;
    o->trace_moves = 0;
    o->wait_timeout_s = 20.0;
    return MC_OK;
}

int mc_create(int32_t n, const double* charges, const double* diameters, const double* positions,
              double radius, double l_B, const mc_options* opt_in, mc_handle** out) {
    if (!out) return fail(nullptr, MC_E_ARG, "out is NULL");
    *out = nullptr;
    mc_options opt;
    mc_options_init(&opt);
    if (opt_in) opt = *opt_in;
    if (n < 1 || n > (1 << 24)) return fail(nullptr, MC_E_ARG, "n out of range [1, 2^24]");
    if (!charges || !diameters || !positions) return fail(nullptr, MC_E_ARG, "null input array");
    if (!is_finite(radius) || radius <= 0) return fail(nullptr, MC_E_ARG, "radius must be finite and > 0");
    if (!is_finite(l_B) || l_B < 0) return fail(nullptr, MC_E_ARG, "l_B must be finite and >= 0");
    if (opt.precision != MC_FP64 && opt.precision != MC_FP32_ACC64)
        return fail(nullptr, MC_E_ARG, "unknown precision");
    if (!is_finite(opt.max_disp) || opt.max_disp <= 0) return fail(nullptr, MC_E_ARG, "max_disp must be > 0");
    if (opt.resum_every < 0 || opt.rdf_every < 0) return fail(nullptr, MC_E_ARG, "negative interval");
    if (opt.rdf_bins < 1 || opt.rdf_bins > 4096 || !is_finite(opt.rdf_rmax) || opt.rdf_rmax <= 0)
        return fail(nullptr, MC_E_ARG, "rdf_bins must be in [1, 4096] and rdf_rmax > 0");
    if (opt.band < -1 || opt.band > kMaxBand) return fail(nullptr, MC_E_ARG, "band out of range");
    if (opt.waves != 0 && opt.waves != 4 && opt.waves != 8) return fail(nullptr, MC_E_ARG, "waves must be 0, 4 or 8");
    if (opt.workgroups < 0 || opt.trace_moves < 0) return fail(nullptr, MC_E_ARG, "negative count");
    if (!is_finite(opt.wait_timeout_s) || opt.wait_timeout_s <= 0) return fail(nullptr, MC_E_ARG, "bad wait_timeout_s");

    double qsum = 0, qabs = 0, smax = 0;
    for (int i = 0; i < n; ++i) {
        if (!is_finite(charges[i]) || !is_finite(diameters[i]) || diameters[i] <= 0)
            return fail(nullptr, MC_E_ARG, "charges must be finite and diameters finite and > 0");
        for (int k = 0; k < 3; ++k)
            if (!is_finite(positions[3 * i + k])) return fail(nullptr, MC_E_ARG, "non-finite position");
        qsum += charges[i];
        qabs += std::fabs(charges[i]);
        smax = std::max(smax, diameters[i]);
    }
    if (std::fabs(qsum) > 1e-9 * std::max(qabs, 1.0))
        return fail(nullptr, MC_E_NOT_NEUTRAL, "sum of charges is not zero");
    for (int i = 0; i < n; ++i) {
        const double* x = positions + 3 * i;
        const double a = radius - 0.5 * diameters[i];
        if (a < 0 || x[0] * x[0] + x[1] * x[1] + x[2] * x[2] > a * a)
            return fail(nullptr, MC_E_WALL, "ion " + std::to_string(i) + " crosses the wall");
    }
    int oa = -1, ob = -1;
    if (find_overlap(n, positions, diameters, smax, &oa, &ob))
        return fail(nullptr, MC_E_OVERLAP,
                    "ions " + std::to_string(oa) + " and " + std::to_string(ob) + " overlap");

    mc_handle* h = new (std::nothrow) mc_handle();
    if (!h) return fail(nullptr, MC_E_OOM, "host allocation failed");
    std::string derr;
    if (!device_info(h->dev, derr)) {
        delete h;
        return fail(nullptr, MC_E_DEVICE, derr);
    }
    h->opt = opt;
    h->n = n;
    h->nb = (n + kGroup - 1) / kGroup;
    h->npad = h->nb * kGroup;
    h->fp64 = opt.precision == MC_FP64;
    h->R = radius;
    h->lB = l_B;
    h->D = 2.0 * opt.max_disp;
    h->q.assign(charges, charges + n);
    h->sigma.assign(diameters, diameters + n);
    h->uniform_sigma = true;
    for (int i = 1; i < n; ++i)
        if (diameters[i] != diameters[0]) h->uniform_sigma = false;
    // species: distinct (q, sigma), decreasing charge then increasing diameter
    for (int i = 0; i < n; ++i) {
        auto key = std::make_pair(charges[i], diameters[i]);
        if (std::find(h->species.begin(), h->species.end(), key) == h->species.end())
            h->species.push_back(key);
    }
    if (h->species.size() > 8) {
        delete h;
        return fail(nullptr, MC_E_ARG, "more than 8 species");
    }
    if (sizeof(unsigned int) * h->species.size() * h->species.size() * (size_t)opt.rdf_bins > 48 * 1024) {
        delete h;
        return fail(nullptr, MC_E_ARG, "species^2 * rdf_bins histogram does not fit in 48 KiB of LDS");
    }
    std::sort(h->species.begin(), h->species.end(), [](const auto& a, const auto& b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
    });
    h->type.resize(h->npad, -1);
    h->n_of_type.assign(h->species.size(), 0);
    for (int i = 0; i < n; ++i) {
        auto it = std::find(h->species.begin(), h->species.end(), std::make_pair(charges[i], diameters[i]));
        h->type[i] = (int32_t)(it - h->species.begin());
        h->n_of_type[h->type[i]] += 1;
    }

    // schedule
    h->band = opt.band >= 0 ? opt.band : 2;
    h->band = std::min(h->band, std::min(kMaxBand, h->nb - 1));
    h->waves = opt.waves ? opt.waves : 4;

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

    const size_t t4 = h->fp64 ? sizeof(double4) : sizeof(float4);
    const size_t t1 = h->fp64 ? sizeof(double) : sizeof(float);
    if ((rc = dalloc(h, &h->pos, 2 * t4 * h->npad)) || (rc = dalloc(h, &h->half, t1 * h->npad)) ||
        (rc = dalloc(h, &h->charge, t1 * h->npad)) ||
        (rc = dalloc(h, &h->wall_a, sizeof(double) * h->npad)) ||
        (rc = dalloc(h, &h->d_type, sizeof(int32_t) * h->npad)) ||
        (rc = dalloc(h, &h->rec, sizeof(GroupRec) * kRing)) ||
        (rc = dalloc(h, &h->stats, sizeof(unsigned long long) * ST_N)) ||
        (rc = dalloc(h, &h->abort_flag, sizeof(int))) ||
        (rc = dalloc(h, &h->e_partial, sizeof(double) * h->nb)) || (rc = dalloc(h, &h->aux, sizeof(EnergyAux))) ||
        (rc = dalloc(h, &h->e_state, sizeof(double))) ||
        (rc = dalloc(h, &h->sweep_tot, sizeof(double) * kMaxLaunchSweeps)) ||
        (rc = dalloc(h, &h->d_desc, sizeof(ChainDesc))))
        return bail(rc);
    const size_t nt = h->species.size();
    const size_t nh = nt * nt * (size_t)opt.rdf_bins;
    if ((rc = dalloc(h, &h->rdf_counts, sizeof(unsigned long long) * nh)) ||
        (rc = dalloc(h, &h->rdf_centres, sizeof(unsigned long long) * nt)))
        return bail(rc);
    if (opt.trace_moves > 0) {
        h->trace_cap = opt.trace_moves;
        if ((rc = dalloc(h, &h->trace_acc, (size_t)h->trace_cap)) ||
            (rc = dalloc(h, &h->trace_de, sizeof(double) * h->trace_cap)))
            return bail(rc);
    }

    // host images: positions carry the version tag of the sweep that produced
    // them; the initial state is the result of virtual sweeps -2 (parity 0)
    // and -1 (parity 1)
    std::vector<char> hpos(2 * t4 * h->npad), hhalf(t1 * h->npad), hq(t1 * h->npad);
    std::vector<double> hwall(h->npad, 0.0);
    for (int i = 0; i < h->npad; ++i) {
        double x, y, z, qq, hh;
        if (i < n) {
            x = positions[3 * i];
            y = positions[3 * i + 1];
            z = positions[3 * i + 2];
            qq = charges[i];
            hh = 0.5 * diameters[i];
            hwall[i] = radius - 0.5 * diameters[i];
        } else {
            // inert padding ion: no charge, no size, far from everything and from each other
            x = 1.0e6 * (double)(i - n + 1);
            y = -2.0e6;
            z = 3.0e6;
            qq = 0.0;
            hh = 0.0;
        }
        for (int par = 0; par < 2; ++par) {
            const uint32_t ver = par == 0 ? 0xFFFFFFFEu : 0xFFFFFFFFu;
            char* dst = &hpos[t4 * ((size_t)par * h->npad + i)];
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
    for (int k = 0; k < kRing; ++k) {
        const int64_t g = (int64_t)k - kRing;  // virtual groups -kRing..-1: decided, nothing accepted
        hrec[(size_t)(g & (kRing - 1))] = GroupRec{(uint32_t)(g + 1), 0u, 0ull};
    }
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream);
    };
    std::vector<unsigned long long> zeros(std::max<size_t>(nh, ST_N), 0ull);
    int zero = 0;
    EnergyAux zaux{0.0, 0.0, 0.0, 0ull};
    hipError_t e = hipSuccess;
    if ((e = up(h->pos, hpos.data(), 2 * t4 * h->npad)) != hipSuccess ||
        (e = up(h->half, hhalf.data(), t1 * h->npad)) != hipSuccess ||
        (e = up(h->charge, hq.data(), t1 * h->npad)) != hipSuccess ||
        (e = up(h->wall_a, hwall.data(), sizeof(double) * h->npad)) != hipSuccess ||
        (e = up(h->d_type, h->type.data(), sizeof(int32_t) * h->npad)) != hipSuccess ||
        (e = up(h->rec, hrec.data(), sizeof(GroupRec) * kRing)) != hipSuccess ||
        (e = up(h->stats, zeros.data(), sizeof(unsigned long long) * ST_N)) != hipSuccess ||
        (e = up(h->abort_flag, &zero, sizeof(int))) != hipSuccess ||
        (e = up(h->aux, &zaux, sizeof(EnergyAux))) != hipSuccess ||
        (e = up(h->e_state, &zaux.e_resum, sizeof(double))) != hipSuccess ||
        (e = up(h->rdf_counts, zeros.data(), sizeof(unsigned long long) * nh)) != hipSuccess ||
        (e = up(h->rdf_centres, zeros.data(), sizeof(unsigned long long) * nt)) != hipSuccess) {
        h->err = std::string("upload failed: ") + hipGetErrorString(e);
        return bail(MC_E_DEVICE);
    }
    if (h->trace_cap) {
        if (hipMemsetAsync(h->trace_acc, 0xFF, (size_t)h->trace_cap, h->stream) != hipSuccess) {
            h->err = "trace init failed";
            return bail(MC_E_DEVICE);
        }
    }

    // launch shape: one workgroup per target group, capped by co-residency
    SweepFn fn = pick_sweep(h->fp64, h->waves, h->uniform_sigma);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, 64 * h->waves, 0) != hipSuccess ||
        per_cu < 1) {
        h->err = "occupancy query failed for the sweep kernel";
        return bail(MC_E_DEVICE);
    }
    // Every workgroup of the cooperative grid must be resident at once.  The
    // occupancy query has been seen to over-promise for workgroups with more
    // than 64 KiB of LDS: such kernels get one workgroup per CU.
    // Kernels that spill to scratch have been seen to run fewer workgroups at
    // once than the query reports: they also get one workgroup per CU.
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, (const void*)fn) == hipSuccess &&
        (fa.sharedSizeBytes > 64 * 1024 || fa.localSizeBytes > 0))
        per_cu = 1;
    const int cap = per_cu * h->dev.cus;
    h->wg = opt.workgroups > 0 ? opt.workgroups : h->nb;
    h->wg = std::max(1, std::min({h->wg, h->nb, cap}));

    ChainDesc& d = h->desc;
    d.n = n;
    d.nb = h->nb;
    d.band = h->band;
    d.wg_count = h->wg;
    d.wg_first = 0;
    d.chain_id = opt.chain_id;
    d.seed = 0;
    d.lB = l_B;
    d.D = h->D;
    d.half_uniform = 0.5 * diameters[0];
    d.pos = h->pos;
    d.charge = h->charge;
    d.half = h->half;
    d.wall_a = h->wall_a;
    d.rec = h->rec;
    d.stats = h->stats;
    d.de_group = nullptr;
    d.trace_acc = h->trace_acc;
    d.trace_de = h->trace_de;
    d.trace_cap = h->trace_cap;
    std::vector<int32_t> wgmap(h->wg, 0);
    if ((rc = dalloc(h, &h->d_wgmap, sizeof(int32_t) * h->wg))) return bail(rc);
    h->wgmap_len = h->wg;
    if ((e = up(h->d_wgmap, wgmap.data(), sizeof(int32_t) * h->wg)) != hipSuccess ||
        (e = up(h->d_desc, &d, sizeof(ChainDesc))) != hipSuccess) {
        h->err = std::string("upload failed: ") + hipGetErrorString(e);
        return bail(MC_E_DEVICE);
    }
    if ((rc = ensure_series(h, 1024))) return bail(rc);
    // initial energy: re-sum into the running energy
    if ((rc = launch_energy(h, 1, 0))) return bail(rc);
    if ((rc = sync_check(h))) return bail(rc);
    *out = h;
    return MC_OK;
}

int mc_sweep(mc_handle* h, int64_t n_sweeps, uint64_t seed) {
    if (!h) return MC_E_ARG;
    if (h->failed) return fail(h, MC_E_STATE, "handle is in a failed state: " + h->err);
    if (n_sweeps < 0 || h->sweeps + n_sweeps > (int64_t)UINT32_MAX)
        return fail(h, MC_E_ARG, "n_sweeps out of range");
    int64_t left = n_sweeps;
    while (left > 0) {
        int64_t step = left;
        const int re = h->opt.resum_every, rd = h->opt.rdf_every;
        if (re > 0) step = std::min<int64_t>(step, re - h->sweeps % re);
        if (rd > 0) step = std::min<int64_t>(step, rd - h->sweeps % rd);
        int rc = launch_sweeps(h, step, seed);
        if (rc) return rc;
        left -= step;
        if (re > 0 && h->sweeps % re == 0 && (rc = launch_energy(h, 1, 1))) return rc;
        if (rd > 0 && h->sweeps % rd == 0 && (rc = launch_rdf(h))) return rc;
    }
    return MC_OK;
}

int mc_energy(mc_handle* h, double* e_running, double* e_exact) {
    if (!h || !e_running) return h ? fail(h, MC_E_ARG, "null output") : MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    HIPCHECK(h, hipMemcpy(e_running, h->e_state, sizeof(double), hipMemcpyDeviceToHost));
    if (e_exact) {
        if ((rc = launch_energy(h, 0, 0))) return rc;
        if ((rc = sync_check(h))) return rc;
        EnergyAux a;
        HIPCHECK(h, hipMemcpy(&a, h->aux, sizeof(EnergyAux), hipMemcpyDeviceToHost));
        *e_exact = a.e_resum;
    }
    return MC_OK;
}

int mc_rdf_sample(mc_handle* h) {
    if (!h) return MC_E_ARG;
    if (h->failed) return fail(h, MC_E_STATE, "handle is in a failed state: " + h->err);
    return launch_rdf(h);
}

int mc_rdf_reset(mc_handle* h) {
    if (!h) return MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    const size_t nt = h->species.size();
    HIPCHECK(h, hipMemsetAsync(h->rdf_counts, 0, sizeof(unsigned long long) * nt * nt * h->opt.rdf_bins, h->stream));
    HIPCHECK(h, hipMemsetAsync(h->rdf_centres, 0, sizeof(unsigned long long) * nt, h->stream));
    h->rdf_samples = 0;
    return sync_check(h);
}

int mc_rdf(mc_handle* h, int32_t bins, double* g, uint64_t* counts, uint64_t* centres, int64_t* n_samples) {
    if (!h) return MC_E_ARG;
    if (bins != h->opt.rdf_bins) return fail(h, MC_E_ARG, "bins differs from the handle's rdf_bins");
    int rc = sync_check(h);
    if (rc) return rc;
    const size_t nt = h->species.size();
    const size_t nh = nt * nt * (size_t)bins;
    std::vector<unsigned long long> c(nh), ce(nt);
    HIPCHECK(h, hipMemcpy(c.data(), h->rdf_counts, sizeof(unsigned long long) * nh, hipMemcpyDeviceToHost));
    HIPCHECK(h, hipMemcpy(ce.data(), h->rdf_centres, sizeof(unsigned long long) * nt, hipMemcpyDeviceToHost));
    if (counts)
        for (size_t k = 0; k < nh; ++k) counts[k] = c[k];
    if (centres)
        for (size_t k = 0; k < nt; ++k) centres[k] = ce[k];
    if (n_samples) *n_samples = h->rdf_samples;
    if (g) {
        const double rmax = h->opt.rdf_rmax, dr = rmax / (double)bins;
        const double pi = 3.14159265358979323846;
        for (size_t a = 0; a < nt; ++a)
            for (size_t b = 0; b < nt; ++b) {
                const double rb = h->R - 0.5 * h->species[b].second;
                const double vb = 4.0 / 3.0 * pi * rb * rb * rb;
                const double nbd = (double)(h->n_of_type[b] - (a == b ? 1 : 0)) / vb;
                for (int k = 0; k < bins; ++k) {
                    const double r0 = k * dr, r1 = (k + 1) * dr;
                    const double vk = 4.0 / 3.0 * pi * (r1 * r1 * r1 - r0 * r0 * r0);
                    const double den = (double)ce[a] * nbd * vk;
                    g[(a * nt + b) * bins + k] = den > 0 ? (double)c[(a * nt + b) * bins + k] / den : 0.0;
                }
            }
    }
    return MC_OK;
}

int mc_species(const mc_handle* h, int32_t* ntypes, double* q, double* s) {
    if (!h) return MC_E_ARG;
    if (ntypes) *ntypes = (int32_t)h->species.size();
    for (size_t k = 0; k < h->species.size(); ++k) {
        if (q) q[k] = h->species[k].first;
        if (s) s[k] = h->species[k].second;
    }
    return MC_OK;
}

int mc_get_positions(mc_handle* h, double* xyz) {
    if (!h || !xyz) return h ? fail(h, MC_E_ARG, "null output") : MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    const int parity = (int)((h->sweeps - 1) & 1);
    if (h->fp64) {
        std::vector<double4> v(h->n);
        HIPCHECK(h, hipMemcpy(v.data(), (double4*)h->pos + (size_t)parity * h->npad, sizeof(double4) * h->n,
                              hipMemcpyDeviceToHost));
        for (int i = 0; i < h->n; ++i) {
            xyz[3 * i] = v[i].x;
            xyz[3 * i + 1] = v[i].y;
            xyz[3 * i + 2] = v[i].z;
        }
    } else {
        std::vector<float4> v(h->n);
        HIPCHECK(h, hipMemcpy(v.data(), (float4*)h->pos + (size_t)parity * h->npad, sizeof(float4) * h->n,
                              hipMemcpyDeviceToHost));
        for (int i = 0; i < h->n; ++i) {
            xyz[3 * i] = v[i].x;
            xyz[3 * i + 1] = v[i].y;
            xyz[3 * i + 2] = v[i].z;
        }
    }
    return MC_OK;
}

int mc_trace(mc_handle* h, int64_t n_moves, uint8_t* acc, double* dE) {
    if (!h) return MC_E_ARG;
    if (n_moves < 0 || n_moves > h->trace_cap || n_moves > h->sweeps * (int64_t)h->n)
        return fail(h, MC_E_ARG, "n_moves exceeds the traced moves");
    int rc = sync_check(h);
    if (rc) return rc;
    if (acc && n_moves) HIPCHECK(h, hipMemcpy(acc, h->trace_acc, (size_t)n_moves, hipMemcpyDeviceToHost));
    if (dE && n_moves) HIPCHECK(h, hipMemcpy(dE, h->trace_de, sizeof(double) * n_moves, hipMemcpyDeviceToHost));
    return MC_OK;
}

int mc_energy_series(mc_handle* h, int64_t n, double* e) {
    if (!h) return MC_E_ARG;
    if (n < 0 || n > h->sweeps || (n && !e)) return fail(h, MC_E_ARG, "n exceeds the sweeps done");
    int rc = sync_check(h);
    if (rc) return rc;
    if (n) HIPCHECK(h, hipMemcpy(e, h->e_series, sizeof(double) * n, hipMemcpyDeviceToHost));
    return MC_OK;
}

int mc_get_stats(mc_handle* h, mc_stats* out) {
    if (!h || !out) return h ? fail(h, MC_E_ARG, "null output") : MC_E_ARG;
    int rc = sync_check(h);
    if (rc) return rc;
    unsigned long long st[ST_N];
    EnergyAux a;
    HIPCHECK(h, hipMemcpy(st, h->stats, sizeof(st), hipMemcpyDeviceToHost));
    HIPCHECK(h, hipMemcpy(&a, h->aux, sizeof(a), hipMemcpyDeviceToHost));
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
    out->band = h->band;
    out->waves = h->waves;
    out->workgroups = h->wg;
    return MC_OK;
}

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
    h->D = 2.0 * max_disp;
    h->desc.D = h->D;
    return upload_desc(h);
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
