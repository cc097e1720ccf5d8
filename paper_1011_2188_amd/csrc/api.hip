// Host runtime of libfdc.so: the C ABI declared in include/fdc.h.
//
// Owns the device state (track database, material table, plans with their
// tallies and spots), validates every argument before touching the GPU, builds
// the per-run work table (spot history ranges cut into 64-history wave units)
// and enqueues the kernels on the caller's stream.
#include "fdc.h"
#include "fdc_device.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace fdc;

namespace {

struct PlanHost {
    int n[3] = {0, 0, 0};
    float vox[3] = {0, 0, 0};
    float org[3] = {0, 0, 0};
    size_t nvox = 0;
    uint16_t *idx = nullptr;
    unsigned long long *E = nullptr;
    unsigned long long *E2 = nullptr;
    unsigned long long *acc = nullptr;      // incident, escaped, deposited scratch
    std::vector<fdc_spot> spots;
    std::vector<uint64_t> h_next;
    uint64_t n_hist = 0;
    bool var_complete = true;
    // per source (parallel to spots): a spot, or a group of listed protons of
    // one energy bin (fdc_add_phase_space); its spots entry then carries the
    // bin energy, the first proton's start and direction, and the group size
    struct Source {
        uint32_t kind = 0;            // 0 spot, 1 listed protons
        uint32_t bin = 0;
        uint64_t first = 0, count = 0;
        uint64_t db_serial = 0;       // the database the grouping was made for
        int32_t dev = -1;             // beam-line device its histories pass (-1 none)
    };
    std::vector<Source> src;
    float4 *ps = nullptr;             // listed protons of the plan, two float4 each
    uint64_t ps_n = 0;
};

// the default material table: synthetic piecewise-linear constants
const double kDefaultTable[4][4] = {
    // hu, rho, rsp, rscp
    {-1000.0, 0.0012, 0.0011, 0.0012},
    {0.0, 1.0, 1.0, 1.0},
    {1000.0, 1.6, 1.5, 2.16},
    {3071.0, 2.84, 2.64, 3.834},
};

} // namespace

struct fdc_ctx {
    int device = 0;
    bool dry = false;                // no device: validation and host bookkeeping only
    uint64_t seed = 0;
    uint32_t R = 64;
    int cus = 256;
    std::string err;

    fdc_alloc_fn alloc = nullptr;
    fdc_free_fn freef = nullptr;
    void *user = nullptr;
    size_t live_allocs = 0;

    // track database
    float4 *steps = nullptr;
    unsigned long long *track_off = nullptr;
    long long *track_T = nullptr;
    uint32_t *bin_first = nullptr;
    std::vector<float> bin_E;
    std::vector<uint32_t> bin_first_h;
    uint32_t n_tracks = 0, n_bins = 0;
    uint64_t db_serial = 0;           // counts database loads
    std::vector<uint64_t> track_off_h;
    uint64_t n_steps_prim = 0;        // primary steps (the secondaries' follow them in `steps`)
    // secondary trajectories (fdc_load_secondaries): per track its first, the
    // table with its end marker, and what they add to each track's energy
    uint32_t *sec_first = nullptr;
    DevSec *secs = nullptr;
    uint32_t n_sec = 0;
    std::vector<long long> sec_T_track;

    // material table
    std::vector<double> table;   // rows of (hu, rho, rsp, rscp)
    double vacuum_below = -990.0;
    float2 *lut = nullptr;
    float *rho_lut = nullptr;

    // plans and spots
    std::vector<PlanHost> plans;
    DevPlan *d_plans = nullptr;
    size_t d_plans_cap = 0;
    bool plans_dirty = true;
    DevSpot *d_spots = nullptr;
    size_t d_spots_cap = 0;
    unsigned long long *d_hnext = nullptr;   // per DevSpot: next history index
    uint64_t gen = 1;                        // bumped whenever device tables move
    std::vector<uint32_t> spot_base;
    bool spots_dirty = true;

    // per-run work table
    WorkItem *d_items = nullptr;
    WorkItem *h_items = nullptr;     // pinned staging
    size_t items_cap = 0;
    hipEvent_t items_ev = nullptr;
    bool items_ev_pending = false;
    unsigned long long *d_queue = nullptr;

    // processing order by start position (launch config source_order = 1)
    uint32_t *d_order = nullptr;             // units x 64
    size_t order_cap = 0;
    uint32_t *d_hist = nullptr;              // whole-item histograms of spots of more than one chunk
    size_t hist_cap = 0;

    // beam-line devices (fdc_add_beam_device): parameters on the host, pixel
    // arrays and the parameter table on the device
    std::vector<DevDevice> devices;
    DevDevice *d_devices = nullptr;
    size_t d_devices_cap = 0;
    bool devices_dirty = false;

    // read-back scratch
    double *d_dose = nullptr, *d_var = nullptr;
    size_t dose_cap = 0;

    fdc_launch_config cfg{};
    hipStream_t cap_stream = nullptr;        // for graph capture
    unsigned char *scratch = nullptr;        // this device's copy of the static run scratch
    hipError_t scratch_err = hipSuccess;     // why it is missing

    // optional timing of the transport kernel: a ring of event pairs
    static constexpr uint32_t kTimeRing = 64;
    bool timing = false;
    hipEvent_t t_start[kTimeRing] = {}, t_end[kTimeRing] = {};
    uint64_t t_count = 0;
};

struct fdc_graph {
    fdc_ctx *ctx = nullptr;
    uint64_t gen = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    WorkItem *d_items = nullptr;
    uint32_t *d_order = nullptr;             // start-position order table (source_order 1)
    uint32_t *d_hist = nullptr;              // and its whole-item histograms
    std::vector<int32_t> plans;
    uint32_t flags = 0;
    bool reset = false;
};

namespace {

int fail(fdc_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(ctx, FDC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void *dalloc(fdc_ctx *ctx, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (ctx->alloc) {
        p = ctx->alloc(bytes, ctx->user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) ctx->live_allocs++;
    return p;
}

void dfree(fdc_ctx *ctx, void *p)
{
    if (!p) return;
    if (ctx->freef) ctx->freef(p, ctx->user);
    else (void)hipFree(p);
    ctx->live_allocs--;
}

template <class T> T *dalloc_n(fdc_ctx *ctx, size_t n) { return (T *)dalloc(ctx, n * sizeof(T)); }

hipStream_t S(void *s) { return (hipStream_t)s; }

bool finite3(const float v[3]) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

int rebuild_lut(fdc_ctx *ctx)
{
    const int n = (int)(ctx->table.size() / 4);
    double *dt = dalloc_n<double>(ctx, ctx->table.size());
    if (!dt) return fail(ctx, FDC_E_NOMEM, "material table: device allocation failed");
    hipError_t e = hipMemcpy(dt, ctx->table.data(), ctx->table.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_build_lut(dt, n, ctx->vacuum_below, ctx->lut, ctx->rho_lut, nullptr);
    // which voxels are vacuum may have changed: every plan's vacuum-skip bits follow the table
    for (size_t p = 0; p < ctx->plans.size() && e == hipSuccess; ++p) {
        const PlanHost &P = ctx->plans[p];
        if (P.idx) e = launch_vacuum_skip(P.idx, ctx->lut, P.n[0], P.n[1], P.n[2], nullptr);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    dfree(ctx, dt);
    if (e != hipSuccess) return fail(ctx, FDC_E_HIP, "material table: %s", hipGetErrorString(e));
    return FDC_OK;
}

// right-handed lateral axes (e1, e2) of a unit direction d; d = +z gives (x, y)
void field_frame(const double d[3], double e1[3], double e2[3])
{
    double a[3] = {0.0, 0.0, 1.0};
    if (std::fabs(d[2]) >= 0.9) { a[0] = 1.0; a[2] = 0.0; }
    e2[0] = d[1] * a[2] - d[2] * a[1];
    e2[1] = d[2] * a[0] - d[0] * a[2];
    e2[2] = d[0] * a[1] - d[1] * a[0];
    const double l = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    for (int q = 0; q < 3; ++q) e2[q] /= l;
    e1[0] = e2[1] * d[2] - e2[2] * d[1];
    e1[1] = e2[2] * d[0] - e2[0] * d[2];
    e1[2] = e2[0] * d[1] - e2[1] * d[0];
}

// spot -> bin (smallest bin energy >= spot energy); -1 if out of range
int spot_bin(const fdc_ctx *ctx, float E)
{
    if (ctx->n_bins == 0 || !(E >= ctx->bin_E.front()) || !(E <= ctx->bin_E.back())) return -1;
    int b = 0;
    while (ctx->bin_E[b] < E) ++b;
    return b;
}

int check_spot(fdc_ctx *ctx, const fdc_spot &s)
{
    if (!finite3(s.pos_cm) || !finite3(s.dir) || !std::isfinite(s.energy_MeV) || !std::isfinite(s.sigma_cm))
        return fail(ctx, FDC_E_ARG, "spot has a non-finite field");
    const double l = std::sqrt((double)s.dir[0] * s.dir[0] + (double)s.dir[1] * s.dir[1] + (double)s.dir[2] * s.dir[2]);
    if (!(l > 1e-6)) return fail(ctx, FDC_E_ARG, "spot direction is zero");
    if (spot_bin(ctx, s.energy_MeV) < 0)
        return fail(ctx, FDC_E_RANGE, "spot energy %g MeV outside the database bins [%g, %g]", s.energy_MeV,
                    ctx->n_bins ? ctx->bin_E.front() : 0.f, ctx->n_bins ? ctx->bin_E.back() : 0.f);
    return FDC_OK;
}

DevSpot make_dev_spot(const fdc_ctx *ctx, const fdc_spot &s, uint32_t plan, uint32_t idx)
{
    DevSpot d{};
    double dir[3] = {s.dir[0], s.dir[1], s.dir[2]};
    const double l = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    for (int q = 0; q < 3; ++q) dir[q] /= l;
    double e1[3], e2[3];
    field_frame(dir, e1, e2);
    for (int q = 0; q < 3; ++q) {
        d.pos[q] = s.pos_cm[q];
        d.e1[q] = e1[q];
        d.e2[q] = e2[q];
        d.d[q] = dir[q];
        d.m[3 * q + 0] = (float)e1[q];
        d.m[3 * q + 1] = (float)e2[q];
        d.m[3 * q + 2] = (float)dir[q];
    }
    d.sigma = s.sigma_cm;
    const int b = spot_bin(ctx, s.energy_MeV);
    d.bin = (uint32_t)b;
    d.plan = plan;
    d.spot = idx;
    d.dev = -1;
    d.skip = to_fp(ctx->bin_E[b]) - to_fp(s.energy_MeV);
    d.n_hist = s.n_histories;
    return d;
}

int ensure_spots(fdc_ctx *ctx)
{
    if (!ctx->spots_dirty) return FDC_OK;
    std::vector<DevSpot> all;
    ctx->spot_base.assign(ctx->plans.size() + 1, 0);
    for (size_t p = 0; p < ctx->plans.size(); ++p) {
        ctx->spot_base[p] = (uint32_t)all.size();
        for (size_t j = 0; j < ctx->plans[p].spots.size(); ++j) {
            const fdc_spot &s = ctx->plans[p].spots[j];
            int rc = check_spot(ctx, s);
            if (rc) return rc;
            DevSpot d = make_dev_spot(ctx, s, (uint32_t)p, (uint32_t)j);
            const PlanHost::Source &src = ctx->plans[p].src[j];
            d.bin_fp = to_fp(ctx->bin_E[d.bin]);
            d.dev = src.dev;
            if (src.kind) {
                if (src.db_serial != ctx->db_serial || src.bin >= ctx->n_bins)
                    return fail(ctx, FDC_E_STATE, "plan %zu: a phase space was grouped for another track database; "
                                "add it again", p);
                d.kind = 1;
                d.bin = src.bin;
                d.bin_fp = to_fp(ctx->bin_E[src.bin]);
                d.ps_first = src.first;
                d.ps_count = src.count;
            }
            all.push_back(d);
        }
    }
    ctx->spot_base[ctx->plans.size()] = (uint32_t)all.size();
    std::vector<unsigned long long> hn;
    for (const PlanHost &P : ctx->plans) hn.insert(hn.end(), P.h_next.begin(), P.h_next.end());
    if (all.size() > ctx->d_spots_cap) {
        DevSpot *n = dalloc_n<DevSpot>(ctx, all.size());
        unsigned long long *h = dalloc_n<unsigned long long>(ctx, all.size());
        if (!n || !h) {
            dfree(ctx, n); dfree(ctx, h);
            return fail(ctx, FDC_E_NOMEM, "spot table: device allocation failed");
        }
        HIPCHK(hipDeviceSynchronize());
        dfree(ctx, ctx->d_spots);
        dfree(ctx, ctx->d_hnext);
        ctx->d_spots = n;
        ctx->d_hnext = h;
        ctx->d_spots_cap = all.size();
    }
    if (!all.empty()) {
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(ctx->d_spots, all.data(), all.size() * sizeof(DevSpot), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(ctx->d_hnext, hn.data(), hn.size() * 8, hipMemcpyHostToDevice));
    }
    ctx->spots_dirty = false;
    ctx->gen++;
    return FDC_OK;
}

int ensure_plans(fdc_ctx *ctx)
{
    if (!ctx->plans_dirty) return FDC_OK;
    std::vector<DevPlan> all(ctx->plans.size());
    for (size_t p = 0; p < ctx->plans.size(); ++p) {
        const PlanHost &P = ctx->plans[p];
        DevPlan &d = all[p];
        d.idx = P.idx;
        d.E = P.E;
        d.E2 = P.E2;
        d.acc = P.acc;
        d.ps = P.ps;
        for (int q = 0; q < 3; ++q) {
            d.n[q] = P.n[q];
            d.vox[q] = P.vox[q];
            d.inv_vox[q] = 1.f / P.vox[q];
            d.org[q] = P.org[q];
            d.vox_d[q] = P.vox[q];
            d.org_d[q] = P.org[q];
        }
    }
    if (all.size() > ctx->d_plans_cap) {
        const size_t cap = std::max<size_t>(all.size(), 2 * ctx->d_plans_cap);
        DevPlan *n = dalloc_n<DevPlan>(ctx, cap);
        if (!n) return fail(ctx, FDC_E_NOMEM, "plan table: device allocation failed");
        HIPCHK(hipDeviceSynchronize());
        dfree(ctx, ctx->d_plans);
        ctx->d_plans = n;
        ctx->d_plans_cap = cap;
    }
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(ctx->d_plans, all.data(), all.size() * sizeof(DevPlan), hipMemcpyHostToDevice));
    ctx->plans_dirty = false;
    ctx->gen++;
    return FDC_OK;
}

// the device table of the beam-line devices (rebuilt when devices were added)
int ensure_devices(fdc_ctx *ctx)
{
    if (!ctx->devices_dirty) return FDC_OK;
    if (ctx->devices.size() > ctx->d_devices_cap) {
        const size_t cap = std::max<size_t>(ctx->devices.size(), 2 * ctx->d_devices_cap);
        DevDevice *n = dalloc_n<DevDevice>(ctx, cap);
        if (!n) return fail(ctx, FDC_E_NOMEM, "device table: device allocation failed");
        HIPCHK(hipDeviceSynchronize());
        dfree(ctx, ctx->d_devices);
        ctx->d_devices = n;
        ctx->d_devices_cap = cap;
        ctx->gen++;                              // captured graphs hold the old table
    }
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(ctx->d_devices, ctx->devices.data(), ctx->devices.size() * sizeof(DevDevice),
                     hipMemcpyHostToDevice));
    ctx->devices_dirty = false;
    return FDC_OK;
}

int ensure_items(fdc_ctx *ctx, size_t n, hipStream_t s)
{
    if (ctx->items_ev_pending) {
        HIPCHK(hipEventSynchronize(ctx->items_ev));
        ctx->items_ev_pending = false;
    }
    if (n <= ctx->items_cap) return FDC_OK;
    const size_t cap = std::max<size_t>(n, 2 * ctx->items_cap);
    WorkItem *d = dalloc_n<WorkItem>(ctx, cap);
    if (!d) return fail(ctx, FDC_E_NOMEM, "work table: device allocation failed");
    WorkItem *h = nullptr;
    if (hipHostMalloc((void **)&h, cap * sizeof(WorkItem), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        dfree(ctx, d);
        return fail(ctx, FDC_E_NOMEM, "work table: pinned host allocation failed");
    }
    HIPCHK(hipStreamSynchronize(s));      // the old table may still be read by a kernel
    dfree(ctx, ctx->d_items);
    if (ctx->h_items) (void)hipHostFree(ctx->h_items);
    ctx->d_items = d;
    ctx->h_items = h;
    ctx->items_cap = cap;
    return FDC_OK;
}

bool valid_plan(const fdc_ctx *ctx, int32_t plan) { return plan >= 0 && (size_t)plan < ctx->plans.size(); }

TransportArgs base_args(const fdc_ctx *ctx)
{
    TransportArgs a{};
    a.steps = ctx->steps;
    a.track_off = ctx->track_off;
    a.track_T = ctx->track_T;
    a.bin_first = ctx->bin_first;
    a.plans = ctx->d_plans;
    a.spots = ctx->d_spots;
    a.items = ctx->d_items;
    a.hnext = ctx->d_hnext;
    a.lut = ctx->lut;
    a.seed_lo = (uint32_t)ctx->seed;
    a.seed_hi = (uint32_t)(ctx->seed >> 32);
    a.R = ctx->R;
    a.devices = ctx->d_devices;
    a.sec_first = ctx->n_sec ? ctx->sec_first : nullptr;
    a.secs = ctx->n_sec ? ctx->secs : nullptr;
    return a;
}

// grow a device buffer to at least n elements (contents not kept; a buffer
// being replaced may still be read by work on s, so s is drained first)
template <class T>
bool grow(fdc_ctx *ctx, T *&buf, size_t &cap, size_t n, hipStream_t s)
{
    n = std::max<size_t>(n, 1);
    if (cap >= n && buf) return true;
    if (buf) {
        if (hipStreamSynchronize(s) != hipSuccess) return false;
        dfree(ctx, buf);
    }
    buf = nullptr;
    cap = 0;
    buf = (T *)dalloc(ctx, n * sizeof(T));
    if (!buf) return false;
    cap = n;
    return true;
}

// ---- scratch of the allocation-free run --------------------------------------
// fdc_run_histories_noalloc keeps its work table, persistent-queue counter and
// start-position lane table in this statically allocated device array instead
// of context buffers.  Every device the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (taken once per device, with the
// device current, when the first context on it is created).  Layout: the
// queue counter at 0, kNoAllocMaxItems work items from 256, then the lane
// table (64 x 4 B per unit) of up to kNoAllocMaxOrderUnits units, then the
// whole-item histograms (4 B per 16 histories of the lane table, plus one
// counter per item and one).
constexpr size_t kNoAllocBytes = 32u << 20;
constexpr uint32_t kNoAllocMaxItems = 16384;
constexpr size_t kNoAllocItemsOff = 256;
constexpr size_t kNoAllocOrderOff = (kNoAllocItemsOff + kNoAllocMaxItems * sizeof(WorkItem) + 255) & ~(size_t)255;
// per unit: 64 lane words and 64 / 16 histogram counters; and the per-item counters
constexpr unsigned long long kNoAllocMaxOrderUnits =
    (kNoAllocBytes - kNoAllocOrderOff - 4 * (kNoAllocMaxItems + 2) - 256) / (4 * (kWave + kWave / 16));
constexpr size_t kNoAllocHistOff = (kNoAllocOrderOff + kNoAllocMaxOrderUnits * kWave * 4 + 255) & ~(size_t)255;
static_assert(kNoAllocHistOff + 4 * (kNoAllocMaxOrderUnits * kWave / 16 + kNoAllocMaxItems + 2) <= kNoAllocBytes,
              "scratch layout");

} // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// the current device's copy of the scratch array (ctx->device must be current)
hipError_t scratch_address(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

} // namespace

extern "C" {

int fdc_create(fdc_ctx **out, int hip_device, uint64_t seed, uint32_t reuse_R)
{
    if (!out) return FDC_E_ARG;
    *out = nullptr;
    if (reuse_R == 0) return FDC_E_ARG;
    if (hip_device == FDC_NO_DEVICE) {
        fdc_ctx *dry = new (std::nothrow) fdc_ctx();
        if (!dry) return FDC_E_NOMEM;
        dry->dry = true;
        dry->device = -1;
        dry->seed = seed;
        dry->R = reuse_R;
        dry->cfg.waves_per_block = 4;
        *out = dry;
        return FDC_OK;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
        (void)hipGetLastError();
        return FDC_E_HIP;
    }
    fdc_ctx *ctx = new (std::nothrow) fdc_ctx();
    if (!ctx) return FDC_E_NOMEM;
    ctx->err.reserve(512);                   // error messages (< 512 chars) then never allocate
    ctx->device = hip_device;
    ctx->seed = seed;
    ctx->R = reuse_R;
    ctx->cfg.waves_per_block = 4;
    ctx->cfg.blocks_per_cu = 0;
    if (hipSetDevice(hip_device) != hipSuccess) { delete ctx; return FDC_E_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) ctx->cus = prop.multiProcessorCount;
    if (hipEventCreateWithFlags(&ctx->items_ev, hipEventDisableTiming) != hipSuccess) { delete ctx; return FDC_E_HIP; }
    if (prepare_lds_kernels() != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(ctx->items_ev);
        delete ctx;
        return FDC_E_HIP;
    }
    // this device's copy of the allocation-free run's scratch; on failure only
    // that entry point is unavailable (it reports the error)
    ctx->scratch_err = scratch_address(hip_device, &ctx->scratch);
    if (ctx->scratch_err != hipSuccess) {
        (void)hipGetLastError();
        ctx->scratch = nullptr;
    }
    *out = ctx;
    return FDC_OK;
}

int fdc_destroy(fdc_ctx *ctx)
{
    if (!ctx) return FDC_E_ARG;
    if (ctx->dry) { delete ctx; return FDC_OK; }
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (PlanHost &P : ctx->plans) {
        dfree(ctx, P.idx); dfree(ctx, P.E); dfree(ctx, P.E2); dfree(ctx, P.acc); dfree(ctx, P.ps);
    }
    dfree(ctx, ctx->steps); dfree(ctx, ctx->track_off); dfree(ctx, ctx->track_T);
    dfree(ctx, ctx->bin_first);
    dfree(ctx, ctx->sec_first); dfree(ctx, ctx->secs);
    dfree(ctx, ctx->lut); dfree(ctx, ctx->rho_lut);
    dfree(ctx, ctx->d_plans); dfree(ctx, ctx->d_spots); dfree(ctx, ctx->d_items); dfree(ctx, ctx->d_queue);
    for (DevDevice &d : ctx->devices) dfree(ctx, (void *)d.pix);
    dfree(ctx, ctx->d_devices);
    dfree(ctx, ctx->d_order);
    dfree(ctx, ctx->d_hist);
    dfree(ctx, ctx->d_hnext);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    dfree(ctx, ctx->d_dose); dfree(ctx, ctx->d_var);
    if (ctx->h_items) (void)hipHostFree(ctx->h_items);
    if (ctx->items_ev) (void)hipEventDestroy(ctx->items_ev);
    for (uint32_t k = 0; k < fdc_ctx::kTimeRing; ++k) {
        if (ctx->t_start[k]) (void)hipEventDestroy(ctx->t_start[k]);
        if (ctx->t_end[k]) (void)hipEventDestroy(ctx->t_end[k]);
    }
    delete ctx;
    return FDC_OK;
}

const char *fdc_last_error(const fdc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int fdc_set_allocator(fdc_ctx *ctx, fdc_alloc_fn alloc, fdc_free_fn free_fn, void *user)
{
    if (!ctx) return FDC_E_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(ctx, FDC_E_ARG, "give both allocator hooks or none");
    if (ctx->live_allocs) return fail(ctx, FDC_E_STATE, "device memory already allocated");
    ctx->alloc = alloc;
    ctx->freef = free_fn;
    ctx->user = user;
    return FDC_OK;
}

static int ensure_table(fdc_ctx *ctx)
{
    if (ctx->lut) return FDC_OK;
    if (ctx->table.empty()) {
        for (auto &row : kDefaultTable) ctx->table.insert(ctx->table.end(), row, row + 4);
        ctx->vacuum_below = -990.0;
    }
    ctx->lut = dalloc_n<float2>(ctx, kLutSize);
    ctx->rho_lut = dalloc_n<float>(ctx, kLutSize);
    if (!ctx->lut || !ctx->rho_lut) {
        dfree(ctx, ctx->lut); dfree(ctx, ctx->rho_lut);
        ctx->lut = nullptr; ctx->rho_lut = nullptr;
        return fail(ctx, FDC_E_NOMEM, "material table: device allocation failed");
    }
    return rebuild_lut(ctx);
}

int fdc_set_hu_table(fdc_ctx *ctx, const float *hu_pts, const float *rho, const float *rsp, const float *rscp,
                     int n_pts, float vacuum_below_hu)
{
    if (!ctx) return FDC_E_ARG;
    if (!hu_pts || !rho || !rsp || !rscp) return fail(ctx, FDC_E_ARG, "material table: NULL array");
    if (n_pts < 2 || n_pts > kMaxTablePts) return fail(ctx, FDC_E_ARG, "material table: n_pts must be 2..%d", kMaxTablePts);
    if (!std::isfinite(vacuum_below_hu)) return fail(ctx, FDC_E_ARG, "material table: vacuum threshold not finite");
    for (int i = 0; i < n_pts; ++i) {
        if (!std::isfinite(hu_pts[i]) || !std::isfinite(rho[i]) || !std::isfinite(rsp[i]) || !std::isfinite(rscp[i]))
            return fail(ctx, FDC_E_ARG, "material table: non-finite value at point %d", i);
        if (rho[i] < 0.f || rsp[i] < 0.f || rscp[i] < 0.f)
            return fail(ctx, FDC_E_ARG, "material table: negative value at point %d", i);
        if (i && !(hu_pts[i] > hu_pts[i - 1])) return fail(ctx, FDC_E_ARG, "material table: HU not increasing");
    }
    if (ctx->dry) {
        ctx->table.clear();
        for (int i = 0; i < n_pts; ++i) {
            ctx->table.push_back(hu_pts[i]); ctx->table.push_back(rho[i]);
            ctx->table.push_back(rsp[i]); ctx->table.push_back(rscp[i]);
        }
        ctx->vacuum_below = vacuum_below_hu;
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<double> old = ctx->table;
    const double old_vac = ctx->vacuum_below;
    ctx->table.clear();
    for (int i = 0; i < n_pts; ++i) {
        ctx->table.push_back(hu_pts[i]); ctx->table.push_back(rho[i]);
        ctx->table.push_back(rsp[i]); ctx->table.push_back(rscp[i]);
    }
    ctx->vacuum_below = vacuum_below_hu;
    int rc = ctx->lut ? rebuild_lut(ctx) : ensure_table(ctx);
    if (rc) { ctx->table = old; ctx->vacuum_below = old_vac; }
    return rc;
}

int fdc_load_track_db(fdc_ctx *ctx, const fdc_step *steps, uint64_t n_steps, const uint64_t *track_off,
                      uint32_t n_tracks, const float *bin_E, const uint32_t *bin_first, uint32_t n_bins,
                      void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!steps || !track_off || !bin_E || !bin_first) return fail(ctx, FDC_E_ARG, "track database: NULL array");
    if (n_steps == 0 || n_tracks == 0 || n_bins == 0) return fail(ctx, FDC_E_ARG, "track database: zero count");
    if (track_off[0] != 0 || track_off[n_tracks] != n_steps)
        return fail(ctx, FDC_E_FORMAT, "track database: offsets must start at 0 and end at n_steps");
    for (uint32_t t = 0; t < n_tracks; ++t)
        if (!(track_off[t + 1] > track_off[t])) return fail(ctx, FDC_E_FORMAT, "track database: track %u empty or offsets not increasing", t);
    if (bin_first[0] != 0 || bin_first[n_bins] != n_tracks)
        return fail(ctx, FDC_E_FORMAT, "track database: bin_first must start at 0 and end at n_tracks");
    for (uint32_t b = 0; b < n_bins; ++b) {
        if (!(bin_first[b + 1] > bin_first[b])) return fail(ctx, FDC_E_FORMAT, "track database: bin %u empty", b);
        if (!std::isfinite(bin_E[b]) || !(bin_E[b] > 0.f)) return fail(ctx, FDC_E_FORMAT, "track database: bad bin energy");
        if (b && !(bin_E[b] > bin_E[b - 1])) return fail(ctx, FDC_E_FORMAT, "track database: bin energies not increasing");
    }
    for (uint64_t k = 0; k < n_steps; ++k) {
        const fdc_step &s = steps[k];
        if (!std::isfinite(s.dx_cm) || !std::isfinite(s.dE_MeV) || !std::isfinite(s.theta_rad) || !std::isfinite(s.phi_rad))
            return fail(ctx, FDC_E_FORMAT, "track database: non-finite value in step %llu", (unsigned long long)k);
        if (!(s.dx_cm > 0.f) || s.dE_MeV < 0.f || s.theta_rad < 0.f)
            return fail(ctx, FDC_E_FORMAT, "track database: step %llu needs dx > 0, dE >= 0, theta >= 0", (unsigned long long)k);
        if (!(s.dE_MeV < 128.f))       // the walk splits a step's energy in 32-bit fixed point
            return fail(ctx, FDC_E_FORMAT, "track database: step %llu loses %g MeV (must be below 128)",
                        (unsigned long long)k, (double)s.dE_MeV);
    }
    if (ctx->dry) {
        ctx->bin_E.assign(bin_E, bin_E + n_bins);
        ctx->bin_first_h.assign(bin_first, bin_first + n_bins + 1);
        ctx->track_off_h.assign(track_off, track_off + (size_t)n_tracks + 1);
        ctx->n_steps_prim = n_steps;
        ctx->n_sec = 0;
        ctx->sec_T_track.clear();
        ctx->n_tracks = n_tracks;
        ctx->n_bins = n_bins;
        ctx->db_serial++;
        ctx->spots_dirty = true;
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_table(ctx);
    if (rc) return rc;
    float4 *d_steps = dalloc_n<float4>(ctx, n_steps);
    unsigned long long *d_off = dalloc_n<unsigned long long>(ctx, (size_t)n_tracks + 1);
    long long *d_T = dalloc_n<long long>(ctx, n_tracks);
    uint32_t *d_bf = dalloc_n<uint32_t>(ctx, (size_t)n_bins + 1);
    if (!d_steps || !d_off || !d_T || !d_bf) {
        dfree(ctx, d_steps); dfree(ctx, d_off); dfree(ctx, d_T); dfree(ctx, d_bf);
        return fail(ctx, FDC_E_NOMEM, "track database: device allocation of %llu bytes failed",
                    (unsigned long long)(n_steps * sizeof(float4)));
    }
    hipStream_t s = S(hip_stream);
    hipError_t e = hipMemcpyAsync(d_steps, steps, n_steps * sizeof(float4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_off, track_off, ((size_t)n_tracks + 1) * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_bf, bin_first, ((size_t)n_bins + 1) * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_track_energy(d_steps, d_off, d_T, n_tracks, s);   // before the compaction
    if (e == hipSuccess) e = launch_compact_steps(d_steps, n_steps, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        dfree(ctx, d_steps); dfree(ctx, d_off); dfree(ctx, d_T); dfree(ctx, d_bf);
        return fail(ctx, FDC_E_HIP, "track database upload: %s", hipGetErrorString(e));
    }
    HIPCHK(hipDeviceSynchronize());
    dfree(ctx, ctx->steps); dfree(ctx, ctx->track_off); dfree(ctx, ctx->track_T);
    dfree(ctx, ctx->bin_first);
    dfree(ctx, ctx->sec_first); dfree(ctx, ctx->secs);
    ctx->sec_first = nullptr;
    ctx->secs = nullptr;
    ctx->n_sec = 0;
    ctx->sec_T_track.clear();
    ctx->steps = d_steps;
    ctx->track_off = d_off;
    ctx->track_T = d_T;
    ctx->bin_first = d_bf;
    ctx->bin_E.assign(bin_E, bin_E + n_bins);
    ctx->bin_first_h.assign(bin_first, bin_first + n_bins + 1);
    ctx->track_off_h.assign(track_off, track_off + (size_t)n_tracks + 1);
    ctx->n_steps_prim = n_steps;
    ctx->n_tracks = n_tracks;
    ctx->n_bins = n_bins;
    ctx->db_serial++;
    ctx->spots_dirty = true;
    ctx->gen++;
    return FDC_OK;
}

int fdc_load_secondaries(fdc_ctx *ctx, const uint32_t *sec_first, const uint64_t *sec_off, uint32_t n_sec,
                         const fdc_step *steps, uint64_t n_sec_steps, const uint32_t *branch, const float *emit,
                         void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (ctx->n_bins == 0) return fail(ctx, FDC_E_STATE, "secondaries: load a track database first");
    if (!sec_first || !sec_off) return fail(ctx, FDC_E_ARG, "secondaries: NULL array");
    if (n_sec && (!steps || !branch || !emit)) return fail(ctx, FDC_E_ARG, "secondaries: NULL array");
    const uint32_t nt = ctx->n_tracks;
    if (sec_first[0] != 0 || sec_first[nt] != n_sec)
        return fail(ctx, FDC_E_FORMAT, "secondaries: sec_first must start at 0 and end at n_sec");
    if (sec_off[0] != 0 || sec_off[n_sec] != n_sec_steps)
        return fail(ctx, FDC_E_FORMAT, "secondaries: offsets must start at 0 and end at n_sec_steps");
    for (uint32_t t = 0; t < nt; ++t) {
        if (sec_first[t + 1] < sec_first[t]) return fail(ctx, FDC_E_FORMAT, "secondaries: sec_first decreases at track %u", t);
        if (sec_first[t + 1] - sec_first[t] > kMaxSecPerTrack)
            return fail(ctx, FDC_E_FORMAT, "secondaries: track %u has %u (at most %u)", t, sec_first[t + 1] - sec_first[t],
                        kMaxSecPerTrack);
        const uint64_t ns = ctx->track_off_h[t + 1] - ctx->track_off_h[t];
        for (uint32_t j = sec_first[t]; j < sec_first[t + 1]; ++j) {
            if (branch[j] >= ns) return fail(ctx, FDC_E_FORMAT, "secondaries: %u branches past its track's last step", j);
            if (j > sec_first[t] && branch[j] < branch[j - 1])
                return fail(ctx, FDC_E_FORMAT, "secondaries: branch steps of track %u not in order", t);
        }
    }
    for (uint32_t j = 0; j < n_sec; ++j) {
        if (!(sec_off[j + 1] > sec_off[j])) return fail(ctx, FDC_E_FORMAT, "secondaries: %u empty or offsets not increasing", j);
        const float th = emit[2 * j], ph = emit[2 * j + 1];
        if (!std::isfinite(th) || !std::isfinite(ph) || th < 0.f || th > 3.14159274f)
            return fail(ctx, FDC_E_FORMAT, "secondaries: %u needs a finite azimuth and a polar angle in [0, pi]", j);
    }
    for (uint64_t k = 0; k < n_sec_steps; ++k) {
        const fdc_step &st = steps[k];
        if (!std::isfinite(st.dx_cm) || !std::isfinite(st.dE_MeV) || !std::isfinite(st.theta_rad) ||
            !std::isfinite(st.phi_rad) || !(st.dx_cm > 0.f) || st.dE_MeV < 0.f || st.theta_rad < 0.f ||
            !(st.dE_MeV < 128.f))
            return fail(ctx, FDC_E_FORMAT, "secondaries: step %llu needs finite values, dx > 0, 0 <= dE < 128 MeV, "
                        "theta >= 0", (unsigned long long)k);
    }
    // the table: each secondary's steps behind the primary steps, its branch
    // step in the same numbering, its energy, and the end marker
    std::vector<DevSec> tab((size_t)n_sec + 1);
    std::vector<long long> add(nt, 0);
    for (uint32_t t = 0; t < nt; ++t) {
        for (uint32_t j = sec_first[t]; j < sec_first[t + 1]; ++j) {
            DevSec &d = tab[j];
            d.k0 = ctx->n_steps_prim + sec_off[j];
            d.k1 = ctx->n_steps_prim + sec_off[j + 1];
            d.kb = ctx->track_off_h[t] + branch[j];
            long long T = 0;
            for (uint64_t k = sec_off[j]; k < sec_off[j + 1]; ++k) T += to_fp(steps[k].dE_MeV);
            d.T = T;
            const double th = emit[2 * j], ph = emit[2 * j + 1];
            d.ct = (float)cos(th);
            d.st = (float)sin(th);
            d.cph = (float)cos(ph);
            d.sph = (float)sin(ph);
            add[t] += T;
        }
    }
    tab[n_sec] = DevSec{~0ull, ~0ull, ~0ull, 0, 1.f, 0.f, 1.f, 0.f};
    if (ctx->dry) {
        ctx->n_sec = n_sec;
        ctx->sec_T_track = add;
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    const uint64_t np = ctx->n_steps_prim;
    float4 *d_steps = dalloc_n<float4>(ctx, np + n_sec_steps);
    uint32_t *d_first = dalloc_n<uint32_t>(ctx, (size_t)nt + 1);
    DevSec *d_tab = dalloc_n<DevSec>(ctx, (size_t)n_sec + 1);
    if (!d_steps || !d_first || !d_tab) {
        dfree(ctx, d_steps); dfree(ctx, d_first); dfree(ctx, d_tab);
        return fail(ctx, FDC_E_NOMEM, "secondaries: device allocation failed");
    }
    // the tracks' energies with the new secondaries in place of the old
    std::vector<long long> T(nt);
    hipStream_t s = S(hip_stream);
    hipError_t e = hipMemcpyAsync(T.data(), ctx->track_T, (size_t)nt * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (uint32_t t = 0; t < nt && e == hipSuccess; ++t)
        T[t] += add[t] - (ctx->sec_T_track.empty() ? 0 : ctx->sec_T_track[t]);
    if (e == hipSuccess) e = hipMemcpyAsync(d_steps, ctx->steps, np * sizeof(float4), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && n_sec_steps)
        e = hipMemcpyAsync(d_steps + np, steps, n_sec_steps * sizeof(float4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n_sec_steps) e = launch_compact_steps(d_steps + np, n_sec_steps, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_first, sec_first, ((size_t)nt + 1) * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_tab, tab.data(), tab.size() * sizeof(DevSec), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->track_T, T.data(), (size_t)nt * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        dfree(ctx, d_steps); dfree(ctx, d_first); dfree(ctx, d_tab);
        return fail(ctx, FDC_E_HIP, "secondaries upload: %s", hipGetErrorString(e));
    }
    dfree(ctx, ctx->steps); dfree(ctx, ctx->sec_first); dfree(ctx, ctx->secs);
    ctx->steps = d_steps;
    ctx->sec_first = d_first;
    ctx->secs = d_tab;
    ctx->n_sec = n_sec;
    ctx->sec_T_track = add;
    ctx->gen++;
    return FDC_OK;
}

// Track-database file: the header below (little-endian), then bin_E
// (f32 x n_bins), bin_first (u32 x n_bins+1), track_off (u64 x n_tracks+1)
// and the steps (4 x f32 each), packed in that order.
namespace {
struct DbFileHeader {
    char magic[8];                   // "FDCTRKDB"
    uint32_t version;                // 1, or 2 with secondary trajectories
    uint32_t n_bins, n_tracks, n_sec;   // (n_sec: version 2 only)
    uint64_t n_steps;
    uint64_t db_seed;
    double physics[8];               // generator constants, informational
};
static_assert(sizeof(DbFileHeader) == 104, "track database header layout");
} // namespace

int fdc_load_track_db_file(fdc_ctx *ctx, const char *path, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!path) return fail(ctx, FDC_E_ARG, "track database file: NULL path");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, FDC_E_ARG, "track database file: cannot open %s", path);
    DbFileHeader h;
    long long size = -1;
    if (std::fseek(f, 0, SEEK_END) == 0) size = std::ftell(f);
    std::rewind(f);
    if (std::fread(&h, sizeof h, 1, f) != 1) { std::fclose(f); return fail(ctx, FDC_E_FORMAT, "track database file: short header"); }
    if (std::memcmp(h.magic, "FDCTRKDB", 8) != 0 || (h.version != 1 && h.version != 2)) {
        std::fclose(f);
        return fail(ctx, FDC_E_FORMAT, "track database file: bad magic or version %u", h.version);
    }
    if (h.n_bins == 0 || h.n_tracks == 0 || h.n_steps == 0 || h.n_steps > (1ull << 40)) {
        std::fclose(f);
        return fail(ctx, FDC_E_FORMAT, "track database file: empty or implausible counts");
    }
    const bool v2 = h.version == 2;
    const uint64_t n_sec = v2 ? h.n_sec : 0;
    const unsigned long long body = sizeof h + 4ull * h.n_bins + 4ull * (h.n_bins + 1ull) +
                                    8ull * (h.n_tracks + 1ull) + 16ull * h.n_steps;
    uint64_t n_sec_steps = 0;
    if (v2) {
        // the secondaries' section: its step count, then sec_first, sec_off,
        // branch, emit and the steps
        if (std::fseek(f, (long)body, SEEK_SET) != 0 || std::fread(&n_sec_steps, 8, 1, f) != 1 ||
            n_sec_steps > (1ull << 40)) {
            std::fclose(f);
            return fail(ctx, FDC_E_FORMAT, "track database file: missing or implausible secondaries section");
        }
        std::fseek(f, (long)sizeof h, SEEK_SET);
    }
    const unsigned long long want = body + (v2 ? 8ull + 4ull * (h.n_tracks + 1ull) + 8ull * (n_sec + 1ull) +
                                                     4ull * n_sec + 8ull * n_sec + 16ull * n_sec_steps
                                               : 0ull);
    if (size < 0 || (unsigned long long)size != want) {
        std::fclose(f);
        return fail(ctx, FDC_E_FORMAT, "track database file: %lld bytes, the header implies %llu", size, want);
    }
    std::vector<float> bin_E, emit;
    std::vector<uint32_t> bin_first, sec_first, branch;
    std::vector<uint64_t> off, sec_off;
    std::vector<fdc_step> steps, sec_steps;
    try {
        bin_E.resize(h.n_bins);
        bin_first.resize(h.n_bins + 1ull);
        off.resize(h.n_tracks + 1ull);
        steps.resize(h.n_steps);
        if (v2) {
            sec_first.resize(h.n_tracks + 1ull);
            sec_off.resize(n_sec + 1ull);
            branch.resize(n_sec);
            emit.resize(2 * n_sec);
            sec_steps.resize(n_sec_steps);
        }
    } catch (const std::bad_alloc &) {
        std::fclose(f);
        return fail(ctx, FDC_E_NOMEM, "track database file: host buffers");
    }
    bool ok = std::fread(bin_E.data(), 4, bin_E.size(), f) == bin_E.size() &&
              std::fread(bin_first.data(), 4, bin_first.size(), f) == bin_first.size() &&
              std::fread(off.data(), 8, off.size(), f) == off.size() &&
              std::fread(steps.data(), sizeof(fdc_step), steps.size(), f) == steps.size();
    if (ok && v2) {
        uint64_t again = 0;
        ok = std::fread(&again, 8, 1, f) == 1 &&
             std::fread(sec_first.data(), 4, sec_first.size(), f) == sec_first.size() &&
             std::fread(sec_off.data(), 8, sec_off.size(), f) == sec_off.size() &&
             std::fread(branch.data(), 4, branch.size(), f) == branch.size() &&
             std::fread(emit.data(), 4, emit.size(), f) == emit.size() &&
             std::fread(sec_steps.data(), sizeof(fdc_step), sec_steps.size(), f) == sec_steps.size();
    }
    std::fclose(f);
    if (!ok) return fail(ctx, FDC_E_FORMAT, "track database file: short read");
    int rc = fdc_load_track_db(ctx, steps.data(), h.n_steps, off.data(), h.n_tracks, bin_E.data(), bin_first.data(),
                               h.n_bins, hip_stream);
    if (rc == FDC_OK && v2)
        rc = fdc_load_secondaries(ctx, sec_first.data(), sec_off.data(), (uint32_t)n_sec, sec_steps.data(),
                                  n_sec_steps, branch.data(), emit.data(), hip_stream);
    return rc;
}

int fdc_load_phantom(fdc_ctx *ctx, int32_t *plan_out, const int16_t *hu, int nx, int ny, int nz,
                     const float voxel_cm[3], const float origin_cm[3], void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!plan_out || !hu || !voxel_cm || !origin_cm) return fail(ctx, FDC_E_ARG, "phantom: NULL argument");
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(ctx, FDC_E_ARG, "phantom: dimensions must be positive");
    const size_t nvox = (size_t)nx * ny * nz;
    if (nvox >= (size_t(1) << 31)) return fail(ctx, FDC_E_ARG, "phantom: more than 2^31 voxels");
    if (!finite3(voxel_cm) || !finite3(origin_cm) || !(voxel_cm[0] > 0.f) || !(voxel_cm[1] > 0.f) || !(voxel_cm[2] > 0.f))
        return fail(ctx, FDC_E_ARG, "phantom: voxel sizes must be positive and finite");
    if (ctx->plans.size() >= (1u << 27)) return fail(ctx, FDC_E_ARG, "phantom: too many plans");
    PlanHost P;
    P.n[0] = nx; P.n[1] = ny; P.n[2] = nz;
    for (int q = 0; q < 3; ++q) { P.vox[q] = voxel_cm[q]; P.org[q] = origin_cm[q]; }
    P.nvox = nvox;
    if (ctx->dry) {
        ctx->plans.push_back(std::move(P));
        *plan_out = (int32_t)(ctx->plans.size() - 1);
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_table(ctx);
    if (rc) return rc;
    int16_t *d_hu = dalloc_n<int16_t>(ctx, nvox);
    P.idx = dalloc_n<uint16_t>(ctx, nvox);
    P.E = dalloc_n<unsigned long long>(ctx, nvox);
    P.E2 = dalloc_n<unsigned long long>(ctx, nvox);
    P.acc = dalloc_n<unsigned long long>(ctx, 8);
    if (!d_hu || !P.idx || !P.E || !P.E2 || !P.acc) {
        dfree(ctx, d_hu); dfree(ctx, P.idx); dfree(ctx, P.E); dfree(ctx, P.E2); dfree(ctx, P.acc);
        return fail(ctx, FDC_E_NOMEM, "phantom: device allocation failed (%zu voxels)", nvox);
    }
    hipStream_t s = S(hip_stream);
    hipError_t e = hipMemcpyAsync(d_hu, hu, nvox * sizeof(int16_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_hu_to_index(d_hu, P.idx, nvox, s);
    if (e == hipSuccess) e = launch_vacuum_skip(P.idx, ctx->lut, nx, ny, nz, s);
    if (e == hipSuccess) e = hipMemsetAsync(P.E, 0, nvox * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(P.E2, 0, nvox * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(P.acc, 0, 64, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(ctx, d_hu);
    if (e != hipSuccess) {
        dfree(ctx, P.idx); dfree(ctx, P.E); dfree(ctx, P.E2); dfree(ctx, P.acc);
        return fail(ctx, FDC_E_HIP, "phantom upload: %s", hipGetErrorString(e));
    }
    ctx->plans.push_back(std::move(P));
    ctx->plans_dirty = true;
    ctx->spots_dirty = true;
    *plan_out = (int32_t)(ctx->plans.size() - 1);
    return FDC_OK;
}

int fdc_add_beam_spots(fdc_ctx *ctx, int32_t plan, const fdc_spot *spots, uint32_t n)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "spots: no plan %d", plan);
    if (n && !spots) return fail(ctx, FDC_E_ARG, "spots: NULL array");
    if (ctx->n_bins == 0) return fail(ctx, FDC_E_STATE, "spots: load a track database first");
    for (uint32_t i = 0; i < n; ++i) {
        int rc = check_spot(ctx, spots[i]);
        if (rc) return rc;
    }
    PlanHost &P = ctx->plans[plan];
    P.spots.insert(P.spots.end(), spots, spots + n);
    P.src.resize(P.spots.size());
    P.h_next.resize(P.spots.size(), 0);
    ctx->spots_dirty = true;
    return FDC_OK;
}

int fdc_add_beam_device(fdc_ctx *ctx, const fdc_beam_device *dev, const float *pixels, int32_t *device_out,
                        void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!dev || !pixels || !device_out) return fail(ctx, FDC_E_ARG, "beam device: NULL argument");
    if (!finite3(dev->origin_cm) || !finite3(dev->dir) || !std::isfinite(dev->pitch_cm[0]) ||
        !std::isfinite(dev->pitch_cm[1]) || !(dev->pitch_cm[0] > 0.f) || !(dev->pitch_cm[1] > 0.f))
        return fail(ctx, FDC_E_ARG, "beam device: non-finite position or direction, or pitch <= 0");
    const double l = std::sqrt((double)dev->dir[0] * dev->dir[0] + (double)dev->dir[1] * dev->dir[1] +
                               (double)dev->dir[2] * dev->dir[2]);
    if (!(l > 1e-6)) return fail(ctx, FDC_E_ARG, "beam device: direction is zero");
    const uint64_t np = (uint64_t)dev->n[0] * dev->n[1];
    if (dev->n[0] == 0 || dev->n[1] == 0 || np > (1ull << 26) || dev->n[0] > 0x7FFFFFFFu || dev->n[1] > 0x7FFFFFFFu)
        return fail(ctx, FDC_E_ARG, "beam device: grid must have 1 .. 2^26 pixels");
    bool material = false;
    for (uint64_t i = 0; i < np; ++i) {
        if (!std::isfinite(pixels[i])) return fail(ctx, FDC_E_ARG, "beam device: non-finite pixel %llu",
                                                   (unsigned long long)i);
        material |= pixels[i] > 0.f;
    }
    if (material && (!(dev->rsp > 0.f) || !(dev->rscp > 0.f) || !std::isfinite(dev->rsp) || !std::isfinite(dev->rscp)))
        return fail(ctx, FDC_E_ARG, "beam device: compensator rsp and rscp must be finite and > 0");
    if (ctx->dry) {
        DevDevice d{};
        ctx->devices.push_back(d);
        *device_out = (int32_t)ctx->devices.size() - 1;
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    float *pix = dalloc_n<float>(ctx, np);
    if (!pix) return fail(ctx, FDC_E_NOMEM, "beam device: pixel allocation failed");
    hipError_t e = hipMemcpyAsync(pix, pixels, np * sizeof(float), hipMemcpyHostToDevice, S(hip_stream));
    if (e == hipSuccess) e = hipStreamSynchronize(S(hip_stream));
    if (e != hipSuccess) {
        dfree(ctx, pix);
        return fail(ctx, FDC_E_HIP, "beam device: %s", hipGetErrorString(e));
    }
    DevDevice d{};
    double nrm[3] = {dev->dir[0] / l, dev->dir[1] / l, dev->dir[2] / l};
    double u1[3], u2[3];
    field_frame(nrm, u1, u2);
    for (int q = 0; q < 3; ++q) {
        d.o[q] = dev->origin_cm[q];
        d.nrm[q] = nrm[q];
        d.u1[q] = u1[q];
        d.u2[q] = u2[q];
    }
    d.pitch[0] = dev->pitch_cm[0];
    d.pitch[1] = dev->pitch_cm[1];
    d.npix[0] = (int)dev->n[0];
    d.npix[1] = (int)dev->n[1];
    d.rsp = material ? dev->rsp : 1.0;
    d.g = material ? (double)dev->rscp / (double)dev->rsp : 1.0;
    d.pix = pix;
    ctx->devices.push_back(d);
    ctx->devices_dirty = true;
    *device_out = (int32_t)ctx->devices.size() - 1;
    return FDC_OK;
}

int fdc_set_spot_device(fdc_ctx *ctx, int32_t plan, uint32_t first_spot, uint32_t n_spots, int32_t device)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "spot device: no plan %d", plan);
    PlanHost &P = ctx->plans[plan];
    if ((uint64_t)first_spot + n_spots > P.spots.size())
        return fail(ctx, FDC_E_ARG, "spot device: spots %u .. %u beyond the plan's %zu", first_spot,
                    first_spot + n_spots, P.spots.size());
    if (device < -1 || device >= (int64_t)ctx->devices.size())
        return fail(ctx, FDC_E_ARG, "spot device: no device %d", device);
    for (uint32_t j = first_spot; j < first_spot + n_spots; ++j)
        if (P.src[j].kind) return fail(ctx, FDC_E_ARG, "spot device: source %u lists protons", j);
    for (uint32_t j = first_spot; j < first_spot + n_spots; ++j) P.src[j].dev = device;
    ctx->spots_dirty = true;
    return FDC_OK;
}

int fdc_add_phase_space(fdc_ctx *ctx, int32_t plan, const fdc_particle *particles, uint64_t n,
                        uint32_t *n_sources_out, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (n_sources_out) *n_sources_out = 0;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "phase space: no plan %d", plan);
    if (n && !particles) return fail(ctx, FDC_E_ARG, "phase space: NULL array");
    if (ctx->n_bins == 0) return fail(ctx, FDC_E_STATE, "phase space: load a track database first");
    if (n > (1ull << 40)) return fail(ctx, FDC_E_ARG, "phase space: too many protons");
    std::vector<uint32_t> bin;
    try {
        bin.resize(n);
    } catch (const std::bad_alloc &) {
        return fail(ctx, FDC_E_NOMEM, "phase space: host buffers");
    }
    for (uint64_t i = 0; i < n; ++i) {
        const fdc_particle &q = particles[i];
        if (!finite3(q.pos_cm) || !finite3(q.dir) || !std::isfinite(q.energy_MeV))
            return fail(ctx, FDC_E_ARG, "phase space: proton %llu has a non-finite field", (unsigned long long)i);
        if (q.dir[0] == 0.f && q.dir[1] == 0.f && q.dir[2] == 0.f)
            return fail(ctx, FDC_E_ARG, "phase space: proton %llu has a zero direction", (unsigned long long)i);
        if (q.reserved != 0.f) return fail(ctx, FDC_E_ARG, "phase space: proton %llu: reserved field not 0",
                                           (unsigned long long)i);
        const int b = spot_bin(ctx, q.energy_MeV);
        if (b < 0 || !(q.energy_MeV >= ctx->bin_E[0]))
            return fail(ctx, FDC_E_RANGE, "phase space: proton %llu energy %g MeV outside the bins [%g, %g]",
                        (unsigned long long)i, (double)q.energy_MeV, (double)ctx->bin_E[0],
                        (double)ctx->bin_E.back());
        bin[i] = (uint32_t)b;
    }
    PlanHost &P = ctx->plans[plan];
    // protons grouped by bin (bins ascending, list order within a bin)
    std::vector<uint64_t> order;
    std::vector<float4> host;
    try {
        order.resize(n);
        host.resize(2 * n);
    } catch (const std::bad_alloc &) {
        return fail(ctx, FDC_E_NOMEM, "phase space: host buffers");
    }
    for (uint64_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint64_t x, uint64_t y) { return bin[x] < bin[y]; });
    for (uint64_t k = 0; k < n; ++k) {
        const fdc_particle &q = particles[order[k]];
        host[2 * k] = make_float4(q.pos_cm[0], q.pos_cm[1], q.pos_cm[2], q.energy_MeV);
        host[2 * k + 1] = make_float4(q.dir[0], q.dir[1], q.dir[2], 0.f);
    }
    if (!ctx->dry && n) {
        HIPCHK(hipSetDevice(ctx->device));
        float4 *d = dalloc_n<float4>(ctx, 2 * (P.ps_n + n));
        if (!d) return fail(ctx, FDC_E_NOMEM, "phase space: device allocation of %llu protons failed",
                            (unsigned long long)(P.ps_n + n));
        hipStream_t s = S(hip_stream);
        hipError_t e = hipSuccess;
        if (P.ps_n) e = hipMemcpyAsync(d, P.ps, 2 * P.ps_n * sizeof(float4), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d + 2 * P.ps_n, host.data(), 2 * n * sizeof(float4),
                                                hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipDeviceSynchronize();     // the old list may be read by earlier work
        if (e != hipSuccess) {
            dfree(ctx, d);
            return fail(ctx, FDC_E_HIP, "phase space upload: %s", hipGetErrorString(e));
        }
        dfree(ctx, P.ps);
        P.ps = d;
        ctx->plans_dirty = true;
    }
    uint32_t added = 0;
    for (uint64_t k = 0; k < n;) {
        uint64_t m = k;
        while (m < n && bin[order[m]] == bin[order[k]]) ++m;
        const fdc_particle &q = particles[order[k]];
        fdc_spot sp{};
        for (int a = 0; a < 3; ++a) { sp.pos_cm[a] = q.pos_cm[a]; sp.dir[a] = q.dir[a]; }
        sp.energy_MeV = ctx->bin_E[bin[order[k]]];
        sp.sigma_cm = 0.f;
        sp.n_histories = m - k;
        PlanHost::Source src;
        src.kind = 1;
        src.bin = bin[order[k]];
        src.first = P.ps_n + k;
        src.count = m - k;
        src.db_serial = ctx->db_serial;
        P.spots.push_back(sp);
        P.src.push_back(src);
        ++added;
        k = m;
    }
    P.ps_n += n;
    P.h_next.resize(P.spots.size(), 0);
    ctx->spots_dirty = true;
    if (n_sources_out) *n_sources_out = added;
    return FDC_OK;
}

int fdc_add_phase_space_file(fdc_ctx *ctx, int32_t plan, const char *path, uint32_t *n_sources_out,
                             void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (n_sources_out) *n_sources_out = 0;
    if (!path) return fail(ctx, FDC_E_ARG, "phase space file: NULL path");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, FDC_E_ARG, "phase space file: cannot open %s", path);
    struct {
        char magic[8];
        uint32_t version, record_bytes;
        uint64_t n, reserved;
    } h;
    static_assert(sizeof(h) == 32, "phase space header layout");
    long long size = -1;
    if (std::fseek(f, 0, SEEK_END) == 0) size = std::ftell(f);
    std::rewind(f);
    if (std::fread(&h, sizeof h, 1, f) != 1) { std::fclose(f); return fail(ctx, FDC_E_FORMAT, "phase space file: short header"); }
    if (std::memcmp(h.magic, "FDCPHSP1", 8) != 0 || h.version != 1 || h.record_bytes != sizeof(fdc_particle)) {
        std::fclose(f);
        return fail(ctx, FDC_E_FORMAT, "phase space file: bad magic, version or record size");
    }
    if (h.n > (1ull << 40) || size < 0 || (unsigned long long)size != sizeof h + h.n * sizeof(fdc_particle)) {
        std::fclose(f);
        return fail(ctx, FDC_E_FORMAT, "phase space file: %lld bytes do not hold the %llu protons of its header",
                    size, (unsigned long long)h.n);
    }
    std::vector<fdc_particle> q;
    try {
        q.resize(h.n);
    } catch (const std::bad_alloc &) {
        std::fclose(f);
        return fail(ctx, FDC_E_NOMEM, "phase space file: host buffer");
    }
    const bool ok = std::fread(q.data(), sizeof(fdc_particle), q.size(), f) == q.size();
    std::fclose(f);
    if (!ok) return fail(ctx, FDC_E_FORMAT, "phase space file: short read");
    return fdc_add_phase_space(ctx, plan, q.data(), h.n, n_sources_out, hip_stream);
}

static int validate_run(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags, uint64_t launches)
{
    if (n_plans && !plans) return fail(ctx, FDC_E_ARG, "run: NULL plan list");
    if (flags & ~(uint32_t)(FDC_RUN_VARIANCE | FDC_RUN_ROTATE_TRACKS | FDC_RUN_COUNT_WORK))
        return fail(ctx, FDC_E_ARG, "run: unknown flag");
    if (ctx->n_bins == 0) return fail(ctx, FDC_E_STATE, "run: no track database loaded");
    for (uint32_t i = 0; i < n_plans; ++i)
        if (!valid_plan(ctx, plans[i])) return fail(ctx, FDC_E_ARG, "run: no plan %d", plans[i]);
    if (n_plans <= kMaxRangePlans) {            // (no host allocation for short lists)
        for (uint32_t i = 1; i < n_plans; ++i)
            for (uint32_t j = 0; j < i; ++j)
                if (plans[i] == plans[j]) return fail(ctx, FDC_E_ARG, "run: plan %d listed twice", plans[i]);
    } else {
        std::vector<char> seen(ctx->plans.size(), 0);
        for (uint32_t i = 0; i < n_plans; ++i)
            if (seen[plans[i]]++) return fail(ctx, FDC_E_ARG, "run: plan %d listed twice", plans[i]);
    }
    // overflow guard: every history deposits at most the largest bin energy
    const double emax = (double)to_fp(ctx->bin_E.back());
    for (uint32_t i = 0; i < n_plans; ++i) {
        const PlanHost &P = ctx->plans[plans[i]];
        double nh = (double)P.n_hist;
        for (const fdc_spot &s : P.spots) nh += (double)s.n_histories * (double)launches;
        if (nh * emax >= 9.2e18) return fail(ctx, FDC_E_OVERFLOW, "run: plan %d would exceed the int64 tally", plans[i]);
    }
    return FDC_OK;
}

// host bookkeeping of a launched run (the device counters advance by themselves)
static void account_run(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags, bool reset)
{
    for (uint32_t i = 0; i < n_plans; ++i) {
        PlanHost &P = ctx->plans[plans[i]];
        if (reset) {
            P.n_hist = 0;
            P.var_complete = true;
        }
        for (size_t j = 0; j < P.spots.size(); ++j) {
            P.h_next[j] += P.spots[j].n_histories;
            P.n_hist += P.spots[j].n_histories;
            if (P.spots[j].n_histories && !(flags & FDC_RUN_VARIANCE)) P.var_complete = false;
        }
    }
}

static unsigned long long build_items(const fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans,
                                      std::vector<WorkItem> &items, uint32_t *n_chunks = nullptr)
{
    unsigned long long units = 0, hist = 0, chunks = 0;
    items.clear();
    for (uint32_t i = 0; i < n_plans; ++i) {
        const PlanHost &P = ctx->plans[plans[i]];
        for (size_t j = 0; j < P.spots.size(); ++j) {
            const uint64_t n = P.spots[j].n_histories;
            if (!n) continue;
            WorkItem w{};
            w.h0 = 0;                              // the spot's device counter is added
            w.n = n;
            w.unit0 = units;
            w.first = hist;
            hist += n;
            w.gspot = ctx->spot_base[plans[i]] + (uint32_t)j;
            w.chunk0 = (uint32_t)chunks;
            items.push_back(w);
            units += units_for(n);
            chunks += source_order_chunks(n);
        }
    }
    if (n_chunks) *n_chunks = (uint32_t)std::min<unsigned long long>(chunks, 0xFFFFFFFFull);
    return units;
}

// the run's processing order by start position (enqueued on s after the
// work table's upload): the per-unit lane table of `units` units, into *order
// grown to fit
static int check_source_order(fdc_ctx *ctx, const std::vector<WorkItem> &items)
{
    unsigned long long chunks = 0;
    for (const WorkItem &w : items) {
        if (w.n >= 0xFFFFFFFFull) return fail(ctx, FDC_E_ARG, "run: source_order needs fewer than 2^32 histories per spot");
        chunks += source_order_chunks(w.n);
    }
    if (chunks > 0x7FFFFFFFull) return fail(ctx, FDC_E_ARG, "run: source_order needs fewer than 2^45 histories per run");
    return FDC_OK;
}

// does the run have spots of more than one ordering chunk (whole-item histograms),
// and how many histogram counters do they need
static bool large_items(const std::vector<WorkItem> &items, unsigned long long *hist_words)
{
    unsigned long long n = 0;
    bool large = false;
    for (const WorkItem &w : items) {
        n += w.n;
        large |= w.n > kOrderWholeSpot;
    }
    *hist_words = order_hist_words(n, items.size());
    return large;
}

static int enqueue_source_order(fdc_ctx *ctx, const WorkItem *d_items, const std::vector<WorkItem> &items,
                                uint32_t n_chunks, unsigned long long units, uint32_t *order, uint32_t *hist,
                                hipStream_t s)
{
    unsigned long long hw = 0;
    const bool large = large_items(items, &hw);
    const OrderTracks ot{ctx->bin_first, ctx->n_sec ? ctx->sec_first : nullptr, ctx->R};
    HIPCHK(launch_source_order(d_items, (uint32_t)items.size(), n_chunks, units, ctx->d_spots, ctx->d_hnext,
                               (uint32_t)ctx->seed, (uint32_t)(ctx->seed >> 32), order, hist, hw, large, ot, s));
    return FDC_OK;
}

static bool one_plan(const int32_t *plans, uint32_t n_plans)
{
    for (uint32_t i = 1; i < n_plans; ++i)
        if (plans[i] != plans[0]) return false;
    return true;
}

// transport launch for a work table already on the device; the queue counter
// is cleared with a kernel so that the sequence can be captured in a graph
static int enqueue_transport_kernel(fdc_ctx *ctx, TransportArgs a, uint32_t flags, hipStream_t s, bool one_plan,
                                    unsigned long long *queue = nullptr);

// the transport kernel, bracketed by the context's timing events when timing
// is on (eager runs only)
static int enqueue_transport(fdc_ctx *ctx, TransportArgs a, uint32_t flags, hipStream_t s, bool one_plan,
                             bool timed = false)
{
    if (!timed || !ctx->timing) return enqueue_transport_kernel(ctx, a, flags, s, one_plan);
    const uint32_t k = (uint32_t)(ctx->t_count % fdc_ctx::kTimeRing);
    if (!ctx->t_start[k]) {
        HIPCHK(hipEventCreate(&ctx->t_start[k]));
        HIPCHK(hipEventCreate(&ctx->t_end[k]));
    }
    HIPCHK(hipEventRecord(ctx->t_start[k], s));
    const int rc = enqueue_transport_kernel(ctx, a, flags, s, one_plan);
    if (rc) return rc;
    HIPCHK(hipEventRecord(ctx->t_end[k], s));
    ctx->t_count++;
    return FDC_OK;
}

// (queue: the persistent launch's counter; null = the context's, allocated on first use)
static int enqueue_transport_kernel(fdc_ctx *ctx, TransportArgs a, uint32_t flags, hipStream_t s, bool one_plan,
                                    unsigned long long *queue)
{
    const uint32_t wpb = ctx->cfg.waves_per_block;
    const bool variance = (flags & FDC_RUN_VARIANCE) != 0;
    if (ctx->cfg.tally_slots &&
        kLutSize * sizeof(float2) + kLdsFixedBytes + lds_tally_bytes(ctx->cfg.tally_slots, variance, ctx->cfg.tally_mode) >
            kMaxLdsBytes)
        return fail(ctx, FDC_E_ARG, "run: LDS sub-tally of %u slots with the squared-energy tally does not fit",
                    ctx->cfg.tally_slots);
    if (flags & FDC_RUN_COUNT_WORK) {
        // the counting kernel: global atomics, one wave per unit, whatever the configuration
        const unsigned long long g = (a.n_units + wpb - 1) / wpb;
        if (g > 0x7fffffffull) return fail(ctx, FDC_E_ARG, "run: too many work units for one launch");
        a.queue = nullptr;
        HIPCHK(launch_transport(a, wpb, (uint32_t)g, variance, false, s, true));
        return FDC_OK;
    }
    const bool persistent = ctx->cfg.tally_slots || ctx->cfg.blocks_per_cu;
    if (persistent) {
        if (!queue) {
            if (!ctx->d_queue) {
                ctx->d_queue = dalloc_n<unsigned long long>(ctx, 1);
                if (!ctx->d_queue) return fail(ctx, FDC_E_NOMEM, "run: queue allocation failed");
            }
            queue = ctx->d_queue;
        }
        HIPCHK(launch_fill_u64(queue, 1, 0, s));
        a.queue = queue;
    }
    if (ctx->cfg.tally_slots) {
        const uint32_t grid = std::max<uint32_t>(1, ctx->cfg.blocks_per_cu) * (uint32_t)ctx->cus;
        // the whole-launch cache (mode 2) needs a launch of one plan; otherwise the rounds cache
        const uint32_t mode = ctx->cfg.tally_mode == 2 && !one_plan ? 1u : ctx->cfg.tally_mode;
        HIPCHK(launch_transport_lds(a, wpb, grid, ctx->cfg.tally_slots, std::max<uint32_t>(1, ctx->cfg.units_per_wave),
                                    variance, mode, s));
    } else if (ctx->cfg.blocks_per_cu) {
        HIPCHK(launch_transport(a, wpb, ctx->cfg.blocks_per_cu * (uint32_t)ctx->cus, variance, false, s));
    } else {
        const unsigned long long g = (a.n_units + wpb - 1) / wpb;
        if (g > 0x7fffffffull) return fail(ctx, FDC_E_ARG, "run: too many work units for one launch");
        HIPCHK(launch_transport(a, wpb, (uint32_t)g, variance, false, s));
    }
    return FDC_OK;
}

int fdc_run_histories(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    int rc = validate_run(ctx, plans, n_plans, flags, 1);
    if (rc) return rc;
    if (ctx->dry) {
        account_run(ctx, plans, n_plans, flags, false);
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    rc = ensure_plans(ctx);
    if (!rc) rc = ensure_spots(ctx);
    if (!rc) rc = ensure_devices(ctx);
    if (rc) return rc;
    hipStream_t s = S(hip_stream);
    std::vector<WorkItem> items;
    uint32_t n_chunks = 0;
    const unsigned long long units = build_items(ctx, plans, n_plans, items, &n_chunks);
    if (items.empty()) return FDC_OK;
    if (ctx->cfg.source_order) {
        rc = check_source_order(ctx, items);
        if (rc) return rc;
        unsigned long long hw = 0;
        const bool large = large_items(items, &hw);
        if (!grow(ctx, ctx->d_order, ctx->order_cap, units * kWave, s) ||
            (large && !grow(ctx, ctx->d_hist, ctx->hist_cap, hw + 1, s)))
            return fail(ctx, FDC_E_NOMEM, "run: source order table");
    }
    rc = ensure_items(ctx, items.size(), s);
    if (rc) return rc;
    std::copy(items.begin(), items.end(), ctx->h_items);
    HIPCHK(hipMemcpyAsync(ctx->d_items, ctx->h_items, items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(ctx->items_ev, s));
    ctx->items_ev_pending = true;
    TransportArgs a = base_args(ctx);
    a.n_items = (uint32_t)items.size();
    a.n_units = units;
    a.flags = flags;
    if (ctx->cfg.source_order) {
        rc = enqueue_source_order(ctx, ctx->d_items, items, n_chunks, units, ctx->d_order, ctx->d_hist, s);
        if (rc) return rc;
        a.order = ctx->d_order;
    }
    rc = enqueue_transport(ctx, a, flags, s, one_plan(plans, n_plans), true);
    if (rc) return rc;
    HIPCHK(launch_advance(ctx->d_items, (uint32_t)items.size(), ctx->d_hnext, ctx->d_spots, ctx->d_plans, s));
    account_run(ctx, plans, n_plans, flags, false);
    return FDC_OK;
}

int fdc_run_histories_noalloc(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    int rc = validate_run(ctx, plans, n_plans, flags, 1);
    if (rc) return rc;
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "run (no allocation): context has no device");
    if (!ctx->scratch)
        return fail(ctx, FDC_E_HIP, "run (no allocation): scratch address: %s", hipGetErrorString(ctx->scratch_err));
    if (n_plans > kMaxRangePlans)
        return fail(ctx, FDC_E_RANGE, "run (no allocation): at most %u plans per run, %u given", kMaxRangePlans, n_plans);
    // the device plan and spot tables must be current: bringing them up to date may allocate
    if (ctx->plans_dirty || ctx->spots_dirty || ctx->devices_dirty)
        return fail(ctx, FDC_E_STATE, "run (no allocation): plans or spots changed since the last run; "
                    "call fdc_run_histories or fdc_prepare_run first");
    // sizes of the work table (as build_items, without building it on the host)
    unsigned long long n_items = 0, units = 0;
    for (uint32_t i = 0; i < n_plans; ++i)
        for (const fdc_spot &sp : ctx->plans[plans[i]].spots)
            if (sp.n_histories) {
                if (ctx->cfg.source_order && sp.n_histories >= 0xFFFFFFFFull)
                    return fail(ctx, FDC_E_ARG, "run: source_order needs fewer than 2^32 histories per spot");
                ++n_items;
                units += units_for(sp.n_histories);
            }
    if (n_items == 0) return FDC_OK;
    if (n_items > kNoAllocMaxItems)
        return fail(ctx, FDC_E_RANGE, "run (no allocation): %llu spots with histories, at most %u",
                    n_items, kNoAllocMaxItems);
    if (ctx->cfg.source_order && units > kNoAllocMaxOrderUnits)
        return fail(ctx, FDC_E_RANGE, "run (no allocation): start-position order of %llu wave units, the scratch "
                    "holds %llu (about %llu histories); use source_order 0 or fdc_run_histories", units,
                    kNoAllocMaxOrderUnits, kNoAllocMaxOrderUnits * 64);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = S(hip_stream);
    SpotRanges r{};
    r.n = n_plans;
    for (uint32_t i = 0; i < n_plans; ++i) {
        r.first[i] = ctx->spot_base[plans[i]];
        r.count[i] = (uint32_t)ctx->plans[plans[i]].spots.size();
    }
    unsigned long long *queue = (unsigned long long *)ctx->scratch;
    WorkItem *d_items = (WorkItem *)(ctx->scratch + kNoAllocItemsOff);
    uint32_t *d_order = (uint32_t *)(ctx->scratch + kNoAllocOrderOff);
    uint32_t *d_hist = (uint32_t *)(ctx->scratch + kNoAllocHistOff);
    HIPCHK(launch_build_items(ctx->d_spots, r, d_items, s));
    TransportArgs a = base_args(ctx);
    a.items = d_items;
    a.n_items = (uint32_t)n_items;
    a.n_units = units;
    a.flags = flags;
    if (ctx->cfg.source_order) {
        unsigned long long chunks = 0, hist = 0;
        bool large = false;
        for (uint32_t i = 0; i < n_plans; ++i)
            for (const fdc_spot &sp : ctx->plans[plans[i]].spots) {
                chunks += source_order_chunks(sp.n_histories);
                hist += sp.n_histories;
                large |= sp.n_histories > kOrderWholeSpot;
            }
        // (n histories <= 64 units: the histograms fit their region)
        const OrderTracks ot{ctx->bin_first, ctx->n_sec ? ctx->sec_first : nullptr, ctx->R};
        HIPCHK(launch_source_order(d_items, (uint32_t)n_items, (uint32_t)chunks, units, ctx->d_spots, ctx->d_hnext,
                                   (uint32_t)ctx->seed, (uint32_t)(ctx->seed >> 32), d_order, d_hist,
                                   order_hist_words(hist, n_items), large, ot, s));
        a.order = d_order;
    }
    rc = enqueue_transport_kernel(ctx, a, flags, s, one_plan(plans, n_plans), queue);
    if (rc) return rc;
    HIPCHK(launch_advance(d_items, (uint32_t)n_items, ctx->d_hnext, ctx->d_spots, ctx->d_plans, s));
    account_run(ctx, plans, n_plans, flags, false);
    return FDC_OK;
}

int fdc_prepare_run(fdc_ctx *ctx)
{
    if (!ctx) return FDC_E_ARG;
    if (ctx->dry) return FDC_OK;
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_plans(ctx);
    if (!rc) rc = ensure_spots(ctx);
    if (!rc) rc = ensure_devices(ctx);
    return rc;
}

int fdc_set_timing(fdc_ctx *ctx, int on)
{
    if (!ctx) return FDC_E_ARG;
    if (ctx->dry && on) return fail(ctx, FDC_E_STATE, "timing: context has no device");
    ctx->timing = on != 0;
    ctx->t_count = 0;
    return FDC_OK;
}

int fdc_transport_times(fdc_ctx *ctx, float *ms, uint32_t n)
{
    if (!ctx) return FDC_E_ARG;
    if (n && !ms) return fail(ctx, FDC_E_ARG, "timing: NULL output");
    const uint64_t have = std::min<uint64_t>(ctx->t_count, fdc_ctx::kTimeRing);
    if (n > have) return fail(ctx, FDC_E_STATE, "timing: %u runs asked, %llu timed and kept", n,
                             (unsigned long long)have);
    if (n == 0) return FDC_OK;
    HIPCHK(hipSetDevice(ctx->device));
    const uint32_t last = (uint32_t)((ctx->t_count - 1) % fdc_ctx::kTimeRing);
    HIPCHK(hipEventSynchronize(ctx->t_end[last]));
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t k = (uint32_t)((ctx->t_count - n + i) % fdc_ctx::kTimeRing);
        HIPCHK(hipEventElapsedTime(&ms[i], ctx->t_start[k], ctx->t_end[k]));
    }
    return FDC_OK;
}

int fdc_graph_create(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags, uint32_t options,
                     double *const *dose_dev, double *const *var_dev, fdc_graph **out)
{
    if (!ctx) return FDC_E_ARG;
    if (!out) return fail(ctx, FDC_E_ARG, "graph: NULL output");
    *out = nullptr;
    if (options & ~(uint32_t)(FDC_GRAPH_RESET_TALLIES | FDC_GRAPH_DOSE)) return fail(ctx, FDC_E_ARG, "graph: unknown option");
    if ((options & FDC_GRAPH_DOSE) && !dose_dev && !var_dev) return fail(ctx, FDC_E_ARG, "graph: dose option without outputs");
    if ((options & FDC_GRAPH_DOSE) && var_dev && !(flags & FDC_RUN_VARIANCE))
        return fail(ctx, FDC_E_ARG, "graph: variance output needs FDC_RUN_VARIANCE");
    if ((options & FDC_GRAPH_DOSE) && var_dev && !(options & FDC_GRAPH_RESET_TALLIES))
        for (uint32_t i = 0; i < n_plans; ++i)
            if (valid_plan(ctx, plans[i]) && !ctx->plans[plans[i]].var_complete)
                return fail(ctx, FDC_E_STATE, "graph: variance output but plan %d has runs without it", plans[i]);
    int rc = validate_run(ctx, plans, n_plans, flags, 1);
    if (rc) return rc;
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "graph: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    rc = ensure_plans(ctx);
    if (!rc) rc = ensure_spots(ctx);
    if (!rc) rc = ensure_devices(ctx);
    if (rc) return rc;
    std::vector<WorkItem> items;
    uint32_t n_chunks = 0;
    const unsigned long long units = build_items(ctx, plans, n_plans, items, &n_chunks);
    const bool ordered = ctx->cfg.source_order && !items.empty();
    if (ordered) {
        rc = check_source_order(ctx, items);
        if (rc) return rc;
    }
    fdc_graph *g = new (std::nothrow) fdc_graph();
    if (!g) return fail(ctx, FDC_E_NOMEM, "graph: host allocation failed");
    g->ctx = ctx;
    g->plans.assign(plans, plans + n_plans);
    g->flags = flags;
    g->reset = (options & FDC_GRAPH_RESET_TALLIES) != 0;
    g->d_items = dalloc_n<WorkItem>(ctx, std::max<size_t>(items.size(), 1));
    unsigned long long hw = 0;
    const bool large = ordered && large_items(items, &hw);
    if (ordered) g->d_order = dalloc_n<uint32_t>(ctx, units * kWave);
    if (large) g->d_hist = dalloc_n<uint32_t>(ctx, hw + 1);
    if (!g->d_items || (ordered && !g->d_order) || (large && !g->d_hist)) {
        dfree(ctx, g->d_items);
        dfree(ctx, g->d_order);
        dfree(ctx, g->d_hist);
        delete g;
        return fail(ctx, FDC_E_NOMEM, "graph: work table allocation failed");
    }
    auto cleanup = [&](int code, const char *what, hipError_t e) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        dfree(ctx, g->d_items);
        dfree(ctx, g->d_order);
        dfree(ctx, g->d_hist);
        delete g;
        return fail(ctx, code, "graph: %s: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipSuccess;
    if (!items.empty()) e = hipMemcpy(g->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(FDC_E_HIP, "work table upload", e);
    if (!ctx->cap_stream) {
        e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return cleanup(FDC_E_HIP, "stream", e);
    }
    if ((ctx->cfg.tally_slots || ctx->cfg.blocks_per_cu) && !ctx->d_queue) {
        ctx->d_queue = dalloc_n<unsigned long long>(ctx, 1);     // no allocation inside the capture
        if (!ctx->d_queue) return cleanup(FDC_E_NOMEM, "queue allocation", hipErrorOutOfMemory);
    }
    hipStream_t s = ctx->cap_stream;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return cleanup(FDC_E_HIP, "begin capture", e);
    rc = FDC_OK;
    for (uint32_t i = 0; i < n_plans && g->reset && e == hipSuccess; ++i) {
        PlanHost &P = ctx->plans[plans[i]];
        e = launch_fill_u64(P.E, P.nvox, 0, s);
        if (e == hipSuccess) e = launch_fill_u64(P.E2, P.nvox, 0, s);
        if (e == hipSuccess) e = launch_fill_u64(P.acc, 8, 0, s);
    }
    if (e == hipSuccess && !items.empty()) {
        TransportArgs a = base_args(ctx);
        a.items = g->d_items;
        a.n_items = (uint32_t)items.size();
        a.n_units = units;
        a.flags = flags;
        if (ordered) {
            rc = enqueue_source_order(ctx, g->d_items, items, n_chunks, units, g->d_order, g->d_hist, s);
            a.order = g->d_order;
        }
        if (!rc) rc = enqueue_transport(ctx, a, flags, s, one_plan(plans, n_plans));
        if (!rc) e = launch_advance(g->d_items, (uint32_t)items.size(), ctx->d_hnext, ctx->d_spots, ctx->d_plans, s);
    }
    for (uint32_t i = 0; i < n_plans && (options & FDC_GRAPH_DOSE) && e == hipSuccess && !rc; ++i) {
        PlanHost &P = ctx->plans[plans[i]];
        const double vol = (double)P.vox[0] * (double)P.vox[1] * (double)P.vox[2];
        e = launch_dose(P.idx, P.E, P.E2, ctx->lut, ctx->rho_lut, P.nvox, vol, P.acc + 3,
                        dose_dev ? dose_dev[i] : nullptr, var_dev ? var_dev[i] : nullptr, s);
    }
    hipError_t e2 = hipStreamEndCapture(s, &g->graph);
    if (rc) { std::string m = ctx->err; cleanup(rc, "capture", hipSuccess); ctx->err = m; return rc; }
    if (e != hipSuccess) return cleanup(FDC_E_HIP, "captured launch", e);
    if (e2 != hipSuccess) return cleanup(FDC_E_HIP, "end capture", e2);
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return cleanup(FDC_E_HIP, "instantiate", e);
    g->gen = ctx->gen;
    *out = g;
    return FDC_OK;
}

int fdc_graph_launch(fdc_graph *g, void *hip_stream)
{
    if (!g) return FDC_E_ARG;
    fdc_ctx *ctx = g->ctx;
    if (g->gen != ctx->gen || ctx->spots_dirty || ctx->plans_dirty || ctx->devices_dirty)
        return fail(ctx, FDC_E_STATE, "graph: plans, spots or database changed since capture; capture again");
    int rc = validate_run(ctx, g->plans.data(), (uint32_t)g->plans.size(), g->flags, 1);
    if (rc && !(rc == FDC_E_OVERFLOW && g->reset)) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipGraphLaunch(g->exec, S(hip_stream)));
    account_run(ctx, g->plans.data(), (uint32_t)g->plans.size(), g->flags, g->reset);
    return FDC_OK;
}

int fdc_graph_destroy(fdc_graph *g)
{
    if (!g) return FDC_E_ARG;
    fdc_ctx *ctx = g->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    dfree(ctx, g->d_items);
    dfree(ctx, g->d_order);
    dfree(ctx, g->d_hist);
    delete g;
    return FDC_OK;
}

// A plan's saved state: this header, then acc[8] (u64), the next-history
// counter of each source (u64), E and E2 (u64 per voxel).
namespace {
struct PlanStateHeader {
    char magic[8];                   // "FDCSTATE"
    uint32_t version;                // 1
    uint32_t var_complete;           // every history so far tallied its squares
    uint64_t nvox, n_sources, n_hist, reserved;
};
static_assert(sizeof(PlanStateHeader) == 48, "plan state header layout");

uint64_t plan_state_bytes(const PlanHost &P)
{
    return sizeof(PlanStateHeader) + 8 * 8 + 8 * (uint64_t)P.spots.size() + 16 * (uint64_t)P.nvox;
}
} // namespace

int fdc_plan_state_bytes(fdc_ctx *ctx, int32_t plan, uint64_t *bytes)
{
    if (!ctx || !bytes) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "state: no plan %d", plan);
    *bytes = plan_state_bytes(ctx->plans[plan]);
    return FDC_OK;
}

int fdc_save_plan_state(fdc_ctx *ctx, int32_t plan, void *buf, uint64_t bytes, void *hip_stream)
{
    if (!ctx || !buf) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "state: no plan %d", plan);
    PlanHost &P = ctx->plans[plan];
    if (bytes != plan_state_bytes(P))
        return fail(ctx, FDC_E_ARG, "state: buffer of %llu bytes, the plan's state takes %llu",
                    (unsigned long long)bytes, (unsigned long long)plan_state_bytes(P));
    unsigned char *o = (unsigned char *)buf;
    PlanStateHeader h{};
    std::memcpy(h.magic, "FDCSTATE", 8);
    h.version = 1;
    h.var_complete = P.var_complete ? 1u : 0u;
    h.nvox = P.nvox;
    h.n_sources = P.spots.size();
    h.n_hist = P.n_hist;
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    unsigned char *acc = o;
    o += 64;
    std::memcpy(o, P.h_next.data(), 8 * P.h_next.size());
    o += 8 * P.h_next.size();
    if (ctx->dry) {                           // no tallies without a device
        std::memset(acc, 0, 64);
        std::memset(o, 0, 16 * P.nvox);
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = S(hip_stream);
    HIPCHK(hipMemcpyAsync(acc, P.acc, 64, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(o, P.E, 8 * P.nvox, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(o + 8 * P.nvox, P.E2, 8 * P.nvox, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return FDC_OK;
}

int fdc_restore_plan_state(fdc_ctx *ctx, int32_t plan, const void *buf, uint64_t bytes, void *hip_stream)
{
    if (!ctx || !buf) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "state: no plan %d", plan);
    PlanHost &P = ctx->plans[plan];
    PlanStateHeader h;
    if (bytes < sizeof h) return fail(ctx, FDC_E_FORMAT, "state: short buffer");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, "FDCSTATE", 8) != 0 || h.version != 1)
        return fail(ctx, FDC_E_FORMAT, "state: bad magic or version");
    if (h.nvox != P.nvox || h.n_sources != P.spots.size())
        return fail(ctx, FDC_E_FORMAT, "state: saved for %llu voxels and %llu sources, the plan has %llu and %llu",
                    (unsigned long long)h.nvox, (unsigned long long)h.n_sources, (unsigned long long)P.nvox,
                    (unsigned long long)P.spots.size());
    if (bytes != plan_state_bytes(P)) return fail(ctx, FDC_E_FORMAT, "state: size does not match its header");
    const unsigned char *in = (const unsigned char *)buf + sizeof h;
    const unsigned char *acc = in;
    in += 64;
    std::vector<uint64_t> hn(P.spots.size());
    std::memcpy(hn.data(), in, 8 * hn.size());
    in += 8 * hn.size();
    if (!ctx->dry) {
        HIPCHK(hipSetDevice(ctx->device));
        hipStream_t s = S(hip_stream);
        HIPCHK(hipMemcpyAsync(P.acc, acc, 64, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P.E, in, 8 * P.nvox, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P.E2, in + 8 * P.nvox, 8 * P.nvox, hipMemcpyHostToDevice, s));
        if (!ctx->spots_dirty && !hn.empty())
            HIPCHK(hipMemcpyAsync(ctx->d_hnext + ctx->spot_base[plan], hn.data(), 8 * hn.size(),
                                  hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    P.h_next = hn;
    P.n_hist = h.n_hist;
    P.var_complete = h.var_complete != 0;
    return FDC_OK;
}

int fdc_read_work_counts(fdc_ctx *ctx, int32_t plan, uint64_t counts[3], void *hip_stream)
{
    if (!ctx || !counts) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "work counts: no plan %d", plan);
    if (ctx->dry) {
        counts[0] = counts[1] = counts[2] = 0;
        return FDC_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = S(hip_stream);
    HIPCHK(hipMemcpyAsync(counts, ctx->plans[plan].acc + 4, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return FDC_OK;
}

int fdc_reset_plan(fdc_ctx *ctx, int32_t plan, int rewind, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "reset: no plan %d", plan);
    PlanHost &P = ctx->plans[plan];
    if (!ctx->dry) {
        HIPCHK(hipSetDevice(ctx->device));
        hipStream_t s = S(hip_stream);
        HIPCHK(launch_fill_u64(P.E, P.nvox, 0, s));
        HIPCHK(launch_fill_u64(P.E2, P.nvox, 0, s));
        HIPCHK(launch_fill_u64(P.acc, 8, 0, s));
        if (rewind && !ctx->spots_dirty && !P.spots.empty())
            HIPCHK(launch_fill_u64(ctx->d_hnext + ctx->spot_base[plan], P.spots.size(), 0, s));
    }
    P.n_hist = 0;
    P.var_complete = true;
    if (rewind) std::fill(P.h_next.begin(), P.h_next.end(), 0);
    return FDC_OK;
}

int fdc_compute_dose(fdc_ctx *ctx, int32_t plan, double *dose_dev, double *var_dev, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "dose: no plan %d", plan);
    const PlanHost &P = ctx->plans[plan];
    if (P.n_hist == 0) return fail(ctx, FDC_E_STATE, "dose: no histories run on plan %d", plan);
    if (var_dev && !P.var_complete)
        return fail(ctx, FDC_E_STATE, "dose: variance asked but a run without FDC_RUN_VARIANCE touched plan %d", plan);
    if (!dose_dev && !var_dev) return FDC_OK;
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "dose: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    const double vol = (double)P.vox[0] * (double)P.vox[1] * (double)P.vox[2];
    HIPCHK(launch_dose(P.idx, P.E, P.E2, ctx->lut, ctx->rho_lut, P.nvox, vol, P.acc + 3, dose_dev, var_dev,
                       S(hip_stream)));
    return FDC_OK;
}

int fdc_read_dose_and_variance(fdc_ctx *ctx, int32_t plan, double *dose, double *var, int64_t *raw_E,
                               uint64_t *raw_E2, fdc_summary *sum, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "read: no plan %d", plan);
    PlanHost &P = ctx->plans[plan];
    if ((dose || var) && P.n_hist == 0) return fail(ctx, FDC_E_STATE, "read: no histories run on plan %d", plan);
    if (var && !P.var_complete)
        return fail(ctx, FDC_E_STATE, "read: variance asked but a run without FDC_RUN_VARIANCE touched plan %d", plan);
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "read: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = S(hip_stream);
    if (dose || var) {
        if (P.nvox > ctx->dose_cap) {
            double *d1 = dalloc_n<double>(ctx, P.nvox), *d2 = dalloc_n<double>(ctx, P.nvox);
            if (!d1 || !d2) { dfree(ctx, d1); dfree(ctx, d2); return fail(ctx, FDC_E_NOMEM, "read: scratch allocation failed"); }
            HIPCHK(hipStreamSynchronize(s));
            dfree(ctx, ctx->d_dose); dfree(ctx, ctx->d_var);
            ctx->d_dose = d1; ctx->d_var = d2; ctx->dose_cap = P.nvox;
        }
        int rc = fdc_compute_dose(ctx, plan, dose ? ctx->d_dose : nullptr, var ? ctx->d_var : nullptr, hip_stream);
        if (rc) return rc;
        if (dose) HIPCHK(hipMemcpyAsync(dose, ctx->d_dose, P.nvox * 8, hipMemcpyDeviceToHost, s));
        if (var) HIPCHK(hipMemcpyAsync(var, ctx->d_var, P.nvox * 8, hipMemcpyDeviceToHost, s));
    }
    if (raw_E) HIPCHK(hipMemcpyAsync(raw_E, P.E, P.nvox * 8, hipMemcpyDeviceToHost, s));
    if (raw_E2) HIPCHK(hipMemcpyAsync(raw_E2, P.E2, P.nvox * 8, hipMemcpyDeviceToHost, s));
    unsigned long long acc[4] = {0, 0, 0, 0};
    if (sum) {
        HIPCHK(launch_fill_u64(P.acc + 2, 1, 0, s));
        HIPCHK(launch_sum_i64(P.E, P.nvox, P.acc + 2, s));
        HIPCHK(hipMemcpyAsync(acc, P.acc, 32, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (sum) {
        sum->n_histories = acc[3];
        sum->incident_fp = (int64_t)acc[0];
        sum->escaped_fp = (int64_t)acc[1];
        sum->deposited_fp = (int64_t)acc[2];
    }
    return FDC_OK;
}

int fdc_debug_endpoints(fdc_ctx *ctx, int32_t plan, uint32_t spot, uint64_t h0, uint32_t n, uint32_t flags,
                        float *xyz_out, int32_t *reason_out, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "endpoints: no plan %d", plan);
    if (spot >= ctx->plans[plan].spots.size()) return fail(ctx, FDC_E_ARG, "endpoints: no spot %u", spot);
    if (n == 0) return FDC_OK;
    if (!xyz_out || !reason_out) return fail(ctx, FDC_E_ARG, "endpoints: NULL output");
    if (flags & ~(uint32_t)(FDC_RUN_VARIANCE | FDC_RUN_ROTATE_TRACKS)) return fail(ctx, FDC_E_ARG, "endpoints: unknown flag");
    if (ctx->n_bins == 0) return fail(ctx, FDC_E_STATE, "endpoints: no track database loaded");
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "endpoints: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_plans(ctx);
    if (!rc) rc = ensure_spots(ctx);
    if (!rc) rc = ensure_devices(ctx);
    if (rc) return rc;
    hipStream_t s = S(hip_stream);
    float *d_xyz = dalloc_n<float>(ctx, 3 * (size_t)n);
    int *d_reason = dalloc_n<int>(ctx, n);
    WorkItem *d_item = dalloc_n<WorkItem>(ctx, 1);
    if (!d_xyz || !d_reason || !d_item) {
        dfree(ctx, d_xyz); dfree(ctx, d_reason); dfree(ctx, d_item);
        return fail(ctx, FDC_E_NOMEM, "endpoints: allocation failed");
    }
    WorkItem w{};
    w.h0 = h0;
    w.n = n;
    w.gspot = ctx->spot_base[plan] + spot;
    const unsigned long long units = units_for(n);
    TransportArgs a = base_args(ctx);
    a.items = d_item;
    a.hnext = nullptr;                       // h0 is absolute here
    a.n_items = 1;
    a.n_units = units;
    a.flags = flags;
    a.ep_xyz = d_xyz;
    a.ep_reason = d_reason;
    hipError_t e = hipMemcpyAsync(d_item, &w, sizeof w, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_transport(a, 4, (uint32_t)((units + 3) / 4), false, true, s);
    if (e == hipSuccess) e = hipMemcpyAsync(xyz_out, d_xyz, 12 * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(reason_out, d_reason, 4 * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(ctx, d_xyz); dfree(ctx, d_reason); dfree(ctx, d_item);
    if (e != hipSuccess) return fail(ctx, FDC_E_HIP, "endpoints: %s", hipGetErrorString(e));
    return FDC_OK;
}

int fdc_debug_philox(fdc_ctx *ctx, const uint32_t *ctr, uint32_t *out, uint32_t n, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (n == 0) return FDC_OK;
    if (!ctr || !out) return fail(ctx, FDC_E_ARG, "philox: NULL array");
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "philox: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = S(hip_stream);
    uint4 *d_c = dalloc_n<uint4>(ctx, n), *d_o = dalloc_n<uint4>(ctx, n);
    if (!d_c || !d_o) { dfree(ctx, d_c); dfree(ctx, d_o); return fail(ctx, FDC_E_NOMEM, "philox: allocation failed"); }
    hipError_t e = hipMemcpyAsync(d_c, ctr, 16 * (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_philox_test(d_c, d_o, n, (uint32_t)ctx->seed, (uint32_t)(ctx->seed >> 32), s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_o, 16 * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(ctx, d_c); dfree(ctx, d_o);
    if (e != hipSuccess) return fail(ctx, FDC_E_HIP, "philox: %s", hipGetErrorString(e));
    return FDC_OK;
}

int fdc_debug_material(fdc_ctx *ctx, float *rsp_out, float *g_out, float *rho_out, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!rsp_out || !g_out || !rho_out) return fail(ctx, FDC_E_ARG, "material: NULL output");
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "material: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_table(ctx);
    if (rc) return rc;
    std::vector<float2> l(kLutSize);
    hipStream_t s = S(hip_stream);
    HIPCHK(hipMemcpyAsync(l.data(), ctx->lut, sizeof(float2) * kLutSize, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rho_out, ctx->rho_lut, sizeof(float) * kLutSize, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < kLutSize; ++i) { rsp_out[i] = l[i].x; g_out[i] = l[i].y; }
    return FDC_OK;
}

int fdc_set_launch_config(fdc_ctx *ctx, const fdc_launch_config *cfg)
{
    if (!ctx) return FDC_E_ARG;
    if (!cfg) return fail(ctx, FDC_E_ARG, "launch config: NULL");
    if (cfg->waves_per_block < 1 || cfg->waves_per_block > 16)
        return fail(ctx, FDC_E_ARG, "launch config: waves_per_block must be 1..16");
    if (cfg->blocks_per_cu > 64) return fail(ctx, FDC_E_ARG, "launch config: blocks_per_cu must be 0..64");
    if (cfg->tally_mode > 2) return fail(ctx, FDC_E_ARG, "launch config: tally_mode must be 0, 1 or 2");
    if (cfg->tally_slots) {
        const uint32_t t = cfg->tally_slots;
        if (cfg->tally_mode == 0 && (t < 256 || t > 8192 || (t & (t - 1))))
            return fail(ctx, FDC_E_ARG, "launch config: tally_slots must be 0 or a power of two 256..8192");
        if (cfg->tally_mode >= 1 && (t < 256 || t % 64))
            return fail(ctx, FDC_E_ARG, "launch config: tally_slots must be 0 or a multiple of 64 from 256");
        if (kLutSize * sizeof(float2) + kLdsFixedBytes + lds_tally_bytes(t, false, cfg->tally_mode) > kMaxLdsBytes)
            return fail(ctx, FDC_E_ARG, "launch config: LDS sub-tally of %u slots does not fit", t);
    }
    if (cfg->units_per_wave > 64) return fail(ctx, FDC_E_ARG, "launch config: units_per_wave must be 0..64");
    if (cfg->tally_slots && cfg->tally_mode == 2 && !ctx->dry) {
        // the whole-launch cache kernel's waves wait for a sibling wave of their
        // workgroup: the workgroup must fit one CU (then its waves are resident together)
        HIPCHK(hipSetDevice(ctx->device));
        for (int var = 0; var < 2; ++var) {
            if (kLutSize * sizeof(float2) + kLdsFixedBytes + lds_tally_bytes(cfg->tally_slots, var, 2) > kMaxLdsBytes)
                continue;                        // (refused at run time for the squared-energy tally)
            int blocks = 0;
            HIPCHK(cache_kernel_occupancy(std::max<uint32_t>(1, cfg->waves_per_block), cfg->tally_slots, var != 0,
                                          &blocks));
            if (blocks < 1)
                return fail(ctx, FDC_E_ARG, "launch config: a workgroup of the whole-launch cache kernel does not fit "
                            "one CU");
        }
    }
    if (cfg->source_order > 1) return fail(ctx, FDC_E_ARG, "launch config: source_order must be 0 or 1");
    ctx->cfg = *cfg;
    return FDC_OK;
}

int fdc_mean_uncertainty(fdc_ctx *ctx, int32_t plan, const double *dose_dev, const double *var_dev, double frac,
                         double *mean_out, uint64_t *n_out, double *dmax_out, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "mean uncertainty: no plan %d", plan);
    if (!dose_dev || !var_dev || !mean_out) return fail(ctx, FDC_E_ARG, "mean uncertainty: NULL argument");
    if (!(frac >= 0.0 && frac < 1.0)) return fail(ctx, FDC_E_ARG, "mean uncertainty: frac must be in [0, 1)");
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "mean uncertainty: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    const PlanHost &P = ctx->plans[plan];
    hipStream_t s = S(hip_stream);
    double *scr = dalloc_n<double>(ctx, metrics_scratch_doubles());
    if (!scr) return fail(ctx, FDC_E_NOMEM, "mean uncertainty: scratch allocation failed");
    double out[3] = {0, 0, 0};
    double *d_out = scr + metrics_scratch_doubles() - 4;
    hipError_t e = launch_mean_uncertainty(dose_dev, var_dev, P.idx, ctx->lut, P.nvox, frac, scr, d_out, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, sizeof out, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(ctx, scr);
    if (e != hipSuccess) return fail(ctx, FDC_E_HIP, "mean uncertainty: %s", hipGetErrorString(e));
    *mean_out = out[2] > 0 ? out[1] / out[2] : 0.0;
    if (n_out) *n_out = (uint64_t)out[2];
    if (dmax_out) *dmax_out = out[0];
    return FDC_OK;
}

int fdc_batch_uncertainty(fdc_ctx *ctx, const double *doses_dev, uint32_t n_batches, uint64_t n_vox,
                          double *mean_dev, double *sigma_dev, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!doses_dev || (!mean_dev && !sigma_dev)) return fail(ctx, FDC_E_ARG, "batch uncertainty: NULL argument");
    if (n_batches < 2 || n_vox == 0) return fail(ctx, FDC_E_ARG, "batch uncertainty: need n_batches >= 2 and voxels");
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "batch uncertainty: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(launch_batch_uncertainty(doses_dev, n_batches, n_vox, mean_dev, sigma_dev, S(hip_stream)));
    return FDC_OK;
}

int fdc_gamma_index(fdc_ctx *ctx, int32_t plan, const double *ref_dev, const double *eval_dev, double dose_frac,
                    double dta_cm, double cutoff_frac, double search_cm, float *gamma_dev, double *pass_rate_out,
                    uint64_t *n_eval_out, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "gamma: no plan %d", plan);
    if (!ref_dev || !eval_dev) return fail(ctx, FDC_E_ARG, "gamma: NULL dose array");
    if (!(dose_frac > 0.0) || !(dta_cm > 0.0) || !(cutoff_frac >= 0.0) || !(search_cm >= dta_cm) ||
        !std::isfinite(search_cm))
        return fail(ctx, FDC_E_ARG, "gamma: need dose_frac > 0, dta > 0, cutoff >= 0, search >= dta");
    const PlanHost &P = ctx->plans[plan];
    // candidate offsets on the twice-upsampled grid, sorted by distance
    std::vector<int4> offs;
    std::vector<double> d2;
    int r[3];
    for (int q = 0; q < 3; ++q) r[q] = (int)std::floor(search_cm / (0.5 * P.vox[q]) + 1e-9);
    if ((double)(2 * r[0] + 1) * (2 * r[1] + 1) * (2 * r[2] + 1) > 4e6)
        return fail(ctx, FDC_E_ARG, "gamma: search radius too large for the voxel size");
    std::vector<std::pair<double, int4>> cand;
    for (int c = -r[2]; c <= r[2]; ++c)
        for (int b = -r[1]; b <= r[1]; ++b)
            for (int a = -r[0]; a <= r[0]; ++a) {
                const double dx = a * 0.5 * P.vox[0], dy = b * 0.5 * P.vox[1], dz = c * 0.5 * P.vox[2];
                const double dist2 = dx * dx + dy * dy + dz * dz;
                if (dist2 <= search_cm * search_cm * (1.0 + 1e-12)) cand.push_back({dist2 / (dta_cm * dta_cm), int4{a, b, c, 0}});
            }
    std::stable_sort(cand.begin(), cand.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    for (auto &p : cand) { d2.push_back(p.first); offs.push_back(p.second); }
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "gamma: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = S(hip_stream);
    const size_t ns = metrics_scratch_doubles();
    // scratch: reduction area (ns doubles), squared distances (n doubles),
    // offsets (n int4 = 2n doubles), two counters
    const size_t no = offs.size();
    double *scr = dalloc_n<double>(ctx, ns + 3 * no + 4);
    if (!scr) return fail(ctx, FDC_E_NOMEM, "gamma: scratch allocation failed");
    double *d_out = scr + ns - 4;
    double *d_d2 = scr + ns;
    int4 *d_offs = (int4 *)(scr + ns + no);
    unsigned long long *d_cnt = (unsigned long long *)(scr + ns + 3 * no);
    unsigned long long cnt[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(d_d2, d2.data(), d2.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_offs, offs.data(), offs.size() * 16, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(d_cnt, 0, 16, s);
    if (e == hipSuccess) e = launch_dmax(ref_dev, P.idx, ctx->lut, P.nvox, scr, d_out, s);
    if (e == hipSuccess)
        e = launch_gamma(ref_dev, eval_dev, P.idx, ctx->lut, P.n[0], P.n[1], P.n[2], d_offs, d_d2, (int)offs.size(),
                         d_out, dose_frac, cutoff_frac, gamma_dev, d_cnt, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, d_cnt, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(ctx, scr);
    if (e != hipSuccess) return fail(ctx, FDC_E_HIP, "gamma: %s", hipGetErrorString(e));
    if (pass_rate_out) *pass_rate_out = cnt[0] ? (double)cnt[1] / (double)cnt[0] : 0.0;
    if (n_eval_out) *n_eval_out = cnt[0];
    return FDC_OK;
}

int fdc_density(fdc_ctx *ctx, int32_t plan, float *rho_dev, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "density: no plan %d", plan);
    if (!rho_dev) return fail(ctx, FDC_E_ARG, "density: NULL output");
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "density: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    const PlanHost &P = ctx->plans[plan];
    HIPCHK(launch_density(P.idx, ctx->rho_lut, P.nvox, rho_dev, S(hip_stream)));
    return FDC_OK;
}

int fdc_denoise_input(fdc_ctx *ctx, int32_t plan, const double *dose_dev, const float *rho_dev, double scale,
                      float *out_dev, void *hip_stream)
{
    if (!ctx) return FDC_E_ARG;
    if (!valid_plan(ctx, plan)) return fail(ctx, FDC_E_ARG, "denoise input: no plan %d", plan);
    if (!dose_dev || !rho_dev || !out_dev || !std::isfinite(scale))
        return fail(ctx, FDC_E_ARG, "denoise input: NULL argument or bad scale");
    if (ctx->dry) return fail(ctx, FDC_E_STATE, "denoise input: context has no device");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(launch_denoise_input(dose_dev, rho_dev, ctx->plans[plan].nvox, scale, out_dev, S(hip_stream)));
    return FDC_OK;
}

int fdc_device_cus(fdc_ctx *ctx, int *cus)
{
    if (!ctx || !cus) return FDC_E_ARG;
    *cus = ctx->cus;
    return FDC_OK;
}

} // extern "C"
