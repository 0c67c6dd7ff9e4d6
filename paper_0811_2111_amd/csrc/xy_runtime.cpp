// xy_runtime.cpp -- host runtime behind the C ABI in include/xy.h: argument
// validation, workspace carve-up, schedule (plan) choice, launch sequencing,
// error mapping and the plan autotuner.  Batches live in xy_batch.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "xy.h"
#include "xy_launch.hpp"
#include "xy_runtime.hpp"

namespace xyr {

thread_local char g_hip_err[256] = "";
// Launch points left before the injected failure (-1: none armed), and whether the
// last failure on this thread was injected.
static std::atomic<int> g_inject_countdown{-1};
thread_local bool g_injected = false;

bool inject_due()
{
    int v = g_inject_countdown.load(std::memory_order_relaxed);
    while (v >= 0) {
        if (g_inject_countdown.compare_exchange_weak(v, v - 1, std::memory_order_relaxed)) {
            if (v == 0) g_injected = true;
            return v == 0;
        }
    }
    return false;
}

int hip_fail(hipError_t e, const char* what)
{
    snprintf(g_hip_err, sizeof(g_hip_err), "%s: %s (%d)%s", what, hipGetErrorString(e), (int)e,
             g_injected ? " [injected]" : "");
    g_injected = false;
    return XY_EHIP;
}

bool valid_L(int32_t L) { return L >= 4 && (L % 2) == 0 && (int64_t)L * (int64_t)L < (1LL << 31); }

bool valid_beta_delta(double beta, double delta)
{
    return std::isfinite(beta) && beta >= 0.0 && std::isfinite(delta) && delta > 0.0 && delta <= M_PI;
}

xyk::SweepArgs sweep_args(uint64_t seed, int L, int precision, double beta, double delta)
{
    xyk::SweepArgs a;
    a.src = a.dst = nullptr;
    a.L = L;
    a.precision = precision;
    a.key0 = (uint32_t)(seed & 0xffffffffu);
    a.key1 = (uint32_t)(seed >> 32);
    a.sweep = 0;
    a.delta = (float)(delta / (2.0 * M_PI));   // radians -> turns, rounded once to FP32
    a.nbl2e = (float)(-beta * 1.4426950408889634073599246810018921);
    return a;
}

xy_plan default_plan(int32_t L, int32_t precision)
{
    // A lattice whose state and ping-pong copy exceed the 256 MiB MALL is read
    // from HBM every sweep; there the strip segments are the fastest plan (over
    // the 256 x 16 tiles, FP32: 2% at L = 8192, 17% at L = 16384 with a record
    // every sweep; FP16: 10% at L = 16384, while at L = 8192, whose two FP16
    // buffers just fit the MALL, the tiles are 4% ahead).
    const uint64_t elem = precision == XY_FP16 ? 2ull : 4ull;
    if (2ull * (uint64_t)L * (uint64_t)L * elem > (256ull << 20) && xyk::strip_supported(L, 512, 64))
        return xy_plan{XY_PLAN_STRIP, 512, 64, 1};
    xy_plan p{XY_PLAN_STREAM, 0, 0, 1};
    static const int cand[][3] = {{256, 16, 1}, {128, 32, 1}, {64, 32, 1}, {64, 16, 1}};
    for (auto& c : cand)
        if (xyk::fused_supported(L, c[0], c[1], c[2])) {
            p.kind = XY_PLAN_FUSED;
            p.tile_x = c[0];
            p.tile_y = c[1];
            p.sweeps_per_pass = c[2];
            return p;
        }
    return p;
}

bool plan_ok(int32_t L, const xy_plan& p)
{
    if (p.kind == XY_PLAN_STREAM) return true;
    if (p.kind == XY_PLAN_FUSED) return xyk::fused_supported(L, p.tile_x, p.tile_y, p.sweeps_per_pass);
    if (p.kind == XY_PLAN_STRIP) return p.sweeps_per_pass == 1 && xyk::strip_supported(L, p.tile_x, p.tile_y);
    if (p.kind == XY_PLAN_RESIDENT) return xyk::resident_supported(L);
    return false;
}

// ---------------------------------------------------------- tune cache (JSON)
// One object, one entry per line:
//   "gfx950/L/precision": {"kind": K, "tile_x": X, "tile_y": Y, "sweeps_per_pass": M, "gupd_s": G},
static std::string cache_key(int32_t L, int32_t precision)
{
    char b[64];
    snprintf(b, sizeof(b), "gfx950/%d/%d", (int)L, (int)precision);
    return b;
}

static bool parse_int_field(const std::string& line, const char* name, int* out)
{
    std::string pat = std::string("\"") + name + "\":";
    size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    *out = atoi(line.c_str() + p + pat.size());
    return true;
}

static std::vector<std::string> read_lines(const char* path)
{
    std::vector<std::string> lines;
    FILE* f = fopen(path, "r");
    if (!f) return lines;
    char buf[1024];
    while (fgets(buf, sizeof(buf), f)) lines.emplace_back(buf);
    fclose(f);
    return lines;
}

bool cache_lookup(const char* path, int32_t L, int32_t precision, xy_plan* plan)
{
    if (!path) return false;
    const std::string key = "\"" + cache_key(L, precision) + "\"";
    for (const std::string& line : read_lines(path)) {
        if (line.find(key) == std::string::npos) continue;
        xy_plan p{0, 0, 0, 1};
        if (!parse_int_field(line, "kind", &p.kind)) return false;
        parse_int_field(line, "tile_x", &p.tile_x);
        parse_int_field(line, "tile_y", &p.tile_y);
        parse_int_field(line, "sweeps_per_pass", &p.sweeps_per_pass);
        if (!plan_ok(L, p)) return false;
        *plan = p;
        return true;
    }
    return false;
}

bool cache_store(const char* path, int32_t L, int32_t precision, const xy_plan& p, double gupd)
{
    const std::string key = "\"" + cache_key(L, precision) + "\"";
    std::vector<std::string> entries;
    for (const std::string& line : read_lines(path)) {
        if (line.find("\"gfx950/") == std::string::npos || line.find(key) != std::string::npos) continue;
        std::string e = line;
        while (!e.empty() && (e.back() == '\n' || e.back() == ',' || e.back() == ' ')) e.pop_back();
        entries.push_back(e);
    }
    char b[256];
    snprintf(b, sizeof(b),
             "  %s: {\"kind\": %d, \"tile_x\": %d, \"tile_y\": %d, \"sweeps_per_pass\": %d, \"gupd_s\": %.3f}",
             key.c_str(), (int)p.kind, (int)p.tile_x, (int)p.tile_y, (int)p.sweeps_per_pass, gupd);
    entries.emplace_back(b);
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fputs("{\n", f);
    for (size_t i = 0; i < entries.size(); ++i) fprintf(f, "%s%s\n", entries[i].c_str(), i + 1 < entries.size() ? "," : "");
    fputs("}\n", f);
    fclose(f);
    return rename(tmp.c_str(), path) == 0;
}

const char* env_cache_path() { return getenv("XY_TUNE_CACHE"); }

}  // namespace xyr

using namespace xyr;

static const uint32_t kMagic = 0x58594c54u;  // "XYLT"

struct xy_lattice {
    uint32_t magic;
    uint64_t seed;
    int32_t L;
    int32_t precision;
    double beta, delta;
    void* state;
    size_t state_len;
    void* work;
    size_t work_len;
    hipStream_t stream;
    uint64_t sweep;
    xy_plan plan;
    xyk::Work w;
    int32_t hmc_steps;     // leap-frog steps per pass of xy_hmc (1 .. 8)
    // kernel timer (xy_kernel_timer): event pairs around the sweep kernel launches
    hipEvent_t* tev;       // 2 * tcap events, or nullptr
    int32_t tcap, tn;
};

static bool live(const xy_lattice* h) { return h && h->magic == kMagic; }

static xyk::SweepArgs args_of(const xy_lattice* h)
{
    xyk::SweepArgs a = sweep_args(h->seed, h->L, h->precision, h->beta, h->delta);
    a.src = a.dst = h->state;
    a.sweep = (uint32_t)h->sweep;
    return a;
}

extern "C" {

int xy_state_bytes(int32_t L, int32_t precision, size_t* state, size_t* workspace)
{
    if (!valid_L(L) || (precision != XY_FP32 && precision != XY_FP16)) return XY_EINVAL;
    if (state) *state = xyk::state_bytes(L, precision);
    if (workspace) *workspace = xyk::work_bytes(L, precision);
    return XY_OK;
}

static int make_handle(xy_lattice** out, uint64_t seed, int32_t L, double beta, double delta, int32_t precision,
                       void* state_dev, size_t state_len, void* work_dev, size_t work_len, void* hip_stream)
{
    if (!out) return XY_ESTATE;
    *out = nullptr;
    if (!valid_L(L) || !valid_beta_delta(beta, delta) || (precision != XY_FP32 && precision != XY_FP16))
        return XY_EINVAL;
    if (!state_dev || !work_dev) return XY_ESTATE;
    if (state_len < xyk::state_bytes(L, precision) || work_len < xyk::work_bytes(L, precision)) return XY_ESIZE;
    xy_lattice* h = new (std::nothrow) xy_lattice;
    if (!h) return XY_ENOMEM;
    h->magic = kMagic;
    h->seed = seed;
    h->L = L;
    h->precision = precision;
    h->beta = beta;
    h->delta = delta;
    h->state = state_dev;
    h->state_len = state_len;
    h->work = work_dev;
    h->work_len = work_len;
    h->stream = (hipStream_t)hip_stream;
    h->sweep = 0;
    h->hmc_steps = 7;
    h->tev = nullptr;
    h->tcap = h->tn = 0;
    h->w = xyk::carve(work_dev, L, precision);
    xy_plan p;
    if (!cache_lookup(env_cache_path(), L, precision, &p)) p = default_plan(L, precision);
    h->plan = p;
    *out = h;
    return XY_OK;
}

int xy_init(xy_lattice** out, uint64_t seed, int32_t L, double beta, double delta, int32_t start,
            int32_t precision, void* state_dev, size_t state_len, void* work_dev, size_t work_len,
            void* hip_stream)
{
    if (out) *out = nullptr;
    if (start != XY_HOT && start != XY_COLD) return XY_EINVAL;
    int rc = make_handle(out, seed, L, beta, delta, precision, state_dev, state_len, work_dev, work_len, hip_stream);
    if (rc != XY_OK) return rc;
    xy_lattice* h = *out;
    hipError_t e = XY_LAUNCH(xyk::launch_init(h->state, L, precision, (uint32_t)(seed & 0xffffffffu),
                                              (uint32_t)(seed >> 32), start == XY_HOT, h->stream));
    if (e == hipSuccess) e = XY_LAUNCH(xyk::launch_zero_u64(h->w.counter, 4, h->stream));
    if (e != hipSuccess) {
        h->magic = 0;
        delete h;
        *out = nullptr;
        return hip_fail(e, "xy_init: launch");
    }
    return XY_OK;
}

int xy_attach(xy_lattice** out, uint64_t seed, int32_t L, double beta, double delta, int32_t precision,
              uint64_t sweep, void* state_dev, size_t state_len, void* work_dev, size_t work_len, void* hip_stream)
{
    if (out) *out = nullptr;
    if (sweep >= 0xffffffffull) return XY_ERANGE;
    int rc = make_handle(out, seed, L, beta, delta, precision, state_dev, state_len, work_dev, work_len, hip_stream);
    if (rc != XY_OK) return rc;
    xy_lattice* h = *out;
    h->sweep = sweep;
    hipError_t e = XY_LAUNCH(xyk::launch_zero_u64(h->w.counter, 4, h->stream));
    if (e != hipSuccess) {
        h->magic = 0;
        delete h;
        *out = nullptr;
        return hip_fail(e, "xy_attach: launch");
    }
    return XY_OK;
}

// One sweep in place by two half-sweep launches.  A failure of the first launch
// leaves the state and counter as they were; a failure of the second leaves the
// red half-sweep done, which is then finished so that state and counter agree.
static int stream_sweep(xy_lattice* h, bool measured, xy_obs* rec, uint8_t* dbg_acc, float* dbg_dE)
{
    xyk::SweepArgs a = args_of(h);
    unsigned long long* cnt = measured ? h->w.counter : nullptr;
    hipError_t e = XY_LAUNCH(xyk::launch_half_sweep(a, 0, cnt, dbg_acc, dbg_dE, h->stream));
    if (e != hipSuccess) return hip_fail(e, "half-sweep launch");
    e = XY_LAUNCH(xyk::launch_half_sweep(a, 1, cnt, dbg_acc, dbg_dE, h->stream));
    if (e != hipSuccess) {
        // finish the sweep; its record is lost, so its accepts are dropped too
        const int rc = hip_fail(e, "half-sweep launch");
        if (xyk::launch_half_sweep(a, 1, cnt, dbg_acc, dbg_dE, h->stream) == hipSuccess) h->sweep += 1;
        if (cnt) (void)xyk::launch_zero_u64(h->w.counter, 4, h->stream);
        return rc;
    }
    h->sweep += 1;
    if (measured) {
        int np = 0;
        e = XY_LAUNCH(xyk::launch_measure(h->state, h->L, h->precision, h->w.partials, h->w.max_partials, &np,
                                          h->stream));
        if (e == hipSuccess)
            e = XY_LAUNCH(xyk::launch_finalize(h->w.partials, np, h->w.counter, rec, h->sweep, h->stream,
                                               h->w.chunks, h->w.arrive));
        if (e != hipSuccess) {
            // the record is lost; its accepts must not leak into the next one
            const int rc = hip_fail(e, "measure launch");
            (void)xyk::launch_zero_u64(h->w.counter, 4, h->stream);
            return rc;
        }
    }
    return XY_OK;
}

int xy_sweep(xy_lattice* h, int64_t n_sweeps, int32_t measure_every, xy_obs* obs_dev)
{
    if (!live(h)) return XY_ESTATE;
    if (n_sweeps < 0 || measure_every < 0) return XY_EINVAL;
    if (h->sweep + (uint64_t)n_sweeps >= 0xffffffffull) return XY_ERANGE;
    const bool meas = measure_every > 0 && obs_dev != nullptr;
    auto measured = [&](int64_t j) { return meas && (j % measure_every) == 0; };  // j = 1-based sweep in call
    auto rec_of = [&](int64_t j) { return obs_dev + (j / measure_every - 1); };

    if (h->plan.kind == XY_PLAN_STREAM) {
        for (int64_t j = 1; j <= n_sweeps; ++j) {
            int rc = stream_sweep(h, measured(j), measured(j) ? rec_of(j) : nullptr, nullptr, nullptr);
            if (rc != XY_OK) return rc;
        }
        return XY_OK;
    }

    if (h->plan.kind == XY_PLAN_RESIDENT) {
        // every sweep of the call in one launch; calls longer than 2^30 sweeps are
        // split at a multiple of measure_every
        const int64_t cap = meas ? ((int64_t)1 << 30) / measure_every * measure_every : ((int64_t)1 << 30);
        for (int64_t done = 0; done < n_sweeps;) {
            const int64_t m = std::min<int64_t>(cap, n_sweeps - done);
            xyk::SweepArgs a = args_of(h);
            hipError_t e = XY_LAUNCH(xyk::launch_resident(a, (int)m, meas ? measure_every : 0,
                                                          meas ? obs_dev + done / measure_every : nullptr,
                                                          h->stream));
            if (e != hipSuccess) return hip_fail(e, "resident sweep launch");
            h->sweep += (uint64_t)m;
            done += m;
        }
        return XY_OK;
    }

    // Tiled schedules: ping-pong passes (state -> pingpong -> state ...); after an
    // odd number of passes the angles are copied back from the ping-pong buffer
    // (one device copy, far cheaper than a streaming sweep at large L), so they
    // end in the caller's buffer; sweeps left over by a two-sweep plan run in
    // place with the streaming schedule (same trajectory).  If a launch fails after
    // an odd number of passes, the latest angles are copied back likewise, so the
    // state and the counter (the sweeps enqueued) always agree and the handle
    // stays usable.
    const bool strip = h->plan.kind == XY_PLAN_STRIP;
    const int m = strip ? 1 : h->plan.sweeps_per_pass;
    const int64_t passes = n_sweeps / m;
    const int nrec = strip ? xyk::strip_records(h->L, h->plan.tile_x, h->plan.tile_y)
                           : xyk::fused_records(h->L, h->plan.tile_x, h->plan.tile_y, m);
    int64_t j = 0;  // sweeps done in this call
    int64_t done_passes = 0;
    auto fail = [&](hipError_t e, const char* what) {
        const int rc = hip_fail(e, what);
        if (done_passes & 1)
            (void)hipMemcpyAsync(h->state, h->w.pingpong, xyk::state_bytes(h->L, h->precision),
                                 hipMemcpyDeviceToDevice, h->stream);
        return rc;
    };
    for (int64_t q = 0; q < passes; ++q) {
        xyk::SweepArgs a = args_of(h);
        a.src = (q & 1) ? h->w.pingpong : h->state;
        a.dst = (q & 1) ? h->state : h->w.pingpong;
        unsigned mask = 0;
        for (int js = 0; js < m; ++js)
            if (measured(j + js + 1)) mask |= 1u << js;
        const bool timing = h->tn < h->tcap;
        if (timing) (void)hipEventRecord(h->tev[2 * h->tn], h->stream);
        hipError_t e = XY_LAUNCH(strip ? xyk::launch_strip(a, h->plan.tile_x, h->plan.tile_y, mask != 0,
                                                           h->w.partials, h->stream)
                                       : xyk::launch_fused(a, h->plan.tile_x, h->plan.tile_y, m, mask,
                                                           h->w.partials, h->stream));
        if (e != hipSuccess) return fail(e, "fused sweep launch");
        if (timing) (void)hipEventRecord(h->tev[2 * h->tn++ + 1], h->stream);
        done_passes = q + 1;
        const uint64_t s0 = h->sweep;
        h->sweep += m;
        j += m;
        for (int js = 0; js < m; ++js) {
            if (!(mask & (1u << js))) continue;
            e = XY_LAUNCH(xyk::launch_finalize(h->w.partials + (size_t)js * nrec * 8, nrec, nullptr,
                                               rec_of(j - m + js + 1), s0 + js + 1, h->stream, h->w.chunks,
                                               h->w.arrive));
            if (e != hipSuccess) return fail(e, "finalize launch");
        }
    }
    if (done_passes & 1) {
        hipError_t e = XY_LAUNCH(hipMemcpyAsync(h->state, h->w.pingpong, xyk::state_bytes(h->L, h->precision),
                                                hipMemcpyDeviceToDevice, h->stream));
        if (e != hipSuccess) return fail(e, "copy back");
        done_passes = 0;
    }
    for (; j < n_sweeps; ++j) {
        int rc = stream_sweep(h, measured(j + 1), measured(j + 1) ? rec_of(j + 1) : nullptr, nullptr, nullptr);
        if (rc != XY_OK) return rc;
    }
    return XY_OK;
}

int xy_measure(xy_lattice* h, xy_obs* obs_dev)
{
    if (!live(h)) return XY_ESTATE;
    if (!obs_dev) return XY_ESTATE;
    int np = 0;
    hipError_t e = XY_LAUNCH(
        xyk::launch_measure(h->state, h->L, h->precision, h->w.partials, h->w.max_partials, &np, h->stream));
    if (e == hipSuccess)
        e = XY_LAUNCH(xyk::launch_finalize(h->w.partials, np, nullptr, obs_dev, h->sweep, h->stream, h->w.chunks,
                                           h->w.arrive));
    if (e != hipSuccess) return hip_fail(e, "measure launch");
    return XY_OK;
}

int xy_hmc_work_bytes(int32_t L, size_t* bytes)
{
    if (!valid_L(L)) return XY_EINVAL;
    if (bytes) *bytes = xyk::hmc_work_bytes(L);
    return XY_OK;
}

int xy_hmc(xy_lattice* h, int64_t n_traj, int32_t n_md, double eps, void* hmc_work, size_t hmc_len,
           xy_hmc_obs* obs_dev)
{
    if (!live(h)) return XY_ESTATE;
    if (h->precision != XY_FP32 || n_traj < 0 || n_md < 1 || !std::isfinite(eps) || !(eps > 0.0)) return XY_EINVAL;
    if (!hmc_work) return XY_ESTATE;
    if (hmc_len < xyk::hmc_work_bytes(h->L)) return XY_ESIZE;
    if (h->sweep + (uint64_t)n_traj >= 0xffffffffull) return XY_ERANGE;
    const xyk::HmcWork w = xyk::hmc_carve(hmc_work, h->L);
    const uint32_t k0 = (uint32_t)(h->seed & 0xffffffffu), k1 = (uint32_t)(h->seed >> 32);
    for (int64_t j = 0; j < n_traj; ++j) {
        hipError_t e = XY_LAUNCH(xyk::launch_hmc_trajectory((float*)h->state, (float*)h->w.pingpong, w, h->L,
                                                            h->beta, eps, n_md, h->hmc_steps, (uint32_t)h->sweep,
                                                            k0, k1, obs_dev ? obs_dev + j : nullptr, h->stream));
        if (e != hipSuccess) return hip_fail(e, "hmc trajectory launch");
        h->sweep += 1;
    }
    return XY_OK;
}

int xy_hmc_set_steps_per_pass(xy_lattice* h, int32_t steps)
{
    if (!live(h)) return XY_ESTATE;
    if (steps < 1 || steps > 8) return XY_EINVAL;
    h->hmc_steps = steps;
    return XY_OK;
}

int xy_hmc_get_steps_per_pass(const xy_lattice* h, int32_t* steps)
{
    if (!live(h) || !steps) return XY_ESTATE;
    *steps = xyk::hmc_multi_supported(h->L) ? h->hmc_steps : 1;
    return XY_OK;
}

int xy_set_params(xy_lattice* h, double beta, double delta)
{
    if (!live(h)) return XY_ESTATE;
    if (!valid_beta_delta(beta, delta)) return XY_EINVAL;
    h->beta = beta;
    h->delta = delta;
    return XY_OK;
}

int xy_get_sweep(const xy_lattice* h, uint64_t* sweep)
{
    if (!live(h) || !sweep) return XY_ESTATE;
    *sweep = h->sweep;
    return XY_OK;
}

int xy_set_sweep(xy_lattice* h, uint64_t sweep)
{
    if (!live(h)) return XY_ESTATE;
    if (sweep >= 0xffffffffull) return XY_ERANGE;
    h->sweep = sweep;
    return XY_OK;
}

int xy_set_stream(xy_lattice* h, void* hip_stream)
{
    if (!live(h)) return XY_ESTATE;
    h->stream = (hipStream_t)hip_stream;
    return XY_OK;
}

int xy_set_plan(xy_lattice* h, const xy_plan* plan)
{
    if (!live(h) || !plan) return XY_ESTATE;
    xy_plan p = *plan;
    if (p.kind == XY_PLAN_AUTO) {
        if (!cache_lookup(env_cache_path(), h->L, h->precision, &p)) p = default_plan(h->L, h->precision);
    }
    if (!plan_ok(h->L, p)) return XY_EINVAL;
    h->plan = p;
    return XY_OK;
}

int xy_get_plan(const xy_lattice* h, xy_plan* plan)
{
    if (!live(h) || !plan) return XY_ESTATE;
    *plan = h->plan;
    return XY_OK;
}

static void drop_timer(xy_lattice* h)
{
    if (h->tev) {
        for (int i = 0; i < 2 * h->tcap; ++i)
            if (h->tev[i]) (void)hipEventDestroy(h->tev[i]);
        delete[] h->tev;
    }
    h->tev = nullptr;
    h->tcap = h->tn = 0;
}

int xy_free(xy_lattice* h)
{
    if (!live(h)) return XY_ESTATE;
    drop_timer(h);
    h->magic = 0;
    delete h;
    return XY_OK;
}

int xy_kernel_timer(xy_lattice* h, int32_t capacity)
{
    if (!live(h)) return XY_ESTATE;
    if (capacity < 0) return XY_EINVAL;
    drop_timer(h);
    if (capacity == 0) return XY_OK;
    h->tev = new (std::nothrow) hipEvent_t[2 * (size_t)capacity]();
    if (!h->tev) return XY_ENOMEM;
    h->tcap = capacity;
    for (int i = 0; i < 2 * capacity; ++i) {
        hipError_t e = hipEventCreate(&h->tev[i]);
        if (e != hipSuccess) {
            h->tev[i] = nullptr;
            drop_timer(h);
            return hip_fail(e, "xy_kernel_timer: hipEventCreate");
        }
    }
    return XY_OK;
}

int xy_kernel_timer_read(xy_lattice* h, double* total_ms, int64_t* launches)
{
    if (!live(h) || !total_ms || !launches) return XY_ESTATE;
    double t = 0.0;
    if (h->tn > 0) {
        hipError_t e = hipEventSynchronize(h->tev[2 * h->tn - 1]);
        if (e != hipSuccess) return hip_fail(e, "xy_kernel_timer_read: hipEventSynchronize");
        for (int i = 0; i < h->tn; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, h->tev[2 * i], h->tev[2 * i + 1]);
            if (e != hipSuccess) return hip_fail(e, "xy_kernel_timer_read: hipEventElapsedTime");
            t += ms;
        }
    }
    *total_ms = t;
    *launches = h->tn;
    h->tn = 0;
    return XY_OK;
}

int xy_debug_sweep(xy_lattice* h, uint8_t* accept_dev, float* dE_dev)
{
    if (!live(h)) return XY_ESTATE;
    if (h->sweep + 1 >= 0xffffffffull) return XY_ERANGE;
    return stream_sweep(h, false, nullptr, accept_dev, dE_dev);
}

int xy_autotune(xy_lattice* h, int32_t sweeps_per_trial, const char* cache_path, xy_plan* best)
{
    if (!live(h)) return XY_ESTATE;
    if (sweeps_per_trial < 2) return XY_EINVAL;
    std::vector<xy_plan> cands;
    cands.push_back({XY_PLAN_STREAM, 0, 0, 1});
    static const int shapes[][3] = {{64, 16, 1}, {64, 32, 1}, {128, 16, 1}, {128, 32, 1}, {128, 64, 1},
                                    {256, 16, 1}, {256, 32, 1}, {64, 32, 2}, {128, 32, 2}};
    for (auto& s : shapes) {
        xy_plan p{XY_PLAN_FUSED, s[0], s[1], s[2]};
        if (plan_ok(h->L, p)) cands.push_back(p);
    }
    if (plan_ok(h->L, xy_plan{XY_PLAN_RESIDENT, 0, 0, 1})) cands.push_back({XY_PLAN_RESIDENT, 0, 0, 1});
    static const int strips[][2] = {{128, 32},  {128, 64},  {128, 128}, {256, 32}, {256, 64},
                                    {256, 128}, {256, 256}, {512, 64},  {512, 128}, {512, 256}};
    for (auto& s : strips) {
        xy_plan p{XY_PLAN_STRIP, s[0], s[1], 1};
        if (plan_ok(h->L, p)) cands.push_back(p);
    }
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    const xy_plan saved = h->plan;
    double best_t = 1e300;
    xy_plan best_p = saved;
    int rc = XY_OK;
    // two rounds over the candidates, each candidate's best trial counting, so
    // that one slow trial (a clock change, another process) does not decide
    std::vector<xy_plan> trials(cands);
    trials.insert(trials.end(), cands.begin(), cands.end());
    for (const xy_plan& p : trials) {
        h->plan = p;
        if (h->sweep + 2ull * (uint64_t)sweeps_per_trial + 2 >= 0xffffffffull) h->sweep = 0;
        rc = xy_sweep(h, sweeps_per_trial, 0, nullptr);  // warm-up (sets LDS attributes, caches)
        if (rc != XY_OK) break;
        if ((e = hipEventRecord(e0, h->stream)) != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
        rc = xy_sweep(h, sweeps_per_trial, 0, nullptr);
        if (rc != XY_OK) break;
        if ((e = hipEventRecord(e1, h->stream)) != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
        if ((e = hipEventSynchronize(e1)) != hipSuccess) { rc = hip_fail(e, "hipEventSynchronize"); break; }
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = hip_fail(e, "hipEventElapsedTime"); break; }
        if (ms < best_t) {
            best_t = ms;
            best_p = p;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->plan = (rc == XY_OK) ? best_p : saved;
    if (rc != XY_OK) return rc;
    if (best) *best = best_p;
    if (cache_path) {
        const double gupd = (double)h->L * h->L * sweeps_per_trial / (best_t * 1e-3) / 1e9;
        if (!cache_store(cache_path, h->L, h->precision, best_p, gupd)) return XY_EIO;
    }
    return XY_OK;
}

int xy_tuned_plan(const char* cache_path, int32_t L, int32_t precision, xy_plan* plan)
{
    if (!plan || !cache_path) return XY_ESTATE;
    if (!valid_L(L)) return XY_EINVAL;
    return cache_lookup(cache_path, L, precision, plan) ? XY_OK : XY_EINVAL;
}

}  // extern "C"

int xyr::sweep_on_work(uint64_t seed, int32_t L, double beta, double delta, int32_t precision, uint64_t sweep,
                       int64_t n_sweeps, int32_t measure_every, void* state_dev, size_t state_len, void* work,
                       size_t work_len, xy_obs* obs_dev, hipStream_t stream)
{
    if (!valid_L(L) || !valid_beta_delta(beta, delta) || (precision != XY_FP32 && precision != XY_FP16) ||
        n_sweeps < 0 || measure_every < 0)
        return XY_EINVAL;
    if (!state_dev || !work) return XY_ESTATE;
    if (state_len < xyk::state_bytes(L, precision) || work_len < xyk::work_bytes(L, precision)) return XY_ESIZE;
    if (sweep >= 0xffffffffull || sweep + (uint64_t)n_sweeps >= 0xffffffffull) return XY_ERANGE;
    xy_lattice h;
    h.magic = kMagic;
    h.seed = seed;
    h.L = L;
    h.precision = precision;
    h.beta = beta;
    h.delta = delta;
    h.state = state_dev;
    h.state_len = state_len;
    h.work = work;
    h.work_len = work_len;
    h.stream = stream;
    h.sweep = sweep;
    h.hmc_steps = 7;
    h.tev = nullptr;
    h.tcap = h.tn = 0;
    h.w = xyk::carve(work, L, precision);
    h.plan = default_plan(L, precision);
    // the workspace keeps the previous call's contents: the accept and arrival
    // counters must start at zero (a kernel, so the call may be graph-captured)
    hipError_t e = XY_LAUNCH(xyk::launch_zero_u64(h.w.counter, 4, stream));
    if (e != hipSuccess) return hip_fail(e, "zero counters");
    const int rc = xy_sweep(&h, n_sweeps, measure_every, obs_dev);
    h.magic = 0;
    return rc;
}

extern "C" {

const char* xy_strerror(int code)
{
    switch (code) {
    case XY_OK: return "ok";
    case XY_EINVAL: return "invalid argument";
    case XY_ESIZE: return "buffer too small";
    case XY_ERANGE: return "sweep counter out of range";
    case XY_EHIP: return "HIP runtime error";
    case XY_ESTATE: return "invalid or freed handle / missing pointer";
    case XY_ENOMEM: return "host allocation failed";
    case XY_EBARRIER: return "batch barrier wait exceeded its spin limit";
    case XY_EIO: return "file could not be written";
    default: return "unknown error";
    }
}

const char* xy_last_hip_error(void) { return g_hip_err; }

int xy_test_inject_failure(int32_t after)
{
    if (after < -1) return XY_EINVAL;
    g_inject_countdown.store(after, std::memory_order_relaxed);
    return XY_OK;
}

}  // extern "C"
