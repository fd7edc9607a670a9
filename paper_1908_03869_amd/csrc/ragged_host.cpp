// ragged_host.cpp - host side of sode_integrate_ragged: argument checks,
// the schedule (lane shape per instance, groups, longest-first order), the
// autotuner and the captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

#include "ctx.hpp"

namespace sode {
namespace {

constexpr int kMaxUnits = 128;

uint64_t fnv1a(const void* data, size_t bytes, uint64_t h = 1469598103934665603ull)
{
    const unsigned char* c = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

template <typename T>
uint64_t mix(uint64_t h, const T& v)
{
    return fnv1a(&v, sizeof v, h);
}

int pow2_at_least(int x)
{
    int p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// Lane shape of an instance with `units` chain units: U units per lane (at
// least units_min, enough for a full wave), then the fewest lanes (4 .. 64)
// that hold the chain.
void lane_shape(int units, int units_min, int* lanes, int* per_lane)
{
    int U = std::max(units_min, pow2_at_least((units + 63) / 64));
    U = std::min(U, 8);
    int L = pow2_at_least((units + U - 1) / U);
    L = std::min(std::max(L, 4), 64);
    *lanes = L;
    *per_lane = U;
}

int validate(const sode_ctx* h, const sode_instance_t* inst, int32_t count, int64_t x0_len,
             int64_t p_len, int64_t out_len)
{
    for (int32_t i = 0; i < count; ++i) {
        const sode_instance_t& d = inst[i];
        if (d.reserved0 != 0 || d.reserved1 != 0)
            return SODE_EINVAL;
        if (d.n < 2 || d.n % 2 != 0 || d.n > 2 * kMaxUnits || d.n > h->n)
            return SODE_EINVAL;
        if (d.nsteps < 0 || d.stride < 1 || d.nsteps % d.stride != 0 || d.nsteps >= (int64_t(1) << 32))
            return SODE_EINVAL;
        if (d.x0_offset < 0 || d.p_offset < 0 || d.out_offset < 0)
            return SODE_EINVAL;
        if (d.x0_offset > x0_len - d.n || d.p_offset > p_len - 5)
            return SODE_EINVAL;
        const int64_t nsave = d.nsteps / d.stride + 1;
        if (nsave > (out_len - d.out_offset) / d.n)
            return SODE_EINVAL;
    }
    return SODE_OK;
}

struct HostPlan {
    std::vector<int32_t> slots;  // [ngroups][kRaggedSlots]
    std::vector<int32_t> shape;  // [ngroups]
};

// Group instances of one lane shape and one save stride (sorted by step
// count, longest first) into groups of 64/L, then order all groups by
// decreasing U x steps.  A group's instances share the stride, so its wave
// follows one save schedule.
void build_plan(const sode_instance_t* inst, int32_t count, int units_min, HostPlan& plan)
{
    struct Member {
        int64_t nsteps;
        int32_t idx;
    };
    std::map<std::pair<int, int64_t>, std::vector<Member>> buckets;  // (shape, stride)
    int lanes_of[kRaggedShapes] = {0}, units_of[kRaggedShapes] = {0};
    for (int32_t i = 0; i < count; ++i) {
        int L, U;
        lane_shape(inst[i].n / 2, units_min, &L, &U);
        const int code = ragged_shape_code(L, U);
        lanes_of[code] = L;
        units_of[code] = U;
        buckets[{code, inst[i].stride}].push_back({inst[i].nsteps, i});
    }
    struct Group {
        int64_t cost;
        int shape;
        int32_t first;
        std::vector<int32_t> members;
    };
    std::vector<Group> groups;
    for (auto& bucket : buckets) {
        const int code = bucket.first.first;
        auto& v = bucket.second;
        std::sort(v.begin(), v.end(), [](const Member& a, const Member& b) {
            return a.nsteps != b.nsteps ? a.nsteps > b.nsteps : a.idx < b.idx;
        });
        const size_t per = 64 / lanes_of[code];
        for (size_t s = 0; s < v.size(); s += per) {
            Group g;
            g.cost = (int64_t)units_of[code] * std::max<int64_t>(v[s].nsteps, 1);
            g.shape = code;
            g.first = v[s].idx;
            for (size_t t = s; t < std::min(v.size(), s + per); ++t)
                g.members.push_back(v[t].idx);
            groups.push_back(std::move(g));
        }
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) {
        return a.cost != b.cost ? a.cost > b.cost : a.first < b.first;
    });
    plan.slots.assign(groups.size() * kRaggedSlots, -1);
    plan.shape.resize(groups.size());
    // Issue priority of the wave that runs a group (bits 8-9 of its shape
    // word): 3 for groups within 2x of the heaviest, 2 within 4x, 1 within
    // 8x, else 0.  The heaviest chains bound the makespan; the waves that
    // share their SIMDs fill the cycles they leave.
    const int64_t top = groups.empty() ? 1 : std::max<int64_t>(groups[0].cost, 1);
    for (size_t g = 0; g < groups.size(); ++g) {
        const int64_t c = groups[g].cost;
        const int prio = 2 * c >= top ? 3 : 4 * c >= top ? 2 : 8 * c >= top ? 1 : 0;
        plan.shape[g] = groups[g].shape | (prio << 8);
        for (size_t t = 0; t < groups[g].members.size(); ++t)
            plan.slots[g * kRaggedSlots + t] = groups[g].members[t];
    }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

void drop_graph(sode_ctx* h)
{
    if (h->rg_exec)
        (void)hipGraphExecDestroy(h->rg_exec);
    if (h->rg_graph)
        (void)hipGraphDestroy(h->rg_graph);
    h->rg_exec = nullptr;
    h->rg_graph = nullptr;
    h->rg_graph_key = 0;
}

// Upload the schedule for (descriptors, units_min) unless it is current.
int install_plan(sode_ctx* h, const sode_instance_t* inst, int32_t count, int units_min,
                 hipStream_t stream)
{
    uint64_t key = fnv1a(inst, sizeof(sode_instance_t) * (size_t)count);
    key = mix(key, count);
    key = mix(key, units_min);
    if (key == h->rg_plan_key && h->rg_buf)
        return SODE_OK;
    HostPlan plan;
    build_plan(inst, count, units_min, plan);
    const int32_t ngroups = (int32_t)plan.shape.size();
    const size_t desc_bytes = sizeof(sode_instance_t) * (size_t)count;
    const size_t slots_off = align256(desc_bytes);
    const size_t shape_off = slots_off + align256(plan.slots.size() * sizeof(int32_t));
    const size_t counter_off = shape_off + align256(plan.shape.size() * sizeof(int32_t));
    const size_t bytes = counter_off + 256;
    // Work still queued on the handle may read the old schedule.
    if (h->launched && hipStreamSynchronize(h->last_stream) != hipSuccess)
        return SODE_EDEVICE;
    if (bytes > h->rg_bytes) {
        drop_graph(h);
        if (h->rg_buf)
            (void)hipFree(h->rg_buf);
        h->rg_buf = nullptr;
        h->rg_bytes = 0;
        if (hipMalloc(&h->rg_buf, bytes) != hipSuccess) {
            h->rg_buf = nullptr;
            return SODE_ENOMEM;
        }
        h->rg_bytes = bytes;
    }
    char* base = static_cast<char*>(h->rg_buf);
    hipError_t e = hipMemcpyAsync(base, inst, desc_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !plan.slots.empty())
        e = hipMemcpyAsync(base + slots_off, plan.slots.data(), plan.slots.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !plan.shape.empty())
        e = hipMemcpyAsync(base + shape_off, plan.shape.data(), plan.shape.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);  // the host vectors die with this call
    if (e != hipSuccess) {
        h->rg_plan_key = 0;
        return SODE_EDEVICE;
    }
    h->rg_slots_off = slots_off;
    h->rg_shape_off = shape_off;
    h->rg_counter_off = counter_off;
    h->rg_ngroups = ngroups;
    h->rg_plan_key = key;
    return SODE_OK;
}

RaggedKernelArgs kernel_args(const sode_ctx* h, const void* X0, const void* p, void* out, double dt)
{
    char* base = static_cast<char*>(h->rg_buf);
    RaggedKernelArgs a;
    a.desc = reinterpret_cast<const sode_instance_t*>(base);
    a.slots = reinterpret_cast<const int32_t*>(base + h->rg_slots_off);
    a.shape = reinterpret_cast<const int32_t*>(base + h->rg_shape_off);
    a.counter = reinterpret_cast<uint32_t*>(base + h->rg_counter_off);
    a.ngroups = h->rg_ngroups;
    a.X0 = static_cast<const float*>(X0);
    a.p = static_cast<const float*>(p);
    a.out = static_cast<float*>(out);
    a.dt = (float)dt;
    a.sqdt = (float)std::sqrt(dt);
    a.compensated = h->compensated;
    int dev = 0;
    const auto it = hipGetDevice(&dev) == hipSuccess ? h->nonfinite.find(dev) : h->nonfinite.end();
    a.nonfinite = it == h->nonfinite.end() ? nullptr : it->second;
    return a;
}

int compute_units()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// Time every candidate (units per lane x waves per CU) on the batch itself,
// twice each (the faster of the two counts), and keep the fastest; a
// candidate with fewer waves per CU wins within 3 % of it (fewer waves
// sharing the SIMD of the batch's longest chain).  Each trial writes the
// same results to `out`.
int autotune(sode_ctx* h, const sode_instance_t* inst, int32_t count, const void* X0,
             const void* p, void* out, double dt, hipStream_t stream, int* best_waves,
             int* best_units)
{
    const int cus = compute_units();
    const int unit_choices[] = {1, 2, 4};
    const int wave_choices[] = {2, 4, 8, 16};
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess)
        return SODE_EDEVICE;
    if (hipEventCreate(&t1) != hipSuccess) {
        (void)hipEventDestroy(t0);
        return SODE_EDEVICE;
    }
    float best = -1.0f;
    struct Trial {
        float ms;
        int waves, units;
    };
    std::vector<Trial> trials;
    int status = SODE_OK;
    bool warmed = false;
    for (int U : unit_choices) {
        if (h->units_per_lane && U != h->units_per_lane)
            continue;
        status = install_plan(h, inst, count, U, stream);
        if (status != SODE_OK)
            break;
        const RaggedKernelArgs a = kernel_args(h, X0, p, out, dt);
        for (int W : wave_choices) {
            if (h->waves_per_cu && W != h->waves_per_cu)
                continue;
            if (!warmed) {
                (void)launch_fhn_ragged(a, 1, W * cus, stream);
                warmed = true;
            }
            float ms = -1.0f;
            hipError_t e = hipSuccess;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                (void)hipEventRecord(t0, stream);
                e = launch_fhn_ragged(a, 1, W * cus, stream);
                (void)hipEventRecord(t1, stream);
                if (e == hipSuccess)
                    e = hipEventSynchronize(t1);
                float t = 0.0f;
                if (e == hipSuccess)
                    e = hipEventElapsedTime(&t, t0, t1);
                if (e == hipSuccess && (ms < 0.0f || t < ms))
                    ms = t;
            }
            if (e != hipSuccess) {
                status = SODE_EDEVICE;
                break;
            }
            trials.push_back({ms, W, U});
            if (best < 0.0f || ms < best)
                best = ms;
        }
        if (status != SODE_OK)
            break;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (status == SODE_OK && best < 0.0f)
        status = SODE_EINVAL;  // fixed options outside the candidate set
    if (status == SODE_OK) {
        // Fewest waves per CU among the trials within 3 % of the fastest,
        // then the faster of those.
        const Trial* pick = nullptr;
        for (const Trial& t : trials) {
            if (t.ms > 1.03f * best)
                continue;
            if (!pick || t.waves < pick->waves || (t.waves == pick->waves && t.ms < pick->ms))
                pick = &t;
        }
        *best_waves = pick->waves;
        *best_units = pick->units;
    }
    return status;
}

}  // namespace

void release_ragged(sode_ctx* h)
{
    drop_graph(h);
    if (h->rg_capture)
        (void)hipStreamDestroy(h->rg_capture);
    if (h->rg_buf)
        (void)hipFree(h->rg_buf);
    h->rg_capture = nullptr;
    h->rg_buf = nullptr;
    h->rg_bytes = 0;
    h->rg_plan_key = 0;
}

}  // namespace sode

extern "C" int sode_integrate_ragged(sode_t h, const sode_instance_t* inst, int32_t count,
                                     const void* X0, int64_t x0_len, const void* p, int64_t p_len,
                                     void* out, int64_t out_len, double t0, double dt, void* stream)
{
    using namespace sode;
    if (!h || count < 0 || (count > 0 && !inst))
        return SODE_EINVAL;
    if (!std::isfinite(t0) || !std::isfinite(dt) || !(dt > 0.0))
        return SODE_EINVAL;
    // FHN noise is additive, so Milstein steps are the Euler-Maruyama steps;
    // the ODE-only methods have no ragged kernel.
    if (h->model != kFHN || h->precision != 32 || (h->method != kEM && h->method != kMilstein))
        return SODE_EUNSUPPORTED;
    if (count == 0)
        return SODE_OK;
    if (!X0 || !p || !out || x0_len < 0 || p_len < 0 || out_len < 0)
        return SODE_EINVAL;
    const int v = validate(h, inst, count, x0_len, p_len, out_len);
    if (v != SODE_OK)
        return v;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!nonfinite_flag(h))
        return SODE_ENOMEM;

    // Lane shape and grid: fixed options, else the tuned pair for this batch
    // shape (autotuning on first sight).
    uint64_t shape_key = 1469598103934665603ull;
    for (int32_t i = 0; i < count; ++i) {
        shape_key = mix(shape_key, inst[i].n);
        shape_key = mix(shape_key, inst[i].nsteps);
    }
    int waves = h->waves_per_cu, units = h->units_per_lane;
    if (!waves || !units) {
        auto it = h->rg_tuned.find(shape_key);
        if (it == h->rg_tuned.end() || (waves && it->second.first != waves) ||
            (units && it->second.second != units)) {
            int bw = 0, bu = 0;
            const int st = autotune(h, inst, count, X0, p, out, dt, s, &bw, &bu);
            if (st != SODE_OK)
                return st;
            if (!h->waves_per_cu && !h->units_per_lane)
                h->rg_tuned[shape_key] = {bw, bu};
            waves = bw;
            units = bu;
        } else {
            waves = it->second.first;
            units = it->second.second;
        }
    }
    int st = install_plan(h, inst, count, units, s);
    if (st != SODE_OK)
        return st;
    const int grid = waves * compute_units();
    const RaggedKernelArgs a = kernel_args(h, X0, p, out, dt);
    h->rg_last_waves = waves;
    h->rg_last_units = units;

    hipError_t e = hipSuccess;
    if (h->graph && h->persistent) {
        uint64_t key = mix(h->rg_plan_key, h->rg_buf);
        key = mix(key, X0);
        key = mix(key, p);
        key = mix(key, out);
        key = mix(key, dt);
        key = mix(key, grid);
        key = mix(key, h->compensated);
        key = mix(key, a.nonfinite);
        if (!h->rg_exec || key != h->rg_graph_key) {
            if (h->launched && hipStreamSynchronize(h->last_stream) != hipSuccess)
                return SODE_EDEVICE;
            drop_graph(h);
            if (!h->rg_capture && hipStreamCreateWithFlags(&h->rg_capture, hipStreamNonBlocking) != hipSuccess) {
                h->rg_capture = nullptr;
                return SODE_EDEVICE;
            }
            e = hipStreamBeginCapture(h->rg_capture, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                const hipError_t le = launch_fhn_ragged(a, 1, grid, h->rg_capture);
                e = hipStreamEndCapture(h->rg_capture, &h->rg_graph);
                if (e == hipSuccess)
                    e = le;
            }
            if (e == hipSuccess)
                e = hipGraphInstantiate(&h->rg_exec, h->rg_graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_graph(h);
                return SODE_EDEVICE;
            }
            h->rg_graph_key = key;
        }
        e = hipGraphLaunch(h->rg_exec, s);
    } else {
        e = launch_fhn_ragged(a, h->persistent, grid, s);
    }
    h->last_error = e;
    h->last_stream = s;
    h->launched = true;
    return e == hipSuccess ? SODE_OK : SODE_EDEVICE;
}
