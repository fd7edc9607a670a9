// stats.hip - ensemble statistics of saved observables: for every column c
// of out[orbits][cols] (cols = saves x values per save) the mean and the
// standard deviation over orbits, in binary64.  These are the statistics
// the accuracy study of Sec. 2.3 reports for the order parameter, <r(t)> and
// sigma(r(t)) over realisations.
//
// Two passes, both in a fixed order, so the result does not depend on
// scheduling: (1) orbit chunk g of column c -> count, mean and sum of
// squared deviations (Welford's update, one thread per column and chunk,
// consecutive threads on consecutive columns so every read is coalesced);
// (2) one thread per column merges the chunks in order with the pairwise
// combination of Chan, Golub & LeVeque.
#include <mutex>

#include "launch.hpp"

namespace sode {
namespace {

struct Partial {
    double n, mean, m2;
};

// Fixed device scratch of the non-allocating entry point: room for the
// partials of kStatsStaticPartials (orbit chunk, column) pairs, 3 MiB.  Each
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes this name to a kernel (on the host it is a stand-in, not
// a device address); it uses the address stats_static_scratch() looks up.
static __device__ __align__(256) Partial scratch[kStatsStaticPartials];

constexpr int kMaxDevices = 64;

template <typename R>
__global__ __launch_bounds__(256) void column_partials(const R* __restrict__ x, int64_t orbits, int64_t cols,
                                                       int64_t chunk, Partial* __restrict__ part)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (c >= cols)
        return;
    const int64_t lo = g * chunk;
    const int64_t hi = lo + chunk < orbits ? lo + chunk : orbits;
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int64_t o = lo; o < hi; ++o) {
        const double v = (double)x[o * cols + c];
        n += 1.0;
        const double delta = v - mean;
        mean += delta / n;
        m2 += delta * (v - mean);
    }
    part[g * cols + c] = Partial{n, mean, m2};
}

__global__ __launch_bounds__(256) void merge_partials(const Partial* __restrict__ part, int64_t groups,
                                                      int64_t cols, double* __restrict__ mean_out,
                                                      double* __restrict__ std_out)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cols)
        return;
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int64_t g = 0; g < groups; ++g) {
        const Partial p = part[g * cols + c];
        if (p.n == 0.0)
            continue;
        const double tot = n + p.n;
        const double delta = p.mean - mean;
        mean += delta * (p.n / tot);
        m2 += p.m2 + delta * delta * (n * p.n / tot);
        n = tot;
    }
    mean_out[c] = mean;
    if (std_out)
        std_out[c] = n > 1.0 ? sqrt(m2 / (n - 1.0)) : 0.0;
}

template <typename R>
hipError_t launch_typed(const StatsRequest& r)
{
    const dim3 g1((unsigned)((r.cols + 255) / 256), (unsigned)r.groups);
    hipLaunchKernelGGL(column_partials<R>, g1, dim3(256), 0, r.stream, static_cast<const R*>(r.x), r.orbits,
                       r.cols, r.chunk, static_cast<Partial*>(r.scratch));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(merge_partials, dim3((unsigned)((r.cols + 255) / 256)), dim3(256), 0, r.stream,
                       static_cast<const Partial*>(r.scratch), r.groups, r.cols, r.mean, r.stddev);
    return hipGetLastError();
}

}  // namespace

size_t stats_partial_bytes() { return sizeof(Partial); }

void* stats_static_scratch(hipError_t* err)
{
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices))
        e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // With device `dev` current: its own copy of the array.
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        addr[dev] = ptr;
    }
    *err = hipSuccess;
    return addr[dev];
}

hipError_t launch_ensemble_stats(const StatsRequest& r)
{
    return r.precision == 64 ? launch_typed<double>(r) : launch_typed<float>(r);
}

}  // namespace sode
