// Kernel-side timing of the field-line passes (profiling mode 2).  With two line groups on two
// streams, events carried in a dispatch also count the time a launch waits for the other
// stream's kernel to free the compute units, so the passes time themselves: every block stamps
// its start and every wave its end on the device's constant-rate wall clock (the earliest start
// and the latest end per launch, over KCLK_SUB sub-slots so that few atomics meet on one word).
#include <climits>

#include "bem_device.h"

namespace bem {
namespace {

__global__ __launch_bounds__(256) void k_kclock_fill(int64_t n, unsigned long long* __restrict__ ts) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) ts[i] = (i & 1) ? 0ull : ULLONG_MAX;
}

// one thread per launch slot: latest end minus earliest start over its sub-slots, in ticks
__global__ __launch_bounds__(256) void k_kclock_span(int64_t m, const unsigned long long* __restrict__ ts,
                                                     unsigned long long* __restrict__ dur) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m) return;
    unsigned long long a = ULLONG_MAX, b = 0;
    for (int s = 0; s < KCLK_SUB; ++s) {
        const unsigned long long x = ts[(k * KCLK_SUB + s) * 2], y = ts[(k * KCLK_SUB + s) * 2 + 1];
        a = x < a ? x : a;
        b = y > b ? y : b;
    }
    dur[k] = (b > a) ? b - a : 0;
}

}  // namespace

void kclock_begin(bem_ctx* c, int64_t max_launches) {
    c->kclk_names.clear();
    if (c->profiling != 2) {
        c->kclk_cap = 0;
        return;
    }
    if (c->kclk_khz == 0) BEM_HIP(hipDeviceGetAttribute(&c->kclk_khz, hipDeviceAttributeWallClockRate, c->device));
    const int64_t words = 2 * KCLK_SUB * max_launches;
    c->kclk.alloc(sizeof(unsigned long long) * (size_t)words);
    c->kclk_dur.alloc(sizeof(unsigned long long) * (size_t)max_launches);
    c->kclk_cap = max_launches;
    hipLaunchKernelGGL(k_kclock_fill, dim3((unsigned)ceil_div(words, 256)), dim3(256), 0, c->stream, words,
                       c->kclk.as<unsigned long long>());
    BEM_CHECK_LAUNCH();
}

unsigned long long* kclock_slot(bem_ctx* c, const char* name) {
    const int64_t k = (int64_t)c->kclk_names.size();
    if (c->profiling != 2 || k >= c->kclk_cap) return nullptr;
    c->kclk_names.emplace_back(name);
    return c->kclk.as<unsigned long long>() + 2 * KCLK_SUB * k;
}

void kclock_end(bem_ctx* c) {
    const int64_t m = (int64_t)c->kclk_names.size();
    if (m == 0 || c->kclk_khz <= 0) {
        c->kclk_names.clear();
        return;
    }
    hipLaunchKernelGGL(k_kclock_span, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, c->stream, m,
                       c->kclk.as<unsigned long long>(), c->kclk_dur.as<unsigned long long>());
    BEM_CHECK_LAUNCH();
    std::vector<unsigned long long> h((size_t)m);
    BEM_HIP(hipMemcpyAsync(h.data(), c->kclk_dur.p, sizeof(unsigned long long) * (size_t)m, hipMemcpyDeviceToHost,
                           c->stream));
    BEM_HIP(hipStreamSynchronize(c->stream));
    for (int64_t k = 0; k < m; ++k) {
        if (h[(size_t)k] == 0) continue;   // a launch whose blocks all left before stamping (none here)
        auto& s = c->stats[c->kclk_names[(size_t)k]];
        s.launches += 1;
        s.ms += (double)h[(size_t)k] / (double)c->kclk_khz;
    }
    c->kclk_names.clear();
}

}  // namespace bem
