// Launch timing for the roofline figures: HIP event pairs around selected kernel
// launches, resolved lazily, plus the algorithmic bytes each launch reports.
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "dg_internal.h"

namespace dg {

namespace {
struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes;
    int id;
};
struct Total {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
int g_next_id = 0;  // launch ids stay valid across resolves (a resolved id is simply not found)
std::vector<hipEvent_t> g_pool;
std::vector<std::string> g_order;
std::unordered_map<std::string, Total> g_tot;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void resolve_locked() {
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto it = g_tot.find(p.name);
            if (it == g_tot.end()) {
                g_order.push_back(p.name);
                it = g_tot.emplace(p.name, Total{}).first;
            }
            it->second.launches += 1;
            it->second.ms += ms;
            it->second.bytes += p.bytes;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

bool prof_on() { return g_on; }

int prof_begin(const char *name, hipStream_t s) {
    if (!g_on) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    Pending p{name, take_event(), take_event(), 0.0, g_next_id};
    if (!p.a || !p.b) return -1;
    g_next_id = (g_next_id + 1) & 0x3fffffff;
    (void)hipEventRecord(p.a, s);
    g_pending.push_back(p);
    if (g_pending.size() > 20000) {
        // keep the pending list bounded: resolve everything but the new entry
        Pending last = g_pending.back();
        g_pending.pop_back();
        resolve_locked();
        g_pending.push_back(last);
    }
    return p.id;
}

static Pending *find_pending(int id) {
    for (size_t i = g_pending.size(); i-- > 0;)
        if (g_pending[i].id == id) return &g_pending[i];
    return nullptr;
}

void prof_end(int slot, hipStream_t s, double bytes) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Pending *p = find_pending(slot);
    if (!p) return;
    (void)hipEventRecord(p->b, s);
    p->bytes += bytes;
}

void prof_drop(int slot) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = g_pending.size(); i-- > 0;) {
        if (g_pending[i].id != slot) continue;
        // the events may still be pending on the stream: wait before reuse
        (void)hipEventSynchronize(g_pending[i].b);
        g_pool.push_back(g_pending[i].a);
        g_pool.push_back(g_pending[i].b);
        g_pending.erase(g_pending.begin() + (std::ptrdiff_t)i);
        return;
    }
}

void prof_add(int slot, double bytes) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Pending *p = find_pending(slot);
    if (p) p->bytes += bytes;
}


// ---- counter calibration ----------------------------------------------------------------
// Kernels with a known number of bytes, to scale the hardware byte counters
// (FETCH_SIZE, WRITE_SIZE) that the roofline's traffic figures come from:
//   kind 0: read every 16-byte word of the buffer once (a stream of `bytes` bytes);
//   kind 1: write every 16-byte word once;
//   kind 2: read one 4-byte word from each 128-byte line (bytes / 128 lines).
// Each workgroup writes one 16-byte word of its reduction (kinds 0, 2) at the
// buffer's start, so the extra writes stay below 16 bytes per workgroup.
__global__ __launch_bounds__(256) void k_cal_read(const int4 *__restrict__ p, int64_t n16, int4 *sink) {
    int4 acc = make_int4(0, 0, 0, 0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x) {
        const int4 v = p[i];
        acc.x ^= v.x; acc.y ^= v.y; acc.z ^= v.z; acc.w ^= v.w;
    }
    __shared__ int s[4];
    if (threadIdx.x < 4) s[threadIdx.x] = 0;
    __syncthreads();
    atomicXor(&s[0], acc.x); atomicXor(&s[1], acc.y); atomicXor(&s[2], acc.z); atomicXor(&s[3], acc.w);
    __syncthreads();
    if (threadIdx.x == 0 && (s[0] | s[1] | s[2] | s[3]) == 0x7fffffff) sink[blockIdx.x] = make_int4(s[0], s[1], s[2], s[3]);
}
__global__ __launch_bounds__(256) void k_cal_write(int4 *p, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_int4((int)i, 1, 2, 3);
}
__global__ __launch_bounds__(256) void k_cal_gather(const int32_t *__restrict__ p, int64_t nlines, int32_t *sink) {
    int acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nlines; i += (int64_t)gridDim.x * blockDim.x)
        acc ^= p[i * 32 + (i & 31)];
    if (acc == 0x7fffffff) sink[0] = acc;
}

// kind 3: CAL_GATHERS 8-byte reads at pseudo-random positions of the first `bytes`
// bytes (SplitMix64 finaliser of the read index, modulo the word count), eight
// independent reads in flight per lane, summed per workgroup; one 16-byte word of
// the sum is written per workgroup at the buffer's start.
constexpr int64_t CAL_GATHERS = 1ll << 26;
__device__ __forceinline__ uint64_t cal_mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__global__ __launch_bounds__(256) void k_cal_rgather(const double *__restrict__ p, int64_t nwords, double *sink) {
    constexpr int U = 8;
    double acc = 0.0;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < CAL_GATHERS; i0 += U * st) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * st;
            v[u] = i < CAL_GATHERS ? p[cal_mix((uint64_t)i) % (uint64_t)nwords] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[2 * blockIdx.x] = red[0];
}

}  // namespace dg

extern "C" int dg_calibrate(int32_t kind, void *buf, int64_t bytes, void *stream) {
    using namespace dg;
    if (!buf || bytes < 4096 || (bytes & 4095) || kind < 0 || kind > 3)
        return set_error(DG_EINVAL, "calibration needs kind 0..3 and a device buffer of a multiple of 4 KiB");
    if (kind == 3 && bytes < 4096 * 16)
        return set_error(DG_EINVAL, "calibration kind 3 needs at least 64 KiB (one 16-byte sum per workgroup)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int blocks = 4096;
    if (kind == 0)
        hipLaunchKernelGGL(k_cal_read, dim3(blocks), dim3(256), 0, s, static_cast<const int4 *>(buf), bytes / 16,
                           static_cast<int4 *>(buf));
    else if (kind == 1)
        hipLaunchKernelGGL(k_cal_write, dim3(blocks), dim3(256), 0, s, static_cast<int4 *>(buf), bytes / 16);
    else if (kind == 2)
        hipLaunchKernelGGL(k_cal_gather, dim3(blocks), dim3(256), 0, s, static_cast<const int32_t *>(buf),
                           bytes / 128, static_cast<int32_t *>(buf));
    else
        hipLaunchKernelGGL(k_cal_rgather, dim3(blocks), dim3(256), 0, s, static_cast<const double *>(buf), bytes / 8,
                           static_cast<double *>(buf));
    DG_HIP(hipGetLastError());
    DG_HIP(hipStreamSynchronize(s));
    return DG_OK;
}

namespace dg {
}  // namespace dg

extern "C" {

int dg_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(dg::g_mu);
    dg::g_on = on != 0;
    return DG_OK;
}

int dg_profile_reset(void) {
    std::lock_guard<std::mutex> lk(dg::g_mu);
    dg::resolve_locked();
    dg::g_tot.clear();
    dg::g_order.clear();
    return DG_OK;
}

int dg_profile_read(dg_kernel_prof *out, int32_t cap, int32_t *count) {
    if (!count || (cap > 0 && !out)) return dg::set_error(DG_EINVAL, "bad profile arguments");
    std::lock_guard<std::mutex> lk(dg::g_mu);
    dg::resolve_locked();
    int32_t c = 0;
    for (const auto &name : dg::g_order) {
        if (c < cap) {
            const auto &t = dg::g_tot[name];
            std::memset(&out[c], 0, sizeof(out[c]));
            std::strncpy(out[c].name, name.c_str(), sizeof(out[c].name) - 1);
            out[c].launches = t.launches;
            out[c].ms = t.ms;
            out[c].bytes = t.bytes;
        }
        ++c;
    }
    *count = c;
    return DG_OK;
}

}  // extern "C"
