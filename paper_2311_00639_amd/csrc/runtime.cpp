// Host runtime of libsyk: error reporting, device term tables, device workspaces.
#include <cstring>
#include <map>
#include <thread>

#include "internal.hpp"

namespace syk {

[[noreturn]] void fail(syk_status s, const std::string &msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(SYK_ENOMEM, std::string(what) + ": out of device memory");
    fail(SYK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------ device tables
static void free_tables(DeviceTables &t) {
    hipFree(t.x);
    hipFree(t.z);
    hipFree(t.c32);
    hipFree(t.c64);
    t = DeviceTables{};
}

const DeviceTables &Hamiltonian::tables(int blk) {
    int dev = 0;
    SYK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(dev_mu);
    for (int b = 0; b < 2; ++b)
        if (static_cast<int>(this->dev[b].size()) <= dev) this->dev[b].resize(dev + 1);
    DeviceTables &t = this->dev[blk][dev];
    if (t.x) return t;
    const auto &bt = block_terms[blk];
    std::vector<uint32_t> hx(K), hz(K);
    std::vector<float> hc32(K);
    std::vector<double> hc64(K);
    for (int a = 0; a < K; ++a) {
        hx[a] = bt[a].x;
        hz[a] = bt[a].z;
        hc64[a] = bt[a].c;
        hc32[a] = static_cast<float>(bt[a].c);
    }
    DeviceTables nt;
    try {
        SYK_HIP(hipMalloc(reinterpret_cast<void **>(&nt.x), K * sizeof(uint32_t)));
        SYK_HIP(hipMalloc(reinterpret_cast<void **>(&nt.z), K * sizeof(uint32_t)));
        SYK_HIP(hipMalloc(reinterpret_cast<void **>(&nt.c32), K * sizeof(float)));
        SYK_HIP(hipMalloc(reinterpret_cast<void **>(&nt.c64), K * sizeof(double)));
        SYK_HIP(hipMemcpy(nt.x, hx.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice));
        SYK_HIP(hipMemcpy(nt.z, hz.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice));
        SYK_HIP(hipMemcpy(nt.c32, hc32.data(), K * sizeof(float), hipMemcpyHostToDevice));
        SYK_HIP(hipMemcpy(nt.c64, hc64.data(), K * sizeof(double), hipMemcpyHostToDevice));
    } catch (...) {
        free_tables(nt);
        throw;
    }
    nt.n_real = n_real[blk];
    nt.K = K;
    t = nt;
    return t;
}

Hamiltonian::~Hamiltonian() {
    int cur = 0;
    bool have = hipGetDevice(&cur) == hipSuccess;
    for (int b = 0; b < 2; ++b)
        for (size_t d = 0; d < dev[b].size(); ++d)
            if (dev[b][d].x) {
                if (have) hipSetDevice(static_cast<int>(d));
                free_tables(dev[b][d]);
            }
    if (have) hipSetDevice(cur);
}

// ------------------------------------------------------------------ workspaces
DeviceBuffer::~DeviceBuffer() { release(); }

void DeviceBuffer::ensure(size_t bytes) {
    if (bytes <= n_) return;
    release();
    void *p = nullptr;
    SYK_HIP(hipMalloc(&p, bytes));
    p_ = static_cast<char *>(p);
    n_ = bytes;
}

void DeviceBuffer::release() {
    if (p_) hipFree(p_);
    p_ = nullptr;
    n_ = 0;
}

namespace {
struct WsKey {
    int dev;
    std::thread::id tid;
    int slot;
    bool operator<(const WsKey &o) const {
        if (dev != o.dev) return dev < o.dev;
        if (tid != o.tid) return tid < o.tid;
        return slot < o.slot;
    }
};
std::mutex ws_mu;
std::map<WsKey, DeviceBuffer> *ws_map() {
    static auto *m = new std::map<WsKey, DeviceBuffer>();   // never destroyed: no HIP calls at exit
    return m;
}
}  // namespace

DeviceBuffer &thread_workspace(int slot) {
    int dev = 0;
    SYK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(ws_mu);
    return (*ws_map())[WsKey{dev, std::this_thread::get_id(), slot}];
}

void release_thread_workspaces() {
    int dev = 0;
    SYK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(ws_mu);
    auto *m = ws_map();
    for (auto it = m->begin(); it != m->end();) {
        if (it->first.dev == dev && it->first.tid == std::this_thread::get_id())
            it = m->erase(it);
        else
            ++it;
    }
}

}  // namespace syk
