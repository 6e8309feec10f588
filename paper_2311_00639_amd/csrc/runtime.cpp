// Host runtime of libsyk: error reporting, device term tables, device workspaces.
#include <algorithm>
#include <cstring>
#include <map>
#include <thread>

#include "apply_plan.hpp"
#include "internal.hpp"

namespace syk {

[[noreturn]] void fail(syk_status s, const std::string &msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(SYK_ENOMEM, std::string(what) + ": out of device memory");
    fail(SYK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------ device tables
void *DeviceSlab::take(size_t bytes, const char *what) {
    const size_t b = (std::max<size_t>(bytes, 1) + 255) & ~static_cast<size_t>(255);
    if (base == nullptr || b > size - used)
        fail(SYK_ENOMEM, std::string(what) + ": " + std::to_string(b) + " bytes do not fit in the " +
                             std::to_string(size - used) + " left of this request's device region");
    void *p = base + used;
    used += b;
    return p;
}

static void free_tables(DeviceTables &t) {
    if (t.in_slab) {
        t = DeviceTables{};
        return;
    }
    ignore_status(hipFree(t.gx));
    ignore_status(hipFree(t.gs));
    ignore_status(hipFree(t.gm));
    ignore_status(hipFree(t.gz));
    ignore_status(hipFree(t.gc32));
    ignore_status(hipFree(t.gc64));
    t = DeviceTables{};
}

int gather_groups(const std::vector<BlockTerm> &terms) {
    std::vector<uint32_t> xs;
    xs.reserve(terms.size());
    for (const BlockTerm &t : terms) xs.push_back(t.x);
    std::sort(xs.begin(), xs.end());
    return static_cast<int>(std::unique(xs.begin(), xs.end()) - xs.begin());
}

template <typename U>
static void upload_vec(U *&d, const std::vector<U> &h, DeviceSlab *slab) {
    const size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(U);
    if (slab)
        d = static_cast<U *>(slab->take(bytes, "term tables"));
    else
        SYK_HIP(hipMalloc(reinterpret_cast<void **>(&d), bytes));
    if (!h.empty()) SYK_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(U), hipMemcpyHostToDevice));
}

const DeviceTables &Hamiltonian::tables(int blk) {
    int dev = 0;
    SYK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(dev_mu);
    for (int b = 0; b < 2; ++b)
        if (static_cast<int>(this->dev[b].size()) <= dev) this->dev[b].resize(dev + 1);
    DeviceTables &t = this->dev[blk][dev];
    if (t.gx) return t;
    const auto &bt = block_terms[blk];
    DeviceTables nt;
    nt.in_slab = slab != nullptr;
    nt.n_real = n_real[blk];
    nt.K = K;
    if (K > 0) {
        // terms ordered by (x, phase): one gather per x group, the group's real- and
        // i-phase coefficients summed per amplitude before the multiply
        std::vector<int> order(K);
        for (int a = 0; a < K; ++a) order[a] = a;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return bt[a].x != bt[b].x ? bt[a].x < bt[b].x : (!bt[a].imag && bt[b].imag);
        });
        std::vector<uint32_t> gx, gs, gm, gz(K);
        std::vector<float> gc32(K);
        std::vector<double> gc64(K);
        for (int i = 0; i < K; ++i) {
            const BlockTerm &t = bt[order[i]];
            if (i == 0 || t.x != bt[order[i - 1]].x) {
                gx.push_back(t.x);
                gs.push_back(static_cast<uint32_t>(i));
                gm.push_back(static_cast<uint32_t>(i));
            }
            if (!t.imag) gm.back() = static_cast<uint32_t>(i + 1);
            gz[i] = t.z;
            gc64[i] = t.c;
            gc32[i] = static_cast<float>(t.c);
        }
        gs.push_back(static_cast<uint32_t>(K));
        try {
            upload_vec(nt.gx, gx, slab);
            upload_vec(nt.gs, gs, slab);
            upload_vec(nt.gm, gm, slab);
            upload_vec(nt.gz, gz, slab);
            upload_vec(nt.gc32, gc32, slab);
            upload_vec(nt.gc64, gc64, slab);
        } catch (...) {
            free_tables(nt);
            throw;
        }
        nt.G = static_cast<int>(gx.size());
    }
    t = nt;
    return t;
}

template <>
const std::vector<TiledVariant> &tiled_variants<float>() {
    static const std::vector<TiledVariant> v = {{13, 3, 2, 1, 1, 0, 0}, {13, 3, 1, 0, 2, 0, 0}, {12, 3, 2, 1, 2, 0, 0},
                                                {12, 2, 4, 3, 1, 0, 0}, {13, 3, 2, 1, 1, 1, 0}, {13, 3, 2, 1, 1, 0, 1},
                                                {13, 3, 2, 1, 1, 0, 2}, {12, 3, 2, 1, 2, 0, 1}, {13, 3, 2, 1, 1, 2, 0},
                                                {13, 3, 2, 1, 1, 2, 1}, {13, 3, 2, 1, 1, 2, 2}, {11, 2, 2, 1, 2, 2, 0},
                                                {10, 2, 2, 1, 4, 2, 0}, {11, 2, 2, 1, 2, 2, 1}, {12, 3, 2, 1, 2, 2, 2},
                                                {12, 2, 2, 1, 2, 2, 2}, {12, 3, 2, 1, 2, 2, 1}};
    return v;
}
template <>
const std::vector<TiledVariant> &tiled_variants<double>() {
    static const std::vector<TiledVariant> v = {{12, 2, 2, 1, 1, 0, 0}, {12, 2, 1, 0, 2, 0, 0}, {11, 2, 2, 1, 2, 0, 0},
                                                {11, 1, 4, 3, 1, 0, 0}, {12, 2, 2, 1, 1, 1, 0}, {12, 2, 2, 1, 1, 0, 1},
                                                {12, 2, 2, 1, 1, 0, 2}, {11, 2, 2, 1, 2, 0, 1}, {12, 2, 2, 1, 1, 2, 0},
                                                {12, 2, 2, 1, 1, 2, 1}, {12, 2, 2, 1, 1, 2, 2}, {11, 2, 2, 1, 2, 2, 0},
                                                {10, 2, 2, 1, 4, 2, 0}, {11, 2, 2, 1, 2, 2, 1}, {11, 2, 2, 1, 2, 2, 2},
                                                {11, 1, 2, 1, 2, 2, 2}, {10, 1, 2, 1, 4, 2, 2}};
    return v;
}
// Before (or without) autotuning: the first of a preference order (control-block records
// with four, two, one tile per workgroup, then the same tile counts with per-term records;
// the fastest at N = 56 when measured) whose grid still has >= 256 workgroups, else the
// variant with the most workgroups.
template <typename T>
int default_variant(int L) {
    const auto &v = tiled_variants<T>();
    for (int pref : {10, 9, 8, 6, 5, 0}) {
        const TiledVariant &tv = v.at(pref);
        if (L >= tv.bt + tv.w + 8) return pref;
    }
    int best = 0;
    for (int i = 1; i < static_cast<int>(v.size()); ++i)
        if (v[i].bt + v[i].w < v[best].bt + v[best].w) best = i;
    return best;
}
template int default_variant<float>(int);
template int default_variant<double>(int);

template <typename T>
const ApplyPlan &Hamiltonian::plan(int blk, int rot, int variant) {
    int d = 0;
    SYK_HIP(hipGetDevice(&d));
    const int prec = sizeof(T) == 8 ? 1 : 0;
    const TiledVariant &tv = tiled_variants<T>().at(variant);
    std::lock_guard<std::mutex> g(dev_mu);
    ApplyPlan &p = plans[std::make_tuple(blk, prec, d, rot, variant)];
    if (p.pi) return p;
    HostPlan hp = build_host_plan(block_terms[blk], L, tv.bt, tv.rb, tv.nbuf, tv.pf, rot, 2 * sizeof(T),
                                  resident_bits(tv), tv.sr, tv.w);
    upload_plan(hp, tv.bt, tv.rb, p, slab);
    p.variant = variant;
    return p;
}
template const ApplyPlan &Hamiltonian::plan<float>(int, int, int);
template const ApplyPlan &Hamiltonian::plan<double>(int, int, int);

template <typename T>
int Hamiltonian::internal_rotation(int variant) {
    if (!use_tiled<T>(L)) return 0;
    const int prec = sizeof(T) == 8 ? 1 : 0;
    const TiledVariant &tv = tiled_variants<T>().at(variant);     // throws for an unknown variant
    std::lock_guard<std::mutex> g(dev_mu);
    auto it = rotation.find({prec, variant});
    if (it == rotation.end())
        it = rotation.emplace(std::make_pair(prec, variant), choose_rotation(block_terms[0], L, tv.bt, resident_bits(tv),
                                                                              tv.w)).first;
    return it->second;
}
template int Hamiltonian::internal_rotation<float>(int);
template int Hamiltonian::internal_rotation<double>(int);

template <typename T>
int Hamiltonian::variant() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) d = 0;       // host-only queries: nothing tuned yet
    std::lock_guard<std::mutex> g(dev_mu);
    auto it = tuned.find({sizeof(T) == 8 ? 1 : 0, d});
    return it == tuned.end() ? default_variant<T>(L) : it->second;
}
template int Hamiltonian::variant<float>();
template int Hamiltonian::variant<double>();

template <typename T>
void apply_block(Hamiltonian &h, int blk, int rot, const T *x, T *y, int nvec, uint64_t ld, hipStream_t s) {
    if (use_tiled<T>(h.L)) {
        launch_apply_tiled<T>(h.plan<T>(blk, rot, h.variant<T>()), x, y, nvec, ld, s);
    } else {
        if (rot != 0) fail(SYK_EDEVICE, "rotated layouts are only planned for tiled blocks");
        launch_apply_h<T>(h.tables(blk), x, y, 1u << h.L, nvec, ld, s);
    }
}
template void apply_block<float>(Hamiltonian &, int, int, const float *, float *, int, uint64_t, hipStream_t);
template void apply_block<double>(Hamiltonian &, int, int, const double *, double *, int, uint64_t, hipStream_t);

template <typename T>
int apply_block_lanczos(Hamiltonian &h, int blk, int rot, const T *x, T *y, const LanczosFuse<T> &lf,
                        hipStream_t s) {
    if (!use_tiled<T>(h.L)) fail(SYK_EDEVICE, "the fused Lanczos step needs a tiled block");
    const ApplyPlan &pl = h.plan<T>(blk, rot, h.variant<T>());
    if (pl.n_wg > lanczos_partials_max(h.L)) fail(SYK_EDEVICE, "partials buffer too small");
    launch_apply_tiled<T>(pl, x, y, 1, 1ULL << h.L, s, &lf);
    return static_cast<int>(pl.n_wg);
}
template int apply_block_lanczos<float>(Hamiltonian &, int, int, const float *, float *,
                                        const LanczosFuse<float> &, hipStream_t);
template int apply_block_lanczos<double>(Hamiltonian &, int, int, const double *, double *,
                                         const LanczosFuse<double> &, hipStream_t);

// Time every compiled variant of the tiled kernel on this Hamiltonian (block U, each in
// its own planned layout) and keep the fastest for the current device.  x, y: scratch
// device vectors of 2^L amplitudes.
template <typename T>
int autotune(Hamiltonian &h, T *x, T *y, hipStream_t s, bool force, std::vector<float> *times) {
    if (!use_tiled<T>(h.L)) return -1;
    int dev = 0;
    SYK_HIP(hipGetDevice(&dev));
    if (!force) {
        std::lock_guard<std::mutex> g(h.dev_mu);
        auto it = h.tuned.find({sizeof(T) == 8 ? 1 : 0, dev});
        if (it != h.tuned.end()) return it->second;
    }
    const auto &vars = tiled_variants<T>();
    const uint64_t n = 1ULL << h.L;
    const int np = reduction_blocks(n);
    double *part = nullptr;
    SYK_HIP(hipMalloc(reinterpret_cast<void **>(&part), (np + 1) * sizeof(double)));
    hipEvent_t e0, e1;
    SYK_HIP(hipEventCreate(&e0));
    SYK_HIP(hipEventCreate(&e1));
    int best = default_variant<T>(h.L);
    float best_ms = 1e30f;
    if (times) times->assign(vars.size(), -1.0f);
    try {
        launch_haar_raw<T>(1, 0, h.L - 1, 0, x, x + n, part, np, s);     // any finite data
        for (int v = 0; v < static_cast<int>(vars.size()); ++v) {
            if (vars[v].bt + vars[v].w + 3 > h.L) continue;              // needs >= 8 workgroups
            const ApplyPlan &pl = h.plan<T>(0, h.internal_rotation<T>(v), v);
            launch_apply_tiled<T>(pl, x, y, 1, n, s);                    // warm-up
            SYK_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < 3; ++k) launch_apply_tiled<T>(pl, x, y, 1, n, s);
            SYK_HIP(hipEventRecord(e1, s));
            SYK_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            SYK_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (times) (*times)[v] = ms / 3.0f;
            if (ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
    } catch (...) {
        ignore_status(hipEventDestroy(e0));
        ignore_status(hipEventDestroy(e1));
        ignore_status(hipFree(part));
        throw;
    }
    ignore_status(hipEventDestroy(e0));
    ignore_status(hipEventDestroy(e1));
    ignore_status(hipFree(part));
    std::lock_guard<std::mutex> g(h.dev_mu);
    h.tuned[{sizeof(T) == 8 ? 1 : 0, dev}] = best;
    return best;
}
template int autotune<float>(Hamiltonian &, float *, float *, hipStream_t, bool, std::vector<float> *);
template int autotune<double>(Hamiltonian &, double *, double *, hipStream_t, bool, std::vector<float> *);

Hamiltonian::~Hamiltonian() {
    int cur = 0;
    bool have = hipGetDevice(&cur) == hipSuccess;
    for (int b = 0; b < 2; ++b) {
        for (size_t d = 0; d < dev[b].size(); ++d)
            if (dev[b][d].gx) {
                if (have) ignore_status(hipSetDevice(static_cast<int>(d)));
                free_tables(dev[b][d]);
            }
    }
    for (auto &kv : plans)
        if (kv.second.pi) {
            if (have) ignore_status(hipSetDevice(std::get<2>(kv.first)));
            free_plan(kv.second);
        }
    if (have) ignore_status(hipSetDevice(cur));
}

// ------------------------------------------------------------------ workspaces
DeviceBuffer::~DeviceBuffer() { release(); }

void DeviceBuffer::ensure(size_t bytes) {
    if (bytes <= n_) return;
    if (!owned_)
        fail(SYK_ENOMEM, "workspace needs " + std::to_string(bytes) + " bytes, its caller-owned region holds " +
                             std::to_string(n_));
    release();
    void *p = nullptr;
    SYK_HIP(hipMalloc(&p, bytes));
    p_ = static_cast<char *>(p);
    n_ = bytes;
}

void DeviceBuffer::release() {
    if (p_ && owned_) ignore_status(hipFree(p_));
    p_ = nullptr;
    n_ = 0;
    owned_ = true;
}

void DeviceBuffer::adopt(void *p, size_t bytes) {
    release();
    p_ = static_cast<char *>(p);
    n_ = bytes;
    owned_ = false;
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
