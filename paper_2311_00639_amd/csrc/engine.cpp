// Request engine: continuous batching of OTOC requests on one device.
//
// Slots are host worker threads, each with its own HIP stream.  A free slot takes the
// first queued request (in arrival order) whose device footprint fits in a free region of
// the engine's arena; the oldest request may be overtaken by smaller ones only max_bypass
// times.  Requests admitted while others run share the GPU: their kernels are enqueued on
// different streams and overlap.  Every request builds its own Hamiltonian and runs the
// same code path as a single syk_otoc call with autotune off, so its result does not
// depend on the mix.
//
// Device memory: the arena is one allocation made when the engine starts (the whole
// budget).  An admitted request gets one region of it, sized by an upper bound of
// everything the request puts on the device: its workspace (Krylov basis, chain vectors,
// reduction partials) and its term tables and apply plans, which are carved from the
// region instead of allocated.  The region goes back to the arena after the request's
// stream has drained, so no hipMalloc or hipFree runs while requests are active (hipFree
// would wait for the whole device and stall the other requests' streams).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "apply_plan.hpp"
#include "engine.hpp"
#include "krylov.hpp"
#include "otoc.hpp"

namespace syk {

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint64_t kRegionAlign = 64ULL << 10;     // arena regions start on 64 KiB boundaries
uint64_t align_up(uint64_t b, uint64_t a) { return (b + a - 1) / a * a; }

// Upper bound of the device bytes of one block's gather tables (runtime.cpp: six arrays of
// at most K + 1 entries, each piece 256-byte aligned in a slab).
uint64_t tables_bound(uint64_t K) { return 4 * 4 * (K + 1) + 4 * (K + 1) + 8 * (K + 1) + 6 * 256; }

// Upper bound of the device bytes of one tiled apply plan (apply_plan.cpp) for K terms on
// 2^L amplitudes, over every compiled variant: at most 2^(L-10) tiles (the smallest tile
// has 2^10 amplitudes); at most 8 tiles per workgroup, so the partner union has at most
// 8 K entries, split steps add at most 8 K / 12 more (a control block holds >= 12
// records), padding to the buffer count and the prefetch entries add at most 8; ranges
// are 3 words per step and tile; records are a 64-word control block per step or at
// most 4 + 2 * 8 words per term; coefficients K + 1 floats and doubles.
uint64_t plan_bound(int L, uint64_t K) {
    const uint64_t steps = 8 * K + (8 * K + 11) / 12 + 8;
    const uint64_t tiles = L > 10 ? (1ULL << (L - 10)) : 1;
    const uint64_t meta = std::max<uint64_t>((steps + 1) * 64 * 4, (K + 1) * 20 * 4);
    return steps * 4 + steps * 8 * 3 * 4 + meta + tiles * 4 + (K + 1) * 12 + 6 * 256;
}

uint64_t footprint_bytes(int N, double k, int m, syk_dtype dt, bool precision_check) {
    const int L = N / 2 - 1;
    const uint64_t n = 1ULL << L;
    // the complex128 re-evaluation of a precision check reuses the workspace
    const size_t e = (dt == SYK_C64 && !precision_check) ? sizeof(float) : sizeof(double);
    const uint64_t K = static_cast<uint64_t>(std::floor(k * N + 0.5));
    // workspace, then per block (U, D) the gather tables and up to two plans per precision
    // (the planner's layout and the standard one)
    const uint64_t dev = otoc_workspace_bytes(n, m, e) + 2 * (tables_bound(K) + 4 * plan_bound(L, K));
    return align_up(dev, kRegionAlign);
}

// First-fit allocator of regions of one device allocation; free ranges are merged with
// their neighbours when returned.  Host bookkeeping only (the caller holds the engine lock).
class Arena {
  public:
    void init(uint64_t bytes) {
        size_ = bytes / kRegionAlign * kRegionAlign;
        if (size_ == 0) fail(SYK_EINVAL, "engine budget below one 64 KiB region");
        void *p = nullptr;
        SYK_HIP(hipMalloc(&p, size_));
        base_ = static_cast<char *>(p);
        free_[0] = size_;
    }
    ~Arena() {
        if (base_) ignore_status(hipFree(base_));
    }
    uint64_t size() const { return size_; }
    char *base() const { return base_; }
    // offset of a free region of `bytes` (a multiple of kRegionAlign), or false
    bool take(uint64_t bytes, uint64_t &off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return true;
        }
        return false;
    }
    void give(uint64_t off, uint64_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    char *base_ = nullptr;
    uint64_t size_ = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> bytes
};

struct Req {
    uint64_t id = 0;
    syk_request r{};
    std::vector<double> t;
    int m_used = 0;
    uint64_t footprint = 0;
    uint64_t offset = 0;        // of its arena region (valid while it runs)
    double t_submit = 0, t_start = 0;
    int bypassed = 0;
    std::atomic<int> cancel{0};
};

struct Done {
    syk_result_info info{};
    std::vector<double> raw, norm, imag;
};

}  // namespace

struct Engine::Impl {
    int dev = 0;
    uint64_t budget = 0, in_use = 0, peak = 0;
    Arena arena;
    int max_active = 4, max_bypass = 8;
    Clock::time_point t0 = Clock::now();

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Req>> pending;
    std::map<uint64_t, std::shared_ptr<Req>> running;
    std::deque<Done> done;
    std::vector<double> latencies;
    long long submitted = 0, completed = 0, failed = 0, cancelled = 0;
    double busy = 0, busy_since = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> workers;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    // caller holds mu; an admitted request leaves with its arena region taken
    std::shared_ptr<Req> pick() {
        if (pending.empty()) return nullptr;
        auto &head = pending.front();
        if (arena.take(head->footprint, head->offset)) {
            auto r = head;
            pending.pop_front();
            return r;
        }
        if (head->bypassed >= max_bypass) return nullptr;
        for (auto it = pending.begin() + 1; it != pending.end(); ++it) {
            if (arena.take((*it)->footprint, (*it)->offset)) {
                auto r = *it;
                pending.erase(it);
                ++head->bypassed;
                return r;
            }
        }
        return nullptr;
    }

    void set_active_changed(int before, int after) {
        const double t = now();
        if (before == 0 && after > 0) busy_since = t;
        if (before > 0 && after == 0) busy += t - busy_since;
    }

    Done run(Req &q, hipStream_t s) {
        Done d;
        d.info.id = q.id;
        d.info.nt = q.r.nt;
        d.info.m_used = q.m_used;
        d.info.footprint_bytes = q.footprint;
        d.info.t_submit = q.t_submit;
        d.info.t_start = q.t_start;
        d.raw.assign(q.r.nt, 0.0);
        d.norm.assign(q.r.nt, 0.0);
        d.imag.assign(q.r.nt, 0.0);
        try {
            // the request's region: its workspace first, then its tables and plans
            DeviceSlab slab;
            slab.base = arena.base() + q.offset;
            slab.size = q.footprint;
            const size_t e = (q.r.dtype == SYK_C64 && !q.r.precision_check) ? sizeof(float) : sizeof(double);
            const size_t ws_bytes = otoc_workspace_bytes(1ULL << (q.r.N / 2 - 1), q.m_used, e);
            DeviceBuffer ws;
            ws.adopt(slab.take(ws_bytes, "workspace"), ws_bytes);
            Hamiltonian h;
            build_hamiltonian(h, q.r.N, q.r.k, q.r.seed);
            h.slab = &slab;
            syk_otoc_opts o{};
            o.nvec = q.r.nvec;
            o.state_seed = q.r.state_seed;
            o.dtype = q.r.dtype;
            syk_krylov_default_opts(q.r.dtype, &o.krylov);
            o.krylov.m = q.m_used;
            if (q.r.tol > 0.0) o.krylov.tol = q.r.tol;
            o.layout = -1;
            o.autotune = 0;
            o.precision_check = q.r.precision_check;
            syk_otoc_stats st{};
            const auto c0 = Clock::now();
            otoc_compute(h, q.r.i, q.r.j, q.r.beta, q.t.data(), q.r.nt, o, ws, s, d.raw.data(), d.norm.data(),
                         d.imag.data(), st, &q.cancel);
            SYK_HIP(hipStreamSynchronize(s));
            st.seconds = std::chrono::duration<double>(Clock::now() - c0).count();
            d.info.stats = st;
            d.info.status = SYK_OK;
        } catch (const Error &e) {
            d.info.status = e.status;
            ignore_status(hipStreamSynchronize(s));
        } catch (const std::bad_alloc &) {
            d.info.status = SYK_ENOMEM;
            ignore_status(hipStreamSynchronize(s));
        } catch (...) {
            d.info.status = SYK_EDEVICE;
            ignore_status(hipStreamSynchronize(s));
        }
        if (d.info.status != SYK_OK) {
            d.raw.assign(q.r.nt, 0.0);
            d.norm.assign(q.r.nt, 0.0);
            d.imag.assign(q.r.nt, 0.0);
        }
        return d;
    }

    void worker() {
        if (hipSetDevice(dev) != hipSuccess) return;
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
        for (;;) {
            std::shared_ptr<Req> q;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || (q = pick()) != nullptr; });
                if (!q) break;                       // stop requested, nothing admitted
                in_use += q->footprint;
                peak = std::max(peak, in_use);
                const int before = static_cast<int>(running.size());
                running[q->id] = q;
                set_active_changed(before, before + 1);
                q->t_start = now();
            }
            Done d = run(*q, s);           // returns with the stream drained
            {
                std::lock_guard<std::mutex> lk(mu);
                arena.give(q->offset, q->footprint);
                in_use -= q->footprint;
                const int before = static_cast<int>(running.size());
                running.erase(q->id);
                set_active_changed(before, before - 1);
                d.info.t_end = now();
                if (d.info.status == SYK_OK) {
                    ++completed;
                    latencies.push_back(d.info.t_end - d.info.t_submit);
                } else if (d.info.status == SYK_ECANCELLED) {
                    ++cancelled;
                } else {
                    ++failed;
                }
                done.push_back(std::move(d));
            }
            cv_done.notify_all();
            cv_work.notify_all();                    // memory returned: others may fit now
        }
        ignore_status(hipStreamDestroy(s));
    }
};

Engine::Engine(const syk_engine_opts &o) : p_(new Impl) {
    SYK_HIP(hipGetDevice(&p_->dev));
    uint64_t budget = o.budget_bytes;
    if (budget == 0) {
        size_t free_b = 0, total_b = 0;
        SYK_HIP(hipMemGetInfo(&free_b, &total_b));
        budget = static_cast<uint64_t>(0.85 * static_cast<double>(free_b));
    }
    p_->arena.init(budget);
    p_->budget = p_->arena.size();
    p_->max_active = o.max_active > 0 ? o.max_active : 4;
    p_->max_bypass = o.max_bypass >= 0 ? o.max_bypass : 8;
    for (int w = 0; w < p_->max_active; ++w) p_->workers.emplace_back([this] { p_->worker(); });
}

Engine::~Engine() {
    {
        std::lock_guard<std::mutex> lk(p_->mu);
        p_->stop = true;
        p_->pending.clear();
        for (auto &kv : p_->running) kv.second->cancel.store(1);
    }
    p_->cv_work.notify_all();
    for (auto &t : p_->workers) t.join();
}

uint64_t Engine::submit(const syk_request &r) {
    auto require = [](bool c, const char *msg) {
        if (!c) fail(SYK_EINVAL, msg);
    };
    require(r.N % 2 == 0 && r.N >= 6 && r.N <= 64, "N must be even with 6 <= N <= 64");
    require(std::isfinite(r.k) && r.k > 0.0, "k must be positive");
    const double K = std::floor(r.k * r.N + 0.5);
    const double nsub = static_cast<double>(r.N) * (r.N - 1) * (r.N - 2) * (r.N - 3) / 24.0;
    require(K >= 1.0 && K <= nsub, "K = round(k N) must lie in [1, C(N,4)]");
    syk_otoc_opts o{};
    o.nvec = r.nvec;
    o.state_seed = r.state_seed;
    o.dtype = r.dtype;
    require(r.dtype == SYK_C64 || r.dtype == SYK_C128, "invalid dtype");
    syk_krylov_default_opts(r.dtype, &o.krylov);
    const int m = r.m > 0 ? r.m : 30;
    const int m_min = r.m_min > 0 ? r.m_min : std::min(m, 8);
    require(m_min <= m, "m_min must not exceed m");
    o.krylov.m = m;
    if (r.tol > 0.0) o.krylov.tol = r.tol;
    o.layout = -1;
    o.precision_check = r.precision_check;
    check_otoc_args(r.N, r.i, r.j, r.beta, r.t, r.nt, o);
    o.krylov.m = m_min;
    check_krylov_opts(o.krylov);

    auto q = std::make_shared<Req>();
    q->r = r;
    q->t.assign(r.t, r.t + r.nt);
    q->r.t = nullptr;
    q->m_used = m;
    std::lock_guard<std::mutex> lk(p_->mu);
    if (p_->stop) fail(SYK_EINVAL, "engine is shutting down");
    const bool pc = r.precision_check != 0;
    while (q->m_used > m_min && footprint_bytes(r.N, r.k, q->m_used, r.dtype, pc) > p_->budget) --q->m_used;
    q->footprint = footprint_bytes(r.N, r.k, q->m_used, r.dtype, pc);
    if (q->footprint > p_->budget) fail(SYK_ENOMEM, "request footprint at m_min exceeds the engine budget");
    q->id = p_->next_id++;
    q->t_submit = p_->now();
    p_->pending.push_back(q);
    ++p_->submitted;
    p_->cv_work.notify_all();
    return q->id;
}

syk_status Engine::poll(int wait_ms, syk_result_info &info, double *raw, double *norm, double *imag, int cap) {
    std::unique_lock<std::mutex> lk(p_->mu);
    auto ready = [&] { return !p_->done.empty(); };
    if (wait_ms < 0) {
        p_->cv_done.wait(lk, [&] { return ready() || (p_->pending.empty() && p_->running.empty()); });
    } else if (wait_ms > 0) {
        p_->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    }
    if (!ready()) return SYK_EAGAIN;
    Done &d = p_->done.front();
    if (cap < d.info.nt) return SYK_EINVAL;
    info = d.info;
    for (int k = 0; k < d.info.nt; ++k) {
        if (raw) raw[k] = d.raw[k];
        if (norm) norm[k] = d.norm[k];
        if (imag) imag[k] = d.imag[k];
    }
    p_->done.pop_front();
    return SYK_OK;
}

void Engine::cancel(uint64_t id) {
    {
        std::lock_guard<std::mutex> lk(p_->mu);
        auto rit = p_->running.find(id);
        if (rit != p_->running.end()) {
            rit->second->cancel.store(1);
            return;
        }
        for (auto it = p_->pending.begin(); it != p_->pending.end(); ++it) {
            if ((*it)->id != id) continue;
            Done d;
            d.info.id = id;
            d.info.status = SYK_ECANCELLED;
            d.info.nt = (*it)->r.nt;
            d.info.m_used = (*it)->m_used;
            d.info.footprint_bytes = (*it)->footprint;
            d.info.t_submit = (*it)->t_submit;
            d.info.t_start = d.info.t_end = p_->now();
            d.raw.assign(d.info.nt, 0.0);
            d.norm.assign(d.info.nt, 0.0);
            d.imag.assign(d.info.nt, 0.0);
            p_->pending.erase(it);
            ++p_->cancelled;
            p_->done.push_back(std::move(d));
            p_->cv_done.notify_all();
            p_->cv_work.notify_all();
            return;
        }
    }
    fail(SYK_EINVAL, "unknown or finished request id");
}

void Engine::stats(syk_engine_stats &st) {
    std::lock_guard<std::mutex> lk(p_->mu);
    st = syk_engine_stats{};
    st.submitted = p_->submitted;
    st.completed = p_->completed;
    st.failed = p_->failed;
    st.cancelled = p_->cancelled;
    st.queued = static_cast<int>(p_->pending.size());
    st.active = static_cast<int>(p_->running.size());
    st.budget_bytes = p_->budget;
    st.bytes_in_use = p_->in_use;
    st.peak_bytes = p_->peak;
    st.busy_seconds = p_->busy + (p_->running.empty() ? 0.0 : p_->now() - p_->busy_since);
    std::vector<double> l = p_->latencies;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        // nearest-rank percentiles
        auto pct = [&](double q) {
            size_t r = static_cast<size_t>(std::ceil(q * static_cast<double>(l.size())));
            r = std::min(std::max<size_t>(r, 1), l.size());
            return l[r - 1];
        };
        st.p50_latency_s = pct(0.50);
        st.p99_latency_s = pct(0.99);
    }
}

}  // namespace syk
