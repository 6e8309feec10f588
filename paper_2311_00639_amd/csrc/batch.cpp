// Host driver of the batched OTOC: term tables and jobs of many realisations, launch-shape
// choice (timed on a sample of the batch), one persistent launch, per-realisation
// averaging over vectors and normalisation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "batch.hpp"

namespace syk {

namespace {

template <typename U>
struct DevArray {
    U *p = nullptr;
    explicit DevArray(size_t n) { SYK_HIP(hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(n, 1) * sizeof(U))); }
    ~DevArray() { ignore_status(hipFree(p)); }
    DevArray(const DevArray &) = delete;
    DevArray &operator=(const DevArray &) = delete;
};

void majorana_form(int N, int n, uint32_t &x, uint32_t &z, int &w, int &top) {
    if (n == N - 1) {
        x = z = 0;
        w = 0;
        top = 1;
    } else {
        block_majorana(N, n, x, z, w);
        top = 0;
    }
}

struct Launch {
    const BatchVariant *v;
    int grid;
};

int device_cus() {
    int dev = 0, cus = 0;
    SYK_HIP(hipGetDevice(&dev));
    SYK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(cus, 1);
}

// run jobs [0, n_jobs) of `jobs_d` with variant v; returns kernel milliseconds
float run_once(const BatchVariant &v, BatchParams p, int n_jobs, int lmax, hipStream_t s, std::vector<char> &hold,
               float2 *&ws, size_t &ws_cap, unsigned *counter) {
    const int grid = std::min(n_jobs, device_cus() * v.occ);
    p.n_jobs = n_jobs;
    p.vec_stride = std::max<uint64_t>(1ULL << lmax, 64);
    p.slot_stride = static_cast<uint64_t>(p.m + 5) * p.vec_stride;
    const size_t need = static_cast<size_t>(grid) * p.slot_stride * sizeof(float2);
    if (need > ws_cap) {
        if (ws) SYK_HIP(hipFree(ws));
        ws = nullptr;
        ws_cap = 0;
        SYK_HIP(hipMalloc(reinterpret_cast<void **>(&ws), need));
        ws_cap = need;
    }
    p.ws = ws;
    p.counter = counter;
    SYK_HIP(hipMemsetAsync(counter, 0, sizeof(unsigned), s));
    hipEvent_t e0, e1;
    SYK_HIP(hipEventCreate(&e0));
    SYK_HIP(hipEventCreate(&e1));
    SYK_HIP(hipEventRecord(e0, s));
    launch_otoc_batch(v, p, grid, s);
    SYK_HIP(hipEventRecord(e1, s));
    SYK_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    const hipError_t te = hipEventElapsedTime(&ms, e0, e1);
    ignore_status(hipEventDestroy(e0));
    ignore_status(hipEventDestroy(e1));
    SYK_HIP(te);
    (void)hold;
    return ms;
}

}  // namespace

void otoc_batch(const syk_batch_item *items, int n_items, const double *t, int nt, const syk_batch_opts &o,
                double *F_raw, double *F_norm, double *F_imag, syk_batch_stats &st, hipStream_t s) {
    const auto t_start = std::chrono::steady_clock::now();
    std::vector<double> ts(t, t + nt);
    const bool prepend = ts[0] != 0.0;
    if (prepend) ts.insert(ts.begin(), 0.0);
    const int ntt = static_cast<int>(ts.size());

    // term tables and jobs
    std::vector<BatchTerm> terms;
    std::vector<BatchJob> jobs;
    int lmax = 0;
    for (int r = 0; r < n_items; ++r) {
        const syk_batch_item &it = items[r];
        Hamiltonian h;
        build_hamiltonian(h, it.N, it.k, it.seed, it.ensemble);
        BatchJob jb{};
        jb.L = h.L;
        jb.N = h.N;
        jb.K = h.K;
        lmax = std::max(lmax, h.L);
        for (int blk = 0; blk < 2; ++blk) {
            jb.term_off[blk] = static_cast<uint32_t>(terms.size());
            std::vector<BatchTerm> bts;
            for (const BlockTerm &bt : h.block_terms[blk])
                bts.push_back(BatchTerm{bt.x, bt.z, static_cast<float>(bt.c), bt.imag ? 1u : 0u});
            std::stable_sort(bts.begin(), bts.end(), [](const BatchTerm &a, const BatchTerm &b) { return a.x < b.x; });
            for (uint32_t g = 0, t = 0; g <= 8; ++g) {
                while (t < bts.size() && (bts[t].x >> 12) < g) ++t;
                jb.gstart[blk][g] = static_cast<uint16_t>(g == 8 ? bts.size() : t);
            }
            terms.insert(terms.end(), bts.begin(), bts.end());
        }
        majorana_form(it.N, it.i, jb.wx, jb.wz, jb.ww, jb.w_top);
        majorana_form(it.N, it.j, jb.vx, jb.vz, jb.vw, jb.v_top);
        jb.beta = o.beta;
        for (int v = 0; v < o.nvec; ++v) {
            jb.base = splitmix_mix(it.state_seed + static_cast<uint64_t>(v + 1) * 0x9E3779B97F4A7C15ULL);
            jobs.push_back(jb);
        }
    }
    const int n_jobs = static_cast<int>(jobs.size());

    // eligible launch shapes
    std::vector<int> elig;
    const auto &vars = batch_variants();
    for (int v = 0; v < static_cast<int>(vars.size()); ++v) {
        bool ok = true;
        for (int r = 0; r < n_items && ok; ++r) ok = batch_variant_supports(vars[v], items[r].N / 2 - 1);
        if (ok) elig.push_back(v);
    }
    if (elig.empty()) fail(SYK_EUNSUPPORTED, "no batched launch shape serves this mix of block sizes");
    if (o.variant >= 0 && std::find(elig.begin(), elig.end(), o.variant) == elig.end())
        fail(SYK_EINVAL, "requested batch variant does not serve this mix of block sizes");

    DevArray<BatchJob> jobs_d(jobs.size());
    DevArray<BatchTerm> terms_d(terms.size());
    DevArray<double> ts_d(ts.size());
    DevArray<double> F_d(static_cast<size_t>(n_jobs) * ntt * 2);
    DevArray<unsigned> counter(1);
    DevArray<int> status_d(jobs.size());
    DevArray<long long> mv_d(jobs.size());
    SYK_HIP(hipMemcpy(jobs_d.p, jobs.data(), jobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice));
    SYK_HIP(hipMemcpy(terms_d.p, terms.data(), terms.size() * sizeof(BatchTerm), hipMemcpyHostToDevice));
    SYK_HIP(hipMemcpy(ts_d.p, ts.data(), ts.size() * sizeof(double), hipMemcpyHostToDevice));

    BatchParams p{};
    p.jobs = jobs_d.p;
    p.terms = terms_d.p;
    p.ts = ts_d.p;
    p.nt = ntt;
    p.m = o.m;
    p.tol = o.tol;
    p.max_substeps = o.max_substeps > 0 ? o.max_substeps : 20000;
    p.F = F_d.p;
    p.status = status_d.p;
    p.matvecs = mv_d.p;
    float2 *ws = nullptr;
    size_t ws_cap = 0;
    std::vector<char> hold;
    try {
        int chosen = o.variant >= 0 ? o.variant : elig[0];
        st.tuned_ms[0] = st.tuned_ms[1] = st.tuned_ms[2] = -1.0;
        if (o.variant < 0 && elig.size() > 1) {
            // time each shape on a sample of the batch (its first jobs, the first two t points)
            BatchParams q = p;
            q.nt = std::min(ntt, 2);
            const int sample = std::min(n_jobs, 2 * device_cus());
            float best = 1e30f;
            for (int v : elig) {
                const float ms = run_once(vars[v], q, sample, lmax, s, hold, ws, ws_cap, counter.p);
                if (v < 3) st.tuned_ms[v] = ms;
                if (ms < best) {
                    best = ms;
                    chosen = v;
                }
            }
        }
        st.variant = chosen;
        st.kernel_ms = run_once(vars[chosen], p, n_jobs, lmax, s, hold, ws, ws_cap, counter.p);
        st.slots = std::min(n_jobs, device_cus() * vars[chosen].occ);
    } catch (...) {
        if (ws) ignore_status(hipFree(ws));
        throw;
    }
    SYK_HIP(hipFree(ws));
    std::vector<double> F(static_cast<size_t>(n_jobs) * ntt * 2);
    std::vector<int> status(jobs.size());
    std::vector<long long> mv(jobs.size());
    SYK_HIP(hipMemcpy(F.data(), F_d.p, F.size() * sizeof(double), hipMemcpyDeviceToHost));
    SYK_HIP(hipMemcpy(status.data(), status_d.p, status.size() * sizeof(int), hipMemcpyDeviceToHost));
    SYK_HIP(hipMemcpy(mv.data(), mv_d.p, mv.size() * sizeof(long long), hipMemcpyDeviceToHost));
    st.matvecs = 0;
    for (int j = 0; j < n_jobs; ++j) {
        st.matvecs += mv[j];
        if (status[j] == SYK_ENOTCONV) fail(SYK_ENOTCONV, "batched Krylov propagation did not converge");
        if (status[j] == SYK_ENUMERIC) fail(SYK_ENUMERIC, "non-finite value in a batched job");
        if (status[j] != 0) fail(SYK_EUNSUPPORTED, "batched job with an unsupported block size");
    }
    // per realisation: mean over vectors, normalised by t = 0
    const int off = prepend ? 1 : 0;
    for (int r = 0; r < n_items; ++r) {
        std::vector<std::complex<double>> acc(ntt, 0.0);
        for (int v = 0; v < o.nvec; ++v) {
            const double *f = F.data() + static_cast<size_t>(r * o.nvec + v) * ntt * 2;
            for (int k = 0; k < ntt; ++k) acc[k] += std::complex<double>(f[2 * k], f[2 * k + 1]);
        }
        for (auto &a : acc) a /= static_cast<double>(o.nvec);
        const double f0 = acc[0].real();
        for (int k = 0; k < nt; ++k) {
            const auto f = acc[k + off];
            if (F_raw) F_raw[static_cast<size_t>(r) * nt + k] = f.real();
            if (F_imag) F_imag[static_cast<size_t>(r) * nt + k] = f.imag();
            if (F_norm) F_norm[static_cast<size_t>(r) * nt + k] = f.real() / f0;
        }
    }
    st.n_jobs = n_jobs;
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
}

}  // namespace syk
