// Request engine (continuous batching of OTOC requests on one device).
#pragma once

#include <memory>

#include "internal.hpp"

namespace syk {

class Engine {
  public:
    explicit Engine(const syk_engine_opts &o);
    ~Engine();
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;

    uint64_t submit(const syk_request &r);
    syk_status poll(int wait_ms, syk_result_info &info, double *raw, double *norm, double *imag, int cap);
    void cancel(uint64_t id);
    void stats(syk_engine_stats &st);

  private:
    struct Impl;
    std::unique_ptr<Impl> p_;
};

}  // namespace syk
