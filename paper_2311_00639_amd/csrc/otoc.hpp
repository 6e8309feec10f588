// OTOC driver (host side).
#pragma once

#include <complex>
#include <vector>

#include "internal.hpp"

namespace syk {

size_t otoc_workspace_bytes(uint64_t n, int m, size_t elem_bytes);

template <typename T>
void apply_gamma(int N, int n, int src, int rot, const T *x, T *y, uint64_t amps, hipStream_t s);

// F[k] = mean over vectors of F_v(ts[k]) (complex); ws: otoc_workspace_bytes(2^L, m, sizeof(T))
template <typename T>
void otoc_run(Hamiltonian &h, int i, int j, double beta, const std::vector<double> &ts, const syk_otoc_opts &o,
              std::vector<std::complex<double>> &F, syk_otoc_stats &st, char *ws, hipStream_t s);

}  // namespace syk
