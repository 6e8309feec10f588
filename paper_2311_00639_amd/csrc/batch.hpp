// Batched OTOC (one persistent launch over many small-N realisations and random vectors).
#pragma once

#include <vector>

#include "internal.hpp"

namespace syk {

constexpr int kMaxKrylov = 60;          // largest Krylov dimension of the batched path

// one term of a block in kernel form: y[m] += c i^imag (-1)^{popc(m & z)} x[m ^ x]
struct BatchTerm {
    uint32_t x, z;
    float c;
    uint32_t imag;
};

// one job: a realisation and one Haar vector, both block chains over the whole t grid
struct BatchJob {
    int L, N, K, pad;
    uint32_t term_off[2];               // first term of block U / D in BatchParams::terms
    uint32_t wx, wz;                    // W = chi_i block form (x, z, phase i^ww), w_top: i == N - 1
    int ww, w_top;
    uint32_t vx, vz;                    // V = chi_j
    int vw, v_top;
    uint64_t base;                      // Haar generator base of this vector
    double beta;
    // each block's terms are sorted by x; gstart[blk][g] = first term with x >> 12 >= g
    // (g <= 8; gstart[blk][8] = K), so the terms of one partner chunk are contiguous
    uint16_t gstart[2][9];
    uint16_t pad2[2];
};

struct BatchParams {
    const BatchJob *jobs;
    int n_jobs;
    const BatchTerm *terms;
    const double *ts;                   // t grid (t[0] = 0)
    int nt;
    int m;                              // Krylov dimension
    double tol;
    int max_substeps;                   // per job, over all propagations
    float2 *ws;                         // per slot: (m + 5) vectors of vec_stride amplitudes
    uint64_t slot_stride, vec_stride;   // in amplitudes
    double *F;                          // per job: nt complex (re, im)
    unsigned *counter;                  // next job; zero at launch
    int *status;                        // per job: 0, SYK_ENOTCONV, SYK_ENUMERIC, SYK_EUNSUPPORTED
    long long *matvecs;                 // per job
};

// launch shape: threads per workgroup, LDS staging chunk 2^chb amplitudes, workgroups per CU
struct BatchVariant {
    int nt, chb, occ;
};
const std::vector<BatchVariant> &batch_variants();
bool batch_variant_supports(const BatchVariant &v, int L);
void launch_otoc_batch(const BatchVariant &v, const BatchParams &p, int grid, hipStream_t s);

// the whole batched request (arguments checked by the caller); synchronises s
void otoc_batch(const syk_batch_item *items, int n_items, const double *t, int nt, const syk_batch_opts &o,
                double *F_raw, double *F_norm, double *F_imag, syk_batch_stats &st, hipStream_t s);

}  // namespace syk
