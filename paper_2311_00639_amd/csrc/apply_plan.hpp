// Host-built launch plan of the tiled apply_H kernel: terms grouped by partner tile.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace syk {

// host description of a plan (see apply_plan.cpp).  A workgroup holds the 2^w output
// tiles t0 ^ hvec[i]; for each partner offset pi (partner tile t0 ^ pi) it applies the
// term group g = pi ^ hvec[i] to tile i, whose records are [first, mid) (real phase) and
// [mid, end) (i phase) at ranges[(step * 2^w + i) * 3].
// record form 2: dwords per record (4 + one more for a double coefficient) and records per
// 64-dword control block (lanes 0..59 hold records, 60 and 62 the counts, 61 the next partner)
inline uint32_t block_record_dwords(uint32_t elem_bytes) { return elem_bytes == 8 ? 4u : 5u; }
inline uint32_t block_records(uint32_t elem_bytes) { return 60u / block_record_dwords(elem_bytes); }

struct HostPlan {
    int rot = 0, w = 0;
    uint32_t n_tiles = 0, n_wg = 0;
    int n_pi = 0;           // padded count; pi holds n_pi + pf entries
    int D = 0, n_partners = 0, classes_xcd = 0, classes_gpu = 0, res_bits = 5;
    std::vector<uint32_t> hvec, pi, ranges, meta, tile_map;
    std::vector<double> c;
};

// rotation s minimising the modelled L2 traffic of the tiled kernel for these terms, with
// 2^res_bits workgroups resident per XCD, each holding 2^w tiles
int choose_rotation(const std::vector<BlockTerm> &terms, int L, int bt, int res_bits, int w);
// partner steps padded to a multiple of `mult`; pi gets `extra` more entries (targets of
// the last prefetches); elem_bytes: bytes per complex amplitude (8 or 16), for the LDS
// offsets in the term records; sr: register-static record form
HostPlan build_host_plan(const std::vector<BlockTerm> &terms, int L, int bt, int rb, int mult, int extra, int s,
                         uint32_t elem_bytes, int res_bits, int sr, int w);
// device copies of a host plan: hipMalloc'ed, or carved from `slab` when it is not null
void upload_plan(const HostPlan &hp, int bt, int rb, ApplyPlan &out, DeviceSlab *slab = nullptr);
void free_plan(ApplyPlan &p);

template <typename T>
void launch_apply_tiled(const ApplyPlan &pl, const T *x, T *y, int nvec, uint64_t ld, hipStream_t s,
                        const LanczosFuse<T> *lf = nullptr);

}  // namespace syk
