// Host-built launch plan of the tiled apply_H kernel: terms grouped by partner tile.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace syk {

// host description of a plan (see apply_plan.cpp)
struct HostPlan {
    int rot = 0;
    uint32_t n_tiles = 0;
    int n_groups = 0;       // padded count; grp_g holds n_groups + pf entries
    int D = 0, classes_xcd = 0, classes_gpu = 0, res_bits = 5;
    std::vector<uint32_t> grp_g, grp_first, grp_mid, meta, tile_map;
    std::vector<double> c;
};

// rotation s minimising the modelled L2 traffic of the tiled kernel for these terms, with
// 2^res_bits workgroups resident per XCD
int choose_rotation(const std::vector<BlockTerm> &terms, int L, int bt, int res_bits);
// groups padded with empty ones to a multiple of `mult`; grp_g gets `extra` more entries
// (targets of the last prefetches); elem_bytes: bytes per complex amplitude (8 or 16), for
// the LDS offsets in the term records
HostPlan build_host_plan(const std::vector<BlockTerm> &terms, int L, int bt, int rb, int mult, int extra, int s,
                         uint32_t elem_bytes, int res_bits);
void upload_plan(const HostPlan &hp, int bt, int rb, ApplyPlan &out);
void free_plan(ApplyPlan &p);

template <typename T>
void launch_apply_tiled(const ApplyPlan &pl, const T *x, T *y, int nvec, uint64_t ld, hipStream_t s,
                        const LanczosFuse<T> *lf = nullptr);

}  // namespace syk
