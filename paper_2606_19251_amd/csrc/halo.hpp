// Host construction of the per-block halo lists used by the fused smoothing kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace amgg {

// Blocks of `rows` consecutive rows of an n-row CSR pattern:
//   hoff[b]..hoff[b+1]   the block's halo rows in `halo` (distinct columns outside the block,
//                        ascending);
//   loc[k]               block-local slot of col[k] (own row j -> j - r0, halo row h -> rows + h);
//   heoff[b]..heoff[b+1] the block's halo entries in `hent`: the stored entries of its halo rows,
//                        row after row, as global entry indices;
//   hend[h]              end of halo row h's entries, relative to heoff[b] (its start is the
//                        previous row's end, 0 for the block's first halo row).
// Returns false (outputs unspecified) when a block has more than row_cap halo rows or ent_cap
// halo entries, or when all blocks together have more than total_cap halo entries.
struct HaloLists {
    std::vector<int32_t> hoff, halo, heoff, hent;
    std::vector<uint16_t> loc, hend;
};
bool build_halo(int32_t n, const int32_t* ptr, const int32_t* col, int rows, int row_cap, int ent_cap,
                size_t total_cap, HaloLists& out);

}  // namespace amgg
