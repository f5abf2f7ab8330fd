// Halo structure of a level for the fused smoothing kernels (host, built once per hierarchy).
//
// Rows are grouped in blocks of `rows` consecutive rows, one workgroup per block. A smoothing
// step u' = u + Q (f - A u) needs the residual at every column its rows touch; the fused
// kernel computes it on the block's own rows and on its halo (the distinct columns outside
// the block), keeps it in LDS and applies Q from there. The lists built here let the kernel
// read the halo rows' entries as one flat, evenly shared stream.
#include "halo.hpp"

#include <algorithm>
#include <cstdint>
#include <vector>

namespace amgg {

bool build_halo(int32_t n, const int32_t* ptr, const int32_t* col, int rows, int row_cap, int ent_cap,
                size_t total_cap, HaloLists& out) {
    if (n <= 0 || rows <= 0) return false;
    const int32_t nb = (n + rows - 1) / rows;
    out.hoff.assign(static_cast<size_t>(nb) + 1, 0);
    out.heoff.assign(static_cast<size_t>(nb) + 1, 0);
    out.halo.clear();
    out.hent.clear();
    out.hend.clear();
    out.loc.assign(static_cast<size_t>(ptr[n]), 0);
    std::vector<int32_t> ext;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t r0 = b * rows, r1 = std::min(r0 + rows, n);
        ext.clear();
        for (int32_t k = ptr[r0]; k < ptr[r1]; ++k)
            if (col[k] < r0 || col[k] >= r1) ext.push_back(col[k]);
        std::sort(ext.begin(), ext.end());
        ext.erase(std::unique(ext.begin(), ext.end()), ext.end());
        if (static_cast<int>(ext.size()) > row_cap) return false;
        for (int32_t k = ptr[r0]; k < ptr[r1]; ++k) {
            const int32_t j = col[k];
            if (j >= r0 && j < r1) {
                out.loc[k] = static_cast<uint16_t>(j - r0);
            } else {
                const auto it = std::lower_bound(ext.begin(), ext.end(), j);
                out.loc[k] = static_cast<uint16_t>(rows + (it - ext.begin()));
            }
        }
        int32_t cnt = 0;
        for (const int32_t j : ext) {
            for (int32_t k = ptr[j]; k < ptr[j + 1]; ++k) out.hent.push_back(k);
            cnt += ptr[j + 1] - ptr[j];
            if (cnt > ent_cap || out.hent.size() > total_cap) return false;
            out.hend.push_back(static_cast<uint16_t>(cnt));
        }
        out.halo.insert(out.halo.end(), ext.begin(), ext.end());
        out.hoff[b + 1] = static_cast<int32_t>(out.halo.size());
        out.heoff[b + 1] = static_cast<int32_t>(out.hent.size());
    }
    return true;
}

}  // namespace amgg
