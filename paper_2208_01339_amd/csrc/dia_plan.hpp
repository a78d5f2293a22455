// Host-side choice of the symmetric stored diagonals from an offset histogram.
#pragma once
#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "kernels.hpp"

// key/cnt: the OFF_SLOTS-entry table k_offsets filled (nonzero entries per
// column offset) for a matrix of n rows.  A stored diagonal costs 8n bytes
// and the slice layout 12 bytes per entry, so the diagonal (offset 0) and
// each offset pair +-o are kept when they cover more than 2n/3 entries; an
// offset whose mirror count differs is unpaired (the matrix is not
// symmetric there) and stays in the slice layout.  At most DMAX diagonals,
// the most populated first.  nd = 0: no diagonal part.
inline ppk::DiaSet choose_diagonals(const unsigned long long *key, const unsigned long long *cnt, int64_t n)
{
    typedef unsigned long long u64;
    ppk::DiaSet D;
    std::vector<std::pair<int64_t, u64>> count;  // (offset, entries)
    for (int q = 0; q < ppk::OFF_SLOTS; ++q)
        if (key[q] != ppk::OFF_EMPTY) count.push_back({(int64_t)key[q], cnt[q]});
    auto entries = [&](int64_t o) -> u64 {
        for (auto &c : count)
            if (c.first == o) return c.second;
        return 0;
    };
    if (3 * entries(0) <= 2 * (u64)n) return D;
    std::vector<std::pair<u64, int64_t>> cand;  // (entries covered, offset > 0)
    for (auto &c : count) {
        if (c.first <= 0 || entries(-c.first) != c.second) continue;
        const u64 cov = 2 * c.second;
        if (3 * cov > 2 * (u64)n) cand.push_back({cov, c.first});
    }
    std::sort(cand.begin(), cand.end(), [](const std::pair<u64, int64_t> &a, const std::pair<u64, int64_t> &b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
    });
    if ((int)cand.size() > ppk::DMAX - 1) cand.resize(ppk::DMAX - 1);
    std::vector<int64_t> offs{0};
    for (auto &c : cand) offs.push_back(c.second);
    std::sort(offs.begin(), offs.end());
    D.nd = (int)offs.size();
    for (int d = 0; d < D.nd; ++d) D.off[d] = offs[d];
    return D;
}
