// Tile schedule of the streaming triangular product (host code only, no
// HIP headers, so it also builds with a plain C++ compiler).
//
// A launch runs one workgroup per schedule entry; entry b holds
// (row tile | context << SCHED_CTX_SHIFT, column tile) or (-1, -1) for an
// idle workgroup.  Workgroup b of a launch runs on XCD b % 8 of the MI355X,
// and each XCD has its own L2, so the schedule decides which tiles share an
// L2: row tiles are taken in groups of consecutive rows, the groups are
// dealt to the XCDs longest first (least-loaded XCD next), and inside a
// group all its row tiles run one chunk of column tiles together.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace gwas {

constexpr int SCHED_CTX_SHIFT = 20;
constexpr int SCHED_ROW_MASK = (1 << SCHED_CTX_SHIFT) - 1;

// tm x tn tile; part_rows rows per partial-sum slice; threads per workgroup;
// rgroup row tiles per L2 group of the schedule; inflight workgroups one XCD
// runs at once.
struct TrmmShape { int tm, tn, part_rows, threads, rgroup, inflight; };

// Row tiles per L2 group.  A workgroup streams A_BYTES per unit of K from
// its L^-1 panel and B_BYTES from its dosage panel; R row tiles x C column
// tiles in flight together on one XCD (R * C = the workgroups that XCD runs
// at once) fetch R * A_BYTES + C * B_BYTES from beyond L2 per unit of K,
// smallest at R = sqrt(inflight * B_BYTES / A_BYTES); R is that rounded
// down to a power of two (on MI355X the rounded-up group was never faster).
inline int row_group_for(int64_t a_bytes, int64_t b_bytes, int inflight) {
    const double r = std::sqrt((double)inflight * (double)b_bytes / (double)a_bytes);
    int g = 1;
    while (g < inflight && (double)(2 * g) <= r * (1.0 + 1e-9)) g *= 2;
    return g;
}

// Schedule of nctx contexts with nrb[c] row tiles each (row tile I of a
// triangular product runs I + 1 tiles of K) and cols SNP columns, all with
// the tiles of sh.  Returns the number of workgroups, 8 times the longest
// XCD list; fills *out (2 ints per workgroup) unless out is null.
inline int64_t trmm_schedule_multi(const int64_t* nrb, int nctx, int64_t cols, const TrmmShape& sh,
                                   std::vector<int>* out) {
    const int64_t ncb = (cols + sh.tn - 1) / sh.tn;
    int64_t total_rows = 0;
    for (int c = 0; c < nctx; ++c) total_rows += nrb[c];
    if (nctx == 1 && total_rows < 16) {
        // too few row tiles to deal over the XCDs: longest rows first
        if (out) {
            out->assign((size_t)(2 * total_rows * ncb), -1);
            int64_t b = 0;
            for (int64_t I = total_rows - 1; I >= 0; --I)
                for (int64_t J = 0; J < ncb; ++J, ++b) {
                    (*out)[2 * b] = (int)I;
                    (*out)[2 * b + 1] = (int)J;
                }
        }
        return total_rows * ncb;
    }
    // groups of R consecutive row tiles of one context, at least two groups
    // per XCD
    const int64_t R = std::max<int64_t>(1, std::min<int64_t>(sh.rgroup, total_rows / 16));
    const int64_t C = std::max<int64_t>(1, sh.inflight / R);
    struct Group { int64_t work; int ctx; int64_t top, rows; };
    std::vector<Group> groups;
    for (int c = 0; c < nctx; ++c)
        for (int64_t top = nrb[c] - 1; top >= 0; top -= R) {
            const int64_t rows = std::min<int64_t>(R, top + 1);
            int64_t w = 0;   // K tiles of the triangular rows top-rows+1 .. top
            for (int64_t I = top; I > top - rows; --I) w += I + 1;
            groups.push_back(Group{w, c, top, rows});
        }
    std::stable_sort(groups.begin(), groups.end(),
                     [](const Group& a, const Group& b) { return a.work > b.work; });
    // Workgroup b runs on XCD b % 8: deal the groups, longest first, to the
    // least loaded XCD
    std::vector<std::vector<int>> lists(8);
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t len[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t g = 0; g < groups.size(); ++g) {
        const int x = (int)(std::min_element(load, load + 8) - load);
        load[x] += groups[g].work;
        len[x] += groups[g].rows * ncb;
        lists[x].push_back((int)g);
    }
    const int64_t per = *std::max_element(len, len + 8);
    if (out) {
        out->assign((size_t)(2 * 8 * per), -1);
        for (int x = 0; x < 8; ++x) {
            int64_t q = 0;
            // within a group: column chunks of C tiles, each run by all R
            // row tiles, so R x C workgroups stream shared panels together
            for (int g : lists[x]) {
                const Group& G = groups[(size_t)g];
                for (int64_t j0 = 0; j0 < ncb; j0 += C)
                    for (int64_t I = G.top; I > G.top - G.rows; --I)
                        for (int64_t J = j0; J < std::min(ncb, j0 + C); ++J, ++q) {
                            (*out)[2 * (8 * q + x)] = (int)(I | ((int64_t)G.ctx << SCHED_CTX_SHIFT));
                            (*out)[2 * (8 * q + x) + 1] = (int)J;
                        }
            }
        }
    }
    return 8 * per;
}

}  // namespace gwas
