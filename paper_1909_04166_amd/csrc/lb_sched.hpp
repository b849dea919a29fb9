// lb_sched.hpp -- work lists of the step kernels: how the strips of tx - 4
// columns and the rows of one or several lattices are spread over workgroups.
// Host code only, free of HIP, so that the cut can be checked on its own.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

namespace cmlb {

// One workgroup's share of a step: rows [y0, y1) of the strip starting at
// column x0 of lattice inst.
struct WorkItem {
    int32_t inst;  // index into the descriptor array
    int32_t x0;    // first column of the strip
    int32_t y0;    // first row collided
    int32_t y1;    // one past the last row collided
};

constexpr int kMaxGrid = 16384;

// Strip width of a TX-lane workgroup: two halo lanes on each side.
inline int strip_w(int tx) { return tx - 4; }

// Work items of one lattice: strips of tx - 4 columns, runs of th rows;
// strip-major so that consecutive items are vertically adjacent (they share
// halo rows).
inline void build_items(int inst, int nx, int ny, int tx, int th, std::vector<WorkItem>& out) {
    for (int x0 = 0; x0 < nx; x0 += strip_w(tx))
        for (int y0 = 0; y0 < ny; y0 += th) out.push_back({inst, x0, y0, std::min(ny, y0 + th)});
}

struct LatShape {
    int inst, nx, ny;
};

// Balanced persistent schedule: the rows of every strip of every lattice, in
// order, are cut into G contiguous segments of nearly equal length; block b
// runs segment b as the items at positions b, b + G, b + 2G, ... (padding
// items are empty).  With exact, block b ends at row position (b + 1) * total / G
// (so when G is a multiple of the strip count, every strip is cut at the same
// rows); otherwise every block but the last takes ceil(total / G) rows.
// Returns false if more than max_items slots are needed.
inline bool build_segments(const std::vector<LatShape>& lats, int tx, int G, int max_items,
                    std::vector<WorkItem>& out, int* nblocks, bool exact = false) {
    *nblocks = 0;
    struct Strip { int inst, x0, ny; };
    std::vector<Strip> strips;
    int64_t total = 0;
    for (const auto& l : lats)
        for (int x0 = 0; x0 < l.nx; x0 += strip_w(tx)) {
            strips.push_back({l.inst, x0, l.ny});
            total += l.ny;
        }
    if (total == 0 || G <= 0) { out.clear(); return true; }
    const int64_t per = std::max<int64_t>(8, (total + G - 1) / G);
    const int nb = exact ? G : (int)std::min<int64_t>(G, (total + per - 1) / per);
    auto end_of = [&](int blk) { return exact ? (blk + 1) * total / nb : (blk + 1) * per; };
    std::vector<std::vector<WorkItem>> blocks(nb);
    int b = 0;
    int64_t pos = 0;
    for (const auto& st : strips) {
        int y = 0;
        while (y < st.ny) {
            const int take = (int)std::min<int64_t>(st.ny - y, end_of(b) - pos);
            if (take > 0) blocks[b].push_back({st.inst, st.x0, y, y + take});
            y += take;
            pos += take;
            if (pos == end_of(b) && b + 1 < nb) ++b;
        }
    }
    size_t maxj = 0;
    for (auto& bl : blocks) maxj = std::max(maxj, bl.size());
    if ((int64_t)maxj * nb > max_items) return false;
    out.assign(maxj * nb, WorkItem{0, 0, 0, 0});
    for (int i = 0; i < nb; ++i)
        for (size_t j = 0; j < blocks[i].size(); ++j) out[j * nb + i] = blocks[i][j];
    *nblocks = nb;
    return true;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Reorder each group of `grid` consecutive items so that the items one XCD
// receives are consecutive in the original order (they share halo rows in the
// XCD's L2).
inline void xcd_permute(std::vector<WorkItem>& items, int grid) {
    if (grid < 16 || grid % 8) return;
    std::vector<WorkItem> out(items.size());
    const size_t n = items.size();
    for (size_t g0 = 0; g0 < n; g0 += grid) {
        const size_t len = std::min<size_t>(grid, n - g0);
        if (len < (size_t)grid) {
            for (size_t i = 0; i < len; ++i) out[g0 + i] = items[g0 + i];
            continue;
        }
        const size_t per = grid / 8;
        for (size_t b = 0; b < len; ++b) out[g0 + b] = items[g0 + (b % 8) * per + b / 8];
    }
    items.swap(out);
}


// How a step is spread over workgroups.
//   mode 0: one work item of th rows per workgroup, grid = number of items,
//           items ordered so that each XCD gets vertically adjacent ones;
//   mode 1: persistent grid of mult * (resident workgroups per CU) * CUs, each
//           workgroup one balanced segment of the concatenated strip rows;
//   mode 2: as mode 1 for lattices of one height, with the grid cut down to
//           strips * bands, bands a multiple of 8: every strip is cut at the
//           same rows, and as block b runs on XCD b % 8, the blocks holding the
//           same rows of neighbouring strips share an XCD and read each other's
//           halo columns from its L2.
struct Sched {
    int tx = 64, th = 64, mode = 0, mult = 1, pf = 0;
    int grid = 0, n_items = 0, rows = 0;
};

// The schedule of a lattice too small to autotune: one work item per workgroup,
// rows halved from 256 until there are two items per CU (down to min_rows).  A
// small lattice's step is bound by the latency of its row loop, so the rows per
// workgroup set its time: the 128^2 droplet ran FP64 at 0.40 GLUPS with 16-row
// items, 0.86 with 8-row items prefetching, 1.89 with 2-row and 2.26 with 1-row
// items.
inline Sched small_lattice_sched(int nx, int ny, bool prefetch, int cus, int min_rows) {
    Sched sc;
    sc.tx = nx >= 1024 ? 256 : (nx >= 256 ? 128 : 64);
    sc.mode = 0;
    sc.pf = prefetch ? 1 : 0;
    const int strips = (nx + strip_w(sc.tx) - 1) / strip_w(sc.tx);
    const int64_t target = 2 * (int64_t)cus;
    sc.th = 256;
    while (sc.th > min_rows && (int64_t)strips * ((ny + sc.th - 1) / sc.th) < target) sc.th /= 2;
    return sc;
}

// Work list of a schedule over the given lattices; `resident` is the number of
// workgroups of the chosen kernel that fit on one CU, `cus` the CU count.
// Fills sc.grid, sc.rows and sc.n_items; false if the schedule does not apply
// (a strip-aligned cut over lattices of different heights, too few rows for
// eight bands) or needs more than max_items work items.
inline bool plan_schedule(const std::vector<LatShape>& lats, int resident, int cus, Sched& sc, int max_items,
                          std::vector<WorkItem>& items) {
    items.clear();
    if (sc.mode == 0) {
        for (const auto& l : lats) build_items(l.inst, l.nx, l.ny, sc.tx, sc.th, items);
        if ((int64_t)items.size() > max_items) return false;
        sc.grid = (int)items.size();
        sc.rows = sc.th;
        xcd_permute(items, sc.grid);
    } else {
        int G = sc.mult * std::max(1, resident) * cus;
        G = std::min(G, kMaxGrid);
        if (sc.mode == 2) {
            int nstrips = 0;
            for (const auto& l : lats) {
                if (l.ny != lats[0].ny) return false;
                nstrips += (l.nx + strip_w(sc.tx) - 1) / strip_w(sc.tx);
            }
            const int bands = nstrips ? G / nstrips / 8 * 8 : 0;
            if (bands < 8 || lats[0].ny < 8 * bands) return false;
            G = nstrips * bands;
        }
        int nb = 0;
        if (!build_segments(lats, sc.tx, G, max_items, items, &nb, sc.mode == 2)) return false;
        sc.grid = nb;
        int64_t total = 0;
        for (const auto& l : lats) total += (int64_t)((l.nx + strip_w(sc.tx) - 1) / strip_w(sc.tx)) * l.ny;
        sc.rows = nb ? (int)((total + nb - 1) / nb) : 0;
    }
    sc.n_items = (int)items.size();
    return true;
}


}  // namespace cmlb
