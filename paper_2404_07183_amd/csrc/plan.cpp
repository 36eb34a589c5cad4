// plan.cpp -- host-side tile planner (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cstring>

namespace pcf {

int64_t lds_record_capacity(int rec_bytes, bool backward)
{
    // the adjoint keeps two 64-bit gradient accumulators per record slot,
    // at a fixed distance from the records
    if (backward)
        return adj_lds_records(rec_bytes);
    return kLdsRecordBytes / rec_bytes;
}

int64_t block_budget(int rec_bytes, bool backward, const TileShape &shape)
{
    const int32_t d = shape.budget_div >= 2 ? shape.budget_div : 2;
    return lds_record_capacity(rec_bytes, backward) / d;
}

void build_blocks(const int64_t *offsets, int64_t lo, int64_t hi,
                  std::vector<int64_t> cuts, int64_t budget, int32_t max_block,
                  std::vector<int32_t> &blocks)
{
    std::sort(cuts.begin(), cuts.end());
    size_t ci = 0;
    int64_t count = 0, recs = 0;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t r = offsets[i + 1] - offsets[i] + kPad;
        bool is_cut = false;
        while (ci < cuts.size() && cuts[ci] <= i) {
            if (cuts[ci] == i)
                is_cut = true;
            ++ci;
        }
        if (count == 0 || is_cut || count == max_block || recs + r > budget) {
            blocks.push_back((int32_t)i);
            count = 0;
            recs = 0;
        }
        ++count;
        recs += r;
    }
}

namespace {

// Index of the block starting at PCF i (i is a block boundary).
int32_t block_at(const std::vector<int32_t> &blocks, int64_t i)
{
    auto it = std::lower_bound(blocks.begin(), blocks.end(), (int32_t)i);
    return (int32_t)(it - blocks.begin());
}

bool check_offsets(int64_t n, const int64_t *offsets, std::string &err)
{
    if (n < 0) {
        err = "n < 0";
        return false;
    }
    if (n > 0 && offsets == nullptr) {
        err = "offsets is NULL";
        return false;
    }
    if (n > 0 && offsets[0] != 0) {
        err = "offsets[0] != 0";
        return false;
    }
    if (n >= ((int64_t)1 << 31)) {
        err = "more than 2^31 - 1 PCFs";
        return false;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (offsets[i + 1] <= offsets[i]) {
            err = "PCF " + std::to_string(i) +
                  " has no rows (every PCF needs at least one row)";
            return false;
        }
        if (offsets[i + 1] - offsets[i] >= kMaxRows) {
            err = "PCF " + std::to_string(i) + " has 2^30 rows or more";
            return false;
        }
    }
    return true;
}

void add_segment(Plan &plan, Segment s, int64_t tiles)
{
    if (tiles <= 0)
        return;
    s.tile_begin = plan.ntiles;
    plan.segs.push_back(s);
    plan.ntiles += tiles;
}

}  // namespace

bool plan_matrix(int64_t n, const int64_t *offsets, int rec_bytes,
                 bool backward, bool windowed, int64_t r0, int64_t r1,
                 int64_t c0, int64_t c1, bool upper_only, int64_t ldo,
                 const TileShape &shape, Plan &plan, std::string &err)
{
    plan = Plan();
    if (!check_offsets(n, offsets, err))
        return false;
    if (!windowed) {
        r0 = c0 = 0;
        r1 = c1 = n;
    }
    if (r0 < 0 || r1 < r0 || r1 > n || c0 < 0 || c1 < c0 || c1 > n) {
        err = "window out of range";
        return false;
    }
    if (ldo < (c1 - c0) || ldo < 1) {
        if (!(r1 == r0 || c1 == c0)) {
            err = "ldo smaller than the window width";
            return false;
        }
    }
    plan.npcf = n;
    plan.rec_count = (n > 0 ? offsets[n] : 0) + n * kPad;
    plan.lds_records = lds_record_capacity(rec_bytes, backward);
    plan.backward = backward;
    if (r1 == r0 || c1 == c0)
        return true;

    const int64_t d0 = std::max(r0, c0), d1 = std::min(r1, c1);
    const bool has_d = d0 < d1;
    const int64_t lo = std::min(r0, c0), hi = std::max(r1, c1);
    std::vector<int64_t> cuts = {r0, r1, c0, c1};
    if (has_d) {
        cuts.push_back(d0);
        cuts.push_back(d1);
    }
    build_blocks(offsets, lo, hi, cuts, block_budget(rec_bytes, backward, shape),
                 shape.max_block, plan.blocks);
    plan.blocks.push_back((int32_t)hi);

    Segment base{};
    base.obase = 0;
    base.ldo = ldo;
    base.row0 = r0;
    base.col0 = c0;

    auto rect = [&](int64_t ra, int64_t rb, int64_t ca, int64_t cb) {
        if (ra >= rb || ca >= cb)
            return;
        Segment s = base;
        s.type = kSegRect;
        s.mirror = 0;
        s.b0 = block_at(plan.blocks, ra);
        s.b1 = block_at(plan.blocks, rb);
        s.c0 = block_at(plan.blocks, ca);
        s.c1 = block_at(plan.blocks, cb);
        add_segment(plan, s, (int64_t)(s.b1 - s.b0) * (s.c1 - s.c0));
    };

    if (has_d) {
        Segment s = base;
        s.type = kSegTriangle;
        s.mirror = upper_only ? 0 : 1;
        s.b0 = block_at(plan.blocks, d0);
        s.b1 = block_at(plan.blocks, d1);
        s.c0 = s.b0;
        s.c1 = s.b1;
        const int64_t nb = s.b1 - s.b0;
        add_segment(plan, s, nb * (nb + 1) / 2);
        // rows outside the overlap against every column; overlap rows
        // against columns outside it (the transposes of these entries lie
        // outside the window, so nothing is mirrored)
        rect(r0, std::min(r1, d0), c0, c1);
        rect(std::max(r0, d1), r1, c0, c1);
        rect(d0, d1, c0, std::min(c1, d0));
        rect(d0, d1, std::max(c0, d1), c1);
    } else {
        rect(r0, r1, c0, c1);
    }
    return true;
}

bool plan_batched(int32_t B, const int64_t *set_offsets,
                  const int64_t *out_offsets, const int64_t *offsets,
                  int64_t n, int rec_bytes, bool upper_only,
                  const TileShape &shape, Plan &plan, std::string &err)
{
    plan = Plan();
    if (B < 0 || (B > 0 && (!set_offsets || !out_offsets))) {
        err = "bad batch description";
        return false;
    }
    if (!check_offsets(n, offsets, err))
        return false;
    for (int32_t b = 0; b < B; ++b) {
        if (set_offsets[b] < 0 || set_offsets[b + 1] < set_offsets[b] ||
            set_offsets[b + 1] > n) {
            err = "set_offsets out of range at problem " + std::to_string(b);
            return false;
        }
        if (out_offsets[b] < 0) {
            err = "negative out_offsets at problem " + std::to_string(b);
            return false;
        }
    }
    plan.npcf = n;
    plan.rec_count = (n > 0 ? offsets[n] : 0) + n * kPad;
    plan.lds_records = lds_record_capacity(rec_bytes, false);
    if (B == 0)
        return true;
    const int64_t lo = set_offsets[0], hi = set_offsets[B];
    std::vector<int64_t> cuts(set_offsets, set_offsets + B + 1);
    build_blocks(offsets, lo, hi, cuts, block_budget(rec_bytes, false, shape),
                 shape.max_block, plan.blocks);
    plan.blocks.push_back((int32_t)hi);

    struct Item {
        double cost;
        Segment s;
        int64_t tiles;
    };
    std::vector<Item> items;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t a = set_offsets[b], e = set_offsets[b + 1];
        if (a == e)
            continue;
        Segment s{};
        s.type = kSegTriangle;
        s.mirror = upper_only ? 0 : 1;
        s.obase = out_offsets[b];
        s.ldo = e - a;
        s.row0 = s.col0 = a;
        s.b0 = block_at(plan.blocks, a);
        s.b1 = block_at(plan.blocks, e);
        s.c0 = s.b0;
        s.c1 = s.b1;
        const int64_t nb = s.b1 - s.b0;
        // merge steps of a set of s PCFs with R rows in total: about
        // s * R (every PCF meets every other once)
        const double cost =
            (double)(e - a) * (double)(offsets[e] - offsets[a]);
        items.push_back({cost, s, nb * (nb + 1) / 2});
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &x, const Item &y) { return x.cost > y.cost; });
    for (auto &it : items)
        add_segment(plan, it.s, it.tiles);
    return true;
}

// FP32 adjoint plans: two 64-bit sums a row for PCF_DETERMINISTIC (FP64
// plans keep them in the gradient arrays themselves).
int64_t adj_acc_bytes(const Plan &plan, int rec_bytes)
{
    if (!plan.backward || rec_bytes == 16)
        return 0;
    const int64_t rows = plan.rec_count - plan.npcf * kPad;
    return align_up(rows * 16, 256);
}

int64_t plan_workspace_bytes(const Plan &plan, int rec_bytes)
{
    int64_t off = kHeaderBytes;
    off += align_up((int64_t)plan.blocks.size() * 4, 256);
    off += align_up((int64_t)plan.segs.size() * (int64_t)sizeof(Segment), 256);
    off += align_up(plan.rec_count * rec_bytes, 256);
    off += adj_acc_bytes(plan, rec_bytes);
    return off;
}

int64_t plan_workspace_bound(const Plan &plan, int rec_bytes)
{
    int64_t off = kHeaderBytes;
    off += align_up((plan.npcf + 1) * 4, 256);
    off += align_up((int64_t)plan.segs.size() * (int64_t)sizeof(Segment), 256);
    off += align_up(plan.rec_count * rec_bytes, 256);
    off += adj_acc_bytes(plan, rec_bytes);
    return off;
}

void plan_serialise(const Plan &plan, int rec_bytes,
                    std::vector<unsigned char> &buf, WsHeader &hdr)
{
    std::memset(&hdr, 0, sizeof(hdr));
    hdr.ntiles = plan.ntiles;
    hdr.nseg = (int64_t)plan.segs.size();
    hdr.nblocks = plan.blocks.empty() ? 0 : (int64_t)plan.blocks.size() - 1;
    hdr.npcf = plan.npcf;
    hdr.off_blocks = kHeaderBytes;
    hdr.off_segs = hdr.off_blocks + align_up((int64_t)plan.blocks.size() * 4, 256);
    hdr.off_rec = hdr.off_segs +
                  align_up((int64_t)plan.segs.size() * (int64_t)sizeof(Segment), 256);
    hdr.rec_count = plan.rec_count;
    hdr.rec_bytes = rec_bytes;
    hdr.first_bad = -1;
    hdr.lds_records = plan.lds_records;
    hdr.off_acc = adj_acc_bytes(plan, rec_bytes) > 0
                      ? hdr.off_rec + align_up(plan.rec_count * rec_bytes, 256)
                      : 0;
    buf.assign((size_t)hdr.off_rec, 0);
    std::memcpy(buf.data(), &hdr, sizeof(hdr));
    if (!plan.blocks.empty())
        std::memcpy(buf.data() + hdr.off_blocks, plan.blocks.data(),
                    plan.blocks.size() * 4);
    if (!plan.segs.empty())
        std::memcpy(buf.data() + hdr.off_segs, plan.segs.data(),
                    plan.segs.size() * sizeof(Segment));
}

}  // namespace pcf
