// plan.hpp -- host-side tile planner for the pairwise PCF kernels.
//
// The matrix F(C) of Section 3.1 is cut into tiles: a tile pairs a block of
// consecutive PCFs (rows) with another block (columns). Blocks are built
// greedily along the PCF order so that the breakpoint records of any two
// blocks fit in one workgroup's LDS together; a PCF too long for that forms
// a block of its own and its tiles read records from global memory. Only the
// upper triangle of each symmetric part is tiled; the transposed entries are
// written from the same result (F is symmetric because h is).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "common.hpp"

namespace pcf {

struct Plan {
    std::vector<int32_t> blocks;  // block start PCF indices; back() = end
    std::vector<Segment> segs;
    int64_t ntiles = 0;
    int64_t npcf = 0;
    int64_t rec_count = 0;        // offsets[n] + n * kPad
    int64_t lds_records = 0;
    bool backward = false;        // an adjoint plan
};

// Tile shape: at most `max_block` PCFs per block and at most 1/`budget_div`
// of a tile's LDS record capacity per block (2: any two blocks fit).
struct TileShape {
    int32_t max_block = kMaxBlock;
    int32_t budget_div = 2;
};

// Records a block may hold.
int64_t block_budget(int rec_bytes, bool backward, const TileShape &shape);
// Records a tile may stage in LDS.
int64_t lds_record_capacity(int rec_bytes, bool backward);

// Greedy blocks over PCFs [lo, hi) with forced boundaries at `cuts`.
// Appends block starts (not the final end) to `blocks`.
void build_blocks(const int64_t *offsets, int64_t lo, int64_t hi,
                  std::vector<int64_t> cuts, int64_t budget, int32_t max_block,
                  std::vector<int32_t> &blocks);

// Plan for one n x n matrix, or the window [r0,r1) x [c0,c1) of it.
// Returns false with a message in `err` on bad input.
bool plan_matrix(int64_t n, const int64_t *offsets, int rec_bytes,
                 bool backward, bool windowed, int64_t r0, int64_t r1,
                 int64_t c0, int64_t c1, bool upper_only, int64_t ldo,
                 const TileShape &shape, Plan &plan, std::string &err);

// Plan for B independent full matrices in one launch.
bool plan_batched(int32_t B, const int64_t *set_offsets,
                  const int64_t *out_offsets, const int64_t *offsets,
                  int64_t n, int rec_bytes, bool upper_only,
                  const TileShape &shape, Plan &plan, std::string &err);

// Bytes of workspace a plan needs (header, blocks, segments, records).
// Bytes of an FP32 adjoint plan's 64-bit gradient sums (0 otherwise).
int64_t adj_acc_bytes(const Plan &plan, int rec_bytes);
int64_t plan_workspace_bytes(const Plan &plan, int rec_bytes);
// Upper bound of plan_workspace_bytes over all tile shapes (every PCF its
// own block).
int64_t plan_workspace_bound(const Plan &plan, int rec_bytes);

// Serialise the plan's header/blocks/segments into a host buffer laid out
// exactly like the workspace prefix (records region excluded).
void plan_serialise(const Plan &plan, int rec_bytes,
                    std::vector<unsigned char> &buf, WsHeader &hdr);

}  // namespace pcf
