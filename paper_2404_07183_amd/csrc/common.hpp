// common.hpp -- types and constants shared by the host planner, the HIP
// kernels and the C-ABI layer of the PCF library (not by the CPU oracle).
#pragma once

#include <stdint.h>

namespace pcf {

// Merge steps per unrolled block of the inner loop. A pair's step count is
// rounded up to a multiple of this; the extra steps run past both
// sentinels and add exactly 0.
constexpr int kStepBlock = 8;
// Padding records after each PCF's last record so that those extra steps
// stay inside the PCF's own records.
constexpr int kPad = kStepBlock - 1;
// Threads per tile workgroup (16 waves of 64 lanes).
constexpr int kThreads = 1024;
// Tile workgroups resident per CU (they share its 160 KiB of LDS).
constexpr int kWgPerCu = 1;
// Most PCFs in one block (so a tile has at most kThreads pairs).
constexpr int kMaxBlock = 32;
constexpr int kMaxPairs = kMaxBlock * kMaxBlock;
// LDS bytes a tile may use for breakpoint records (of 160 KiB per CU on
// gfx950; the rest holds per-pair prefix sums, accumulators and block
// metadata).
#ifndef PCF_LDSREC
#define PCF_LDSREC (136 * 1024)
#endif
constexpr int kLdsRecordBytes = PCF_LDSREC;
// The adjoint's LDS bytes for records and gradient slots: its tile state
// holds partial-sum slots for one value a pair only (the pair weights), 8 KiB
// less than the forward's, which go to the records.
constexpr int kAdjLdsBytes = kLdsRecordBytes + 8 * 1024;
// The adjoint keeps two 64-bit gradient slots per record in two arrays after
// its records, dL/dv then dL/dt (8-byte strides, so that random slots spread
// over the LDS banks): adj_lds_records(rec_bytes) records a tile (a multiple
// of 64), and adj_gt_offset(rec_bytes) bytes from a record's dL/dv slot to
// its dL/dt slot (a constant offset of the LDS atomics, which holds 16 bits).
constexpr int adj_lds_records(int rec_bytes)
{
    return kAdjLdsBytes / (rec_bytes + 16) / 64 * 64;
}
constexpr uint32_t adj_gt_offset(int rec_bytes)
{
    return (uint32_t)adj_lds_records(rec_bytes) * 8;
}
// Records per thread when the adjoint stages a tile through registers.
constexpr int adj_stage_unroll(int rec_bytes)
{
    return (adj_lds_records(rec_bytes) + kThreads - 1) / kThreads;
}
static_assert(adj_gt_offset(16) + 8 * 8 <= 65535 && adj_gt_offset(8) + 8 * 8 <= 65535,
              "adjoint LDS layout");
static_assert(adj_lds_records(16) * (16 + 16) <= kAdjLdsBytes &&
                  adj_lds_records(8) * (8 + 16) <= kAdjLdsBytes,
              "adjoint LDS capacity");

// Rows a PCF may have (exclusive): keeps a pair's merge steps below 2^31.
constexpr int64_t kMaxRows = (int64_t)1 << 30;
// Number of hardware XCDs (each with its own L2) on MI355X.
constexpr int kXcds = 8;

enum SegType : int32_t { kSegTriangle = 0, kSegRect = 1 };

// A run of tiles sharing one output mapping. Triangle: all block pairs
// (I, J) with b0 <= I <= J < b1, column-major over the upper triangle.
// Rectangle: I in [b0, b1), J in [c0, c1), row-major.
struct Segment {
    int64_t tile_begin;  // index of the segment's first tile
    int64_t obase;       // output element offset of entry (row0, col0)
    int64_t ldo;         // output leading dimension (elements)
    int64_t row0, col0;  // PCF indices of output row 0 / column 0
    int32_t b0, b1, c0, c1;
    int32_t type;
    int32_t mirror;      // 1: also write the transposed entry
};

// Head of the device workspace. Written by the host planner (copied in
// once per plan) and read by every kernel, so a call that reuses a plan
// needs nothing from the host.
struct WsHeader {
    uint32_t counter[kXcds];  // tile counters, reset before each launch
    int64_t ntiles;
    int64_t nseg;
    int64_t nblocks;
    int64_t npcf;
    int64_t off_blocks;   // byte offsets inside the workspace
    int64_t off_segs;
    int64_t off_rec;
    int64_t rec_count;    // records in the packed array
    int64_t rec_bytes;    // bytes per record (8 FP32, 16 FP64)
    int64_t first_bad;    // validation result (PCF index or -1)
    int64_t lds_records;  // records a tile may hold in LDS
    // deterministic adjoint: the largest |W|, |v| and piece length, as bit
    // patterns (non-negative doubles order like their patterns)
    unsigned long long adj_max[3];
    int64_t off_acc;      // FP32 adjoint plans: 64-bit sums of dL/dt, dL/dv (2 x 8 bytes
                          // a row) for PCF_DETERMINISTIC; else 0
    int64_t reserved[1];
};
static_assert(sizeof(WsHeader) <= 256, "header must fit its slot");

constexpr int64_t kHeaderBytes = 256;

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace pcf
