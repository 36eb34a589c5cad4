// reduce.hpp -- launch interface of the reductions of groups of PCFs
// (reduce.hip): the tree levels, the standard deviation's sums and the
// root's row rule.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcf {

// Reductions of groups of PCFs (reduce.hip). Ops as in pcf_reduce_op.
// RO_SUB, RO_MUL and RO_SQDIFF (a - b, ab, (a - b)^2) are combinations of two
// PCFs only: not associative, so never reduced over more than a pair.
enum { RO_SUM = 0, RO_MEAN = 1, RO_MAX = 2, RO_MIN = 3, RO_STD = 4, RO_SUB = 5, RO_MUL = 6, RO_SQDIFF = 7 };
struct RedLevelArgs {
    const int64_t *offsets;  // the set's CSR offsets (device, n+1)
    const int64_t *groups;   // group offsets (device, B+1)
    const int32_t *row_pcf;  // the PCF of every row (device, P)
    int64_t n;
    int32_t B;
    int level;               // inputs are items of 2^level PCFs
    const void *tin, *vin;
    void *tout, *vout;
};
struct RedStdArgs {
    const int64_t *offsets, *groups;
    int32_t B;
    int64_t rows;            // the set's total rows
    const void *t, *v;       // the set
    const void *rt, *rv;     // the sum tree's roots
    void *q;                 // out: sum of squared deviations per root row
    int64_t nchunks;         // the root pass's chunks (red_std_small)
    const int64_t *chunk_row, *chunk_grp;
    int64_t *chunk_first;    // scratch, 64 per chunk: PCF i's row at or before
                             // the chunk's first time
};
struct RedEmitArgs {
    const int64_t *offsets, *groups;
    int op;
    const void *rt, *rv;     // roots: times, and the values the rule compares
    int64_t nchunks;         // chunks of at most 1024 rows of one group
    const int64_t *chunk_row, *chunk_grp;
    int fill;                // 0: chunk_cnt[c] = kept rows; 1: write them
    int64_t *chunk_cnt;
    const int64_t *chunk_off;
    const int64_t *out_end;  // device: the output's total rows (fill)
    void *t_out, *v_out;
};
hipError_t launch_red_level(bool f64, int op, const RedLevelArgs &a, int64_t rows,
                            hipStream_t s);
hipError_t launch_red_interleave(bool f64, int64_t n, const int64_t *xo, const void *xt,
                                 const void *xv, const int64_t *yo, const void *yt,
                                 const void *yv, const int64_t *zo, void *zt, void *zv,
                                 hipStream_t s);
hipError_t launch_red_rowmap(const int64_t *offsets, int64_t n, int32_t *row_pcf, hipStream_t s);
// groups of more than 64 PCFs (a search per PCF and root row)
hipError_t launch_red_std(bool f64, const RedStdArgs &a, hipStream_t s);
// groups of at most 64 PCFs (a block per chunk of root rows, the PCF rows
// it selects staged in LDS)
hipError_t launch_red_std_small(bool f64, const RedStdArgs &a, hipStream_t s);
hipError_t launch_red_emit(bool f64, const RedEmitArgs &a, hipStream_t s);

}  // namespace pcf
