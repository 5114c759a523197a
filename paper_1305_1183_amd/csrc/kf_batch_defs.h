// kf_batch_defs.h -- tables shared by the batched host runtime and its kernel.
//
// A batch is many independent BiCGK and GEMVER instances (square, n <= 2048)
// whose operands sit in one float arena. The work of the batch is cut into
// items: whole instances, or row blocks of a larger instance. One persistent
// launch dequeues the items in a fixed order; cross-item dependencies (the
// column reductions of A^T r and B^T y, and GEMVER's w = alpha B x after x is
// complete) go through per-instance counters in the workspace.
#pragma once
#include <stdint.h>

#define KFB_MAX_N 2048
#define KFB_BUCKETS 6
#define KFB_THREADS 256

// item phases
#define KFB_BICGK 0     // rows of A: q rows, column partial of A^T r
#define KFB_GEMVER_K1 1 // rows of A: B rows, column partial of B^T y (whole instance: also K2)
#define KFB_GEMVER_K2 2 // rows of B: w rows, after x is complete

// sync words (uint32) at the start of the sync area
#define KFB_SYNC_QUEUE 0
#define KFB_SYNC_EXIT 1
#define KFB_SYNC_ERROR 2
#define KFB_SYNC_HEADER 16
// per split instance j: [HEADER + 4 j + 0] arrivals of phase-1 items,
// [+1] x complete flag, [+2] arrivals of K2 items
#define KFB_SYNC_PER_INST 4

// error bits
#define KFB_ERR_SPIN 1u

// vector slots: BiCGK p r q s; GEMVER u1 v1 u2 v2 y z x w
struct kfb_inst {
    int32_t kind;    // 0 BiCGK, 1 GEMVER
    int32_t n;       // rows = columns
    int32_t ld;      // row pitch of A and B in floats (multiple of 4)
    int32_t bucket;  // size bucket (tile shape)
    int32_t nblk;    // row blocks (1 = the instance is one item)
    int32_t rows;    // rows per block
    int32_t sync;    // index of the counters of a split instance, -1 if whole
    float alpha, beta;
    int32_t tile;    // entry of the tile menu of (kind, bucket)
    int64_t a, b;    // arena offsets of A and B (floats)
    int64_t v[8];    // arena offsets of the vectors
    int64_t ws;      // workspace offset of the column partials (floats), -1 if whole
};

struct kfb_item {
    int32_t inst;
    int32_t phase_blk;  // phase << 24 | block
};

static inline int kfb_bucket(int n) {
    return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : n <= 512 ? 3 : n <= 1024 ? 4 : 5;
}
// Tile menu per kind and size bucket; entry 0 is the default. A whole-row tile
// <LTPR, K, LG> lets TPR = 2^LTPR lanes share a row, K float4 chunks per lane
// (TPR K 4 >= the bucket's largest n), and walks 256 / TPR rows per step, G =
// 2^LG steps per row reduction. A wide tile (BiCGK above n = 512) lets the
// four waves split each row, K float4 chunks per lane of the workgroup, G =
// 2^LG rows per step. Entries with k = 0 are absent.
#define KFB_TILES 3
struct kfb_tile {
    int8_t wide, ltpr, k, lg;
};
constexpr kfb_tile kfb_tile_menu[2][KFB_BUCKETS][KFB_TILES] = {
    {   // BiCGK
        {{0, 4, 1, 2}, {0, 4, 1, 1}, {0, 3, 2, 2}},
        {{0, 5, 1, 2}, {0, 5, 1, 1}, {0, 4, 2, 2}},
        {{0, 6, 1, 2}, {0, 6, 1, 1}, {0, 5, 2, 2}},
        {{0, 6, 2, 2}, {0, 6, 2, 1}, {0, 5, 4, 1}},
        {{1, 0, 1, 3}, {1, 0, 1, 2}, {0, 6, 4, 1}},
        {{1, 0, 2, 2}, {1, 0, 2, 1}, {0, 6, 8, 0}},
    },
    {   // GEMVER
        {{0, 4, 1, 2}, {0, 4, 1, 1}, {0, 3, 2, 2}},
        {{0, 5, 1, 2}, {0, 5, 1, 1}, {0, 4, 2, 2}},
        {{0, 6, 1, 2}, {0, 6, 1, 1}, {0, 5, 2, 2}},
        {{0, 6, 2, 2}, {0, 6, 2, 1}, {0, 5, 4, 1}},
        {{0, 6, 4, 1}, {0, 6, 4, 0}, {0, 5, 8, 0}},
        {{0, 6, 8, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    },
};
// number of tiles on the menu of (kind, bucket)
static inline int kfb_tile_count(int kind, int bucket) {
    int c = 0;
    for (int t = 0; t < KFB_TILES; ++t) c += kfb_tile_menu[kind][bucket][t].k > 0;
    return c;
}
// rows one workgroup step covers with tile t of (kind, bucket) (the tile's row extent)
static inline int kfb_rows_per_step(int kind, int bucket, int t) {
    const kfb_tile& x = kfb_tile_menu[kind][bucket][t];
    return x.wide ? (1 << x.lg) : ((KFB_THREADS >> x.ltpr) << x.lg);
}
